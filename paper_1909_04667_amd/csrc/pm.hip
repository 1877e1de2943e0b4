// Particle-mesh long-range force for gfx950 (Sec. 3.3 and 3.4 of the Arepo
// paper): CIC deposit, FFT Poisson solve with the Gaussian long-range filter
// exp(-k^2 rs^2) and CIC deconvolution, four-point finite differences, CIC
// interpolation.  Mean density removed (k = 0 set to zero, Sec. 2.2).
//
// Layout: mesh index (i * ng + j) * ng + k, i <-> x.  The deposit accumulates
// fixed-point masses with integer atomics, so the mesh is independent of
// particle order (deterministic).  One 64-bit word per cell holds the mass at
// 2^-62 of the total: a mean cell of a 256^3 mesh then keeps only about 38
// bits, which for FP64 left errors of ~1e-11 of the mean density and up to
// ~5e-10 in the forces of weakly accelerated particles.  The FP64 solve
// therefore adds a second plane: each contribution's rounding residual,
// in [-1/2, 1/2] units of the first word, rounded at 2^-20 of that unit (so
// the residual sums of any cell stay below 2^52 in magnitude); the two
// integer sums are exact and order-independent, and the cell's mass is
// (hi + lo 2^-20) units, rounded once.  The 3-D FFT runs as five passes over
// the half spectrum of the real mesh (kz = 0 .. ng/2): forward z (reading the
// fixed-point mesh, two real lines per complex transform), forward y,
// [forward x, Green's function, inverse x] fused in LDS, inverse y, inverse z
// (writing the real potential, again two lines per transform).  Each pass
// holds a block of lines in registers and LDS (coalesced along the
// contiguous axis).
// The gradient is taken inside the interpolation kernel from the potential.
#include "pm_device.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace tpm {
namespace {

using namespace pmk;

constexpr int kBlock = 256;
constexpr size_t kFftLds = 64 * 1024;  // LDS budget of one FFT block

template <typename T>
struct Cx {
    T re, im;
};

// CIC base cell and weights of the particle at sorted slot s (Sec. 3.3):
// mesh points at i h, weights (1 - w, w) on cells i0 and i0 + 1 per axis.
// Any input (even outside the box or NaN) stays on the mesh.
__device__ __forceinline__ void cic_cell(const double *__restrict__ ps, int64_t n, int64_t s,
                                         const MeshGeom &mg, int i0[3], double w[3]) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double u = ps[(size_t)a * n + s] - mg.lo[a];
        if (mg.box > 0.0) {
            if (u < 0.0)
                u += mg.box;
            if (u >= mg.box)
                u -= mg.box;
        }
        const double f = u / mg.h;
        const double fl = floor(f);
        w[a] = f - fl;
        int i = (int)fmin(fmax(fl, -1.0e9), 1.0e9) % mg.ng;
        if (i < 0)
            i += mg.ng;
        i0[a] = i;
    }
}

// The deposit as fixed-point integers (order-independent, hence
// deterministic).  A workgroup takes kDepChunk consecutive particles in curve
// order, a compact region of the mesh: their contributions are summed in an
// LDS tile over the region's bounding box (cell offsets from the chunk's
// first particle, nearest image), and the tile is added to the mesh row by
// row, so the device-scope atomics of a wavefront hit consecutive cells.  A
// chunk whose box exceeds the tile adds its contributions directly.
// TWO: the second plane of residuals (mesh + plane) described above.
constexpr int kDepPer = 1;
constexpr int kDepChunk = kBlock * kDepPer;
constexpr int kDepTile = 3072;  // cells (24 KB per plane)

// Fixed-point parts of one contribution v (in units of the first word):
// hi = v rounded to an integer; lo = (v - hi) 2^20 rounded, two's complement.
// v - hi is exact (Sterbenz), as is its scaling by 2^20.
template <bool TWO>
__device__ __forceinline__ void fixed_parts(double v, unsigned long long &hi,
                                            unsigned long long &lo) {
    const double vr = rint(v);
    hi = (unsigned long long)vr;
    lo = TWO ? (unsigned long long)(long long)rint((v - vr) * 0x1p20) : 0ull;
}

template <bool TWO>
__global__ __launch_bounds__(kBlock) void k_deposit(const double *__restrict__ ps,
                                                    const double *__restrict__ ms, int64_t n,
                                                    const Rec64 *__restrict__ rec, MeshGeom mg,
                                                    unsigned long long *__restrict__ mesh,
                                                    size_t plane) {
    __shared__ unsigned long long tile[TWO ? 2 * kDepTile : kDepTile];
    __shared__ int red[6][kBlock / 64];
    __shared__ int refc[3];
    const int ng = mg.ng, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t s0 = (int64_t)blockIdx.x * kDepChunk;  // < n
    int ex;
    frexp(rec[0].mass, &ex);  // total mass < 2^ex
    const double scale = ldexp(1.0, 62 - ex);
    int i0[kDepPer][3], o[kDepPer][3];
    double w[kDepPer][3], m[kDepPer];
    bool live[kDepPer];
#pragma unroll
    for (int p = 0; p < kDepPer; p++) {
        const int64_t s = s0 + p * kBlock + tid;
        live[p] = s < n;
        cic_cell(ps, n, live[p] ? s : s0, mg, i0[p], w[p]);
        m[p] = live[p] ? ms[s] : 0.0;
    }
    if (tid == 0) {  // the chunk's first particle is thread 0's first
        refc[0] = i0[0][0];
        refc[1] = i0[0][1];
        refc[2] = i0[0][2];
    }
    __syncthreads();
    int lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        lo[a] = ng;
        hi[a] = -ng;
#pragma unroll
        for (int p = 0; p < kDepPer; p++) {
            int d = i0[p][a] - refc[a];  // nearest image, |d| <= ng / 2
            if (2 * d > ng)
                d -= ng;
            if (2 * d < -ng)
                d += ng;
            o[p][a] = live[p] ? d : 0;
            lo[a] = min(lo[a], o[p][a]);
            hi[a] = max(hi[a], o[p][a]);
        }
        for (int k = 1; k < 64; k <<= 1) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], k));
            hi[a] = max(hi[a], __shfl_xor(hi[a], k));
        }
        if (lane == 0) {
            red[a][wv] = lo[a];
            red[3 + a][wv] = hi[a];
        }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; a++) {
        lo[a] = red[a][0];
        hi[a] = red[3 + a][0];
        for (int q = 1; q < kBlock / 64; q++) {
            lo[a] = min(lo[a], red[a][q]);
            hi[a] = max(hi[a], red[3 + a][q]);
        }
    }
    // the tile spans offsets lo .. hi + 1 (the upper CIC neighbours)
    const int D0 = hi[0] - lo[0] + 2, D1 = hi[1] - lo[1] + 2, D2 = hi[2] - lo[2] + 2;
    const int64_t V = (int64_t)D0 * D1 * D2;
    if (V <= kDepTile) {
        for (int k = tid; k < (int)V; k += kBlock) {
            tile[k] = 0ull;
            if (TWO)
                tile[kDepTile + k] = 0ull;
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < kDepPer; p++) {
            if (!live[p])
                continue;
#pragma unroll
            for (int c = 0; c < 8; c++) {
                double wt = 1.0;
                int t[3];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const int up = (c >> (2 - a)) & 1;
                    wt *= up ? w[p][a] : 1.0 - w[p][a];
                    t[a] = o[p][a] - lo[a] + up;
                }
                unsigned long long qh, ql;
                fixed_parts<TWO>(m[p] * wt * scale, qh, ql);
                const int cell = (t[0] * D1 + t[1]) * D2 + t[2];
                atomicAdd(&tile[cell], qh);
                if (TWO)
                    atomicAdd(&tile[kDepTile + cell], ql);
            }
        }
        __syncthreads();
        for (int k = tid; k < (int)V; k += kBlock) {
            const unsigned long long v = tile[k];
            const unsigned long long vl = TWO ? tile[kDepTile + k] : 0ull;
            if (v || vl) {
                const int l2 = k % D2, l1 = (k / D2) % D1, l0 = k / (D1 * D2);
                int g[3] = {refc[0] + lo[0] + l0, refc[1] + lo[1] + l1, refc[2] + lo[2] + l2};
#pragma unroll
                for (int a = 0; a < 3; a++)
                    g[a] = ((g[a] % ng) + ng) % ng;
                const size_t cell = ((size_t)g[0] * ng + g[1]) * ng + g[2];
                atomicAdd(&mesh[cell], v);
                if (TWO)
                    atomicAdd(&mesh[plane + cell], vl);
            }
        }
    } else {
#pragma unroll
        for (int p = 0; p < kDepPer; p++) {
            if (!live[p])
                continue;
#pragma unroll
            for (int c = 0; c < 8; c++) {
                double wt = 1.0;
                int t[3];
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const int up = (c >> (2 - a)) & 1;
                    wt *= up ? w[p][a] : 1.0 - w[p][a];
                    t[a] = up ? (i0[p][a] + 1 == ng ? 0 : i0[p][a] + 1) : i0[p][a];
                }
                unsigned long long qh, ql;
                fixed_parts<TWO>(m[p] * wt * scale, qh, ql);
                const size_t cell = ((size_t)t[0] * ng + t[1]) * ng + t[2];
                atomicAdd(&mesh[cell], qh);
                if (TWO)
                    atomicAdd(&mesh[plane + cell], ql);
            }
        }
    }
}

// ---- FFT: four-step decomposition in registers ------------------------------
//
// A line of ng = R1 * R2 points (n = R2 n1 + n2, k = k1 + R1 k2) is handled by
// R2 threads.  Thread n2 loads x[R2 n1 + n2] (n1 = 0 .. R1-1), takes an R1-point
// DFT in registers, multiplies by W_ng^(n2 k1), and writes the row to LDS;
// after one exchange, thread t takes the R2-point DFTs of the columns
// k1 = t (+ R2) and holds X[k1 + R1 k2].  Small DFTs are radix-2
// decimation-in-frequency with compile-time twiddles (the output comes out in
// bit-reversed order, which is only a renaming of registers).

// cos(pi k / 16), k = 0 .. 8 (exact 0, 1 and sqrt(2)/2 where they occur)
__device__ constexpr double kCosQ[9] = {1.0,
                                        0.9807852804032304,
                                        0.9238795325112867,
                                        0.8314696123025452,
                                        0.7071067811865476,
                                        0.5555702330196023,
                                        0.38268343236508984,
                                        0.19509032201612833,
                                        0.0};

// exp(-2 pi i m / 32), compile-time m
template <int M>
struct W32 {
    static constexpr int m = M & 31, q = m / 8, r = m % 8;
    static constexpr double c = q == 0 ? kCosQ[r] : q == 1 ? -kCosQ[8 - r] : q == 2 ? -kCosQ[r] : kCosQ[8 - r];
    static constexpr double s = q == 0 ? kCosQ[8 - r] : q == 1 ? kCosQ[r] : q == 2 ? -kCosQ[8 - r] : -kCosQ[r];
    // W = cos - i sin
};

template <int R>
__device__ constexpr int bitrev(int k) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (k & 1);
        k >>= 1;
    }
    return r;
}

template <typename T, bool INV, int M>
__device__ __forceinline__ Cx<T> twiddle_mul(Cx<T> v) {
    if constexpr ((M & 31) == 0) {
        return v;
    } else if constexpr ((M & 31) == 8) {  // -i (forward) / +i (inverse)
        return INV ? Cx<T>{-v.im, v.re} : Cx<T>{v.im, -v.re};
    } else if constexpr ((M & 31) == 16) {
        return Cx<T>{-v.re, -v.im};
    } else if constexpr ((M & 31) == 24) {
        return INV ? Cx<T>{v.im, -v.re} : Cx<T>{-v.im, v.re};
    } else {
        const T c = (T)W32<M>::c, sn = INV ? (T)W32<M>::s : (T)-W32<M>::s;
        return Cx<T>{v.re * c - v.im * sn, v.re * sn + v.im * c};
    }
}

// One DIF butterfly stage of length LEN on an R-point register array.
template <typename T, bool INV, int R, int LEN, int J>
__device__ __forceinline__ void dif_j(Cx<T> *v) {
    if constexpr (J < LEN / 2) {
#pragma unroll
        for (int i = 0; i < R; i += LEN) {
            const Cx<T> a = v[i + J], b = v[i + J + LEN / 2];
            v[i + J] = Cx<T>{a.re + b.re, a.im + b.im};
            v[i + J + LEN / 2] = twiddle_mul<T, INV, J * (32 / LEN)>(Cx<T>{a.re - b.re, a.im - b.im});
        }
        dif_j<T, INV, R, LEN, J + 1>(v);
    }
}

template <typename T, bool INV, int R, int LEN>
__device__ __forceinline__ void dif_stages(Cx<T> *v) {
    if constexpr (LEN >= 2) {
        dif_j<T, INV, R, LEN, 0>(v);
        dif_stages<T, INV, R, LEN / 2>(v);
    }
}

// In-register R-point DFT; the result X[k] is left in v[bitrev(k)].
template <typename T, bool INV, int R>
__device__ __forceinline__ void dft_regs(Cx<T> *v) {
    dif_stages<T, INV, R, R>(v);
}

struct FftPass {
    int axis;        // 0: x, 1: y, 2: z (contiguous)
    int in_fixed;    // read the fixed-point deposit (axis 2, forward only)
    int out_real;    // write the scaled real part (axis 2, inverse only)
    int inverse;
    int green;       // forward, multiply by the Green's function, inverse
    // Half spectrum of a real mesh: the complex mesh holds kz = 0 .. ng/2
    // only, (i * ng + j) * (ng/2 + 1) + kz.  The z passes then transform two
    // real lines (j, j + 1) as one complex line: forward, their spectra are
    // C[k] +- conj(C[ng - k]) halves; inverse, C = A + i B is rebuilt from the
    // two half spectra by Hermitian symmetry and its real and imaginary parts
    // are the two real lines.  Otherwise the mesh is fully complex.
    int half;
};

// One line transform: on entry thread n2 holds a[n1] = x[R2 n1 + n2]; on exit
// it holds, for column c (k1 = n2 + c R2), X[k1 + R1 k2] in out[c * R2 + k2].
template <typename T, bool INV, int R1, int R2>
__device__ __forceinline__ void line_fft(Cx<T> *a, Cx<T> *out, Cx<T> *row, int n2,
                                         const Cx<T> *__restrict__ tw, bool active) {
    constexpr int NG = R1 * R2, C = R1 / R2, PAD = R2 + 1;
    if (active) {
        dft_regs<T, INV, R1>(a);
#pragma unroll
        for (int k1 = 0; k1 < R1; k1++) {
            Cx<T> v = a[bitrev<R1>(k1)];
            if (k1 && n2) {
                Cx<T> w = tw[(n2 * k1) & (NG - 1)];
                if (INV)
                    w.im = -w.im;
                v = Cx<T>{v.re * w.re - v.im * w.im, v.re * w.im + v.im * w.re};
            }
            row[k1 * PAD + n2] = v;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int c = 0; c < C; c++) {
            const int k1 = n2 + c * R2;
            Cx<T> b[R2];
#pragma unroll
            for (int m = 0; m < R2; m++)
                b[m] = row[k1 * PAD + m];
            dft_regs<T, INV, R2>(b);
#pragma unroll
            for (int k2 = 0; k2 < R2; k2++)
                out[c * R2 + k2] = b[bitrev<R2>(k2)];
        }
    }
    __syncthreads();
}

// Mass of cell g in units of the first word: hi, plus lo 2^-20 when the
// residual plane exists (plane > 0); one rounding.
__device__ __forceinline__ double fixed_value(const unsigned long long *__restrict__ mq,
                                              size_t plane, size_t g) {
    const double hi = (double)mq[g];
    return plane ? fma((double)(long long)mq[plane + g], 0x1p-20, hi) : hi;
}

template <typename T, int R1, int R2>
__global__ __launch_bounds__(kBlock) void k_fft(FftPass ps, int B, Cx<T> *__restrict__ mesh,
                                                const unsigned long long *__restrict__ mq,
                                                T *__restrict__ phi, const Cx<T> *__restrict__ tw,
                                                const double *__restrict__ gk2,
                                                const double *__restrict__ gq, double gconst,
                                                const double *__restrict__ gtab,
                                                const Rec64 *__restrict__ rec, double vinv,
                                                double norm, size_t plane) {
    constexpr int NG = R1 * R2, C = R1 / R2, PAD = R2 + 1, H = NG / 2 + 1;
    extern __shared__ unsigned char lds_raw[];
    Cx<T> *lds = (Cx<T> *)lds_raw;  // B rows of R1 x (R2 + 1)
    const int tid = threadIdx.x;
    int b, n2;
    if (ps.axis == 2) {  // contiguous lines: a line's threads adjacent
        b = tid / R2;
        n2 = tid % R2;
    } else {  // strided lines: neighbouring lines adjacent (coalesced)
        n2 = tid / B;
        b = tid % B;
    }
    bool active = b < B && n2 < R2 && tid < B * R2;
    size_t base, stride;
    size_t hb = 0;             // half spectrum of the first line of a z pair
    int jline = 0, kline = 0;  // (y, z) of an x line, for the Green's function
    if (ps.axis == 2) {
        if (ps.half) {  // line pair (j, j + 1): real lines base, base + NG
            const size_t pr = (size_t)blockIdx.x * B + b;
            const size_t i = pr / (NG / 2), j = 2 * (pr % (NG / 2));
            base = (i * NG + j) * NG;
            hb = (i * NG + j) * H;
        } else {
            base = ((size_t)blockIdx.x * B + b) * NG;
        }
        stride = 1;
    } else {
        const int W = ps.half ? H : NG;  // lines per value of the outer index
        const int per = (W + B - 1) / B;
        const size_t outer = blockIdx.x / per, kz = (size_t)(blockIdx.x % per) * B + b;
        active = active && kz < (size_t)W;
        base = ps.axis == 1 ? outer * NG * W + kz : outer * W + kz;
        stride = ps.axis == 1 ? (size_t)W : (size_t)NG * W;
        jline = (int)outer;
        kline = (int)kz;
    }
    Cx<T> *row = lds + (size_t)(active ? b : 0) * R1 * PAD;
    double qscale = 0.0;
    if (ps.in_fixed) {
        int ex;
        frexp(rec[0].mass, &ex);
        qscale = ldexp(1.0, ex - 62) * vinv;
    }
    Cx<T> a[R1], o[R1];
    if (active) {
#pragma unroll
        for (int n1 = 0; n1 < R1; n1++) {
            const int pos = R2 * n1 + n2;
            if (ps.in_fixed) {
                const size_t g = base + (size_t)pos;
                a[n1] = Cx<T>{(T)(fixed_value(mq, plane, g) * qscale),
                              ps.half ? (T)(fixed_value(mq, plane, g + NG) * qscale) : (T)0};
            } else if (ps.half && ps.axis == 2) {
                // C[k] = A_k + i B_k; above ng/2 from A_(ng-k) = conj(A_k)
                const int kk = pos <= NG / 2 ? pos : NG - pos;
                const Cx<T> A = mesh[hb + kk], Bv = mesh[hb + H + kk];
                a[n1] = pos <= NG / 2 ? Cx<T>{A.re - Bv.im, A.im + Bv.re}
                                      : Cx<T>{A.re + Bv.im, Bv.re - A.im};
            } else {
                a[n1] = mesh[base + (size_t)pos * stride];
            }
        }
    }
    if (ps.inverse && !ps.green)
        line_fft<T, true, R1, R2>(a, o, row, n2, tw, active);
    else
        line_fft<T, false, R1, R2>(a, o, row, n2, tw, active);
    if (ps.green) {
        // natural order through LDS, Green's function, inverse transform
        Cx<T> *line = row;  // reuse this line's LDS (NG <= R1 * PAD)
        if (active) {
#pragma unroll
            for (int c = 0; c < C; c++)
#pragma unroll
                for (int k2 = 0; k2 < R2; k2++)
                    line[(n2 + c * R2) + R1 * k2] = o[c * R2 + k2];
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int n1 = 0; n1 < R1; n1++) {
                const int i = R2 * n1 + n2;
                double g = 0.0;
                if (gtab) {
                    // isolated: the table holds one octant of the (even)
                    // transformed kernel, (NG/2 + 1)^3 values
                    constexpr int GH = NG / 2 + 1;
                    const int ii = i <= NG / 2 ? i : NG - i;
                    const int jj = jline <= NG / 2 ? jline : NG - jline;
                    const int kk = kline <= NG / 2 ? kline : NG - kline;
                    g = gconst * gtab[((size_t)ii * GH + jj) * GH + kk];
                } else {
                    const double k2s = (gk2[i] + gk2[jline]) + gk2[kline];
                    const double q = (gq[i] * gq[jline]) * gq[kline];
                    if (k2s != 0.0)
                        g = gconst * q / k2s;
                }
                const Cx<T> v = line[i];
                a[n1] = Cx<T>{(T)(v.re * g), (T)(v.im * g)};
            }
        }
        __syncthreads();
        line_fft<T, true, R1, R2>(a, o, row, n2, tw, active);
    }
    if (ps.half && ps.in_fixed) {
        // two real lines from one transform: A_k = (C_k + conj C_-k) / 2,
        // B_k = (C_k - conj C_-k) / 2i, k = 0 .. ng/2
        Cx<T> *line = row;
        if (active) {
#pragma unroll
            for (int c = 0; c < C; c++)
#pragma unroll
                for (int k2 = 0; k2 < R2; k2++)
                    line[(n2 + c * R2) + R1 * k2] = o[c * R2 + k2];
        }
        __syncthreads();
        if (active) {
            for (int k = n2; k <= NG / 2; k += R2) {
                const Cx<T> ck = line[k], cm = line[(NG - k) & (NG - 1)];
                mesh[hb + k] = Cx<T>{(T)0.5 * (ck.re + cm.re), (T)0.5 * (ck.im - cm.im)};
                mesh[hb + H + k] = Cx<T>{(T)0.5 * (ck.im + cm.im), (T)0.5 * (cm.re - ck.re)};
            }
        }
        return;
    }
    if (active) {
#pragma unroll
        for (int c = 0; c < C; c++)
#pragma unroll
            for (int k2 = 0; k2 < R2; k2++) {
                const size_t pos = (size_t)((n2 + c * R2) + R1 * k2);
                const Cx<T> v = o[c * R2 + k2];
                if (ps.out_real) {
                    phi[base + pos] = (T)(v.re * norm);
                    if (ps.half)
                        phi[base + NG + pos] = (T)(v.im * norm);
                } else {
                    mesh[base + pos * stride] = v;
                }
            }
    }
}

// Fused four-point difference and CIC interpolation, over the active slots
// in curve order (neighbouring threads read neighbouring mesh cells); the
// results go to slot order and are scattered to caller order afterwards.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_interp(const uint32_t *__restrict__ act,
                                                   const uint32_t *__restrict__ nuniq,
                                                   int64_t n, const double *__restrict__ ps,
                                                   const T *__restrict__ phi, MeshGeom mg,
                                                   T *__restrict__ res, T *__restrict__ rpot) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= (int64_t)*nuniq)
        return;
    double F[3], P;
    interp_at<T>(ps, n, act[k], phi, mg, F, P);
    T *r = res + 4 * (size_t)k;  // the slot's record (fourth value unused)
    r[0] = (T)F[0];
    r[1] = (T)F[1];
    r[2] = (T)F[2];
    rpot[k] = (T)P;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_out(
    const int32_t *__restrict__ idx, int64_t n_act, int64_t n, const int32_t *__restrict__ rank,
    const uint32_t *__restrict__ slot, const uint32_t *__restrict__ nuniq,
    const T *__restrict__ res, const T *__restrict__ rpot, T *__restrict__ acc,
    T *__restrict__ pot, uint32_t *__restrict__ err) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_act)
        return;
    const int32_t i = idx[k];
    if (i < 0 || (int64_t)i >= n) {
        acc[k] = acc[n_act + k] = acc[2 * n_act + k] = (T)NAN;
        if (pot)
            pot[k] = (T)NAN;
        atomicOr(err, 1u);
        return;
    }
    // with every particle active the slots are the ranks
    const uint32_t rk = (uint32_t)rank[i];
    const uint32_t sl = *nuniq == (uint32_t)n ? rk : slot[rk];
    const T *r = res + 4 * (size_t)sl;
    acc[k] = r[0];
    acc[n_act + k] = r[1];
    acc[2 * n_act + k] = r[2];
    if (pot)
        pot[k] = rpot[sl];
}

struct FftArgs {
    const double *gk2 = nullptr, *gq = nullptr, *gtab = nullptr;
    double gconst = 0.0, vinv = 1.0, norm = 1.0;
    const Rec64 *rec = nullptr;
    size_t plane = 0;  // offset of the residual plane of the deposit (0: none)
};

template <typename T, int R1, int R2>
int launch_fft(tpm_ctx *c, const FftPass &fp, Cx<T> *mc, const unsigned long long *mq, T *phi,
               const Cx<T> *tw, const FftArgs &fa) {
    constexpr int NG = R1 * R2;
    // lines per block: one wavefront group of R2 threads per line, at most
    // kBlock threads, the LDS rows within the budget, and B | NG
    int B = kBlock / R2;
    while ((size_t)B * R1 * (R2 + 1) * sizeof(Cx<T>) > kFftLds)
        B >>= 1;
    if (B > NG)
        B = NG;
    const size_t lds = (size_t)B * R1 * (R2 + 1) * sizeof(Cx<T>);
    size_t lines = (size_t)NG * NG;
    if (fp.half)  // z: line pairs; x, y: ng/2 + 1 lines per outer index
        lines = fp.axis == 2 ? (size_t)NG * (NG / 2)
                             : (size_t)NG * (((NG / 2 + 1) + B - 1) / B) * B;
    const unsigned blocks = (unsigned)(lines / B);
    k_fft<T, R1, R2><<<blocks, kBlock, lds, c->stream>>>(fp, B, mc, mq, phi, tw, fa.gk2,
                                                         fa.gq, fa.gconst, fa.gtab, fa.rec,
                                                         fa.vinv, fa.norm, fa.plane);
    TPM_LAUNCHED(c, "k_fft");
    return TPM_OK;
}

// One pass over an ng^3 mesh with the register decomposition of ng.
template <typename T>
int fft_pass(tpm_ctx *c, int ng, const FftPass &fp, Cx<T> *mc, const unsigned long long *mq,
             T *phi, const Cx<T> *tw, const FftArgs &fa) {
    switch (ng) {
    case 8: return launch_fft<T, 4, 2>(c, fp, mc, mq, phi, tw, fa);
    case 16: return launch_fft<T, 4, 4>(c, fp, mc, mq, phi, tw, fa);
    case 32: return launch_fft<T, 8, 4>(c, fp, mc, mq, phi, tw, fa);
    case 64: return launch_fft<T, 8, 8>(c, fp, mc, mq, phi, tw, fa);
    case 128: return launch_fft<T, 16, 8>(c, fp, mc, mq, phi, tw, fa);
    case 256: return launch_fft<T, 16, 16>(c, fp, mc, mq, phi, tw, fa);
    case 512: return launch_fft<T, 32, 16>(c, fp, mc, mq, phi, tw, fa);
    case 1024: return launch_fft<T, 32, 32>(c, fp, mc, mq, phi, tw, fa);
    default: return fail(c, TPM_EINVAL, "unsupported mesh size");
    }
}

template <typename T>
std::vector<Cx<T>> twiddles(int ng) {
    std::vector<Cx<T>> tw(ng);
    for (int k = 0; k < ng; k++) {
        const double a = 2.0 * M_PI * k / ng;
        tw[k] = Cx<T>{(T)std::cos(a), (T)-std::sin(a)};
    }
    return tw;
}

// Isolated mesh: the long-range kernel -erf(rho / 2 a) / rho in units of the
// mesh spacing (rho = r / h, a = r_s / h), value -1 / (sqrt(pi) a) at rho = 0,
// at the signed offsets of the padded M^3 mesh.
__global__ __launch_bounds__(kBlock) void k_green_fill(Cx<double> *__restrict__ mesh, int M,
                                                       double inv2a) {
    const size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t m3 = (size_t)M * M * M;
    if (q >= m3)
        return;
    const int k = (int)(q % M), j = (int)((q / M) % M), i = (int)(q / ((size_t)M * M));
    const int h = M / 2;
    const double o0 = i < h ? i : i - M, o1 = j < h ? j : j - M, o2 = k < h ? k : k - M;
    const double rho = sqrt(o0 * o0 + o1 * o1 + o2 * o2);
    const double v = rho == 0.0 ? -2.0 * inv2a / sqrt(M_PI) : -erf(rho * inv2a) / rho;
    mesh[q] = Cx<double>{v, 0.0};
}

// One octant of the transformed kernel (real: the kernel is even), divided
// by the CIC deconvolution prod_a sinc^4(pi n_a / M).
__global__ __launch_bounds__(kBlock) void k_green_table(const Cx<double> *__restrict__ mesh,
                                                        int M, double *__restrict__ tab) {
    const int gh = M / 2 + 1;
    const size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (size_t)gh * gh * gh)
        return;
    const int idx[3] = {(int)(q / ((size_t)gh * gh)), (int)((q / gh) % gh), (int)(q % gh)};
    double dc = 1.0;
    for (int a = 0; a < 3; a++) {
        const double sarg = M_PI * idx[a] / M;
        const double sc = idx[a] == 0 ? 1.0 : sin(sarg) / sarg;
        dc *= sc * sc * sc * sc;
    }
    tab[q] = mesh[((size_t)idx[0] * M + idx[1]) * M + idx[2]].re / dc;
}

// Builds the isolated Green's function table once per context (it depends
// only on pm_grid and asmth, in units of the mesh spacing).
int build_green_isolated(tpm_ctx *c) {
    const int ng = c->P.pm_grid, M = 2 * ng, gh = ng + 1;
    if (c->green_tab_ng == ng && c->green_tab.p)
        return TPM_OK;
    const size_t m3 = (size_t)M * M * M;
    hipStream_t st = c->stream;
    DBuf tmp, twb;
    auto release = [&] {
        (void)hipStreamSynchronize(st);
        if (tmp.p)
            (void)hipFree(tmp.p);
        if (twb.p)
            (void)hipFree(twb.p);
        tmp.p = twb.p = nullptr;
    };
    if (hipMalloc(&tmp.p, m3 * sizeof(Cx<double>)) != hipSuccess ||
        hipMalloc(&twb.p, (size_t)M * sizeof(Cx<double>)) != hipSuccess) {
        (void)hipGetLastError();
        release();
        return fail(c, TPM_ENOMEM, "isolated Green's function: out of device memory");
    }
    const std::vector<Cx<double>> tw = twiddles<double>(M);
    int rc = TPM_OK;
    if (hipMemcpyAsync(twb.p, tw.data(), tw.size() * sizeof(Cx<double>), hipMemcpyHostToDevice,
                       st) != hipSuccess)
        rc = fail(c, TPM_EDEVICE, "isolated Green's function: copy failed");
    if (rc == TPM_OK)
        rc = ensure(c, c->green_tab, (size_t)gh * gh * gh * sizeof(double));
    if (rc == TPM_OK) {
        k_green_fill<<<(unsigned)((m3 + kBlock - 1) / kBlock), kBlock, 0, st>>>(
            (Cx<double> *)tmp.p, M, 0.5 / c->P.asmth);
        if (hipGetLastError() != hipSuccess)
            rc = fail(c, TPM_EDEVICE, "k_green_fill launch failed");
    }
    const FftPass fwd[3] = {{2, 0, 0, 0, 0}, {1, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
    for (int k = 0; k < 3 && rc == TPM_OK; k++)
        rc = fft_pass<double>(c, M, fwd[k], (Cx<double> *)tmp.p, nullptr, nullptr,
                              (const Cx<double> *)twb.p, FftArgs{});
    if (rc == TPM_OK) {
        const size_t g3 = (size_t)gh * gh * gh;
        k_green_table<<<(unsigned)((g3 + kBlock - 1) / kBlock), kBlock, 0, st>>>(
            (const Cx<double> *)tmp.p, M, (double *)c->green_tab.p);
        if (hipGetLastError() != hipSuccess)
            rc = fail(c, TPM_EDEVICE, "k_green_table launch failed");
    }
    release();  // waits for the stream: the table is complete
    if (rc == TPM_OK)
        c->green_tab_ng = ng;
    return rc;
}

template <typename T>
int solve_t(tpm_ctx *c) {
    const tpm_params &P = c->P;
    const bool iso = !P.periodic;
    const MeshGeom mg = mesh_geom(c);
    const int M = mg.ng;  // transformed mesh
    const size_t n3 = (size_t)M * M * M;
    hipStream_t st = c->stream;
    if (iso)
        TPM_TRY(build_green_isolated(c));
    // FP64: a second plane of deposit residuals
    constexpr bool kTwo = sizeof(T) == sizeof(double);
    const size_t planes = kTwo ? 2 : 1;
    TPM_TRY(ensure(c, c->mesh_q, planes * n3 * 8));
    // half spectrum of the real mesh: kz = 0 .. M/2
    TPM_TRY(ensure(c, c->mesh_c, (size_t)M * M * (M / 2 + 1) * sizeof(Cx<T>)));
    TPM_TRY(ensure(c, c->mesh_phi, n3 * sizeof(T)));
    TPM_TRY(ensure(c, c->twiddle, (size_t)M * sizeof(Cx<T>) + 64));
    TPM_TRY(ensure(c, c->green_axis, (size_t)2 * M * sizeof(double)));
    // tables, computed in double on the host once per context (they depend
    // on the mesh size and the fixed parameters only).  Periodic Green's
    // function per axis: k_a^2 and exp(-k_a^2 r_s^2) / sinc^4(k_a h / 2);
    // the filter and the deconvolution are products over the axes, so a
    // mesh point needs three multiplications and one division.
    if (c->axis_tables_M != M) {
        const std::vector<Cx<T>> tw = twiddles<T>(M);
        std::vector<double> g(2 * M, 0.0);
        if (!iso) {
            const double box = P.box_size, h = mg.h;
            const double rs = P.asmth * P.box_size / P.pm_grid;
            for (int i = 0; i < M; i++) {
                const int nn = i < M / 2 ? i : i - M;
                const double kv = 2.0 * M_PI * nn / box;
                const double s = 0.5 * kv * h;
                const double sc = nn == 0 ? 1.0 : std::sin(s) / s;
                g[i] = kv * kv;
                g[M + i] = std::exp(-(kv * kv) * (rs * rs)) / (sc * sc * sc * sc);
            }
        }
        TPM_HIP(c, hipMemcpyAsync(c->twiddle.p, tw.data(), tw.size() * sizeof(Cx<T>),
                                  hipMemcpyHostToDevice, st));
        TPM_HIP(c, hipMemcpyAsync(c->green_axis.p, g.data(), g.size() * sizeof(double),
                                  hipMemcpyHostToDevice, st));
        // host vectors die at scope end: wait for the copies
        TPM_HIP(c, hipStreamSynchronize(st));
        c->axis_tables_M = M;
    }
    unsigned long long *mq = (unsigned long long *)c->mesh_q.p;
    TPM_TRY(timer_begin(c, TPM_TIMER_DEPOSIT));
    TPM_TRY(fill_u64(c, (uint64_t *)mq, 0ull, (int64_t)(planes * n3)));
    k_deposit<kTwo><<<grid_for(c->n, kDepChunk), kBlock, 0, st>>>(
        (const double *)c->ps.p, (const double *)c->ms.p, c->n, (const Rec64 *)c->rec64.p, mg,
        mq, kTwo ? n3 : 0);
    TPM_LAUNCHED(c, "k_deposit");
    TPM_TRY(timer_end(c, TPM_TIMER_DEPOSIT));
    FftArgs fa;
    fa.rec = (const Rec64 *)c->rec64.p;
    fa.plane = kTwo ? n3 : 0;
    fa.norm = 1.0 / (double)n3;
    if (iso) {
        // masses on the mesh, Phi = IFFT(FFT(M) T) (G / h) / M^3
        fa.gtab = (const double *)c->green_tab.p;
        fa.gconst = P.G / mg.h;
        fa.vinv = 1.0;
    } else {
        fa.gk2 = (const double *)c->green_axis.p;
        fa.gq = fa.gk2 + M;
        fa.gconst = -4.0 * M_PI * P.G;
        fa.vinv = 1.0 / (mg.h * mg.h * mg.h);
    }
    Cx<T> *mc = (Cx<T> *)c->mesh_c.p;
    T *phi = (T *)c->mesh_phi.p;
    const Cx<T> *tw = (const Cx<T> *)c->twiddle.p;
    const FftPass passes[5] = {{2, 1, 0, 0, 0, 1}, {1, 0, 0, 0, 0, 1}, {0, 0, 0, 0, 1, 1},
                               {1, 0, 0, 1, 0, 1}, {2, 0, 1, 1, 0, 1}};
    TPM_TRY(timer_begin(c, TPM_TIMER_FFT));
    for (const FftPass &fp : passes)
        TPM_TRY(fft_pass<T>(c, M, fp, mc, mq, phi, tw, fa));
    return timer_end(c, TPM_TIMER_FFT);
}

template <typename T>
int interp_t(tpm_ctx *c, int64_t n_act, const int32_t *idx, void *acc, void *pot) {
    const int64_t n = c->n;
    const MeshGeom mg = mesh_geom(c);
    TPM_TRY(ensure(c, c->res, (size_t)4 * n * sizeof(T)));
    TPM_TRY(ensure(c, c->rpot, (size_t)n * sizeof(T)));
    TPM_TRY(select_active(c, n_act, idx));
    const unsigned g = grid_for(std::min<int64_t>(n_act, n), kBlock);
    k_interp<T><<<g, kBlock, 0, c->stream>>>(
        (const uint32_t *)c->act.p, (const uint32_t *)c->counters.p + 40, n,
        (const double *)c->ps.p, (const T *)c->mesh_phi.p, mg, (T *)c->res.p, (T *)c->rpot.p);
    TPM_LAUNCHED(c, "k_interp");
    k_scatter_out<T><<<grid_for(n_act, kBlock), kBlock, 0, c->stream>>>(
        idx, n_act, n, (const int32_t *)c->rank.p, (const uint32_t *)c->slot.p,
        (const uint32_t *)c->counters.p + 40, (const T *)c->res.p, (const T *)c->rpot.p,
        (T *)acc, (T *)pot,
        (uint32_t *)c->err_flag.p);
    TPM_LAUNCHED(c, "k_scatter_out");
    return TPM_OK;
}

template <typename T>
int export_t(tpm_ctx *c, double *rho, double *phi) {
    const MeshGeom mg = mesh_geom(c);
    const size_t M = (size_t)mg.ng, n3 = M * M * M;
    constexpr bool kTwo = sizeof(T) == sizeof(double);
    TPM_HIP(c, hipStreamSynchronize(c->stream));
    if (rho) {
        Rec64 root;
        TPM_HIP(c, hipMemcpy(&root, c->rec64.p, sizeof(Rec64), hipMemcpyDeviceToHost));
        int ex;
        std::frexp(root.mass, &ex);
        const double vinv = c->P.periodic ? 1.0 / (mg.h * mg.h * mg.h) : 1.0;
        const double qscale = std::ldexp(1.0, ex - 62) * vinv;
        std::vector<unsigned long long> q((kTwo ? 2 : 1) * n3);
        TPM_HIP(c, hipMemcpy(q.data(), c->mesh_q.p, q.size() * 8, hipMemcpyDeviceToHost));
        for (size_t g = 0; g < n3; g++) {
            const double hi = (double)q[g];
            const double v = kTwo ? std::fma((double)(long long)q[n3 + g], 0x1p-20, hi) : hi;
            rho[g] = v * qscale;
        }
    }
    if (phi) {
        std::vector<T> f(n3);
        TPM_HIP(c, hipMemcpy(f.data(), c->mesh_phi.p, n3 * sizeof(T), hipMemcpyDeviceToHost));
        for (size_t g = 0; g < n3; g++)
            phi[g] = (double)f[g];
    }
    return TPM_OK;
}

}  // namespace

// Mesh geometry of the current build: periodic box of ng cells, or the
// isolated ng-cell mesh of spacing L_root / (ng - 4) starting two cells
// below the root cube, zero-padded to (2 ng)^3.
MeshGeom pmk::mesh_geom(const tpm_ctx *c) {
    const tpm_params &P = c->P;
    MeshGeom g{};
    if (P.periodic) {
        g.box = P.box_size;
        g.h = P.box_size / P.pm_grid;
        g.ng = P.pm_grid;
    } else {
        g.box = 0.0;
        g.h = c->frame_host.L / (P.pm_grid - 4);
        for (int a = 0; a < 3; a++)
            g.lo[a] = c->frame_host.x0[a] - 2.0 * g.h;
        g.ng = 2 * P.pm_grid;
    }
    return g;
}

int pm_export(tpm_ctx *c, double *rho, double *phi) {
    if (c->P.precision == TPM_FP32)
        return export_t<float>(c, rho, phi);
    return export_t<double>(c, rho, phi);
}

int pm_solve(tpm_ctx *c) {
    if (c->P.precision == TPM_FP32)
        return solve_t<float>(c);
    return solve_t<double>(c);
}

int pm_interp(tpm_ctx *c, int64_t n_act, const int32_t *idx, void *acc, void *pot) {
    if (n_act == 0)
        return TPM_OK;
    // the interpolation yields the potential anyway: written whenever the
    // caller passes a buffer, whatever want_potential says (that flag prices
    // the tree walk's potential)
    if (c->P.precision == TPM_FP32)
        return interp_t<float>(c, n_act, idx, acc, pot);
    return interp_t<double>(c, n_act, idx, acc, pot);
}

}  // namespace tpm
