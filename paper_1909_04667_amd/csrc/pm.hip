// Particle-mesh long-range force for gfx950 (Sec. 3.3 and 3.4 of the Arepo
// paper): CIC deposit, FFT Poisson solve with the Gaussian long-range filter
// exp(-k^2 rs^2) and CIC deconvolution, four-point finite differences, CIC
// interpolation.  Mean density removed (k = 0 set to zero, Sec. 2.2).
//
// Layout: mesh index (i * ng + j) * ng + k, i <-> x.  The deposit accumulates
// 62-bit fixed-point masses with integer atomics, so the mesh is independent
// of particle order (deterministic).  The 3-D FFT runs as five passes over
// the complex mesh: forward z (reading the fixed-point mesh), forward y,
// [forward x, Green's function, inverse x] fused in LDS, inverse y, inverse z
// (writing the real potential).  Each pass loads a block of lines into LDS
// (coalesced along the contiguous axis) and runs a radix-2 Stockham FFT.
// The gradient is taken inside the interpolation kernel from the potential.
#include "tpm_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace tpm {
namespace {

constexpr int kBlock = 256;
constexpr size_t kFftLds = 64 * 1024;  // two ping-pong buffers per block

template <typename T>
struct Cx {
    T re, im;
};

__global__ __launch_bounds__(kBlock) void k_deposit(const double *__restrict__ ps,
                                                    const double *__restrict__ ms, int64_t n,
                                                    const Rec64 *__restrict__ rec, double box,
                                                    double h, int ng,
                                                    unsigned long long *__restrict__ mesh) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = s < n;
    const int lane = threadIdx.x & 63;
    const uint64_t le = ~0ull >> (63 - lane);  // lanes 0..lane
    int ex;
    frexp(rec[0].mass, &ex);  // total mass < 2^ex
    const double scale = ldexp(1.0, 62 - ex);
    int i0[3] = {0, 0, 0};
    double w[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double u = live ? ps[(size_t)a * n + s] : 0.0;
        if (u < 0.0)
            u += box;
        if (u >= box)
            u -= box;
        const double f = u / h;
        const double fl = floor(f);
        w[a] = f - fl;
        // any input (even outside the box or NaN) stays on the mesh
        int i = (int)fmin(fmax(fl, -1.0e9), 1.0e9) % ng;
        if (i < 0)
            i += ng;
        i0[a] = i;
    }
    const double m = live ? ms[s] : 0.0;
    // Particles are in curve order, so neighbouring lanes often hit the same
    // cells: sum equal cells across the wavefront first (integers, so the
    // result does not depend on the grouping) and issue one atomic per run.
#pragma unroll
    for (int c = 0; c < 8; c++) {
        double wt = 1.0;
        int t[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const int up = (c >> (2 - a)) & 1;
            wt *= up ? w[a] : 1.0 - w[a];
            t[a] = up ? (i0[a] + 1 == ng ? 0 : i0[a] + 1) : i0[a];
        }
        const uint32_t cell =
            live ? (uint32_t)(((size_t)t[0] * ng + t[1]) * ng + t[2]) : 0xffffffffu;
        unsigned long long q = live ? __double2ull_rn(m * wt * scale) : 0ull;
        const uint32_t prev = __shfl_up(cell, 1, 64);
        const bool head = lane == 0 || prev != cell;
        const uint64_t heads = __ballot(head);
        const uint32_t seg = (uint32_t)__popcll(heads & le);  // run id of this lane
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {  // suffix sums within each run
            const unsigned long long oq = __shfl_down(q, off, 64);
            const uint32_t os = __shfl_down(seg, off, 64);
            if (lane + off < 64 && os == seg)
                q += oq;
        }
        if (live && head)
            atomicAdd(&mesh[cell], q);
    }
}

// One 1-D transform direction over a block of B lines held in LDS.
template <typename T>
__device__ __forceinline__ Cx<T> *stockham(Cx<T> *x, Cx<T> *y, int B, int ng, int logn,
                                           const Cx<T> *__restrict__ tw, bool inverse) {
    const int half = ng >> 1;
    int s = 1;
    for (int st = 0; st < logn; st++) {
        const int m = half / s;  // n/2 at this stage
        for (int id = threadIdx.x; id < B * half; id += kBlock) {
            const int b = id / half;
            const int j = id - b * half;
            const int p = j / s, q = j - p * s;
            const Cx<T> *xb = x + b * ng;
            Cx<T> *yb = y + b * ng;
            const Cx<T> a = xb[q + s * p];
            const Cx<T> c = xb[q + s * (p + m)];
            Cx<T> w = tw[p * s];
            if (inverse)
                w.im = -w.im;
            const T dr = a.re - c.re, di = a.im - c.im;
            yb[q + 2 * s * p] = Cx<T>{a.re + c.re, a.im + c.im};
            yb[q + 2 * s * p + s] = Cx<T>{dr * w.re - di * w.im, dr * w.im + di * w.re};
        }
        __syncthreads();
        Cx<T> *t = x;
        x = y;
        y = t;
        s <<= 1;
    }
    return x;
}

struct FftPass {
    int axis;        // 0: x (stride ng^2), 1: y (stride ng), 2: z (contiguous)
    int in_fixed;    // read the fixed-point deposit (axis 2, forward only)
    int out_real;    // write the scaled real part (axis 2, inverse only)
    int inverse;
    int green;       // forward, multiply by the Green's function, inverse
};

// Per-axis tables for the Green's function: k_a^2 and sinc^4(k_a h / 2).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fft(FftPass ps, int ng, int logn, int B,
                                                Cx<T> *__restrict__ mesh,
                                                const unsigned long long *__restrict__ mq,
                                                T *__restrict__ phi, const Cx<T> *__restrict__ tw,
                                                const double *__restrict__ gk2,
                                                const double *__restrict__ gdc, double gconst,
                                                double rs, const Rec64 *__restrict__ rec,
                                                double vinv, double norm) {
    extern __shared__ unsigned char lds_raw[];
    Cx<T> *buf0 = (Cx<T> *)lds_raw;
    Cx<T> *buf1 = buf0 + (size_t)B * ng;
    const size_t ng2 = (size_t)ng * ng;
    // line base offsets and element stride
    size_t base0;
    size_t stride;
    int lines_contig;  // 1: lines are contiguous (axis z)
    if (ps.axis == 2) {
        base0 = (size_t)blockIdx.x * B * ng;
        stride = 1;
        lines_contig = 1;
    } else {
        const int per = ng / B;
        const size_t outer = blockIdx.x / per, kb = blockIdx.x % per;
        if (ps.axis == 1)
            base0 = outer * ng2 + kb * B;
        else
            base0 = outer * ng + kb * B;
        stride = ps.axis == 1 ? (size_t)ng : ng2;
        lines_contig = 0;
    }
    double qscale = 0.0;
    if (ps.in_fixed) {
        int ex;
        frexp(rec[0].mass, &ex);
        qscale = ldexp(1.0, ex - 62) * vinv;
    }
    const int total = B * ng;
    for (int id = threadIdx.x; id < total; id += kBlock) {
        int b, k;
        size_t g;
        if (lines_contig) {
            b = id / ng;
            k = id - b * ng;
            g = base0 + (size_t)b * ng + k;
        } else {
            k = id / B;
            b = id - k * B;
            g = base0 + b + (size_t)k * stride;
        }
        Cx<T> v;
        if (ps.in_fixed) {
            v.re = (T)((double)mq[g] * qscale);
            v.im = (T)0;
        } else {
            v = mesh[g];
        }
        buf0[b * ng + k] = v;
    }
    __syncthreads();
    Cx<T> *res = stockham<T>(buf0, buf1, B, ng, logn, tw, ps.inverse && !ps.green);
    if (ps.green) {
        // x lines: the block fixes (j, k) = (outer, kb * B + b); i runs along the line
        const int per = ng / B;
        const int j = blockIdx.x / per, kb = blockIdx.x % per;
        for (int id = threadIdx.x; id < total; id += kBlock) {
            const int b = id / ng, i = id - b * ng;
            const int k = kb * B + b;
            const double k2 = (gk2[i] + gk2[j]) + gk2[k];
            const double dc = (gdc[i] * gdc[j]) * gdc[k];
            double g = 0.0;
            if (k2 != 0.0)
                g = gconst * exp(-k2 * rs * rs) / (k2 * dc);
            Cx<T> v = res[b * ng + i];
            v.re = (T)(v.re * g);
            v.im = (T)(v.im * g);
            res[b * ng + i] = v;
        }
        __syncthreads();
        Cx<T> *other = (res == buf0) ? buf1 : buf0;
        res = stockham<T>(res, other, B, ng, logn, tw, true);
    }
    for (int id = threadIdx.x; id < total; id += kBlock) {
        int b, k;
        size_t g;
        if (lines_contig) {
            b = id / ng;
            k = id - b * ng;
            g = base0 + (size_t)b * ng + k;
        } else {
            k = id / B;
            b = id - k * B;
            g = base0 + b + (size_t)k * stride;
        }
        const Cx<T> v = res[b * ng + k];
        if (ps.out_real)
            phi[g] = (T)(v.re * norm);
        else
            mesh[g] = v;
    }
}

// Fused four-point difference and CIC interpolation, over the active slots
// in curve order (neighbouring threads read neighbouring mesh cells); the
// results go to slot order and are scattered to caller order afterwards.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_interp(const uint32_t *__restrict__ act,
                                                   const uint32_t *__restrict__ nuniq,
                                                   int64_t n, const double *__restrict__ ps,
                                                   const T *__restrict__ phi, int ng, double box,
                                                   double h, T *__restrict__ res,
                                                   T *__restrict__ rpot) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= (int64_t)*nuniq)
        return;
    const int64_t s = act[k];
    int i0[3];
    double w[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        double u = ps[(size_t)a * n + s];
        if (u < 0.0)
            u += box;
        if (u >= box)
            u -= box;
        const double f = u / h;
        const double fl = floor(f);
        w[a] = f - fl;
        // any input (even outside the box or NaN) stays on the mesh
        int i = (int)fmin(fmax(fl, -1.0e9), 1.0e9) % ng;
        if (i < 0)
            i += ng;
        i0[a] = i;
    }
    const int mask = ng - 1;
    auto at = [&](int x, int y, int z) -> double {
        return (double)phi[((size_t)(x & mask) * ng + (y & mask)) * ng + (z & mask)];
    };
    double F[3] = {0.0, 0.0, 0.0}, P = 0.0;
#pragma unroll
    for (int c = 0; c < 8; c++) {
        double wt = 1.0;
        int t[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const int up = (c >> (2 - a)) & 1;
            wt *= up ? w[a] : 1.0 - w[a];
            t[a] = i0[a] + up;
        }
        // -grad Phi at mesh point t
        {
            const double g = ((2.0 / 3.0) * (at(t[0] + 1, t[1], t[2]) - at(t[0] - 1, t[1], t[2])) -
                              (1.0 / 12.0) * (at(t[0] + 2, t[1], t[2]) - at(t[0] - 2, t[1], t[2]))) /
                             h;
            F[0] += wt * -g;
        }
        {
            const double g = ((2.0 / 3.0) * (at(t[0], t[1] + 1, t[2]) - at(t[0], t[1] - 1, t[2])) -
                              (1.0 / 12.0) * (at(t[0], t[1] + 2, t[2]) - at(t[0], t[1] - 2, t[2]))) /
                             h;
            F[1] += wt * -g;
        }
        {
            const double g = ((2.0 / 3.0) * (at(t[0], t[1], t[2] + 1) - at(t[0], t[1], t[2] - 1)) -
                              (1.0 / 12.0) * (at(t[0], t[1], t[2] + 2) - at(t[0], t[1], t[2] - 2))) /
                             h;
            F[2] += wt * -g;
        }
        P += wt * at(t[0], t[1], t[2]);
    }
    res[k] = (T)F[0];
    res[n + k] = (T)F[1];
    res[2 * n + k] = (T)F[2];
    rpot[k] = (T)P;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_out(
    const int32_t *__restrict__ idx, int64_t n_act, int64_t n, const int32_t *__restrict__ rank,
    const uint32_t *__restrict__ slot, const T *__restrict__ res, const T *__restrict__ rpot,
    T *__restrict__ acc, T *__restrict__ pot, uint32_t *__restrict__ err) {
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
    const uint32_t sl = slot[rank[i]];
    acc[k] = res[sl];
    acc[n_act + k] = res[n + sl];
    acc[2 * n_act + k] = res[2 * n + sl];
    if (pot)
        pot[k] = rpot[sl];
}

template <typename T>
int solve_t(tpm_ctx *c) {
    const tpm_params &P = c->P;
    const int ng = P.pm_grid;
    int logn = 0;
    while ((1 << logn) < ng)
        logn++;
    const size_t n3 = (size_t)ng * ng * ng;
    hipStream_t st = c->stream;
    TPM_TRY(ensure(c, c->mesh_q, n3 * 8));
    TPM_TRY(ensure(c, c->mesh_c, n3 * sizeof(Cx<T>)));
    TPM_TRY(ensure(c, c->mesh_phi, n3 * sizeof(T)));
    TPM_TRY(ensure(c, c->twiddle, (size_t)ng / 2 * sizeof(Cx<T>) + 64));
    TPM_TRY(ensure(c, c->green_axis, (size_t)2 * ng * sizeof(double)));
    // tables, computed in double on the host
    {
        std::vector<Cx<T>> tw(ng / 2);
        for (int k = 0; k < ng / 2; k++) {
            const double a = 2.0 * M_PI * k / ng;
            tw[k] = Cx<T>{(T)std::cos(a), (T)-std::sin(a)};
        }
        const double box = P.box_size, h = box / ng;
        std::vector<double> g(2 * ng);
        for (int i = 0; i < ng; i++) {
            const int nn = i < ng / 2 ? i : i - ng;
            const double kv = 2.0 * M_PI * nn / box;
            const double s = 0.5 * kv * h;
            const double sc = nn == 0 ? 1.0 : std::sin(s) / s;
            g[i] = kv * kv;
            g[ng + i] = sc * sc * sc * sc;
        }
        TPM_HIP(c, hipMemcpyAsync(c->twiddle.p, tw.data(), tw.size() * sizeof(Cx<T>),
                                  hipMemcpyHostToDevice, st));
        TPM_HIP(c, hipMemcpyAsync(c->green_axis.p, g.data(), g.size() * sizeof(double),
                                  hipMemcpyHostToDevice, st));
        // host vectors die at scope end: wait for the copies
        TPM_HIP(c, hipStreamSynchronize(st));
    }
    unsigned long long *mq = (unsigned long long *)c->mesh_q.p;
    TPM_TRY(fill_u64(c, (uint64_t *)mq, 0ull, (int64_t)n3));
    const double box = P.box_size, h = box / ng;
    k_deposit<<<grid_for(c->n, kBlock), kBlock, 0, st>>>(
        (const double *)c->ps.p, (const double *)c->ms.p, c->n, (const Rec64 *)c->rec64.p, box, h,
        ng, mq);
    TPM_LAUNCHED(c, "k_deposit");
    int B = (int)(kFftLds / (2 * (size_t)ng * sizeof(Cx<T>)));
    if (B > ng)
        B = ng;
    if (B < 1)
        return fail(c, TPM_EINVAL, "pm_grid too large for the LDS line block");
    const size_t lds = 2 * (size_t)B * ng * sizeof(Cx<T>);
    const unsigned blocks = (unsigned)((size_t)ng * ng / B);
    const double *gk2 = (const double *)c->green_axis.p;
    const double *gdc = gk2 + ng;
    const double gconst = -4.0 * M_PI * P.G;
    const double rs = P.asmth * P.box_size / P.pm_grid;
    const double vinv = 1.0 / (h * h * h);
    const double norm = 1.0 / (double)n3;
    Cx<T> *mc = (Cx<T> *)c->mesh_c.p;
    T *phi = (T *)c->mesh_phi.p;
    const Cx<T> *tw = (const Cx<T> *)c->twiddle.p;
    const Rec64 *rec = (const Rec64 *)c->rec64.p;
    const FftPass passes[5] = {
        {2, 1, 0, 0, 0}, {1, 0, 0, 0, 0}, {0, 0, 0, 0, 1}, {1, 0, 0, 1, 0}, {2, 0, 1, 1, 0}};
    for (const FftPass &fp : passes) {
        k_fft<T><<<blocks, kBlock, lds, st>>>(fp, ng, logn, B, mc, mq, phi, tw, gk2, gdc, gconst,
                                              rs, rec, vinv, norm);
        TPM_LAUNCHED(c, "k_fft");
    }
    return TPM_OK;
}

template <typename T>
int interp_t(tpm_ctx *c, int64_t n_act, const int32_t *idx, void *acc, void *pot) {
    const tpm_params &P = c->P;
    const int ng = P.pm_grid;
    const int64_t n = c->n;
    const double box = P.box_size, h = box / ng;
    TPM_TRY(ensure(c, c->res, (size_t)3 * n * sizeof(T)));
    TPM_TRY(ensure(c, c->rpot, (size_t)n * sizeof(T)));
    TPM_TRY(select_active(c, n_act, idx));
    const unsigned g = grid_for(std::min<int64_t>(n_act, n), kBlock);
    k_interp<T><<<g, kBlock, 0, c->stream>>>(
        (const uint32_t *)c->act.p, (const uint32_t *)c->counters.p + 40, n,
        (const double *)c->ps.p, (const T *)c->mesh_phi.p, ng, box, h, (T *)c->res.p,
        (T *)c->rpot.p);
    TPM_LAUNCHED(c, "k_interp");
    k_scatter_out<T><<<grid_for(n_act, kBlock), kBlock, 0, c->stream>>>(
        idx, n_act, n, (const int32_t *)c->rank.p, (const uint32_t *)c->slot.p,
        (const T *)c->res.p, (const T *)c->rpot.p, (T *)acc, (T *)pot,
        (uint32_t *)c->err_flag.p);
    TPM_LAUNCHED(c, "k_scatter_out");
    return TPM_OK;
}

}  // namespace

int pm_solve(tpm_ctx *c) {
    if (c->P.precision == TPM_FP32)
        return solve_t<float>(c);
    return solve_t<double>(c);
}

int pm_interp(tpm_ctx *c, int64_t n_act, const int32_t *idx, void *acc, void *pot) {
    if (n_act == 0)
        return TPM_OK;
    void *p = (pot && c->P.want_potential) ? pot : nullptr;
    if (c->P.precision == TPM_FP32)
        return interp_t<float>(c, n_act, idx, acc, p);
    return interp_t<double>(c, n_act, idx, acc, p);
}

}  // namespace tpm
