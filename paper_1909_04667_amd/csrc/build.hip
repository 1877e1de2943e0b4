// Tree build for gfx950 (Sec. 3.1 of the Arepo paper: enclosing cube, a tree
// rebuilt for every force computation, monopole moments; Sec. 8: Peano-
// Hilbert ordering).
//
// Instead of inserting particles one by one, the tree is derived from the
// sorted 63-bit keys: a node is a key prefix shared by at least two particles,
// which is exactly the tree sequential insertion produces.  Every particle
// starts the nodes whose prefix level lies between its common-prefix depths
// with its left and right neighbours, so one scan over per-particle counts
// gives the depth-first position of every entry, and skip pointers (end of a
// subtree) come from a galloping search for the end of each prefix run.
#include "tpm_internal.h"

#include <vector>

namespace tpm {
namespace {

constexpr int kBlock = 256;

// ---- root cube -------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_bbox_partial(const double *__restrict__ x,
                                                         const double *__restrict__ y,
                                                         const double *__restrict__ z,
                                                         int64_t n, double *__restrict__ part) {
    __shared__ double s[6][kBlock];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const double *c[3] = {x, y, z};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            double v = c[a][i];
            lo[a] = fmin(lo[a], v);
            hi[a] = fmax(hi[a], v);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; a++) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
#pragma unroll
            for (int a = 0; a < 3; a++) {
                s[a][threadIdx.x] = fmin(s[a][threadIdx.x], s[a][threadIdx.x + w]);
                s[3 + a][threadIdx.x] = fmax(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + w]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6)
        part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// Smallest power of two >= ext (1 + 2^-20) (1 when every particle coincides);
// the corner sits below the minimum by a fraction shift of the slack.
__global__ __launch_bounds__(kBlock) void k_frame_final(const double *__restrict__ part,
                                                        int nparts, Frame *F, double s0,
                                                        double s1, double s2) {
    // min/max of the block partials: strided over the threads, then a tree in
    // LDS (both exact, so the order does not matter)
    __shared__ double sh[6][kBlock];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nparts; b += kBlock)
        for (int a = 0; a < 3; a++) {
            lo[a] = fmin(lo[a], part[b * 6 + a]);
            hi[a] = fmax(hi[a], part[b * 6 + 3 + a]);
        }
    for (int a = 0; a < 3; a++) {
        sh[a][threadIdx.x] = lo[a];
        sh[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int a = 0; a < 3; a++) {
                sh[a][threadIdx.x] = fmin(sh[a][threadIdx.x], sh[a][threadIdx.x + w]);
                sh[3 + a][threadIdx.x] = fmax(sh[3 + a][threadIdx.x], sh[3 + a][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x != 0)
        return;
    for (int a = 0; a < 3; a++) {
        lo[a] = sh[a][0];
        hi[a] = sh[3 + a][0];
    }
    double ext = 0.0;
    for (int a = 0; a < 3; a++) {
        double e = hi[a] - lo[a];
        ext = e > ext ? e : ext;
    }
    double L = 1.0;
    if (ext > 0.0) {
        double t = ext * (1.0 + 0x1p-20);
        int ex;
        double m = frexp(t, &ex);
        L = (m == 0.5) ? ldexp(1.0, ex - 1) : ldexp(1.0, ex);
    }
    const double shift[3] = {s0, s1, s2};
    for (int a = 0; a < 3; a++)
        F->x0[a] = lo[a] - shift[a] * (L - (hi[a] - lo[a]));
    F->L = L;
    F->S = 2097152.0 / L;
    F->box = 0.0;
    F->periodic = 0;
}

// ---- keys ------------------------------------------------------------------

// Tree-frame coordinate and 21-bit cell index of one coordinate value.
__device__ __forceinline__ void to_frame(double xv, double x0, const Frame &F, double &p,
                                         uint32_t &q) {
    p = xv;
    double u = p - x0;
    if (F.periodic) {
        if (u >= F.L) {
            p = xv - F.L;
            u = p - x0;
        } else if (u < 0.0) {
            p = xv + F.L;
            u = p - x0;
        }
    }
    double f = floor(u * F.S);
    f = fmax(f, 0.0);
    f = fmin(f, 2097151.0);
    q = (uint32_t)f;
}

// Spread the low 21 bits of v to every third bit.
__device__ __forceinline__ uint64_t dilate3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Peano-Hilbert index of a 21-bit cell (Skilling 2004, transpose form),
// branch-free: each level either inverts the low bits of axis 0 or exchanges
// them with the axis whose bit is clear; the closing Gray-code correction is
// a suffix parity computed with shifts.
__device__ __forceinline__ uint64_t hilbert_key(uint32_t a0, uint32_t a1, uint32_t a2) {
    uint32_t X0 = a0, X1 = a1, X2 = a2;
#pragma unroll
    for (int b = kBits - 1; b >= 1; --b) {
        const uint32_t P = (1u << b) - 1u;
        const uint32_t m0 = 0u - ((X0 >> b) & 1u);
        X0 ^= P & m0;
        const uint32_t m1 = 0u - ((X1 >> b) & 1u);
        const uint32_t t1 = (X0 ^ X1) & P & ~m1;
        X0 ^= (P & m1) | t1;
        X1 ^= t1;
        const uint32_t m2 = 0u - ((X2 >> b) & 1u);
        const uint32_t t2 = (X0 ^ X2) & P & ~m2;
        X0 ^= (P & m2) | t2;
        X2 ^= t2;
    }
    X1 ^= X0;
    X2 ^= X1;
    uint32_t z = X2;  // z_j = parity of bits >= j of X2
    z ^= z >> 1;
    z ^= z >> 2;
    z ^= z >> 4;
    z ^= z >> 8;
    z ^= z >> 16;
    const uint32_t t = z >> 1;
    X0 ^= t;
    X1 ^= t;
    X2 ^= t;
    return (dilate3(X0) << 2) | (dilate3(X1) << 1) | dilate3(X2);
}

// Keys, and the caller's position and mass of each particle packed into one
// 32-byte record (caller order), so that the gather into curve order reads
// one record per particle instead of four scattered values.
__global__ __launch_bounds__(kBlock) void k_keys(const double *__restrict__ x,
                                                 const double *__restrict__ y,
                                                 const double *__restrict__ z,
                                                 const double *__restrict__ mass, int64_t n,
                                                 const Frame *__restrict__ Fp,
                                                 uint64_t *__restrict__ key,
                                                 uint32_t *__restrict__ idx,
                                                 double4 *__restrict__ xyzm) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n)
        return;
    const Frame F = *Fp;
    const double xi = x[i], yi = y[i], zi = z[i];
    double p;
    uint32_t q0, q1, q2;
    to_frame(xi, F.x0[0], F, p, q0);
    to_frame(yi, F.x0[1], F, p, q1);
    to_frame(zi, F.x0[2], F, p, q2);
    key[i] = hilbert_key(q0, q1, q2);
    idx[i] = (uint32_t)i;
    xyzm[i] = make_double4(xi, yi, zi, mass ? mass[i] : 1.0 / (double)n);
}

// ---- gather into curve order -------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_gather(
    const double4 *__restrict__ xyzm, int64_t n, const Frame *__restrict__ Fp,
    const uint32_t *__restrict__ sidx, int32_t *__restrict__ perm, int32_t *__restrict__ rank,
    double *__restrict__ ps, double *__restrict__ ms, uint64_t *__restrict__ qs,
    const double *__restrict__ eps, double *__restrict__ hs, uint32_t *__restrict__ bad_eps) {
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n)
        return;
    const Frame F = *Fp;
    const uint32_t i = sidx[s];
    perm[s] = (int32_t)i;
    rank[i] = (int32_t)s;
    const double4 r = xyzm[i];
    double p0, p1, p2;
    uint32_t q0, q1, q2;
    to_frame(r.x, F.x0[0], F, p0, q0);
    to_frame(r.y, F.x0[1], F, p1, q1);
    to_frame(r.z, F.x0[2], F, p2, q2);
    ps[s] = p0;
    ps[n + s] = p1;
    ps[2 * n + s] = p2;
    ms[s] = r.w;
    qs[s] = ((uint64_t)q0 << 42) | ((uint64_t)q1 << 21) | (uint64_t)q2;
    if (eps) {  // individual softening: spline support 2.8 eps, in curve order
        const double e = eps[i];
        if (!(e > 0.0) || !isfinite(e))
            atomicOr(bad_eps, 1u);
        hs[s] = 2.8 * e;
    }
}

// ---- topology ----------------------------------------------------------------

// Number of leading 3-bit groups two keys share (0..21).
__device__ __forceinline__ int common_levels(uint64_t a, uint64_t b) {
    uint64_t d = a ^ b;
    if (d == 0)
        return kMaxLevel;
    int top = 63 - __clzll((long long)d);
    return (kMaxLevel - 1) - top / 3;
}

// Per particle: depth shared with the right neighbour, entries it starts
// (nodes at levels (dL, dR] plus itself), and per block and level the number
// of nodes its particles start: hist[level * nb + block] (a counting sort by
// level, so node lists come out in particle order without global atomics).
__global__ __launch_bounds__(kBlock) void k_count(const uint64_t *__restrict__ key, int64_t n,
                                                  int8_t *__restrict__ dR,
                                                  uint32_t *__restrict__ cnt,
                                                  uint32_t *__restrict__ hist, uint32_t nb) {
    __shared__ uint32_t h[kLevels][kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int r = -1, l = -1;
    if (s < n) {
        const uint64_t k = key[s];
        r = (s + 1 < n) ? common_levels(k, key[s + 1]) : -1;
        l = (s > 0) ? common_levels(key[s - 1], k) : -1;
        dR[s] = (int8_t)r;
        const int nn = r > l ? r - l : 0;
        cnt[s] = (uint32_t)nn + 1u;
    }
    for (int lev = 0; lev < kLevels; lev++) {
        const uint64_t m = __ballot(lev > l && lev <= r);
        if (lane == 0)
            h[lev][w] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (threadIdx.x < kLevels) {
        uint32_t t = 0;
#pragma unroll
        for (int q = 0; q < kBlock / 64; q++)
            t += h[threadIdx.x][q];
        hist[(size_t)threadIdx.x * nb + blockIdx.x] = t;
    }
}

// Start offset of every level's node list (the scanned histogram's first
// block) into out[0..21].
__global__ void k_level_starts(const uint32_t *__restrict__ off, uint32_t nb,
                               uint32_t *__restrict__ out) {
    if (threadIdx.x < kLevels)
        out[threadIdx.x] = off[(size_t)threadIdx.x * nb];
}

__device__ __forceinline__ uint64_t prefix_at(uint64_t k, int lev) {
    return k >> (3 * (kMaxLevel - lev));
}

// FP32 record of an entry: exact integer centre of its cell at level lev
// (units of L 2^-22, shifted left by sh so that 32-bit differences wrap
// modulo a periodic box), level and particle flag in the freed low bits of x.
__device__ __forceinline__ void rec32_centre(Rec32 &o, const uint32_t q[3], int lev, int sh,
                                             bool part) {
    int32_t C[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const uint32_t P = q[a] >> (kBits - lev);
        C[a] = (int32_t)(((2u * P + 1u) << (kBits - lev)));
    }
    o.cx_meta = (int32_t)((uint32_t)C[0] << sh) | lev | (part ? kRecParticle : 0);
    o.cy = (int32_t)((uint32_t)C[1] << sh);
    o.cz = (int32_t)((uint32_t)C[2] << sh);
}

// Emit the particle entry and the node entries a particle starts.  Skip
// pointers and counts of nodes are filled bottom-up by k_moments: every
// entry carries a depth (nodes: their level; a particle: the level of the
// cell it occupies alone, one below its deepest shared prefix), and the
// subtree of a node of level l ends at the first later entry of depth <= l.
// FP32 contexts (out32 set): a particle's FP32 record is written here, a
// node's by k_moments.
__global__ __launch_bounds__(kBlock) void k_emit(
    const uint64_t *__restrict__ key, int64_t n, const int8_t *__restrict__ dR,
    const uint32_t *__restrict__ base, const Frame *__restrict__ Fp,
    const double *__restrict__ ps, const double *__restrict__ ms,
    const uint64_t *__restrict__ qs, Rec64 *__restrict__ rec, uint32_t *__restrict__ efirst,
    uint32_t *__restrict__ ecount, uint32_t *__restrict__ pe,
    const uint32_t *__restrict__ loff, uint32_t nb, uint32_t *__restrict__ lvl_list,
    const double *__restrict__ hs, double *__restrict__ eh, double G, Rec32 *__restrict__ out32,
    float *__restrict__ eh32) {
    __shared__ uint32_t h[kLevels][kBlock / 64];
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool live = s < n;
    const int r = live ? (int)dR[s] : -1;
    const int l = (live && s > 0) ? (int)dR[s - 1] : -1;
    const uint32_t b = live ? base[s] : 0u;
    const int nn = r > l ? r - l : 0;
    // level lists in particle order: block offset (scanned histogram) +
    // preceding wavefronts of the block + preceding lanes of the wavefront
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int lev = 0; lev < kLevels; lev++) {
        const uint64_t m = __ballot(lev > l && lev <= r);
        if (lane == 0)
            h[lev][w] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    for (int lev = 0; lev < kLevels; lev++) {
        const bool has = lev > l && lev <= r;
        const uint64_t m = __ballot(has);
        if (has) {
            uint32_t at = loff[(size_t)lev * nb + blockIdx.x];
            for (int q = 0; q < w; q++)
                at += h[lev][q];
            lvl_list[at + (uint32_t)__popcll(m & lt)] = b + (uint32_t)(lev - l - 1);
        }
    }
    if (!live)
        return;
    const Frame F = *Fp;
    const uint32_t ep = b + (uint32_t)nn;
    const int sh = F.periodic ? kRecShiftPer : kRecShiftIso;
    const uint64_t qq = qs[s];
    const uint32_t q[3] = {(uint32_t)(qq >> 42) & 0x1fffffu, (uint32_t)(qq >> 21) & 0x1fffffu,
                           (uint32_t)qq & 0x1fffffu};
    {
        Rec64 R;
        R.com[0] = ps[s];
        R.com[1] = ps[n + s];
        R.com[2] = ps[2 * n + s];
        R.mass = ms[s];
        R.cen[0] = R.com[0];
        R.cen[1] = R.com[1];
        R.cen[2] = R.com[2];
        R.skip = ep + 1u;
        R.meta = kParticleFlag | (uint32_t)((r > l ? r : l) + 1);
        rec[ep] = R;
        efirst[ep] = (uint32_t)s;
        ecount[ep] = 1u;
        pe[s] = ep;
        if (eh)
            eh[ep] = hs[s];
        if (out32) {  // offset from the centre of its depth-21 cell
            Rec32 o;
            rec32_centre(o, q, kMaxLevel, sh, true);
            const double len = ldexp(F.L, -kMaxLevel);
            o.dx = (float)(R.com[0] - (F.x0[0] + ((double)q[0] + 0.5) * len));
            o.dy = (float)(R.com[1] - (F.x0[1] + ((double)q[1] + 0.5) * len));
            o.dz = (float)(R.com[2] - (F.x0[2] + ((double)q[2] + 0.5) * len));
            o.gm = (float)(G * R.mass);
            o.skip = R.skip;
            out32[ep] = o;
            if (eh32)
                eh32[ep] = (float)hs[s];
        }
    }
    if (nn == 0)
        return;
    for (int lev = l + 1; lev <= r; ++lev) {
        const uint32_t e = b + (uint32_t)(lev - l - 1);
        Rec64 R;
        const double len = ldexp(F.L, -lev);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const uint32_t P_a = q[a] >> (kBits - lev);
            R.cen[a] = F.x0[a] + ((double)P_a + 0.5) * len;
            R.com[a] = 0.0;
        }
        R.mass = 0.0;
        R.skip = 0u;  // set by k_moments
        R.meta = (uint32_t)lev;
        rec[e] = R;
        efirst[e] = (uint32_t)s;
    }
}

// Nodes of one level (deepest level first): walk the children through their
// skip pointers (all deeper, so already final), sum the monopole moments in
// curve order -- M = (M1 + M2) + ..., X = fma(M_k, s_k, X), s = X / M -- and
// set the node's particle count, skip pointer and leaf-parent flag.  With individual
// softening the node also takes the largest spline support of its children.
// The particle count follows from the first particles of the node and of the
// entry after its subtree (particles of a subtree are consecutive on the
// curve), so the children's counts are not read.
// FP32 contexts (out32 set): the node's FP32 record is written too (exact
// integer centre from its first particle's cell, float offset of the centre of
// mass from it, G m, skip, leaf-parent flag).
__global__ __launch_bounds__(kBlock) void k_moments(Rec64 *__restrict__ rec, uint32_t E,
                                                    uint32_t n, const uint32_t *__restrict__ efirst,
                                                    uint32_t *__restrict__ ecount,
                                                    const uint32_t *__restrict__ list,
                                                    uint32_t count, uint32_t lev,
                                                    double *__restrict__ eh, double G,
                                                    const uint64_t *__restrict__ qs, int sh,
                                                    Rec32 *__restrict__ out32,
                                                    float *__restrict__ eh32) {
    uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= count)
        return;
    const uint32_t e = list[i];
    // what does not depend on the children first, so that its loads overlap
    // the walk over them
    Rec64 R = rec[e];
    const uint32_t f = efirst[e];
    const uint64_t qq = out32 ? qs[f] : 0ull;
    double M = 0.0, X0 = 0.0, X1 = 0.0, X2 = 0.0, hmax = 0.0;
    uint32_t k = e + 1;
    while (k < E && (rec[k].meta & 0xffu) > lev) {
        if (eh)
            hmax = eh[k] > hmax ? eh[k] : hmax;
        const double mk = rec[k].mass;
        M = M + mk;
        X0 = fma(mk, rec[k].com[0], X0);
        X1 = fma(mk, rec[k].com[1], X1);
        X2 = fma(mk, rec[k].com[2], X2);
        k = rec[k].skip;
    }
    const uint32_t cnt = (k < E ? efirst[k] : n) - f;
    const bool leaf_parent = k - e - 1u == cnt;  // no entry below but the particles themselves
    R.mass = M;
    R.com[0] = X0 / M;
    R.com[1] = X1 / M;
    R.com[2] = X2 / M;
    R.skip = k;
    R.meta |= leaf_parent ? kLeafParentFlag : 0u;
    rec[e] = R;
    ecount[e] = cnt;
    if (eh)
        eh[e] = hmax;
    if (out32) {  // exact integer centre from the node's first particle
        const uint32_t q[3] = {(uint32_t)(qq >> 42) & 0x1fffffu,
                               (uint32_t)(qq >> 21) & 0x1fffffu, (uint32_t)qq & 0x1fffffu};
        Rec32 o;
        rec32_centre(o, q, (int)lev, sh, false);
        o.dx = (float)(R.com[0] - R.cen[0]);
        o.dy = (float)(R.com[1] - R.cen[1]);
        o.dz = (float)(R.com[2] - R.cen[2]);
        o.gm = (float)(G * M);
        o.cx_meta |= leaf_parent ? kRecLeafParent : 0;
        o.skip = k;
        out32[e] = o;
        if (eh32)
            eh32[e] = (float)hmax;
    }
}


}  // namespace

size_t topology_hist_bytes(int64_t n) {
    return (size_t)2 * kLevels * grid_for(n, kBlock) * sizeof(uint32_t);
}

size_t bbox_bytes(int64_t n) {
    return (size_t)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock) * 6 * sizeof(double);
}

int build(tpm_ctx *c, int64_t n, const double *x, const double *y, const double *z,
          const double *mass, const double *eps) {
    hipStream_t st = c->stream;
    const tpm_params &P = c->P;
    // per-particle buffers
    TPM_TRY(ensure(c, c->frame, sizeof(Frame)));
    for (int b = 0; b < 2; b++) {
        TPM_TRY(ensure(c, c->key[b], (size_t)n * 8));
        TPM_TRY(ensure(c, c->idx[b], (size_t)n * 4));
    }
    TPM_TRY(ensure(c, c->perm, (size_t)n * 4));
    TPM_TRY(ensure(c, c->xyzm, (size_t)n * 32));
    TPM_TRY(ensure(c, c->rank, (size_t)n * 4));
    TPM_TRY(ensure(c, c->ps, (size_t)n * 24));
    TPM_TRY(ensure(c, c->ms, (size_t)n * 8));
    TPM_TRY(ensure(c, c->qs, (size_t)n * 8));
    TPM_TRY(ensure(c, c->dR, (size_t)n));
    TPM_TRY(ensure(c, c->cnt, (size_t)n * 4));
    TPM_TRY(ensure(c, c->base, (size_t)n * 4));
    TPM_TRY(ensure(c, c->pe, (size_t)n * 4));
    TPM_TRY(ensure(c, c->counters, 64 * sizeof(uint32_t)));
    TPM_TRY(ensure(c, c->lvl_cursor, 32 * sizeof(uint32_t)));
    Frame *F = (Frame *)c->frame.p;

    // 1. root cube
    TPM_TRY(timer_begin(c, TPM_TIMER_KEYS));
    if (P.periodic) {
        Frame h{};
        for (int a = 0; a < 3; a++)
            h.x0[a] = -(P.shift[a] * P.box_size);
        h.L = P.box_size;
        h.S = 2097152.0 / P.box_size;
        h.box = P.box_size;
        h.periodic = 1;
        c->frame_host = h;
        TPM_HIP(c, hipMemcpyAsync(F, &c->frame_host, sizeof(Frame), hipMemcpyHostToDevice, st));
    } else {
        const int nparts = (int)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
        TPM_TRY(ensure(c, c->bbox, bbox_bytes(n)));
        k_bbox_partial<<<nparts, kBlock, 0, st>>>(x, y, z, n, (double *)c->bbox.p);
        TPM_LAUNCHED(c, "k_bbox_partial");
        k_frame_final<<<1, kBlock, 0, st>>>((const double *)c->bbox.p, nparts, F, P.shift[0],
                                            P.shift[1], P.shift[2]);
        TPM_LAUNCHED(c, "k_frame_final");
    }
    // 2. keys, 3. sort, gather
    k_keys<<<grid_for(n, kBlock), kBlock, 0, st>>>(x, y, z, mass, n, F,
                                                   (uint64_t *)c->key[0].p,
                                                   (uint32_t *)c->idx[0].p, (double4 *)c->xyzm.p);
    TPM_LAUNCHED(c, "k_keys");
    TPM_TRY(timer_end(c, TPM_TIMER_KEYS));
    TPM_TRY(radix_sort_pairs(c, n));
    // individual softening: spline supports in curve order; a bad value
    // sets the second error word, read back with the sizes below
    c->mixed = eps != nullptr;
    uint32_t *bad_eps = (uint32_t *)c->err_flag.p + 1;
    if (c->mixed)
        TPM_TRY(ensure(c, c->hs, (size_t)n * 8));
    TPM_TRY(timer_begin(c, TPM_TIMER_GATHER));
    k_gather<<<grid_for(n, kBlock), kBlock, 0, st>>>(
        (const double4 *)c->xyzm.p, n, F, (const uint32_t *)c->idx[0].p, (int32_t *)c->perm.p,
        (int32_t *)c->rank.p, (double *)c->ps.p, (double *)c->ms.p, (uint64_t *)c->qs.p, eps,
        c->mixed ? (double *)c->hs.p : nullptr, bad_eps);
    TPM_LAUNCHED(c, "k_gather");
    TPM_TRY(timer_end(c, TPM_TIMER_GATHER));
    // 4. topology: counts, scan, one readback of the sizes
    const uint64_t *key = (const uint64_t *)c->key[0].p;
    uint32_t *lvl_count = (uint32_t *)c->counters.p;  // [0..21] level starts, [32] E, [33] nodes
    const uint32_t nb = grid_for(n, kBlock);
    TPM_TRY(ensure(c, c->hist, topology_hist_bytes(n)));
    uint32_t *lhist = (uint32_t *)c->hist.p;
    uint32_t *loff = lhist + (size_t)kLevels * nb;
    TPM_TRY(timer_begin(c, TPM_TIMER_TOPOLOGY));
    k_count<<<nb, kBlock, 0, st>>>(key, n, (int8_t *)c->dR.p, (uint32_t *)c->cnt.p, lhist, nb);
    TPM_LAUNCHED(c, "k_count");
    TPM_TRY(scan_u32(c, (const uint32_t *)c->cnt.p, (uint32_t *)c->base.p, n, lvl_count + 32));
    TPM_TRY(scan_u32(c, lhist, loff, (int64_t)kLevels * nb, lvl_count + 33));
    k_level_starts<<<1, 64, 0, st>>>(loff, nb, lvl_count);
    TPM_LAUNCHED(c, "k_level_starts");
    TPM_TRY(timer_end(c, TPM_TIMER_TOPOLOGY));
    TPM_HIP(c, hipMemcpyAsync(c->hpin, lvl_count, 64 * sizeof(uint32_t), hipMemcpyDeviceToHost,
                              st));
    if (!P.periodic)
        TPM_HIP(c, hipMemcpyAsync(&c->frame_host, F, sizeof(Frame), hipMemcpyDeviceToHost, st));
    TPM_HIP(c, hipMemcpyAsync(c->hpin + 128, bad_eps, sizeof(uint32_t), hipMemcpyDeviceToHost,
                              st));
    TPM_HIP(c, hipStreamSynchronize(st));
    if (c->hpin[128]) {
        TPM_TRY(fill_u32(c, bad_eps, 0u, 1));
        return fail(c, TPM_EINVAL, "softening lengths must be positive and finite");
    }
    // the FP32 walk works in units of L 2^-22 and scales sizes by 2^-level
    // through the exponent: both need a root size well inside float range
    if (P.precision == TPM_FP32 &&
        !(c->frame_host.L >= 0x1p-80 && c->frame_host.L <= 0x1p+80))
        return fail(c, TPM_EINVAL, "FP32 path: root cube size outside [2^-80, 2^80]");
    const uint32_t E = c->hpin[32];
    const uint32_t nodes = c->hpin[33];
    if ((uint64_t)E != (uint64_t)n + nodes)
        return fail(c, TPM_EDEVICE, "tree build: entry count mismatch");
    for (int l = 0; l < kLevels; l++)
        c->level_off[l] = c->hpin[l];
    c->level_off[kLevels] = nodes;
    for (int l = 0; l < kLevels; l++)
        c->level_count[l] = c->level_off[l + 1] - c->level_off[l];
    const uint32_t off = nodes;
    TPM_TRY(ensure(c, c->rec64, (size_t)E * sizeof(Rec64)));
    TPM_TRY(ensure(c, c->efirst, (size_t)E * 4));
    TPM_TRY(ensure(c, c->ecount, (size_t)E * 4));
    TPM_TRY(ensure(c, c->lvl_list, (size_t)(off > 0 ? off : 1) * 4));
    Rec64 *rec = (Rec64 *)c->rec64.p;
    // FP32 records: particles' written by the emission, nodes' by the moments
    Rec32 *rec32 = nullptr;
    float *eh32 = nullptr;
    if (P.precision == TPM_FP32) {
        TPM_TRY(ensure(c, c->rec32, (size_t)E * sizeof(Rec32)));
        rec32 = (Rec32 *)c->rec32.p;
        if (c->mixed) {
            TPM_TRY(ensure(c, c->eh32, (size_t)E * 4));
            eh32 = (float *)c->eh32.p;
        }
    }
    double *eh = nullptr;
    if (c->mixed) {
        TPM_TRY(ensure(c, c->eh64, (size_t)E * 8));
        eh = (double *)c->eh64.p;
    }
    TPM_TRY(timer_begin(c, TPM_TIMER_TOPOLOGY));
    k_emit<<<grid_for(n, kBlock), kBlock, 0, st>>>(
        key, n, (const int8_t *)c->dR.p, (const uint32_t *)c->base.p, F,
        (const double *)c->ps.p, (const double *)c->ms.p, (const uint64_t *)c->qs.p, rec,
        (uint32_t *)c->efirst.p, (uint32_t *)c->ecount.p, (uint32_t *)c->pe.p, loff, nb,
        (uint32_t *)c->lvl_list.p, (const double *)c->hs.p, eh, P.G, rec32, eh32);
    TPM_LAUNCHED(c, "k_emit");
    TPM_TRY(timer_end(c, TPM_TIMER_TOPOLOGY));
    // 5. moments, deepest level first
    TPM_TRY(timer_begin(c, TPM_TIMER_MOMENTS));
    for (int l = kMaxLevel; l >= 0; l--) {
        const uint32_t cnt = c->level_count[l];
        if (!cnt)
            continue;
        k_moments<<<grid_for(cnt, kBlock), kBlock, 0, st>>>(
            rec, E, (uint32_t)n, (const uint32_t *)c->efirst.p, (uint32_t *)c->ecount.p,
            (const uint32_t *)c->lvl_list.p + c->level_off[l],
            cnt, (uint32_t)l, eh, P.G, (const uint64_t *)c->qs.p,
            P.periodic ? kRecShiftPer : kRecShiftIso, rec32, eh32);
        TPM_LAUNCHED(c, "k_moments");
    }
    TPM_TRY(timer_end(c, TPM_TIMER_MOMENTS));
    c->n = n;
    c->E = E;
    return TPM_OK;
}

}  // namespace tpm
