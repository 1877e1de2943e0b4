// Device code of the tree walks (Sec. 3.1, 3.2, 3.4), shared by the
// single-system launches (walk.hip) and the resident serving loop
// (server.hip).  See walk.hip for the description of the walks.
#pragma once

#include "tpm_internal.h"
#include "erfc_poly.h"

namespace tpm {
namespace wk {

constexpr int kBlock = 256;

struct WalkArgs {
    const void *rec;
    uint32_t E;
    uint32_t n;
    const uint32_t *act;
    const uint32_t *nuniq;
    const double *ps;
    const uint64_t *qs;
    const uint32_t *pe;
    const int32_t *perm;
    const double *anorm;
    double x0[3];
    double L;
    double box, half;
    double G, theta2, alpha, h, hinv, h3inv, rc2, inv2rs;
    // root cube: L^2, 0.6 L (box rule), L/2; a level-l cube's values follow
    // by exponent arithmetic
    double L2r, limr, hlr;
    // single-precision copies
    float fu, fL, ftheta2, falpha, fh2, fhinv, fh3inv, frc2, finv2rs;
    float fgexp;  // -log2(e) / (2 r_s)^2: exp(-x^2) = exp2(d^2 fgexp), x = r / (2 r_s)
    float fL2r, flimr, fhlr;
    // leaf-run prefilter: (r_cut + tolerance)^2, and the largest group
    // extent from its reference cell for which the reference cell's nearest
    // image is every member's (periodic)
    float fpf2, fpf_ext;
    double pf2, pf_ext;
    void *res;   // [n][4] per slot: acceleration x, y, z and the interaction count
    void *rpot;  // [n]
    // individual softening (Sec. 3.2): spline support per target (curve
    // order) and the largest support per entry (double, or float for FP32)
    const double *hs;
    const void *eh;
    // largest extent of a group's targets for the shared cursor in the
    // census of compact groups (squared; TreePM: half the cutoff radius)
    double group_ext2;
    const uint32_t *census;  // count of compact groups (sparse sets with a cutoff)
    // results stored device-coherently (written through to memory at once):
    // set by the resident server, whose later work items read them inside
    // the same kernel; other launches store plainly (visible at kernel end)
    uint32_t coherent;
};

// Wavefront masks: ballot of a lane predicate, and a mask read back as the
// predicate of each lane.
__device__ __forceinline__ uint64_t wave_mask(bool p) { return __builtin_amdgcn_ballot_w64(p); }
// a - b modulo 2^32 (the periodic wrap of the shifted integer coordinates of
// the FP32 records), without signed overflow
__device__ __forceinline__ int32_t wsub(int32_t a, int32_t b) {
    return (int32_t)((uint32_t)a - (uint32_t)b);
}
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// ---- FP64 arithmetic (fixed operation order, explicit fma) -------------------

// 1/d from the hardware reciprocal and two Newton steps (within an ulp, not
// correctly rounded: used only inside erfc, d >= 4).
__device__ __forceinline__ double rcp_refined64(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// e^y for y <= 0 (the argument is -x^2): Cody & Waite's reduction y = k ln2 +
// r, |r| <= ln2 / 2, with ln2 split into a double and its remainder, then the
// Taylor series of e^r to degree 13 (remainder below 6e-18 relative) scaled
// by 2^k.  Arguments below -1000 give 0, as e^y does in double.
__device__ __forceinline__ double exp_neg64(double y) {
    constexpr double kLog2e = 0x1.71547652b82fep+0;
    constexpr double kLn2Hi = 0x1.62e42fefa39efp-1, kLn2Lo = 0x1.abc9e3b39803fp-56;
    constexpr double kInvFact[14] = {1.0,
                                     1.0,
                                     1.0 / 2.0,
                                     1.0 / 6.0,
                                     1.0 / 24.0,
                                     1.0 / 120.0,
                                     1.0 / 720.0,
                                     1.0 / 5040.0,
                                     1.0 / 40320.0,
                                     1.0 / 362880.0,
                                     1.0 / 3628800.0,
                                     1.0 / 39916800.0,
                                     1.0 / 479001600.0,
                                     1.0 / 6227020800.0};
    y = y > -1000.0 ? y : -1000.0;
    const double k = rint(y * kLog2e);
    double r = fma(-k, kLn2Hi, y);
    r = fma(-k, kLn2Lo, r);
    double p = kInvFact[13];
#pragma unroll
    for (int j = 12; j >= 0; j--)
        p = fma(p, r, kInvFact[j]);
    return ldexp(p, (int)k);
}

// Scaled complementary error function exp(x^2) erfc(x) = t g(t), t = 4/(4+x),
// g a degree-20 polynomial in s = (4 - x)/(4 + x) (coefficients in
// erfc_poly.h, relative error below 5e-15 for x >= 0): no branches, and
// exp(-x^2) is shared with the Gaussian term of the short-range factor.
__device__ __forceinline__ double erfc_scaled64(double x) {
    const double rd = rcp_refined64(4.0 + x);
    const double sv = (4.0 - x) * rd;
    double g = kErfcPoly[kErfcDegree];
#pragma unroll
    for (int j = kErfcDegree - 1; j >= 0; j--)
        g = fma(g, sv, kErfcPoly[j]);
    return (4.0 * rd) * g;
}

__device__ __forceinline__ double spline_g64(double u) {
    if (u < 0.5) {
        double u2 = u * u;
        return fma(u2, fma(32.0, u, -38.4), 32.0 / 3.0);
    }
    double cubic = fma(fma(fma(-32.0 / 3.0, u, 38.4), u, -48.0), u, 64.0 / 3.0);
    return cubic - 1.0 / (15.0 * (u * u * u));
}

__device__ __forceinline__ double spline_phi64(double u) {
    double u2 = u * u;
    if (u < 0.5)
        return u2 * (16.0 / 3.0 + u2 * (-48.0 / 5.0 + u * (32.0 / 5.0))) - 14.0 / 5.0;
    return u2 * (32.0 / 3.0 + u * (-16.0 + u * (48.0 / 5.0 + u * (-32.0 / 15.0)))) - 16.0 / 5.0 +
           1.0 / (15.0 * u);
}

// r = |d| and 1 / r from d^2: the hardware reciprocal square root refined by
// two Newton steps (relative error about one ulp, far below the FP64 path's
// tolerance), in place of a correctly rounded square root and division.  A
// coincident pair, or one closer than 2^-500 (d^2 below the normal range,
// where the estimate is not reliable), gets r = 0 and a 1 / r that no result
// uses: it takes the softened branch.
__device__ __forceinline__ void r_rinv64(double dd, double &r, double &rinv) {
    double y = __builtin_amdgcn_rsq(dd);
    const double hd = 0.5 * dd;
    y = y * fma(-hd * y, y, 1.5);
    y = y * fma(-hd * y, y, 1.5);
    rinv = y;
    r = dd >= 0x1p-1000 ? dd * y : 0.0;
}

// hp: the pair's spline support with individual softening (MIXED), else
// the common one of the parameters.
template <bool TPM, bool POT, bool MIXED>
__device__ __forceinline__ void interact64(const WalkArgs &A, double m, double d0, double d1,
                                           double d2, double dd, double hp, double &a0,
                                           double &a1, double &a2, double &pot) {
    const double Gm = A.G * m;
    double r, rinv;
    r_rinv64(dd, r, rinv);
    const double h = MIXED ? hp : A.h;
    double fac, phi = 0.0;
    if (r >= h) {
        fac = Gm * rinv * rinv * rinv;
        if (POT)
            phi = -Gm * rinv;
    } else {
        double hinv = A.hinv, h3inv = A.h3inv;
        if (MIXED) {
            hinv = 1.0 / h;
            h3inv = hinv * hinv * hinv;
        }
        const double u = r / h;
        fac = (Gm * h3inv) * spline_g64(u);
        if (POT)
            phi = (Gm * hinv) * spline_phi64(u);
    }
    if (TPM) {
        const double x = r * A.inv2rs;
        const double gx = exp_neg64(-(x * x));
        const double ec = gx * erfc_scaled64(x);
        fac = fac * (ec + (x * 1.1283791670955126) * gx);
        if (POT)
            phi = phi * ec;
    }
    a0 = fma(fac, d0, a0);
    a1 = fma(fac, d1, a1);
    a2 = fma(fac, d2, a2);
    if (POT)
        pot += phi;
}

// Nearest image of a difference |d| < box: d - box if d > box / 2, d + box
// if d < -box / 2 (the same operations and results as the two-sided test,
// without branches).
template <bool PER>
__device__ __forceinline__ double wrap64(double d, double box, double half) {
    if (PER) {
        const double t = d - copysign(box, d);
        d = fabs(d) > half ? t : d;
    }
    return d;
}

__device__ __forceinline__ double spline_g64_sel(double u) {
    const double u2 = u * u;
    const double inner = fma(u2, fma(32.0, u, -38.4), 32.0 / 3.0);
    const double cubic = fma(fma(fma(-32.0 / 3.0, u, 38.4), u, -48.0), u, 64.0 / 3.0);
    const double outer = cubic - 1.0 / (15.0 * (u * u * u));
    return u < 0.5 ? inner : outer;
}

__device__ __forceinline__ double spline_phi64_sel(double u) {
    const double u2 = u * u;
    const double inner = u2 * (16.0 / 3.0 + u2 * (-48.0 / 5.0 + u * (32.0 / 5.0))) - 14.0 / 5.0;
    const double outer =
        u2 * (32.0 / 3.0 + u * (-16.0 + u * (48.0 / 5.0 + u * (-32.0 / 15.0)))) - 16.0 / 5.0 +
        1.0 / (15.0 * u);
    return u < 0.5 ? inner : outer;
}

// The force and potential factors of interact64 (fac and phi, before the
// products with the difference vector), computed by the whole wavefront for
// one pair per lane; `used` marks the lanes whose factors are used (the
// others may hold any pair, even a coincident one).  Per-lane choices are
// selects, so each lane gets exactly interact64's factors for its pair.
template <bool TPM, bool POT, bool MIXED>
__device__ __forceinline__ void factor64(const WalkArgs &A, uint64_t used, double m, double dd,
                                         double hp, double &fac, double &phi) {
    const double Gm = A.G * m;
    double r, rinv;
    r_rinv64(dd, r, rinv);
    const double h = MIXED ? hp : A.h;
    fac = Gm * rinv * rinv * rinv;
    phi = 0.0;
    if (POT)
        phi = -Gm * rinv;
    const bool soft = r < h;
    if (used & wave_mask(soft)) {
        double hinv = A.hinv, h3inv = A.h3inv;
        if (MIXED) {
            hinv = 1.0 / h;
            h3inv = hinv * hinv * hinv;
        }
        const double u = r / h;
        fac = soft ? (Gm * h3inv) * spline_g64_sel(u) : fac;
        if (POT)
            phi = soft ? (Gm * hinv) * spline_phi64_sel(u) : phi;
    }
    if (TPM) {
        const double x = r * A.inv2rs;
        const double gx = exp_neg64(-(x * x));
        const double ec = gx * erfc_scaled64(x);
        fac = fac * (ec + (x * 1.1283791670955126) * gx);
        if (POT)
            phi = phi * ec;
    }
}

// Interaction queue of one wavefront in the FP64 walk with a cutoff.  A step
// of the walk interacts some of the 64 targets with one entry, and with the
// cutoff most steps take only a few lanes.  So a step appends its pairs (in
// lane order) and its lane mask instead of evaluating at once; when more
// than 64 pairs are pending, the pairs queued before the last step are
// evaluated one per lane, and each target then adds its own pairs in the
// order of the steps: the same products and sums, in the same order, as an
// immediate evaluation.  Pairs and steps sit in rings of 128, so a step is
// stored before the evaluation that it triggers (its values need not stay in
// registers across it).  Without a cutoff nearly every step takes most lanes
// and the walk evaluates at once.
constexpr uint32_t kQueue = 64;
constexpr uint32_t kAccSteps = 2;
constexpr uint32_t kRing = 128;
struct IQ64 {
    double d[3][kRing];  // difference vector, entry minus target
    double m[kRing];     // mass; after evaluation the force factor
    double h[kRing];     // larger softening; after evaluation the potential factor
    uint64_t step[kRing];
};

// Device-coherent accesses (relaxed device-scope atomics: they bypass the
// caches that are not coherent across the chip's dies) for the data one
// phase of the resident serving loop hands to the next: the active slots,
// |a| and the walk results.  Single-system launches use the same code.
template <typename T>
__device__ __forceinline__ T coherent_ld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void coherent_st(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The number of unique active targets, written by an earlier kernel or, in
// the resident server, by another wavefront of the same kernel: read with a
// coherent vector load (never through the scalar cache) and made uniform.
__device__ __forceinline__ uint32_t load_count(const uint32_t *p) {
    return __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// A slot's results are one record of four values: the acceleration and, in
// the fourth, the interaction count carried in the value's bits (so the
// output gathers read one record per target).
__device__ __forceinline__ float count_bits(uint32_t n, float) { return __uint_as_float(n); }
__device__ __forceinline__ double count_bits(uint32_t n, double) {
    return __longlong_as_double((long long)n);
}
__device__ __forceinline__ uint32_t count_of(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t count_of(double v) {
    return (uint32_t)__double_as_longlong(v);
}
template <typename T>
__device__ __forceinline__ void store_result(const WalkArgs &A, uint32_t slot, T a0, T a1, T a2,
                                             bool pot_on, T pot, uint32_t nint) {
    T *r = (T *)A.res + 4 * (size_t)slot;
    if (A.coherent) {
        coherent_st(r, a0);
        coherent_st(r + 1, a1);
        coherent_st(r + 2, a2);
        coherent_st(r + 3, count_bits(nint, T()));
        if (pot_on)
            coherent_st((T *)A.rpot + slot, pot);
    } else {  // the whole record in one (FP32) or two (FP64) 16-byte stores
        if constexpr (sizeof(T) == 4) {
            typedef T T4 __attribute__((ext_vector_type(4)));
            *(T4 *)r = T4{a0, a1, a2, count_bits(nint, T())};
        } else {
            typedef T T2 __attribute__((ext_vector_type(2)));
            ((T2 *)r)[0] = T2{a0, a1};
            ((T2 *)r)[1] = T2{a2, count_bits(nint, T())};
        }
        if (pot_on)
            ((T *)A.rpot)[slot] = pot;
    }
}

// Orders the wavefront's LDS accesses (lanes read what other lanes wrote).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Number of lanes of m below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Record i for a wavefront-uniform i, read through the constant address
// space (the tree does not change during a walk): scalar loads, whatever
// fences the walk holds for its LDS queue.
__device__ __forceinline__ Rec64 uniform_rec(const Rec64 *R, uint32_t i) {
    typedef __attribute__((address_space(4))) const uint64_t cword;
    const cword *w = (const cword *)(R + i);
    uint64_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        v[k] = w[k];
    Rec64 r;
    __builtin_memcpy(&r, v, sizeof r);
    return r;
}

// The same for FP32 records, and for one value of a per-entry array.
__device__ __forceinline__ Rec32 uniform_rec32(const Rec32 *R, uint32_t i) {
    typedef __attribute__((address_space(4))) const uint64_t cword;
    const cword *w = (const cword *)(R + i);
    uint64_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        v[k] = w[k];
    Rec32 r;
    __builtin_memcpy(&r, v, sizeof r);
    return r;
}

template <typename T>
__device__ __forceinline__ T uniform_at(const void *p, uint32_t i) {
    typedef __attribute__((address_space(4))) const T cval;
    return ((const cval *)p)[i];
}

// A wavefront-uniform pointer kept in scalar registers (it may have been
// read from memory the compiler cannot prove unchanging).
template <typename T>
__device__ __forceinline__ const T *uniform_ptr(const void *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const T *)(((uint64_t)hi << 32) | lo);
}

// Side of a level-`lev` cube, scaled from the root side through the exponent
// field (exact: the root side is a normal number and lev <= 21).
__device__ __forceinline__ double scale_level(double v, uint32_t lev) {
    return __longlong_as_double(__double_as_longlong(v) - ((long long)lev << 52));
}

// One wavefront walks group `wave` (slots 64 wave .. 64 wave + 63).  The
// cursor and the entry are wavefront-uniform; each lane decides for itself
// (as masks) and only branches on wavefront-uniform conditions are taken.
template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__device__ __forceinline__ void walk_group64(const WalkArgs &A, uint32_t wave, IQ64 *Q) {
    const int lane = threadIdx.x & 63;
    const uint32_t nu = load_count(A.nuniq);
    if (wave * 64u >= nu)
        return;  // whole wavefront
    const uint32_t slot = wave * 64u + lane;
    const bool valid = slot < nu;
    const uint32_t s = coherent_ld(A.act + (valid ? slot : wave * 64u));
    const double x0 = A.ps[s], x1 = A.ps[A.n + s], x2 = A.ps[2 * (size_t)A.n + s];
    const uint32_t self = A.pe[s];
    double an = 0.0;
    if (OPEN == TPM_OPEN_REL)
        an = coherent_ld(A.anorm + A.perm[s]);
    const double alpha_an = A.alpha * an;
    const double hi = MIXED ? A.hs[s] : 0.0;  // the target's own support
    // the lane's walk stands at the cursor when next <= cursor (next moves
    // to the skip pointer only when the lane accepts or discards a cube)
    uint32_t next = valid ? 0u : 0xffffffffu;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, pot = 0.0;
    uint32_t nint = 0;
    const Rec64 *__restrict__ R = uniform_ptr<Rec64>(A.rec);

    // leaf-run prefilter (as in the FP32 walk): bounding box of the targets
    // relative to lane 0's position
    double xr0 = 0.0, xr1 = 0.0, xr2 = 0.0;
    double lo0 = 0.0, hi0 = 0.0, lo1 = 0.0, hi1 = 0.0, lo2 = 0.0, hi2 = 0.0;
    bool prefilter = false;
    if (TPM) {
        auto uni = [](double v) {
            const uint64_t b = (uint64_t)__double_as_longlong(v);
            const uint32_t l = __builtin_amdgcn_readfirstlane((uint32_t)b);
            const uint32_t h = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
            return __longlong_as_double((long long)(((uint64_t)h << 32) | l));
        };
        xr0 = uni(x0), xr1 = uni(x1), xr2 = uni(x2);
        lo0 = hi0 = wrap64<PER>(x0 - xr0, A.box, A.half);
        lo1 = hi1 = wrap64<PER>(x1 - xr1, A.box, A.half);
        lo2 = hi2 = wrap64<PER>(x2 - xr2, A.box, A.half);
        for (int o = 1; o < 64; o <<= 1) {
            lo0 = fmin(lo0, __shfl_xor(lo0, o));
            hi0 = fmax(hi0, __shfl_xor(hi0, o));
            lo1 = fmin(lo1, __shfl_xor(lo1, o));
            hi1 = fmax(hi1, __shfl_xor(hi1, o));
            lo2 = fmin(lo2, __shfl_xor(lo2, o));
            hi2 = fmax(hi2, __shfl_xor(hi2, o));
        }
        lo0 = uni(lo0), hi0 = uni(hi0), lo1 = uni(lo1), hi1 = uni(hi1), lo2 = uni(lo2),
        hi2 = uni(hi2);
        const double ext = fmax(fmax(fmax(-lo0, hi0), fmax(-lo1, hi1)), fmax(-lo2, hi2));
        prefilter = ext < A.pf_ext;
    }

    // queue state (wavefront-uniform): ring heads of the pending pairs and
    // steps, and their counts
    uint32_t qh = 0, qn = 0, sh = 0, ns = 0;
    // evaluate the first n (<= 64) pending pairs, then add those of the
    // first `steps` pending steps to their targets
    auto flush = [&](uint32_t n, uint32_t steps) {
        wave_sync();
        const bool own = (uint32_t)lane < n;
        const uint32_t i = (qh + (own ? (uint32_t)lane : 0u)) & (kRing - 1u);
        {
            const double d0 = Q->d[0][i], d1 = Q->d[1][i], d2 = Q->d[2][i];
            double fac, phi;
            factor64<TPM, POT, MIXED>(A, wave_mask(own), Q->m[i],
                                      fma(d0, d0, fma(d1, d1, d2 * d2)),
                                      MIXED ? Q->h[i] : 0.0, fac, phi);
            wave_sync();
            if (own) {
                Q->m[i] = fac;
                if (POT)
                    Q->h[i] = phi;
            }
        }
        // lane j holds the mask of step j
        const uint64_t sv = Q->step[(sh + (uint32_t)lane) & (kRing - 1u)];
        const uint32_t svl = (uint32_t)sv, svh = (uint32_t)(sv >> 32);
        wave_sync();
        // kAccSteps steps at a time: their loads are issued together, and
        // each lane adds only the pairs of steps that it is in, in order
        uint32_t b = qh;
        for (uint32_t j = 0; j < steps; j += kAccSteps) {
            bool in[kAccSteps];
            uint32_t pp[kAccSteps];
#pragma unroll
            for (uint32_t u = 0; u < kAccSteps; ++u) {
                const uint32_t jj = min(j + u, 63u);
                const uint32_t ml = __builtin_amdgcn_readlane(svl, jj);
                const uint32_t mh = __builtin_amdgcn_readlane(svh, jj);
                const uint64_t m = j + u < steps ? ((uint64_t)mh << 32) | ml : 0ull;
                in[u] = lane_in(m);
                pp[u] = (b + lanes_below(m)) & (kRing - 1u);
                b += (uint32_t)__builtin_popcountll(m);
            }
            double f[kAccSteps], x[kAccSteps], y[kAccSteps], z[kAccSteps], ph[kAccSteps];
#pragma unroll
            for (uint32_t u = 0; u < kAccSteps; ++u) {
                f[u] = Q->m[pp[u]];
                x[u] = Q->d[0][pp[u]];
                y[u] = Q->d[1][pp[u]];
                z[u] = Q->d[2][pp[u]];
                ph[u] = POT ? Q->h[pp[u]] : 0.0;
            }
#pragma unroll
            for (uint32_t u = 0; u < kAccSteps; ++u) {
                a0 = in[u] ? fma(f[u], x[u], a0) : a0;
                a1 = in[u] ? fma(f[u], y[u], a1) : a1;
                a2 = in[u] ? fma(f[u], z[u], a2) : a2;
                if (POT)
                    pot = in[u] ? pot + ph[u] : pot;
            }
        }
        wave_sync();
        qh = (qh + n) & (kRing - 1u);
        sh = (sh + steps) & (kRing - 1u);
    };
    // the lanes in `inter` (not empty) interact with an entry of mass m
    auto push = [&](uint64_t inter, double m, double d0, double d1, double d2, double dd,
                    double hp) {
        nint += lane_in(inter) ? 1u : 0u;
        if (!TPM) {  // evaluate at once (fma(0, d, a) == a for the other lanes)
            double fac, phi;
            factor64<TPM, POT, MIXED>(A, inter, m, dd, hp, fac, phi);
            const bool in = lane_in(inter);
            fac = in ? fac : 0.0;
            a0 = fma(fac, d0, a0);
            a1 = fma(fac, d1, a1);
            a2 = fma(fac, d2, a2);
            if (POT)
                pot += in ? phi : 0.0;
            return;
        }
        const uint32_t k = (uint32_t)__builtin_popcountll(inter);
        if (lane_in(inter)) {
            const uint32_t p = (qh + qn + lanes_below(inter)) & (kRing - 1u);
            Q->d[0][p] = d0;
            Q->d[1][p] = d1;
            Q->d[2][p] = d2;
            Q->m[p] = m;
            if (MIXED)
                Q->h[p] = hp;
        }
        if (lane == 0)
            Q->step[(sh + ns) & (kRing - 1u)] = inter;
        if (qn + k > kQueue) {  // at most 64 pending before this step
            flush(qn, ns);
            qn = k;
            ns = 1;
        } else {
            qn += k;
            ++ns;
        }
    };

    // one particle entry e (wavefront-uniform) for the lanes in m
    auto particle = [&](const Rec64 &r, uint32_t e, uint64_t m) {
        const double he = MIXED ? uniform_at<double>(A.eh, e) : 0.0;
        const double hp = hi > he ? hi : he;  // the larger support
        const double d0 = wrap64<PER>(r.com[0] - x0, A.box, A.half);
        const double d1 = wrap64<PER>(r.com[1] - x1, A.box, A.half);
        const double d2 = wrap64<PER>(r.com[2] - x2, A.box, A.half);
        const double dd = fma(d0, d0, fma(d1, d1, d2 * d2));
        uint64_t inter = m & wave_mask(e != self);
        if (TPM)
            inter &= wave_mask(dd < A.rc2);
        if (inter)
            push(inter, r.mass, d0, d1, d2, dd, hp);
    };

    uint32_t c = 0;
    while (c < A.E) {
        const uint32_t cu = __builtin_amdgcn_readfirstlane(c);
        const Rec64 r = uniform_rec(R, cu);
        const uint64_t mine = wave_mask(next <= cu);
        if (r.meta & kParticleFlag) {
            particle(r, cu, mine);
            c = cu + 1u;
            continue;
        }
        const double he = MIXED ? uniform_at<double>(A.eh, cu) : 0.0;
        const double hp = hi > he ? hi : he;  // the larger support
        const uint32_t lev = r.meta & 0xffu;
        const double c0 = wrap64<PER>(r.cen[0] - x0, A.box, A.half);
        const double c1 = wrap64<PER>(r.cen[1] - x1, A.box, A.half);
        const double c2 = wrap64<PER>(r.cen[2] - x2, A.box, A.half);
        uint64_t keep = ~0ull;
        if (TPM) {
            const double hl = scale_level(A.hlr, lev);
            double e0 = fabs(c0) - hl, e1 = fabs(c1) - hl, e2 = fabs(c2) - hl;
            e0 = e0 > 0.0 ? e0 : 0.0;
            e1 = e1 > 0.0 ? e1 : 0.0;
            e2 = e2 > 0.0 ? e2 : 0.0;
            keep = wave_mask(!(fma(e0, e0, fma(e1, e1, e2 * e2)) > A.rc2));
            if (!(mine & keep)) {  // every lane here discards the cube
                next = lane_in(mine) ? r.skip : next;
                c = r.skip;
                continue;
            }
        }
        const double d0 = wrap64<PER>(r.com[0] - x0, A.box, A.half);
        const double d1 = wrap64<PER>(r.com[1] - x1, A.box, A.half);
        const double d2 = wrap64<PER>(r.com[2] - x2, A.box, A.half);
        const double dd = fma(d0, d0, fma(d1, d1, d2 * d2));
        const double L2 = scale_level(scale_level(A.L2r, lev), lev);
        uint64_t open;
        if (OPEN == TPM_OPEN_BH)
            open = wave_mask(L2 > A.theta2 * dd);
        else
            open = wave_mask((A.G * r.mass) * L2 > alpha_an * (dd * dd));
        const double lim = scale_level(A.limr, lev);
        open |= wave_mask(fabs(c0) < lim) & wave_mask(fabs(c1) < lim) &
                wave_mask(fabs(c2) < lim);
        // larger softening inside the node, target within it of the
        // centre of mass: open (Sec. 3.2)
        if (MIXED)
            open |= wave_mask(hi < he) & wave_mask(dd < he * he);
        open &= keep;
        const uint64_t inter = mine & keep & ~open;
        const uint64_t desc = mine & open;
        next = lane_in(mine & ~open) ? r.skip : next;
        if (inter)
            push(inter, r.mass, d0, d1, d2, dd, hp);
        {
            // an opened leaf parent (with the prefilter): its particle
            // children walked here; for any other cube the run is empty
            const bool run = TPM && desc && (r.meta & kLeafParentFlag) && prefilter;
            const uint32_t end = run ? r.skip : cu + 1u;
            for (uint32_t base = cu + 1u; base < end; base += 64u) {
                const uint32_t k = min(64u, end - base);
                bool near = false;
                if ((uint32_t)lane < k) {
                    const double *t = R[base + lane].com;
                    const double p0 = wrap64<PER>(t[0] - xr0, A.box, A.half);
                    const double p1 = wrap64<PER>(t[1] - xr1, A.box, A.half);
                    const double p2 = wrap64<PER>(t[2] - xr2, A.box, A.half);
                    const double g0 = fmax(fmax(lo0 - p0, p0 - hi0), 0.0);
                    const double g1 = fmax(fmax(lo1 - p1, p1 - hi1), 0.0);
                    const double g2 = fmax(fmax(lo2 - p2, p2 - hi2), 0.0);
                    near = fma(g0, g0, fma(g1, g1, g2 * g2)) < A.pf2;
                }
                for (uint64_t m = wave_mask(near); m; m &= m - 1) {
                    const uint32_t e = base + (uint32_t)__builtin_ctzll(m);
                    particle(uniform_rec(R, e), e, desc);
                }
            }
            c = run ? r.skip : desc ? cu + 1u : r.skip;
        }
    }
    if (TPM && qn)
        flush(qn, ns);
    if (valid)
        store_result<double>(A, slot, a0, a1, a2, POT, pot, nint);
}

// ---- FP32 walk ----------------------------------------------------------------

__device__ __forceinline__ float spline_g32(float u) {
    if (u < 0.5f) {
        const float u2 = u * u;
        return fmaf(u2, fmaf(32.0f, u, -38.4f), 10.6666667f);
    }
    const float cubic = fmaf(fmaf(fmaf(-10.6666667f, u, 38.4f), u, -48.0f), u, 21.3333333f);
    return cubic - __builtin_amdgcn_rcpf(15.0f * u * u * u);
}

__device__ __forceinline__ float spline_phi32(float u) {
    const float u2 = u * u;
    if (u < 0.5f)
        return fmaf(u2, fmaf(u2, fmaf(u, 6.4f, -9.6f), 5.33333333f), -2.8f);
    return fmaf(u2, fmaf(u, fmaf(u, fmaf(u, -2.13333333f, 9.6f), -16.0f), 10.6666667f), -3.2f) +
           __builtin_amdgcn_rcpf(15.0f * u);
}

template <bool TPM, bool POT, bool MIXED>
__device__ __forceinline__ void interact32(const WalkArgs &A, float gm, float d0, float d1,
                                           float d2, float dd, float hp, float &a0, float &a1,
                                           float &a2, float &pot) {
    float fac, phi = 0.0f, r = 0.0f;
    if (dd >= (MIXED ? hp * hp : A.fh2)) {
        const float rinv = __builtin_amdgcn_rsqf(dd);
        fac = gm * rinv * rinv * rinv;
        if (POT)
            phi = -gm * rinv;
        if (TPM)
            r = dd * rinv;
    } else {
        float hinv = A.fhinv, h3inv = A.fh3inv;
        if (MIXED) {
            hinv = 1.0f / hp;
            h3inv = hinv * hinv * hinv;
        }
        r = __builtin_amdgcn_sqrtf(dd);
        const float u = r * hinv;
        fac = (gm * h3inv) * spline_g32(u);
        if (POT)
            phi = (gm * hinv) * spline_phi32(u);
    }
    if (TPM) {
        // erfc(x) = t P(t) exp(-x^2) by Abramowitz & Stegun 7.1.26 (|error|
        // < 1.5e-7); the force factor erfc(x) + (2/sqrt(pi)) x exp(-x^2)
        // shares exp(-x^2), taken from d^2 directly
        const float x = r * A.finv2rs;
        const float g = __builtin_amdgcn_exp2f(dd * A.fgexp);
        const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
        const float tp =
            t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f),
                             -0.284496736f),
                     0.254829592f);
        fac *= g * fmaf(x, 1.12837917f, tp);
        if (POT)
            phi *= tp * g;
    }
    a0 = fmaf(fac, d0, a0);
    a1 = fmaf(fac, d1, a1);
    a2 = fmaf(fac, d2, a2);
    if (POT)
        pot += phi;
}

__device__ __forceinline__ float spline_g32_sel(float u) {
    const float u2 = u * u;
    const float inner = fmaf(u2, fmaf(32.0f, u, -38.4f), 10.6666667f);
    const float cubic = fmaf(fmaf(fmaf(-10.6666667f, u, 38.4f), u, -48.0f), u, 21.3333333f);
    const float outer = cubic - __builtin_amdgcn_rcpf(15.0f * u * u * u);
    return u < 0.5f ? inner : outer;
}

__device__ __forceinline__ float spline_phi32_sel(float u) {
    const float u2 = u * u;
    const float inner = fmaf(u2, fmaf(u2, fmaf(u, 6.4f, -9.6f), 5.33333333f), -2.8f);
    const float outer =
        fmaf(u2, fmaf(u, fmaf(u, fmaf(u, -2.13333333f, 9.6f), -16.0f), 10.6666667f), -3.2f) +
        __builtin_amdgcn_rcpf(15.0f * u);
    return u < 0.5f ? inner : outer;
}

// interact32 for the lanes with `inter` set, executed by the whole wavefront
// (callers branch on "some lane interacts", a uniform condition); per-lane
// choices are selects, so the interacting lanes get exactly interact32's result.
template <bool TPM, bool POT, bool MIXED>
__device__ __forceinline__ void interact32_wave(const WalkArgs &A, uint64_t inter_m, float gm,
                                                float d0, float d1, float d2, float dd, float hp,
                                                float &a0, float &a1, float &a2, float &pot,
                                                uint32_t &nint) {
    const bool inter = lane_in(inter_m);
    const float rinv = __builtin_amdgcn_rsqf(dd);
    float fac = gm * rinv * rinv * rinv;
    float phi = 0.0f, r = 0.0f;
    if (POT)
        phi = -gm * rinv;
    if (TPM)
        r = dd * rinv;
    const bool soft = dd < (MIXED ? hp * hp : A.fh2);
    if (inter_m & wave_mask(soft)) {
        float hinv = A.fhinv, h3inv = A.fh3inv;
        if (MIXED) {
            hinv = 1.0f / hp;
            h3inv = hinv * hinv * hinv;
        }
        const float rr = __builtin_amdgcn_sqrtf(dd);
        const float u = rr * hinv;
        fac = soft ? (gm * h3inv) * spline_g32_sel(u) : fac;
        if (POT)
            phi = soft ? (gm * hinv) * spline_phi32_sel(u) : phi;
        if (TPM)
            r = soft ? rr : r;
    }
    if (TPM) {  // as in interact32
        const float x = r * A.finv2rs;
        const float g = __builtin_amdgcn_exp2f(dd * A.fgexp);
        const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
        const float tp =
            t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f),
                             -0.284496736f),
                     0.254829592f);
        fac *= g * fmaf(x, 1.12837917f, tp);
        if (POT)
            phi *= tp * g;
    }
    fac = inter ? fac : 0.0f;
    a0 = fmaf(fac, d0, a0);
    a1 = fmaf(fac, d1, a1);
    a2 = fmaf(fac, d2, a2);
    if (POT)
        pot += inter ? phi : 0.0f;
    nint += inter ? 1u : 0u;
}

__device__ __forceinline__ float scale_level32(float v, uint32_t lev) {
    return __int_as_float(__float_as_int(v) - (int)(lev << 23));
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__device__ __forceinline__ void walk_group32(const WalkArgs &A, uint32_t wave) {
    constexpr int SH = PER ? kRecShiftPer : kRecShiftIso;
    const int lane = threadIdx.x & 63;
    const uint32_t nu = load_count(A.nuniq);
    if (wave * 64u >= nu)
        return;
    const uint32_t slot = wave * 64u + lane;
    const bool valid = slot < nu;
    const uint32_t s = coherent_ld(A.act + (valid ? slot : wave * 64u));
    // own depth-21 cell centre (integer, shifted like the records) and the
    // float offset of the particle from it
    const uint64_t qq = A.qs[s];
    const uint32_t q0 = (uint32_t)(qq >> 42) & 0x1fffffu, q1 = (uint32_t)(qq >> 21) & 0x1fffffu,
                   q2 = (uint32_t)qq & 0x1fffffu;
    int32_t G0 = (int32_t)((2u * q0 + 1u) << SH), G1 = (int32_t)((2u * q1 + 1u) << SH),
            G2 = (int32_t)((2u * q2 + 1u) << SH);
    // keep each centre whole in one register: split into (2 q << SH) plus a
    // constant, it would cost a second subtraction per coordinate and entry
    asm("" : "+v"(G0), "+v"(G1), "+v"(G2));
    const double len21 = ldexp(A.L, -kMaxLevel);
    const float xr0 = (float)(A.ps[s] - (A.x0[0] + ((double)q0 + 0.5) * len21));
    const float xr1 = (float)(A.ps[A.n + s] - (A.x0[1] + ((double)q1 + 0.5) * len21));
    const float xr2 = (float)(A.ps[2 * (size_t)A.n + s] - (A.x0[2] + ((double)q2 + 0.5) * len21));
    const uint32_t self = A.pe[s];
    float an = 0.0f;
    if (OPEN == TPM_OPEN_REL)
        an = (float)coherent_ld(A.anorm + A.perm[s]);
    const float alpha_an = A.falpha * an;
    const float hi = MIXED ? (float)A.hs[s] : 0.0f;
    // A lane's walk stands at the cursor when next <= cursor: next is only
    // moved (to the skip pointer) when the lane accepts or discards a cube,
    // so a lane that opened a cube follows the cursor through its subtree,
    // particles included, without per-entry bookkeeping.
    uint32_t next = valid ? 0u : 0xffffffffu;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, pot = 0.0f;
    uint32_t nint = 0;
    const Rec32 *__restrict__ R = uniform_ptr<Rec32>(A.rec);

    // With a cutoff, the particles below an opened leaf parent are first
    // tested together, one per lane, against the bounding box of the group's
    // targets (positions relative to lane 0's cell, r_cut padded by a
    // tolerance above the rounding); only those that can lie within r_cut of
    // some target are visited.  The others would interact with no lane, so
    // results and interaction lists are unchanged.
    int32_t Gr0 = 0, Gr1 = 0, Gr2 = 0;
    float lo0 = 0.f, hi0 = 0.f, lo1 = 0.f, hi1 = 0.f, lo2 = 0.f, hi2 = 0.f;
    bool prefilter = false;
    if (TPM) {
        Gr0 = __builtin_amdgcn_readfirstlane(G0);
        Gr1 = __builtin_amdgcn_readfirstlane(G1);
        Gr2 = __builtin_amdgcn_readfirstlane(G2);
        lo0 = hi0 = fmaf((float)wsub(G0, Gr0), A.fu, xr0);
        lo1 = hi1 = fmaf((float)wsub(G1, Gr1), A.fu, xr1);
        lo2 = hi2 = fmaf((float)wsub(G2, Gr2), A.fu, xr2);
        for (int o = 1; o < 64; o <<= 1) {
            lo0 = fminf(lo0, __shfl_xor(lo0, o));
            hi0 = fmaxf(hi0, __shfl_xor(hi0, o));
            lo1 = fminf(lo1, __shfl_xor(lo1, o));
            hi1 = fmaxf(hi1, __shfl_xor(hi1, o));
            lo2 = fminf(lo2, __shfl_xor(lo2, o));
            hi2 = fmaxf(hi2, __shfl_xor(hi2, o));
        }
        auto uni = [](float v) {
            return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
        };
        lo0 = uni(lo0), hi0 = uni(hi0), lo1 = uni(lo1), hi1 = uni(hi1), lo2 = uni(lo2),
        hi2 = uni(hi2);
        // in a periodic box the reference cell's nearest image must be every
        // target's: a group wider than that walks without the prefilter
        const float ext = fmaxf(fmaxf(fmaxf(-lo0, hi0), fmaxf(-lo1, hi1)), fmaxf(-lo2, hi2));
        prefilter = ext < A.fpf_ext;
    }

    // one particle entry e (wavefront-uniform) for the lanes in m
    auto particle = [&](const Rec32 &r, uint32_t e, uint64_t m) {
        const float he = MIXED ? uniform_at<float>(A.eh, e) : 0.0f;
        const float hp = hi > he ? hi : he;
        const float d0 = fmaf((float)wsub(r.cx_meta & -(1 << SH), G0), A.fu, -xr0) + r.dx;
        const float d1 = fmaf((float)wsub(r.cy, G1), A.fu, -xr1) + r.dy;
        const float d2 = fmaf((float)wsub(r.cz, G2), A.fu, -xr2) + r.dz;
        const float dd = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        uint64_t inter = m & wave_mask(e != self);
        if (TPM)
            inter &= wave_mask(dd < A.frc2);
        // unconditional: nearly every visited particle interacts with some
        // lane, and a branch here costs more than the rare empty evaluation
        interact32_wave<TPM, POT, MIXED>(A, inter, r.gm, d0, d1, d2, dd, hp, a0, a1, a2, pot,
                                         nint);
    };

    // level sizes follow from the root's by exponent arithmetic (exact; on
    // the scalar unit, since the entry is wavefront-uniform)
    uint32_t c = 0;
    while (c < A.E) {
        const uint32_t cu = __builtin_amdgcn_readfirstlane(c);
        const Rec32 r = uniform_rec32(R, cu);
        const uint64_t mine = wave_mask(next <= cu);
        const int32_t cm = r.cx_meta;
        if (cm & kRecParticle) {
            particle(r, cu, mine);
            c = cu + 1u;
            continue;
        }
        const float he = MIXED ? uniform_at<float>(A.eh, cu) : 0.0f;
        const float hp = hi > he ? hi : he;
        // target -> centre of the cube (32-bit differences wrap modulo the
        // periodic box), and target -> centre of mass
        const float c0 = fmaf((float)wsub(cm & -(1 << SH), G0), A.fu, -xr0);
        const float c1 = fmaf((float)wsub(r.cy, G1), A.fu, -xr1);
        const float c2 = fmaf((float)wsub(r.cz, G2), A.fu, -xr2);
        const uint32_t lev = (uint32_t)cm & kRecLevel;
        uint64_t keep = ~0ull;
        if (TPM) {
            const float hl = scale_level32(A.fhlr, lev);
            const float e0 = fmaxf(fabsf(c0) - hl, 0.0f);
            const float e1 = fmaxf(fabsf(c1) - hl, 0.0f);
            const float e2 = fmaxf(fabsf(c2) - hl, 0.0f);
            keep = wave_mask(!(fmaf(e0, e0, fmaf(e1, e1, e2 * e2)) > A.frc2));
            if (!(mine & keep)) {  // every lane here discards the cube
                next = lane_in(mine) ? r.skip : next;
                c = r.skip;
                continue;
            }
        }
        const float d0 = c0 + r.dx, d1 = c1 + r.dy, d2 = c2 + r.dz;
        const float dd = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        const float L2 = scale_level32(scale_level32(A.fL2r, lev), lev);
        uint64_t open;
        if (OPEN == TPM_OPEN_BH)
            open = wave_mask(L2 > A.ftheta2 * dd);
        else
            open = wave_mask(r.gm * L2 > alpha_an * (dd * dd));
        const float lim = scale_level32(A.flimr, lev);
        open |= wave_mask(fabsf(c0) < lim) & wave_mask(fabsf(c1) < lim) &
                wave_mask(fabsf(c2) < lim);
        if (MIXED)
            open |= wave_mask(hi < he) & wave_mask(dd < he * he);
        open &= keep;
        const uint64_t inter = mine & keep & ~open;
        const uint64_t desc = mine & open;
        next = lane_in(mine & ~open) ? r.skip : next;
        if (inter)
            interact32_wave<TPM, POT, MIXED>(A, inter, r.gm, d0, d1, d2, dd, hp, a0, a1, a2, pot,
                                             nint);
        {
            // an opened leaf parent (with the prefilter): the children
            // cu + 1 .. skip - 1 are particles, walked here by the lanes that
            // opened the cube, and the cursor then moves past them; for any
            // other cube the run is empty (one path through the loop for the
            // accumulators either way)
            const bool run = TPM && desc && (cm & kRecLeafParent) && prefilter;
            const uint32_t end = run ? r.skip : cu + 1u;
            for (uint32_t base = cu + 1u; base < end; base += 64u) {
                const uint32_t k = min(64u, end - base);
                bool near = false;
                if ((uint32_t)lane < k) {
                    const Rec32 t = R[base + lane];
                    const float p0 = fmaf((float)wsub(t.cx_meta & -(1 << SH), Gr0), A.fu, t.dx);
                    const float p1 = fmaf((float)wsub(t.cy, Gr1), A.fu, t.dy);
                    const float p2 = fmaf((float)wsub(t.cz, Gr2), A.fu, t.dz);
                    const float g0 = fmaxf(fmaxf(lo0 - p0, p0 - hi0), 0.0f);
                    const float g1 = fmaxf(fmaxf(lo1 - p1, p1 - hi1), 0.0f);
                    const float g2 = fmaxf(fmaxf(lo2 - p2, p2 - hi2), 0.0f);
                    near = fmaf(g0, g0, fmaf(g1, g1, g2 * g2)) < A.fpf2;
                }
                for (uint64_t m = wave_mask(near); m; m &= m - 1) {
                    const uint32_t e = base + (uint32_t)__builtin_ctzll(m);
                    particle(uniform_rec32(R, e), e, desc);
                }
            }
            c = run ? r.skip : desc ? cu + 1u : r.skip;
        }
    }
    if (valid)
        store_result<float>(A, slot, a0, a1, a2, POT, pot, nint);
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Remap so that each XCD takes a contiguous eighth of the groups: a
// compact region of space whose part of the tree stays in that XCD's L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
    const uint32_t full = nb & ~7u;
    if (b >= full)
        return b;
    return (b & 7u) * (full >> 3) + (b >> 3);
}

__device__ __forceinline__ uint32_t wave_id() {
    return (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) >> 6;
}

// ---- lane-independent walks ------------------------------------------------
//
// Each lane walks its own targets: its cursor follows exactly the depth-first
// sequence of its own walk (open -> next entry, accept/discard -> skip), so
// the accumulation order per target is the same as in the shared-cursor walk
// and in a sequential walk.  Entries are gathered per lane.  A wavefront owns
// a chunk of 64 * K consecutive slots; lane l takes slots l, l + 64, ... of
// the chunk one after the other, which evens out the lanes' work while the
// wave's targets stay spatially close on the curve.
//
// FRONT (sparse active sets, too few targets to fill the chip one per lane):
// a wavefront walks ONE target (slot `wave`).  Phase 1 takes the walk's upper
// part breadth first: the lanes take the entries of the current frontier one
// each; an entry whose subtree holds at most kFrontLeaf entries is set aside
// undecided for phase 2, a larger one is decided as the sequential walk
// decides it (interacting where it interacts) and, when it is a cube that is
// opened, its children (found along the skip pointers) form the next
// frontier.  A cube with more than 8 children (coincident particles in a
// depth-21 cell) is set aside whole; phase 2 decides it again (the same
// decision: opened).  Phase 2: lane l walks the set-aside subtrees l, l + 64,
// ... depth first, so no lane walks more than kFrontLeaf entries per subtree
// while the work near the target is spread over the lanes.  Every
// interaction of the sequential walk happens once, in one lane, with the same
// operands; the 64 partial sums are added in a fixed tree order, so results
// are deterministic but rounded differently from the other variants
// (interaction counts are identical).  Phase 1 expands level by level while
// the frontier and the set-aside list together hold at most 512 entries
// (each level's frontier taken 64 entries at a time); then the rest of the
// frontier is set aside undecided.  `front`: 2048 words of LDS per wavefront
// (two frontiers of 512, 1024 set aside).
constexpr uint32_t kFrontWords = 2048;
constexpr uint32_t kFrontLeaf = 128;

// LDS of one wavefront in kernels that run either walk: the FP64 queue or
// the FRONT walk's frontiers.
union WaveLds {
    IQ64 q;
    uint32_t front[kFrontWords];
};

// Partial sums of a wavefront's lanes to lane 0, in a fixed tree order.
template <typename T>
__device__ __forceinline__ void lanes_to_first(T &a0, T &a1, T &a2, T &pot, uint32_t &nint,
                                               bool pot_on) {
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_down(a0, o);
        a1 += __shfl_down(a1, o);
        a2 += __shfl_down(a2, o);
        if (pot_on)
            pot += __shfl_down(pot, o);
        nint += __shfl_down(nint, o);
    }
}

// Phase 1 of the FRONT walk.  visit(e, r) decides entry e for the target
// (with its interaction) and returns true to descend; recs(e) loads record e.
// Leaves the final frontier in *cur (nf entries).
__device__ __forceinline__ bool is_particle(const Rec64 &r) {
    return (r.meta & kParticleFlag) != 0;
}
__device__ __forceinline__ bool is_particle(const Rec32 &r) {
    return (r.cx_meta & kRecParticle) != 0;
}

// Exclusive prefix over the wavefront's lanes of v, and the total.
__device__ __forceinline__ uint32_t lanes_prefix(uint32_t v, uint32_t &total) {
    const int lane = threadIdx.x & 63;
    uint32_t in = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(in, o);
        if (lane >= o)
            in += t;
    }
    total = __builtin_amdgcn_readfirstlane(__shfl(in, 63));
    return in - v;
}

// Phase 1 of the FRONT walk.  visit(e, r) decides entry e for the target
// (with its interaction) and returns true to descend.  Leaves the set-aside
// subtrees in *aside (na entries).
template <typename Rec, typename Visit>
__device__ __forceinline__ void expand_front(const Rec *__restrict__ R, uint32_t *front,
                                             uint32_t *&aside, uint32_t &na, Visit &visit) {
    const int lane = threadIdx.x & 63;
    uint32_t *cur = front, *nxt = front + 512;
    aside = front + 1024;
    na = 0u;
    if (lane == 0)
        cur[0] = 0u;  // the root
    uint32_t nf = 1u;
    wave_sync();
    // one level per pass, its frontier taken 64 entries at a time.  Bounds:
    // the next frontier holds at most 512 entries (an opened cube whose
    // children do not fit any more is set aside whole, to be opened again in
    // phase 2), and a level starts only while na + nf <= 512, so that the
    // set-aside list (1024 words) also takes the final frontier
    while (nf != 0u && na + nf <= 512u) {
        uint32_t nn = 0u;
        for (uint32_t b = 0; b < nf; b += 64u) {
            uint32_t nkid = 0u, nset = 0u, e = 0u;
            if (b + (uint32_t)lane < nf) {
                e = cur[b + lane];
                const Rec r = R[e];
                const uint32_t skip = r.skip;
                if (skip - e <= kFrontLeaf) {
                    nset = 1u;  // small subtree: walked whole in phase 2
                } else if (visit(e, r) && !is_particle(r)) {  // an opened cube
                    uint32_t c = e + 1u;
                    while (c < skip && nkid < 8u) {
                        nkid++;
                        c = R[c].skip;
                    }
                    if (c < skip) {  // more than 8 children: set aside whole
                        nkid = 0u;
                        nset = 1u;
                    }
                }
            }
            uint32_t tk, ts;
            uint32_t ok = lanes_prefix(nkid, tk);
            if (nn + tk > 512u) {  // the lanes whose children no longer fit
                if (nkid && nn + ok + nkid > 512u) {
                    nkid = 0u;
                    nset = 1u;
                }
                ok = lanes_prefix(nkid, tk);
            }
            const uint32_t os = lanes_prefix(nset, ts);
            if (nset)
                aside[na + os] = e;
            if (nkid) {
                uint32_t c = e + 1u;
                for (uint32_t k = 0; k < nkid; k++) {
                    nxt[nn + ok + k] = c;
                    c = R[c].skip;
                }
            }
            nn += tk;
            na += ts;
        }
        wave_sync();
        uint32_t *t = cur;
        cur = nxt;
        nxt = t;
        nf = nn;
    }
    // the rest of the frontier (at most 512 entries), set aside undecided
    for (uint32_t k = (uint32_t)lane; k < nf; k += 64u)
        aside[na + k] = cur[k];
    na += nf;
    wave_sync();
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED, bool FRONT = false>
__device__ __forceinline__ void walk_lanes64(const WalkArgs &A, uint32_t wave, uint32_t K,
                                             uint32_t *front = nullptr) {
    const int lane = threadIdx.x & 63;
    const uint32_t nu = load_count(A.nuniq);
    const uint32_t base = FRONT ? wave : wave * 64u * K;
    if (base >= nu)
        return;
    const uint32_t chunk_end = min(nu, base + 64u * K);
    const Rec64 *__restrict__ R = (const Rec64 *)A.rec;
    double x0 = 0.0, x1 = 0.0, x2 = 0.0, an = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0, pot = 0.0,
           hi = 0.0;
    uint32_t self = 0, nint = 0;
    auto start = [&](uint32_t sl) {
        const uint32_t s = coherent_ld(A.act + sl);
        x0 = A.ps[s];
        x1 = A.ps[A.n + s];
        x2 = A.ps[2 * (size_t)A.n + s];
        self = A.pe[s];
        if (OPEN == TPM_OPEN_REL)
            an = coherent_ld(A.anorm + A.perm[s]);
        if (MIXED)
            hi = A.hs[s];
        a0 = a1 = a2 = pot = 0.0;
        nint = 0;
    };
    // entry e for this lane's target: the decision and the interaction, as
    // in a sequential walk; true: descend into e
    auto visit = [&](uint32_t e, const Rec64 &r) -> bool {
        const double he = MIXED ? ((const double *)A.eh)[e] : 0.0;
        const double d0 = wrap64<PER>(r.com[0] - x0, A.box, A.half);
        const double d1 = wrap64<PER>(r.com[1] - x1, A.box, A.half);
        const double d2 = wrap64<PER>(r.com[2] - x2, A.box, A.half);
        const double dd = fma(d0, d0, fma(d1, d1, d2 * d2));
        bool inter, step_in;
        if (r.meta & kParticleFlag) {
            step_in = true;
            inter = e != self && (!TPM || dd < A.rc2);
        } else {
            const double L = ldexp(A.L, -(int)(r.meta & 0xffu));
            const double c0 = wrap64<PER>(r.cen[0] - x0, A.box, A.half);
            const double c1 = wrap64<PER>(r.cen[1] - x1, A.box, A.half);
            const double c2 = wrap64<PER>(r.cen[2] - x2, A.box, A.half);
            bool discard = false;
            if (TPM) {
                const double hl = 0.5 * L;
                double e0 = fabs(c0) - hl, e1 = fabs(c1) - hl, e2 = fabs(c2) - hl;
                e0 = e0 > 0.0 ? e0 : 0.0;
                e1 = e1 > 0.0 ? e1 : 0.0;
                e2 = e2 > 0.0 ? e2 : 0.0;
                discard = fma(e0, e0, fma(e1, e1, e2 * e2)) > A.rc2;
            }
            bool open = false;
            if (!discard) {
                if (OPEN == TPM_OPEN_BH)
                    open = (L * L) > A.theta2 * dd;
                else
                    open = (A.G * r.mass) * (L * L) > (A.alpha * an) * (dd * dd);
                const double lim = 0.6 * L;
                if (fabs(c0) < lim && fabs(c1) < lim && fabs(c2) < lim)
                    open = true;
                if (MIXED && hi < he && dd < he * he)
                    open = true;
            }
            step_in = open;
            inter = !discard && !open;
        }
        if (inter) {
            interact64<TPM, POT, MIXED>(A, r.mass, d0, d1, d2, dd, hi > he ? hi : he, a0, a1,
                                        a2, pot);
            nint++;
        }
        return step_in;
    };
    if constexpr (!FRONT) {
        uint32_t slot = base + lane;
        bool live = slot < chunk_end;
        uint32_t e = 0;
        if (live)
            start(slot);
        while (__ballot(live)) {
            if (live) {
                const Rec64 r = R[e];
                e = visit(e, r) ? e + 1u : r.skip;
                if (e >= A.E) {
                    store_result<double>(A, slot, a0, a1, a2, POT, pot, nint);
                    slot += 64u;
                    live = slot < chunk_end;
                    e = 0;
                    if (live)
                        start(slot);
                }
            }
        }
    } else {
        start(base);
        uint32_t *cur, nf;  // the set-aside subtrees
        expand_front<Rec64>(R, front, cur, nf, visit);
        // phase 2: the set-aside subtrees lane, lane + 64, ...
        uint32_t k = (uint32_t)lane;
        bool live = k < nf;
        uint32_t e = 0, end = 0;
        if (live) {
            e = cur[k];
            end = R[e].skip;
        }
        while (__ballot(live)) {
            if (live) {
                const Rec64 r = R[e];
                e = visit(e, r) ? e + 1u : r.skip;
                if (e >= end) {
                    k += 64u;
                    live = k < nf;
                    if (live) {
                        e = cur[k];
                        end = R[e].skip;
                    }
                }
            }
        }
        lanes_to_first(a0, a1, a2, pot, nint, POT);
        if (lane == 0)
            store_result<double>(A, base, a0, a1, a2, POT, pot, nint);
    }
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED, bool FRONT = false>
__device__ __forceinline__ void walk_lanes32(const WalkArgs &A, uint32_t wave, uint32_t K,
                                             uint32_t *front = nullptr) {
    const int lane = threadIdx.x & 63;
    const uint32_t nu = load_count(A.nuniq);
    const uint32_t base = FRONT ? wave : wave * 64u * K;
    if (base >= nu)
        return;
    const uint32_t chunk_end = min(nu, base + 64u * K);
    const Rec32 *__restrict__ R = (const Rec32 *)A.rec;
    const double len21 = ldexp(A.L, -kMaxLevel);
    constexpr int SH = PER ? kRecShiftPer : kRecShiftIso;
    int32_t G0 = 0, G1 = 0, G2 = 0;
    float xr0 = 0.f, xr1 = 0.f, xr2 = 0.f, alpha_an = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f,
          pot = 0.f, hi = 0.f;
    uint32_t self = 0, nint = 0;
    auto start = [&](uint32_t sl) {
        const uint32_t s = coherent_ld(A.act + sl);
        const uint64_t qq = A.qs[s];
        const uint32_t q0 = (uint32_t)(qq >> 42) & 0x1fffffu,
                       q1 = (uint32_t)(qq >> 21) & 0x1fffffu, q2 = (uint32_t)qq & 0x1fffffu;
        G0 = (int32_t)((2u * q0 + 1u) << SH);
        G1 = (int32_t)((2u * q1 + 1u) << SH);
        G2 = (int32_t)((2u * q2 + 1u) << SH);
        xr0 = (float)(A.ps[s] - (A.x0[0] + ((double)q0 + 0.5) * len21));
        xr1 = (float)(A.ps[A.n + s] - (A.x0[1] + ((double)q1 + 0.5) * len21));
        xr2 = (float)(A.ps[2 * (size_t)A.n + s] - (A.x0[2] + ((double)q2 + 0.5) * len21));
        self = A.pe[s];
        alpha_an = 0.f;
        if (OPEN == TPM_OPEN_REL)
            alpha_an = A.falpha * (float)coherent_ld(A.anorm + A.perm[s]);
        if (MIXED)
            hi = (float)A.hs[s];
        a0 = a1 = a2 = pot = 0.f;
        nint = 0;
    };
    // entry e for this lane's target: the decision and the interaction, as
    // in a sequential walk; true: descend into e
    auto visit = [&](uint32_t e, const Rec32 &r) -> bool {
        const float he = MIXED ? ((const float *)A.eh)[e] : 0.0f;
        const int32_t cm = r.cx_meta;
        const float c0 = fmaf((float)wsub(cm & -(1 << SH), G0), A.fu, -xr0);
        const float c1 = fmaf((float)wsub(r.cy, G1), A.fu, -xr1);
        const float c2 = fmaf((float)wsub(r.cz, G2), A.fu, -xr2);
        const float d0 = c0 + r.dx, d1 = c1 + r.dy, d2 = c2 + r.dz;
        const float dd = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        const bool part = (cm & kRecParticle) != 0;
        const float L = __builtin_amdgcn_ldexpf(A.fL, -(cm & kRecLevel));
        bool discard = false;
        if (TPM) {
            const float hl = 0.5f * L;
            const float e0 = fmaxf(fabsf(c0) - hl, 0.0f);
            const float e1 = fmaxf(fabsf(c1) - hl, 0.0f);
            const float e2 = fmaxf(fabsf(c2) - hl, 0.0f);
            discard = !part && fmaf(e0, e0, fmaf(e1, e1, e2 * e2)) > A.frc2;
        }
        const float L2 = L * L;
        bool crit;
        if (OPEN == TPM_OPEN_BH)
            crit = L2 > A.ftheta2 * dd;
        else
            crit = r.gm * L2 > alpha_an * (dd * dd);
        const float lim = 0.6f * L;
        const bool box = fabsf(c0) < lim && fabsf(c1) < lim && fabsf(c2) < lim;
        const bool soft_open = MIXED && hi < he && dd < he * he;
        const bool open = !part && !discard && (crit || box || soft_open);
        const bool inter = part ? (e != self && (!TPM || dd < A.frc2)) : (!discard && !open);
        if (inter) {
            interact32<TPM, POT, MIXED>(A, r.gm, d0, d1, d2, dd, hi > he ? hi : he, a0, a1, a2,
                                        pot);
            nint++;
        }
        return part || open;
    };
    if constexpr (!FRONT) {
        uint32_t slot = base + lane;
        bool live = slot < chunk_end;
        uint32_t e = 0;
        if (live)
            start(slot);
        while (__ballot(live)) {
            if (live) {
                const Rec32 r = R[e];
                e = visit(e, r) ? e + 1u : r.skip;
                if (e >= A.E) {
                    store_result<float>(A, slot, a0, a1, a2, POT, pot, nint);
                    slot += 64u;
                    live = slot < chunk_end;
                    e = 0;
                    if (live)
                        start(slot);
                }
            }
        }
    } else {
        start(base);
        uint32_t *cur, nf;  // the set-aside subtrees
        expand_front<Rec32>(R, front, cur, nf, visit);
        // phase 2: the set-aside subtrees lane, lane + 64, ...
        uint32_t k = (uint32_t)lane;
        bool live = k < nf;
        uint32_t e = 0, end = 0;
        if (live) {
            e = cur[k];
            end = R[e].skip;
        }
        while (__ballot(live)) {
            if (live) {
                const Rec32 r = R[e];
                e = visit(e, r) ? e + 1u : r.skip;
                if (e >= end) {
                    k += 64u;
                    live = k < nf;
                    if (live) {
                        e = cur[k];
                        end = R[e].skip;
                    }
                }
            }
        }
        lanes_to_first(a0, a1, a2, pot, nint, POT);
        if (lane == 0)
            store_result<float>(A, base, a0, a1, a2, POT, pot, nint);
    }
}

// Host side (walk.hip): the walk arguments of one call from the context and
// its working memory, and the choice of the lane-independent walk.
void fill_args(tpm_ctx *c, const double *anorm, const Work &w, WalkArgs &A);
// Walk variant for an active set of n_act: shared cursor (64 targets per
// wavefront), independent lanes, one wavefront per target (FRONT), or the
// shared cursor or lanes as a census of the groups' extents decides on the
// device (the two give the same results).
enum Variant : uint32_t { kGroupWalk = 0, kLaneWalk = 1, kSplitWalk = 2, kGroupOrLanes = 3 };
// The walk for an active set of n_act targets.  census_ok: kGroupOrLanes may
// be returned (single-system launches; the batch and the resident server
// take the lanes there).
Variant walk_variant(const tpm_ctx *c, int64_t n_act, bool census_ok = false);

// Whether the targets of group `wave` (its 64 slots; the caller has checked
// that the group is not empty) lie within a box of side sqrt(A.group_ext2)
// (nearest images in a periodic box), so that a shared cursor walks little
// more than each target's own walk.  Wavefront-uniform.
template <bool PER>
__device__ __forceinline__ bool group_compact(const WalkArgs &A, uint32_t wave) {
    const int lane = threadIdx.x & 63;
    const uint32_t nu = load_count(A.nuniq);
    const uint32_t slot = wave * 64u + lane;
    const uint32_t s = coherent_ld(A.act + (slot < nu ? slot : wave * 64u));
    double lo[3], hi[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double x = A.ps[(size_t)a * A.n + s];
        const double x0 = __shfl(x, 0);
        double d = x - x0;
        if (PER)
            d = fabs(d) > A.half ? d - copysign(A.box, d) : d;
        lo[a] = hi[a] = d;
    }
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            lo[a] = fmin(lo[a], __shfl_xor(lo[a], o));
            hi[a] = fmax(hi[a], __shfl_xor(hi[a], o));
        }
    }
    double e = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++)
        e = fmax(e, hi[a] - lo[a]);
    return __builtin_amdgcn_readfirstlane((int)(e * e <= A.group_ext2)) != 0;
}

}  // namespace wk
}  // namespace tpm
