// Tree walk for gfx950 (Sec. 3.1 opening criteria and box rule, Sec. 3.2
// spline softening, Sec. 3.4 short-range truncation and cutoff).
//
// One wavefront walks the depth-first entry list for 64 active particles that
// are adjacent on the Peano-Hilbert curve.  The wave keeps ONE cursor: every
// lane owns a "next" index (the entry its own depth-first walk needs next,
// or an earlier one while it is inside a cube it opened); lanes whose next
// is at or before the cursor evaluate the entry, lanes that accepted or
// discarded an ancestor sit out until the cursor reaches their next.  The
// cursor descends (c + 1) when any lane opens the entry and otherwise jumps
// to the entry's skip pointer -- the next entry of some lane's walk, since
// subtrees nest.  Entries are read with wave-uniform (scalar) loads, so each
// lane sees exactly the entry sequence of its own recursive walk, in order:
// the FP64 path reproduces a sequential FP64 walk bit for bit apart from the
// last bits of erfc/exp.  With a cutoff, entries that can interact with no
// lane of the wavefront are skipped (particles of opened leaf parents beyond
// r_cut of the group's bounding box, cubes every lane discards).
#include "tpm_internal.h"
#include "erfc_poly.h"

#include <algorithm>
#include <new>
#include <string>
#include <vector>

namespace tpm {
namespace {

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
    void *res;
    void *rpot;
    uint32_t *rnint;
    // individual softening (Sec. 3.2): spline support per target (curve
    // order) and the largest support per entry (double, or float for FP32)
    const double *hs;
    const void *eh;
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
    const uint32_t nu = *A.nuniq;
    if (wave * 64u >= nu)
        return;  // whole wavefront
    const uint32_t slot = wave * 64u + lane;
    const bool valid = slot < nu;
    const uint32_t s = A.act[valid ? slot : wave * 64u];
    const double x0 = A.ps[s], x1 = A.ps[A.n + s], x2 = A.ps[2 * (size_t)A.n + s];
    const uint32_t self = A.pe[s];
    double an = 0.0;
    if (OPEN == TPM_OPEN_REL)
        an = A.anorm[A.perm[s]];
    const double alpha_an = A.alpha * an;
    const double hi = MIXED ? A.hs[s] : 0.0;  // the target's own support
    // the lane's walk stands at the cursor when next <= cursor (next moves
    // to the skip pointer only when the lane accepts or discards a cube)
    uint32_t next = valid ? 0u : 0xffffffffu;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, pot = 0.0;
    uint32_t nint = 0;
    const Rec64 *__restrict__ R = (const Rec64 *)A.rec;

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
        const double he = MIXED ? ((const double *)A.eh)[e] : 0.0;
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
        const double he = MIXED ? ((const double *)A.eh)[cu] : 0.0;
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
        if (TPM && desc && (r.meta & kLeafParentFlag) && prefilter) {
            const uint32_t end = r.skip;
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
            c = end;
        } else {
            c = desc ? cu + 1u : r.skip;
        }
    }
    if (TPM && qn)
        flush(qn, ns);
    if (valid) {
        double *res = (double *)A.res;
        res[slot] = a0;
        res[A.n + slot] = a1;
        res[2 * (size_t)A.n + slot] = a2;
        if (POT)
            ((double *)A.rpot)[slot] = pot;
        A.rnint[slot] = nint;
    }
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
    const uint32_t nu = *A.nuniq;
    if (wave * 64u >= nu)
        return;
    const uint32_t slot = wave * 64u + lane;
    const bool valid = slot < nu;
    const uint32_t s = A.act[valid ? slot : wave * 64u];
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
        an = (float)A.anorm[A.perm[s]];
    const float alpha_an = A.falpha * an;
    const float hi = MIXED ? (float)A.hs[s] : 0.0f;
    // A lane's walk stands at the cursor when next <= cursor: next is only
    // moved (to the skip pointer) when the lane accepts or discards a cube,
    // so a lane that opened a cube follows the cursor through its subtree,
    // particles included, without per-entry bookkeeping.
    uint32_t next = valid ? 0u : 0xffffffffu;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, pot = 0.0f;
    uint32_t nint = 0;
    const Rec32 *__restrict__ R = (const Rec32 *)A.rec;

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
        const float he = MIXED ? ((const float *)A.eh)[e] : 0.0f;
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
        const Rec32 r = R[cu];
        const uint64_t mine = wave_mask(next <= cu);
        const int32_t cm = r.cx_meta;
        if (cm & kRecParticle) {
            particle(r, cu, mine);
            c = cu + 1u;
            continue;
        }
        const float he = MIXED ? ((const float *)A.eh)[cu] : 0.0f;
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
        if (TPM && desc && (cm & kRecLeafParent) && prefilter) {
            // the children cu + 1 .. skip - 1 are particles, walked by the
            // lanes that opened the cube; the cursor then moves past them
            const uint32_t end = r.skip;
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
                    particle(R[e], e, desc);
                }
            }
            c = end;
        } else {
            c = desc ? cu + 1u : r.skip;
        }
    }
    if (valid) {
        float *res = (float *)A.res;
        res[slot] = a0;
        res[A.n + slot] = a1;
        res[2 * (size_t)A.n + slot] = a2;
        if (POT)
            ((float *)A.rpot)[slot] = pot;
        A.rnint[slot] = nint;
    }
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

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk64(const WalkArgs A) {
    IQ64 *Q = nullptr;  // the interaction queue, with a cutoff
    if constexpr (TPM) {
        __shared__ IQ64 q[kBlock / 64];
        Q = &q[threadIdx.x >> 6];
    }
    walk_group64<PER, TPM, OPEN, POT, MIXED>(A, wave_id(), Q);
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk32(const WalkArgs A) {
    walk_group32<PER, TPM, OPEN, POT, MIXED>(A, wave_id());
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

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__device__ __forceinline__ void walk_lanes64(const WalkArgs &A, uint32_t wave, uint32_t K) {
    const int lane = threadIdx.x & 63;
    const uint32_t nu = *A.nuniq;
    const uint32_t base = wave * 64u * K;
    if (base >= nu)
        return;
    const uint32_t chunk_end = min(nu, base + 64u * K);
    const Rec64 *__restrict__ R = (const Rec64 *)A.rec;
    uint32_t slot = base + lane;
    bool live = slot < chunk_end;
    double x0 = 0.0, x1 = 0.0, x2 = 0.0, an = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0, pot = 0.0,
           hi = 0.0;
    uint32_t self = 0, nint = 0, e = 0;
    auto start = [&](uint32_t sl) {
        const uint32_t s = A.act[sl];
        x0 = A.ps[s];
        x1 = A.ps[A.n + s];
        x2 = A.ps[2 * (size_t)A.n + s];
        self = A.pe[s];
        if (OPEN == TPM_OPEN_REL)
            an = A.anorm[A.perm[s]];
        if (MIXED)
            hi = A.hs[s];
        a0 = a1 = a2 = pot = 0.0;
        nint = 0;
        e = 0;
    };
    if (live)
        start(slot);
    while (__ballot(live)) {
        if (live) {
            const Rec64 r = R[e];
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
            e = step_in ? e + 1u : r.skip;
            if (e >= A.E) {
                double *res = (double *)A.res;
                res[slot] = a0;
                res[A.n + slot] = a1;
                res[2 * (size_t)A.n + slot] = a2;
                if (POT)
                    ((double *)A.rpot)[slot] = pot;
                A.rnint[slot] = nint;
                slot += 64u;
                live = slot < chunk_end;
                if (live)
                    start(slot);
            }
        }
    }
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__device__ __forceinline__ void walk_lanes32(const WalkArgs &A, uint32_t wave, uint32_t K) {
    const int lane = threadIdx.x & 63;
    const uint32_t nu = *A.nuniq;
    const uint32_t base = wave * 64u * K;
    if (base >= nu)
        return;
    const uint32_t chunk_end = min(nu, base + 64u * K);
    const Rec32 *__restrict__ R = (const Rec32 *)A.rec;
    const double len21 = ldexp(A.L, -kMaxLevel);
    uint32_t slot = base + lane;
    bool live = slot < chunk_end;
    constexpr int SH = PER ? kRecShiftPer : kRecShiftIso;
    int32_t G0 = 0, G1 = 0, G2 = 0;
    float xr0 = 0.f, xr1 = 0.f, xr2 = 0.f, alpha_an = 0.f, a0 = 0.f, a1 = 0.f, a2 = 0.f,
          pot = 0.f, hi = 0.f;
    uint32_t self = 0, nint = 0, e = 0;
    auto start = [&](uint32_t sl) {
        const uint32_t s = A.act[sl];
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
            alpha_an = A.falpha * (float)A.anorm[A.perm[s]];
        if (MIXED)
            hi = (float)A.hs[s];
        a0 = a1 = a2 = pot = 0.f;
        nint = 0;
        e = 0;
    };
    if (live)
        start(slot);
    while (__ballot(live)) {
        if (live) {
            const Rec32 r = R[e];
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
                interact32<TPM, POT, MIXED>(A, r.gm, d0, d1, d2, dd, hi > he ? hi : he, a0, a1,
                                            a2, pot);
                nint++;
            }
            e = (part || open) ? e + 1u : r.skip;
            if (e >= A.E) {
                float *res = (float *)A.res;
                res[slot] = a0;
                res[A.n + slot] = a1;
                res[2 * (size_t)A.n + slot] = a2;
                if (POT)
                    ((float *)A.rpot)[slot] = pot;
                A.rnint[slot] = nint;
                slot += 64u;
                live = slot < chunk_end;
                if (live)
                    start(slot);
            }
        }
    }
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk64i(const WalkArgs A, uint32_t K) {
    walk_lanes64<PER, TPM, OPEN, POT, MIXED>(A, wave_id(), K);
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk32i(const WalkArgs A, uint32_t K) {
    walk_lanes32<PER, TPM, OPEN, POT, MIXED>(A, wave_id(), K);
}

// ---- active set -> slots in curve order --------------------------------------

__global__ __launch_bounds__(kBlock) void k_mark(const int32_t *__restrict__ idx, int64_t n_act,
                                                 int64_t n, const int32_t *__restrict__ rank,
                                                 uint32_t *__restrict__ mark, uint32_t epoch) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_act)
        return;
    const int32_t i = idx[k];
    if (i < 0 || (int64_t)i >= n)
        return;  // reported by the output kernel
    mark[rank[i]] = epoch;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_output(
    const int32_t *__restrict__ idx, int64_t n_act, int64_t n, const int32_t *__restrict__ rank,
    const uint32_t *__restrict__ slot, const T *__restrict__ res, const T *__restrict__ rpot,
    const uint32_t *__restrict__ rnint, T *__restrict__ acc, T *__restrict__ pot,
    uint32_t *__restrict__ nint, uint32_t *__restrict__ err) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_act)
        return;
    const int32_t i = idx[k];
    if (i < 0 || (int64_t)i >= n) {
        const T nan = (T)NAN;
        acc[k] = nan;
        acc[n_act + k] = nan;
        acc[2 * n_act + k] = nan;
        if (pot)
            pot[k] = nan;
        if (nint)
            nint[k] = 0xffffffffu;
        atomicOr(err, 1u);
        return;
    }
    const uint32_t sl = slot[rank[i]];
    acc[k] = res[sl];
    acc[n_act + k] = res[n + sl];
    acc[2 * n_act + k] = res[2 * n + sl];
    if (pot)
        pot[k] = rpot[sl];
    if (nint)
        nint[k] = rnint[sl];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_accel_norm(const int32_t *__restrict__ idx,
                                                       int64_t n_act, int64_t n,
                                                       const T *__restrict__ a,
                                                       const T *__restrict__ b,
                                                       double *__restrict__ out,
                                                       uint32_t *__restrict__ err) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_act)
        return;
    const int32_t i = idx[k];
    if (i < 0 || (int64_t)i >= n) {
        atomicOr(err, 1u);
        return;
    }
    double v[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        v[d] = (double)a[d * n_act + k];
        if (b)
            v[d] += (double)b[d * n_act + k];
    }
    out[i] = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

struct Launch {
    bool fp32;
    bool lanes;       // lane-independent walk
    uint32_t K;       // slots per lane (lane-independent walk)
    unsigned blocks;
};

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
void launch_walk(const WalkArgs &A, const Launch &L, hipStream_t st) {
    if (L.lanes) {
        if (L.fp32)
            k_walk32i<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A, L.K);
        else
            k_walk64i<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A, L.K);
    } else {
        if (L.fp32)
            k_walk32<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A);
        else
            k_walk64<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A);
    }
}

template <bool PER, bool TPM, bool MIXED>
void dispatch_open_pot(const WalkArgs &A, const Launch &L, int open, bool pot, hipStream_t st) {
    if (open == TPM_OPEN_BH) {
        if (pot)
            launch_walk<PER, TPM, TPM_OPEN_BH, true, MIXED>(A, L, st);
        else
            launch_walk<PER, TPM, TPM_OPEN_BH, false, MIXED>(A, L, st);
    } else {
        if (pot)
            launch_walk<PER, TPM, TPM_OPEN_REL, true, MIXED>(A, L, st);
        else
            launch_walk<PER, TPM, TPM_OPEN_REL, false, MIXED>(A, L, st);
    }
}

template <bool PER, bool TPM>
void dispatch_mixed(const WalkArgs &A, const Launch &L, int open, bool pot, bool mixed,
                    hipStream_t st) {
    if (mixed)
        dispatch_open_pot<PER, TPM, true>(A, L, open, pot, st);
    else
        dispatch_open_pot<PER, TPM, false>(A, L, open, pot, st);
}

}  // namespace

int accel_norm(tpm_ctx *c, int64_t n_act, const int32_t *idx, const void *a, const void *b,
               double *out) {
    if (n_act == 0)
        return TPM_OK;
    const unsigned g = grid_for(n_act, kBlock);
    if (c->P.precision == TPM_FP32)
        k_accel_norm<float><<<g, kBlock, 0, c->stream>>>(idx, n_act, c->n, (const float *)a,
                                                         (const float *)b, out,
                                                         (uint32_t *)c->err_flag.p);
    else
        k_accel_norm<double><<<g, kBlock, 0, c->stream>>>(idx, n_act, c->n, (const double *)a,
                                                          (const double *)b, out,
                                                          (uint32_t *)c->err_flag.p);
    TPM_LAUNCHED(c, "k_accel_norm");
    return TPM_OK;
}

int work_of_ctx(tpm_ctx *c, bool results, Work &w) {
    const int64_t n = c->n;
    TPM_TRY(ensure(c, c->mark, (size_t)n * 4));
    TPM_TRY(ensure(c, c->act, (size_t)n * 4));
    TPM_TRY(ensure(c, c->slot, (size_t)n * 4));
    TPM_TRY(ensure(c, c->scan_tmp, (size_t)compaction_tiles(n) * 4));
    if (results) {
        const size_t esz = c->P.precision == TPM_FP32 ? 4 : 8;
        TPM_TRY(ensure(c, c->res, (size_t)3 * n * esz));
        TPM_TRY(ensure(c, c->rpot, (size_t)n * esz));
        TPM_TRY(ensure(c, c->rnint, (size_t)n * 4));
    }
    w = Work{};
    w.mark = (uint32_t *)c->mark.p;
    w.clear = false;
    if (++c->epoch == 0 || c->epoch == 1) {  // fresh or wrapped: clear the marks
        w.clear = true;
        c->epoch = 1;
    }
    w.epoch = c->epoch;
    w.act = (uint32_t *)c->act.p;
    w.slot = (uint32_t *)c->slot.p;
    w.counts = (uint32_t *)c->scan_tmp.p;
    w.nuniq = (uint32_t *)c->counters.p + 40;
    w.res = c->res.p;
    w.rpot = c->rpot.p;
    w.rnint = (uint32_t *)c->rnint.p;
    return TPM_OK;
}

int select_active_into(tpm_ctx *c, int64_t n_act, const int32_t *idx, const Work &w) {
    const int64_t n = c->n;
    hipStream_t st = c->stream;
    if (w.clear)
        TPM_TRY(fill_u32(c, w.mark, 0u, n));
    if (n_act > 0) {
        k_mark<<<grid_for(n_act, kBlock), kBlock, 0, st>>>(idx, n_act, n,
                                                           (const int32_t *)c->rank.p, w.mark,
                                                           w.epoch);
        TPM_LAUNCHED(c, "k_mark");
    }
    return compact_marked(c, w.mark, w.epoch, n, w.act, w.slot, w.nuniq, w.counts);
}

int select_active(tpm_ctx *c, int64_t n_act, const int32_t *idx) {
    Work w;
    TPM_TRY(work_of_ctx(c, false, w));
    return select_active_into(c, n_act, idx, w);
}

// Walk variant (both give identical results): independent lanes for sparse
// active sets, whose groups are too spread out for a shared cursor (it would
// visit the union of their walks), and for FP64 TreePM of isolated systems
// (their outer groups span many cutoff radii, and the FP64 interaction is
// costly); the shared cursor otherwise (measured on the 128^3 box and the
// Hernquist sphere).
static bool use_lanes(const tpm_ctx *c, int64_t n_act) {
    if (c->walk_mode != 0)
        return c->walk_mode == 2;
    const bool fp64_iso_tpm =
        c->P.precision == TPM_FP64 && c->P.pm_grid > 0 && !c->P.periodic;
    return fp64_iso_tpm || 4 * n_act < c->n;
}

static void fill_args(tpm_ctx *c, const double *anorm, const Work &w, WalkArgs &A) {
    const tpm_params &P = c->P;
    const int64_t n = c->n;
    const bool fp32 = P.precision == TPM_FP32;
    A.rec = fp32 ? c->rec32.p : c->rec64.p;
    A.E = (uint32_t)c->E;
    A.n = (uint32_t)n;
    A.act = w.act;
    A.nuniq = w.nuniq;
    A.ps = (const double *)c->ps.p;
    A.qs = (const uint64_t *)c->qs.p;
    A.pe = (const uint32_t *)c->pe.p;
    A.perm = (const int32_t *)c->perm.p;
    A.anorm = anorm;
    for (int a = 0; a < 3; a++)
        A.x0[a] = c->frame_host.x0[a];
    A.L = c->frame_host.L;
    A.box = P.periodic ? P.box_size : 0.0;
    A.half = 0.5 * A.box;
    const bool tpm_on = P.pm_grid > 0;
    // split scale r_s = asmth x mesh spacing; the isolated mesh spans the
    // root cube in pm_grid - 4 cells
    double rs = 1.0;
    if (tpm_on)
        rs = P.periodic ? P.asmth * P.box_size / P.pm_grid
                        : P.asmth * (c->frame_host.L / (P.pm_grid - 4));
    const double rcut = tpm_on ? P.rcut * rs : 0.0;
    A.G = P.G;
    A.theta2 = P.theta * P.theta;
    A.alpha = P.alpha;
    A.h = 2.8 * P.eps;
    A.hinv = 1.0 / A.h;
    A.h3inv = A.hinv * A.hinv * A.hinv;
    A.rc2 = rcut * rcut;
    A.inv2rs = 0.5 / rs;
    // unit of the shifted integer coordinates of the FP32 records
    A.fu = (float)ldexp(A.L, -22 - (P.periodic ? kRecShiftPer : kRecShiftIso));
    A.fL = (float)A.L;
    A.ftheta2 = (float)A.theta2;
    A.falpha = (float)A.alpha;
    A.fh2 = (float)(A.h * A.h);
    A.fhinv = (float)A.hinv;
    A.fh3inv = (float)A.h3inv;
    A.frc2 = (float)A.rc2;
    {
        // the prefilter's rounding (positions relative to a group's reference
        // cell, all below L_root in magnitude) stays far below L_root 2^-16
        const double tol = ldexp(A.L, -16);
        A.fpf2 = (float)((rcut + tol) * (rcut + tol));
        A.fpf_ext = P.periodic ? (float)(0.5 * P.box_size - rcut - 2.0 * tol) : 3.0e38f;
        const double tol64 = ldexp(A.L, -40);
        A.pf2 = (rcut + tol64) * (rcut + tol64);
        A.pf_ext = P.periodic ? 0.5 * P.box_size - rcut - 2.0 * tol64 : 1.0e300;
    }
    A.finv2rs = (float)A.inv2rs;
    A.fgexp = (float)(-1.4426950408889634 * A.inv2rs * A.inv2rs);
    A.res = w.res;
    A.rpot = w.rpot;
    A.rnint = w.rnint;
    A.L2r = A.L * A.L;
    A.limr = 0.6 * A.L;
    A.hlr = 0.5 * A.L;
    A.hs = c->mixed ? (const double *)c->hs.p : nullptr;
    A.eh = c->mixed ? (fp32 ? c->eh32.p : c->eh64.p) : nullptr;
    A.fL2r = A.fL * A.fL;
    A.flimr = 0.6f * A.fL;
    A.fhlr = 0.5f * A.fL;
}

int forces(tpm_ctx *c, int32_t opening, int64_t n_act, const int32_t *idx, const double *anorm,
           void *acc, void *pot, uint32_t *nint) {
    if (n_act == 0)
        return TPM_OK;
    Work w;
    TPM_TRY(work_of_ctx(c, true, w));
    return forces_into(c, opening, n_act, idx, anorm, acc, pot, nint, w, true);
}

int forces_into(tpm_ctx *c, int32_t opening, int64_t n_act, const int32_t *idx,
                const double *anorm, void *acc, void *pot, uint32_t *nint, const Work &w,
                bool timed) {
    const tpm_params &P = c->P;
    const int64_t n = c->n;
    hipStream_t st = c->stream;
    const bool fp32 = P.precision == TPM_FP32;
    if (n_act == 0)
        return TPM_OK;
    TPM_TRY(select_active_into(c, n_act, idx, w));

    WalkArgs A{};
    fill_args(c, anorm, w, A);
    const bool tpm_on = P.pm_grid > 0;
    const int64_t groups = (std::min<int64_t>(n_act, n) + 63) / 64;
    Launch LA;
    LA.fp32 = fp32;
    // lane-independent walks pay off where the interaction is expensive and
    // the wavefront's union of cutoff spheres is large: FP64 with TreePM
    LA.lanes = use_lanes(c, n_act);
    LA.K = 1;
    if (LA.lanes) {
        // several slots per lane once there are enough wavefronts to fill the chip
        const int64_t slots_per_chip = 256 * 4 * 8;
        while (LA.K < 8 && groups / (2 * LA.K) >= 2 * slots_per_chip)
            LA.K *= 2;
    }
    const int64_t waves = (groups + LA.K - 1) / LA.K;
    LA.blocks = (unsigned)((waves + 3) / 4);
    const bool want_pot = pot != nullptr && P.want_potential;
    const int tkind = opening == TPM_OPEN_REL ? TPM_TIMER_WALK_REL : TPM_TIMER_WALK;
    if (timed)
        TPM_TRY(timer_begin(c, tkind));
    // periodic boxes always carry the mesh (validated at creation)
    if (P.periodic)
        dispatch_mixed<true, true>(A, LA, opening, want_pot, c->mixed, st);
    else if (tpm_on)
        dispatch_mixed<false, true>(A, LA, opening, want_pot, c->mixed, st);
    else
        dispatch_mixed<false, false>(A, LA, opening, want_pot, c->mixed, st);
    TPM_LAUNCHED(c, "k_walk");
    if (timed)
        TPM_TRY(timer_end(c, tkind));
    const unsigned ob = grid_for(n_act, kBlock);
    if (fp32)
        k_output<float><<<ob, kBlock, 0, st>>>(
            idx, n_act, n, (const int32_t *)c->rank.p, w.slot, (const float *)w.res,
            (const float *)w.rpot, w.rnint, (float *)acc, want_pot ? (float *)pot : nullptr,
            nint, (uint32_t *)c->err_flag.p);
    else
        k_output<double><<<ob, kBlock, 0, st>>>(
            idx, n_act, n, (const int32_t *)c->rank.p, w.slot, (const double *)w.res,
            (const double *)w.rpot, w.rnint, (double *)acc, want_pot ? (double *)pot : nullptr,
            nint, (uint32_t *)c->err_flag.p);
    TPM_LAUNCHED(c, "k_output");
    return TPM_OK;
}

}  // namespace tpm

// ---- batched walks over many systems (continuous batching) -------------------
//
// One persistent launch per precision walks the groups of every request staged
// in a batch: wavefronts pop work items (one group of one request) from a
// device counter until the finite item list is exhausted.  A work item runs
// the same per-group code as a single-system launch, so each result is the
// same whether its request runs alone or in a mix.

namespace tpm {
namespace {

struct BatchReq {
    WalkArgs A;
    uint32_t variant;  // bit 0 relative criterion, 1 TreePM, 2 lanes, 3 periodic,
                       // 4 individual softening
    uint32_t first;    // first work item of the request
};

template <bool FP32, bool PER, bool TPM, int OPEN, bool MIXED>
__device__ __forceinline__ void batch_group(const WalkArgs &A, uint32_t g, bool lanes, IQ64 *Q) {
    if constexpr (FP32) {
        if (lanes)
            walk_lanes32<PER, TPM, OPEN, false, MIXED>(A, g, 1u);
        else
            walk_group32<PER, TPM, OPEN, false, MIXED>(A, g);
    } else {
        if (lanes)
            walk_lanes64<PER, TPM, OPEN, false, MIXED>(A, g, 1u);
        else
            walk_group64<PER, TPM, OPEN, false, MIXED>(A, g, Q);
    }
}

template <bool FP32, int OPEN, bool MIXED>
__device__ __forceinline__ void batch_geometry(const BatchReq &R, uint32_t g, bool lanes,
                                               IQ64 *Q) {
    if (R.variant & 8u)  // periodic box (always with the mesh)
        batch_group<FP32, true, true, OPEN, MIXED>(R.A, g, lanes, Q);
    else if (R.variant & 2u)  // isolated TreePM
        batch_group<FP32, false, true, OPEN, MIXED>(R.A, g, lanes, Q);
    else
        batch_group<FP32, false, false, OPEN, MIXED>(R.A, g, lanes, Q);
}

// The FP64 instance inlines every walk variant and would take 143 VGPRs
// (three wavefronts per SIMD); held to 128 (four) it spills 13 dwords and
// serves 4-5 % more force evaluations per second.
template <bool FP32>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_walk_batch(const BatchReq *__restrict__ reqs,
                                                       uint32_t nreq, uint32_t nitems,
                                                       uint32_t *__restrict__ counter) {
    const int lane = threadIdx.x & 63;
    IQ64 *Q = nullptr;  // the FP64 walk's interaction queue (used with a cutoff)
    if constexpr (!FP32) {
        __shared__ IQ64 q[kBlock / 64];
        Q = &q[threadIdx.x >> 6];
    }
    for (;;) {
        uint32_t item = 0;
        if (lane == 0)
            item = atomicAdd(counter, 1u);
        item = __builtin_amdgcn_readfirstlane(__shfl(item, 0, 64));
        if (item >= nitems)
            break;  // every wavefront reaches this once the items are exhausted
        uint32_t lo = 0, hi = nreq;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (reqs[mid].first <= item)
                lo = mid;
            else
                hi = mid;
        }
        const BatchReq &R = reqs[lo];
        const uint32_t g = item - R.first;
        const bool lanes = (R.variant & 4u) != 0;
        const bool rel = (R.variant & 1u) != 0, mixed = (R.variant & 16u) != 0;
        if (rel) {
            if (mixed)
                batch_geometry<FP32, TPM_OPEN_REL, true>(R, g, lanes, Q);
            else
                batch_geometry<FP32, TPM_OPEN_REL, false>(R, g, lanes, Q);
        } else {
            if (mixed)
                batch_geometry<FP32, TPM_OPEN_BH, true>(R, g, lanes, Q);
            else
                batch_geometry<FP32, TPM_OPEN_BH, false>(R, g, lanes, Q);
        }
    }
}

}  // namespace
}  // namespace tpm

struct tpm_batch {
    hipStream_t stream = nullptr;
    std::string err;
    struct Pending {
        tpm_ctx *c;
        int32_t opening;
        int64_t n_act;
        const int32_t *idx;
        const double *anorm;
        void *acc;
        uint32_t *nint;
    };
    std::vector<Pending> pend;
    tpm::BatchReq *host = nullptr;  // pinned staging of the request table
    size_t host_cap = 0;
    void *dev = nullptr;            // device request table
    size_t dev_cap = 0;
    uint32_t *counter = nullptr;    // two work counters
    hipEvent_t done = nullptr;      // last launch finished: staging reusable
    bool launched = false;
};

using namespace tpm;

static int bfail(tpm_batch *b, int code, const std::string &m) {
    b->err = m;
    return code;
}

#define BHIP(b, expr)                                                        \
    do {                                                                     \
        hipError_t _e = (expr);                                              \
        if (_e != hipSuccess)                                                \
            return bfail((b), _e == hipErrorOutOfMemory ? TPM_ENOMEM : TPM_EDEVICE, \
                         std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

extern "C" {

int tpm_batch_create(void *hip_stream, tpm_batch **out) {
    if (!out)
        return TPM_EINVAL;
    *out = nullptr;
    tpm_batch *b = new (std::nothrow) tpm_batch();
    if (!b)
        return TPM_ENOMEM;
    b->stream = (hipStream_t)hip_stream;
    if (hipMalloc((void **)&b->counter, 16) != hipSuccess ||
        hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
        if (b->counter)
            (void)hipFree(b->counter);
        delete b;
        return TPM_ENOMEM;
    }
    *out = b;
    return TPM_OK;
}

int tpm_batch_destroy(tpm_batch *b) {
    if (!b)
        return TPM_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    if (b->host)
        (void)hipHostFree(b->host);
    if (b->dev)
        (void)hipFree(b->dev);
    if (b->counter)
        (void)hipFree(b->counter);
    if (b->done)
        (void)hipEventDestroy(b->done);
    delete b;
    return TPM_OK;
}

const char *tpm_batch_last_error(const tpm_batch *b) { return b ? b->err.c_str() : "NULL batch"; }

int tpm_batch_add(tpm_batch *b, tpm_ctx *c, int32_t opening, int64_t n_act,
                  const int32_t *idx, const double *anorm, void *acc, uint32_t *nint) {
    if (!b)
        return TPM_EINVAL;
    if (!c || !c->built)
        return bfail(b, TPM_ESTATE, "context missing or not built");
    if (opening != TPM_OPEN_BH && opening != TPM_OPEN_REL)
        return bfail(b, TPM_EINVAL, "opening must be TPM_OPEN_BH or TPM_OPEN_REL");
    if (n_act < 0 || n_act > (int64_t(1) << 31) - 1)
        return bfail(b, TPM_EINVAL, "n_act out of range");
    if (n_act > 0 && (!idx || !acc))
        return bfail(b, TPM_EINVAL, "active_idx and acc must not be NULL");
    if (opening == TPM_OPEN_REL && n_act > 0 && !anorm)
        return bfail(b, TPM_EINVAL, "the relative criterion needs a_old_norm");
    for (const auto &p : b->pend)
        if (p.c == c)
            return bfail(b, TPM_EINVAL, "a context may appear once per batch");
    b->pend.push_back({c, opening, n_act, idx, anorm, acc, nint});
    return TPM_OK;
}

int tpm_batch_launch(tpm_batch *b) {
    if (!b)
        return TPM_EINVAL;
    if (b->pend.empty())
        return TPM_OK;
    if (b->launched)
        BHIP(b, hipEventSynchronize(b->done));  // the staging table is free again
    const size_t np = b->pend.size();
    if (b->host_cap < np) {
        if (b->host)
            BHIP(b, hipHostFree(b->host));
        b->host = nullptr;
        BHIP(b, hipHostMalloc((void **)&b->host, 2 * np * sizeof(BatchReq), hipHostMallocDefault));
        b->host_cap = 2 * np;
    }
    if (b->dev_cap < np * sizeof(BatchReq)) {
        if (b->dev)
            BHIP(b, hipFree(b->dev));
        b->dev = nullptr;
        BHIP(b, hipMalloc(&b->dev, 2 * np * sizeof(BatchReq)));
        b->dev_cap = 2 * np * sizeof(BatchReq);
    }
    // stage: active sets of every request on the batch stream, FP32 first
    uint32_t items[2] = {0, 0}, nreq[2] = {0, 0};
    std::vector<size_t> order;
    for (int pass = 0; pass < 2; pass++)
        for (size_t k = 0; k < np; k++)
            if ((b->pend[k].c->P.precision == TPM_FP32) == (pass == 0))
                order.push_back(k);
    for (size_t o = 0; o < np; o++) {
        const auto &p = b->pend[order[o]];
        tpm_ctx *c = p.c;
        const int which = c->P.precision == TPM_FP32 ? 0 : 1;
        hipStream_t saved = c->stream;
        c->stream = b->stream;
        Work w;
        int rc = work_of_ctx(c, true, w);
        if (rc == TPM_OK && p.n_act > 0)
            rc = select_active_into(c, p.n_act, p.idx, w);
        c->stream = saved;
        if (rc != TPM_OK)
            return bfail(b, rc, c->err);
        BatchReq &R = b->host[o];
        R = BatchReq{};
        fill_args(c, p.anorm, w, R.A);
        R.variant = (p.opening == TPM_OPEN_REL ? 1u : 0u) | (c->P.pm_grid > 0 ? 2u : 0u) |
                    (use_lanes(c, p.n_act) ? 4u : 0u) | (c->P.periodic ? 8u : 0u) |
                    (c->mixed ? 16u : 0u);
        R.first = items[which];
        const int64_t groups = p.n_act > 0 ? (std::min<int64_t>(p.n_act, c->n) + 63) / 64 : 0;
        items[which] += (uint32_t)groups;
        nreq[which]++;
    }
    BHIP(b, hipMemcpyAsync(b->dev, b->host, np * sizeof(BatchReq), hipMemcpyHostToDevice,
                           b->stream));
    {
        tpm_ctx tmp;  // fill kernels only need a stream
        tmp.stream = b->stream;
        if (fill_u32(&tmp, b->counter, 0u, 2) != TPM_OK)
            return bfail(b, TPM_EDEVICE, tmp.err);
    }
    const BatchReq *dreq = (const BatchReq *)b->dev;
    const uint32_t max_blocks = 2048;
    if (items[0]) {
        const uint32_t blocks = std::min<uint32_t>(max_blocks, (items[0] + 3) / 4);
        k_walk_batch<true><<<blocks, kBlock, 0, b->stream>>>(dreq, nreq[0], items[0], b->counter);
        BHIP(b, hipGetLastError());
    }
    if (items[1]) {
        const uint32_t blocks = std::min<uint32_t>(max_blocks, (items[1] + 3) / 4);
        k_walk_batch<false><<<blocks, kBlock, 0, b->stream>>>(dreq + nreq[0], nreq[1], items[1],
                                                              b->counter + 1);
        BHIP(b, hipGetLastError());
    }
    // outputs in each request's caller order
    for (const auto &p : b->pend) {
        if (p.n_act == 0)
            continue;
        tpm_ctx *c = p.c;
        const unsigned ob = grid_for(p.n_act, kBlock);
        if (c->P.precision == TPM_FP32)
            k_output<float><<<ob, kBlock, 0, b->stream>>>(
                p.idx, p.n_act, c->n, (const int32_t *)c->rank.p, (const uint32_t *)c->slot.p,
                (const float *)c->res.p, (const float *)c->rpot.p, (const uint32_t *)c->rnint.p,
                (float *)p.acc, nullptr, p.nint, (uint32_t *)c->err_flag.p);
        else
            k_output<double><<<ob, kBlock, 0, b->stream>>>(
                p.idx, p.n_act, c->n, (const int32_t *)c->rank.p, (const uint32_t *)c->slot.p,
                (const double *)c->res.p, (const double *)c->rpot.p,
                (const uint32_t *)c->rnint.p, (double *)p.acc, nullptr, p.nint,
                (uint32_t *)c->err_flag.p);
        BHIP(b, hipGetLastError());
    }
    BHIP(b, hipEventRecord(b->done, b->stream));
    b->launched = true;
    b->pend.clear();
    return TPM_OK;
}

}  // extern "C"
