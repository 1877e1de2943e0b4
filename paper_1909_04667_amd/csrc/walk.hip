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
#include "walk_device.h"

#include <algorithm>
#include <new>
#include <string>
#include <vector>

namespace tpm {
namespace {

using namespace wk;

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

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk64i(const WalkArgs A, uint32_t K) {
    walk_lanes64<PER, TPM, OPEN, POT, MIXED>(A, wave_id(), K);
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk32i(const WalkArgs A, uint32_t K) {
    walk_lanes32<PER, TPM, OPEN, POT, MIXED>(A, wave_id(), K);
}

// Sparse active sets with a cutoff: a census counts the compact groups
// (group_compact), then one of two launches walks every group -- with the
// shared cursor when at least half of the groups are compact (a set of dense
// clumps, as the deepest time bins are), with independent lanes otherwise;
// the other launch returns at once.  The two walks give the same results.
// Measured on the clustered 256^3 box, FP32 relative walk, against lanes for
// every sparse set: the densest 1 % 1.17 against 1.65 ms, the densest 10 %
// 3.81 against 4.44, random 1 % and 10 % unchanged (lanes: 1.66, 6.18).
// (Choosing per group inside one kernel made its lane walk slower: 7.6
// against 6.0 ms on the random 10 %.)
template <bool PER>
__global__ __launch_bounds__(kBlock) void k_census(const WalkArgs A, uint32_t *census) {
    const uint32_t wave = wave_id();
    if (wave * 64u >= load_count(A.nuniq))
        return;
    if (group_compact<PER>(A, wave) && (threadIdx.x & 63) == 0)
        atomicAdd(census, 1u);
}

__device__ __forceinline__ bool mostly_compact(const WalkArgs &A) {
    const uint32_t groups = (load_count(A.nuniq) + 63u) / 64u;
    return 2ull * load_count(A.census) >= groups;
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk64m(const WalkArgs A) {
    __shared__ IQ64 q[kBlock / 64];
    if (mostly_compact(A))
        walk_group64<PER, TPM, OPEN, POT, MIXED>(A, wave_id(), &q[threadIdx.x >> 6]);
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk64im(const WalkArgs A) {
    if (!mostly_compact(A))
        walk_lanes64<PER, TPM, OPEN, POT, MIXED>(A, wave_id(), 1u);
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk32m(const WalkArgs A) {
    if (mostly_compact(A))
        walk_group32<PER, TPM, OPEN, POT, MIXED>(A, wave_id());
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk32im(const WalkArgs A) {
    if (!mostly_compact(A))
        walk_lanes32<PER, TPM, OPEN, POT, MIXED>(A, wave_id(), 1u);
}

// one wavefront per target (sparse active sets)
template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk64s(const WalkArgs A) {
    __shared__ uint32_t front[kBlock / 64][kFrontWords];
    walk_lanes64<PER, TPM, OPEN, POT, MIXED, true>(A, wave_id(), 1u, front[threadIdx.x >> 6]);
}

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
__global__ __launch_bounds__(kBlock) void k_walk32s(const WalkArgs A) {
    __shared__ uint32_t front[kBlock / 64][kFrontWords];
    walk_lanes32<PER, TPM, OPEN, POT, MIXED, true>(A, wave_id(), 1u, front[threadIdx.x >> 6]);
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
    const uint32_t *__restrict__ slot, const uint32_t *__restrict__ nuniq,
    const T *__restrict__ res, const T *__restrict__ rpot, T *__restrict__ acc,
    T *__restrict__ pot, uint32_t *__restrict__ nint, uint32_t *__restrict__ err) {
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
    // the slot's record: acceleration and interaction count together (with
    // every particle active the slots are the ranks, and the lookup is skipped)
    const uint32_t rk = (uint32_t)rank[i];
    const uint32_t sl = *nuniq == (uint32_t)n ? rk : slot[rk];
    const T *r = res + 4 * (size_t)sl;
    acc[k] = r[0];
    acc[n_act + k] = r[1];
    acc[2 * n_act + k] = r[2];
    if (pot)
        pot[k] = rpot[sl];
    if (nint)
        nint[k] = count_of(r[3]);
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
    Variant variant;
    uint32_t K;       // slots per lane (lane-independent walk)
    unsigned blocks;
};

template <bool PER, bool TPM, int OPEN, bool POT, bool MIXED>
void launch_walk(const WalkArgs &A, const Launch &L, hipStream_t st) {
    if (L.variant == kSplitWalk) {
        if (L.fp32)
            k_walk32s<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A);
        else
            k_walk64s<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A);
    } else if (L.variant == kLaneWalk) {
        if (L.fp32)
            k_walk32i<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A, L.K);
        else
            k_walk64i<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A, L.K);
    } else if (L.variant == kGroupOrLanes) {
        if constexpr (TPM) {  // chosen only with a cutoff
            k_census<PER><<<L.blocks, kBlock, 0, st>>>(A, (uint32_t *)A.census);
            if (L.fp32) {
                k_walk32m<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A);
                k_walk32im<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A);
            } else {
                k_walk64m<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A);
                k_walk64im<PER, TPM, OPEN, POT, MIXED><<<L.blocks, kBlock, 0, st>>>(A);
            }
        }
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
        TPM_TRY(ensure(c, c->res, (size_t)4 * n * esz));
        TPM_TRY(ensure(c, c->rpot, (size_t)n * esz));
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

// Walk variant.  Independent lanes (results identical to the shared cursor)
// for sparse active sets, whose groups are too spread out for a shared cursor
// (it would visit the union of their walks), and for FP64 TreePM of isolated
// systems (their outer groups span many cutoff radii, and the FP64
// interaction is costly); the shared cursor otherwise (measured on the 128^3
// box and the Hernquist sphere).  One wavefront per target for active sets
// of at most 4096 targets, and of at most 65536 in trees of 2^22 particles or
// more: with that few wavefronts a lane's serial walk (the longest, which
// grows with the tree) is the critical path, while the frontier walk spreads
// each target over its wavefront and fills the chip.  Measured, FP32
// relative walk, lanes against one wavefront per target: the densest targets
// of the clustered 256^3 box, 16777 targets 1.41 / 0.35 ms, 41943: 1.41 /
// 0.75, 83886: 1.46 / 1.28, 167772: 1.73 / 2.41 (FP64 even at 84 k); the
// 4096-particle Plummer sphere 0.74 -> 0.32 ms.  In smaller trees the lane
// walks are short and the frontier walk's larger work per target loses
// (block steps of a 2^18 Hernquist sphere with sets up to 65536: 15.6 ms
// against 25.5 ms for the integration; the serving mix, up to 2^21
// particles per system: half the burst capacity).
// TPM_WALK_MODE (1 shared cursor, 2 lanes, 3 one wavefront per target)
// overrides the choice.
Variant wk::walk_variant(const tpm_ctx *c, int64_t n_act, bool census_ok) {
    if (c->walk_mode != 0)
        return c->walk_mode == 1 ? kGroupWalk : c->walk_mode == 2 ? kLaneWalk : kSplitWalk;
    const int64_t targets = std::min<int64_t>(n_act, c->n);
    if (targets <= 4096 || (targets <= 65536 && c->n >= (int64_t(1) << 22)))
        return kSplitWalk;
    const bool fp64_iso_tpm =
        c->P.precision == TPM_FP64 && c->P.pm_grid > 0 && !c->P.periodic;
    if (fp64_iso_tpm)
        return kLaneWalk;
    if (4 * n_act >= c->n)
        return kGroupWalk;
    // a sparse set: with a cutoff, as the census of its groups decides
    return census_ok && c->P.pm_grid > 0 ? kGroupOrLanes : kLaneWalk;
}

void wk::fill_args(tpm_ctx *c, const double *anorm, const Work &w, WalkArgs &A) {
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
    A.coherent = 0u;
    A.census = nullptr;
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
    A.group_ext2 = 0.25 * A.rc2;
    A.finv2rs = (float)A.inv2rs;
    A.fgexp = (float)(-1.4426950408889634 * A.inv2rs * A.inv2rs);
    A.res = w.res;
    A.rpot = w.rpot;
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
    LA.variant = walk_variant(c, n_act, true);
    if (LA.variant == kGroupOrLanes) {  // the census word follows the unique count
        A.census = w.nuniq + 1;
        TPM_TRY(fill_u32(c, w.nuniq + 1, 0u, 1));
    }
    LA.K = 1;
    if (LA.variant == kLaneWalk) {
        // several slots per lane once there are enough wavefronts to fill the chip
        const int64_t slots_per_chip = 256 * 4 * 8;
        while (LA.K < 8 && groups / (2 * LA.K) >= 2 * slots_per_chip)
            LA.K *= 2;
    }
    const int64_t waves = LA.variant == kSplitWalk ? std::min<int64_t>(n_act, n)
                                                  : (groups + LA.K - 1) / LA.K;
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
            idx, n_act, n, (const int32_t *)c->rank.p, w.slot, w.nuniq, (const float *)w.res,
            (const float *)w.rpot, (float *)acc, want_pot ? (float *)pot : nullptr,
            nint, (uint32_t *)c->err_flag.p);
    else
        k_output<double><<<ob, kBlock, 0, st>>>(
            idx, n_act, n, (const int32_t *)c->rank.p, w.slot, w.nuniq, (const double *)w.res,
            (const double *)w.rpot, (double *)acc, want_pot ? (double *)pot : nullptr,
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
    uint32_t variant;  // bit 0 relative criterion, 1 TreePM, 3 periodic, 4 individual
                       // softening, bits 5-6 the walk variant (wk::Variant)
    uint32_t first;    // first work item of the request
};

// The batch kernel holds the shared-cursor and lane walks only; requests
// that take one wavefront per target are launched on their own (inlined
// here, that walk would push the kernel's registers into heavy spills).
template <bool FP32, bool PER, bool TPM, int OPEN, bool MIXED>
__device__ __forceinline__ void batch_group(const WalkArgs &A, uint32_t g, uint32_t var,
                                            IQ64 *Q) {
    if constexpr (FP32) {
        if (var == kLaneWalk)
            walk_lanes32<PER, TPM, OPEN, false, MIXED>(A, g, 1u);
        else
            walk_group32<PER, TPM, OPEN, false, MIXED>(A, g);
    } else {
        if (var == kLaneWalk)
            walk_lanes64<PER, TPM, OPEN, false, MIXED>(A, g, 1u);
        else
            walk_group64<PER, TPM, OPEN, false, MIXED>(A, g, Q);
    }
}

template <bool FP32, int OPEN, bool MIXED>
__device__ __forceinline__ void batch_geometry(const BatchReq &R, uint32_t g, uint32_t lanes,
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
        const uint32_t lanes = (R.variant >> 5) & 3u;  // walk variant
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
    struct Own {  // a request walked by a launch of its own
        WalkArgs A;
        Launch L;
        int32_t opening;
        bool mixed, periodic, tpm;
    };
    std::vector<Own> own;
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
                    ((uint32_t)walk_variant(c, p.n_act) << 5) | (c->P.periodic ? 8u : 0u) |
                    (c->mixed ? 16u : 0u);
        R.first = items[which];
        const int64_t tg = std::min<int64_t>(p.n_act, c->n);
        const bool split = p.n_act > 0 && walk_variant(c, p.n_act) == kSplitWalk;
        if (split) {  // its own launch, after the staging below
            Launch LA{c->P.precision == TPM_FP32, kSplitWalk, 1u,
                      (unsigned)((tg + 3) / 4)};
            own.push_back({R.A, LA, p.opening, c->mixed != 0, c->P.periodic != 0,
                           c->P.pm_grid > 0});
        }
        const int64_t groups = (p.n_act > 0 && !split) ? (tg + 63) / 64 : 0;
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
    for (const Own &o : own) {
        if (o.periodic)
            dispatch_mixed<true, true>(o.A, o.L, o.opening, false, o.mixed, b->stream);
        else if (o.tpm)
            dispatch_mixed<false, true>(o.A, o.L, o.opening, false, o.mixed, b->stream);
        else
            dispatch_mixed<false, false>(o.A, o.L, o.opening, false, o.mixed, b->stream);
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
                (const uint32_t *)c->counters.p + 40, (const float *)c->res.p, (const float *)c->rpot.p, (float *)p.acc, nullptr,
                p.nint, (uint32_t *)c->err_flag.p);
        else
            k_output<double><<<ob, kBlock, 0, b->stream>>>(
                p.idx, p.n_act, c->n, (const int32_t *)c->rank.p, (const uint32_t *)c->slot.p,
                (const uint32_t *)c->counters.p + 40, (const double *)c->res.p, (const double *)c->rpot.p, (double *)p.acc, nullptr,
                p.nint, (uint32_t *)c->err_flag.p);
        BHIP(b, hipGetLastError());
    }
    BHIP(b, hipEventRecord(b->done, b->stream));
    b->launched = true;
    b->pend.clear();
    return TPM_OK;
}

}  // extern "C"
