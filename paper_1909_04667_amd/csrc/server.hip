// Device-resident serving loop: one persistent kernel per precision takes
// force requests for many resident systems (uneven N, uneven active
// fractions -- the time-step bins of Sec. 7.2) while it runs.  A request is
// one tree pass (geometric or relative criterion), or the paper's whole
// first force computation (Sec. 3.1): geometric pass, mesh force (Sec. 3.3,
// when the context has a mesh), |a| of their sum, relative pass.
//
// Host side: a request is a descriptor (walk arguments of its context, the
// active list, the outputs) written into a ring in coherent pinned host
// memory; publishing it is one release store of the ring's tail.  Device
// side: whichever wavefront finds no work takes a lock and copies new
// descriptors into the device slot table, then publishes the request's first
// job.  A request runs as phases, each a job of independent work items of one
// wavefront: [clear the marks] -> mark the active list -> count marked ranks
// per tile -> compact them into curve order -> walk groups of 64 targets ->
// [mesh interpolation -> |a| -> walk again with the relative criterion] ->
// write the outputs in caller order.  The wavefront that completes a phase's
// last item publishes the next phase; the last item of the output phase
// stores the request's ticket into pinned host memory (system scope), which
// the host polls.  Work items of different requests interleave on the device:
// a request's phases run while other requests' items occupy the rest of the
// chip.  Every work item runs the same code as the single-system path (marks,
// per-tile counts and compaction in increasing rank, the same walk per group,
// the same output gather), so each result is bit-identical alone and in any
// mix.
//
// Coherence: the chip's dies each have their own L2, so data one work item
// hands to a later one (marks, counts, active slots, results, |a|, job
// entries) is written and read with device-scope relaxed accesses, which
// bypass the non-coherent caches, and every counter that publishes it is
// incremented only after the wavefront's own stores have completed.  No
// acquire or release fence (cache invalidation or write-back) runs at all:
// the outputs for the host are written through to memory with system-scope
// stores before the request's ticket is stored into pinned memory.  The kernel outlives many requests, so nothing it
// reads through the scalar cache may change while it runs.  Each request's descriptor goes
// to its own entry of a ring of kDescRing entries (index = ticket modulo the
// ring), and the host launches the kernel anew after kRelaunch requests, so
// within one launch no entry is written twice: the walks read the arguments
// with scalar loads as they do in a single-system launch.  Counts written by
// other wavefronts are read with coherent vector loads; claims are
// agent-scope acquires (they invalidate the vector L1).  The tree records,
// also read with scalar loads, change only when a tree is rebuilt or device
// memory is freed (and possibly reused): the library counts both, and a
// submit after such an event drains the kernel and launches it again (a
// launch starts with fresh caches) before the request runs.  Exit: every
// wavefront leaves when the host asks (stop or drain) or when the fetcher has
// seen no live request for idle_ms; the host relaunches the kernel whenever
// it finds it gone with requests pending.
#include <atomic>
#include <cstring>
#include <type_traits>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "pm_device.h"
#include "walk_device.h"

namespace tpm {
namespace {

using namespace wk;

constexpr uint32_t kSrvTile = 2048;   // ranks per count / compact item
constexpr uint32_t kSrvChunk = 4096;  // list entries per clear / mark / output item
constexpr uint32_t kSrvSlots = 1024;  // active slots per mesh / |a| item
constexpr uint32_t kJobCap = 1u << 16;  // job ring (one live job per request)
constexpr int kMaxSlots = 256;        // live requests per server
constexpr uint32_t kDescRing = 1u << 16;  // device descriptors (index = ticket mod ring)
constexpr uint64_t kRelaunch = 1u << 14;  // requests per launch, well below the ring

enum : uint32_t {
    kPhClear = 0, kPhMark, kPhCount, kPhCompact, kPhWalk, kPhPm, kPhNorm, kPhWalk2, kPhOutput
};
constexpr uint32_t kStep = 1u;   // flags: the whole first force computation
constexpr uint32_t kMesh = 2u;   //        with the mesh part

// One request, as the host prepares it.  variant: bit 0 relative criterion,
// 1 TreePM, 3 periodic, 4 individual softening, bits 5-6 the walk variant
// (wk::Variant).
// Whole 64-byte lines, so no scalar-cache line holds parts of two
// descriptors.
// Whole 128-byte L2 lines per descriptor: a wavefront that reads descriptor i
// must not bring any part of descriptor i + 1 into its die's L2 before the
// fetcher has written it (the fetcher's stores from another die would not
// replace that stale copy, and later scalar loads of i + 1 would read it).
struct alignas(128) SrvReq {
    WalkArgs A;
    const int32_t *idx;   // caller's active list [n_act]
    const int32_t *rank;  // build index -> rank
    uint32_t *mark;
    uint32_t *slot;
    uint32_t *counts;
    void *acc;            // [3][n_act], the precision of the server
    uint32_t *nint;       // [n_act] or null
    uint32_t *err;        // the context's sticky error word
    uint32_t n_act;
    uint32_t epoch;
    uint32_t clear;
    uint32_t variant;
    uint32_t flags;       // kStep, kMesh
    uint32_t pad0;
    pmk::MeshGeom mg;     // mesh geometry (kMesh)
    const void *phi;      // potential mesh (kMesh)
    void *res_pm;         // [n][4] mesh force in slot order (kMesh)
    void *acc_pm;         // [3][n_act] mesh force in caller order (kMesh)
    double *anorm_out;    // [n] |a| in build order, read by the relative pass (kStep)
    uint64_t ticket;
    uint32_t slot_id;     // host slot: completion flag and ring entry
    uint32_t desc;        // device descriptor index
};
static_assert(sizeof(SrvReq) % 128 == 0, "descriptors own whole L2 lines");
static_assert(sizeof(SrvReq) % 8 == 0, "descriptor copied in 8-byte words");
constexpr uint32_t kReqWords = sizeof(SrvReq) / 8;

// A job (one phase of one request): `claim` holds (sequence << 32) | next
// item, 0 while the entry is being written; a wavefront claims an item by
// compare-and-swap only while the sequence is the one it read, after reading
// the fields between two equal reads of `claim`.
struct Job {
    unsigned long long claim;
    uint32_t slot, phase, nitems, pad;
};

struct SrvDev {
    uint32_t job_reserve;  // next job index to publish
    uint32_t job_head;     // oldest job that may still have items
    uint32_t host_head;    // ring entries copied to the device
    uint32_t live;         // requests taken from the ring and not yet finished
    uint32_t ctl;          // the host's control word, mirrored by the fetcher;
                           // 3: the fetcher found the server idle
    uint32_t done[kDescRing];  // items finished in the live phase of each request
};

// Coherent pinned host memory shared with the kernel.
struct SrvHost {
    unsigned long long tail;       // descriptors published (host writes)
    unsigned int ctl;              // 0 run, 1 stop, 2 drain (host writes)
    unsigned int pad;
    unsigned long long done[kMaxSlots];  // ticket + 1 when a slot's request finished
    SrvReq ring[kMaxSlots];
};

template <typename T>
__device__ __forceinline__ T ld_rlx(T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A result for the host: a system-scope store, written through to memory.
template <typename T>
__device__ __forceinline__ void out_st(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Waits until the wavefront's memory operations have completed (its
// device-scope stores are then visible chip-wide), and keeps the compiler
// from moving memory accesses across this point.
__device__ __forceinline__ void wait_mem() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ uint32_t phase_items(uint32_t n, uint32_t n_act, uint32_t ph,
                                                uint32_t nuniq, uint32_t variant) {
    switch (ph) {
    case kPhClear: return (n + kSrvChunk - 1) / kSrvChunk;
    case kPhMark:
    case kPhOutput: return (n_act + kSrvChunk - 1) / kSrvChunk;
    case kPhCount:
    case kPhCompact: return (n + kSrvTile - 1) / kSrvTile;
    case kPhPm:
    case kPhNorm: return (nuniq + kSrvSlots - 1) / kSrvSlots;
    default: return (variant >> 5) == kSplitWalk ? nuniq            // one target per item
                                                 : (nuniq + 63) / 64;  // 64 per item
    }
}

// The phase after ph.
__device__ __forceinline__ uint32_t next_phase(uint32_t ph, uint32_t flags) {
    switch (ph) {
    case kPhWalk: return (flags & kStep) ? ((flags & kMesh) ? kPhPm : kPhNorm) : kPhOutput;
    case kPhPm: return kPhNorm;
    case kPhNorm: return kPhWalk2;
    case kPhWalk2: return kPhOutput;
    default: return ph + 1u;
    }
}

// Publishes one job (called by lane 0).
__device__ void publish(SrvDev *st, Job *jobs, uint32_t slot, uint32_t phase, uint32_t n) {
    const uint32_t j = __hip_atomic_fetch_add(&st->job_reserve, 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
    Job *J = &jobs[j % kJobCap];
    coherent_st(&J->claim, 0ull);
    coherent_st(&st->done[slot], 0u);
    wait_mem();
    coherent_st(&J->slot, slot);
    coherent_st(&J->phase, phase);
    coherent_st(&J->nitems, n);
    wait_mem();
    coherent_st(&J->claim, (unsigned long long)(j + 1u) << 32);
}

// Lane 0: claims the next item of the oldest job that has one: a load sees
// items left, then one fetch-and-add takes an item (no compare-and-swap
// retries when many wavefronts look at once).  The item taken is always
// honoured: should the entry have been republished in between (it is reused
// only after kJobCap newer jobs), it is that job's item.  Returns false when
// no published job has an item left.
__device__ bool claim(SrvDev *st, Job *jobs, uint32_t &slot, uint32_t &phase, uint32_t &nitems,
                      uint32_t &item) {
    for (int guard = 0; guard < 64; guard++) {
        const uint32_t h = ld_rlx(&st->job_head);
        Job *J = &jobs[h % kJobCap];
        const unsigned long long c1 = ld_rlx(&J->claim);
        if ((uint32_t)(c1 >> 32) != h + 1u)
            return false;  // not (yet) published
        wait_mem();
        const uint32_t ni = ld_rlx(&J->nitems);
        if ((uint32_t)c1 >= ni) {  // exhausted: move the head on
            uint32_t e = h;
            __hip_atomic_compare_exchange_strong(&st->job_head, &e, h + 1u, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const unsigned long long c = __hip_atomic_fetch_add(&J->claim, 1ull, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
        wait_mem();
        const uint32_t seq = (uint32_t)(c >> 32);
        if (seq == 0)
            continue;  // being written: the publisher's final store replaces the add
        // the job whose item this is (normally the one at h)
        const uint32_t jn = ld_rlx(&J->nitems);
        if ((uint32_t)c >= jn)
            continue;  // exhausted meanwhile
        slot = ld_rlx(&J->slot);
        phase = ld_rlx(&J->phase);
        nitems = jn;
        item = (uint32_t)c;
        return true;
    }
    return false;
}

// The fetcher wavefront (the kernel's first): copies new host descriptors
// into the slot table (all lanes copy, lane 0 publishes each request's first
// job) and mirrors the host's control word into device memory.  It is the
// only wavefront that reads host memory.  Returns the descriptors taken.
__device__ uint32_t fetch(SrvDev *st, SrvHost *host, SrvReq *slots, Job *jobs) {
    const int lane = threadIdx.x & 63;
    uint32_t head = 0, tail = 0;
    if (lane == 0) {
        head = ld_rlx(&st->host_head);
        // relaxed: the descriptor words are read after it (wait_mem below)
        // with system-scope loads, which do not go through the caches
        tail = (uint32_t)__hip_atomic_load(&host->tail, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
        const uint32_t ctl = __hip_atomic_load(&host->ctl, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_SYSTEM);
        coherent_st(&st->ctl, ctl);
    }
    head = __builtin_amdgcn_readfirstlane(head);
    tail = __builtin_amdgcn_readfirstlane(tail);
    wait_mem();
    uint32_t n = 0;
    for (uint32_t r = head; r != tail && n < 16; r++, n++) {
        SrvReq *hr = &host->ring[r % kMaxSlots];
        const uint32_t sid = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&hr->desc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
        const unsigned long long *src = (const unsigned long long *)hr;
        unsigned long long *dst = (unsigned long long *)&slots[sid];
        for (uint32_t w = lane; w < kReqWords; w += 64)
            coherent_st(&dst[w], __hip_atomic_load(&src[w], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_SYSTEM));
        wait_mem();
        if (lane == 0) {
            const uint32_t nn = __hip_atomic_load(&hr->A.n, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM);
            const uint32_t na = __hip_atomic_load(&hr->n_act, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM);
            const uint32_t ph = __hip_atomic_load(&hr->clear, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM)
                                    ? kPhClear
                                    : kPhMark;
            __hip_atomic_fetch_add(&st->live, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            publish(st, jobs, sid, ph, phase_items(nn, na, ph, 0, 0));
        }
    }
    if (lane == 0 && n)
        coherent_st(&st->host_head, head + n);
    return n;
}

// True while a published job may still have items (the head job is
// published): the fetcher stays while there is work.
__device__ __forceinline__ bool jobs_pending(SrvDev *st, Job *jobs) {
    const uint32_t h = ld_rlx(&st->job_head);
    return (uint32_t)(ld_rlx(&jobs[h % kJobCap].claim) >> 32) == h + 1u;
}

// ---- the work items -----------------------------------------------------------

__device__ __forceinline__ void item_clear(const SrvReq &R, uint32_t it) {
    const int lane = threadIdx.x & 63;
    const uint32_t n = R.A.n;
    for (uint32_t k = it * kSrvChunk + lane; k < min(n, (it + 1) * kSrvChunk); k += 64)
        coherent_st(R.mark + k, 0u);
}

__device__ __forceinline__ void item_mark(const SrvReq &R, uint32_t it) {
    const int lane = threadIdx.x & 63;
    const uint32_t n = R.A.n;
    for (uint32_t k = it * kSrvChunk + lane; k < min(R.n_act, (it + 1) * kSrvChunk); k += 64) {
        const int32_t i = R.idx[k];
        if (i >= 0 && (uint32_t)i < n)
            coherent_st(R.mark + R.rank[i], R.epoch);  // out-of-range indices: the output phase
    }
}

// Marked ranks of one tile, counted (as the single-system compaction does).
__device__ __forceinline__ void item_count(const SrvReq &R, uint32_t it) {
    const int lane = threadIdx.x & 63;
    const uint32_t n = R.A.n, base = it * kSrvTile;
    uint32_t t = 0;
    for (uint32_t j = 0; j < kSrvTile; j += 64) {
        const uint32_t r = base + j + lane;
        t += (uint32_t)__popcll(__ballot(r < n && coherent_ld(R.mark + r) == R.epoch));
    }
    if (lane == 0)
        coherent_st(R.counts + it, t);
}

// The tile's marked ranks in increasing order at their positions in the
// compacted list (the earlier tiles' counts give the offset); the item of
// tile 0 also writes the total.
__device__ __forceinline__ void item_compact(const SrvReq &R, uint32_t it) {
    const int lane = threadIdx.x & 63;
    const uint32_t n = R.A.n, base = it * kSrvTile;
    const uint32_t nt = (n + kSrvTile - 1) / kSrvTile;
    uint32_t before = 0, all = 0;
    for (uint32_t q = lane; q < nt; q += 64) {
        const uint32_t v = coherent_ld(R.counts + q);
        before += q < it ? v : 0u;
        all += v;
    }
    for (int o = 1; o < 64; o <<= 1) {
        before += __shfl_xor(before, o);
        all += __shfl_xor(all, o);
    }
    if (it == 0 && lane == 0)
        coherent_st((uint32_t *)R.A.nuniq, all);
    uint32_t pos = before;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (uint32_t j = 0; j < kSrvTile; j += 64) {
        const uint32_t r = base + j + lane;
        const bool f = r < n && coherent_ld(R.mark + r) == R.epoch;
        const uint64_t m = __ballot(f);
        if (f) {
            const uint32_t p = pos + (uint32_t)__popcll(m & below);
            coherent_st((uint32_t *)R.A.act + p, r);
            coherent_st(R.slot + r, p);
        }
        pos += (uint32_t)__popcll(m);
    }
}

template <bool FP32, bool PER, bool TPM, int OPEN, bool MIXED>
__device__ __forceinline__ void srv_group(const WalkArgs &A, uint32_t g, uint32_t var,
                                          WaveLds *Q) {
    if constexpr (FP32) {
        if (var == kSplitWalk)
            walk_lanes32<PER, TPM, OPEN, false, MIXED, true>(A, g, 1u, Q->front);
        else if (var == kLaneWalk)
            walk_lanes32<PER, TPM, OPEN, false, MIXED>(A, g, 1u);
        else
            walk_group32<PER, TPM, OPEN, false, MIXED>(A, g);
    } else {
        if (var == kSplitWalk)
            walk_lanes64<PER, TPM, OPEN, false, MIXED, true>(A, g, 1u, Q->front);
        else if (var == kLaneWalk)
            walk_lanes64<PER, TPM, OPEN, false, MIXED>(A, g, 1u);
        else
            walk_group64<PER, TPM, OPEN, false, MIXED>(A, g, &Q->q);
    }
}

template <bool FP32, int OPEN, bool MIXED>
__device__ __forceinline__ void srv_geometry(const SrvReq &R, uint32_t g, uint32_t lanes,
                                             WaveLds *Q) {
    if (R.variant & 8u)
        srv_group<FP32, true, true, OPEN, MIXED>(R.A, g, lanes, Q);
    else if (R.variant & 2u)
        srv_group<FP32, false, true, OPEN, MIXED>(R.A, g, lanes, Q);
    else
        srv_group<FP32, false, false, OPEN, MIXED>(R.A, g, lanes, Q);
}

template <bool FP32>
__device__ __forceinline__ void item_walk(const SrvReq &R, uint32_t g, WaveLds *Q, bool rel) {
    const uint32_t lanes = (R.variant >> 5) & 3u;  // walk variant
    const bool mixed = (R.variant & 16u) != 0;
    if (rel) {
        if (mixed)
            srv_geometry<FP32, TPM_OPEN_REL, true>(R, g, lanes, Q);
        else
            srv_geometry<FP32, TPM_OPEN_REL, false>(R, g, lanes, Q);
    } else {
        if (mixed)
            srv_geometry<FP32, TPM_OPEN_BH, true>(R, g, lanes, Q);
        else
            srv_geometry<FP32, TPM_OPEN_BH, false>(R, g, lanes, Q);
    }
}

// Mesh force at the active slots (as the single-system interpolation kernel).
template <typename T>
__device__ __forceinline__ void item_pm(const SrvReq &R, uint32_t it, uint32_t nu) {
    const int lane = threadIdx.x & 63;
    const uint32_t n = R.A.n;
    T *res = (T *)R.res_pm;
    for (uint32_t k = it * kSrvSlots + lane; k < min(nu, (it + 1) * kSrvSlots); k += 64) {
        double F[3], P;
        pmk::interp_at<T, true>(R.A.ps, n, coherent_ld(R.A.act + k), (const T *)R.phi, R.mg, F,
                                P);
        coherent_st(res + 4 * (size_t)k, (T)F[0]);
        coherent_st(res + 4 * (size_t)k + 1, (T)F[1]);
        coherent_st(res + 4 * (size_t)k + 2, (T)F[2]);
    }
}

// |a| of the geometric pass plus the mesh force, into build order (as the
// single-system |a| kernel: the sum and the norm in double).
template <typename T>
__device__ __forceinline__ void item_norm(const SrvReq &R, uint32_t it, uint32_t nu) {
    const int lane = threadIdx.x & 63;
    const T *a = (const T *)R.A.res, *b = (const T *)R.res_pm;
    const bool mesh = (R.flags & kMesh) != 0;
    for (uint32_t k = it * kSrvSlots + lane; k < min(nu, (it + 1) * kSrvSlots); k += 64) {
        double v[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            v[d] = (double)coherent_ld(a + 4 * (size_t)k + d);
            if (mesh)
                v[d] += (double)coherent_ld(b + 4 * (size_t)k + d);
        }
        coherent_st(R.anorm_out + R.A.perm[coherent_ld(R.A.act + k)],
                    sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
    }
}

// Results in caller order (as the single-system output kernels).
template <typename T>
__device__ __forceinline__ void item_output(const SrvReq &R, uint32_t it) {
    const int lane = threadIdx.x & 63;
    const uint32_t n = R.A.n, na = R.n_act;
    const T *res = (const T *)R.A.res, *rpm = (const T *)R.res_pm;
    T *acc = (T *)R.acc, *apm = (T *)R.acc_pm;
    const bool mesh = (R.flags & kMesh) != 0;
    for (uint32_t k = it * kSrvChunk + lane; k < min(na, (it + 1) * kSrvChunk); k += 64) {
        const int32_t i = R.idx[k];
        T v[6] = {(T)NAN, (T)NAN, (T)NAN, (T)NAN, (T)NAN, (T)NAN};
        uint32_t ni = 0xffffffffu;
        if (i < 0 || (uint32_t)i >= n) {
            atomicOr(R.err, 1u);
        } else {
            const uint32_t sl = coherent_ld(R.slot + R.rank[i]);
            for (int d = 0; d < 3; d++)
                v[d] = coherent_ld(res + 4 * (size_t)sl + d);
            if (mesh)
                for (int d = 0; d < 3; d++)
                    v[3 + d] = coherent_ld(rpm + 4 * (size_t)sl + d);
            if (R.nint)
                ni = count_of(coherent_ld(res + 4 * (size_t)sl + 3));
        }
        // outputs written through to memory (other dies' caches are not
        // written back for the host)
        for (int d = 0; d < 3; d++)
            out_st(acc + (size_t)d * na + k, v[d]);
        if (mesh)
            for (int d = 0; d < 3; d++)
                out_st(apm + (size_t)d * na + k, v[3 + d]);
        if (R.nint)
            out_st(R.nint + k, ni);
    }
}

// Both instances inline every walk variant (FP32: 80 VGPRs, FP64: 170, no
// spills); each is launched with two wavefronts per SIMD.
template <bool FP32>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(FP32 ? 4 : 2))) void k_server(
    SrvDev *st, SrvHost *host, SrvReq *slots, Job *jobs, unsigned long long idle_ticks) {
    const int lane = threadIdx.x & 63;
    __shared__ WaveLds q[kBlock / 64];  // the walks' queue or frontiers
    WaveLds *Q = &q[threadIdx.x >> 6];
    // per block: bumped when one of its wavefronts sees more items left, so
    // its sleeping siblings wake up and claim (an LDS read, no memory traffic)
    __shared__ uint32_t s_hint;
    if (threadIdx.x == 0)
        s_hint = 0u;
    __syncthreads();
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the kernel's first wavefront only fetches requests from the host; it
    // also decides, for the whole kernel, when the server has been idle
    // (no request live, none fetched) for idle_ticks, and then tells every
    // wavefront to leave.  (Wavefronts deciding that each for themselves would
    // thin the server out under sparse arrivals.)
    if (blockIdx.x == 0 && wv == 0) {
        unsigned long long last = wall_clock64();
        for (;;) {
            const uint32_t got = fetch(st, host, slots, jobs);
            uint32_t ctl = 0, busy = 0;
            if (lane == 0) {
                ctl = ld_rlx(&st->ctl);
                busy = (ld_rlx(&st->live) != 0u || jobs_pending(st, jobs)) ? 1u : 0u;
            }
            if (__builtin_amdgcn_readfirstlane(ctl) != 0)
                break;
            if (got || __builtin_amdgcn_readfirstlane(busy)) {
                last = wall_clock64();
            } else if (wall_clock64() - last > idle_ticks) {
                if (lane == 0)
                    coherent_st(&st->ctl, 3u);
                break;
            }
            if (got && lane == 0)
                __hip_atomic_fetch_add(&s_hint, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __builtin_amdgcn_s_sleep(16);
        }
        return;
    }
    // one wavefront in every 24 blocks (a few per die) polls the job queue
    // often; the others sleep on their block's hint and look themselves
    // every ~30 us
    const bool hot = wv == (blockIdx.x == 0 ? 1u : 0u) && (blockIdx.x % 24u) == 0;
    for (;;) {
        uint32_t has = 0, sid = 0, ph = 0, nitems = 0, item = 0;
        if (lane == 0)
            has = claim(st, jobs, sid, ph, nitems, item) ? 1u : 0u;
        has = __builtin_amdgcn_readfirstlane(has);
        if (!has) {
            uint32_t ctl = 0;
            if (lane == 0)
                ctl = ld_rlx(&st->ctl);
            if (__builtin_amdgcn_readfirstlane(ctl) != 0)
                break;  // stop, drain or idle: every wavefront reaches this
            if (hot) {
                __builtin_amdgcn_s_sleep(64);  // ~2 us
            } else {
                const uint32_t seen = __hip_atomic_load(&s_hint, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_WORKGROUP);
                for (int k = 0; k < 16; k++) {
                    __builtin_amdgcn_s_sleep(64);
                    if (__hip_atomic_load(&s_hint, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP) != seen)
                        break;
                }
            }
            continue;
        }
        if (lane == 0 && item + 1u < nitems)  // more left: wake the block
            __hip_atomic_fetch_add(&s_hint, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        sid = __builtin_amdgcn_readfirstlane(sid);
        ph = __builtin_amdgcn_readfirstlane(ph);
        nitems = __builtin_amdgcn_readfirstlane(nitems);
        item = __builtin_amdgcn_readfirstlane(item);
        // the descriptor was written once in this launch, before its job was
        // published: read it through the constant address space (scalar loads,
        // like kernel arguments)
        typedef __attribute__((address_space(4))) const SrvReq creq;
        const SrvReq &R = *(const SrvReq *)(const creq *)&slots[sid];
        using T = typename std::conditional<FP32, float, double>::type;
        switch (ph) {
        case kPhClear: item_clear(R, item); break;
        case kPhMark: item_mark(R, item); break;
        case kPhCount: item_count(R, item); break;
        case kPhCompact: item_compact(R, item); break;
        case kPhWalk:
        case kPhWalk2:  // the request's own criterion; a step: geometric, then relative
            item_walk<FP32>(R, item, Q,
                            ph == kPhWalk2 || (!(R.flags & kStep) && (R.variant & 1u)));
            break;
        case kPhPm: item_pm<T>(R, item, load_count(R.A.nuniq)); break;
        case kPhNorm: item_norm<T>(R, item, load_count(R.A.nuniq)); break;
        default: item_output<T>(R, item); break;
        }
        wait_mem();  // this item's stores are visible before it counts as done
        if (lane == 0) {
            const uint32_t d = __hip_atomic_fetch_add(&st->done[sid], 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            wait_mem();
            if (d + 1u == nitems) {  // this wavefront finished the phase
                if (ph == kPhOutput) {
                    // every output item wrote through to memory and waited
                    // for its stores before counting itself done
                    out_st(&host->done[R.slot_id], R.ticket + 1ull);
                    __hip_atomic_fetch_sub(&st->live, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    uint32_t nph = next_phase(ph, R.flags), nu = 0;
                    if (nph >= kPhWalk)
                        nu = coherent_ld(R.A.nuniq);
                    if (nph >= kPhWalk && nph != kPhOutput && nu == 0)
                        nph = kPhOutput;  // no valid target: only the outputs remain
                    publish(st, jobs, sid, nph, phase_items(R.A.n, R.n_act, nph, nu, R.variant));
                    __hip_atomic_fetch_add(&s_hint, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
        wave_sync();
    }
}

}  // namespace
}  // namespace tpm

struct tpm_server {
    int precision = TPM_FP32;
    int device = 0;
    hipStream_t stream = nullptr;  // non-blocking, default priority
    hipEvent_t exited = nullptr;   // recorded after each launch
    bool launched = false;
    uint64_t launch_epoch = 0;     // memory epoch (builds and frees) at the last launch
    double idle_ms = 5.0;
    unsigned long long idle_ticks = 0;
    std::string err;
    tpm::SrvDev *dev = nullptr;
    tpm::SrvReq *slots = nullptr;
    tpm::Job *jobs = nullptr;
    tpm::SrvHost *host = nullptr;      // host address
    tpm::SrvHost *host_dev = nullptr;  // the same memory, device address
    std::vector<int> free_slots;
    std::vector<uint64_t> slot_ticket;  // ticket of the request in each slot (0: free)
    std::vector<tpm_ctx *> slot_ctx;
    uint64_t next_ticket = 1;
    uint64_t published = 0;
    uint64_t published_at_launch = 0;
    int64_t launches = 0;
    int blocks = 0;
};

using namespace tpm;

namespace {

int sfail(tpm_server *s, int code, const std::string &m) {
    s->err = m;
    return code;
}

#define SHIP(s, expr)                                                                      \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess)                                                              \
            return sfail((s), _e == hipErrorOutOfMemory ? TPM_ENOMEM : TPM_EDEVICE,        \
                         std::string(#expr) + ": " + hipGetErrorString(_e));               \
    } while (0)

int launch(tpm_server *s) {
    s->host->ctl = 0;
    std::atomic_thread_fence(std::memory_order_seq_cst);
    // the device mirror of the control word starts at "run"
    SHIP(s, hipMemsetAsync(&s->dev->ctl, 0, sizeof(uint32_t), s->stream));
    if (s->precision == TPM_FP32)
        k_server<true><<<s->blocks, kBlock, 0, s->stream>>>(s->dev, s->host_dev, s->slots,
                                                            s->jobs, s->idle_ticks);
    else
        k_server<false><<<s->blocks, kBlock, 0, s->stream>>>(s->dev, s->host_dev, s->slots,
                                                             s->jobs, s->idle_ticks);
    SHIP(s, hipGetLastError());
    SHIP(s, hipEventRecord(s->exited, s->stream));
    s->launched = true;
    s->published_at_launch = s->published;
    s->launch_epoch = memory_epoch();
    s->launches++;
    return TPM_OK;
}

bool running(tpm_server *s) { return s->launched && hipEventQuery(s->exited) == hipErrorNotReady; }

// Asks the kernel to leave and waits for it.
int drain(tpm_server *s, unsigned int how) {
    if (!s->launched)
        return TPM_OK;
    __atomic_store_n(&s->host->ctl, how, __ATOMIC_SEQ_CST);
    SHIP(s, hipEventSynchronize(s->exited));
    s->launched = false;
    s->host->ctl = 0;
    return TPM_OK;
}

// Relaunches the kernel if it left while requests are pending.
int keep_alive(tpm_server *s) {
    bool pending = false;
    for (uint64_t t : s->slot_ticket)
        pending = pending || t != 0;
    if (pending && !running(s))
        return launch(s);
    return TPM_OK;
}

}  // namespace

extern "C" {

int tpm_server_create(int32_t precision, double idle_ms, tpm_server **out) {
    if (!out)
        return TPM_EINVAL;
    *out = nullptr;
    if ((precision != TPM_FP32 && precision != TPM_FP64) || !(idle_ms > 0.0) || idle_ms > 1e4)
        return TPM_EINVAL;
    tpm_server *s = new (std::nothrow) tpm_server();
    if (!s)
        return TPM_ENOMEM;
    s->precision = precision;
    s->idle_ms = idle_ms;
    int rc = TPM_OK;
    int cus = 0, clock_khz = 0;
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) !=
            hipSuccess ||
        hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, s->device) !=
            hipSuccess)
        rc = TPM_EDEVICE;
    // Two wavefronts per SIMD each: FP32 (80 VGPRs) and FP64 (170) then fit
    // in a SIMD's registers beside each other (and four blocks of 32 KiB in
    // a CU's LDS); kernels of other work (builds of newly admitted systems)
    // run when the servers drain or idle.  Measured on the serving mix of 16
    // systems: burst capacity 6.3e7 evals/s against 5.0e7 with three FP32
    // and one FP64 wavefront per SIMD (FP64 requests were latency-bound with
    // one wavefront per SIMD).
    s->blocks = cus * 2;
    if (clock_khz <= 0)
        clock_khz = 100000;  // the usual 100 MHz constant clock
    s->idle_ticks = (unsigned long long)(idle_ms * (double)clock_khz);
    if (rc == TPM_OK &&
        (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&s->exited, hipEventDisableTiming) != hipSuccess))
        rc = TPM_EDEVICE;
    if (rc == TPM_OK &&
        (hipMalloc((void **)&s->dev, sizeof(SrvDev)) != hipSuccess ||
         hipMalloc((void **)&s->slots, kDescRing * sizeof(SrvReq)) != hipSuccess ||
         hipMalloc((void **)&s->jobs, kJobCap * sizeof(Job)) != hipSuccess ||
         hipHostMalloc((void **)&s->host, sizeof(SrvHost),
                       hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess))
        rc = TPM_ENOMEM;
    if (rc == TPM_OK && hipHostGetDevicePointer((void **)&s->host_dev, s->host, 0) != hipSuccess)
        rc = TPM_EDEVICE;
    if (rc == TPM_OK &&
        (hipMemsetAsync(s->dev, 0, sizeof(SrvDev), s->stream) != hipSuccess ||
         hipMemsetAsync(s->jobs, 0, kJobCap * sizeof(Job), s->stream) != hipSuccess ||
         hipStreamSynchronize(s->stream) != hipSuccess))
        rc = TPM_EDEVICE;
    if (rc != TPM_OK) {
        tpm_server_destroy(s);
        return rc;
    }
    std::memset(s->host, 0, sizeof(SrvHost));
    for (int k = kMaxSlots - 1; k >= 0; k--)
        s->free_slots.push_back(k);
    s->slot_ticket.assign(kMaxSlots, 0);
    s->slot_ctx.assign(kMaxSlots, nullptr);
    *out = s;
    return TPM_OK;
}

int tpm_server_destroy(tpm_server *s) {
    if (!s)
        return TPM_EINVAL;
    if (s->host && s->launched)
        (void)drain(s, 1u);
    if (s->stream)
        (void)hipStreamSynchronize(s->stream);
    if (s->dev)
        (void)hipFree(s->dev);
    if (s->slots)
        (void)hipFree(s->slots);
    if (s->jobs)
        (void)hipFree(s->jobs);
    if (s->host)
        (void)hipHostFree(s->host);
    if (s->exited)
        (void)hipEventDestroy(s->exited);
    if (s->stream)
        (void)hipStreamDestroy(s->stream);
    delete s;
    return TPM_OK;
}

const char *tpm_server_last_error(const tpm_server *s) { return s ? s->err.c_str() : "NULL server"; }

namespace {

int submit_impl(tpm_server *s, tpm_ctx *c, bool step, int32_t opening, int64_t n_act,
                const int32_t *idx, const double *anorm, void *acc, void *acc_pm,
                uint32_t *nint, uint64_t *ticket) {
    if (!s || !c || !ticket)
        return TPM_EINVAL;
    *ticket = 0;
    if (!c->built)
        return sfail(s, TPM_ESTATE, "submit before build_tree");
    if (c->P.precision != s->precision)
        return sfail(s, TPM_EINVAL, "context precision differs from the server's");
    if (!step && opening != TPM_OPEN_BH && opening != TPM_OPEN_REL)
        return sfail(s, TPM_EINVAL, "opening must be TPM_OPEN_BH or TPM_OPEN_REL");
    if (n_act < 1 || n_act > (int64_t(1) << 31) - 1 || !idx || !acc)
        return sfail(s, TPM_EINVAL, "n_act must be >= 1 with active_idx and acc");
    if (!step && opening == TPM_OPEN_REL && !anorm)
        return sfail(s, TPM_EINVAL, "the relative criterion needs a_old_norm");
    const bool mesh = step && c->P.pm_grid > 0;
    if (mesh != (acc_pm != nullptr))
        return sfail(s, TPM_EINVAL, "acc_pm is required exactly when the step has a mesh");
    if (c->device != s->device)
        return sfail(s, TPM_EINVAL, "context on another device");
    for (int k = 0; k < kMaxSlots; k++)
        if (s->slot_ticket[k] && s->slot_ctx[k] == c)
            return sfail(s, TPM_ESTATE, "the context already has a request in flight");
    if (s->free_slots.empty())
        return sfail(s, TPM_ESTATE, "every request slot is in use");
    // the context's earlier work (its build, the inputs of this request) is
    // complete before the request is published
    Work w;
    TPM_TRY(work_of_ctx(c, true, w));
    const size_t esz = c->P.precision == TPM_FP32 ? 4 : 8;
    if (step) {
        TPM_TRY(ensure(c, c->srv_an, (size_t)c->n * 8));
        if (mesh) {
            TPM_TRY(ensure(c, c->srv_pm, (size_t)4 * c->n * esz));
            if (!c->pm_ready) {
                TPM_TRY(pm_solve(c));
                c->pm_ready = 1;
            }
        }
    }
    TPM_HIP(c, hipStreamSynchronize(c->stream));
    // trees are read through the scalar cache: after any rebuild or free
    // since the running kernel started, drain it and launch it again
    if (running(s) && memory_epoch() != s->launch_epoch)
        TPM_TRY(drain(s, 2u));
    // a launch takes at most kRelaunch requests (descriptors unique per launch)
    if (running(s) && s->published - s->published_at_launch >= kRelaunch)
        TPM_TRY(drain(s, 2u));
    const int sid = s->free_slots.back();
    s->free_slots.pop_back();
    SrvReq R{};
    wk::fill_args(c, step ? (const double *)c->srv_an.p : anorm, w, R.A);
    R.A.coherent = 1u;  // later items of the request read the results in this kernel
    R.idx = idx;
    R.rank = (const int32_t *)c->rank.p;
    R.mark = w.mark;
    R.slot = w.slot;
    R.counts = w.counts;
    R.acc = acc;
    R.nint = nint;
    R.err = (uint32_t *)c->err_flag.p;
    R.n_act = (uint32_t)n_act;
    R.epoch = w.epoch;
    R.clear = w.clear ? 1u : 0u;
    R.variant = (opening == TPM_OPEN_REL ? 1u : 0u) | (c->P.pm_grid > 0 ? 2u : 0u) |
                ((uint32_t)wk::walk_variant(c, n_act) << 5) | (c->P.periodic ? 8u : 0u) |
                (c->mixed ? 16u : 0u);
    R.flags = (step ? kStep : 0u) | (mesh ? kMesh : 0u);
    if (mesh) {
        R.mg = pmk::mesh_geom(c);
        R.phi = c->mesh_phi.p;
        R.res_pm = c->srv_pm.p;
        R.acc_pm = acc_pm;
    }
    R.anorm_out = step ? (double *)c->srv_an.p : nullptr;
    R.ticket = s->next_ticket++;
    R.slot_id = (uint32_t)sid;
    R.desc = (uint32_t)(R.ticket % kDescRing);
    s->host->done[sid] = 0;
    std::memcpy(&s->host->ring[s->published % kMaxSlots], &R, sizeof(SrvReq));
    s->slot_ticket[sid] = R.ticket;
    s->slot_ctx[sid] = c;
    s->published++;
    __atomic_store_n(&s->host->tail, (unsigned long long)s->published, __ATOMIC_RELEASE);
    if (!running(s))
        TPM_TRY(launch(s));
    *ticket = R.ticket;
    return TPM_OK;
}

}  // namespace

int tpm_server_submit(tpm_server *s, tpm_ctx *c, int32_t opening, int64_t n_act,
                      const int32_t *idx, const double *anorm, void *acc, uint32_t *nint,
                      uint64_t *ticket) {
    return submit_impl(s, c, false, opening, n_act, idx, anorm, acc, nullptr, nint, ticket);
}

int tpm_server_submit_step(tpm_server *s, tpm_ctx *c, int64_t n_act, const int32_t *idx,
                           void *acc, void *acc_pm, uint32_t *nint, uint64_t *ticket) {
    return submit_impl(s, c, true, TPM_OPEN_REL, n_act, idx, nullptr, acc, acc_pm, nint,
                       ticket);
}

// 1: the request finished (outputs complete and visible); 0: pending.
int tpm_server_poll(tpm_server *s, uint64_t ticket) {
    if (!s || ticket == 0)
        return TPM_EINVAL;
    int sid = -1;
    for (int k = 0; k < kMaxSlots; k++)
        if (s->slot_ticket[k] == ticket)
            sid = k;
    if (sid < 0)
        return 1;  // already reported
    if (__atomic_load_n(&s->host->done[sid], __ATOMIC_ACQUIRE) == ticket + 1ull) {
        s->slot_ticket[sid] = 0;
        s->slot_ctx[sid] = nullptr;
        s->free_slots.push_back(sid);
        return 1;
    }
    TPM_TRY(keep_alive(s));
    return 0;
}

int tpm_server_wait(tpm_server *s, uint64_t ticket) {
    for (;;) {
        const int r = tpm_server_poll(s, ticket);
        if (r != 0)
            return r < 0 ? r : TPM_OK;
        std::this_thread::yield();
    }
}

int tpm_server_info(const tpm_server *s, int64_t *launches, int64_t *in_flight) {
    if (!s)
        return TPM_EINVAL;
    if (launches)
        *launches = s->launches;
    if (in_flight) {
        int64_t k = 0;
        for (uint64_t t : s->slot_ticket)
            k += t != 0;
        *in_flight = k;
    }
    return TPM_OK;
}

}  // extern "C"
