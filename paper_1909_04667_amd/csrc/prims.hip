// Device-wide primitives for gfx950: exclusive scan and a stable LSD radix
// sort of (63-bit key, 32-bit index) pairs.  Wave64 throughout: ranks inside
// a wavefront come from 64-bit ballots, across wavefronts from LDS.
#include "tpm_internal.h"

namespace tpm {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;  // 2048

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off)
            v += t;
    }
    return v;
}

// Exclusive scan of one 256-thread block's values; returns the block total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_w, uint32_t &excl) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v, lane);
    if (lane == 63)
        s_w[w] = inc;
    __syncthreads();
    uint32_t wbase = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanBlock / 64; k++) {
        uint32_t t = s_w[k];
        if (k < w)
            wbase += t;
        tot += t;
    }
    excl = wbase + inc - v;
    __syncthreads();
    return tot;
}

// Phase 1: per-tile exclusive scan into out, tile totals into sums.
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const uint32_t *__restrict__ in,
                                                           uint32_t *__restrict__ out,
                                                           int64_t n, uint32_t *sums) {
    __shared__ uint32_t s_data[kScanTile];
    __shared__ uint32_t s_w[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kScanBlock) {
        int64_t i = base + k;
        s_data[k] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanItems], t = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        v[j] = s_data[threadIdx.x * kScanItems + j];
        t += v[j];
    }
    uint32_t excl;
    uint32_t tot = block_excl_scan(t, s_w, excl);
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        s_data[threadIdx.x * kScanItems + j] = excl;
        excl += v[j];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kScanTile; k += kScanBlock) {
        int64_t i = base + k;
        if (i < n)
            out[i] = s_data[k];
    }
    if (threadIdx.x == 0)
        sums[blockIdx.x] = tot;
}

// Phase 2: one block scans the tile totals in place (any count), with total.
__global__ __launch_bounds__(kScanBlock) void k_scan_sums(uint32_t *sums, int64_t nb,
                                                          uint32_t *d_total) {
    __shared__ uint32_t s_w[kScanBlock / 64];
    uint32_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
        int64_t i = b0 + threadIdx.x;
        uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t excl;
        uint32_t tot = block_excl_scan(v, s_w, excl);
        if (i < nb)
            sums[i] = carry + excl;
        carry += tot;
    }
    if (threadIdx.x == 0 && d_total)
        *d_total = carry;
}

// Phase 3: add tile offsets.
__global__ __launch_bounds__(kScanBlock) void k_scan_add(uint32_t *out, int64_t n,
                                                         const uint32_t *sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const uint32_t add = sums[blockIdx.x];
    for (int k = threadIdx.x; k < kScanTile; k += kScanBlock) {
        int64_t i = base + k;
        if (i < n)
            out[i] += add;
    }
}

// Radix sort ---------------------------------------------------------------
//
// Stable LSD sort, eight 8-bit digits, one kernel per digit (a single sweep
// in the manner of Merrill & Garland's decoupled look-back scan).  The eight
// digit histograms of all keys are counted once up front.  A pass's blocks
// take tiles of 8192 keys in the order they start (an atomic tile counter),
// rank their tile stably in LDS, publish the tile's digit counts, and find
// the counts of all earlier tiles by looking back through the published
// words; a tile then writes each digit's keys as one contiguous run.  With
// every tile resident at once, the inclusive counts advance a few tiles per
// look-back round trip, so large tiles (fewer of them) shorten the pass.
constexpr int kSortBlock = 1024;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortBlock * kSortRounds;  // 8192 keys per block
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kRadix = 256;  // digit values; threads 0 .. 255 own one each
constexpr int kPasses = 8;
constexpr int kLook = 4;  // look-back words per step (8 and 16 were slower)
// Look-back word of (tile, digit): flag in bits 32-33, count in bits 0-31.
constexpr uint64_t kAggregate = 1ull << 32;  // this tile's own count
constexpr uint64_t kInclusive = 2ull << 32;  // count of this and all earlier tiles

// The eight digit histograms of all keys (one read of the keys).
__global__ __launch_bounds__(kSortBlock) void k_radix_count(const uint64_t *__restrict__ keys,
                                                            int64_t n,
                                                            unsigned long long *__restrict__ hist) {
    __shared__ uint32_t h[kPasses][kRadix];
    for (int k = threadIdx.x; k < kPasses * kRadix; k += kSortBlock)
        (&h[0][0])[k] = 0u;
    __syncthreads();
    // a wavefront takes chunks of 1024 keys, lane l the keys 16 l .. 16 l + 15
    // of a chunk: keys of neighbouring lanes lie 16 apart in the input, whose
    // order is often spatial, which keeps one instruction's atomics apart
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * (kSortBlock / 64);
    for (int64_t ch = (int64_t)blockIdx.x * (kSortBlock / 64) + (threadIdx.x >> 6);
         ch * 1024 < n; ch += nw) {
#pragma unroll 4
        for (int j = 0; j < 16; j++) {
            const int64_t i = ch * 1024 + lane * 16 + j;
            if (i < n) {
                const uint64_t k = keys[i];
#pragma unroll
                for (int p = 0; p < kPasses; p++)
                    atomicAdd(&h[p][(uint32_t)(k >> (8 * p)) & 255u], 1u);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kPasses * kRadix; k += kSortBlock) {
        const uint32_t v = (&h[0][0])[k];
        if (v)
            atomicAdd(&hist[k], (unsigned long long)v);
    }
}

__device__ __forceinline__ uint64_t load_word(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_word(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One digit pass.  ctr: this pass's tile counter; hist: its digit histogram;
// look: its nb x 256 look-back words (all zero on entry).
__global__ __launch_bounds__(kSortBlock) void k_radix_pass(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    unsigned long long *ctr, const unsigned long long *__restrict__ hist, uint64_t *look) {
    __shared__ uint64_t s_k[kSortTile];
    __shared__ uint32_t s_v[kSortTile];
    __shared__ uint32_t s_wc[kSortWaves][kRadix];  // per-wavefront digit counts
    __shared__ uint32_t s_loc[kRadix];          // start of each digit's run in the tile
    __shared__ uint32_t s_out[kRadix];          // output position of a run's first key
    __shared__ uint32_t s_sc[kRadix / 64];
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const bool owner = tid < kRadix;  // thread tid owns digit tid
    if (tid == 0)
        s_tile = (uint32_t)atomicAdd(ctr, 1ull);
    for (int q = tid; q < kSortWaves * kRadix; q += kSortBlock)
        (&s_wc[0][0])[q] = 0u;
    __syncthreads();
    const uint32_t t = s_tile;
    const int64_t base = (int64_t)t * kSortTile;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // 1. stable rank of every key among the keys with its digit in its
    // wavefront's share of the tile (contiguous keys, no block barrier):
    // a ballot match finds the lanes with the same digit, the wavefront's
    // own counter in LDS gives the keys of that digit in earlier rounds
    uint64_t k[kSortRounds];
    uint32_t v[kSortRounds], pos[kSortRounds];
    const int64_t wbase = base + (int64_t)w * (kSortTile / kSortWaves);
#pragma unroll
    for (int r = 0; r < kSortRounds; r++) {
        const int64_t i = wbase + (int64_t)r * 64 + lane;
        const bool valid = i < n;
        k[r] = valid ? kin[i] : 0ull;
        v[r] = valid ? vin[i] : 0u;
        const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        const uint32_t prev = s_wc[w][d];
        pos[r] = prev + rank;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0)
            s_wc[w][d] = prev + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    uint32_t cnt = 0u;  // wavefront counts of digit tid -> wavefront bases
    if (owner) {
#pragma unroll
        for (int q = 0; q < kSortWaves; q++) {
            const uint32_t cq = s_wc[q][tid];
            s_wc[q][tid] = cnt;
            cnt += cq;
        }
    }

    // 2. publish this tile's count of digit tid, then add up the earlier tiles
    uint32_t before = 0u;
    if (owner) {
        uint64_t *mine = look + (size_t)t * kRadix + tid;
        if (t == 0) {
            store_word(mine, kInclusive | cnt);
        } else {
            store_word(mine, kAggregate | cnt);
            // every earlier tile has started (tile numbers follow start order)
            // and publishes its own count before it looks back itself, so each
            // wait below ends
            // (kLook earlier tiles' words per step, loaded together; tile 0 is
            // inclusive, so the walk never reads before it)
            for (int64_t j = (int64_t)t - 1;;) {
                uint64_t wd[kLook];
#pragma unroll
                for (int q = 0; q < kLook; q++)
                    wd[q] = j - q >= 0 ? load_word(look + (size_t)(j - q) * kRadix + tid) : 0ull;
                bool done = false;
                int used = 0;
#pragma unroll
                for (int q = 0; q < kLook; q++) {
                    if (done || used < q || !(wd[q] & (kAggregate | kInclusive)))
                        continue;
                    before += (uint32_t)wd[q];
                    used = q + 1;
                    done = (wd[q] & kInclusive) != 0;
                }
                if (done)
                    break;
                j -= used;
                if (used < kLook)
                    __builtin_amdgcn_s_sleep(1);  // tile j not published yet
            }
            store_word(mine, kInclusive | (before + cnt));
        }
    }

    // 3. runs of the tile in digit order; global start of each run (the
    // digit owners are wavefronts 0 .. kRadix/64 - 1)
    {
        const uint32_t hd = owner ? (uint32_t)hist[tid] : 0u;
        const uint32_t inc = wave_incl_scan(cnt, lane);
        const uint32_t ginc = wave_incl_scan(hd, lane);
        if (owner && lane == 63)
            s_sc[w] = inc;
        __syncthreads();
        uint32_t wb = 0u;
#pragma unroll
        for (int q = 0; q < kRadix / 64; q++)
            wb += q < w ? s_sc[q] : 0u;
        const uint32_t loc = wb + inc - cnt;
        __syncthreads();
        if (owner && lane == 63)
            s_sc[w] = ginc;
        __syncthreads();
        uint32_t gb = 0u;
#pragma unroll
        for (int q = 0; q < kRadix / 64; q++)
            gb += q < w ? s_sc[q] : 0u;
        if (owner) {
            s_loc[tid] = loc;
            s_out[tid] = gb + ginc - hd + before;  // keys with a smaller digit + earlier tiles
        }
    }
    __syncthreads();

    // 4. place the keys in tile order by digit, then write the runs out
#pragma unroll
    for (int r = 0; r < kSortRounds; r++) {
        const int64_t i = wbase + (int64_t)r * 64 + lane;
        if (i < n) {
            const uint32_t d = (uint32_t)(k[r] >> shift) & 255u;
            const uint32_t slot = s_loc[d] + s_wc[w][d] + pos[r];
            s_k[slot] = k[r];
            s_v[slot] = v[r];
        }
    }
    __syncthreads();
    const int64_t m = n - base < kSortTile ? n - base : kSortTile;
    for (int j = tid; j < m; j += kSortBlock) {
        const uint64_t kk = s_k[j];
        const uint32_t d = (uint32_t)(kk >> shift) & 255u;
        const uint32_t g = s_out[d] + ((uint32_t)j - s_loc[d]);
        kout[g] = kk;
        vout[g] = s_v[j];
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

// Compaction of the slots r with mark[r] == epoch, in increasing r: phase 1
// counts them per tile of kScanTile slots.
__global__ __launch_bounds__(kScanBlock) void k_mark_count(const uint32_t *__restrict__ mark,
                                                           int64_t n, uint32_t epoch,
                                                           uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_w[kScanBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t t = 0;
    for (int k = threadIdx.x; k < kScanTile; k += kScanBlock) {
        const int64_t r = base + k;
        t += (r < n && mark[r] == epoch) ? 1u : 0u;
    }
    uint32_t excl;
    const uint32_t tot = block_excl_scan(t, s_w, excl);
    if (threadIdx.x == 0)
        counts[blockIdx.x] = tot;
}

// Phase 2: a tile's offset is the sum of the earlier tiles' counts (read
// here, a few per thread); the tile's own slots are ranked with a block scan.
// Writes act[pos] = r and slot[r] = pos; workgroup 0 also writes the total.
__global__ __launch_bounds__(kScanBlock) void k_mark_compact(
    const uint32_t *__restrict__ mark, int64_t n, uint32_t epoch,
    const uint32_t *__restrict__ counts, uint32_t *__restrict__ act,
    uint32_t *__restrict__ slot, uint32_t *__restrict__ d_total) {
    __shared__ uint32_t s_w[kScanBlock / 64];
    const uint32_t b = blockIdx.x, nb = gridDim.x;
    uint32_t before = 0, all = 0;
    for (uint32_t q = threadIdx.x; q < nb; q += kScanBlock) {
        const uint32_t v = counts[q];
        before += q < b ? v : 0u;
        all += v;
    }
    uint32_t excl;
    const uint32_t off = block_excl_scan(before, s_w, excl);
    const uint32_t total = block_excl_scan(all, s_w, excl);
    if (b == 0 && threadIdx.x == 0)
        *d_total = total;
    // kScanItems rounds of kScanBlock consecutive slots: lanes take
    // consecutive slots, so the outputs of a full set are written contiguously
    const int64_t base = (int64_t)b * kScanTile;
    uint32_t pos = off;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
        const int64_t r = base + j * kScanBlock + threadIdx.x;
        const uint32_t f = (r < n && mark[r] == epoch) ? 1u : 0u;
        uint32_t ex;
        const uint32_t tot = block_excl_scan(f, s_w, ex);
        if (f) {
            act[pos + ex] = (uint32_t)r;
            slot[r] = pos + ex;
        }
        pos += tot;
    }
}

}  // namespace

int64_t compaction_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

int compact_marked(tpm_ctx *c, const uint32_t *mark, uint32_t epoch, int64_t n, uint32_t *act,
                   uint32_t *slot, uint32_t *d_total, uint32_t *counts) {
    if (n <= 0)
        return fill_u32(c, d_total, 0u, 1);
    const int64_t nb = compaction_tiles(n);
    k_mark_count<<<(unsigned)nb, kScanBlock, 0, c->stream>>>(mark, n, epoch, counts);
    TPM_LAUNCHED(c, "k_mark_count");
    k_mark_compact<<<(unsigned)nb, kScanBlock, 0, c->stream>>>(mark, n, epoch, counts, act, slot,
                                                               d_total);
    TPM_LAUNCHED(c, "k_mark_compact");
    return TPM_OK;
}


int scan_u32(tpm_ctx *c, const uint32_t *in, uint32_t *out, int64_t n, uint32_t *d_total) {
    if (n <= 0) {
        if (d_total)
            TPM_TRY(fill_u32(c, d_total, 0u, 1));
        return TPM_OK;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    TPM_TRY(ensure(c, c->scan_tmp, (size_t)nb * sizeof(uint32_t)));
    uint32_t *sums = (uint32_t *)c->scan_tmp.p;
    k_scan_tiles<<<(unsigned)nb, kScanBlock, 0, c->stream>>>(in, out, n, sums);
    TPM_LAUNCHED(c, "k_scan_tiles");
    k_scan_sums<<<1, kScanBlock, 0, c->stream>>>(sums, nb, d_total);
    TPM_LAUNCHED(c, "k_scan_sums");
    if (nb > 1) {
        k_scan_add<<<(unsigned)nb, kScanBlock, 0, c->stream>>>(out, n, sums);
        TPM_LAUNCHED(c, "k_scan_add");
    }
    return TPM_OK;
}

size_t sort_scratch_bytes(int64_t n) {
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    // tile counters, digit histograms, look-back words of every pass
    return (size_t)(kPasses + kPasses * kRadix + kPasses * nb * kRadix) * sizeof(uint64_t);
}

int radix_sort_pairs(tpm_ctx *c, int64_t n) {
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t words = (int64_t)(sort_scratch_bytes(n) / sizeof(uint64_t));
    TPM_TRY(ensure(c, c->hist, (size_t)words * sizeof(uint64_t)));
    unsigned long long *ctr = (unsigned long long *)c->hist.p;
    unsigned long long *hist = ctr + kPasses;
    uint64_t *look = (uint64_t *)(hist + kPasses * kRadix);
    TPM_TRY(timer_begin(c, TPM_TIMER_SORT));
    TPM_TRY(fill_u64(c, (uint64_t *)ctr, 0ull, words));
    const int64_t cb = nb < 1024 ? nb : 1024;
    k_radix_count<<<(unsigned)cb, kSortBlock, 0, c->stream>>>(
        (const uint64_t *)c->key[0].p, n, hist);
    TPM_LAUNCHED(c, "k_radix_count");
    int cur = 0;
    for (int p = 0; p < kPasses; p++) {
        k_radix_pass<<<(unsigned)nb, kSortBlock, 0, c->stream>>>(
            (const uint64_t *)c->key[cur].p, (const uint32_t *)c->idx[cur].p,
            (uint64_t *)c->key[cur ^ 1].p, (uint32_t *)c->idx[cur ^ 1].p, n, 8 * p, ctr + p,
            hist + (size_t)p * kRadix, look + (size_t)p * nb * kRadix);
        TPM_LAUNCHED(c, "k_radix_pass");
        cur ^= 1;
    }
    return timer_end(c, TPM_TIMER_SORT);  // eight passes: the result is back in buffer 0
}

int fill_u32(tpm_ctx *c, uint32_t *p, uint32_t v, int64_t n) {
    if (n <= 0)
        return TPM_OK;
    k_fill_u32<<<grid_for(n, 256), 256, 0, c->stream>>>(p, v, n);
    TPM_LAUNCHED(c, "k_fill_u32");
    return TPM_OK;
}

int fill_u64(tpm_ctx *c, uint64_t *p, uint64_t v, int64_t n) {
    if (n <= 0)
        return TPM_OK;
    k_fill_u64<<<grid_for(n, 256), 256, 0, c->stream>>>(p, v, n);
    TPM_LAUNCHED(c, "k_fill_u64");
    return TPM_OK;
}

}  // namespace tpm
