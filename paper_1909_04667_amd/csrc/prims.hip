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
constexpr int kSortBlock = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortBlock * kSortRounds;  // 4096 keys per block
constexpr int kRadix = 256;

__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const uint64_t *__restrict__ keys,
                                                           int64_t n, int shift,
                                                           uint32_t *__restrict__ hist,
                                                           int nb) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int r = 0; r < kSortRounds; r++) {
        int64_t i = base + (int64_t)r * kSortBlock + threadIdx.x;
        if (i < n)
            atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: each round ranks 256 consecutive keys (4 wavefronts in
// order); within a wavefront equal digits are matched with 8 ballots.
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const uint32_t *__restrict__ offs, int nb) {
    __shared__ uint32_t s_run[kRadix];
    __shared__ uint32_t s_w[kSortBlock / 64][kRadix];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    s_run[tid] = offs[(int64_t)tid * nb + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; r++) {
        const int64_t i = base + (int64_t)r * kSortBlock + tid;
        const bool valid = i < n;
        uint64_t k = valid ? kin[i] : 0ull;
        uint32_t v = valid ? vin[i] : 0u;
        uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        const uint32_t cnt = (uint32_t)__popcll(peers);
#pragma unroll
        for (int q = 0; q < kSortBlock / 64; q++)
            s_w[q][tid] = 0;
        __syncthreads();
        if (valid && rank == 0)
            s_w[w][d] = cnt;
        __syncthreads();
        {   // thread tid owns digit tid: turn wave counts into wave bases
            uint32_t t = s_run[tid];
#pragma unroll
            for (int q = 0; q < kSortBlock / 64; q++) {
                uint32_t c = s_w[q][tid];
                s_w[q][tid] = t;
                t += c;
            }
            s_run[tid] = t;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = s_w[w][d] + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
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

}  // namespace

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

int radix_sort_pairs(tpm_ctx *c, int64_t n) {
    const int nb = (int)((n + kSortTile - 1) / kSortTile);
    TPM_TRY(ensure(c, c->hist, (size_t)2 * kRadix * nb * sizeof(uint32_t)));
    uint32_t *hist = (uint32_t *)c->hist.p;
    uint32_t *offs = hist + (size_t)kRadix * nb;
    int cur = 0;
    TPM_TRY(timer_begin(c, TPM_TIMER_SORT));
    for (int shift = 0; shift < 64; shift += 8) {
        const uint64_t *kin = (const uint64_t *)c->key[cur].p;
        const uint32_t *vin = (const uint32_t *)c->idx[cur].p;
        k_radix_hist<<<nb, kSortBlock, 0, c->stream>>>(kin, n, shift, hist, nb);
        TPM_LAUNCHED(c, "k_radix_hist");
        TPM_TRY(scan_u32(c, hist, offs, (int64_t)kRadix * nb, nullptr));
        k_radix_scatter<<<nb, kSortBlock, 0, c->stream>>>(
            kin, vin, (uint64_t *)c->key[cur ^ 1].p, (uint32_t *)c->idx[cur ^ 1].p, n, shift,
            offs, nb);
        TPM_LAUNCHED(c, "k_radix_scatter");
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
