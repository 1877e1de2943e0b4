// Measured denominators of the roofline figures, taken on the device the
// library runs on: the issue rate of dependent vector FMAs in FP32 (built
// without packed FP32 instructions, as the whole library is) and in FP64,
// and the bandwidth of a streaming copy through HBM.
#include "tpm_internal.h"

namespace tpm {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kChains = 8;   // independent dependency chains per lane
constexpr int kUnroll = 16;  // FMAs per chain per loop iteration

template <typename T>
__global__ __launch_bounds__(kProbeBlock) void k_fma_chains(T *__restrict__ sink, T seed,
                                                            int iters) {
    T a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; k++)
        a[k] = seed + (T)(threadIdx.x + k);
    const T b = (T)0.999, c = (T)0.001;
    for (int i = 0; i < iters; i++) {
#pragma unroll
        for (int u = 0; u < kUnroll; u++)
#pragma unroll
            for (int k = 0; k < kChains; k++)
                a[k] = fma(a[k], b, c);
    }
    T s = (T)0;
#pragma unroll
    for (int k = 0; k < kChains; k++)
        s += a[k];
    if (s == (T)-1)  // never true: keeps the chains live
        sink[0] = s;
}

__global__ __launch_bounds__(kProbeBlock) void k_copy16(const uint4 *__restrict__ src,
                                                        uint4 *__restrict__ dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
    for (int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

// Best of reps timed launches of f on stream st, in milliseconds.
template <typename F>
int best_ms(hipStream_t st, int reps, F f, double *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0)
            (void)hipEventDestroy(e0);
        return TPM_EDEVICE;
    }
    int rc = TPM_OK;
    double best = 1e300;
    for (int r = 0; r < reps + 1 && rc == TPM_OK; r++) {  // first launch: warm-up
        if (hipEventRecord(e0, st) != hipSuccess)
            rc = TPM_EDEVICE;
        f();
        if (hipGetLastError() != hipSuccess)
            rc = TPM_EDEVICE;
        if (rc == TPM_OK && hipEventRecord(e1, st) != hipSuccess)
            rc = TPM_EDEVICE;
        float t = 0.0f;
        if (rc == TPM_OK &&
            (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            rc = TPM_EDEVICE;
        if (rc == TPM_OK && r > 0 && t < best)
            best = t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = best;
    return rc;
}

}  // namespace
}  // namespace tpm

using namespace tpm;

extern "C" {

int tpm_probe_fma(int32_t precision, void *sink, void *hip_stream, double *tflops) {
    if (!sink || !tflops || (precision != TPM_FP64 && precision != TPM_FP32))
        return TPM_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return TPM_EDEVICE;
    const unsigned blocks = (unsigned)cus * 16;  // 16 wavefronts per SIMD
    const int iters = 256;
    double ms = 0.0;
    int rc;
    if (precision == TPM_FP32)
        rc = best_ms(st, 5, [&] {
            k_fma_chains<float><<<blocks, kProbeBlock, 0, st>>>((float *)sink, 1.0f, iters);
        }, &ms);
    else
        rc = best_ms(st, 5, [&] {
            k_fma_chains<double><<<blocks, kProbeBlock, 0, st>>>((double *)sink, 1.0, iters);
        }, &ms);
    if (rc != TPM_OK)
        return rc;
    const double flops = 2.0 * kChains * kUnroll * (double)iters * blocks * kProbeBlock;
    *tflops = flops / (ms * 1e-3) / 1e12;
    return TPM_OK;
}

int tpm_probe_copy(const void *src, void *dst, int64_t bytes, void *hip_stream,
                   double *gbps) {
    if (!src || !dst || !gbps || bytes < 16 || bytes % 16)
        return TPM_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return TPM_EDEVICE;
    const int64_t n16 = bytes / 16;
    const unsigned blocks = (unsigned)cus * 8;
    double ms = 0.0;
    const int rc = best_ms(st, 5, [&] {
        k_copy16<<<blocks, kProbeBlock, 0, st>>>((const uint4 *)src, (uint4 *)dst, n16);
    }, &ms);
    if (rc != TPM_OK)
        return rc;
    *gbps = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;  // read + write
    return TPM_OK;
}

}  // extern "C"
