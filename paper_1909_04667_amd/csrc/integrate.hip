// Time integration kernels (Sec. 7.1-7.3 of the Arepo paper): the leapfrog's
// kicks and drifts, the power-of-two time bins with their synchronisation
// rule, and the order-preserving selections a block-step or split-Hamiltonian
// driver needs (which particles close a step at a tick; the slow and fast
// parts of a set).  All arithmetic in FP64: a kick is v + a dt with
// dt = 0.5 dt_max 2^-bin (or a given dt), a drift x + v dt, products rounded
// before the sums (built with -ffp-contract=off).
#include "tpm_internal.h"

#include <cmath>

namespace tpm {
namespace {

constexpr int kBlock = 256;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_kick(int64_t n_act, const int32_t *__restrict__ idx,
                                                 int64_t n, const T *__restrict__ acc,
                                                 const T *__restrict__ acc_b, double b_sign,
                                                 const int32_t *__restrict__ bins, double dt_max,
                                                 double dt, double *__restrict__ vx,
                                                 double *__restrict__ vy,
                                                 double *__restrict__ vz,
                                                 uint32_t *__restrict__ err) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_act)
        return;
    const int32_t i = idx[k];
    if (i < 0 || (int64_t)i >= n) {
        atomicOr(err, 1u);
        return;
    }
    const double h = bins ? ldexp(0.5 * dt_max, -bins[i]) : dt;
    double *v[3] = {vx, vy, vz};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        double a = (double)acc[c * n_act + k];
        if (acc_b)
            a = b_sign > 0.0 ? a + (double)acc_b[c * n_act + k]
                             : a - (double)acc_b[c * n_act + k];
        v[c][i] = v[c][i] + a * h;
    }
}

__global__ __launch_bounds__(kBlock) void k_drift(int64_t n_act, const int32_t *__restrict__ idx,
                                                  int64_t n, double *__restrict__ x,
                                                  double *__restrict__ y, double *__restrict__ z,
                                                  const double *__restrict__ vx,
                                                  const double *__restrict__ vy,
                                                  const double *__restrict__ vz, double dt,
                                                  double box, uint32_t *__restrict__ err) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_act)
        return;
    const int64_t i = idx ? (int64_t)idx[k] : k;
    if (i < 0 || i >= n) {
        atomicOr(err, 1u);
        return;
    }
    double *p[3] = {x, y, z};
    const double *v[3] = {vx, vy, vz};
#pragma unroll
    for (int c = 0; c < 3; c++) {
        double u = p[c][i] + v[c][i] * dt;
        if (box > 0.0)
            u = u >= box ? u - box : (u < 0.0 ? u + box : u);
        p[c][i] = u;
    }
}

// New time bin of each listed particle from its acceleration: the largest
// step dt_max 2^-b not above sqrt(2 C eps / |a|) (Sec. 7.1); a longer step
// than the current one only if the tick t is a multiple of it (Sec. 7.2).
// hist[b] counts the new bins.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_time_bins(
    int64_t n_act, const int32_t *__restrict__ idx, int64_t n, const T *__restrict__ acc,
    const T *__restrict__ acc_b, const double *__restrict__ eps, double eps0, double C,
    double dt_max, int max_bin, int64_t t, int32_t *__restrict__ bins,
    uint32_t *__restrict__ hist, uint32_t *__restrict__ err) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n_act)
        return;
    const int32_t i = idx[k];
    if (i < 0 || (int64_t)i >= n) {
        atomicOr(err, 1u);
        return;
    }
    double a[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        a[c] = (double)acc[c * n_act + k];
        if (acc_b)
            a[c] = a[c] + (double)acc_b[c * n_act + k];
    }
    const double an = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    int b = 0;
    if (an > 0.0) {
        const double e = eps ? eps[i] : eps0;
        const double dt = sqrt(2.0 * C * e / an);
        while (b < max_bin && ldexp(dt_max, -b) > dt)
            b++;
    }
    const int old = bins[i];
    if (b < old)
        while (b < old && (t & ((int64_t(1) << (max_bin - b)) - 1)) != 0)
            b++;
    bins[i] = b;
    atomicAdd(&hist[b], 1u);
}

// Selection predicates over a list of particles (the list, or 0..n-1):
// 0: closes a step at tick t (t a multiple of 2^(max_bin - bin));
// 1: bin <= level; 2: bin > level.
__global__ __launch_bounds__(kBlock) void k_select_flags(int64_t m,
                                                         const int32_t *__restrict__ list,
                                                         const int32_t *__restrict__ bins,
                                                         int mode, int64_t t, int level,
                                                         int max_bin,
                                                         uint32_t *__restrict__ flag) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m)
        return;
    const int32_t i = list ? list[k] : (int32_t)k;
    const int b = bins[i];
    bool f;
    if (mode == 0)
        f = (t & ((int64_t(1) << (max_bin - b)) - 1)) == 0;
    else if (mode == 1)
        f = b <= level;
    else
        f = b > level;
    flag[k] = f ? 1u : 0u;
}

// Keeps list order: out[off[k]] = (local ? k : list[k]) for flagged k.
__global__ __launch_bounds__(kBlock) void k_select_scatter(int64_t m,
                                                           const int32_t *__restrict__ list,
                                                           const uint32_t *__restrict__ flag,
                                                           const uint32_t *__restrict__ off,
                                                           int local,
                                                           int32_t *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m || !flag[k])
        return;
    out[off[k]] = local ? (int32_t)k : (list ? list[k] : (int32_t)k);
}

__global__ __launch_bounds__(kBlock) void k_gather(int64_t m, const int32_t *__restrict__ idx,
                                                   int64_t n, const double *__restrict__ src,
                                                   double *__restrict__ dst,
                                                   uint32_t *__restrict__ err) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m)
        return;
    const int32_t i = idx[k];
    if (i < 0 || (int64_t)i >= n) {
        atomicOr(err, 1u);
        dst[k] = NAN;
        return;
    }
    dst[k] = src[i];
}

int ensure_err(tpm_ctx *c) {
    if (!c->err_flag.p) {
        TPM_TRY(ensure(c, c->err_flag, 16));
        TPM_TRY(fill_u32(c, (uint32_t *)c->err_flag.p, 0u, 4));
    }
    return TPM_OK;
}

}  // namespace
}  // namespace tpm

using namespace tpm;

extern "C" {

int tpm_kick(tpm_ctx *c, int64_t n, int64_t n_act, const int32_t *idx, int32_t precision,
             const void *acc, const void *acc_b, int32_t b_sign, const int32_t *bins,
             double dt_max, double dt, double *vx, double *vy, double *vz) {
    if (!c)
        return TPM_EINVAL;
    if (n < 1 || n_act < 0 || n_act > (int64_t(1) << 31) - 1)
        return fail(c, TPM_EINVAL, "kick: sizes out of range");
    if (precision != TPM_FP64 && precision != TPM_FP32)
        return fail(c, TPM_EINVAL, "kick: precision must be TPM_FP64 or TPM_FP32");
    if (acc_b && b_sign != 1 && b_sign != -1)
        return fail(c, TPM_EINVAL, "kick: b_sign must be +1 or -1");
    if (!std::isfinite(dt) || !std::isfinite(dt_max))
        return fail(c, TPM_EINVAL, "kick: time steps must be finite");
    if (n_act == 0)
        return TPM_OK;
    if (!idx || !acc || !vx || !vy || !vz)
        return fail(c, TPM_EINVAL, "kick: NULL array");
    TPM_HIP(c, hipSetDevice(c->device));
    TPM_TRY(ensure_err(c));
    const unsigned g = grid_for(n_act, kBlock);
    uint32_t *err = (uint32_t *)c->err_flag.p;
    if (precision == TPM_FP32)
        k_kick<float><<<g, kBlock, 0, c->stream>>>(n_act, idx, n, (const float *)acc,
                                                   (const float *)acc_b, (double)b_sign, bins,
                                                   dt_max, dt, vx, vy, vz, err);
    else
        k_kick<double><<<g, kBlock, 0, c->stream>>>(n_act, idx, n, (const double *)acc,
                                                    (const double *)acc_b, (double)b_sign, bins,
                                                    dt_max, dt, vx, vy, vz, err);
    TPM_LAUNCHED(c, "k_kick");
    return TPM_OK;
}

int tpm_drift(tpm_ctx *c, int64_t n, int64_t n_act, const int32_t *idx, double *x, double *y,
              double *z, const double *vx, const double *vy, const double *vz, double dt,
              double box) {
    if (!c)
        return TPM_EINVAL;
    if (n < 1 || n_act < 0 || n_act > n)
        return fail(c, TPM_EINVAL, "drift: sizes out of range");
    if (!std::isfinite(dt) || !(box >= 0.0) || !std::isfinite(box))
        return fail(c, TPM_EINVAL, "drift: dt must be finite and box >= 0");
    if (n_act == 0)
        return TPM_OK;
    if (!x || !y || !z || !vx || !vy || !vz)
        return fail(c, TPM_EINVAL, "drift: NULL array");
    TPM_HIP(c, hipSetDevice(c->device));
    TPM_TRY(ensure_err(c));
    k_drift<<<grid_for(n_act, kBlock), kBlock, 0, c->stream>>>(
        n_act, idx, n, x, y, z, vx, vy, vz, dt, box, (uint32_t *)c->err_flag.p);
    TPM_LAUNCHED(c, "k_drift");
    return TPM_OK;
}

int tpm_time_bins(tpm_ctx *c, int64_t n, int64_t n_act, const int32_t *idx, int32_t precision,
                  const void *acc, const void *acc_b, const double *eps, double eps0, double C,
                  double dt_max, int32_t max_bin, int64_t t, int32_t *bins, uint32_t *hist) {
    if (!c)
        return TPM_EINVAL;
    if (n < 1 || n_act < 0 || n_act > (int64_t(1) << 31) - 1)
        return fail(c, TPM_EINVAL, "time_bins: sizes out of range");
    if (precision != TPM_FP64 && precision != TPM_FP32)
        return fail(c, TPM_EINVAL, "time_bins: precision must be TPM_FP64 or TPM_FP32");
    if (max_bin < 0 || max_bin > 40 || t < 0)
        return fail(c, TPM_EINVAL, "time_bins: max_bin must lie in [0, 40], t >= 0");
    if (!(C > 0.0) || !(dt_max > 0.0) || !std::isfinite(C) || !std::isfinite(dt_max) ||
        (!eps && !(eps0 > 0.0)))
        return fail(c, TPM_EINVAL, "time_bins: C, dt_max and eps must be positive");
    if (n_act == 0)
        return TPM_OK;
    if (!idx || !acc || !bins || !hist)
        return fail(c, TPM_EINVAL, "time_bins: NULL array");
    TPM_HIP(c, hipSetDevice(c->device));
    TPM_TRY(ensure_err(c));
    const unsigned g = grid_for(n_act, kBlock);
    uint32_t *err = (uint32_t *)c->err_flag.p;
    if (precision == TPM_FP32)
        k_time_bins<float><<<g, kBlock, 0, c->stream>>>(n_act, idx, n, (const float *)acc,
                                                        (const float *)acc_b, eps, eps0, C,
                                                        dt_max, max_bin, t, bins, hist, err);
    else
        k_time_bins<double><<<g, kBlock, 0, c->stream>>>(n_act, idx, n, (const double *)acc,
                                                         (const double *)acc_b, eps, eps0, C,
                                                         dt_max, max_bin, t, bins, hist, err);
    TPM_LAUNCHED(c, "k_time_bins");
    return TPM_OK;
}

int tpm_select_bins(tpm_ctx *c, int64_t m, const int32_t *list, const int32_t *bins,
                    int32_t mode, int64_t t, int32_t level, int32_t max_bin, int32_t local,
                    int32_t *out, int64_t *n_out) {
    if (!c)
        return TPM_EINVAL;
    if (m < 0 || m > (int64_t(1) << 31) - 1 || !n_out)
        return fail(c, TPM_EINVAL, "select_bins: size out of range or n_out NULL");
    if (mode < 0 || mode > 2 || max_bin < 0 || max_bin > 40 || t < 0)
        return fail(c, TPM_EINVAL, "select_bins: bad mode, max_bin or tick");
    *n_out = 0;
    if (m == 0)
        return TPM_OK;
    if (!bins || !out)
        return fail(c, TPM_EINVAL, "select_bins: NULL array");
    TPM_HIP(c, hipSetDevice(c->device));
    TPM_TRY(ensure(c, c->ig_flag, (size_t)m * 4));
    TPM_TRY(ensure(c, c->ig_off, (size_t)m * 4 + 64));
    uint32_t *flag = (uint32_t *)c->ig_flag.p, *off = (uint32_t *)c->ig_off.p;
    uint32_t *total = off + ((m + 15) & ~int64_t(15));
    const unsigned g = grid_for(m, kBlock);
    k_select_flags<<<g, kBlock, 0, c->stream>>>(m, list, bins, mode, t, level, max_bin, flag);
    TPM_LAUNCHED(c, "k_select_flags");
    TPM_TRY(scan_u32(c, flag, off, m, total));
    k_select_scatter<<<g, kBlock, 0, c->stream>>>(m, list, flag, off, local, out);
    TPM_LAUNCHED(c, "k_select_scatter");
    TPM_HIP(c, hipMemcpyAsync(c->hpin + 130, total, 4, hipMemcpyDeviceToHost, c->stream));
    TPM_HIP(c, hipStreamSynchronize(c->stream));
    *n_out = (int64_t)c->hpin[130];
    return TPM_OK;
}

int tpm_gather(tpm_ctx *c, int64_t n, int64_t m, const int32_t *idx, const double *src,
               double *dst) {
    if (!c)
        return TPM_EINVAL;
    if (n < 1 || m < 0 || m > (int64_t(1) << 31) - 1)
        return fail(c, TPM_EINVAL, "gather: sizes out of range");
    if (m == 0)
        return TPM_OK;
    if (!idx || !src || !dst)
        return fail(c, TPM_EINVAL, "gather: NULL array");
    TPM_HIP(c, hipSetDevice(c->device));
    TPM_TRY(ensure_err(c));
    k_gather<<<grid_for(m, kBlock), kBlock, 0, c->stream>>>(m, idx, n, src, dst,
                                                            (uint32_t *)c->err_flag.p);
    TPM_LAUNCHED(c, "k_gather");
    return TPM_OK;
}

}  // extern "C"
