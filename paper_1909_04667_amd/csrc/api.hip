// C ABI of the gfx950 TreePM library: argument validation, buffer ownership,
// error reporting and the verification export.  The hot path lives in
// build.hip, walk.hip and pm.hip.
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "tpm_internal.h"

namespace tpm {

static std::atomic<uint64_t> g_memory_epoch{0};

uint64_t memory_epoch() { return g_memory_epoch.load(std::memory_order_acquire); }
void bump_memory_epoch() { g_memory_epoch.fetch_add(1, std::memory_order_acq_rel); }

int fail(tpm_ctx *c, int code, const std::string &msg) {
    if (c)
        c->err = msg;
    return code;
}

int hip_check(tpm_ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess)
        return TPM_OK;
    const int code = (e == hipErrorOutOfMemory) ? TPM_ENOMEM : TPM_EDEVICE;
    return fail(c, code, std::string(what) + ": " + hipGetErrorString(e));
}

int ensure(tpm_ctx *c, DBuf &b, size_t bytes) {
    if (bytes == 0)
        bytes = 16;
    if (b.cap >= bytes)
        return TPM_OK;
    if (c->arena) {  // carve from the arena: nothing is freed or allocated
        const size_t sz = (bytes + 255) & ~size_t(255);
        if (c->arena_hi - c->arena_lo < sz)
            return fail(c, TPM_ENOMEM,
                        "arena of " + std::to_string(c->arena_size) + " bytes exhausted (" +
                            std::to_string(c->arena_hi - c->arena_lo) + " free, " +
                            std::to_string(sz) + " needed)");
        if (b.persistent) {
            c->arena_hi -= sz;
            b.p = c->arena + c->arena_hi;
        } else {
            b.p = c->arena + c->arena_lo;
            c->arena_lo += sz;
        }
        b.cap = sz;
        return TPM_OK;
    }
    if (b.p) {
        TPM_HIP(c, hipStreamSynchronize(c->stream));
        bump_memory_epoch();
        TPM_HIP(c, hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    const size_t want = bytes + bytes / 8;  // headroom for slightly larger rebuilds
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, TPM_ENOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    b.p = p;
    b.cap = want;
    return TPM_OK;
}

std::vector<DBuf *> all_bufs(tpm_ctx *c) {
    return {&c->frame, &c->bbox, &c->key[0], &c->key[1], &c->idx[0], &c->idx[1],
            &c->hist, &c->scan_tmp, &c->perm, &c->rank, &c->xyzm, &c->ps, &c->ms, &c->qs,
            &c->dR, &c->cnt, &c->base, &c->lvl_cursor, &c->lvl_list, &c->rec64,
            &c->rec32, &c->efirst, &c->ecount, &c->pe, &c->mark, &c->act, &c->slot,
            &c->counters, &c->res, &c->rpot, &c->srv_pm, &c->srv_an,
            &c->err_flag, &c->mesh_q, &c->mesh_c, &c->mesh_phi, &c->twiddle,
            &c->green_axis, &c->green_tab, &c->hs, &c->eh64, &c->eh32, &c->ig_flag,
            &c->ig_off};
}

size_t bytes_held(const tpm_ctx *c) {
    if (c->arena)
        return c->arena_size;
    size_t s = 0;
    for (const DBuf *b : all_bufs(const_cast<tpm_ctx *>(c)))
        s += b->cap;
    return s;
}

void visit_sizes(tpm_ctx *c, const tpm_params &P, int64_t n, int64_t E, bool mixed,
                 const std::function<void(DBuf &, size_t, int)> &f) {
    const size_t N = (size_t)n, NE = (size_t)E;
    const size_t esz = P.precision == TPM_FP32 ? 4 : 8;
    // fixed size, kept across builds
    f(c->frame, sizeof(Frame), 2);
    f(c->counters, 64 * sizeof(uint32_t), 2);
    f(c->lvl_cursor, 32 * sizeof(uint32_t), 2);
    f(c->err_flag, 16, 2);
    // per particle: build (keys, sort, ranks, sorted copies, topology)
    for (int b = 0; b < 2; b++) {
        f(c->key[b], 8 * N, 0);
        f(c->idx[b], 4 * N, 0);
    }
    f(c->hist, std::max(sort_scratch_bytes(n), topology_hist_bytes(n)), 0);
    f(c->scan_tmp, (size_t)compaction_tiles(n) * 4, 0);
    f(c->perm, 4 * N, 0);
    f(c->xyzm, 32 * N, 0);
    f(c->rank, 4 * N, 0);
    f(c->ps, 24 * N, 0);
    f(c->ms, 8 * N, 0);
    f(c->qs, 8 * N, 0);
    f(c->dR, N, 0);
    f(c->cnt, 4 * N, 0);
    f(c->base, 4 * N, 0);
    f(c->pe, 4 * N, 0);
    if (!P.periodic)
        f(c->bbox, bbox_bytes(n), 0);
    if (mixed)
        f(c->hs, 8 * N, 0);
    // per particle: active sets, results, resident-server steps, selections
    f(c->mark, 4 * N, 0);
    f(c->act, 4 * N, 0);
    f(c->slot, 4 * N, 0);
    f(c->res, 4 * N * esz, 0);
    f(c->rpot, N * esz, 0);
    f(c->srv_an, 8 * N, 0);
    if (P.pm_grid > 0)
        f(c->srv_pm, 4 * N * esz, 0);
    f(c->ig_flag, 4 * N, 0);
    f(c->ig_off, 4 * N + 64, 0);
    // per entry
    if (E > 0) {
        f(c->rec64, NE * sizeof(Rec64), 1);
        f(c->efirst, 4 * NE, 1);
        f(c->ecount, 4 * NE, 1);
        f(c->lvl_list, 4 * std::max<size_t>(NE - std::min(NE, N), 1), 1);
        if (P.precision == TPM_FP32)
            f(c->rec32, NE * sizeof(Rec32), 1);
        if (mixed) {
            f(c->eh64, 8 * NE, 1);
            if (P.precision == TPM_FP32)
                f(c->eh32, 4 * NE, 1);
        }
    }
    // mesh, transforms and tables (Sec. 3.3)
    if (P.pm_grid > 0) {
        const size_t M = P.periodic ? (size_t)P.pm_grid : 2 * (size_t)P.pm_grid;
        const size_t n3 = M * M * M;
        f(c->mesh_q, (esz == 8 ? 2 : 1) * n3 * 8, 2);
        f(c->mesh_c, M * M * (M / 2 + 1) * 2 * esz, 2);
        f(c->mesh_phi, n3 * esz, 2);
        f(c->twiddle, M * 2 * esz + 64, 2);
        f(c->green_axis, 2 * M * sizeof(double), 2);
        if (!P.periodic) {
            const size_t gh = (size_t)P.pm_grid + 1;
            f(c->green_tab, gh * gh * gh * sizeof(double), 2);
        }
    }
}

static hipEvent_t take_event(tpm_ctx *c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

int timer_begin(tpm_ctx *c, int kind) {
    if (!c->timing)
        return TPM_OK;
    hipEvent_t e = take_event(c);
    if (!e)
        return fail(c, TPM_EDEVICE, "hipEventCreate failed");
    TPM_HIP(c, hipEventRecord(e, c->stream));
    c->timed[kind].push_back({e, nullptr});
    return TPM_OK;
}

int timer_end(tpm_ctx *c, int kind) {
    if (!c->timing || c->timed[kind].empty() || c->timed[kind].back().second)
        return TPM_OK;
    hipEvent_t e = take_event(c);
    if (!e)
        return fail(c, TPM_EDEVICE, "hipEventCreate failed");
    TPM_HIP(c, hipEventRecord(e, c->stream));
    c->timed[kind].back().second = e;
    return TPM_OK;
}

static void free_all(tpm_ctx *c) {
    bump_memory_epoch();
    for (auto &v : c->timed) {
        for (auto &pr : v) {
            if (pr.first)
                (void)hipEventDestroy(pr.first);
            if (pr.second)
                (void)hipEventDestroy(pr.second);
        }
        v.clear();
    }
    for (hipEvent_t e : c->event_pool)
        (void)hipEventDestroy(e);
    c->event_pool.clear();
    for (DBuf *b : all_bufs(c)) {
        if (b->p && !c->arena)
            (void)hipFree(b->p);
        b->p = nullptr;
        b->cap = 0;
    }
    if (c->arena)
        (void)hipFree(c->arena);
    c->arena = nullptr;
    c->arena_size = c->arena_lo = c->arena_hi = 0;
    c->green_tab_ng = 0;
    c->axis_tables_M = 0;
    if (c->hpin)
        (void)hipHostFree(c->hpin);
    c->hpin = nullptr;
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static const char *validate(const tpm_params *p) {
    if (!p)
        return "params is NULL";
    if (p->precision != TPM_FP64 && p->precision != TPM_FP32)
        return "precision must be TPM_FP64 or TPM_FP32";
    if (!(p->G > 0.0) || !std::isfinite(p->G))
        return "G must be positive";
    if (!(p->eps > 0.0) || !std::isfinite(p->eps))
        return "eps must be positive";
    if (!(p->theta >= 0.0) || !std::isfinite(p->theta))
        return "theta must be >= 0";
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha))
        return "alpha must be positive";
    for (int a = 0; a < 3; a++)
        if (!(p->shift[a] >= 0.0 && p->shift[a] < 1.0))
            return "shift must lie in [0, 1)";
    if (p->periodic) {
        if (!(p->box_size > 0.0) || !std::isfinite(p->box_size))
            return "periodic box_size must be positive";
        if (p->pm_grid == 0)
            return "a periodic box needs the PM mesh (pm_grid > 0)";
    }
    if (p->pm_grid != 0) {
        if (!(p->asmth > 0.0) || !(p->rcut > 0.0) || !std::isfinite(p->asmth) ||
            !std::isfinite(p->rcut))
            return "asmth and rcut must be positive";
        if (p->periodic) {
            if (!is_pow2(p->pm_grid) || p->pm_grid < 8 || p->pm_grid > 1024)
                return "pm_grid must be a power of two in [8, 1024]";
            const double rs = p->asmth * p->box_size / p->pm_grid;
            if (!(p->rcut * rs < 0.5 * p->box_size))
                return "cutoff radius must be below half the box";
        } else {
            // isolated: zero-padded (2 pm_grid)^3 transform
            if (!is_pow2(p->pm_grid) || p->pm_grid < 16 || p->pm_grid > 256)
                return "isolated pm_grid must be a power of two in [16, 256]";
        }
    }
    if (p->want_potential != 0 && p->want_potential != 1)
        return "want_potential must be 0 or 1";
    return nullptr;
}

}  // namespace tpm

using namespace tpm;

extern "C" {

int tpm_create(const tpm_params *p, void *hip_stream, tpm_ctx **out) {
    return tpm_create_arena(p, hip_stream, 0, out);
}

int tpm_create_arena(const tpm_params *p, void *hip_stream, int64_t arena_bytes,
                     tpm_ctx **out) {
    if (!out)
        return TPM_EINVAL;
    *out = nullptr;
    if (validate(p) || arena_bytes < 0)
        return TPM_EINVAL;
    tpm_ctx *c = new (std::nothrow) tpm_ctx();
    if (!c)
        return TPM_ENOMEM;
    c->P = *p;
    c->stream = (hipStream_t)hip_stream;
    // tuning override of the walk variant (0 automatic, 1 shared cursor,
    // 2 independent lanes, 3 one wavefront per target); 1 and 2 give
    // identical results, 3 the same interactions summed in another order
    if (const char *m = std::getenv("TPM_WALK_MODE")) {
        const int v = std::atoi(m);
        c->walk_mode = (v >= 1 && v <= 3) ? v : 0;
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return TPM_EDEVICE;
    }
    noalloc_attach(c->device);
    if (hipHostMalloc((void **)&c->hpin, 256 * sizeof(uint32_t), hipHostMallocDefault) !=
        hipSuccess) {
        delete c;
        return TPM_ENOMEM;
    }
    // buffers kept across builds take the arena's top end
    visit_sizes(c, c->P, 1, 0, false, [](DBuf &b, size_t, int kind) {
        if (kind == 2)
            b.persistent = true;
    });
    if (arena_bytes > 0) {
        void *a = nullptr;
        if (hipMalloc(&a, (size_t)arena_bytes) != hipSuccess) {
            (void)hipGetLastError();
            free_all(c);
            delete c;
            return TPM_ENOMEM;
        }
        c->arena = (unsigned char *)a;
        c->arena_size = (size_t)arena_bytes;
        c->arena_lo = 0;
        // every carved buffer starts on a 256-byte boundary (scalar loads and
        // atomics need aligned addresses): the top end too
        c->arena_hi = (size_t)arena_bytes & ~size_t(255);
    }
    *out = c;
    return TPM_OK;
}

int tpm_destroy(tpm_ctx *c) {
    if (!c)
        return TPM_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
    return TPM_OK;
}

const char *tpm_last_error(const tpm_ctx *c) { return c ? c->err.c_str() : "NULL context"; }

int tpm_set_stream(tpm_ctx *c, void *s) {
    if (!c)
        return TPM_EINVAL;
    c->stream = (hipStream_t)s;
    return TPM_OK;
}

int64_t tpm_bytes_needed(const tpm_params *p, int64_t n) {
    if (validate(p) || n < 1)
        return -1;
    // every buffer at its largest size for n particles and at most 2.5 n + 64
    // entries, with individual softening, plus the headroom (an eighth) and
    // the alignment of either allocation mode
    tpm_ctx tmp;
    tmp.P = *p;
    size_t b = 0;
    visit_sizes(&tmp, *p, n, n * 5 / 2 + 64, true, [&](DBuf &, size_t bytes, int) {
        b += bytes + bytes / 8 + 256;
    });
    return (int64_t)b;
}

int64_t tpm_bytes_held(const tpm_ctx *c) { return c ? (int64_t)bytes_held(c) : -1; }

int tpm_build_tree(tpm_ctx *c, int64_t n, const double *x, const double *y, const double *z,
                   const double *mass) {
    return tpm_build_tree_eps(c, n, x, y, z, mass, nullptr);
}

int tpm_build_tree_eps(tpm_ctx *c, int64_t n, const double *x, const double *y,
                       const double *z, const double *mass, const double *eps) {
    if (!c)
        return TPM_EINVAL;
    if (n < 1 || n > (int64_t(1) << 30))
        return fail(c, TPM_EINVAL, "n must lie in [1, 2^30]");
    if (!x || !y || !z)
        return fail(c, TPM_EINVAL, "positions must not be NULL");
    TPM_HIP(c, hipSetDevice(c->device));
    c->built = 0;
    c->pm_ready = 0;
    bump_memory_epoch();
    c->epoch = 0;  // marks must be cleared before the next active set
    if (c->arena) {
        // the previous build's buffers are released (later work on this
        // stream runs after what was queued before); every per-particle
        // buffer is carved now at its largest size, so that a context whose
        // arena cannot hold them fails here, before any kernel runs
        for (DBuf *b : all_bufs(c))
            if (!b->persistent) {
                b->p = nullptr;
                b->cap = 0;
            }
        c->arena_lo = 0;
        int rc = TPM_OK;
        visit_sizes(c, c->P, n, 0, eps != nullptr, [&](DBuf &b, size_t bytes, int kind) {
            if (rc == TPM_OK && kind == 0)
                rc = ensure(c, b, bytes);
        });
        TPM_TRY(rc);
    }
    if (!c->err_flag.p) {
        TPM_TRY(ensure(c, c->err_flag, 16));
        TPM_TRY(fill_u32(c, (uint32_t *)c->err_flag.p, 0u, 4));
    }
    TPM_TRY(timer_begin(c, TPM_TIMER_BUILD));
    TPM_TRY(build(c, n, x, y, z, mass, eps));
    TPM_TRY(timer_end(c, TPM_TIMER_BUILD));
    c->built = 1;
    return TPM_OK;
}

int tpm_compute_forces(tpm_ctx *c, int32_t opening, int64_t n_act, const int32_t *idx,
                       const double *anorm, void *acc, void *pot, uint32_t *nint) {
    if (!c)
        return TPM_EINVAL;
    if (!c->built)
        return fail(c, TPM_ESTATE, "compute_forces before build_tree");
    if (opening != TPM_OPEN_BH && opening != TPM_OPEN_REL)
        return fail(c, TPM_EINVAL, "opening must be TPM_OPEN_BH or TPM_OPEN_REL");
    if (n_act < 0 || n_act > (int64_t(1) << 31) - 1)
        return fail(c, TPM_EINVAL, "n_act out of range");
    if (n_act > 0 && (!idx || !acc))
        return fail(c, TPM_EINVAL, "active_idx and acc must not be NULL");
    if (opening == TPM_OPEN_REL && n_act > 0 && !anorm)
        return fail(c, TPM_EINVAL, "the relative criterion needs a_old_norm");
    TPM_HIP(c, hipSetDevice(c->device));
    return forces(c, opening, n_act, idx, anorm, acc, pot, nint);
}

int tpm_pm_long_range(tpm_ctx *c, int64_t n_act, const int32_t *idx, void *acc, void *pot) {
    if (!c)
        return TPM_EINVAL;
    if (c->P.pm_grid <= 0)
        return fail(c, TPM_EINVAL, "no PM mesh configured");
    if (!c->built)
        return fail(c, TPM_ESTATE, "pm_long_range before build_tree");
    if (n_act < 0 || n_act > (int64_t(1) << 31) - 1)
        return fail(c, TPM_EINVAL, "n_act out of range");
    if (n_act > 0 && (!idx || !acc))
        return fail(c, TPM_EINVAL, "active_idx and acc must not be NULL");
    TPM_HIP(c, hipSetDevice(c->device));
    if (!c->pm_ready) {
        TPM_TRY(timer_begin(c, TPM_TIMER_PM_SOLVE));
        TPM_TRY(pm_solve(c));
        TPM_TRY(timer_end(c, TPM_TIMER_PM_SOLVE));
        c->pm_ready = 1;
    }
    TPM_TRY(timer_begin(c, TPM_TIMER_PM_INTERP));
    TPM_TRY(pm_interp(c, n_act, idx, acc, pot));
    return timer_end(c, TPM_TIMER_PM_INTERP);
}

int tpm_export_mesh(tpm_ctx *c, double *rho, double *phi) {
    if (!c)
        return TPM_EINVAL;
    if (c->P.pm_grid <= 0)
        return fail(c, TPM_EINVAL, "no PM mesh configured");
    if (!c->built)
        return fail(c, TPM_ESTATE, "export_mesh before build_tree");
    TPM_HIP(c, hipSetDevice(c->device));
    if (!c->pm_ready) {
        TPM_TRY(pm_solve(c));
        c->pm_ready = 1;
    }
    return pm_export(c, rho, phi);
}

int tpm_accel_norm(tpm_ctx *c, int64_t n_act, const int32_t *idx, const void *a, const void *b,
                   double *out) {
    if (!c)
        return TPM_EINVAL;
    if (!c->built)
        return fail(c, TPM_ESTATE, "accel_norm before build_tree");
    if (n_act < 0 || n_act > (int64_t(1) << 31) - 1)
        return fail(c, TPM_EINVAL, "n_act out of range");
    if (n_act > 0 && (!idx || !a || !out))
        return fail(c, TPM_EINVAL, "active_idx, acc_a and out must not be NULL");
    TPM_HIP(c, hipSetDevice(c->device));
    return accel_norm(c, n_act, idx, a, b, out);
}

int tpm_set_shift(tpm_ctx *c, const double *shift) {
    if (!c)
        return TPM_EINVAL;
    if (!shift)
        return fail(c, TPM_EINVAL, "shift must not be NULL");
    for (int a = 0; a < 3; a++)
        if (!(shift[a] >= 0.0 && shift[a] < 1.0))
            return fail(c, TPM_EINVAL, "shift must lie in [0, 1)");
    for (int a = 0; a < 3; a++)
        c->P.shift[a] = shift[a];
    return TPM_OK;
}

int tpm_timing_enable(tpm_ctx *c, int on) {
    if (!c)
        return TPM_EINVAL;
    c->timing = on ? 1 : 0;
    return TPM_OK;
}

// Elapsed milliseconds of every timed launch of one class since the last
// read, in launch order; the events go back to the pool.
static int drain_timer(tpm_ctx *c, int kind, std::vector<float> &out) {
    TPM_HIP(c, hipStreamSynchronize(c->stream));
    out.clear();
    int rc = TPM_OK;
    for (auto &pr : c->timed[kind]) {
        if (pr.first && pr.second && rc == TPM_OK) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, pr.first, pr.second) != hipSuccess)
                rc = fail(c, TPM_EDEVICE, "hipEventElapsedTime failed");
            out.push_back(t);
        }
        if (pr.first)
            c->event_pool.push_back(pr.first);
        if (pr.second)
            c->event_pool.push_back(pr.second);
    }
    c->timed[kind].clear();
    return rc;
}

int tpm_timing_read(tpm_ctx *c, int kind, double *ms, int64_t *launches) {
    if (!c || kind < 0 || kind >= TPM_TIMER_KINDS)
        return TPM_EINVAL;
    std::vector<float> d;
    TPM_TRY(drain_timer(c, kind, d));
    double sum = 0.0;
    for (float t : d)
        sum += t;
    if (ms)
        *ms = sum;
    if (launches)
        *launches = (int64_t)d.size();
    return TPM_OK;
}

int tpm_timing_durations(tpm_ctx *c, int kind, double *ms, int64_t cap, int64_t *launches) {
    if (!c || kind < 0 || kind >= TPM_TIMER_KINDS || cap < 0 || (cap > 0 && !ms))
        return TPM_EINVAL;
    std::vector<float> d;
    TPM_TRY(drain_timer(c, kind, d));
    for (size_t k = 0; k < d.size() && (int64_t)k < cap; k++)
        ms[k] = d[k];
    if (launches)
        *launches = (int64_t)d.size();
    return TPM_OK;
}

int tpm_check(tpm_ctx *c) {
    if (!c)
        return TPM_EINVAL;
    TPM_HIP(c, hipStreamSynchronize(c->stream));
    if (!c->err_flag.p)
        return TPM_OK;
    uint32_t f = 0;
    TPM_HIP(c, hipMemcpy(&f, c->err_flag.p, 4, hipMemcpyDeviceToHost));
    if (f) {
        TPM_TRY(fill_u32(c, (uint32_t *)c->err_flag.p, 0u, 4));
        TPM_HIP(c, hipStreamSynchronize(c->stream));
        return fail(c, TPM_EINDEX, "an active index was out of range");
    }
    return TPM_OK;
}

int tpm_tree_info(tpm_ctx *c, int64_t *n, int64_t *ne, double *frame4) {
    if (!c)
        return TPM_EINVAL;
    if (!c->built)
        return fail(c, TPM_ESTATE, "no tree built");
    TPM_HIP(c, hipStreamSynchronize(c->stream));
    if (n)
        *n = c->n;
    if (ne)
        *ne = c->E;
    if (frame4) {
        for (int a = 0; a < 3; a++)
            frame4[a] = c->frame_host.x0[a];
        frame4[3] = c->frame_host.L;
    }
    return TPM_OK;
}

int tpm_export_tree(tpm_ctx *c, int32_t *level, int64_t *first, int64_t *count, int64_t *skip,
                    int64_t *pidx, double *mass, double *com, double *cen, uint64_t *key,
                    int64_t *perm) {
    if (!c)
        return TPM_EINVAL;
    if (!c->built)
        return fail(c, TPM_ESTATE, "no tree built");
    TPM_HIP(c, hipStreamSynchronize(c->stream));
    const int64_t n = c->n, E = c->E;
    std::vector<Rec64> rec(E);
    std::vector<uint32_t> ef(E), ec(E);
    std::vector<int32_t> pm(n);
    TPM_HIP(c, hipMemcpy(rec.data(), c->rec64.p, E * sizeof(Rec64), hipMemcpyDeviceToHost));
    TPM_HIP(c, hipMemcpy(ef.data(), c->efirst.p, E * 4, hipMemcpyDeviceToHost));
    TPM_HIP(c, hipMemcpy(ec.data(), c->ecount.p, E * 4, hipMemcpyDeviceToHost));
    TPM_HIP(c, hipMemcpy(pm.data(), c->perm.p, n * 4, hipMemcpyDeviceToHost));
    if (key)
        TPM_HIP(c, hipMemcpy(key, c->key[0].p, n * 8, hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < E; e++) {
        const Rec64 &R = rec[e];
        const bool part = (R.meta & kParticleFlag) != 0;
        if (level)
            level[e] = part ? -1 : (int32_t)(R.meta & 0xffu);
        if (first)
            first[e] = ef[e];
        if (count)
            count[e] = ec[e];
        if (skip)
            skip[e] = R.skip;
        if (pidx)
            pidx[e] = part ? pm[ef[e]] : -1;
        if (mass)
            mass[e] = R.mass;
        for (int a = 0; a < 3; a++) {
            if (com)
                com[a * E + e] = R.com[a];
            if (cen)
                cen[a * E + e] = R.cen[a];
        }
    }
    if (perm)
        for (int64_t s = 0; s < n; s++)
            perm[s] = pm[s];
    return TPM_OK;
}

}  // extern "C"
