// Internal declarations of the gfx950 TreePM library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <utility>
#include <vector>

#include "treepm.h"

namespace tpm {

constexpr int kBits = 21;          // bits per axis of the integer coordinate
constexpr int kMaxLevel = 21;      // deepest octree level (63-bit keys)
constexpr int kLevels = kMaxLevel + 1;
constexpr uint32_t kParticleFlag = 1u << 8;
constexpr uint32_t kLeafParentFlag = 1u << 9;  // a cube whose children are all particles

// Root frame of the last build, resident in device memory.
struct Frame {
    double x0[3];     // corner of the root cube (tree frame)
    double L;         // side of the root cube
    double S;         // 2^21 / L
    double box;       // periodic box side (0 when isolated)
    int32_t periodic;
    int32_t pad;
};

// FP64 walk record, one per depth-first entry (64 bytes: one scalar-cache
// line).  Particle entries: com = position, cen = position.
struct alignas(64) Rec64 {
    double com[3];
    double mass;
    double cen[3];
    uint32_t skip;    // index of the entry after this subtree
    uint32_t meta;    // level (bits 0-7) | kParticleFlag
};

// FP32 walk record (32 bytes).  Geometry is exact integer: the centre of the
// cube is C * u with C = (2 P + 1) 2^(21-level), u = L_root 2^-22, P the
// cube's integer corner at its level; a particle uses its depth-21 cell.
// dcom = (centre of mass - centre) rounded to float; gm = G * mass.
// The integer coordinates are stored as C << kRecShift: in a periodic box
// (10 bits) a 32-bit difference then wraps modulo the box of 2^22 units with
// no further work; otherwise (9 bits) every difference of two coordinates
// below 2^22 still fits an int32.  The freed low bits of cx hold the level
// and the particle flag.
constexpr int kRecShiftPer = 10;
constexpr int kRecShiftIso = 9;
constexpr int32_t kRecLevel = 31;     // level, bits 0-4 of cx_meta
constexpr int32_t kRecParticle = 32;  // particle flag, bit 5 of cx_meta
constexpr int32_t kRecLeafParent = 64;  // cube with particle children only, bit 6
struct alignas(32) Rec32 {
    float dx, dy, dz, gm;
    int32_t cx_meta;  // C_x << shift | leaf parent << 6 | particle << 5 | level
    int32_t cy, cz;   // C_y << shift, C_z << shift
    uint32_t skip;
};

struct DBuf {
    void *p = nullptr;
    size_t cap = 0;
    bool persistent = false;  // arena: kept across builds (top end of the arena)
};

}  // namespace tpm

struct tpm_ctx {
    tpm_params P;
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    int64_t n = 0;          // particles of the last build
    int64_t E = 0;          // depth-first entries of the last build
    int built = 0;
    int pm_ready = 0;
    uint32_t epoch = 0;     // active-set marking generation
    int walk_mode = 0;      // 0: automatic, 1: shared cursor, 2: independent lanes,
                            // 3: one wavefront per target
    tpm::Frame frame_host{};
    uint32_t level_count[tpm::kLevels] = {};
    uint32_t level_off[tpm::kLevels + 1] = {};
    // host pinned scratch for small readbacks
    uint32_t *hpin = nullptr;
    // device buffers
    tpm::DBuf frame;            // Frame
    tpm::DBuf bbox;             // per-block min/max partials
    tpm::DBuf key[2], idx[2];   // sort ping-pong
    tpm::DBuf hist;             // radix histograms / offsets
    tpm::DBuf scan_tmp;         // scan block sums
    tpm::DBuf perm, rank;       // rank -> build index, build index -> rank
    tpm::DBuf xyzm;             // caller-order position and mass records [n] (build)
    tpm::DBuf ps, ms, qs;       // sorted positions [3][n], masses, packed q
    tpm::DBuf dR, cnt, base;    // build: neighbour depth, entries per particle
    tpm::DBuf lvl_cursor, lvl_list;
    tpm::DBuf rec64, rec32, efirst, ecount;
    tpm::DBuf pe;               // rank -> entry
    tpm::DBuf mark, act, slot, counters;
    tpm::DBuf res, rpot;        // walk results in slot order ([n][4], [n])
    tpm::DBuf srv_pm, srv_an;   // resident server steps: mesh force (slot order), |a|
    tpm::DBuf err_flag;         // [0] bad active index, [1] bad softening length
    // individual softening (Sec. 3.2): spline supports per particle in curve
    // order, and per entry the largest of its particles (FP64, FP32 copy)
    int mixed = 0;
    tpm::DBuf hs, eh64, eh32;
    // time integration: selection flags and offsets
    tpm::DBuf ig_flag, ig_off;
    // particle mesh
    tpm::DBuf mesh_q;           // fixed-point deposit
    tpm::DBuf mesh_c;           // complex work mesh
    tpm::DBuf mesh_phi;         // real potential
    tpm::DBuf twiddle;          // FFT twiddles
    tpm::DBuf green_axis;       // per-axis k^2 and filter / deconvolution tables
    tpm::DBuf green_tab;        // isolated mesh: transformed kernel, one octant
    int green_tab_ng = 0;       // pm_grid the table was built for (0: none)
    int axis_tables_M = 0;      // mesh size the twiddle and axis tables hold (0: none)
    // device arena (tpm_create_arena): one allocation; per-build buffers are
    // carved upward from its start and released at every build, persistent
    // ones (mesh, tables, flags) downward from its end.  Null: each buffer is
    // its own allocation, made when first needed.
    unsigned char *arena = nullptr;
    size_t arena_size = 0, arena_lo = 0, arena_hi = 0;
    // measurement: event pairs per timer class, and a pool of spare events
    int timing = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed[TPM_TIMER_KINDS];
    std::vector<hipEvent_t> event_pool;
};

namespace tpm {

// Error plumbing ---------------------------------------------------------
int fail(tpm_ctx *c, int code, const std::string &msg);
int hip_check(tpm_ctx *c, hipError_t e, const char *what);
int ensure(tpm_ctx *c, DBuf &b, size_t bytes);
size_t bytes_held(const tpm_ctx *c);
// Every device buffer of a context.
std::vector<DBuf *> all_bufs(tpm_ctx *c);
// Every device buffer a build of n particles with E entries (mixed: with
// individual softening) and the calls after it take, at its largest size:
// f(buffer, bytes, kind), kind 0 per particle, 1 per entry, 2 persistent.
void visit_sizes(tpm_ctx *c, const tpm_params &P, int64_t n, int64_t E, bool mixed,
                 const std::function<void(DBuf &, size_t, int)> &f);
// Scratch of the radix sort of n keys (tile counters, histograms, look-back),
// of the build's per-level node histograms, and of its bounding-box partials.
size_t sort_scratch_bytes(int64_t n);
size_t topology_hist_bytes(int64_t n);
size_t bbox_bytes(int64_t n);
// Count of events that rewrite tree records or free device memory (builds,
// frees), library-wide: a kernel that outlives such an event may hold stale
// scalar-cache lines of the affected addresses.
uint64_t memory_epoch();
void bump_memory_epoch();

#define TPM_TRY(expr)            \
    do {                         \
        int _rc = (expr);        \
        if (_rc != TPM_OK)       \
            return _rc;          \
    } while (0)

#define TPM_HIP(c, expr) TPM_TRY(::tpm::hip_check((c), (expr), #expr))
#define TPM_LAUNCHED(c, name) TPM_TRY(::tpm::hip_check((c), hipGetLastError(), name))

// Working memory of one active-set call: marks and slot maps of the active
// set, per-tile compaction counts, the count of unique actives, and the walk
// results in slot order.  Either the context's own buffers (allocated on
// demand) or a fixed region the caller provides.
struct Work {
    uint32_t *mark = nullptr;   // [n] epoch marks
    uint32_t epoch = 0;         // the mark of this call
    bool clear = false;         // clear the marks [0, n) before marking
    uint32_t *act = nullptr;    // [n] active slots in curve order
    uint32_t *slot = nullptr;   // [n] rank -> position in act
    uint32_t *counts = nullptr; // [ceil(n / scan tile)] compaction tile counts
    uint32_t *nuniq = nullptr;  // [1] number of unique actives
    void *res = nullptr;        // [n][4] results in slot order (dtype of the context):
                                // acceleration and the interaction count's bits
    void *rpot = nullptr;       // [n]
};

// Primitives (prims.hip) ---------------------------------------------------
// Exclusive scan of n uint32 values; total written to d_total if non-null.
int scan_u32(tpm_ctx *c, const uint32_t *in, uint32_t *out, int64_t n, uint32_t *d_total);
// act[0 .. total) = the slots r < n with mark[r] == epoch, increasing;
// slot[r] = the position of r in act; the total goes to *d_total (device);
// counts: compaction_tiles(n) words of scratch.
int compact_marked(tpm_ctx *c, const uint32_t *mark, uint32_t epoch, int64_t n, uint32_t *act,
                   uint32_t *slot, uint32_t *d_total, uint32_t *counts);
int64_t compaction_tiles(int64_t n);
// Stable ascending sort of (key, value) pairs; result lands in key[0]/idx[0].
int radix_sort_pairs(tpm_ctx *c, int64_t n);
int fill_u32(tpm_ctx *c, uint32_t *p, uint32_t v, int64_t n);
int fill_u64(tpm_ctx *c, uint64_t *p, uint64_t v, int64_t n);

// Build (build.hip) --------------------------------------------------------
int build(tpm_ctx *c, int64_t n, const double *x, const double *y, const double *z,
          const double *mass, const double *eps);

// Walk (walk.hip) ----------------------------------------------------------
int forces(tpm_ctx *c, int32_t opening, int64_t n_act, const int32_t *idx, const double *anorm,
           void *acc, void *pot, uint32_t *nint);
// forces() with the working memory given (allocates nothing, records no
// timers when timed = false)
int forces_into(tpm_ctx *c, int32_t opening, int64_t n_act, const int32_t *idx,
                const double *anorm, void *acc, void *pot, uint32_t *nint, const Work &w,
                bool timed);
// the context's own working memory, allocated as needed (results: res and
// rpot too); advances the context's mark epoch
int work_of_ctx(tpm_ctx *c, bool results, Work &w);
int select_active(tpm_ctx *c, int64_t n_act, const int32_t *idx);
int select_active_into(tpm_ctx *c, int64_t n_act, const int32_t *idx, const Work &w);

// Particle mesh (pm.hip) -----------------------------------------------------
int pm_solve(tpm_ctx *c);
int pm_interp(tpm_ctx *c, int64_t n_act, const int32_t *idx, void *acc, void *pot);
// Host copies of the deposited mesh (density, or mass per cell when isolated)
// and of the potential mesh of the last solve (synchronises).
int pm_export(tpm_ctx *c, double *rho, double *phi);

// Allocation-free forces (noalloc.hip): look up this device's scratch array
// (once per device, the device current).
void noalloc_attach(int device);

// Bracket kernels of one timer class with events (no-op unless enabled).
int timer_begin(tpm_ctx *c, int kind);
int timer_end(tpm_ctx *c, int kind);
int accel_norm(tpm_ctx *c, int64_t n_act, const int32_t *idx, const void *a, const void *b,
               double *out);

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace tpm
