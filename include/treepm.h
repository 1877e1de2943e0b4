/*
 * treepm.h -- C ABI of the MI355X (gfx950) TreePM gravity library.
 *
 * The library computes the gravitational accelerations of the currently
 * active particles of an N-body system by the TreePM method of the Arepo code
 * (Weinberger, Springel & Pakmor, "The AREPO public code release", ApJS 2020):
 *
 *   tpm_build_tree      Sec. 3.1  enclosing cube, Peano-Hilbert keys (the
 *                                 ordering of Sec. 8), radix sort, octree with
 *                                 monopole moments, rebuilt for every call
 *                                 sequence (no dynamic updates)
 *   tpm_compute_forces  Sec. 3.1  tree walk with the relative or geometric
 *                                 opening criterion and the 1.2 L box rule;
 *                       Sec. 3.2  spline softening (zero-lag potential -Gm/eps,
 *                                 Newtonian beyond 2.8 eps);
 *                       Sec. 3.4  short-range truncation and cutoff when a PM
 *                                 mesh is configured
 *   tpm_pm_long_range   Sec. 3.3/3.4  CIC deposit, FFT Poisson solve with the
 *                                 long-range Gaussian filter and CIC
 *                                 deconvolution, four-point finite difference,
 *                                 CIC interpolation; periodic boxes, or
 *                                 isolated systems on a zero-padded mesh
 *   tpm_build_tree_eps  Sec. 3.2  individual softening lengths
 *   tpm_kick, tpm_drift, tpm_time_bins, tpm_select_bins, tpm_gather
 *                       Sec. 7    leapfrog with power-of-two time bins and
 *                                 the split-Hamiltonian variant
 *   tpm_batch_*         many systems' walks in one persistent launch
 *
 * Conventions for every entry point:
 *   - All particle arrays are DEVICE pointers (HIP global memory), borrowed
 *     for the duration of the stream work the call enqueues; the library never
 *     frees or writes caller inputs (the integration kernels update the
 *     velocity, position and bin arrays they are given).  Outputs are
 *     written by kernels on the
 *     context's stream; they are valid once that stream has reached the call.
 *   - Returns TPM_OK (0) or a negative error code.  Arguments are validated on
 *     the host before anything is enqueued: on an error no output is written.
 *     Index arrays live on the device and are checked there: an out-of-range
 *     index yields NaN outputs for that position and sets a sticky device flag
 *     that tpm_check() reports (and clears).
 *   - Not thread-safe per context; different contexts are independent.
 *   - Layouts: "[3][n]" means three contiguous planes x, y, z of n values.
 */
#ifndef TREEPM_H
#define TREEPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPM_OK 0
#define TPM_EINVAL (-1)   /* invalid argument or parameter */
#define TPM_ENOMEM (-2)   /* device or pinned-host allocation failed */
#define TPM_EDEVICE (-3)  /* a HIP runtime call failed (text in tpm_last_error) */
#define TPM_ESTATE (-4)   /* call out of order (e.g. forces before a build) */
#define TPM_EINDEX (-5)   /* tpm_check(): an active index was out of range */

#define TPM_OPEN_BH 0     /* geometric criterion  L > theta d            (Sec. 3.1) */
#define TPM_OPEN_REL 1    /* relative  G m L^2 / d^4 > alpha |a_old|      (Sec. 3.1) */

#define TPM_FP64 0        /* FP64 walk: bit-compatible with the FP64 reference contract */
#define TPM_FP32 1        /* FP32 walk on node-relative offsets, FP64 moments */

/* Run-time parameters (the gravity parameters of the paper's Table 1). */
typedef struct tpm_params {
    int32_t periodic;       /* 1: periodic cube of side box_size (requires pm_grid > 0) */
    int32_t precision;      /* TPM_FP64 or TPM_FP32 (walk and mesh arithmetic) */
    int32_t want_potential; /* 1: compute potentials too */
    int32_t pm_grid;        /* PM mesh cells per side; 0: no PM.  Periodic: power of two,
                               8..1024, the mesh tiles the box.  Isolated (periodic == 0,
                               Sec. 3.3 zero padding): power of two, 16..256; the mesh
                               spans the root cube in pm_grid - 4 cells with two spare
                               cells per side and is transformed zero-padded at
                               (2 pm_grid)^3 */
    double box_size;        /* periodic box side (ignored when periodic == 0) */
    double G;               /* gravitational constant (> 0) */
    double eps;             /* softening length; spline support 2.8 eps (> 0) */
    double theta;           /* ErrTolTheta (>= 0) */
    double alpha;           /* ErrTolForceAcc (> 0) */
    double asmth;           /* ASMTH: r_s = asmth * mesh spacing (> 0 with PM): periodic
                               box_size / pm_grid, isolated L_root / (pm_grid - 4) with
                               L_root the root cube of the last build */
    double rcut;            /* RCUT: short-range cutoff r_cut = rcut * r_s (> 0 with PM) */
    double shift[3];        /* root placement in [0,1)^3: non-periodic, fraction of the
                               slack of the power-of-two root cube; periodic, box shift
                               as a fraction of box_size (Sec. 3.1, random placement) */
} tpm_params;

typedef struct tpm_ctx tpm_ctx;

/* Create a context bound to a HIP stream (NULL: the null stream) on the
 * current device.  Validates *p (TPM_EINVAL).  No device memory is allocated
 * until the first build; each buffer is then allocated when first needed and
 * reallocated when a larger build needs more.  *out receives the context,
 * NULL on error. */
int tpm_create(const tpm_params *p, void *hip_stream, tpm_ctx **out);

/* Create a context whose device memory is one arena of arena_bytes, allocated
 * here (the memory manager of Sec. 9.4: one allocation, carved by the
 * library); arena_bytes 0 is tpm_create.  No later call allocates or frees
 * device memory.  A build releases the previous build's buffers and carves
 * every per-particle buffer at once; buffers kept across builds (mesh,
 * tables, flags) sit at the arena's end.  A call that would need more than
 * the arena holds returns TPM_ENOMEM before it writes any output (a build
 * then leaves the context without a tree).  tpm_bytes_needed(p, n) bytes
 * hold every call on trees of at most n particles and 2.5 n + 64 entries
 * (any input without many near-coincident particles).  Rebuilding must not
 * overlap work still reading the context on another stream (the resident
 * server).  TPM_EINVAL for invalid parameters or arena_bytes < 0,
 * TPM_ENOMEM when the arena cannot be allocated. */
int tpm_create_arena(const tpm_params *p, void *hip_stream, int64_t arena_bytes,
                     tpm_ctx **out);

/* Free every device and host buffer of the context (synchronises its stream). */
int tpm_destroy(tpm_ctx *ctx);

/* Text of the last error of this context (never NULL; "" when none). */
const char *tpm_last_error(const tpm_ctx *ctx);

/* Rebind the context to another stream. */
int tpm_set_stream(tpm_ctx *ctx, void *hip_stream);

/* Upper bound of the device bytes a context holds for builds of at most n
 * particles (trees of at most 2.5 n + 64 entries) and every call on them
 * (forces, mesh, resident-server steps, time-bin selections), with or
 * without individual softening, in either allocation mode: the admission
 * estimate for a memory budget and a sufficient arena size.  Returns -1 on
 * invalid parameters. */
int64_t tpm_bytes_needed(const tpm_params *p, int64_t n);

/* Device bytes the context holds now (an arena context: the arena size). */
int64_t tpm_bytes_held(const tpm_ctx *ctx);

/* Build the tree (Sec. 3.1) of n >= 1 particles.
 * x, y, z: device double[n] positions; periodic inputs must lie in
 *          [0, box_size) (other values are folded by one box length and then
 *          clamped to the root cube).
 * mass:    device double[n], or NULL for equal masses 1/n.
 * Steps: root cube -> 63-bit Peano-Hilbert keys -> stable radix sort (ties by
 * index) -> depth-first threaded octree (internal node = cell holding >= 2
 * particles; a depth-21 cell holding several particles lists them in index
 * order) -> FP64 monopole moments, children summed in curve order.
 * Synchronises the stream once (to size the node arrays).  Invalidates any
 * cached PM mesh. */
int tpm_build_tree(tpm_ctx *ctx, int64_t n, const double *x, const double *y,
                   const double *z, const double *mass);

/* As tpm_build_tree, with an individual softening length per particle
 * (Sec. 3.2: softening set per particle or per type).
 * eps: device double[n] (> 0, finite; build order), or NULL for params.eps
 *      for all (then identical to tpm_build_tree).
 * A pair interacts with the larger of its two spline supports 2.8 eps; every
 * tree entry carries the largest support of its particles; a node whose
 * support exceeds the target's is opened when the target lies within that
 * support of the node's centre of mass, and otherwise interacts with the
 * larger of the two supports.  A non-positive or non-finite value is found
 * during the build: TPM_EINVAL, no tree.  The setting holds until the next
 * build. */
int tpm_build_tree_eps(tpm_ctx *ctx, int64_t n, const double *x, const double *y,
                       const double *z, const double *mass, const double *eps);

/* Random placement of the tree domain (Sec. 3.1: each tree construction
 * places the root anew so that force errors decorrelate in time; a periodic
 * box is shifted as a whole by a new random vector).  shift: host double[3],
 * each in [0, 1): non-periodic, the fraction of the root cube's slack below
 * the particles' minimum along each axis; periodic, the shift of the box
 * origin as a fraction of box_size.  The caller draws the numbers; they apply
 * to every build that follows (the initial value is params.shift) and leave
 * the current tree and a cached mesh unchanged.  TPM_EINVAL for a value
 * outside [0, 1) or NaN (the setting is then unchanged). */
int tpm_set_shift(tpm_ctx *ctx, const double *shift);

/* Tree force on the active particles (Sec. 3.1, 3.2, 3.4).
 * opening:     TPM_OPEN_BH or TPM_OPEN_REL.
 * n_act:       number of active particles (>= 0).
 * active_idx:  device int32[n_act], indices into the build's particle order,
 *              any order; duplicates are allowed (each gets the same result).
 * a_old_norm:  device double[n] in build order, |a| of the previous force
 *              (needed by TPM_OPEN_REL; ignored by TPM_OPEN_BH, may be NULL).
 * acc:         device [3][n_act] in active_idx order; double for TPM_FP64,
 *              float for TPM_FP32.  With a PM mesh this is the short-range
 *              (truncated) part only; add tpm_pm_long_range for the total.
 * pot:         device [n_act] of the same type, or NULL.
 * n_interactions: device uint32[n_act] node + particle interactions per
 *              target (the cost factor g_i of Sec. 8), or NULL.
 * Results are deterministic.  Small active sets (at most 4096 targets, or
 * 65536 in trees of 2^22 particles or more) are walked with one wavefront per
 * target, which adds a target's interactions in another order than larger
 * sets do: its force may then differ in the last bits between sets of the
 * two kinds; interaction counts never differ.
 * Enqueues work only; does not synchronise. */
int tpm_compute_forces(tpm_ctx *ctx, int32_t opening, int64_t n_act, const int32_t *active_idx,
                       const double *a_old_norm, void *acc, void *pot,
                       uint32_t *n_interactions);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): tpm_compute_forces
 * with the same arguments, kernels and results, whose per-call working
 * memory (active-set marks and slot lists, compaction counts, results in
 * curve order) lives in one fixed device array of the library instead of the
 * context's buffers.  It calls no hipMalloc, hipFree or other allocating
 * routine and records no timer events.  Limit: trees of at most
 * tpm_noalloc_max_n() = 2^20 particles (TPM_EINVAL beyond, before anything
 * is enqueued); the array takes 52 MiB on every GPU the library runs on,
 * held until the process ends.  All calls on one GPU share that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race;
 * each call clears what it needs.  The tree itself comes from
 * tpm_build_tree, which does allocate.  TPM_EDEVICE if the array's address
 * could not be looked up when the context was created. */
int tpm_compute_forces_noalloc(tpm_ctx *ctx, int32_t opening, int64_t n_act,
                               const int32_t *active_idx, const double *a_old_norm, void *acc,
                               void *pot, uint32_t *n_interactions);
int64_t tpm_noalloc_max_n(void);

/* Long-range PM acceleration at the active particles (Sec. 3.3, 3.4).
 * Requires pm_grid > 0 (else TPM_EINVAL).  Periodic box: Green's function
 * -4 pi G exp(-k^2 r_s^2) / k^2, mean density removed.  Isolated system:
 * zero-padded mesh, Green's function = the transform of the sampled
 * long-range kernel -G erf(r / 2 r_s) / r (built once per context).  Both
 * divide by the CIC deconvolution.  The mesh is solved from ALL particles
 * of the last build on first use after that build and cached; every call
 * interpolates.  acc: device [3][n_act], pot: device
 * [n_act] or NULL (written whenever given, whatever want_potential says),
 * dtype as in tpm_compute_forces.  Does not synchronise. */
int tpm_pm_long_range(tpm_ctx *ctx, int64_t n_act, const int32_t *active_idx, void *acc,
                      void *pot);

/* Verification export of the mesh of the last PM solve (Sec. 3.3), solving
 * it first if no solve has run since the build.  rho: host double[M^3], the
 * CIC-deposited mass density of all particles of the build (periodic: mass
 * per unit volume on the pm_grid^3 mesh; isolated: mass per cell of the
 * zero-padded (2 pm_grid)^3 mesh); phi: host double[M^3], the potential on
 * the same mesh (converted from float in TPM_FP32).  Layout (i M + j) M + k,
 * i along x.  Either pointer may be NULL.  TPM_EINVAL without a mesh,
 * TPM_ESTATE before a build.  Synchronises. */
int tpm_export_mesh(tpm_ctx *ctx, double *rho, double *phi);

/* |a| per particle for the relative criterion of the next pass (Sec. 3.1:
 * |a| of the previous force computation).  For k < n_act:
 *   out[active_idx[k]] = |acc_a[:,k] + acc_b[:,k]|  (computed in double)
 * acc_a, acc_b: device [3][n_act] of the context's dtype (acc_b may be NULL,
 * e.g. the tree part and the PM part of a TreePM force); out: device
 * double[n] in build order (entries of inactive particles are untouched).
 * Out-of-range indices are skipped and flagged for tpm_check. */
int tpm_accel_norm(tpm_ctx *ctx, int64_t n_act, const int32_t *active_idx, const void *acc_a,
                   const void *acc_b, double *out);

/* Measurement: when enabled, the library records HIP events on its stream
 * immediately around the kernels of one class, so the elapsed time is the
 * kernels' own duration.  tpm_timing_read synchronises the stream, returns
 * the summed milliseconds and the number of timed launches of class kind
 * since the last read, and resets them. */
#define TPM_TIMER_WALK 0       /* tree-walk kernel, geometric criterion */
#define TPM_TIMER_BUILD 1      /* whole tree build (keys .. moments) */
#define TPM_TIMER_PM_SOLVE 2   /* deposit + FFT solve */
#define TPM_TIMER_PM_INTERP 3  /* difference + interpolation kernel */
#define TPM_TIMER_SORT 4       /* radix sort within the build */
#define TPM_TIMER_WALK_REL 5   /* tree-walk kernel, relative criterion */
#define TPM_TIMER_KEYS 6       /* root cube and Peano-Hilbert keys (within the build) */
#define TPM_TIMER_GATHER 7     /* gather into curve order (within the build) */
#define TPM_TIMER_TOPOLOGY 8   /* depth-first entries: counts and scans, then emission
                                  (two records per build) */
#define TPM_TIMER_MOMENTS 9    /* monopole moments and FP32 records (within the build) */
#define TPM_TIMER_DEPOSIT 10   /* mesh clear and CIC deposit (within the solve) */
#define TPM_TIMER_FFT 11       /* the five FFT passes with the Green's function */
#define TPM_TIMER_KINDS 12
int tpm_timing_enable(tpm_ctx *ctx, int on);
int tpm_timing_read(tpm_ctx *ctx, int kind, double *ms, int64_t *launches);

/* As tpm_timing_read, but returns each timed launch's milliseconds in launch
 * order: ms receives min(cap, *launches) values (host array), *launches the
 * number of launches recorded; the records are reset either way. */
int tpm_timing_durations(tpm_ctx *ctx, int kind, double *ms, int64_t cap, int64_t *launches);

/* Measured roofline denominators (measurement only, not part of the method):
 * tpm_probe_fma times dependent vector FMAs (eight chains per lane, sixteen
 * wavefronts per SIMD) in TPM_FP32 (unpacked, as the library is built) or
 * TPM_FP64 and returns the best of five launches in TFLOP/s (FMA = 2 flops);
 * sink: device memory of at least 8 bytes (never written in practice).
 * tpm_probe_copy copies bytes (a multiple of 16) from src to dst (device
 * buffers) and returns read + write bytes per second of the best of five
 * launches, in GB/s.  Both run on hip_stream on the current device and
 * synchronise it. */
int tpm_probe_fma(int32_t precision, void *sink, void *hip_stream, double *tflops);
int tpm_probe_copy(const void *src, void *dst, int64_t bytes, void *hip_stream, double *gbps);

/* Synchronise the stream and report sticky device-side errors
 * (TPM_EINDEX for an out-of-range active index); clears them. */
int tpm_check(tpm_ctx *ctx);

/* Sizes of the current tree: particles, depth-first entries (nodes +
 * particles), and the root frame {x0, y0, z0, L_root}.  Synchronises. */
int tpm_tree_info(tpm_ctx *ctx, int64_t *n, int64_t *n_entries, double *frame4);

/* Copy the tree to caller-owned HOST buffers for verification (any pointer
 * may be NULL; array sizes are n_entries or n as noted).  Entry e, in
 * depth-first order: level[e] (0..21; -1 for a particle entry), first[e]
 * (rank of its first particle in key order), count[e] (particles below),
 * skip[e] (index of the entry after its subtree), pidx[e] (build index of the
 * particle, -1 for nodes), mass[e], com[3][n_entries] (centre of mass, tree
 * frame), cen[3][n_entries] (geometric centre of nodes, position of
 * particles); key[n] sorted keys and perm[n] build index of the particle of
 * each rank.  Synchronises. */
int tpm_export_tree(tpm_ctx *ctx, int32_t *level, int64_t *first, int64_t *count,
                    int64_t *skip, int64_t *pidx, double *mass, double *com, double *cen,
                    uint64_t *key, int64_t *perm);

/* ---- Serving: continuous batching over many systems ---------------------
 * A batch stages tree-force requests (one per context per batch) of many
 * resident systems with uneven N and active fractions (the time-step bins of
 * Sec. 7.2) and walks all of them in ONE persistent launch per precision:
 * wavefronts pop work items (a group of 64 curve-adjacent targets of one
 * request) from a device counter until the finite list is exhausted.  Every
 * work item runs the same per-group walk as tpm_compute_forces, so each
 * request's result is bit-identical alone and in any mix.
 * All work is enqueued on the batch's stream; the caller orders each
 * context's build (and PM solve) before the launch (same stream or an
 * event).  Potentials are not produced by batches. */
typedef struct tpm_batch tpm_batch;

int tpm_batch_create(void *hip_stream, tpm_batch **out);
int tpm_batch_destroy(tpm_batch *batch);
const char *tpm_batch_last_error(const tpm_batch *batch);

/* Stage one request: arguments as tpm_compute_forces (acc [3][n_act] of the
 * context's dtype, n_interactions nullable).  TPM_EINVAL if the context is
 * already staged in this batch; TPM_ESTATE if it has no tree. */
int tpm_batch_add(tpm_batch *batch, tpm_ctx *ctx, int32_t opening, int64_t n_act,
                  const int32_t *active_idx, const double *a_old_norm, void *acc,
                  uint32_t *n_interactions);

/* Enqueue the staged requests: active-set selection per request, one
 * persistent walk per precision, outputs per request; then clear the
 * stage.  Does not synchronise (except to reuse its pinned staging table
 * after the previous launch). */
int tpm_batch_launch(tpm_batch *batch);

/* ---- Serving: a device-resident request loop ------------------------------
 * A server is one persistent kernel per precision that keeps running while
 * requests arrive: tree-force requests (the same arguments as
 * tpm_compute_forces) for resident contexts of uneven N and uneven active
 * fractions (the time-step bins of Sec. 7.2).  Submitting writes a
 * descriptor into a ring in pinned host memory; the running kernel picks it
 * up, runs the request's phases (active-set marking and compaction in curve
 * order, the per-group walks, the outputs in caller order) as work items
 * interleaved with other requests' items, and stores the request's ticket
 * back into pinned memory when its outputs are complete.  Every work item
 * runs the single-system code, so results are bit-identical to
 * tpm_compute_forces alone or in any mix.  The kernel leaves after idle_ms
 * without work and is launched again by the next submit or poll.
 * Requirements: the context's precision is the server's; one request per
 * context in flight; inputs (the tree, active_idx, a_old_norm) complete
 * before submission -- submit synchronises the context's stream -- and
 * outputs untouched until tpm_server_poll reports the request finished.
 * The running kernels leave room on the chip for other kernels.
 * A context rebuilt while the kernel runs makes the next submit drain the
 * kernel and launch it again.  Potentials are not produced. */
typedef struct tpm_server tpm_server;

/* precision: TPM_FP32 or TPM_FP64; idle_ms in (0, 1e4]: how long the
 * kernel waits for work before it leaves.  Creates its own non-blocking
 * stream on the current device. */
int tpm_server_create(int32_t precision, double idle_ms, tpm_server **out);
/* Stops the kernel, waits for it, frees everything. */
int tpm_server_destroy(tpm_server *server);
const char *tpm_server_last_error(const tpm_server *server);
/* Submit a request (n_act >= 1); *ticket identifies it.  TPM_ESTATE if the
 * context has a request in flight or all 256 request slots are in use. */
int tpm_server_submit(tpm_server *server, tpm_ctx *ctx, int32_t opening, int64_t n_act,
                      const int32_t *active_idx, const double *a_old_norm, void *acc,
                      uint32_t *n_interactions, uint64_t *ticket);
/* The paper's first force computation as one request (Sec. 3.1): the
 * geometric pass, the mesh force when the context has a mesh (Sec. 3.3,
 * 3.4; the mesh is solved first if needed), |a| of their sum for every
 * active particle, and the relative pass with that |a|.  acc: the relative
 * pass's tree force [3][n_act] in caller order; acc_pm: the mesh force
 * [3][n_act] (required exactly when the context has a mesh, else NULL);
 * n_interactions: the relative pass's counts or NULL.  Results equal
 * tpm_compute_forces(BH), tpm_pm_long_range, tpm_accel_norm and
 * tpm_compute_forces(REL) in sequence, bit for bit. */
int tpm_server_submit_step(tpm_server *server, tpm_ctx *ctx, int64_t n_act,
                           const int32_t *active_idx, void *acc, void *acc_pm,
                           uint32_t *n_interactions, uint64_t *ticket);
/* 1 once the request's outputs are complete and visible to the host and to
 * later work on any stream, 0 while pending (never blocks). */
int tpm_server_poll(tpm_server *server, uint64_t ticket);
/* Blocks until tpm_server_poll would return 1. */
int tpm_server_wait(tpm_server *server, uint64_t ticket);
/* Kernel launches so far and requests in flight (either may be NULL). */
int tpm_server_info(const tpm_server *server, int64_t *launches, int64_t *in_flight);

/* ---- time integration (Sec. 7.1-7.3) --------------------------------------
 *
 * Kernels for a leapfrog driver with the power-of-two time-step hierarchy
 * (Sec. 7.2) and the split-Hamiltonian variant (Sec. 7.3).  They run on the
 * context's stream and use its error word for out-of-range indices (reported
 * by tpm_check); positions, velocities, bins and indices are caller-owned
 * device arrays of the n particles in build order.  FP64 arithmetic, products
 * rounded before sums: a kick is v + a dt, a drift x + v dt. */

/* Kick: v[idx[k]] += (acc[k] + b_sign acc_b[k]) * h for k < n_act, with
 * h = 0.5 dt_max 2^-bins[idx[k]] (half the particle's step) if bins is not
 * NULL, else h = dt.  acc, acc_b: device [3][n_act] of the given precision
 * (acc_b may be NULL; b_sign = +1 adds it, e.g. the PM force, -1 subtracts
 * it, e.g. a part's own force to leave the mutual one). */
int tpm_kick(tpm_ctx *ctx, int64_t n, int64_t n_act, const int32_t *idx, int32_t precision,
             const void *acc, const void *acc_b, int32_t b_sign, const int32_t *bins,
             double dt_max, double dt, double *vx, double *vy, double *vz);

/* Drift: x[i] += v[i] dt for i = idx[k] (k < n_act), or for i < n_act when
 * idx is NULL; box > 0 folds the result back into [0, box) by one length. */
int tpm_drift(tpm_ctx *ctx, int64_t n, int64_t n_act, const int32_t *idx, double *x,
              double *y, double *z, const double *vx, const double *vy, const double *vz,
              double dt, double box);

/* Time bins (Sec. 7.1, 7.2) of the listed particles from their acceleration
 * acc (+ acc_b, may be NULL): the largest step dt_max 2^-b, b <= max_bin, not
 * above sqrt(2 C eps / |a|) (eps[i], or eps0 when eps is NULL); a step longer
 * than the current bins[i] only if the tick t (in units of dt_max 2^-max_bin)
 * is a multiple of it, else the longest such step.  Writes bins[i]; adds the
 * count of each new bin to hist[0..max_bin] (device uint32, caller-zeroed).
 * t = 0 (every step synchronised) assigns fresh bins. */
int tpm_time_bins(tpm_ctx *ctx, int64_t n, int64_t n_act, const int32_t *idx,
                  int32_t precision, const void *acc, const void *acc_b, const double *eps,
                  double eps0, double C, double dt_max, int32_t max_bin, int64_t t,
                  int32_t *bins, uint32_t *hist);

/* Order-preserving selection from a list of m particles (list, or 0..m-1
 * when NULL) by their bins: mode 0, those closing a step at tick t (t a
 * multiple of 2^(max_bin - bin)); mode 1, bin <= level; mode 2, bin > level.
 * out (device int32[m]) receives the selected particles (local = 0) or their
 * positions in the list (local = 1); *n_out (host) their number.
 * Synchronises the stream (the count is needed on the host). */
int tpm_select_bins(tpm_ctx *ctx, int64_t m, const int32_t *list, const int32_t *bins,
                    int32_t mode, int64_t t, int32_t level, int32_t max_bin, int32_t local,
                    int32_t *out, int64_t *n_out);

/* dst[k] = src[idx[k]], k < m (device FP64 arrays): positions, masses or
 * softenings of a subset, contiguous for a build over that subset. */
int tpm_gather(tpm_ctx *ctx, int64_t n, int64_t m, const int32_t *idx, const double *src,
               double *dst);

#ifdef __cplusplus
}
#endif

#endif /* TREEPM_H */
