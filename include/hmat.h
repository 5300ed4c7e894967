/*
 * hmat.h — lattice H-matrix library for boundary-element earthquake-sequence
 * models on AMD Instinct MI355X (gfx950).
 *
 * The library builds a lattice H-matrix approximation of an element
 * stiffness matrix and applies it to slip-rate vectors on the GPU.
 *
 *   Method (Ozawa, Ida, Hoshino, Ando, "Large-scale earthquake sequence
 *   simulations on 3D nonplanar faults using the boundary element method
 *   accelerated by lattice H-matrices"):
 *     - stiffness entries: section 2.1, eqs. (5)-(6)
 *     - cluster tree, admissibility, partition: section 3.1.1, eq. (17)
 *     - adaptive cross approximation: section 3.1.2, eqs. (18)-(19)
 *     - H-matrix-vector product: section 3.1.3, eq. (20)
 *     - lattice structure: section 3.2
 *     - rate-and-state right-hand side: section 2.2, eqs. (7)-(13), (21)-(22)
 *
 * Conventions shared by every entry point
 *   - Every call returns hmat_status: HMAT_OK (0) or a negative error code.
 *     No C++ exception crosses this interface.  After an error,
 *     hmat_last_error() returns a message for the calling thread.
 *   - A handle (hmat_t) owns all device memory it allocates: factor storage,
 *     block descriptors, schedules and scratch.  The caller owns every array
 *     passed in; the library never frees or retains caller pointers beyond
 *     the call (except where stated).
 *   - "Device" pointers are addresses returned by hipMalloc (or a PyTorch
 *     CUDA/HIP tensor's data_ptr()) on the device that was current when the
 *     handle was created.  "Host" pointers are ordinary process memory.
 *   - Calls that take a stream are stream-ordered on that hipStream_t
 *     (NULL = the null stream): they enqueue work and return without waiting
 *     for the GPU, unless stated otherwise.
 *   - A handle is not safe to use from two streams or threads at once: its
 *     products share one scratch buffer.
 *   - Vectors at the interface are FP64 in the caller's element order.
 */
#ifndef HMAT_H_
#define HMAT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hmat_s* hmat_t;

typedef enum {
  HMAT_OK = 0,
  HMAT_EINVAL = -1,       /* invalid argument (null pointer, bad size, bad option, bad mesh) */
  HMAT_ENOMEM = -2,       /* host or device allocation failed */
  HMAT_EDEVICE = -3,      /* a HIP runtime call failed (message names it) */
  HMAT_ESTATE = -4,       /* handle in an unusable state */
  HMAT_EUNSUPPORTED = -5  /* valid request the library does not implement */
} hmat_status;

/* Storage precision of the factors on the device.  Products always take and
 * return FP64 vectors and accumulate in FP64. */
typedef enum { HMAT_F64 = 0, HMAT_F32 = 1 } hmat_prec;

/* Product kernel.
 *   HMAT_KERNEL_PLAIN:   two launches over the block list in its natural
 *                        layout (column-major dense blocks and factors).
 *   HMAT_KERNEL_BATCHED: blocks repacked into lane-coalesced panels and
 *                        processed as one list of work units: two launches
 *                        (SPLIT) or one persistent launch (PERSISTENT).  The
 *                        persistent launch's wait for phase 1 is bounded; a
 *                        launch that gives up (never observed) is reported
 *                        as HMAT_EDEVICE by the next hmat_check,
 *                        hmat_profile or rs_rk45_attempt / _step / _run on
 *                        the handle.
 *   HMAT_KERNEL_AUTO:    BATCHED with the schedule picked by hmat_autotune. */
typedef enum {
  HMAT_KERNEL_PLAIN = 0,
  HMAT_KERNEL_BATCHED_SPLIT = 1,
  HMAT_KERNEL_BATCHED_PERSISTENT = 2,
  HMAT_KERNEL_AUTO = 3
} hmat_kernel;

/* Green's function families. */
typedef enum {
  /* Unbounded isotropic medium, all elements rectangles in one plane, slip
   * along a common in-plane direction (closed form; eqs. (5)-(6) with the
   * full-space kernel).  The normal-stress matrix B of such a fault is 0. */
  HMAT_GF_FS_RECT_COPLANAR = 1,
  /* Unbounded isotropic medium, triangular elements of any orientation
   * (nonplanar faults), slip along each element's own in-plane direction.
   * Closed form: the stress of a triangular dislocation loop as a line
   * integral over its three edges (Peach-Koehler), at the centroids.  B is
   * in general nonzero. */
  HMAT_GF_FS_TRIANGLE = 2
} hmat_green_kind;

/* Element mesh (host memory, read during hmat_build only). */
typedef struct {
  int64_t n;               /* number of elements, >= 1 */
  int32_t nvert;           /* vertices per element: 4 (rectangles) or 3 (triangles) */
  const double* verts;     /* n * nvert * 3 coordinates [m], element-major;
                              counter-clockwise seen from the +normal side */
  const double* slip_dir;  /* n * 3 unit slip directions in the element plane */
} hmat_mesh;

typedef struct {
  int32_t kind;            /* hmat_green_kind */
  int32_t component;       /* 0: shear traction along the slip direction (A),
                              1: normal traction, compression positive (B) */
  double mu;               /* rigidity [Pa] */
  double nu;               /* Poisson ratio, in (-1, 0.5) */
} hmat_green;

typedef struct {
  double aca_eps;          /* ACA tolerance of eq. (19), > 0 */
  double eta;              /* admissibility parameter of eq. (17), > 0 */
  int32_t leaf;            /* maximum cluster size of a tree leaf, >= 1 */
  int32_t lattice;         /* lattice blocks per side (power of two); 1 = normal H-matrix */
  int32_t max_rank;        /* rank cap before the dense fallback; 0 = min(m, n) / 2 */
  int32_t prec;            /* hmat_prec: factor storage on the device */
  int32_t kernel;          /* hmat_kernel */
  int32_t n_threads;       /* host threads for construction and packing; 0 = every CPU of the process affinity mask */
  int32_t wg_waves;        /* BATCHED: waves per workgroup (4, 8 or 16); 0 = default */
  int32_t unit_kib;        /* BATCHED: target bytes per work unit in KiB; 0 = default */
  int32_t wg_waves_p1;     /* BATCHED split: waves per workgroup of phase 1 (4, 8, 16);
                              0 = default (4) */
  int32_t max_nrhs;        /* > 0: allocate the buffers of hmat_matmat at creation (needs
                              HMAT_F32 and a BATCHED kernel); 0: none */
  int32_t transpose;       /* 1: also lay out H^T for hmat_matvec_T (doubles the factor
                              storage); 0: hmat_matvec_T returns HMAT_ESTATE */
  int32_t build_device;    /* hmat_build: 1 = evaluate entries and run ACA on the GPU (same
                              rules; blocks beyond rank 64 fall back to the host); 0 = host
                              threads.  Ignored by hmat_build_host. */
  int32_t mm_groups;       /* hmat_matmat: groups of four waves sharing each 64-output slice
                              (1 or 2) in both phases and modes; 3 = phase 2 on pairs of row
                              intervals that stage their common inputs once (phase 1 one
                              group); 0 = per phase and mode the fastest of these, timed at
                              creation (and by hmat_autotune) */
} hmat_opts;

/* Arithmetic of hmat_matmat: FP32 factors and member values are split into
 * bf16 parts (each the bf16 rounding of the remaining error) and the cross
 * products with part indices i + j < parts are accumulated in FP32 on MFMA. */
typedef enum {
  HMAT_MM_BF16X3 = 2,      /* 2 parts, 3 products: about 16 significant bits */
  HMAT_MM_BF16X6 = 3       /* 3 parts (exact FP32), 6 products: FP32-level accuracy */
} hmat_mm_mode;

/* Fill *opts with defaults (eps 1e-6, eta 2, leaf 32, lattice 1, FP64, AUTO,
 * transpose 1). */
void hmat_default_opts(hmat_opts* opts);

/* Statistics of a handle (hmat_info). */
typedef struct {
  int64_t n;               /* matrix order */
  int64_t n_dense;         /* dense (inadmissible) blocks */
  int64_t n_lr;            /* low-rank blocks (rank 0 blocks included) */
  int64_t dense_entries;   /* sum m*n over dense blocks */
  int64_t lr_entries;      /* sum r*(m+n) over low-rank blocks */
  int64_t max_rank;
  int64_t sum_rank;        /* total rank = length of the intermediate vector t */
  int64_t n_leaves;        /* row units of the product (leaf row clusters) */
  int64_t tree_depth;
  int64_t device_bytes;    /* device memory held by the handle */
  int64_t factor_bytes;    /* bytes of stored factors read per product: s*(dense+lr entries) */
  int64_t alg_bytes;       /* algorithmic bytes per single-vector product:
                              factor_bytes + 8N (x) + 16N (y read+write) + 4N (perm) */
  int64_t n_units_p1;      /* BATCHED: work units of phase 1 (t = V^T x) */
  int64_t n_units_p2;      /* BATCHED: work units of phase 2 (y = D x + U t) */
  int32_t prec;
  int32_t kernel;          /* kernel actually used (AUTO resolved) */
  int32_t wg_waves;
  int32_t lattice;
  int32_t wg_waves_p1;
  int32_t mm_groups;       /* hmat_matmat schedule, 4 bits each: BF16x3 phase 1, phase 2,
                              BF16x6 phase 1, phase 2 from the low bits (1 or 2 wave groups, 3
                              pairs of row intervals); 0 without max_nrhs */
} hmat_stats;

/* Host copy of the blocks of a handle, in cluster order (hmat_export /
 * hmat_import).  Block b occupies rows [r0, r0+m) and columns [c0, c0+n) of
 * the cluster-ordered matrix; cluster position k is user element perm[k].
 *   desc[6*b + 0] = kind (0 dense, 1 low rank)
 *   desc[6*b + 1..5] = r0, m, c0, n, rank (0 for dense)
 *   off[b] = first value of the block in values[]:
 *     dense:    m*n values, column-major;
 *     low rank: U (m x rank, column-major) then V (n x rank, column-major),
 *               block = U V^T (the paper's g = U^T, h = V^T, eq. (18)). */
typedef struct {
  int64_t n;
  int64_t nblocks;
  int64_t nvalues;
  const int32_t* perm;     /* n */
  const int64_t* desc;     /* 6 * nblocks */
  const int64_t* off;      /* nblocks */
  const double* values;    /* nvalues */
} hmat_host_blocks;

/*
 * hmat_build — construct the lattice H-matrix of one stiffness matrix.
 * Section 3.1.1 (cluster tree on element centres, eq. (17) admissibility),
 * section 3.2 (lattice: tree cut at depth log2(lattice), each lattice block
 * partitioned on its own), section 3.1.2 (ACA, eqs. (18)-(19), FP64, on host
 * threads or, with opts.build_device, on the current device), then packing
 * and upload of the factors to the current device.
 *   mesh, green, opts: host structs, validated (EINVAL on any bad field,
 *     non-finite coordinate, non-planar or non-rectangular element for the
 *     coplanar kernel, lattice not a power of two or deeper than the tree).
 *   stream: hipStream_t for the uploads; the call returns after they finish.
 *   out: receives the new handle; untouched on error.
 */
hmat_status hmat_build(const hmat_mesh* mesh, const hmat_green* green, const hmat_opts* opts,
                       void* stream, hmat_t* out);

/*
 * hmat_build_host — the construction of hmat_build (same validation, same
 * blocks) without any device work: the handle holds only the FP64 host
 * blocks, for hmat_export / hmat_info / hmat_destroy, e.g. to build on a
 * machine without a GPU and hmat_import elsewhere.  Products, rs_rhs and
 * hmat_autotune on such a handle return HMAT_ESTATE.
 */
hmat_status hmat_build_host(const hmat_mesh* mesh, const hmat_green* green, const hmat_opts* opts, hmat_t* out);

/*
 * hmat_import — create a handle from host blocks (layout of hmat_host_blocks)
 * instead of building them; opts selects prec/kernel/schedule (the
 * construction fields are ignored).  Blocks must tile the n x n matrix
 * exactly once and perm must be a permutation (EINVAL otherwise).  The
 * arrays are copied; the caller keeps ownership.
 */
hmat_status hmat_import(const hmat_host_blocks* blocks, const hmat_opts* opts, void* stream,
                        hmat_t* out);

/*
 * hmat_export — host view of the handle's blocks in FP64 (as built, before
 * any storage rounding).  The pointers in *out are owned by the handle and
 * stay valid until hmat_destroy.
 */
hmat_status hmat_export(hmat_t h, hmat_host_blocks* out);

/*
 * hmat_matvec — y = alpha * H x + beta * y   (eq. (20): dense blocks by plain
 * products, low-rank blocks as U (V^T x_M), all contributions to a row summed
 * by the single owner of that row, no atomics on y).
 *   x, y: DEVICE FP64, caller's element order, column-major n x nrhs with
 *     leading dimension ld >= n; x and y must not overlap.
 *   nrhs >= 0 (0 is a no-op); beta == 0 ignores the old contents of y.
 *   With the split schedule the columns go in passes of 4 (then 2) vectors
 *   that read each stored entry once per pass; the remaining columns, and
 *   other schedules, one at a time.  The sums of a row are taken in the same
 *   order either way up to the length of the staging rounds: results agree
 *   with single-vector products to rounding.
 *   Allocates nothing and does not wait for the GPU.
 */
hmat_status hmat_matvec(hmat_t h, const double* x, double* y, int64_t nrhs, int64_t ld,
                        double alpha, double beta, void* stream);

/* hmat_matvec_T — y = alpha * H^T x + beta * y; same arguments and rules.
 * Runs the product kernels on the packed blocks of H^T (dense blocks
 * transposed, U and V exchanged); needs a handle created with transpose = 1
 * (HMAT_ESTATE otherwise).  The backward of the product y = H x. */
hmat_status hmat_matvec_T(hmat_t h, const double* x, double* y, int64_t nrhs, int64_t ld,
                          double alpha, double beta, void* stream);

/*
 * hmat_matmat — Y = alpha * H X + beta * Y for nrhs members at once
 * (ensemble of simulations; eq. (20) applied to a block of vectors): the
 * products of every work unit run on MFMA (v_mfma_f32_16x16x32_bf16) with the
 * split arithmetic of `mode` (hmat_mm_mode).
 *   X, Y: DEVICE FP64, caller's element order, element-major:
 *     X[i * ldx + r], Y[i * ldy + r] for element i < n, member r < nrhs;
 *     ldx, ldy >= nrhs; X and Y must not overlap.  Members are processed in
 *     groups of 64.
 *   Requires a handle created with max_nrhs > 0 (HMAT_ESTATE otherwise).
 *   Allocates nothing and does not wait for the GPU.  Results are
 *   reproducible for a handle; the wave-group choice (hmat_opts.mm_groups)
 *   sets the order of the FP32 sums, so two handles whose timed choices
 *   differ agree to rounding only (fix mm_groups for identical results).
 */
hmat_status hmat_matmat(hmat_t h, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t nrhs, double alpha,
                        double beta, int32_t mode, void* stream);

/* hmat_info — statistics of the handle (host struct filled, no GPU work). */
hmat_status hmat_info(hmat_t h, hmat_stats* out);

/*
 * hmat_autotune — time the plain product and the BATCHED schedules (waves
 * per workgroup of each phase, split or persistent launch) on the handle's
 * own blocks and keep the fastest.  Synchronises the stream.  Products before and after give
 * results equal to within rounding (the summation order of a row can
 * change with the schedule).  reps: timed products per candidate (>= 1).
 * The choice is remembered for the life of the process, keyed by the block
 * list, the storage and schedule options and the device model: a later
 * call on a handle with the same key re-lays it out with that choice
 * without timing.  The choices timed at creation (the small-matrix layout,
 * the ensemble wave groups) are remembered the same way.
 */
hmat_status hmat_autotune(hmat_t h, int32_t reps, void* stream);

/* Launch timings of the product (hmat_profile). */
typedef struct {
  int32_t n_launches;      /* kernel launches per product: 2 (plain, split) or 1 (persistent) */
  int32_t reps;
  double ms[2];            /* mean duration of each launch [ms] (HIP events on the stream) */
  double ms_product;       /* mean duration of a whole product [ms] */
  int64_t alg_bytes[2];    /* algorithmic bytes of each launch: launch 1 (phase 1) reads the
                              V factors, x and the permutation and writes t; launch 2 (phase 2)
                              reads the dense blocks, the U factors, t, x, the permutation and
                              reads/writes y.  A single persistent launch reports alg_bytes. */
} hmat_profile_t;

/*
 * hmat_profile — run reps products y = H x (after one warm-up) with HIP
 * events around each kernel launch on `stream` and report mean durations.
 * x, y: DEVICE FP64 vectors of length n (not overlapping).  Synchronises the
 * stream; creates and destroys its own events.
 */
hmat_status hmat_profile(hmat_t h, const double* x, double* y, int32_t reps, void* stream, hmat_profile_t* out);

/*
 * hmat_check — report whether every product on the handle since the last
 * check produced valid results.  Only the persistent schedule can fail
 * silently (a workgroup that gave up its bounded wait for phase 1): for a
 * handle using it, waits for `stream`, reads the device flag, clears it and
 * returns HMAT_EDEVICE if it was set.  Other handles: HMAT_OK at once,
 * without waiting.  The asynchronous calls (hmat_matvec, _matvec_T,
 * rs_rk45_replay, rs_rk45_adjoint) do not check by themselves; call this
 * after them where their results are used.
 */
hmat_status hmat_check(hmat_t h, void* stream);

/* Rate-and-state parameters for rs_rhs (section 2.2; section 4.1 loading). */
typedef struct {
  int64_t n;               /* elements; must equal the order of A (and B) */
  double V0;               /* reference slip rate [m/s] */
  double f0;               /* reference friction coefficient */
  double eta_rad;          /* radiation damping mu / (2 c_s) [Pa s / m] */
  double V_pl;             /* plate (backslip loading) rate [m/s] */
  const double* a;         /* DEVICE n: direct-effect coefficient */
  const double* b;         /* DEVICE n: evolution-effect coefficient */
  const double* dc;        /* DEVICE n: characteristic slip distance [m] */
} rs_params;

/*
 * rs_rhs — right-hand side dy/dt of the 3N ODEs (eqs. (8), (10), (12) with
 * the partial derivatives of eq. (13) and backslip loading, eqs. (21)-(22)).
 *   y: DEVICE 3n = (phi | tau | sigma); dydt: DEVICE 3n, same layout;
 *   V_out: DEVICE n or NULL (slip rate from eq. (7)).
 *   B may be NULL: dsigma/dt = 0 (coplanar faults in a full space).
 *   Uses the handle's scratch for the slip-rate vector; allocates nothing.
 */
hmat_status rs_rhs(hmat_t A, hmat_t B, const rs_params* p, const double* y, double* dydt,
                   double* V_out, void* stream);

/* State of the adaptive Runge-Kutta integration (host struct, read and
 * updated by rs_rk45_attempt / rs_rk45_step). */
typedef struct {
  double t;                /* simulated time [s] */
  double dt;               /* step to try next [s] (> 0) */
  double eps_rk;           /* allowance eps_RK of section 2.2; <= 0 means 1e-4 */
  double last_err;         /* err / eps_RK of the last attempt */
  int64_t accepted;        /* accepted steps so far */
  int64_t rejected;        /* rejected attempts so far */
} rs_rk45_state;

/* Streams of the integration calls (rs_rk45_attempt, _run, _step, _replay,
 * _adjoint, rs_ens_rk45_run).  With a B handle other than A, the products
 * with A and with B of each stage run side by side: A's on `stream`, B's on
 * a stream that B owns (created at B's first such call unless `stream` is
 * being captured then, in which case both go on `stream`), forked from
 * `stream` and joined back before the right-hand side.  Every call stays
 * ordered on `stream`; the results do not depend on the overlap.  Under the
 * graph capture of rs_rk45_run / rs_ens_rk45_run the two become parallel
 * branches of the graph (a handle is used by one stream at a time, as
 * everywhere: B's own stream is no exception). */

/* Bytes of device workspace rs_rk45_attempt needs for n elements:
 * 8 * (28 n + 288).  n < 0 returns -1. */
int64_t rs_rk45_workspace_bytes(int64_t n);

/*
 * rs_rk45_attempt — one attempt of the embedded Runge-Kutta 5(4) pair of
 * Cash & Karp on the 3N ODEs (section 2.2): six right-hand-side evaluations
 * (slip rate of eq. (7), products with A and B, eqs. (8), (12)), the largest
 * relative difference err between the 5th- and 4th-order solutions, and the
 * step control of eqs. (14)-(15) with r = err / eps_RK (non-finite err:
 * reject with dt/2).  On acceptance y becomes the 5th-order solution, the
 * slip D advances by eq. (16), t += dt and accepted += 1; otherwise y and D
 * are unchanged and rejected += 1.  st->dt becomes the next step.
 *   y: DEVICE 3n (phi | tau | sigma), updated in place; D: DEVICE n slip.
 *   workspace: DEVICE, at least rs_rk45_workspace_bytes(n), 8-byte aligned;
 *     it also holds the device copy of the integration state.
 *   force: -1 let the controller decide; 1 accept / 0 reject regardless of
 *     err and leave st->dt unchanged (replay of a recorded step sequence).
 *   Synchronises the stream (state copied in and out).  Allocates nothing.
 */
hmat_status rs_rk45_attempt(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace,
                            rs_rk45_state* st, int32_t force, void* stream);

/*
 * rs_rk45_run — advance until n_accept more steps are accepted.  The step
 * control runs on the GPU (the state lives in the workspace), so attempts
 * are enqueued back to back with no host round trip; the host reads the
 * state once per batch (a batch is as many attempts as steps still missing;
 * attempts after the target is reached change nothing).  use_graph != 0 and
 * a non-null stream: one attempt is captured once as a HIP graph (cached in
 * A, re-captured when any argument changes) and replayed.
 * max_attempts > 0 bounds the attempts (HMAT_ESTATE if the target is not
 * reached; the state stays consistent).  st is updated on return.
 * dt_log: DEVICE, n_accept doubles, or NULL; entry m receives the step of
 * the m-th step accepted by this call (the list rs_rk45_replay takes).
 */
hmat_status rs_rk45_run(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace,
                        rs_rk45_state* st, int64_t n_accept, int64_t max_attempts, double* dt_log,
                        int32_t use_graph, void* stream);

/* GPU time of a timed run (rs_rk45_run_timed), from the device wall clock. */
typedef struct {
  double product_ms;       /* summed time of the stages' products (with B: the pair, side by side) */
  double attempt_ms;       /* summed time of the attempts, first kernel to last */
  int64_t attempts;        /* attempts launched */
} rs_rk45_timing;

/*
 * rs_rk45_run_timed — rs_rk45_run with the products' share of the GPU time
 * measured in the run itself: each attempt (graph-captured like
 * rs_rk45_run's, cached separately) also launches one-thread kernels that
 * read the device wall clock at its start and end and before and after each
 * stage's products, and sum the intervals on the device; *timing receives
 * the totals.  The stamps add about one small kernel each (13 per attempt)
 * to the run.  Same arguments, state and results as rs_rk45_run otherwise.
 */
hmat_status rs_rk45_run_timed(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace,
                              rs_rk45_state* st, int64_t n_accept, int64_t max_attempts, double* dt_log,
                              int32_t use_graph, void* stream, rs_rk45_timing* timing);

/* rs_rk45_step — rs_rk45_run for one accepted step, without a graph. */
hmat_status rs_rk45_step(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace,
                         rs_rk45_state* st, int32_t max_attempts, void* stream);

/*
 * rs_rk45_replay — the integration of rs_rk45_run on a frozen list of steps
 * (section 2.2 stages, eq. (16) slip; no error control: every step is taken).
 * Replaying the dt_log of a controlled run reproduces that run.
 *   y: DEVICE 3n, advanced in place; D: DEVICE n slip, accumulated, or NULL.
 *   dts: HOST, n_steps steps (> 0, finite).
 *   ckpt: DEVICE, ceil(n_steps / ckpt_every) * 3n doubles, or NULL; block c
 *     receives y before step c * ckpt_every (the checkpoints rs_rk45_adjoint
 *     starts its segments from).
 *   workspace: DEVICE, rs_rk45_workspace_bytes(n), 8-byte aligned.
 *   Asynchronous on `stream`; allocates nothing.
 */
hmat_status rs_rk45_replay(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, const double* dts,
                           int64_t n_steps, double* ckpt, int64_t ckpt_every, void* workspace, void* stream);

/*
 * rs_rk45_replay_noalloc — rs_rk45_replay without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc).  Same arguments, results
 * and stream ordering as rs_rk45_replay; the 24 n doubles of workspace come
 * from a static device array of 32 MiB in the library (one per device,
 * held until the process ends), so n is at most
 * rs_rk45_replay_noalloc_max_n() = 174762 (HMAT_EINVAL beyond).  Calls no
 * allocating routine.  Every call on a device shares that array: two calls
 * that overlap on one device (on different streams, or from two threads)
 * race and give wrong results; calls ordered on one stream are safe.
 */
int64_t rs_rk45_replay_noalloc_max_n(void);
hmat_status rs_rk45_replay_noalloc(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D,
                                   const double* dts, int64_t n_steps, double* ckpt, int64_t ckpt_every,
                                   void* stream);

/* Bytes of device workspace rs_rk45_adjoint needs: 8 (36 n K + 31 n + 32)
 * with K = min(ckpt_every, n_steps) (-1 on bad arguments or overflow). */
int64_t rs_rk45_adjoint_workspace_bytes(int64_t n, int64_t ckpt_every);

/*
 * rs_rk45_adjoint — reverse-mode derivative of rs_rk45_replay (the discrete
 * adjoint of the frozen-step integration).  For a loss L(y_M, D_M) of the
 * state and slip after the n_steps steps, given Dbar = dL/dD_M and
 * ybar = dL/dy_M, it returns dL/dy_0 in y_bar and adds dL/da and dL/dd_c to
 * a_bar and dc_bar (b held fixed, so dL/da is also the derivative with
 * respect to a - b).  Each segment of ckpt_every steps is recomputed from its
 * checkpoint with every stage kept, then swept backwards: per stage one
 * product with A^T (and B^T), eqs. (8), (12), (13) differentiated element by
 * element.  The handles need transposed products (opts.transpose, or the
 * plain kernel), else HMAT_ESTATE.
 *   ckpt: DEVICE, as written by rs_rk45_replay with the same ckpt_every, dts.
 *   D_bar: DEVICE n, or NULL (zero).  y_bar: DEVICE 3n, in dL/dy_M, out dL/dy_0.
 *   a_bar, dc_bar: DEVICE n, accumulated (+=).
 *   workspace: DEVICE, at least rs_rk45_adjoint_workspace_bytes(n,
 *     min(ckpt_every, n_steps)) bytes (workspace_bytes), 8-byte aligned.
 *   Asynchronous on `stream`; allocates nothing.
 */
hmat_status rs_rk45_adjoint(hmat_t A, hmat_t B, const rs_params* p, const double* ckpt, int64_t ckpt_every,
                            const double* dts, int64_t n_steps, const double* D_bar, double* y_bar, double* a_bar,
                            double* dc_bar, void* workspace, int64_t workspace_bytes, void* stream);

/* Ensemble of up to 64 rate-and-state simulations on one fault (section
 * 2.2 for each member), advanced together: every member has its own
 * friction parameters, state, slip, step and step control; at each
 * Runge-Kutta stage the slip rates of all members go through one ensemble
 * product (hmat_matmat's MFMA kernels).  Layout, member-fastest:
 * element i, member r at [i * members + r]; state components (phi | tau |
 * sigma) in three such blocks of n * members. */
typedef struct {
  int64_t n;               /* elements; must equal the order of A (and B) */
  int32_t members;         /* 1..64 */
  int32_t mode;            /* HMAT_MM_BF16X3 or HMAT_MM_BF16X6 */
  double V0, f0, eta_rad, V_pl;   /* as in rs_params, shared by the members */
  const double* a;         /* DEVICE n * members */
  const double* b;         /* DEVICE n * members */
  const double* dc;        /* DEVICE n * members */
} rs_ens_params;

/* Host state of an ensemble integration (per member). */
typedef struct {
  double eps_rk;           /* allowance eps_RK; <= 0 means 1e-4 */
  double t[64];            /* simulated time of each member [s] */
  double dt[64];           /* step each member tries next [s] (> 0) */
  double last_err[64];     /* err / eps_RK of the member's last attempt */
  int64_t accepted[64];
  int64_t rejected[64];
} rs_ens_state;

/* Bytes of device workspace rs_ens_rk45_run needs: 8 * 28 * n * members plus
 * the device state (about 5 KB); -1 on bad arguments. */
int64_t rs_ens_workspace_bytes(int64_t n, int32_t members);

/*
 * rs_ens_rk45_run — advance every member until it has n_accept more
 * accepted steps (members that reach it stop changing while the others
 * continue).  Each attempt: six stages of per-member stage combinations,
 * slip rates (eq. (7)), one ensemble product with A (and B) for all members,
 * per-member right-hand sides (eqs. (8), (12), (13)); then per-member error
 * (largest relative difference of the 5th- and 4th-order solutions) and
 * step control (eqs. (14)-(15)); accepted members advance y and D (eq. (16)).
 * The controllers run on the GPU; the host reads the state once per batch.
 *   A: built with max_nrhs >= members (FP32 storage, a BATCHED kernel).
 *   y: DEVICE 3 * n * members; D: DEVICE n * members; updated in place.
 *   workspace: DEVICE, rs_ens_workspace_bytes(n, members), 8-byte aligned.
 *   use_graph != 0 and a non-null stream: one attempt is captured as a HIP
 *     graph (cached in A) and replayed.
 *   max_attempts > 0 bounds the attempts (HMAT_ESTATE if a member misses
 *     its target).  st is updated on return.
 */
hmat_status rs_ens_rk45_run(hmat_t A, hmat_t B, const rs_ens_params* p, double* y, double* D, void* workspace,
                            rs_ens_state* st, int64_t n_accept, int64_t max_attempts, int32_t use_graph,
                            void* stream);

/*
 * hmat_kernel_entries — evaluate kernel entries on the host, without building
 * an H-matrix: out[k] = A[rows[k], cols[k]] (green->component 0) or B
 * (component 1), from the same closed forms hmat_build uses (eqs. (5)-(6)).
 * The mesh is validated as in hmat_build.  rows, cols, out: HOST, count
 * entries; indices in [0, mesh->n).  No GPU work.
 */
hmat_status hmat_kernel_entries(const hmat_mesh* mesh, const hmat_green* green, int64_t count, const int64_t* rows,
                                const int64_t* cols, double* out);

/* Release the handle and all its device memory (NULL is ignored).
 * Synchronises the device first. */
void hmat_destroy(hmat_t h);

/* Message of the last failed call on this thread ("" if none). */
const char* hmat_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HMAT_H_ */
