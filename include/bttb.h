/*
 * bttb.h -- C ABI of the MI355X (gfx950) BTTB operator and joint RRCG library.
 *
 * What it computes (Vatankhah, Renaut, Huang, Mickus, Gharloghi, arXiv:2112.15562):
 *
 *   * Sec. 2.1, eq. (d=gm): d = A m, A the m x n sensitivity of the vertical gravity
 *     (A^(1)) or the total-field anomaly (A^(2)) of right rectangular prisms.
 *   * Sec. 2.7.1: A = [A_(1) ... A_(nz)] by depth layer, A x = sum_r A_(r) x_(r); each
 *     A_(r) is BTTB and fixed by an array T_(r) of (sx+nx-1) x (sy+ny-1) values; its
 *     products are IFFT2(FFT2(T) . FFT2(X)) (forward) and IFFT2(conj(FFT2(T)) . FFT2(V))
 *     (transpose) with X / V embedded in the upper-left corner of a zero array.
 *   * eq. (matrixvector): weighted products A~ x = W_d . (A (W^-1 . x)),
 *     A~^T y = W^-1 . (A^T (W_d . y)), the diagonals passed as vectors.
 *   * Sec. 2.4, eqs. (RRCG:1-8) with Sec. 2.5 (bounds), 2.6 (chi^2 test) and 2.8
 *     (alpha schedule, fixed Lagrange parameters): the joint RRCG solver.
 *
 * Conventions shared by every entry point:
 *   * Every function returns an int status: BTTB_OK (0) or a negative bttb_status.
 *     None throws, aborts or exits.  bttb_last_error() returns a message for the
 *     calling thread's last failure.
 *   * Array layouts are C order.  A model vector is [nz][nx][ny] (x = East index a,
 *     y = North index b, layer r); a data vector is [sx][sy] (station p, q).  The
 *     kernel array is [nz][sx+nx-1][sy+ny-1] with
 *       kernels[r][i][j] = K_r(u = i-(nx-1), v = j-(ny-1)),
 *     u = station x index minus prism x index, v likewise along y, K_r the response
 *     at the station of a unit-property prism of layer r.
 *   * "dev" pointers are HIP device pointers; the caller owns them, the library
 *     only reads or writes them.  A handle owns its device memory (a plan its eigenvalues
 *     and scratch), allocated by the call that creates it (bttb_setup, bttb_group_create,
 *     rrcg_create, rrcg_group_create) and freed by its destroy call; the autotuners and the
 *     timing calls allocate too.  Products (one-plan, group, bttb_apply_noalloc) and RRCG
 *     steps of a solver created with use_graph = 0 only launch kernels -- no allocation,
 *     copy, memset or synchronisation -- so a caller may capture them in a HIP graph and
 *     replay it (a solver with use_graph = 1 captures and replays its own graphs).
 *   * Data type: vectors are double for a BTTB_F64 plan and float for a BTTB_F32 plan.
 *     RRCG scalars are always double.
 *   * Every call is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *     returns without waiting, except where stated.  One plan or RRCG handle must not
 *     be used from two streams at once.
 *   * Pointers must be non-NULL unless stated nullable, and aligned to their element
 *     size; sizes must be >= 1.  Violations return BTTB_EINVAL.  The padded transform
 *     sizes must not exceed BTTB_MAX_TRANSFORM, else BTTB_ESIZE.
 */
#ifndef BTTB_H
#define BTTB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define BTTB_API __attribute__((visibility("default")))
#else
#define BTTB_API
#endif

#define BTTB_MAX_TRANSFORM 2048

typedef struct bttb_plan_s* bttb_plan;
typedef struct rrcg_s* rrcg_handle;
typedef struct bttb_group_s* bttb_group;
typedef struct rrcg_group_s* rrcg_group;

typedef enum {
  BTTB_OK = 0,
  BTTB_EINVAL = -1, /* bad argument: NULL / misaligned pointer, size < 1, bad enum */
  BTTB_ENOMEM = -2, /* device allocation failed (setup / create only) */
  BTTB_EHIP = -3,   /* a HIP runtime call or kernel launch failed */
  BTTB_ESIZE = -4,  /* padded transform size above BTTB_MAX_TRANSFORM, or batch too large */
  BTTB_ESTATE = -5, /* incompatible plans or handle state */
  BTTB_ENAN = -6    /* a non-finite value was produced (RRCG status) */
} bttb_status;

typedef enum { BTTB_F64 = 0, BTTB_F32 = 1 } bttb_precision;
/* Flag or-ed into bttb_setup's precision: pad to powers of two (>= 32) instead of the
 * smallest 5-smooth multiples of 8, so that the plan takes the register-FFT kernels of the
 * one-plan products.  (Groups and solvers also take 5-smooth plans: see bttb_group_create.) */
#define BTTB_PAD_POW2 0x10
/* Flag or-ed into bttb_setup's precision (not with BTTB_PAD_POW2): for each axis, the transform size
 * of least estimated cost for products in a group -- the next power of two (>= 32) or a 5-smooth
 * size below it that the group kernels cover, weighing each size's points by a cost factor of its
 * pass plan (1 for a power of two, from 1.5 for 5-smooth ones).  For uneven batches, where the
 * power-of-two padding of some grids is up to 4 times the area. */
#define BTTB_PAD_AUTO 0x40
/* Flag or-ed into bttb_setup's precision: keep the full complex eigenvalues even when the
 * operator is symmetric.  Without it, a plan (any padding) whose eigenvalues are real and
 * even along x to 1e-14 (FP64) / 1e-6 (FP32) of their largest magnitude -- the case of a
 * kernel even in both lags, e.g. gravity with the stations above the prism centres, in FP32
 * (in FP64 its closed forms are symmetric only to their evaluation noise) --
 * stores only Re lambda[0 .. Px/2] of each column (eig_real_even in bttb_plan_desc),
 * which the column passes read instead of the complex array. */
#define BTTB_EIG_FULL 0x20
typedef enum { BTTB_GRAVITY = 0, BTTB_MAGNETIC = 1 } bttb_kind;
typedef enum { BTTB_OP_FORWARD = 0, BTTB_OP_ADJOINT = 1 } bttb_op;

/* Station and prism grid.  x = East, y = North, z = down.  Prism (a, b, r) spans
 * [a dx,(a+1) dx] x [b dy,(b+1) dy] x [top + r dz, top + (r+1) dz]; station (p, q) sits at
 * ((p+ox+1/2) dx, (q+oy+1/2) dy, -height), i.e. above the centre of prism column
 * (p+ox, q+oy) (Sec. 2.7.1; ox = oy = 0 with sx = nx, sy = ny is the paper's layout, a
 * station grid over the interior of a padded model domain has sx < nx and an offset).
 * The inducing field has inclination incl_deg, declination decl_deg and intensity
 * field_nt (nT).  Units: metres, g/cc -> mGal, SI susceptibility -> nT. */
typedef struct {
  int sx, sy, nx, ny, nz;
  double dx, dy, dz, height, top;
  double incl_deg, decl_deg, field_nt;
  int ox, oy;
} bttb_geometry;

/* Plan description returned by bttb_plan_info. */
typedef struct {
  int sx, sy, nx, ny, nz;
  int Px, Py;              /* padded BCCB transform sizes (powers of two, or 5-smooth multiples of 8) */
  int precision;           /* bttb_precision */
  int max_batch;
  size_t eig_bytes;        /* bytes of the stored eigenvalues (see eig_real_even) */
  size_t scratch_bytes;    /* bytes of the product scratch */
  int col_fft_per_block;   /* launch shape in use (see bttb_set_launch) */
  int row_fft_per_block;
  int layer_chunks;
  int eig_real_even;       /* 1: stored as real [nz][Py/2+1][Px/2+1] (symmetric operator,
                              see BTTB_EIG_FULL); 0: complex [nz][Py/2+1][Px] */
} bttb_plan_desc;

/* Kernel array of eq. (d=gm) for one operator, computed on the GPU in FP64 from the
 * closed forms of the prism's vertical gravity (kind = BTTB_GRAVITY, Haaz) or total
 * field anomaly for induced magnetisation (kind = BTTB_MAGNETIC, Rao & Babu),
 * Sec. 2.1.  out: dev double [nz][sx+nx-1][sy+ny-1] in the layout above. */
BTTB_API int bttb_prism_kernels(int kind, const bttb_geometry* g, double* out, void* stream);

/* Build a plan: place each layer's kernel array on a Px x Py circle (Px, Py the
 * smallest 5-smooth multiples of 8 >= sx+nx-1, sy+ny-1) and take its FFT2 once
 * (the BCCB eigenvalues, Sec. 2.7.1), in FP64; a BTTB_F32 plan rounds them to float.
 * kernels: dev double [nz][sx+nx-1][sy+ny-1], read during the call only.
 * max_batch: batch members one product launch transforms together (>= 1); a product call
 * with a larger batch runs max_batch members at a time (the plan's scratch holds max_batch).
 * Synchronises `stream` before returning.  *out receives the plan. */
BTTB_API int bttb_setup(const double* kernels, int sx, int sy, int nx, int ny, int nz,
               int precision, int max_batch, void* stream, bttb_plan* out);

/* y = A x  (Sec. 2.7.1 forward).  x: dev [nz][nx][ny]; y: dev [sx][sy]. */
BTTB_API int bttb_matvec(bttb_plan plan, const void* x, void* y, void* stream);

/* z = A^T r  (Sec. 2.7.1 transpose, conj eigenvalues).  r: dev [sx][sy]; z: dev [nz][nx][ny]. */
BTTB_API int bttb_rmatvec(bttb_plan plan, const void* r, void* z, void* stream);

/* General product, batched and weighted (eq. matrixvector):
 *   op = BTTB_OP_FORWARD: out_b = wd . (A (winv . in_b))        in_b [nz][nx][ny] -> out_b [sx][sy]
 *   op = BTTB_OP_ADJOINT: out_b = winv . (A^T (wd . in_b))      in_b [sx][sy] -> out_b [nz][nx][ny]
 * for b < batch (batch >= 1, else BTTB_EINVAL; max_batch members per launch), element
 * strides in_stride / out_stride between batch members (>= the member size when batch > 1).  winv (dev [nz][nx][ny], = 1/W) and wd (dev [sx][sy])
 * are nullable (NULL = identity) and shared by the whole batch. */
BTTB_API int bttb_apply(bttb_plan plan, int op, int batch, const void* in, long long in_stride,
               void* out, long long out_stride, const void* winv, const void* wd, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): bttb_apply with batch 1 (same arguments, same
 * kernels, same results), with the products' intermediates (the row spectra and the data-side
 * spectra) in a fixed array of BTTB_NOALLOC_MAX_SCRATCH bytes that the library holds on every GPU
 * it runs on until the process ends, instead of the plan's scratch.  Allocates nothing.  Call it
 * with the plan's device current.  A plan whose intermediates need more than the array returns
 * BTTB_ESIZE (at 32 MiB: 256x256x32 in FP32 fits, in FP64 it does not).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (two streams, or two host threads) race.
 * The first call on a device looks up the array's address there (no allocation). */
#define BTTB_NOALLOC_MAX_SCRATCH (32u << 20)
BTTB_API int bttb_apply_noalloc(bttb_plan plan, int op, const void* in, void* out, const void* winv,
                                const void* wd, void* stream);

/* Launch shape: FFTs per block for the column and row passes and the number of layer
 * chunks of the forward column pass.  Values <= 0 keep the current choice.  Changes
 * only the work split, never the arithmetic of an output element.  BTTB_EINVAL if a
 * value does not fit the plan (LDS or size limits). */
BTTB_API int bttb_set_launch(bttb_plan plan, int col_fft_per_block, int row_fft_per_block, int layer_chunks);

BTTB_API int bttb_plan_info(bttb_plan plan, bttb_plan_desc* out);

/* Copy the plan's eigenvalues as complex [nz][Py/2+1][Px] of the plan's type, interleaved
 * re, im, already scaled by 1/(Px Py), into the dev buffer `out` (nz (Py/2+1) Px complex
 * values; a real-even store is expanded), enqueued on `stream`.  For inspection and tests. */
BTTB_API int bttb_plan_eigenvalues(bttb_plan plan, void* out, void* stream);

BTTB_API int bttb_destroy(bttb_plan plan);

/* Per-kernel timing with HIP events recorded on the launch stream around each kernel
 * of the products, for measurement.  bttb_timing_enable(plan, n, repeat) allocates n
 * event pairs (n = 0 disables and frees them; not to be called during stream capture);
 * launches beyond n are not timed.  While timing is on, each timed kernel is launched
 * `repeat` (>= 1) times back to back between its two events; every kernel reads one
 * buffer and writes another, so the repeats leave the results unchanged and the
 * per-launch time excludes the event overhead.  bttb_timing_read synchronises on the
 * events, adds the elapsed milliseconds and launch counts (repeats included) of every
 * timed kernel into total_ms[BTTB_NKERNELS] and count[BTTB_NKERNELS] (overwritten),
 * and starts over.
 * Kernel ids: 0 forward row transform, 1 forward column pass (eigenvalue multiply and
 * layer sum), 2 forward inverse row transform, 3 transpose row transform, 4 transpose
 * column pass (conjugate eigenvalue multiply), 5 transpose inverse row transform. */
#define BTTB_NKERNELS 6
BTTB_API int bttb_timing_enable(bttb_plan plan, int max_launches, int repeat);
BTTB_API int bttb_timing_read(bttb_plan plan, double* total_ms, int* count);

/* ---------------------------------------------------------------------------------- */
/* Groups: the products of many plans in one launch per stage                           */
/* ---------------------------------------------------------------------------------- */

/* A group runs the products (Sec. 2.7.1, eq. matrixvector) of up to 64 plans -- e.g. the
 * gravity and magnetic operators of many inversions of uneven sizes -- as one kernel
 * launch per stage (row transform, column pass, inverse row transform), each member
 * with its own plan's eigenvalues and scratch.  Members are plans of one precision whose
 * transform sizes are powers of two from 32 to 2048 (bttb_setup with BTTB_PAD_POW2), or
 * 5-smooth sizes up to 640 that are not powers of two (radix-3 and -5 passes, the default
 * padding of bttb_setup) where the rows and columns, model and data side, fill at most half of
 * the transform (stations over the prism centres always do); otherwise BTTB_ESTATE.  Each
 * plan at most once (a member's intermediates live in its plan; a repeated plan is
 * BTTB_EINVAL).
 * The group refers to the plans, which must outlive it and must not be used on another
 * stream while a group product runs.  Creation allocates a small device table and
 * synchronises `stream`. */
BTTB_API int bttb_group_create(const bttb_plan* plans, int count, void* stream, bttb_group* out);

/* For every member i: op = BTTB_OP_FORWARD: out_i = wd_i . (A_i (winv_i . in_i));
 * op = BTTB_OP_ADJOINT: out_i = winv_i . (A_i^T (wd_i . in_i)); shapes as bttb_apply
 * with batch 1.  in, out: DEVICE arrays of `count` device pointers (caller-owned, read
 * by the kernels when they run, so a captured graph may be replayed with new contents
 * of the same buffers).  winv, wd: device pointer arrays or NULL (identity for all);
 * entries may be NULL. */
BTTB_API int bttb_group_apply(bttb_group g, int op, const void* const* in, void* const* out,
                              const void* const* winv, const void* const* wd, void* stream);

/* Launch shape: threads per block of the model-side row transforms, the data-side row
 * transforms and the column passes (powers of two, at least N/8 of every member, at
 * most 512; columns at most 256 in FP64), and the layer chunks of the forward column
 * pass (bounded per member by its plan).  Values <= 0 keep the current choice.  Only
 * the work split changes.  Synchronises `stream`. */
BTTB_API int bttb_group_set_launch(bttb_group g, int model_row_threads, int data_row_threads, int col_threads,
                                   int layer_chunks, void* stream);

typedef struct {
  int count, precision;
  int model_row_threads, data_row_threads, col_threads, layer_chunks;
  int blocks[6]; /* blocks of each launch: forward row, column, inverse row; transpose likewise */
} bttb_group_desc;

BTTB_API int bttb_group_info(bttb_group g, bttb_group_desc* out);
BTTB_API int bttb_group_destroy(bttb_group g);

/* Event timing of a group's launches, as bttb_timing_enable / bttb_timing_read for a plan
 * (kernel ids as there; each id covers every member of the launch).  Launches captured
 * into a graph are not timed.  In a solver's products (rrcg_products, rrcg_group_products),
 * whose stages carry CG pieces, the repeats before the last launch of a stage write the
 * in-place direction update (RRCG:5) to a scratch vector and record no scalars: they read
 * what the last launch reads, so the solver's state is that of one launch. */
BTTB_API int bttb_group_timing_enable(bttb_group g, int max_launches, int repeat);
BTTB_API int bttb_group_timing_read(bttb_group g, double* total_ms, int* count);
/* The timed launches since the last read, one by one, in launch order: kernel id and the
 * milliseconds of one launch (the time between its events divided by its repeats), at most
 * `cap` of them; *n receives how many were written.  Synchronises on the events and starts
 * over, as bttb_group_timing_read does (call one or the other). */
BTTB_API int bttb_group_timing_list(bttb_group g, int cap, int* kernel_id, double* ms, int* n);

/* ---------------------------------------------------------------------------------- */
/* Launch-shape autotuning                                                              */
/* ---------------------------------------------------------------------------------- */

/* Result of an autotuning call. */
typedef struct {
  double us_per_pair; /* time of one forward plus one transpose product (per member set
                         for a group) with the chosen shape, microseconds */
  int shape[4];       /* plan: column FFTs per block, row FFTs per block, layer chunks, 0;
                         group: model-row, data-row and column threads per block, layer chunks */
  int tried;          /* candidate shapes timed */
} bttb_tune_result;

/* Time the products of a plan (or group) under candidate launch shapes and keep the
 * fastest: `reps` (1..1000) forward and transpose products per candidate on zero-filled
 * scratch vectors, between HIP events on `stream`.  A plan sweeps every valid
 * combination of column FFTs per block, row FFTs per block (1, 2, 4, 8) and layer chunks
 * (1, 2, 4, 8, 16); a group tunes its four coordinates one at a time, twice round.
 * Results of later products are unchanged up to the grouping of the forward layer sums.
 * Allocates and frees the scratch vectors; synchronises `stream`.  Tune a plan before
 * creating a solver on it (a solver captures the shapes in its graphs).  out nullable. */
BTTB_API int bttb_autotune(bttb_plan plan, int reps, void* stream, bttb_tune_result* out);
BTTB_API int bttb_group_autotune(bttb_group g, int reps, void* stream, bttb_tune_result* out);

/* ---------------------------------------------------------------------------------- */
/* Joint RRCG (Sec. 2.4 eqs. RRCG:1-8, Sec. 2.5-2.6, Sec. 2.8)                          */
/* ---------------------------------------------------------------------------------- */

/* Description of one joint inversion.  Index 0 = gravity (density), 1 = magnetic
 * (susceptibility); both plans share nx, ny, nz, sx, sy and precision.  All vectors are
 * dev, caller-owned, of the plans' type, and must stay alive until rrcg_destroy.
 * State (read and written by the solver):
 *   m[i]      [nz][nx][ny] the model m in the original space; holds the starting model
 *             at rrcg_create (m_0 = m_apr for the paper's start) and m_k after k steps
 *   p[i]      [nz][nx][ny] the last search direction (weighted space); zero it for a
 *             fresh start
 *   resid[i]  [sx][sy] the weighted residual W_d (A m - d) of the current m
 * Inputs:
 *   dobs[i]   [sx][sy] observed data
 *   wd[i]     [sx][sy] diagonal of W_d = 1/sigma
 *   wdepth[i] [nz][nx][ny] diagonal of W_depth
 *   whard[i]  [nz][nx][ny] diagonal of W_hard, nullable (= 1)
 *   mapr[i]   [nz][nx][ny] a-priori model, nullable (= 0)
 * Scalars: bounds lo/hi (Sec. 2.5), alpha0, decay q and floor alpha_min (eq. regpara),
 * lambda (fixed Lagrange parameters), eps2 (eq. WL; the paper uses 1e-9).
 * Flags: coupled = 1 joint beta and step length (eqs. RRCG:5-6), 0 = per data set
 *        (the stand-alone form of Sec. 3.1.1);
 *        restart = 1 sets beta = 0 at the first CG step of every outer step;
 *        p_norm = 1 refreshes W_L1 from the iterate (eq. WL), 2 keeps W_L1 = I;
 *        gramian_weighted = 0 takes the Gramian directions on m (eqs. RRCG:2-3),
 *        1 on m~ (eqs. steepestascenta/b);
 *        anchor: the vector the regularisation term of RRCG:4 pulls toward,
 *        alpha (m~ - anchor): BTTB_ANCHOR_APR (0) W m_apr, the gradient of eq. (GlobalFunction2);
 *        BTTB_ANCHOR_PREV (1) the previous iterate as printed in RRCG:4, read as W m_prev with
 *        m_prev the model at the start of the previous CG step (inside one reweighting this is
 *        -alpha s_{k-1} p_{k-1}; at the first step m_prev = m_0, so the term vanishes).
 *   mprev[i]  [nz][nx][ny] state for BTTB_ANCHOR_PREV (ignored, may be NULL, otherwise): the
 *             model at the start of the last CG step, read by the gradient and rewritten by
 *             every update; set it equal to m for a fresh start. */
typedef enum { BTTB_ANCHOR_APR = 0, BTTB_ANCHOR_PREV = 1 } bttb_anchor;
typedef struct {
  bttb_plan plan[2];
  void* m[2];
  void* p[2];
  void* resid[2];
  const void* dobs[2];
  const void* wd[2];
  const void* wdepth[2];
  const void* whard[2];
  const void* mapr[2];
  double lo[2], hi[2];
  double alpha0[2], q[2], alpha_min[2], lambda[2];
  double eps2;
  int coupled, restart, p_norm, gramian_weighted;
  int use_graph;  /* 1: the step's kernel sequences are captured into HIP graphs and replayed by
                     rrcg_step (fewer launches); 0: launched one by one */
  int anchor;     /* bttb_anchor */
  void* mprev[2];
} rrcg_desc;

/* Scalar state (FP64) of a handle. */
typedef struct {
  double alpha[2];     /* alpha^(i) used by the next outer step */
  double L_prev[2];    /* ||l^(i)||^2 of the last CG step (0 = none: next beta is 0) */
  double phi[2];       /* ||W_d (A m - d)||^2 after the last outer step */
  double threshold;    /* chi^2 threshold m + sqrt(2m), eq. (chi2) */
  double beta[2];      /* beta and step length of the last CG step */
  double step[2];
  double gramian;      /* S_G(m1, m2) after the last outer step */
  int frozen[2];       /* chi^2 met at some outer step: alpha^(i) no longer decays */
  int k;               /* outer steps taken */
  int converged;       /* both chi^2 tests met at the last outer step */
  int nonfinite;       /* a NaN / Inf reached a reduction */
  double similarity;   /* |(m1, m2)| / (||m1|| ||m2||) of the current models (0 if one is zero): the
                          cosine the Gramian S_G = ||m1||^2 ||m2||^2 (1 - cos^2) drives to one, by
                          which a scan over fixed Lagrange parameters (Sec. 3.1.3) compares runs;
                          computed on the device with S_G after every outer step (read only) */
} rrcg_scalars;

/* Create a solver for one inversion: the scalars start at alpha = alpha0, no previous
 * gradient, k = 0, and resid / Phi / S_G are computed from the given m.  Allocates the
 * solver's own work vectors.  When both plans can join a product group (bttb_group_create) the
 * solver runs as a one-inversion group solver (rrcg_group_create): both operators' products
 * share each launch and the CG pieces ride on their row transforms.  Synchronises `stream`. */
BTTB_API int rrcg_create(const rrcg_desc* d, void* stream, rrcg_handle* out);

/* One outer step: n_inner >= 1 CG steps at the outer step's W and alpha (RRCG:1-7, the
 * residual taken exactly at the first and by r~ <- r~ - s A~ p after), then RRCG:8,
 * projection onto [lo, hi], Phi^(i), the chi^2 test and the alpha update.
 * n_inner = 1 with restart = 0 is the single loop printed in the paper.  Asynchronous:
 * no device-to-host transfer. */
BTTB_API int rrcg_step(rrcg_handle h, int n_inner, void* stream);

/* Capture the graph of an outer step with n_inner CG steps ahead of its first use (a
 * solver on group plans (bttb_group_create) with use_graph replays each outer step as one graph,
 * captured on first use per step length; otherwise this does nothing). */
BTTB_API int rrcg_prepare(rrcg_handle h, int n_inner);

/* Copy the scalar state to / from the host.  Synchronises `stream`. */
BTTB_API int rrcg_read_scalars(rrcg_handle h, rrcg_scalars* out, void* stream);
BTTB_API int rrcg_write_scalars(rrcg_handle h, const rrcg_scalars* in, void* stream);

/* Recompute resid, Phi and S_G of the current m, e.g. after m was written to resume
 * from a checkpoint (with rrcg_write_scalars for the scalar state). */
BTTB_API int rrcg_refresh(rrcg_handle h, void* stream);

/* rrcg_group_autotune for a solver on group plans (BTTB_ESTATE otherwise). */
BTTB_API int rrcg_autotune(rrcg_handle h, int reps, void* stream, bttb_tune_result* out);

/* The product group of a solver on group plans (owned by the solver), for
 * inspection and timing; BTTB_ESTATE for other plans. */
BTTB_API int rrcg_products(rrcg_handle h, bttb_group* out);

BTTB_API int rrcg_destroy(rrcg_handle h);

/* Group solver: up to 32 joint inversions of uneven sizes stepped together.  Each
 * inversion is described by its own rrcg_desc and keeps its own state, scalars and
 * parameters, with the same arithmetic as a one-inversion solver; every phase of a step
 * is one launch over all of them (the products of all their operators through one
 * product group, the CG pieces fused into the row transforms, and the elementwise
 * updates over the concatenated vectors).  All plans must be able to join a product group
 * (bttb_group_create) and share one precision, each used by one inversion once (as in
 * bttb_group_create); descs[0].use_graph decides graph capture for the whole group.
 * Creation allocates the work vectors and synchronises `stream`. */
BTTB_API int rrcg_group_create(const rrcg_desc* descs, int count, void* stream, rrcg_group* out);

/* One outer step of every inversion (as rrcg_step).  Asynchronous.  With use_graph the whole
 * outer step is one graph, captured on the first step with this n_inner (the four most
 * recent step lengths are kept; rrcg_group_prepare captures ahead). */
BTTB_API int rrcg_group_step(rrcg_group g, int n_inner, void* stream);
BTTB_API int rrcg_group_prepare(rrcg_group g, int n_inner);

/* Scalars of inversion `index` (0-based); synchronise `stream`. */
BTTB_API int rrcg_group_read_scalars(rrcg_group g, int index, rrcg_scalars* out, void* stream);
BTTB_API int rrcg_group_write_scalars(rrcg_group g, int index, const rrcg_scalars* in, void* stream);

/* Recompute resid, Phi and S_G of every inversion from its current m. */
BTTB_API int rrcg_group_refresh(rrcg_group g, void* stream);

/* Launch shape of the group's products (as bttb_group_set_launch); recaptures the step
 * graphs.  Synchronises `stream`. */
BTTB_API int rrcg_group_set_launch(rrcg_group g, int model_row_threads, int data_row_threads, int col_threads,
                                   int layer_chunks, void* stream);

/* Launch shape of the solver's products chosen by timing `reps` CG steps per candidate (the
 * fused forms the solve runs), one coordinate at a time; the solver state is saved before
 * and restored after, so the solve is unchanged.  Allocates a temporary copy of the state;
 * recaptures the step graphs; synchronises `stream`.  us_per_pair in `out` is the CG step
 * time divided by the operator pairs of a step (2 per inversion). */
BTTB_API int rrcg_group_autotune(rrcg_group g, int reps, void* stream, bttb_tune_result* out);

/* The product group the solver uses (owned by the solver; valid until rrcg_group_destroy),
 * for inspection and timing. */
BTTB_API int rrcg_group_products(rrcg_group g, bttb_group* out);

BTTB_API int rrcg_group_destroy(rrcg_group g);

/* ---------------------------------------------------------------------------------- */

BTTB_API const char* bttb_strerror(int status);
BTTB_API const char* bttb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BTTB_H */
