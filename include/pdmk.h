/*
 * pdmk.h -- C interface of an MI355X (gfx950) implementation of periodic
 * dual-space multilevel kernel splitting (periodic DMK) for Laplace lattice
 * sums in oblique 2D and triclinic 3D cells.
 *
 * The operation (Introduction, eq:potential and eq:greens): for a lattice
 * matrix L = [a_1 ... a_d] (columns are the lattice vectors), sources y_j with
 * charges q_j and targets x_i, return
 *
 *     Phi(x_i) = sum_{n in Z^d} sum_j G(x_i - y_j - L n) q_j,
 *     G(r) = -log(r)/(2 pi) in 2D,  1/(4 pi r) in 3D,
 *
 * in the tin-foil sense (the k = 0 Fourier mode is zero), with the singular
 * self pair (n = 0, coincident source) excluded, and optionally grad Phi.
 * The charges must be neutral (sum q = 0) unless PDMK_ALLOW_NONNEUTRAL is set,
 * in which case the result is the potential of the charges plus a uniform
 * neutralising background.  Units: G exactly as above, no Coulomb constant.
 *
 * The method is Algorithm 1 (Periodic DMK): orient L (Section 3.2,
 * eq:Ltri), cover the cell with root cubes of side r_c = L_min / kappa
 * (eq:mi), add a halo of image sources (Sections 3.3-3.4), build an adaptive
 * tree on the extended root grid, evaluate the compactly supported near
 * field G - W_0 by free-space DMK on it (Section 3.5), evaluate the smooth
 * periodic far field W_0^(p) by spreading -> FFT -> diagonal scaling ->
 * inverse FFT -> interpolation without upsampling (Section 3.6, eq:W0p,
 * eq:diag, eq:Mi), and remove the self terms (Section 3.8, eq:W0zero).
 *
 * Conventions shared by every entry point:
 *   - L is a HOST pointer to d*d doubles, column-major (L[i + d*j] is the
 *     i-th Cartesian component of a_j).
 *   - Position, charge, potential and gradient arrays are DEVICE pointers
 *     (memory of the current HIP device).  Positions are row-major n x d
 *     doubles, potentials n doubles, gradients row-major n x d doubles.
 *   - Positions may lie anywhere in R^d; they are wrapped into the cell.
 *   - The caller owns every buffer.  Inputs are never modified.  The library
 *     keeps no caller pointer after a call returns.
 *   - Calls are ordered on the HIP stream passed in (NULL = default stream)
 *     and block until the results are written (the call synchronises its
 *     stream before returning), except pdmk_plan_execute, which only
 *     enqueues (its status comes from pdmk_plan_status).  The tree build
 *     needs the sizes of each refinement level on the host before it can
 *     launch the next one, so every call that builds a tree waits on the
 *     device; pdmk_plan_execute builds none.  Inside a call, part of the work runs on a
 *     second stream (default priority; owned by the plan, created on its
 *     first evaluation, or by the batch worker) forked from and joined back
 *     to the caller's stream by events.
 *   - Errors: every function returns a pdmk_status.  On an error detected on
 *     the host the output arrays are not written.  pdmk_last_error() returns a
 *     thread-local message for the last failure.
 */
#ifndef PDMK_H
#define PDMK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PDMK_OK = 0,
  PDMK_ERR_INVALID_ARG = -1,     /* bad dimension, null pointer, n < 0 ... */
  PDMK_ERR_SINGULAR_LATTICE = -2,/* det L == 0 or not finite */
  PDMK_ERR_NOT_NEUTRAL = -3,     /* |sum q| > 1e-8 sum |q| without ALLOW_NONNEUTRAL */
  PDMK_ERR_EPS_RANGE = -4,       /* eps outside [1e-12, 1e-2] */
  PDMK_ERR_NONFINITE = -5,       /* NaN or Inf in positions or charges */
  PDMK_ERR_OUT_OF_MEMORY = -6,   /* device allocation failed */
  PDMK_ERR_HIP = -7,             /* a HIP runtime call failed */
  PDMK_ERR_NO_DEVICE = -8,       /* no HIP device available */
  PDMK_ERR_UNSUPPORTED = -9,     /* option combination not implemented */
  PDMK_ERR_SCRATCH = -10         /* pdmk_plan_eval_noalloc: the input needs more
                                    device scratch than the library's fixed array */
} pdmk_status;

/* Arithmetic of the evaluation.
 *   PDMK_PREC_FP64 : every stage in double precision.
 *   PDMK_PREC_MIXED: FP64 kept for wrapping, box assignment, residual-pair
 *                    offsets and r^2, the far-field diagonal scaling and the
 *                    final accumulation; FP32 for the stages in fp32_stages:
 *                    3D: residual-series sums, proxy charges / potentials and
 *                    plane-wave transforms (on FP32 matrix cores; BF16 hi/lo
 *                    products with FP32 accumulation at eps >= 1e-3), far-field
 *                    window weights.  2D: residual-series sums and window
 *                    weights only (2D proxies and plane waves stay FP64).
 *                    FP32 cannot reach eps below 1e-6: for eps < 1e-6 a mixed
 *                    plan computes every stage in FP64 (the same arithmetic as
 *                    PDMK_PREC_FP64), so the result still meets eps. */
enum { PDMK_PREC_FP64 = 0, PDMK_PREC_MIXED = 1 };

/* Stages a mixed plan may compute in FP32 (pdmk_opts.fp32_stages). */
enum {
  PDMK_FP32_RESIDUAL = 1,      /* leaf residual-series sums */
  PDMK_FP32_PROXY = 2,         /* proxy tensors and plane-wave transforms (3D) */
  PDMK_FP32_WINDOW = 4,        /* far-field spreading / interpolation weights */
  PDMK_BF16_PLANE_WAVES = 8    /* BF16 hi/lo plane-wave products at eps >= 1e-3 (3D) */
};

/* Flags */
enum {
  PDMK_WANT_GRAD = 1,          /* gradients wanted: accurate grad Phi (see pdmk_eval) */
  PDMK_ALLOW_NONNEUTRAL = 2,   /* accept sum q != 0 (uniform background) */
  PDMK_DETERMINISTIC = 4,      /* fixed-order reductions: repeated calls on the same
                                  input return bitwise-equal results (see below) */
  PDMK_VECTOR_PLANE_WAVES = 8, /* use the vector-ALU plane-wave, anterpolation,
                                  transfer and leaf-evaluation kernels instead of the
                                  matrix-core ones (same arithmetic type; for
                                  comparing the two implementations) */
  PDMK_ONE_STREAM = 16,        /* run every stage on the caller's stream (no second
                                  stream for the far field's grid steps; each stage
                                  then has the device to itself, so its timings in
                                  pdmk_stats are stand-alone durations) */
  PDMK_BLOCH = 32,             /* quasi-periodic conditions with the Bloch vector
                                  pdmk_opts.bloch (see pdmk_plan_eval_bloch) */
  PDMK_BALANCE = 128,          /* 2:1 balance of the adaptive tree (Algorithm 1): every
                                  leaf holding points is split while a colleague of it
                                  has grandchildren, the tree being rebuilt with the
                                  forced splits until none is left.  The result is the
                                  same (the interaction rule is exact for any tree); the
                                  work moves from the residual sums to plane waves. */
  PDMK_ALL_PAIRS = 256,        /* evaluate every residual pair from both ends.  By
                                  default, when the targets are the sources and the
                                  call asks for no gradients, is not deterministic
                                  and keeps no tree, each pair of points in two
                                  different leaves is evaluated once, since R_h
                                  depends on |x - y| alone, and the result is added
                                  to both points; this flag turns that off (for
                                  comparing the two; the results agree to rounding) */
  PDMK_VIRTUAL_IMAGES = 64     /* the cube-cell construction of rem:cube for rectangular
                                  cells whose edges are whole multiples of
                                  r_c = L_min / kappa (a cube with integer kappa): the
                                  root cubes tile the cell, a boundary box's colleagues
                                  across a face are the boxes on the other side shifted
                                  by L n (n in {-1,0,1}^d), and no image point is placed,
                                  sorted or stored.  Other cells: PDMK_ERR_UNSUPPORTED.
                                  Not with PDMK_BLOCH. */
};

typedef struct {
  int dim;          /* 2 or 3 */
  double eps;       /* requested relative l2 accuracy, [1e-12, 1e-2] */
  int precision;    /* PDMK_PREC_FP64 or PDMK_PREC_MIXED */
  double kappa;     /* root cube side r_c = L_min / kappa (Section 5); <= 0: default */
  int n_s;          /* leaf capacity (Section 5, Table tab:tuning); <= 0: default */
  unsigned flags;   /* PDMK_WANT_GRAD | PDMK_ALLOW_NONNEUTRAL | PDMK_DETERMINISTIC |
                       PDMK_VECTOR_PLANE_WAVES | PDMK_ONE_STREAM | PDMK_BLOCH */
  int porder;       /* Chebyshev proxy points per axis; <= 0: chosen from eps */
  int npw;          /* plane-wave half count J per axis (modes -J..J); <= 0: from eps */
  int nufft_w;      /* spreading-window width in grid cells; <= 0: from eps (two
                       cells more when PDMK_WANT_GRAD is set) */
  double sigma;     /* Fourier grid per axis = sigma * M_i of eq:Mi rounded up to a
                       2,3,5-smooth even size; <= 0: 1 (no upsampling, as in the
                       paper) for eps >= 1e-7, 2 below */
  unsigned fp32_stages; /* PDMK_PREC_MIXED only: PDMK_FP32_* / PDMK_BF16_* bits of the
                       stages computed in reduced precision; 0: all of them (the
                       default).  Ignored (every stage FP64) when eps < 1e-6. */
  double bloch[3];  /* with PDMK_BLOCH: the Bloch vector beta (Cartesian, the
                       caller's frame; d components used) */
} pdmk_opts;

/*
 * PDMK_DETERMINISTIC.  Without it, the leaf residual sums (segments of one
 * target's list), the far-field spreading, the child -> parent proxy-charge
 * transfers and the charge sum accumulate with floating-point atomics, so
 * repeated calls agree to rounding only.  With it every such reduction has a
 * fixed order or is exact: residual segments write partial sums that one
 * thread per target adds in segment order; spreading accumulates each
 * block's subgrid in program order (one wave per block) and adds the
 * subgrids into the grid in two-word 64-bit fixed point (integer atomics,
 * order-independent; resolution 2^-82 of sum |q|); child -> parent
 * transfers run one octant per launch.  Repeated calls with the same inputs,
 * options and device then return bitwise-equal potentials and gradients,
 * also through pdmk_batch_eval with any number of workers.  It costs time
 * and is off by default.
 */

/* Fill *out with the defaults for (dim, eps); nufft_w is left 0 (chosen at
 * plan creation from eps and the flags).  Host only; no device needed. */
int pdmk_default_opts(int dim, double eps, pdmk_opts* out);

/*
 * One evaluation (Algorithm 1).  Targets are the sources when trg == NULL
 * (then n_trg is ignored and the self pair of every source is excluded);
 * otherwise targets are n_trg separate points and no self pair is removed.
 * grad may be NULL; when it is not NULL, grad Phi at the targets is written.
 * PDMK_WANT_GRAD in the options asks for gradients of full accuracy (it
 * widens the far-field window at plan creation); pdmk_eval with that flag
 * requires grad to be non-NULL.
 */
int pdmk_eval(const pdmk_opts* opts, const double* L, int64_t n_src,
              const double* src, const double* q, int64_t n_trg,
              const double* trg, double* pot, double* grad, void* stream);

/*
 * Plans keep the host tables for one (opts, L) pair and the device
 * workspace between calls (the tree is rebuilt every call, as in the
 * paper).  The workspace is one device buffer that grows to the largest call
 * seen; a call that needs more than it holds allocates the difference for
 * itself, and the plan then grows the buffer, so repeated calls of one size
 * allocate nothing after the first.  It is freed by pdmk_plan_destroy.  A
 * plan is bound to the device that was current at creation and serves one
 * call at a time (calls on one plan from several threads must not overlap).
 */
typedef struct pdmk_plan pdmk_plan;
int pdmk_plan_create(const pdmk_opts* opts, const double* L, pdmk_plan** out);
int pdmk_plan_eval(pdmk_plan* plan, int64_t n_src, const double* src,
                   const double* q, int64_t n_trg, const double* trg,
                   double* pot, double* grad, void* stream);
void pdmk_plan_destroy(pdmk_plan* plan);

/*
 * Quasi-periodic (Bloch) conditions (Section 4.1, eq:qp_def): for a plan made
 * with PDMK_BLOCH and beta = opts.bloch,
 *
 *     Phi(x_i) = sum_n sum_j q_j e^{i beta.L n} G(x_i - y_j - L n),
 *
 * the self pair removed, so that Phi(x + L n) = e^{i beta.L n} Phi(x).
 * Positions are taken literally: the image of y_j at y_j + L n carries the
 * charge q_j e^{i beta.L n} (a point given outside the cell is wrapped in with
 * the matching phase on its charge, and a target's value is carried back by
 * the phase of its wrap).  The method is that of the periodic case with the
 * paper's three changes: phased image charges in the near field (evaluated
 * as two real near fields, of the real and the imaginary parts of the image
 * charges), the far field of eq:qp_far (sources pre-modulated by
 * e^{-i beta.y}, scaling by What_0(|k_m + beta|) with the m = 0 mode kept,
 * targets post-modulated by e^{i beta.x}) on the grid M_i = 2 ceil((c/r_c +
 * |beta|) |a_i| / 2 pi).  Charges are real and need not be neutral.  beta
 * must not lie in the reciprocal lattice 2 pi L^{-T} Z^d (that is the
 * periodic case: pdmk_plan_create returns PDMK_ERR_INVALID_ARG).  Potentials
 * only: PDMK_WANT_GRAD, PDMK_DETERMINISTIC and kept trees are not supported
 * with PDMK_BLOCH (PDMK_ERR_UNSUPPORTED), and pdmk_plan_eval rejects a Bloch
 * plan.  pot: DEVICE, 2 n_trg doubles, (real, imaginary) per target.
 * Other arguments, blocking and errors as pdmk_plan_eval.
 */
int pdmk_plan_eval_bloch(pdmk_plan* plan, int64_t n_src, const double* src, const double* q,
                         int64_t n_trg, const double* trg, double* pot, void* stream);

/*
 * The two halves of one evaluation (for checking each on its own): the
 * far field pot_far = the interpolated Fourier sum of eq:W0p over the modes
 * of eq:Mi with m = 0 omitted (Section 3.6), which includes every
 * source's own W_0(0); and the near field pot_near = everything else: the
 * plane-wave and residual sums of G - W_0 over the images within r_c
 * (Section 3.5) minus the self terms W_0(0) q of Section 3.8, plus the
 * uniform-background constant for non-neutral charges.  pot_near + pot_far
 * is what pdmk_plan_eval returns.  Arguments as pdmk_plan_eval (potentials
 * only; pot_near and pot_far: n_trg doubles, DEVICE).  Blocks.
 */
int pdmk_plan_eval_parts(pdmk_plan* plan, int64_t n_src, const double* src, const double* q,
                         int64_t n_trg, const double* trg, double* pot_near, double* pot_far,
                         void* stream);

/*
 * pdmk_plan_eval without device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, results and blocking as pdmk_plan_eval.  Its
 * workspace is one fixed device array inside the library,
 * PDMK_NOALLOC_SCRATCH_BYTES (64 MiB) per device, held from the first such
 * call on a device until the process ends; the call makes no hipMalloc,
 * hipFree, stream or event creation (the far field runs on the caller's
 * stream, no stage timings are recorded).  Inputs whose tree, lists and
 * buffers do not fit the array are rejected with PDMK_ERR_SCRATCH, with the
 * outputs unwritten (roughly up to 5e4 points in 3D at eps = 1e-6; the exact
 * limit depends on the distribution).  The array is shared by every call on
 * one device: the library holds a per-device lock for the whole call, so
 * calls from several threads on one device run one after another.
 */
#define PDMK_NOALLOC_SCRATCH_BYTES (64ull << 20)
int pdmk_plan_eval_noalloc(pdmk_plan* plan, int64_t n_src, const double* src, const double* q,
                           int64_t n_trg, const double* trg, double* pot, double* grad,
                           void* stream);

/*
 * Kept trees: evaluate many charge vectors (and small displacements) on one
 * tree.  Algorithm 1 rebuilds the tree for every evaluation (the
 * preprocessing and tree steps depend only on the positions); when the
 * positions do not change -- new charges, the adjoint charges of a backward
 * pass, a finite-difference stencil -- those steps can be done once.
 *
 * pdmk_plan_bind: one full evaluation (arguments and results as
 * pdmk_plan_eval; blocks) that also keeps, in device memory owned by the
 * plan, everything that depends on the positions alone: wrapped and sorted
 * sources, images and targets, the tree, colleague and residual lists.  A
 * previous binding is released first.  It also allocates the workspace an
 * execute needs, so that executes allocate nothing.  When the targets are the
 * sources, the plan was made without PDMK_WANT_GRAD (nor PDMK_DETERMINISTIC
 * or PDMK_ALL_PAIRS) and the bind asks for no gradients, the kept lists
 * evaluate each residual pair once (see PDMK_ALL_PAIRS); an execute on such a
 * tree that asks for gradients returns PDMK_ERR_UNSUPPORTED before enqueuing
 * anything.
 *
 * pdmk_plan_execute: the near field, far field and assembly of Algorithm 1
 * for charges q (n_src, DEVICE) on the kept tree, into pot (n_trg) and, when
 * grad is not NULL, grad (n_trg x d).  It only enqueues work on `stream` and
 * returns: no host synchronisation, no allocation, no memset nodes, so a
 * caller may capture it into a HIP graph and replay it (the graph then reads
 * q and writes pot / grad at the addresses given at capture).  src / trg
 * (DEVICE, caller layout, may be NULL = the bound positions) are moved
 * positions of the bound points: the kept tree, lists, images and wrap are
 * used with each point displaced by (new - bound) position ("frozen tree").
 * The result is accurate to eps while every displacement stays well below
 * the smallest leaf side (the near-field lists and proxy grids of the bound
 * boxes remain valid: the residual kernel is continuous at the edge of its
 * support and vanishes there to within eps); it is a smooth function of the
 * positions, as finite-difference checks need.  trg must be NULL when the
 * bound targets are the sources.  Errors of the inputs (non-finite values,
 * charges not neutral without PDMK_ALLOW_NONNEUTRAL) are found on the
 * device: the assembly then leaves pot / grad unwritten and the error is
 * kept until the next pdmk_plan_status.  Calls on one plan are ordered by
 * their streams; an execute must not overlap another call on the same plan.
 *
 * pdmk_plan_status: waits for the plan's last execute and returns the first
 * error any execute since the previous status call found on the device
 * (PDMK_ERR_NONFINITE, PDMK_ERR_NOT_NEUTRAL), else PDMK_OK; clears it.
 *
 * pdmk_plan_unbind releases the kept tree (pdmk_plan_destroy does too).
 */
int pdmk_plan_bind(pdmk_plan* plan, int64_t n_src, const double* src, const double* q,
                   int64_t n_trg, const double* trg, double* pot, double* grad, void* stream);
int pdmk_plan_execute(pdmk_plan* plan, const double* src, const double* trg, const double* q,
                      double* pot, double* grad, void* stream);
int pdmk_plan_status(pdmk_plan* plan);
void pdmk_plan_unbind(pdmk_plan* plan);

/*
 * Adjoint of an evaluation, for a loss l(Phi) with g = dl/dPhi at the n_trg
 * targets.  The Laplace kernel is symmetric, so the adjoint is one more
 * evaluation with the roles of sources and targets swapped: with
 * Psi(y) = sum_i g_i K(y - x_i) (the potential of the charges g at the targets,
 * uniform background for sum g != 0, the same convention the evaluation uses
 * for non-neutral charges; the method's split G - W_0 + W_0 is unchanged),
 *     dq_j   = Psi(y_j)
 *     dsrc_j = q_j grad Psi(y_j)   (+ g_j grad Phi(y_j) when targets are the sources)
 *     dtrg_i = g_i grad Phi(x_i)   (separate targets only)
 * Arguments: src, q, trg as in the evaluation (trg == NULL: targets are the
 * sources); g: n_trg doubles; grad_phi: the gradient the forward evaluation
 * returned (n_trg x d, row-major), required for dsrc with targets = sources and
 * for dtrg; dq (n_src), dsrc (n_src x d), dtrg (n_trg x d): outputs, each may be
 * NULL.  Device pointers; the plan keeps a device buffer of n_src (d + 1)
 * doubles for Psi between calls.  Blocks until the outputs are written.
 */
int pdmk_plan_adjoint(pdmk_plan* plan, int64_t n_src, const double* src, const double* q,
                      int64_t n_trg, const double* trg, const double* g,
                      const double* grad_phi, double* dq, double* dsrc, double* dtrg,
                      void* stream);

/*
 * Batches of independent systems (many small cells in one call; the adaptive
 * tuning remark of Section 5 leaves per-problem planning to future work, and
 * a batch is where it pays).  All systems share the
 * options; system s has its own lattice L + s*d*d (HOST, column-major) and the
 * sources offsets[s] .. offsets[s+1]-1 of the concatenated arrays (offsets is a
 * HOST array of n_sys + 1 nondecreasing entries; targets are the sources, the
 * self pair excluded).  src (row-major N x d), q, pot (N) and grad (N x d, may
 * be NULL; required with PDMK_WANT_GRAD) are DEVICE arrays.  Every system must
 * be neutral unless PDMK_ALLOW_NONNEUTRAL is set.
 *
 * pdmk_batch_create builds one plan per system (host tables, geometry) and
 * n_workers host workers (<= 0: 8), each with its own non-blocking HIP stream
 * and device workspace; pdmk_batch_eval hands the systems to the workers, so
 * the pipelines of different systems run concurrently on the device.  The call
 * first synchronises `stream` (the inputs must be complete) and returns when
 * every output is written.  On the first failing system the remaining ones are
 * skipped and its status is returned.  pdmk_batch_stats reads the counters of
 * system `sys`.  pdmk_eval_batched = create + eval + destroy.
 */
typedef struct pdmk_batch pdmk_batch;
int pdmk_batch_create(const pdmk_opts* opts, int n_sys, const double* L, int n_workers,
                      pdmk_batch** out);
int pdmk_batch_eval(pdmk_batch* batch, const int64_t* offsets, const double* src,
                    const double* q, double* pot, double* grad, void* stream);
void pdmk_batch_destroy(pdmk_batch* batch);

/*
 * Kept trees for a batch (repeated evaluation with new charges, e.g. the
 * adjoint after a forward call or charge updates at fixed positions):
 * pdmk_batch_bind is one evaluation of every system (as pdmk_batch_eval,
 * blocking; targets are the sources) that keeps each system's tree as
 * pdmk_plan_bind does; pdmk_batch_execute then evaluates new charges q
 * (DEVICE, offsets as bound) into pot (and grad with PDMK_WANT_GRAD) by
 * enqueueing every system's pdmk_plan_execute round-robin over the batch's
 * worker streams, forked from and joined back into `stream` with events, from
 * the calling thread only: it does not block, allocates nothing and makes no
 * host read, so a caller can capture the whole call into one graph.
 * pdmk_batch_status waits and returns the first device-detected input error
 * of the systems (as pdmk_plan_status).  A new bind replaces the kept trees;
 * pdmk_batch_eval and pdmk_batch_tune leave them in place only if they do not
 * re-plan (pdmk_batch_tune re-plans: bind again after it).
 */
int pdmk_batch_bind(pdmk_batch* batch, const int64_t* offsets, const double* src,
                    const double* q, double* pot, double* grad, void* stream);
int pdmk_batch_execute(pdmk_batch* batch, const double* q, double* pot, double* grad,
                       void* stream);
int pdmk_batch_status(pdmk_batch* batch);
int pdmk_eval_batched(const pdmk_opts* opts, int n_sys, const double* L,
                      const int64_t* offsets, const double* src, const double* q,
                      double* pot, double* grad, void* stream);

/*
 * Batch autotuner (the run-time choice of (kappa, n_s) that Section 5 leaves
 * for later, per size class of a batch).  The systems of `batch` with n > 0
 * sources are grouped by floor(log2 n);
 * for each class and candidate (kappa[i], n_s[i]) (<= 0: the batch's value),
 * up to n_workers systems spread evenly over the class's sizes are planned
 * and evaluated concurrently, one per worker stream as in pdmk_batch_eval:
 * one warm-up round and `trials` (>= 1) timed rounds, outputs discarded.
 * Every system of the class is then re-planned with the candidate of the
 * shortest rounds.  Any
 * (kappa, n_s) is a valid plan (the split of Section 3 is exact for any
 * tree), so tuning changes speed, not the tolerance.  offsets, src, q: as for
 * pdmk_batch_eval (offsets HOST, src and q DEVICE); the call synchronises
 * `stream` first.  kappa_out, n_s_out: HOST arrays of n_sys entries or NULL;
 * they receive each system's plan parameters after tuning (systems with no
 * sources keep their plan).  Blocks; allocates device buffers for the
 * sampled systems' outputs for the duration of the call.  Errors:
 * PDMK_ERR_INVALID_ARG for null arguments, n_cand < 1, trials < 1 or
 * decreasing offsets; the first planning error of a class none of whose
 * candidates could be planned; evaluation errors (for instance a
 * non-neutral system) at once.  After an error the batch stays usable:
 * classes tuned before it keep their new plans, the others their old ones.
 */
int pdmk_batch_tune(pdmk_batch* batch, const int64_t* offsets, const double* src,
                    const double* q, int n_cand, const double* kappa, const int* n_s,
                    int trials, void* stream, double* kappa_out, int* n_s_out);

/*
 * Runtime planning of the method's two free parameters, the root-cube side
 * r_c = L_min / kappa and the leaf capacity n_s (Section 5; the paper leaves
 * planning them at run time for later).  Each candidate (kappa[i], n_s[i])
 * (<= 0: the value in opts) is planned and timed on the caller's input: one
 * warm-up evaluation and `trials` timed ones (>= 1), results discarded.  The
 * fastest pair is written to *best_kappa, *best_n_s.  The result of the
 * method does not depend on (kappa, n_s) beyond the tolerance eps (the split
 * of Section 3 is exact for any tree), so every candidate is a valid choice.
 * opts, L: as for pdmk_plan_create (HOST).  kappa, n_s: n_cand candidates
 * (HOST).  src, q, trg, n_src, n_trg: as for pdmk_plan_eval (DEVICE).  pot:
 * DEVICE scratch of n_trg doubles (overwritten).  times_ms: HOST, n_cand
 * doubles or NULL; receives each candidate's mean time per evaluation in
 * milliseconds, -1 where the candidate could not be planned (for instance
 * kappa out of range).  Blocks.  Errors: PDMK_ERR_INVALID_ARG for null
 * arguments or n_cand < 1; the status of the first candidate when none
 * could be planned; evaluation errors of a planned candidate are returned
 * at once (they do not depend on the candidate).
 */
int pdmk_plan_tune(const pdmk_opts* opts, const double* L, int n_cand, const double* kappa,
                   const int* n_s, int trials, int64_t n_src, const double* src,
                   const double* q, int64_t n_trg, const double* trg, double* pot,
                   void* stream, double* times_ms, double* best_kappa, int* best_n_s);

/* Geometry and parameters a plan derived from (opts, L); host only. */
typedef struct {
  int dim;
  double L_oriented[9];   /* upper-triangular L after orientation (eq:Ltri), column-major */
  double Q[9];            /* x_oriented = Q^T x ; column-major */
  int perm[3];            /* input lattice vector feeding oriented column i */
  double volume;          /* |det L| */
  double rc;              /* root cube side */
  int nroot[3];           /* m_i, inner block of root cubes (eq:mi) */
  double origin[3];       /* corner of the extended root grid (x^- - r_c) */
  int fgrid[3];           /* Fourier grid per axis actually used (>= M_i of eq:Mi) */
  int fgrid_paper[3];     /* M_i of eq:Mi */
  int n_shifts;           /* lattice shifts passing the bounds of eq:shift_bounds */
  double c;               /* PSWF bandwidth with psi(1)/psi(0) = eps */
  double w0_zero_rc;      /* 3D: W_0(0) * r_c (eq:W0zero); 2D: W_0(0) at r_c = 1 */
  int porder, npw, nufft_w, n_s;
  double nufft_beta, kappa;
} pdmk_geometry;
int pdmk_plan_geometry(const pdmk_plan* plan, pdmk_geometry* out);
/* The same geometry computed on the host from (opts, L) without a device. */
int pdmk_geometry_get(const pdmk_opts* opts, const double* L, pdmk_geometry* out);

/* Counters and stage times (milliseconds, from HIP events) of the last
 * pdmk_plan_eval on this plan. */
typedef struct {
  int64_t n_src, n_trg, n_images;   /* n_images: N' (originals + images) */
  int n_levels;
  int64_t n_boxes, n_leaves, n_nonleaf;
  int64_t n_direct_pairs;           /* target-source pairs visited by the residual sums */
  int64_t n_pw_pairs;               /* plane-wave box pairs */
  double t_build_ms, t_near_ms, t_far_ms, t_total_ms;
                                    /* t_far_ms: the far field's grid steps (run on the
                                       plan's second stream beside the build and near
                                       field, so they overlap those times) plus the
                                       interpolation */
  double t_direct_ms, t_pw_ms, t_proxy_ms;
  int64_t n_support_pairs;          /* visited pairs inside the residual support (r < h) */
  int series_len;                   /* terms of the residual series the residual sums used */
  double t_call_ms;                 /* host wall time of the whole call */
  int64_t workspace_bytes;          /* device workspace the call used */
  int64_t n_pwout_boxes;            /* boxes given outgoing plane waves (all levels) */
  int64_t n_pwin_boxes;             /* boxes given incoming plane waves (with targets) */
  double t_pwout_ms, t_pwin_ms;     /* time of the outgoing / incoming plane-wave kernels */
  double t_pwtr_ms;                 /* time of the colleague translation kernel (matrix-core
                                       path; 0 where the incoming kernel translates itself) */
  int64_t n_staged_pairs;           /* pairs the residual sums evaluated after dropping the
                                       list sources out of reach of each 64-target pass */
  double t_spread_ms;               /* far field: spreading (on the second stream unless
                                       PDMK_ONE_STREAM, so it may overlap other stages) */
  double t_fft_ms;                  /* far field: forward FFT, scaling, inverse FFT */
  double t_interp_ms;               /* far field: interpolation at the targets */
  int64_t n_forced_splits;          /* PDMK_BALANCE: leaves split for the 2:1 balance */
  int balance_rounds;               /* PDMK_BALANCE: tree builds until balanced */
  int pairs_once;                   /* 1: the residual sums evaluated each pair of points in
                                       different leaves once and added it to both (see
                                       PDMK_ALL_PAIRS); the pair counts are those evaluated */
} pdmk_stats;
int pdmk_plan_stats(const pdmk_plan* plan, pdmk_stats* out);
int pdmk_batch_stats(const pdmk_batch* batch, int sys, pdmk_stats* out);

/* Kernel-splitting scalars for (dim, eps); host only.  Pins the host
 * implementation of the PSWF calibration (Section 2.2) and of the split
 * kernels (eq:pswf_split, eq:W0zero) without a device. */
typedef struct {
  double c;          /* bandwidth: psi(1)/psi(0) = eps */
  double lambda0;    /* eigenvalue of eq:pswf_eig */
  double c0_over_psi0; /* int_0^1 psi / psi(0) */
  double w0_zero;    /* 3D: W_0(0) for r_c = 1 (eq:W0zero); 2D: W_0(0) for r_c = 1 */
} pdmk_kernel_info;
int pdmk_kernel_info_get(int dim, double eps, pdmk_kernel_info* out);

/* Residual kernel R_h(r) = G(r) - W_h(r) (zero for r >= h) and the smooth
 * far-field transform What_0(k) = psi~(k r_c / c) / k^2 evaluated on the host
 * from the same tables the device uses; for tests. */
int pdmk_kernel_eval_residual(int dim, double eps, double h, int64_t n,
                              const double* r, double* out);
int pdmk_kernel_eval_w0hat(int dim, double eps, double rc, int64_t n,
                           const double* k, double* out);

/* Status text and the thread-local message of the last failure. */
const char* pdmk_status_string(int status);
const char* pdmk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PDMK_H */
