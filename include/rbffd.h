/*
 * rbffd.h -- C ABI of the MI355X (gfx950) RBF-FD library.
 *
 * The library computes, on one GPU, the data-parallel hot path of the
 * polyharmonic-spline + polynomial RBF-FD method (Barnett, Flyer & Wicker,
 * arXiv 1509.02615):
 *   A1  stencil search: the n nodes nearest each centre           (Section 6, App. A)
 *   A2-A4 batched weights: one saddle-point solve per stencil    (Section 3, Eq. weights;
 *                                                                 Section 5.3, Eq. eqn:laplacian)
 *   B1  ghost-node closure per Runge-Kutta stage                 (Section 5.2, Eq. bcEqn;
 *                                                                 BCs of Section 6.4)
 *   B2-B3 fused gather-stencil products + PDE right-hand side   (Section 6.1; Eqs. uEq-piEq)
 *   B4  Runge-Kutta stages fused into the right-hand side        (Section 6: RK4)
 *
 * Conventions (every entry point):
 *   - Every array argument is a DEVICE pointer on the context's device,
 *     owned by the caller, unless stated otherwise. Scalars are by value.
 *   - All work is enqueued on the context's HIP stream; an entry point returns
 *     once the work is enqueued, except where it says it synchronises.
 *   - Return value: RBFFD_OK (0) or a negative rbffd_status code. Nothing is
 *     thrown across the ABI. On RBFFD_EINVAL nothing has been written.
 *     rbffd_last_error() gives a message for the last failing call.
 *   - A context (and the models created from it) is used by one host thread
 *     at a time.
 *   - Node coordinates are (x, z) pairs in FP64, [n_nodes][2] row-major.
 *   - Field arrays ("state") are [n_nodes][E][F] row-major: node-major, then
 *     ensemble member, then field. F = 1 (psi) for transport, F = 4
 *     (u, w, theta', pi') for Navier-Stokes. The element type is the model's
 *     field dtype.
 */
#ifndef RBFFD_H
#define RBFFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbffd_ctx rbffd_ctx;     /* opaque, library-owned */
typedef struct rbffd_model rbffd_model; /* opaque, library-owned */

typedef enum {
  RBFFD_OK = 0,
  RBFFD_EINVAL = -1,     /* bad argument; nothing written                         */
  RBFFD_ENOMEM = -2,     /* device or host allocation failed                      */
  RBFFD_EDEVICE = -3,    /* HIP runtime error                                     */
  RBFFD_ESINGULAR = -4,  /* some stencil systems are singular (see status[])      */
  RBFFD_ENONFINITE = -5  /* a state value became Inf/NaN during rbffd_step        */
} rbffd_status;

/* Differential operators L (Section 3: "the operator L"). */
typedef enum {
  RBFFD_DX = 1,        /* d/dx                                                   */
  RBFFD_DZ = 2,        /* d/dz (the second coordinate; d/dy in the unit square)  */
  RBFFD_LAP = 3,       /* Laplacian                                              */
  RBFFD_HYPERLAP = 4,  /* Laplacian^k, k = rbffd_op.k (Section 5.3)              */
  RBFFD_DZZ = 5,       /* d2/dz2 (wall closure of w, Section 6.4)                */
  RBFFD_DXX = 6        /* d2/dx2 (lateral-wall closure of u, Section 6.5)        */
} rbffd_op_kind;

typedef struct {
  int32_t kind;       /* rbffd_op_kind                                              */
  int32_t k;          /* power for RBFFD_HYPERLAP; 0 = (m_eff - 1)/2, the largest power
                         for which Laplacian^k r^m stays continuous (m >= 2k+1)        */
  int32_t phs_order;  /* PHS order m used for this operator; 0 = the stencil's m.
                         Operators of equal order share one factorisation.           */
  int32_t reserved;   /* must be 0                                                   */
} rbffd_op;

/* Node set and per-stencil method parameters (Section 3: node set, stencil
 * size n, PHS order m (odd, phi = r^m), polynomial degree l). */
typedef struct {
  int64_t n_nodes;          /* N: nodes searched as neighbours                         */
  const double *xy;         /* [N][2] FP64 (x, z)                                      */
  double period_x;          /* x period for the minimum image; 0 = not periodic.
                               With a period all x must lie in one interval of that
                               length.                                                  */
  int64_t n_centers;        /* Nc: number of stencils (0: an empty batch, a no-op)     */
  const int32_t *centers;   /* [Nc] centre node indices, or NULL = 0..Nc-1             */
  int32_t n_max;            /* stencil row length of idx/w (1..120)                    */
  const int32_t *n_per;     /* [Nc] stencil size per centre (<= n_max), or NULL = n_max */
  int32_t m_uniform;        /* odd PHS order, 1 <= m <= 15, used when m_per is NULL     */
  const int32_t *m_per;     /* [Nc] or NULL                                            */
  int32_t l_uniform;        /* polynomial degree 0..6, used when l_per is NULL          */
  const int32_t *l_per;     /* [Nc] or NULL                                            */
  const int32_t *idx_in;    /* [Nc][n_max] given stencils (skip the search), or NULL    */
} rbffd_stencils;

enum { RBFFD_SOLVE_FP64 = 0, RBFFD_SOLVE_FP32_IR = 1 };
enum { RBFFD_F64 = 0, RBFFD_F32 = 1, RBFFD_BF16 = 2 };
enum { RBFFD_PHYS_ADVECTION = 1, RBFFD_PHYS_NS = 2 };
enum { RBFFD_RK4 = 0, RBFFD_WSRK3 = 1 };

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`; `hip_stream` is a hipStream_t
 * (NULL = the null stream) that every call of this context is ordered on. */
int rbffd_create(rbffd_ctx **out, int device, void *hip_stream);
int rbffd_destroy(rbffd_ctx *ctx);
/* Message of the last failing call on this context (never NULL). */
const char *rbffd_last_error(rbffd_ctx *ctx);
/* Block until all work enqueued on the context's stream has finished. */
int rbffd_sync(rbffd_ctx *ctx);

/* ---- A1: stencil search ------------------------------------------------- */

/* For each centre c: the n_c nodes with the smallest key (d^2, j), in that
 * order, where d^2 = dx*dx + dz*dz is evaluated in IEEE FP64 with two
 * rounded products and a rounded sum (no fused multiply-add) and dx is the
 * minimum image for a periodic x (shifted by one period when |dx| > period/2).
 * Section 6 uses the n = 37 nearest nodes (a complete symmetric set on
 * Cartesian and hexagonal lattices, Appendix A).
 * Output idx [Nc][n_max] int32, entries past n_c set to -1. Ignores m and l.
 * Synchronises (argument checks, grid set-up). EINVAL (nothing written): a
 * centre outside the node set, n_c outside 1..min(n_max, N), non-finite
 * coordinates. Dense clusters (more candidates near a centre than the
 * search holds on chip) are searched by a slower exact kernel. */
int rbffd_knn(rbffd_ctx *ctx, const rbffd_stencils *st, int32_t *idx);

/* ---- A1-A4: batched weights -------------------------------------------- */

/* One row of each differentiation matrix per centre (Section 3, Eq. weights):
 * with phi(r) = r^m and all monomials of degree <= l, solve
 *     [Phi P; P^T 0] [w; v] = [L phi(|x - x_j|) at x_c ; L p(x_c)]
 * and keep w. The system is formed in a frame centred at x_c and scaled by
 * the largest centre-to-node distance, solved by LU with partial pivoting in
 * FP64 (or an FP32 factorisation when precision = RBFFD_SOLVE_FP32_IR) plus
 * iterative refinement with double-double residuals, then rescaled.
 * Runs the A1 search first unless st->idx_in is given (then idx is a copy).
 * Outputs: idx [Nc][n_max] (may be NULL when idx_in is given),
 *          w [n_ops][Nc][n_max] FP64 (zero past n_c),
 *          status [Nc] (NULL allowed): 0 ok, 1 singular (smallest pivot below
 *          1e-13 max|A|, or refinement did not converge: it stops when the
 *          error left after a correction d, estimated as |d|^2 / |d_prev|
 *          from the contraction of successive corrections, is below
 *          2^-52 |x|, or when |d| <= 2^-48 |x|), 3 ok after an FP64 solve
 *          (RBFFD_SOLVE_FP32_IR only: stencils whose FP32-factorisation
 *          refinement stalls are solved again with the FP64 factorisation).
 * Returns RBFFD_ESINGULAR (after writing everything) when any status is 1;
 * synchronises to read the status count. EINVAL (nothing written: every
 * per-stencil parameter and given index is checked on the device before the
 * search or a solve starts): even m, l > 6, n_c < M, K = n_c + M > 128,
 * Laplacian^k with m < 2k+1, n_ops outside 1..8, a centre or given stencil
 * index outside the node set. */
int rbffd_weights(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops,
                  int precision, int32_t *idx, double *w, int32_t *status);

/* Autotuning of the batched weights (Section 3's O(n^3 N) preprocessing):
 * stencils are grouped by system size K = n + M into RBFFD_WEIGHT_BUCKETS
 * buckets (K <= 32, 48, 64, 80, 96, 128), each solved by one launch that
 * drains the bucket's queue; stencils the two-systems-per-wavefront kernel
 * cannot pair, and (FP32 factorisation) systems whose refinement stalls, go
 * to further device-side queues drained without a host round trip. A launch
 * shape per bucket sets the grid (workgroups per compute unit of a
 * persistent grid, or one workgroup per system) and, for K <= 32, two systems
 * per wavefront or one; shapes never change a system's arithmetic, so every
 * shape gives bit-identical results. This call computes the same outputs as
 * rbffd_weights; for every bucket whose shapes[b] is -1 it runs each of the
 * bucket's shapes twice (the batch is solved twice per shape), times the
 * bucket's launches with HIP events and keeps the fastest in the context for
 * later rbffd_weights calls; shapes[b] >= 0 forces that shape (0 is the
 * default).
 * shapes (host, [RBFFD_WEIGHT_BUCKETS], in/out, or NULL = tune all) returns
 * the chosen shapes, bucket_ms (host or NULL) the chosen shapes' times.
 * Shape counts: 4 for bucket 0 (two systems per wavefront with one wavefront
 * per pair (0) or a persistent grid (1); one system per wavefront, one
 * wavefront per system (2) or persistent (3)), 2 for buckets 1-2 (one
 * wavefront per system, or persistent), 4 for buckets 3-5 (one workgroup per
 * system, or 1, 2, 4 persistent workgroups per compute unit). A persistent
 * grid holds as many wavefronts as the compute units keep resident. Synchronises. Errors as rbffd_weights; EINVAL
 * for a shape outside its bucket's range. */
#define RBFFD_WEIGHT_BUCKETS 6
int rbffd_weights_tune(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops, int precision,
                       int32_t *idx, double *w, int32_t *status, int32_t *shapes, double *bucket_ms);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * operation as rbffd_weights (same arguments, outputs, status codes and
 * kernels, bit-identical results) without any device allocation. Its scratch
 * (search grid, bucket lists, status when `status` is NULL) is a fixed
 * region of about 64 MiB that the library holds on every device it runs on
 * until the process ends, set up by rbffd_create. Limits: n_nodes <=
 * RBFFD_NOALLOC_MAX_NODES and n_centers <= RBFFD_NOALLOC_MAX_CENTERS, else
 * RBFFD_EINVAL with nothing written. Every call on a device shares that
 * device's region: calls that overlap on one device (from several contexts
 * or threads) race and must be serialised by the caller. It still
 * synchronises like rbffd_weights. */
#define RBFFD_NOALLOC_MAX_NODES 2097152
#define RBFFD_NOALLOC_MAX_CENTERS 2097152
int rbffd_weights_noalloc(rbffd_ctx *ctx, const rbffd_stencils *st, const rbffd_op *ops, int n_ops,
                          int precision, int32_t *idx, double *w, int32_t *status);

/* ---- B1-B4: right-hand side model -------------------------------------- */

typedef struct {
  int32_t physics;        /* RBFFD_PHYS_ADVECTION or RBFFD_PHYS_NS                      */
  int32_t field_dtype;    /* RBFFD_F64 or RBFFD_F32 (state element type)                */
  int32_t weight_dtype;   /* RBFFD_F64, RBFFD_F32 or RBFFD_BF16 storage of the weights
                             (closure weights stay FP64). F32: every weight as its FP32
                             rounding plus a small correction of Lap^k (within about
                             2^-30 of FP64), Dx and Dz (about 2^-29). BF16: Dx, Dz and
                             Lap as bfloat16 plus an 8-bit correction (about 2^-16),
                             Lap^k as FP32 plus an 8-bit correction (about 2^-32). With
                             F32 and BF16 the hyperviscosity sums and the divergence
                             u_x + w_z run in FP64 on the corrected weights, the other
                             sums in FP32; ghost values are kept in FP64 beside the FP32
                             state for the sums of the nodes next to walls; Lap^k
                             weights must lie in the FP32 normal range. F32/BF16 need
                             field_dtype F32. */
  int32_t n;              /* stencil length (row length of idx and w)                    */
  int64_t n_total;        /* N: all nodes including ghosts                               */
  int64_t n_active;       /* nodes 0..n_active-1 carry stencils and prognostic values;
                             n_active..N-1 are ghost nodes                               */
  int32_t ensemble;       /* E >= 1 members sharing the weights                          */
  int32_t reserved0;
  const int32_t *idx;     /* [n_active][n] stencils (indices < N)                        */
  const double *w;        /* [n_ops][n_active][n] weights. Transport: Dx, Dz, Lap^k.
                             Navier-Stokes: Dx, Dz, Lap, Lap^k.                         */
  const double *xy;       /* [N][2] node coordinates (z gives pi-bar(z))                 */
  double hv_coeff;        /* coefficient of the Lap^k term added to every field's
                             tendency (sign included; +gamma for k = 3)                 */
  /* transport (Section 6.1, flux form): velocity (U, V)(x) * cos(pi t / vel_period) */
  const double *vel_u;    /* [n_total] U at the nodes (read at stencil neighbours)       */
  const double *vel_v;    /* [n_total] V at the nodes                                    */
  double vel_period;
  /* Navier-Stokes constants (Section 6.2, 6.4) */
  double c_p, c_v, R_d, g, theta_bar, mu;
  double u_bar;           /* uniform background wind added to u in the advective terms
                             (translating density current, Section 6.4.2); 0 otherwise */
  /* ghost closure (Section 5.2), Navier-Stokes only. One boundary row per
   * (boundary node, wall): a corner node of a closed box has two rows, one
   * per wall, each with its own ghost. Row r's stencil is idx[bnd_nodes[r]].
   * Walls normal to z (bottom, top; Section 6.4): du/dz = dtheta'/dz = 0,
   * dpi'/dz = g theta' / (c_p theta_bar (theta_bar + theta')), w = 0 and
   * d2w/dz2 = 0. Walls normal to x (lateral; Section 6.5): u = 0,
   * d2u/dx2 = 0, dw/dx = dtheta'/dx = dpi'/dx = 0. */
  int32_t n_bnd;          /* number of boundary rows (0: no walls)                       */
  int32_t reserved1;
  const int32_t *bnd_nodes;   /* [n_bnd] active index of each row's boundary node        */
  const int32_t *bnd_ghosts;  /* [n_bnd] its ghost node (each ghost in exactly one row;
                                 every node >= n_active is a ghost)                      */
  const int32_t *bnd_normal;  /* [n_bnd] 0: wall normal to z, 1: wall normal to x         */
  const double *bnd_d1;   /* [n_bnd][n] weights of the first derivative along the normal
                             (Dz or Dx) at the boundary node                             */
  const double *bnd_d2;   /* [n_bnd][n] weights of the second derivative along the normal
                             (Dzz or Dxx)                                                */
  /* transport mirror boundary (Section 6.1): nodes past n_active are mirror
   * ghosts whose values are copied from active node mirror_src[k] before
   * every right-hand side; required for transport when n_total > n_active */
  const int32_t *mirror_src;  /* [n_total - n_active] or NULL                           */
} rbffd_model_desc;

/* Build a model: repack stencils and weights into the library's slot-major
 * layout, mark wall nodes, and factor and invert the ghost blocks W_G
 * (Section 5.2; one per field's operator set, split into the independent
 * groups of rows that share no ghost) once on the host, keeping each inverse
 * row to rounding accuracy as its entries above a certified cut-off.
 * Synchronises. The caller's arrays may be freed after. EINVAL:
 * inconsistent sizes or indices, a ghost listed twice or missing, F32
 * hyperviscosity weights outside the FP32 normal range; ESINGULAR: a
 * singular W_G. */
int rbffd_model_create(rbffd_ctx *ctx, const rbffd_model_desc *desc, rbffd_model **out);
int rbffd_model_destroy(rbffd_model *model);

/* B1 alone: set w = 0 on the wall nodes and fill the ghost rows of `state`
 * ([N][E][F]) from W_G u_G = bc - W_I u_I - W_B u_B for u, theta' (bc 0),
 * pi' (bc = g theta'/(c_p theta_bar (theta_bar + theta'))) with the Dz rows
 * and w (bc 0) with the Dzz rows. No-op for transport models. */
int rbffd_ghost(rbffd_ctx *ctx, rbffd_model *model, void *state);

/* B1-B3: one right-hand-side evaluation at time t. Runs the closure on
 * `state` (its wall-w and ghost entries are overwritten), then writes
 * tendency [N][E][F] for the active nodes (ghost rows and wall dw/dt set 0). */
int rbffd_rhs(rbffd_ctx *ctx, rbffd_model *model, double t, void *state, void *tendency);

/* B1-B4: advance `state` in place by n_steps steps of size dt with the
 * tableau (RBFFD_RK4: classical RK4; RBFFD_WSRK3: y1 = y + dt/3 f(y),
 * y2 = y + dt/2 f(y1), y + dt f(y2)). Each stage is closure -> fused
 * RHS + stage update. Eight steps and one step are captured as HIP graphs
 * when a call first needs them (recaptured when state, dt or the tableau
 * change); a call replays the eight-step graph n_steps / 8 times and the
 * one-step graph for the rest.
 * *t (host) is advanced. Synchronises at the end to check for non-finite
 * values: returns RBFFD_ENONFINITE and names the first bad step in
 * rbffd_last_error. */
int rbffd_step(rbffd_ctx *ctx, rbffd_model *model, void *state, double *t, double dt,
               int64_t n_steps, int tableau);

/* Bytes of the slot-major stencil stream (indices + weights of every
 * operator) plus per-node constants that the fused right-hand-side kernel
 * reads per node and evaluation; field traffic is not included. */
int64_t rbffd_model_bytes_per_node(rbffd_model *model);

/* Kernel timing for measurement: while enabled (enable != 0), rbffd_rhs and
 * rbffd_step launch every stage without graph replay and record a pair of
 * HIP events on the context stream around each fused right-hand-side
 * kernel. rbffd_model_profile_read synchronises and returns the summed
 * kernel time (ms) and the number of launches since the last read or
 * enable, then resets both. */
int rbffd_model_profile(rbffd_model *model, int enable);
int rbffd_model_profile_read(rbffd_model *model, double *total_ms, int64_t *launches);

/* Autotuning of the fused right-hand-side kernel: run the closure on `state`
 * (its ghost entries are overwritten), time every compiled launch shape of
 * the kernel (block size, slot unrolling, cached or non-temporal weight
 * loads) on a few evaluations of this model's data, and keep the fastest
 * for all later calls. Models of a multiple of 64 members also try
 * traversing the nodes in Morton order of their coordinates (shape index + 6).
 * *chosen on entry: -1 to time every shape, or one shape index to time and
 * keep that one alone (EINVAL, nothing changed, if it is out of range); on
 * return the shape kept and its time per launch (us). Synchronises.
 * Transport models keep their single shape (chosen = -1). */
int rbffd_model_tune(rbffd_ctx *ctx, rbffd_model *model, void *state, int *chosen, double *best_us);

/* ---- learned coarse closure (a per-node network on stencil-gathered fields) */

/* A small network corrects the right-hand side of a coarse Navier-Stokes
 * model: for node i and member e its input is the stencil-gathered state --
 * slot 0 the node's own four fields, slots k >= 1 the differences
 * f(j_k) - f(i), each field divided by in_scale[field] (37 x 4 = 148 values) --
 * plus one per-node value (node_feature[i], e.g. height / domain height),
 * zero-padded to 160. Layers: h1 = a(W1 x + b1), h2 = a(W2 h1 + b2),
 * y = W3 h2 + b3, with 128 hidden units, activation a = tanh or relu
 * (max(v, 0), one vector operation per value where tanh costs about
 * twenty), BF16 weights and activations and FP32 accumulation on the
 * matrix cores; the correction in physical units
 * is y[c] * out_scale[c]. Training minimises the mean of (y - target)^2 over
 * samples and fields with Adam on FP32 master weights.
 * Parameter layout (FP32, contiguous): W1 [128][160], b1 [128], W2 [128][128],
 * b2 [128], W3 [16][128] (rows 4..15 unused, kept 0), b3 [16] (4..15 unused). */
#define RBFFD_CLOSURE_NPARAMS (128 * 160 + 128 + 128 * 128 + 128 + 16 * 128 + 16)

typedef struct rbffd_closure rbffd_closure;  /* opaque, library-owned */

enum { RBFFD_ACT_TANH = 0, RBFFD_ACT_RELU = 1 };

typedef struct {
  int64_t max_samples;          /* largest n_active * E used with this closure        */
  const float *init_params;     /* [RBFFD_CLOSURE_NPARAMS] device, copied at creation  */
  const double *node_feature;   /* [n_active] device, copied at creation               */
  float in_scale[4];            /* input scale per field                               */
  float out_scale[4];           /* output scale per field                              */
  int32_t activation;           /* RBFFD_ACT_TANH or RBFFD_ACT_RELU                    */
} rbffd_closure_desc;

/* Bind a closure to a Navier-Stokes model (its stencils, node count and E). */
int rbffd_closure_create(rbffd_ctx *ctx, rbffd_model *model, const rbffd_closure_desc *desc,
                         rbffd_closure **out);
int rbffd_closure_destroy(rbffd_closure *cl);
/* Device pointer to the FP32 master parameters (library-owned, layout above). */
float *rbffd_closure_params(rbffd_closure *cl);
/* Correction y * out_scale for every active node and member of `state`
 * ([N][E][4] FP32, ghost rows filled): out [n_active][E][4] FP32. */
int rbffd_closure_forward(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, float *out);
/* Autotuning of the fused forward pass: times each compiled launch shape
 * (16-sample tiles per wavefront 1 or 2, wavefronts per block 4, 8 or 16,
 * wavefronts per SIMD 2 or 4: shapes 0-4) on `state` and keeps the fastest for
 * later forward, step and training calls; every shape computes the same
 * correction bit for bit. *chosen (host, in/out): -1 on entry tunes, a shape
 * 0-4 is timed and kept as given; on return the shape kept and its time per
 * call (us). Synchronises. EINVAL for a shape above 4. */
int rbffd_closure_tune(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, int *chosen, double *best_us);
/* Loss and its gradient with respect to the parameters for targets
 * [n_active][E][4] FP32 (already divided by out_scale); grad
 * [RBFFD_CLOSURE_NPARAMS] FP32 device (overwritten); *loss on the host.
 * Synchronises. */
int rbffd_closure_gradient(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, const float *target,
                           float *grad, double *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the same loss; the
 * step counter is kept inside. Synchronises to return *loss. */
int rbffd_closure_train_step(rbffd_ctx *ctx, rbffd_closure *cl, const void *state, const float *target,
                             double lr, double *loss);
/* Coarse time stepping with the correction: each of n_steps steps is one
 * rbffd_step of the model followed by state += dt * correction(state before
 * the step) on the active nodes. A member whose correction is not finite
 * keeps the plain step (the fallback); *n_fallback counts such
 * (member, step) pairs (host, may be NULL). */
int rbffd_closure_step(rbffd_ctx *ctx, rbffd_closure *cl, void *state, double *t, double dt, int64_t n_steps,
                       int tableau, int64_t *n_fallback);

/* Measurement helper: copy `bytes` (a multiple of 16, 16-byte aligned
 * pointers) from src to dst with a plain streaming kernel, so that hardware
 * memory counters can be calibrated against a kernel of known traffic. */
int rbffd_stream_copy(rbffd_ctx *ctx, void *dst, const void *src, int64_t bytes);

/* Measurement helper: a matrix-core throughput probe. Every wavefront of
 * 4 x (number of compute units) 256-thread blocks runs `iters` rounds of four
 * independent BF16 matrix products on register operands (no memory
 * traffic), of shape 16x16x32 (shape 0) or 32x32x16 (shape 1), so the
 * launch's rate (timed by the caller on the context stream) is that shape's
 * dense BF16 ceiling on this device. out: device, at least
 * 1024 x (number of compute units) floats, one value per thread is written;
 * *flops (host) receives the launch's flop count. RBFFD_EINVAL for another
 * shape, a short out or iters < 1. */
int rbffd_mfma_probe(rbffd_ctx *ctx, int shape, float *out, int64_t n_out, int iters, int64_t *flops);

#ifdef __cplusplus
}
#endif
#endif /* RBFFD_H */
