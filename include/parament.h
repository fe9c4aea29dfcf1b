/*
 * parament.h -- C ABI of the MI355X parallel-in-time Schrodinger propagator.
 *
 * The library computes the propagator of
 *     i dU/dt = H(t) U,   H(t) = H0 + sum_k c_k(t) H_k         (hbar = 1)
 * (eq. schroedinger with H = hbar * calH; control decomposition
 * eq. format_control) over N equal slices of width h, following the pipeline
 * of the Computational approach section (Fig. 1):
 *   1. expand: one Hermitian exponent G_j per slice, by the midpoint rule
 *      (order 2) or by 4th-order commutator Magnus with Simpson quadrature
 *      (order 4, Magnus integrators section, eq. magnus_coeffs), or -- the
 *      commutator-free alternative the same section names -- two
 *      exponents per slice without commutators (PM_ORDER_CF4), or by the
 *      sixth-order Magnus scheme the same section points to for higher
 *      order (PM_ORDER_MAGNUS6);
 *   2. exponentiate all slices at once, U_j = exp(-i G_j), by scaling and
 *      squaring with a truncated Taylor series (Matrix exponential section);
 *   3. reduce U(T) = U_{N-1} ... U_1 U_0 (eq. slices) by chunked products and
 *      a log-depth product tree (Reduction by matrix multiplication section).
 * The usage model is the state machine of the PARAMENT library section
 * (Fig. state_machine): create a context, set the Hamiltonians once, then
 * propagate any number of control sequences.
 *
 * Conventions for every entry point
 *   - Complex arrays are interleaved (re, im) pairs of double (complex128) or
 *     float (complex64), row-major: element (r, c) of a d x d matrix is at
 *     pair index r*d + c.  Matrix stacks are [n][d][d].
 *   - Control samples are float64, laid out [n_ctrl][n_samples] (control k
 *     contiguous).  Order 2: n_samples = N, sample j is H's control value at
 *     the slice midpoint (j + 1/2) h.  Order 4: n_samples = 2N + 1 (odd,
 *     >= 3), sample i at t = i h / 2; slice j uses samples 2j, 2j+1, 2j+2.
 *     PM_ORDER_CF4 samples exactly as order 4.  PM_ORDER_MAGNUS6:
 *     n_samples = 3N, samples 3j, 3j+1, 3j+2 at the Gauss-Legendre nodes
 *     t = (j + c_i) h, c = 1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10.
 *   - dt is the slice width h for every order (for order 4 the paper's
 *     sample spacing is h/2).
 *   - Product order: later slices multiply from the left.
 *   - The caller owns every buffer passed in.  pm_set_hamiltonian copies its
 *     inputs; they persist across propagations until replaced.
 *   - Errors are reported only through pm_status; no exception or abort
 *     crosses the ABI.  On error, outputs are left untouched and the context
 *     stays usable, except after PM_E_DEVICE.  pm_last_error() describes the
 *     most recent failure on a context.
 *   - A context is neither thread-safe nor reentrant; distinct contexts are
 *     independent (PARAMENT library section).
 */
#ifndef PARAMENT_H
#define PARAMENT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pm_ctx pm_ctx;

/* Integrator codes of the `order` argument. */
enum {
    PM_ORDER_MIDPOINT = 2,  /* G_j = h H(t_j + h/2)                                 */
    PM_ORDER_MAGNUS4 = 4,   /* commutator Magnus, eq. magnus_coeffs                 */
    /* Commutator-free 4th order (the alternative to higher commutator Magnus
     * that the Magnus integrators section names; the two-exponential scheme
     * of Blanes and Moan): with A1, A2, A3 = H at the slice's three samples,
     *   U_j = exp(-i (h/12)(-A1 + 4 A2 + 3 A3)) exp(-i (h/12)(3 A1 + 4 A2 - A3)),
     * whose exponents are built from H0, H_k alone (basis 1 + n_ctrl).  The
     * 2N exponentials are propagated as the factors of the product in
     * order; per-slice output is not available (PM_E_INVALID_ARG).        */
    PM_ORDER_CF4 = 5,
    /* Sixth-order Magnus (the higher-order Magnus integrators the Magnus
     * integrators section points to; the three-node scheme of Blanes, Casas
     * and Ros).  With A1, A2, A3 = H at the slice's Gauss-Legendre nodes,
     * the moments P1 = h A2, P2 = (sqrt(15) h/3)(A3 - A1) and
     * P3 = (10 h/3)(A3 - 2 A2 + A1) give R1 = -i[P1, P2],
     * R2 = (i/60)[P1, 2 P3 + R1] and the slice exponent
     *   G_j = P1 + P3/12 - (i/240)[-20 P1 - P3 + R1, P2 + R2],
     * formed on the device from the basis {H0, H_k} (1 + n_ctrl matrices)
     * by three products per slice, then exponentiated like every other
     * exponent.  PM_FP64 contexts only (pm_set_hamiltonian returns
     * PM_E_UNSUPPORTED otherwise); per-slice output is available; the
     * gradient, trajectory, GRAPE and batch entry points do not take it
     * (PM_E_UNSUPPORTED).                                                 */
    PM_ORDER_MAGNUS6 = 6
};

typedef enum pm_status {
    PM_OK = 0,
    PM_E_INVALID_ARG = 1,   /* bad size, order, pointer or sample count      */
    PM_E_NOT_READY = 2,     /* propagation before pm_set_hamiltonian         */
    PM_E_NOT_HERMITIAN = 3, /* max|H - H^H| > 1e-12 * max(1, max|H|)        */
    PM_E_OOM = 4,           /* device or host allocation failed              */
    PM_E_DEVICE = 5,        /* HIP runtime error; the context is unusable    */
    PM_E_UNSUPPORTED = 6    /* dimension or mode not built into this library */
} pm_status;

/* Arithmetic of the exponentiate and reduce steps.  Planning (norms, choice
 * of Taylor degree and scaling exponent) is FP64 in every mode. */
typedef enum pm_precision {
    PM_FP64 = 0,       /* complex128 throughout                                */
    PM_FP32 = 1,       /* complex64 products (4 real FP32 products each);
                          squarings and the tree above the chunks in FP64      */
    PM_FP32_3M = 2,    /* complex64 with 3-real-product complex multiplication;
                          squarings and tree top in FP64                       */
    PM_BF16_SPLIT = 3  /* 3M products on BF16 hi/lo split operands with FP32
                          accumulation; squarings and tree top in FP64         */
} pm_precision;

/* Largest dimension served.  Dimensions that are not a power of two are
 * embedded (zero-padded) in the next supported size. */
#define PM_MAX_DIM 64
/* Largest Taylor degree the planner may choose. */
#define PM_MAX_TAYLOR_DEGREE 21
/* Largest Chebyshev degree (Table 1 of the paper ends at 25). */
#define PM_MAX_CHEBYSHEV_DEGREE 25

/* How the slice exponentials are evaluated (Matrix exponential section). */
typedef enum pm_expm_method {
    PM_EXPM_TAYLOR = 0,    /* truncated Taylor series with scaling and squaring (default) */
    PM_EXPM_CHEBYSHEV = 1  /* the paper's Chebyshev series (eq. chebychev_series) with
                              scaling and squaring; dimensions <= 4 by the Clenshaw
                              recurrence (Algorithm 1) in the algebra of G, larger ones
                              split into even and odd halves over T_i(2X^2 - I) */
} pm_expm_method;

/* Create a context on HIP device `device` computing in `precision`.
 * *out receives the handle (NULL on failure).  Allocates nothing on the
 * device until pm_set_hamiltonian. */
pm_status pm_create(pm_ctx **out, int device, int precision);

/* Release a context and every device buffer it owns.  NULL is accepted. */
pm_status pm_destroy(pm_ctx *ctx);

/* Upload the drift H0 [dim][dim] and controls Hk [n_ctrl][dim][dim]
 * (complex128, Hermitian; Hk may be NULL when n_ctrl == 0) and choose the
 * integrator (PM_ORDER_MIDPOINT, PM_ORDER_MAGNUS4, PM_ORDER_CF4 or
 * PM_ORDER_MAGNUS6).  For order 4 the
 * host forms the effective control Hamiltonians of eq. magnus_coeffs,
 * i[H0,H_k] and i[H_k,H_k'] (k<k'), all Hermitian, and uploads them too
 * (setHamiltonian of the PARAMENT library section).  Inputs are symmetrised
 * to exact Hermiticity after the check.  1 <= dim <= PM_MAX_DIM,
 * 0 <= n_ctrl <= 8. */
pm_status pm_set_hamiltonian(pm_ctx *ctx, int64_t dim, const double *H0,
                             int64_t n_ctrl, const double *Hk, int order);

/* Propagate with host buffers (equiprop of the PARAMENT library section).
 * samples: host [n_ctrl][n_samples] float64.  U_out: host [dim][dim]
 * complex128, receives U(T).  slices_out: NULL, or host [N][dim][dim]
 * receiving every U_j, complex128 for PM_FP64 and complex64 otherwise.
 * Synchronous.  slices_out must be NULL for PM_ORDER_CF4. */
pm_status pm_equiprop(pm_ctx *ctx, const double *samples, int64_t n_samples,
                      double dt, double *U_out, void *slices_out);

/* Same with device buffers, enqueued on `stream` (a hipStream_t; NULL = the
 * null stream) without synchronising.  samples_dev: device float64
 * [n_ctrl][n_samples]; U_out_dev: device complex128 [dim][dim];
 * slices_out_dev: NULL or device [N][dim][dim] (complex128 for PM_FP64,
 * complex64 otherwise).  Buffers must stay valid until the stream reaches
 * the end of this call's work.  The context's workspace is reused by the
 * next call on the context, so calls on one context must be ordered on one
 * stream. */
pm_status pm_equiprop_dev(pm_ctx *ctx, const double *samples_dev,
                          int64_t n_samples, double dt, double *U_out_dev,
                          void *slices_out_dev, void *stream);

/* pm_equiprop_dev for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and stream semantics as
 * pm_equiprop_dev (bitwise the same U(T) and slices), but the product
 * tree's tickets and nodes -- the propagation's only scratch memory -- live
 * in a fixed 64 MiB device array that the library holds on each device
 * until the process ends, instead of the context's buffers, and no
 * allocation of any kind is made (the context's basis, uploaded by
 * pm_set_hamiltonian, and the caller's buffers are used as given).  A
 * propagation whose tree needs more than the array (4 KiB per tree node at
 * dimensions 5..16, 16 KiB at 17..32, 64 KiB at 33..64; about
 * 2 * chains / 4 + 64 nodes at 5..16 and 2 * chains + 64 above) returns
 * PM_E_INVALID_ARG; longer chains (pm_set_chunk) shrink the tree.  The
 * array is shared by every call on a device and keeps the last call's
 * contents; its tickets are cleared on `stream` (by a fill kernel) before
 * each launch.  Calls whose work overlaps on one device (other streams,
 * other threads, other contexts) race on the array: order them on one
 * stream. */
pm_status pm_equiprop_dev_noalloc(pm_ctx *ctx, const double *samples_dev,
                                  int64_t n_samples, double dt, double *U_out_dev,
                                  void *slices_out_dev, void *stream);

/* Adjoint gradient (the paper's outlook on GRAPE-style optimal control,
 * Applications and outlook section).  For a real loss L of U(T) with
 * dL = Re Tr(W^H dU(T)) -- W is 2 dL/d conj(U), the convention of PyTorch's
 * complex gradients -- writes dL/d samples into grad_dev (float64
 * [n_ctrl][n_samples]).  Runs its own forward pass (U(T) written to
 * U_out_dev when non-NULL, complex128 [dim][dim], which must not overlap
 * W_dev, samples or grad_dev; the backward pass reads it there) keeping one checkpoint
 * product per chain of consecutive slices (see pm_set_chunk) and the product
 * tree's nodes, then a backward pass that recomputes each chain's slice
 * propagators from its checkpoint and contracts the Frechet derivatives of
 * exp(-i G_j) with the basis (the chain rule through the expand step's
 * weights gives the sample gradient).  W_dev: device complex128 [dim][dim].
 * Enqueued on `stream`; PM_FP64 contexts only (PM_E_UNSUPPORTED otherwise). */
pm_status pm_backward_dev(pm_ctx *ctx, const double *samples_dev, int64_t n_samples,
                          double dt, const double *W_dev, double *grad_dev,
                          double *U_out_dev, void *stream);

/* What a trajectory holds at every slice boundary t_j = j h, j = 0..N
 * (P_j = U_{j-1} ... U_0, P_0 = I): */
typedef enum pm_trajectory_kind {
    PM_TRAJ_PROPAGATORS = 0,  /* P_j                        out [N+1][dim][dim]   */
    PM_TRAJ_STATES = 1,       /* P_j Psi_0, Psi_0 [dim][n]  out [N+1][dim][n]     */
    PM_TRAJ_DENSITY = 2       /* P_j rho_0 P_j^H            out [N+1][dim][dim]   */
} pm_trajectory_kind;

/* Time evolution at every slice boundary (the trajectory of eq. slices'
 * partial products; states psi(t) = U(t) psi_0 and rho(t) = U(t) rho_0
 * U(t)^H, Computational approach section).  A forward pass keeps the
 * product tree (as the gradient does); each chain then starts from its
 * checkpoint product and multiplies its recomputed slices in, writing the
 * prefix before each slice.  x0_dev: NULL for PM_TRAJ_PROPAGATORS, device
 * complex128 [dim][n_vec] states (1 <= n_vec <= dim) for PM_TRAJ_STATES,
 * device complex128 [dim][dim] for PM_TRAJ_DENSITY.  out_dev: device
 * complex128, N+1 blocks as listed above.  Enqueued on `stream`; PM_FP64
 * contexts only (PM_E_UNSUPPORTED otherwise); Taylor series. */
pm_status pm_trajectory_dev(pm_ctx *ctx, const double *samples_dev, int64_t n_samples, double dt,
                            int kind, const double *x0_dev, int64_t n_vec, double *out_dev,
                            void *stream);

/* Optimisers of pm_grape_dev. */
typedef enum pm_optimizer {
    PM_OPT_GD = 0,    /* c <- c - step * grad                                        */
    PM_OPT_ADAM = 1   /* Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments) */
} pm_optimizer;

/* Gradient-based optimal control of the gate fidelity (GRAPE, Applications
 * and outlook section): `iters` updates of the control samples samples_dev
 * (device float64 [n_ctrl][n_samples], overwritten with the optimised
 * controls) for L = 1 - |Tr(V^H U(T))|^2 / dim^2, V_dev device complex128
 * [dim][dim].  Each iteration runs the checkpointed forward pass, the loss
 * (on the device), the adjoint and the update; loss_dev (device float64,
 * iters + 1 values) receives L before every update and after the last.  The
 * whole loop is enqueued on `stream` without host synchronisation.  PM_FP64
 * contexts only; Taylor series. */
pm_status pm_grape_dev(pm_ctx *ctx, double *samples_dev, int64_t n_samples, double dt,
                       const double *V_dev, int iters, double step, int optimizer,
                       double *loss_dev, void *stream);

/* Gate-fidelity loss and its gradient with host buffers (synchronous):
 * L = 1 - |Tr(V^H U(T))|^2 / dim^2 for the target V (host complex128
 * [dim][dim]); *loss receives L, grad (host float64 [n_ctrl][n_samples])
 * dL/d samples, U_out (NULL or host complex128 [dim][dim]) U(T).  PM_FP64
 * contexts only. */
pm_status pm_fidelity_grad(pm_ctx *ctx, const double *samples, int64_t n_samples,
                           double dt, const double *V, double *loss, double *grad,
                           double *U_out);

/* ---- batches of independent, uneven instances ---------------------------
 * Many propagation problems (any mix of dimensions, control counts, slice
 * counts and orders) in one persistent launch on one device.  Each instance
 * follows the same conventions as a single context; its U(T) lands in a
 * concatenated output [instance][dim][dim] complex128.  Chains of
 * consecutive slices from every instance are grouped in packets (a block's
 * worth of work) and served longest-first from a shared queue; the launch is
 * captured once in a HIP graph and replayed.  Instances of dimension <= 16
 * are embedded in 16 (32 and 64 use their own tile layouts). */
typedef struct pm_batch pm_batch;

typedef struct pm_instance {
    int64_t dim;             /* 1..PM_MAX_DIM                                  */
    int64_t n_ctrl;          /* 0..8                                           */
    int order;               /* PM_ORDER_MIDPOINT, _MAGNUS4 or _CF4            */
    const double *H0;        /* host complex128 [dim][dim]                     */
    const double *Hk;        /* host complex128 [n_ctrl][dim][dim] (or NULL)   */
    const double *samples;   /* host float64 [n_ctrl][n_samples] (or NULL)     */
    int64_t n_samples;       /* order 2: N; order 4 and CF4: 2N + 1            */
    double dt;               /* slice width h                                  */
} pm_instance;

/* Create / release a batch on `device` computing in `precision`. */
pm_status pm_batch_create(pm_batch **out, int device, int precision);
pm_status pm_batch_destroy(pm_batch *b);

/* Validate, build every instance's basis and plan, and upload everything
 * (copies the caller's buffers; replaces a previous set).  Inputs are checked
 * like pm_set_hamiltonian / pm_equiprop; on error nothing is kept. */
pm_status pm_batch_set(pm_batch *b, const pm_instance *inst, int64_t n_inst);

/* Slices per chain for the instances of embedding dimension dim_class (16, 32
 * or 64); 0 restores the default.  Takes effect at the next pm_batch_set. */
pm_status pm_batch_set_chunk(pm_batch *b, int dim_class, int64_t chunk);

/* Enqueue the whole batch on `stream` (a hipStream_t, NULL = null stream). */
pm_status pm_batch_run(pm_batch *b, void *stream);

/* Synchronise and copy every U(T) (concatenated complex128, instance order)
 * into the host buffer U_out of n_doubles doubles (2 * sum dim^2 needed). */
pm_status pm_batch_result(pm_batch *b, double *U_out, int64_t n_doubles);

/* Device pointer to the concatenated results (valid until the next
 * pm_batch_set or pm_batch_destroy). */
pm_status pm_batch_output_dev(pm_batch *b, const double **out);

/* Packets of the current set and the number of doubles of its output. */
int64_t pm_batch_packets(const pm_batch *b);
int64_t pm_batch_output_doubles(const pm_batch *b);

/* Most recent failure on b; with b == NULL, why the calling thread's last
 * pm_batch_create / pm_create failed. */
const char *pm_batch_last_error(const pm_batch *b);

/* Process-wide tuning (normally loaded from the autotuner's table):
 * key "chains": the number of slice chains the automatic chunking aims for on
 * engine class dim_class (2, 4, 16, 32, 64) in `precision`;
 * key "batch_chunk": slices per chain of batched instances of class 16, 32
 * or 64 in `precision`.  value 0 restores the built-in default.  Not
 * thread-safe; set before propagating. */
pm_status pm_tuning_set(const char *key, int dim_class, int precision, int64_t value);

/* Numerics helpers (PARAMENT library section: e.g. a different maximum
 * degree).  max_taylor_degree in [1, PM_MAX_TAYLOR_DEGREE] caps the degree
 * the planner may pick (default PM_MAX_TAYLOR_DEGREE); force_s >= 0 fixes the
 * number of squarings for every slice (the degree is then the smallest that
 * meets the precision's threshold, or the cap), -1 restores automatic choice.
 * chunk > 0 fixes how many consecutive slices one wave team multiplies before
 * the tree, 0 restores the automatic choice. */
pm_status pm_set_expm_policy(pm_ctx *ctx, int max_taylor_degree, int force_s);
pm_status pm_set_chunk(pm_ctx *ctx, int64_t chunk);

/* Uneven chain lengths (the Reduction section's chains need not be equal;
 * only their order matters).  When a propagation of dimension <= 16 runs
 * exactly two blocks of chains per compute unit, the chains of the blocks
 * each unit receives first take `percent` percent more slices and the others
 * correspondingly fewer: the first-dispatched waves win the SIMD's issue
 * arbitration and would otherwise finish early, leaving the second ones to
 * run alone.  percent in [0, 100] (0: equal chains), -1 (default) the
 * automatic choice: 25 in PM_FP64; in the other precisions 20 for dimensions
 * 5..16 (and slice pairs of dimension <= 8), 0 for dimensions <= 4.  Chains
 * of dimensions <= 4 stay whole multiples of 1024 slices.  U(T) changes only
 * by the association of the chain products (rounding).  Not applied to the
 * gradient's or the trajectory's forward pass.  PM_E_INVALID_ARG outside
 * that range. */
pm_status pm_set_chain_skew(pm_ctx *ctx, int percent);

/* ---- device workspace ---------------------------------------------------
 * Besides the basis uploaded by pm_set_hamiltonian, a context allocates
 * per-call workspace on its device and keeps it for the next call: the
 * product tree's nodes and tickets; for the gradient and the trajectory the
 * checkpoints (U(T) and one product per chain of slices) and, for the
 * gradient, the weight gradients of every slice (N x basis count doubles);
 * the host-buffer entry points also stage their inputs and outputs there.
 * Kinds of call for pm_workspace_plan: */
typedef enum pm_work_kind {
    PM_WORK_PROPAGATE = 0,    /* pm_equiprop_dev returning U(T) (per-slice output in the caller's buffer) */
    PM_WORK_GRADIENT = 1,     /* pm_backward_dev                                                          */
    PM_WORK_TRAJECTORY = 2    /* pm_trajectory_dev                                                        */
} pm_work_kind;

/* Limit the context's device workspace to `bytes` (0: no limit, the
 * default).  Every later call plans its chain length so that its workspace
 * fits: the automatic length is doubled until it does -- fewer tree nodes
 * and, for the gradient and the trajectory, checkpoints further apart
 * (each chain's slices are recomputed from its checkpoint, so memory is
 * traded for recomputation: the checkpoint interval grows as the limit
 * shrinks).  A call whose workspace cannot fit even as a single chain, or
 * at a chain length fixed by pm_set_chunk, returns PM_E_OOM before
 * allocating anything.  Before a call the context releases what it holds
 * from earlier calls if that plus the call's need would pass the limit.
 * Setting a limit below what is held releases it now (synchronising the
 * device).  The fixed-workspace entry point pm_equiprop_dev_noalloc does
 * not use the context's workspace. */
pm_status pm_set_workspace_limit(pm_ctx *ctx, int64_t bytes);

/* Bytes of device workspace the context holds now (-1 for NULL). */
int64_t pm_workspace_held(const pm_ctx *ctx);

/* Host-only: the chain length (*chunk_out) and device workspace in bytes
 * (*bytes_out, may be NULL) a call of `kind` with n_samples samples would
 * use on a context of this dimension, control count, order and precision
 * with no chunk override, under the workspace limit `limit` (0: none);
 * PM_E_OOM if it cannot fit, PM_E_UNSUPPORTED for a kind or order the
 * precision does not take.  No GPU is touched. */
pm_status pm_workspace_plan(int64_t dim, int64_t n_ctrl, int order, int precision,
                            int64_t n_samples, int kind, int64_t limit, int64_t *chunk_out,
                            int64_t *bytes_out);

/* Choose the exponential (pm_expm_method) for pm_equiprop / pm_equiprop_dev.
 * PM_EXPM_CHEBYSHEV: per slice, with nu = ||G_j||_1 (the spectrum lies in
 * [-nu, nu]), the planner picks the degree m <= PM_MAX_CHEBYSHEV_DEGREE and
 * squarings s minimising P(m) + s with nu / 2^s <= theta_m, P(m) = 0, 1 and
 * floor(m/2) + 1 for m = 1, 2 and m >= 3 (the products of the even/odd split
 * evaluation), ties to the smaller s, then the smaller m; theta_m from
 * pm_chebyshev_theta; the series is taken
 * on the interval [-theta_m, theta_m] (it contains the scaled spectrum), so
 * its coefficients a_k = (-i)^k J_k(theta_m) depend on m only.  Dimensions
 * <= 4 first shift G by tr G / D.  PM_FP64 contexts only (PM_E_UNSUPPORTED
 * otherwise); the gradient entry points always use the Taylor series. */
pm_status pm_set_expm_method(pm_ctx *ctx, int method);

/* The decomposition a propagation of n_samples samples that returns U(T)
 * only would use on this context (after pm_set_hamiltonian; host-only,
 * nothing is launched): *chunk slices per chain, *chains chains, *leaves
 * leaves of the product tree (chains are combined per block before the tree,
 * so leaves <= chains).  The reduction performs chains - 1 products after the
 * chains.  Without a pm_set_chunk override, a propagation with per-slice
 * output on dimensions 1 and 2 uses one chain per resident wave instead of the
 * tuned count.  *chunk is the length before the uneven split of
 * pm_set_chain_skew (which keeps the number of chains and leaves). */
pm_status pm_launch_shape(pm_ctx *ctx, int64_t n_samples, int64_t *chunk, int64_t *chains,
                          int64_t *leaves);

/* Human-readable name of a status code (static storage). */
const char *pm_status_string(pm_status s);

/* Description of the most recent failure on ctx ("" if none; static storage
 * owned by the context, valid until the next call on it).  With ctx == NULL:
 * why the calling thread's last pm_create / pm_batch_create failed. */
const char *pm_last_error(const pm_ctx *ctx);

/* ---- host-only helpers: no GPU is touched ------------------------------ */

/* Number of Hermitian basis matrices: 1 + n_ctrl (order 2, CF4 and 6), or
 * 1 + 2 n_ctrl + n_ctrl (n_ctrl - 1) / 2 (order 4, eq. magnus_coeffs:
 * 3K/2 + K^2/2 effective controls besides H0).  -1 on bad arguments. */
int64_t pm_basis_count(int64_t n_ctrl, int order);

/* The basis the device receives, in FP64: basis_out [M][dim][dim]
 * complex128 in the order H0, H_1..H_K, then for order 4 i[H0,H_k]
 * (k = 1..K), then i[H_k,H_k'] for k < k' in lexicographic order;
 * norms_out [M] their 1-norms (max column sum of |entries|).  Either output
 * may be NULL. */
pm_status pm_build_basis_host(int64_t dim, const double *H0, int64_t n_ctrl,
                              const double *Hk, int order, double *basis_out,
                              double *norms_out);

/* Real weights w_{j,m} of slice j on that basis (the expand step):
 * order 2: w = h (1, c_1[j], ..., c_K[j]);
 * CF4: `slice` numbers the 2N exponentials in product order, e = 2j + f
 *   (f = 0 the first factor of slice j, f = 1 the second):
 *   w_H0 = h/2, w_Hk = (h/12)(3 s0_k + 4 s1_k - s2_k) for f = 0 and
 *   (h/12)(-s0_k + 4 s1_k + 3 s2_k) for f = 1;
 * order 4 with s0, s1, s2 = samples 2j, 2j+1, 2j+2:
 *   w_H0 = h, w_Hk = (h/6)(s0_k + 4 s1_k + s2_k),
 *   w_i[H0,Hk] = (h^2/12)(s2_k - s0_k),
 *   w_i[Hk,Hk'] = (h^2/12)(s0_k s2_k' - s2_k s0_k').
 * weights_out [M]; for PM_ORDER_MAGNUS6 weights_out [3][M] receives the
 * weights of the moments P1, P2, P3 (see PM_ORDER_MAGNUS6) with
 * s1, s2, s3 = samples 3j, 3j+1, 3j+2:
 *   P1: (h, h s2_k),  P2: (0, (sqrt(15) h/3)(s3_k - s1_k)),
 *   P3: (0, (10 h/3)(s3_k - 2 s2_k + s1_k)). */
pm_status pm_slice_weights_host(int64_t n_ctrl, const double *samples,
                                int64_t n_samples, double dt, int order,
                                int64_t slice, double *weights_out);

/* Truncation threshold theta_m of the degree-m Taylor polynomial used for a
 * propagation of n_slices slices.  With the remainder bound
 *     R_m(theta) = theta^(m+1)/(m+1)! / (1 - theta/(m+2))
 * of exp(X) - T_m(X) for ||X|| <= theta:
 *   PM_FP64: the largest theta with R_m(theta) <= 2^-53;
 *   reduced modes: the largest theta with R_m(theta) / theta <= u / sqrt(N),
 *     u = 2^-24 (FP32 modes) or 2^-16 (BF16 split).  These modes carry each
 *     slice propagator as I + E and accumulate the chain as Q + E Q, so
 *     their rounding error per slice scales with ||E|| ~ ||G||; truncation
 *     errors of neighbouring slices add coherently (~N) while rounding errors
 *     add like a random walk (~sqrt(N)), hence the target relative to ||G||
 *     with the sqrt(N).
 * n_slices >= 1. */
pm_status pm_taylor_theta(int m, int precision, int64_t n_slices, double *theta_out);

/* Table 1 of the paper: the largest ||G|| for which the degree-m Chebyshev
 * series meets Lubich's estimate (eq. error_chebychev)
 *     4 (exp(1 - rho^2) rho)^(m+1) <= u,   rho = 2 ||G|| / (4m + 4),
 * with u = 2^-53 (PM_FP64), 2^-24 (FP32 modes) or 2^-16 (BF16 split).
 * 1 <= m <= PM_MAX_CHEBYSHEV_DEGREE. */
pm_status pm_chebyshev_theta(int m, int precision, double *theta_out);

/* The Chebyshev planner's (m, s) for ||G||_1 = nu (see pm_set_expm_method);
 * force_s >= 0 fixes s and takes the smallest feasible degree. */
pm_status pm_plan_chebyshev(double nu, int precision, int max_degree, int force_s, int *m_out,
                            int *s_out);

/* The planner's choice for a slice with ||G||_1 = nu in a propagation of
 * n_slices slices: Taylor degree m and squarings s minimising the product
 * count (ties to the smaller s), subject to nu / 2^s <= theta_m and
 * m <= max_degree. */
pm_status pm_plan_expm(double nu, int precision, int max_degree, int64_t n_slices,
                       int *m_out, int *s_out);

#ifdef __cplusplus
}
#endif

#endif /* PARAMENT_H */
