/*
 * crv.h - C ABI of libcrv, the MI355X (gfx950) hot path of the hybrid
 * IGA-ADS-CRVPINN CO2-sequestration time step (arXiv 2604.20731).
 *
 * The calls follow the paper's statement of the IGA-ADS-CRVPINN algorithm:
 *   crv_init              step 1: permeability, porosity, wells, viscosities,
 *                         initial saturation given as B-spline coefficients;
 *   crv_pretrain_pressure step 2: Adam on the robust loss (eq. 27) with S^0;
 *   crv_step              steps 4-7: L2 projection of the network pressure,
 *                         ten explicit saturation substeps (eq. 6 in the
 *                         Galerkin form of eq. 10-13, mass matrix of eq. 14),
 *                         retraining of the pressure network;
 *   crv_get_fields        the pressure map and the saturation.
 * Further calls expose single pieces of the path (robust loss and its
 * gradients, Gram and mass solves, projection, substeps) and the training
 * state, for verification, differentiation and checkpoint/resume, and the
 * paper's direct-solver pressure path that CRVPINN replaces (the IGA
 * Galerkin system of eq. 15-20: crv_pressure_galerkin, crv_step_galerkin).
 *
 * Discretisation (readings of the paper, fixed here):
 *   - unit square/cube, Ne elements per axis; collocation N = Ne, nodes
 *     x_i = i/N, i = 0..N (eq. 21), (N+1)^d nodes;
 *   - B-splines of degree r on open uniform knots, nb = Ne + r per axis;
 *   - pressure -div(alpha grad p) = q - div(g F_b), p = 0 on the boundary,
 *     g = -gravity e_v (zero unless crv_config.gravity is set; see there);
 *     alpha = K (kr_w(s)/mu_w + kr_g(s)/mu_g), kr_w = (1-s)^n, kr_g = s^n at
 *     s = clamp(S, 0, 1) (second eq. 23 with Brooks-Corey mobilities);
 *   - RES_k = a_h(u, delta_k) - (q, delta_k)_h at interior nodes (eq. 24-25),
 *     G = (delta, delta)_{nabla,h} (eq. 26, no h^-2 factor), LOSS = RES.G^-1 RES;
 *   - network u = f NN_theta(2x - 1), f the trial-function factor (zero on
 *     the boundary; crv_config.boundary_factor), tanh hidden layers, linear
 *     output.
 *
 * Array layouts (all host arrays are float64, C order, x fastest):
 *   nodal      (N+1)^d        index ((k*(N+1)) + j)*(N+1) + i
 *   interior   (N-1)^d        node (i,j[,k]) with 1 <= i,j,k <= N-1
 *   coefs      nb^d           index ((c*nb) + b)*nb + a
 *   wells      n_wells        crv_well records (x, y, rate); rate > 0 injects gas
 *   theta      n_params       per layer W (out x in, row-major) then b (out),
 *                             layers d -> width (x hidden, tanh) -> 1
 *
 * Ownership: host input arrays are read during the call and may be freed
 * afterwards.  The device workspace (d_workspace, ws_bytes) belongs to the
 * caller, must stay alive until crv_destroy and is never freed by the
 * library; with d_workspace == NULL the library allocates and owns it.
 * Output arrays are caller-allocated host buffers of the stated sizes.
 *
 * Errors: every call returns a crv_status; no C++ exception crosses the ABI.
 * crv_last_error() returns a thread-local message for the last failure.
 * A context is not thread-safe; all its work is ordered on its stream.
 */
#ifndef CRV_H
#define CRV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CRV_OK = 0,
  CRV_EINVAL = -1,   /* bad configuration, shape, value or argument */
  CRV_ENOMEM = -2,   /* workspace too small or device allocation failed */
  CRV_EHIP = -3,     /* HIP runtime error */
  CRV_ENUMERIC = -4, /* NaN/Inf found in the loss or the saturation */
  CRV_ESTATE = -5    /* call not allowed in the current state */
} crv_status;

typedef enum {
  CRV_PREC_FP32 = 0,   /* fields, solves and network in float32 (network on
                          fp32 MFMA where the shape allows) */
  CRV_PREC_BF16 = 1,   /* hidden-layer products on bf16 MFMA, float32
                          accumulate; everything else float32 */
  CRV_PREC_FP64 = 2,   /* everything in float64 (verification mode) */
  CRV_PREC_BF16X3 = 3, /* hidden-layer products as three bf16 MFMAs on
                          hi/lo-split operands (about 2^-16 relative error),
                          float32 accumulate; everything else float32 */
  CRV_PREC_BF16X3F = 4 /* split-bf16 forward (the pressure that the residual,
                          loss and projection see); in the network backward
                          the weights stay split and activations and deltas
                          are rounded to bf16 (gradient error about 2^-9,
                          random across nodes); everything else float32 */
} crv_precision;

typedef struct {
  int dim;              /* 2 or 3 */
  int n_elem;           /* Ne per axis, 4 <= Ne <= 1024 (3D: <= 256) */
  int degree;           /* B-spline degree r: 1, 2 or 3 */
  int width;            /* hidden width: 16, 32, 64 or 128 (bf16 network
                           paths: 32 or 64 with 3 or 4 hidden layers, 4 in
                           3D; plain bf16 and the mixed form also 128) */
  int hidden;           /* number of tanh hidden layers, 1..8 */
  int precision;        /* crv_precision */
  double mu_w, mu_g;    /* brine and gas viscosities */
  double relperm_exp;   /* Brooks-Corey exponent n */
  double lr, beta1, beta2, eps; /* Adam */
  int adam_iters;       /* Adam iterations per coupled step (100) */
  int substeps;         /* saturation substeps per coupled step (10) */
  double well_radius;   /* well disc radius */
  /* Gravity (eq. 5 and 9-10): g = -gravity e_v, e_v the last coordinate
   * (y in 2D, z in 3D), gravity >= 0; rho_w, rho_g >= 0 the brine and gas
   * densities.  The pressure right-hand side becomes
   * q - div_+(g K (kr_w rho_w/mu_w + kr_g rho_g/mu_g)) (forward difference
   * along e_v), the gas flux lambda_g K (grad p - rho_g g).  0 = off. */
  double gravity, rho_w, rho_g;
  /* Trial-function factor u = f NN (eq. 23: the trial functions vanish on
   * the boundary): 0 = interior indicator (default), 1 = distance factor
   * prod_a 4 x_a (1 - x_a) (also zero on the boundary, one at the centre);
   * other values CRV_EINVAL. */
  int boundary_factor;
} crv_config;

typedef struct crv_ctx crv_ctx;

/* One well (IGA-ADS-CRVPINN algorithm, step 1: the sources q_w, q_g): a disc
 * of radius crv_config.well_radius around (x, y) in 2D, a vertical cylinder
 * over the interior z nodes in 3D; rate > 0 injects gas, rate < 0 produces.
 * Three doubles, the same bytes as a row of an n x 3 float64 array. */
typedef struct {
  double x, y, rate;
} crv_well;

/* Defaults: 2D, Ne 32, r 2, width 32, 3 hidden layers, FP32, mu_w 1,
 * mu_g 0.1, n 2, Adam lr 1e-4 (the paper's value), beta (0.9, 0.999),
 * eps 1e-8, 100 iterations and 10 substeps per step, well radius 0.06,
 * no gravity. */
crv_status crv_config_default(crv_config* cfg);

/* Number of network parameters for cfg. */
crv_status crv_param_count(const crv_config* cfg, int64_t* n);

/* Device bytes crv_init needs for cfg: every array of IGA-ADS-CRVPINN
 * algorithm steps 1-7 (inputs, fields, network state, Adam moments, Gram and
 * mass factors, scratch), 256-byte aligned; the serving admission budget. */
crv_status crv_workspace_size(const crv_config* cfg, size_t* bytes);

/* Algorithm step 1.  log_perm, porosity: nodal (N+1)^d; porosity > 0.
 * wells: n_wells records; every well disc (3D: vertical cylinder over the
 * interior z nodes) must cover at least one node and no boundary node.
 * s0_coefs: nb^d initial saturation coefficients, NULL for zero.
 * theta0: initial network parameters (crv_param_count values), or NULL for
 * the seeded default: Xavier-uniform weights a (2u - 1), a = sqrt(6 /
 * (fan_in + fan_out)), u = (x_k >> 11) 2^-53 with x_k output k of SplitMix64
 * started at seed (k counts the weights in the theta layout), zero biases.
 * seed is read only when theta0 is NULL.
 * stream: a hipStream_t (NULL = default stream).  On success *out holds the
 * context.  Returns CRV_EINVAL for invalid input, CRV_ENOMEM when ws_bytes
 * is below crv_workspace_size. */
crv_status crv_init(const crv_config* cfg, const double* log_perm, const double* porosity,
                    const crv_well* wells, int n_wells, const double* s0_coefs,
                    const double* theta0, uint64_t seed, void* d_workspace, size_t ws_bytes,
                    void* stream, crv_ctx** out);

/* Algorithm step 2 (and step 7): iters Adam iterations on the robust loss
 * with the current saturation.  final_loss (nullable) receives the loss of
 * the last iteration (evaluated before its update).  Blocks until done. */
crv_status crv_pretrain_pressure(crv_ctx* ctx, int iters, double* final_loss);

/* Same iterations as crv_pretrain_pressure, enqueued on the context's stream
 * without waiting (for schedulers overlapping several contexts). */
crv_status crv_train_async(crv_ctx* ctx, int iters);

/* Wait for all work enqueued on the context's stream; CRV_ENUMERIC if a
 * non-finite saturation was flagged. */
crv_status crv_sync(crv_ctx* ctx);

/* Preconditioners of the Galerkin conjugate-gradient solve. */
#define CRV_PRECOND_JACOBI 0 /* the diagonal of S */
#define CRV_PRECOND_KRON 1   /* D (V x V) L^-1 (V x V) D: V the DST-I basis of the
                              * interior coefficients, L the symbol of the
                              * constant-coefficient operator K x M + M x K of
                              * uniform B-splines, D = sqrt(diag of that operator /
                              * diag S) (a scaled fast-diagonalisation inverse) */

/* The paper's direct-solver pressure path (eq. 15-20; 2D only): the IGA
 * Galerkin system S P = F on the B-spline space, S = int alpha grad B .
 * grad B, F = int q B + int (g F_b) . grad B with alpha and the buoyancy
 * flux F_b from the current saturation, P = 0 on the boundary coefficients.
 * Solved matrix-free by conjugate gradients with preconditioner precond
 * (CRV_PRECOND_*), from P = 0, until |F - S P| <= rtol |F| (the recursively
 * updated residual, tested on the device after every iteration) or
 * max_iters.  The solution replaces the pressure
 * coefficients the saturation substeps use.  p_coefs (nullable, host,
 * nb^2) receives them; iters and rel_residual (nullable) the iteration count
 * and |r|/|F|.  The first call allocates the solver's device arrays (owned
 * by the context, about 3 (Ne (r+1))^2 + 8 nb^2 + 5 mp^2 values, mp = nb - 2
 * rounded up to 64); CRV_EINVAL in 3D, for max_iters < 0, a negative rtol or
 * an unknown precond; blocks until done. */
crv_status crv_pressure_galerkin(crv_ctx* ctx, int max_iters, double rtol, int precond,
                                 double* p_coefs, int* iters, double* rel_residual);

/* One pass of that algorithm: cfg.substeps saturation substeps of
 * tau = dt/substeps with the current pressure coefficients, refresh, and the
 * Galerkin pressure of the new saturation (crv_pressure_galerkin).  No
 * network training.  Blocks until done. */
crv_status crv_step_galerkin(crv_ctx* ctx, double dt, int max_iters, double rtol, int precond,
                             int* iters, double* rel_residual);

/* Algorithm steps 4-7, one coupled step of length dt > 0: project the
 * network pressure, cfg.substeps substeps of tau = dt/substeps, refresh
 * alpha from the new saturation, cfg.adam_iters Adam iterations.
 * Asynchronous on the context's stream; errors of the device work (NaN
 * saturation) surface as CRV_ENUMERIC at the next synchronising call. */
crv_status crv_step(crv_ctx* ctx, double dt);

/* Serving form of crv_step (IGA-ADS-CRVPINN algorithm, steps 4-7, for n
 * scenarios): one coupled step of length dts[i] for each of the n contexts
 * (all validated first: CRV_EINVAL for a NULL context or a bad dt,
 * CRV_ESTATE for a context not pretrained; nothing is enqueued then), with
 * exactly the results of n crv_step calls.  Contexts of one configuration
 * (2D, matrix-core network) whose workspaces lie at one stride, in order and
 * without overlap, advance together: every kernel of the step runs once for
 * all of them (the scenario selects the workspace), on the first context's
 * stream, ordered after the work queued on the others' streams and before
 * their later work.  Any other set of contexts steps each on its own stream
 * with no host wait.  Asynchronous like crv_step.
 * crv_step_batch_shared: the same, except that a batched network backward
 * shares the blocks that fit on the device among the scenarios (each
 * scenario's gradient is the same sum grouped into fewer partial rows), which
 * is faster for large grids; results then match crv_step to rounding, which
 * Adam's normalised steps carry on (within each precision form's parity
 * bound), not bitwise.
 * crv_step_batch_shared_part: crv_step_batch_shared whose batched backward
 * takes 1/part of the device's resident blocks (part in [1, 16], else
 * CRV_EINVAL; part = 1 is crv_step_batch_shared), for batches stepped on
 * several streams at once: each leaves room for the others' kernels.  The
 * grouping of the gradient sums depends on part (same bound as above). */
crv_status crv_step_batch(crv_ctx* const* ctxs, const double* dts, int n);
crv_status crv_step_batch_shared(crv_ctx* const* ctxs, const double* dts, int n);
crv_status crv_step_batch_shared_part(crv_ctx* const* ctxs, const double* dts, int n, int part);

/* Outputs (any may be NULL): p_nodal (N+1)^d network pressure m*NN,
 * s_coefs nb^d, s_nodal (N+1)^d saturation at the nodes. Synchronises. */
crv_status crv_get_fields(crv_ctx* ctx, double* p_nodal, double* s_coefs, double* s_nodal);

/* Robust loss of the current parameters and its gradients (differentiation
 * form): dtheta (n_params) and dlogperm ((N+1)^d), both nullable.  Does not
 * change the training state. */
crv_status crv_loss_grad(crv_ctx* ctx, double* loss, double* dtheta, double* dlogperm);

/* Training state for checkpoint/resume: theta, Adam m and v (n_params
 * each, nullable) and the Adam step count.  crv_set_state with t = -1 keeps
 * the current step count (replacing theta alone, as the differentiation
 * form does); t < -1 is CRV_EINVAL. */
crv_status crv_get_state(crv_ctx* ctx, double* theta, double* adam_m, double* adam_v, int64_t* t);
crv_status crv_set_state(crv_ctx* ctx, const double* theta, const double* adam_m,
                         const double* adam_v, int64_t t);

/* Replace the saturation coefficients (nb^d) and refresh alpha. */
crv_status crv_set_saturation(crv_ctx* ctx, const double* s_coefs);

/* Replace the nodal log-permeability ((N+1)^d, host, finite, else
 * CRV_EINVAL) and refresh alpha = lambda_t(S) K (eq. 23, nodal form); the
 * saturation transport reads the same K.  Used by the differentiation form
 * to evaluate the loss at a new log K. */
crv_status crv_set_log_perm(crv_ctx* ctx, const double* log_perm);

/* Differentiation form on device arrays (float32 contexts; a float64
 * context gives CRV_EINVAL).  Every pointer is device memory of the
 * context's GPU, owned by the caller; a host pointer is CRV_EINVAL.
 * crv_set_params_device: theta (n_params float32, nullable) replaces the
 *   network parameters as crv_set_state(theta, NULL, NULL, -1) does;
 *   log_perm ((N+1)^d float32, nullable) replaces the nodal log K as
 *   crv_set_log_perm does (K = exp(log K) in float64, rounded once).  A
 *   non-finite log K is CRV_EINVAL and changes nothing: the check waits for
 *   the context's stream once.  The copies read the arrays in stream order.
 * crv_loss_grad_device: crv_loss_grad's loss (one float64, eq. 21-28),
 *   dtheta (n_params float32) and dlogperm ((N+1)^d float32), each nullable,
 *   written in stream order on the context's stream without waiting for
 *   it: a caller on another stream orders itself after the context's
 *   stream before reading them.  Does not change the training state. */
crv_status crv_set_params_device(crv_ctx* ctx, const float* theta, const float* log_perm);
crv_status crv_loss_grad_device(crv_ctx* ctx, double* loss, float* dtheta, float* dlogperm);

/* Inverse problem (the paper's conclusions name recovering reservoir
 * parameters as future work), read as a joint Adam on the network parameters
 * and the nodal log K.
 * crv_set_observations: host (N+1)^d arrays of pressure data d and weights
 *   w >= 0 (0: not observed; boundary nodes are ignored); data NULL clears
 *   them.  With observations every training call (pretrain, step, loss_grad,
 *   invert) uses the objective LOSS + sum_p w_p (u_p - d_p)^2, whose
 *   gradient in u gains 2 w (u - d).  CRV_EINVAL for non-finite entries or
 *   negative weights.
 * crv_invert: iters joint iterations, each: the objective's gradients in
 *   theta and in log K (dLOSS/dlogK = dLOSS/dalpha * alpha) at the current
 *   point; Adam on theta with the configured rate; Adam on log K with rate
 *   lr_logk (same betas and eps, its own moments and step count, started at
 *   zero by crv_init); then K = exp(log K) and alpha.  The objective of each
 *   iteration joins the loss history.  Synchronises with the host at the end.
 * crv_get_log_perm: the current nodal log K into a host (N+1)^d array. */
crv_status crv_set_observations(crv_ctx* ctx, const double* data, const double* weights);
crv_status crv_invert(crv_ctx* ctx, int iters, double lr_logk);
crv_status crv_get_log_perm(crv_ctx* ctx, double* log_perm);

/* Loss of each Adam iteration so far (oldest first, at most cap entries,
 * the most recent ones when more were run); *n receives the count. */
crv_status crv_loss_history(crv_ctx* ctx, double* out, int cap, int* n);

/* Single pieces, host in / host out, for verification:
 * crv_gram_solve  q = G^-1 res on the interior grid (eq. 26-28);
 * crv_mass_solve  x = (M^x (x) M^y [(x) M^z])^-1 b on coefficient arrays (eq. 14);
 * crv_project_pressure  p coefs of the L2 projection of the network
 *                       pressure (algorithm step 4);
 * crv_saturation_substeps  steps 4-6 only: project the pressure and run n
 *                       substeps of length tau (no retraining). */
crv_status crv_gram_solve(crv_ctx* ctx, const double* res, double* q);

/* crv_gram_solve without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops): the same
 * q = G^-1 res (2D) on caller-owned device arrays, with no context.
 *   n_elem  Ne, 4 <= Ne <= 512 (larger: CRV_EINVAL, before any device work)
 *   d_res   device float32, (Ne-1)^2 interior residual entries, x fastest
 *   d_q     device float32, (Ne-1)^2 entries, receives G^-1 res
 *   d_loss  device double, nullable: receives res . q (the robust loss)
 *   stream  hipStream_t the kernels are enqueued on (NULL: the null stream)
 * The call only enqueues kernels and returns; no host synchronisation, no
 * device or host allocation.  Its tables and work arrays live in one fixed
 * device array of about 7.3 MB that every GPU the library runs on holds
 * until the process ends; the call rebuilds what it reads there.  Calls
 * that overlap on one GPU (other streams, other threads) share that array
 * and race: order them on one stream.  Errors: CRV_EINVAL for a bad size or
 * a NULL array, CRV_EHIP for a launch or symbol-lookup failure. */
crv_status crv_gram_solve_noalloc(int n_elem, const float* d_res, float* d_q, double* d_loss,
                                  void* stream);
crv_status crv_mass_solve(crv_ctx* ctx, const double* b, double* x);
crv_status crv_project_pressure(crv_ctx* ctx, double* p_coefs);
crv_status crv_saturation_substeps(crv_ctx* ctx, double tau, int n);

/* Kernel timing with HIP events on the context's stream (bench and
 * profiling).  While enabled, every launch of the kernels below is bracketed
 * by an event pair; crv_profile_read synchronises and returns, for one
 * kernel id, the summed duration in milliseconds and the number of launches
 * since the last crv_profile_enable(ctx, 1). */
typedef enum {
  CRV_K_MLP_FWD = 0,   /* network forward (u at the nodes) */
  CRV_K_MLP_BWD,       /* network backward (recompute + backprop + partials;
                          on the matrix cores also the adjoint field and the
                          loss partials) */
  CRV_K_RESIDUAL,      /* collocation residual */
  CRV_K_GRAM_DST,      /* DST-I products of the Gram solve (2 events per
                          solve; in 3D each spans the z and y products) */
  CRV_K_GRAM_LINES,    /* shifted tridiagonal line solves */
  CRV_K_ADJOINT,       /* adjoint stencil + loss partials (per-node network
                          path only) */
  CRV_K_LOSS,          /* loss reduction */
  CRV_K_GRAD_REDUCE,   /* gradient partial reduction passes */
  CRV_K_ADAM,          /* fused Adam */
  CRV_K_REFRESH,       /* alpha refresh */
  CRV_K_PROJECT,       /* pressure projection assembly */
  CRV_K_ADS_ASSEMBLE,  /* saturation right-hand side */
  CRV_K_MASS_ROWS,     /* mass solve, contiguous direction */
  CRV_K_MASS_COLS,     /* mass solve, strided direction */
  CRV_K_COUNT
} crv_kernel;
crv_status crv_profile_enable(crv_ctx* ctx, int enable);
crv_status crv_profile_read(crv_ctx* ctx, int kernel, double* total_ms, int64_t* count);

crv_status crv_destroy(crv_ctx* ctx);
const char* crv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CRV_H */
