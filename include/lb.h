/*
 * lb.h - C ABI of the MI355X IMEX trust-region library for the
 * Landau-Brazovskii (LB) energy (Bao, Deng, Jiang, Zhang, arXiv 2603.03933).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid (Section 2, grid set T_M^d): a periodic orthorhombic box
 * [0,box[0]) x ... with n[a] points per axis, x_j = j * box[a] / n[a];
 * reciprocal lattice B = diag(2 pi / box), reciprocal indices k_a in
 * [-n_a/2, n_a/2); lb_plan_set_lattice replaces the box by a general
 * Bravais lattice. Supported axis lengths: 2^a 3^b with 8 <= n <= 512.
 *
 * Fields are real arrays of N = prod(n) doubles in C order (last axis
 * fastest), `batch` instances back to back. Every array argument is a DEVICE
 * pointer owned by the caller (for example a torch tensor's data_ptr()); the
 * library never frees or keeps it beyond the call. Structs (lb_grid,
 * lb_params, *_opts, *_info) are HOST pointers.
 *
 * Inner products and norms are those of the paper's Psi_hat coordinates
 * (Section 2, discrete inner product): <a,b> = (1/N) sum_x a(x) b(x) and
 * ||a|| = sqrt(<a,a>) = RMS(a). The mass constraint (Section 2, e_1^T
 * Psi_hat = 0) is enforced by removing the k = 0 Fourier mode (projection P
 * of Section 3); inputs are expected to have zero mean.
 *
 * Energy (eq. lb_energy, discretised in eq. interaction_bulk_energy):
 *   E = 1/2 sum_k Lambda_k |psi_hat_k|^2 + (1/N) sum_x F(psi(x)),
 *   Lambda_k = xi^2 (q^2 - |Bk|^2)^2, F = tau/2 psi^2 - gamma/6 psi^3 + psi^4/24.
 * The paper has xi = q = 1.
 *
 * Streams: all work is enqueued on the plan's HIP stream (`stream` is a
 * hipStream_t; NULL means the null stream). Calls that only launch kernels
 * return before the GPU finishes; calls that fill a host `info` struct
 * synchronise the stream before returning. A plan is not thread safe: use one
 * plan per stream. Plans allocate all their device workspace in
 * lb_plan_create; no other call allocates, except lb_lanczos_min, which adds
 * its Krylov basis to the plan the first time it needs more vectors.
 *
 * Return codes: LB_OK, LB_NOT_CONVERGED (outputs valid, details in info), or a
 * negative error; lb_last_error() returns a message for the last error of the
 * calling thread.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_NOT_CONVERGED 1
#define LB_ERR_ARG (-1)         /* null pointer, bad size, radius <= 0, ...  */
#define LB_ERR_HIP (-2)         /* HIP runtime error                        */
#define LB_ERR_MISMATCH (-3)    /* call does not fit the plan (batch, ...)  */
#define LB_ERR_NONFINITE (-4)   /* NaN or Inf met in a reduction            */
#define LB_ERR_UNSUPPORTED (-5) /* grid size or box the library has no kernels for */

/* Arithmetic of the FFT and pointwise stages of lb_hessvec and of the inner
 * subproblem iteration. Energies, gradients, norms, dot products, the
 * Lagrange-multiplier update and the trust-region ratio are always FP64. */
#define LB_FP64 0
#define LB_FP32 1

typedef struct lb_grid {
  int dim;        /* 2 or 3 */
  int n[3];       /* points per axis (n[2] unused when dim == 2) */
  double box[3];  /* box side per axis, > 0 */
} lb_grid;

typedef struct lb_params {
  double tau;   /* reduced temperature (eq. lb_energy) */
  double gamma; /* three-body coefficient (eq. lb_energy) */
  double xi;    /* interaction strength, 1 in the paper */
  double q;     /* critical wave number, 1 in the paper */
} lb_params;

/* Options of the subproblem solver (Algorithm 3). */
typedef struct lb_sub_opts {
  double eta;            /* IMEX step size eta (Section 4: 0.1) */
  double eps_sub;        /* stop when ||g + (H + lambda I) d|| < eps_sub (Section 4: 1e-13) */
  double eps_sub_rel;    /* ... or < eps_sub_rel * ||g|| (0 disables) */
  int max_inner;         /* cap on iterations of Algorithm 3 */
  int max_newton;        /* cap on Newton steps per iteration */
  double newton_rtol;    /* Newton stops when phi(lambda) - r^2 <= newton_rtol r^2 */
  double newton_steptol; /* ... or |delta lambda| <= newton_steptol max(1, lambda) */
  int poll_every;        /* iterations enqueued between host reads of the stop flag */
  int newton_phi;        /* root of phi(lambda) = r^2 (eq. lambda_update_rule) by Newton applied
                            to: 1 -> phi(lambda) - r^2 from lambda = 0, as printed;
                            0 (default) -> the equivalent 1/sqrt(phi) - 1/r from the previous
                            iteration's multiplier: concave, so it converges monotonically to
                            the same root in fewer steps */
  int newton_direct;     /* 1: every Newton evaluation sums phi over the whole spectrum, as
                            printed; 0 (default): from power sums of |b|^2 taken once per
                            iteration (a truncated series with a rigorous tail bound far below
                            rounding), falling back to the full sum when the bound fails */
  int single_workgroup;  /* 1 (default): on square 2D grids up to 64 x 64 one workgroup runs
                            every iteration in a single launch (same arithmetic); 0: one
                            launch sequence per iteration, as on every other grid */
  int graph;             /* 1: subproblems with max_inner >= 127 replay a captured HIP graph
                            of two iterations' launches on a private stream (same kernels,
                            same results); 0 (default, faster on the current runtime): direct
                            launches. Not used while kernel timing is on. */
  int fused_newton;      /* The multiplier step of each iteration (Newton on eq.
                            lambda_update_rule, and the stop test) in the next iteration's
                            first pass, where every workgroup sums all the update pass's
                            partials in the same order (one launch fewer per iteration, at
                            the price of those redundant reads); an iteration whose series
                            Newton needs sums over the spectrum falls back to the separate
                            launch. 1 (default): fused where the redundant reads stay below
                            16 MB per pass (grids up to about 96^3; not 128^3); 2: always;
                            0: always the separate one-workgroup launch. The results are the
                            same bits either way. Not used with newton_direct or graph. */
} lb_sub_opts;

typedef struct lb_sub_info {
  double lambda;      /* Lagrange multiplier of the returned d */
  double resid;       /* ||g + (H + lambda I) d|| of the returned d */
  double dnorm;       /* ||d|| */
  double gnorm;       /* ||g|| */
  int iters;          /* iterations of Algorithm 3 performed */
  int newton_iters;   /* Newton steps summed over the iterations */
  int newton_direct;  /* Newton evaluations that summed phi over the spectrum */
  int status;         /* LB_OK or LB_NOT_CONVERGED (cap reached) */
} lb_sub_info;

/* Options of the outer IMEX-TR loop (Algorithms 1 and 2). Defaults from
 * lb_tr_opts_default are the paper's Section 4 values plus the readings
 * documented with each field. */
typedef struct lb_tr_opts {
  double theta, gamma_c, gamma_e, gamma_lambda; /* 1e-4, 0.5, 2, 1.5 */
  double mu_lo, mu_hi, mu0, r0, nu0;            /* 1, 1e5, 1, 1, 5 */
  double eps;           /* gradient tolerance (1e-10 with grad_norm_inf) */
  int grad_norm_inf;    /* 1: ||g||_inf < eps (Algorithm 1); 0: ||g||_2 < eps */
  double eta;           /* IMEX step size (0.1) */
  int eta_safe;         /* 1: eta_j = min(eta, 0.9 / max|Gamma'(psi_j)|) so that the
                           descent lemma's bound holds; 0: fixed eta */
  int rho_taylor;       /* 1: E(v) - E(v+s) from the exact quartic expansion;
                           0: from two energy evaluations */
  int contract_else_old_step; /* CONTRACT else-branch radius: 0 -> gamma_C ||s|| with
                                 the new s (as printed), 1 -> gamma_C ||s_j|| */
  double nu_tol;        /* ||s_j|| = nu_j tested with relative tolerance nu_tol */
  int max_outer;
  lb_sub_opts sub;      /* subproblem options (eta is overwritten per iteration) */
  double cg_rtol;       /* CONTRACT: CG relative tolerance on (H + lambda I) s = -g */
  int cg_maxiter;
  int verbose;          /* 1: one line per outer iteration on stderr */
  /* Nearly hard subproblems (Remark on the hard case, Section 3.2; Section 4.3):
     with hard_case = 1, each outer iteration j estimates sigma_1 and its unit
     eigenvector xi by hard_lanczos_steps Lanczos steps (preconditioner shift
     hard_precond_shift, start lb_random_ball(1, seed, 2j + 1)); when sigma_1 < 0
     and |<xi, g>| <= hard_tol, Algorithm 3 starts from lb_random_ball(r_j, seed,
     2j) instead of -r g/||g||. */
  int hard_case;              /* 0 (default): always the deterministic start */
  double hard_tol;            /* 1e-12, the paper's threshold on |g^(1)| */
  int hard_lanczos_steps;     /* 30 */
  double hard_precond_shift;  /* 1.0 */
  unsigned long long seed;    /* key of the random draws (0) */
  double cg_precond_shift;    /* CONTRACT's CG (the paper leaves the solver open): c > 0 (default 1)
                                 preconditions (H + lambda~ I) by (Lambda + lambda~ + c)^-1, as in
                                 lb_shifted_solve; 0: plain CG */
  int capped_reject;          /* Algorithm 1 takes s_j from a subproblem that meets its optimality
                                 conditions; one stopped by max_inner does not. 0 (default): its
                                 step is still tested by the ratio (counted in sub_capped);
                                 1: it is rejected without a ratio test, the field stays and
                                 r_{j+1} = gamma_C r_j */
} lb_tr_opts;

typedef struct lb_tr_info {
  double energy;     /* E at the returned psi */
  double gnorm;      /* ||g||_2 at the returned psi */
  double gnorm_inf;  /* max_k |g_hat_k| at the returned psi */
  int outer;         /* outer iterations performed */
  int inner_total;   /* subproblem iterations summed */
  int cg_total;      /* CG iterations spent in CONTRACT */
  int accepted, contracted, expanded;
  int status;        /* LB_OK or LB_NOT_CONVERGED */
  int hard_cases;    /* subproblems started from a random point (hard_case = 1) */
  int newton_total;  /* Newton steps of the multiplier, summed over all subproblem iterations */
  int newton_direct; /* of their evaluations, those that summed phi over the spectrum */
  int sub_capped;    /* outer iterations whose subproblem stopped at sub.max_inner before its
                        stop test held; Algorithm 1 then takes that iterate as s_j although it
                        need not satisfy the optimality conditions (eq.
                        tr_subproblem_optimal_condition) */
} lb_tr_info;

typedef struct lb_plan lb_plan;

/* Library version (major * 10000 + minor * 100 + patch). */
int lb_version(void);

/* Message describing the last error returned on the calling thread. */
const char *lb_last_error(void);

/* Fill option structs with the defaults described above. */
void lb_sub_opts_default(lb_sub_opts *opts);
void lb_tr_opts_default(lb_tr_opts *opts);

/* Create a plan for `batch` instances of `grid` computing in `precision`
 * (LB_FP64 or LB_FP32) on `stream`. Allocates twiddle tables, |Bk|^2 tables
 * and every device workspace.
 * Errors: LB_ERR_ARG, LB_ERR_UNSUPPORTED (axis length), LB_ERR_HIP. */
int lb_plan_create(lb_plan **out, const lb_grid *grid, int batch, int precision, void *stream);
int lb_plan_destroy(lb_plan *plan);
int lb_plan_set_stream(lb_plan *plan, void *stream);

/* General Bravais lattice (Section 2: the grid T_M^d = {A (j / M)}, reciprocal
 * matrix B with A B^T = 2 pi I). A: dim x dim doubles (host), row major, whose
 * column a is the cell vector along grid axis a; grid point j is
 * x = sum_a A[:, a] j_a / n_a. The interaction multiplier becomes
 * Lambda_k = xi^2 (q^2 - |Bk|^2)^2 with |Bk|^2 = k^T B^T B k. A Nyquist index
 * (-n_a/2) and its conjugate partner carry different |Bk|^2 when B has
 * off-diagonal terms; both take their mean, so Lambda keeps real fields real.
 * A diagonal A is the orthorhombic box diag(A) (the same results as a plan
 * created with that box); A = NULL returns to the grid's box. Errors:
 * LB_ERR_ARG (non-finite or singular A). Applies to every later call on the
 * plan; lb_hessvec_noalloc takes orthorhombic boxes only. */
int lb_plan_set_lattice(lb_plan *plan, const double *A);
/* Device bytes held by the plan. */
size_t lb_plan_workspace_bytes(const lb_plan *plan);

/* Kernel timing, a measurement aid. When enabled, every kernel launch of the
 * plan whose name is listed in `filter` (comma-separated names; all launches
 * when filter is NULL or "") is bracketed by HIP events on the plan's stream;
 * durations accumulate per kernel name until timing is set again. Names
 * include rows_r2c, rows_c2r, rows_c2r_hv, rows_energy, rows_inner, col1_fwd,
 * col1_inv, col0_fwd, col0_inv, col0_fwd_mul_inv, col0_inv_scale_d,
 * plane_inner, col0_fwd_update, col0_fwd_hess, plane_fwd_phys,
 * plane_inv_phys, newton, sub2d, grad_assemble, spec_reduce, finalize,
 * lincomb, init_b, final_d, gamma_p, energy_out, add_real, axpy_real.
 * lb_plan_set_timing_sampled times only launches 0, every, 2 every, ... of
 * each listed kernel (every >= 1), an unbiased sample of the durations at a
 * fraction of the events' cost. */
int lb_plan_set_timing(lb_plan *plan, int enable, const char *filter);
int lb_plan_set_timing_sampled(lb_plan *plan, int enable, const char *filter, int every);
/* Entry `index` (0-based) of the accumulated timings: kernel name, launches
 * and total milliseconds. Synchronises the stream. LB_ERR_ARG past the end. */
int lb_plan_timing_entry(lb_plan *plan, int index, char *name, int name_len, long *count, double *total_ms);

/* Energy and projected gradient (Section 2: grad G = Lambda Psi_hat,
 * grad F = F_N Gamma F_N^{-1} Psi_hat; Section 3: projection P).
 *   params : `batch` entries (host)
 *   psi    : batch * N doubles (device, zero mean)
 *   energy : batch doubles (device), written
 *   grad   : batch * N doubles (device) or NULL; the physical form of the
 *            projected gradient g = P(F_N^{-1} Lambda psi_hat + F'(psi)),
 *            whose norm ||g|| is the paper's ||grad E_bar||.
 * Always FP64. Asynchronous. */
int lb_energy_grad(lb_plan *plan, const lb_params *params, const double *psi, double *energy, double *grad);

/* Hessian-vector product (Section 2: grad^2 G = Lambda, grad^2 F = F_N Gamma' F_N^{-1};
 * Section 3.2: H = D + T):
 *   hv = P( F_N^{-1} Lambda F_N v + Gamma'(psi) v ),  Gamma' = tau - gamma psi + psi^2/2.
 * The interaction part is applied after a forward FFT, the bulk part pointwise.
 *   psi, v : batch * N doubles (device); hv : batch * N doubles (device), written
 *   project: 1 removes the mean of hv (the operator on the zero-mean subspace);
 *            0 returns F_N^{-1} P Lambda F_N v + Gamma' v.
 * FFT arithmetic in the plan's precision. Asynchronous. */
int lb_hessvec(lb_plan *plan, const lb_params *params, const double *psi, const double *v, double *hv, int project);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * Hessian-vector product of lb_hessvec for one FP64 instance of `grid`
 * without a plan and without any allocation. Its workspace (twiddle tables,
 * the partial sums of the projection's mean, the half spectrum) is a fixed
 * 8 MiB device array of the library, one per GPU, held until the process
 * ends; grids whose half spectrum exceeds about 520 000 modes (for example
 * 128^3) are rejected with LB_ERR_ARG. Every call on a GPU shares that GPU's
 * array, so calls that overlap on one GPU (different streams, threads) race:
 * serialise them. The twiddle tables are regenerated on the device in each
 * call, so results agree with lb_hessvec to rounding, not bit for bit.
 *   grid    : host; params : host, one entry; psi, v, hv : N doubles (device)
 *   project : as for lb_hessvec; stream : hipStream_t (NULL: null stream)
 * Asynchronous. Errors: LB_ERR_ARG, LB_ERR_UNSUPPORTED, LB_ERR_HIP. */
int lb_hessvec_noalloc(const lb_grid *grid, const lb_params *params, const double *psi, const double *v, double *hv,
                       int project, void *stream);

/* Derivatives with respect to the N grid values (for automatic
 * differentiation frameworks), of E as printed in eq. lb_energy with the sum
 * over every k including k = 0 and no mass constraint (on zero-mean fields
 * this is the paper's E):
 *   lb_energy_grad_raw: energy (batch doubles, device) and
 *     grad[x] = dE/dpsi_x = (F_N^{-1} Lambda psi_hat + F'(psi))_x / N
 *     (batch * N doubles, device). Always FP64. Asynchronous.
 *   lb_hessvec_raw: hv = (F_N^{-1} Lambda F_N v + Gamma'(psi) v) / N, the
 *     Hessian of E in these coordinates times v. FFT arithmetic in the plan's
 *     precision. Asynchronous.
 * Arguments as for lb_energy_grad / lb_hessvec; psi need not have zero mean. */
int lb_energy_grad_raw(lb_plan *plan, const lb_params *params, const double *psi, double *energy, double *grad);
int lb_hessvec_raw(lb_plan *plan, const lb_params *params, const double *psi, const double *v, double *hv);

/* Field moments per instance, the parameter derivatives of E (eq. lb_energy:
 * dE/dtau = mean(psi^2)/2, dE/dgamma = -mean(psi^3)/6) and of its gradient:
 *   out[4 b + 0] = mean(psi^2), out[4 b + 1] = mean(psi^3),
 *   out[4 b + 2] = mean(w psi), out[4 b + 3] = mean(w psi^2)  (0 if w is NULL)
 *   psi, w : batch * N doubles (device; w nullable); out : 4 * batch doubles
 *   (device), written. FP64. Asynchronous. */
int lb_field_moments(lb_plan *plan, const double *psi, const double *w, double *out);

/* Parameter derivatives of E (eq. lb_energy), per instance b:
 *   out[4 b + 0] = dE/dtau   = mean(psi^2) / 2
 *   out[4 b + 1] = dE/dgamma = -mean(psi^3) / 6
 *   out[4 b + 2] = d<w, grad_raw E>/dtau   = mean(w psi)
 *   out[4 b + 3] = d<w, grad_raw E>/dgamma = -mean(w psi^2) / 2
 * with grad_raw E the gradient with respect to the N grid values
 * (lb_energy_grad_raw) and <w, .> the plain sum over grid points; entries 2
 * and 3 are 0 when w is NULL.
 *   psi, w : batch * N doubles (device; w nullable); out : 4 * batch doubles
 *   (device), written. FP64. Asynchronous. */
int lb_param_grad(lb_plan *plan, const double *psi, const double *w, double *out);

/* Gradient with respect to the N grid values of
 * ct[2 b] dE/dtau + ct[2 b + 1] dE/dgamma (eq. lb_energy), per instance b:
 *   out[x] = (ct[2 b] psi_x - ct[2 b + 1] psi_x^2 / 2) / N.
 *   psi : batch * N doubles (device); ct : 2 * batch doubles (device);
 *   out : batch * N doubles (device), written. FP64. Asynchronous. */
int lb_param_grad_vjp(lb_plan *plan, const double *psi, const double *ct, double *out);

/* Trust-region subproblem min_{||d|| <= radius} <g,d> + <d,Hd>/2 by the
 * adaptive IMEX iteration (Section 3.2, Algorithm 3; eqs. imex-scheme and
 * lambda_update_rule), batch must be 1.
 *   psi   : N doubles (device); grad : N doubles (device), the projected
 *           gradient g (as written by lb_energy_grad), nonzero
 *   d0    : N doubles (device) initial feasible point, or NULL for the
 *           paper's d_0 = -radius g / ||g||
 *   d_out : N doubles (device), the step d (zero mean)
 *   info  : host, filled on return (the call synchronises the stream)
 * Returns LB_OK, LB_NOT_CONVERGED (max_inner reached, d_out valid) or an error. */
int lb_tr_subproblem(lb_plan *plan, const lb_params *params, const double *psi, const double *grad, double radius,
                     const lb_sub_opts *opts, const double *d0, double *d_out, lb_sub_info *info);

/* Full IMEX-TR solve (Section 3.1, Algorithms 1 and 2 around Algorithm 3),
 * batch must be 1. psi (device, N doubles, zero mean) is overwritten with
 * the final iterate. info is filled on return. */
int lb_imex_tr_solve(lb_plan *plan, const lb_params *params, double *psi, const lb_tr_opts *opts, lb_tr_info *info);

/* CONTRACT's linear system (Algorithm 2): conjugate gradients for
 * (H + shift I) s = -g on the zero-mean subspace (H + shift I must be
 * positive definite), stopped when ||r|| <= rtol ||g|| or after maxiter steps.
 * precond_shift = c > 0: preconditioned by the diagonal (Lambda_k + shift + c)^-1
 * in Fourier space (same system, far fewer steps on stiff spectra); 0: plain
 * CG; negative or non-finite: LB_ERR_ARG. grad, s_out: N doubles (device).
 * batch must be 1. *iters receives the CG iteration count. */
int lb_shifted_solve(lb_plan *plan, const lb_params *params, const double *psi, const double *grad, double shift,
                     double rtol, int maxiter, double precond_shift, double *s_out, int *iters);

/* Second-order check (the paper's SP-II test, Section 1 definition: grad = 0
 * and H >= 0): an estimate of sigma_1, the smallest eigenvalue of H on the
 * zero-mean subspace, by `steps` Lanczos steps with full reorthogonalisation
 * from v0 (device, N doubles).
 *   precond_shift <= 0: Lanczos on H; *ritz_min is its smallest Ritz value and
 *     *resid the Ritz residual norm.
 *   precond_shift = c > 0: Lanczos on K = S H S with S = (Lambda_k + c)^(-1/2)
 *     diagonal in Fourier space. K is congruent to H (same inertia) with a
 *     clustered spectrum, so its lowest Ritz vector y converges in few steps;
 *     *ritz_min is the Rayleigh quotient of H at x = S y and *resid is
 *     ||Hx - ritz x|| / ||x||.
 * Either value bounds sigma_1 from above. batch must be 1. Host outputs;
 * evec (device, N doubles, nullable) receives the unit Ritz vector (y, or
 * x / ||x|| with preconditioning), mean zero.
 * Allocates steps + 1 spectral vectors on first use (kept by the plan). */
int lb_lanczos_min(lb_plan *plan, const lb_params *params, const double *psi, const double *v0, int steps,
                   double precond_shift, double *ritz_min, double *resid, double *evec);

/* A random feasible initial point for nearly hard subproblems (Remark on the
 * hard case, Section 3.2: a continuous distribution supported on the ball
 * ||s|| <= r): d uniformly distributed in the ball of radius `radius` of the
 * (N-1)-dimensional zero-mean subspace (||.|| = RMS). z_x is standard normal
 * by the Box-Muller transform of the two first words of Philox4x64-10 (Salmon
 * et al., SC'11) at counter (x, 0, 0, 0) and key (seed, draw) (x the C-order
 * index, words mapped to (0, 1) by ((w >> 11) + 1/2) 2^-53); d = radius
 * u^(1/(N-1)) (z - mean z) / rms(z - mean z) with u from word 0 at counter
 * (0, 1, 0, 0). d_out: N doubles (device), written; batch must be 1.
 * Asynchronous. */
int lb_random_ball(lb_plan *plan, double radius, unsigned long long seed, unsigned long long draw, double *d_out);

/* IMEX-TR solves of the plan's `batch` instances together (Algorithms 1-3 for
 * each): every pass of the subproblem iteration and of the outer loop is one
 * launch for all instances still iterating, with per-instance multipliers,
 * stop flags, radii and branches; an instance leaves the launches when its
 * gradient test holds. Each instance's result equals its lb_imex_tr_solve on
 * a plan of batch 1, bit for bit.
 *   params : batch entries (host); psi : batch * N doubles (device, zero-mean
 *   fields, updated); infos, status : batch entries (host, written; status is
 *   LB_OK, LB_NOT_CONVERGED or a negative error per instance).
 * Nearly hard starts (hard_case) and the direct ratio numerator (rho_taylor = 0)
 * need batch 1 (LB_ERR_UNSUPPORTED otherwise). Returns LB_OK, or the first
 * instance's error. Synchronises the stream. */
int lb_imex_tr_solve_batch(lb_plan *plan, const lb_params *params, double *psi, const lb_tr_opts *opts,
                           lb_tr_info *infos, int *status);

/* `count` independent jobs run concurrently, e.g. a sweep of instances of
 * different grid sizes and parameters: a pool of `workers` host threads, each
 * with its own HIP stream, takes the jobs largest first. Job i solves the
 * plans[i]->batch instances of plans[i] (distinct plans) as
 * lb_imex_tr_solve_batch does, with the fields psi[i] (device,
 * batch_i * N_i doubles, updated). params, infos and status (host) hold one
 * entry per instance, job after job (job i's first instance at
 * sum_{k<i} batch_k). opts (nullable: defaults) apply to all. Each job starts
 * after the work already enqueued on its plan's stream, and later work on that
 * stream sees its result. Returns LB_OK when no instance failed, else the first
 * failure's code (its message in lb_last_error). Blocks until all jobs are done. */
int lb_imex_tr_solve_many(lb_plan *const *plans, const lb_params *params, double *const *psi, int count,
                          const lb_tr_opts *opts, int workers, lb_tr_info *infos, int *status);

/* Autotuner: on grids whose inner iteration has a plane pass or a split
 * order (3D with n1 = n2), time the inner iteration's passes (Section 3.2:
 * the scaled inverse, the product with Gamma', the forward update) in each
 * built variant: one workgroup per plane with 256, 512 or 1024 threads (or
 * the five passes where the plane does not fit in LDS), or the
 * split order with 2 or 4 parts (lb_plan_set_plane_split) with each built
 * thread count of its split-plane pass, each with every built radix plan of
 * the axis-0 passes
 * (lb_plan_set_column_plan), `reps` iterations each on the plan's own buffers
 * (Gamma' from psi) in two interleaved rounds (each candidate keeps its faster
 * round), and use the fastest from then on; the built-in variant stays unless
 * another is more than 2 % faster. *threads receives the
 * chosen plane stage's thread count (0 when the plan has nothing to tune;
 * lb_plan_get_variant tells the whole choice). Synchronises the stream;
 * overwrites workspaces only. */
int lb_plan_autotune(lb_plan *plan, const lb_params *params, const double *psi, int reps, int *threads);

/* Pins the plane-pass variant the autotuner would choose: threads = 256, 512
 * or 1024, or 0 for the built-in choice (1024 from n1 = 96, else 512). Only
 * the plans lb_plan_autotune can tune (3D, n1 = n2 >= 64) accept a nonzero
 * value (LB_ERR_UNSUPPORTED otherwise; LB_ERR_ARG for any other count). The
 * variants differ only in how many threads share a plane; their results agree
 * to rounding, and each variant is deterministic. */
int lb_plan_set_plane_threads(lb_plan *plan, int threads);

/* Order of the inner iteration on 3D grids with n1 = n2 (the product T d of
 * Section 3.2 by pointwise products and FFTs). split = 1 or 2 splits the
 * axis-1 transform by x1 mod K with K = 2 or 4 parts: the axis-0 inverse pass
 * does its first K-point step across the column groups (k1 + q n1/K), the
 * forward update pass its last, and a split-plane pass with K workgroups per
 * plane, each holding 1/K of the plane in LDS, does the rest (twice or four
 * times the workgroups of the plane pass; with 4 parts a 256^3 grid keeps
 * three passes instead of the five of the column and row kernels).
 * split = 0 runs one workgroup per plane where the plane fits in LDS, else
 * the five passes. threads = 256, 512 or 1024 pins the (split-)plane pass's
 * thread count where that variant is built, 0 keeps the built-in one.
 * Without a call the plan takes the built-in order: one workgroup per plane
 * where the plane fits, else the five passes (measured faster at 256^3 than
 * the four-part order, whose axis-0 passes move 4-column runs). LB_ERR_UNSUPPORTED when the grid
 * has no such order (the (n1/K)(n2/2 + 1) columns of a part must fill whole
 * column-workgroup shares; four parts need 16 columns per workgroup);
 * LB_ERR_ARG for other values. All orders compute the same iteration: results
 * agree to rounding, and each is deterministic. The Hessian products of
 * CONTRACT and Lanczos keep one workgroup per plane (or the five passes). */
int lb_plan_set_plane_split(lb_plan *plan, int split, int threads);

/* Order of lb_hessvec and lb_hessvec_raw (see lb_plan_set_plane_split):
 * split = 1 or 2 runs the three passes of the product in the split order
 * with 2 or 4 parts (K split-plane workgroups per plane, the axis-1 K-point
 * steps in the axis-0 pass); 0 one workgroup per plane, or the five passes
 * where the plane does not fit; -1 the built-in choice (2 parts for FP64
 * planes of 96 points and more that fit in LDS, else none; where the plane
 * does not fit, 4 parts in FP32 and the five passes in FP64). lb_hessvec_noalloc always takes the
 * built-in choice. LB_ERR_UNSUPPORTED when the grid has no such order. All
 * orders compute the same product; results agree to rounding. */
int lb_plan_set_hessvec_split(lb_plan *plan, int split);

/* Plan of the inner iteration's two axis-0 passes: 0, radix 8 first (the
 * built-in plan); 1, radix 4 first (more threads per transform, one pass
 * more at length 128); 2, radix 16 first (fewer threads, one pass fewer),
 * with the same columns per workgroup; 3, radix 8 first with twice the
 * columns per workgroup (longer contiguous runs per row in the split order,
 * half the workgroups and partial sums; one or two parts only: with four,
 * or where a part's columns do not fill its workgroups, the passes run plan
 * 0). Plans 1 to 3 exist for axis-0 lengths 64 to 256 (LB_ERR_UNSUPPORTED
 * otherwise; LB_ERR_ARG for other values). The plans compute the same
 * transforms: results agree to rounding, and each is deterministic. */
int lb_plan_set_column_plan(lb_plan *plan, int column_plan);

/* The inner iteration's variant in use: *split = 0, 1 or 2 (no split, 2 or
 * 4 parts), *threads the plane or split-plane pass's thread count (0 when the
 * inner iteration runs the five passes), *column_plan the axis-0 passes'
 * plan (as they run it: 0 where plan 3 does not apply). */
int lb_plan_get_variant(lb_plan *plan, int *split, int *threads, int *column_plan);

#ifdef __cplusplus
}
#endif
#endif /* LB_H */
