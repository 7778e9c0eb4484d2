/*
 * automat.h -- C ABI of libautomat, an MI355X (gfx950) FP64 evaluator for
 * generalized standard materials (GSM) by one implicit-Euler step per
 * material point.
 *
 * The method (AutoMat paper):
 *  - a GSM is given by a free energy omega(eps, a) and a force potential
 *    Psi(A); sigma = d omega / d eps and a' = dPsi/dA (-d omega / d a)
 *    (Section "Generalized Standard Materials", equations gsm_sigma and
 *    gsm_internal);
 *  - one material-law evaluation takes eps_{n+1} and a_n and returns
 *    a_{n+1}, sigma_{n+1} and optionally the consistent tangent
 *    C_{n+1} = d sigma_{n+1} / d eps_{n+1} (same section, the evaluation
 *    contract). Implicit Euler evaluates the rate at t_{n+1} only, so eps_n
 *    is not an input;
 *  - the step a_{n+1} = a_n + h f(eps_{n+1}, a_{n+1}) is solved by Newton
 *    with gradients and Hessians of omega and Psi from automatic
 *    differentiation, and the tangent follows from the implicit function
 *    theorem with the Newton matrix at the converged point (Section
 *    "Single Implicit Euler Step", equations implicit_euler and
 *    tangent_formula);
 *  - the material family is the Michel-Suquet elasto-viscoplastic GSM
 *    (Section "Example", equations michel_suquet_omega and
 *    michel_suquet_psi): kind 1; kind 0 is its purely elastic special case
 *    (Psi = 0).
 *
 * Conventions for every entry point:
 *  - all floating point is IEEE double (FP64); units are the caller's
 *    (the presets use MPa and s);
 *  - strains and internal variables are 6-vectors in engineering-shear Voigt
 *    order (11, 22, 33, 23, 13, 12); stresses are plain Voigt in the same
 *    order;
 *  - fields are device pointers in structure-of-arrays, component-major
 *    layout with leading dimension n: component c of point i is at
 *    ptr[c * n + i]. A tangent field holds 36 components, row-major 6x6 per
 *    point: entry (r, c) of point i is at ptr[(6 * r + c) * n + i];
 *  - phase ids are uint8 per point, indexing automat_params.phase;
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are asynchronous and stream-ordered; the library keeps no pointer
 *    after it returns;
 *  - the caller owns all memory. Output arrays must not alias inputs, except
 *    that a_out may equal a_old (in-place update);
 *  - return value 0 on success, a negative AUTOMAT_E* code otherwise; an
 *    error return launches nothing.
 */
#ifndef AUTOMAT_H
#define AUTOMAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AUTOMAT_MAX_PHASES 16
/* Differentiable material parameters, in this order:
 * E, nu, H, sigma_y, sigma0, eps0, n. */
#define AUTOMAT_NPAR 7

#define AUTOMAT_OK 0
#define AUTOMAT_EINVAL (-1)  /* bad pointer, size, scalar or parameter */
#define AUTOMAT_EHIP (-2)    /* HIP runtime or launch error */
#define AUTOMAT_ENOMEM (-3)  /* device or host allocation failed */
#define AUTOMAT_EBUDGET (-4) /* serving request larger than the memory budget */

/* Flags of automat_evaluate_ex. */
#define AUTOMAT_SIGMA_CRITERION 1u /* stop Newton on ||C F||_inf <= tol ||sigma||_inf,
                                      i.e. converge the stress (Section "Stress-Driven
                                      Error Control", last paragraph) */
#define AUTOMAT_HAND_PARTIALS 2u   /* semi-automatic strategy: the same Newton solve and
                                      tangent with hand-derived partials of omega and Psi
                                      instead of automatic differentiation (Section
                                      "Example", comparison of evaluation strategies) */

/* One material phase (Section "Example", Table misu_parameters names the
 * same quantities).
 *  kind     0 = elastic (Psi = 0), 1 = Michel-Suquet elasto-viscoplastic
 *  E, nu    Young's modulus (> 0) and Poisson's ratio (-1 < nu < 0.5)
 *  H        linear kinematic hardening modulus (>= 0)
 *  sigma_y  initial yield stress (>= 0)
 *  sigma0   drag stress sigma_d (> 0)
 *  eps0     reference strain rate (>= 0)
 *  n        rate sensitivity (>= 1)
 * For kind 0 only E and nu are read and checked. */
typedef struct automat_phase {
    int32_t kind;
    int32_t reserved;
    double E, nu, H, sigma_y, sigma0, eps0, n;
} automat_phase;

/* Host struct, read during the call and copied into the launch. */
typedef struct automat_params {
    int32_t n_phases; /* 1 .. AUTOMAT_MAX_PHASES */
    int32_t reserved;
    automat_phase phase[AUTOMAT_MAX_PHASES];
} automat_params;

/* One implicit-Euler material-law evaluation of n points.
 *
 *  eps_new     [6][n] strain at t_{n+1}                               (in)
 *  a_old       [6][n] internal variables a_n (viscoplastic strain)    (in)
 *  phase       [n]    phase id per point                              (in)
 *  params      host   phase table                                     (in)
 *  h           step length t_{n+1} - t_n, finite and > 0
 *  tol         Newton tolerance (> 0): converged when
 *              ||F||_inf <= max(tol ||a_{n+1} - a_n||_inf,
 *                               2^-48 ||eps_new - a_old||_inf)
 *              (F the implicit-Euler residual; the second term is the
 *              rounding level of the trial elastic strain, reached by flows
 *              just above the yield stress), or when F vanishes exactly
 *  max_iter    maximum number of Newton updates (>= 1)
 *  sigma_out   [6][n] stress sigma_{n+1}                              (out)
 *  a_out       [6][n] a_{n+1}, may equal a_old; NULL skips the write  (out)
 *  tangent_out [36][n] consistent tangent, NULL skips it              (out)
 *
 * Per-point failures do not fail the call: a point that does not converge
 * keeps its last Newton iterate; a point with non-finite input or a phase id
 * >= n_phases gets NaN outputs. Use automat_evaluate_ex to see them.
 * n = 0 is a no-op returning 0. Errors: AUTOMAT_EINVAL (NULL required
 * pointer, n < 0, h or tol not finite and > 0, max_iter < 1, invalid
 * params), AUTOMAT_EHIP. */
int32_t automat_evaluate(int64_t n, const double *eps_new, const double *a_old,
                         const uint8_t *phase, const automat_params *params, double h,
                         double tol, int32_t max_iter, double *sigma_out, double *a_out,
                         double *tangent_out, void *stream);

/* As automat_evaluate, plus
 *  iters_out    [n] device int32, number of Newton updates per point, -1 if not
 *               converged or invalid input; NULL skips it             (out)
 *  nonconverged device uint64 counter, incremented once per point with
 *               iters = -1 (not reset by the call); NULL skips it     (inout)
 *  flags        0, or AUTOMAT_SIGMA_CRITERION and/or AUTOMAT_HAND_PARTIALS */
int32_t automat_evaluate_ex(int64_t n, const double *eps_new, const double *a_old,
                            const uint8_t *phase, const automat_params *params, double h,
                            double tol, int32_t max_iter, double *sigma_out, double *a_out,
                            double *tangent_out, int32_t *iters_out, uint64_t *nonconverged,
                            uint32_t flags, void *stream);

/* Vector-Jacobian product of one evaluation at its converged state
 * (implicit function theorem through the Newton system of Section "Single
 * Implicit Euler Step"; the step length carries no derivative and the
 * equation solve is treated as one elementary operation, as in Theorem
 * ad_integration_step).
 *
 *  eps_new, a_old, phase, params, h   as passed to automat_evaluate  (in)
 *  a_new       [6][n] a_{n+1} returned by the forward call            (in)
 *  grad_sigma  [6][n] cotangent of sigma_{n+1}; NULL = zero           (in)
 *  grad_a      [6][n] cotangent of a_{n+1}; NULL = zero               (in)
 *  grad_eps    [6][n] cotangent of eps_{n+1}                          (out)
 *  grad_a_old  [6][n] cotangent of a_n; NULL skips it                 (out)
 *  grad_params [n_phases][AUTOMAT_NPAR] device array, ACCUMULATED (+=)
 *              over points, in the order E, nu, H, sigma_y, sigma0,
 *              eps0, n; NULL skips it                               (inout)
 * Points with a phase id >= n_phases get NaN cotangents and add nothing.
 * Errors as automat_evaluate. */
int32_t automat_evaluate_backward(int64_t n, const double *eps_new, const double *a_old,
                                  const double *a_new, const uint8_t *phase,
                                  const automat_params *params, double h,
                                  const double *grad_sigma, const double *grad_a,
                                  double *grad_eps, double *grad_a_old, double *grad_params,
                                  void *stream);

/* ------------------------------------------------------------------------
 * Moulinec-Suquet basic scheme (FFT-based homogenization around the
 * material-point evaluation; the paper's Section "Example", paragraph
 * "Material Law Evaluations": each fixed-point iteration makes one material
 * sweep without tangent). Periodic grid nx * ny * nz, x fastest (point
 * i = x + nx (y + ny z)); strain-controlled macroscopic load; isotropic
 * reference medium C0 = (lambda0, mu0); Green operator
 * Gamma0(xi) = [d_ki q_h q_j + d_hi q_k q_j + d_kj q_h q_i + d_hj q_k q_i]/(4 mu0)
 *              - (lambda0 + mu0)/(mu0 (lambda0 + 2 mu0)) q_i q_j q_k q_h,
 * q = xi/|xi|, at every non-zero frequency except where a Nyquist index
 * N/2 of an even dimension meets another non-zero component (+N/2 and -N/2
 * are one index there but different directions): there Gamma0 = C0^-1, so
 * the converged stress has no content at those frequencies and the
 * converged fields do not depend on C0. The zero frequency carries the
 * macroscopic strain. Mixed boundary conditions (the paper's Section
 * "Example", paragraph "Boundary Conditions": a uniaxial
 * tension-compression test) prescribe the mean stress on a chosen set of
 * components and the mean strain on the rest; the reference stiffness is
 * fixed or adjusted to the tangent field at the start of every load step
 * (paragraph "Material Law Evaluations").
 * ------------------------------------------------------------------------ */
typedef struct automat_ms automat_ms; /* opaque; owns its FFT plans and work buffers */

typedef struct automat_ms_options {
    double tol;              /* stop when ||eps' - eps||_2 / ||E|| <= tol (tensor norms,
                                voxel-averaged L2); > 0 unless fixed_iter */
    int32_t max_iter;        /* maximum fixed-point iterations per load step, >= 1 */
    int32_t fixed_iter;      /* nonzero: run exactly max_iter iterations, no test */
    double lambda0, mu0;     /* reference medium; <= 0 selects the means of the smallest
                                and largest Lame constants of the phases */
    double newton_tol;       /* per-point Newton tolerance, > 0 */
    int32_t newton_max_iter; /* per-point Newton update limit, >= 1 */
    int32_t ref_update;      /* 1: at the start of every load step, after the initial
                                guess, one sweep with tangent sets C0 to the means of
                                the smallest and largest Lame constants of the isotropic
                                parts of the tangents (lambda = K - 2 mu / 3 with
                                3K = sum of the normal block / 3 and
                                10 mu = C11 + C22 + C33 + 2 (C44 + C55 + C66) - 3K);
                                the reference then stays in use until the next update
                                (automat_ms_reference reports it). 0: fixed. Needs
                                36 more doubles per voxel (allocated on the first step) */
    int32_t warm_start;      /* 1: each sweep's per-point Newton solves start from the
                                increments of the previous sweep (the last step's for a
                                step's first sweep; a start without flow is replaced by
                                the elastic trial state), which saves Newton updates for
                                strongly nonlinear laws at 96 bytes per voxel and sweep
                                of extra traffic; 0: every solve starts from the elastic
                                trial state */
    int32_t reserved;        /* must be 0 */
} automat_ms_options;

/* Create a solver for an nx * ny * nz grid (each >= 2). params and opts are
 * copied. Allocates about 9.4 doubles per voxel of device memory on the
 * current device. Errors: AUTOMAT_EINVAL, AUTOMAT_ENOMEM. */
int32_t automat_ms_create(int32_t nx, int32_t ny, int32_t nz, const automat_params *params,
                          const automat_ms_options *opts, automat_ms **out);

/* One load step to the macroscopic strain E_macro[6] (host, engineering
 * Voigt) with step length h. eps [6][n] (device, in/out) holds the strain
 * field of the previous step on entry (zeros before the first step) and is
 * shifted by E_macro - E_previous as the initial guess; on return it is the
 * converged field. a [6][n] (device, in/out): a_n on entry, a_{n+1} on
 * return (committed by a final sweep at the converged strain). sigma_out
 * [6][n] (device) receives that sweep's stress, or NULL. sigma_mean[6]
 * (host) its voxel average, or NULL. iters (host): fixed-point iterations
 * used; residual (host): the last ||eps' - eps||_2 / ||E||. Synchronizes
 * the stream once per iteration (convergence test) unless fixed_iter. */
int32_t automat_ms_step(automat_ms *ms, const uint8_t *phase, const double *E_macro, double h,
                        double *eps, double *a, double *sigma_out, double *sigma_mean,
                        int32_t *iters, double *residual, void *stream);

/* automat_ms_step for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid
 * allocation): the step's work space (the polarization field, its half
 * spectrum, the reduction partials and scalars, the failed-solve counter)
 * lives in a 64 MiB device array of the library, one per device, held
 * until the process ends, instead of the handle's buffers; the call makes
 * no allocation (the handle, with its transform plans, is created
 * beforehand). Same arguments, results and synchronization as
 * automat_ms_step. AUTOMAT_EINVAL if the work space does not fit in 64 MiB
 * (6 n doubles + 6 (nx/2 + 1) ny nz complex doubles + 50 KiB, i.e. grids up
 * to about 86^3 voxels) or if the handle adjusts its reference every step
 * (ref_update: that sweep needs a tangent field). Every call on one device
 * shares the array: calls that overlap on one device (other streams, other
 * threads) race. */
int32_t automat_ms_step_noalloc(automat_ms *ms, const uint8_t *phase, const double *E_macro,
                                double h, double *eps, double *a, double *sigma_out,
                                double *sigma_mean, int32_t *iters, double *residual,
                                void *stream);

/* One load step under mixed boundary conditions. Bit c of stress_mask
 * (0 <= stress_mask < 64, components in engineering Voigt order 11 22 33 23
 * 13 12) selects a stress-controlled component, whose mean stress is
 * S_macro[c] (host [6], or NULL for zero targets); the other components
 * have the mean strain E_macro[c] (host [6]; stress-controlled entries are
 * ignored). Every update sets the zero frequency to the macroscopic strain
 * E that solves mean(tau) + C0 E = S_macro on the stress-controlled set
 * (closed form for the isotropic C0), so at convergence the mean stress
 * meets the targets. The initial guess shifts the previous field by the
 * prescribed strain increments and, on stress-controlled components, by
 * the increments that keep the reference medium's stress there unchanged.
 * E_reached (host [6], or NULL) receives the macroscopic strain of the last
 * update, and the next step starts from it. The convergence test divides by
 * the norm of that strain. Other arguments, synchronization and errors as
 * automat_ms_step (AUTOMAT_EINVAL also for an adjusted reference that is
 * not positive definite). The reverse step (automat_ms_adjoint_step)
 * covers strain-controlled steps only. */
int32_t automat_ms_step_mixed(automat_ms *ms, const uint8_t *phase, const double *E_macro,
                              const double *S_macro, uint32_t stress_mask, double h, double *eps,
                              double *a, double *sigma_out, double *sigma_mean, double *E_reached,
                              int32_t *iters, double *residual, void *stream);

/* Set the macroscopic strain the next step starts from (e.g. after loading
 * a checkpointed strain field). */
int32_t automat_ms_set_macro(automat_ms *ms, const double *E_previous);

/* Point solves of the last completed load step (all its sweeps, the
 * reference and commit sweeps included) that did not converge within
 * newton_max_iter updates; their results are the last iterates. */
int32_t automat_ms_newton_failures(const automat_ms *ms, uint64_t *count);

/* The reference medium in use. */
int32_t automat_ms_reference(const automat_ms *ms, double *lambda0, double *mu0);

/* Reverse step: vector-Jacobian product of one converged load step. The
 * paper obtains tangents by the implicit function theorem applied to the
 * converged Newton system (section "Implicit Euler", consistent tangent);
 * here the same theorem is applied one level up, to the converged fixed
 * point eps = E - Gamma0 (sigma(eps) - C0 eps) of the basic scheme. For the
 * functional
 *   L = w . mean(sigma_k) + sum_x grad_sigma(x) . sigma_k(x)
 *       + sum_x grad_a(x) . a_k(x)
 * of the step's stress and internal variables, the adjoint field lam solves
 *   lam = b - (C - C0) Gamma0 lam,   b = direct strain cotangent of L,
 * with C the consistent tangent field at the converged strain (the same
 * fixed-point iteration as the forward scheme, in transposed form). Then
 * dL/dE_k = sum_x lam(x), and the cotangent g + w/n - Gamma0 lam of the
 * stress, taken through the point-level vector-Jacobian product, gives
 * dL/da_{k-1} and dL/dp.
 *   eps    device [6][n]: the step's converged strain (as left by
 *          automat_ms_step); a_prev, a_next: internal variables before and
 *          after the step (device [6][n]).
 *   w      host [6] or NULL; grad_sigma, grad_a: device [6][n] or NULL
 *          (zero).
 *   grad_E       host [6], out: dL/dE_k.
 *   grad_a_prev  device [6][n] or NULL, out: dL/da_{k-1}; must not alias
 *                an input.
 *   grad_params  device [n_phases][AUTOMAT_NPAR] or NULL, accumulated:
 *                dL/dp.
 *   iters, residual: adjoint iterations and the last relative change
 *   ||lam' - lam||_2 / ||b||_2; the iteration stops at opts.tol (or runs
 *   opts.max_iter times with fixed_iter). Work space (54 doubles per
 *   point) is allocated on the first call. Synchronizes the stream. */
int32_t automat_ms_adjoint_step(automat_ms *ms, const uint8_t *phase, double h,
                                const double *eps, const double *a_prev, const double *a_next,
                                const double *w, const double *grad_sigma, const double *grad_a,
                                double *grad_E, double *grad_a_prev, double *grad_params,
                                int32_t *iters, double *residual, void *stream);

int32_t automat_ms_destroy(automat_ms *ms);

/* ------------------------------------------------------------------------
 * Continuous-batching service (the paper's chunked evaluation with streams
 * that overlap transfers and computation, section "Computational Layout,
 * Profiling and Performance Limiters", recast for device-resident state).
 * Requests of uneven sizes, each with several load steps and its own phase
 * table, are admitted in arrival order while their device block (97 bytes
 * per point plus the phase tables) fits in the server's arena, one device
 * allocation of the whole budget made at creation. Every batch is one
 * kernel over the next load step of admitted requests (the least remaining
 * work first, up to the point cap); the next batch is queued behind the
 * running one; requests that arrive meanwhile are admitted by a second host
 * thread, uploaded on a second stream while the kernels run, and join a
 * later batch. Internal variables stay on the device between steps. The strain of step j of K at point i is (j / K) E_final +
 * noise_std z, z standard normal from Philox4x32-10 (Salmon et al. 2011)
 * keyed by seed with counter (i, j, w) and the Box-Muller transform.
 * Results do not depend on the rest of the batch beyond rounding (flowing
 * points are packed into full waves, and a wave decides together whether a
 * trial point is evaluated to first order; measured differences stay below
 * 1e-12 relative).
 * ------------------------------------------------------------------------ */
typedef struct automat_server automat_server; /* opaque; owns a scheduler thread, an
                                                 admission thread, three streams and
                                                 the arena */

typedef struct automat_request {
    int64_t n;             /* points, >= 1 */
    const uint8_t *phase;  /* host [n] phase ids; must stay valid until the result arrives */
    automat_params params; /* phase table of this request */
    double h;              /* step length, > 0 */
    double tol;            /* Newton tolerance, > 0 */
    int32_t max_iter;      /* Newton update limit, >= 1 */
    int32_t steps;         /* load steps K, >= 1 */
    double E_final[6];     /* macro strain at step K (engineering Voigt) */
    double noise_std;      /* standard deviation of the per-point strain noise, >= 0 */
    uint64_t seed;         /* generator key */
    const double *a_init;  /* host [6][n] initial internal variables, or NULL for zero */
    double *sigma_host;    /* host [6][n] stress after the last step, or NULL */
    double *a_host;        /* host [6][n] internal variables after the last step, or NULL */
    double t_arrival;      /* arrival time on the server clock (latency origin); < 0: at submit */
} automat_request;

typedef struct automat_result {
    uint64_t id;
    int32_t status;        /* AUTOMAT_OK, AUTOMAT_ENOMEM, AUTOMAT_EHIP; AUTOMAT_EINVAL if cancelled */
    int32_t steps_done;
    int64_t n;
    int64_t nonconverged;  /* point-steps that did not converge */
    double t_arrival, t_admit, t_done; /* server clock, seconds */
} automat_result;

typedef struct automat_server_stats_t {
    double clock_s;        /* server clock now */
    int64_t pending, active, used_bytes, launches, updates;
    double busy_s;         /* time spent in batch launches */
} automat_server_stats_t;

/* Start a server on the current device. hbm_budget_bytes (>= 4096) is
 * allocated at once as the arena that holds every admitted request;
 * max_batch_points (0 = unbounded) bounds the points of one launch (at least
 * one request is always taken; requests with the least remaining work, points
 * times load steps left, go first, and one left out of 16 consecutive
 * launches goes before all others; while the next queued request waits for
 * arena space a launch may take four times as many points, since the device
 * is saturated then); sequential != 0 admits one request at a
 * time (the per-request baseline). Errors: AUTOMAT_EINVAL, AUTOMAT_ENOMEM
 * (the budget cannot be allocated), AUTOMAT_EHIP. */
int32_t automat_server_create(size_t hbm_budget_bytes, int64_t max_batch_points,
                              int32_t sequential, automat_server **out);

/* Queue a request (copied; the host arrays it points to must stay valid until
 * its result is polled). Errors: AUTOMAT_EINVAL, AUTOMAT_EBUDGET (larger than
 * the whole budget). */
int32_t automat_server_submit(automat_server *server, const automat_request *req, uint64_t *id);

/* Move up to max finished results to out; *count receives their number. */
int32_t automat_server_poll(automat_server *server, automat_result *out, int32_t max,
                            int32_t *count);

int32_t automat_server_stats(automat_server *server, automat_server_stats_t *stats);

/* Finish the admitted requests, cancel the queued ones, stop the scheduler. */
int32_t automat_server_destroy(automat_server *server);

/* ------------------------------------------------------------------------
 * The paper's "conventional" evaluation strategy (Section "Single Implicit
 * Euler Step" and Table "implicit_euler_timings"): the same implicit-Euler
 * step of the same material, reduced by hand to a scalar equation for the
 * equivalent stress (radial return), without automatic differentiation. A
 * comparison point for automat_evaluate. The flow keeps the direction of
 * the trial deviator and q solves
 *   q + (3 mu + H) h eps0 ((q - sigma_y)^+ / sigma0)^n = q_tr
 * by Newton from q_tr (monotone), stopped when a step is <= tol q.
 * Arguments and layout as automat_evaluate_ex (no tangent, no flags; the
 * tangent comes with automat_evaluate_conventional_ex);
 * iters_out: Newton steps (0 without flow), -1 for invalid input or no
 * convergence within max_iter. */
int32_t automat_evaluate_conventional(int64_t n, const double *eps_new, const double *a_old,
                                      const uint8_t *phase, const automat_params *params,
                                      double h, double tol, int32_t max_iter, double *sigma_out,
                                      double *a_out, int32_t *iters_out, uint64_t *nonconverged,
                                      void *stream);

/* The conventional strategy with its consistent tangent (Section "Single
 * Implicit Euler Step", the tangent of the converged step; Table
 * "implicit_euler_timings" compares the strategies with and without it),
 * derived by hand from the same scalar reduction:
 *   C_tan = kappa I (x) I + 2 mu theta I_dev + 2 mu (beta - theta) N (x) N,
 * N the unit trial deviator, theta = 1 - 3 mu dp / q_tr,
 * beta = 1 - 3 mu c / (1 + c (3 mu + H)), dp = h eps0 x^n,
 * c = h eps0 n x^(n-1) / sigma0, x = (q - sigma_y) / sigma0 at the converged
 * q; the elastic stiffness without flow.
 * tangent_out: device [36][n] (row-major 6x6 per point, engineering-shear
 * Voigt, d sigma / d eps at fixed a_n), or NULL (then exactly
 * automat_evaluate_conventional); it must not overlap another argument
 * array (AUTOMAT_EINVAL for the same base pointer). NaN for invalid points.
 * Other arguments and errors as automat_evaluate_conventional. */
int32_t automat_evaluate_conventional_ex(int64_t n, const double *eps_new, const double *a_old,
                                         const uint8_t *phase, const automat_params *params,
                                         double h, double tol, int32_t max_iter,
                                         double *sigma_out, double *a_out, double *tangent_out,
                                         int32_t *iters_out, uint64_t *nonconverged,
                                         void *stream);

/* ------------------------------------------------------------------------
 * Adaptive explicit Runge-Kutta evaluation (Section "Rosenbrock and
 * Runge-Kutta Schemes with Adaptive Step Size"; error measure on stresses as
 * in Section "Error Control"). Over one load step of length h the strain
 * moves linearly from eps_n to eps_new; a' = dPsi/dA(A(eps(t), a)) is
 * integrated from a_old with the embedded Bogacki-Shampine 3(2) pair (the
 * pair of MATLAB's ode23) and automatic step size control: a step of size
 * dt is accepted when the rms over the six stress components of
 * (sigma_3rd - sigma_2nd) / (atol + rtol max(|sigma_start|, |sigma_end|)) is
 * <= 1; the next dt is dt min(5, max(1/5, 0.9 err^(-1/3))) (growth capped at 1
 * right after a rejection); the first try is the whole load step.
 *   eps_n, eps_new, a_old  device [6][n]; a_out may equal a_old.
 *   sigma_out, a_out       device [6][n]: stress and internal variables at
 *                          the end of the step.
 *   steps_out              device [n] or NULL: accepted steps, -1 if the
 *                          point is invalid or needed more than max_steps
 *                          attempts (its outputs are then the last state,
 *                          or NaN for invalid input), counted in
 *                          *nonconverged (device uint64, or NULL).
 * atol >= 0, rtol > 0 (MATLAB's defaults are 1e-6 and 1e-3), max_steps >= 1.
 * Stream-ordered, asynchronous. The consistent tangent of this scheme is
 * computed by automat_evaluate_rk23_ex. */
int32_t automat_evaluate_rk23(int64_t n, const double *eps_n, const double *eps_new,
                              const double *a_old, const uint8_t *phase,
                              const automat_params *params, double h, double atol, double rtol,
                              int32_t max_steps, double *sigma_out, double *a_out,
                              int32_t *steps_out, uint64_t *nonconverged, void *stream);

/* The lower-order embedded pair of the same section (the paper's ode12):
 * explicit Euler inside Heun's method, k1 = f(t, a), k2 = f(t + dt, a + dt k1),
 * a_{2nd} = a + dt/2 (k1 + k2), a_{1st} = a + dt k1; error measure, step
 * acceptance, first try and growth limits as automat_evaluate_rk23 with the
 * step factor 0.9 err^(-1/2). Arguments, layout, ownership and errors as
 * automat_evaluate_rk23. */
int32_t automat_evaluate_rk12(int64_t n, const double *eps_n, const double *eps_new,
                              const double *a_old, const uint8_t *phase,
                              const automat_params *params, double h, double atol, double rtol,
                              int32_t max_steps, double *sigma_out, double *a_out,
                              int32_t *steps_out, uint64_t *nonconverged, void *stream);

/* The adaptive schemes above with their consistent tangent (Section
 * "Rosenbrock and Runge-Kutta Schemes with Adaptive Step Size", the theorem
 * on differentiating an integration step; Section "Error Control" for the
 * error measure). The sensitivity Y = d a / d eps_new (6x6, Y = 0 at the
 * start of the step) follows Y' = Psi''(A) ((t/h) C - K Y), with C the
 * elastic stiffness and K = d^2 omega / da^2, and is advanced with the same
 * stages and accepted steps as a; the error measure of a step is the rms over
 * 42 components: the six stresses as above and the 36 entries of
 * T = C ((t/h) I - Y), scaled the same way, so the tangent's accuracy also
 * controls the step size (steps_out can exceed that of the plain call). On
 * return tangent_out holds C_{n+1} = d sigma / d eps_new = C (I - Y(h)),
 * device [36][n], row-major 6x6 per point (entry (r, c) at [(6 r + c) n + i]);
 * C for points without flow, NaN for invalid points. tangent_out must not
 * overlap the other arrays; NULL gives the plain evaluation. Other
 * arguments, layout, ownership and errors as automat_evaluate_rk23 (rk23_ex)
 * and automat_evaluate_rk12 (rk12_ex). */
int32_t automat_evaluate_rk23_ex(int64_t n, const double *eps_n, const double *eps_new,
                                 const double *a_old, const uint8_t *phase,
                                 const automat_params *params, double h, double atol,
                                 double rtol, int32_t max_steps, double *sigma_out,
                                 double *a_out, double *tangent_out, int32_t *steps_out,
                                 uint64_t *nonconverged, void *stream);
int32_t automat_evaluate_rk12_ex(int64_t n, const double *eps_n, const double *eps_new,
                                 const double *a_old, const uint8_t *phase,
                                 const automat_params *params, double h, double atol,
                                 double rtol, int32_t max_steps, double *sigma_out,
                                 double *a_out, double *tangent_out, int32_t *steps_out,
                                 uint64_t *nonconverged, void *stream);

/* Single-precision evaluation (Section "Example", paragraph
 * "Parallelization": single precision works for this material law and pays
 * off most with tangent). As automat_evaluate_ex with float fields:
 *   eps_new, a_old  device float [6][n] (in); sigma_out, a_out (may equal
 *   a_old, or NULL), tangent_out (NULL skips it) device float (out);
 *   iters_out, nonconverged as automat_evaluate_ex.
 * Arithmetic is FP32 throughout, with closed-form partials of omega and Psi
 * (the semi-automatic strategy) and the same Newton solve, line search and
 * tangent as the FP64 kernels; the convergence test is
 * ||F||_inf <= max(tol ||a_{n+1} - a_n||_inf, 2^-19 ||eps_new - a_old||_inf),
 * the floor being the FP32 rounding level of the trial elastic strain, so
 * a tol below FP32 resolution converges at that floor; an update smaller
 * than 2^-21 ||a_{n+1} - a_n||_inf (the increment cannot improve in FP32)
 * also counts as converged. Results agree with
 * the FP64 evaluation of the same (float) inputs to a few units of FP32
 * rounding times the conditioning of the step. No flags. Errors as
 * automat_evaluate_ex. */
int32_t automat_evaluate_f32(int64_t n, const float *eps_new, const float *a_old,
                             const uint8_t *phase, const automat_params *params, double h,
                             double tol, int32_t max_iter, float *sigma_out, float *a_out,
                             float *tangent_out, int32_t *iters_out, uint64_t *nonconverged,
                             void *stream);

/* Human-readable text of a return code. */
const char *automat_strerror(int32_t code);

/* Library version string. */
const char *automat_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AUTOMAT_H */
