/*
 * automat_oracle.c -- plain FP64 CPU oracle for one implicit-Euler step of the
 * Michel-Suquet generalized standard material (GSM).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it. It shares no code with the GPU path: the derivatives below
 * are derived by hand (no automatic differentiation) and the Newton system is
 * the paper's nonsymmetric one, solved by Gaussian elimination with partial
 * pivoting.
 *
 * What it computes (paper: Section "Generalized Standard Materials",
 * equations gsm_sigma and gsm_internal; Section "Example", equations
 * michel_suquet_omega and michel_suquet_psi; Section "Single Implicit Euler
 * Step", equations implicit_euler and tangent_formula):
 *
 *   omega(eps, a) = 1/2 (eps - a)^T C (eps - a) + 1/3 a^T Hm a,
 *                   Hm = H diag(1, 1, 1, 1/2, 1/2, 1/2)
 *   Psi(A)        = sigma0 eps0 / (n + 1) ((q(A) - sigma_y)^+ / sigma0)^(n + 1),
 *                   q = von Mises norm of dev A
 *   sigma = d omega / d eps,  A = -d omega / d a,  a' = dPsi/dA (A)
 *
 * with a = viscoplastic strain (engineering-shear Voigt, order 11 22 33 23 13
 * 12) and the isotropic-hardening integral dropped: with K(alpha) = sigma_y
 * constant, alpha only accumulates and never feeds back, and sigma_y enters
 * through Psi. One implicit-Euler step solves
 *
 *   F(Delta) = Delta - h f(A(a_n + Delta)) = 0,   Delta = a_{n+1} - a_n,
 *
 * by Newton from Delta = 0 (a^{(0)} = a_n) with the Jacobian
 * dF/dDelta = I + h Psi''(A) K, K = d^2 omega / d a^2 = C + 2/3 Hm.
 *
 * Readings of the paper where it is silent (each also listed in the design
 * notes): increment unknown Delta; stop when
 * ||F||_inf <= max(tol ||Delta||_inf, 16 u ||eps - a_n||_inf), u = 2^-52:
 * relative to the increment, or at the rounding level of the trial elastic
 * strain that F is computed from (for a flow just above the yield stress
 * the increment is so small that the relative test asks for more digits
 * than F carries); optional stress
 * criterion ||C F||_inf <= tol ||sigma||_inf (the paper's suggestion to
 * converge sigma instead of a); Armijo backtracking on the convex merit
 * function Phi(Delta) = 1/2 Delta^T K Delta + h Psi(A(Delta)), whose gradient
 * is K F, with a rounding allowance of 1e-13 Phi; f = Psi'' = 0 where
 * (q - sigma_y)^+ = 0, except n = 1, sigma_y = 0, where Psi is the smooth
 * quadratic 3 eps0 J2 / (2 sigma0) and Psi'' = 3 eps0 / (2 sigma0) P.
 *
 * Parameter rows (one per phase, 8 doubles):
 *   kind (0 elastic, 1 viscoplastic), E, nu, H, sigma_y, sigma0, eps0, n
 * Parameter-gradient rows (7 doubles): E, nu, H, sigma_y, sigma0, eps0, n.
 *
 * Field layout: structure-of-arrays, component-major, element (c, i) at c*n+i.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_NPAR_IN 8
#define ORACLE_NPAR_GRAD 7
#define ORACLE_SIGMA_CRITERION 1u

typedef struct {
    int kind;
    double E, nu, H, sy, s0, e0, n;
} phase_t;

static void load_phase(const double *row, phase_t *p)
{
    p->kind = (int)row[0];
    p->E = row[1];
    p->nu = row[2];
    p->H = row[3];
    p->sy = row[4];
    p->s0 = row[5];
    p->e0 = row[6];
    p->n = row[7];
}

/* Validation of one phase; 0 if valid. */
static int check_phase(const phase_t *p)
{
    if (!(p->kind == 0 || p->kind == 1)) return -1;
    if (!(p->E > 0.0) || !isfinite(p->E)) return -1;
    if (!(p->nu > -1.0 && p->nu < 0.5)) return -1;
    if (p->kind == 1) {
        if (!(p->H >= 0.0) || !isfinite(p->H)) return -1;
        if (!(p->sy >= 0.0) || !isfinite(p->sy)) return -1;
        if (!(p->s0 > 0.0) || !isfinite(p->s0)) return -1;
        if (!(p->e0 >= 0.0) || !isfinite(p->e0)) return -1;
        if (!(p->n >= 1.0) || !isfinite(p->n)) return -1;
    }
    return 0;
}

/* Isotropic stiffness in engineering-shear Voigt form:
 * normal block lambda + 2 mu on the diagonal, lambda off it; shear block mu I. */
static void stiffness(double E, double nu, double C[6][6])
{
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    double mu = E / (2.0 * (1.0 + nu));
    memset(C, 0, 36 * sizeof(double));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[i][j] = lam + (i == j ? 2.0 * mu : 0.0);
    for (int i = 3; i < 6; ++i) C[i][i] = mu;
}

/* Derivative of the stiffness with respect to nu (hand-derived):
 * d lambda / d nu = E (1 + 2 nu^2) / ((1 + nu)^2 (1 - 2 nu)^2),
 * d mu / d nu = -E / (2 (1 + nu)^2). */
static void stiffness_dnu(double E, double nu, double C[6][6])
{
    double den = (1.0 + nu) * (1.0 - 2.0 * nu);
    double dlam = E * (1.0 + 2.0 * nu * nu) / (den * den);
    double dmu = -E / (2.0 * (1.0 + nu) * (1.0 + nu));
    memset(C, 0, 36 * sizeof(double));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[i][j] = dlam + (i == j ? 2.0 * dmu : 0.0);
    for (int i = 3; i < 6; ++i) C[i][i] = dmu;
}

static const double DIAG_D[6] = {1.0, 1.0, 1.0, 0.5, 0.5, 0.5};

/* K = d^2 omega / d a^2 = C + 2/3 H D */
static void hessian_omega_aa(const phase_t *p, const double C[6][6], double K[6][6])
{
    memcpy(K, C, 36 * sizeof(double));
    for (int i = 0; i < 6; ++i) K[i][i] += (2.0 / 3.0) * p->H * DIAG_D[i];
}

static void matvec(const double M[6][6], const double x[6], double y[6])
{
    for (int i = 0; i < 6; ++i) {
        double s = 0.0;
        for (int j = 0; j < 6; ++j) s += M[i][j] * x[j];
        y[i] = s;
    }
}

/* A = -d omega / d a = C (eps - a) - 2/3 H D a */
static void gen_stress(const phase_t *p, const double C[6][6], const double eps[6],
                       const double a[6], double A[6])
{
    double e[6];
    for (int i = 0; i < 6; ++i) e[i] = eps[i] - a[i];
    matvec(C, e, A);
    for (int i = 0; i < 6; ++i) A[i] -= (2.0 / 3.0) * p->H * DIAG_D[i] * a[i];
}

/* Projection P = d^2 J2 / dA^2 (plain Voigt stress argument). */
static double proj_P(int i, int j)
{
    if (i < 3 && j < 3) return (i == j ? 1.0 : 0.0) - 1.0 / 3.0;
    if (i == j) return 2.0;
    return 0.0;
}

/* g = grad J2 = (s1, s2, s3, 2 A4, 2 A5, 2 A6) with the deviator written as
 * s1 = (2 A1 - A2 - A3) / 3 etc., which is exactly zero for a hydrostatic
 * state (A1 = A2 = A3), so such a state has no flow at all. */
static void deviator(const double A[6], double g[6])
{
    g[0] = (2.0 * A[0] - A[1] - A[2]) / 3.0;
    g[1] = (2.0 * A[1] - A[0] - A[2]) / 3.0;
    g[2] = (2.0 * A[2] - A[0] - A[1]) / 3.0;
    g[3] = 2.0 * A[3];
    g[4] = 2.0 * A[4];
    g[5] = 2.0 * A[5];
}

/* Force potential value, gradient f = dPsi/dA and (optionally) Hessian.
 * Hand-derived:
 *   s = dev(A) (normal part), J2 = 1/2 (s1^2 + s2^2 + s3^2) + A4^2 + A5^2 + A6^2,
 *   q = sqrt(3 J2), g = grad J2 = (s1, s2, s3, 2 A4, 2 A5, 2 A6),
 *   grad q = 3/(2q) g, hess q = 3/(2q) P - grad q grad q^T / q,
 *   x = (q - sigma_y)^+, r = x / sigma0,
 *   Psi = sigma0 eps0 / (n+1) r^(n+1), f = eps0 r^n grad q,
 *   Psi'' = eps0 n / sigma0 r^(n-1) grad q grad q^T + eps0 r^n hess q. */
static double force_potential(const phase_t *p, const double A[6], double f[6],
                              double P2[6][6])
{
    double g[6];
    deviator(A, g);
    double J2 = 0.5 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + A[3] * A[3] + A[4] * A[4] +
                A[5] * A[5];
    if (p->n == 1.0 && p->sy == 0.0) {
        /* smooth quadratic: Psi = eps0/(2 sigma0) q^2 = 3 eps0 J2 / (2 sigma0) */
        double c = 1.5 * p->e0 / p->s0;
        for (int i = 0; i < 6; ++i) f[i] = c * g[i];
        if (P2)
            for (int i = 0; i < 6; ++i)
                for (int j = 0; j < 6; ++j) P2[i][j] = c * proj_P(i, j);
        return c * J2;
    }
    double q = sqrt(3.0 * J2);
    double x = q - p->sy;
    if (!(x > 0.0)) {
        for (int i = 0; i < 6; ++i) f[i] = 0.0;
        if (P2) memset(P2, 0, 36 * sizeof(double));
        return 0.0;
    }
    double r = x / p->s0;
    double rn = pow(r, p->n);
    double gq[6];
    for (int i = 0; i < 6; ++i) gq[i] = 1.5 / q * g[i];
    double fm = p->e0 * rn; /* dPsi/dq */
    for (int i = 0; i < 6; ++i) f[i] = fm * gq[i];
    if (P2) {
        double c1 = p->e0 * p->n / p->s0 * pow(r, p->n - 1.0); /* d2Psi/dq2 */
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double hq = 1.5 / q * proj_P(i, j) - gq[i] * gq[j] / q;
                P2[i][j] = c1 * gq[i] * gq[j] + fm * hq;
            }
    }
    return p->s0 * p->e0 / (p->n + 1.0) * r * rn;
}

/* Solve M X = B for nrhs right-hand sides stored column-wise in B[6][nrhs]
 * (row-major, leading dimension ldb) by Gaussian elimination with partial
 * pivoting. M is overwritten. Returns 0, or -1 if a pivot is exactly zero. */
static int gauss_solve(double M[6][6], double *B, int nrhs, int ldb)
{
    for (int k = 0; k < 6; ++k) {
        int piv = k;
        double best = fabs(M[k][k]);
        for (int i = k + 1; i < 6; ++i)
            if (fabs(M[i][k]) > best) {
                best = fabs(M[i][k]);
                piv = i;
            }
        if (best == 0.0) return -1;
        if (piv != k) {
            for (int j = 0; j < 6; ++j) {
                double t = M[k][j];
                M[k][j] = M[piv][j];
                M[piv][j] = t;
            }
            for (int r = 0; r < nrhs; ++r) {
                double t = B[k * ldb + r];
                B[k * ldb + r] = B[piv * ldb + r];
                B[piv * ldb + r] = t;
            }
        }
        for (int i = k + 1; i < 6; ++i) {
            double l = M[i][k] / M[k][k];
            for (int j = k; j < 6; ++j) M[i][j] -= l * M[k][j];
            for (int r = 0; r < nrhs; ++r) B[i * ldb + r] -= l * B[k * ldb + r];
        }
    }
    for (int k = 5; k >= 0; --k) {
        for (int r = 0; r < nrhs; ++r) {
            double s = B[k * ldb + r];
            for (int j = k + 1; j < 6; ++j) s -= M[k][j] * B[j * ldb + r];
            B[k * ldb + r] = s / M[k][k];
        }
    }
    return 0;
}

static double norm_inf(const double *x)
{
    double m = 0.0;
    for (int i = 0; i < 6; ++i) m = fmax(m, fabs(x[i]));
    return m;
}

/* Residual state at one Newton iterate. */
typedef struct {
    double A[6], f[6], F[6], KD[6];
    double psi, phi;
} resid_t;

static void residual(const phase_t *p, const double C[6][6], const double K[6][6],
                     const double eps[6], const double an[6], const double D[6], double h,
                     resid_t *r)
{
    double a[6];
    for (int i = 0; i < 6; ++i) a[i] = an[i] + D[i];
    gen_stress(p, C, eps, a, r->A);
    r->psi = force_potential(p, r->A, r->f, NULL);
    for (int i = 0; i < 6; ++i) r->F[i] = D[i] - h * r->f[i];
    matvec(K, D, r->KD);
    double dkd = 0.0;
    for (int i = 0; i < 6; ++i) dkd += D[i] * r->KD[i];
    r->phi = 0.5 * dkd + h * r->psi;
}

static int all_finite(const double *x, int m)
{
    for (int i = 0; i < m; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

/* One material point. Returns the number of Newton updates, or -1 if not
 * converged within max_iter (the last iterate is kept) or if the input is
 * invalid (non-finite data, unknown phase: outputs NaN). */
static int eval_point(const phase_t *ph, int nph, int pid, const double eps[6],
                      const double an[6], double h, double tol, int max_iter, unsigned flags,
                      double sig[6], double aout[6], double tan_[36])
{
    if (pid >= nph || !all_finite(eps, 6) || !all_finite(an, 6)) {
        for (int i = 0; i < 6; ++i) sig[i] = aout[i] = NAN;
        if (tan_)
            for (int i = 0; i < 36; ++i) tan_[i] = NAN;
        return -1;
    }
    const phase_t *p = &ph[pid];
    double C[6][6], K[6][6];
    stiffness(p->E, p->nu, C);
    hessian_omega_aa(p, C, K);

    if (p->kind == 0) {
        /* Psi = 0: no evolution, sigma = C (eps - a_n) */
        double e[6];
        for (int i = 0; i < 6; ++i) e[i] = eps[i] - an[i];
        matvec(C, e, sig);
        memcpy(aout, an, 6 * sizeof(double));
        if (tan_) memcpy(tan_, C, 36 * sizeof(double));
        return 0;
    }

    double D[6] = {0, 0, 0, 0, 0, 0};
    double floor_F = 0.0; /* 16 u ||eps - a_n||_inf */
    for (int i = 0; i < 6; ++i) floor_F = fmax(floor_F, fabs(eps[i] - an[i]));
    floor_F *= 16.0 * 0x1p-52;
    resid_t cur, trial;
    residual(p, C, K, eps, an, D, h, &cur);
    int k = 0, status = -1;
    for (;;) {
        int zero = 1;
        for (int i = 0; i < 6; ++i)
            if (cur.F[i] != 0.0) zero = 0;
        if (zero) {
            status = k;
            break;
        }
        if (flags & ORACLE_SIGMA_CRITERION) {
            if (k >= 1) {
                double CF[6], s[6], e[6];
                matvec(C, cur.F, CF);
                for (int i = 0; i < 6; ++i) e[i] = eps[i] - an[i] - D[i];
                matvec(C, e, s);
                if (norm_inf(CF) <= tol * norm_inf(s)) {
                    status = k;
                    break;
                }
            }
        } else if (norm_inf(cur.F) <= fmax(tol * norm_inf(D), floor_F)) {
            status = k;
            break;
        }
        if (k >= max_iter) break;
        /* Newton step: (I + h Psi'' K) delta = F */
        double P2[6][6], J[6][6], delta[6];
        force_potential(p, cur.A, cur.f, P2);
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double s = 0.0;
                for (int l = 0; l < 6; ++l) s += P2[i][l] * K[l][j];
                J[i][j] = (i == j ? 1.0 : 0.0) + h * s;
            }
        memcpy(delta, cur.F, sizeof delta);
        if (gauss_solve(J, delta, 1, 1) != 0) break;
        /* Armijo backtracking on the merit function; slope = (K F) . delta */
        double KF[6], slope = 0.0;
        matvec(K, cur.F, KF);
        for (int i = 0; i < 6; ++i) slope += KF[i] * delta[i];
        double t = 1.0, Dt[6];
        for (;;) {
            for (int i = 0; i < 6; ++i) Dt[i] = D[i] - t * delta[i];
            residual(p, C, K, eps, an, Dt, h, &trial);
            if (trial.phi <= cur.phi - 1e-4 * t * slope + 1e-13 * cur.phi) break;
            if (t < 0x1p-30) break; /* accept the shortest step */
            t *= 0.5;
        }
        memcpy(D, Dt, sizeof D);
        cur = trial;
        ++k;
    }

    for (int i = 0; i < 6; ++i) aout[i] = an[i] + D[i];
    {
        double e[6];
        for (int i = 0; i < 6; ++i) e[i] = eps[i] - aout[i];
        matvec(C, e, sig);
    }
    if (tan_) {
        /* (I + h Psi'' K) Z = h Psi'' C; tangent = C - C Z */
        double P2[6][6], J[6][6], Z[6 * 6];
        double f[6];
        force_potential(p, cur.A, f, P2);
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double s = 0.0, z = 0.0;
                for (int l = 0; l < 6; ++l) {
                    s += P2[i][l] * K[l][j];
                    z += P2[i][l] * C[l][j];
                }
                J[i][j] = (i == j ? 1.0 : 0.0) + h * s;
                Z[i * 6 + j] = h * z;
            }
        if (gauss_solve(J, Z, 6, 6) != 0) {
            for (int i = 0; i < 36; ++i) tan_[i] = NAN;
        } else {
            for (int i = 0; i < 6; ++i)
                for (int j = 0; j < 6; ++j) {
                    double s = 0.0;
                    for (int l = 0; l < 6; ++l) s += C[i][l] * Z[l * 6 + j];
                    tan_[i * 6 + j] = C[i][j] - s;
                }
        }
    }
    return status;
}

static int load_all(int nph, const double *par, phase_t *ph)
{
    if (nph < 1 || nph > 256) return -1;
    for (int k = 0; k < nph; ++k) {
        load_phase(par + (size_t)k * ORACLE_NPAR_IN, &ph[k]);
        if (check_phase(&ph[k]) != 0) return -1;
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (the CPU timing's one-core run). */
void oracle_set_num_threads(int nt)
{
#ifdef _OPENMP
    if (nt >= 1) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

/* Evaluate n points. eps, a_old: [6][n]; sigma, a_out: [6][n]; tangent
 * [36][n] (row-major 6x6 per point) or NULL; iters [n] or NULL. Returns 0,
 * or -1 on invalid arguments. */
int oracle_evaluate(int64_t n, const double *eps, const double *a_old, const uint8_t *phase,
                    int n_phases, const double *par, double h, double tol, int max_iter,
                    unsigned flags, double *sigma, double *a_out, double *tangent,
                    int32_t *iters)
{
    phase_t ph[256];
    if (n < 0 || !eps || !a_old || !phase || !par || !sigma || !a_out) return -1;
    if (!(h > 0.0) || !isfinite(h) || !(tol > 0.0) || max_iter < 1) return -1;
    if (load_all(n_phases, par, ph) != 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double e[6], an[6], s[6], ao[6], t[36];
        for (int c = 0; c < 6; ++c) {
            e[c] = eps[c * n + i];
            an[c] = a_old[c * n + i];
        }
        int it = eval_point(ph, n_phases, phase[i], e, an, h, tol, max_iter, flags, s, ao,
                            tangent ? t : NULL);
        for (int c = 0; c < 6; ++c) {
            sigma[c * n + i] = s[c];
            a_out[c * n + i] = ao[c];
        }
        if (tangent)
            for (int c = 0; c < 36; ++c) tangent[c * n + i] = t[c];
        if (iters) iters[i] = it;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Backward (vector-Jacobian product) through the converged step.
 *
 * Outputs sigma(eps, a_{n+1}; p) and a_{n+1}(eps, a_n; p), where a_{n+1}
 * solves F(a; eps, a_n, p) = a - a_n - h f(eps, a; p) = 0. Given cotangents
 * gs (of sigma) and ga (of a_{n+1}), with the implicit function theorem:
 *   abar = ga + d sigma/d a ^T gs = ga - C gs
 *   J^T w = abar,  J = I + h Psi'' K
 *   grad a_n  = w
 *   grad eps  = C gs + h C Psi'' w
 *   grad p    = gs . d sigma/dp + h w . df/dp   (partials at fixed eps, a)
 * with df/dp = Psi'' dA/dp for the elastic parameters (E, nu, H) and the
 * hand-derived partials of f for the viscous ones:
 *   df/dsigma_y = -eps0 n / sigma0 r^(n-1) grad q, df/dsigma0 = -(n/sigma0) f,
 *   df/deps0 = r^n grad q, df/dn = log(r) f.
 * ------------------------------------------------------------------------ */
static void backward_point(const phase_t *p, const double eps[6], const double an[6],
                           const double anew[6], double h, const double gs[6],
                           const double ga[6], double geps[6], double gan[6],
                           double gp[ORACLE_NPAR_GRAD])
{
    double C[6][6], K[6][6], Cn[6][6];
    (void)an; /* the backward needs only the converged state a_{n+1} */
    stiffness(p->E, p->nu, C);
    stiffness_dnu(p->E, p->nu, Cn);
    hessian_omega_aa(p, C, K);
    double e[6], sig[6], Cgs[6];
    for (int i = 0; i < 6; ++i) e[i] = eps[i] - anew[i];
    matvec(C, e, sig);
    matvec(C, gs, Cgs);

    double A[6], f[6], P2[6][6];
    memset(P2, 0, sizeof P2);
    memset(f, 0, sizeof f);
    if (p->kind == 1) {
        gen_stress(p, C, eps, anew, A);
        force_potential(p, A, f, P2);
    }
    /* J^T w = abar */
    double JT[6][6], w[6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0; /* (P2 K)^T_{ij} = (P2 K)_{ji} */
            for (int l = 0; l < 6; ++l) s += P2[j][l] * K[l][i];
            JT[i][j] = (i == j ? 1.0 : 0.0) + h * s;
        }
    for (int i = 0; i < 6; ++i) w[i] = ga[i] - Cgs[i];
    if (gauss_solve(JT, w, 1, 1) != 0)
        for (int i = 0; i < 6; ++i) w[i] = NAN;
    double P2w[6], CP2w[6];
    matvec(P2, w, P2w);
    matvec(C, P2w, CP2w);
    for (int i = 0; i < 6; ++i) {
        gan[i] = w[i];
        geps[i] = Cgs[i] + h * CP2w[i];
    }

    /* parameter partials */
    double dAdE[6], dAdnu[6], dAdH[6], dsdnu[6];
    for (int i = 0; i < 6; ++i) dAdE[i] = sig[i] / p->E; /* C is linear in E */
    matvec(Cn, e, dsdnu);
    for (int i = 0; i < 6; ++i) {
        dAdnu[i] = dsdnu[i];
        dAdH[i] = -(2.0 / 3.0) * DIAG_D[i] * anew[i];
    }
    double gsE = 0.0, gsnu = 0.0, wP2AE = 0.0, wP2Anu = 0.0, wP2AH = 0.0;
    for (int i = 0; i < 6; ++i) {
        gsE += gs[i] * sig[i] / p->E;
        gsnu += gs[i] * dsdnu[i];
        wP2AE += P2w[i] * dAdE[i]; /* w . Psi'' dA/dp = (Psi'' w) . dA/dp */
        wP2Anu += P2w[i] * dAdnu[i];
        wP2AH += P2w[i] * dAdH[i];
    }
    gp[0] = gsE + h * wP2AE;
    gp[1] = gsnu + h * wP2Anu;
    gp[2] = h * wP2AH;
    gp[3] = gp[4] = gp[5] = gp[6] = 0.0;
    if (p->kind == 1 && !(p->n == 1.0 && p->sy == 0.0)) {
        double g[6];
        deviator(A, g);
        double J2 = 0.5 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + A[3] * A[3] +
                    A[4] * A[4] + A[5] * A[5];
        double q = sqrt(3.0 * J2);
        double x = q - p->sy;
        if (x > 0.0) {
            double r = x / p->s0;
            double wgq = 0.0;
            for (int i = 0; i < 6; ++i) wgq += w[i] * 1.5 / q * g[i];
            double rn = pow(r, p->n);
            double wf = p->e0 * rn * wgq;
            gp[3] = h * (-p->e0 * p->n / p->s0 * pow(r, p->n - 1.0) * wgq);
            gp[4] = h * (-(p->n / p->s0) * wf);
            gp[5] = h * (rn * wgq);
            gp[6] = h * (log(r) * wf);
        }
    } else if (p->kind == 1) {
        /* n = 1, sigma_y = 0: f = 3 eps0 / (2 sigma0) g; the n-derivative of
         * r^n at n = 1 is r log r, taken from the general branch when x > 0 */
        double g[6];
        deviator(A, g);
        double J2 = 0.5 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + A[3] * A[3] +
                    A[4] * A[4] + A[5] * A[5];
        double q = sqrt(3.0 * J2);
        double wg = 0.0;
        for (int i = 0; i < 6; ++i) wg += w[i] * g[i];
        double c = 1.5 * p->e0 / p->s0;
        gp[3] = (q > 0.0) ? h * (-p->e0 / p->s0 * 1.5 / q * wg) : 0.0;
        gp[4] = h * (-(1.0 / p->s0) * c * wg);
        gp[5] = h * (1.5 / p->s0 * wg);
        gp[6] = (q > 0.0) ? h * (log(q / p->s0) * c * wg) : 0.0;
    }
}

/* gpar [n_phases][7] is accumulated (+=). grad_sigma / grad_a may be NULL
 * (treated as zero); grad_a_old may be NULL. Returns 0 or -1. */
int oracle_backward(int64_t n, const double *eps, const double *a_old, const double *a_new,
                    const uint8_t *phase, int n_phases, const double *par, double h,
                    const double *gsig, const double *ga, double *geps, double *ga_old,
                    double *gpar)
{
    phase_t ph[256];
    if (n < 0 || !eps || !a_old || !a_new || !phase || !par || !geps) return -1;
    if (!(h > 0.0) || !isfinite(h)) return -1;
    if (load_all(n_phases, par, ph) != 0) return -1;
    int nt = oracle_num_threads();
    double *part = NULL;
    if (gpar) {
        part = (double *)calloc((size_t)nt * n_phases * ORACLE_NPAR_GRAD, sizeof(double));
        if (!part) return -1;
    }
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double e[6], an[6], anw[6], gs[6], gaa[6], ge[6], gan[6], gp[ORACLE_NPAR_GRAD];
            int pid = phase[i];
            for (int c = 0; c < 6; ++c) {
                e[c] = eps[c * n + i];
                an[c] = a_old[c * n + i];
                anw[c] = a_new[c * n + i];
                gs[c] = gsig ? gsig[c * n + i] : 0.0;
                gaa[c] = ga ? ga[c * n + i] : 0.0;
            }
            if (pid >= n_phases) {
                for (int c = 0; c < 6; ++c) ge[c] = gan[c] = NAN;
                for (int c = 0; c < ORACLE_NPAR_GRAD; ++c) gp[c] = 0.0;
            } else {
                backward_point(&ph[pid], e, an, anw, h, gs, gaa, ge, gan, gp);
            }
            for (int c = 0; c < 6; ++c) {
                geps[c * n + i] = ge[c];
                if (ga_old) ga_old[c * n + i] = gan[c];
            }
            if (part && pid < n_phases)
                for (int c = 0; c < ORACLE_NPAR_GRAD; ++c)
                    part[((size_t)tid * n_phases + pid) * ORACLE_NPAR_GRAD + c] += gp[c];
        }
    }
    if (gpar) {
        for (int t = 0; t < nt; ++t)
            for (int k = 0; k < n_phases * ORACLE_NPAR_GRAD; ++k)
                gpar[k] += part[(size_t)t * n_phases * ORACLE_NPAR_GRAD + k];
        free(part);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Forward (Jacobian-vector) product through the converged step, the same
 * implicit-function argument as the tangent (Section "Single Implicit Euler
 * Step", equation tangent_formula) with perturbed inputs instead of a
 * perturbed strain only. At the converged a_{n+1} = a_n + Delta,
 *   F(Delta; eps, a_n, p) = Delta - h f(A(eps, a_n + Delta; p); p) = 0,
 *   A = C(p) (eps - a) - 2/3 H D a,   sigma = C(p) (eps - a_{n+1}).
 * For a direction (d eps, d a_n, d p):
 *   dA_x    = C d eps - K d a_n + (dA/dp) d p      (explicit part)
 *   J d Delta = h Psi'' dA_x + h (df/dp) d p,      J = I + h Psi'' K
 *   d a_{n+1} = d a_n + d Delta
 *   d sigma   = C (d eps - d a_{n+1}) + (dC/dp) (eps - a_{n+1}) d p
 * with dA/dE = C (eps - a) / E, dA/dnu = dC/dnu (eps - a), dA/dH = -2/3 D a,
 * and the hand-derived partials of f in the viscous parameters:
 *   df/dsigma_y = -eps0 n / sigma0 r^(n-1) grad q,  df/dsigma0 = -(n/sigma0) f,
 *   df/deps0 = r^n grad q,  df/dn = log(r) f   (r = (q - sigma_y)^+ / sigma0;
 * all zero where r = 0, one-sided in sigma_y at sigma_y = 0).
 * ------------------------------------------------------------------------ */
static void jvp_point(const phase_t *p, const double eps[6], const double anew[6], double h,
                      const double de[6], const double dan[6], const double dp[7],
                      double dsig[6], double danew[6])
{
    double C[6][6], K[6][6], Cn[6][6];
    stiffness(p->E, p->nu, C);
    stiffness_dnu(p->E, p->nu, Cn);
    hessian_omega_aa(p, C, K);
    double e[6], sig[6], dsnu[6];
    for (int i = 0; i < 6; ++i) e[i] = eps[i] - anew[i];
    matvec(C, e, sig);   /* = C (eps - a_{n+1}), also C (eps - a) in dA/dE */
    matvec(Cn, e, dsnu); /* dC/dnu (eps - a_{n+1}) */

    double A[6], f[6], P2[6][6];
    memset(f, 0, sizeof f);
    memset(P2, 0, sizeof P2);
    memset(A, 0, sizeof A);
    if (p->kind == 1) {
        gen_stress(p, C, eps, anew, A);
        force_potential(p, A, f, P2);
    }
    /* explicit change of A */
    double Cde[6], Kda[6], dAx[6];
    matvec(C, de, Cde);
    matvec(K, dan, Kda);
    for (int i = 0; i < 6; ++i)
        dAx[i] = Cde[i] - Kda[i] + sig[i] / p->E * dp[0] + dsnu[i] * dp[1] -
                 (2.0 / 3.0) * DIAG_D[i] * anew[i] * dp[2];
    /* df/dp d p for the viscous parameters */
    double dfp[6] = {0, 0, 0, 0, 0, 0};
    if (p->kind == 1) {
        double g[6];
        deviator(A, g);
        double J2 = 0.5 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + A[3] * A[3] +
                    A[4] * A[4] + A[5] * A[5];
        double q = sqrt(3.0 * J2);
        double x = q - p->sy;
        if (x > 0.0) {
            double r = x / p->s0;
            double rn = pow(r, p->n);
            for (int i = 0; i < 6; ++i) {
                double gq = 1.5 / q * g[i];
                double fi = p->e0 * rn * gq;
                dfp[i] = -p->e0 * p->n / p->s0 * pow(r, p->n - 1.0) * gq * dp[3] -
                         (p->n / p->s0) * fi * dp[4] + rn * gq * dp[5] + log(r) * fi * dp[6];
            }
        }
    }
    /* J d Delta = h Psi'' dA_x + h df/dp dp */
    double J[6][6], dD[6], P2dA[6];
    matvec(P2, dAx, P2dA);
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int l = 0; l < 6; ++l) s += P2[i][l] * K[l][j];
            J[i][j] = (i == j ? 1.0 : 0.0) + h * s;
        }
        dD[i] = h * (P2dA[i] + dfp[i]);
    }
    if (gauss_solve(J, dD, 1, 1) != 0)
        for (int i = 0; i < 6; ++i) dD[i] = NAN;
    double da1[6], dee[6], Cdee[6];
    for (int i = 0; i < 6; ++i) {
        da1[i] = dan[i] + dD[i];
        dee[i] = de[i] - da1[i];
    }
    matvec(C, dee, Cdee);
    for (int i = 0; i < 6; ++i) {
        dsig[i] = Cdee[i] + sig[i] / p->E * dp[0] + dsnu[i] * dp[1];
        danew[i] = da1[i];
    }
}

/* d_eps, d_a_old: [6][n] or NULL (zero); d_par: [n_phases][7] or NULL
 * (zero), the parameter direction of each phase; d_sigma [6][n];
 * d_a_new [6][n] or NULL. a_new is the converged state of oracle_evaluate.
 * Unknown phases give NaN. Returns 0, or -1 on invalid arguments. */
int oracle_jvp(int64_t n, const double *eps, const double *a_new, const uint8_t *phase,
               int n_phases, const double *par, double h, const double *d_eps,
               const double *d_a_old, const double *d_par, double *d_sigma, double *d_a_new)
{
    phase_t ph[256];
    if (n < 0 || !eps || !a_new || !phase || !par || !d_sigma) return -1;
    if (!(h > 0.0) || !isfinite(h)) return -1;
    if (load_all(n_phases, par, ph) != 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double e[6], anw[6], de[6], dan[6], dp[7] = {0, 0, 0, 0, 0, 0, 0}, ds[6], da[6];
        int pid = phase[i];
        for (int c = 0; c < 6; ++c) {
            e[c] = eps[c * n + i];
            anw[c] = a_new[c * n + i];
            de[c] = d_eps ? d_eps[c * n + i] : 0.0;
            dan[c] = d_a_old ? d_a_old[c * n + i] : 0.0;
        }
        if (pid >= n_phases) {
            for (int c = 0; c < 6; ++c) ds[c] = da[c] = NAN;
        } else {
            if (d_par)
                for (int c = 0; c < ORACLE_NPAR_GRAD; ++c)
                    dp[c] = d_par[pid * ORACLE_NPAR_GRAD + c];
            jvp_point(&ph[pid], e, anw, h, de, dan, dp, ds, da);
        }
        for (int c = 0; c < 6; ++c) {
            d_sigma[c * n + i] = ds[c];
            if (d_a_new) d_a_new[c * n + i] = da[c];
        }
    }
    return 0;
}

/* Convenience for tests: Psi'' and f at one generalized stress. */
int oracle_force_potential(const double *row, const double A[6], double f[6], double P2[36],
                           double *psi)
{
    phase_t p;
    load_phase(row, &p);
    if (check_phase(&p) != 0) return -1;
    double H[6][6];
    *psi = force_potential(&p, A, f, H);
    memcpy(P2, H, sizeof H);
    return 0;
}

/* ------------------------------------------------------------------------
 * Adaptive explicit Runge-Kutta evaluation (paper: Section "Rosenbrock and
 * Runge-Kutta Schemes with Adaptive Step Size" and Section "Error Control";
 * the embedded Bogacki-Shampine 3(2) pair behind MATLAB's ode23, with the
 * automatic step size control of Hairer, Norsett and Wanner).
 *
 * On the load step [t_n, t_n + h] the strain moves linearly,
 *   eps(s) = eps_n + (s / h) (eps_{n+1} - eps_n),  0 <= s <= h,
 * and the internal variables follow a' = f(A(eps(s), a)). With the tangent,
 * the sensitivity Y = d a / d eps_{n+1} (6x6, Y(0) = 0) follows
 *   Y' = Psi''(A) ((s / h) C - K Y)
 * and is advanced by the same stages and the same accepted steps (the
 * combined system of the paper's Theorem "ad_integration_step").
 *
 * One step of size dt from (s, y) (k1 is the last stage of the previous
 * accepted step, first same as last):
 *   k2 = f(s + dt/2, y + dt/2 k1),  k3 = f(s + 3dt/4, y + 3dt/4 k2),
 *   y1 = y + dt (2/9 k1 + 1/3 k2 + 4/9 k3),  k4 = f(s + dt, y1),
 *   yh = y + dt (7/24 k1 + 1/4 k2 + 1/3 k3 + 1/8 k4).
 * Error measure on stresses: sigma = C (eps(s) - a) (and, with the tangent,
 * T = C ((s/h) I - Y)),
 *   err = sqrt(mean over components of ((z1 - zh) / (atol + rtol max(|z0|, |z1|)))^2)
 * with z0 at the start, z1 and zh from y1 and yh at the end of the step.
 * The step is accepted when err <= 1. New step size
 *   dt * min(fmax, max(1/5, 9/10 err^(-1/3))),  fmax = 5, or 1 right after a
 * rejection; the first try is the whole load step, and a step never passes
 * s = h. Elastic phases (f = 0) take one step.
 * ------------------------------------------------------------------------ */

static void rk_rhs(const phase_t *p, const double C[6][6], const double e0[6],
                   const double de[6], double theta, const double a[6], double k[6],
                   double P2[6][6])
{
    double eps[6], A[6];
    for (int i = 0; i < 6; ++i) eps[i] = e0[i] + theta * de[i];
    gen_stress(p, C, eps, a, A);
    if (p->kind == 0) {
        for (int i = 0; i < 6; ++i) k[i] = 0.0;
        if (P2) memset(P2, 0, 36 * sizeof(double));
        return;
    }
    force_potential(p, A, k, P2);
}

/* tangent stage: Ydot = Psi'' (theta C - K Y) */
static void rk_rhs_tan(const double P2[6][6], const double C[6][6], const double K[6][6],
                       double theta, const double Y[36], double KY[36])
{
    double B[6][6];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = theta * C[i][j];
            for (int q = 0; q < 6; ++q) s -= K[i][q] * Y[q * 6 + j];
            B[i][j] = s;
        }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0.0;
            for (int q = 0; q < 6; ++q) s += P2[i][q] * B[q][j];
            KY[i * 6 + j] = s;
        }
}

static double rk_scale(double atol, double rtol, double z0, double z1)
{
    return atol + rtol * fmax(fabs(z0), fabs(z1));
}

/* Returns the number of accepted steps, or -1 (invalid input or more than
 * max_steps attempts). sigma, a_out [6]; tangent [36] or NULL. */
static int rk23_point(const phase_t *ph, int nph, int pid, const double eps_n[6],
                      const double eps1[6], const double an[6], double h, double atol,
                      double rtol, int max_steps, double sigma[6], double a_out[6],
                      double *tangent, int *rejected)
{
    *rejected = 0;
    int bad = pid >= nph || !all_finite(eps_n, 6) || !all_finite(eps1, 6) || !all_finite(an, 6);
    if (bad) {
        for (int i = 0; i < 6; ++i) sigma[i] = a_out[i] = NAN;
        if (tangent)
            for (int i = 0; i < 36; ++i) tangent[i] = NAN;
        return -1;
    }
    const phase_t *p = &ph[pid];
    double C[6][6], K[6][6], de[6];
    stiffness(p->E, p->nu, C);
    hessian_omega_aa(p, C, K);
    for (int i = 0; i < 6; ++i) de[i] = eps1[i] - eps_n[i];
    const int tan = tangent != NULL;
    double y[6], Y[36], k1[6], k2[6], k3[6], k4[6], yt[6], y1[6], yh[6];
    double K1[36], K2[36], K3[36], K4[36], Yt[36], Y1[36], Yh[36], P2[6][6];
    memcpy(y, an, sizeof y);
    memset(Y, 0, sizeof Y);
    rk_rhs(p, C, eps_n, de, 0.0, y, k1, tan ? P2 : NULL);
    if (tan) rk_rhs_tan(P2, C, K, 0.0, Y, K1);
    double s = 0.0, dt = h, fmax_ = 5.0;
    int accepted = 0, attempts = 0, status = 0;
    while (s < h) {
        if (++attempts > max_steps) {
            status = -1;
            break;
        }
        const int last = dt >= h - s;
        if (last) dt = h - s;
        const double th0 = s / h, th2 = (s + 0.5 * dt) / h, th3 = (s + 0.75 * dt) / h;
        const double th4 = last ? 1.0 : (s + dt) / h;
        for (int i = 0; i < 6; ++i) yt[i] = y[i] + 0.5 * dt * k1[i];
        rk_rhs(p, C, eps_n, de, th2, yt, k2, tan ? P2 : NULL);
        if (tan) {
            for (int i = 0; i < 36; ++i) Yt[i] = Y[i] + 0.5 * dt * K1[i];
            rk_rhs_tan(P2, C, K, th2, Yt, K2);
        }
        for (int i = 0; i < 6; ++i) yt[i] = y[i] + 0.75 * dt * k2[i];
        rk_rhs(p, C, eps_n, de, th3, yt, k3, tan ? P2 : NULL);
        if (tan) {
            for (int i = 0; i < 36; ++i) Yt[i] = Y[i] + 0.75 * dt * K2[i];
            rk_rhs_tan(P2, C, K, th3, Yt, K3);
        }
        for (int i = 0; i < 6; ++i)
            y1[i] = y[i] + dt * (2.0 / 9.0 * k1[i] + 1.0 / 3.0 * k2[i] + 4.0 / 9.0 * k3[i]);
        rk_rhs(p, C, eps_n, de, th4, y1, k4, tan ? P2 : NULL);
        if (tan) {
            for (int i = 0; i < 36; ++i)
                Y1[i] = Y[i] + dt * (2.0 / 9.0 * K1[i] + 1.0 / 3.0 * K2[i] + 4.0 / 9.0 * K3[i]);
            rk_rhs_tan(P2, C, K, th4, Y1, K4);
        }
        for (int i = 0; i < 6; ++i)
            yh[i] = y[i] + dt * (7.0 / 24.0 * k1[i] + 0.25 * k2[i] + 1.0 / 3.0 * k3[i] +
                                 0.125 * k4[i]);
        /* error measure on the stresses (and tangents) */
        double e_s[6], e_1[6];
        for (int i = 0; i < 6; ++i) {
            e_s[i] = eps_n[i] + th0 * de[i];
            e_1[i] = eps_n[i] + th4 * de[i];
        }
        double d0[6], d1[6], dh[6], z0[6], z1[6], zh[6];
        for (int i = 0; i < 6; ++i) {
            d0[i] = e_s[i] - y[i];
            d1[i] = e_1[i] - y1[i];
            dh[i] = e_1[i] - yh[i];
        }
        matvec(C, d0, z0);
        matvec(C, d1, z1);
        matvec(C, dh, zh);
        double sum = 0.0;
        int cnt = 6;
        for (int i = 0; i < 6; ++i) {
            const double r = (z1[i] - zh[i]) / rk_scale(atol, rtol, z0[i], z1[i]);
            sum += r * r;
        }
        if (tan) {
            for (int j = 0; j < 6; ++j)
                for (int i = 0; i < 6; ++i) {
                    /* T = C (theta I - Y): entry (i, j) */
                    double t0 = th0 * C[i][j], t1 = th4 * C[i][j], tq = th4 * C[i][j];
                    for (int q = 0; q < 6; ++q) {
                        t0 -= C[i][q] * Y[q * 6 + j];
                        t1 -= C[i][q] * Y1[q * 6 + j];
                    }
                    for (int q = 0; q < 6; ++q) {
                        double yhq = Y[q * 6 + j] + dt * (7.0 / 24.0 * K1[q * 6 + j] +
                                                           0.25 * K2[q * 6 + j] +
                                                           1.0 / 3.0 * K3[q * 6 + j] +
                                                           0.125 * K4[q * 6 + j]);
                        Yh[q * 6 + j] = yhq;
                        tq -= C[i][q] * yhq;
                    }
                    const double r = (t1 - tq) / rk_scale(atol, rtol, t0, t1);
                    sum += r * r;
                }
            cnt += 36;
        }
        const double err = sqrt(sum / cnt);
        double fac = err > 0.0 ? 0.9 * pow(err, -1.0 / 3.0) : fmax_;
        fac = fmin(fmax_, fmax(0.2, fac));
        if (err <= 1.0) {
            ++accepted;
            s = last ? h : s + dt;
            memcpy(y, y1, sizeof y);
            memcpy(k1, k4, sizeof k1);
            if (tan) {
                memcpy(Y, Y1, sizeof Y);
                memcpy(K1, K4, sizeof K1);
            }
            dt *= fac;
            fmax_ = 5.0;
        } else {
            ++*rejected;
            dt *= fmin(1.0, fac);
            fmax_ = 1.0;
        }
    }
    (void)Yh;
    double d[6];
    for (int i = 0; i < 6; ++i) {
        a_out[i] = y[i];
        d[i] = eps1[i] - y[i];
    }
    matvec(C, d, sigma);
    if (tangent)
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double t = C[i][j];
                for (int q = 0; q < 6; ++q) t -= C[i][q] * Y[q * 6 + j];
                tangent[i * 6 + j] = t;
            }
    return status < 0 ? -1 : accepted;
}

/* Adaptive ode23 evaluation of n points: eps_n, eps1, a_old [6][n]; sigma,
 * a_out [6][n]; tangent [36][n] or NULL; steps, rejected [n] or NULL.
 * Returns 0, or -1 on invalid arguments. */
int oracle_evaluate_rk23(int64_t n, const double *eps_n, const double *eps1,
                         const double *a_old, const uint8_t *phase, int n_phases,
                         const double *par, double h, double atol, double rtol, int max_steps,
                         double *sigma, double *a_out, double *tangent, int32_t *steps,
                         int32_t *rejected)
{
    phase_t ph[256];
    if (n < 0 || !eps_n || !eps1 || !a_old || !phase || !par || !sigma || !a_out) return -1;
    if (!(h > 0.0) || !isfinite(h) || !(atol >= 0.0) || !(rtol > 0.0) || max_steps < 1)
        return -1;
    if (load_all(n_phases, par, ph) != 0) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double e0[6], e1[6], an[6], s[6], ao[6], t[36];
        for (int c = 0; c < 6; ++c) {
            e0[c] = eps_n[c * n + i];
            e1[c] = eps1[c * n + i];
            an[c] = a_old[c * n + i];
        }
        int rej = 0;
        int st = rk23_point(ph, n_phases, phase[i], e0, e1, an, h, atol, rtol, max_steps, s, ao,
                            tangent ? t : NULL, &rej);
        for (int c = 0; c < 6; ++c) {
            sigma[c * n + i] = s[c];
            a_out[c * n + i] = ao[c];
        }
        if (tangent)
            for (int c = 0; c < 36; ++c) tangent[c * n + i] = t[c];
        if (steps) steps[i] = st;
        if (rejected) rejected[i] = rej;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * The lower-order pair the paper calls ode12: explicit Euler embedded in
 * Heun's method. One step of size dt from (s, y):
 *   k1 = f(s, y),  k2 = f(s + dt, y + dt k1),
 *   y1 = y + dt/2 (k1 + k2)  (second order),  yh = y + dt k1  (first order).
 * Same error measure on stresses (and tangents) and the same step size
 * rule as above with exponent 1/2 (the lower order is 1). k1 is evaluated
 * afresh at every step (the pair is not first-same-as-last).
 * ------------------------------------------------------------------------ */
static int rk12_point(const phase_t *ph, int nph, int pid, const double eps_n[6],
                      const double eps1[6], const double an[6], double h, double atol,
                      double rtol, int max_steps, double sigma[6], double a_out[6],
                      double *tangent, int *rejected)
{
    *rejected = 0;
    int bad = pid >= nph || !all_finite(eps_n, 6) || !all_finite(eps1, 6) || !all_finite(an, 6);
    if (bad) {
        for (int i = 0; i < 6; ++i) sigma[i] = a_out[i] = NAN;
        if (tangent)
            for (int i = 0; i < 36; ++i) tangent[i] = NAN;
        return -1;
    }
    const phase_t *p = &ph[pid];
    double C[6][6], K[6][6], de[6];
    stiffness(p->E, p->nu, C);
    hessian_omega_aa(p, C, K);
    for (int i = 0; i < 6; ++i) de[i] = eps1[i] - eps_n[i];
    const int tan = tangent != NULL;
    double y[6], Y[36], k1[6], k2[6], yt[6], y1[6], yh[6], K1[36], K2[36], Yt[36], Y1[36];
    double P2[6][6];
    memcpy(y, an, sizeof y);
    memset(Y, 0, sizeof Y);
    double s = 0.0, dt = h, fmax_ = 5.0;
    int accepted = 0, attempts = 0, status = 0;
    while (s < h) {
        if (++attempts > max_steps) {
            status = -1;
            break;
        }
        const int last = dt >= h - s;
        if (last) dt = h - s;
        const double th0 = s / h, th1 = last ? 1.0 : (s + dt) / h;
        rk_rhs(p, C, eps_n, de, th0, y, k1, tan ? P2 : NULL);
        if (tan) rk_rhs_tan(P2, C, K, th0, Y, K1);
        for (int i = 0; i < 6; ++i) yt[i] = y[i] + dt * k1[i];
        rk_rhs(p, C, eps_n, de, th1, yt, k2, tan ? P2 : NULL);
        if (tan) {
            for (int i = 0; i < 36; ++i) Yt[i] = Y[i] + dt * K1[i];
            rk_rhs_tan(P2, C, K, th1, Yt, K2);
        }
        for (int i = 0; i < 6; ++i) {
            y1[i] = y[i] + 0.5 * dt * (k1[i] + k2[i]);
            yh[i] = y[i] + dt * k1[i];
        }
        double d0[6], d1[6], dh[6], z0[6], z1[6], zh[6];
        for (int i = 0; i < 6; ++i) {
            const double e0 = eps_n[i] + th0 * de[i], e1 = eps_n[i] + th1 * de[i];
            d0[i] = e0 - y[i];
            d1[i] = e1 - y1[i];
            dh[i] = e1 - yh[i];
        }
        matvec(C, d0, z0);
        matvec(C, d1, z1);
        matvec(C, dh, zh);
        double sum = 0.0;
        int cnt = 6;
        for (int i = 0; i < 6; ++i) {
            const double r = (z1[i] - zh[i]) / rk_scale(atol, rtol, z0[i], z1[i]);
            sum += r * r;
        }
        if (tan) {
            for (int i = 0; i < 36; ++i) Y1[i] = Y[i] + 0.5 * dt * (K1[i] + K2[i]);
            for (int j = 0; j < 6; ++j)
                for (int i = 0; i < 6; ++i) {
                    double t0 = th0 * C[i][j], t1 = th1 * C[i][j], tq = th1 * C[i][j];
                    for (int q = 0; q < 6; ++q) {
                        t0 -= C[i][q] * Y[q * 6 + j];
                        t1 -= C[i][q] * Y1[q * 6 + j];
                        tq -= C[i][q] * (Y[q * 6 + j] + dt * K1[q * 6 + j]);
                    }
                    const double r = (t1 - tq) / rk_scale(atol, rtol, t0, t1);
                    sum += r * r;
                }
            cnt += 36;
        }
        const double err = sqrt(sum / cnt);
        double fac = err > 0.0 ? 0.9 * pow(err, -0.5) : fmax_;
        fac = fmin(fmax_, fmax(0.2, fac));
        if (err <= 1.0) {
            ++accepted;
            s = last ? h : s + dt;
            memcpy(y, y1, sizeof y);
            if (tan) memcpy(Y, Y1, sizeof Y);
            dt *= fac;
            fmax_ = 5.0;
        } else {
            ++*rejected;
            dt *= fmin(1.0, fac);
            fmax_ = 1.0;
        }
    }
    double d[6];
    for (int i = 0; i < 6; ++i) {
        a_out[i] = y[i];
        d[i] = eps1[i] - y[i];
    }
    matvec(C, d, sigma);
    if (tangent)
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) {
                double t = C[i][j];
                for (int q = 0; q < 6; ++q) t -= C[i][q] * Y[q * 6 + j];
                tangent[i * 6 + j] = t;
            }
    return status < 0 ? -1 : accepted;
}

int oracle_evaluate_rk12(int64_t n, const double *eps_n, const double *eps1,
                         const double *a_old, const uint8_t *phase, int n_phases,
                         const double *par, double h, double atol, double rtol, int max_steps,
                         double *sigma, double *a_out, double *tangent, int32_t *steps,
                         int32_t *rejected)
{
    phase_t ph[256];
    if (n < 0 || !eps_n || !eps1 || !a_old || !phase || !par || !sigma || !a_out) return -1;
    if (!(h > 0.0) || !isfinite(h) || !(atol >= 0.0) || !(rtol > 0.0) || max_steps < 1)
        return -1;
    if (load_all(n_phases, par, ph) != 0) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double e0[6], e1[6], an[6], s[6], ao[6], t[36];
        for (int c = 0; c < 6; ++c) {
            e0[c] = eps_n[c * n + i];
            e1[c] = eps1[c * n + i];
            an[c] = a_old[c * n + i];
        }
        int rej = 0;
        int st = rk12_point(ph, n_phases, phase[i], e0, e1, an, h, atol, rtol, max_steps, s, ao,
                            tangent ? t : NULL, &rej);
        for (int c = 0; c < 6; ++c) {
            sigma[c * n + i] = s[c];
            a_out[c * n + i] = ao[c];
        }
        if (tangent)
            for (int c = 0; c < 36; ++c) tangent[c * n + i] = t[c];
        if (steps) steps[i] = st;
        if (rejected) rejected[i] = rej;
    }
    return 0;
}
