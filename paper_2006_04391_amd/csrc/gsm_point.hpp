// gsm_point.hpp -- per-point implicit-Euler solve of a GSM, generic over the
// material model (paper: Section "Single Implicit Euler Step").
//
// Unknown: the increment D = a_{n+1} - a_n, started at 0 (a^{(0)} = a_n).
// Residual F(D) = D - h f(A(a_n + D)), f = dPsi/dA, A = -d omega / d a, both
// from reverse sweeps of the AD layer. Newton's matrix is
// J = I + h Psi''(A) K with K = d^2 omega / d a^2. Instead of J, the solver
// factors the symmetric positive definite matrix
//
//   M = K^{-1} + h Psi''(A)       (J = M K),
//
// by an in-register Cholesky factorization: with y = M^{-1} F the Newton
// update is delta = K^{-1} y, exactly J^{-1} F. K^{-1} is a per-phase
// constant (omega is quadratic in a) computed once per block from the AD
// Hessian of omega.
//
// Step control: Armijo backtracking on the convex merit function
// Phi(D) = 1/2 D^T K D + h Psi(A(D)), whose gradient is K F, so the Newton
// direction has slope -F^T y < 0. Along D - t delta (K delta = y) the change
// is Phi(D - t delta) - Phi(D) = -t D.y + t^2/2 delta.y + h (Psi_t - Psi),
// so only scalars are carried; Phi itself is accumulated from these
// differences. A rounding allowance of 1e-13 Phi keeps round-off from
// rejecting steps once the residual is at machine level.
//
// Stopping: F vanishes exactly (no flow), or after at least one update
// ||F||_inf <= tol ||D||_inf (or, with the stress criterion,
// ||d sigma/d a F||_inf <= tol ||sigma||_inf); otherwise at max_iter updates
// the point is flagged as not converged and keeps its last iterate. The
// wave leaves the loop as soon as a ballot shows every lane done.
//
// Consistent tangent (equation tangent_formula with the implicit function
// theorem): with R = K^{-1} d^2 omega/(da deps) and
// C0 = d^2 omega/deps^2 - d^2 omega/(deps da) R (both per-phase constants),
//
//   C_{n+1} = C0 + R^T M^{-1} R = C0 + W^T W,   W = L^{-1} R,  M = L L^T,
//
// which reuses the Cholesky factor at the converged point and is symmetric
// by construction.
#pragma once

#include "linalg6.hpp"
#include "msgsm.hpp"

#pragma clang fp reassociate(on)

namespace automat {

// Per-phase constants, built on the device from the AD Hessian of omega.
template <class Model>
struct PhaseConst {
    typename Model::Phase prm;
    double Kinv[21];   // (d2 omega / da2)^-1, packed
    double K[21];      // d2 omega / da2, packed (merit value at a warm start)
    double Cee[21];    // d2 omega / deps2, packed (elastic stiffness)
    double C0[21];     // Cee - Kea Kinv Kae, packed
    double R[36];      // Kinv Kae, row-major (row a, column eps)
};

template <class Model>
AD_FN bool build_phase_const(const typename Model::Phase &p, PhaseConst<Model> &pc,
                             bool tangent) {
    pc.prm = p;
    Model::derive(pc.prm);
    double Kaa[21], Kae[6][6], Kee[21];
    Model::omega_hessian(pc.prm, Kaa, Kae, Kee);
    double L[21];
#pragma unroll
    for (int i = 0; i < 21; ++i) {
        L[i] = Kaa[i];
        pc.K[i] = Kaa[i];
        pc.Cee[i] = Kee[i];
    }
    const bool ok = la::cholesky6(L);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double col[6] = {0, 0, 0, 0, 0, 0};
        col[j] = 1.0;
        la::chol_solve6(L, col);
#pragma unroll
        for (int i = j; i < 6; ++i) pc.Kinv[la::pk(i, j)] = col[i];
    }
    if (tangent) {
        // R = Kinv Kae, C0 = Kee - Kae^T R
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            double col[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) col[i] = Kae[i][j];
            double r[6];
            la::symv6(pc.Kinv, col, r);
#pragma unroll
            for (int i = 0; i < 6; ++i) pc.R[i * 6 + j] = r[i];
        }
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < 6; ++k) s += Kae[k][i] * pc.R[k * 6 + j];
                pc.C0[la::pk(i, j)] = Kee[la::pk(i, j)] - s;
            }
    }
    return ok;
}

// Read-only view of a 6-vector stored with a stride (e.g. a lane's column of
// an LDS staging array); plain arrays work too.
template <int S>
struct Strided {
    const double *p;
    AD_FN double operator[](int i) const { return p[i * S]; }
};

// State of one residual evaluation: generalized stress, residual, Psi.
struct Resid {
    double A[6], F[6];
    double psi;
};

template <class Model, class V>
AD_FN void residual(const typename Model::Phase &prm, const V &eps, const V &an,
                    const double *D, double h, Resid &r) {
    double a[6], e[6], f[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        a[i] = an[i] + D[i];
        e[i] = eps[i];
    }
    Model::gen_stress(prm, e, a, r.A);
    asm volatile("" ::: "memory");  // re-read the phase constants for the Psi sweep
    r.psi = Model::psi_grad(prm, r.A, f);
#pragma unroll
    for (int i = 0; i < 6; ++i) r.F[i] = D[i] - h * f[i];
}

// Residual together with the Newton matrix of the same point,
// M = K^{-1} + h Psi''(A), from one forward-over-reverse sweep of Psi: the
// next Newton step (or the tangent, at the converged point) factors this M,
// so the transcendental part of Psi is evaluated once per trial point.
struct Resid2 : Resid {
    double M[21];
};

template <class Model, class V>
AD_FN void residual2(const typename Model::Phase &prm, const double *Kinv, const V &eps,
                     const V &an, const double *D, double h, Resid2 &r) {
    double a[6], e[6], f[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        a[i] = an[i] + D[i];
        e[i] = eps[i];
    }
    Model::gen_stress(prm, e, a, r.A);
    asm volatile("" ::: "memory");  // re-read the phase constants for the Psi sweep
    r.psi = Model::psi_grad_hess(prm, r.A, f, r.M);
#pragma unroll
    for (int i = 0; i < 6; ++i) r.F[i] = D[i] - h * f[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) r.M[i] = Kinv[i] + h * r.M[i];
}

// Newton matrix M = K^-1 + h Psi''(A) at the point of a first-order
// residual.
template <class Model>
AD_FN void newton_matrix(const typename Model::Phase &prm, const double *Kinv, double h,
                         Resid2 &r) {
    Model::psi_hess(prm, r.A, r.M);
#pragma unroll
    for (int i = 0; i < 21; ++i) r.M[i] = Kinv[i] + h * r.M[i];
}

// Stress-criterion test: ||d sigma / d a . F||_inf <= tol ||sigma||_inf at
// a = a_n + D, with both terms from the AD layer.
template <class Model, class V>
AD_FN bool sigma_converged(const typename Model::Phase &prm, const V &epsv, const V &an,
                           const double *D, const double *F, double tol) {
    double a[6], sig[6], eps[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        a[i] = an[i] + D[i];
        eps[i] = epsv[i];
    }
    Model::stress(prm, eps, a, sig);
    Leaves6<Model::OM_EPS> le(eps);
    Leaves6<Model::OM_A> la_(a);
    ad::VecDir<6, Model::OM_A> dir;
#pragma unroll
    for (int i = 0; i < 6; ++i) dir.d[i] = F[i];
    ad::GradT<6, Model::OM_EPS> dsig;
    ad::sweep2(Model::omega(le, la_, prm.lam, prm.mu, prm.H), dir, dsig);
    return la::norm_inf6(dsig.g) <= tol * la::norm_inf6(sig);
}

}  // namespace automat

#pragma clang fp reassociate(off)
