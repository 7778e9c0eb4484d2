// msgsm_hand.hpp -- the semi-automatic evaluation strategy: the generic
// implicit-Euler Newton solve and consistent tangent of the automatic
// strategy, fed with hand-derived partials of omega and Psi instead of
// automatic differentiation (the paper's Section "Example", paragraph on the
// evaluation strategies, which compares conventional, automatic and
// semi-automatic evaluations).
//
// Same model as MSGSM (engineering Voigt strains, plain Voigt stresses):
//   sigma = C (eps - a),  A = -d omega/da = sigma - Hm a,
//   Hm = diag(2H/3, 2H/3, 2H/3, H/3, H/3, H/3),
//   J2(A) = (s1^2 + s2^2 + s3^2)/2 + A4^2 + A5^2 + A6^2,
//   g = dJ2/dA = (s1, s2, s3, 2 A4, 2 A5, 2 A6),
//   d2J2/dA2 = [I - 11^T/3 on the normal block, 2 I on the shear block].
// Without a yield threshold Psi = coef u^(pq/2) with u = 3 J2 / sigma0^2;
// with one, Psi = coef x^pq with x = (q - sigma_y)^+ / sigma0, q = sqrt(3 J2)
// (coef = sigma0 eps0 / (n + 1), pq = n + 1). Where Psi is flat (below the
// threshold, or at u = 0 for n > 1) f and Psi'' vanish; for n = 1 without a
// threshold Psi is the quadratic coef u.
#pragma once

#include "linalg6.hpp"
#include "msgsm.hpp"

#pragma clang fp reassociate(on)

namespace automat {

struct MSGSMHand : MSGSM {
    AD_FN static void stress(const Phase &p, const double *eps, const double *a, double *sig) {
        double e[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) e[i] = eps[i] - a[i];
        const double tr = p.lam * (e[0] + e[1] + e[2]);
#pragma unroll
        for (int i = 0; i < 3; ++i) sig[i] = tr + 2.0 * p.mu * e[i];
#pragma unroll
        for (int i = 3; i < 6; ++i) sig[i] = p.mu * e[i];
    }

    AD_FN static void gen_stress(const Phase &p, const double *eps, const double *a, double *A) {
        stress(p, eps, a, A);
        const double h2 = (2.0 / 3.0) * p.H, h1 = (1.0 / 3.0) * p.H;
#pragma unroll
        for (int i = 0; i < 3; ++i) A[i] -= h2 * a[i];
#pragma unroll
        for (int i = 3; i < 6; ++i) A[i] -= h1 * a[i];
    }

    // J2 and its gradient g
    AD_FN static double j2_grad(const double *A, double *g) {
        constexpr double third = 1.0 / 3.0;
        g[0] = (2.0 * A[0] - A[1] - A[2]) * third;
        g[1] = (2.0 * A[1] - A[0] - A[2]) * third;
        g[2] = (2.0 * A[2] - A[0] - A[1]) * third;
        g[3] = 2.0 * A[3];
        g[4] = 2.0 * A[4];
        g[5] = 2.0 * A[5];
        return 0.5 * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) + A[3] * A[3] + A[4] * A[4] +
               A[5] * A[5];
    }

    // Scalar factors of Psi = Psi(J2): value, d Psi/dJ2 (= a1) and
    // d2 Psi/dJ2^2 (= a2), so that f = a1 g and Psi'' = a2 g g^T + a1 d2J2.
    // Returns false where Psi is flat (f = Psi'' = 0).
    AD_FN static bool psi_j2(const Phase &p, double J2, double &val, double &a1, double &a2) {
        if (p.sy == 0.0) {
            const double k = 3.0 * p.is0 * p.is0;  // u = k J2
            const double u = k * J2;
            const double c = 0.5 * p.pq;
            if (!(u > 0.0)) {
                if (p.n != 1.0) return false;
                val = 0.0;  // Psi = coef u
                a1 = p.coef * k;
                a2 = 0.0;
                return true;
            }
            const double uc1 = fm::pow_pos(u, c - 1.0);  // u^(c - 1)
            val = p.coef * uc1 * u;
            a1 = p.coef * c * uc1 * k;
            a2 = p.coef * c * (c - 1.0) * uc1 / u * k * k;
            return true;
        }
        const double q = sqrt(3.0 * J2);
        const double x = (q - p.sy) * p.is0;
        if (!(x > 0.0)) return false;
        const double n = p.pq - 1.0;
        const double xn1 = fm::pow_pos(x, n - 1.0);  // x^(n - 1)
        const double xn = xn1 * x;
        val = p.coef * xn * x;
        // dPsi/dq = coef pq x^n / sigma0 = eps0 x^n, d2Psi/dq2 = eps0 n x^(n-1) / sigma0;
        // dq/dJ2 = 3 / (2 q), d2q/dJ2^2 = -9 / (4 q^3)
        const double dq = 1.5 / q;
        const double p1 = p.coef * p.pq * p.is0 * xn;
        const double p2 = p.coef * p.pq * p.is0 * p.is0 * n * xn1;
        a1 = p1 * dq;
        a2 = p2 * dq * dq - p1 * dq * dq / q;
        return true;
    }

    AD_FN static double psi_grad(const Phase &p, const double *A, double *f) {
        double g[6];
        const double J2 = j2_grad(A, g);
        double val, a1, a2;
        if (!psi_j2(p, J2, val, a1, a2)) {
#pragma unroll
            for (int i = 0; i < 6; ++i) f[i] = 0.0;
            return 0.0;
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) f[i] = a1 * g[i];
        return val;
    }

    AD_FN static double psi_grad_hess(const Phase &p, const double *A, double *f, double *Hp) {
        double g[6];
        const double J2 = j2_grad(A, g);
        double val, a1, a2;
        if (!psi_j2(p, J2, val, a1, a2)) {
#pragma unroll
            for (int i = 0; i < 6; ++i) f[i] = 0.0;
#pragma unroll
            for (int i = 0; i < 21; ++i) Hp[i] = 0.0;
            return 0.0;
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) f[i] = a1 * g[i];
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                double d2 = 0.0;  // d2J2 / dA_i dA_j
                if (i < 3 && j < 3) d2 = (i == j ? 2.0 : -1.0) * (1.0 / 3.0);
                else if (i == j) d2 = 2.0;
                Hp[la::pk(i, j)] = a2 * g[i] * g[j] + a1 * d2;
            }
        return val;
    }

    AD_FN static void psi_hess(const Phase &p, const double *A, double *Hp) {
        double f[6];
        (void)psi_grad_hess(p, A, f, Hp);
    }

    // omega is quadratic: Kaa = C + Hm, Kae = -C, Kee = C
    AD_FN static void omega_hessian(const Phase &p, double *Kaa, double (&Kae)[6][6],
                                    double *Kee) {
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                double c = 0.0;
                if (i < 3 && j < 3) c = p.lam + (i == j ? 2.0 * p.mu : 0.0);
                else if (i == j) c = p.mu;
                Kae[i][j] = -c;
                if (j <= i) {
                    Kee[la::pk(i, j)] = c;
                    const double hm = i == j ? (i < 3 ? 2.0 : 1.0) * (1.0 / 3.0) * p.H : 0.0;
                    Kaa[la::pk(i, j)] = c + hm;
                }
            }
    }
};

}  // namespace automat

#pragma clang fp reassociate(off)
