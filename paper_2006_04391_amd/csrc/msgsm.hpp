// msgsm.hpp -- the Michel-Suquet elasto-viscoplastic GSM as two potentials
// written over the AD layer (paper: Section "Example", equations
// michel_suquet_omega and michel_suquet_psi).
//
//   omega(eps, a) = 1/2 (eps - a)^T C(E, nu) (eps - a) + 1/3 a^T Hm a,
//                   Hm = H diag(1, 1, 1, 1/2, 1/2, 1/2)
//   Psi(A)        = sigma0 eps0 / (n + 1) ((|dev A|_eq - sigma_y)^+ / sigma0)^(n + 1)
//
// a is the viscoplastic strain in engineering-shear Voigt form (the 1/2 on
// the shear entries of Hm is what engineering shears require). With the
// isotropic-hardening function equal to the constant sigma_y, the
// equivalent plastic strain never feeds back and is not carried; sigma_y
// enters Psi instead.
//
// Everything the solver needs is derived from these two scalar expressions
// by the AD layer: A = -d omega / d a and sigma = d omega / d eps by reverse
// sweeps, f = dPsi/dA and Psi'' by one forward-over-reverse sweep, the
// Hessian blocks of omega likewise, and parameter partials by sweeps seeded
// on the parameter leaves. The potentials are written once, over parameter
// arguments that are plain numbers on the hot path (derived per phase: the
// Lame constants, sigma0 eps0 / (n + 1), 1 / sigma0, n + 1) and expressions
// of parameter leaves when parameter derivatives are wanted.
#pragma once

#include "ad.hpp"

#pragma clang fp reassociate(on)

namespace automat {

// Six consecutive leaves BASE .. BASE+5.
template <int B>
struct Leaves6 {
    ad::Var<B + 0> c0;
    ad::Var<B + 1> c1;
    ad::Var<B + 2> c2;
    ad::Var<B + 3> c3;
    ad::Var<B + 4> c4;
    ad::Var<B + 5> c5;
    AD_FN Leaves6() {}
    AD_FN explicit Leaves6(const double *x) { set(x); }
    AD_FN void set(const double *x) {
        c0.val = x[0];
        c1.val = x[1];
        c2.val = x[2];
        c3.val = x[3];
        c4.val = x[4];
        c5.val = x[5];
    }
};

struct MSGSM {
    // Per-phase parameters: raw as in the ABI (kind 0 elastic, 1 flowing),
    // then the derived constants filled by derive().
    struct Phase {
        int kind;
        int reserved;
        double E, nu, H, sy, s0, e0, n;
        double lam, mu, coef, is0, pq;
    };

    // Leaf ids. omega: eps 0..5, a 6..11, E 12, nu 13, H 14.
    //           Psi:   A 0..5, sigma_y 6, sigma0 7, eps0 8, n 9.
    static constexpr int OM_EPS = 0, OM_A = 6, OM_E = 12, OM_NU = 13, OM_H = 14;
    static constexpr int PS_A = 0, PS_SY = 6, PS_S0 = 7, PS_E0 = 8, PS_N = 9;

    template <class TE, class TN>
    AD_FN static auto lame_lambda(const TE &E, const TN &nu) {
        using namespace ad;
        return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    }
    template <class TE, class TN>
    AD_FN static auto lame_mu(const TE &E, const TN &nu) {
        using namespace ad;
        return E / (2.0 * (1.0 + nu));
    }

    AD_FN static void derive(Phase &p) {
        p.lam = lame_lambda(p.E, p.nu);
        p.mu = lame_mu(p.E, p.nu);
        p.coef = p.s0 * p.e0 / (p.n + 1.0);
        p.is0 = 1.0 / p.s0;
        p.pq = p.n + 1.0;
    }

    // The free energy over Lame constants lam, mu and hardening modulus H.
    template <class EL, class AL, class TL, class TM, class TH>
    AD_FN static auto omega(const EL &e, const AL &a, const TL &lam, const TM &mu, const TH &H) {
        using namespace ad;
        auto e0 = e.c0 - a.c0;
        auto e1 = e.c1 - a.c1;
        auto e2 = e.c2 - a.c2;
        auto e3 = e.c3 - a.c3;
        auto e4 = e.c4 - a.c4;
        auto e5 = e.c5 - a.c5;
        auto elastic = 0.5 * lam * sq(e0 + e1 + e2) + mu * (sq(e0) + sq(e1) + sq(e2)) +
                       0.5 * mu * (sq(e3) + sq(e4) + sq(e5));
        auto hardening = H * (1.0 / 3.0) *
                         (sq(a.c0) + sq(a.c1) + sq(a.c2) + 0.5 * (sq(a.c3) + sq(a.c4) + sq(a.c5)));
        return elastic + hardening;
    }

    // J2 of a plain-Voigt stress-like 6-vector of leaves. The deviator is
    // written as s1 = (2 A1 - A2 - A3) / 3 etc., exactly zero for a
    // hydrostatic state, so such a state does not flow at all.
    template <class AL>
    AD_FN static auto j2(const AL &A) {
        using namespace ad;
        constexpr double third = 1.0 / 3.0;
        auto s0 = (2.0 * A.c0 - A.c1 - A.c2) * third;
        auto s1 = (2.0 * A.c1 - A.c0 - A.c2) * third;
        auto s2 = (2.0 * A.c2 - A.c0 - A.c1) * third;
        return 0.5 * (sq(s0) + sq(s1) + sq(s2)) + sq(A.c3) + sq(A.c4) + sq(A.c5);
    }

    // The force potential over coef = sigma0 eps0 / (n + 1), is0 = 1 / sigma0,
    // pq = n + 1 and sigma_y, handed to f(expr). Without a yield threshold
    // the power of the equivalent stress is written as a power of 3 J2,
    // which avoids the square root (and its cone point) altogether; with a
    // threshold the positive part of (q - sigma_y) is taken.
    template <class AL, class TY, class TC, class TI, class TP, class F>
    AD_FN static void with_psi(const AL &A, const TY &sy, const TC &coef, const TI &is0,
                               const TP &pq, bool no_threshold, F &&f) {
        using namespace ad;
        if (no_threshold) {
            auto u = 3.0 * j2(A) * sq(is0);
            f(coef * pow(u, 0.5 * pq));
        } else {
            auto x = pos(sqrt(3.0 * j2(A)) - sy) * is0;
            f(coef * pow(x, pq));
        }
    }

    AD_FN static bool flows(const Phase &p) { return p.kind != 0; }

    // ---- first-order quantities used in the Newton loop -------------------

    // A = -d omega / d a at (eps, a)
    AD_FN static void gen_stress(const Phase &p, const double *eps, const double *a, double *A) {
        Leaves6<OM_EPS> le(eps);
        Leaves6<OM_A> la(a);
        ad::Grad<6, OM_A> g;
        ad::value_grad(omega(le, la, p.lam, p.mu, p.H), g);
#pragma unroll
        for (int i = 0; i < 6; ++i) A[i] = -g.g[i];
    }

    // sigma = d omega / d eps at (eps, a)
    AD_FN static void stress(const Phase &p, const double *eps, const double *a, double *sig) {
        Leaves6<OM_EPS> le(eps);
        Leaves6<OM_A> la(a);
        ad::Grad<6, OM_EPS> g;
        ad::value_grad(omega(le, la, p.lam, p.mu, p.H), g);
#pragma unroll
        for (int i = 0; i < 6; ++i) sig[i] = g.g[i];
    }

    // Psi(A) and f = dPsi/dA
    AD_FN static double psi_grad(const Phase &p, const double *A, double *f) {
        Leaves6<PS_A> la(A);
        double val = 0.0;
        ad::Grad<6, PS_A> g;
        with_psi(la, p.sy, p.coef, p.is0, p.pq, p.sy == 0.0,
                 [&](const auto &e) { val = ad::value_grad(e, g); });
#pragma unroll
        for (int i = 0; i < 6; ++i) f[i] = g.g[i];
        return val;
    }

    // Psi(A), f = dPsi/dA and Psi''(A) (packed lower triangle) by one sweep
    AD_FN static double psi_grad_hess(const Phase &p, const double *A, double *f, double *Hp) {
        Leaves6<PS_A> la(A);
        double val = 0.0;
        with_psi(la, p.sy, p.coef, p.is0, p.pq, p.sy == 0.0,
                 [&](const auto &e) { val = ad::value_grad_hess6<PS_A>(e, f, Hp); });
        return val;
    }

    // Psi''(A), packed lower triangle, by one sweep
    AD_FN static void psi_hess(const Phase &p, const double *A, double *Hp) {
        Leaves6<PS_A> la(A);
        double g[6];
        with_psi(la, p.sy, p.coef, p.is0, p.pq, p.sy == 0.0,
                 [&](const auto &e) { ad::value_grad_hess6<PS_A>(e, g, Hp); });
    }

    // ---- second-order quantities for the vector-Jacobian product ----------

    // Psi''(A) w by one forward-over-reverse sweep (same form of Psi as the
    // Newton solve).
    AD_FN static void psi_hvp(const Phase &p, const double *A, const double *w, double *out) {
        Leaves6<PS_A> la(A);
        ad::VecDir<6, PS_A> dir;
#pragma unroll
        for (int i = 0; i < 6; ++i) dir.d[i] = w[i];
        ad::GradT<6, PS_A> acc;
        with_psi(la, p.sy, p.coef, p.is0, p.pq, p.sy == 0.0,
                 [&](const auto &e) { ad::sweep2(e, dir, acc); });
#pragma unroll
        for (int i = 0; i < 6; ++i) out[i] = acc.g[i];
    }

    // (omega_ee u, omega_ae u): the tangent of the gradient of omega in the
    // direction u on eps.
    AD_FN static void omega_hvp_eps(const Phase &p, const double *eps, const double *a,
                                    const double *u, double *ge, double *ga) {
        Leaves6<OM_EPS> le(eps);
        Leaves6<OM_A> la(a);
        ad::VecDir<6, OM_EPS> dir;
#pragma unroll
        for (int i = 0; i < 6; ++i) dir.d[i] = u[i];
        ad::GradT<12, OM_EPS> acc;
        ad::sweep2(omega(le, la, p.lam, p.mu, p.H), dir, acc);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            ge[i] = acc.g[i];
            ga[i] = acc.g[6 + i];
        }
    }

    // With direction (u on eps, v on a) and E, nu, H as leaves:
    // ge = d/deps (grad omega . (u, v)), gp = d/d(E, nu, H) (grad omega . (u, v)).
    AD_FN static void omega_hvp_params(const Phase &p, const double *eps, const double *a,
                                       const double *u, const double *v, double *ge,
                                       double *gp) {
        Leaves6<OM_EPS> le(eps);
        Leaves6<OM_A> la(a);
        ad::Var<OM_E> E(p.E);
        ad::Var<OM_NU> nu(p.nu);
        ad::Var<OM_H> H(p.H);
        ad::VecDir<12, OM_EPS> dir;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            dir.d[i] = u[i];
            dir.d[6 + i] = v[i];
        }
        ad::GradT<15, OM_EPS> acc;
        ad::sweep2(omega(le, la, lame_lambda(E, nu), lame_mu(E, nu), H), dir, acc);
#pragma unroll
        for (int i = 0; i < 6; ++i) ge[i] = acc.g[i];
        gp[0] = acc.g[OM_E];
        gp[1] = acc.g[OM_NU];
        gp[2] = acc.g[OM_H];
    }

    // d/d(sigma_y, sigma0, eps0, n) of (w . dPsi/dA) at fixed A. Uses the
    // thresholded form of Psi, whose sigma_y-derivative is the one-sided
    // one at sigma_y = 0.
    AD_FN static void psi_param_partials(const Phase &p, const double *A, const double *w,
                                         double *gp) {
        using namespace ad;
        Leaves6<PS_A> la(A);
        Var<PS_SY> sy(p.sy);
        Var<PS_S0> s0(p.s0);
        Var<PS_E0> e0(p.e0);
        Var<PS_N> n(p.n);
        VecDir<6, PS_A> dir;
#pragma unroll
        for (int i = 0; i < 6; ++i) dir.d[i] = w[i];
        GradT<4, PS_SY> acc;
        auto coef = s0 * e0 / (n + 1.0);
        auto is0 = 1.0 / s0;
        auto pq = n + 1.0;
        with_psi(la, sy, coef, is0, pq, false, [&](const auto &e) { sweep2(e, dir, acc); });
#pragma unroll
        for (int i = 0; i < 4; ++i) gp[i] = acc.g[i];
    }

    // Hessian blocks of omega: Kaa = d2/da2 (packed), Kae = d2/(da deps)
    // (row a, column eps), Kee = d2/deps2 (packed). omega is quadratic, so
    // they do not depend on the point; they are taken at (0, 0).
    AD_FN static void omega_hessian(const Phase &p, double *Kaa, double (&Kae)[6][6],
                                    double *Kee) {
        const double z[6] = {0, 0, 0, 0, 0, 0};
        Leaves6<OM_EPS> le(z);
        Leaves6<OM_A> la(z);
        auto om = omega(le, la, p.lam, p.mu, p.H);
        double g[6];
        ad::value_grad_hess6<OM_A>(om, g, Kaa);
        ad::value_grad_hess6<OM_EPS>(om, g, Kee);
        ad::hessian_block6<OM_A, OM_EPS>(om, Kae);
    }
};

}  // namespace automat

#pragma clang fp reassociate(off)
