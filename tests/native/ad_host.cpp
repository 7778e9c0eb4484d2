// Host build of the device AD layer, model potentials and fast math, for
// the CPU tests (compiled by tests/test_ad_host.py; test infrastructure).
#include <cstdint>

#include "ad.hpp"
#include "gsm_point.hpp"
#include "msgsm.hpp"

using namespace automat;
using M = MSGSM;

static M::Phase phase_from_row(const double *row) {
    M::Phase p{};
    p.kind = (int)row[0];
    p.E = row[1];
    p.nu = row[2];
    p.H = row[3];
    p.sy = row[4];
    p.s0 = row[5];
    p.e0 = row[6];
    p.n = row[7];
    M::derive(p);
    return p;
}

extern "C" {

void fm_vec(int which, const double *x, double *y, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        switch (which) {
        case 0: y[i] = fm::log(x[i]); break;
        case 1: y[i] = fm::exp(x[i]); break;
        case 2: y[i] = fm::rcp(x[i]); break;
        default: y[i] = fm::rsqrt(x[i]); break;
        }
    }
}

void fm_pow(const double *x, const double *e, double *y, int64_t n) {
    for (int64_t i = 0; i < n; ++i) y[i] = fm::pow_pos(x[i], e[i]);
}

// pow node of the AD layer with a constant exponent: value, first and
// second derivative in u
void ad_pow_const(const double *u, double e, double *val, double *d1, double *d2, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        ad::Var<0> a(u[i]);
        ad::HessRows<1, 1, 0> acc;
        val[i] = ad::sweep2(pow(a, e), ad::UnitDirs<1, 0>{}, acc);
        d1[i] = acc.g[0];
        d2[i] = acc.H[0][0];
    }
}

// Psi, f = dPsi/dA (first-order sweep) and Psi'' (one vector sweep).
void ad_psi(const double *row, const double *A, double *psi, double *f, double *Hp, double *f2) {
    M::Phase p = phase_from_row(row);
    *psi = M::psi_grad(p, A, f);
    double g[6];
    Leaves6<0> la(A);
    M::with_psi(la, p.sy, p.coef, p.is0, p.pq, p.sy == 0.0,
                [&](const auto &e) { ad::value_grad_hess6<0>(e, g, Hp); });
    for (int i = 0; i < 6; ++i) f2[i] = g[i];
}

// A = -d omega/da, sigma = d omega/deps, and the omega Hessian blocks.
void ad_omega(const double *row, const double *eps, const double *a, double *A, double *sig,
              double *Kaa, double *Kae, double *Kee) {
    M::Phase p = phase_from_row(row);
    M::gen_stress(p, eps, a, A);
    M::stress(p, eps, a, sig);
    double B[6][6];
    M::omega_hessian(p, Kaa, B, Kee);
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) Kae[i * 6 + j] = B[i][j];
}

// Parameter partials: d/d(sy, s0, e0, n) of w . dPsi/dA, and of
// grad omega . (u on eps, v on a) w.r.t. (E, nu, H).
void ad_params(const double *row, const double *A, const double *w, const double *eps,
               const double *a, const double *u, const double *v, double *gpsi, double *gom,
               double *ge) {
    M::Phase p = phase_from_row(row);
    M::psi_param_partials(p, A, w, gpsi);
    M::omega_hvp_params(p, eps, a, u, v, ge, gom);
}

// A generic expression over three leaves exercising every node type:
// value, gradient and Hessian (row-major 3x3) by one vector sweep.
void ad_generic(const double *x, double *val, double *g, double *H) {
    using namespace ad;
    Var<0> a(x[0]);
    Var<1> b(x[1]);
    Var<2> c(x[2]);
    auto e = pow(a * b + exp(c), sqrt(b) + 1.0) / log(a + 2.0) - sq(c - a) * pos(b - 0.5) +
             (-c) / (1.0 + a * a);
    HessRows<3, 3, 0> acc;
    *val = sweep2(e, UnitDirs<3, 0>{}, acc);
    for (int i = 0; i < 3; ++i) {
        g[i] = acc.g[i];
        for (int j = 0; j < 3; ++j) H[i * 3 + j] = acc.H[i][j];
    }
}

// Symmetric 6x6 Cholesky solve (packed lower input).
int la_solve(const double *Mp, double *b) {
    double L[21];
    for (int i = 0; i < 21; ++i) L[i] = Mp[i];
    const bool ok = la::cholesky6(L);
    la::chol_solve6(L, b);
    return ok ? 0 : -1;
}

}  // extern "C"
