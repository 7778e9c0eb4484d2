"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle (never the GPU path) against an independent
route: a closed form, a textbook reduction, finite differences, an invariant
the paper states (Theorem 1) or a physical law. A plausible mistake in the
oracle (a dropped hardening term, a wrong shear factor, a transposed
Jacobian, a sign) fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs
from tests import _tensor as T

HERE = os.path.dirname(os.path.abspath(__file__))


def _phase_row(**kw):
    base = dict(kind=1, E=2500.0, nu=0.35, H=0.0, sigma_y=0.0, sigma0=50.0, eps0=1e-3, n=5.0)
    base.update(kw)
    return base


def _single(eps, a_old, ph, h=0.1, tol=1e-12, max_iter=50, tangent=False, flags=0):
    eps = np.asarray(eps, dtype=np.float64).reshape(6, -1)
    a_old = np.asarray(a_old, dtype=np.float64).reshape(6, -1)
    phase = np.zeros(eps.shape[1], dtype=np.uint8)
    return oracle.evaluate(eps, a_old, phase, [ph], h=h, tol=tol, max_iter=max_iter,
                           tangent=tangent, flags=flags)


# ---------------------------------------------------------------------------
# parameters and the elastic closed form
# ---------------------------------------------------------------------------

def test_paper_parameter_table_golden():
    """The paper preset reproduces Table misu_parameters (GPa -> MPa)."""
    g = json.load(open(os.path.join(HERE, "golden", "misu_parameters.json")))
    m, f = inputs.paper_phases()
    al = g["aluminum"]
    assert m["E"] == al["E"] * 1000 and m["nu"] == al["nu"]
    assert m["sigma_y"] == al["sigma_Y"] and m["H"] == al["H"] * 1000
    assert m["eps0"] == al["eps0_dot"] and m["sigma0"] == al["sigma_d"] and m["n"] == al["n"]
    assert f["E"] == g["al2o3"]["E"] * 1000 and f["nu"] == g["al2o3"]["nu"]
    assert m["kind"] == 1 and f["kind"] == 0


def test_elastic_phase_is_hooke_tensor_form():
    """Elastic phase: sigma = lambda tr(e) I + 2 mu e with e = eps - a_n
    (tensor form, independent of the Voigt matrix), a_{n+1} = a_n bitwise,
    tangent = the Voigt image of the isotropic stiffness tensor."""
    rng = np.random.default_rng(11)
    n = 64
    eps = rng.normal(0, 1e-3, (6, n))
    a_old = rng.normal(0, 1e-4, (6, n))
    ph = dict(kind=0, E=72000.0, nu=0.22, H=0.0, sigma_y=0.0, sigma0=1.0, eps0=0.0, n=1.0)
    r = oracle.evaluate(eps, a_old, np.zeros(n, np.uint8), [ph], tangent=True)
    sig_ref = T.stress_voigt(T.hooke(72000.0, 0.22, T.strain_tensor(eps - a_old)))
    np.testing.assert_allclose(r["sigma"], sig_ref, rtol=1e-13, atol=1e-13 * np.abs(sig_ref).max())
    assert np.array_equal(r["a_out"], a_old)
    assert np.all(r["iters"] == 0)
    lam, mu = T.lame(72000.0, 0.22)
    C4 = lam * np.einsum("ij,kl->ijkl", np.eye(3), np.eye(3)) + 2 * mu * T.identity4_sym()
    Cv = T.voigt_matrix_from_tensor4(C4)
    np.testing.assert_allclose(r["tangent"][:, 0].reshape(6, 6), Cv, rtol=1e-14, atol=1e-9)


def test_uniaxial_stress_and_shear_recover_E_nu():
    """Physical pin of the Voigt convention: the uniaxial-stress strain state
    (1, -nu, -nu, 0, 0, 0) s gives sigma = (E s, 0, ...); an engineering shear
    gamma_12 = g gives sigma_12 = mu g = E g / (2 (1 + nu))."""
    E, nu, s, g = 72000.0, 0.22, 1e-3, 2e-3
    ph = dict(kind=0, E=E, nu=nu, H=0.0, sigma_y=0.0, sigma0=1.0, eps0=0.0, n=1.0)
    r = _single([s, -nu * s, -nu * s, 0, 0, 0], np.zeros(6), ph)
    np.testing.assert_allclose(r["sigma"][:, 0], [E * s, 0, 0, 0, 0, 0], atol=1e-12 * E * s)
    r = _single([0, 0, 0, 0, 0, g], np.zeros(6), ph)
    np.testing.assert_allclose(r["sigma"][5, 0], E * g / (2 * (1 + nu)), rtol=1e-15)


def test_hydrostatic_strain_is_elastic_in_matrix():
    """q = 0: no flow (F vanishes exactly), zero updates, sigma = C eps."""
    ph = _phase_row()
    r = _single([1e-3, 1e-3, 1e-3, 0, 0, 0], np.zeros(6), ph)
    assert r["iters"][0] == 0
    assert np.array_equal(r["a_out"][:, 0], np.zeros(6))
    lam, mu = T.lame(2500.0, 0.35)
    np.testing.assert_allclose(r["sigma"][:3, 0], (3 * lam + 2 * mu) * 1e-3, rtol=1e-14)


# ---------------------------------------------------------------------------
# the textbook radial return (the paper's "conventional strategy")
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("preset", ["config", "paper", "hardening_only", "threshold_only"])
def test_radial_return_agreement(preset):
    """The full 6-D Newton agrees with the scalar J2 return mapping (the
    conventional strategy the paper automates; it states both give the same
    results to machine precision)."""
    rng = np.random.default_rng(3)
    n = 2000
    if preset == "config":
        ph = _phase_row()
        e11, std = 5e-3, 2e-4
    elif preset == "paper":
        ph = inputs.paper_phases()[0]
        e11, std = 1e-2, 2e-3
    elif preset == "hardening_only":
        ph = _phase_row(H=1800.0, eps0=1.0, n=3.0)
        e11, std = 2e-2, 3e-3
    else:
        ph = _phase_row(sigma_y=5.0, eps0=0.5, n=2.5)
        e11, std = 2e-2, 3e-3
    eps = inputs.uniaxial_strain(n, e11, std, rng)
    a_old = inputs.deviatoric_draw(n, 1e-3 if preset != "config" else 1e-4, rng)
    r = oracle.evaluate(eps, a_old, np.zeros(n, np.uint8), [ph], h=0.1)
    assert np.all(r["iters"] >= 0)
    sig, a_new, q, q_tr = T.radial_return(eps, a_old, ph["E"], ph["nu"], ph["H"], ph["sigma_y"],
                                          ph["sigma0"], ph["eps0"], ph["n"], 0.1)
    rel_s = np.abs(r["sigma"] - sig).max(0) / np.abs(sig).max(0)
    rel_a = np.abs(r["a_out"] - a_new).max(0) / np.abs(a_new).max(0)
    assert rel_s.max() <= 1e-13, rel_s.max()
    assert rel_a.max() <= 1e-12, rel_a.max()
    # the increment itself (not only a_{n+1} = a_n + increment)
    d_or = r["a_out"] - a_old
    d_rr = a_new - a_old
    rel_d = np.abs(d_or - d_rr).max(0) / np.maximum(np.abs(d_rr).max(0), 1e-300)
    flowing = q < q_tr * (1 - 1e-12)
    assert rel_d[flowing].max() <= 1e-9, rel_d[flowing].max()


def test_linear_viscous_one_update_closed_form():
    """n = 1, sigma_y = 0, H = 0: f is linear in A, so Newton lands on the
    root in exactly one update, with q = q_trial / (1 + 3 mu h eps0 / sigma0)."""
    rng = np.random.default_rng(5)
    n = 200
    ph = _phase_row(n=1.0, eps0=0.3)
    eps = inputs.uniaxial_strain(n, 1e-2, 2e-3, rng)
    r = oracle.evaluate(eps, np.zeros((6, n)), np.zeros(n, np.uint8), [ph], h=0.1)
    assert np.all(r["iters"] == 1)
    lam, mu = T.lame(2500.0, 0.35)
    q_tr = T.mises(T.dev(T.hooke(2500.0, 0.35, T.strain_tensor(eps))))
    q = T.mises(T.dev(T.stress_tensor(r["sigma"])))
    np.testing.assert_allclose(q, q_tr / (1 + 3 * mu * 0.1 * 0.3 / 50.0), rtol=1e-13)


def test_relaxation_converges_first_order_to_ode_solution():
    """Stress relaxation at fixed strain (H = sigma_y = 0) has the exact
    solution q(t)^(1-n) = q0^(1-n) + 3 mu eps0 (n-1) sigma0^-n t. Repeated
    implicit-Euler steps converge to it at first order in h."""
    ph = _phase_row()
    lam, mu = T.lame(2500.0, 0.35)
    e11, Tend, nexp = 5e-2, 1.0, 5.0
    q0 = 2 * mu * e11
    q_exact = (q0 ** (1 - nexp) + 3 * mu * 1e-3 * (nexp - 1) * 50.0 ** (-nexp) * Tend) ** (1 / (1 - nexp))
    errs = []
    for N in (10, 20, 40, 80):
        a = np.zeros((6, 1))
        eps = np.array([e11, 0, 0, 0, 0, 0.0]).reshape(6, 1)
        for _ in range(N):
            r = _single(eps, a, ph, h=Tend / N)
            assert r["iters"][0] >= 0
            a = r["a_out"]
        q = T.mises(T.dev(T.stress_tensor(r["sigma"])))[0]
        errs.append(abs(q - q_exact))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert errs[0] / q_exact < 0.1
    for rr in ratios:
        assert 1.8 < rr < 2.2, ratios


# ---------------------------------------------------------------------------
# derivatives of the force potential
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("preset", ["config", "paper", "n1"])
def test_force_potential_derivatives_fd(preset):
    """f = dPsi/dA and Psi'' = df/dA against central differences."""
    ph = {"config": _phase_row(), "paper": inputs.paper_phases()[0],
          "n1": _phase_row(n=1.0, sigma_y=3.0)}[preset]
    row = inputs.phases_array([ph])[0]
    rng = np.random.default_rng(7)
    for _ in range(20):
        A = rng.normal(0, 60.0, 6)
        psi, f, P2 = oracle.force_potential(row, A)
        step = 1e-6 * np.abs(A).max()
        fd_f = np.zeros(6)
        fd_P = np.zeros((6, 6))
        for j in range(6):
            dA = np.zeros(6)
            dA[j] = step
            pp, fp, _ = oracle.force_potential(row, A + dA)
            pm, fm, _ = oracle.force_potential(row, A - dA)
            fd_f[j] = (pp - pm) / (2 * step)
            fd_P[:, j] = (fp - fm) / (2 * step)
        np.testing.assert_allclose(f, fd_f, rtol=1e-6, atol=1e-8 * np.abs(f).max())
        np.testing.assert_allclose(P2, fd_P, rtol=1e-5, atol=1e-6 * np.abs(P2).max())
        np.testing.assert_allclose(P2, P2.T, rtol=0, atol=1e-14 * np.abs(P2).max())


def test_dissipation_homogeneity_and_incompressibility():
    """With sigma_y = 0, Psi is homogeneous of degree n+1 in A, so the
    dissipation A_{n+1} . Delta = h A . f = h (n+1) Psi(A_{n+1}) >= 0;
    the increment is trace-free (plastic incompressibility) and the free
    energy does not increase."""
    ps = inputs.points_random(500, seed=9, e11=2e-2, std=3e-3)
    ph = _phase_row(eps0=0.2)
    phase = np.zeros(ps.n, np.uint8)
    r = oracle.evaluate(ps.eps, ps.a_old, phase, [ph], h=0.1)
    d = r["a_out"] - ps.a_old
    A_t = T.hooke(2500.0, 0.35, T.strain_tensor(ps.eps - r["a_out"]))
    A = T.stress_voigt(A_t)
    diss = np.einsum("ij,ij->j", A, d)
    row = inputs.phases_array([ph])[0]
    psi = np.array([oracle.force_potential(row, A[:, i])[0] for i in range(ps.n)])
    np.testing.assert_allclose(diss, 0.1 * 6.0 * psi, rtol=1e-9)
    assert np.all(diss >= 0)
    # rounding of a_{n+1} - a_n is at the scale of |a_{n+1}|
    assert np.abs(d[:3].sum(0)).max() <= 8 * np.finfo(float).eps * np.abs(r["a_out"]).max()

    def omega(a):
        e = T.strain_tensor(ps.eps - a)
        return 0.5 * np.einsum("ij...,ij...->...", T.hooke(2500.0, 0.35, e), e)
    assert np.all(omega(r["a_out"]) <= omega(ps.a_old) * (1 + 1e-15))


def test_rotation_equivariance():
    """Isotropy: rotating eps and a_n rotates sigma and a_{n+1}."""
    rng = np.random.default_rng(13)
    ph = inputs.paper_phases()[0]
    n = 50
    eps = inputs.uniaxial_strain(n, 1e-2, 3e-3, rng)
    a_old = inputs.deviatoric_draw(n, 1e-3, rng)
    r0 = oracle.evaluate(eps, a_old, np.zeros(n, np.uint8), [ph])
    R = T.random_rotation(rng)
    rot = lambda t: np.einsum("ik,kl...,jl->ij...", R, t, R)
    eps_r = T.strain_voigt(rot(T.strain_tensor(eps)))
    a_r = T.strain_voigt(rot(T.strain_tensor(a_old)))
    r1 = oracle.evaluate(eps_r, a_r, np.zeros(n, np.uint8), [ph])
    sig_exp = T.stress_voigt(rot(T.stress_tensor(r0["sigma"])))
    a_exp = T.strain_voigt(rot(T.strain_tensor(r0["a_out"])))
    np.testing.assert_allclose(r1["sigma"], sig_exp, rtol=0, atol=1e-11 * np.abs(sig_exp).max())
    np.testing.assert_allclose(r1["a_out"], a_exp, rtol=0, atol=1e-11 * np.abs(a_exp).max())


def test_theorem1_jacobian_eigenvalues_nonpositive():
    """Theorem 1: the Jacobian -Psi''(A) K of the right-hand side has real,
    non-positive eigenvalues."""
    rng = np.random.default_rng(17)
    for ph in (inputs.paper_phases()[0], _phase_row(H=500.0, sigma_y=2.0)):
        row = inputs.phases_array([ph])[0]
        lam, mu = T.lame(ph["E"], ph["nu"])
        C4 = lam * np.einsum("ij,kl->ijkl", np.eye(3), np.eye(3)) + 2 * mu * T.identity4_sym()
        K = T.voigt_matrix_from_tensor4(C4) + (2 / 3) * ph["H"] * np.diag([1, 1, 1, .5, .5, .5])
        for _ in range(50):
            A = rng.normal(0, 200.0, 6)
            _, _, P2 = oracle.force_potential(row, A)
            ev = np.linalg.eigvals(-P2 @ K)
            scale = np.abs(P2 @ K).max()
            assert np.abs(ev.imag).max() <= 1e-9 * scale
            assert ev.real.max() <= 1e-12 * scale


# ---------------------------------------------------------------------------
# consistent tangent
# ---------------------------------------------------------------------------

def _fd_tangent(eps, a_old, ph, h=0.1, rel=1e-7):
    n = eps.shape[1]
    out = np.zeros((36, n))
    for j in range(6):
        st = rel * np.abs(eps).max(0)
        ep = eps.copy()
        em = eps.copy()
        ep[j] += st
        em[j] -= st
        sp = _single(ep, a_old, ph, h=h, tol=1e-14)["sigma"]
        sm = _single(em, a_old, ph, h=h, tol=1e-14)["sigma"]
        for i in range(6):
            out[i * 6 + j] = (sp[i] - sm[i]) / (2 * st)
    return out


@pytest.mark.parametrize("preset", ["config", "paper"])
def test_tangent_fd_symmetry_definiteness(preset):
    rng = np.random.default_rng(19)
    n = 100
    if preset == "config":
        ph, e11, std = _phase_row(eps0=0.1), 2e-2, 3e-3
    else:
        ph, e11, std = inputs.paper_phases()[0], 1e-2, 2e-3
    eps = inputs.uniaxial_strain(n, e11, std, rng)
    a_old = inputs.deviatoric_draw(n, 1e-3, rng)
    r = _single(eps, a_old, ph, tangent=True, tol=1e-14)
    C = r["tangent"]
    fd = _fd_tangent(eps, a_old, ph)
    rel = np.abs(C - fd).max(0) / np.abs(C).max(0)
    assert rel.max() <= 1e-6, rel.max()
    for i in range(n):
        M = C[:, i].reshape(6, 6)
        assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
        assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_tangent_woodbury_identity_no_hardening():
    """H = 0: C_{n+1} = (C^-1 + h Psi''(sigma_{n+1}))^-1 (the IFT tangent
    rewritten; sigma = A when H = 0)."""
    rng = np.random.default_rng(23)
    ph = _phase_row(eps0=0.1, sigma_y=2.0)
    row = inputs.phases_array([ph])[0]
    n = 60
    eps = inputs.uniaxial_strain(n, 2e-2, 3e-3, rng)
    a_old = inputs.deviatoric_draw(n, 1e-3, rng)
    r = _single(eps, a_old, ph, tangent=True)
    lam, mu = T.lame(2500.0, 0.35)
    C4 = lam * np.einsum("ij,kl->ijkl", np.eye(3), np.eye(3)) + 2 * mu * T.identity4_sym()
    Ce = T.voigt_matrix_from_tensor4(C4)
    for i in range(n):
        _, _, P2 = oracle.force_potential(row, r["sigma"][:, i])
        ref = np.linalg.inv(np.linalg.inv(Ce) + 0.1 * P2)
        M = r["tangent"][:, i].reshape(6, 6)
        assert np.abs(M - ref).max() <= 1e-12 * np.abs(ref).max()


def test_tangent_radial_return_closed_form():
    """H = 0: the consistent tangent of the J2 return mapping,
    C = kappa I(x)I + 2 mu theta I_dev + 2 mu (beta - theta) N(x)N,
    theta = q / q_tr, beta = 1 / (1 + 3 mu h eps0 n (q - sigma_y)^(n-1) / sigma0^n),
    N the unit trial deviator (tensor form, converted to Voigt)."""
    rng = np.random.default_rng(29)
    ph = _phase_row(eps0=0.1, sigma_y=3.0, n=4.2)
    n = 40
    eps = inputs.uniaxial_strain(n, 2e-2, 3e-3, rng)
    a_old = inputs.deviatoric_draw(n, 1e-3, rng)
    r = _single(eps, a_old, ph, tangent=True)
    lam, mu = T.lame(2500.0, 0.35)
    kappa = lam + 2 * mu / 3
    _, _, q, q_tr = T.radial_return(eps, a_old, 2500.0, 0.35, 0.0, 3.0, 50.0, 0.1, 4.2, 0.1)
    s_tr = T.dev(T.hooke(2500.0, 0.35, T.strain_tensor(eps - a_old)))
    I = np.eye(3)
    Idev = T.identity4_sym() - np.einsum("ij,kl->ijkl", I, I) / 3
    for i in range(n):
        theta = q[i] / q_tr[i]
        beta = 1.0 / (1 + 3 * mu * 0.1 * 0.1 * 4.2 * (q[i] - 3.0) ** 3.2 / 50.0 ** 4.2)
        Nt = s_tr[:, :, i] / np.sqrt(np.sum(s_tr[:, :, i] ** 2))
        C4 = (kappa * np.einsum("ij,kl->ijkl", I, I) + 2 * mu * theta * Idev
              + 2 * mu * (beta - theta) * np.einsum("ij,kl->ijkl", Nt, Nt))
        ref = T.voigt_matrix_from_tensor4(C4)
        M = r["tangent"][:, i].reshape(6, 6)
        assert np.abs(M - ref).max() <= 1e-10 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# backward (vector-Jacobian product)
# ---------------------------------------------------------------------------

def _loss(eps, a_old, phases, gs, ga, h=0.1):
    r = oracle.evaluate(eps, a_old, np.zeros(eps.shape[1], np.uint8), phases, h=h, tol=1e-15,
                        max_iter=100)
    return (gs * r["sigma"]).sum() + (ga * r["a_out"]).sum()


@pytest.mark.parametrize("preset", ["config", "paper", "elastic"])
def test_backward_fd(preset):
    """grad eps, grad a_n and every parameter gradient against central
    differences of <g_sigma, sigma> + <g_a, a_{n+1}> through the forward
    oracle."""
    rng = np.random.default_rng(31)
    if preset == "config":
        ph = _phase_row(eps0=0.1, H=300.0, sigma_y=2.0)
        e11, std = 2e-2, 3e-3
    elif preset == "paper":
        ph = inputs.paper_phases()[0]
        e11, std = 1e-2, 2e-3
    else:
        ph = inputs.config_phases()[1]
        e11, std = 2e-3, 1e-4
    n = 1
    eps = inputs.uniaxial_strain(n, e11, std, rng)
    a_old = inputs.deviatoric_draw(n, 1e-3, rng)
    gs = rng.normal(size=(6, n))
    ga = rng.normal(size=(6, n)) * 1e4
    r = oracle.evaluate(eps, a_old, np.zeros(n, np.uint8), [ph], tol=1e-15, max_iter=100)
    b = oracle.backward(eps, a_old, r["a_out"], np.zeros(n, np.uint8), [ph], 0.1, gs, ga)
    for j in range(6):
        st = 1e-7 * np.abs(eps).max()
        ep, em = eps.copy(), eps.copy()
        ep[j] += st
        em[j] -= st
        fd = (_loss(ep, a_old, [ph], gs, ga) - _loss(em, a_old, [ph], gs, ga)) / (2 * st)
        assert abs(fd - b["grad_eps"][j, 0]) <= 1e-6 * np.abs(b["grad_eps"]).max()
        st = 1e-7 * np.abs(eps).max()
        ap, am = a_old.copy(), a_old.copy()
        ap[j] += st
        am[j] -= st
        fd = (_loss(eps, ap, [ph], gs, ga) - _loss(eps, am, [ph], gs, ga)) / (2 * st)
        assert abs(fd - b["grad_a_old"][j, 0]) <= 1e-6 * np.abs(b["grad_a_old"]).max()
    keys = oracle.GRAD_KEYS if ph["kind"] == 1 else ("E", "nu")
    for k in keys:
        kk = oracle.GRAD_KEYS.index(k)
        base = ph[k]
        st = 1e-6 * abs(base) if base != 0 else 1e-6
        pp = dict(ph, **{k: base + st})
        pm = dict(ph, **{k: base - st}) if base - st >= 0 or k == "nu" else dict(ph)
        den = (2 * st) if pm is not ph and pm[k] != base else st
        fd = (_loss(eps, a_old, [pp], gs, ga) - _loss(eps, a_old, [pm], gs, ga)) / den
        got = b["grad_params"][0, kk]
        scale = max(abs(got), abs(fd), 1e-300)
        assert abs(fd - got) <= 2e-5 * scale + 1e-9 * np.abs(b["grad_params"]).max(), (k, fd, got)


def test_backward_adjoint_identity_and_elastic_E():
    """<g_sigma, C deps> = <grad eps, deps> with g_a = 0; for the elastic
    phase d sigma / dE = sigma / E exactly."""
    rng = np.random.default_rng(37)
    ph = inputs.paper_phases()
    n = 100
    ps = inputs.points_random(n, seed=41, phases=ph, e11=1e-2, std=2e-3, a_std=1e-3)
    r = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ph, tangent=True)
    gs = rng.normal(size=(6, n))
    b = oracle.backward(ps.eps, ps.a_old, r["a_out"], ps.phase, ph, 0.1, gs, None)
    d = rng.normal(size=(6, n))
    Cd = np.einsum("ijn,jn->in", r["tangent"].reshape(6, 6, n), d)
    lhs = np.einsum("in,in->n", gs, Cd)
    rhs = np.einsum("in,in->n", b["grad_eps"], d)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-11, atol=1e-11 * np.abs(lhs).max())
    el = ps.phase == 1
    exp_E = np.sum(gs[:, el] * r["sigma"][:, el]) / ph[1]["E"]
    np.testing.assert_allclose(b["grad_params"][1, 0], exp_E, rtol=1e-12)


# ---------------------------------------------------------------------------
# forward (Jacobian-vector) product
# ---------------------------------------------------------------------------

def _outputs(eps, a_old, phases, h=0.1):
    r = oracle.evaluate(eps, a_old, np.zeros(eps.shape[1], np.uint8), phases, h=h, tol=1e-15,
                        max_iter=100)
    return r["sigma"], r["a_out"]


@pytest.mark.parametrize("preset", ["config", "paper", "linear", "elastic"])
def test_jvp_central_differences(preset):
    """d sigma and d a_{n+1} in a random direction of (eps, a_n) and along
    each parameter against central differences of the forward oracle."""
    rng = np.random.default_rng(43)
    if preset == "config":
        ph = _phase_row(eps0=0.1, H=300.0, sigma_y=2.0)
        e11, std = 2e-2, 3e-3
    elif preset == "paper":
        ph = inputs.paper_phases()[0]
        e11, std = 1e-2, 2e-3
    elif preset == "linear":
        ph = _phase_row(n=1.0, eps0=0.1)
        e11, std = 2e-2, 3e-3
    else:
        ph = inputs.config_phases()[1]
        e11, std = 2e-3, 1e-4
    n = 3
    eps = inputs.uniaxial_strain(n, e11, std, rng)
    a_old = inputs.deviatoric_draw(n, 1e-3, rng)
    r = oracle.evaluate(eps, a_old, np.zeros(n, np.uint8), [ph], tol=1e-15, max_iter=100)
    de = rng.normal(size=(6, n)) * np.abs(eps).max()
    da = rng.normal(size=(6, n)) * 1e-3
    j = oracle.jvp(eps, r["a_out"], np.zeros(n, np.uint8), [ph], 0.1, d_eps=de, d_a_old=da)
    st = 1e-6
    sp, ap = _outputs(eps + st * de, a_old + st * da, [ph])
    sm, am = _outputs(eps - st * de, a_old - st * da, [ph])
    for got, fd in ((j["d_sigma"], (sp - sm) / (2 * st)), (j["d_a_new"], (ap - am) / (2 * st))):
        assert np.abs(got - fd).max() <= 1e-6 * max(np.abs(fd).max(), 1e-300), (got, fd)
    keys = oracle.GRAD_KEYS if ph["kind"] == 1 else ("E", "nu")
    for k in keys:
        kk = oracle.GRAD_KEYS.index(k)
        base = ph[k]
        stp = 1e-6 * abs(base) if base != 0 else 1e-6
        dp = np.zeros((1, 7))
        dp[0, kk] = 1.0
        j = oracle.jvp(eps, r["a_out"], np.zeros(n, np.uint8), [ph], 0.1, d_params=dp)
        sp, ap = _outputs(eps, a_old, [dict(ph, **{k: base + stp})])
        lower = {"n": 1.0, "nu": -1.0}.get(k, 0.0)        # smallest valid value
        if base - stp >= lower:
            sm, am = _outputs(eps, a_old, [dict(ph, **{k: base - stp})])
            den = 2 * stp
        else:                                  # one-sided at sigma_y = 0 or n = 1
            sm, am = _outputs(eps, a_old, [ph])
            den = stp
        for got, fd in ((j["d_sigma"], (sp - sm) / den), (j["d_a_new"], (ap - am) / den)):
            scale = max(np.abs(fd).max(), np.abs(got).max(), 1e-300)
            assert np.abs(got - fd).max() <= 2e-5 * scale, (k, got, fd)


def test_jvp_adjoint_identity_with_vjp():
    """<g_s, d sigma> + <g_a, d a_{n+1}> = <grad eps, d eps> + <grad a_n, d a_n>
    + sum over phases of grad p . d p: the forward and reverse products are
    transposes of one linear map (two separate hand derivations)."""
    rng = np.random.default_rng(47)
    ph = [dict(inputs.paper_phases()[0]), inputs.paper_phases()[1],
          _phase_row(n=1.0, eps0=0.1)]
    n = 300
    ps = inputs.points_random(n, seed=49, phases=ph[:2], e11=1e-2, std=2e-3, a_std=1e-3)
    phase = rng.integers(0, 3, n).astype(np.uint8)
    r = oracle.evaluate(ps.eps, ps.a_old, phase, ph)
    gs, ga = rng.normal(size=(6, n)), rng.normal(size=(6, n)) * 1e4
    de, da = rng.normal(size=(6, n)) * 1e-3, rng.normal(size=(6, n)) * 1e-4
    dp = rng.normal(size=(3, 7)) * np.array([[p.get(k, 1.0) or 1.0 for k in oracle.GRAD_KEYS]
                                               for p in ph]) * 1e-2
    j = oracle.jvp(ps.eps, r["a_out"], phase, ph, 0.1, d_eps=de, d_a_old=da, d_params=dp)
    b = oracle.backward(ps.eps, ps.a_old, r["a_out"], phase, ph, 0.1, gs, ga)
    lhs = np.sum(gs * j["d_sigma"]) + np.sum(ga * j["d_a_new"])
    terms = [np.sum(b["grad_eps"] * de), np.sum(b["grad_a_old"] * da), np.sum(b["grad_params"] * dp)]
    assert abs(lhs - sum(terms)) <= 1e-11 * max(abs(t) for t in terms + [lhs])


# ---------------------------------------------------------------------------
# failure handling
# ---------------------------------------------------------------------------

def test_nonconvergence_flag_and_nan_inputs():
    ph = inputs.paper_phases()
    eps = np.array([[5e-2, 2e-3, 1e-3], [0, 1e-3, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0]])
    a_old = np.zeros((6, 3))
    eps[2, 1] = np.nan
    phase = np.array([0, 0, 7], np.uint8)      # point 2: unknown phase id
    r = oracle.evaluate(eps, a_old, phase, ph, h=1.0, max_iter=1)
    assert r["iters"][0] == -1                   # nonlinear point, one update allowed
    assert np.all(np.isfinite(r["sigma"][:, 0]))
    assert r["iters"][1] == -1 and np.all(np.isnan(r["sigma"][:, 1]))
    assert r["iters"][2] == -1 and np.all(np.isnan(r["a_out"][:, 2]))
    r = oracle.evaluate(eps[:, :1], a_old[:, :1], phase[:1], ph, h=1.0, max_iter=50)
    assert r["iters"][0] > 1


def test_invalid_arguments_rejected():
    ps = inputs.points_c0(n=8)
    with pytest.raises(ValueError):
        oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=0.0)
    with pytest.raises(ValueError):
        oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, max_iter=0)
    bad = [dict(ps.phases[0], E=0.0), ps.phases[1]]
    with pytest.raises(ValueError):
        oracle.evaluate(ps.eps, ps.a_old, ps.phase, bad)


def test_c0_iteration_profile_and_sigma_criterion():
    """The c0 set converges everywhere; the stress criterion gives the same
    answer to well within the parity tolerance."""
    ps = inputs.points_c0()
    r = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases)
    assert np.all(r["iters"][ps.phase == 1] == 0)
    assert np.all(r["iters"][ps.phase == 0] >= 1)
    r2 = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, flags=oracle.SIGMA_CRITERION)
    assert np.all(r2["iters"] >= 0)
    rel = np.abs(r2["sigma"] - r["sigma"]).max(0) / np.abs(r["sigma"]).max(0)
    assert rel.max() <= 1e-12
