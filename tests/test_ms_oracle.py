"""Pins of the oracle's Moulinec-Suquet driver (CPU)."""
import numpy as np
import pytest

import oracle
from oracle import ms as oms
from paper_2006_04391_amd import inputs
from tests import _tensor as T

ELASTIC = lambda E, nu: dict(kind=0, E=E, nu=nu, H=0.0, sigma_y=0.0, sigma0=1.0, eps0=0.0, n=1.0)


def _voigt_from_sym(t):
    return np.array([t[0, 0], t[1, 1], t[2, 2], 2 * t[1, 2], 2 * t[0, 2], 2 * t[0, 1]])


def test_green_operator_projects_compatible_strains_and_kills_equilibrated_stress():
    """Gamma0 : C0 : sym(xi (x) u) = sym(xi (x) u) (compatible fields are
    reproduced) and Gamma0 : s = 0 for s . xi = 0 (equilibrated fields)."""
    rng = np.random.default_rng(0)
    shape = (4, 5, 6)
    lam0, mu0 = 700.0, 350.0
    nz, ny, nx = shape
    for _ in range(10):
        # away from the Nyquist planes, where +xi and its alias -xi differ per component
        kz, ky, kx = rng.integers(-1, 2), rng.integers(-2, 3), rng.integers(1, 3)
        xi = np.array([kx / nx, ky / ny, kz / nz])
        u = rng.normal(size=3) + 1j * rng.normal(size=3)
        e = 0.5 * (np.outer(xi, u) + np.outer(u, xi))
        s = lam0 * np.trace(e) * np.eye(3) + 2 * mu0 * e        # C0 : e
        tau = np.zeros((6, nz, ny, nx // 2 + 1), dtype=complex)
        tau[:, kz % nz, ky % ny, kx] = [s[0, 0], s[1, 1], s[2, 2], s[1, 2], s[0, 2], s[0, 1]]
        out = oms.gamma_apply(tau, shape, lam0, mu0)[:, kz % nz, ky % ny, kx]
        np.testing.assert_allclose(-out, _voigt_from_sym(e), rtol=1e-12, atol=1e-14)
        # an equilibrated stress: s . xi = 0
        w = np.cross(xi, rng.normal(size=3))
        z = np.cross(xi, w)
        sq = np.outer(w, w) + np.outer(z, z) * 0.3
        tau[:, kz % nz, ky % ny, kx] = [sq[0, 0], sq[1, 1], sq[2, 2], sq[1, 2], sq[0, 2], sq[0, 1]]
        out = oms.gamma_apply(tau, shape, lam0, mu0)[:, kz % nz, ky % ny, kx]
        assert np.abs(out).max() <= 1e-14 * np.abs(sq).max() / mu0


def test_homogeneous_cell_one_iteration():
    N = 8
    ph = [ELASTIC(2500.0, 0.35)]
    E = np.array([1e-3, -2e-4, 0, 0, 5e-4, 0])
    r = oms.ms_step(np.zeros((6, N ** 3)), np.zeros((6, N ** 3)), np.zeros(N ** 3, np.uint8), ph,
                    (N, N, N), E, np.zeros(6), 0.1, lam0=500.0, mu0=300.0, tol=1e-12)
    assert r["iters"] == 1
    np.testing.assert_allclose(r["eps"], np.repeat(E[:, None], N ** 3, 1), atol=1e-15)
    sig = T.stress_voigt(T.hooke(2500.0, 0.35, T.strain_tensor(E)))
    np.testing.assert_allclose(r["sigma_mean"], sig, rtol=1e-12, atol=1e-12)


def laminate_sigma(phases_x, fr, E):
    """Exact mean stress of an elastic laminate with layers normal to x.
    Tangential strains (yy, zz, yz) are uniform, tractions (xx, xy, xz) are
    uniform; the remaining strain components average to E."""
    lam = np.array([T.lame(p["E"], p["nu"])[0] for p in phases_x])
    mu = np.array([T.lame(p["E"], p["nu"])[1] for p in phases_x])
    fr = np.asarray(fr)
    M = lam + 2 * mu
    Exx, Eyy, Ezz, Eyz, Exz, Exy = E
    sxx = (Exx + np.sum(fr * lam / M) * (Eyy + Ezz)) / np.sum(fr / M)
    exx = (sxx - lam * (Eyy + Ezz)) / M
    sxy = Exy / np.sum(fr / mu)
    sxz = Exz / np.sum(fr / mu)
    syy = np.sum(fr * (lam * (exx + Ezz) + M * Eyy))
    szz = np.sum(fr * (lam * (exx + Eyy) + M * Ezz))
    syz = np.sum(fr * mu) * Eyz
    return np.array([sxx, syy, szz, syz, sxz, sxy])


def test_laminate_exact():
    """A voxel laminate (phase varying along x only) reproduces the exact
    laminate mean stress."""
    nz, ny, nx = 4, 4, 16
    ph = [ELASTIC(2500.0, 0.35), ELASTIC(72000.0, 0.22)]
    layer = (np.arange(nx) >= 11).astype(np.uint8)           # 5 of 16 layers stiff
    phase = np.broadcast_to(layer[None, None, :], (nz, ny, nx)).reshape(-1).copy()
    E = np.array([1e-3, 3e-4, -2e-4, 4e-4, -5e-4, 6e-4])
    r = oms.ms_step(np.zeros((6, phase.size)), np.zeros((6, phase.size)), phase, ph, (nz, ny, nx),
                    E, np.zeros(6), 0.1, tol=1e-11, max_iter=5000)
    ref = laminate_sigma(ph, [11 / 16, 5 / 16], E)
    np.testing.assert_allclose(r["sigma_mean"], ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


def test_spheres_within_hashin_shtrikman_bounds():
    N = 16
    phase = inputs.sphere_phase(N, seed=5, radius=3.0, vol_frac=0.2)
    c2 = phase.mean()
    m, f = ELASTIC(2500.0, 0.35), ELASTIC(72000.0, 0.22)
    l1, m1 = T.lame(m["E"], m["nu"])
    l2, m2 = T.lame(f["E"], f["nu"])
    k1, k2 = l1 + 2 * m1 / 3, l2 + 2 * m2 / 3
    c1 = 1 - c2
    k_lo = k1 + c2 / (1 / (k2 - k1) + 3 * c1 / (3 * k1 + 4 * m1))
    k_hi = k2 + c1 / (1 / (k1 - k2) + 3 * c2 / (3 * k2 + 4 * m2))
    m_lo = m1 + c2 / (1 / (m2 - m1) + 6 * c1 * (k1 + 2 * m1) / (5 * m1 * (3 * k1 + 4 * m1)))
    m_hi = m2 + c1 / (1 / (m1 - m2) + 6 * c2 * (k2 + 2 * m2) / (5 * m2 * (3 * k2 + 4 * m2)))
    z = np.zeros((6, N ** 3))
    e = 1e-3
    r = oms.ms_step(z, z, phase, [m, f], (N, N, N), [e, e, e, 0, 0, 0], np.zeros(6), 0.1,
                    tol=1e-8, max_iter=5000)
    k_eff = r["sigma_mean"][:3].sum() / (9 * e)
    assert k_lo <= k_eff <= k_hi, (k_lo, k_eff, k_hi)
    r = oms.ms_step(z, z, phase, [m, f], (N, N, N), [0, 0, 0, 0, 0, e], np.zeros(6), 0.1,
                    tol=1e-8, max_iter=5000)
    m_eff = r["sigma_mean"][5] / e
    assert m_lo <= m_eff <= m_hi, (m_lo, m_eff, m_hi)


def test_viscoplastic_step_commits_state_and_relaxes():
    """Two steps with a flowing matrix: a_{n+1} is committed, the scheme
    converges below tol, and the mean stress is below the elastic one."""
    N = 8
    phase = inputs.sphere_phase(N, seed=6, radius=2.0, vol_frac=0.2)
    ph = inputs.paper_phases()
    z = np.zeros((6, N ** 3))
    E1 = np.array([5e-3, 0, 0, 0, 0, 0])
    r1 = oms.ms_step(z, z, phase, ph, (N, N, N), E1, np.zeros(6), 1.0, tol=1e-8)
    assert r1["residual"] <= 1e-8 and r1["iters"] > 1
    assert np.abs(r1["a"][:, phase == 0]).max() > 0 and np.all(r1["a"][:, phase == 1] == 0)
    el = [ph[0] | dict(kind=0), ph[1]]
    r_el = oms.ms_step(z, z, phase, el, (N, N, N), E1, np.zeros(6), 1.0, tol=1e-8)
    assert r1["sigma_mean"][0] < r_el["sigma_mean"][0]
    r2 = oms.ms_step(r1["eps"], r1["a"], phase, ph, (N, N, N), 2 * E1, E1, 1.0, tol=1e-8)
    assert np.allclose(r2["eps"].mean(axis=1), 2 * E1, atol=1e-14)


def _gamma_full(tau_full, shape, lam0, mu0):
    """The operator on the full (signed) frequency grid: the reference
    compliance where a Nyquist component meets another non-zero component,
    the continuous operator at the signed frequency elsewhere."""
    nz, ny, nx = shape
    F = np.stack(np.broadcast_arrays(np.fft.fftfreq(nx)[None, None, :],
                                     np.fft.fftfreq(ny)[None, :, None],
                                     np.fft.fftfreq(nz)[:, None, None]), axis=0)
    nyq = np.abs(F) == 0.5
    T = np.empty((3, 3) + tau_full.shape[1:], dtype=complex)
    for c, (i, j) in enumerate(oms.VOIGT_PAIRS):
        T[i, j] = tau_full[c]
        T[j, i] = tau_full[c]
    nrm = np.sqrt((F ** 2).sum(axis=0))
    nrm[nrm == 0] = 1.0
    cont = oms._gamma_unit(T, F / nrm, lam0, mu0)
    amb = nyq.any(axis=0) & ((F != 0).sum(axis=0) >= 2)
    comp = np.empty_like(tau_full)
    for idx in np.ndindex(*tau_full.shape[1:]):
        if amb[idx]:
            t = tau_full[(slice(None),) + idx]
            st = T[(slice(None), slice(None)) + idx]
            # isotropic compliance in tensor form: e = (s - lam0/(3 lam0 + 2 mu0) tr(s) I) / (2 mu0)
            e = (st - lam0 / (3 * lam0 + 2 * mu0) * np.trace(st) * np.eye(3)) / (2 * mu0)
            comp[(slice(None),) + idx] = -_voigt_from_sym(e)
    return np.where(amb[None], comp, cont)


@pytest.mark.parametrize("shape", [(6, 8, 10), (5, 7, 9), (4, 6, 6)])
def test_green_operator_keeps_fields_real(shape):
    """The half-spectrum update equals the full complex-FFT update and the
    latter is real: the operator is Hermitian-consistent on even grids
    (Nyquist planes included)."""
    rng = np.random.default_rng(1)
    tau = rng.normal(size=(6,) + shape)
    lam0, mu0 = 600.0, 400.0
    half = oms.gamma_apply(np.fft.rfftn(tau, axes=(1, 2, 3)), shape, lam0, mu0)
    half[:, 0, 0, 0] = 0
    e_half = np.fft.irfftn(half, s=shape, axes=(1, 2, 3))
    full = _gamma_full(np.fft.fftn(tau, axes=(1, 2, 3)), shape, lam0, mu0)
    full[:, 0, 0, 0] = 0
    e_full = np.fft.ifftn(full, axes=(1, 2, 3))
    assert np.abs(e_full.imag).max() <= 1e-12 * np.abs(e_full.real).max()
    np.testing.assert_allclose(e_half, e_full.real, rtol=0, atol=1e-12 * np.abs(e_half).max())


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 7, 8)])
def test_fixed_point_does_not_depend_on_the_reference(shape):
    """Two reference media (both stiff enough for convergence) give the same
    converged fields on a heterogeneous cell with even dimensions."""
    nz, ny, nx = shape
    n = nx * ny * nz
    phase = (np.random.default_rng(2).random(n) < 0.3).astype(np.uint8)
    ph = [ELASTIC(2500.0, 0.35), ELASTIC(72000.0, 0.22)]
    z = np.zeros((6, n))
    E = np.array([1e-3, -2e-4, 3e-4, 5e-4, 0, -4e-4])
    lam0, mu0 = oms.reference_medium(ph)
    r1 = oms.ms_step(z, z, phase, ph, shape, E, np.zeros(6), 0.1, lam0=lam0, mu0=mu0, tol=1e-14,
                     max_iter=3000)
    r2 = oms.ms_step(z, z, phase, ph, shape, E, np.zeros(6), 0.1, lam0=1.7 * lam0,
                     mu0=1.4 * mu0, tol=1e-14, max_iter=3000)
    assert r1["residual"] <= 1e-14 and r2["residual"] <= 1e-14
    scale = np.abs(r1["sigma"]).max()
    assert np.abs(r1["sigma"] - r2["sigma"]).max() <= 1e-10 * scale
    assert np.abs(r1["eps"] - r2["eps"]).max() <= 1e-10 * np.abs(r1["eps"]).max()


def test_central_differences_of_the_scheme_give_the_laminate_stiffness():
    """The derivative reference of the reverse step (central differences of
    the oracle's scheme run a fixed number of iterations past convergence)
    reproduces the exact stiffness of an elastic laminate."""
    nz, ny, nx = 2, 2, 8
    ph = [ELASTIC(2500.0, 0.35), ELASTIC(72000.0, 0.22)]
    layer = (np.arange(nx) >= 5).astype(np.uint8)
    phase = np.broadcast_to(layer[None, None, :], (nz, ny, nx)).reshape(-1).copy()
    lam0, mu0 = oms.reference_medium(ph)
    z = np.zeros((6, phase.size))
    C = np.array([laminate_sigma(ph, [5 / 8, 3 / 8], np.eye(6)[c]) for c in range(6)]).T
    d = 1e-7
    for c in range(6):
        E = np.zeros(6)
        E[c] = d
        sp = oms.ms_step(z, z, phase, ph, (nz, ny, nx), E, np.zeros(6), 0.1, lam0=lam0, mu0=mu0,
                         tol=0.0, max_iter=800, fixed_iter=True)["sigma_mean"]
        sm = oms.ms_step(z, z, phase, ph, (nz, ny, nx), -E, np.zeros(6), 0.1, lam0=lam0, mu0=mu0,
                         tol=0.0, max_iter=800, fixed_iter=True)["sigma_mean"]
        np.testing.assert_allclose((sp - sm) / (2 * d), C[:, c], rtol=1e-7,
                                   atol=1e-7 * np.abs(C).max())


UNIAXIAL = 0b111110    # every component but xx stress-controlled


def test_uniaxial_stress_homogeneous_gives_young_and_poisson():
    """Mixed boundary conditions, eps_xx prescribed and every other mean
    stress zero: a homogeneous elastic cell returns sigma_xx = E eps_xx and
    the lateral contraction -nu eps_xx (for any reference medium)."""
    N = 6
    Ey, nu = 2500.0, 0.35
    e = 1e-3
    z = np.zeros((6, N ** 3))
    r = oms.ms_step(z, z, np.zeros(N ** 3, np.uint8), [ELASTIC(Ey, nu)], (N, N, N),
                    [e, 0, 0, 0, 0, 0], np.zeros(6), 0.1, lam0=900.0, mu0=700.0, tol=1e-13,
                    max_iter=500, stress_mask=UNIAXIAL)
    np.testing.assert_allclose(r["E"], [e, -nu * e, -nu * e, 0, 0, 0], rtol=1e-11, atol=1e-17)
    np.testing.assert_allclose(r["sigma_mean"], [Ey * e, 0, 0, 0, 0, 0], atol=1e-11 * Ey * e)


def _laminate_stiffness(ph, fr):
    """Exact effective stiffness (6x6, engineering Voigt) of a laminate with
    layers normal to x, column by column from the exact mean stress."""
    return np.stack([laminate_sigma(ph, fr, np.eye(6)[j]) for j in range(6)], axis=1)


@pytest.mark.parametrize("mask", [UNIAXIAL, 0b011010])
def test_mixed_conditions_on_a_laminate(mask):
    """A laminate under mixed conditions reaches the state that the exact
    effective stiffness gives for the same mixed problem, solved directly."""
    nz, ny, nx = 4, 4, 16
    ph = [ELASTIC(2500.0, 0.35), ELASTIC(72000.0, 0.22)]
    layer = (np.arange(nx) >= 11).astype(np.uint8)
    phase = np.broadcast_to(layer[None, None, :], (nz, ny, nx)).reshape(-1).copy()
    Ebar = np.array([1e-3, 3e-4, -2e-4, 4e-4, -5e-4, 6e-4])
    Sbar = np.array([0.0, 2.0, -1.0, 0.5, 0.0, -0.7])
    z = np.zeros((6, phase.size))
    r = oms.ms_step(z, z, phase, ph, (nz, ny, nx), Ebar, np.zeros(6), 0.1, tol=1e-12,
                    max_iter=5000, stress_mask=mask, S_macro=Sbar)
    Ceff = _laminate_stiffness(ph, [11 / 16, 5 / 16])
    S = np.array([bool(mask >> c & 1) for c in range(6)])
    Eref = Ebar.copy()
    Eref[S] = np.linalg.solve(Ceff[np.ix_(S, S)], Sbar[S] - Ceff[np.ix_(S, ~S)] @ Ebar[~S])
    sref = Ceff @ Eref
    np.testing.assert_allclose(r["E"], Eref, rtol=1e-8, atol=1e-8 * np.abs(Eref).max())
    np.testing.assert_allclose(r["sigma_mean"], sref, rtol=1e-8, atol=1e-8 * np.abs(sref).max())
    np.testing.assert_allclose(r["sigma_mean"][S], Sbar[S], atol=1e-8 * np.abs(sref).max())


def test_isotropic_part_of_stiffnesses():
    """The isotropic part returns the Lame constants of an isotropic
    stiffness, and for an anisotropic one it is the closest isotropic tensor
    in the Frobenius norm of the full fourth-order tensors."""
    lam, mu = oms.isotropic_part(np.stack([oms.voigt_stiffness(40.0, 21.0).ravel(),
                                           oms.voigt_stiffness(-3.0, 7.5).ravel()], axis=1))
    np.testing.assert_allclose(lam, [40.0, -3.0], rtol=1e-14)
    np.testing.assert_allclose(mu, [21.0, 7.5], rtol=1e-14)
    rng = np.random.default_rng(3)
    A = rng.normal(size=(6, 6))
    C = A @ A.T + 6 * np.eye(6)
    l0, m0 = oms.isotropic_part(C.reshape(36, 1))

    def dist(l, m):
        return np.sum((oms.full_tensor(C.reshape(36, 1)) -
                       oms.full_tensor(oms.voigt_stiffness(l, m).reshape(36, 1))) ** 2)
    d0 = dist(l0[0], m0[0])
    for dl, dm in [(1e-3, 0), (-1e-3, 0), (0, 1e-3), (0, -1e-3), (1e-3, -1e-3)]:
        assert dist(l0[0] + dl, m0[0] + dm) > d0


def test_reference_update_elastic_equals_fixed_rule():
    """On an elastic field the tangent-based reference equals the fixed
    reference from the elastic constants."""
    N = 8
    phase = inputs.sphere_phase(N, seed=5, radius=2.0, vol_frac=0.2)
    ph = [ELASTIC(2500.0, 0.35), ELASTIC(72000.0, 0.22)]
    z = np.zeros((6, N ** 3))
    r = oms.ms_step(z, z, phase, ph, (N, N, N), [1e-3, 0, 0, 0, 0, 0], np.zeros(6), 0.1,
                    tol=1e-8, ref_update=True)
    np.testing.assert_allclose([r["lam0"], r["mu0"]], oms.reference_medium(ph), rtol=1e-13)


def test_reference_update_same_solution_fewer_iterations():
    """With a flowing matrix the tangent-based reference is softer; the
    converged state does not depend on the reference (up to the tolerance),
    and the softer reference needs fewer iterations."""
    N = 8
    phase = inputs.sphere_phase(N, seed=6, radius=2.0, vol_frac=0.2)
    ph = inputs.paper_phases()
    z = np.zeros((6, N ** 3))
    E1 = np.array([4e-3, 0, 0, 0, 0, 0])
    r1 = oms.ms_step(z, z, phase, ph, (N, N, N), E1, np.zeros(6), 1.0, tol=1e-10,
                     stress_mask=UNIAXIAL)
    runs = {}
    for upd in (False, True):
        runs[upd] = oms.ms_step(r1["eps"], r1["a"], phase, ph, (N, N, N), 2 * E1, r1["E"], 1.0,
                                tol=1e-10, stress_mask=UNIAXIAL, ref_update=upd)
    f, u = runs[False], runs[True]
    assert u["mu0"] < 0.9 * f["mu0"]
    assert u["iters"] < f["iters"]
    scale = np.abs(f["sigma"]).max()
    assert np.abs(u["sigma"] - f["sigma"]).max() <= 1e-7 * scale
    np.testing.assert_allclose(u["E"], f["E"], rtol=1e-7)
    assert abs(f["sigma_mean"][1:]).max() <= 1e-8 * abs(f["sigma_mean"][0])


# ---------------------------------------------------------------------------
# linearized scheme (forward derivative of converged load steps)
# ---------------------------------------------------------------------------

def test_linearized_step_gives_the_laminate_stiffness():
    """On an elastic laminate the linearized Lippmann-Schwinger solve for a
    unit macroscopic strain returns the column of the exact laminate
    stiffness (tangential strains and normal tractions uniform)."""
    nz, ny, nx = 4, 4, 16
    ph = [ELASTIC(2500.0, 0.35), ELASTIC(72000.0, 0.22)]
    layer = (np.arange(nx) >= 11).astype(np.uint8)
    phase = np.broadcast_to(layer[None, None, :], (nz, ny, nx)).reshape(-1).copy()
    z = np.zeros((6, phase.size))
    C = np.array([laminate_sigma(ph, [11 / 16, 5 / 16], np.eye(6)[c]) for c in range(6)]).T
    for c in range(6):
        r = oms.linearized_step(z, z, z, phase, ph, (nz, ny, nx), 0.1, np.eye(6)[c])
        assert r["gmres_info"] == 0
        np.testing.assert_allclose(r["d_sigma_mean"], C[:, c], rtol=1e-10,
                                   atol=1e-10 * np.abs(C).max())


def _converged_history(shape, phase, ph, loads, h, tol=1e-13):
    n = phase.size
    eps, a, prev = np.zeros((6, n)), np.zeros((6, n)), np.zeros(6)
    hist = []
    for E in loads:
        r = oms.ms_step(eps, a, phase, ph, shape, E, prev, h, tol=tol, max_iter=5000,
                        newton_tol=1e-14)
        assert r["residual"] <= tol
        hist.append((r["eps"], a, r["a"]))
        eps, a, prev = r["eps"], r["a"], np.asarray(E, dtype=float)
    return hist, r["sigma_mean"]


def test_linearized_history_against_central_differences_of_the_scheme():
    """Two flowing load steps on a random two-phase grid: the forward
    derivative of <sigma_2> in E_2, in E_1 (through the history of a) and in
    the matrix parameters E, sigma0 and n, against central differences of
    the scheme converged to 1e-13 (relative step 1e-5: the stopping rules
    make the discrete map piecewise smooth with jumps near 1e-13; truncation
    and those jumps stay near 1e-10 relative, gate 1e-8)."""
    shape = (4, 6, 8)
    nz, ny, nx = shape
    rng = np.random.default_rng(11)
    phase = (rng.random(nz * ny * nx) < 0.25).astype(np.uint8)
    ph = inputs.paper_phases()
    h = 1.0
    loads = [[2e-3 * k, -5e-4 * k, 0, 0, 3e-4 * k, 0] for k in (1, 2)]
    hist, _ = _converged_history(shape, phase, ph, loads, h)

    def mean_after(loads_, ph_):
        return _converged_history(shape, phase, ph_, loads_, h)[1]

    step = 1e-5 * np.linalg.norm(loads[-1])
    for k, c in ((1, 0), (1, 5), (0, 0)):
        dE = np.zeros((2, 6))
        dE[k, c] = 1.0
        lin = oms.linearized_history(hist, phase, ph, shape, h, dE)
        lp = [list(x) for x in loads]
        lm = [list(x) for x in loads]
        lp[k][c] += step
        lm[k][c] -= step
        fd = (mean_after(lp, ph) - mean_after(lm, ph)) / (2 * step)
        assert np.abs(lin - fd).max() <= 1e-8 * np.abs(fd).max(), (k, c, lin, fd)
    for key in ("E", "sigma0", "n"):
        p0 = ph[0][key]
        d = 1e-5 * abs(p0)
        dp = np.zeros((2, 7))
        dp[0, oracle.GRAD_KEYS.index(key)] = 1.0
        lin = oms.linearized_history(hist, phase, ph, shape, h, np.zeros((2, 6)), d_params=dp)
        fd = (mean_after(loads, [dict(ph[0], **{key: p0 + d}), ph[1]])
              - mean_after(loads, [dict(ph[0], **{key: p0 - d}), ph[1]])) / (2 * d)
        assert np.abs(lin - fd).max() <= 1e-8 * np.abs(fd).max(), (key, lin, fd)
