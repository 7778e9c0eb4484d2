"""Moulinec-Suquet basic scheme with the CPU oracle as material law.

TEST INFRASTRUCTURE ONLY (see the package docstring). numpy + scipy.fft,
written from the textbook scheme (the homogenization the paper embeds its
material law in: one material sweep without tangent per fixed-point
iteration):

  sigma = material(eps, a_n);  tau = sigma - C0 eps
  eps^(xi) = -Gamma0(xi) : tau^(xi) (xi != 0),  eps^(0) = E
  Gamma0_khij = [d_ki q_h q_j + d_hi q_k q_j + d_kj q_h q_i + d_hj q_k q_i] / (4 mu0)
                - (lambda0 + mu0) / (mu0 (lambda0 + 2 mu0)) q_i q_j q_k q_h,  q = xi/|xi|
  err = ||eps' - eps||_2 / ||E||  (tensor norms, voxel-averaged)

and, once converged (or after a fixed number of iterations), one more
material sweep at the final strain that commits a_{n+1}. Fields are (6, n)
with n = nz * ny * nx, x fastest.

Driver extensions (the paper's Section "Example": the uniaxial
tension-compression test under mixed boundary conditions, and the reference
stiffness that is either fixed from the elastic stiffness or adjusted to the
tangent stiffness at the start of every load step):

* mixed boundary conditions: components in the stress-controlled set S take
  the macroscopic stress S_bar, the others the macroscopic strain E_bar.
  The zero frequency of every update is the macroscopic strain E that makes
  the reference medium's average stress meet the targets,
  mean(tau) + C0 E = S_bar on S, E = E_bar elsewhere (a linear solve);
  at the fixed point mean(sigma) = mean(tau) + C0 mean(eps) = S_bar on S.
  The load step's initial guess shifts the previous field by dE with
  dE = E_bar - E_prev off S and C0[S,S] dE_S = -C0[S,F] dE_F;
* reference update: after that shift, a material sweep with tangent gives the
  isotropic part of every local tangent (projection onto the isotropic
  fourth-order tensors, written on the full tensor), and C0 takes the means
  of the smallest and largest of those Lame constants, the rule the fixed
  reference applies to the elastic constants.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from . import evaluate

VOIGT_PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def tensor_sq(x):
    """Squared tensor norm of engineering-Voigt strains along axis 0."""
    return x[0] ** 2 + x[1] ** 2 + x[2] ** 2 + 0.5 * (x[3] ** 2 + x[4] ** 2 + x[5] ** 2)


def reference_medium(phases):
    lam = [p["E"] * p["nu"] / ((1 + p["nu"]) * (1 - 2 * p["nu"])) for p in phases]
    mu = [p["E"] / (2 * (1 + p["nu"])) for p in phases]
    return 0.5 * (min(lam) + max(lam)), 0.5 * (min(mu) + max(mu))


def _freqs(shape):
    """Frequencies k/N_d (half spectrum along x) and masks of the Nyquist
    entries k = N_d/2 of even dimensions."""
    nz, ny, nx = shape
    fx = np.fft.rfftfreq(nx)[None, None, :]
    fy = np.fft.fftfreq(ny)[None, :, None]
    fz = np.fft.fftfreq(nz)[:, None, None]
    F = np.stack(np.broadcast_arrays(fx, fy, fz), axis=0).copy()      # (3, nz, ny, nxh)
    F = np.abs(F) * np.sign(F)
    nyq = np.stack([np.abs(F[d]) == 0.5 for d in range(3)], axis=0)   # only for even N_d
    F[nyq] = 0.5
    return F, nyq


def _gamma_unit(T, q, lam0, mu0):
    """eps^ = -Gamma0(q) : T for unit vectors q (3, ...) and tensors T (3, 3, ...)."""
    v = np.einsum("ij...,j...->i...", T, q)
    s = np.einsum("i...,i...->...", q, v)
    c1 = 1.0 / (2.0 * mu0)
    c2 = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0))
    out = np.empty((6,) + T.shape[2:], dtype=complex)
    for c, (k, h) in enumerate(VOIGT_PAIRS):
        e = c1 * (q[k] * v[h] + q[h] * v[k]) - c2 * s * q[k] * q[h]
        out[c] = -(1.0 if c < 3 else 2.0) * e
    return out


def gamma_apply(tau_hat, shape, lam0, mu0):
    """-Gamma0 : tau^ on the half spectrum (the zero frequency is set by the
    caller). Where a component sits at the Nyquist index N_d/2 of an even
    dimension and another component is non-zero, +N_d/2 and -N_d/2 are one
    index but give different directions q; there the operator is the
    reference compliance C0^-1 (so the converged stress has no content at
    those frequencies and the fixed point does not depend on C0). Elsewhere,
    pure Nyquist axes included (the operator is even in q), it is the
    continuous operator."""
    F, nyq = _freqs(shape)
    T = np.empty((3, 3) + tau_hat.shape[1:], dtype=complex)
    for c, (i, j) in enumerate(VOIGT_PAIRS):
        T[i, j] = tau_hat[c]
        T[j, i] = tau_hat[c]
    norm = np.sqrt((F ** 2).sum(axis=0))
    norm[norm == 0] = 1.0
    out = _gamma_unit(T, F / norm, lam0, mu0)
    ambiguous = nyq.any(axis=0) & ((F != 0).sum(axis=0) >= 2)
    S0 = np.linalg.inv(voigt_stiffness(lam0, mu0))
    comp = -np.einsum("cd,d...->c...", S0, tau_hat)
    return np.where(ambiguous[None], comp, out)


def gamma_matrix(shape, lam0, mu0):
    """The operator of gamma_apply as one complex 6x6 matrix per frequency of
    the half spectrum, (6, 6, nz, ny, nx//2 + 1): column d is the image of
    the unit polarization e_d (the operator is linear and acts frequency by
    frequency), so that an iteration applies it by one matrix product."""
    nz, ny, nx = shape
    G = np.empty((6, 6, nz, ny, nx // 2 + 1), dtype=complex)
    for d in range(6):
        unit = np.zeros((6, nz, ny, nx // 2 + 1), dtype=complex)
        unit[d] = 1.0
        G[:, d] = gamma_apply(unit, shape, lam0, mu0)
    return G


def voigt_stiffness(lam, mu):
    """Isotropic stiffness in engineering Voigt form (stress = C @ strain)."""
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[[0, 1, 2], [0, 1, 2]] += 2.0 * mu
    C[[3, 4, 5], [3, 4, 5]] = mu
    return C


def full_tensor(tan):
    """(36, n) row-major engineering-Voigt stiffnesses -> (3, 3, 3, 3, n)
    tensors with sigma_ij = C_ijkl eps_kl (a shear column of the Voigt form
    acts on the engineering strain 2 eps_kl, shared by kl and lk, so every
    tensor entry equals its Voigt entry)."""
    V = np.asarray(tan).reshape(6, 6, -1)
    idx = {}
    for c, (i, j) in enumerate(VOIGT_PAIRS):
        idx[(i, j)] = idx[(j, i)] = c
    T = np.empty((3, 3, 3, 3, V.shape[2]))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    T[i, j, k, l] = V[idx[(i, j)], idx[(k, l)]]
    return T


def isotropic_part(tan):
    """Lame constants (lam, mu) of the isotropic part of each stiffness:
    C_iso = 3K P1 + 2mu P2 with the projectors P1 = I x I / 3 and
    P2 = I_sym - P1, K = (I : C : I) / 9, 2mu = (P2 :: C) / 5."""
    T = full_tensor(tan)
    c_iijj = np.einsum("iijj...->...", T)
    c_ijij = np.einsum("ijij...->...", T)
    K = c_iijj / 9.0
    mu = (c_ijij - c_iijj / 3.0) / 10.0
    return K - 2.0 * mu / 3.0, mu


def reference_from_tangent(tan):
    lam, mu = isotropic_part(tan)
    return 0.5 * (np.nanmin(lam) + np.nanmax(lam)), 0.5 * (np.nanmin(mu) + np.nanmax(mu))


def _macro_strain(tau_mean, E_bar, S_bar, smask, lam0, mu0):
    """E with E = E_bar off the stress-controlled set S and
    (tau_mean + C0 E)_S = S_bar_S."""
    E = np.array(E_bar, dtype=np.float64)
    S = np.array([bool(smask >> c & 1) for c in range(6)])
    if S.any():
        C0 = voigt_stiffness(lam0, mu0)
        F = ~S
        rhs = np.asarray(S_bar, dtype=np.float64)[S] - tau_mean[S] - C0[np.ix_(S, F)] @ E[F]
        E[S] = np.linalg.solve(C0[np.ix_(S, S)], rhs)
    return E


def ms_step(eps, a, phase, phases, shape, E, E_prev, h, lam0=None, mu0=None, tol=1e-6,
            max_iter=1000, fixed_iter=False, newton_tol=1e-12, newton_max_iter=50,
            stress_mask=0, S_macro=None, ref_update=False):
    """One load step. E is the macroscopic strain (its stress-controlled
    components are ignored), E_prev the macroscopic strain the previous step
    reached. Returns dict(eps, a, sigma, sigma_mean, E (reached), iters,
    residual, lam0, mu0 (the reference used))."""
    if lam0 is None or mu0 is None:
        lam0, mu0 = reference_medium(phases)
    nz, ny, nx = shape
    n = nx * ny * nz
    E = np.asarray(E, dtype=np.float64)
    E_prev = np.asarray(E_prev, dtype=np.float64)
    S_bar = np.zeros(6) if S_macro is None else np.asarray(S_macro, dtype=np.float64)
    S = np.array([bool(stress_mask >> c & 1) for c in range(6)])
    dE = E - E_prev
    if S.any():
        C0 = voigt_stiffness(lam0, mu0)
        dE[S] = np.linalg.solve(C0[np.ix_(S, S)], -C0[np.ix_(S, ~S)] @ dE[~S])
    eps = np.array(eps, dtype=np.float64) + dE[:, None]
    Ecur = E_prev + dE
    if ref_update:
        rt = evaluate(eps, a, phase, phases, h=h, tol=newton_tol, max_iter=newton_max_iter,
                      tangent=True)
        lam0, mu0 = reference_from_tangent(rt["tangent"])
    err = 0.0
    it = 0
    G = gamma_matrix(shape, lam0, mu0)
    for it in range(1, max_iter + 1):
        r = evaluate(eps, a, phase, phases, h=h, tol=newton_tol, max_iter=newton_max_iter)
        tr = lam0 * (eps[0] + eps[1] + eps[2])
        tau = r["sigma"].copy()
        tau[:3] -= tr + 2.0 * mu0 * eps[:3]
        tau[3:] -= mu0 * eps[3:]
        th = scipy.fft.rfftn(tau.reshape(6, nz, ny, nx), axes=(1, 2, 3))
        eh = np.einsum("cd...,d...->c...", G, th)
        Ecur = _macro_strain(th[:, 0, 0, 0].real / n, E, S_bar, stress_mask, lam0, mu0)
        eh[:, 0, 0, 0] = Ecur * n
        new = scipy.fft.irfftn(eh, s=(nz, ny, nx), axes=(1, 2, 3)).reshape(6, n)
        En = max(np.sqrt(tensor_sq(Ecur)), 1e-300)
        err = np.sqrt(np.mean(tensor_sq(new - eps))) / En
        eps = new
        if not fixed_iter and err <= tol:
            break
    r = evaluate(eps, a, phase, phases, h=h, tol=newton_tol, max_iter=newton_max_iter)
    return dict(eps=eps, a=r["a_out"], sigma=r["sigma"], sigma_mean=r["sigma"].mean(axis=1),
                E=Ecur, iters=it, residual=err, lam0=lam0, mu0=mu0)


def _gamma_field(x, G, shape):
    """-Gamma0 * x for a real (6, n) field with the zero frequency removed."""
    nz, ny, nx = shape
    xh = scipy.fft.rfftn(x.reshape(6, nz, ny, nx), axes=(1, 2, 3))
    yh = np.einsum("cd...,d...->c...", G, xh)
    yh[:, 0, 0, 0] = 0.0
    return scipy.fft.irfftn(yh, s=(nz, ny, nx), axes=(1, 2, 3)).reshape(6, -1)


def linearized_step(eps, a_prev, a, phase, phases, shape, h, dE, d_a_prev=None, d_params=None,
                    lam0=None, mu0=None, tol=1e-12, max_iter=2000):
    """Forward derivative of one converged strain-controlled load step.

    (eps, a) is the converged state that the step reached from a_prev under
    the macroscopic strain E. The implicit function theorem (the paper's
    Section "Single Implicit Euler Step", applied here to the fixed point of
    the basic scheme instead of the Newton system) gives the change d eps of
    the fixed point for a change (dE, d a_prev, d p) of the step's inputs as
    the solution of the linearized Lippmann-Schwinger equation

        d eps = dE - Gamma0 * (d sigma - C0 d eps),
        d sigma = C_tan d eps + s,

    with C_tan the consistent tangent field at the converged state and s the
    stress change at fixed strain (from d a_prev and d p, the oracle's
    Jacobian-vector product). Rearranged,
        d eps + Gamma0 * ((C_tan - C0) d eps) = dE - Gamma0 * s,
    a linear system for the 6n strain values, solved by GMRES (the converged
    derivative does not depend on C0).

    d_params: (n_phases, 7) over the oracle's GRAD_KEYS, or None.
    Returns dict(d_eps, d_sigma (fields), d_sigma_mean (6,), d_a (the change
    of a_{n+1}, for the next step's history), gmres_info)."""
    from scipy.sparse.linalg import LinearOperator, gmres
    from . import jvp
    if lam0 is None or mu0 is None:
        lam0, mu0 = reference_medium(phases)
    nz, ny, nx = shape
    n = nx * ny * nz
    G = gamma_matrix(shape, lam0, mu0)
    C0 = voigt_stiffness(lam0, mu0)
    r = evaluate(eps, a_prev, phase, phases, h=h, tol=1e-14, max_iter=100, tangent=True)
    Ct = r["tangent"].reshape(6, 6, n)
    dCt = Ct - C0[:, :, None]
    s = jvp(eps, a, phase, phases, h, d_a_old=d_a_prev, d_params=d_params)["d_sigma"]

    def op(v):
        x = v.reshape(6, n)
        return (x - _gamma_field(np.einsum("cdn,dn->cn", dCt, x), G, shape)).reshape(-1)

    dE = np.asarray(dE, dtype=np.float64)
    b = (dE[:, None] + _gamma_field(s, G, shape)).reshape(-1)
    L = LinearOperator((6 * n, 6 * n), matvec=op, dtype=np.float64)
    x, info = gmres(L, b, x0=np.repeat(dE, n), rtol=tol, atol=0.0, restart=60,
                    maxiter=max_iter)
    de = x.reshape(6, n)
    j = jvp(eps, a, phase, phases, h, d_eps=de, d_a_old=d_a_prev, d_params=d_params)
    return dict(d_eps=de, d_sigma=j["d_sigma"], d_sigma_mean=j["d_sigma"].mean(axis=1),
                d_a=j["d_a_new"], gmres_info=info)


def linearized_history(history, phase, phases, shape, h, dE_steps, d_params=None, lam0=None,
                       mu0=None, tol=1e-12):
    """Forward derivative of the last step's mean stress over a load history.

    history: the converged steps [(eps_1, a_0, a_1), ..., (eps_K, a_{K-1}, a_K)]
    of a strain-controlled run from a_0; dE_steps: (K, 6) changes of the
    macroscopic strains; d_params as in linearized_step. The change of a_k
    carries into step k + 1. Returns d mean(sigma_K) (6,)."""
    d_a = None
    out = None
    for (eps, a_prev, a), dE in zip(history, dE_steps):
        out = linearized_step(eps, a_prev, a, phase, phases, shape, h, dE, d_a_prev=d_a,
                              d_params=d_params, lam0=lam0, mu0=mu0, tol=tol)
        if out["gmres_info"] != 0:
            raise RuntimeError(f"GMRES did not converge ({out['gmres_info']})")
        d_a = out["d_a"]
    return out["d_sigma_mean"]
