"""Second- and fourth-order tensor helpers for the tests (numpy, 3x3 form).

These give the tests an independent route to the quantities that the oracle
and the GPU path compute in 6-component Voigt form: strains in engineering
shear (gamma_ij = 2 eps_ij), stresses plain, order 11 22 33 23 13 12.
"""
import numpy as np

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def strain_tensor(v):
    """(6, ...) engineering Voigt -> (3, 3, ...) symmetric tensor."""
    v = np.asarray(v, dtype=np.float64)
    t = np.zeros((3, 3) + v.shape[1:])
    for k, (i, j) in enumerate(VOIGT):
        val = v[k] if i == j else 0.5 * v[k]
        t[i, j] = val
        t[j, i] = val
    return t


def stress_tensor(v):
    v = np.asarray(v, dtype=np.float64)
    t = np.zeros((3, 3) + v.shape[1:])
    for k, (i, j) in enumerate(VOIGT):
        t[i, j] = v[k]
        t[j, i] = v[k]
    return t


def strain_voigt(t):
    return np.stack([t[i, j] if i == j else 2.0 * t[i, j] for (i, j) in VOIGT])


def stress_voigt(t):
    return np.stack([t[i, j] for (i, j) in VOIGT])


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def hooke(E, nu, eps_t):
    """sigma_ij = lambda tr(eps) delta_ij + 2 mu eps_ij (tensor form)."""
    lam, mu = lame(E, nu)
    tr = np.trace(eps_t)
    return lam * tr * np.eye(3).reshape((3, 3) + (1,) * (eps_t.ndim - 2)) + 2 * mu * eps_t


def dev(t):
    tr = np.trace(t) / 3.0
    return t - tr * np.eye(3).reshape((3, 3) + (1,) * (t.ndim - 2))


def mises(s_t):
    """sqrt(3/2 s:s) of a deviatoric tensor."""
    return np.sqrt(1.5 * np.einsum("ij...,ij...->...", s_t, s_t))


def voigt_matrix_from_tensor4(T):
    """Engineering-strain -> stress Voigt matrix of a minor-symmetric 4th-order tensor."""
    M = np.zeros((6, 6))
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            M[I, J] = T[i, j, k, l]
    return M


def identity4_sym():
    d = np.eye(3)
    return 0.5 * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d))


def random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def radial_return(eps, a_old, E, nu, H, sy, s0, e0, n, h):
    """Textbook J2 return mapping for the Perzyna power law with linear
    kinematic hardening, reduced to the scalar equation
        q + (3 mu + H) h eps0 ((q - sigma_y)^+ / sigma0)^n = q_trial
    on [0, q_trial], solved by bisection to the last bit. Vectorised over
    points: eps, a_old (6, n) engineering Voigt. Returns (sigma, a_new, q,
    q_trial) with sigma (6, n) plain Voigt."""
    lam, mu = lame(E, nu)
    e_t = strain_tensor(eps)
    a_t = strain_tensor(a_old)
    A_tr = hooke(E, nu, e_t - a_t) - (2.0 / 3.0) * H * a_t     # generalized stress
    s_tr = dev(A_tr)
    q_tr = mises(s_tr)
    lo = np.zeros_like(q_tr)
    hi = q_tr.copy()
    c = (3 * mu + H) * h * e0

    def phi(q):
        x = np.maximum(q - sy, 0.0)
        return q + c * (x / s0) ** n - q_tr

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        pos = phi(mid) > 0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
    q = 0.5 * (lo + hi)
    dp = h * e0 * (np.maximum(q - sy, 0.0) / s0) ** n
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(q_tr > 0, dp / q_tr, 0.0)
    d_t = 1.5 * ratio * s_tr                                  # tensor increment
    a_new_t = a_t + d_t
    sig_t = hooke(E, nu, e_t - a_new_t)
    return stress_voigt(sig_t), strain_voigt(a_new_t), q, q_tr
