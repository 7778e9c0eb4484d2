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
    caller). A component k = N_d/2 of an even dimension stands for both
    +N_d/2 and -N_d/2; the operator is averaged over those sign choices,
    which keeps the spectrum Hermitian (and equals the continuous operator
    on the pure Nyquist axes, the operator being even in xi)."""
    F, nyq = _freqs(shape)
    T = np.empty((3, 3) + tau_hat.shape[1:], dtype=complex)
    for c, (i, j) in enumerate(VOIGT_PAIRS):
        T[i, j] = tau_hat[c]
        T[j, i] = tau_hat[c]
    out = np.zeros_like(tau_hat)
    count = np.zeros(tau_hat.shape[1:])
    for sx in (1.0, -1.0):
        for sy in (1.0, -1.0):
            for sz in (1.0, -1.0):
                sgn = np.array([sx, sy, sz])
                # a sign flip applies only where that component is at Nyquist
                use = np.ones(tau_hat.shape[1:], dtype=bool)
                for d in range(3):
                    if sgn[d] < 0:
                        use &= nyq[d]
                q = F * np.where(nyq, sgn[:, None, None, None], 1.0)
                norm = np.sqrt((q ** 2).sum(axis=0))
                norm[norm == 0] = 1.0
                g = _gamma_unit(T, q / norm, lam0, mu0)
                out += np.where(use, g, 0.0)
                count += use
    return out / count


def ms_step(eps, a, phase, phases, shape, E, E_prev, h, lam0=None, mu0=None, tol=1e-6,
            max_iter=1000, fixed_iter=False, newton_tol=1e-12, newton_max_iter=50):
    """One load step. Returns dict(eps, a, sigma, sigma_mean, iters, residual)."""
    if lam0 is None or mu0 is None:
        lam0, mu0 = reference_medium(phases)
    nz, ny, nx = shape
    n = nx * ny * nz
    E = np.asarray(E, dtype=np.float64)
    eps = np.array(eps, dtype=np.float64) + (E - np.asarray(E_prev, dtype=np.float64))[:, None]
    En = max(np.sqrt(tensor_sq(E)), 1e-300)
    err = 0.0
    it = 0
    for it in range(1, max_iter + 1):
        r = evaluate(eps, a, phase, phases, h=h, tol=newton_tol, max_iter=newton_max_iter)
        tr = lam0 * (eps[0] + eps[1] + eps[2])
        tau = r["sigma"].copy()
        tau[:3] -= tr + 2.0 * mu0 * eps[:3]
        tau[3:] -= mu0 * eps[3:]
        th = scipy.fft.rfftn(tau.reshape(6, nz, ny, nx), axes=(1, 2, 3))
        eh = gamma_apply(th, shape, lam0, mu0)
        eh[:, 0, 0, 0] = E * n
        new = scipy.fft.irfftn(eh, s=(nz, ny, nx), axes=(1, 2, 3)).reshape(6, n)
        err = np.sqrt(np.mean(tensor_sq(new - eps))) / En
        eps = new
        if not fixed_iter and err <= tol:
            break
    r = evaluate(eps, a, phase, phases, h=h, tol=newton_tol, max_iter=newton_max_iter)
    return dict(eps=eps, a=r["a_out"], sigma=r["sigma"], sigma_mean=r["sigma"].mean(axis=1),
                iters=it, residual=err)
