"""Torch-facing binding of libautomat: device memory and streams come from
torch, every computation runs in the library's HIP kernels.

Tensors: fields are float64 CUDA tensors of shape (6, n) (tangent (36, n)),
contiguous, component-major; phase ids uint8 (n,). Calls are enqueued on the
current torch stream of the tensors' device.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check, load, make_params


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _field(t, name, rows, n=None, dev=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU (got {t.device}); there is no CPU path")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.dim() != 2 or t.shape[0] != rows or (n is not None and t.shape[1] != n):
        raise ValueError(f"{name} must have shape ({rows}, n)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dev is not None and t.device != dev:
        raise ValueError(f"{name} is on {t.device}, expected {dev}")
    return t


def _phase_ids(t, n, dev):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or t.dim() != 1 or t.shape[0] != n:
        raise ValueError("phase must be a uint8 tensor of shape (n,)")
    if t.device != dev or not t.is_contiguous():
        raise ValueError("phase must be contiguous and on the fields' device")
    return t


def evaluate(eps, a_old, phase, phases, h=0.1, tol=1e-12, max_iter=50, *, tangent=False,
             a_out=None, sigma_out=None, write_a=True, return_iters=False, flags=0):
    """One implicit-Euler evaluation of every point.

    Returns (sigma, a_new) plus the tangent (36, n) if ``tangent`` and
    (iters, nonconverged_count) if ``return_iters``. ``a_out`` may be
    ``a_old`` for an in-place update; ``write_a=False`` skips the state
    write (a_new is then None).
    """
    eps = _field(eps, "eps", 6)
    n, dev = eps.shape[1], eps.device
    a_old = _field(a_old, "a_old", 6, n, dev)
    phase = _phase_ids(phase, n, dev)
    params = make_params(phases)
    sigma = torch.empty_like(eps) if sigma_out is None else _field(sigma_out, "sigma_out", 6, n, dev)
    if write_a:
        a_new = torch.empty_like(a_old) if a_out is None else _field(a_out, "a_out", 6, n, dev)
    else:
        a_new = None
    C = torch.empty((36, n), dtype=torch.float64, device=dev) if tangent else None
    iters = torch.empty(n, dtype=torch.int32, device=dev) if return_iters else None
    count = torch.zeros(1, dtype=torch.int64, device=dev) if return_iters else None
    lib = load()
    with torch.cuda.device(dev):
        rc = lib.automat_evaluate_ex(n, _ptr(eps), _ptr(a_old), _ptr(phase), ctypes.byref(params),
                                     float(h), float(tol), int(max_iter), _ptr(sigma), _ptr(a_new),
                                     _ptr(C), _ptr(iters), _ptr(count), int(flags), _stream(dev))
    check("automat_evaluate_ex", rc)
    out = [sigma, a_new]
    if tangent:
        out.append(C)
    if return_iters:
        out += [iters, count]
    return tuple(out)


def evaluate_backward(eps, a_old, a_new, phase, phases, h, grad_sigma=None, grad_a=None, *,
                      want_a_old=True, want_params=True):
    """Vector-Jacobian product at a converged evaluation.

    Returns (grad_eps, grad_a_old or None, grad_params (n_phases, 7) or None)."""
    eps = _field(eps, "eps", 6)
    n, dev = eps.shape[1], eps.device
    a_old = _field(a_old, "a_old", 6, n, dev)
    a_new = _field(a_new, "a_new", 6, n, dev)
    phase = _phase_ids(phase, n, dev)
    if grad_sigma is not None:
        grad_sigma = _field(grad_sigma, "grad_sigma", 6, n, dev)
    if grad_a is not None:
        grad_a = _field(grad_a, "grad_a", 6, n, dev)
    params = make_params(phases)
    geps = torch.empty_like(eps)
    gan = torch.empty_like(eps) if want_a_old else None
    gpar = torch.zeros((len(phases), _lib.NPAR), dtype=torch.float64, device=dev) if want_params else None
    lib = load()
    with torch.cuda.device(dev):
        rc = lib.automat_evaluate_backward(n, _ptr(eps), _ptr(a_old), _ptr(a_new), _ptr(phase),
                                           ctypes.byref(params), float(h), _ptr(grad_sigma),
                                           _ptr(grad_a), _ptr(geps), _ptr(gan), _ptr(gpar),
                                           _stream(dev))
    check("automat_evaluate_backward", rc)
    return geps, gan, gpar


def version() -> str:
    return load().automat_version().decode()


class MS:
    """Moulinec-Suquet basic-scheme solver on a periodic grid (the library's
    automat_ms_* entry points). shape = (nz, ny, nx), x fastest."""

    def __init__(self, shape, phases, *, tol=1e-6, max_iter=1000, fixed_iter=False, lambda0=0.0,
                 mu0=0.0, newton_tol=1e-12, newton_max_iter=50, device=None):
        if isinstance(shape, int):
            shape = (shape, shape, shape)
        self.shape = tuple(int(s) for s in shape)
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        self.phases = list(phases)
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self._params = make_params(self.phases)
        opts = _lib.MsOptions()
        opts.tol = float(tol)
        opts.max_iter = int(max_iter)
        opts.fixed_iter = 1 if fixed_iter else 0
        opts.lambda0 = float(lambda0)
        opts.mu0 = float(mu0)
        opts.newton_tol = float(newton_tol)
        opts.newton_max_iter = int(newton_max_iter)
        self._opts = opts
        self._h = ctypes.c_void_p()
        lib = load()
        nz, ny, nx = self.shape
        with torch.cuda.device(self.device):
            rc = lib.automat_ms_create(nx, ny, nz, ctypes.byref(self._params), ctypes.byref(opts),
                                       ctypes.byref(self._h))
        check("automat_ms_create", rc)

    def reference(self):
        lam, mu = ctypes.c_double(), ctypes.c_double()
        check("automat_ms_reference", load().automat_ms_reference(self._h, ctypes.byref(lam),
                                                                   ctypes.byref(mu)))
        return lam.value, mu.value

    def set_macro(self, E_prev):
        E = (ctypes.c_double * 6)(*[float(x) for x in E_prev])
        check("automat_ms_set_macro", load().automat_ms_set_macro(self._h, E))

    def step(self, phase, E_macro, h, eps, a, sigma_out=None):
        """Advance one load step in place (eps, a). Returns (sigma_mean (6,),
        iterations, last relative strain change)."""
        dev = self.device
        eps = _field(eps, "eps", 6, self.n, dev)
        a = _field(a, "a", 6, self.n, dev)
        phase = _phase_ids(phase, self.n, dev)
        if sigma_out is not None:
            sigma_out = _field(sigma_out, "sigma_out", 6, self.n, dev)
        E = (ctypes.c_double * 6)(*[float(x) for x in E_macro])
        mean = (ctypes.c_double * 6)()
        iters = ctypes.c_int32()
        res = ctypes.c_double()
        with torch.cuda.device(dev):
            rc = load().automat_ms_step(self._h, _ptr(phase), E, float(h), _ptr(eps), _ptr(a),
                                        _ptr(sigma_out), mean, ctypes.byref(iters),
                                        ctypes.byref(res), _stream(dev))
        check("automat_ms_step", rc)
        return list(mean), iters.value, res.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().automat_ms_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
