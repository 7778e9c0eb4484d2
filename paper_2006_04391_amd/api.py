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


def _field(t, name, rows, n=None, dev=None, dtype=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU (got {t.device}); there is no CPU path")
    dtype = torch.float64 if dtype is None else dtype
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
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
             a_out=None, sigma_out=None, tangent_out=None, write_a=True, return_iters=False,
             flags=0):
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
    if tangent:
        C = (torch.empty((36, n), dtype=torch.float64, device=dev) if tangent_out is None
             else _field(tangent_out, "tangent_out", 36, n, dev))
    else:
        C = None
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


def evaluate_conventional(eps, a_old, phase, phases, h=0.1, tol=1e-12, max_iter=50, *,
                          tangent=False, a_out=None, sigma_out=None, tangent_out=None):
    """Hand-reduced radial-return evaluation (the paper's conventional
    strategy). Returns (sigma, a_new[, C (36, n)], iters (n,) int32,
    failed-point count)."""
    eps = _field(eps, "eps", 6)
    n, dev = eps.shape[1], eps.device
    a_old = _field(a_old, "a_old", 6, n, dev)
    phase = _phase_ids(phase, n, dev)
    params = make_params(phases)
    sigma = torch.empty_like(eps) if sigma_out is None else _field(sigma_out, "sigma_out", 6, n, dev)
    a_new = torch.empty_like(a_old) if a_out is None else _field(a_out, "a_out", 6, n, dev)
    C = None
    if tangent:
        C = (torch.empty((36, n), dtype=torch.float64, device=dev) if tangent_out is None
             else _field(tangent_out, "tangent_out", 36, n, dev))
    iters = torch.empty(n, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    with torch.cuda.device(dev):
        rc = load().automat_evaluate_conventional_ex(n, _ptr(eps), _ptr(a_old), _ptr(phase),
                                                     ctypes.byref(params), float(h), float(tol),
                                                     int(max_iter), _ptr(sigma), _ptr(a_new),
                                                     _ptr(C), _ptr(iters), _ptr(count),
                                                     _stream(dev))
    check("automat_evaluate_conventional_ex", rc)
    if tangent:
        return sigma, a_new, C, iters, count
    return sigma, a_new, iters, count


def evaluate_f32(eps, a_old, phase, phases, h=0.1, tol=1e-6, max_iter=50, *, tangent=False,
                 a_out=None, sigma_out=None, tangent_out=None, write_a=True, return_iters=False):
    """Single-precision evaluation (float32 fields and arithmetic). Returns
    (sigma, a_new) plus the tangent (36, n) if ``tangent`` and (iters,
    nonconverged_count) if ``return_iters``."""
    f32 = torch.float32
    eps = _field(eps, "eps", 6, dtype=f32)
    n, dev = eps.shape[1], eps.device
    a_old = _field(a_old, "a_old", 6, n, dev, dtype=f32)
    phase = _phase_ids(phase, n, dev)
    params = make_params(phases)
    sigma = torch.empty_like(eps) if sigma_out is None else _field(sigma_out, "sigma_out", 6, n,
                                                                   dev, dtype=f32)
    if write_a:
        a_new = torch.empty_like(a_old) if a_out is None else _field(a_out, "a_out", 6, n, dev,
                                                                     dtype=f32)
    else:
        a_new = None
    if tangent:
        C = (torch.empty((36, n), dtype=f32, device=dev) if tangent_out is None
             else _field(tangent_out, "tangent_out", 36, n, dev, dtype=f32))
    else:
        C = None
    iters = torch.empty(n, dtype=torch.int32, device=dev) if return_iters else None
    count = torch.zeros(1, dtype=torch.int64, device=dev) if return_iters else None
    with torch.cuda.device(dev):
        rc = load().automat_evaluate_f32(n, _ptr(eps), _ptr(a_old), _ptr(phase),
                                         ctypes.byref(params), float(h), float(tol), int(max_iter),
                                         _ptr(sigma), _ptr(a_new), _ptr(C), _ptr(iters),
                                         _ptr(count), _stream(dev))
    check("automat_evaluate_f32", rc)
    out = (sigma, a_new) + ((C,) if tangent else ())
    if return_iters:
        out = out + (iters, count)
    return out


def evaluate_rk23(eps_n, eps_new, a_old, phase, phases, h=0.1, atol=1e-6, rtol=1e-3,
                  max_steps=100000, *, tangent=False, a_out=None, sigma_out=None,
                  tangent_out=None, _pair="rk23"):
    """Adaptive Bogacki-Shampine 3(2) evaluation over one load step with the
    strain moving linearly from eps_n to eps_new. Returns (sigma, a_new,
    steps (n,) int32, failed-point count), with the consistent tangent
    (36, n) after a_new if ``tangent`` (its entries then also enter the
    step size control)."""
    eps_n = _field(eps_n, "eps_n", 6)
    n, dev = eps_n.shape[1], eps_n.device
    eps_new = _field(eps_new, "eps_new", 6, n, dev)
    a_old = _field(a_old, "a_old", 6, n, dev)
    phase = _phase_ids(phase, n, dev)
    params = make_params(phases)
    sigma = torch.empty_like(eps_n) if sigma_out is None else _field(sigma_out, "sigma_out", 6, n, dev)
    a_new = torch.empty_like(a_old) if a_out is None else _field(a_out, "a_out", 6, n, dev)
    tan = None
    if tangent:
        tan = (torch.empty((36, n), dtype=torch.float64, device=dev) if tangent_out is None
               else _field(tangent_out, "tangent_out", 36, n, dev))
    steps = torch.empty(n, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    lib = load()
    with torch.cuda.device(dev):
        args = (n, _ptr(eps_n), _ptr(eps_new), _ptr(a_old), _ptr(phase), ctypes.byref(params),
                float(h), float(atol), float(rtol), int(max_steps), _ptr(sigma), _ptr(a_new))
        if tangent:
            entry = f"automat_evaluate_{_pair}_ex"
            rc = getattr(lib, entry)(*args, _ptr(tan), _ptr(steps), _ptr(count), _stream(dev))
        else:
            entry = f"automat_evaluate_{_pair}"
            rc = getattr(lib, entry)(*args, _ptr(steps), _ptr(count), _stream(dev))
    check(entry, rc)
    if tangent:
        return sigma, a_new, tan, steps, count
    return sigma, a_new, steps, count


def evaluate_rk12(eps_n, eps_new, a_old, phase, phases, h=0.1, atol=1e-6, rtol=1e-3,
                  max_steps=100000, *, tangent=False, a_out=None, sigma_out=None,
                  tangent_out=None):
    """As evaluate_rk23 with the Heun-Euler 2(1) pair (ode12)."""
    return evaluate_rk23(eps_n, eps_new, a_old, phase, phases, h, atol, rtol, max_steps,
                         tangent=tangent, a_out=a_out, sigma_out=sigma_out,
                         tangent_out=tangent_out, _pair="rk12")


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
                 mu0=0.0, newton_tol=1e-12, newton_max_iter=50, ref_update=False, warm_start=True,
                 device=None):
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
        opts.ref_update = 1 if ref_update else 0
        opts.warm_start = 1 if warm_start else 0
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

    def newton_failures(self):
        """Point solves of the last load step that did not converge."""
        c = ctypes.c_uint64()
        check("automat_ms_newton_failures", load().automat_ms_newton_failures(self._h,
                                                                             ctypes.byref(c)))
        return c.value

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

    def step_noalloc(self, phase, E_macro, h, eps, a, sigma_out=None):
        """step() through automat_ms_step_noalloc: the work space is the
        library's fixed device array, so the call allocates nothing (grids
        up to about 86^3, no reference update). Same returns as step()."""
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
            rc = load().automat_ms_step_noalloc(self._h, _ptr(phase), E, float(h), _ptr(eps),
                                                _ptr(a), _ptr(sigma_out), mean,
                                                ctypes.byref(iters), ctypes.byref(res),
                                                _stream(dev))
        check("automat_ms_step_noalloc", rc)
        return list(mean), iters.value, res.value

    def step_mixed(self, phase, E_macro, h, eps, a, stress_mask, S_macro=None, sigma_out=None):
        """Advance one load step under mixed conditions (automat_ms_step_mixed):
        bit c of stress_mask makes component c stress-controlled with mean
        stress S_macro[c] (zero if None). Returns (sigma_mean (6,), E reached
        (6,), iterations, last relative strain change)."""
        dev = self.device
        eps = _field(eps, "eps", 6, self.n, dev)
        a = _field(a, "a", 6, self.n, dev)
        phase = _phase_ids(phase, self.n, dev)
        if sigma_out is not None:
            sigma_out = _field(sigma_out, "sigma_out", 6, self.n, dev)
        E = (ctypes.c_double * 6)(*[float(x) for x in E_macro])
        S = (ctypes.c_double * 6)(*[float(x) for x in S_macro]) if S_macro is not None else None
        mean = (ctypes.c_double * 6)()
        Er = (ctypes.c_double * 6)()
        iters = ctypes.c_int32()
        res = ctypes.c_double()
        with torch.cuda.device(dev):
            rc = load().automat_ms_step_mixed(self._h, _ptr(phase), E, S, int(stress_mask),
                                              float(h), _ptr(eps), _ptr(a), _ptr(sigma_out), mean,
                                              Er, ctypes.byref(iters), ctypes.byref(res),
                                              _stream(dev))
        check("automat_ms_step_mixed", rc)
        return list(mean), list(Er), iters.value, res.value

    def adjoint_step(self, phase, h, eps, a_prev, a_next, w=None, grad_sigma=None, grad_a=None,
                     grad_a_prev=None, grad_params=None):
        """Reverse step of one converged load step (automat_ms_adjoint_step).
        Returns (dL/dE (6,), adjoint iterations, last relative change);
        grad_a_prev (6, n) receives dL/da_{k-1}, grad_params (n_phases, 7)
        accumulates dL/dp."""
        dev = self.device
        eps = _field(eps, "eps", 6, self.n, dev)
        a_prev = _field(a_prev, "a_prev", 6, self.n, dev)
        a_next = _field(a_next, "a_next", 6, self.n, dev)
        phase = _phase_ids(phase, self.n, dev)
        if grad_sigma is not None:
            grad_sigma = _field(grad_sigma, "grad_sigma", 6, self.n, dev)
        if grad_a is not None:
            grad_a = _field(grad_a, "grad_a", 6, self.n, dev)
        if grad_a_prev is not None:
            grad_a_prev = _field(grad_a_prev, "grad_a_prev", 6, self.n, dev)
        if grad_params is not None:
            grad_params = _field(grad_params, "grad_params", len(self.phases), _lib.NPAR, dev)
        wv = (ctypes.c_double * 6)(*[float(x) for x in w]) if w is not None else None
        gE = (ctypes.c_double * 6)()
        iters = ctypes.c_int32()
        res = ctypes.c_double()
        with torch.cuda.device(dev):
            rc = load().automat_ms_adjoint_step(
                self._h, _ptr(phase), float(h), _ptr(eps), _ptr(a_prev), _ptr(a_next), wv,
                _ptr(grad_sigma), _ptr(grad_a), gE, _ptr(grad_a_prev), _ptr(grad_params),
                ctypes.byref(iters), ctypes.byref(res), _stream(dev))
        check("automat_ms_adjoint_step", rc)
        return list(gE), iters.value, res.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().automat_ms_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ms_gradients(shape, phase, phases, loads, h, **opts):
    """Run the basic scheme over the load steps `loads` (macro strains E_1..E_K)
    from zero state, keeping each converged step (strain and internal
    variables) on the device, then differentiate the last step's mean
    stress by reverse steps. Returns dict(sigma_mean (6,), dsig_dE (6, K, 6):
    d mean(sigma_K)_j / d (E_k)_c, dsig_dp (6, n_phases, 7):
    d mean(sigma_K)_j / d p, forward and adjoint iteration counts)."""
    import numpy as np
    ms = MS(shape, phases, **opts)
    try:
        n, dev = ms.n, ms.device
        ph = _phase_ids(torch.as_tensor(np.ascontiguousarray(phase)).to(dev), n, dev)
        eps = torch.zeros((6, n), dtype=torch.float64, device=dev)
        a = torch.zeros_like(eps)
        states = [a.clone()]                 # a_0 .. a_K
        strains = []                         # eps_1 .. eps_K
        fwd_iters = []
        mean = None
        for E in loads:
            mean, it, _ = ms.step(ph, E, h, eps, a)
            strains.append(eps.clone())
            states.append(a.clone())
            fwd_iters.append(it)
        K = len(loads)
        dE = np.zeros((6, K, 6))
        dp = np.zeros((6, len(phases), _lib.NPAR))
        adj_iters = []
        ga = torch.empty_like(eps)
        ga_prev = torch.empty_like(eps)
        for j in range(6):
            w = [0.0] * 6
            w[j] = 1.0
            gp = torch.zeros((len(phases), _lib.NPAR), dtype=torch.float64, device=dev)
            carry = None
            for k in range(K - 1, -1, -1):
                gE, it, _ = ms.adjoint_step(ph, h, strains[k], states[k], states[k + 1],
                                            w=w if k == K - 1 else None, grad_a=carry,
                                            grad_a_prev=ga_prev if k > 0 else None,
                                            grad_params=gp)
                dE[j, k] = gE
                adj_iters.append(it)
                if k > 0:
                    ga, ga_prev = ga_prev, ga
                    carry = ga
            dp[j] = gp.cpu().numpy()
        return dict(sigma_mean=np.array(mean), dsig_dE=dE, dsig_dp=dp, fwd_iters=fwd_iters,
                    adj_iters=adj_iters)
    finally:
        ms.close()


def _phases_from_tensor(params, kinds):
    vals = params.detach().to("cpu", torch.float64).tolist()
    return [dict(kind=int(k), E=v[0], nu=v[1], H=v[2], sigma_y=v[3], sigma0=v[4], eps0=v[5], n=v[6])
            for k, v in zip(kinds, vals)]


class AutoMatFn(torch.autograd.Function):
    """Differentiable implicit-Euler evaluation.

    forward(eps (6, n), a_old (6, n), params (n_phases, 7), phase (n,), kinds,
            h, tol, max_iter) -> (sigma (6, n), a_new (6, n))

    params rows are (E, nu, H, sigma_y, sigma0, eps0, n) per phase and may
    require grad; kinds is a sequence of phase kinds (0 elastic, 1
    viscoplastic). The backward is the library's vector-Jacobian product
    (implicit function theorem through the converged Newton system; the step
    length carries no derivative)."""

    @staticmethod
    def forward(ctx, eps, a_old, params, phase, kinds, h=0.1, tol=1e-12, max_iter=50):
        phases = _phases_from_tensor(params, kinds)
        sigma, a_new = evaluate(eps.detach(), a_old.detach(), phase, phases, h, tol, max_iter)
        ctx.save_for_backward(eps, a_old, a_new, phase)
        ctx.phases = phases
        ctx.h = h
        ctx.params_device = params.device
        return sigma, a_new

    @staticmethod
    def backward(ctx, g_sigma, g_a):
        eps, a_old, a_new, phase = ctx.saved_tensors
        gs = g_sigma.contiguous() if g_sigma is not None else None
        ga = g_a.contiguous() if g_a is not None else None
        geps, gan, gpar = evaluate_backward(eps.detach(), a_old.detach(), a_new, phase, ctx.phases,
                                            ctx.h, gs, ga,
                                            want_a_old=ctx.needs_input_grad[1],
                                            want_params=ctx.needs_input_grad[2])
        if gpar is not None:
            gpar = gpar.to(ctx.params_device)
        return geps, gan, gpar, None, None, None, None, None


def automat(eps, a_old, params, phase, kinds, h=0.1, tol=1e-12, max_iter=50):
    """Functional form of AutoMatFn.apply."""
    return AutoMatFn.apply(eps, a_old, params, phase, tuple(kinds), h, tol, max_iter)


class Server:
    """Continuous-batching evaluation service (the library's
    automat_server_* entry points). submit() queues a request whose host
    arrays stay referenced here until its result is polled."""

    def __init__(self, budget_bytes, max_batch_points=0, sequential=False, device=None):
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = load().automat_server_create(ctypes.c_size_t(int(budget_bytes)),
                                              int(max_batch_points), 1 if sequential else 0,
                                              ctypes.byref(self._h))
        check("automat_server_create", rc)
        self._keep = {}

    def clock(self):
        return self.stats()["clock_s"]

    def submit(self, phase, phases, steps, E_final, noise_std, seed, h=0.1, tol=1e-12,
               max_iter=50, a_init=None, want_fields=False, arrival=-1.0):
        """phase: numpy uint8 (n,). Returns the request id; with want_fields
        the final sigma and a (6, n) arrive in the polled result."""
        import numpy as np
        phase = np.ascontiguousarray(phase, dtype=np.uint8)
        n = phase.shape[0]
        req = _lib.Request()
        req.n = n
        req.phase = phase.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        req.params = make_params(phases)
        req.h, req.tol, req.max_iter, req.steps = float(h), float(tol), int(max_iter), int(steps)
        for c in range(6):
            req.E_final[c] = float(E_final[c])
        req.noise_std = float(noise_std)
        req.seed = int(seed) & ((1 << 64) - 1)
        keep = [phase]
        if a_init is not None:
            a_init = np.ascontiguousarray(a_init, dtype=np.float64)
            req.a_init = a_init.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            keep.append(a_init)
        sig = a = None
        if want_fields:
            sig = np.empty((6, n))
            a = np.empty((6, n))
            req.sigma_host = sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            req.a_host = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        req.t_arrival = float(arrival)
        rid = ctypes.c_uint64()
        check("automat_server_submit", load().automat_server_submit(self._h, ctypes.byref(req),
                                                                     ctypes.byref(rid)))
        self._keep[rid.value] = (keep, sig, a)
        return rid.value

    def poll(self, max_results=1024):
        buf = (_lib.Result * max_results)()
        cnt = ctypes.c_int32()
        check("automat_server_poll", load().automat_server_poll(self._h, buf, max_results,
                                                                 ctypes.byref(cnt)))
        out = []
        for k in range(cnt.value):
            r = buf[k]
            d = dict(id=r.id, status=r.status, steps_done=r.steps_done, n=r.n,
                     nonconverged=r.nonconverged, t_arrival=r.t_arrival, t_admit=r.t_admit,
                     t_done=r.t_done)
            _, sig, a = self._keep.pop(r.id, (None, None, None))
            if sig is not None:
                d["sigma"], d["a"] = sig, a
            out.append(d)
        return out

    def stats(self):
        st = _lib.ServerStats()
        check("automat_server_stats", load().automat_server_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().automat_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
