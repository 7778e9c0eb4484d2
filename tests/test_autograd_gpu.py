"""AutoMatFn (torch.autograd.Function over the HIP forward and backward)
against central finite differences in FP64 and against the oracle's VJP."""
import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs
from tests.test_parity_gpu import N, T

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KEYS = ("E", "nu", "H", "sigma_y", "sigma0", "eps0", "n")


def _setup(n=300, seed=60):
    ph = inputs.paper_phases()
    ph[0] = dict(ph[0], H=400.0, sigma_y=5.0)
    ps = inputs.points_random(n, seed=seed, phases=ph, e11=1e-2, std=3e-3, a_std=1e-3)
    params = torch.tensor([[p[k] for k in KEYS] for p in ph], dtype=torch.float64,
                          device="cuda")
    kinds = [p["kind"] for p in ph]
    return ps, params, kinds


def test_autograd_matches_oracle_vjp():
    from paper_2006_04391_amd import api
    ps, params, kinds = _setup()
    eps = T(ps.eps).requires_grad_(True)
    a_old = T(ps.a_old).requires_grad_(True)
    p = params.clone().requires_grad_(True)
    sigma, a_new = api.automat(eps, a_old, p, T(ps.phase), kinds, h=1.0, tol=1e-14, max_iter=100)
    rng = np.random.default_rng(0)
    gs, ga = rng.normal(size=(6, ps.n)), rng.normal(size=(6, ps.n)) * 1e3
    loss = (sigma * T(gs)).sum() + (a_new * T(ga)).sum()
    loss.backward()
    ref_f = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=1.0, tol=1e-14, max_iter=100)
    ref = oracle.backward(ps.eps, ps.a_old, ref_f["a_out"], ps.phase, ps.phases, 1.0, gs, ga)
    for got, want in ((eps.grad, ref["grad_eps"]), (a_old.grad, ref["grad_a_old"])):
        got = N(got)
        rel = np.abs(got - want).max(0) / np.maximum(np.abs(want).max(0), 1e-300)
        assert rel.max() <= 1e-9
    gp = N(p.grad)
    scale = np.abs(ref["grad_params"]).max(axis=0)
    assert np.all(np.abs(gp - ref["grad_params"]) <= 1e-9 * np.maximum(scale, 1e-300))


def test_autograd_central_differences():
    """d/dp of a scalar loss against central differences with relative
    steps 1e-6 for every parameter of the flowing phase and for strains."""
    from paper_2006_04391_amd import api
    ps, params, kinds = _setup(n=64, seed=61)
    rng = np.random.default_rng(1)
    gs = T(rng.normal(size=(6, ps.n)))
    ga = T(rng.normal(size=(6, ps.n)) * 1e3)

    def loss(eps, a_old, p):
        s, a = api.automat(eps, a_old, p, T(ps.phase), kinds, h=1.0, tol=1e-15, max_iter=100)
        return (s * gs).sum() + (a * ga).sum()

    eps, a_old = T(ps.eps), T(ps.a_old)
    p = params.clone().requires_grad_(True)
    e = eps.clone().requires_grad_(True)
    L = loss(e, a_old, p)
    L.backward()
    for k in range(7):
        st = 1e-6 * abs(float(params[0, k]))
        pp, pm = params.clone(), params.clone()
        pp[0, k] += st
        pm[0, k] -= st
        fd = (loss(eps, a_old, pp) - loss(eps, a_old, pm)).item() / (2 * st)
        got = float(p.grad[0, k])
        assert abs(fd - got) <= 1e-5 * max(abs(fd), abs(got)) + 1e-12, (KEYS[k], fd, got)
    d = T(rng.normal(size=(6, ps.n)) * 1e-4)
    fd = (loss(eps + 1e-4 * d, a_old, params) - loss(eps - 1e-4 * d, a_old, params)).item() / 2e-4
    got = float((e.grad * d).sum())
    assert abs(fd - got) <= 1e-6 * abs(got)


def test_gradcheck_small():
    from paper_2006_04391_amd import api
    ps, params, kinds = _setup(n=3, seed=62)
    eps = T(ps.eps).requires_grad_(True)
    a_old = T(ps.a_old).requires_grad_(True)

    def f(e, a):
        return api.automat(e, a, params, T(ps.phase), kinds, h=1.0, tol=1e-15, max_iter=100)

    assert torch.autograd.gradcheck(f, (eps, a_old), eps=1e-8, atol=1e-6, rtol=1e-5)
