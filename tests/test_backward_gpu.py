"""Vector-Jacobian product on the GPU vs the oracle's hand-derived one."""
import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs
from tests.test_parity_gpu import N, T, rel_per_point

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _case(preset, n, seed):
    if preset == "paper":
        ps = inputs.points_random(n, seed=seed, phases=inputs.paper_phases(), e11=1e-2, std=3e-3,
                                  a_std=1e-3)
    elif preset == "threshold":
        ph = inputs.config_phases()
        ph[0] = dict(ph[0], H=900.0, sigma_y=4.0, eps0=0.5, n=3.3)
        ps = inputs.points_random(n, seed=seed, phases=ph, e11=3e-2, std=5e-3, a_std=2e-3)
    elif preset == "linear":
        ph = inputs.config_phases()
        ph[0] = dict(ph[0], n=1.0, eps0=0.1)
        ps = inputs.points_random(n, seed=seed, phases=ph, e11=3e-2, std=5e-3, a_std=2e-3)
    else:
        ps = inputs.points_random(n, seed=seed)
    return ps


@pytest.mark.parametrize("preset,n", [("config", 256 * 4 + 3), ("paper", 777),
                                      ("threshold", 1500), ("linear", 300)])
@pytest.mark.parametrize("which", ["both", "sigma_only", "a_only"])
def test_backward_parity(preset, n, which):
    from paper_2006_04391_amd import api
    ps = _case(preset, n, seed=40 + n)
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, tol=1e-14, max_iter=100)
    rng = np.random.default_rng(n)
    gs = rng.normal(size=(6, ps.n)) if which != "a_only" else None
    ga = rng.normal(size=(6, ps.n)) * 1e3 if which != "sigma_only" else None
    b_ref = oracle.backward(ps.eps, ps.a_old, ref["a_out"], ps.phase, ps.phases, ps.h, gs, ga)
    ge, gan, gp = api.evaluate_backward(T(ps.eps), T(ps.a_old), T(ref["a_out"]), T(ps.phase),
                                        ps.phases, ps.h, None if gs is None else T(gs),
                                        None if ga is None else T(ga))
    torch.cuda.synchronize()
    assert rel_per_point(N(ge), b_ref["grad_eps"]).max() <= TOL
    assert rel_per_point(N(gan), b_ref["grad_a_old"]).max() <= TOL
    gp = N(gp)
    scale = np.abs(b_ref["grad_params"]).max(axis=0, keepdims=True)
    err = np.abs(gp - b_ref["grad_params"])
    # sums over points in a different order: relative to the largest phase sum
    assert np.all(err <= 1e-9 * np.maximum(scale, 1e-300) + 1e-300), (gp, b_ref["grad_params"])


def test_backward_accumulates_and_handles_invalid_phase():
    from paper_2006_04391_amd import api
    ps = _case("paper", 600, seed=77)
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases)
    gs = np.ones((6, ps.n))
    ge1, _, gp1 = api.evaluate_backward(T(ps.eps), T(ps.a_old), T(ref["a_out"]), T(ps.phase),
                                        ps.phases, ps.h, T(gs), None)
    ph = ps.phase.copy()
    ph[3] = 200
    ge2, gan2, gp2 = api.evaluate_backward(T(ps.eps), T(ps.a_old), T(ref["a_out"]), T(ph),
                                           ps.phases, ps.h, T(gs), None)
    torch.cuda.synchronize()
    assert np.all(np.isnan(N(ge2)[:, 3])) and np.all(np.isnan(N(gan2)[:, 3]))
    keep = np.ones(ps.n, bool)
    keep[3] = False
    assert np.array_equal(N(ge2)[:, keep], N(ge1)[:, keep])
    assert np.all(np.isfinite(N(gp2)))


def test_backward_full_batch_128():
    """The vector-Jacobian product on the 128^3 fibre batch (2^21 points:
    the grid of four blocks per compute unit strides over 8 tiles per
    block), random cotangents, against the oracle's hand-derived product."""
    from paper_2006_04391_amd import api
    ps = inputs.points_c1(N=128)
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, tol=1e-14, max_iter=100)
    rng = np.random.default_rng(128)
    gs = rng.normal(size=(6, ps.n))
    ga = rng.normal(size=(6, ps.n)) * 1e3
    b_ref = oracle.backward(ps.eps, ps.a_old, ref["a_out"], ps.phase, ps.phases, ps.h, gs, ga)
    ge, gan, gp = api.evaluate_backward(T(ps.eps), T(ps.a_old), T(ref["a_out"]), T(ps.phase),
                                        ps.phases, ps.h, T(gs), T(ga))
    torch.cuda.synchronize()
    assert rel_per_point(N(ge), b_ref["grad_eps"]).max() <= TOL
    assert rel_per_point(N(gan), b_ref["grad_a_old"]).max() <= TOL
    gp = N(gp)
    scale = np.abs(b_ref["grad_params"]).max(axis=0, keepdims=True)
    assert np.all(np.abs(gp - b_ref["grad_params"]) <= 1e-9 * np.maximum(scale, 1e-300)), \
        (gp, b_ref["grad_params"])
