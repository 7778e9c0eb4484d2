"""The hand-reduced radial-return kernel (the paper's conventional strategy)
against the oracle's full six-dimensional Newton solve of the same step."""
import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs
from tests.test_parity_gpu import TOL, N, T, rel_per_point

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(preset, n):
    if preset == "config":
        ps = inputs.points_random(n, seed=31, e11=2e-2, std=3e-3, a_std=1e-3)
        ps.phases = [dict(ps.phases[0], eps0=0.2), ps.phases[1]]
    elif preset == "paper":
        ps = inputs.points_random(n, seed=32, phases=inputs.paper_phases(), e11=1e-2, std=3e-3,
                                  a_std=1e-3)
    elif preset == "hardening":
        ph = inputs.config_phases()
        ph[0] = dict(ph[0], H=900.0, sigma_y=4.0, eps0=0.5, n=3.3)
        ps = inputs.points_random(n, seed=33, phases=ph, e11=3e-2, std=5e-3, a_std=2e-3)
    elif preset == "threshold_int":                 # x^5, x^4 by products
        ph = inputs.config_phases()
        ph[0] = dict(ph[0], H=400.0, sigma_y=6.0, eps0=0.3)
        ps = inputs.points_random(n, seed=35, phases=ph, e11=2e-2, std=4e-3, a_std=1e-3)
    else:
        ph = inputs.config_phases()
        ph[0] = dict(ph[0], n=1.0, eps0=0.1)
        ps = inputs.points_random(n, seed=34, phases=ph, e11=3e-2, std=5e-3, a_std=2e-3)
    return ps


@pytest.mark.parametrize("preset,n", [("config", 4133), ("paper", 1025), ("hardening", 999),
                                      ("linear", 300), ("threshold_int", 700)])
def test_radial_return_matches_the_automatic_solution(preset, n):
    from paper_2006_04391_amd import api
    ps = _case(preset, n)
    sig, a, it, cnt = api.evaluate_conventional(T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases,
                                                h=ps.h)
    torch.cuda.synchronize()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h)
    assert int(cnt.item()) == 0 and np.all(N(it) >= 0)
    assert rel_per_point(N(sig), ref["sigma"]).max() <= TOL
    assert rel_per_point(N(a), ref["a_out"]).max() <= TOL
    flow = (ref["iters"] > 0)
    assert flow.sum() > 0 and np.all(N(it)[flow] >= 1)
    if preset == "linear":
        assert N(it)[flow].max() <= 2           # n = 1: one step to the root, one to confirm


def test_c1_batch_and_invalid_points():
    from paper_2006_04391_amd import api
    ps = inputs.points_c0()
    ps.eps[2, 3] = np.nan
    ps.phase[9] = 7
    sig, a, it, cnt = api.evaluate_conventional(T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases,
                                                h=ps.h)
    torch.cuda.synchronize()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h)
    it = N(it)
    assert it[3] == -1 and it[9] == -1 and int(cnt.item()) == 2
    assert np.all(np.isnan(N(sig)[:, [3, 9]]))
    ok = np.ones(ps.n, bool)
    ok[[3, 9]] = False
    assert rel_per_point(N(sig)[:, ok], ref["sigma"][:, ok]).max() <= TOL


@pytest.mark.parametrize("preset,n", [("config", 4133), ("paper", 1025), ("hardening", 999),
                                      ("linear", 300), ("threshold_int", 700)])
def test_conventional_tangent_matches_the_oracle(preset, n):
    """The hand-derived radial-return tangent against the oracle's implicit
    function theorem tangent on the nonsymmetric Newton system."""
    from paper_2006_04391_amd import api
    ps = _case(preset, n)
    sig, a, C, it, cnt = api.evaluate_conventional(T(ps.eps), T(ps.a_old), T(ps.phase),
                                                   ps.phases, h=ps.h, tangent=True)
    torch.cuda.synchronize()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tangent=True)
    assert int(cnt.item()) == 0
    assert rel_per_point(N(sig), ref["sigma"]).max() <= TOL
    assert rel_per_point(N(a), ref["a_out"]).max() <= TOL
    assert rel_per_point(N(C), ref["tangent"]).max() <= TOL
    # symmetric (a Hessian of the condensed incremental potential)
    M = N(C).reshape(6, 6, -1)
    assert np.abs(M - M.transpose(1, 0, 2)).max() <= 1e-12 * np.abs(M).max()


def test_conventional_tangent_linear_flow_at_zero_deviator():
    """n = 1 without threshold: the flow is linear in the trial deviator, so
    hydrostatic points (q_tr = 0) still have the viscous tangent."""
    from paper_2006_04391_amd import api
    ps = _case("linear", 256)
    ps.eps[:] = 0.0
    ps.eps[:3] = 1e-3
    ps.a_old[:] = 0.0
    sig, a, C, it, cnt = api.evaluate_conventional(T(ps.eps), T(ps.a_old), T(ps.phase),
                                                   ps.phases, h=ps.h, tangent=True)
    torch.cuda.synchronize()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tangent=True)
    assert rel_per_point(N(C), ref["tangent"]).max() <= TOL
    # the matrix's shear stiffness is below the elastic one there
    m = ps.phase == 0
    mu = ps.phases[0]["E"] / (2 * (1 + ps.phases[0]["nu"]))
    assert m.sum() > 0 and np.all(N(C)[3 * 6 + 3, m] < 0.99 * mu)


def test_conventional_tangent_on_the_128_cubed_batch():
    """The fibre batch at 128^3 (2^21 points, the grid strides 4 times)."""
    from paper_2006_04391_amd import api
    ps = inputs.points_c1(N=128)
    sig, a, C, it, cnt = api.evaluate_conventional(T(ps.eps), T(ps.a_old), T(ps.phase),
                                                   ps.phases, h=ps.h, tangent=True)
    torch.cuda.synchronize()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tangent=True)
    assert int(cnt.item()) == 0
    assert rel_per_point(N(sig), ref["sigma"]).max() <= TOL
    assert rel_per_point(N(a), ref["a_out"]).max() <= TOL
    assert rel_per_point(N(C), ref["tangent"]).max() <= TOL


def test_conventional_tangent_arguments():
    from paper_2006_04391_amd import _lib, api
    ps = _case("config", 300)
    e, a0, ph = T(ps.eps), T(ps.a_old), T(ps.phase)
    L = _lib.load()
    params = _lib.make_params(ps.phases)
    sig = torch.empty_like(e)
    an = torch.empty_like(e)
    it = torch.empty(ps.n, dtype=torch.int32, device="cuda")
    p = lambda t: t.data_ptr()
    for bad in (sig, an, e, a0):
        rc = L.automat_evaluate_conventional_ex(ps.n, p(e), p(a0), p(ph), _lib.ctypes.byref(params),
                                                0.1, 1e-12, 50, p(sig), p(an), p(bad), p(it),
                                                None, None)
        assert rc == _lib.EINVAL
    s1, a1, i1, _ = api.evaluate_conventional(e, a0, ph, ps.phases)
    rc = L.automat_evaluate_conventional_ex(ps.n, p(e), p(a0), p(ph), _lib.ctypes.byref(params),
                                            0.1, 1e-12, 50, p(sig), p(an), None, p(it), None, None)
    torch.cuda.synchronize()
    assert rc == 0
    assert torch.equal(sig, s1) and torch.equal(an, a1) and torch.equal(it, i1)
