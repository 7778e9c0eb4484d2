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
