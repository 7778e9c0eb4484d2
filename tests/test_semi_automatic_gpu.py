"""Semi-automatic strategy on the GPU (hand-derived partials of omega and Psi
inside the generic Newton solve and tangent) vs the oracle, on the same
seeded inputs and with the same bar as the automatic kernel; and against the
automatic kernel itself."""
import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs
from tests.test_parity_gpu import N, T, TOL, check, rel_per_point

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu(ps, tangent, flags, h=None, max_iter=None):
    from paper_2006_04391_amd import api
    out = api.evaluate(T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases,
                       h=ps.h if h is None else h, tol=ps.tol,
                       max_iter=ps.max_iter if max_iter is None else max_iter, tangent=tangent,
                       return_iters=True, flags=flags)
    torch.cuda.synchronize()
    g = dict(sigma=N(out[0]), a_out=N(out[1]), iters=N(out[-2]), count=int(out[-1].item()))
    if tangent:
        g["tangent"] = N(out[2])
    return g


def _presets():
    out = []
    ps = inputs.points_random(256 * 5 + 37, seed=31, e11=2e-2, std=3e-3, a_std=1e-3)
    ps.phases = [dict(ps.phases[0], eps0=0.2), ps.phases[1]]
    out.append(("config", ps))
    out.append(("paper", inputs.points_random(256 * 3 + 1, seed=32, phases=inputs.paper_phases(),
                                              e11=1e-2, std=3e-3, a_std=1e-3)))
    ph = inputs.config_phases()
    ph[0] = dict(ph[0], H=900.0, sigma_y=4.0, eps0=0.5, n=3.3)
    out.append(("hardening", inputs.points_random(999, seed=33, phases=ph, e11=3e-2, std=5e-3,
                                                  a_std=2e-3)))
    ph = inputs.config_phases()
    ph[0] = dict(ph[0], n=1.0, eps0=0.1)
    out.append(("linear", inputs.points_random(300, seed=34, phases=ph, e11=3e-2, std=5e-3,
                                               a_std=2e-3)))
    ph = inputs.config_phases()
    ph[0] = dict(ph[0], H=400.0, sigma_y=6.0, eps0=0.3)      # x^6 by products
    out.append(("threshold_int", inputs.points_random(700, seed=35, phases=ph, e11=2e-2,
                                                      std=4e-3, a_std=1e-3)))
    return out


@pytest.mark.parametrize("name,ps", _presets(), ids=[p[0] for p in _presets()])
@pytest.mark.parametrize("tangent", [False, True])
def test_semi_automatic_matches_oracle(name, ps, tangent):
    from paper_2006_04391_amd import _lib
    g = _gpu(ps, tangent, _lib.HAND_PARTIALS)
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tol=ps.tol,
                          max_iter=ps.max_iter, tangent=tangent)
    check(g, ref, ps, tangent)
    assert g["count"] == 0


def test_semi_automatic_matches_automatic_on_the_c0_batch():
    from paper_2006_04391_amd import _lib
    ps = inputs.points_c0()
    a = _gpu(ps, True, 0)
    s = _gpu(ps, True, _lib.HAND_PARTIALS)
    for key in ("sigma", "a_out", "tangent"):
        assert rel_per_point(s[key], a[key]).max() <= 1e-12, key
    assert np.mean(s["iters"] == a["iters"]) > 0.99


def test_semi_automatic_many_iterations_and_sigma_flag():
    from paper_2006_04391_amd import _lib
    ps = inputs.points_random(700, seed=35, phases=inputs.paper_phases(), e11=3e-2, std=1e-2,
                              a_std=3e-3)
    g = _gpu(ps, True, _lib.HAND_PARTIALS, h=10.0)
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=10.0, tol=ps.tol,
                          max_iter=ps.max_iter, tangent=True)
    check(g, ref, ps, tangent=True)
    assert ref["iters"].max() >= 4
    g = _gpu(ps, False, _lib.HAND_PARTIALS | _lib.SIGMA_CRITERION)
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tol=ps.tol,
                          max_iter=ps.max_iter, flags=oracle.SIGMA_CRITERION)
    check(g, ref, ps)


def test_semi_automatic_full_size_parity():
    """The 256^3 fibre batch (the benchmark's launch configuration), every
    point against the oracle."""
    from paper_2006_04391_amd import _lib
    ps = inputs.points_c1()
    g = _gpu(ps, False, _lib.HAND_PARTIALS)
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tol=ps.tol,
                          max_iter=ps.max_iter)
    check(g, ref, ps)
    assert g["count"] == 0
