"""Adaptive explicit Runge-Kutta evaluation on the GPU (Bogacki-Shampine 3(2)
and Heun-Euler 2(1)) vs the oracle, point by point on the same seeded inputs
(same accepted steps, results within the parity bar)."""
import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs
from tests.test_parity_gpu import TOL, N, T, rel_per_point

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


PAIRS = ["rk23", "rk12"]


def _run(e0, ps, h, pair="rk23", **kw):
    from paper_2006_04391_amd import api
    fn = getattr(api, "evaluate_" + pair)
    sig, a, steps, cnt = fn(T(e0), T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases, h=h, **kw)
    torch.cuda.synchronize()
    ref = getattr(oracle, "evaluate_" + pair)(e0, ps.eps, ps.a_old, ps.phase, ps.phases, h=h, **kw)
    return dict(sigma=N(sig), a_out=N(a), steps=N(steps), count=int(cnt.item())), ref


def _check(g, ref):
    assert np.array_equal(g["steps"], ref["steps"])
    ok = ref["steps"] >= 0
    assert rel_per_point(g["sigma"][:, ok], ref["sigma"][:, ok]).max() <= TOL
    assert rel_per_point(g["a_out"][:, ok], ref["a_out"][:, ok]).max() <= TOL
    assert g["count"] == int((ref["steps"] < 0).sum())


@pytest.mark.parametrize("pair", PAIRS)
@pytest.mark.parametrize("preset,n,seed", [("config", 4133, 1), ("paper", 1031, 2)])
def test_ramp_parity(preset, n, seed, pair):
    phases = inputs.config_phases() if preset == "config" else inputs.paper_phases()
    # loads that make the matrix flow enough for several steps
    e11, h = (2e-2, 10.0) if preset == "config" else (4e-3, 1.0)
    ps = inputs.points_random(n, seed=seed, phases=phases, e11=e11, std=3e-4, a_std=1e-4)
    e0 = 0.5 * ps.eps + 1e-4 * np.random.default_rng(seed).normal(size=ps.eps.shape)
    g, ref = _run(e0, ps, h=h, pair=pair)
    assert ref["steps"].max() > 1
    _check(g, ref)


@pytest.mark.parametrize("pair,rtol", [("rk23", 1e-9), ("rk12", 1e-6)])
def test_tight_tolerances_many_steps(pair, rtol):
    ps = inputs.points_random(700, seed=5, phases=inputs.paper_phases(), e11=6e-3, std=5e-4)
    e0 = np.zeros_like(ps.eps)
    g, ref = _run(e0, ps, h=1.0, pair=pair, atol=1e-3 * rtol, rtol=rtol)
    assert ref["steps"].max() > 20
    _check(g, ref)


@pytest.mark.parametrize("pair", PAIRS)
def test_invalid_points_and_step_limit(pair):
    ps = inputs.points_random(300, seed=6, phases=inputs.paper_phases(), e11=6e-3, std=5e-4)
    ps.eps[0, 7] = np.inf
    ps.phase[11] = 9
    e0 = np.zeros_like(ps.eps)
    g, ref = _run(e0, ps, h=1.0, pair=pair, max_steps=3)
    assert (ref["steps"] < 0).sum() > 2 and g["steps"][7] == -1 and g["steps"][11] == -1
    _check(g, ref)


@pytest.mark.parametrize("pair", PAIRS)
def test_empty_and_invalid_arguments(pair):
    from paper_2006_04391_amd import api, _lib
    fn = getattr(api, "evaluate_" + pair)
    ps = inputs.points_random(10, seed=7, phases=inputs.config_phases())
    z = T(np.zeros_like(ps.eps))
    with pytest.raises(_lib.AutomatError):
        fn(z, T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases, h=0.0)
    with pytest.raises(_lib.AutomatError):
        fn(z, T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases, rtol=0.0)
    e = torch.empty((6, 0), dtype=torch.float64, device="cuda")
    out = fn(e, e, e, torch.empty(0, dtype=torch.uint8, device="cuda"), ps.phases)
    assert out[0].shape == (6, 0)


def _run_tan(e0, ps, h, pair, **kw):
    from paper_2006_04391_amd import api
    fn = getattr(api, "evaluate_" + pair)
    sig, a, tan, steps, cnt = fn(T(e0), T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases, h=h,
                                 tangent=True, **kw)
    torch.cuda.synchronize()
    ref = getattr(oracle, "evaluate_" + pair)(e0, ps.eps, ps.a_old, ps.phase, ps.phases, h=h,
                                              tangent=True, **kw)
    return dict(sigma=N(sig), a_out=N(a), tangent=N(tan), steps=N(steps),
                count=int(cnt.item())), ref


@pytest.mark.parametrize("pair", PAIRS)
@pytest.mark.parametrize("preset,n,seed", [("config", 1031, 11), ("paper", 517, 12)])
def test_tangent_parity(preset, n, seed, pair):
    """Consistent tangent of the adaptive schemes: the sensitivity system is
    integrated with the same stages and steps, and its entries enter the
    error measure, so the accepted steps, the state and the tangent all
    match the oracle point by point."""
    phases = inputs.config_phases() if preset == "config" else inputs.paper_phases()
    e11, h = (2e-2, 10.0) if preset == "config" else (4e-3, 1.0)
    ps = inputs.points_random(n, seed=seed, phases=phases, e11=e11, std=3e-4, a_std=1e-4)
    e0 = 0.5 * ps.eps + 1e-4 * np.random.default_rng(seed).normal(size=ps.eps.shape)
    g, ref = _run_tan(e0, ps, h=h, pair=pair)
    assert ref["steps"].max() > 1
    _check(g, ref)
    ok = ref["steps"] >= 0
    assert rel_per_point(g["tangent"][:, ok], ref["tangent"][:, ok]).max() <= TOL
    # elastic points: the elastic stiffness exactly
    el = ps.phase == 1
    assert np.array_equal(g["tangent"][:, el], ref["tangent"][:, el])


@pytest.mark.parametrize("pair", PAIRS)
def test_tangent_invalid_points_and_step_limit(pair):
    ps = inputs.points_random(300, seed=13, phases=inputs.paper_phases(), e11=6e-3, std=5e-4)
    ps.eps[0, 7] = np.inf
    ps.phase[11] = 9
    e0 = np.zeros_like(ps.eps)
    g, ref = _run_tan(e0, ps, h=1.0, pair=pair, max_steps=3)
    assert (ref["steps"] < 0).sum() > 2 and g["steps"][7] == -1 and g["steps"][11] == -1
    _check(g, ref)
    assert np.all(np.isnan(g["tangent"][:, [7, 11]]))
    ok = ref["steps"] >= 0
    assert rel_per_point(g["tangent"][:, ok], ref["tangent"][:, ok]).max() <= TOL


@pytest.mark.parametrize("pair,rtol", [("rk23", 1e-6), ("rk12", 1e-4)])
def test_tangent_tight_tolerances_many_steps(pair, rtol):
    ps = inputs.points_random(300, seed=14, phases=inputs.paper_phases(), e11=6e-3, std=5e-4)
    e0 = np.zeros_like(ps.eps)
    g, ref = _run_tan(e0, ps, h=1.0, pair=pair, atol=1e-3 * rtol, rtol=rtol)
    assert ref["steps"].max() > 10
    _check(g, ref)
    ok = ref["steps"] >= 0
    assert rel_per_point(g["tangent"][:, ok], ref["tangent"][:, ok]).max() <= TOL


def test_tangent_argument_errors():
    from paper_2006_04391_amd import _lib, api
    ps = inputs.points_random(64, seed=15, phases=inputs.config_phases())
    e0, e1, a0, ph = T(np.zeros_like(ps.eps)), T(ps.eps), T(ps.a_old), T(ps.phase)
    L = _lib.load()
    params = _lib.make_params(ps.phases)
    sig = torch.empty_like(e1)
    an = torch.empty_like(e1)
    steps = torch.empty(ps.n, dtype=torch.int32, device="cuda")
    ptr = lambda t: t.data_ptr()
    for bad_tan in (sig, an, e1):            # the tangent must not overlap another array
        rc = L.automat_evaluate_rk23_ex(ps.n, ptr(e0), ptr(e1), ptr(a0), ptr(ph),
                                        _lib.ctypes.byref(params), 0.1, 1e-6, 1e-3, 100,
                                        ptr(sig), ptr(an), ptr(bad_tan), ptr(steps), None, None)
        assert rc == _lib.EINVAL
    # NULL tangent: the plain evaluation, same results as the plain entry point
    s1, a1, st1, _ = api.evaluate_rk23(e0, e1, a0, ph, ps.phases)
    rc = L.automat_evaluate_rk23_ex(ps.n, ptr(e0), ptr(e1), ptr(a0), ptr(ph),
                                    _lib.ctypes.byref(params), 0.1, 1e-6, 1e-3, 100000,
                                    ptr(sig), ptr(an), None, ptr(steps), None, None)
    torch.cuda.synchronize()
    assert rc == 0
    assert torch.equal(sig, s1) and torch.equal(an, a1) and torch.equal(steps, st1)


@pytest.mark.parametrize("pair", PAIRS)
def test_full_size_ramp_parity(pair):
    """The benchmark's adaptive leg: the 256^3 fibre batch with the strain
    ramping from 0.8 eps to eps over h = 0.1 s, in its launch configuration
    (a grid of four blocks per compute unit, so every wave strides over
    about 64 tiles): accepted steps, stress and internal variables of every
    point against the oracle."""
    from tests.test_parity_gpu import points_c1
    ps = points_c1()
    e0 = 0.8 * ps.eps
    g, ref = _run(e0, ps, h=ps.h, pair=pair)
    _check(g, ref)
    assert g["count"] == 0


@pytest.mark.parametrize("pair", PAIRS)
def test_strided_flowing_many_steps(pair):
    """More points than the grid holds resident threads (2^19 + 77), strongly
    flowing so that lanes of one wave take different numbers of steps
    across the stride loop."""
    n = (1 << 19) + 77
    ps = inputs.points_random(n, seed=16, phases=inputs.config_phases(), e11=2e-2, std=3e-4,
                              a_std=1e-4)
    e0 = 0.5 * ps.eps + 1e-4 * np.random.default_rng(16).normal(size=ps.eps.shape)
    g, ref = _run(e0, ps, h=10.0, pair=pair)
    assert ref["steps"].max() > 2
    _check(g, ref)


@pytest.mark.parametrize("pair", PAIRS)
def test_tangent_full_batch_128(pair):
    """The tangent kernels on the 128^3 fibre batch (2^21 points, one wave
    per 64 points) with the benchmark's ramp: accepted steps, state and all
    tangent entries of every point against the oracle."""
    ps = inputs.points_c1(N=128)
    e0 = 0.8 * ps.eps
    g, ref = _run_tan(e0, ps, h=ps.h, pair=pair)
    _check(g, ref)
    assert rel_per_point(g["tangent"], ref["tangent"]).max() <= TOL
