"""GPU path vs the CPU oracle, element by element on the same seeded inputs.

Bar (per point, per output): ||x_gpu - x_oracle||_inf / ||x_oracle||_inf
<= 1e-10 for stress, internal variables and tangent; where the oracle value is
exactly zero the GPU value must be exactly zero. Elastic points must return
a_{n+1} = a_n bitwise.
"""
import functools

import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _dev():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch.device("cuda:0")


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


def N(t):
    return t.detach().cpu().numpy()


def rel_per_point(x, y):
    """max_c |x - y| / max_c |y| per column; 0/0 -> 0, x/0 -> inf."""
    num = np.abs(x - y).max(axis=0)
    den = np.abs(y).max(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(den > 0, num / den, np.where(num > 0, np.inf, 0.0))
    return r


def run_both(ps, tangent=False, flags=0, max_iter=None, h=None):
    from paper_2006_04391_amd import api
    mi = ps.max_iter if max_iter is None else max_iter
    hh = ps.h if h is None else h
    out = api.evaluate(T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases, h=hh, tol=ps.tol,
                       max_iter=mi, tangent=tangent, return_iters=True, flags=flags)
    torch.cuda.synchronize()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=hh, tol=ps.tol, max_iter=mi,
                          tangent=tangent, flags=flags)
    g = dict(sigma=N(out[0]), a_out=N(out[1]))
    if tangent:
        g["tangent"] = N(out[2])
    g["iters"] = N(out[-2])
    g["count"] = int(out[-1].item())
    return g, ref


def check(g, ref, ps, tangent=False):
    for key in ("sigma", "a_out") + (("tangent",) if tangent else ()):
        r = rel_per_point(g[key], ref[key])
        assert r.max() <= TOL, (key, r.max(), int(r.argmax()))
    kinds = np.array([p["kind"] for p in ps.phases] + [-1] * 256)
    el = kinds[ps.phase] == 0
    assert np.array_equal(g["a_out"][:, el].view(np.uint64), ps.a_old[:, el].view(np.uint64))
    assert np.all(g["iters"][el] == 0)
    assert np.all((g["iters"] >= 0) == (ref["iters"] >= 0))
    # iteration counts agree except where rounding decides at the threshold
    assert np.mean(g["iters"] == ref["iters"]) > 0.99


@pytest.mark.parametrize("tangent", [False, True])
def test_c0_4096_points(tangent):
    ps = inputs.points_c0()
    g, ref = run_both(ps, tangent=tangent)
    check(g, ref, ps, tangent)
    assert g["count"] == 0


@pytest.mark.parametrize("preset,n", [("config", 256 * 5 + 37), ("paper", 256 * 3 + 1),
                                      ("hardening", 999), ("linear", 300),
                                      ("threshold_int", 700), ("n3", 513)])
def test_random_presets_ragged(preset, n):
    """Several tiles plus a ragged tail, in the nonlinear regimes (integer
    exponents take the power by products, the others exp/log)."""
    if preset == "config":
        ps = inputs.points_random(n, seed=21, e11=2e-2, std=3e-3, a_std=1e-3)
        ps.phases = [dict(ps.phases[0], eps0=0.2), ps.phases[1]]
    elif preset == "paper":
        ps = inputs.points_random(n, seed=22, phases=inputs.paper_phases(), e11=1e-2, std=3e-3,
                                  a_std=1e-3)
    elif preset == "hardening":
        ph = inputs.config_phases()
        ph[0] = dict(ph[0], H=900.0, sigma_y=4.0, eps0=0.5, n=3.3)
        ps = inputs.points_random(n, seed=23, phases=ph, e11=3e-2, std=5e-3, a_std=2e-3)
    elif preset == "linear":
        ph = inputs.config_phases()
        ph[0] = dict(ph[0], n=1.0, eps0=0.1)
        ps = inputs.points_random(n, seed=24, phases=ph, e11=3e-2, std=5e-3, a_std=2e-3)
    elif preset == "threshold_int":                 # x^6 with a yield threshold
        ph = inputs.config_phases()
        ph[0] = dict(ph[0], H=400.0, sigma_y=6.0, eps0=0.3)
        ps = inputs.points_random(n, seed=28, phases=ph, e11=2e-2, std=4e-3, a_std=1e-3)
    else:                                           # n = 3: u^2 without threshold
        ph = inputs.config_phases()
        ph[0] = dict(ph[0], n=3.0, eps0=0.05)
        ps = inputs.points_random(n, seed=29, phases=ph, e11=2e-2, std=4e-3, a_std=1e-3)
    for tangent in (False, True):
        g, ref = run_both(ps, tangent=tangent)
        check(g, ref, ps, tangent)


def test_large_step_many_iterations_and_damping_regime():
    """h = 10 s with the paper preset at 3 % strain: many Newton updates."""
    ps = inputs.points_random(700, seed=25, phases=inputs.paper_phases(), e11=3e-2, std=1e-2,
                              a_std=3e-3)
    g, ref = run_both(ps, tangent=True, h=10.0)
    check(g, ref, ps, tangent=True)
    assert ref["iters"].max() >= 4


def test_sigma_criterion_flag():
    ps = inputs.points_random(1000, seed=26, phases=inputs.paper_phases(), e11=1e-2, std=2e-3)
    g, ref = run_both(ps, flags=oracle.SIGMA_CRITERION)
    check(g, ref, ps)


def test_hydrostatic_points_do_not_flow():
    ps = inputs.points_c0(n=512)
    ps.eps[:] = 0.0
    ps.eps[:3] = 1e-3
    g, ref = run_both(ps, tangent=True)
    check(g, ref, ps, tangent=True)
    assert np.all(g["iters"] == 0)


def test_nonconvergence_and_invalid_points_flagged():
    from paper_2006_04391_amd import api
    ps = inputs.points_random(300, seed=27, phases=inputs.paper_phases(), e11=5e-2, std=1e-2,
                              a_std=1e-3, incl_frac=0.3)
    ps.eps[1, 5] = np.nan
    ps.phase[7] = 9                          # no such phase
    g, ref = run_both(ps, max_iter=1, h=5.0)
    assert np.array_equal(g["iters"] < 0, ref["iters"] < 0)
    assert g["count"] == int(np.sum(ref["iters"] < 0))
    for idx in (5, 7):
        assert g["iters"][idx] == -1
        assert np.all(np.isnan(g["sigma"][:, idx])) and np.all(np.isnan(g["a_out"][:, idx]))
    ok = ref["iters"] >= 0
    r = rel_per_point(g["sigma"][:, ok], ref["sigma"][:, ok])
    assert r.max() <= TOL
    # non-converged points keep the iterate after one update, like the oracle
    bad = (ref["iters"] < 0) & np.all(np.isfinite(ref["sigma"]), axis=0)
    assert bad.sum() > 0
    r = rel_per_point(g["a_out"][:, bad], ref["a_out"][:, bad])
    assert r.max() <= 1e-8


def test_in_place_update_and_skipped_outputs():
    from paper_2006_04391_amd import api
    ps = inputs.points_random(2000, seed=28)
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, tangent=False)
    a = T(ps.a_old)
    sig, a2 = api.evaluate(T(ps.eps), a, T(ps.phase), ps.phases, a_out=a)
    torch.cuda.synchronize()
    assert a2.data_ptr() == a.data_ptr()
    assert rel_per_point(N(a), ref["a_out"]).max() <= TOL
    sig, none = api.evaluate(T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases, write_a=False)
    assert none is None
    assert rel_per_point(N(sig), ref["sigma"]).max() <= TOL


def test_empty_and_single_point():
    from paper_2006_04391_amd import api
    ps = inputs.points_c0(n=1)
    e = torch.empty((6, 0), dtype=torch.float64, device=_dev())
    p = torch.empty((0,), dtype=torch.uint8, device=_dev())
    s, a = api.evaluate(e, e.clone(), p, ps.phases)
    assert s.shape == (6, 0)
    g, ref = run_both(ps, tangent=True)
    check(g, ref, ps, tangent=True)


def test_invalid_arguments():
    from paper_2006_04391_amd import api, _lib
    ps = inputs.points_c0(n=64)
    args = (T(ps.eps), T(ps.a_old), T(ps.phase))
    for kw in (dict(h=0.0), dict(h=float("nan")), dict(tol=0.0), dict(max_iter=0), dict(flags=8)):
        with pytest.raises(_lib.AutomatError) as e:
            api.evaluate(*args, ps.phases, **kw)
        assert e.value.code == _lib.EINVAL
    for bad in ([dict(ps.phases[0], nu=0.5), ps.phases[1]],
                [dict(ps.phases[0], n=0.5), ps.phases[1]],
                [dict(ps.phases[0], sigma0=0.0), ps.phases[1]],
                [dict(ps.phases[0], kind=2), ps.phases[1]]):
        with pytest.raises(_lib.AutomatError):
            api.evaluate(*args, bad)
    with pytest.raises(ValueError):
        api.evaluate(*args, ps.phases * 9)


def test_many_phases_table():
    """16 phases with jittered parameters, phase ids spread over all of them."""
    rng = np.random.default_rng(29)
    phases = []
    for k in range(16):
        base = inputs.paper_phases()[k % 2]
        phases.append(inputs.jitter_phases([base], rng)[0])
    ps = inputs.points_random(3000, seed=30, phases=phases, e11=1e-2, std=2e-3, a_std=1e-3)
    ps.phase = rng.integers(0, 16, ps.n).astype(np.uint8)
    ps.a_old[:, [phases[p]["kind"] == 0 for p in ps.phase]] = 0.0
    g, ref = run_both(ps, tangent=True)
    check(g, ref, ps, tangent=True)


@functools.lru_cache(maxsize=1)
def points_c1():
    return inputs.points_c1()


def test_c1_full_size_parity():
    """The 256^3 fibre batch in the benchmark's launch configuration: every
    point against the oracle."""
    from paper_2006_04391_amd import api
    ps = points_c1()
    out = api.evaluate(T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases, h=ps.h, tol=ps.tol,
                       max_iter=ps.max_iter, return_iters=True)
    torch.cuda.synchronize()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tol=ps.tol,
                          max_iter=ps.max_iter)
    g = dict(sigma=N(out[0]), a_out=N(out[1]), iters=N(out[2]), count=int(out[3].item()))
    del out
    check(g, ref, ps)
    assert g["count"] == 0
    assert abs(float(np.mean(ps.phase)) - 0.15) < 0.01


def test_c1_full_size_tangent_parity():
    """The 256^3 fibre batch with the consistent tangent, in the benchmark's
    launch configuration (four rounds of resident blocks, so every wave
    strides over many chunks and its LDS ring wraps): stress, internal
    variables and all 36 tangent entries of every point against the
    oracle, compared in slices to bound host memory."""
    from paper_2006_04391_amd import api
    ps = points_c1()
    n = ps.n
    tan = torch.empty((36, n), dtype=torch.float64, device=_dev())
    sig, a_new, C, iters, cnt = api.evaluate(T(ps.eps), T(ps.a_old), T(ps.phase), ps.phases,
                                             h=ps.h, tol=ps.tol, max_iter=ps.max_iter,
                                             tangent=True, tangent_out=tan, return_iters=True)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tol=ps.tol,
                          max_iter=ps.max_iter, tangent=True)
    g = dict(sigma=N(sig), a_out=N(a_new), iters=N(iters), count=0)
    del sig, a_new
    check(g, ref, ps)
    step = 1 << 21
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        r = rel_per_point(N(C[:, lo:hi]), ref["tangent"][:, lo:hi])
        assert r.max() <= TOL, (lo, r.max(), lo + int(r.argmax()))
