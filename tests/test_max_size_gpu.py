"""Maximum sizes: fields of more than 2^31 elements.

The point kernels address component c of point i of a component-major field
at c n + i (36 components for a tangent) in 64-bit arithmetic, so a batch
may hold more points than a 32-bit element index reaches: 6 n > 2^31 for
the state and stress fields (n > 357,913,941) and 36 n > 2^31 for a tangent
(n > 59,652,323). Each test tiles a seeded 4096-point set along the points
to such an n, with a ragged last tile, runs the HIP path once over the whole
batch and compares every output element on the device with the oracle's
result for the same base point, at the bar of the corresponding parity test
(1e-10 per point in FP64; the single-precision bars for FP32). Exact
quantities (accepted step counts, elastic points returning a_n bit for bit)
are compared exactly; the parameter gradients of the backward, a sum over
all points, against the base sums times the tile count within 1e-10 of the
sum of the per-point magnitudes (the bound of the summation's rounding).
These batches take up to about 130 GB of device memory."""
import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10
TOL32 = 5e-5
B = 4096
N_STATE = 92160 * B + 1000    # 6 n = 2.26e9 > 2^31
N_TANGENT = 15000 * B + 1000  # 36 n = 2.21e9 > 2^31
GB = 1 << 30


def _dev(need_bytes):
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info(0)
    if need_bytes > 0.9 * free:
        pytest.skip(f"needs {need_bytes / GB:.0f} GiB of device memory, {free / GB:.0f} GiB free")
    return torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _release():
    yield
    if torch.cuda.is_available():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


def _tile(base, n, dev, dtype=None):
    """Device tensor with base[..., j] at every point i = j (mod B); the last
    tile is cut short. base: (rows, B) or (B,)."""
    b = torch.from_numpy(np.ascontiguousarray(base)).to(dev)
    if dtype is not None:
        b = b.to(dtype)
    full, tail = divmod(n, B)
    if b.dim() == 1:
        out = torch.empty(n, dtype=b.dtype, device=dev)
        out[:full * B].view(full, B).copy_(b.unsqueeze(0).expand(full, B))
        out[full * B:].copy_(b[:tail])
    else:
        rows = b.shape[0]
        out = torch.empty((rows, n), dtype=b.dtype, device=dev)
        out[:, :full * B].view(rows, full, B).copy_(b.unsqueeze(1).expand(rows, full, B))
        out[:, full * B:].copy_(b[:, :tail])
    return out


def _slices(n):
    """The batch in slices of about 2^22 points: (lo, hi, whole tiles in it),
    tiles None for the ragged last tile."""
    full, tail = divmod(n, B)
    step = max(1, (1 << 22) // B)
    for t0 in range(0, full, step):
        t1 = min(full, t0 + step)
        yield t0 * B, t1 * B, t1 - t0
    if tail:
        yield full * B, n, None


def _view(x, lo, hi, tiles):
    if x.dim() == 1:
        s = x[lo:hi]
        return s.view(tiles, B) if tiles else s
    s = x[:, lo:hi]
    return s.view(x.shape[0], tiles, B) if tiles else s


def _worst(got, ref, den):
    """max over points of max_c |got - ref| / den (point's reference scale;
    where den = 0 the difference must be 0). got: (rows, n) on the device,
    ref: (rows, B) and den: (B,) from the oracle on the base set."""
    dev = got.device
    r = torch.from_numpy(np.ascontiguousarray(ref, dtype=np.float64)).to(dev)
    d = torch.from_numpy(np.ascontiguousarray(den, dtype=np.float64)).to(dev)
    worst = 0.0
    n = got.shape[1]
    for lo, hi, tiles in _slices(n):
        g = _view(got, lo, hi, tiles).double()
        rr = r.unsqueeze(1) if tiles else r[:, :hi - lo]
        dd = d if tiles else d[:hi - lo]
        num = torch.nan_to_num((g - rr).abs().amax(0), nan=float("inf"))
        pos = dd > 0
        rel = torch.where(pos, num / torch.where(pos, dd, torch.ones_like(dd)),
                          torch.where(num > 0, torch.full_like(num, float("inf")),
                                      torch.zeros_like(num)))
        worst = max(worst, rel.max().item())
    return worst


def _rel_worst(got, ref):
    return _worst(got, ref, np.abs(ref).max(axis=0))


def _count_equal(got, ref, mask=None):
    """Number of points where got equals ref exactly (bitwise for floats),
    over the points whose base column is in mask (all if None); and the
    number of points checked."""
    dev = got.device
    r = torch.from_numpy(np.ascontiguousarray(ref)).to(dev)
    m = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask)).to(dev)
    eq = total = 0
    n = got.shape[-1]
    for lo, hi, tiles in _slices(n):
        g = _view(got, lo, hi, tiles)
        if got.dim() == 1:
            rr = r if tiles else r[:hi - lo]
            same = g == rr
        else:
            rr = r.unsqueeze(1) if tiles else r[:, :hi - lo]
            if g.dtype.is_floating_point:
                same = (g.view(torch.int64 if g.dtype == torch.float64 else torch.int32) ==
                        rr.view(torch.int64 if rr.dtype == torch.float64 else torch.int32)).all(0)
            else:
                same = (g == rr).all(0)
        if m is not None:
            mm = m if tiles else m[:hi - lo]
            same = same[..., mm]
        eq += int(same.sum().item())
        total += same.numel()
    return eq, total


def test_forward_beyond_32bit_indices():
    from paper_2006_04391_amd import api
    n = N_STATE
    dev = _dev(n * (4 * 48 + 1 + 4) + 4 * GB)
    ps = inputs.points_c0()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tol=ps.tol,
                          max_iter=ps.max_iter)
    eps = _tile(ps.eps, n, dev)
    a_old = _tile(ps.a_old, n, dev)
    phase = _tile(ps.phase, n, dev)
    sig, a_new, iters, count = api.evaluate(eps, a_old, phase, ps.phases, h=ps.h, tol=ps.tol,
                                            max_iter=ps.max_iter, return_iters=True)
    torch.cuda.synchronize()
    del eps
    assert int(count.item()) == 0
    assert _rel_worst(sig, ref["sigma"]) <= TOL
    assert _rel_worst(a_new, ref["a_out"]) <= TOL
    kinds = np.array([p["kind"] for p in ps.phases])
    el = kinds[ps.phase] == 0
    assert el.any() and (~el).any()
    eq, tot = _count_equal(a_new, ps.a_old, el)
    assert eq == tot > 0
    eq, tot = _count_equal(iters, ref["iters"])
    assert tot == n and eq / tot > 0.99


def test_tangent_beyond_32bit_indices():
    from paper_2006_04391_amd import api
    n = N_TANGENT
    dev = _dev(n * (4 * 48 + 288 + 1) + 4 * GB)
    ps = inputs.points_c0()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tol=ps.tol,
                          max_iter=ps.max_iter, tangent=True)
    sig, a_new, C = api.evaluate(_tile(ps.eps, n, dev), _tile(ps.a_old, n, dev),
                                 _tile(ps.phase, n, dev), ps.phases, h=ps.h, tol=ps.tol,
                                 max_iter=ps.max_iter, tangent=True)
    torch.cuda.synchronize()
    assert _rel_worst(sig, ref["sigma"]) <= TOL
    assert _rel_worst(a_new, ref["a_out"]) <= TOL
    assert _rel_worst(C, ref["tangent"]) <= TOL


def test_f32_beyond_32bit_indices():
    from paper_2006_04391_amd import api
    n = N_STATE
    dev = _dev(n * (4 * 24 + 1 + 4) + 4 * GB)
    ps = inputs.points_c0()
    eps32 = np.asarray(ps.eps, np.float32)
    a32 = np.asarray(ps.a_old, np.float32)
    ref = oracle.evaluate(eps32.astype(np.float64), a32.astype(np.float64), ps.phase, ps.phases,
                          h=ps.h, tol=1e-13, max_iter=100)
    sig, a_new, iters, count = api.evaluate_f32(_tile(eps32, n, dev), _tile(a32, n, dev),
                                                _tile(ps.phase, n, dev), ps.phases, h=ps.h,
                                                tol=1e-6, max_iter=ps.max_iter,
                                                return_iters=True)
    torch.cuda.synchronize()
    assert int(count.item()) == 0
    assert _rel_worst(sig, ref["sigma"]) <= TOL32
    scale = np.maximum(np.abs(ref["a_out"]).max(0), np.abs(eps32.astype(np.float64)).max(0))
    assert _worst(a_new, ref["a_out"], scale) <= TOL32


@pytest.mark.parametrize("tangent", [False, True])
def test_conventional_beyond_32bit_indices(tangent):
    from paper_2006_04391_amd import api
    n = N_TANGENT if tangent else N_STATE
    dev = _dev(n * (4 * 48 + 1 + 4 + (288 if tangent else 0)) + 4 * GB)
    ps = inputs.points_c0()
    ref = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, h=ps.h, tol=ps.tol,
                          max_iter=ps.max_iter, tangent=tangent)
    out = api.evaluate_conventional(_tile(ps.eps, n, dev), _tile(ps.a_old, n, dev),
                                    _tile(ps.phase, n, dev), ps.phases, h=ps.h, tol=ps.tol,
                                    max_iter=ps.max_iter, tangent=tangent)
    torch.cuda.synchronize()
    assert int(out[-1].item()) == 0
    assert _rel_worst(out[0], ref["sigma"]) <= TOL
    assert _rel_worst(out[1], ref["a_out"]) <= TOL
    if tangent:
        assert _rel_worst(out[2], ref["tangent"]) <= TOL


def _ramp_base(seed):
    """4096 points whose matrix flows enough for several adaptive steps
    (the loads of the adaptive schemes' parity tests)."""
    ps = inputs.points_random(B, seed=seed, phases=inputs.config_phases(), e11=2e-2, std=3e-4,
                              a_std=1e-4)
    e0 = 0.5 * ps.eps + 1e-4 * np.random.default_rng(seed).normal(size=ps.eps.shape)
    return ps, e0, 10.0


@pytest.mark.parametrize("pair", ["rk23", "rk12"])
@pytest.mark.parametrize("tangent", [False, True])
def test_adaptive_beyond_32bit_indices(pair, tangent):
    from paper_2006_04391_amd import api
    n = N_TANGENT if tangent else N_STATE
    dev = _dev(n * (5 * 48 + 1 + 4 + (288 if tangent else 0)) + 4 * GB)
    ps, e0, h = _ramp_base(seed=91 if pair == "rk23" else 92)
    ref = getattr(oracle, "evaluate_" + pair)(e0, ps.eps, ps.a_old, ps.phase, ps.phases, h=h,
                                              tangent=tangent)
    assert ref["steps"].max() > 1 and ref["steps"].min() >= 1
    out = getattr(api, "evaluate_" + pair)(_tile(e0, n, dev), _tile(ps.eps, n, dev),
                                           _tile(ps.a_old, n, dev), _tile(ps.phase, n, dev),
                                           ps.phases, h=h, tangent=tangent)
    torch.cuda.synchronize()
    steps, count = out[-2], out[-1]
    assert int(count.item()) == 0
    eq, tot = _count_equal(steps, ref["steps"])
    assert eq == tot == n
    assert _rel_worst(out[0], ref["sigma"]) <= TOL
    assert _rel_worst(out[1], ref["a_out"]) <= TOL
    if tangent:
        assert _rel_worst(out[2], ref["tangent"]) <= TOL


def test_backward_beyond_32bit_indices():
    from paper_2006_04391_amd import api
    n = N_STATE
    dev = _dev(n * (7 * 48 + 1) + 4 * GB)
    ps = inputs.points_random(B, seed=93, phases=inputs.paper_phases(), e11=1e-2, std=3e-3,
                              a_std=1e-3)
    ev = oracle.evaluate(ps.eps, ps.a_old, ps.phase, ps.phases, tol=1e-14, max_iter=100)
    rng = np.random.default_rng(93)
    gs = rng.normal(size=(6, B))
    ga = rng.normal(size=(6, B)) * 1e3
    ref = oracle.backward(ps.eps, ps.a_old, ev["a_out"], ps.phase, ps.phases, ps.h, gs, ga)
    full, tail = divmod(n, B)
    head = oracle.backward(ps.eps[:, :tail], ps.a_old[:, :tail], ev["a_out"][:, :tail],
                           ps.phase[:tail], ps.phases, ps.h, gs[:, :tail], ga[:, :tail])
    # sum over points of |per-point parameter gradient|, the scale of the
    # summation's rounding
    mags = np.zeros_like(ref["grad_params"])
    for j in range(B):
        one = oracle.backward(ps.eps[:, j:j + 1], ps.a_old[:, j:j + 1], ev["a_out"][:, j:j + 1],
                              ps.phase[j:j + 1], ps.phases, ps.h, gs[:, j:j + 1], ga[:, j:j + 1])
        mags += np.abs(one["grad_params"]) * (full + (1 if j < tail else 0))
    ge, gan, gp = api.evaluate_backward(_tile(ps.eps, n, dev), _tile(ps.a_old, n, dev),
                                        _tile(ev["a_out"], n, dev), _tile(ps.phase, n, dev),
                                        ps.phases, ps.h, _tile(gs, n, dev), _tile(ga, n, dev))
    torch.cuda.synchronize()
    assert _rel_worst(ge, ref["grad_eps"]) <= TOL
    assert _rel_worst(gan, ref["grad_a_old"]) <= TOL
    want = full * ref["grad_params"] + head["grad_params"]
    err = np.abs(gp.cpu().numpy() - want)
    assert np.all(err <= TOL * mags + 1e-300), (err, mags)
    assert np.any(mags > 0)
