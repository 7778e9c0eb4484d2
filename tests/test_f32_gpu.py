"""Single-precision evaluation on the GPU vs the FP64 oracle on the same
(float-rounded) inputs.

Bar: per point, ||x_f32 - x_oracle||_inf <= TOL32 * ||x_oracle||_inf for
the stress, TOL32_TAN for the tangent, and for the internal variables
(strains) TOL32 times the point's strain scale max(||a_oracle||_inf,
||eps||_inf): an increment below the FP32 resolution of the strain is not
resolved (a_{n+1} = a_n there), so a bar relative to |a| alone would ask for
digits FP32 does not hold where a_n = 0. The kernel stops
Newton at the FP32 rounding level of the trial elastic strain
(2^-19 ||eps - a_n||_inf); J = I + h Psi'' K has its spectrum in [1, inf)
(Psi'' K is similar to a symmetric positive semi-definite matrix), so the
increment error stays below that floor, and the stress error below the
floor times the stiffness, about 2e-6 of the trial stress; rounding in the
stress and the tangent's Cholesky solves adds a few units of 2^-24 times
the conditioning. The bars leave a factor ~5 over the largest errors
measured on these inputs."""
import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs
from tests.test_parity_gpu import N, rel_per_point

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL32 = 5e-5
TOL32_TAN = 5e-4


def _run(ps, tangent, h=None):
    from paper_2006_04391_amd import api
    eps = np.asarray(ps.eps, np.float32)
    a_old = np.asarray(ps.a_old, np.float32)
    hh = ps.h if h is None else h
    dev = torch.device("cuda:0")
    out = api.evaluate_f32(torch.from_numpy(eps).to(dev), torch.from_numpy(a_old).to(dev),
                           torch.from_numpy(ps.phase).to(dev), ps.phases, h=hh, tol=1e-6,
                           max_iter=ps.max_iter, tangent=tangent, return_iters=True)
    torch.cuda.synchronize()
    g = dict(sigma=N(out[0]).astype(np.float64), a_out=N(out[1]).astype(np.float64),
             iters=N(out[-2]), count=int(out[-1].item()))
    if tangent:
        g["tangent"] = N(out[2]).astype(np.float64)
    ref = oracle.evaluate(eps.astype(np.float64), a_old.astype(np.float64), ps.phase, ps.phases,
                          h=hh, tol=1e-13, max_iter=100, tangent=tangent)
    return g, ref, a_old


def _check(g, ref, ps, a_old, tangent):
    for key, tol in (("sigma", TOL32),) + ((("tangent", TOL32_TAN),) if tangent else ()):
        r = rel_per_point(g[key], ref[key])
        assert r.max() <= tol, (key, r.max(), int(r.argmax()))
    scale = np.maximum(np.abs(ref["a_out"]).max(0), np.abs(ps.eps).max(0))
    r = np.abs(g["a_out"] - ref["a_out"]).max(0) / scale
    assert r.max() <= TOL32, ("a_out", r.max(), int(r.argmax()))
    el = np.array([ps.phases[p]["kind"] == 0 for p in ps.phase])
    assert np.array_equal(g["a_out"][:, el].astype(np.float32), a_old[:, el])
    assert np.all(g["iters"][el] == 0)
    assert g["count"] == 0 and np.all(g["iters"] >= 0)


def _presets():
    out = [("c0", inputs.points_c0())]
    ps = inputs.points_random(256 * 5 + 37, seed=41, e11=2e-2, std=3e-3, a_std=1e-3)
    ps.phases = [dict(ps.phases[0], eps0=0.2), ps.phases[1]]
    out.append(("config", ps))
    out.append(("paper", inputs.points_random(256 * 3 + 1, seed=42, phases=inputs.paper_phases(),
                                              e11=1e-2, std=3e-3, a_std=1e-3)))
    ph = inputs.config_phases()
    ph[0] = dict(ph[0], H=900.0, sigma_y=4.0, eps0=0.5, n=3.3)
    out.append(("hardening", inputs.points_random(999, seed=43, phases=ph, e11=3e-2, std=5e-3,
                                                  a_std=2e-3)))
    ph = inputs.config_phases()
    ph[0] = dict(ph[0], n=1.0, eps0=0.1)
    out.append(("linear", inputs.points_random(300, seed=44, phases=ph, e11=3e-2, std=5e-3,
                                               a_std=2e-3)))
    return out


@pytest.mark.parametrize("name,ps", _presets(), ids=[p[0] for p in _presets()])
@pytest.mark.parametrize("tangent", [False, True])
def test_f32_matches_fp64_oracle(name, ps, tangent):
    g, ref, a_old = _run(ps, tangent)
    _check(g, ref, ps, a_old, tangent)


def test_f32_invalid_points_and_arguments():
    from paper_2006_04391_amd import api, _lib
    ps = inputs.points_c0(n=300)
    ps.eps[0, 5] = np.inf
    ps.phase[7] = 9
    eps = torch.from_numpy(np.asarray(ps.eps, np.float32)).cuda()
    a = torch.from_numpy(np.asarray(ps.a_old, np.float32)).cuda()
    ph = torch.from_numpy(ps.phase).cuda()
    s, an, it, cnt = api.evaluate_f32(eps, a, ph, ps.phases, return_iters=True)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 2 and N(it)[5] == -1 and N(it)[7] == -1
    assert np.all(np.isnan(N(s)[:, 5])) and np.all(np.isnan(N(an)[:, 7]))
    with pytest.raises(_lib.AutomatError):
        api.evaluate_f32(eps, a, ph, ps.phases, h=0.0)
    with pytest.raises(TypeError):
        api.evaluate_f32(eps.double(), a, ph, ps.phases)


def test_f32_full_size():
    """The 256^3 fibre batch rounded to float, every point against the FP64
    oracle on the same inputs."""
    ps = inputs.points_c1()
    g, ref, a_old = _run(ps, False)
    _check(g, ref, ps, a_old, False)
