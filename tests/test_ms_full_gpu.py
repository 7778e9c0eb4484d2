"""The basic scheme at the workloads' full sizes against the oracle's
stored runs (``tests/golden/make_ms_golden.py``, which calls only the
oracle): fixed iteration counts on both sides (lockstep), so the fields
agree to rounding.

* 128^3 spheres, benchmark phases, two strain-controlled steps of 12
  iterations, cold Newton starts as in the benchmark;
* 150^3 synthetic metal-matrix composite, the paper's phases, two steps of
  the tension-compression cycle under uniaxial mixed conditions with the
  reference stiffness adjusted from the tangent field every step (2-D
  hipFFT plans in-plane, the length-150 z transforms with the Green
  operator in one kernel), 10 iterations each;
* the same on a 128^3 composite, 8 iterations each (the in-plane slab
  transforms and the fused z transform with the Green operator, whose
  zero frequency then carries the mixed conditions);
* 64^3 spheres, five converged steps: the reverse steps' derivatives of the
  last mean stress against the oracle's linearized scheme (forward
  derivatives, an independent route to the same numbers).

Sampled voxels: |x_gpu - x_oracle| <= 1e-10 max |x_oracle| per field and
component; per-component means and L2 norms of the whole fields at 1e-10.
"""
import json
import os

import numpy as np
import pytest

from paper_2006_04391_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
UNIAXIAL = 0b111110
GRAD_INDEX = {"E": 0, "nu": 1, "H": 2, "sigma_y": 3, "sigma0": 4, "eps0": 5, "n": 6}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def _check_fields(g, ref, k, idx):
    for key, x in g.items():
        xs = x[:, idx]
        o = ref[f"step{k}_{key}_samples"]
        scale = np.abs(o).max(axis=1, keepdims=True)
        scale = np.where(scale > 0, scale, 1.0)
        err = (np.abs(xs - o) / scale).max()
        assert err <= 1e-10, (k, key, err)
        for stat, val in (("mean", x.mean(axis=1)), ("norm", np.linalg.norm(x, axis=1))):
            o = ref[f"step{k}_{key}_{stat}"]
            tol = 1e-10 * max(np.abs(o).max(), 1e-300)
            if stat == "mean":
                tol = 1e-10 * np.abs(ref[f"step{k}_{key}_norm"]).max() / np.sqrt(x.shape[1])
            assert np.abs(val - o).max() <= tol, (k, key, stat, val, o)


def test_spheres128_lockstep_against_oracle():
    from paper_2006_04391_amd import api
    _need_gpu()
    ref = np.load(os.path.join(GOLDEN, "ms_spheres128_lockstep.npz"))
    N = 128
    n = N ** 3
    it = int(ref["iterations"])
    h = float(ref["h"])
    phase = torch.from_numpy(inputs.sphere_phase(N, seed=2)).cuda()
    ms = api.MS((N, N, N), inputs.config_phases(), tol=1e-30, max_iter=it, fixed_iter=True,
                warm_start=False)
    eps = torch.zeros((6, n), dtype=torch.float64, device="cuda")
    a = torch.zeros_like(eps)
    sig = torch.empty_like(eps)
    idx = ref["indices"]
    for k in (1, 2):
        mean, iters, res = ms.step(phase, ref[f"step{k}_E"], h, eps, a, sigma_out=sig)
        torch.cuda.synchronize()
        assert iters == it
        assert ms.newton_failures() == 0
        o = ref[f"step{k}_sigma_mean"]
        np.testing.assert_allclose(mean, o, rtol=1e-10, atol=1e-10 * np.abs(o).max())
        assert abs(res - float(ref[f"step{k}_residual"])) <= 1e-8 * float(ref[f"step{k}_residual"])
        _check_fields(dict(eps=eps.cpu().numpy(), sigma=sig.cpu().numpy(), a=a.cpu().numpy()),
                      ref, k, idx)
    ms.close()


@pytest.mark.parametrize("N,seed,name", [(150, 4, "ms_mmc150_mixed_lockstep.npz"),
                                          (128, 5, "ms_mmc128_mixed_lockstep.npz")])
def test_mmc_mixed_reference_update_lockstep_against_oracle(N, seed, name):
    from paper_2006_04391_amd import api
    _need_gpu()
    ref = np.load(os.path.join(GOLDEN, name))
    n = N ** 3
    it = int(ref["iterations"])
    h = float(ref["h"])
    phase = torch.from_numpy(inputs.mmc_phase(N, seed=seed)).cuda()
    ms = api.MS((N, N, N), inputs.paper_phases(), tol=1e-30, max_iter=it, fixed_iter=True,
                ref_update=True)
    eps = torch.zeros((6, n), dtype=torch.float64, device="cuda")
    a = torch.zeros_like(eps)
    sig = torch.empty_like(eps)
    idx = ref["indices"]
    for k in (1, 2):
        mean, Er, iters, res = ms.step_mixed(phase, ref[f"step{k}_E_target"], h, eps, a,
                                             UNIAXIAL, sigma_out=sig)
        torch.cuda.synchronize()
        assert iters == it
        assert ms.newton_failures() == 0
        np.testing.assert_allclose(ms.reference(), ref[f"step{k}_reference"], rtol=1e-12)
        o = ref[f"step{k}_E"]
        np.testing.assert_allclose(Er, o, rtol=1e-10, atol=1e-10 * abs(o[0]))
        o = ref[f"step{k}_sigma_mean"]
        np.testing.assert_allclose(mean, o, rtol=1e-10, atol=1e-10 * np.abs(o).max())
        assert abs(res - float(ref[f"step{k}_residual"])) <= 1e-8 * float(ref[f"step{k}_residual"])
        _check_fields(dict(eps=eps.cpu().numpy(), sigma=sig.cpu().numpy(), a=a.cpu().numpy()),
                      ref, k, idx)
    # the matrix flows, and the reference follows the tangent field
    assert np.abs(ref["step2_a_samples"]).max() > 0
    mu = [p["E"] / (2 * (1 + p["nu"])) for p in inputs.paper_phases()]
    assert ref["step1_reference"][1] < 0.95 * 0.5 * (min(mu) + max(mu))


def test_spheres64_derivatives_against_oracle_linearized_scheme():
    """The 64^3 differentiation workload: d<sigma_5>/dE_5 (6 x 6) and
    d<sigma_5>/d(E, nu, sigma0, n) of the matrix over the five-step history
    from the GPU's reverse steps, against the oracle's forward derivatives
    (linearized Lippmann-Schwinger solves on the oracle's tangent field).
    Both sides converge the scheme to 1e-12 or below; the derivatives agree
    to 1e-7 of their scale (the fixed-point residual enters them at about
    the contrast times 1e-12)."""
    from paper_2006_04391_amd import api
    _need_gpu()
    with open(os.path.join(GOLDEN, "ms_spheres64_derivatives.json")) as f:
        ref = json.load(f)
    N = 64
    phase = inputs.sphere_phase(N, seed=3)
    ph = inputs.config_phases()
    r = api.ms_gradients((N, N, N), phase, ph, ref["loads"], ref["h"], tol=1e-13, max_iter=5000)
    np.testing.assert_allclose(r["sigma_mean"], ref["sigma_mean"], rtol=1e-9,
                               atol=1e-9 * np.abs(ref["sigma_mean"]).max())
    C = np.array(ref["dsig_dE_last"])
    got = r["dsig_dE"][:, -1, :]
    assert np.abs(got - C).max() <= 1e-7 * np.abs(C).max(), (got, C)
    for key, col in ref["dsig_dp_matrix"].items():
        col = np.array(col)
        g = r["dsig_dp"][:, 0, GRAD_INDEX[key]]
        assert np.abs(g - col).max() <= 1e-7 * np.abs(col).max(), (key, g, col)
