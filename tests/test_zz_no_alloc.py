"""The basic-scheme load step without allocation (automat_ms_step_noalloc)
against the step with the handle's own work space (automat_ms_step),
through the C ABI: the same kernels run on the same inputs, so the fields,
mean stresses, iteration counts and residuals agree exactly. Calls in a
row, each on a smaller grid than the one before, and the rejections."""
import numpy as np
import pytest

from paper_2006_04391_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def _run(shape, phase, ph, loads, h, noalloc, **opts):
    from paper_2006_04391_amd import api
    n = shape[0] * shape[1] * shape[2]
    ms = api.MS(shape, ph, **opts)
    eps = torch.zeros((6, n), dtype=torch.float64, device="cuda")
    a = torch.zeros_like(eps)
    sig = torch.empty_like(eps)
    ph_t = torch.from_numpy(phase).cuda()
    out = []
    for E in loads:
        step = ms.step_noalloc if noalloc else ms.step
        mean, it, res = step(ph_t, E, h, eps, a, sigma_out=sig)
        torch.cuda.synchronize()
        out.append(dict(eps=eps.cpu().numpy(), a=a.cpu().numpy(), sigma=sig.cpu().numpy(),
                        mean=np.array(mean), iters=it, residual=res,
                        failures=ms.newton_failures()))
    ms.close()
    return out


@pytest.mark.parametrize("warm", [False, True])
def test_noalloc_step_equals_the_handle_step(warm):
    _need_gpu()
    ph = inputs.paper_phases()
    h = 1.0
    loads = [[2e-3 * k, -5e-4 * k, 0, 0, 3e-4 * k, 0] for k in (1, 2)]
    # a 4 x 128 x 128 grid (the plane transform kernels, z by hipFFT), then
    # a smaller 24 x 20 x 28 one and a still smaller 12 x 10 x 16 one (3-D
    # hipFFT plans)
    for shape, seed in (((4, 128, 128), 2), ((24, 20, 28), 3), ((12, 10, 16), 4)):
        rng = np.random.default_rng(seed)
        phase = (rng.random(shape[0] * shape[1] * shape[2]) < 0.2).astype(np.uint8)
        opts = dict(tol=1e-8, max_iter=2000, warm_start=warm)
        ref = _run(shape, phase, ph, loads, h, False, **opts)
        got = _run(shape, phase, ph, loads, h, True, **opts)
        for r, g in zip(ref, got):
            assert g["iters"] == r["iters"] and g["failures"] == r["failures"] == 0
            for key in ("eps", "a", "sigma", "mean"):
                assert np.array_equal(g[key], r[key]), (shape, key)
            assert g["residual"] == r["residual"]
        assert np.abs(got[-1]["a"]).max() > 0


def test_noalloc_step_rejects_what_does_not_fit():
    from paper_2006_04391_amd import api, _lib
    _need_gpu()
    ph = inputs.config_phases()
    # 96^3: 42 MB polarization + 43 MB spectrum > 64 MiB
    ms = api.MS((96, 96, 96), ph)
    z = torch.zeros((6, 96 ** 3), dtype=torch.float64, device="cuda")
    p = torch.zeros(96 ** 3, dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.AutomatError) as e:
        ms.step_noalloc(p, [1e-4, 0, 0, 0, 0, 0], 0.1, z, z.clone())
    assert e.value.code == _lib.EINVAL
    ms.close()
    ms = api.MS((8, 8, 8), ph, ref_update=True)
    z = torch.zeros((6, 512), dtype=torch.float64, device="cuda")
    p = torch.zeros(512, dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.AutomatError):
        ms.step_noalloc(p, [1e-4, 0, 0, 0, 0, 0], 0.1, z, z.clone())
    ms.close()
