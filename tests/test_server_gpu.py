"""Continuous-batching service on the GPU: each request's final fields equal
the oracle's run of the same load steps on the reproduced strains, and a
request's results do not depend on what it was batched with (to 1e-12 per
point)."""
import time

import numpy as np
import pytest

import oracle
from paper_2006_04391_amd import inputs
from tests.test_parity_gpu import TOL, rel_per_point

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _server(**kw):
    from paper_2006_04391_amd import api
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return api.Server(kw.pop("budget", 8 << 30), **kw)


def _drain(srv, ids, timeout=60.0):
    got = {}
    t0 = time.time()
    while len(got) < len(ids):
        for r in srv.poll():
            got[r["id"]] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.002)
    return [got[i] for i in ids]


def _request(side, structure, seed, steps, phases=None, noise=2e-4, E=(5e-3, 0, 0, 0, 0, 0)):
    rng = np.random.default_rng(seed)
    # inclusions scaled to the small test cells
    phase = (inputs.fibre_phase(side, seed=seed, radius=max(1.0, side / 12), length=side / 2)
             if structure == "fibre" else
             inputs.sphere_phase(side, seed=seed, radius=max(1.5, side / 6)))
    ph = phases if phases is not None else inputs.jitter_phases(inputs.config_phases(), rng)
    return dict(phase=phase, phases=ph, steps=steps, E_final=E, noise_std=noise,
                seed=int(rng.integers(1 << 62)))


def _oracle_final(q, h=0.1, max_iter=50):
    """The oracle's run of the request's load steps: final sigma and a, the
    failed point solves, and the per-point strain scale max(||a||, ||eps||)
    of the last step (see _check)."""
    n = q["phase"].size
    a = np.zeros((6, n)) if q.get("a_init") is None else np.array(q["a_init"], dtype=np.float64)
    fails = 0
    for j in range(1, q["steps"] + 1):
        eps = inputs.served_strain(n, j, q["steps"], q["E_final"], q["noise_std"], q["seed"])
        r = oracle.evaluate(eps, a, q["phase"], q["phases"], h=h, tol=1e-12, max_iter=max_iter)
        a = r["a_out"]
        fails += int((r["iters"] < 0).sum())
    return r["sigma"], a, fails, np.maximum(np.abs(a).max(0), np.abs(eps).max(0))


def _check(res, sig_ref, a_ref, scale):
    """sigma within TOL per point; a (a strain) within TOL of the point's
    strain scale max(||a||, ||eps||): both Newton solves stop at
    ||F|| <= max(tol ||Delta||, 2^-48 ||eps - a_n||), so where the increment
    of a point that starts from a_n = 0 is tiny (a flow just above the yield
    stress) each side determines a only to about 2^-48 ||eps||, which is
    far below TOL ||eps|| but can exceed TOL ||a||."""
    assert rel_per_point(res["sigma"], sig_ref).max() <= TOL
    r = np.abs(res["a"] - a_ref).max(0) / scale
    assert r.max() <= TOL, (r.max(), int(r.argmax()))


def test_single_request_matches_oracle():
    q = _request(12, "sphere", 3, 4)
    srv = _server()
    rid = srv.submit(**q, want_fields=True)
    (res,) = _drain(srv, [rid])
    srv.close()
    assert res["status"] == 0 and res["steps_done"] == 4 and res["n"] == 12 ** 3
    sig, a, fails, scale = _oracle_final(q)
    assert res["nonconverged"] == fails == 0
    _check(res, sig, a, scale)
    assert np.abs(a).max() > 0
    assert res["t_arrival"] <= res["t_admit"] <= res["t_done"]


def test_batched_mix_matches_oracle_and_running_alone():
    reqs = [_request(s, k, 10 + j, steps) for j, (s, k, steps) in
            enumerate([(9, "fibre", 3), (17, "sphere", 1), (13, "fibre", 5), (10, "sphere", 2),
                       (21, "fibre", 4), (8, "sphere", 3)])]
    srv = _server()
    ids = [srv.submit(**q, want_fields=True) for q in reqs]
    mixed = _drain(srv, ids)
    st = srv.stats()
    srv.close()
    assert st["updates"] == sum(q["phase"].size * q["steps"] for q in reqs)
    assert st["used_bytes"] == 0 and st["active"] == 0 and st["pending"] == 0
    # several requests shared launches
    assert st["launches"] < sum(q["steps"] for q in reqs)
    seq = _server(sequential=True)
    ids = [seq.submit(**q, want_fields=True) for q in reqs]
    alone = _drain(seq, ids)
    st = seq.stats()
    seq.close()
    assert st["launches"] == sum(q["steps"] for q in reqs)
    for q, m, s in zip(reqs, mixed, alone):
        assert m["status"] == s["status"] == 0
        # the same points meet different batch-mates in the two runs; the
        # wave-wide choice of a first-order trial evaluation may change the
        # last bits, never more
        assert rel_per_point(m["sigma"], s["sigma"]).max() <= 1e-12
        assert rel_per_point(m["a"], s["a"]).max() <= 1e-12
        sig, a, fails, scale = _oracle_final(q)
        assert m["nonconverged"] == fails
        _check(m, sig, a, scale)


def test_point_cap_splits_batches():
    reqs = [_request(s, "sphere", 30 + s, 2) for s in (8, 12, 16)]
    srv = _server(max_batch_points=16 ** 3)
    ids = [srv.submit(**q, want_fields=True) for q in reqs]
    out = _drain(srv, ids)
    st = srv.stats()
    srv.close()
    assert st["launches"] >= 4
    for q, r in zip(reqs, out):
        sig, a, _, scale = _oracle_final(q)
        _check(r, sig, a, scale)


def test_budget_admission_and_rejection():
    from paper_2006_04391_amd import _lib
    q = _request(16, "fibre", 5, 3)
    fp = 16 ** 3 * 97 + 8192
    srv = _server(budget=fp)                   # room for about one request at a time
    ids = [srv.submit(**q, want_fields=True) for _ in range(3)]
    out = _drain(srv, ids)
    for r in out[1:]:
        assert rel_per_point(r["sigma"], out[0]["sigma"]).max() <= 1e-12
        assert r["t_admit"] >= out[0]["t_done"] - 1e-3
    big = _request(24, "sphere", 6, 1)
    with pytest.raises(_lib.AutomatError) as e:
        srv.submit(**big)
    assert e.value.code == _lib.EBUDGET
    srv.close()


def test_first_step_state_in_a_reused_block():
    """A request without an initial state starts from a_n = 0: its first load
    step takes a_n = 0 without reading the field and writes the zeros of its
    points without flow itself, so what an earlier request left in the same
    arena block does not leak in (here the block of a request whose matrix
    flowed, reused by one whose inclusions sit where that matrix was). A
    request with an initial state starts from it."""
    side = 16
    n = side ** 3
    first = _request(side, "sphere", 71, 3)
    second = _request(side, "fibre", 72, 1)
    a0 = inputs.deviatoric_draw(n, 1e-3, np.random.default_rng(73))
    third = dict(_request(side, "sphere", 74, 2), a_init=a0)
    srv = _server(budget=n * 97 + 8192)    # one request at a time, each in the block before
    ids = [srv.submit(**q, want_fields=True) for q in (first, second, third)]
    out = _drain(srv, ids)
    srv.close()
    finals = []
    for q, r in zip((first, second, third), out):
        assert r["status"] == 0
        sig, a, fails, scale = _oracle_final(q)
        assert r["nonconverged"] == fails == 0
        _check(r, sig, a, scale)
        finals.append(a)
    kinds = np.array([p["kind"] for p in second["phases"]])
    leftover = (np.abs(finals[0]).max(axis=0) > 0) & (kinds[second["phase"]] == 0)
    assert leftover.sum() > 0
    assert np.all(out[1]["a"][:, leftover] == 0.0)
    assert not np.array_equal(finals[2], _oracle_final(dict(third, a_init=None))[1])


def test_nonconverged_points_are_counted():
    ph = inputs.paper_phases()
    q = _request(10, "sphere", 7, 2, phases=ph, E=(2e-2, 0, 0, 0, 0, 0))
    srv = _server()
    rid = srv.submit(**q, want_fields=True, max_iter=2)
    (res,) = _drain(srv, [rid])
    srv.close()
    _, _, fails, _ = _oracle_final(q, max_iter=2)
    assert fails > 0 and res["nonconverged"] == fails


def test_invalid_requests():
    from paper_2006_04391_amd import _lib
    q = _request(6, "sphere", 8, 1)
    srv = _server()
    for bad in (dict(steps=0), dict(noise_std=-1.0), dict(h=0.0)):
        with pytest.raises(_lib.AutomatError):
            srv.submit(**(q | bad))
    bad_phase = q["phases"] + [dict(q["phases"][0], nu=0.6)]
    with pytest.raises(_lib.AutomatError):
        srv.submit(**(q | dict(phases=bad_phase)))
    rid = srv.submit(**q)
    (res,) = _drain(srv, [rid])
    assert res["status"] == 0 and "sigma" not in res
    srv.close()


def test_mix_larger_than_the_resident_grid():
    """Many more tiles in one batch than the batch kernel's resident grid
    holds blocks (four 84^3 requests: 9270 tiles of 256 points against at
    most a few blocks per compute unit), so blocks stride over many tiles
    and move from one request to the next inside a launch (drain the wave
    queues, reload the descriptor and phase table): every request against
    the oracle and against the same request served alone."""
    reqs = [_request(s, k, 60 + j, steps) for j, (s, k, steps) in
            enumerate([(84, "fibre", 3), (84, "sphere", 2), (84, "fibre", 1), (84, "sphere", 4),
                       (11, "fibre", 2)])]
    tiles = sum((q["phase"].size + 255) // 256 for q in reqs)
    assert tiles > 8 * 4 * torch.cuda.get_device_properties(0).multi_processor_count
    srv = _server()
    ids = [srv.submit(**q, want_fields=True) for q in reqs]
    mixed = _drain(srv, ids, timeout=120.0)
    st = srv.stats()
    srv.close()
    assert st["launches"] < sum(q["steps"] for q in reqs)
    seq = _server(sequential=True)
    ids = [seq.submit(**q, want_fields=True) for q in reqs]
    alone = _drain(seq, ids, timeout=120.0)
    seq.close()
    for q, m, s in zip(reqs, mixed, alone):
        assert m["status"] == s["status"] == 0
        assert rel_per_point(m["sigma"], s["sigma"]).max() <= 1e-12
        assert rel_per_point(m["a"], s["a"]).max() <= 1e-12
        sig, a, fails, scale = _oracle_final(q)
        assert m["nonconverged"] == fails == 0
        _check(m, sig, a, scale)
        assert np.abs(a).max() > 0
