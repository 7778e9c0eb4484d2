"""Seeded input generators shared by the oracle side and the GPU side (CPU)."""
import json
import os

import numpy as np

from paper_2006_04391_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def test_philox_known_answers():
    for case in json.load(open(GOLDEN))["cases"]:
        c = [np.array([int(x, 16)], dtype=np.uint64) for x in case["counter"]]
        k = [int(x, 16) for x in case["key"]]
        out = inputs.philox4x32_10(*c, *k)
        assert [int(o[0]) for o in out] == [int(x, 16) for x in case["out"]]


def test_served_strain_statistics_and_mean_path():
    n = 100000
    E = np.array([5e-3, 0, 0, 0, 0, 0])
    z = (inputs.served_strain(n, 3, 4, E, 2e-4, 99) - 0.75 * E[:, None]) / 2e-4
    assert np.all(np.abs(z.mean(axis=1)) < 5 / np.sqrt(n))
    assert np.all(np.abs(z.std(axis=1) - 1) < 5 / np.sqrt(2 * n))
    cc = np.corrcoef(z)
    assert np.abs(cc - np.eye(6)).max() < 5 / np.sqrt(n)
    # points, steps and seeds draw distinct streams; a prefix is stable
    a = inputs.served_strain(50, 1, 2, E, 1.0, 7)
    assert np.array_equal(a, inputs.served_strain(80, 1, 2, E, 1.0, 7)[:, :50])
    assert not np.allclose(a, inputs.served_strain(50, 2, 2, E, 1.0, 7) - 0.5 * E[:, None])
    assert not np.allclose(a, inputs.served_strain(50, 1, 2, E, 1.0, 8))


def test_request_stream_shape():
    reqs = inputs.serving_requests(count=400, seed=4)
    t = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert abs(np.diff(t).mean() - 5e-3) < 1e-3
    sides = np.array([r.side for r in reqs])
    assert sides.min() >= 32 and sides.max() <= 256
    assert 1 <= min(r.steps for r in reqs) and max(r.steps for r in reqs) <= 10
    assert {r.structure for r in reqs} == {"fibre", "sphere"}
    base = inputs.config_phases()
    for r in reqs[:20]:
        for p, b in zip(r.phases, base):
            assert 0.9 * b["E"] <= p["E"] <= 1.1 * b["E"]
