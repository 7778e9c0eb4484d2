"""Write the oracle's expected values for the full-size basic-scheme checks.

The basic scheme's fixed point couples every voxel, so at the workloads'
full sizes the oracle cannot compute a sample of voxels alone, and a full
run takes minutes on the CPU. This script runs the oracle (``oracle/`` only,
on the seeded inputs of ``paper_2006_04391_amd.inputs``) once and stores
what the GPU tests compare with:

* ``ms_spheres128_lockstep.npz``: the 128^3 sphere microstructure (20 %,
  r = 6, seed 2), benchmark phases, strain path 1e-3 t e11 with h = 0.1 s,
  two load steps of exactly 12 fixed-point iterations each; per step the
  mean stress, the last relative strain change, the per-component mean and
  L2 norm of the strain, stress and internal-variable fields and those
  fields at 512 seeded voxel indices;
* ``ms_mmc150_mixed_lockstep.npz``: the 150^3 synthetic metal-matrix
  composite (seed 4), the paper's phase parameters, the first two steps of
  the tension-compression cycle cut into 8 steps (the first step already
  passes the matrix's yield stress), uniaxial mixed conditions, reference
  stiffness adjusted from the tangent field every step, 10 fixed-point
  iterations per step; the same quantities plus the macroscopic strain
  reached and the reference Lame constants;
* ``ms_mmc128_mixed_lockstep.npz``: the same test on a 128^3 synthetic
  metal-matrix composite (seed 5), 8 fixed-point iterations per step (the
  grid size on which the basic scheme's transforms run in-plane and along z
  in kernels of their own);
* ``ms_spheres64_derivatives.json``: the 64^3 sphere microstructure (seed
  3), five load steps of the same strain path converged to 1e-12; the
  derivative of the last mean stress with respect to the last macroscopic
  strain (6 x 6) and to the matrix's E, nu, sigma0 and n over the whole
  history, from the oracle's linearized scheme (forward derivatives).

Run from the repository root: ``python tests/golden/make_ms_golden.py``
(about 25 minutes on 8 cores; ``--only NAME`` runs one of lockstep128,
mixed150, mixed128, derivatives64).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import ms as oms  # noqa: E402
from paper_2006_04391_amd import inputs  # noqa: E402

N_SAMPLES = 512
UNIAXIAL = 0b111110


def sample_indices(n, seed):
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(n, N_SAMPLES - 2, replace=False))
    return np.unique(np.concatenate([[0], idx, [n - 1]]))


def _log(msg):
    print(msg, flush=True)


def _field_stats(out, prefix, r, idx):
    for key in ("eps", "sigma", "a"):
        x = r[key]
        out[f"{prefix}{key}_mean"] = x.mean(axis=1)
        out[f"{prefix}{key}_norm"] = np.linalg.norm(x, axis=1)
        out[f"{prefix}{key}_samples"] = x[:, idx]


def lockstep128():
    N, h, iters = 128, 0.1, 12
    shape = (N, N, N)
    phase = inputs.sphere_phase(N, seed=2)
    ph = inputs.config_phases()
    n = N ** 3
    idx = sample_indices(n, 128)
    out = dict(indices=idx, iterations=np.array(iters), h=np.array(h))
    eps, a, prev = np.zeros((6, n)), np.zeros((6, n)), np.zeros(6)
    for k in (1, 2):
        t0 = time.perf_counter()
        E = np.array([1e-3 * h * k, 0, 0, 0, 0, 0])
        r = oms.ms_step(eps, a, phase, ph, shape, E, prev, h, tol=0.0, max_iter=iters,
                        fixed_iter=True)
        out[f"step{k}_E"] = E
        out[f"step{k}_sigma_mean"] = r["sigma_mean"]
        out[f"step{k}_residual"] = np.array(r["residual"])
        _field_stats(out, f"step{k}_", r, idx)
        eps, a, prev = r["eps"], r["a"], E
        _log(f"lockstep128 step {k}: {time.perf_counter() - t0:.1f} s, "
             f"residual {r['residual']:.3e}, mean sigma {r['sigma_mean']}")
    np.savez(os.path.join(HERE, "ms_spheres128_lockstep.npz"), **out)


def mixed150(N=150, iters=10, seed=4, name="ms_mmc150_mixed_lockstep.npz"):
    shape = (N, N, N)
    phase = inputs.mmc_phase(N, seed=seed)
    ph = inputs.paper_phases()
    h, path = inputs.tension_compression_path(8)
    n = N ** 3
    idx = sample_indices(n, 150)
    out = dict(indices=idx, iterations=np.array(iters), h=np.array(h))
    eps, a, prev = np.zeros((6, n)), np.zeros((6, n)), np.zeros(6)
    lam0, mu0 = oms.reference_medium(ph)
    for k in (1, 2):
        t0 = time.perf_counter()
        E = np.array([path[k - 1], 0, 0, 0, 0, 0])
        r = oms.ms_step(eps, a, phase, ph, shape, E, prev, h, lam0=lam0, mu0=mu0, tol=0.0,
                        max_iter=iters, fixed_iter=True, stress_mask=UNIAXIAL, ref_update=True)
        out[f"step{k}_E_target"] = E
        out[f"step{k}_E"] = r["E"]
        out[f"step{k}_sigma_mean"] = r["sigma_mean"]
        out[f"step{k}_residual"] = np.array(r["residual"])
        out[f"step{k}_reference"] = np.array([r["lam0"], r["mu0"]])
        _field_stats(out, f"step{k}_", r, idx)
        eps, a, prev, lam0, mu0 = r["eps"], r["a"], r["E"], r["lam0"], r["mu0"]
        _log(f"mixed{N} step {k}: {time.perf_counter() - t0:.1f} s, residual "
             f"{r['residual']:.3e}, E {r['E']}, reference {r['lam0']:.1f} {r['mu0']:.1f}")
    np.savez(os.path.join(HERE, name), **out)


def mixed128():
    mixed150(N=128, iters=8, seed=5, name="ms_mmc128_mixed_lockstep.npz")


def derivatives64():
    N, h, tol = 64, 0.1, 1e-12
    shape = (N, N, N)
    phase = inputs.sphere_phase(N, seed=3)
    ph = inputs.config_phases()
    n = N ** 3
    loads = [np.array([1e-3 * h * k, 0, 0, 0, 0, 0]) for k in range(1, 6)]
    lam0, mu0 = oms.reference_medium(ph)
    eps, a, prev = np.zeros((6, n)), np.zeros((6, n)), np.zeros(6)
    hist, iters = [], []
    for E in loads:
        t0 = time.perf_counter()
        r = oms.ms_step(eps, a, phase, ph, shape, E, prev, h, lam0=lam0, mu0=mu0, tol=tol,
                        max_iter=5000, newton_tol=1e-14)
        hist.append((r["eps"], a, r["a"]))
        iters.append(int(r["iters"]))
        eps, a, prev = r["eps"], r["a"], E
        _log(f"derivatives64 forward step: {r['iters']} iterations, {time.perf_counter() - t0:.1f} s")
    sigma_mean = r["sigma_mean"]
    K = len(loads)
    dE = np.zeros((6, 6))
    for c in range(6):
        t0 = time.perf_counter()
        d = np.zeros((K, 6))
        d[-1, c] = 1.0
        dE[:, c] = oms.linearized_history(hist[-1:], phase, ph, shape, h, d[-1:], lam0=lam0,
                                          mu0=mu0)
        _log(f"derivatives64 d sigma / d E5[{c}]: {time.perf_counter() - t0:.1f} s")
    dp = {}
    for key in ("E", "nu", "sigma0", "n"):
        t0 = time.perf_counter()
        d = np.zeros((len(ph), 7))
        d[0, oracle.GRAD_KEYS.index(key)] = 1.0
        dp[key] = oms.linearized_history(hist, phase, ph, shape, h, np.zeros((K, 6)),
                                         d_params=d, lam0=lam0, mu0=mu0).tolist()
        _log(f"derivatives64 d sigma / d {key}: {time.perf_counter() - t0:.1f} s")
    out = {
        "what": "64^3 spheres (20 %, r = 6, seed 3), benchmark phases, strain path "
                "1e-3 t e11, five steps of h = 0.1 s from zero state, basic scheme converged "
                "to 1e-12 (Newton 1e-14); forward derivatives of the last mean stress from "
                "the oracle's linearized scheme",
        "loads": [E.tolist() for E in loads],
        "h": h,
        "forward_iterations": iters,
        "sigma_mean": sigma_mean.tolist(),
        "dsig_dE_last": dE.tolist(),
        "dsig_dp_matrix": dp,
    }
    with open(os.path.join(HERE, "ms_spheres64_derivatives.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=["lockstep128", "mixed150", "mixed128", "derivatives64"])
    args = ap.parse_args()
    jobs = dict(lockstep128=lockstep128, mixed150=mixed150, mixed128=mixed128,
                derivatives64=derivatives64)
    for name, fn in jobs.items():
        if args.only in (None, name):
            fn()


if __name__ == "__main__":
    main()
