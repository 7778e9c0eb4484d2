"""Seeded synthetic inputs for the material-point evaluation.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle. It holds no arithmetic of the material law: only random draws,
microstructure geometry (phase fields) and material parameter presets.

Conventions used by every producer and consumer of these arrays:

* strains are 6-vectors in engineering-shear Voigt order
  (11, 22, 33, 23, 13, 12), stresses in plain Voigt order, units MPa and s;
* fields are structure-of-arrays, component-major: element (c, i) is at
  ``c * n + i`` (numpy shape ``(6, n)``);
* a voxel grid of side N is flattened x-fastest: ``i = x + N * (y + N * z)``;
* phase ids are ``uint8``; phase 0 is the matrix, phase 1 the inclusion.

The paper's workload is a short-fibre metal-matrix composite (Section
"Example", paragraph "Microstructure"); its voxel image is not available, so
the fibre and sphere generators below stand in for it with the same kind of
structure.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PHASE_KEYS = ("kind", "E", "nu", "H", "sigma_y", "sigma0", "eps0", "n")

# Elastic phase: the force potential vanishes, so only E and nu matter. The
# viscous entries are placeholders that pass validation.
_ELASTIC_FILL = dict(H=0.0, sigma_y=0.0, sigma0=1.0, eps0=0.0, n=1.0)


def config_phases() -> list[dict]:
    """Matrix + inclusion of the benchmark workloads (MPa, 1/s).

    Matrix: isotropic elastic E = 2.5 GPa, nu = 0.35 with a Perzyna power-law
    viscoplastic potential (drag stress 50 MPa, reference rate 1e-3/s,
    exponent 5), no hardening and no yield threshold. Inclusion: elastic,
    E = 72 GPa, nu = 0.22.
    """
    return [
        dict(kind=1, E=2500.0, nu=0.35, H=0.0, sigma_y=0.0, sigma0=50.0, eps0=1e-3, n=5.0),
        dict(kind=0, E=72000.0, nu=0.22, **_ELASTIC_FILL),
    ]


def paper_phases() -> list[dict]:
    """Aluminium matrix and Al2O3 fibre of Table ``misu_parameters`` (MPa, 1/s).

    E = 55 GPa, nu = 0.33, sigma_Y = 25 MPa, H = 1.8 GPa, reference rate 1/s,
    drag stress 130 MPa, n = 3.6 for the matrix; E = 300 GPa, nu = 0.25 for
    the fibre. Strongly nonlinear at percent strains, so it exercises the
    many-iteration Newton paths.
    """
    return [
        dict(kind=1, E=55000.0, nu=0.33, H=1800.0, sigma_y=25.0, sigma0=130.0, eps0=1.0, n=3.6),
        dict(kind=0, E=300000.0, nu=0.25, **_ELASTIC_FILL),
    ]


def jitter_phases(phases: list[dict], rng: np.random.Generator, rel: float = 0.1) -> list[dict]:
    """Multiply every continuous parameter of every phase by U(1-rel, 1+rel).

    Zero-valued parameters stay zero; Poisson's ratio stays below 0.5 and the
    exponent stays >= 1 because the presets are far enough from those limits.
    """
    out = []
    for p in phases:
        q = dict(p)
        for k in PHASE_KEYS[1:]:
            q[k] = float(p[k] * rng.uniform(1.0 - rel, 1.0 + rel))
        if q["kind"] == 0:
            q.update(_ELASTIC_FILL)
        out.append(q)
    return out


def phases_array(phases: list[dict]) -> np.ndarray:
    """Rows (kind, E, nu, H, sigma_y, sigma0, eps0, n) as float64, one per phase."""
    return np.array([[float(p[k]) for k in PHASE_KEYS] for p in phases], dtype=np.float64)


# ----------------------------------------------------------------------------
# material-point sets
# ----------------------------------------------------------------------------

@dataclass
class PointSet:
    eps: np.ndarray      # (6, n) float64, strain at t_{n+1}
    a_old: np.ndarray    # (6, n) float64, internal variables at t_n
    phase: np.ndarray    # (n,) uint8
    phases: list         # phase parameter dicts
    h: float = 0.1
    tol: float = 1e-12
    max_iter: int = 50

    @property
    def n(self) -> int:
        return int(self.phase.shape[0])


def uniaxial_strain(n: int, e11: float, std: float, rng: np.random.Generator) -> np.ndarray:
    """(e11, 0, 0, 0, 0, 0) plus iid N(0, std^2) on every Voigt component."""
    eps = rng.normal(0.0, std, size=(6, n))
    eps[0] += e11
    return eps


def deviatoric_draw(n: int, std: float, rng: np.random.Generator) -> np.ndarray:
    """Six iid N(0, std^2) components, then the mean of the three normal
    components is subtracted from each of them (trace-free)."""
    a = rng.normal(0.0, std, size=(6, n))
    a[:3] -= a[:3].mean(axis=0, keepdims=True)
    return a


def points_c0(seed: int = 0, n: int = 4096) -> PointSet:
    """4096 independent points: 70 % matrix / 30 % inclusion.

    Exactly round(0.3 n) inclusion points at positions from a seeded
    permutation; strain (2e-3, 0...) + N(0, 1e-4^2); a_old = 0; h = 0.1 s.
    """
    rng = np.random.default_rng(seed)
    phase = np.zeros(n, dtype=np.uint8)
    perm = rng.permutation(n)
    phase[perm[: int(round(0.3 * n))]] = 1
    eps = uniaxial_strain(n, 2e-3, 1e-4, rng)
    a_old = np.zeros((6, n))
    return PointSet(eps, a_old, phase, config_phases())


def points_random(n: int, seed: int, phases: list[dict] | None = None, e11: float = 5e-3,
                  std: float = 2e-4, a_std: float = 1e-4, incl_frac: float = 0.3) -> PointSet:
    """Random material points with random phases and a deviatoric prior a_n
    in the matrix (zero in inclusions). Used for parity sweeps at any size."""
    rng = np.random.default_rng(seed)
    phase = (rng.random(n) < incl_frac).astype(np.uint8)
    eps = uniaxial_strain(n, e11, std, rng)
    a_old = deviatoric_draw(n, a_std, rng)
    a_old[:, phase != 0] = 0.0
    return PointSet(eps, a_old, phase, phases if phases is not None else config_phases())


# ----------------------------------------------------------------------------
# periodic microstructures
# ----------------------------------------------------------------------------

def _unit_vectors(rng: np.random.Generator) -> np.ndarray:
    """One direction uniform on the unit sphere."""
    z = rng.uniform(-1.0, 1.0)
    phi = rng.uniform(0.0, 2.0 * math.pi)
    r = math.sqrt(max(0.0, 1.0 - z * z))
    return np.array([r * math.cos(phi), r * math.sin(phi), z])


def fibre_phase(N: int, seed: int, radius: float = 4.0, length: float = 64.0,
                vol_frac: float = 0.15) -> np.ndarray:
    """Periodic N^3 phase field of straight capped fibres (phase 1) in a matrix.

    Fibres have centres uniform in the cell and directions uniform on the
    sphere; overlap is allowed. A voxel (centre at integer coordinates) is
    fibre if its minimum-image distance to the fibre's axis segment is at most
    ``radius``. Fibres are added until the fibre fraction reaches
    ``vol_frac``. Returns a flat uint8 array, x-fastest.
    """
    rng = np.random.default_rng(seed)
    grid = np.zeros((N, N, N), dtype=np.uint8)        # indexed [z, y, x]
    target = vol_frac * N ** 3
    count = 0
    half = 0.5 * length
    r2 = radius * radius
    while count < target:
        c = rng.uniform(0.0, N, size=3)               # (x, y, z)
        d = _unit_vectors(rng)
        lo = [int(math.floor(c[k] - (abs(d[k]) * half + radius))) - 1 for k in range(3)]
        hi = [int(math.ceil(c[k] + (abs(d[k]) * half + radius))) + 1 for k in range(3)]
        xs = np.arange(lo[0], hi[0] + 1, dtype=np.float64)
        ys = np.arange(lo[1], hi[1] + 1, dtype=np.float64)
        zs = np.arange(lo[2], hi[2] + 1, dtype=np.float64)
        dx = xs - c[0]
        dy = ys - c[1]
        dz = zs - c[2]
        # projection onto the axis, clamped to the segment
        t = (dz[:, None, None] * d[2] + dy[None, :, None] * d[1] + dx[None, None, :] * d[0])
        t = np.clip(t, -half, half)
        rx = dx[None, None, :] - t * d[0]
        ry = dy[None, :, None] - t * d[1]
        rz = dz[:, None, None] - t * d[2]
        inside = (rx * rx + ry * ry + rz * rz) <= r2
        zi, yi, xi = np.nonzero(inside)
        if zi.size == 0:
            continue
        zz = (zs[zi].astype(np.int64)) % N
        yy = (ys[yi].astype(np.int64)) % N
        xx = (xs[xi].astype(np.int64)) % N
        before = grid[zz, yy, xx]
        count += int(np.count_nonzero(before == 0))
        grid[zz, yy, xx] = 1
        # a voxel hit twice in one fibre (only if length + radius >= N) is
        # counted twice above; recount exactly in that rare case
        if 2 * (half + radius) >= N:
            count = int(np.count_nonzero(grid))
    return grid.reshape(-1)


def tension_compression_path(steps: int = 80, rate: float = 1.4e-3, e_max: float = 3.58454e-3,
                             e_min: float = -3.48441e-3):
    """Macroscopic axial strain of a uniaxial tension-compression cycle at
    constant absolute strain rate: 0 -> e_max -> e_min, cut into `steps`
    equal time steps (the test of the paper's Section "Example", paragraph
    "Boundary Conditions"; its default of 80 load steps). Returns (h, list of
    the axial strains at the ends of the steps)."""
    t1 = e_max / rate
    T = t1 + (e_max - e_min) / rate
    h = T / steps

    def e(t):
        return rate * t if t <= t1 else e_max - rate * (t - t1)
    return h, [e(k * h) for k in range(1, steps + 1)]


def mmc_phase(N: int = 150, seed: int = 0, vol_frac: float = 0.102, aspect: float = 15.0,
              radius: float = 2.5) -> np.ndarray:
    """Synthetic metal-matrix-composite microstructure standing in for the
    paper's GeoDict volume element: straight fibres of length/diameter
    `aspect`, isotropic directions, `vol_frac` fibre content."""
    return fibre_phase(N, seed, radius=radius, length=2.0 * radius * aspect, vol_frac=vol_frac)


def sphere_phase(N: int, seed: int, radius: float = 6.0, vol_frac: float = 0.20) -> np.ndarray:
    """Periodic N^3 phase field of non-overlapping spheres (phase 1).

    Random sequential addition: centres uniform in the cell, a candidate is
    rejected if its minimum-image centre distance to any accepted sphere is
    below 2 * radius. Spheres are added until the voxel fraction of sphere
    reaches ``vol_frac`` (a voxel is inside if its centre is within
    ``radius`` of a sphere centre, minimum image). Returns a flat uint8
    array, x-fastest.
    """
    rng = np.random.default_rng(seed)
    grid = np.zeros((N, N, N), dtype=np.uint8)
    target = vol_frac * N ** 3
    centres = np.zeros((0, 3))
    count = 0
    r2 = radius * radius
    tries = 0
    while count < target:
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("sphere packing did not reach the volume fraction")
        c = rng.uniform(0.0, N, size=3)
        if centres.shape[0]:
            dd = centres - c
            dd -= N * np.round(dd / N)
            if np.min(np.einsum("ij,ij->i", dd, dd)) < (2.0 * radius) ** 2:
                continue
        centres = np.vstack([centres, c])
        lo = [int(math.floor(c[k] - radius)) - 1 for k in range(3)]
        hi = [int(math.ceil(c[k] + radius)) + 1 for k in range(3)]
        xs = np.arange(lo[0], hi[0] + 1, dtype=np.float64)
        ys = np.arange(lo[1], hi[1] + 1, dtype=np.float64)
        zs = np.arange(lo[2], hi[2] + 1, dtype=np.float64)
        inside = ((zs[:, None, None] - c[2]) ** 2 + (ys[None, :, None] - c[1]) ** 2
                  + (xs[None, None, :] - c[0]) ** 2) <= r2
        zi, yi, xi = np.nonzero(inside)
        zz = zs[zi].astype(np.int64) % N
        yy = ys[yi].astype(np.int64) % N
        xx = xs[xi].astype(np.int64) % N
        count += int(np.count_nonzero(grid[zz, yy, xx] == 0))
        grid[zz, yy, xx] = 1
    return grid.reshape(-1)


def points_c1(seed: int = 1, N: int = 256) -> PointSet:
    """The 256^3 headline batch: fibre microstructure (r = 4, L = 64, 15 %),
    strain (5e-3, 0...) + N(0, 2e-4^2), deviatoric prior a_n with std 1e-4 in
    the matrix and zero in the fibres; h = 0.1 s."""
    rng = np.random.default_rng(seed)
    phase = fibre_phase(N, seed=seed)
    n = N ** 3
    eps = uniaxial_strain(n, 5e-3, 2e-4, rng)
    a_old = deviatoric_draw(n, 1e-4, rng)
    a_old[:, phase != 0] = 0.0
    return PointSet(eps, a_old, phase, config_phases())


# ----------------------------------------------------------------------------
# counter-based strain generator of the serving path (Philox4x32-10)
# ----------------------------------------------------------------------------

_M32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw 2011), vectorized
    over counters; returns four uint32 arrays."""
    c = [np.asarray(x, dtype=np.uint64) & _M32 for x in (c0, c1, c2, c3)]
    k0, k1 = np.uint64(k0) & _M32, np.uint64(k1) & _M32
    M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
    W0, W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & _M32
            k1 = (k1 + W1) & _M32
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & _M32, (p0 >> np.uint64(32)) ^ c[3] ^ k1,
             p0 & _M32]
    return [x.astype(np.uint32) for x in c]


def _u01(u):
    return (u.astype(np.float64) + 0.5) * 2.0 ** -32


def _box_muller(a, b):
    r = np.sqrt(-2.0 * np.log(_u01(a)))
    t = 2.0 * np.pi * _u01(b)
    return r * np.cos(t), r * np.sin(t)


def served_strain(n, step, steps, E_final, noise_std, seed):
    """Strain of load step `step` (1-based) of `steps` at points 0..n-1:
    (step / steps) E_final + noise_std z, z from Philox4x32-10 keyed by the
    seed with counter (i_lo, i_hi, step, w) and Box-Muller pairs."""
    i = np.arange(n, dtype=np.uint64)
    lo, hi = i & _M32, i >> np.uint64(32)
    k0, k1 = int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF
    r0 = philox4x32_10(lo, hi, np.uint64(step), np.uint64(0), k0, k1)
    r1 = philox4x32_10(lo, hi, np.uint64(step), np.uint64(1), k0, k1)
    z = np.empty((6, n))
    z[0], z[1] = _box_muller(r0[0], r0[1])
    z[2], z[3] = _box_muller(r0[2], r0[3])
    z[4], z[5] = _box_muller(r1[0], r1[1])
    E = np.asarray(E_final, dtype=np.float64) * (step / steps)
    return E[:, None] + noise_std * z


@dataclass
class ServeRequest:
    side: int
    structure: str          # "fibre" or "sphere"
    structure_seed: int
    phases: list
    steps: int
    seed: int
    arrival: float          # seconds after the start of the run
    E_final: tuple = (5e-3, 0.0, 0.0, 0.0, 0.0, 0.0)
    noise_std: float = 2e-4
    h: float = 0.1

    @property
    def n(self):
        return self.side ** 3


def serving_requests(count=1000, rate=200.0, seed=4, min_side=32, max_side=256):
    """The request stream of the serving workload: exponential inter-arrival
    times (rate per second), cube side log-uniform in [min_side, max_side],
    fibre (as the 256^3 batch) or sphere (20 %, r = 6) structure by a fair
    coin, every parameter of both phases jittered by U(0.9, 1.1), 1..10 load
    steps, a strain seed per request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        side = int(round(math.exp(rng.uniform(math.log(min_side), math.log(max_side)))))
        kind = "fibre" if rng.random() < 0.5 else "sphere"
        out.append(ServeRequest(side=side, structure=kind, structure_seed=int(rng.integers(1 << 31)),
                                phases=jitter_phases(config_phases(), rng),
                                steps=int(rng.integers(1, 11)), seed=int(rng.integers(1 << 62)),
                                arrival=t))
    return out


def request_phase_field(req: ServeRequest) -> np.ndarray:
    if req.structure == "fibre":
        return fibre_phase(req.side, seed=req.structure_seed)
    return sphere_phase(req.side, seed=req.structure_seed)
