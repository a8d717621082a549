"""Seeded synthetic particle sets for the PMMM far-field workloads.

This module holds random-number recipes only: positions, charges and the
per-system parameters of the batched workload.  It contains none of the
method's arithmetic, so both the HIP path and the FP64 oracle may consume
its output.

Every generator uses ``numpy.random.Generator(PCG64(seed))``.  Positions are
produced directly in the working precision (float32 for the FP32 paths,
float64 for the FP64 workload) inside the half-open unit cube, so a value of
exactly 1.0 can never appear.  The charge recipes follow the paper's
accuracy test (Sec. 4: uniform positions in a unit box, charges drawn in
[0, 1/N) and shifted to zero mean) and the workload descriptions below.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "ParticleSet",
    "uniform_positions",
    "neutral_pm1",
    "open_equal_mass",
    "periodic_pm1",
    "periodic_pm1_blocks",
    "plummer_sphere",
    "uniform_open_shape",
    "periodic_pm1_edge",
    "paper_accuracy_set",
    "batched_systems",
    "multi_charge_sets",
    "WORKLOADS",
    "make_workload",
]


@dataclasses.dataclass
class ParticleSet:
    """Positions ``x, y, z`` and charges ``q`` (same dtype), plus the mesh
    and method parameters the workload is defined with."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray
    n_cells: int
    p: int
    boundary: str  # "open" or "periodic"
    box: float = 1.0
    cutoff: int = 2
    shape: tuple | None = None   # open: (nx, ny, nz) cells, n_cells = nx, box = x edge

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def pos(self) -> np.ndarray:
        """(N, 3) float64 copy of the positions (exact widening)."""
        return np.stack([self.x, self.y, self.z], axis=1).astype(np.float64)

    def subset(self, idx: np.ndarray) -> "ParticleSet":
        return dataclasses.replace(
            self, x=self.x[idx], y=self.y[idx], z=self.z[idx], q=self.q[idx]
        )


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_positions(rng: np.random.Generator, n: int, dtype=np.float32):
    """Three arrays of ``n`` positions uniform in [0, 1)."""
    dt = np.dtype(dtype)
    return tuple(rng.random(n, dtype=dt) for _ in range(3))


def neutral_pm1(rng: np.random.Generator, n: int, dtype=np.float32) -> np.ndarray:
    """Charges +1 for a random half of the particles and -1 for the rest
    (``n`` must be even), so the total is exactly zero."""
    if n % 2:
        raise ValueError("neutral +/-1 charges need an even particle count")
    q = np.ones(n, dtype=dtype)
    q[rng.permutation(n)[: n // 2]] = -1
    return q


def open_equal_mass(n=4096, n_cells=8, p=4, seed=1, dtype=np.float64) -> ParticleSet:
    """Open boundary, uniform in the unit cube, equal masses 1/N."""
    rng = _rng(seed)
    x, y, z = uniform_positions(rng, n, dtype)
    q = np.full(n, 1.0 / n, dtype=dtype)
    return ParticleSet(x, y, z, q, n_cells, p, "open")


def periodic_pm1(n=32768, n_cells=16, p=5, seed=2, dtype=np.float32) -> ParticleSet:
    """Periodic boundary, uniform in the unit cube, exactly neutral +/-1."""
    rng = _rng(seed)
    x, y, z = uniform_positions(rng, n, dtype)
    q = neutral_pm1(rng, n, dtype)
    return ParticleSet(x, y, z, q, n_cells, p, "periodic")


def periodic_pm1_blocks(n_blocks=32, block=32768, n_cells=32, p=7, seed=3,
                        dtype=np.float32) -> ParticleSet:
    """Periodic, ``n_blocks`` consecutive blocks of ``block`` uniform
    particles, each block exactly neutral +/-1.  Block 0 on its own is the
    32768-particle slice used for the Ewald check."""
    rng = _rng(seed)
    xs, ys, zs, qs = [], [], [], []
    for _ in range(n_blocks):
        x, y, z = uniform_positions(rng, block, dtype)
        xs.append(x)
        ys.append(y)
        zs.append(z)
        qs.append(neutral_pm1(rng, block, dtype))
    return ParticleSet(np.concatenate(xs), np.concatenate(ys), np.concatenate(zs),
                       np.concatenate(qs), n_cells, p, "periodic")


def plummer_sphere(n=1 << 22, n_cells=64, p=6, seed=4, scale=0.05,
                   dtype=np.float32) -> ParticleSet:
    """Plummer sphere of scale radius ``scale`` centred in the unit cube.

    Radii come from the textbook inverse of the Plummer cumulative mass
    ``m(r) = r^3 / (r^2 + a^2)^{3/2}``, directions are isotropic, and draws
    that land outside [0, 1)^3 are rejected and redrawn.  Equal masses 1/N.
    """
    rng = _rng(seed)
    out = np.empty((0, 3), dtype=np.float64)
    while out.shape[0] < n:
        m = n - out.shape[0]
        batch = int(m * 1.05) + 1024
        u = rng.random(batch)
        u = np.clip(u, 1e-300, 1.0)
        r = scale / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        cz = 2.0 * rng.random(batch) - 1.0
        ph = 2.0 * np.pi * rng.random(batch)
        sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
        pts = 0.5 + r[:, None] * np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)
        pts = pts.astype(dtype).astype(np.float64)
        ok = np.all((pts >= 0.0) & (pts < 1.0), axis=1)
        out = np.concatenate([out, pts[ok]], axis=0)
    out = out[:n].astype(dtype)
    q = np.full(n, 1.0 / n, dtype=dtype)
    return ParticleSet(out[:, 0].copy(), out[:, 1].copy(), out[:, 2].copy(), q,
                       n_cells, p, "open")


def uniform_open_shape(n=1 << 21, dims=(48, 40, 32), p=6, edge=1.0 / 64, seed=8,
                       dtype=np.float32) -> ParticleSet:
    """Open box of dims cubic cells of edge ``edge`` (not a cube, not powers
    of two), ``n`` uniform particles with neutral +/-1 charges.  Positions
    are drawn in float64 and rounded to ``dtype``; a rounding that reaches
    the box edge is moved one step inside."""
    rng = _rng(seed)
    ext = np.asarray(dims, dtype=np.float64) * edge
    pos = (rng.random((n, 3)) * ext).astype(dtype)
    top = ext.astype(dtype)
    pos = np.where(pos >= top, np.nextafter(top, dtype(0)), pos)
    q = neutral_pm1(rng, n, dtype)
    return ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), q, int(dims[0]), p,
                       "open", box=float(dims[0] * edge), shape=tuple(int(d) for d in dims))


def periodic_pm1_edge(n=1 << 20, n_cells=24, p=6, edge=1.0 / 32, seed=9,
                      dtype=np.float32) -> ParticleSet:
    """Periodic box of n_cells^3 cells of edge ``edge`` (an edge count that
    is not a power of two), ``n`` uniform particles, neutral +/-1 charges.
    Positions are drawn in float64 and rounded to ``dtype``; a rounding that
    reaches the box edge is moved one step inside."""
    rng = _rng(seed)
    box = n_cells * edge
    pos = (rng.random((n, 3)) * box).astype(dtype)
    top = dtype(box)
    pos = np.where(pos >= top, np.nextafter(top, dtype(0)), pos)
    q = neutral_pm1(rng, n, dtype)
    return ParticleSet(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), q, n_cells, p,
                       "periodic", box=float(box))


def paper_accuracy_set(n=16384, n_cells=8, p=4, boundary="open", cutoff=2,
                       seed=7, dtype=np.float64) -> ParticleSet:
    """The paper's accuracy-test recipe (Sec. 4): N uniform particles in a
    unit box on an 8^3 mesh, charges uniform in [0, 1/N) then shifted by
    their mean so that the system is neutral."""
    rng = _rng(seed)
    x, y, z = uniform_positions(rng, n, dtype)
    q = rng.random(n) / n
    q = (q - q.mean()).astype(dtype)
    return ParticleSet(x, y, z, q, n_cells, p, boundary, cutoff=cutoff)


def batched_systems(n_sys=256, seed=5, dtype=np.float32):
    """Independent periodic systems with uneven sizes: N uniform in
    [2048, 65536] (rounded to even), mesh edge drawn from {8, 16, 32} and
    order from {4, 5, 6}, each exactly neutral +/-1."""
    rng = _rng(seed)
    systems = []
    ns = rng.integers(2048, 65537, size=n_sys)
    meshes = rng.choice(np.array([8, 16, 32]), size=n_sys)
    orders = rng.choice(np.array([4, 5, 6]), size=n_sys)
    for s in range(n_sys):
        n = int(ns[s]) & ~1
        x, y, z = uniform_positions(rng, n, dtype)
        q = neutral_pm1(rng, n, dtype)
        systems.append(ParticleSet(x, y, z, q, int(meshes[s]), int(orders[s]), "periodic"))
    return systems


def multi_charge_sets(n=1 << 20, n_sets=64, n_cells=32, p=6, seed=6, dtype=np.float32):
    """One set of uniform positions with ``n_sets`` independent exactly
    neutral +/-1 charge assignments.  Returns (ParticleSet of set 0,
    charges of shape (n_sets, n))."""
    rng = _rng(seed)
    x, y, z = uniform_positions(rng, n, dtype)
    qs = np.stack([neutral_pm1(rng, n, dtype) for _ in range(n_sets)])
    return ParticleSet(x, y, z, qs[0].copy(), n_cells, p, "periodic"), qs


#: Named workloads: name -> (factory, description)
WORKLOADS = {
    "open_n4096_m8_p4_f64": (open_equal_mass,
                             "open, N=4096 uniform, equal masses 1/N, 8^3 cells (16^3 padded FFT), p=4, FP64"),
    "periodic_n32768_m16_p5": (periodic_pm1,
                               "periodic, N=32768 uniform, neutral +/-1, 16^3 cells, p=5, FP32"),
    "periodic_n1048576_m32_p7": (periodic_pm1_blocks,
                                 "periodic, N=2^20 uniform, neutral +/-1, 32^3 cells, p=7, FP32"),
    "open_plummer_n4194304_m64_p6": (plummer_sphere,
                                     "open, N=2^22 Plummer a=0.05, 64^3 cells (128^3 padded FFT), p=6, FP32"),
    "periodic_n1048576_m24_p6": (periodic_pm1_edge,
                                 "periodic, N=2^20 uniform, neutral +/-1, 24^3 cells of edge 1/32 "
                                 "(direct DFTs), p=6, FP32"),
    "open_n2097152_m48x40x32_p6": (uniform_open_shape,
                                   "open, N=2^21 uniform, neutral +/-1, 48x40x32 cells of edge 1/64 "
                                   "(computed in the 64^3 cube, 128^3 padded FFT), p=6, FP32"),
}


def make_workload(name: str) -> ParticleSet:
    return WORKLOADS[name][0]()
