"""Host-side accounting of bench.py (CPU): the per-stage algorithmic bytes
sum to the closed form of the unfused FP32 pipeline, and the pair counts
behind the near-field and hierarchical roofline figures equal brute-force
enumeration."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

STAGES = ("bin", "p2m", "fft_fwd", "column", "fft_inv", "l2p")


@pytest.mark.parametrize("N,n,p,nf", [(4096, 8, 4, 16), (32768, 16, 5, 16), (1 << 20, 32, 7, 32),
                                      (1 << 22, 64, 6, 128)])
def test_stage_bytes_sum_to_closed_form(N, n, p, nf):
    """One far-field call moves 80N + 8K + 16PK + (32P + 4Q)F bytes in FP32
    with every stage reading its inputs and writing its outputs once
    (K = n^3 cells, F = nf^2 (nf/2 + 1) half-spectrum frequencies,
    P = (p+1)^2 moments, Q = (2p+1)^2 kernel components)."""
    K, P, Q = n ** 3, (p + 1) ** 2, (2 * p + 1) ** 2
    F = nf * nf * (nf // 2 + 1)
    total = sum(bench.algorithmic_work(s, N, n, p, nf)[0] for s in STAGES)
    assert total == 80 * N + 8 * K + 16 * P * K + (32 * P + 4 * Q) * F


def test_stage_bytes_of_the_plummer_workload():
    """2^22 particles, 64^3 cells in the 128^3 transform, p = 6: 2.93 GB."""
    total = sum(bench.algorithmic_work(s, 1 << 22, 64, 6, 128)[0] for s in STAGES)
    assert abs(total / 2.93e9 - 1) < 0.005


def _near_pairs_brute(x, y, z, nc, c):
    I = np.clip((np.stack([x, y, z], 1) * nc).astype(np.int64), 0, nc - 1)
    d = np.abs(I[:, None, :] - I[None, :, :]).max(-1)
    return int((d <= c).sum()) - len(x)


@pytest.mark.parametrize("nc,c,n", [(4, 1, 700), (5, 2, 600), (8, 1, 900), (3, 1, 1)])
def test_near_pairs_brute_force(nc, c, n):
    rng = np.random.default_rng(nc * 10 + c)
    x, y, z = rng.random((3, n))
    if n > 1:
        x[: n // 3] = 0.31 + 0.01 * rng.random(n // 3)     # a crowded slab of cells
    assert bench._near_pairs(x, y, z, nc, c) == _near_pairs_brute(x, y, z, nc, c)


@pytest.mark.parametrize("n,r,c", [(4, 2, 1), (2, 4, 1), (4, 2, 2), (8, 1, 1), (3, 2, 1)])
def test_fine_pairs_brute_force(n, r, c):
    """Ordered (target, source) fine-cell pairs whose coarse cells are within
    c and fine cells are not (Chebyshev distances)."""
    nf = n * r
    g = np.stack(np.meshgrid(*(np.arange(nf),) * 3, indexing="ij"), -1).reshape(-1, 3)
    fine = np.abs(g[:, None, :] - g[None, :, :]).max(-1)
    coarse = np.abs(g[:, None, :] // r - g[None, :, :] // r).max(-1)
    brute = int(np.sum((coarse <= c) & (fine > c)))
    assert bench._fine_pairs(n, r, c) == brute
    if r == 1:
        assert brute == 0
