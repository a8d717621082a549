"""Pins for oracle.exact: closed forms, Newton's third law, alpha
independence of the Ewald sum and the rock-salt Madelung constant."""
import os

import numpy as np

from oracle import exact, pmmm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_direct_two_bodies_closed_form():
    pos = np.array([[0.1, 0.2, 0.3], [0.4, 0.6, 0.9]])
    q = np.array([0.7, -1.3])
    phi, g = exact.direct(pos, q)
    d = pos[0] - pos[1]
    r = np.linalg.norm(d)
    assert abs(phi[0] - q[1] / r) < 1e-15
    assert abs(phi[1] - q[0] / r) < 1e-15
    np.testing.assert_allclose(g[0], -q[1] * d / r ** 3, rtol=1e-14)
    np.testing.assert_allclose(g[1], q[0] * d / r ** 3, rtol=1e-14)


def test_direct_newton_third_law():
    rng = np.random.default_rng(1)
    pos = rng.random((300, 3))
    q = rng.random(300) - 0.5
    _, g = exact.direct(pos, q)
    f = q[:, None] * g
    assert np.max(np.abs(f.sum(axis=0))) < 1e-12 * np.max(np.abs(f))


def test_ewald_alpha_independent_and_momentum_conserving():
    rng = np.random.default_rng(2)
    pos = rng.random((400, 3))
    q = rng.random(400) - 0.5
    q -= q.mean()
    p1, g1 = exact.ewald(pos, q)                     # alpha = 14, minimum image
    p2, g2 = exact.ewald(pos, q, alpha=6.0, images=1, rcut=0.999)
    assert exact.rel_rms(p2, p1) < 1e-12
    assert exact.rel_rms(g2, g1) < 1e-12
    f = q[:, None] * g1
    assert np.max(np.abs(f.sum(axis=0))) < 1e-11 * np.max(np.abs(f))


def test_ewald_charged_system_alpha_independent():
    """With Q_tot != 0 the -pi/(V alpha^2) Q_tot term keeps Phi independent
    of alpha (the reading of eq. refewald taken here)."""
    rng = np.random.default_rng(3)
    pos = rng.random((100, 3))
    q = rng.random(100)
    p1, _ = exact.ewald(pos, q)
    p2, _ = exact.ewald(pos, q, alpha=7.0, images=1, rcut=0.999)
    assert exact.rel_rms(p2, p1) < 1e-12


def test_ewald_madelung():
    with open(os.path.join(GOLDEN, "madelung.txt")) as f:
        Mad = float([l for l in f if not l.startswith("#")][0])
    n = 6
    i = np.arange(n)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    I = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    pos = (I + 0.5) / n
    q = (-1.0) ** I.sum(axis=1)
    phi, g = exact.ewald(pos, q)
    np.testing.assert_allclose(phi, -Mad * q * n, rtol=1e-12)
    assert np.max(np.abs(g)) < 1e-10


def test_near_field_counts_only_near_cells():
    """The near field plus the direct sum over the remaining cells is the
    full direct sum (open boundary)."""
    rng = np.random.default_rng(4)
    pos = rng.random((500, 3))
    q = rng.random(500) - 0.5
    cfg = pmmm.Config(n=6, p=1, boundary="open", cutoff=1)
    nphi, _ = exact.near(pos, q, cfg)
    I, _, _, _ = pmmm.cells(pos, cfg)
    full, _ = exact.direct(pos, q)
    for i in range(0, 500, 50):
        far = np.max(np.abs(I - I[i]), axis=1) > 1
        r = np.linalg.norm(pos[far] - pos[i], axis=1)
        assert abs(nphi[i] + np.sum(q[far] / r) - full[i]) < 1e-12 * np.sum(np.abs(q) / 0.01)


def test_direct_at_is_rows_of_direct():
    """direct_at(pos, q, idx) returns rows idx of the all-pairs sum."""
    rng = np.random.default_rng(23)
    pos = rng.random((700, 3))
    q = rng.random(700) - 0.5
    phi, g = exact.direct(pos, q)
    idx = np.array([0, 5, 699, 123, 5])
    p2, g2 = exact.direct_at(pos, q, idx)
    assert np.allclose(p2, phi[idx], rtol=1e-14, atol=0)
    assert np.allclose(g2, g[idx], rtol=1e-13, atol=1e-13 * np.abs(g).max())
