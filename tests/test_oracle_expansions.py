"""Pins for oracle.expansions (App. A.3-A.4): the transformations against
direct sums and exact polynomial identities."""
import numpy as np

from oracle import expansions as ex
from oracle.harmonics import get, ntri, tri


def _cluster(n, centre, size, seed):
    rng = np.random.default_rng(seed)
    pos = np.asarray(centre) + size * (rng.random((n, 3)) - 0.5)
    q = rng.random(n) - 0.3
    return pos, q


def _direct(src, q, tgt):
    d = tgt[:, None, :] - src[None, :, :]
    r = np.linalg.norm(d, axis=2)
    return (q[None, :] / r).sum(axis=1), -(q[None, :, None] * d / r[:, :, None] ** 3).sum(axis=1)


def test_p2m_m2p_converges():
    """eq. P2M + eq. M2P reproduce the cluster's potential outside the
    multipole sphere; the error falls geometrically with p."""
    src, q = _cluster(40, [0, 0, 0], 0.5, 1)
    tgt, _ = _cluster(10, [2.0, 0.5, -0.3], 0.5, 2)
    ref, _ = _direct(src, q, tgt)
    errs = []
    for p in (2, 4, 8, 12):
        M = ex.p2m(p, np.zeros(3), src, q)
        errs.append(np.max(np.abs(ex.m2p(p, M, np.zeros(3), tgt) - ref)))
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-6 * np.max(np.abs(ref))


def test_m2l_l2p_against_direct():
    """eq. M2L + eq. L2P for two well separated clusters converge to the
    direct sum; the gradient from eq. L2L at order one + eq. phigrad too."""
    src, q = _cluster(30, [0, 0, 0], 0.4, 3)
    tgt, _ = _cluster(8, [1.5, -1.2, 2.0], 0.4, 4)
    rM, rL = np.zeros(3), np.array([1.5, -1.2, 2.0])
    ref_phi, ref_g = _direct(src, q, tgt)
    prev = None
    for p in (3, 6, 10):
        L = ex.m2l(p, ex.p2m(p, rM, src, q), rM, rL)
        phi = ex.l2p(p, L, rL, tgt)
        g = np.stack([ex.gradient_from_L1(ex.l2l(p, L, rL, t, pout=1)) for t in tgt])
        e = max(np.max(np.abs(phi - ref_phi)) / np.max(np.abs(ref_phi)),
                np.max(np.abs(g - ref_g)) / np.max(np.abs(ref_g)))
        if prev is not None:
            assert e < 0.3 * prev
        prev = e
    assert prev < 1e-6


def test_l2l_is_exact_reexpansion():
    """L2P after eq. L2L equals L2P of the original expansion exactly
    (a finite polynomial re-expansion)."""
    p = 7
    rng = np.random.default_rng(7)
    L = rng.standard_normal(ntri(p)) + 1j * rng.standard_normal(ntri(p))
    for l in range(p + 1):
        L[tri(l, 0)] = L[tri(l, 0)].real
    rL, rL2 = np.zeros(3), np.array([0.2, -0.1, 0.15])
    pts = rng.random((5, 3)) - 0.5
    L2 = ex.l2l(p, L, rL, rL2)
    np.testing.assert_allclose(ex.l2p(p, L2, rL2, pts), ex.l2p(p, L, rL, pts), rtol=1e-12, atol=1e-12)


def test_m2m_equals_p2m_at_new_centre():
    """eq. M2M of the moments equals eq. P2M about the new centre (exact)."""
    p = 6
    src, q = _cluster(20, [0.1, 0.0, -0.1], 0.3, 8)
    rM, rM2 = np.array([0.1, 0.0, -0.1]), np.array([0.3, -0.2, 0.1])
    M = ex.p2m(p, rM, src, q)
    np.testing.assert_allclose(ex.m2m(p, M, rM, rM2), ex.p2m(p, rM2, src, q), rtol=1e-12, atol=1e-13)


def test_gradient_one_charge_closed_form():
    """A single charge q at r_s: L_1^0 = -q d_z/|d|^3 and Re L_1^1 = q d_x/|d|^3,
    Im L_1^1 = -q d_y/|d|^3 with d = r_L - r_s, so eq. phigrad gives
    grad(q/|r - r_s|) at r_L."""
    p = 3
    rs, rL = np.array([0.3, -0.4, 0.2]), np.array([2.0, 1.0, -1.5])
    q = 0.7
    M = ex.p2m(p, rs, rs[None, :], np.array([q]))
    L = ex.m2l(p, M, rs, rL)
    d = rL - rs
    r3 = np.linalg.norm(d) ** 3
    assert abs(L[tri(1, 0)] - (-q * d[2] / r3)) < 1e-15
    assert abs(L[tri(1, 1)] - (q * d[0] / r3 - 1j * q * d[1] / r3)) < 1e-15
    np.testing.assert_allclose(ex.gradient_from_L1(L), -q * d / r3, rtol=1e-13)
    assert abs(L[tri(0, 0)] - q / np.linalg.norm(d)) < 1e-15


def test_gradient_matches_finite_differences():
    """eq. phigrad at a particle equals the finite-difference gradient of eq. L2P."""
    p = 6
    rng = np.random.default_rng(9)
    L = rng.standard_normal(ntri(p)) + 1j * rng.standard_normal(ntri(p))
    for l in range(p + 1):
        L[tri(l, 0)] = L[tri(l, 0)].real
    rL = np.zeros(3)
    x = np.array([0.21, -0.13, 0.3])
    g = ex.gradient_from_L1(ex.l2l(p, L, rL, x, pout=1))
    h = 1e-6
    fd = [(ex.l2p(p, L, rL, (x + h * e)[None])[0] - ex.l2p(p, L, rL, (x - h * e)[None])[0]) / (2 * h)
          for e in np.eye(3)]
    np.testing.assert_allclose(g, fd, rtol=1e-7, atol=1e-8)


def test_real_matrix_equals_complex_m2l():
    """eq. realmatrix (A, B, C, D of G^{m,mu}) reproduces eq. M2L exactly."""
    p = 5
    rng = np.random.default_rng(10)
    M = rng.standard_normal(ntri(p)) + 1j * rng.standard_normal(ntri(p))
    for l in range(p + 1):
        M[tri(l, 0)] = M[tri(l, 0)].real
    d = np.array([2.1, -1.3, 2.7])
    L = ex.m2l(p, M, np.zeros(3), d)
    from oracle.harmonics import solid_S
    S = solid_S(2 * p, *d)
    for l in range(p + 1):
        for m in range(l + 1):
            re = im = 0.0
            for lam in range(p + 1):
                G0 = get(S, l + lam, -m)
                re += G0.real * M[tri(lam, 0)].real
                im += G0.imag * M[tri(lam, 0)].real
                for mu in range(1, lam + 1):
                    A, B = get(S, l + lam, -(m + mu)).real, get(S, l + lam, -(m + mu)).imag
                    C = (-1) ** mu * get(S, l + lam, -(m - mu)).real
                    D = (-1) ** mu * get(S, l + lam, -(m - mu)).imag
                    Mr, Mi = M[tri(lam, mu)].real, M[tri(lam, mu)].imag
                    re += (A + C) * Mr - (B - D) * Mi
                    im += (B + D) * Mr + (A - C) * Mi
            assert abs(L[tri(l, m)].real - re) < 1e-12 * (1 + abs(re))
            assert abs(L[tri(l, m)].imag - im) < 1e-12 * (1 + abs(im))
