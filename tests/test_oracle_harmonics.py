"""Pins for oracle.harmonics: the paper's Table RSlm, the textbook associated
Legendre functions, Laplace's equation, the ladder operators and the
addition theorems (App. A.1-A.3)."""
import os
from math import factorial

import numpy as np
import pytest
from scipy.special import lpmv

from oracle.harmonics import (from_real, get, nreal, ridx, solid_R, solid_S, to_real, tri)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pts(n=16, seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * (rng.random((n, 3)) * 2 - 1)


def test_table_rslm():
    """Table RSlm, both signs of m, at random points: exact to rounding."""
    pts = _pts(32, 1)
    x, y, z = pts.T
    r = np.sqrt(x * x + y * y + z * z)
    R = solid_R(2, x, y, z)
    S = solid_S(2, x, y, z)
    rows = 0
    with open(os.path.join(GOLDEN, "table_rslm.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, re_, se_ = [s.strip() for s in line.split("|")]
            l, m = map(int, head.split())
            env = {"x": x, "y": y, "z": z, "r": r}
            np.testing.assert_allclose(get(R, l, m), eval(re_, env), rtol=1e-14, atol=1e-15)
            np.testing.assert_allclose(get(S, l, m), eval(se_, env), rtol=1e-13, atol=1e-14)
            rows += 1
    assert rows == 9


@pytest.mark.parametrize("lmax", [14])
def test_textbook_legendre(lmax):
    """Spherical definitions of App. A.1 with scipy's P_l^m, which carries the
    Condon-Shortley factor (-1)^m exactly as the paper's (-sin t)^m."""
    pts = _pts(24, 2, 1.7)
    x, y, z = pts.T
    r = np.sqrt(x * x + y * y + z * z)
    ct = z / r
    ph = np.arctan2(y, x)
    R = solid_R(lmax, x, y, z)
    S = solid_S(lmax, x, y, z)
    for l in range(lmax + 1):
        for m in range(l + 1):
            P = lpmv(m, l, ct)
            Rref = r ** l / factorial(l + m) * P * np.exp(1j * m * ph)
            Sref = (-1) ** (l + m) * factorial(l - m) / r ** (l + 1) * P * np.exp(1j * m * ph)
            scale_r = np.max(np.abs(Rref)) + 1e-300
            scale_s = np.max(np.abs(Sref)) + 1e-300
            assert np.max(np.abs(R[:, tri(l, m)] - Rref)) <= 1e-12 * scale_r, (l, m)
            assert np.max(np.abs(S[:, tri(l, m)] - Sref)) <= 1e-12 * scale_s, (l, m)


def _fd_second(f, pts, h=1e-4):
    """Central second differences along x, y, z."""
    f0 = f(pts)
    out = []
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        out.append((f(pts + e) + f(pts - e) - 2 * f0) / h ** 2)
    return out


def test_laplace():
    """R and S solve Laplace's equation (App. A.1): the three second
    derivatives cancel to the finite-difference truncation level."""
    pts = _pts(8, 3) + np.array([0.0, 0.0, 2.5])
    p = 8
    for f in (lambda q: solid_R(p, *q.T), lambda q: solid_S(p, *q.T)):
        dxx, dyy, dzz = _fd_second(f, pts)
        lap = np.abs(dxx + dyy + dzz)
        scale = np.abs(dxx) + np.abs(dyy) + np.abs(dzz) + 1e-300
        big = scale > 1e-6 * np.max(scale)
        assert np.max(lap[big] / scale[big]) < 1e-5


def _grad_fd(f, pts, h=1e-5):
    g = []
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        g.append((f(pts + e) - f(pts - e)) / (2 * h))
    return g


def test_ladder_operators():
    """d+ = dx + i dy, dz, d- = -dx + i dy lower R by one order and raise S by
    one order while shifting m by +1, 0, -1 (App. A.2)."""
    p = 7
    pts = _pts(6, 4) + np.array([0.3, -0.2, 1.9])
    fR = lambda q: np.stack([get(solid_R(p, *q.T), l, m) for l in range(p + 1)
                             for m in range(-l, l + 1)], axis=1)
    fS = lambda q: np.stack([get(solid_S(p + 1, *q.T), l, m) for l in range(p + 1)
                             for m in range(-l, l + 1)], axis=1)
    gx, gy, gz = _grad_fd(fR, pts)
    sx, sy, sz = _grad_fd(fS, pts)
    R = solid_R(p, *pts.T)
    S = solid_S(p + 1, *pts.T)
    col = 0
    for l in range(p + 1):
        for m in range(-l, l + 1):
            dp, dz, dm = gx[:, col] + 1j * gy[:, col], gz[:, col], -gx[:, col] + 1j * gy[:, col]
            np.testing.assert_allclose(dp, get(R, l - 1, m + 1), atol=1e-8)
            np.testing.assert_allclose(dz, get(R, l - 1, m), atol=1e-8)
            np.testing.assert_allclose(dm, get(R, l - 1, m - 1), atol=1e-8)
            tp = sx[:, col] + 1j * sy[:, col]
            tm = -sx[:, col] + 1j * sy[:, col]
            sc = np.max(np.abs(get(S, l + 1, m))) + 1e-12
            assert np.max(np.abs(tp - get(S, l + 1, m + 1))) < 1e-6 * sc
            assert np.max(np.abs(sz[:, col] - get(S, l + 1, m))) < 1e-6 * sc
            assert np.max(np.abs(tm - get(S, l + 1, m - 1))) < 1e-6 * sc
            col += 1


def test_addition_theorem_R():
    """eq. additionR is a finite identity for regular harmonics."""
    p = 10
    rng = np.random.default_rng(5)
    r = rng.random(3) - 0.5
    d = rng.random(3) - 0.5
    lhs = solid_R(p, *(r + d))
    Rr = solid_R(p, *r)
    Rd = solid_R(p, *d)
    for l in range(p + 1):
        for m in range(l + 1):
            acc = 0j
            for lam in range(l + 1):
                for mu in range(-lam, lam + 1):
                    acc += get(Rr, l - lam, m - mu) * get(Rd, lam, mu)
            assert abs(acc - lhs[tri(l, m)]) < 1e-14 * max(1.0, abs(lhs[tri(l, m)]))


def test_addition_theorem_S_and_expand():
    """eq. additionS and eq. expand: the series converges to S (resp. 1/r)
    for |dr| < |r|; truncating at high order leaves only rounding."""
    L = 40
    rng = np.random.default_rng(6)
    rs = np.array([0.4, -0.3, 1.1])
    rr = 0.25 * (rng.random(3) - 0.5)
    S = solid_S(L, *rs)
    Rm = solid_R(L, *(-rr))
    approx = sum(get(S, lam, -mu) * get(Rm, lam, mu)
                 for lam in range(L + 1) for mu in range(-lam, lam + 1))
    assert abs(approx - 1.0 / np.linalg.norm(rs - rr)) < 1e-14
    # addition theorem for S_3^{-1}
    l, m = 3, 1
    lhs = get(solid_S(3, *(rs + rr)), l, -m)
    Rd = solid_R(L, *rr)
    acc = sum(get(S, l + lam, -(m + mu)) * get(Rd, lam, mu)
              for lam in range(L - l + 1) for mu in range(-lam, lam + 1))
    assert abs(acc - lhs) < 1e-12 * abs(lhs)


def test_real_storage_roundtrip():
    """App. A.6 storage: index l(l+1)+m holds Re X_l^|m| (m>=0), Im (m<0)."""
    p = 6
    X = solid_R(p, 0.3, -0.7, 0.2)
    Xr = to_real(X, p)
    assert Xr.shape == (nreal(p),)
    assert Xr[ridx(2, -1)] == X[tri(2, 1)].imag
    assert Xr[ridx(3, 2)] == X[tri(3, 2)].real
    np.testing.assert_array_equal(from_real(Xr, p), X)
