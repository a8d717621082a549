"""Solid harmonics R_l^m and S_l^m in FP64 (test infrastructure; oracle).

Definitions (App. A.1):
    R_l^m = r^l / (l+m)! P_l^m(cos t) e^{i m phi}
    S_l^m = (-1)^{l+m} (l-m)! / r^{l+1} P_l^m(cos t) e^{i m phi}
for 0 <= m <= l, with P_l^m carrying the Condon-Shortley factor
(-sin t)^m, and X_l^{-m} = (-1)^m conj(X_l^m) for negative m.

They are evaluated in Cartesian form with the scaled Legendre recursion of
App. A.5:  Ptilde_m^m = (-1)^m (2m-1)!!,  Ptilde_{m+1}^m = (2m+1) z Ptilde_m^m,
Ptilde_l^m = ((2l-1) z Ptilde_{l-1}^m - (l+m-1) r^2 Ptilde_{l-2}^m) / (l-m);
Q_l^m = Ptilde_l^m (x+iy)^m;  R_l^m = Q_l^m / (l+m)!;
S_l^{-m}(x,y,z) = (l-m)! / r^{2l+1} Q_l^m(-x, y, -z).

Complex harmonics for m >= 0 are returned in "triangular" arrays with the
last axis indexed by tri(l, m) = l(l+1)/2 + m.  Real storage (App. A.6):
X[l(l+1)+m] = Re X_l^|m| (m >= 0), Im X_l^|m| (m < 0).
"""
from __future__ import annotations

from math import factorial

import numpy as np


def tri(l: int, m: int) -> int:
    return l * (l + 1) // 2 + m


def ntri(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def nreal(p: int) -> int:
    return (p + 1) * (p + 1)


def ridx(l: int, m: int) -> int:
    """Real-storage index l(l+1)+m (m may be negative)."""
    return l * (l + 1) + m


def scaled_legendre(p: int, r2, z):
    """Ptilde_l^m(r, z) for 0 <= m <= l <= p; last axis tri(l, m)."""
    r2 = np.asarray(r2, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros(np.broadcast(r2, z).shape + (ntri(p),))
    for m in range(p + 1):
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        out[..., tri(m, m)] = (-1) ** m * dfact
        if m + 1 <= p:
            out[..., tri(m + 1, m)] = (2 * m + 1) * z * out[..., tri(m, m)]
        for l in range(m + 2, p + 1):
            out[..., tri(l, m)] = ((2 * l - 1) * z * out[..., tri(l - 1, m)]
                                   - (l + m - 1) * r2 * out[..., tri(l - 2, m)]) / (l - m)
    return out


def _Q(p: int, x, y, z):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    r2 = x * x + y * y + z * z
    P = scaled_legendre(p, r2, z)
    w = x + 1j * y
    Q = np.empty(P.shape, dtype=np.complex128)
    wm = np.ones(np.broadcast(x, y).shape, dtype=np.complex128)
    for m in range(p + 1):
        for l in range(m, p + 1):
            Q[..., tri(l, m)] = P[..., tri(l, m)] * wm
        wm = wm * w
    return Q, r2


def solid_R(p: int, x, y, z):
    """R_l^m(x, y, z) for 0 <= m <= l <= p (complex; last axis tri)."""
    Q, _ = _Q(p, x, y, z)
    for l in range(p + 1):
        for m in range(l + 1):
            Q[..., tri(l, m)] /= factorial(l + m)
    return Q


def solid_S(p: int, x, y, z):
    """S_l^m(x, y, z) for 0 <= m <= l <= p (complex; last axis tri)."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    Q, r2 = _Q(p, -x, y, -z)
    rinv2 = 1.0 / r2
    rpow = np.sqrt(rinv2)  # 1 / r^{2l+1} at l = 0
    out = np.empty(Q.shape, dtype=np.complex128)
    for l in range(p + 1):
        for m in range(l + 1):
            s_neg = factorial(l - m) * rpow * Q[..., tri(l, m)]  # S_l^{-m}
            out[..., tri(l, m)] = (-1) ** m * np.conj(s_neg)
        rpow = rpow * rinv2
    return out


def get(X, l: int, m: int):
    """X_l^m for any -l <= m <= l from a triangular (m >= 0) array, via the
    conjugate relation X_l^{-m} = (-1)^m conj(X_l^m); zero outside |m| <= l."""
    if l < 0 or abs(m) > l:
        return np.zeros(X.shape[:-1], dtype=np.complex128)
    if m >= 0:
        return X[..., tri(l, m)]
    return (-1) ** (-m) * np.conj(X[..., tri(l, -m)])


def to_real(X, p: int):
    """Real storage of a triangular complex array (last axis -> (p+1)^2)."""
    out = np.empty(X.shape[:-1] + (nreal(p),))
    for l in range(p + 1):
        out[..., ridx(l, 0)] = X[..., tri(l, 0)].real
        for m in range(1, l + 1):
            out[..., ridx(l, m)] = X[..., tri(l, m)].real
            out[..., ridx(l, -m)] = X[..., tri(l, m)].imag
    return out


def from_real(Xr, p: int):
    """Inverse of :func:`to_real` (Im X_l^0 is taken as zero)."""
    out = np.empty(Xr.shape[:-1] + (ntri(p),), dtype=np.complex128)
    for l in range(p + 1):
        out[..., tri(l, 0)] = Xr[..., ridx(l, 0)]
        for m in range(1, l + 1):
            out[..., tri(l, m)] = Xr[..., ridx(l, m)] + 1j * Xr[..., ridx(l, -m)]
    return out
