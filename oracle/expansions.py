"""Single-centre multipole transformations of App. A.3, complex form, FP64
(test infrastructure; oracle).

All coefficient sets are triangular complex arrays (m >= 0, last axis
tri(l, m)); negative m follows from the conjugate relation.  These are used
to pin the mesh pipeline in :mod:`oracle.pmmm` against first principles.
"""
from __future__ import annotations

import numpy as np

from .harmonics import get, ntri, solid_R, solid_S, tri


def p2m(p, centre, pos, q):
    """eq. P2M: M_l^m = sum_i q_i R_l^m(r_M - r_i)."""
    d = np.asarray(centre)[None, :] - np.asarray(pos)
    R = solid_R(p, d[:, 0], d[:, 1], d[:, 2])
    return (np.asarray(q)[:, None] * R).sum(axis=0)


def m2p(p, M, centre, pts):
    """eq. M2P: Phi(r) = sum_{l,m} M_l^m S_l^{-m}(r - r_M)."""
    d = np.asarray(pts) - np.asarray(centre)[None, :]
    S = solid_S(p, d[:, 0], d[:, 1], d[:, 2])
    out = np.zeros(d.shape[0], dtype=np.complex128)
    for l in range(p + 1):
        for m in range(-l, l + 1):
            out += get(M, l, m) * get(S, l, -m)
    return out.real


def m2l(p, M, rM, rL):
    """eq. M2L: L_l^m = sum_{lam,mu} M_lam^mu S_{l+lam}^{-(m+mu)}(r_L - r_M)."""
    d = np.asarray(rL, dtype=np.float64) - np.asarray(rM, dtype=np.float64)
    S = solid_S(2 * p, d[0], d[1], d[2])
    L = np.zeros(ntri(p), dtype=np.complex128)
    for l in range(p + 1):
        for m in range(l + 1):
            acc = 0j
            for lam in range(p + 1):
                for mu in range(-lam, lam + 1):
                    acc += get(M, lam, mu) * get(S, l + lam, -(m + mu))
            L[tri(l, m)] = acc
    return L


def l2p(p, L, rL, pts):
    """eq. L2P: Phi(r) = sum_{l,m} L_l^m R_l^m(r - r_L)."""
    d = np.asarray(pts) - np.asarray(rL)[None, :]
    R = solid_R(p, d[:, 0], d[:, 1], d[:, 2])
    out = np.zeros(d.shape[0], dtype=np.complex128)
    for l in range(p + 1):
        for m in range(-l, l + 1):
            out += get(L, l, m) * get(R, l, m)
    return out.real


def l2l(p, L, rL, rL2, pout=None):
    """eq. L2L: L'_l^m = sum_{lam>=l} sum_mu L_lam^mu R_{lam-l}^{mu-m}(r_L' - r_L),
    for 0 <= m <= l <= pout (default p)."""
    pout = p if pout is None else pout
    d = np.asarray(rL2, dtype=np.float64) - np.asarray(rL, dtype=np.float64)
    R = solid_R(p, d[0], d[1], d[2])
    out = np.zeros(ntri(pout), dtype=np.complex128)
    for l in range(pout + 1):
        for m in range(l + 1):
            acc = 0j
            for lam in range(l, p + 1):
                for mu in range(-lam, lam + 1):
                    acc += get(L, lam, mu) * get(R, lam - l, mu - m)
            out[tri(l, m)] = acc
    return out


def m2m(p, M, rM, rM2):
    """eq. M2M: M'_l^m = sum_{lam<=l} sum_mu M_{l-lam}^{m-mu} R_lam^mu(r_M' - r_M)."""
    d = np.asarray(rM2, dtype=np.float64) - np.asarray(rM, dtype=np.float64)
    R = solid_R(p, d[0], d[1], d[2])
    out = np.zeros(ntri(p), dtype=np.complex128)
    for l in range(p + 1):
        for m in range(l + 1):
            acc = 0j
            for lam in range(l + 1):
                for mu in range(-lam, lam + 1):
                    acc += get(M, l - lam, m - mu) * get(R, lam, mu)
            out[tri(l, m)] = acc
    return out


def gradient_from_L1(L1):
    """eq. phigrad: grad Phi at the expansion centre from the order-1 local
    coefficients: (-Re L_1^1, Im L_1^1, L_1^0)."""
    return np.array([-L1[tri(1, 1)].real, L1[tri(1, 1)].imag, L1[tri(1, 0)].real])
