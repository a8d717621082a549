"""Exact references in FP64 (test infrastructure; oracle): the open-boundary
direct sum, the Ewald sum for periodic boundaries, and the PMMM near field.

Phi = sum_j q_j / |r - r_j| everywhere; returned gradients are grad Phi.
"""
from __future__ import annotations

import ctypes
from math import ceil, erfc, pi, sqrt

import numpy as np

from . import _clib
from .pmmm import Config, cells


def direct(pos, q):
    """O(N^2) open-boundary potential and gradient (all pairs j != i)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = len(q)
    phi = np.empty(n)
    grad = np.empty((n, 3))
    _clib.lib().ora_direct(n, _clib.dptr(pos), _clib.dptr(q), _clib.dptr(phi), _clib.dptr(grad))
    return phi, grad


def direct_at(pos, q, idx):
    """Rows idx of direct(pos, q): the open-boundary potential and gradient
    at the listed particles from all other particles."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = len(idx)
    phi = np.empty(m)
    grad = np.empty((m, 3))
    _clib.lib().ora_direct_at(len(q), _clib.dptr(pos), _clib.dptr(q), m,
                              idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              _clib.dptr(phi), _clib.dptr(grad))
    return phi, grad


def ewald_params(box: float, tol: float = 1e-16, alpha: float | None = None):
    """Real-space cutoff below b/2 (minimum image) and the reciprocal radius
    for a requested truncation level; alpha defaults to 14/b."""
    a = 14.0 / box if alpha is None else alpha
    # real space: erfc(a r) / r < tol
    rc = 0.5 * box
    r = 1e-3 * box
    while r < 0.5 * box and erfc(a * r) / r > tol:
        r += 1e-3 * box
    rc = min(r, 0.5 * box)
    # reciprocal: exp(-(pi k / a)^2) / (pi V k^2) < tol
    kmax = int(ceil(sqrt(-np.log(tol)) * a * box / pi)) + 1
    return a, rc, kmax


def ewald(pos, q, box: float = 1.0, alpha: float | None = None, tol: float = 1e-16,
          images: int = 0, rcut: float | None = None, kmax: int | None = None):
    """Ewald reference of App. B (eq. refewald, read with the charge factor
    q_j in both sums and the self term -(2 alpha/sqrt(pi)) q_i; tin-foil
    boundary, k = 0 omitted, plus -(pi/(V alpha^2)) Q_tot)."""
    a, rc, km = ewald_params(box, tol, alpha)
    if rcut is not None:
        rc = rcut
    if kmax is not None:
        km = kmax
    pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64) % box)
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = len(q)
    phi = np.empty(n)
    grad = np.empty((n, 3))
    _clib.lib().ora_ewald(n, _clib.dptr(pos), _clib.dptr(q), box, a, images, rc, km,
                          _clib.dptr(phi), _clib.dptr(grad))
    return phi, grad


def near(pos, q, cfg: Config):
    """Near field of PMMM (Sec. 2.1): direct 1/r sum over the particles of
    the (2c+1)^3 cells around each particle's cell; periodic meshes wrap the
    cell offset with the matching image shift."""
    I, _, _, wpos = cells(pos, cfg)
    if cfg.shape is not None and len(set(cfg.dims)) > 1:
        return _near_pairs(wpos, q, I, cfg.cutoff)
    wpos = np.ascontiguousarray(wpos, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    ci = np.ascontiguousarray(I.astype(np.int32))
    n = len(q)
    phi = np.empty(n)
    grad = np.empty((n, 3))
    _clib.lib().ora_near(n, _clib.dptr(wpos), _clib.dptr(q), _clib.iptr(ci), cfg.n, cfg.box,
                         cfg.cutoff, 1 if cfg.boundary == "periodic" else 0,
                         _clib.dptr(phi), _clib.dptr(grad))
    return phi, grad


def _near_pairs(pos, q, I, cutoff, chunk=512):
    """Open-boundary near field by brute force over all pairs: the pairs
    whose cells lie within the near cube, max_a |I_a - J_a| <= c."""
    q = np.asarray(q, dtype=np.float64)
    n = len(q)
    phi = np.zeros(n)
    grad = np.zeros((n, 3))
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        d = pos[s:e, None, :] - pos[None, :, :]            # r_i - r_j
        r2 = np.sum(d * d, axis=2)
        near = np.max(np.abs(I[s:e, None, :] - I[None, :, :]), axis=2) <= cutoff
        near[np.arange(e - s), np.arange(s, e)] = False
        w = np.where(near, q[None, :] / np.sqrt(np.where(near, r2, 1.0)), 0.0)
        phi[s:e] = w.sum(axis=1)
        grad[s:e] = -np.einsum("ij,ijk->ik", w / np.where(near, r2, 1.0), d)
    return phi, grad


def rel_rms(a, b):
    """sqrt(sum |a - b|^2 / sum |b|^2) over all entries."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))
