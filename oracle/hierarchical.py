"""Two-level hierarchical PMMM (Sec. 5.2), FP64 (test infrastructure; oracle).
Only tests/ use this module.

An open coarse mesh of n^3 cells is refined by r per axis into a fine mesh
of (n r)^3 cells of the same box; c is the near-cube half width on both
levels.  A pair of particles i, j is counted by
  * the coarse PMMM when their coarse cells are more than c apart
    (Chebyshev distance; oracle.pmmm.far_field on the coarse mesh);
  * the fine level when their coarse cells are within c but their fine cells
    are more than c apart: the local expansion of fine cell I gathers
    eq. M2L of the moments of every such fine cell J (written in the
    real-matrix form of eq. realmatrix with the real values of S at the
    displacement r_I - r_J), then eq. L2P and the order-one eq. L2L give the
    potential and gradient;
  * the near field when their fine cells are within c (the direct sum).
Far field of the hierarchy = coarse part + fine part.  The coarse
neighbourhood of a source cell spans fine displacements up to
D = (c + 1) r - 1 per axis, the margin of the paper's local convolution.

Readings: the paper describes the split and its cost, not an algorithm
listing; the coarse level here is the uniform open PMMM of the coarse mesh,
the fine moments are eq. P2M about the fine-cell centres, and the fine level
evaluates the restricted sum directly, offset by offset (the paper's local
FFT convolution computes the same sum).

Parity status: pinned by tests/test_oracle_hierarchical.py against the
complex single-centre eq. M2L summed pair by pair, the r = 1 reduction to
the coarse PMMM, and the direct sum.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import pmmm as opm
from .harmonics import solid_S, to_real


def fine_config(cfg: opm.Config, r: int) -> opm.Config:
    """The fine mesh: r times the cells per axis, same box, order and c."""
    if cfg.boundary != "open" or cfg.shape is not None:
        raise ValueError("the hierarchy is built on an open cubic coarse mesh")
    return dataclasses.replace(cfg, n=cfg.n * r)


def fine_local_mesh(M, cfg: opm.Config, r: int):
    """Fine local expansions [P, nz, ny, nx] (physical units) from fine
    moments M [P, nz, ny, nx] for the pairs of fine cells whose coarse cells
    are within c and whose fine cells are farther than c."""
    fcfg = fine_config(cfg, r)
    nf, c, p, h = fcfg.n, cfg.cutoff, cfg.p, fcfg.h
    D = (c + 1) * r - 1
    coarse = np.arange(nf) // r
    L = np.zeros(M.shape, dtype=np.complex128)
    for dz in range(-D, D + 1):
        for dy in range(-D, D + 1):
            for dx in range(-D, D + 1):
                if max(abs(dx), abs(dy), abs(dz)) <= c:
                    continue                       # fine near cube: direct sum
                idx = []
                for d in (dz, dy, dx):             # targets i, sources i - d
                    i = np.arange(max(0, d), min(nf, nf + d))
                    keep = np.abs(coarse[i] - coarse[i - d]) <= c
                    idx.append(i[keep])
                if any(len(a) == 0 for a in idx):
                    continue
                iz, iy, ix = idx
                S = solid_S(2 * p, np.float64(dx * h), np.float64(dy * h), np.float64(dz * h))
                G = to_real(S, 2 * p)[:, None, None, None]
                src = M[:, (iz - dz)[:, None, None], (iy - dy)[None, :, None], (ix - dx)[None, None, :]]
                L[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]] += opm.m2l_wave(G, src, p)
    return L.real


def far_field(pos, q, cfg: opm.Config, r: int):
    """Far field of the hierarchy: (phi, grad) of the coarse PMMM plus the
    fine level."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    coarse = opm.far_field(pos, q, cfg)
    fcfg = fine_config(cfg, r)
    M, _ = opm.p2m_mesh(pos, q, fcfg)
    L = fine_local_mesh(M, cfg, r)
    phi, grad = opm.l2p(L, pos, fcfg)
    return coarse.phi + phi, coarse.grad + grad


__all__ = ["fine_config", "fine_local_mesh", "far_field"]
