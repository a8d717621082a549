"""Literal FP64 PMMM far field (test infrastructure; oracle).

Follows the paper's procedure step by step (Sec. 2.1 and App. A-C), in
physical units, with numpy's FFT as the transform primitive:

  1. cells        each particle belongs to cell I = floor(r/h) (periodic
                  positions are wrapped into the box first), centre (I+1/2)h
  2. p2m_mesh     eq. P2M per cell: M_l^m = sum_i q_i R_l^m(r_M - r_i)
  3. green_open / green_periodic
                  transfer-kernel meshes of S_n^k, n <= 2p, in real storage
                  (App. C layout for open boundaries, eq. greenPBC for
                  periodic ones), masked on the near cells
  4. spectra      unnormalised forward DFT of each mesh component
  5. m2l_wave     the real-matrix M2L (eq. realmatrix) with every real
                  coefficient replaced by its complex spectrum value
  6. local_mesh   inverse DFT (1/n_f^3), open: the [0, n)^3 octant
                  (open meshes may have nx, ny, nz cells of one edge h: the
                  zero padding and the octant are taken per axis)
  7. periodic_corrections
                  dipole, self and r^2 corrections (App. B, correction
                  procedure) and the charged-system terms
  8. l2p          eq. L2P for Phi and eq. L2L to order one + eq. phigrad
                  for grad Phi

Returned quantities are the FAR field only: Phi_i and grad Phi_i, with
Phi = sum_j q_j / |r - r_j|.
"""
from __future__ import annotations

import dataclasses
from math import pi, sqrt

import numpy as np

from . import _clib
from .harmonics import from_real, get, nreal, ridx, solid_R, solid_S, to_real, tri


@dataclasses.dataclass(frozen=True)
class Config:
    n: int                 # cells per axis (cubic mesh of a cubic box)
    p: int                 # expansion order
    boundary: str          # "open" or "periodic"
    box: float = 1.0       # box edge b
    cutoff: int = 2        # near cube half-width c (27 cells: 1, 125 cells: 2)
    alpha: float | None = None   # periodic splitting parameter (default 1.5/b)
    images: int = 4        # lattice-sum radius: |r + n b| <= images b (real), |n| <= images (reciprocal)
    shape: tuple | None = None   # open boundary: (nx, ny, nz) cells of edge h = box / nx; None: n^3

    def __post_init__(self):
        if self.shape is not None:
            if self.boundary != "open":
                raise ValueError("a non-cubic mesh needs the open boundary")
            if tuple(self.shape)[0] != self.n:
                raise ValueError("shape[0] must equal n (box is the x edge)")

    @property
    def dims(self) -> tuple:
        """Cells per axis (x, y, z)."""
        return tuple(self.shape) if self.shape is not None else (self.n, self.n, self.n)

    @property
    def extent(self) -> np.ndarray:
        """Box edges (x, y, z): cubic cells of edge h."""
        return self.h * np.asarray(self.dims, dtype=np.float64)

    @property
    def h(self) -> float:
        return self.box / self.n

    @property
    def nf(self) -> int:
        return 2 * self.n if self.boundary == "open" else self.n

    @property
    def a(self) -> float:
        return 1.5 / self.box if self.alpha is None else self.alpha

    @property
    def V(self) -> float:
        return self.box ** 3


# ---------------------------------------------------------------- step 1
def cells(pos, cfg: Config):
    """Integer cell (N, 3) [x, y, z], cell centres and positions relative to
    them.  Open boundaries reject particles outside [0, b)."""
    pos = np.asarray(pos, dtype=np.float64)
    if cfg.boundary == "periodic":
        pos = pos - cfg.box * np.floor(pos / cfg.box)
    elif np.any((pos < 0) | (pos >= cfg.extent[None, :])):
        raise ValueError("open boundary: particle outside the box")
    I = np.floor(pos / cfg.h).astype(np.int64)
    I = np.clip(I, 0, np.asarray(cfg.dims)[None, :] - 1)
    centre = (I + 0.5) * cfg.h
    return I, centre, pos - centre, pos


def linear_cell(I, dims):
    """Cell index (z ny + y) nx + x; dims = (nx, ny, nz), or n for n^3."""
    nx, ny, _ = (dims, dims, dims) if np.isscalar(dims) else dims
    return (I[:, 2] * ny + I[:, 1]) * nx + I[:, 0]


# ---------------------------------------------------------------- step 2
def p2m_mesh(pos, q, cfg: Config, chunk: int = 1 << 16):
    """Moment meshes M[P, z, y, x] (real storage) and the per-cell sums
    sum_k q_k |r_k^rel|^2 [z, y, x] used by the periodic correction."""
    P = nreal(cfg.p)
    nx, ny, nz = cfg.dims
    K = nx * ny * nz
    I, centre, rel, _ = cells(pos, cfg)
    lin = linear_cell(I, cfg.dims)
    q = np.asarray(q, dtype=np.float64)
    M = np.zeros((P, K))
    for s in range(0, len(q), chunk):
        e = min(len(q), s + chunk)
        d = -rel[s:e]                      # r_M - r_i
        R = solid_R(cfg.p, d[:, 0], d[:, 1], d[:, 2])
        Mr = to_real(q[s:e, None] * R, cfg.p)
        for c in range(P):
            M[c] += np.bincount(lin[s:e], weights=Mr[:, c], minlength=K)
    qr2 = np.bincount(lin, weights=q * np.sum(rel * rel, axis=1), minlength=K)
    return M.reshape(P, nz, ny, nx), qr2.reshape(nz, ny, nx)


# ---------------------------------------------------------------- step 3
def green_open(cfg: Config):
    """Open-boundary transfer-kernel mesh on the zero-padded mesh of twice
    the cells per axis (App. C, Fig. green; per axis a of n_a cells): index
    d -> displacement d (d < n_a) or d - 2 n_a (d > n_a); the index-n_a
    planes and the near cube max|delta| <= c are zero; elsewhere
    S_k^j(delta h) for orders k <= 2p, real storage, [Q, 2nz, 2ny, 2nx]."""
    p2 = 2 * cfg.p
    ax = []
    for na in cfg.dims:
        d = np.arange(2 * na)
        ax.append((np.where(d < na, d, d - 2 * na), d == na))
    (dx, px), (dy, py), (dz, pz) = ax
    DZ, DY, DX = np.meshgrid(dz, dy, dx, indexing="ij")
    onplane = pz[:, None, None] | py[None, :, None] | px[None, None, :]
    cheb = np.maximum(np.maximum(np.abs(DX), np.abs(DY)), np.abs(DZ))
    zero = onplane | (cheb <= cfg.cutoff)
    h = cfg.h
    X = np.where(zero, 1.0, DX * h)
    S = solid_S(p2, X, DY * h, DZ * h)
    G = to_real(S, p2)
    G[zero] = 0.0
    return np.moveaxis(G, -1, 0).copy()


def green_periodic(cfg: Config):
    """Periodic transfer-kernel mesh on the n^3 mesh (App. B, eq. greenPBC
    minus the near images), computed by the oracle's C lattice sums."""
    n, p2 = cfg.n, 2 * cfg.p
    if n < 2 * cfg.cutoff + 1:
        raise ValueError("periodic mesh needs n >= 2c + 1")
    G = np.zeros((nreal(p2), n, n, n))
    _clib.lib().ora_green_periodic(n, cfg.box, p2, cfg.cutoff, cfg.a, cfg.images,
                                   _clib.dptr(G))
    return G


def lower_gamma_half(lmax: int, x: float):
    """Regularised lower incomplete gamma P(l + 1/2, x) for l = 0..lmax (the
    C series the periodic kernel uses for the subtracted near image)."""
    out = np.zeros(lmax + 1)
    _clib.lib().ora_lower_gamma_half(int(lmax), float(x), _clib.dptr(out))
    return out


def green(cfg: Config):
    return green_open(cfg) if cfg.boundary == "open" else green_periodic(cfg)


# ---------------------------------------------------------------- step 4
def spectra(mesh):
    """Unnormalised forward real-to-complex DFT over the last three axes."""
    return np.fft.rfftn(mesh, axes=(-3, -2, -1))


# ---------------------------------------------------------------- step 5
def _re_S(Gt, n, k):
    """Spectrum of the mesh Re S_n^k for any k (conjugate relation)."""
    if abs(k) > n:
        return 0.0
    if k >= 0:
        return Gt[ridx(n, k)]
    return (-1) ** (-k) * Gt[ridx(n, -k)]


def _im_S(Gt, n, k):
    """Spectrum of the mesh Im S_n^k for any k (conjugate relation)."""
    if abs(k) > n or k == 0:
        return 0.0
    if k > 0:
        return Gt[ridx(n, -k)]
    return -((-1) ** (-k)) * Gt[ridx(n, k)]


def m2l_wave(Gt, Mt, p: int):
    """eq. realmatrix in wave space.  For output (l, m >= 0), input (lam, mu):
    G^{m,mu}_{l,lam} = S_{l+lam}^{-(m+mu)} (eq. M2L);
    A = Re G^{m,mu}, B = Im G^{m,mu}, C = (-1)^mu Re G^{m,-mu},
    D = (-1)^mu Im G^{m,-mu};
    Re L += A M^0 + sum_{mu>=1} [(A+C) Re M - (B-D) Im M];
    Im L += B M^0 + sum_{mu>=1} [(B+D) Re M + (A-C) Im M]."""
    Lt = np.zeros((nreal(p),) + Mt.shape[1:], dtype=np.complex128)
    for l in range(p + 1):
        for m in range(l + 1):
            acc_re = np.zeros(Mt.shape[1:], dtype=np.complex128)
            acc_im = np.zeros(Mt.shape[1:], dtype=np.complex128)
            for lam in range(p + 1):
                nn = l + lam
                A = _re_S(Gt, nn, -m)
                B = _im_S(Gt, nn, -m)
                acc_re = acc_re + A * Mt[ridx(lam, 0)]
                acc_im = acc_im + B * Mt[ridx(lam, 0)]
                for mu in range(1, lam + 1):
                    A = _re_S(Gt, nn, -(m + mu))
                    B = _im_S(Gt, nn, -(m + mu))
                    sg = (-1) ** mu
                    C = sg * _re_S(Gt, nn, -(m - mu))
                    D = sg * _im_S(Gt, nn, -(m - mu))
                    Mre, Mim = Mt[ridx(lam, mu)], Mt[ridx(lam, -mu)]
                    acc_re = acc_re + (A + C) * Mre - (B - D) * Mim
                    acc_im = acc_im + (B + D) * Mre + (A - C) * Mim
            Lt[ridx(l, m)] = acc_re
            if m > 0:
                Lt[ridx(l, -m)] = acc_im
    return Lt


# ---------------------------------------------------------------- step 6
def local_mesh(M, cfg: Config, Gt=None):
    """L = F^{-1}{ G~ M~ } on the FFT mesh; open boundaries zero-pad M into
    the [0, n)^3 octant of the (2n)^3 mesh and keep that octant of L."""
    if Gt is None:
        Gt = spectra(green(cfg))
    nx, ny, nz = cfg.dims
    if cfg.boundary == "open":
        sf = (2 * nz, 2 * ny, 2 * nx)
        Mp = np.zeros((M.shape[0],) + sf)
        Mp[:, :nz, :ny, :nx] = M
    else:
        sf = (nz, ny, nx)
        Mp = M
    Lt = m2l_wave(Gt, spectra(Mp), cfg.p)
    L = np.fft.irfftn(Lt, s=sf, axes=(-3, -2, -1))
    return L[:, :nz, :ny, :nx].copy()


# ---------------------------------------------------------------- step 7
def periodic_corrections(L, M, qr2, cfg: Config):
    """Correction procedure of App. B for periodic boundaries:
    L_1^0 += 4 pi/(3V) sum_J M_1^0;  L_1^1 += 8 pi/(3V) conj(sum_J M_1^1);
    L_0^0 += -(2 alpha/sqrt(pi)) M_0^0(cell) + 2 pi/(3V) sum_k q_k |r_k^rel|^2.
    Returns the corrected local mesh and the total charge."""
    L = L.copy()
    V, a = cfg.V, cfg.a
    sM = M.reshape(M.shape[0], -1).sum(axis=1)
    if cfg.p >= 1:
        # the dipole terms act on L_1^m, which a p = 0 expansion does not carry
        L[ridx(1, 0)] += 4 * pi / (3 * V) * sM[ridx(1, 0)]
        L[ridx(1, 1)] += 8 * pi / (3 * V) * sM[ridx(1, 1)]
        L[ridx(1, -1)] += -8 * pi / (3 * V) * sM[ridx(1, -1)]
    L[ridx(0, 0)] += -(2 * a / sqrt(pi)) * M[ridx(0, 0)] + 2 * pi / (3 * V) * qr2.sum()
    return L, sM[ridx(0, 0)]


# ---------------------------------------------------------------- step 8
def l2p(L, pos, cfg: Config, chunk: int = 1 << 16):
    """eq. L2P for Phi and eq. L2L (destination order one) with eq. phigrad
    for grad Phi, at each particle from the local expansion of its cell."""
    p = cfg.p
    I, centre, rel, _ = cells(pos, cfg)
    lin = linear_cell(I, cfg.dims)
    Lf = L.reshape(L.shape[0], -1)
    N = len(lin)
    phi = np.empty(N)
    grad = np.empty((N, 3))
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        Lc = from_real(Lf[:, lin[s:e]].T, p)
        d = rel[s:e]                       # r - r_L
        R = solid_R(p, d[:, 0], d[:, 1], d[:, 2])
        ph = np.zeros(e - s, dtype=np.complex128)
        for lam in range(p + 1):
            for mu in range(-lam, lam + 1):
                ph += get(Lc, lam, mu) * get(R, lam, mu)
        phi[s:e] = ph.real
        L10 = np.zeros(e - s, dtype=np.complex128)
        L11 = np.zeros(e - s, dtype=np.complex128)
        for lam in range(1, p + 1):
            for mu in range(-lam, lam + 1):
                L10 += get(Lc, lam, mu) * get(R, lam - 1, mu)
                L11 += get(Lc, lam, mu) * get(R, lam - 1, mu - 1)
        grad[s:e, 0] = -L11.real
        grad[s:e, 1] = L11.imag
        grad[s:e, 2] = L10.real
    return phi, grad


def charged_system_terms(pos, qtot, cfg: Config):
    """Per-particle terms for a periodic system with nonzero total charge:
    Phi += 2 pi/(3V) Q (|r^rel|^2 - 3/(2 alpha^2)),  grad += 4 pi/(3V) Q r^rel."""
    _, _, rel, _ = cells(pos, cfg)
    V, a = cfg.V, cfg.a
    dphi = 2 * pi / (3 * V) * qtot * (np.sum(rel * rel, axis=1) - 3.0 / (2 * a * a))
    dgrad = 4 * pi / (3 * V) * qtot * rel
    return dphi, dgrad


# ---------------------------------------------------------------- pipeline
@dataclasses.dataclass
class FarResult:
    phi: np.ndarray
    grad: np.ndarray
    M: np.ndarray          # moment mesh [P, n, n, n]
    L: np.ndarray          # local mesh [P, n, n, n] (after corrections)
    qr2: np.ndarray


def far_field(pos, q, cfg: Config, Gt=None, eval_idx=None) -> FarResult:
    """The whole far-field pipeline.  ``Gt`` may carry precomputed transfer
    spectra; ``eval_idx`` restricts L2P to a subset of particles (P2M still
    uses every particle)."""
    pos = np.asarray(pos, dtype=np.float64)
    M, qr2 = p2m_mesh(pos, q, cfg)
    L = local_mesh(M, cfg, Gt)
    qtot = 0.0
    if cfg.boundary == "periodic":
        L, qtot = periodic_corrections(L, M, qr2, cfg)
    ev = pos if eval_idx is None else pos[eval_idx]
    phi, grad = l2p(L, ev, cfg)
    if cfg.boundary == "periodic":
        dphi, dgrad = charged_system_terms(ev, qtot, cfg)
        phi = phi + dphi
        grad = grad + dgrad
    return FarResult(phi, grad, M, L, qr2)


def mesh_scales(cfg: Config):
    """Factors that convert physical-unit meshes to cell units:
    M_l (cell units) = M_l / h^l, L_l (cell units) = L_l h^{l+1}."""
    p, h = cfg.p, cfg.h
    sm = np.empty(nreal(p))
    sl = np.empty(nreal(p))
    for l in range(p + 1):
        for m in range(-l, l + 1):
            sm[ridx(l, m)] = h ** (-l)
            sl[ridx(l, m)] = h ** (l + 1)
    return sm, sl
