"""Coefficient storage variants of the paper, FP64/integer (test infrastructure;
oracle).  Only tests/, the package's smoke check and the benchmark's CPU
baseline use this module.

1. Per-order fixed point (Sec. 5.3 and its footnote).  A coefficient of order
   l is held in b_l = 3 (p + 1 - l) bits, so the (2l + 1) real words of order
   l cost 3 (2l + 1)(p + 1 - l) bits and a whole cell
   3 (p + 1)(p + 2)(2p + 3) / 6 bits (612 at p = 7, where order 0 starts at
   24 bits).  The paper fixes the bit counts only; the readings used here:
     * words are the real storage of the moments or local expansions (App. A
       real form: index l(l+1)+m holds Re X_l^|m| for m >= 0 and Im X_l^|m|
       for m < 0), one float32 value per word;
     * the unit of order l is a power of two 2^e_l shared by the whole mesh;
       chosen automatically, it is the smallest one under which the largest
       |word| A of that order still rounds inside the signed range: with
       A = f 2^E (1/2 <= f < 1), e_l = E - (b_l - 1), plus one when
       rint(A / 2^e_l) reaches 2^(b_l - 1); an order whose words are all
       zero takes e_l = 0; an order holding a non-finite word takes the
       marker EXP_INVALID and decodes to NaN;
     * code = rint(word / 2^e_l) (round half to even) clamped to
       +-(2^(b_l - 1) - 1), NaN coded as 0, stored as b_l-bit two's
       complement;
     * a cell's codes follow each other in real-storage order in one bit
       stream, bit j of the stream being bit (j mod 32) of 32-bit word
       j div 32; the record is padded with zero bits to whole 32-bit words.
   Scaling by a power of two is exact, so the rounding decision is the same
   in any binary precision that holds the word.

2. Complex composition of two real sets (App. D).  Two coefficient sets A
   and B, each obeying X_l^{-m} = (-1)^m conj(X_l^m), are carried as one
   complex set C_l^m = A_l^m + i B_l^m over every m in [-l, l]; by linearity
   the M2L of C is the composite of the M2Ls of A and B, and the split below
   recovers the two sets.

Parity status: pinned by tests/test_oracle_storage.py against the bit counts
the paper prints, a big-integer re-reading of the bit stream, hand-computed
codes, the round-trip error bound of the rounding, and eq. M2L of the
single-centre oracle applied to each set apart.
"""
from __future__ import annotations

import numpy as np

from .harmonics import from_real, get, nreal, ridx, solid_S

EXP_INVALID = -(2 ** 31)


# ----------------------------------------------------------------- fixed point
def order_bits(p: int) -> list[int]:
    """Bits per word of each order l = 0..p (footnote of Sec. 5.3)."""
    return [3 * (p + 1 - l) for l in range(p + 1)]


def word_order(p: int) -> np.ndarray:
    """Order l of each real-storage word k = l(l+1)+m."""
    return np.array([l for l in range(p + 1) for _ in range(2 * l + 1)], dtype=np.int64)


def cell_bits(p: int) -> int:
    """Bits of one cell record: the sum over all (p+1)^2 words."""
    b = order_bits(p)
    return int(sum(b[l] for l in word_order(p)))


def cell_words(p: int) -> int:
    """32-bit words of one (zero-padded) cell record."""
    return (cell_bits(p) + 31) // 32


def auto_exponents(coef, p: int) -> np.ndarray:
    """Exponents e_l of the units 2^e_l chosen from the mesh.

    coef: float32 array [(p+1)^2, ncell] (real storage, component-major)."""
    c = np.asarray(coef, dtype=np.float32).reshape(nreal(p), -1)
    lw = word_order(p)
    b = order_bits(p)
    e = np.zeros(p + 1, dtype=np.int64)
    for l in range(p + 1):
        words = c[lw == l].astype(np.float64)
        if words.size == 0:
            continue
        if not np.all(np.isfinite(words)):
            e[l] = EXP_INVALID
            continue
        amax = np.abs(words).max()
        if amax == 0.0:
            e[l] = 0
            continue
        _, E = np.frexp(amax)
        e[l] = int(E) - (b[l] - 1)
        if np.rint(np.ldexp(amax, -int(e[l]))) > 2 ** (b[l] - 1) - 1:
            e[l] += 1
    return e


def encode(coef, p: int, exps) -> np.ndarray:
    """Integer codes [ncell, (p+1)^2] of float32 words under units 2^e_l."""
    c = np.asarray(coef, dtype=np.float32).reshape(nreal(p), -1).astype(np.float64)
    lw = word_order(p)
    b = np.array(order_bits(p), dtype=np.int64)
    ex = np.asarray(exps, dtype=np.int64)
    codes = np.zeros(c.shape, dtype=np.int64)
    for k in range(nreal(p)):
        l = lw[k]
        if ex[l] == EXP_INVALID:
            continue
        lim = float(2 ** (int(b[l]) - 1) - 1)
        with np.errstate(over="ignore", invalid="ignore"):
            v = np.rint(np.ldexp(c[k], -int(ex[l])))
        v = np.where(np.isnan(v), 0.0, np.clip(v, -lim, lim))
        codes[k] = v.astype(np.int64)
    return codes.T.copy()


def pack(codes, p: int) -> np.ndarray:
    """Bit-stream records [ncell, cell_words(p)] (uint32) of the codes."""
    codes = np.asarray(codes, dtype=np.int64)
    ncell = codes.shape[0]
    words = np.zeros((ncell, cell_words(p)), dtype=np.uint64)
    lw = word_order(p)
    b = order_bits(p)
    off = 0
    for k in range(nreal(p)):
        nb = b[lw[k]]
        u = codes[:, k].astype(np.uint64) & np.uint64((1 << nb) - 1)   # two's complement field
        w, s = divmod(off, 32)
        words[:, w] |= (u << np.uint64(s)) & np.uint64(0xFFFFFFFF)
        if s + nb > 32:
            words[:, w + 1] |= (u >> np.uint64(32 - s)) & np.uint64(0xFFFFFFFF)
        off += nb
    return words.astype(np.uint32)


def unpack(packed, p: int) -> np.ndarray:
    """Codes [ncell, (p+1)^2] from bit-stream records."""
    wd = np.asarray(packed, dtype=np.uint32).astype(np.uint64)
    ncell = wd.shape[0]
    codes = np.zeros((ncell, nreal(p)), dtype=np.int64)
    lw = word_order(p)
    b = order_bits(p)
    off = 0
    for k in range(nreal(p)):
        nb = b[lw[k]]
        w, s = divmod(off, 32)
        u = wd[:, w] >> np.uint64(s)
        if s + nb > 32:
            u |= wd[:, w + 1] << np.uint64(32 - s)
        u &= np.uint64((1 << nb) - 1)
        v = u.astype(np.int64)
        codes[:, k] = np.where(v >= (1 << (nb - 1)), v - (1 << nb), v)
        off += nb
    return codes


def decode(codes, p: int, exps) -> np.ndarray:
    """Float64 words [(p+1)^2, ncell] = code 2^e_l (NaN for invalid orders)."""
    codes = np.asarray(codes, dtype=np.int64)
    lw = word_order(p)
    ex = np.asarray(exps, dtype=np.int64)
    out = np.empty((nreal(p), codes.shape[0]))
    for k in range(nreal(p)):
        e = ex[lw[k]]
        out[k] = np.nan if e == EXP_INVALID else np.ldexp(codes[:, k].astype(np.float64), int(e))
    return out


# ---------------------------------------------------------------- App. D
def compose(a_real, b_real, p: int) -> np.ndarray:
    """C_l^m = A_l^m + i B_l^m for every -l <= m <= l.

    a_real, b_real: real storage [..., (p+1)^2]; returns complex [..., (p+1)^2]
    indexed l(l+1)+m (full m range, no symmetry)."""
    A = from_real(np.asarray(a_real, dtype=np.float64), p)
    B = from_real(np.asarray(b_real, dtype=np.float64), p)
    C = np.zeros(A.shape[:-1] + (nreal(p),), dtype=np.complex128)
    for l in range(p + 1):
        for m in range(-l, l + 1):
            C[..., ridx(l, m)] = get(A, l, m) + 1j * get(B, l, m)
    return C


def split(C, p: int):
    """App. D: A_l^m and B_l^m (m >= 0) from C_l^m and C_l^{-m}, returned in
    real storage [..., (p+1)^2] each."""
    C = np.asarray(C, dtype=np.complex128)
    a = np.zeros(C.shape[:-1] + (nreal(p),))
    b = np.zeros(C.shape[:-1] + (nreal(p),))
    for l in range(p + 1):
        for m in range(l + 1):
            cp = C[..., ridx(l, m)]
            cm = (-1) ** m * C[..., ridx(l, -m)]
            s, d = cp + cm, cp - cm
            A = 0.5 * s.real + 0.5j * d.imag
            B = 0.5 * s.imag - 0.5j * d.real
            a[..., ridx(l, m)] = A.real
            b[..., ridx(l, m)] = B.real
            if m > 0:
                a[..., ridx(l, -m)] = A.imag
                b[..., ridx(l, -m)] = B.imag
    return a, b


def m2l_full(p, C, rM, rL):
    """eq. M2L for an arbitrary complex coefficient set held over the full m
    range (no conjugate relation assumed): L_l^m = sum_{lam,mu} C_lam^mu
    S_{l+lam}^{-(m+mu)}(r_L - r_M), every -l <= m <= l, indexed l(l+1)+m."""
    d = np.asarray(rL, dtype=np.float64) - np.asarray(rM, dtype=np.float64)
    S = solid_S(2 * p, d[0], d[1], d[2])
    L = np.zeros(nreal(p), dtype=np.complex128)
    for l in range(p + 1):
        for m in range(-l, l + 1):
            acc = 0j
            for lam in range(p + 1):
                for mu in range(-lam, lam + 1):
                    acc += C[ridx(lam, mu)] * get(S, l + lam, -(m + mu))
            L[ridx(l, m)] = acc
    return L


def full_from_tri(X, p: int) -> np.ndarray:
    """Full-m complex array (index l(l+1)+m) of a triangular set with the
    conjugate relation."""
    out = np.zeros(np.shape(X)[:-1] + (nreal(p),), dtype=np.complex128)
    for l in range(p + 1):
        for m in range(-l, l + 1):
            out[..., ridx(l, m)] = get(X, l, m)
    return out


__all__ = ["EXP_INVALID", "order_bits", "word_order", "cell_bits", "cell_words", "auto_exponents",
           "encode", "pack", "unpack", "decode", "compose", "split", "m2l_full", "full_from_tri"]
