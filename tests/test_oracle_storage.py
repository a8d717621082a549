"""Pins for oracle.storage: the per-order fixed point of Sec. 5.3 (the bit
counts the paper prints, an independent big-integer reading of the bit
stream, hand-computed codes, the rounding bound) and the complex composition
of App. D (checked against eq. M2L applied to each set apart)."""
import numpy as np
import pytest

from oracle import expansions as ex
from oracle.harmonics import nreal, ridx, to_real
from oracle.storage import (EXP_INVALID, auto_exponents, cell_bits, cell_words, compose, decode,
                            encode, full_from_tri, m2l_full, order_bits, pack, split, unpack)


def test_bits_per_cell_printed_values():
    """Sec. 5.3: 24 bits at order 0 and 612 bits per cell at p = 7; the
    footnote's closed form 3 (p+1)(p+2)(2p+3)/6 for every order."""
    assert order_bits(7)[0] == 24
    assert order_bits(7)[7] == 3
    assert cell_bits(7) == 612
    for p in range(11):
        assert cell_bits(p) == 3 * (p + 1) * (p + 2) * (2 * p + 3) // 6
        assert cell_words(p) * 32 >= cell_bits(p) > (cell_words(p) - 1) * 32


def _random_codes(p, ncell, rng):
    b = order_bits(p)
    cols = []
    for l in range(p + 1):
        lim = 2 ** (b[l] - 1) - 1
        for _ in range(2 * l + 1):
            cols.append(rng.integers(-lim, lim + 1, ncell))
    codes = np.stack(cols, axis=1)
    codes[0, :] = [2 ** (b[l] - 1) - 1 for l in range(p + 1) for _ in range(2 * l + 1)]
    codes[1, :] = [-(2 ** (b[l] - 1) - 1) for l in range(p + 1) for _ in range(2 * l + 1)]
    return codes


@pytest.mark.parametrize("p", [0, 1, 3, 6, 7, 10])
def test_bit_stream_against_big_integers(p):
    """Each record, read as one little-endian integer of 32 * words bits,
    yields the codes as consecutive b_l-bit two's-complement fields in
    real-storage order, followed by zero padding."""
    rng = np.random.default_rng(p)
    codes = _random_codes(p, 40, rng)
    rec = pack(codes, p)
    assert rec.shape == (40, cell_words(p)) and rec.dtype == np.uint32
    b = order_bits(p)
    for c in range(40):
        big = sum(int(w) << (32 * i) for i, w in enumerate(rec[c]))
        for l in range(p + 1):
            for m in range(-l, l + 1):
                field = big & ((1 << b[l]) - 1)
                big >>= b[l]
                val = field - (1 << b[l]) if field >> (b[l] - 1) else field
                assert val == codes[c, ridx(l, m)]
        assert big == 0
    np.testing.assert_array_equal(unpack(rec, p), codes)


def test_hand_computed_codes():
    """p = 7: order 0 has 24 bits, order 1 has 21.  Max |word| 1.0 at order 0
    gives the unit 2^-22; max 3.0 at order 1 gives the unit 2^-18 and halves
    round to even; a largest word just below 1.0 would round to 2^23 under
    the unit 2^-23, so the unit stays 2^-22; under a caller's unit 2^-23 it
    is clamped to 2^23 - 1."""
    p = 7
    coef = np.zeros((nreal(p), 4), dtype=np.float32)
    coef[0] = [1.0, -1.0, 0.25, 0.0]
    coef[1] = [3.0, 2.0 ** -19, 3 * 2.0 ** -19, -5 * 2.0 ** -19]
    e = auto_exponents(coef, p)
    assert e[0] == -22 and e[1] == -18 and all(e[2:] == 0)
    codes = encode(coef, p, e)
    assert list(codes[:, 0]) == [2 ** 22, -(2 ** 22), 2 ** 20, 0]
    assert list(codes[:, 1]) == [3 * 2 ** 18, 0, 2, -2]
    coef[0, 0] = np.nextafter(np.float32(1.0), np.float32(0.0))
    coef[0, 1] = -0.5
    e = auto_exponents(coef, p)
    assert e[0] == -22
    assert encode(coef, p, e)[0, 0] == 2 ** 22
    coef[0, 2] = 2.0 ** -24
    assert encode(coef, p, auto_exponents(coef, p))[2, 0] == 0     # 1/4 of the unit
    e[0] = -23
    assert encode(coef, p, e)[0, 0] == 2 ** 23 - 1


@pytest.mark.parametrize("p", [2, 6, 10])
def test_round_trip_within_half_a_unit(p):
    """|decode(encode(x)) - x| <= 2^(e_l - 1) for every word, the largest word
    of each order fills the top bit of its range, and words that are
    multiples of the unit come back exactly."""
    rng = np.random.default_rng(10 + p)
    ncell = 300
    scale = np.array([4.0 ** -l for l in range(p + 1) for _ in range(2 * l + 1)])
    coef = (rng.standard_normal((nreal(p), ncell)) * scale[:, None]).astype(np.float32)
    e = auto_exponents(coef, p)
    codes = encode(coef, p, e)
    back = decode(unpack(pack(codes, p), p), p, e)
    lw = np.array([l for l in range(p + 1) for _ in range(2 * l + 1)])
    unit = np.ldexp(1.0, e[lw])
    assert np.all(np.abs(back - coef) <= 0.5 * unit[:, None])
    b = order_bits(p)
    for l in range(p + 1):
        top = np.abs(codes[:, lw == l]).max()
        assert 2 ** (b[l] - 2) <= top <= 2 ** (b[l] - 1) - 1
    exact = (np.rint(coef / unit[:, None]) * unit[:, None]).astype(np.float32)
    ce = encode(exact, p, e)
    np.testing.assert_array_equal(decode(ce, p, e), exact.astype(np.float64))


def test_zero_and_non_finite_orders():
    p = 3
    coef = np.ones((nreal(p), 5), dtype=np.float32)
    coef[1:4] = 0.0                      # order 1 all zero
    coef[4, 2] = np.inf                  # order 2 holds a non-finite word
    e = auto_exponents(coef, p)
    assert e[1] == 0 and e[2] == EXP_INVALID and e[0] == 1 - 11
    codes = encode(coef, p, e)
    assert np.all(codes[:, 1:4] == 0) and np.all(codes[:, 4:9] == 0)
    d = decode(codes, p, e)
    assert np.all(np.isnan(d[4:9])) and np.all(d[0] == 1.0)
    # caller-fixed units: saturation and NaN
    e2 = np.array([-20, -10, -10, -10])
    c2 = coef.copy()
    c2[0, 0] = 1e30
    c2[0, 1] = -np.inf
    c2[0, 2] = np.nan
    codes2 = encode(c2, p, e2)
    lim0 = 2 ** (order_bits(p)[0] - 1) - 1
    assert list(codes2[:3, 0]) == [lim0, -lim0, 0]


def _sets(p, rng, ncell=3):
    """Genuine multipole sets: eq. P2M of random particles about a centre."""
    out = []
    for _ in range(ncell):
        pos = rng.random((7, 3)) - 0.5
        q = rng.standard_normal(7)
        out.append(ex.p2m(p, np.zeros(3), pos, q))
    return np.stack(out)


def test_compose_matches_printed_parts():
    """App. D: C_l^m = (Re A - Im B) + i (Re B + Im A) and
    (-1)^m C_l^{-m} = (Re A + Im B) + i (Re B - Im A)."""
    p = 4
    rng = np.random.default_rng(5)
    A, B = _sets(p, rng), _sets(p, rng)
    C = compose(to_real(A, p), to_real(B, p), p)
    from oracle.harmonics import tri
    for l in range(p + 1):
        for m in range(l + 1):
            a, b = A[:, tri(l, m)], B[:, tri(l, m)]
            np.testing.assert_allclose(C[:, ridx(l, m)], (a.real - b.imag) + 1j * (b.real + a.imag),
                                       rtol=0, atol=1e-15)
            np.testing.assert_allclose((-1) ** m * C[:, ridx(l, -m)],
                                       (a.real + b.imag) + 1j * (b.real - a.imag), rtol=0, atol=1e-15)


def test_split_inverts_compose():
    p = 6
    rng = np.random.default_rng(6)
    a = rng.standard_normal((11, nreal(p)))
    b = rng.standard_normal((11, nreal(p)))
    a2, b2 = split(compose(a, b, p), p)
    np.testing.assert_allclose(a2, a, rtol=0, atol=1e-15)
    np.testing.assert_allclose(b2, b, rtol=0, atol=1e-15)


def test_composite_m2l_is_the_two_m2ls():
    """App. D linearity: the full-range M2L of C = A + iB, split, equals eq.
    M2L applied to A and to B apart (the single-centre oracle); on a set with
    the conjugate relation the full-range M2L is that M2L itself."""
    p = 4
    rng = np.random.default_rng(7)
    A, B = _sets(p, rng, 1)[0], _sets(p, rng, 1)[0]
    rM, rL = np.zeros(3), np.array([2.5, -1.0, 3.0])
    LA, LB = ex.m2l(p, A, rM, rL), ex.m2l(p, B, rM, rL)
    np.testing.assert_allclose(m2l_full(p, full_from_tri(A, p), rM, rL), full_from_tri(LA, p),
                               rtol=1e-13, atol=1e-16)
    C = compose(to_real(A, p), to_real(B, p), p)
    la, lb = split(m2l_full(p, C, rM, rL), p)
    np.testing.assert_allclose(la, to_real(LA, p), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(lb, to_real(LB, p), rtol=1e-12, atol=1e-15)
    # a sign slip in the split would mix the two sets: check they differ
    assert np.abs(to_real(LA, p) - to_real(LB, p)).max() > 1e-3


def test_far_field_change_within_the_rounding_bound():
    """Local-expansion mesh of an open far field (p = 7, 612-bit records, cell
    units): after the round trip, every particle's potential moves by no
    more than the sum over words of half a unit times that word's weight in
    eq. L2P (|R_l^0| for m = 0, 2 |Re R_l^m| or 2 |Im R_l^m| otherwise).
    The relative RMS change of the gradient is printed: the per-order bit
    budget of Sec. 5.3 trades about 3e-4 of the gradient for a 3.3x smaller
    mesh at p = 7."""
    from oracle import exact
    from oracle import pmmm as opm
    from oracle.harmonics import get, solid_R
    p, n = 7, 8
    cfg = opm.Config(n=n, p=p, boundary="open")
    rng = np.random.default_rng(1)
    pos = rng.random((4096, 3))
    q = np.where(np.arange(4096) % 2 == 0, 1.0, -1.0) / 4096
    r = opm.far_field(pos, q, cfg)
    _, sl = opm.mesh_scales(cfg)
    Lc = (r.L.reshape(nreal(p), -1) * sl[:, None]).astype(np.float32)
    e = auto_exponents(Lc, p)
    Lq = (decode(encode(Lc, p, e), p, e) / sl[:, None]).reshape(r.L.shape)
    phi, grad = opm.l2p(Lq, pos, cfg)
    _, _, rel, _ = opm.cells(pos, cfg)
    R = solid_R(p, rel[:, 0], rel[:, 1], rel[:, 2])
    bound = np.zeros(len(pos))
    for l in range(p + 1):
        half = 0.5 * np.ldexp(1.0, int(e[l])) / cfg.h ** (l + 1)
        w = np.abs(get(R, l, 0).real)
        for m in range(1, l + 1):
            w = w + 2 * (np.abs(get(R, l, m).real) + np.abs(get(R, l, m).imag))
        bound += half * w
    assert np.all(np.abs(phi - r.phi) <= bound * (1 + 1e-9))
    g = exact.rel_rms(grad, r.grad)
    print(f"612-bit records at p = 7: rel-RMS change of Phi {exact.rel_rms(phi, r.phi):.2e}, grad {g:.2e}")
    assert 1e-6 < g < 3e-3
