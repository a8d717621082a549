"""Pins for the literal mesh pipeline oracle.pmmm (Sec. 2, App. B-C):
FFT convolution against first-principles cell-pair sums, the p = 0 (NGP)
limit, cell-centre exactness, the periodic transfer kernel against Ewald
and brute-force image sums, alpha independence, the Madelung constant,
error decay with p, and structural identities."""
import os
from math import pi, sqrt

import numpy as np
import pytest

from oracle import exact
from oracle import expansions as ex
from oracle import pmmm
from oracle.harmonics import from_real, get, nreal, ridx, solid_S, to_real, tri

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(n, seed, neutral=True):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    q = rng.random(n) - 0.5
    if neutral:
        q -= q.mean()
    return pos, q


def _cell_centres(n, box=1.0):
    i = np.arange(n)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    return (np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1) + 0.5) * (box / n)


def test_open_fft_convolution_equals_cell_pair_m2l():
    """Steps 3-6 on an open 4^3 mesh equal the explicit sum over cell pairs
    of eq. M2L (complex form) for all cells outside the near cube."""
    cfg = pmmm.Config(n=4, p=3, boundary="open", cutoff=1)
    pos, q = _rand(300, 1)
    M, _ = pmmm.p2m_mesh(pos, q, cfg)
    L = pmmm.local_mesh(M, cfg)
    n, h, P = cfg.n, cfg.h, nreal(cfg.p)
    Mc = from_real(M.reshape(P, -1).T, cfg.p)
    cen = _cell_centres(n)
    for I in range(n ** 3):
        acc = np.zeros(Mc.shape[1], dtype=complex)
        iI = np.array([I % n, (I // n) % n, I // n ** 2])
        for J in range(n ** 3):
            iJ = np.array([J % n, (J // n) % n, J // n ** 2])
            if np.max(np.abs(iI - iJ)) <= cfg.cutoff:
                continue
            acc += ex.m2l(cfg.p, Mc[J], cen[J], cen[I])
        np.testing.assert_allclose(L.reshape(P, -1)[:, I], to_real(acc, cfg.p), rtol=1e-11,
                                   atol=1e-11 * np.max(np.abs(L)))


def test_periodic_fft_convolution_equals_cyclic_sum():
    """Steps 4-6 on a periodic 5^3 mesh equal the cyclic real-space sum
    L_i = sum_j T(G_{i-j}) M_j with T the real matrix of eq. realmatrix."""
    cfg = pmmm.Config(n=5, p=2, boundary="periodic", cutoff=2)
    pos, q = _rand(200, 2)
    M, _ = pmmm.p2m_mesh(pos, q, cfg)
    G = pmmm.green_periodic(cfg)
    L = pmmm.local_mesh(M, cfg, pmmm.spectra(G))
    n, p, P = cfg.n, cfg.p, nreal(cfg.p)
    Gc = from_real(np.moveaxis(G, 0, -1), 2 * p)     # [z, y, x, tri] complex
    Mc = from_real(np.moveaxis(M, 0, -1), p)
    ref = np.zeros((n, n, n, P))
    for iz in range(n):
        for iy in range(n):
            for ix in range(n):
                acc = np.zeros(Mc.shape[-1], dtype=complex)
                for jz in range(n):
                    for jy in range(n):
                        for jx in range(n):
                            g = Gc[(iz - jz) % n, (iy - jy) % n, (ix - jx) % n]
                            m = Mc[jz, jy, jx]
                            for l in range(p + 1):
                                for mm in range(l + 1):
                                    acc[tri(l, mm)] += sum(
                                        get(m, lam, mu) * get(g, l + lam, -(mm + mu))
                                        for lam in range(p + 1) for mu in range(-lam, lam + 1))
                ref[iz, iy, ix] = to_real(acc, p)
    np.testing.assert_allclose(np.moveaxis(L, 0, -1), ref, rtol=1e-10, atol=1e-10 * np.max(np.abs(ref)))


def test_p0_is_nearest_grid_point_pm():
    """At p = 0 the far potential of a particle is sum_J Q_J / |c_I - c_J|
    over the cells J outside its near cube (Sec. 2.2, NGP limit)."""
    cfg = pmmm.Config(n=6, p=0, boundary="open", cutoff=2)
    pos, q = _rand(400, 3)
    far = pmmm.far_field(pos, q, cfg)
    I, cen, _, _ = pmmm.cells(pos, cfg)
    lin = pmmm.linear_cell(I, cfg.n)
    Qc = np.bincount(lin, weights=q, minlength=cfg.n ** 3)
    allc = _cell_centres(cfg.n)
    idx3 = np.stack([np.arange(cfg.n ** 3) % cfg.n, (np.arange(cfg.n ** 3) // cfg.n) % cfg.n,
                     np.arange(cfg.n ** 3) // cfg.n ** 2], axis=1)
    for i in range(0, 400, 37):
        far_mask = np.max(np.abs(idx3 - I[i]), axis=1) > cfg.cutoff
        ref = np.sum(Qc[far_mask] / np.linalg.norm(allc[far_mask] - cen[i], axis=1))
        assert abs(far.phi[i] - ref) < 1e-12 * abs(ref)
    assert np.all(far.grad == 0.0)


@pytest.mark.parametrize("p", [1, 4])
def test_open_cell_centres_exact(p):
    """With every particle at its cell centre, the far field equals the exact
    sum over particles outside the near cube for any p."""
    cfg = pmmm.Config(n=6, p=p, boundary="open", cutoff=1)
    cen = _cell_centres(cfg.n)
    rng = np.random.default_rng(4)
    q = rng.random(len(cen)) - 0.5
    far = pmmm.far_field(cen, q, cfg)
    dphi, dg = exact.direct(cen, q)
    nphi, ng = exact.near(cen, q, cfg)
    assert exact.rel_rms(far.phi, dphi - nphi) < 1e-13
    assert exact.rel_rms(far.grad, dg - ng) < 1e-13


@pytest.mark.parametrize("boundary,n", [("open", 4), ("periodic", 5), ("periodic", 8)])
def test_green_spectrum_parity(boundary, n):
    """G(-d) = (-1)^k G(d) for order k on the whole mesh, the half-box
    (Nyquist) offsets of an even periodic mesh included, so the spectra of
    even orders are real and those of odd orders imaginary (to rounding)."""
    cfg = pmmm.Config(n=n, p=3, boundary=boundary, cutoff=2 if boundary == "periodic" else 1)
    G = pmmm.green(cfg)
    nf = G.shape[1]
    mirror = (-np.arange(nf)) % nf
    Gt = pmmm.spectra(G)
    for k in range(2 * cfg.p + 1):
        sl = slice(k * k, (k + 1) * (k + 1))
        Gm = G[sl][:, mirror][:, :, mirror][:, :, :, mirror]
        assert np.max(np.abs(Gm - (-1) ** k * G[sl])) <= 1e-14 * np.max(np.abs(G[sl])), k
        for j in range(-k, k + 1):
            c = Gt[ridx(k, j)]
            big = np.max(np.abs(c))
            bad = np.max(np.abs(c.imag)) if k % 2 == 0 else np.max(np.abs(c.real))
            assert bad <= 1e-14 * big, (k, j)


def test_periodic_green_low_orders_match_ewald():
    """Order 0 of the periodic kernel is the Ewald potential of a unit charge
    (up to the constant pi/(V alpha^2) of the omitted k = 0 term) and order
    1 is its gradient (App. B, below eq. greenPBC); near images subtracted."""
    cfg = pmmm.Config(n=5, p=1, boundary="periodic", cutoff=1)
    G = pmmm.green_periodic(cfg).reshape(nreal(2), -1)
    n, h, a, V = cfg.n, cfg.h, cfg.a, cfg.V
    for lin in [1, 7, 31, 62, 124]:
        ix, iy, iz = lin % n, (lin // n) % n, lin // n ** 2
        d = np.array([ix if ix <= n // 2 else ix - n, iy if iy <= n // 2 else iy - n,
                      iz if iz <= n // 2 else iz - n])
        r = d * h
        pos = np.stack([np.zeros(3), r % 1.0])
        phi, grad = exact.ewald(pos, np.array([1.0, 0.0]), alpha=10.0)
        near = np.max(np.abs(d)) <= cfg.cutoff
        Sd = solid_S(1, *r)
        g00 = phi[1] + pi / (V * a * a) - (Sd[tri(0, 0)].real if near else 0.0)
        assert abs(G[0, lin] - g00) < 1e-12, lin
        gz = grad[1, 2] - (Sd[tri(1, 0)].real if near else 0.0)
        gx = grad[1, 0] - (Sd[tri(1, 1)].real if near else 0.0)
        gy = grad[1, 1] - (Sd[tri(1, 1)].imag if near else 0.0)
        assert abs(G[ridx(1, 0), lin] - gz) < 1e-11
        assert abs(G[ridx(1, 1), lin] - gx) < 1e-11
        assert abs(G[ridx(1, -1), lin] - gy) < 1e-11


def test_periodic_green_high_orders_match_image_sum():
    """For orders >= 5 the lattice sum converges absolutely; a brute-force
    sum over a large cube of images agrees with eq. greenPBC."""
    cfg = pmmm.Config(n=5, p=4, boundary="periodic", cutoff=1)
    G = pmmm.green_periodic(cfg).reshape(nreal(8), -1)
    n, h = cfg.n, cfg.h
    R = 14
    g = np.arange(-R, R + 1)
    NZ, NY, NX = np.meshgrid(g, g, g, indexing="ij")
    imgs = np.stack([NX.ravel(), NY.ravel(), NZ.ravel()], axis=1).astype(float)
    for lin in [3, 40, 88]:
        ix, iy, iz = lin % n, (lin // n) % n, lin // n ** 2
        d = np.array([ix if ix <= n // 2 else ix - n, iy if iy <= n // 2 else iy - n,
                      iz if iz <= n // 2 else iz - n])
        v = d * h + imgs
        if np.max(np.abs(d)) <= cfg.cutoff:
            v = v[np.any(imgs != 0, axis=1)]
        S = solid_S(8, v[:, 0], v[:, 1], v[:, 2]).sum(axis=0)
        ref = to_real(S, 8)
        for k in range(6, 9):
            for j in range(-k, k + 1):
                scale = np.max(np.abs(G[ridx(k, -k):ridx(k, k) + 1, lin]))
                assert abs(G[ridx(k, j), lin] - ref[ridx(k, j)]) < 1e-5 * scale, (lin, k, j)


def test_lower_incomplete_gamma_matches_scipy():
    """The series the periodic kernel uses for the subtracted near image,
    P(l + 1/2, x) = 1 - Q(l + 1/2, x), against scipy's regularised lower
    incomplete gamma over the orders and arguments the kernels reach (and
    beyond), including x where P is far below the rounding of 1 - Q."""
    from scipy.special import gammainc
    for x in [1e-8, 1e-4, 0.01, 0.1, 0.42, 1.0, 1.7, 4.0, 9.0, 25.0, 60.0]:
        P = pmmm.lower_gamma_half(20, x)
        for l in range(21):
            ref = gammainc(l + 0.5, x)
            if ref < 1e-290:
                assert P[l] < 1e-280
                continue
            assert abs(P[l] - ref) <= 1e-13 * ref, (x, l, P[l], ref)


def test_periodic_green_near_image_term():
    """Subtracting the near image (App. B): at an offset of Chebyshev
    distance 2 the c = 2 kernel equals the c = 1 kernel, where that offset
    is not near and nothing is subtracted, minus S(delta h).  The c = 2
    kernel takes the primary image's real-space term as -P S; the reference
    here subtracts S in full, so they agree to the rounding of S."""
    c2 = pmmm.Config(n=8, p=5, boundary="periodic", cutoff=2)
    c1 = pmmm.Config(n=8, p=5, boundary="periodic", cutoff=1)
    G2 = pmmm.green_periodic(c2).reshape(nreal(10), -1)
    G1 = pmmm.green_periodic(c1).reshape(nreal(10), -1)
    n, h = c2.n, c2.h
    for d in [(2, 0, 0), (2, 1, -1), (-2, 2, 2), (1, -2, 0)]:
        ix, iy, iz = (v % n for v in d)
        lin = (iz * n + iy) * n + ix
        S = to_real(solid_S(10, np.array([d[0] * h]), np.array([d[1] * h]),
                            np.array([d[2] * h]))[0], 10)
        ref = G1[:, lin] - S
        assert np.max(np.abs(G2[:, lin] - ref) / (np.abs(S) + np.abs(G1[:, lin]))) < 1e-14, d


def test_periodic_green_alpha_and_images_independent():
    """The split of eq. greenPBC does not depend on alpha or on the image
    radius once converged, apart from the order-0 constant pi/(V alpha^2)."""
    base = pmmm.Config(n=5, p=3, boundary="periodic", cutoff=2)
    G0 = pmmm.green_periodic(base)
    for alpha, images in [(1.3, 6), (1.8, 5), (1.5, 6), (2.2, 6)]:
        cfg = pmmm.Config(n=5, p=3, boundary="periodic", cutoff=2, alpha=alpha, images=images)
        G1 = pmmm.green_periodic(cfg)
        diff = G1 - G0
        # order 0 carries +pi/(V alpha^2) (omitted k = 0 term) and, at d = 0,
        # the smooth self part 2 alpha/sqrt(pi) that the self correction removes
        diff[0] -= pi / (cfg.V * cfg.a ** 2) - pi / (base.V * base.a ** 2)
        diff[0, 0, 0, 0] -= 2 * (cfg.a - base.a) / sqrt(pi)
        assert np.max(np.abs(diff)) < 1e-11 * np.max(np.abs(G0)), (alpha, images)


def test_madelung_rock_salt_any_p():
    """Rock salt, one +/-1 charge at every cell centre: far + near equals
    Ewald exactly for any p (App. B), i.e. Phi_i = -M q_i / h with the
    textbook Madelung constant M, and zero gradient."""
    with open(os.path.join(GOLDEN, "madelung.txt")) as f:
        Mad = float([l for l in f if not l.startswith("#")][0])
    n = 8
    cen = _cell_centres(n)
    I = np.floor(cen * n).astype(int)
    q = (-1.0) ** I.sum(axis=1)
    for p in (1, 3):
        cfg = pmmm.Config(n=n, p=p, boundary="periodic", cutoff=2)
        far = pmmm.far_field(cen, q, cfg)
        nphi, ng = exact.near(cen, q, cfg)
        np.testing.assert_allclose(far.phi + nphi, -Mad * q * n, rtol=1e-11)
        assert np.max(np.abs(far.grad + ng)) < 1e-9


def test_periodic_cell_centres_equal_ewald():
    """Random charges sitting on cell centres: PMMM equals Ewald to lattice
    sum precision for any p (statement below eq. phicorr)."""
    n = 6
    cen = _cell_centres(n)
    rng = np.random.default_rng(12)
    q = rng.random(len(cen)) - 0.5     # charged system: exercises the Q_tot terms
    ephi, eg = exact.ewald(cen, q)
    for p in (1, 2):
        cfg = pmmm.Config(n=n, p=p, boundary="periodic", cutoff=2)
        far = pmmm.far_field(cen, q, cfg)
        nphi, ng = exact.near(cen, q, cfg)
        assert exact.rel_rms(far.phi + nphi, ephi) < 1e-11
        assert exact.rel_rms(far.grad + ng, eg) < 1e-10


def _errest(c):
    s = sqrt(3) / 2
    return s / ((c + 1) - s)


def test_errest_ratios_golden():
    with open(os.path.join(GOLDEN, "errest_ratios.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            c, r = line.split()
            assert abs(_errest(int(c)) - float(r)) < 0.006


@pytest.mark.parametrize("boundary", ["open", "periodic"])
@pytest.mark.parametrize("cutoff", [1, 2])
def test_error_decays_with_p(boundary, cutoff):
    """Sec. 4: the error against the exact reference falls by a ratio as p
    grows, at or below eq. errest, and the larger cutoff converges faster."""
    rng = np.random.default_rng(13)
    pos = rng.random((1500, 3))
    q = rng.random(1500) / 1500
    q -= q.mean()
    ref_phi, ref_g = exact.direct(pos, q) if boundary == "open" else exact.ewald(pos, q)
    errs = []
    for p in range(1, 6):
        cfg = pmmm.Config(n=8, p=p, boundary=boundary, cutoff=cutoff)
        far = pmmm.far_field(pos, q, cfg)
        nphi, ng = exact.near(pos, q, cfg)
        errs.append(exact.rel_rms(far.grad + ng, ref_g))
    ratio = _errest(cutoff)
    for a, b in zip(errs, errs[1:]):
        assert b < a
    # observed per-order ratio stays below the worst-case estimate
    assert (errs[-1] / errs[0]) ** (1 / 4) < ratio
    assert errs[-1] < (5e-4 if cutoff == 1 else 1e-4)


@pytest.mark.parametrize("cutoff", [1, 2])
def test_paper_accuracy_protocol(cutoff):
    """The accuracy test of Sec. 4 (reading: 8^3 open mesh, N = 16384 uniform
    particles, charges U[0, 1/N) minus their mean, p = 1..7): the total field
    (far + near) against the direct sum.  The plotted data is not in the
    text, so the check is eq. errest: the error at order p stays below the
    worst-case ((sqrt 3/2) / (c + 1 - sqrt 3/2))^(p+1), falls at every order
    by at most that ratio on average, and c = 2 beats c = 1 (the smaller
    ratio of the larger cutoff)."""
    from paper_1409_5981_amd import inputs
    ps = inputs.paper_accuracy_set(cutoff=cutoff)
    pos, q = ps.pos, ps.q.astype(np.float64)
    ref_phi, ref_g = exact.direct(pos, q)
    ratio = _errest(cutoff)
    errs, errs_phi = [], []
    for p in range(1, 8):
        cfg = pmmm.Config(n=ps.n_cells, p=p, boundary="open", cutoff=cutoff)
        far = pmmm.far_field(pos, q, cfg)
        nphi, ng = exact.near(pos, q, cfg)
        errs.append(exact.rel_rms(far.grad + ng, ref_g))
        errs_phi.append(exact.rel_rms(far.phi + nphi, ref_phi))
        print(f"c={cutoff} p={p}: grad {errs[-1]:.3e} phi {errs_phi[-1]:.3e} "
              f"(worst case {ratio ** (p + 1):.2e})")
        assert errs[-1] < ratio ** (p + 1) and errs_phi[-1] < ratio ** (p + 1)
    for a, b in zip(errs, errs[1:]):
        assert b < a
    for a, b in zip(errs_phi, errs_phi[1:]):
        assert b < a
    assert (errs[-1] / errs[0]) ** (1 / 6) < ratio
    if cutoff == 2:
        # the same particles with c = 1 at p = 7 (fewer near cells, slower decay)
        c1 = pmmm.Config(n=ps.n_cells, p=7, boundary="open", cutoff=1)
        far1 = pmmm.far_field(pos, q, c1)
        _, ng1 = exact.near(pos, q, c1)
        assert errs[-1] < exact.rel_rms(far1.grad + ng1, ref_g)


def test_energy_identity():
    """sum_i q_i Phi_i^far = sum_I sum_{l,m} (-1)^l L_l^m M_l^m (complex sum
    over all m), from eq. P2M and eq. L2P with R(-r) = (-1)^l R(r)."""
    cfg = pmmm.Config(n=4, p=4, boundary="open", cutoff=1)
    pos, q = _rand(500, 14)
    far = pmmm.far_field(pos, q, cfg)
    P = nreal(cfg.p)
    Mc = from_real(far.M.reshape(P, -1).T, cfg.p)
    Lc = from_real(far.L.reshape(P, -1).T, cfg.p)
    tot = 0j
    for l in range(cfg.p + 1):
        for m in range(-l, l + 1):
            tot += (-1) ** l * np.sum(get(Lc, l, m) * get(Mc, l, m))
    lhs = np.sum(q * far.phi)
    assert abs(tot.imag) < 1e-12 * abs(lhs)
    assert abs(tot.real - lhs) < 1e-12 * abs(lhs)


def test_periodic_whole_cell_translation():
    """Shifting every particle by whole cells (with wrap) leaves each
    particle's far field unchanged."""
    cfg = pmmm.Config(n=6, p=3, boundary="periodic", cutoff=2)
    pos, q = _rand(600, 15)
    a = pmmm.far_field(pos, q, cfg)
    shift = np.array([2, 5, 1]) * cfg.h
    b = pmmm.far_field((pos + shift) % 1.0, q, cfg)
    assert exact.rel_rms(b.phi, a.phi) < 1e-12
    assert exact.rel_rms(b.grad, a.grad) < 1e-12


def test_open_rejects_outside_particles():
    cfg = pmmm.Config(n=4, p=2, boundary="open")
    with pytest.raises(ValueError):
        pmmm.cells(np.array([[0.5, 1.0, 0.5]]), cfg)


# ------------------------------------------------- open meshes of nx x ny x nz cells
def test_open_non_cubic_fft_convolution_equals_cell_pair_m2l():
    """Steps 3-6 on an open 3 x 4 x 5 mesh of cubic cells equal the explicit
    sum over cell pairs of eq. M2L outside the near cube (Sec. 1: the mesh
    may be any product of three integers; App. C padding per axis)."""
    dims = (3, 4, 5)
    cfg = pmmm.Config(n=3, p=2, boundary="open", cutoff=1, box=0.75, shape=dims)
    rng = np.random.default_rng(2)
    pos = rng.random((300, 3)) * cfg.extent
    q = rng.random(300) - 0.5
    M, _ = pmmm.p2m_mesh(pos, q, cfg)
    assert M.shape == (nreal(2), 5, 4, 3)
    L = pmmm.local_mesh(M, cfg)
    P, h = nreal(cfg.p), cfg.h
    Mc = from_real(M.reshape(P, -1).T, cfg.p)
    nx, ny, nz = dims
    idx = np.array([[i % nx, (i // nx) % ny, i // (nx * ny)] for i in range(nx * ny * nz)])
    cen = (idx + 0.5) * h
    for I in range(len(idx)):
        acc = np.zeros(Mc.shape[1], dtype=complex)
        for J in range(len(idx)):
            if np.max(np.abs(idx[I] - idx[J])) <= cfg.cutoff:
                continue
            acc += ex.m2l(cfg.p, Mc[J], cen[J], cen[I])
        np.testing.assert_allclose(L.reshape(P, -1)[:, I], to_real(acc, cfg.p), rtol=1e-11,
                                   atol=1e-11 * np.max(np.abs(L)))


def test_open_non_cubic_equals_its_cubic_embedding():
    """The open far field on an nx x ny x nz mesh equals the far field on the
    cube of 8^3 equal cells holding it (the extra cells are empty and the
    near cubes are the same), and a cubic shape equals the plain n^3 mesh."""
    rng = np.random.default_rng(3)
    h = 1.0 / 8
    cfg = pmmm.Config(n=5, p=4, boundary="open", cutoff=2, box=5 * h, shape=(5, 8, 3))
    pos = rng.random((500, 3)) * cfg.extent
    q = rng.random(500) - 0.5
    a = pmmm.far_field(pos, q, cfg)
    b = pmmm.far_field(pos, q, pmmm.Config(n=8, p=4, boundary="open", cutoff=2, box=1.0))
    assert exact.rel_rms(a.phi, b.phi) < 1e-12 and exact.rel_rms(a.grad, b.grad) < 1e-12
    pos2 = rng.random((500, 3))
    c = pmmm.far_field(pos2, q, pmmm.Config(n=8, p=4, boundary="open", shape=(8, 8, 8)))
    d = pmmm.far_field(pos2, q, pmmm.Config(n=8, p=4, boundary="open"))
    assert np.array_equal(c.phi, d.phi) and np.array_equal(c.grad, d.grad)


def test_near_pairs_match_cell_near_field():
    """The brute-force near field used for non-cubic meshes equals the
    cell-list near field of the C oracle on a cubic mesh."""
    pos, q = _rand(700, 9)
    cfg = pmmm.Config(n=6, p=2, boundary="open", cutoff=2)
    I, _, _, wpos = pmmm.cells(pos, cfg)
    a = exact._near_pairs(wpos, q, I, cfg.cutoff)
    b = exact.near(pos, q, cfg)
    assert exact.rel_rms(a[0], b[0]) < 1e-13 and exact.rel_rms(a[1], b[1]) < 1e-13


def test_open_non_cubic_total_field_matches_direct_sum():
    """Far + near on a 12 x 6 x 9 mesh against the direct sum: the method
    error at p = 6, c = 2 is of the size the cubic meshes give."""
    rng = np.random.default_rng(5)
    cfg = pmmm.Config(n=12, p=6, boundary="open", cutoff=2, box=1.0, shape=(12, 6, 9))
    pos = rng.random((3000, 3)) * cfg.extent
    q = rng.random(3000) - 0.5
    q -= q.mean()
    far = pmmm.far_field(pos, q, cfg)
    nphi, ng = exact.near(pos, q, cfg)
    dphi, dg = exact.direct(pos, q)
    e = exact.rel_rms(far.grad + ng, dg)
    print(f"12x6x9 open mesh, p = 6, c = 2: rel-RMS grad error {e:.2e}")
    assert e < 1e-5
