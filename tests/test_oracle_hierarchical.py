"""Pins for oracle.hierarchical (Sec. 5.2): the fine level against eq. M2L
in complex form summed pair by pair, the r = 1 reduction to the coarse
PMMM, and the hierarchy's total field against the direct sum."""
import numpy as np
import pytest

from oracle import exact
from oracle import expansions as ex
from oracle import hierarchical as hier
from oracle import pmmm as opm
from oracle.harmonics import from_real, nreal, to_real


def _set(n, seed):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    q = rng.random(n) - 0.5
    return pos, q - q.mean()


def test_fine_level_equals_pairwise_m2l():
    """Coarse 3^3, r = 2, c = 1: the fine local expansion of every fine cell
    is the sum over fine cells whose coarse cells are within c and whose
    fine cells are not, of the complex single-centre eq. M2L."""
    cfg = opm.Config(n=3, p=2, boundary="open", cutoff=1)
    r = 2
    pos, q = _set(400, 1)
    fcfg = hier.fine_config(cfg, r)
    M, _ = opm.p2m_mesh(pos, q, fcfg)
    L = hier.fine_local_mesh(M, cfg, r)
    nf, P, h = fcfg.n, nreal(cfg.p), fcfg.h
    Mc = from_real(M.reshape(P, -1).T, cfg.p)
    idx = np.array([[i % nf, (i // nf) % nf, i // nf ** 2] for i in range(nf ** 3)])
    cen = (idx + 0.5) * h
    ref = np.zeros((nf ** 3, P))
    for I in range(nf ** 3):
        acc = 0
        for J in range(nf ** 3):
            if np.max(np.abs(idx[I] // r - idx[J] // r)) > cfg.cutoff:
                continue
            if np.max(np.abs(idx[I] - idx[J])) <= cfg.cutoff:
                continue
            acc = acc + ex.m2l(cfg.p, Mc[J], cen[J], cen[I])
        ref[I] = to_real(acc, cfg.p) if not np.isscalar(acc) else 0.0
    np.testing.assert_allclose(L.reshape(P, -1).T, ref, rtol=1e-11,
                               atol=1e-11 * np.abs(ref).max())


def test_refinement_one_is_the_coarse_pmmm():
    """r = 1: the fine cells are the coarse cells, no pair is left to the
    fine level, and the hierarchy is the uniform PMMM."""
    cfg = opm.Config(n=6, p=3, boundary="open", cutoff=1)
    pos, q = _set(600, 2)
    phi, grad = hier.far_field(pos, q, cfg, 1)
    ref = opm.far_field(pos, q, cfg)
    assert np.array_equal(phi, ref.phi) and np.array_equal(grad, ref.grad)


@pytest.mark.parametrize("cutoff", [1, 2])
def test_hierarchy_total_field_matches_direct_sum(cutoff):
    """Coarse 4^3 refined by 2: far field of the hierarchy + the fine near
    field against the direct sum, an error that falls with p and stays of
    the size of the uniform fine mesh's."""
    pos, q = _set(2000, 3)
    dphi, dg = exact.direct(pos, q)
    errs = []
    for p in (2, 4, 6):
        cfg = opm.Config(n=4, p=p, boundary="open", cutoff=cutoff)
        phi, grad = hier.far_field(pos, q, cfg, 2)
        nphi, ng = exact.near(pos, q, hier.fine_config(cfg, 2))
        errs.append(exact.rel_rms(grad + ng, dg))
    uni = opm.far_field(pos, q, hier.fine_config(opm.Config(n=4, p=6, boundary="open",
                                                            cutoff=cutoff), 2))
    nphi, ng = exact.near(pos, q, hier.fine_config(opm.Config(n=4, p=6, boundary="open",
                                                              cutoff=cutoff), 2))
    e_uni = exact.rel_rms(uni.grad + ng, dg)
    print(f"c = {cutoff}: hierarchy grad errors {['%.2e' % e for e in errs]}, uniform 8^3 p = 6 {e_uni:.2e}")
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 5 * e_uni + 1e-6
