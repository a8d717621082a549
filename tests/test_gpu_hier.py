"""GPU parity of the two-level hierarchical far field (pmmm_hier_*, Sec. 5.2)
against oracle.hierarchical at the FP32 bounds of gpu_helpers.BOUNDS: the
far field for refinements 2 and 4 and both cutoffs, the total field against
the oracle's far + fine near field and the direct sum, the r = 1 reduction
to the uniform plan, and the box check."""
import numpy as np
import pytest

from gpu_helpers import assert_parity
from oracle import exact
from oracle import hierarchical as ohier
from oracle import pmmm as opm
from paper_1409_5981_amd import inputs

pytestmark = pytest.mark.gpu


def _set(N, seed):
    rng = np.random.default_rng(seed)
    x, y, z = inputs.uniform_positions(rng, N, np.float32)
    q = inputs.neutral_pm1(rng, N, np.float32)
    return np.stack([x, y, z], 1), q


def _run(n, p, r, c, pos, q, mode="far"):
    import torch
    from paper_1409_5981_amd._lib import Hier
    h = Hier(n, p, r, cutoff=c)
    x, y, z = (torch.from_numpy(np.ascontiguousarray(pos[:, a])).cuda() for a in range(3))
    qt = torch.from_numpy(q).cuda()
    phi, gx, gy, gz = getattr(h, mode)(x, y, z, qt)
    torch.cuda.synchronize()
    h.sync_status()
    return {"phi": phi.double().cpu().numpy(), "grad": torch.stack([gx, gy, gz], 1).double().cpu().numpy()}


# p = 3, 4: the fine-level kernel with one row group; 5 to 10: two to seven
# row groups.
@pytest.mark.parametrize("n,p,r,c,N", [(4, 4, 2, 1, 3000), (4, 3, 2, 2, 3000), (4, 3, 4, 1, 4000),
                                       (8, 5, 2, 2, 6000), (4, 6, 2, 1, 3000), (4, 7, 2, 1, 3000),
                                       (4, 8, 2, 1, 2000), (4, 10, 2, 1, 2000)])
def test_hier_far_matches_oracle(n, p, r, c, N):
    print(f"hier coarse {n}^3 p={p} r={r} c={c} N={N}", flush=True)
    pos, q = _set(N, 10 * n + r + c)
    cfg = opm.Config(n=n, p=p, boundary="open", cutoff=c)
    ref_phi, ref_grad = ohier.far_field(pos.astype(np.float64), q.astype(np.float64), cfg, r)
    res = _run(n, p, r, c, pos, q)
    assert_parity(res, ref_phi, ref_grad, "f32", f"hier n={n} r={r} c={c} p={p}")


def test_hier_total_matches_oracle_and_direct_sum():
    n, p, r, c = 4, 5, 2, 2
    pos, q = _set(5000, 7)
    p64, q64 = pos.astype(np.float64), q.astype(np.float64)
    cfg = opm.Config(n=n, p=p, boundary="open", cutoff=c)
    fphi, fgrad = ohier.far_field(p64, q64, cfg, r)
    nphi, ng = exact.near(p64, q64, ohier.fine_config(cfg, r))
    res = _run(n, p, r, c, pos, q, mode="total")
    assert_parity(res, fphi + nphi, fgrad + ng, "f32", "hier total")
    dphi, dg = exact.direct(p64, q64)
    e = exact.rel_rms(res["grad"], dg)
    print(f"hierarchy total field vs direct sum: rel-RMS grad {e:.2e}", flush=True)
    assert e < 1e-4


def test_hier_refine_one_is_the_plan():
    """r = 1 leaves no pair to the fine level: the hierarchy's far field is
    bitwise the plan's."""
    import torch
    from paper_1409_5981_amd._lib import Plan
    pos, q = _set(3000, 3)
    res = _run(8, 4, 1, 2, pos, q)
    plan = Plan(8, 4, "open", cutoff=2)
    x, y, z = (torch.from_numpy(np.ascontiguousarray(pos[:, a])).cuda() for a in range(3))
    phi, gx, gy, gz = plan.far(x, y, z, torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(res["phi"], phi.double().cpu().numpy())
    assert np.array_equal(res["grad"], torch.stack([gx, gy, gz], 1).double().cpu().numpy())


def test_hier_box_check_and_arguments():
    import torch
    from paper_1409_5981_amd._lib import PMMM_EDOMAIN, Hier, PMMMError
    pos, q = _set(500, 5)
    pos[3, 2] = 1.25
    h = Hier(4, 3, 2, cutoff=1)
    x, y, z = (torch.from_numpy(np.ascontiguousarray(pos[:, a])).cuda() for a in range(3))
    h.far(x, y, z, torch.from_numpy(q).cuda())
    with pytest.raises(PMMMError) as e:
        h.sync_status()
    assert e.value.code == PMMM_EDOMAIN
    with pytest.raises(PMMMError):
        Hier(4, 3, 3)                          # refine must be 1, 2, 4 or 8
    with pytest.raises(PMMMError):
        Hier(64, 3, 4)                         # fine mesh above 128 cells per axis


def test_hier_empty_single_and_smaller_second_call():
    """N = 0 returns at once; one particle has no far field (every pair is
    its own); a second, smaller call on the same object matches the oracle
    on its own particles."""
    import torch
    from paper_1409_5981_amd._lib import Hier
    h = Hier(4, 4, 2, cutoff=1)
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    out = h.far(e, e, e, e)
    torch.cuda.synchronize()
    h.sync_status()
    assert all(o.numel() == 0 for o in out)
    pos = np.array([[0.3, 0.6, 0.45]], dtype=np.float32)
    q = np.ones(1, dtype=np.float32)
    x, y, z = (torch.from_numpy(np.ascontiguousarray(pos[:, a])).cuda() for a in range(3))
    phi, gx, gy, gz = h.far(x, y, z, torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    h.sync_status()
    # only FFT round-off of the coarse mesh's masked convolution is left
    scale = 4.0                                  # |q| / (coarse cell edge)
    assert float(torch.stack([phi, gx, gy, gz]).abs().max()) < 1e-6 * scale
    cfg = opm.Config(n=4, p=4, boundary="open", cutoff=1)
    for N, seed in ((3000, 21), (1200, 22)):
        pos, q = _set(N, seed)
        x, y, z = (torch.from_numpy(np.ascontiguousarray(pos[:, a])).cuda() for a in range(3))
        phi, gx, gy, gz = h.far(x, y, z, torch.from_numpy(q).cuda())
        torch.cuda.synchronize()
        h.sync_status()
        ref_phi, ref_grad = ohier.far_field(pos.astype(np.float64), q.astype(np.float64), cfg, 2)
        res = {"phi": phi.double().cpu().numpy(),
               "grad": torch.stack([gx, gy, gz], 1).double().cpu().numpy()}
        assert_parity(res, ref_phi, ref_grad, "f32", f"hier call N={N}")


def test_hier_refine_eight_total_field_vs_direct_sum():
    """r = 8 (fine 32^3 from 4^3, offsets up to 15 cells per axis): the
    oracle's hierarchy takes minutes here, so the total field is checked
    against the direct sum within the method error.  On these particles at
    p = 5, c = 1 the oracle's hierarchy (far + fine near field) is 5.6e-4
    from the direct sum at r = 2 and 8.4e-4 at r = 4, and 7.5e-2 at r = 2
    without its fine level; the bound 5e-3 keeps a wide margin on the first
    and is fifteen times below the last."""
    pos, q = _set(3000, 31)
    res = _run(4, 5, 8, 1, pos, q, mode="total")
    dphi, dg = exact.direct(pos.astype(np.float64), q.astype(np.float64))
    e = exact.rel_rms(res["grad"], dg)
    print(f"hier r=8 total field vs direct sum: rel-RMS grad {e:.2e}", flush=True)
    assert e < 5e-3


def test_hier_stage_profiling():
    """pmmm_hier_set_profiling / _read_profile: the fine level's eq. M2L sums
    are timed as its column stage, the coarse PMMM's stages on level 0, and
    another level is rejected."""
    import torch
    from paper_1409_5981_amd._lib import Hier, PMMMError
    pos, q = _set(2000, 41)
    h = Hier(4, 3, 2, cutoff=1)
    x, y, z = (torch.from_numpy(np.ascontiguousarray(pos[:, a])).cuda() for a in range(3))
    qt = torch.from_numpy(q).cuda()
    h.set_profiling(["bin", "column", "l2p"])
    for _ in range(3):
        h.far(x, y, z, qt)
    torch.cuda.synchronize()
    fine, coarse = h.read_profile(1), h.read_profile(0)
    for prof in (fine, coarse):
        for st in ("bin", "column", "l2p"):
            ms, cnt = prof[st]
            assert cnt == 3 and ms > 0.0
        assert prof["p2m"] == (0.0, 0)
    assert h.read_profile(1)["column"] == (0.0, 0)      # reset by the read before
    h.set_profiling([])
    h.far(x, y, z, qt)
    torch.cuda.synchronize()
    assert h.read_profile(1)["column"] == (0.0, 0)
    with pytest.raises(PMMMError):
        h.read_profile(2)
