"""GPU parity of the multi-charge path (pmmm_far_multi_f32: many charge sets
on one set of positions and one periodic mesh, M2L as a product on the BF16
matrix cores with split operands) against the FP64 oracle run set by set.

Tolerances: PMMM_F32 plans keep three bf16 terms of every M2L operand (all
24 bits of an FP32 value), so the FP32 bound of 1e-6 relative RMS applies.
PMMM_BF16X3 plans keep two terms: each operand keeps 16 bits (relative
error at most 2^-17 after round-to-nearest), the dropped product h1 g1 is
below 2^-16 of |t m|, so every product carries a relative error of a few
2^-16 (~5e-5 worst case); rounding errors of the 49-term sums and of the
frequencies are independent, so the RMS over the mesh is several times
smaller.  The bound used is 5e-5."""
import numpy as np
import pytest

from gpu_helpers import oracle_cfg
from oracle import exact
from oracle import pmmm as opm
from paper_1409_5981_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-6, "bf16x3": 5e-5}


def _run_multi(ps, qs, precision="f32", cutoff=2, plan=None):
    """qs: (n_sets, n) charges; returns numpy dict of [n_sets, n] arrays."""
    import torch
    from paper_1409_5981_amd._lib import Plan
    if plan is None:
        plan = Plan(ps.n_cells, ps.p, "periodic", box=ps.box, cutoff=cutoff, precision=precision)
    dev = "cuda"
    x, y, z = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
               for a in (ps.x, ps.y, ps.z))
    q = torch.from_numpy(np.ascontiguousarray(qs.T, dtype=np.float32)).to(dev)
    phi, gx, gy, gz = plan.far_multi(x, y, z, q)
    torch.cuda.synchronize()
    plan.sync_status()
    out = {"phi": phi.double().cpu().numpy().T,
           "grad": torch.stack([gx, gy, gz], dim=2).double().cpu().numpy().transpose(1, 0, 2)}
    return out, plan


def _check_sets(ps, qs, out, sets, precision, cutoff=2):
    cfg = oracle_cfg(ps, cutoff)
    worst = 0.0
    for s in sets:
        ref = opm.far_field(ps.pos, qs[s].astype(np.float64), cfg)
        eg = exact.rel_rms(out["grad"][s], ref.grad)
        ep = exact.rel_rms(out["phi"][s], ref.phi)
        print(f"n={ps.n_cells} p={ps.p} N={ps.n} set {s} {precision}: "
              f"rel-RMS grad {eg:.3e} phi {ep:.3e}", flush=True)
        worst = max(worst, eg, ep)
        assert eg <= TOL[precision], (s, eg)
        assert ep <= TOL[precision], (s, ep)
    return worst


@pytest.mark.parametrize("n_cells,p,cutoff", [(8, 4, 2), (16, 5, 2), (4, 3, 1)])
def test_multi_small_f32(n_cells, p, cutoff):
    ps, qs = inputs.multi_charge_sets(n=4000, n_sets=8, n_cells=n_cells, p=p, seed=21)
    out, _ = _run_multi(ps, qs, "f32", cutoff=cutoff)
    _check_sets(ps, qs, out, range(8), "f32", cutoff=cutoff)


def test_multi_bf16x3_error_stated():
    """Two-term splits: the measured error is printed and bounded."""
    ps, qs = inputs.multi_charge_sets(n=6000, n_sets=16, n_cells=16, p=6, seed=22)
    out, _ = _run_multi(ps, qs, "bf16x3")
    worst = _check_sets(ps, qs, out, [0, 7, 15], "bf16x3")
    print(f"bf16x3 worst rel-RMS {worst:.3e}")


def test_multi_more_than_one_chunk():
    """70 sets: a full chunk of 64 and a partial one of 6 (a partial set
    tile), against the oracle at both ends of each chunk."""
    ps, qs = inputs.multi_charge_sets(n=2000, n_sets=70, n_cells=8, p=4, seed=23)
    out, _ = _run_multi(ps, qs, "f32")
    _check_sets(ps, qs, out, [0, 37, 63, 64, 69], "f32")


def test_multi_32_mesh_p6():
    """32^3 periodic mesh at p = 6 (the multi-charge workload's mesh and
    order) with a moderate particle count."""
    ps, qs = inputs.multi_charge_sets(n=32768, n_sets=4, n_cells=32, p=6, seed=24)
    out, _ = _run_multi(ps, qs, "f32")
    _check_sets(ps, qs, out, [0, 3], "f32")


def test_multi_matches_single_charge_path():
    """Each set's multi-charge result equals the single-charge FP32 path's
    result for that set (both within FP32 rounding of the oracle)."""
    import torch
    from gpu_helpers import gpu_far
    ps, qs = inputs.multi_charge_sets(n=5000, n_sets=8, n_cells=8, p=5, seed=25)
    out, plan = _run_multi(ps, qs, "f32")
    for s in (0, 5):
        single = inputs.ParticleSet(ps.x, ps.y, ps.z, qs[s].copy(), ps.n_cells, ps.p, "periodic")
        res, _ = gpu_far(single, "f32")
        assert exact.rel_rms(out["grad"][s], res["grad"]) < 1e-6
        assert exact.rel_rms(out["phi"][s], res["phi"]) < 1e-6


def test_multi_charged_sets_and_reuse():
    """Non-neutral charge sets (the per-particle terms of a charged periodic
    system) and a second, smaller call on the same plan."""
    rng = np.random.default_rng(26)
    n = 3000
    x, y, z = (rng.random(n).astype(np.float32) for _ in range(3))
    qs = rng.random((5, n)).astype(np.float32)       # all positive: charged systems
    ps = inputs.ParticleSet(x, y, z, qs[0].copy(), 8, 4, "periodic")
    out, plan = _run_multi(ps, qs, "f32")
    _check_sets(ps, qs, out, range(5), "f32")
    small = ps.subset(np.arange(1000))
    out2, _ = _run_multi(small, qs[:3, :1000].copy(), "f32", plan=plan)
    _check_sets(small, qs[:3, :1000], out2, range(3), "f32")


def test_multi_empty_and_errors():
    import torch
    from paper_1409_5981_amd._lib import PMMM_EINVAL, PMMM_EUNSUPPORTED, Plan, PMMMError
    plan = Plan(8, 3, "periodic")
    e = torch.empty(0, dtype=torch.float32, device="cuda")
    out = plan.far_multi(e, e, e, torch.empty(0, 4, dtype=torch.float32, device="cuda"))
    assert all(o.shape == (0, 4) for o in out)
    open_plan = Plan(8, 3, "open")
    one = torch.full((2,), 0.3, dtype=torch.float32, device="cuda")
    with pytest.raises(PMMMError) as ei:
        open_plan.far_multi(one, one, one, torch.ones(2, 3, device="cuda"))
    assert ei.value.code == PMMM_EUNSUPPORTED
    f64 = Plan(8, 3, "periodic", precision="f64")
    d = one.double()
    with pytest.raises((PMMMError, ValueError)):
        f64.far_multi(d, d, d, torch.ones(2, 3, dtype=torch.float64, device="cuda"))
    assert PMMM_EINVAL == 1


def test_multi_full_size_sampled():
    """The multi-charge workload at full size (2^20 positions, 64 neutral
    +/-1 charge sets, 32^3 mesh, p = 6) in the benchmark's launch
    configuration; FP64 oracle values of 4096 sampled particles for four of
    the sets were written by tests/golden/make_oracle_refs.py."""
    import os
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden",
                               "ref_multi_periodic_n1048576_m32_p6_s64.npz"))
    ps, qs = inputs.multi_charge_sets()
    assert ps.n == int(ref["n"]) and qs.shape[0] == int(ref["n_sets"])
    out, _ = _run_multi(ps, qs, "f32")
    idx = ref["idx"]
    for k, s in enumerate(ref["sets"]):
        eg = exact.rel_rms(out["grad"][s][idx], ref["grad"][k])
        ep = exact.rel_rms(out["phi"][s][idx], ref["phi"][k])
        print(f"multi full size set {s}: sampled rel-RMS grad {eg:.3e} phi {ep:.3e}", flush=True)
        assert eg <= TOL["f32"], (s, eg)
        assert ep <= TOL["f32"], (s, ep)
