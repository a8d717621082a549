"""The allocation-free far field (pmmm_far_f32_noalloc, through the C ABI)
against pmmm_far_f32 on the same inputs, to the FP32 parity bounds: two
calls in a row on one plan, the second with a smaller input, at both ends
of the size range (the sorted-order result path at the full static
capacity); the call allocates no device memory; sizes beyond the static
scratch are refused before anything runs."""
import numpy as np
import pytest

from gpu_helpers import assert_parity
from paper_1409_5981_amd import inputs

pytestmark = pytest.mark.gpu


def _particles(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    x, y, z = (rng.random(n).astype(np.float32) for _ in range(3))
    q = inputs.neutral_pm1(rng, n, np.float32)
    return [torch.from_numpy(a).cuda() for a in (x, y, z, q)]


def _np(out):
    import torch
    return {"phi": out[0].double().cpu().numpy(),
            "grad": torch.stack(list(out[1:]), 1).double().cpu().numpy()}


@pytest.mark.parametrize("n_cells,p,boundary", [(16, 5, "periodic"), (16, 4, "open")])
def test_noalloc_matches_far_f32(n_cells, p, boundary):
    import torch
    from paper_1409_5981_amd._lib import PMMM_NOALLOC_MAX_N, Plan
    ref_plan = Plan(n_cells, p, boundary)
    plan = Plan(n_cells, p, boundary)          # no particle capacity of its own
    for k, n in enumerate((PMMM_NOALLOC_MAX_N, 40000)):
        t = _particles(n, 70 + k)
        ref = _np(ref_plan.far(*t))
        out = tuple(torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(4))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        got = plan.far_noalloc(*t, out=out)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        plan.sync_status()
        assert free0 - free1 < (1 << 20), (free0, free1)
        assert_parity(_np(got), ref["phi"], ref["grad"], "f32",
                      f"noalloc vs far_f32 {boundary} n={n_cells} p={p} N={n} call {k + 1}")


def test_noalloc_refuses_oversize_and_fp64():
    import torch
    from paper_1409_5981_amd._lib import PMMM_EINVAL, PMMM_NOALLOC_MAX_N, Plan, PMMMError
    plan = Plan(8, 3, "periodic")
    n = PMMM_NOALLOC_MAX_N + 1
    t = [torch.full((n,), 0.5, dtype=torch.float32, device="cuda") for _ in range(4)]
    out = tuple(torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(4))
    with pytest.raises(PMMMError) as ei:
        plan.far_noalloc(*t, out=out)
    assert ei.value.code == PMMM_EINVAL
    f64 = Plan(8, 3, "periodic", precision="f64")
    d = [torch.full((4,), 0.5, dtype=torch.float64, device="cuda") for _ in range(4)]
    with pytest.raises((PMMMError, ValueError)):
        f64.far_noalloc(*d, out=tuple(torch.empty(4, dtype=torch.float64, device="cuda")
                                      for _ in range(4)))
