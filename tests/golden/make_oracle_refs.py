"""Write FP64 oracle references for the large workloads (test
infrastructure).  Calls only the oracle and the seeded input generators.

For each workload the oracle computes the moments from ALL particles and
evaluates the far field on a seeded sample of 4096 particles; the sample
indices and the values are stored in tests/golden/ref_<workload>.npz.

    python tests/golden/make_oracle_refs.py [workload ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import pmmm as opm  # noqa: E402
from paper_1409_5981_amd import inputs  # noqa: E402

SAMPLE = 4096
JOBS = {
    "periodic_n1048576_m32_p7": inputs.periodic_pm1_blocks,
    "open_plummer_n4194304_m64_p6": inputs.plummer_sphere,
}


def make(name: str) -> str:
    t0 = time.time()
    ps = JOBS[name]()
    cfg = opm.Config(n=ps.n_cells, p=ps.p, boundary=ps.boundary, box=ps.box, cutoff=2)
    rng = np.random.Generator(np.random.PCG64(1234))
    idx = np.sort(rng.choice(ps.n, size=SAMPLE, replace=False))
    res = opm.far_field(ps.pos, ps.q.astype(np.float64), cfg, eval_idx=idx)
    path = os.path.join(HERE, f"ref_{name}.npz")
    np.savez_compressed(path, idx=idx, phi=res.phi, grad=res.grad,
                        n=ps.n, n_cells=ps.n_cells, p=ps.p, boundary=ps.boundary)
    print(f"{name}: {time.time() - t0:.0f} s -> {path}", flush=True)
    return path


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(JOBS)):
        make(nm)
