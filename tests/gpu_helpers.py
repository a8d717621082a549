"""Helpers shared by the GPU tests: run the HIP far field through the C ABI
binding on numpy inputs, and convert oracle meshes to the library's cell
units and layouts."""
from __future__ import annotations

import numpy as np

from oracle import pmmm as opm
from oracle.harmonics import nreal


def gpu_far(ps, precision="f32", cutoff=2, near=False, plan=None, alpha=0.0, images=0):
    import torch
    from paper_1409_5981_amd._lib import Plan
    dt = torch.float32 if precision == "f32" else torch.float64
    npdt = np.float32 if precision == "f32" else np.float64
    if plan is None:
        plan = Plan(ps.n_cells, ps.p, ps.boundary, box=ps.box, cutoff=cutoff,
                    precision=precision, alpha=alpha, images=images,
                    shape=getattr(ps, "shape", None))
    dev = "cuda"
    x, y, z, q = (torch.from_numpy(np.ascontiguousarray(a, dtype=npdt)).to(dev)
                  for a in (ps.x, ps.y, ps.z, ps.q))
    phi, gx, gy, gz = plan.far(x, y, z, q)
    out = {"phi": phi, "grad": torch.stack([gx, gy, gz], dim=1)}
    if near:
        nphi, nx, ny, nz = plan.near(x, y, z, q)
        out["near_phi"] = nphi
        out["near_grad"] = torch.stack([nx, ny, nz], dim=1)
    torch.cuda.synchronize()
    res = {k: v.double().cpu().numpy() for k, v in out.items()}
    plan.sync_status()
    return res, plan


# Parity bounds: (relative RMS over all particles, 99th percentile and
# maximum of the per-particle error e_i = |x_i - x_ref,i| / (|x_ref,i| +
# rms_j |x_ref,j|)), x = Phi or grad Phi.  e_i is the particle's own relative
# error, floored at the RMS magnitude so that particles whose field nearly
# cancels do not dominate.  FP32 rounding leaves a few 1e-7 relative RMS;
# the per-particle error of independent roundings stays within about ten
# times that over tens of thousands of particles, so p99 and max get 3x and
# 20x the RMS bound.
BOUNDS = {"f32": (1e-6, 3e-6, 2e-5), "f64": (1e-12, 3e-12, 2e-11)}


def err_stats(x, ref):
    """(relative RMS, p99, max of e_i) as defined above; x and ref are [N]
    (Phi) or [N, 3] (grad Phi)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.ndim == 1:
        d, mag = np.abs(x - ref), np.abs(ref)
    else:
        d, mag = np.linalg.norm(x - ref, axis=1), np.linalg.norm(ref, axis=1)
    rms = float(np.sqrt(np.mean(mag ** 2)))
    e = d / (mag + rms)
    rel = float(np.sqrt(np.sum(d ** 2) / np.sum(mag ** 2)))
    return rel, float(np.percentile(e, 99)), float(np.max(e))


def assert_parity(res, ref_phi, ref_grad, precision, what, bounds=None, idx=None):
    """Assert Phi and grad Phi of a GPU result (dict of numpy arrays) against
    the oracle within the bounds of `precision` (or `bounds`); idx selects a
    sample of the GPU particles that the references belong to."""
    b = bounds if bounds is not None else BOUNDS[precision]
    phi, grad = res["phi"], res["grad"]
    if idx is not None:
        phi, grad = phi[idx], grad[idx]
    out = {}
    for name, x, r in (("grad", grad, ref_grad), ("phi", phi, ref_phi)):
        st = err_stats(x, r)
        out[name] = st
        print(f"{what} {name}: rel-RMS {st[0]:.2e} p99 {st[1]:.2e} max {st[2]:.2e}", flush=True)
        assert st[0] <= b[0] and st[1] <= b[1] and st[2] <= b[2], (what, name, st, b)
    return out


def oracle_cfg(ps, cutoff=2):
    return opm.Config(n=ps.n_cells, p=ps.p, boundary=ps.boundary, box=ps.box, cutoff=cutoff,
                      shape=getattr(ps, "shape", None))


def cell_unit_mesh(mesh, cfg, kind):
    """Physical-unit oracle mesh [P, n, n, n] -> cell units (M_l / h^l or
    L_l h^(l+1))."""
    sm, sl = opm.mesh_scales(cfg)
    s = sm if kind == "M" else sl
    return mesh * s[:, None, None, None]


def folded_green(cfg):
    """Oracle transfer-kernel spectra in cell units, folded like the library:
    [ky, kx, Q, kz] on ky, kz <= nf/2, holding Re (even order) or Im (odd
    order)."""
    Gt = opm.spectra(opm.green(cfg))        # [Q, kz, ky, kx] physical units
    p2 = 2 * cfg.p
    Q = nreal(p2)
    out = np.empty(Gt.shape[2:] + (Q, Gt.shape[1]))
    for k in range(p2 + 1):
        scale = cfg.h ** (k + 1)            # S_k(delta h) h^(k+1) = S_k(delta)
        for j in range(k * k, (k + 1) * (k + 1)):
            v = Gt[j].imag if k % 2 else Gt[j].real
            out[:, :, j, :] = np.transpose(v, (1, 2, 0)) * scale
    nh = Gt.shape[1] // 2 + 1
    out = out[:nh, :, :, :nh]
    if cfg.boundary == "periodic":
        # the library folds the self term -(2 alpha/sqrt(pi)) M_0^0 of the
        # correction procedure into component 0 (cell units: alpha h)
        out[:, :, 0, :] += -2.0 * cfg.a * cfg.h / np.sqrt(np.pi)
    return out
