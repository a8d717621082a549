#!/usr/bin/env python
"""Benchmark of the PMMM far field on one MI355X.

Workload: periodic boundary, N = 32768 particles uniform in the unit cube
with exactly neutral +/-1 charges, 16^3 cells, p = 5, cutoff c = 2, FP32
(seeded synthetic data, see paper_1409_5981_amd.inputs).  One step is one
pmmm_far_f32 call on inputs already resident in HBM: binning, P2M, forward
FFTs, wave-space M2L (with the periodic corrections), inverse FFTs and L2P.  The
transfer kernel is built once when the plan is created, outside the timed
region (the paper precomputes it at the start of a simulation).

Prints one JSON line (rank 0) with the throughput in particles/s, the
roofline of the dominant kernel (its duration measured with HIP events on
the library's stream over the timed region) and the FP64 CPU oracle timed
on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particles/s, PMMM far field (P2M+FFT M2L+L2P) at rel. RMS force err <=1e-6"
HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
FP32_PEAK = 157.3e12         # FLOP/s, MI355X FP32 vector
FP64_PEAK = 78.6e12
BF16_PEAK = 2.5e15           # FLOP/s, MI355X dense BF16 matrix cores
MULTI_METRIC = ("particle x charge-set evaluations/s, PMMM far field of many charge sets "
                "on one mesh (M2L on BF16 matrix cores, split operands)")


def stage_work(stage, N, n, p, nf, open_bc, tsize=4):
    """Algorithmic HBM bytes and flops of one launch of a stage (each array
    read or written once by the stage, no cache reuse assumed)."""
    P, Q = (p + 1) ** 2, (2 * p + 1) ** 2
    K = n ** 3
    ncol = nf * (nf // 2 + 1)
    F = ncol * nf
    spec = n * ncol                  # complex values per component between kernels
    c = 2 * tsize
    lg = nf.bit_length() - 1
    harm = 4 * (p + 1) * (p + 2)     # regular harmonics, per particle
    if stage == "bin":
        return 4 * tsize * N * 2 + 4 * 4 * N + 3 * 4 * K, 10 * N
    if stage == "p2m":
        return 4 * tsize * N + tsize * (P + 1) * K, (harm + 2 * P + 6) * N
    if stage == "fft_fwd":
        return tsize * P * K + c * P * spec, 5 * P * n * nf * (nf // 2 + 1) * 2 * lg
    if stage == "column":
        nh = nf // 2 + 1
        green = tsize * Q * nh * nh * ((nh + 3) & ~3)      # stored quadrant of the kernel
        return 2 * c * P * spec + green, 4 * P * P * F + 2 * 5 * P * ncol * nf * lg
    if stage == "fft_inv":
        return c * P * spec + tsize * P * K, 5 * P * n * nf * (nf // 2 + 1) * 2 * lg
    if stage == "l2p":
        return tsize * P * K + 4 * tsize * N + 2 * 4 * N + 4 * tsize * N, (harm + 14 * P) * N
    raise KeyError(stage)


def multi_stage_work(stage, N, S, n, p, nprod):
    """Algorithmic HBM bytes, useful FP32 flops and executed matrix-core
    flops of one launch of a multi-charge stage (S charge sets, periodic
    n^3 mesh, FP32 storage)."""
    P, Q = (p + 1) ** 2, (2 * p + 1) ** 2
    PD = p * p
    K = n ** 3
    nh = n // 2 + 1
    ncol = n * nh
    F = ncol * n
    lg = n.bit_length() - 1
    harm = 4 * (p + 1) * (p + 2)
    spec = 8 * S * P * F                    # split-z spectra, complex FP32
    if stage == "bin":
        return 4 * 3 * N + 16 * N + 4 * 4 * N + 3 * 4 * K, 10 * N, 0
    if stage == "p2m":
        return 20 * N + 4 * S * N + 4 * S * (P + 1) * K, (harm + 2 * S * (P + 1)) * N, 0
    if stage == "fft_fwd":
        return 4 * S * (P + 1) * K + spec, 5 * S * P * K * 2 * lg, 0
    if stage == "column":
        rt, ks = -(-P // 16) * 16, -(-P // 32) * 32
        mfma = nprod * 2 * rt * ks * (-(-2 * S // 16) * 16) * F
        return 2 * spec + 4 * Q * nh * nh * ((nh + 3) & ~3), 4 * P * P * S * F, mfma
    if stage == "fft_inv":
        return spec + 4 * S * P * K, 5 * S * P * K * 2 * lg, 0
    if stage == "l2p":
        return 4 * S * P * K + 20 * N + 16 * S * N, (harm + 2 * S * (P + 3 * PD)) * N, 0
    raise KeyError(stage)


def kernel_source_hash():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1409_5981_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(stage, workload, src_hash):
    """HBM traffic of the dominant kernel from committed rocprofv3 counter
    runs (FETCH_SIZE / WRITE_SIZE scaled by the copy-kernel calibration),
    only if the kernel sources are unchanged since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != src_hash:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(ps, target_s, max_n=32768):
    """The FP64 oracle's far field (P2M, FFT M2L, corrections, L2P) on the
    workload's mesh and order, repeated for about target_s seconds.  Large
    workloads use their first max_n particles as the sample.  The plan-time
    transfer spectra are computed once beforehand and not timed."""
    import numpy as np
    from oracle import pmmm as opm
    cfg = opm.Config(n=ps.n_cells, p=ps.p, boundary=ps.boundary, box=ps.box)
    Gt = opm.spectra(opm.green(cfg))
    sub = ps if ps.n <= max_n else ps.subset(np.arange(max_n))
    pos, q = sub.pos, sub.q.astype(np.float64)
    reps, t0 = 0, time.perf_counter()
    while True:
        opm.far_field(pos, q, cfg, Gt=Gt)
        reps += 1
        el = time.perf_counter() - t0
        if el >= target_s or reps >= 1000:
            break
    what = "the same workload" if sub is ps else f"the first {sub.n} particles of the workload"
    return {"value": sub.n * reps / el, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} full far-field passes over {what} (N={sub.n}, "
                      f"{ps.n_cells}^3 cells, p={ps.p}; FP64 numpy, single thread), {el:.1f} s; "
                      "transfer spectra precomputed"}


WORKLOADS = {
    # name: (generator, boundary, precision)
    "periodic_n32768_m16_p5": ("periodic_pm1", "periodic", "f32"),
    "open_n4096_m8_p4_f64": ("open_equal_mass", "open", "f64"),
    "periodic_n1048576_m32_p7": ("periodic_pm1_blocks", "periodic", "f32"),
    "open_plummer_n4194304_m64_p6": ("plummer_sphere", "open", "f32"),
    "multi_periodic_n1048576_m32_p6_s64": ("multi_charge_sets", "periodic", "f32"),
    "batch_periodic_256sys": ("batched_systems", "periodic", "f32"),
}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="periodic_n32768_m16_p5", choices=sorted(WORKLOADS),
                    help="default: the headline workload; the others are the remaining "
                         "single-GPU configurations")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the plan-time launch-shape autotuner (single-system workloads)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB before the "
                         "benchmark (calibration of the HBM traffic counters)")
    ap.add_argument("--split", default="f32", choices=["f32", "bf16x3"],
                    help="multi-charge workload: three-term (f32) or two-term (bf16x3) "
                         "bf16 splits in the M2L product")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the far-field pipeline runs on a single MI355X); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1409_5981_amd import inputs
    from paper_1409_5981_amd._lib import Plan, STAGES

    if args.copy_mb > 0:
        # a plain copy kernel of known size: reads and writes copy_mb MiB once
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    workload = args.workload
    if workload.startswith("multi_"):
        return bench_multi(args, workload)
    if workload.startswith("batch_"):
        return bench_batch(args, workload)
    gen, boundary, prec = WORKLOADS[workload]
    ps = getattr(inputs, gen)()
    N, n, p = ps.n, ps.n_cells, ps.p
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x, y, z, q = (torch.from_numpy(a).to(dev) for a in (ps.x, ps.y, ps.z, ps.q))
    plan = Plan(n, p, boundary, cutoff=2, precision=prec, n_max=N)
    tdt = torch.float32 if prec == "f32" else torch.float64
    out = tuple(torch.empty(N, dtype=tdt, device=dev) for _ in range(4))
    # a dedicated stream (the legacy default stream adds implicit synchronisation)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    torch.cuda.set_stream(stream)
    tuning = None
    if not args.no_autotune:
        # plan-time choice of launch shapes on this workload (not timed)
        tuning = plan.autotune(x, y, z, q, out=out)

    # warm-up; the second half also times every stage to pick the dominant kernel
    half = max(1, args.warmup // 2)
    for i in range(args.warmup):
        if i == half:
            plan.set_profiling(STAGES)
        plan.far(x, y, z, q, out=out)
    torch.cuda.synchronize()
    prof = plan.read_profile(reset=True)
    means = {st: (ms / c if c else 0.0) for st, (ms, c) in prof.items()}
    dominant = max(means, key=means.get)
    print("stage means (ms): " + ", ".join(f"{k}={v*1e3:.1f}us" for k, v in means.items()),
          file=sys.stderr)

    # timed region: only the dominant stage carries events
    plan.set_profiling([dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.far(x, y, z, q, out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.sync_status()
    prof = plan.read_profile(reset=True)
    plan.set_profiling([])
    ms_k, cnt = prof[dominant]
    t_k = ms_k / cnt / 1e3

    nf = 2 * n if boundary == "open" else n
    tsize = 4 if prec == "f32" else 8
    peak_alu = FP32_PEAK if prec == "f32" else FP64_PEAK
    bytes_k, flops_k = stage_work(dominant, N, n, p, nf, boundary == "open", tsize)
    t_hbm, t_alu = bytes_k / HBM_PEAK, flops_k / peak_alu
    if t_hbm >= t_alu:
        roof = {"bound": "hbm", "achieved": bytes_k / t_k / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": flops_k / t_k / 1e12, "peak": peak_alu / 1e12,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = load_traffic(dominant, workload, kernel_source_hash())
    roof["kernel"] = dominant
    roof["kernel_us"] = t_k * 1e6
    roof["algorithmic_bytes"] = bytes_k
    roof["algorithmic_flops"] = flops_k

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(ps, args.cpu_seconds)

    rec = {
        "metric": METRIC,
        "value": N * args.steps / el,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": workload, "boundary": boundary, "n_particles": N,
                   "cells": f"{n}^3", "fft_mesh": f"{nf}^3", "p": p, "cutoff": 2,
                   "tuning": {"column_width": tuning[0], "p2m_lanes": tuning[1]} if tuning else None,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def _roofline(t_k, bytes_k, flops_k, peak_flops, mfma_flops=0):
    t_hbm = bytes_k / HBM_PEAK
    t_alu = flops_k / peak_flops
    t_mfma = mfma_flops / BF16_PEAK
    if t_mfma > max(t_hbm, t_alu):
        roof = {"bound": "mfma", "achieved": mfma_flops / t_k / 1e12, "peak": BF16_PEAK / 1e12,
                "unit": "TFLOP/s"}
    elif t_hbm >= t_alu:
        roof = {"bound": "hbm", "achieved": bytes_k / t_k / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": flops_k / t_k / 1e12, "peak": peak_flops / 1e12,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    return roof


def bench_multi(args, workload):
    """Multi-charge workload: 2^20 uniform positions, 64 neutral +/-1 charge
    sets, periodic 32^3 mesh, p = 6; one step is one pmmm_far_multi_f32 call
    (binning once, then P2M, split-z FFTs, M2L on the matrix cores, inverse
    FFTs and L2P for every set)."""
    import torch
    from paper_1409_5981_amd import inputs
    from paper_1409_5981_amd._lib import Plan, STAGES

    ps, qs = inputs.multi_charge_sets()
    N, S, n, p = ps.n, qs.shape[0], ps.n_cells, ps.p
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x, y, z = (torch.from_numpy(a).to(dev) for a in (ps.x, ps.y, ps.z))
    q = torch.from_numpy(qs.T.copy()).to(dev)
    plan = Plan(n, p, "periodic", cutoff=2, precision=args.split, n_max=N)
    out = tuple(torch.empty(N, S, dtype=torch.float32, device=dev) for _ in range(4))
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    torch.cuda.set_stream(stream)
    warm = max(2, args.warmup)
    half = max(1, warm // 2)
    for i in range(warm):
        if i == half:
            plan.set_profiling(STAGES)
        plan.far_multi(x, y, z, q, out=out)
    torch.cuda.synchronize()
    prof = plan.read_profile(reset=True)
    means = {st: (ms / c if c else 0.0) for st, (ms, c) in prof.items()}
    dominant = max(means, key=means.get)
    print("stage means: " + ", ".join(f"{k}={v*1e3:.1f}us" for k, v in means.items()),
          file=sys.stderr)
    plan.set_profiling([dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.far_multi(x, y, z, q, out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.sync_status()
    prof = plan.read_profile(reset=True)
    plan.set_profiling([])
    ms_k, cnt = prof[dominant]
    t_k = ms_k / cnt / 1e3
    nprod = 6 if args.split == "f32" else 3
    bytes_k, flops_k, mfma_k = multi_stage_work(dominant, N, S, n, p, nprod)
    roof = _roofline(t_k, bytes_k, flops_k, FP32_PEAK, mfma_k)
    roof["traffic"] = load_traffic(dominant, workload, kernel_source_hash())
    roof["kernel"] = dominant
    roof["kernel_us"] = t_k * 1e6
    roof["algorithmic_bytes"] = bytes_k
    roof["algorithmic_flops"] = flops_k
    # matrix-core share of the column stage (mean over the warm-up profile)
    t_col = means.get("column", 0.0) / 1e3
    col_bytes, col_flops, col_mfma = multi_stage_work("column", N, S, n, p, nprod)
    stages = {st: {"us": means[st] * 1e3} for st in STAGES}
    for st in STAGES:
        b_, f_, m_ = multi_stage_work(st, N, S, n, p, nprod)
        if means[st] > 0:
            stages[st]["hbm_frac"] = b_ / (means[st] / 1e3) / HBM_PEAK
            if m_:
                stages[st]["mfma_frac"] = m_ / (means[st] / 1e3) / BF16_PEAK
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(ps, args.cpu_seconds)
        cpu["unit"] = "particle x charge-set evaluations/s"
        cpu["sample"] += "; one charge set per pass"
    rec = {
        "metric": MULTI_METRIC,
        "value": N * S * args.steps / el,
        "unit": "particle x charge-set evaluations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warm,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.split == "f32" else "f32+bf16x3",
        "data": "synthetic",
        "config": {"workload": workload, "boundary": "periodic", "n_particles": N,
                   "charge_sets": S, "cells": f"{n}^3", "fft_mesh": f"{n}^3", "p": p,
                   "cutoff": 2, "m2l_products": nprod, "positions_per_s": N * args.steps / el,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "stages": stages,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


def bench_batch(args, workload):
    """Batched workload: 256 independent periodic systems (N uniform in
    [2048, 65536], meshes 8^3/16^3/32^3, p in {4, 5, 6}, neutral +/-1); one
    step is one pmmm_batch_far_f32 call over all of them (graph replay after
    the second call)."""
    import numpy as np
    import torch
    from paper_1409_5981_amd import inputs
    from paper_1409_5981_amd._lib import Batch

    systems = inputs.batched_systems()
    offs = np.zeros(len(systems) + 1, dtype=np.int64)
    for i, ps in enumerate(systems):
        offs[i + 1] = offs[i] + ps.n
    N = int(offs[-1])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x, y, z, q = (torch.from_numpy(np.concatenate([getattr(ps, a) for ps in systems])).to(dev)
                  for a in ("x", "y", "z", "q"))
    batch = Batch([{"n": ps.n_cells, "p": ps.p, "boundary": "periodic"} for ps in systems])
    out = tuple(torch.empty(N, dtype=torch.float32, device=dev) for _ in range(4))
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    torch.cuda.set_stream(stream)
    for _ in range(max(3, args.warmup)):
        batch.far(offs, x, y, z, q, out=out, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.far(offs, x, y, z, q, out=out, stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    batch.sync_status()
    cpu = None
    if not args.no_cpu_baseline:
        big = max(systems, key=lambda ps: ps.n)
        cpu = cpu_baseline(big, args.cpu_seconds)
        cpu["sample"] += "; the largest system of the batch"
    meshes = {m: sum(1 for ps in systems if ps.n_cells == m) for m in (8, 16, 32)}
    rec = {
        "metric": "particles/s over a batch of independent periodic systems, PMMM far field",
        "value": N * args.steps / el,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(3, args.warmup),
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "systems": len(systems), "n_particles": N,
                   "classes": batch.classes, "meshes": meshes, "cutoff": 2,
                   "parallelism": "single GPU"},
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
