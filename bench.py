#!/usr/bin/env python
"""Benchmark of the PMMM far field on one MI355X.

Default workload (the largest single-GPU configuration): open boundary,
N = 2^22 equal-mass particles from a Plummer sphere (scale radius 0.05,
truncated to the unit cube), 64^3 cells (128^3 zero-padded FFT), p = 6,
cutoff c = 2, FP32 (seeded synthetic data, see paper_1409_5981_amd.inputs).
One step is one pmmm_far_f32 call on inputs already resident in HBM:
binning, P2M, forward FFTs, wave-space M2L, inverse FFTs and L2P.  The
transfer kernel is built once when the plan is created, outside the timed
region (the paper precomputes it at the start of a simulation).

Prints one JSON line with the throughput in particles/s, the error of the
timed result against the stored FP64 oracle sample (the line is marked
failed, exit status 3, above the FP32 bound of 1e-6), the roofline of the
dominant kernel on its algorithmic bytes (its duration measured with HIP
events on the library's stream over the timed region), the roofline of the
whole step, and the FP64 CPU oracle timed on a bounded sample on this
host in a child process running beside the GPU measurement.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particles/s, PMMM far field (P2M+FFT M2L+L2P) at rel. RMS force err <=1e-6"
HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
FP32_PEAK = 157.3e12         # FLOP/s, MI355X FP32 vector
# FP32 operations of one near-field pair (k_near): the offset (4), r^2 (5),
# rsq (1), q/r and the potential sum (2), 1/r^3 (2), three gradient FMAs (6)
NEAR_FLOPS_PER_PAIR = 20
FP64_PEAK = 78.6e12
BF16_PEAK = 2.5e15           # FLOP/s, MI355X dense BF16 matrix cores
MULTI_METRIC = ("particle x charge-set evaluations/s, PMMM far field of many charge sets "
                "on one mesh (M2L on BF16 matrix cores, split operands)")
ERR_BOUND = {"f32": 1e-6, "f64": 1e-12}
DEFAULT_WORKLOAD = "open_plummer_n4194304_m64_p6"


def algorithmic_work(stage, N, n, p, nf, tsize=4):
    """Algorithmic HBM bytes and flops of one stage: what the method itself
    must move, each array read or written once, no transfer-kernel symmetry
    compression, stages unfused (F = nf^2 (nf/2+1) half-spectrum
    frequencies, K = n^3 cells, P = (p+1)^2, Q = (2p+1)^2).  The library's
    launches map onto the stages one to one: binning, P2M, the forward
    plane FFTs, the column kernel (wave-space M2L; its z transforms are
    counted with the FFT stages), the inverse plane FFTs and L2P."""
    t = tsize
    P, Q, K = (p + 1) ** 2, (2 * p + 1) ** 2, n ** 3
    F = nf * nf * (nf // 2 + 1)
    lg = round(3 * math.log2(nf))                # log2(nf^3)
    harm = 4 * (p + 1) * (p + 2)
    fft = 5 * P * nf ** 3 * lg // 2              # one direction, real-to-complex
    if stage == "bin":
        return 8 * t * N + 4 * N + 8 * K, 10 * N
    if stage == "p2m":
        return 4 * t * N + t * P * K, (harm + 2 * P + 6 * p) * N
    if stage == "fft_fwd":
        return t * P * K + 2 * t * P * F, fft
    if stage == "column":
        return 4 * t * P * F + t * Q * F, 4 * P * P * F
    if stage == "fft_inv":
        return 2 * t * P * F + t * P * K, fft
    if stage == "l2p":
        return t * P * K + 7 * t * N, (harm + 14 * P) * N
    if stage == "near":
        return 8 * t * N, 0
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
        return 2 * spec + 4 * Q * F, 4 * P * P * S * F, mfma
    if stage == "fft_inv":
        return spec + 4 * S * P * K, 5 * S * P * K * 2 * lg, 0
    if stage == "l2p":
        return 4 * S * P * K + 20 * N + 16 * S * N, (harm + 2 * S * (P + 3 * PD)) * N, 0
    raise KeyError(stage)


# Sources that build each stage's kernels (a traffic record stays valid while
# they are unchanged); stages not listed hash every kernel source.
STAGE_SOURCES = {
    "column": ["pmmm_column.h", "pmmm_column_inst.hip", "pmmm_internal.h"],
}


def kernel_source_hash(stage=None):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1409_5981_amd", "csrc")
    for f in STAGE_SOURCES.get(stage) or sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(stage, workload, src_hash, form=None):
    """HBM traffic of the dominant kernel from committed rocprofv3 counter
    runs (FETCH_SIZE / WRITE_SIZE scaled by the copy-kernel calibration),
    only if the kernel sources are unchanged since the counters were taken.
    A record may hold one figure per kernel form (the column stage's forms);
    `form` picks it, the record's default form when None or "default"."""
    path = os.path.join(ROOT, "profiles", f"traffic_{stage}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != src_hash:
        return None
    forms = rec.get("forms")
    if forms:
        key = form if form not in (None, "default") else rec.get("default_form")
        return forms.get(key, {}).get("bytes_per_launch")
    return rec.get("bytes_per_launch")


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


def host_cpu():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


# ------------------------------------------------------------ CPU baseline
def cpu_baseline_child(workload, n_sample):
    """Runs in a child process.  The FP64 oracle's far field on the
    workload, timed stage by stage: its particle stages (binning and P2M,
    L2P) on a random sample of n_sample particles, scaled linearly to N, and
    its mesh stage (forward FFTs, wave-space M2L, inverse FFTs) once on the
    full mesh; the transfer spectra are computed beforehand and not timed.
    Prints one JSON object."""
    import numpy as np
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import pmmm as opm
    from paper_1409_5981_amd import inputs
    ps = inputs.make_workload(workload)
    cfg = opm.Config(n=ps.n_cells, p=ps.p, boundary=ps.boundary, box=ps.box, shape=ps.shape)
    t0 = time.perf_counter()
    Gt = opm.spectra(opm.green(cfg))
    t_green = time.perf_counter() - t0
    rng = np.random.Generator(np.random.PCG64(99))
    ns = min(n_sample, ps.n)
    idx = np.sort(rng.choice(ps.n, size=ns, replace=False))
    pos, q = ps.pos[idx], ps.q[idx].astype(np.float64)
    t0 = time.perf_counter()
    M, qr2 = opm.p2m_mesh(pos, q, cfg)
    t_p2m = time.perf_counter() - t0
    t0 = time.perf_counter()
    L = opm.local_mesh(M, cfg, Gt)
    if cfg.boundary == "periodic":
        L, _ = opm.periodic_corrections(L, M, qr2, cfg)
    t_mesh = time.perf_counter() - t0
    t0 = time.perf_counter()
    opm.l2p(L, pos, cfg)
    t_l2p = time.perf_counter() - t0
    scale = ps.n / ns
    t_full = (t_p2m + t_l2p) * scale + t_mesh
    model, ncpu = host_cpu()
    if t_full < 5.0:
        # small workload: whole far-field calls on all particles, repeated
        pos, q = ps.pos, ps.q.astype(np.float64)
        reps, t0 = 0, time.perf_counter()
        while True:
            opm.far_field(pos, q, cfg, Gt=Gt)
            reps += 1
            el = time.perf_counter() - t0
            if el >= 10.0 or reps >= 1000:
                break
        print(json.dumps({
            "value": ps.n * reps / el, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 oracle (numpy, single thread) on this host ({model}, {ncpu} logical "
                       f"CPUs): {reps} whole far-field calls on all {ps.n} particles, {el:.1f} s; "
                       f"transfer spectra precomputed ({t_green:.1f} s, not timed)"),
        }), flush=True)
        return
    print(json.dumps({
        "value": ps.n / t_full, "unit": "particles/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 oracle (numpy, single thread) on this host ({model}, {ncpu} logical CPUs): "
                   f"binning+P2M and L2P on {ns} randomly sampled particles of the workload "
                   f"({t_p2m:.1f} s + {t_l2p:.1f} s, scaled x{scale:.0f} to N={ps.n}), FFTs + "
                   f"wave-space M2L + inverse FFTs once on the full "
                   f"{'x'.join(str(2 * d if cfg.boundary == 'open' else d) for d in cfg.dims)} mesh "
                   f"({t_mesh:.1f} s); estimated {t_full:.1f} s per far-field call; "
                   f"transfer spectra precomputed ({t_green:.1f} s, not timed)"),
        "stage_seconds": {"p2m_sample": t_p2m, "mesh": t_mesh, "l2p_sample": t_l2p,
                          "green_untimed": t_green},
    }), flush=True)


def start_cpu_baseline(workload, n_sample):
    code = (f"import sys; sys.path.insert(0, {ROOT!r}); import bench; "
            f"bench.cpu_baseline_child({workload!r}, {int(n_sample)})")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    return subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE,
                            stderr=subprocess.PIPE, text=True, env=env, cwd=ROOT)


def finish_cpu_baseline(proc, timeout=600):
    try:
        out, err = proc.communicate(timeout=timeout)
    except subprocess.TimeoutExpired:
        proc.kill()
        return None
    if proc.returncode != 0:
        print("cpu baseline failed: " + err[-2000:], file=sys.stderr)
        return None
    rec = json.loads(out.strip().splitlines()[-1])
    rec.pop("stage_seconds", None)
    return rec


# ------------------------------------------------------------------- errors
def golden_error(workload, outs, precision):
    """Error of the GPU result against the stored FP64 oracle sample of the
    workload (written by tests/golden/make_oracle_refs.py): relative RMS and
    the maximum per-particle error |x - x_ref| / (|x_ref| + rms |x_ref|)."""
    import numpy as np
    import torch
    path = os.path.join(ROOT, "tests", "golden", f"ref_{workload}.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    idx = torch.from_numpy(ref["idx"]).to(outs[0].device)
    phi = outs[0][idx].double().cpu().numpy()
    grad = torch.stack([o[idx] for o in outs[1:]], 1).double().cpu().numpy()
    res = {}
    for name, x, r in (("grad", grad, ref["grad"]), ("phi", phi, ref["phi"])):
        d = np.abs(x - r) if r.ndim == 1 else np.linalg.norm(x - r, axis=1)
        mag = np.abs(r) if r.ndim == 1 else np.linalg.norm(r, axis=1)
        rms = float(np.sqrt(np.mean(mag ** 2)))
        res[f"rel_rms_{name}"] = float(np.sqrt(np.sum(d ** 2) / np.sum(mag ** 2)))
        res[f"max_{name}"] = float(np.max(d / (mag + rms)))
    res["sample"] = int(len(ref["idx"]))
    res["bound"] = ERR_BOUND[precision]
    res["ok"] = bool(res["rel_rms_grad"] <= res["bound"] and res["rel_rms_phi"] <= res["bound"])
    return res


WORKLOADS = {
    # name: (boundary, precision)
    "open_plummer_n4194304_m64_p6": ("open", "f32"),
    "periodic_n32768_m16_p5": ("periodic", "f32"),
    "open_n4096_m8_p4_f64": ("open", "f64"),
    "periodic_n1048576_m32_p7": ("periodic", "f32"),
    "open_n2097152_m48x40x32_p6": ("open", "f32"),
    "periodic_n1048576_m24_p6": ("periodic", "f32"),
    "multi_periodic_n1048576_m32_p6_s64": ("periodic", "f32"),
    "batch_periodic_256sys": ("periodic", "f32"),
    "hier_open_n1048576_m16r2_p4_c1": ("open", "f32"),
    "hier_total_plummer_n4194304_m64r2_p4_c1": ("open", "f32"),
}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=1 << 16,
                    help="particles of the oracle's particle stages in the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graphs", type=int, default=0,
                    help="1: replay the repeated far-field call as a HIP graph (pmmm_plan_set_graphs); "
                         "stage profiling makes the calls eager again, so only the step time changes")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS),
                    help="default: the largest single-GPU configuration; the others are the "
                         "remaining configurations")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the plan-time launch-shape autotuner (single-system workloads)")
    ap.add_argument("--column-kernel", default=None,
                    choices=["tile", "stream1", "stream2", "stream4"],
                    help="fix the column-kernel form instead of tuning it")
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

    workload = args.workload
    single = not workload.startswith(("multi_", "batch_", "hier_"))
    cpu_proc = None
    if single and not args.no_cpu_baseline:
        # the oracle runs on the host beside the GPU measurement
        cpu_proc = start_cpu_baseline(workload, args.cpu_sample)

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
    if workload.startswith("multi_"):
        return bench_multi(args, workload)
    if workload.startswith("batch_"):
        return bench_batch(args, workload)
    if workload.startswith("hier_"):
        return bench_hier(args, workload)
    boundary, prec = WORKLOADS[workload]
    ps = inputs.make_workload(workload)
    N, n, p = ps.n, ps.n_cells, ps.p
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    x, y, z, q = (torch.from_numpy(a).to(dev) for a in (ps.x, ps.y, ps.z, ps.q))
    plan = Plan(n, p, boundary, box=ps.box, cutoff=2, precision=prec, n_max=N, shape=ps.shape)
    n = plan.n_mesh             # cells per axis of the computed mesh
    tdt = torch.float32 if prec == "f32" else torch.float64
    out = tuple(torch.empty(N, dtype=tdt, device=dev) for _ in range(4))
    # a dedicated stream (the legacy default stream adds implicit synchronisation)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    torch.cuda.set_stream(stream)
    tuning = None
    if args.column_kernel is not None:
        plan.set_tuning(column_kernel=args.column_kernel)
        tuning = plan.tuning()
    elif not args.no_autotune:
        # plan-time choice of launch shapes on this workload (not timed)
        tuning = plan.autotune(x, y, z, q, out=out)

    plan.set_graphs(bool(args.graphs))
    # warm-up; the second half also times every stage to pick the dominant kernel
    half = max(1, args.warmup // 2)
    far_stages = [s for s in STAGES if s != "near"]
    for i in range(max(2, args.warmup)):
        if i == half:
            plan.set_profiling(far_stages)
        plan.far(x, y, z, q, out=out)
    torch.cuda.synchronize()
    prof = plan.read_profile(reset=True)
    means = {st: (ms / c if c else 0.0) for st, (ms, c) in prof.items() if st in far_stages}
    dominant = max(means, key=means.get)
    print("stage means: " + ", ".join(f"{k}={v*1e3:.1f}us" for k, v in means.items()),
          file=sys.stderr)

    # timed region: exactly K steps between two synchronisations; per-step
    # events on the stream give the median, and only the dominant stage
    # carries the library's stage events
    K = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    plan.set_profiling([dominant])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(K):
        plan.far(x, y, z, q, out=out)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.sync_status()
    prof = plan.read_profile(reset=True)
    plan.set_profiling([])
    step_ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(K))
    ms_k, cnt = prof[dominant]
    t_k = ms_k / cnt / 1e3

    err = golden_error(workload, out, prec)

    # the near field beside it (not part of the metric): median of a few
    # pmmm_near calls and of a few pmmm_total calls (one binning for both)
    near_t = []
    for fn in (plan.near, plan.total):
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn(x, y, z, q, out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        near_t.append(sorted(ts)[len(ts) // 2])
    near_rec = {"near_ms": near_t[0], "total_ms": near_t[1],
                "note": "pmmm_near_* and pmmm_total_* (far + near, one binning), median of 5 calls; "
                        "not part of the far-field metric"}

    storage_rec = bench_storage(plan, p, stream) if prec == "f32" else None

    nf = 2 * n if boundary == "open" else n
    tsize = 4 if prec == "f32" else 8
    peak_alu = FP32_PEAK if prec == "f32" else FP64_PEAK
    bytes_k, flops_k = algorithmic_work(dominant, N, n, p, nf, tsize)
    roof = _roofline(t_k, bytes_k, flops_k, peak_alu)
    form = tuning.get("column_kernel") if (tuning and dominant == "column") else None
    roof["traffic"] = load_traffic(dominant, workload, kernel_source_hash(dominant), form)
    roof["kernel"] = dominant if form in (None, "default") else f"{dominant} ({form})"
    roof["kernel_us"] = t_k * 1e6
    roof["algorithmic_bytes"] = bytes_k
    roof["algorithmic_flops"] = flops_k
    # whole step: sum over the stages of their roofline times, over the
    # median step time
    t_med = step_ms[len(step_ms) // 2] / 1e3
    t_roof = sum(max(b / HBM_PEAK, f / peak_alu)
                 for b, f in (algorithmic_work(s, N, n, p, nf, tsize) for s in far_stages))
    step_roof = {"algorithmic_bytes": sum(algorithmic_work(s, N, n, p, nf, tsize)[0]
                                          for s in far_stages),
                 "roofline_time_us": t_roof * 1e6, "median_step_us": t_med * 1e6,
                 "frac": t_roof / t_med}

    cpu = finish_cpu_baseline(cpu_proc) if cpu_proc is not None else None

    rec = {
        "metric": METRIC,
        "value": N * K / el,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": el / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": workload, "boundary": boundary, "n_particles": N,
                   "cells": (f"{n}^3" if ps.shape is None else
                             "x".join(map(str, ps.shape)) + f" (computed in {n}^3)"),
                   "fft_mesh": f"{nf}^3", "p": p, "cutoff": 2,
                   "tuning": tuning,
                   "parallelism": "single GPU"},
        "step_ms": {"median": step_ms[len(step_ms) // 2], "min": step_ms[0],
                    "max": step_ms[-1], "events": K},
        "error": err,
        "roofline": roof,
        "step_roofline": step_roof,
        "stage_us": {k: v * 1e3 for k, v in means.items()},
        "near_field": near_rec,
        "coef_storage": storage_rec,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    if err is not None and not err["ok"]:
        print("error above the bound: the line is not a valid measurement", file=sys.stderr)
        sys.exit(3)


def bench_storage(plan, p, stream, reps=50):
    """Coefficient storage calls on the workload's own meshes (outside the
    far-field metric): per-order fixed-point records of the local-expansion
    mesh (Sec. 5.3) and the App. D composition of the local-expansion and
    moment meshes.  The stream is held by a spin kernel while the calls are
    queued, so the events time back-to-back kernels, not host launch gaps."""
    import numpy as np
    import torch
    from paper_1409_5981_amd import _lib
    P = (p + 1) ** 2
    Lh = plan.mesh(_lib.PMMM_MESH_L).reshape(P, -1).astype(np.float32)
    Mh = plan.mesh(_lib.PMMM_MESH_M).reshape(P, -1).astype(np.float32)
    dev = torch.device("cuda")
    L, M = torch.from_numpy(Lh).to(dev), torch.from_numpy(Mh).to(dev)
    ncell = L.shape[1]
    W = _lib.coef_record_words(p)
    rec, ex = _lib.coef_pack(p, L, stream=stream)
    back = _lib.coef_unpack(p, rec, ex, stream=stream)
    comp = _lib.coef_compose(p, L, M, stream=stream)
    sa, sb = _lib.coef_split(p, comp, stream=stream)
    torch.cuda.synchronize()
    d = (back - L).double()
    rt_err = float(torch.sqrt((d * d).sum() / (L.double() ** 2).sum()))

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            torch.cuda._sleep(20_000_000)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    fw, cw = 4 * P * ncell, 4 * W * ncell
    cases = {
        "pack_auto_units": (lambda: _lib.coef_pack(p, L, rec, ex, True, stream), 2 * fw + cw),
        "pack_given_units": (lambda: _lib.coef_pack(p, L, rec, ex, False, stream), fw + cw),
        "unpack": (lambda: _lib.coef_unpack(p, rec, ex, back, stream), cw + fw),
        "compose": (lambda: _lib.coef_compose(p, L, M, comp, stream), 4 * fw),
        "split": (lambda: _lib.coef_split(p, comp, sa, sb, stream), 4 * fw),
    }
    kern = {}
    for name, (fn, nbytes) in cases.items():
        t = timed(fn)
        kern[name] = {"us": t * 1e6, "algorithmic_bytes": nbytes, "GB/s": nbytes / t / 1e9,
                      "frac": nbytes / t / HBM_PEAK}
    return {"mesh": f"local-expansion mesh of the workload, {P} x {ncell} float32",
            "bits_per_cell": 3 * (p + 1) * (p + 2) * (2 * p + 3) // 6,
            "record_bytes_per_cell": 4 * W, "float_bytes_per_cell": 4 * P,
            "round_trip_rel_rms": rt_err, "calls": kern,
            "note": "pmmm_coef_* calls (Sec. 5.3 records, App. D composite); not part of the "
                    "far-field metric; HIP events over %d back-to-back calls each" % reps}


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
    stages5 = [s for s in STAGES if s != "near"]
    warm = max(2, args.warmup)
    half = max(1, warm // 2)
    for i in range(warm):
        if i == half:
            plan.set_profiling(stages5)
        plan.far_multi(x, y, z, q, out=out)
    torch.cuda.synchronize()
    prof = plan.read_profile(reset=True)
    means = {st: (ms / c if c else 0.0) for st, (ms, c) in prof.items() if st in stages5}
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
    roof["traffic"] = load_traffic(dominant, workload, kernel_source_hash(dominant))
    roof["kernel"] = dominant
    roof["kernel_us"] = t_k * 1e6
    roof["algorithmic_bytes"] = bytes_k
    roof["algorithmic_flops"] = flops_k
    stages = {st: {"us": means[st] * 1e3} for st in stages5}
    for st in stages5:
        b_, f_, m_ = multi_stage_work(st, N, S, n, p, nprod)
        if means[st] > 0:
            stages[st]["hbm_frac"] = b_ / (means[st] / 1e3) / HBM_PEAK
            if m_:
                stages[st]["mfma_frac"] = m_ / (means[st] / 1e3) / BF16_PEAK
    # error of four sets on the stored oracle sample
    err = None
    path = os.path.join(ROOT, "tests", "golden", f"ref_{workload}.npz")
    if os.path.exists(path) and args.split == "f32":
        import numpy as np
        ref = np.load(path)
        idx = torch.from_numpy(ref["idx"]).to(dev)
        worst = 0.0
        for k, s in enumerate(ref["sets"]):
            g = torch.stack([o[idx, int(s)] for o in out[1:]], 1).double().cpu().numpy()
            ph = out[0][idx, int(s)].double().cpu().numpy()
            eg = float(np.sqrt(np.sum((g - ref["grad"][k]) ** 2) / np.sum(ref["grad"][k] ** 2)))
            ep = float(np.sqrt(np.sum((ph - ref["phi"][k]) ** 2) / np.sum(ref["phi"][k] ** 2)))
            worst = max(worst, eg, ep)
        err = {"worst_rel_rms": worst, "sets": [int(s) for s in ref["sets"]],
               "sample": int(len(ref["idx"])), "bound": ERR_BOUND["f32"],
               "ok": worst <= ERR_BOUND["f32"]}
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
        "error": err,
        "roofline": roof,
        "stages": stages,
        "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def bench_batch(args, workload):
    """Batched workload: 256 independent periodic systems (N uniform in
    [2048, 65536], meshes 8^3/16^3/32^3, p in {4, 5, 6}, neutral +/-1); one
    step is one pmmm_batch_far_f32 call over all of them (graph replay after
    the second call).  The roofline sums the algorithmic bytes of every
    stage of every system."""
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
    K = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(K):
        batch.far(offs, x, y, z, q, out=out, stream=stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    batch.sync_status()
    step_ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(K))
    t_med = step_ms[len(step_ms) // 2] / 1e3
    stages = ["bin", "p2m", "fft_fwd", "column", "fft_inv", "l2p"]
    tot_b = tot_t = 0.0
    for ps in systems:
        for st in stages:
            b, f = algorithmic_work(st, ps.n, ps.n_cells, ps.p, ps.n_cells)
            tot_b += b
            tot_t += max(b / HBM_PEAK, f / FP32_PEAK)
    roof = {"bound": "hbm", "achieved": tot_b / t_med / 1e9, "peak": HBM_PEAK / 1e9,
            "unit": "GB/s", "frac": tot_b / t_med / HBM_PEAK, "traffic": None,
            "kernel": "whole batch call", "algorithmic_bytes": tot_b,
            "roofline_time_us": tot_t * 1e6, "roofline_frac": tot_t / t_med}
    meshes = {m: sum(1 for ps in systems if ps.n_cells == m) for m in (8, 16, 32)}
    rec = {
        "metric": "particles/s over a batch of independent periodic systems, PMMM far field",
        "value": N * K / el,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": max(3, args.warmup),
        "ms_per_step": el / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "systems": len(systems), "n_particles": N,
                   "classes": batch.classes, "meshes": meshes, "cutoff": 2,
                   "parallelism": "single GPU"},
        "step_ms": {"median": step_ms[len(step_ms) // 2], "min": step_ms[0],
                    "max": step_ms[-1], "events": K},
        "roofline": roof,
        "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


def _near_pairs(x, y, z, nc, c):
    """Ordered pairs i != j whose cells (nc^3 over the unit box) are within c
    of each other (Chebyshev): the near field's pair count."""
    import numpy as np
    idx = [np.clip((np.asarray(a, dtype=np.float64) * nc).astype(np.int64), 0, nc - 1)
           for a in (x, y, z)]
    cnt = np.bincount((idx[2] * nc + idx[1]) * nc + idx[0], minlength=nc ** 3)
    cnt = cnt.reshape(nc, nc, nc).astype(np.float64)
    pad = np.pad(cnt, c)
    tot = 0.0
    for dz in range(-c, c + 1):
        for dy in range(-c, c + 1):
            for dx in range(-c, c + 1):
                tot += float(np.sum(cnt * pad[c + dz:c + dz + nc, c + dy:c + dy + nc,
                                              c + dx:c + dx + nc]))
    return int(tot) - len(idx[0])


def _fine_pairs(n, r, c):
    """Pairs of fine cells (target, source) whose coarse cells are within c
    and fine cells are not: the fine level's eq. M2L products, counted
    exactly."""
    import numpy as np
    nf = n * r
    cells = np.arange(nf)
    D = (c + 1) * r - 1
    per_axis = {}                 # offset d -> targets i with source i - d in a near coarse cell
    for d in range(-D, D + 1):
        i = cells[max(0, d):min(nf, nf + d)]
        per_axis[d] = int(np.sum(np.abs(i // r - (i - d) // r) <= c))
    pairs = 0
    for dz in range(-D, D + 1):
        for dy in range(-D, D + 1):
            for dx in range(-D, D + 1):
                if max(abs(dx), abs(dy), abs(dz)) <= c:
                    continue
                pairs += per_axis[dx] * per_axis[dy] * per_axis[dz]
    return pairs


def bench_hier(args, workload):
    """Two-level hierarchical PMMM (pmmm_hier_*, Sec. 5.2).  One step is one
    call.
      hier_open_n1048576_m16r2_p4_c1: the far field of 2^20 uniform
        particles with neutral +/-1 charges in the unit box, coarse 16^3
        open mesh refined by 2 (fine 32^3), p = 4, c = 1;
      hier_total_plummer_n4194304_m64r2_p4_c1: the total field (far + near)
        of the 2^22-particle Plummer sphere of the default workload, coarse
        64^3 refined by 2 (fine 128^3), p = 4, c = 1, beside the total field
        of the uniform 64^3 plan at the same p and c on the same particles
        (the clustered case the hierarchy is for: the near field shrinks
        with the finer cells).
    The far-field line's roofline takes the fine level's algorithmic work,
    one real (P x P) eq. M2L product per pair of fine cells whose coarse
    cells are near and fine cells are not, over that kernel's own time (HIP
    events around it); the total-field line's takes the near-field pairs
    and those products over the whole call."""
    import numpy as np
    import torch
    from paper_1409_5981_amd import inputs
    from paper_1409_5981_amd._lib import Hier, Plan

    total = workload.startswith("hier_total_")
    if total:
        ps = inputs.plummer_sphere()
        x, y, z, q = ps.x, ps.y, ps.z, ps.q
        N, n, r, p, c = ps.n, 64, 2, 4, 1
        K, W = min(args.steps, 10), min(args.warmup, 2)
    else:
        N, n, r, p, c = 1 << 20, 16, 2, 4, 1
        rng = np.random.Generator(np.random.PCG64(10))
        x, y, z = inputs.uniform_positions(rng, N, np.float32)
        q = inputs.neutral_pm1(rng, N, np.float32)
        K, W = args.steps, max(3, args.warmup)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    xt, yt, zt, qt = (torch.from_numpy(a).to(dev) for a in (x, y, z, q))
    h = Hier(n, p, r, cutoff=c, n_max=N)
    out = tuple(torch.empty(N, dtype=torch.float32, device=dev) for _ in range(4))
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    torch.cuda.set_stream(stream)
    call = h.total if total else h.far
    for _ in range(W):
        call(xt, yt, zt, qt, out=out, stream=stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(K):
        call(xt, yt, zt, qt, out=out, stream=stream)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    h.sync_status()
    step_ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(K))
    t_med = step_ms[len(step_ms) // 2] / 1e3
    # the fine level's kernel alone: HIP events around it on the call's
    # stream, in calls of their own after the timed ones
    h.set_profiling(["column"])
    h.read_profile(1)
    for _ in range(min(K, 20)):
        call(xt, yt, zt, qt, out=out, stream=stream)
    torch.cuda.synchronize()
    fms, fcnt = h.read_profile(1)["column"]
    h.set_profiling([])
    t_fine = fms / max(fcnt, 1) / 1e3
    nf = n * r
    pairs = _fine_pairs(n, r, c)
    P = (p + 1) ** 2
    flops = 2 * P * P * pairs
    roof = {"bound": "alu", "achieved": flops / t_fine / 1e12, "peak": FP32_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": flops / t_fine / FP32_PEAK, "traffic": None,
            "kernel": "fine-level eq. M2L sums (k_hier_m2l_cell)", "kernel_us": t_fine * 1e6,
            "algorithmic_flops": flops, "fine_pairs": pairs,
            "call_frac": flops / t_med / FP32_PEAK}
    extra = {}
    if total:
        # the near field's pairs on the fine mesh at NEAR_FLOPS_PER_PAIR
        # FP32 operations each, with the fine level's products, over the
        # whole call (the near field takes most of it)
        near_h = _near_pairs(x, y, z, nf, c)
        work = flops + NEAR_FLOPS_PER_PAIR * near_h
        roof.update({"achieved": work / t_med / 1e12, "frac": work / t_med / FP32_PEAK,
                     "kernel": "whole hierarchical total call (near-field pairs and fine-level flops)",
                     "algorithmic_flops": work, "near_pairs": near_h,
                     "fine_frac": flops / t_fine / FP32_PEAK})
        roof.pop("call_frac")
        # the uniform plan's total field on the same particles, and how
        # closely the two agree (the same method error, other cells)
        hout = [o.double().cpu().numpy() for o in out]
        plan = Plan(n, p, "open", cutoff=c, n_max=N)
        uout = tuple(torch.empty(N, dtype=torch.float32, device=dev) for _ in range(4))
        plan.total(xt, yt, zt, qt, out=uout, stream=stream)
        torch.cuda.synchronize()
        ut = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            plan.total(xt, yt, zt, qt, out=uout, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ut.append(e0.elapsed_time(e1))
        plan.sync_status()
        u = [o.double().cpu().numpy() for o in uout]
        gh, gu = np.stack(hout[1:], 1), np.stack(u[1:], 1)
        extra = {"uniform_total_ms": sorted(ut)[1], "hier_total_ms": step_ms[len(step_ms) // 2],
                 "speedup_vs_uniform": sorted(ut)[1] / step_ms[len(step_ms) // 2],
                 "near_pairs_hier": near_h,
                 "near_pairs_uniform": _near_pairs(x, y, z, n, c),
                 "grad_rel_rms_hier_vs_uniform":
                     float(np.sqrt(np.sum((gh - gu) ** 2) / np.sum(gu ** 2)))}
    rec = {
        "metric": ("particles/s, two-level hierarchical PMMM total field (far + near)" if total
                   else "particles/s, two-level hierarchical PMMM far field"),
        "value": N * K / el,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": el / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "n_particles": N, "coarse": f"{n}^3", "refine": r,
                   "fine": f"{nf}^3", "p": p, "cutoff": c, "parallelism": "single GPU"},
        "step_ms": {"median": step_ms[len(step_ms) // 2], "min": step_ms[0],
                    "max": step_ms[-1], "events": K},
        "roofline": roof,
        **extra,
        "cpu_baseline": None,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
