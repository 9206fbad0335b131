#!/usr/bin/env python3
"""Throughput of the OD2Pm ADMM frame sweep on one MI355X.

One step = one full ADMM iteration of Algorithm 2 over the whole synthetic scan:
the frame sweep (gather, 2-D FFT, ST-AGM prox, Gamma update, inverse FFT,
overlap-add) followed by the pixel update (u, Lam and the consensus v).
Workload: 512 x 512 complex image, 64 x 64 disk probe, raster step 16 with +-2 px
jitter (29 x 29 = 841 frames), Poisson noise at peak 1e4 photons, 4 x 4 subdomains.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  Options: --steps K --warmup W --gpus 1 (one GPU only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ADMM frame-iters/s (FP32 FFT vs split-BF16 MFMA DFT) at fixed rel. error"
HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_sweep_c2_pmc.md")
KERNEL_SOURCES = ["paper_2011_00162_amd/csrc/kernels.hip", "paper_2011_00162_amd/csrc/fft_frame.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per sweep launch from the committed PMC summary, if it matches the kernel source."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    txt = open(PMC_SUMMARY).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not (m_hash and m_bytes) or m_hash.group(1) != kernel_hash():
        return None
    return float(m_bytes.group(1))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def gpu_leg(args, torch, odp, synthetic):
    spec = synthetic.CONFIGS["c2"]
    pr = synthetic.draw_problem(spec)
    n, p = spec.n, spec.p
    dev = "cuda"
    u_true = torch.from_numpy(pr["u_true"].astype("complex64")).to(dev)
    w = torch.from_numpy(pr["w"].astype("complex64")).to(dev)
    J = len(pr["offsets"])
    # measured intensities: the library's own forward operator, then seeded Poisson counts
    synth = odp.Plan(n, n, p, pr["offsets"], pr["frame_sub"], r=1.0)
    synth.bind(torch.ones((J, p, p), dtype=torch.float32, device=dev), w)
    f = (synth.forward(u_true, w).abs() ** 2).double().cpu().numpy()
    del synth
    f = synthetic.poisson_counts(f, spec.peak, pr["rng_poisson"])
    sqrt_f = torch.from_numpy(f ** 0.5).float().to(dev)
    eps, eta = 0.5, 0.1
    plan = odp.Plan(n, n, p, pr["offsets"], pr["frame_sub"], eps=eps, eta=eta, r=1.0)
    plan.bind(sqrt_f, w)
    r = 0.5 * eta * plan.illum_max()
    plan.set_params(r=r)
    state = plan.new_state()
    info = plan.info

    plan.iterate(state, args.warmup)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    plan.iterate(state, args.steps)
    t1.record()
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)

    # per-kernel timing of the frame sweep, events on the launch stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        plan.frame_sweep(state)
        b.record()
        plan.pixel_update(state)
    torch.cuda.synchronize()
    sweep_ms = sorted(a.elapsed_time(b) for a, b in ev)
    sweep_avg_ms = sum(sweep_ms) / len(sweep_ms)
    alg_bytes = 20.0 * J * p * p + 16.0 * info.p_sub
    return dict(J=J, n=n, p=p, D=info.D, total_ms=total_ms, sweep_avg_ms=sweep_avg_ms,
                sweep_median_ms=sweep_ms[len(sweep_ms) // 2], alg_bytes=alg_bytes, r=r, eta=eta, eps=eps,
                p_sub=info.p_sub, n_pairs=info.n_pairs)


def cpu_leg(args, torch, odp, synthetic):
    """The FP64 oracle on a bounded sample of the same workload, and the GPU on the same data."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import operators as ops
    from oracle.geometry import build_geometry
    from oracle.od2p import merge, od2pm_run, subdomain_illumination

    spec = synthetic.CONFIGS["c2"]
    pr = synthetic.draw_problem(spec)
    f = synthetic.poisson_counts(ops.intensities(pr["u_true"], pr["w"], pr["offsets"]), spec.peak,
                                 pr["rng_poisson"])
    sf32 = np.sqrt(f).astype(np.float32)
    f = sf32.astype(np.float64) ** 2
    w = pr["w"].astype(np.complex64).astype(np.complex128)
    g = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
    eps, eta = 0.5, 0.1
    r = 0.5 * eta * max(float(subdomain_illumination(g, w, d).max()) for d in range(g.D))
    K = args.cpu_iters
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        st, _ = od2pm_run(g, w, f, eps, eta, r, K)
        dt = time.perf_counter() - t
    u_or = merge(g, st.u)
    # the GPU path on the identical data and iteration count
    plan = odp.Plan(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"], eps=eps, eta=eta, r=r)
    plan.bind(torch.from_numpy(sf32).cuda(), torch.from_numpy(w.astype(np.complex64)).cuda())
    state = plan.new_state()
    plan.iterate(state, K)
    u_gpu = plan.merge(state).cpu().numpy().astype(np.complex128)
    rel_err = float(np.linalg.norm(u_gpu - u_or) / np.linalg.norm(u_or))
    return dict(value=g.J * K / dt, unit="frame-iters/s", cores=1, kind="oracle",
                sample=f"{K} OD2Pm iterations of the full 512x512 / 841-frame workload (FP64 NumPy, "
                       f"single thread) in {dt:.1f} s on {cpu_model()} ({os.cpu_count()} logical CPUs)",
                rel_err_gpu_vs_oracle=rel_err, rel_err_iters=K)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-iters", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (scales the HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the subdomains of one problem run as workgroups of one device).", file=sys.stderr)
        return 2
    if args.steps < 1:
        print("--steps must be >= 1", file=sys.stderr)
        return 2

    import torch
    import synthetic
    import paper_2011_00162_amd as odp

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    g = gpu_leg(args, torch, odp, synthetic)
    ms_per_step = g["total_ms"] / args.steps
    value = g["J"] * args.steps / (g["total_ms"] / 1e3)
    achieved = g["alg_bytes"] / (g["sweep_avg_ms"] / 1e3) / 1e9
    traffic = measured_traffic()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "frame-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "non-blind OD2Pm, 512x512 image, 64x64 disk probe (R=24, phase 0.02 r^2), raster step 16 "
                        "+-2 px jitter, 841 frames, Poisson peak 1e4, 4x4 subdomains, eps=0.5, eta=0.1, "
                        "r=0.5*eta*max(diag A*A)",
            "transform": "fft_f32",
            "frames": g["J"], "probe": g["p"], "image": g["n"], "subdomains": g["D"], "pairs": g["n_pairs"],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_sweep<64> (frame sweep)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": g["alg_bytes"],
            "avg_launch_ms": g["sweep_avg_ms"],
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_leg(args, torch, odp, synthetic)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
