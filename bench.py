"""Benchmark of the ternary free-energy entropic LBM update on one MI355X.

Default workload: D2Q9 1024x1024 periodic, liquid/gas density ratio 1000, two
seeded drops (the FP64-vs-FP32-mixed workload).  `value` is the FP64 path's
whole-job MLUPS; the FP32-mixed path and the D3Q27 256^3 ratio-1000 collision
box are measured in the same run and reported beside it.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def library_params(T, wl, precision):
    import paper_1710_07486_amd as T_
    nz, ny, nx = wl.shape
    ph = wl.physics()
    return T_.Params(lattice=wl.lattice, precision=precision, nx=nx, ny=ny, nz=nz, T=T,
                     lambda1=ph["lambda1"], lambda2=ph["lambda2"], lambda3=ph["lambda3"],
                     kappa1=ph["kappa1"], kappa2=ph["kappa2"], kappa3=ph["kappa3"], chi=ph["chi"],
                     nu=ph["nu"], mobility=ph["mobility"], tau_phi=ph["tau_phi"])


def measure(wl, precision, steps, warmup, fields=None):
    """Whole-step MLUPS with HIP events on the solver's stream, and the mean
    duration of each kernel kind.  Drops start at the discretised model's own
    coexistence densities (a 1D slab relaxed by the library)."""
    import torch
    import paper_1710_07486_amd as T_
    from paper_1710_07486_amd.calibrate import discrete_coexistence
    from synth import workloads as W
    T = T_.temperature_for_ratio(wl.ratio)
    p = library_params(T, wl, precision)
    if fields is None:
        rg, rl = discrete_coexistence(library_params(T, wl, T_.FP64))
        log("discrete coexistence densities", rg, rl)
        fields = W.fields(wl, rg, rl)
    rho, phi, u = fields
    s = T_.Solver(p)
    uu = u if np.abs(u).max() > 0 else None
    s.init_fields(rho, phi, uu)
    s.step(warmup)
    s.sync()
    stream = s.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kern = s.time_kernels(max(3, min(steps, 20)))
    d = s.diagnostics(check=False)
    out = {"mlups": wl.nodes * steps / (ms * 1e-3) / 1e6, "ms_per_step": ms / steps, "kernels_ms": kern,
           "bytes_per_update": s.algorithmic_bytes_per_update(), "diag": d}
    out["rho"] = s.read("rho", check=False)
    s.close()
    del s
    torch.cuda.empty_cache()
    return out, fields


def cpu_baseline(wl, budget_s=15.0):
    """The FP64 oracle on the host cores, on a bounded number of steps of the
    same workload."""
    from oracle import oracle as O
    from synth import workloads as W
    O.build(force=False)
    p = O.coexisting_params(wl.ratio, **wl.physics())
    rho, phi, u = W.fields(wl, p.rho_g, p.rho_l)
    st = O.State(p, rho, phi, u if np.abs(u).max() > 0 else None)
    t0 = time.perf_counter()
    st.run(1)
    t1 = time.perf_counter()
    n = max(1, min(200, int(budget_s / max(t1 - t0, 1e-3))))
    t0 = time.perf_counter()
    st.run(n)
    dt = time.perf_counter() - t0
    return {"value": wl.nodes * n / dt / 1e6, "unit": "MLUPS", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{wl.name}: {n} time steps of the full lattice (FP64 oracle, OpenMP)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU-baseline leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the D3Q27 256^3 measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the lattice would shard by slabs, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1710_07486_amd as T_
    from synth import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    wl = W.drops_2d(1024, ratio=1000.0, seed=0)
    log("workload", wl.name, "steps", args.steps, "warmup", args.warmup)
    r64, fields = measure(wl, T_.FP64, args.steps, args.warmup)
    log("fp64", {k: v for k, v in r64.items() if k != "rho"})
    r32, _ = measure(wl, T_.FP32_MIXED, args.steps, args.warmup, fields)
    log("fp32-mixed", {k: v for k, v in r32.items() if k != "rho"})
    rel_rho = float(np.abs(r32["rho"] - r64["rho"]).max() / np.abs(r64["rho"]).max())

    kern = r64["kernels_ms"]
    dom = max(kern, key=kern.get)
    achieved = r64["bytes_per_update"] * wl.nodes / (kern["collide"] * 1e-3) / 1e9
    result = {
        "metric": "ternary ELBM MLUPS & % HBM roofline; FP32-mixed vs FP64 at stated error",
        "value": round(r64["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded drops, SplitMix64 noise)",
        "config": {"workload": wl.name, "lattice": "D2Q9", "nx": 1024, "ny": 1024, "density_ratio": 1000,
                   "precision": "fp64", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "collide", "kernels_ms": {k: round(v, 5) for k, v in kern.items()},
                     "dominant": dom},
        "fp32_mixed": {"value": round(r32["mlups"], 2), "unit": "MLUPS",
                       "speedup_vs_fp64": round(r32["mlups"] / r64["mlups"], 3),
                       "rel_density_error_vs_fp64": rel_rho,
                       "kernels_ms": {k: round(v, 5) for k, v in r32["kernels_ms"].items()}},
        "whole_step_hbm_frac": round(r64["mlups"] * 1e6 * r64["bytes_per_update"] / (HBM_PEAK_GBS * 1e9), 4),
    }
    if not args.no_3d:
        wl3 = W.collision_3d(256, radius=32, ratio=1000.0, v_rel=0.04, kappa2=0.1, kappa3=0.1)
        s3 = max(10, args.steps // 4)
        log("workload", wl3.name, "steps", s3)
        r3, f3 = measure(wl3, T_.FP64, s3, 5)
        r3m, _ = measure(wl3, T_.FP32_MIXED, s3, 5, f3)
        k3 = r3["kernels_ms"]
        result["d3q27_256"] = {
            "fp64_mlups": round(r3["mlups"], 2), "fp32_mixed_mlups": round(r3m["mlups"], 2),
            "fp64_collide_GBs": round(r3["bytes_per_update"] * wl3.nodes / (k3["collide"] * 1e-3) / 1e9, 1),
            "fp64_whole_step_hbm_frac": round(r3["mlups"] * 1e6 * r3["bytes_per_update"] / (HBM_PEAK_GBS * 1e9), 4),
            "fp64_kernels_ms": {k: round(v, 5) for k, v in k3.items()},
            "fp32_mixed_kernels_ms": {k: round(v, 5) for k, v in r3m["kernels_ms"].items()},
            "rel_density_error_mixed_vs_fp64": float(np.abs(r3m["rho"] - r3["rho"]).max() / np.abs(r3["rho"]).max()),
        }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
