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
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak, TFLOP/s

# HBM bytes per launch of the D2Q9 1024x1024 FP64 step kernel (chemical
# potentials, collision and next-step moments in one launch) from two rocprofv3
# counter passes (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0, scales from a 1 GiB copy
# in the same runs; profiles/collide_d2q9_1024_fp64_traffic.md), valid only for
# the kernel sources whose hash is recorded with it.
COLLIDE_TRAFFIC = {"bytes_per_launch": 348263540, "sources_sha256_16": "23c3c63e8f701e57"}


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "node_ops.hpp", "lattice.hpp"):
        with open(os.path.join(ROOT, "paper_1710_07486_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def library_params(T, wl, precision, eos=None, extra=None):
    """Solver parameters of workload `wl`; `eos` optionally names another free
    energy as {"eos": kind, "a": a, "b": b}; `extra` adds fields (walls,
    contact angles)."""
    import paper_1710_07486_amd as T_
    nz, ny, nx = wl.shape
    ph = wl.physics()
    return T_.Params(lattice=wl.lattice, precision=precision, nx=nx, ny=ny, nz=nz, T=T,
                     lambda1=ph["lambda1"], lambda2=ph["lambda2"], lambda3=ph["lambda3"],
                     kappa1=ph["kappa1"], kappa2=ph["kappa2"], kappa3=ph["kappa3"], chi=ph["chi"],
                     nu=ph["nu"], mobility=ph["mobility"], tau_phi=ph["tau_phi"], walls=ph.get("walls", 0),
                     **(eos or {}), **(extra or {}))


def measure(wl, precision, steps, warmup, fields=None, coex=None, eos=None, extra=None):
    """Whole-step MLUPS with HIP events on the solver's stream, and the mean
    duration of each kernel kind.  Drops start at the discretised model's own
    coexistence densities (a 1D slab relaxed by the library, unless `coex`
    gives them)."""
    import torch
    import paper_1710_07486_amd as T_
    from paper_1710_07486_amd.calibrate import discrete_coexistence
    from synth import workloads as W
    T = T_.temperature_for_ratio(wl.ratio, **(eos or {}))
    p = library_params(T, wl, precision, eos, extra)
    rg = rl = None
    if fields is None:
        slab = library_params(T, wl, T_.FP64, eos)
        slab.walls = 0
        rg, rl = coex if coex else discrete_coexistence(slab)
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
    taken = s.steps
    out = {"mlups": wl.nodes * steps / (ms * 1e-3) / 1e6, "ms_per_step": ms / steps, "kernels_ms": kern,
           "bytes_per_update": s.algorithmic_bytes_per_update(), "diag": d, "coex": [rg, rl], "steps_taken": taken}
    out["rho"] = s.read("rho", check=False)
    s.close()
    del s
    torch.cuda.empty_cache()
    return out, fields


def batch_throughput(steps=100, warmup=10, count=64, lo=256, hi=1024):
    """The batching form: `count` uneven D2Q9 instances (sides U{256..1024},
    ratio U[100, 1000], FP32-mixed) advanced together (persistent launches,
    graph-captured runs of steps, tile shape and workgroups per CU from the
    autotuner's timed sweep), against the same instances advanced one after
    another by the single-instance solver.  Aggregate MLUPS both ways."""
    import torch
    import paper_1710_07486_amd as T_
    from paper_1710_07486_amd import autotune
    from paper_1710_07486_amd.batch import Batch
    from synth import workloads as W
    insts = W.batch_instances(count, seed=3, lo=lo, hi=hi)
    params, fields = [], []
    for wl in insts:
        T = T_.temperature_for_ratio(wl.ratio)
        rg, rl, _, _ = T_.coexistence(T)
        p = library_params(T, wl, T_.FP32_MIXED)
        p.rho_g, p.rho_l = rg, rl
        params.append(p)
        fields.append(W.fields(wl, rg, rl))
    nodes = sum(wl.nodes for wl in insts)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with Batch(params) as b:
        for i, (r, ph, u) in enumerate(fields):
            b.init_fields(i, r, ph, u)
        rec = autotune.tune(b, steps=10, warmup=4, cache=None)
        b.step(warmup)
        b.sync()
        e0.record(b.stream)
        b.step(steps)
        e1.record(b.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        finite = all(bool(np.isfinite(b.read(i, "rho")).all()) for i in range(0, count, 8))
    seq_ms = 0.0
    s_steps = max(10, steps // 5)
    for p, (r, ph, u) in zip(params, fields):
        with T_.Solver(p) as s:
            s.init_fields(r, ph, u)
            s.step(3)
            s.sync()
            e0.record(s.stream)
            s.step(s_steps)
            e1.record(s.stream)
            torch.cuda.synchronize()
            seq_ms += e0.elapsed_time(e1) / s_steps
        torch.cuda.empty_cache()
    return {"instances": count, "sides": [lo, hi], "nodes": nodes, "precision": "fp32_mixed",
            "batched_mlups": round(nodes / ms / 1e3, 2),
            "ms_per_step": round(ms, 4), "one_by_one_mlups": round(nodes / seq_ms / 1e3, 2),
            "speedup_vs_one_by_one": round(seq_ms / ms, 3),
            "mode": {0: "persistent three-phase", 1: "fused per instance", 2: "fused, one launch"}[rec.get("mode", 0)],
            "persistent_best_mlups": round(nodes / min(r["ms_per_step"] for r in rec["table"] if r["mode"] == 0) / 1e3, 2),
            "tile_shape": rec["shape"], "wg_per_cu": rec["wg_per_cu"],
            "finite": finite}


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


def surrogate_throughput(n=256, batch=8, reps=10):
    """Training-step and forward throughput of the convolutional surrogate
    (six 3x3 layers, BF16 on the matrix cores) at the family's image size,
    timed with HIP events on the network's stream, and the mean duration of
    its dominant kernel (the 64->64 forward convolution, 4 of 6 layers)."""
    import torch
    from paper_1710_07486_amd import surrogate as S
    net = S.Network(seed=0)
    x = torch.zeros(batch * n * n * S.CH, dtype=torch.int16, device="cuda")
    y = torch.zeros_like(x)
    st = net.stream
    for _ in range(3):
        net.train_step(x, y, batch, n, n, 1e-5)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        net.train_step(x, y, batch, n, n, 1e-5)
    e1.record(st)
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / reps
    e0.record(st)
    for _ in range(reps):
        net.forward(x, batch, n, n)
    e1.record(st)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    a = net.a[1]
    out = net.a[2]
    e0.record(st)
    for _ in range(reps):
        S.conv_forward(a, batch, n, n, 64, net.wf[1], net.b[1], 64, 1, y_bf16=out, stream=st, dil=2)
    e1.record(st)
    torch.cuda.synchronize()
    conv_ms = e0.elapsed_time(e1) / reps
    px = batch * n * n
    fl_fwd = S.flops_per_pixel(padded=True) * px
    conv_tf = 2 * 9 * 64 * 64 * px / (conv_ms * 1e-3) / 1e12
    return {"image": f"{n}x{n}", "batch": batch, "train_step_ms": round(train_ms, 3),
            "train_tflops": round(3 * fl_fwd / (train_ms * 1e-3) / 1e12, 1),
            "forward_ms": round(fwd_ms, 3), "forward_tflops": round(fl_fwd / (fwd_ms * 1e-3) / 1e12, 1),
            "roofline": {"bound": "mfma", "kernel": "conv 64->64 forward (bf16)", "achieved": round(conv_tf, 1),
                         "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(conv_tf / BF16_PEAK_TFLOPS, 4),
                         "kernel_ms": round(conv_ms, 4)}}


def copy_probe(nbytes=1 << 30):
    """A plain device copy of known size (read nbytes, write nbytes): its
    FETCH_SIZE / WRITE_SIZE counters calibrate the byte counts read for the
    solver's kernels in the same profiled run."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy probe", nbytes, "bytes")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 1000 timed steps after 200 warm-up (80 ms of D2Q9 FP64 work): with 200
    # after 20 the short timed region read 5-15 % below the steady rate
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU-baseline leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the D3Q27 256^3 measurement")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-mixed measurement")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--no-reduced", action="store_true", help="skip the reduced phase-field lattice measurement")
    ap.add_argument("--no-walls", action="store_true", help="skip the wall-bounded channel measurement")
    ap.add_argument("--no-eos", action="store_true", help="skip the van der Waals / Peng-Robinson measurement")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate throughput measurement")
    ap.add_argument("--coex2d", type=float, nargs=2, metavar=("RHO_G", "RHO_L"),
                    help="coexistence densities of the 2D workload (skips their calibration run)")
    ap.add_argument("--coex3d", type=float, nargs=2, metavar=("RHO_G", "RHO_L"),
                    help="coexistence densities of the 3D workload (skips their calibration run)")
    ap.add_argument("--copy-probe", action="store_true", help="run a 1 GiB device copy first (counter scale)")
    ap.add_argument("--coex-cache", default=None,
                    help="JSON file of calibrated coexistence densities: read if present, else written")
    args = ap.parse_args()
    cache = {}
    if args.coex_cache and os.path.exists(args.coex_cache):
        with open(args.coex_cache) as fh:
            cache = json.load(fh)
        args.coex2d = args.coex2d or cache.get("2d")
        args.coex3d = args.coex3d or cache.get("3d")
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1710_07486_amd as T_
    from synth import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.copy_probe:
        copy_probe()
    wl = W.drops_2d(1024, ratio=1000.0, seed=0)
    log("workload", wl.name, "steps", args.steps, "warmup", args.warmup)
    r64, fields = measure(wl, T_.FP64, args.steps, args.warmup, coex=args.coex2d)
    cache["2d"] = r64["coex"]
    log("fp64", {k: v for k, v in r64.items() if k != "rho"})

    kern = r64["kernels_ms"]
    dom = max(kern, key=kern.get)
    traffic = (COLLIDE_TRAFFIC["bytes_per_launch"]
               if kernel_sources_hash() == COLLIDE_TRAFFIC["sources_sha256_16"] else None)
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
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_launch": int(r64["bytes_per_update"] * wl.nodes),
                     "kernel": "collide", "kernels_ms": {k: round(v, 5) for k, v in kern.items()},
                     "dominant": dom},
        "whole_step_hbm_frac": round(r64["mlups"] * 1e6 * r64["bytes_per_update"] / (HBM_PEAK_GBS * 1e9), 4),
    }
    if not args.no_fp32:
        r32, _ = measure(wl, T_.FP32_MIXED, args.steps, args.warmup, fields)
        log("fp32-mixed", {k: v for k, v in r32.items() if k != "rho"})
        diff = np.abs(r32["rho"] - r64["rho"])
        rel_rho = float(diff.max() / np.abs(r64["rho"]).max())
        # the max-norm error sits on the interfaces (a shift of an interface
        # by a small fraction of a node at ratio 1000); the mean-norm one is
        # what the bulk sees.  Both runs have taken the same steps.
        result["fp32_mixed"] = {"value": round(r32["mlups"], 2), "unit": "MLUPS",
                                "speedup_vs_fp64": round(r32["mlups"] / r64["mlups"], 3),
                                "rel_density_error_vs_fp64": rel_rho,
                                "rel_density_error_mean_norm_vs_fp64": float(diff.mean() / np.abs(r64["rho"]).mean()),
                                "error_after_steps": r32["steps_taken"],
                                "kernels_ms": {k: round(v, 5) for k, v in r32["kernels_ms"].items()}}
    if not args.no_eos:
        # the same drops with the other two free energies: Peng-Robinson at
        # ratio 1000; van der Waals at ratio 100, since its moving drops at
        # ratio 1000 diverge (the oracle's too, for a = 0.5/49 .. 1/49)
        result["other_eos"] = {}
        for name, e, ratio in (("van_der_waals", {"eos": T_.EOS_VDW, "a": 2.0 / 49.0, "b": 2.0 / 21.0}, 100.0),
                               ("peng_robinson", {"eos": T_.EOS_PR, "a": 2.0 / 49.0, "b": 2.0 / 21.0}, 1000.0)):
            wle = W.drops_2d(1024, ratio=ratio, seed=0)
            re_, _ = measure(wle, T_.FP64, args.steps, args.warmup, eos=e)
            log(name, {k: v for k, v in re_.items() if k != "rho"})
            result["other_eos"][name] = {"workload": wle.name, "a": e["a"], "b": e["b"],
                                         "fp64_mlups": round(re_["mlups"], 2),
                                         "vs_carnahan_starling": round(re_["mlups"] / r64["mlups"], 3),
                                         "collide_ms": round(re_["kernels_ms"]["collide"], 5),
                                         "finite": bool(np.isfinite(re_["rho"]).all())}
    if not args.no_walls:
        # a channel between wetting walls (60 / 120 degrees), caps of liquid 1
        # and 2 on the walls, same size and ratio as the drops
        wlw = W.wall_drops(1024, 1024, radius=200.0, ratio=1000.0)
        ang = {"theta_rho_lo": math.radians(60.0), "theta_phi_lo": math.radians(60.0),
               "theta_rho_hi": math.radians(120.0), "theta_phi_hi": math.radians(120.0)}
        result["walls"] = {"workload": wlw.name, "angles_deg": [60.0, 120.0]}
        for tag, prec in (("fp64", T_.FP64), ("fp32_mixed", T_.FP32_MIXED)):
            rw, _ = measure(wlw, prec, args.steps, args.warmup, coex=r64["coex"], extra=ang)
            log("walls", tag, {k: v for k, v in rw.items() if k != "rho"})
            result["walls"][tag + "_mlups"] = round(rw["mlups"], 2)
            result["walls"][tag + "_vs_periodic"] = round(rw["mlups"] / (r64["mlups"] if tag == "fp64" else
                                                                         result.get("fp32_mixed", {}).get("value", float("nan"))), 3)
            result["walls"][tag + "_finite"] = bool(np.isfinite(rw["rho"]).all())
    if not args.no_reduced:
        # the same drops with the phase field on D2Q5 (fewer bytes per update)
        rr, _ = measure(wl, T_.FP64, args.steps, args.warmup, fields, extra={"glattice": 1})
        log("reduced g lattice", {k: v for k, v in rr.items() if k != "rho"})
        result["reduced_g_lattice"] = {"lattice": "D2Q9 + D2Q5", "fp64_mlups": round(rr["mlups"], 2),
                                       "vs_full": round(rr["mlups"] / r64["mlups"], 3),
                                       "bytes_per_update": rr["bytes_per_update"],
                                       "collide_ms": round(rr["kernels_ms"]["collide"], 5)}
    if not args.no_3d:
        wl3 = W.collision_3d(256, radius=32, ratio=1000.0, v_rel=0.04, kappa2=0.1, kappa3=0.1)
        s3 = max(10, args.steps // 4)
        log("workload", wl3.name, "steps", s3)
        r3, f3 = measure(wl3, T_.FP64, s3, 5, coex=args.coex3d)
        cache["3d"] = r3["coex"]
        r3m, _ = measure(wl3, T_.FP32_MIXED, s3, 5, f3)
        r3r = None if args.no_reduced else measure(wl3, T_.FP64, s3, 5, f3, extra={"glattice": 1})[0]
        k3 = r3["kernels_ms"]
        result["d3q27_256"] = {
            "fp64_mlups": round(r3["mlups"], 2), "fp32_mixed_mlups": round(r3m["mlups"], 2),
            "fp64_collide_GBs": round(r3["bytes_per_update"] * wl3.nodes / (k3["collide"] * 1e-3) / 1e9, 1),
            "fp64_whole_step_hbm_frac": round(r3["mlups"] * 1e6 * r3["bytes_per_update"] / (HBM_PEAK_GBS * 1e9), 4),
            "fp64_kernels_ms": {k: round(v, 5) for k, v in k3.items()},
            "fp32_mixed_kernels_ms": {k: round(v, 5) for k, v in r3m["kernels_ms"].items()},
            "rel_density_error_mixed_vs_fp64": float(np.abs(r3m["rho"] - r3["rho"]).max() / np.abs(r3["rho"]).max()),
            "rel_density_error_mean_norm_mixed_vs_fp64": float(np.abs(r3m["rho"] - r3["rho"]).mean()
                                                               / np.abs(r3["rho"]).mean()),
            "error_after_steps": r3m["steps_taken"],
        }
        if r3r is not None:
            result["d3q27_256"]["fp64_reduced_g_mlups"] = round(r3r["mlups"], 2)
            result["d3q27_256"]["fp64_reduced_g_vs_full"] = round(r3r["mlups"] / r3["mlups"], 3)
    if args.coex_cache and not os.path.exists(args.coex_cache):
        with open(args.coex_cache, "w") as fh:
            json.dump(cache, fh)
    if not args.no_batch:
        log("batched form")
        # the batch workload (sides 256..1024), and small lattices (32..128)
        # whose single launches leave most of the GPU idle
        result["batch"] = batch_throughput()
        log("batch", result["batch"])
        result["batch_small"] = batch_throughput(steps=2000, warmup=200, count=64, lo=32, hi=128)
        log("batch_small", result["batch_small"])
    if not args.no_surrogate:
        log("surrogate throughput")
        result["surrogate"] = surrogate_throughput()
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
