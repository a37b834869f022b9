"""Benchmark of the ternary free-energy entropic LBM update on one MI355X.

Headline workload: D3Q27 256^3 periodic box, binary collision of a liquid-1
and a liquid-2 drop (radius 32) in gas at a lattice liquid/gas density ratio
of 800 (the temperature at which the lattice model's relaxed flat interface
holds that ratio; its Maxwell ratio, 6,715, is reported beside it; at a
lattice ratio of 1000 this drop start diverges), FP64.  `value` is the whole-job MLUPS of exactly --steps timed steps
after --warmup untimed ones (one HIP event pair around them on the solver's
stream), with the conservation diagnostics every 100 steps inside the timed
region.  `roofline` is that of the step's dominant kernel (the collision,
k_collide_next3), from HIP events around each of its launches over as many
steps again, right after the timed region (events around every launch would
lengthen a step: by 7 us on a 77 us D2Q9 step).

Extra legs (each with its own roofline object where it has a dominant
kernel): the FP32-mixed form of the same box, the D2Q9 1024^2 drops in FP64
and FP32-mixed (with the FP32-mixed error against FP64 after 20,000 steps per
field), other free energies, walls, the reduced phase-field lattice, the
batched form, the surrogate's MFMA kernels, and the FP64 oracle on the host
cores on a bounded sample of the headline workload.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak, TFLOP/s
METRIC = "ternary ELBM MLUPS & % HBM roofline; FP32-mixed vs FP64 at stated error"

# HBM bytes per launch of the dominant kernel of each step, from two rocprofv3
# counter passes (FETCH_SIZE, then WRITE_SIZE, each scaled by what the same
# counter reads for a 1 GiB device copy in the same run: x2.0 and x1.0),
# valid only for the kernel sources whose hash is recorded with them
# (profiles/step_kernels_d3q27_256_d2q9_1024_stats_and_traffic.md): the D3Q27
# 256^3 FP64 collision of a step without diagnostics, the FP32 pair-split
# collision, the D2Q9 1024^2 one-launch steps, and the two kernels of a
# three-liquid D3Q27 step together.
TRAFFIC = {
    "d3q27_fp64_collide": {"bytes_per_launch": 16640641082, "sources_sha256_16": "9b98837135b95332"},
    "d3q27_fp32_collide": {"bytes_per_launch": 9809648396, "sources_sha256_16": "9b98837135b95332"},
    "d2q9_fp64_step": {"bytes_per_launch": 348253973, "sources_sha256_16": "9b98837135b95332"},
    "d2q9_fp32_step": {"bytes_per_launch": 213560016, "sources_sha256_16": "9b98837135b95332"},
    "d3q27_three_liquid_step": {"bytes_per_launch": 26384209065, "sources_sha256_16": "9b98837135b95332"},
}


# The sources of the step kernels the stored traffic was counted on (the
# kernel files and every local header they include).
KERNEL_SOURCES = ("kernels.hip", "kernels.hpp", "node_ops.hpp", "lattice.hpp", "next_sums.hpp", "nliquid.hip")


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1710_07486_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_of(key):
    t = TRAFFIC.get(key)
    return t["bytes_per_launch"] if t and t["sources_sha256_16"] == kernel_sources_hash() else None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def temperature_of(wl, eos=None):
    import paper_1710_07486_amd as T_
    return wl.T if wl.T else T_.temperature_for_ratio(wl.ratio, **(eos or {}))


def library_params(T, wl, precision, eos=None, extra=None, diag_every=0):
    """Solver parameters of workload `wl`; `eos` optionally names another free
    energy as {"eos": kind, "a": a, "b": b}; `extra` adds fields (walls,
    contact angles, glattice)."""
    import paper_1710_07486_amd as T_
    nz, ny, nx = wl.shape
    ph = wl.physics()
    return T_.Params(lattice=wl.lattice, precision=precision, nx=nx, ny=ny, nz=nz, T=T,
                     lambda1=ph["lambda1"], lambda2=ph["lambda2"], lambda3=ph["lambda3"],
                     kappa1=ph["kappa1"], kappa2=ph["kappa2"], kappa3=ph["kappa3"], chi=ph["chi"],
                     nu=ph["nu"], mobility=ph["mobility"], tau_phi=ph["tau_phi"], walls=ph.get("walls", 0),
                     diag_every=diag_every, **(eos or {}), **(extra or {}))


def ratios(wl, T, coex, eos=None):
    """Maxwell and lattice density ratios of a workload at temperature T."""
    import paper_1710_07486_amd as T_
    e = eos or {}
    rg, rl, _, _ = T_.coexistence(T, e.get("a", 0.037), e.get("b", 0.2), 1.0, e.get("eos", 0))
    tc = T_.critical_temperature(e.get("a", 0.037), e.get("b", 0.2), 1.0, e.get("eos", 0))
    out = {"T": T, "T_over_Tc": round(T / tc, 6), "density_ratio_maxwell": round(rl / rg, 1)}
    if coex and coex[0]:
        out["density_ratio_lattice"] = round(coex[1] / coex[0], 1)
        out["coexisting_densities_lattice"] = [round(coex[0], 6), round(coex[1], 5)]
    return out


def measure(wl, precision, steps, warmup, fields=None, coex=None, eos=None, extra=None, diag_every=0,
            keep=False):
    """Exactly `steps` timed steps after `warmup` untimed ones, timed by one
    HIP event pair on the solver's stream (the time per step), then as many
    steps again with an event pair around every kernel launch (the mean
    duration of each kernel kind).  Drops start at the discretised model's
    own coexistence densities (a 1D slab relaxed by the library, unless
    `coex` gives them)."""
    import torch
    import paper_1710_07486_amd as T_
    from paper_1710_07486_amd.calibrate import discrete_coexistence
    from synth import workloads as W
    T = temperature_of(wl, eos)
    p = library_params(T, wl, precision, eos, extra, diag_every)
    if fields is None:
        slab = library_params(T, wl, T_.FP64, eos)
        slab.walls = 0
        coex = coex if coex else discrete_coexistence(slab)
        log("lattice coexistence densities", coex)
        fields = W.fields(wl, coex[0], coex[1])
    rho, phi, u = fields
    s = T_.Solver(p)
    uu = u if np.abs(u).max() > 0 else None
    s.init_fields(rho, phi, uu)
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    span_ms = e0.elapsed_time(e1) / steps
    d = s.diagnostics(check=False)
    kern, inst_ms = s.time_kernels(steps, span=True)
    torch.cuda.synchronize()
    out = {"mlups": wl.nodes / (span_ms * 1e-3) / 1e6, "ms_per_step": span_ms, "kernels_ms": kern,
           "instrumented_ms_per_step": inst_ms, "host_wall_s": wall,
           "bytes_per_update": s.algorithmic_bytes_per_update(), "diag": d,
           "coex": list(coex) if coex else None, "steps_taken": s.steps, "T": T}
    out["rho"] = s.read("rho", check=False)
    if keep:
        out["solver"] = s
    else:
        s.close()
        del s
        torch.cuda.empty_cache()
    return out, fields


def roofline_of(r, nodes, kernel_name, kind="collide", traffic_key=None, one_launch=False):
    """HBM roofline of the dominant kernel: algorithmic bytes (read and write
    of every population once, per node) times the nodes of one launch, over
    the kernel's mean event-timed duration.  A step of one launch takes the
    time per step of the timed region instead (the kernel back to back with
    itself; the events around each launch lengthen it by a few us)."""
    ms = r["kernels_ms"][kind]
    if one_launch:
        ms = min(ms, r["ms_per_step"])
    alg = r["bytes_per_update"] * nodes
    achieved = alg / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_of(traffic_key) if traffic_key else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": kernel_name, "kernel_ms": round(ms, 5),
            "algorithmic_bytes_per_launch": int(alg),
            "algorithmic_bytes_per_node": r["bytes_per_update"]}


def precision_errors(a, b, steps):
    """Errors of FP32-mixed fields `b` against FP64 fields `a` (dicts of
    numpy arrays: rho, phi, ux, uy[, uz]), per field: max-norm and mean-norm
    relative density error, the density error in the bulk phases and on the
    interfaces, phase-field and velocity errors relative to their largest
    magnitudes, and the spurious-current magnitude of both runs."""
    r64, r32 = a["rho"], b["rho"]
    rmax = np.abs(r64).max()
    # interfaces: where the FP64 density is between 1.5 rho_g and 0.95 rho_l
    lo, hi = r64.min(), r64.max()
    iface = (r64 > 1.5 * lo) & (r64 < 0.95 * hi)
    bulk = ~iface
    dr = np.abs(r32 - r64)
    u64 = np.stack([a[k] for k in ("ux", "uy", "uz") if k in a])
    u32 = np.stack([b[k] for k in ("ux", "uy", "uz") if k in b])
    m64, m32 = np.sqrt((u64 ** 2).sum(0)), np.sqrt((u32 ** 2).sum(0))
    return {"after_steps": steps,
            "rel_density_error_max_norm": float(dr.max() / rmax),
            "rel_density_error_mean_norm": float(dr.mean() / np.abs(r64).mean()),
            "rel_density_error_bulk_pointwise_max": float((dr[bulk] / np.abs(r64[bulk])).max()),
            "rel_density_error_interface_max_norm": float(dr[iface].max() / rmax) if iface.any() else 0.0,
            "rel_phase_field_error_max_norm": float(np.abs(b["phi"] - a["phi"]).max() / np.abs(a["phi"]).max()),
            "rel_velocity_error_max_norm": float(np.abs(u32 - u64).max() / max(m64.max(), 1e-300)),
            "spurious_current_max_fp64": float(m64.max()), "spurious_current_max_fp32_mixed": float(m32.max()),
            "interface_nodes": int(iface.sum())}


def fp32_horizon(wl, fields, steps):
    """FP64 and FP32-mixed runs of `steps` steps from the same start: the
    precision form's error per field at that horizon."""
    import torch
    import paper_1710_07486_amd as T_
    T = temperature_of(wl)
    out = {}
    for tag, prec in (("fp64", T_.FP64), ("fp32", T_.FP32_MIXED)):
        s = T_.Solver(library_params(T, wl, prec))
        s.init_fields(*fields[:2], None)
        s.step(steps)
        out[tag] = {k: s.read(k, check=False) for k in ("rho", "phi", "ux", "uy")}
        s.close()
        del s
        torch.cuda.empty_cache()
    return precision_errors(out["fp64"], out["fp32"], steps)


def batch_throughput(steps=100, warmup=10, count=64, lo=256, hi=1024):
    """The batching form: `count` uneven D2Q9 instances (sides U{256..1024},
    Maxwell ratio U[100, 1000], FP32-mixed) advanced together (the mode, tile
    shape and workgroups per CU from the autotuner's timed sweep), against
    the same instances advanced one after another by the single-instance
    solver.  Aggregate MLUPS both ways."""
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
            "density_ratio": "Maxwell U[100, 1000]",
            "batched_mlups": round(nodes / ms / 1e3, 2),
            "ms_per_step": round(ms, 4), "one_by_one_mlups": round(nodes / seq_ms / 1e3, 2),
            "speedup_vs_one_by_one": round(seq_ms / ms, 3),
            "whole_step_hbm_frac": round(nodes / ms / 1e3 * 1e6 * 144 / (HBM_PEAK_GBS * 1e9), 4),
            "mode": {0: "persistent three-phase", 1: "fused per instance", 2: "fused, one launch"}[rec.get("mode", 0)],
            "persistent_best_mlups": round(nodes / min(r["ms_per_step"] for r in rec["table"] if r["mode"] == 0) / 1e3, 2),
            "tile_shape": rec["shape"], "wg_per_cu": rec["wg_per_cu"],
            "finite": finite}


def cpu_baseline(wl, coex, budget_s=20.0):
    """The FP64 oracle on the host cores, on a bounded number of time steps
    of the full headline lattice (same temperature and starting densities)."""
    from oracle import oracle as O
    from synth import workloads as W
    O.build(force=False)
    p = O.workload_params(wl)
    rho, phi, u = W.fields(wl, coex[0], coex[1])
    st = O.State(p, rho, phi, u if np.abs(u).max() > 0 else None)
    t0 = time.perf_counter()
    st.run(1)
    t1 = time.perf_counter()
    n = max(1, min(200, int(budget_s / max(t1 - t0, 1e-3))))
    t0 = time.perf_counter()
    st.run(n)
    dt = time.perf_counter() - t0
    return {"value": round(wl.nodes * n / dt / 1e6, 3), "unit": "MLUPS", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{wl.name}: {n} time steps of the full {'x'.join(map(str, wl.shape[::-1]))} lattice "
                      f"after one warm-up step (FP64 oracle, OpenMP, {dt:.1f} s)"}


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
            "roofline": {"bound": "mfma", "kernel": "k_conv_lds 64->64 forward (bf16)", "achieved": round(conv_tf, 1),
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


def nliquid_throughput(wl3, coex, steps, warmup):
    """Three liquids and the gas on the 3D workload: its second drop is
    liquid 3 (psi = chi) and liquid 2 is absent, liquid 3 with liquid 2's
    lambda and kappa.  FP64, two launches per step (the collision that leaves
    the next moments as partial sums, then the pass that completes them and
    computes the potentials), timed with an event pair around the `steps`
    timed steps on the solver's stream."""
    import torch
    import paper_1710_07486_amd as T_
    from paper_1710_07486_amd import nliquid as NL
    from synth import workloads as W
    T = temperature_of(wl3, None)
    p = library_params(T, wl3, T_.FP64, None, None, 0)
    rho, phi, u = W.fields(wl3, coex[0], coex[1])
    psi = np.maximum(-phi, 0.0)
    phi = np.maximum(phi, 0.0)
    s = NL.NLSolver(p, NL.NLParams(lambda4=p.lambda2, kappa4=p.kappa2))
    s.init_fields(rho, phi, psi, u if np.abs(u).max() > 0 else None)
    del rho, phi, psi, u
    s.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    c3 = s.read("c3")
    finite = bool(np.isfinite(c3).all())
    per_node = 2.0 * 3 * 27 * 8  # read and write of f, g and h once
    achieved = per_node * wl3.nodes / (ms * 1e-3) / 1e9
    out = {"workload": wl3.name + "_liquid3", "lattice": "D3Q27, f + two phase-field lattices",
           "mlups": round(wl3.nodes / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 4),
           "steps": steps, "warmup": warmup, "launches_per_step": 2,
           "whole_step_roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                                   "algorithmic_bytes_per_node": per_node,
                                   "traffic": traffic_of("d3q27_three_liquid_step"),
                                   "traffic_unit": "HBM bytes per step, its two kernels (rocprofv3 FETCH_SIZE + "
                                                   "WRITE_SIZE, copy-calibrated)"},
           "liquid3_max_c": round(float(c3.max()), 4), "finite": finite}
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


LEGS = ("fp32", "2d", "eos", "walls", "reduced", "nliquid", "batch", "surrogate", "cpu")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=20, help="untimed steps before them")
    ap.add_argument("--steps2d", type=int, default=1000, help="timed steps of the D2Q9 legs")
    ap.add_argument("--horizon", type=int, default=20000, help="steps of the FP32-mixed vs FP64 error run (2D)")
    ap.add_argument("--skip", default="", help="comma-separated legs to skip: " + ",".join(LEGS))
    ap.add_argument("--only-headline", action="store_true", help="skip every extra leg")
    ap.add_argument("--coex3d", type=float, nargs=2, metavar=("RHO_G", "RHO_L"),
                    help="lattice coexistence densities of the 3D workload (skips their calibration run)")
    ap.add_argument("--coex2d", type=float, nargs=2, metavar=("RHO_G", "RHO_L"),
                    help="lattice coexistence densities of the 2D workload (skips their calibration run)")
    ap.add_argument("--copy-probe", action="store_true", help="run a 1 GiB device copy first (counter scale)")
    args = ap.parse_args()
    skip = set(LEGS) if args.only_headline else set(filter(None, args.skip.split(",")))
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1710_07486_amd as T_
    from synth import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.copy_probe:
        copy_probe()
    wl3 = W.collision_3d(256, radius=32, ratio=800.0, v_rel=0.04, kappa2=0.2, kappa3=0.2, lattice_ratio=True)
    log("workload", wl3.name, "steps", args.steps, "warmup", args.warmup)
    r3, f3 = measure(wl3, T_.FP64, args.steps, args.warmup, coex=args.coex3d, diag_every=100)
    log("fp64 3d", {k: v for k, v in r3.items() if k != "rho"})
    cfg = {"workload": wl3.name, "lattice": "D3Q27", "nx": 256, "ny": 256, "nz": 256, "drop_radius": 32,
           "relative_velocity": 0.04, "precision": "fp64", "diag_every": 100, "parallelism": "single GPU"}
    cfg.update(ratios(wl3, r3["T"], r3["coex"]))
    result = {
        "metric": METRIC,
        "value": round(r3["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r3["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded drops, SplitMix64 noise)",
        "config": cfg,
        "roofline": roofline_of(r3, wl3.nodes, "k_collide_next3", traffic_key="d3q27_fp64_collide"),
        "whole_step_hbm_frac": round(r3["mlups"] * 1e6 * r3["bytes_per_update"] / (HBM_PEAK_GBS * 1e9), 4),
        "kernels_ms": {k: round(v, 5) for k, v in r3["kernels_ms"].items()},
        "ms_per_step_with_launch_events": round(r3["instrumented_ms_per_step"], 4),
        "host_wall_s_timed_region": round(r3["host_wall_s"], 4),
        "diagnostics": {k: r3["diag"][k] for k in ("mass", "max_u", "min_rho", "nonfinite")}
        if isinstance(r3["diag"], dict) else None,
    }
    if "fp32" not in skip:
        r3m, _ = measure(wl3, T_.FP32_MIXED, args.steps, args.warmup, f3, coex=r3["coex"], diag_every=100)
        log("fp32-mixed 3d", {k: v for k, v in r3m.items() if k != "rho"})
        diff = np.abs(r3m["rho"] - r3["rho"])
        result["fp32_mixed"] = {
            "workload": wl3.name, "value": round(r3m["mlups"], 2), "unit": "MLUPS",
            "speedup_vs_fp64": round(r3m["mlups"] / r3["mlups"], 3),
            "ms_per_step": round(r3m["ms_per_step"], 4),
            "kernels_ms": {k: round(v, 5) for k, v in r3m["kernels_ms"].items()},
            "roofline": roofline_of(r3m, wl3.nodes, "k_collide (pair split, fp32)",
                                    traffic_key="d3q27_fp32_collide"),
            "whole_step_hbm_frac": round(r3m["mlups"] * 1e6 * r3m["bytes_per_update"] / (HBM_PEAK_GBS * 1e9), 4),
            "rel_density_error_vs_fp64_max_norm": float(diff.max() / np.abs(r3["rho"]).max()),
            "rel_density_error_vs_fp64_mean_norm": float(diff.mean() / np.abs(r3["rho"]).mean()),
            "error_after_steps": r3m["steps_taken"]}
    if "2d" not in skip:
        wl = W.drops_2d(1024, ratio=1000.0, seed=0, lattice_ratio=True)
        log("workload", wl.name)
        r64, fields = measure(wl, T_.FP64, args.steps2d, 200, coex=args.coex2d, diag_every=100)
        log("fp64 2d", {k: v for k, v in r64.items() if k != "rho"})
        d2 = {"workload": wl.name, "fp64_mlups": round(r64["mlups"], 2),
              "fp64_ms_per_step": round(r64["ms_per_step"], 5),
              "fp64_roofline": roofline_of(r64, wl.nodes, "k_collide_fused2 (fp64, one launch per step)",
                                           traffic_key="d2q9_fp64_step", one_launch=True),
              "fp64_kernels_ms": {k: round(v, 5) for k, v in r64["kernels_ms"].items()}}
        d2.update(ratios(wl, r64["T"], r64["coex"]))
        if "fp32" not in skip:
            r32, _ = measure(wl, T_.FP32_MIXED, args.steps2d, 200, fields, coex=r64["coex"], diag_every=100)
            log("fp32-mixed 2d", {k: v for k, v in r32.items() if k != "rho"})
            d2["fp32_mixed_mlups"] = round(r32["mlups"], 2)
            d2["fp32_mixed_speedup_vs_fp64"] = round(r32["mlups"] / r64["mlups"], 3)
            d2["fp32_mixed_roofline"] = roofline_of(r32, wl.nodes, "k_collide_fused2 (fp32-mixed, one launch per step)",
                                                    traffic_key="d2q9_fp32_step", one_launch=True)
            d2["fp32_mixed_kernels_ms"] = {k: round(v, 5) for k, v in r32["kernels_ms"].items()}
            d2["fp32_mixed_error_vs_fp64"] = fp32_horizon(wl, fields, args.horizon)
            log("fp32 horizon", d2["fp32_mixed_error_vs_fp64"])
        result["d2q9_1024"] = d2
        if "reduced" not in skip:
            rr, _ = measure(wl, T_.FP64, args.steps2d, 200, fields, coex=r64["coex"], extra={"glattice": 1})
            log("reduced g lattice 2d", {k: v for k, v in rr.items() if k != "rho"})
            d2["reduced_g_lattice"] = {"lattice": "D2Q9 + D2Q5", "fp64_mlups": round(rr["mlups"], 2),
                                       "vs_full": round(rr["mlups"] / r64["mlups"], 3),
                                       "bytes_per_update": rr["bytes_per_update"],
                                       "collide_ms": round(rr["kernels_ms"]["collide"], 5)}
        if "eos" not in skip:
            # the same drops with the other two free energies: Peng-Robinson at
            # Maxwell ratio 1000; van der Waals at 100, since its moving drops at
            # 1000 diverge (the oracle's too, for a = 0.5/49 .. 1/49)
            d2["other_eos"] = {}
            for name, e, ratio in (("van_der_waals", {"eos": T_.EOS_VDW, "a": 2.0 / 49.0, "b": 2.0 / 21.0}, 100.0),
                                   ("peng_robinson", {"eos": T_.EOS_PR, "a": 2.0 / 49.0, "b": 2.0 / 21.0}, 1000.0)):
                wle = W.drops_2d(1024, ratio=ratio, seed=0)
                re_, _ = measure(wle, T_.FP64, args.steps2d, 200, eos=e)
                log(name, {k: v for k, v in re_.items() if k != "rho"})
                d2["other_eos"][name] = {"workload": wle.name, "a": e["a"], "b": e["b"],
                                         "fp64_mlups": round(re_["mlups"], 2),
                                         "vs_carnahan_starling": round(re_["mlups"] / r64["mlups"], 3),
                                         "collide_ms": round(re_["kernels_ms"]["collide"], 5),
                                         "finite": bool(np.isfinite(re_["rho"]).all())}
                d2["other_eos"][name].update(ratios(wle, re_["T"], re_["coex"], e))
        if "walls" not in skip:
            # a channel between wetting walls (60 / 120 degrees), caps of liquid
            # 1 and 2 on the walls, same size and temperature as the drops
            wlw = W.wall_drops(1024, 1024, radius=200.0, ratio=1000.0)
            wlw.T = wl.T
            ang = {"theta_rho_lo": math.radians(60.0), "theta_phi_lo": math.radians(60.0),
                   "theta_rho_hi": math.radians(120.0), "theta_phi_hi": math.radians(120.0)}
            d2["walls"] = {"workload": wlw.name, "angles_deg": [60.0, 120.0]}
            for tag, prec in (("fp64", T_.FP64), ("fp32_mixed", T_.FP32_MIXED)):
                rw, _ = measure(wlw, prec, args.steps2d, 200, coex=r64["coex"], extra=ang)
                log("walls", tag, {k: v for k, v in rw.items() if k != "rho"})
                d2["walls"][tag + "_mlups"] = round(rw["mlups"], 2)
                d2["walls"][tag + "_finite"] = bool(np.isfinite(rw["rho"]).all())
    if "reduced" not in skip:
        r3r, _ = measure(wl3, T_.FP64, args.steps, args.warmup, f3, coex=r3["coex"], extra={"glattice": 1})
        log("reduced g lattice 3d", {k: v for k, v in r3r.items() if k != "rho"})
        result["d3q27_reduced_g_lattice"] = {"lattice": "D3Q27 + D3Q7", "fp64_mlups": round(r3r["mlups"], 2),
                                             "vs_full": round(r3r["mlups"] / r3["mlups"], 3),
                                             "bytes_per_update": r3r["bytes_per_update"],
                                             "kernels_ms": {k: round(v, 5) for k, v in r3r["kernels_ms"].items()}}
    if "nliquid" not in skip:
        result["three_liquids"] = nliquid_throughput(wl3, r3["coex"], args.steps, args.warmup)
        log("three liquids", result["three_liquids"])
    if "batch" not in skip:
        log("batched form")
        # the batch workload (sides 256..1024), and small lattices (32..128)
        # whose single launches leave most of the GPU idle
        result["batch"] = batch_throughput()
        log("batch", result["batch"])
        result["batch_small"] = batch_throughput(steps=2000, warmup=200, count=64, lo=32, hi=128)
        log("batch_small", result["batch_small"])
    if "surrogate" not in skip:
        log("surrogate throughput")
        result["surrogate"] = surrogate_throughput()
    if "cpu" not in skip:
        log("cpu baseline (oracle)")
        torch.cuda.empty_cache()
        result["cpu_baseline"] = cpu_baseline(wl3, r3["coex"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
