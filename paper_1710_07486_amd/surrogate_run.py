"""Train and judge the surrogate of one family end to end on the GPU.

    python -m paper_1710_07486_amd.surrogate_run --family lens --out result.json

Generates trajectories with the batched solver, trains the network with the
library's kernels, evaluates held-out prediction error, and compares
surrogate-started runs with plain runs (steps to the judged equilibrium,
lead time, wall time including inference).  Prints progress lines and
writes one JSON document.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--family", default="lens")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--train", type=int, default=256, help="training trajectories")
    ap.add_argument("--jumps", type=int, default=3, help="chained pairs per training trajectory")
    ap.add_argument("--held", type=int, default=16, help="held-out trajectories for the MSE")
    ap.add_argument("--iters", type=int, default=8000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--compare", type=int, default=8, help="held-out seeds judged against plain runs")
    ap.add_argument("--ref-steps", type=int, default=40000)
    ap.add_argument("--window", type=int, default=500)
    ap.add_argument("--tol", type=float, default=1e-2)
    ap.add_argument("--out", default=None)
    ap.add_argument("--save-net", default=None)
    a = ap.parse_args(argv)

    import torch
    from . import surrogate as S

    def log(msg):
        print(msg, flush=True)

    fam = S.Family(**{**S.FAMILIES[a.family].__dict__, "n": a.n, "jumps": a.jumps})
    res = {"family": fam.__dict__.copy(), "dilations": list(S.DILATIONS)}
    t0 = time.time()
    ph = S.physics(fam)
    res["physics"] = ph.__dict__.copy()
    log(f"physics {ph}")
    t = time.time()
    data = S.generate(fam, list(range(10000, 10000 + a.train)), ph)
    held = S.generate(fam, list(range(20000, 20000 + a.held)), ph)
    torch.cuda.synchronize()
    res["generate_s"] = time.time() - t
    log(f"generated {len(data)} + {len(held)} pairs in {res['generate_s']:.1f} s")
    net = S.Network(seed=0)
    t = time.time()
    hist = S.train(net, data, a.iters, batch=a.batch, lr=a.lr, lr_final=a.lr / 20,
                   log_every=max(1, a.iters // 10), log=log)
    torch.cuda.synchronize()
    res["train_s"] = time.time() - t
    res["train_mse_history"] = hist
    flop = 3 * S.flops_per_pixel(True) * a.batch * fam.n * fam.n * a.iters
    res["train_tflops"] = flop / res["train_s"] / 1e12
    mp, m0, cp, c0 = S.evaluate(net, held, per_channel=True)
    res["heldout_mse"] = {"surrogate": mp, "identity": m0, "ratio": mp / m0,
                          "per_channel_surrogate": cp.tolist(), "per_channel_identity": c0.tolist()}
    log(f"held-out MSE {mp:.3e} vs identity {m0:.3e} (ratio {mp / m0:.3f})")
    if a.save_net:
        np.savez(a.save_net, **net.state_dict())
    runs = []
    for seed in range(20000, 20000 + a.compare):
        t = time.time()
        r = S.compare_to_plain(net, fam, seed, ph, a.ref_steps, window=a.window, tol=a.tol, jumps=1, log=log)
        r["wall_s"] = time.time() - t
        runs.append({k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in r.items()
                     if k not in ("plain_distance", "surrogate_distance")})
    # inference wall time of one jump at this size
    import torch as _t
    r0, f0 = S.initial_fields(fam, 20000, ph)
    rt, ft = _t.from_numpy(r0).cuda(), _t.from_numpy(f0).cuda()
    S.jump(net, rt, ft, ph)
    _t.cuda.synchronize()
    t = time.time()
    for _ in range(10):
        S.jump(net, rt, ft, ph)
    _t.cuda.synchronize()
    res["jump_ms"] = (time.time() - t) * 100.0
    res["runs"] = runs
    ok = [r for r in runs if r["gain_steps"] is not None]
    res["summary"] = {
        "fallbacks": sum(r["fallback"] for r in runs),
        "settled_both": len(ok),
        "mean_plain_steps": float(np.mean([r["plain_steps"] for r in ok])) if ok else None,
        "mean_surrogate_steps": float(np.mean([r["surrogate_steps"] for r in ok])) if ok else None,
        "mean_gain_steps": float(np.mean([r["gain_steps"] for r in ok])) if ok else None,
        "mean_lead_steps": float(np.mean([r["lead_steps"] for r in runs if "lead_steps" in r])),
    }
    res["total_s"] = time.time() - t0
    log(json.dumps(res["summary"]))
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1, default=float)
    return 0


if __name__ == "__main__":
    sys.exit(main())
