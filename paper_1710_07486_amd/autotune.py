"""Autotuner of the batched form's tile shape and persistent grid size.

For every compiled tile shape (threads along x and y of a workgroup) and
every workgroups-per-CU count, the batch is stepped on the device and timed
with HIP events on its stream; a D2Q9 batch is also timed in its two fused
modes (the single solver's fused step per instance, or for all instances in
one launch).  The fastest configuration is
applied and cached in a JSON file keyed by lattice, precision, device and
problem-size class.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional, Sequence

from .batch import Batch, tile_variants

DEFAULT_CACHE = os.environ.get("TELBM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "telbm",
                                                                "tune.json"))


def cache_key(batch: Batch) -> str:
    import torch
    p0 = batch.params[0]
    nodes = sum(p.nodes for p in batch.params)
    size_class = 2 ** int(round(math.log2(max(nodes, 1))))
    dev = torch.cuda.get_device_name(0).replace(" ", "_")
    return f"lat{p0.lattice}-prec{p0.precision}-{dev}-n{size_class}-k{len(batch.params)}"


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_config(batch: Batch, variant: int, wg: int, steps: int, warmup: int) -> float:
    import torch
    batch.set_tiles(variant, wg)
    batch.step(warmup)
    batch.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    batch.step(steps)
    e1.record(batch.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(batch: Batch, steps: int = 20, warmup: int = 10, wg_options: Sequence[int] = (1, 2, 4, 8),
         cache: Optional[str] = DEFAULT_CACHE, force: bool = False) -> Dict:
    """Pick and apply the fastest (tile shape, workgroups per CU); returns the record."""
    key = cache_key(batch)
    db = _load(cache) if cache else {}
    if not force and key in db:
        rec = db[key]
        batch.set_tiles(rec["variant"], rec["wg_per_cu"])
        batch.set_mode(rec.get("mode", 0))
        return rec
    shapes = tile_variants()
    table = []
    batch.set_mode(0)
    for v, shape in enumerate(shapes):
        for wg in wg_options:
            ms = time_config(batch, v, wg, steps, warmup)
            table.append({"mode": 0, "variant": v, "shape": list(shape), "wg_per_cu": wg, "ms_per_step": ms})
    best0 = min(table, key=lambda r: r["ms_per_step"])
    if batch.params[0].lattice == 0:
        # the fused modes: one fused launch per instance, or one for all
        for mode in (1, 2):
            batch.set_mode(mode)
            ms = time_config(batch, best0["variant"], best0["wg_per_cu"], steps, warmup)
            table.append({"mode": mode, "variant": best0["variant"], "shape": best0["shape"],
                          "wg_per_cu": best0["wg_per_cu"], "ms_per_step": ms})
    best = min(table, key=lambda r: r["ms_per_step"])
    rec = {"mode": best["mode"], "variant": best["variant"], "shape": best["shape"], "wg_per_cu": best["wg_per_cu"],
           "ms_per_step": best["ms_per_step"], "table": table}
    batch.set_tiles(rec["variant"], rec["wg_per_cu"])
    batch.set_mode(rec["mode"])
    if cache:
        db[key] = rec
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, cache)
    return rec
