"""Equilibrium detector used to judge a run.

The observables are the interface measures L_k = sum_x |grad s_k| of the
scaled density s_0 = (rho - rho_g)/(rho_l - rho_g) and of the two liquid
concentrations s_1 = C1, s_2 = C2 (central differences, periodic): in two
dimensions they are the lengths of the liquid-gas outline and of each
liquid's outline.  Relaxation to the equilibrium lens (or engulfed drop)
lowers them toward their final values.  They do not change when the whole
structure drifts, which it does slowly through the periodic box, so a
pointwise field difference is no test of settling.  The velocity is no test
either: near the triple points the spurious currents stay at O(1e-3) in
lattice units at a density ratio of 10.

The detector fires when every L_k changes by less than `tol` (relative)
over each of `patience` consecutive windows of steps (capillary waves make
a single quiet window a poor sign); the steps counted are those at the end
of the first quiet window.  Analysis only; the state is read back through
the library.
"""
from __future__ import annotations

import dataclasses
from typing import List, Tuple

import numpy as np


@dataclasses.dataclass
class Detector:
    window: int = 500
    tol: float = 1e-3
    max_steps: int = 60000
    patience: int = 2


def _grad_norm_sum(s: np.ndarray) -> float:
    g2 = np.zeros_like(s)
    for ax in range(s.ndim):
        if s.shape[ax] > 1:
            d = 0.5 * (np.roll(s, -1, axis=ax) - np.roll(s, 1, axis=ax))
            g2 += d * d
    return float(np.sum(np.sqrt(g2)))


def interface_measures(rho: np.ndarray, phi: np.ndarray, rho_g: float, rho_l: float,
                       chi: float = 5.0) -> np.ndarray:
    s = (np.squeeze(rho) - rho_g) / (rho_l - rho_g)
    q = np.squeeze(phi) / chi
    return np.array([_grad_norm_sum(s), _grad_norm_sum(0.5 * (s + q)), _grad_norm_sum(0.5 * (s - q))])


def measures_of(solver, rho_g, rho_l, chi=5.0) -> np.ndarray:
    return interface_measures(solver.read("rho"), solver.read("phi"), rho_g, rho_l, chi)


def run_to_equilibrium(solver, rho_g: float, rho_l: float, chi: float = 5.0, det: Detector = Detector(),
                       trace=None) -> Tuple[int, List[float]]:
    """Step `solver` in windows until the detector fires.  Returns the steps
    taken (max_steps + window if it never fires) and the per-window largest
    relative change of the interface measures."""
    prev = measures_of(solver, rho_g, rho_l, chi)
    steps = 0
    hist = []
    quiet = 0
    while steps < det.max_steps + det.window * (det.patience - 1):
        solver.step(det.window)
        steps += det.window
        cur = measures_of(solver, rho_g, rho_l, chi)
        ch = float(np.max(np.abs(cur - prev) / np.maximum(cur, 1e-30)))
        hist.append(ch)
        if trace:
            trace(steps, ch, cur)
        quiet = quiet + 1 if ch < det.tol else 0
        if quiet >= det.patience:
            return steps - det.window * (det.patience - 1), hist
        prev = cur
    return det.max_steps + det.window, hist
