"""Equilibrium detectors used to judge a run.

The observables are shape measures: for the scaled density s_0 = (rho -
rho_g)/(rho_l - rho_g) and the two liquid concentrations s_1 = C1, s_2 =
C2, L_k = sum_x |grad r(s_k)| with the indicator ramp r(v) = clip((v -
1/4)/(1/2), 0, 1) (central differences, periodic).  In two dimensions L_0 is
the length of the liquid-gas outline and L_1, L_2 those of each liquid's
outline.  The ramp is flat in the bulk phases, so the measures see the
shapes and not the slow drift of the bulk densities toward the curved-
interface coexistence values; and they do not change when the whole
structure drifts through the periodic box, which it does slowly.  The
velocity is no test either: near the triple points the spurious currents
stay at O(1e-3) in lattice units at a density ratio of 10.

Two detectors:
  - online (run_to_equilibrium): fires when every L_k changes by less than
    `tol` (relative) over each of `patience` consecutive windows of steps
    (capillary waves make a single quiet window a poor sign);
  - judged (settle_step): given a run's trajectory of measures and the
    equilibrium measures of a long plain reference run, the first step from
    which every L_k stays within `tol` (relative) of its equilibrium value
    until the end of the trajectory.
Analysis only; the state is read back through the library.
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


def _ramp(v: np.ndarray) -> np.ndarray:
    return np.clip((v - 0.25) / 0.5, 0.0, 1.0)


def _grad_norm_sum(s: np.ndarray) -> float:
    s = _ramp(s)
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


def trajectory(solver, steps: int, window: int, rho_g: float, rho_l: float, chi: float = 5.0) -> np.ndarray:
    """Interface measures at t = 0, window, 2 window, ..., steps (rows)."""
    out = [measures_of(solver, rho_g, rho_l, chi)]
    for _ in range(steps // window):
        solver.step(window)
        out.append(measures_of(solver, rho_g, rho_l, chi))
    return np.array(out)


def distance(traj: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-row largest relative distance of the measures to `ref`."""
    return np.max(np.abs(traj - ref[None, :]) / np.maximum(np.abs(ref[None, :]), 1e-30), axis=1)


def settle_step(traj: np.ndarray, ref: np.ndarray, tol: float, window: int) -> int:
    """First step from which the trajectory stays within tol of ref; -1 if
    it never settles (its last point is outside)."""
    d = distance(traj, ref)
    outside = np.nonzero(d >= tol)[0]
    if outside.size == 0:
        return 0
    k = int(outside[-1]) + 1
    return -1 if k >= len(d) else k * window
