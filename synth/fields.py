"""Initial density / phase-field / velocity arrays for drop configurations.

Each drop k contributes a smooth indicator C_k = (1 - tanh((r_k - R_k)/w))/2
(minimum-image distance r_k on the periodic box).  Drops of liquid 1 and
liquid 2 sum into C1 and C2; then rho = rho_g + (rho_l - rho_g) min(1, C1+C2),
phi = chi (C1 - C2), plus i.i.d. uniform noise drawn from SplitMix64, and
u = sum_k C_k v_k.  The densities and chi are inputs: nothing here evaluates
the equation of state.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np

from .rng import uniform


def _coords(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def _min_image(d, n):
    return d - n * np.round(d / n)


def drop_indicator(shape, center: Sequence[float], radius: float, width: float = 3.0,
                   periodic_y: bool = True) -> np.ndarray:
    """Smooth indicator of a disc/ball of ``radius`` at ``center`` (x, y[, z]);
    with periodic_y False the distance along y is not wrapped (a box bounded
    by walls in y)."""
    nz, ny, nx = shape
    x, y, z = _coords(shape)
    cx, cy = center[0], center[1]
    cz = center[2] if len(center) > 2 else 0.0
    dy = _min_image(y - cy, ny) if periodic_y else y - cy
    r2 = _min_image(x - cx, nx) ** 2 + dy ** 2
    if nz > 1:
        r2 = r2 + _min_image(z - cz, nz) ** 2
    r = np.sqrt(r2)
    return 0.5 * (1.0 - np.tanh((r - radius) / width))


def two_drop_fields(shape, drops, rho_g: float, rho_l: float, chi: float, seed: int,
                    noise: float = 1e-4, width: float = 3.0, periodic_y: bool = True):
    """Fields for a list of drops.

    ``drops`` is a sequence of dicts with keys ``center``, ``radius``,
    ``liquid`` (1 or 2) and optionally ``velocity`` (3-vector).
    Returns (rho, phi, u) with shapes (nz, ny, nx), (nz, ny, nx), (3, nz, ny, nx).
    """
    c1 = np.zeros(shape)
    c2 = np.zeros(shape)
    u = np.zeros((3,) + tuple(shape))
    for d in drops:
        ind = drop_indicator(shape, d["center"], d["radius"], width, periodic_y)
        if d["liquid"] == 1:
            c1 += ind
        else:
            c2 += ind
        v = d.get("velocity")
        if v is not None:
            for a in range(min(3, len(v))):
                u[a] += ind * v[a]
    s = np.minimum(1.0, c1 + c2)
    rho = rho_g + (rho_l - rho_g) * s
    phi = chi * (c1 - c2)
    n = int(np.prod(shape))
    if noise > 0.0:
        rho = rho + uniform(seed, n, -noise, noise).reshape(shape)
        phi = phi + uniform(seed, n, -noise, noise, offset=n).reshape(shape)
    return np.ascontiguousarray(rho), np.ascontiguousarray(phi), np.ascontiguousarray(u)


def lens_drops(nx: int, ny: int, radius: float = 20.0, gap: float = 0.0):
    """Two touching drops (liquid 1 left, liquid 2 right) centred in a 2D box."""
    cx, cy = nx / 2.0, ny / 2.0
    off = radius + gap / 2.0
    return [
        {"center": (cx - off, cy), "radius": radius, "liquid": 1},
        {"center": (cx + off, cy), "radius": radius, "liquid": 2},
    ]


def collision_drops(shape, radius: float, v_rel: float, impact: float = 0.0, gap: float = 8.0):
    """Two drops approaching along x with relative speed ``v_rel``.

    ``impact`` is the impact parameter B = b / D with b the offset along y.
    """
    nz, ny, nx = shape
    cx, cy = nx / 2.0, ny / 2.0
    cz = nz / 2.0 if nz > 1 else 0.0
    off = radius + gap / 2.0
    b = impact * 2.0 * radius
    return [
        {"center": (cx - off, cy - b / 2.0, cz), "radius": radius, "liquid": 1,
         "velocity": (0.5 * v_rel, 0.0, 0.0)},
        {"center": (cx + off, cy + b / 2.0, cz), "radius": radius, "liquid": 2,
         "velocity": (-0.5 * v_rel, 0.0, 0.0)},
    ]
