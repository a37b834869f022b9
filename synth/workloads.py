"""Named synthetic workloads shaped like the paper's simulations.

The paper simulates a liquid lens (Fig. 2), liquid-gas coexistence over
temperature (Fig. 3) and binary collisions of immiscible drops (Figs. 4-5),
but gives no grid sizes.  These workloads stand in for them.  Shared free
energy parameters follow the paper's lens caption and text: lambda1 = 0.6,
kappa1 = 1e-3, lambda_i = 3.125 kappa_i, chi = 5, nu = 0.167, M = 0.5.

A workload names its liquid/gas density ratio.  By default that is the
Maxwell ratio of the equation of state, and the temperature and coexisting
densities that realise it are computed by whoever consumes the workload (the
oracle in tests, the library in the benchmark).  A workload built with
``lattice_ratio=True`` instead carries a fixed temperature ``T`` at which the
lattice model's relaxed flat interface holds the named ratio; those
temperatures were computed once by the oracle (``python -m
oracle.lattice_ratio``) and are stored below as inputs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from .rng import uniform

D2Q9, D3Q27 = 0, 1

# Temperatures at which the relaxed flat liquid-1 slab in gas (256 nodes)
# holds the named lattice density ratio, computed by oracle.lattice_ratio.
# Keys: ("drops_2d", seed, ratio) with that seed's liquid coefficients, and
# ("collision_3d", kappa2 = kappa3, ratio).  Maxwell ratios at these
# temperatures: 12,864 and 6,715.
LATTICE_RATIO_T = {
    ("drops_2d", 0, 1000.0): 0.027515478,
    ("collision_3d", 0.2, 800.0): 0.028859406,
}


def lattice_ratio_temperature(*key) -> float:
    try:
        return LATTICE_RATIO_T[tuple(key)]
    except KeyError:
        raise KeyError(f"no lattice-ratio temperature stored for {key}")


@dataclasses.dataclass
class Workload:
    name: str
    lattice: int
    shape: tuple            # (nz, ny, nx)
    ratio: float            # liquid/gas density ratio (Maxwell's, unless T is set)
    kappa2: float
    kappa3: float
    drops: list
    steps: int
    seed: int = 0
    lambda1: float = 0.6
    kappa1: float = 1e-3
    chi: float = 5.0
    nu: float = 0.167
    mobility: float = 0.5
    tau_phi: float = 1.0
    noise: float = 1e-4
    width: float = 3.0
    walls: int = 0          # 1: solid walls at y = -1/2 and y = ny - 1/2
    T: float = 0.0          # temperature; 0: the one whose Maxwell ratio is `ratio`

    @property
    def lambda2(self) -> float:
        return 3.125 * self.kappa2

    @property
    def lambda3(self) -> float:
        return 3.125 * self.kappa3

    @property
    def nodes(self) -> int:
        return int(np.prod(self.shape))

    def physics(self) -> dict:
        """Parameters other than the EOS temperature and coexisting densities."""
        nz, ny, nx = self.shape
        return dict(lattice=self.lattice, nx=nx, ny=ny, nz=nz, lambda1=self.lambda1,
                    lambda2=self.lambda2, lambda3=self.lambda3, kappa1=self.kappa1,
                    kappa2=self.kappa2, kappa3=self.kappa3, chi=self.chi, nu=self.nu,
                    mobility=self.mobility, tau_phi=self.tau_phi, walls=self.walls)


def lens(nx: int = 128, ny: int = 128, radius: float = 20.0, ratio: float = 10.0,
         kappa: float = 0.045, steps: int = 1000, seed: int = 0) -> Workload:
    """Liquid-1 drop touching a liquid-2 drop in gas, equal liquid tensions."""
    cx, cy = nx / 2.0, ny / 2.0
    drops = [{"center": (cx - radius, cy), "radius": radius, "liquid": 1},
             {"center": (cx + radius, cy), "radius": radius, "liquid": 2}]
    return Workload(f"lens_d2q9_{nx}x{ny}_ratio{ratio:g}", D2Q9, (1, ny, nx), ratio,
                    kappa, kappa, drops, steps, seed)


def drops_2d(n: int = 1024, ratio: float = 1000.0, seed: int = 0, steps: int = 20000,
             lattice_ratio: bool = False) -> Workload:
    """Two touching drops of seeded radii in [n*80/1024, n*160/1024] and a seeded
    axis angle; liquid gradient coefficients drawn log-uniformly around 0.37,
    so that the tension ratios span partial wetting and encapsulation.  With
    ``lattice_ratio`` the temperature is the one at which a flat slab of
    liquid 1 in gas with this seed's coefficients holds ``ratio`` on the
    lattice (stored for seed 0 and ratio 1000)."""
    r = uniform(seed * 7919 + 17, 5)
    s = n / 1024.0
    R1 = s * (80.0 + 80.0 * r[0])
    R2 = s * (80.0 + 80.0 * r[1])
    ang = 2.0 * math.pi * r[2]
    k2 = 0.37 * math.exp(math.log(0.5) + (math.log(2.0) - math.log(0.5)) * r[3])
    k3 = 0.37 * math.exp(math.log(0.5) + (math.log(2.0) - math.log(0.5)) * r[4])
    c = n / 2.0
    d = 0.5 * (R1 + R2)
    drops = [
        {"center": (c - d * math.cos(ang) * R1 / d, c - d * math.sin(ang) * R1 / d), "radius": R1, "liquid": 1},
        {"center": (c + d * math.cos(ang) * R2 / d, c + d * math.sin(ang) * R2 / d), "radius": R2, "liquid": 2},
    ]
    T = lattice_ratio_temperature("drops_2d", seed, ratio) if lattice_ratio else 0.0
    tag = "latticeratio" if lattice_ratio else "ratio"
    return Workload(f"drops_d2q9_{n}x{n}_{tag}{ratio:g}_seed{seed}", D2Q9, (1, n, n), ratio,
                    k2, k3, drops, steps, seed, T=T)


def collision_3d(n: int = 256, radius: float = 32.0, ratio: float = 1000.0, v_rel: float = 0.04,
                 impact: float = 0.0, kappa2: float = 0.37, kappa3: float = 0.37,
                 steps: int = 10000, seed: int = 0, lattice_ratio: bool = False) -> Workload:
    """Binary collision of a liquid-1 and a liquid-2 drop in a periodic cube.
    With ``lattice_ratio`` (kappa2 = kappa3 required) the temperature is the
    one at which a flat slab holds ``ratio`` on the lattice."""
    shape = (n, n, n)
    off = radius + 4.0
    b = impact * 2.0 * radius
    c = n / 2.0
    drops = [
        {"center": (c - off, c - b / 2.0, c), "radius": radius, "liquid": 1,
         "velocity": (0.5 * v_rel, 0.0, 0.0)},
        {"center": (c + off, c + b / 2.0, c), "radius": radius, "liquid": 2,
         "velocity": (-0.5 * v_rel, 0.0, 0.0)},
    ]
    T = 0.0
    if lattice_ratio:
        assert kappa2 == kappa3, "lattice-ratio temperatures are stored for equal liquid coefficients"
        T = lattice_ratio_temperature("collision_3d", kappa2, ratio)
    tag = "latticeratio" if lattice_ratio else "ratio"
    return Workload(f"collision_d3q27_{n}^3_{tag}{ratio:g}_B{impact:g}", D3Q27, shape, ratio,
                    kappa2, kappa3, drops, steps, seed, T=T)


def batch_instances(count: int = 64, seed: int = 3, lo: int = 256, hi: int = 1024,
                    steps: int = 5000) -> List[Workload]:
    """Uneven 2D head-on collision instances: sides U{lo..hi}, ratio U[100, 1000],
    relative speed log-uniform (standing in for We log-U[1, 100])."""
    out = []
    r = uniform(seed, 6 * count)
    for k in range(count):
        nx = lo + int(r[6 * k] * (hi - lo + 1))
        ny = lo + int(r[6 * k + 1] * (hi - lo + 1))
        nx, ny = min(nx, hi), min(ny, hi)
        ratio = 100.0 + 900.0 * r[6 * k + 2]
        we = math.exp(math.log(100.0) * r[6 * k + 3])
        v_rel = 0.01 * math.sqrt(we / 10.0)
        R = min(nx, ny) / 8.0
        cx, cy = nx / 2.0, ny / 2.0
        off = R + 4.0
        drops = [
            {"center": (cx - off, cy), "radius": R, "liquid": 1, "velocity": (0.5 * v_rel, 0.0, 0.0)},
            {"center": (cx + off, cy), "radius": R, "liquid": 2, "velocity": (-0.5 * v_rel, 0.0, 0.0)},
        ]
        out.append(Workload(f"batch{k}_d2q9_{nx}x{ny}", D2Q9, (1, ny, nx), ratio, 0.045, 0.045,
                            drops, steps, seed * 1000 + k))
    return out


def fields(w: Workload, rho_g: float, rho_l: float, noise: Optional[float] = None):
    """(rho, phi, u) for a workload, given its coexisting densities."""
    from .fields import two_drop_fields
    return two_drop_fields(w.shape, w.drops, rho_g, rho_l, w.chi, w.seed,
                           w.noise if noise is None else noise, w.width, periodic_y=not w.walls)


def wall_drops(nx: int = 96, ny: int = 48, nz: int = 1, radius: float = 14.0, ratio: float = 10.0,
               kappa: float = 0.1, start_deg=(70.0, 110.0), steps: int = 2000, seed: int = 0) -> Workload:
    """A channel bounded by solid walls at y = -1/2 and y = ny - 1/2: a cap of
    liquid 1 on the bottom wall and one of liquid 2 on the top wall, each a
    disc of ``radius`` cut by its wall at the angle start_deg (inside the
    drop).  D3Q27 when nz > 1."""
    c0, c1 = math.cos(math.radians(start_deg[0])), math.cos(math.radians(start_deg[1]))
    zc = nz / 2.0
    drops = [
        {"center": (nx / 3.0, -0.5 - radius * c0, zc), "radius": radius, "liquid": 1},
        {"center": (2.0 * nx / 3.0, ny - 0.5 + radius * c1, zc), "radius": radius, "liquid": 2},
    ]
    return Workload(name=f"wall_drops_{'d3q27' if nz > 1 else 'd2q9'}_{nx}x{ny}x{nz}_ratio{ratio:g}",
                    lattice=D3Q27 if nz > 1 else D2Q9, shape=(nz, ny, nx), ratio=ratio, kappa2=kappa,
                    kappa3=kappa, drops=drops, steps=steps, seed=seed, width=2.0, walls=1)
