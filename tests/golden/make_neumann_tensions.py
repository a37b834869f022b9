"""Write neumann_tensions.json: the oracle's own Laplace tensions of the three
interfaces of the Neumann-lens parameters (test infrastructure; calls only
the oracle).

Laplace's law (the paper's tension measurement, stated with Fig. 2): a
relaxed 2D drop of radius R has a bulk pressure jump dp = dp0 + gamma / R,
with the bulk pressure p = rho mu_rho + phi mu_phi - f_B of the free energy.
dp0 is the lattice's pressure offset across an interface two to four nodes
wide (it vanishes in the continuum); it and gamma are fitted by least squares
over three radii.  Drops of liquid 1 in liquid 2 ("12"), liquid 1 in gas
("1g") and liquid 2 in gas ("2g").

Run from the repository root: python -m tests.golden.make_neumann_tensions
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402

# the lens parameters: Maxwell density ratio 3, lambda_i = kappa_i = 0.1
# (liquid-liquid interface 2 nodes wide), the paper's lambda1, kappa1, chi
RATIO, KAPPA, LAMBDA = 3.0, 0.1, 0.1
N, RADII, STEPS = 160, (24.0, 32.0, 40.0), 20000


def params():
    return O.coexisting_params(RATIO, lattice=0, nx=N, ny=N, nz=1, kappa2=KAPPA, kappa3=KAPPA,
                               lambda2=LAMBDA, lambda3=LAMBDA)


def fields(kind, c, rg, rl, chi):
    if kind == "12":
        return np.full(c.shape, rl), chi * (2.0 * c - 1.0)
    if kind == "2g":
        return rg + (rl - rg) * c, -chi * c
    return rg + (rl - rg) * c, chi * c


def laplace(p, kind, rg, rl):
    yy, xx = np.mgrid[0:N, 0:N]
    rr = np.hypot(xx - N / 2, yy - N / 2)
    dps, rads = [], []
    for R in RADII:
        c = 0.5 * (1.0 - np.tanh((rr - R) / 2.0))
        rho, phi = fields(kind, c, rg, rl, p.chi)
        st = O.State(p, rho[None], phi[None])
        st.run(STEPS)
        f = st.fields()
        r, ph = f["rho"][0], f["phi"][0]
        c0 = N // 2
        pin = O.bulk_pressure(p, r[c0 - 1:c0 + 2, c0 - 1:c0 + 2].mean(), ph[c0 - 1:c0 + 2, c0 - 1:c0 + 2].mean())
        pout = O.bulk_pressure(p, r[0:3, 0:3].mean(), ph[0:3, 0:3].mean())
        ind = (ph / p.chi + 1.0) / 2.0 if kind == "12" else (r - r[0:3, 0:3].mean()) / (r[c0, c0] - r[0:3, 0:3].mean())
        dps.append(pin - pout)
        rads.append(math.sqrt(ind.sum() / math.pi))
        print(kind, R, dps[-1], rads[-1], flush=True)
    A = np.stack([1.0 / np.array(rads), np.ones(len(rads))], axis=1)
    g, off = np.linalg.lstsq(A, np.array(dps), rcond=None)[0]
    return float(g), float(off), dps, rads


def main():
    O.build(force=False)
    p = params()
    rg, rl = O.discrete_coexistence(p, steps=20000, n=256)
    out = {"ratio": RATIO, "kappa": KAPPA, "lambda": LAMBDA, "box": N, "radii": RADII, "steps": STEPS,
           "start_densities": [rg, rl], "tensions": {}, "offsets": {}, "raw": {}}
    for kind in ("12", "1g", "2g"):
        g, off, dps, rads = laplace(p, kind, rg, rl)
        out["tensions"][kind] = g
        out["offsets"][kind] = off
        out["raw"][kind] = {"dp": dps, "R": rads}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "neumann_tensions.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(out["tensions"])


if __name__ == "__main__":
    main()
