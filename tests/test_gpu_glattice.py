"""GPU runs on the reduced phase-field lattice (D2Q5 with D2Q9, D3Q7 with
D3Q27) against the FP64 oracle with the same lattice: FP64 within 1e-10,
FP32-mixed within 1e-5 (densities), also with walls and after reads
between steps."""
import dataclasses
import math

import numpy as np
import pytest

from synth import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b, floor=1e-300):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))


def run(orc, wl, steps, precision=0, extra=None, read_at=None):
    import paper_1710_07486_amd as T
    extra = dict(extra or {})
    po = dataclasses.replace(orc.coexisting_params(wl.ratio, **wl.physics()), glattice=1, **extra)
    rho, phi, u = W.fields(wl, po.rho_g, po.rho_l)
    uu = u if np.abs(u).max() > 0 else None
    nz, ny, nx = wl.shape
    pl = T.Params(lattice=wl.lattice, precision=precision, nx=nx, ny=ny, nz=nz, T=po.T, rho_g=po.rho_g,
                  rho_l=po.rho_l, lambda1=po.lambda1, lambda2=po.lambda2, lambda3=po.lambda3, kappa1=po.kappa1,
                  kappa2=po.kappa2, kappa3=po.kappa3, chi=po.chi, nu=po.nu, mobility=po.mobility,
                  tau_phi=po.tau_phi, walls=po.walls, glattice=1, **{k: v for k, v in extra.items() if k != "walls"})
    st = orc.State(po, rho, phi, uu)
    st.run(steps)
    fo = st.fields()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, uu)
        if read_at:
            s.step(read_at)
            s.read("phi")
            s.diagnostics(check=False)
            s.step(steps - read_at)
        else:
            s.step(steps)
        fg = s.fields()
    assert np.isfinite(fo["rho"]).all()
    e = {k: rel(fg[k], fo[k]) for k in ("rho", "phi")}
    e["u"] = rel(fg["u"], fo["u"], 1e-14)
    e["mu_rho"] = rel(fg["mu_rho"], fo["mu_rho"], 1e-3)
    print("errors", e, flush=True)
    return e


CASES_2D = [(96, 64), (100, 37), (70, 9)]


@pytest.mark.parametrize("shape", CASES_2D, ids=[f"{a}x{b}" for a, b in CASES_2D])
def test_d2q5_phase_field_fp64(orc, shape):
    nx, ny = shape
    wl = W.lens(nx, ny, radius=min(nx, ny) / 5, ratio=100.0, kappa=0.1)
    say("D2Q9 + D2Q5 FP64", shape)
    for k, v in run(orc, wl, 300).items():
        assert v <= 1e-10, (k, v)


def test_d2q5_phase_field_fp32_mixed(orc):
    wl = W.lens(96, 64, radius=12.0, ratio=100.0, kappa=0.1)
    say("D2Q9 + D2Q5 FP32-mixed")
    e = run(orc, wl, 300, precision=1)
    assert e["rho"] <= 1e-5 and e["phi"] <= 1e-5 and e["u"] <= 1e-4, e


SHAPES_3D = [(16, 18, 20), (33, 10, 7)]


@pytest.mark.parametrize("shape", SHAPES_3D, ids=[f"{a}x{b}x{c}" for a, b, c in SHAPES_3D])
def test_d3q7_phase_field_fp64(orc, shape):
    nx, ny, nz = shape
    r = 0.25 * min(shape)
    wl = W.Workload(name="box", lattice=1, shape=(nz, ny, nx), ratio=100.0, kappa2=0.1, kappa3=0.1,
                    drops=[{"center": (nx / 2 - r, ny / 2, nz / 2), "radius": r, "liquid": 1,
                            "velocity": (0.02, 0.0, 0.0)},
                           {"center": (nx / 2 + r, ny / 2, nz / 2), "radius": r, "liquid": 2,
                            "velocity": (-0.02, 0.0, 0.0)}], steps=40, seed=3)
    say("D3Q27 + D3Q7 FP64", shape)
    for k, v in run(orc, wl, 40).items():
        assert v <= 1e-10, (k, v)


@pytest.mark.parametrize("lattice", [0, 1])
def test_reduced_phase_field_with_walls_and_reads(orc, lattice):
    wl = W.wall_drops(64, 24, radius=10.0, ratio=100.0) if lattice == 0 else \
        W.wall_drops(20, 14, 12, radius=6.0, ratio=100.0)
    ang = dict(walls=1, theta_rho_lo=math.radians(60.0), theta_phi_lo=math.radians(70.0),
               theta_rho_hi=math.radians(120.0), theta_phi_hi=math.radians(100.0))
    say("reduced phase field with walls, reads between steps, lattice", lattice)
    for k, v in run(orc, wl, 24, extra=ang, read_at=9).items():
        assert v <= 1e-10, (k, v)
