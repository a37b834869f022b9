"""GPU runs with solid walls (halfway bounce-back, geometric wetting) against
the FP64 oracle and a closed form.

Parity: a liquid-1 cap on the bottom wall and a liquid-2 cap on the top wall
of a channel (walls at y = -1/2 and ny - 1/2), wetting angles that differ per
wall and per field, several grid shapes including ragged tiles; FP64 within
1e-10 of the oracle, FP32-mixed (D2Q9 and D3Q27) within 1e-5 (densities).
Closed form: a shear wave between the walls decays at nu k^2, k = pi / ny."""
import math

import numpy as np
import pytest

from synth import workloads as W

pytestmark = pytest.mark.gpu

ANGLES = dict(theta_rho_lo=math.radians(60.0), theta_phi_lo=math.radians(70.0),
              theta_rho_hi=math.radians(120.0), theta_phi_hi=math.radians(100.0))


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b, floor=1e-300):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))


def both(orc, wl, precision=0, angles=ANGLES):
    import paper_1710_07486_amd as T
    po = orc.coexisting_params(wl.ratio, **wl.physics())
    for k, v in angles.items():
        setattr(po, k, v)
    rho, phi, u = W.fields(wl, po.rho_g, po.rho_l)
    nz, ny, nx = wl.shape
    pl = T.Params(lattice=wl.lattice, precision=precision, nx=nx, ny=ny, nz=nz, T=po.T, rho_g=po.rho_g,
                  rho_l=po.rho_l, lambda1=po.lambda1, lambda2=po.lambda2, lambda3=po.lambda3, kappa1=po.kappa1,
                  kappa2=po.kappa2, kappa3=po.kappa3, chi=po.chi, nu=po.nu, mobility=po.mobility,
                  tau_phi=po.tau_phi, walls=1, **angles)
    return po, pl, rho, phi


def run(orc, wl, steps, precision=0):
    import paper_1710_07486_amd as T
    po, pl, rho, phi = both(orc, wl, precision)
    st = orc.State(po, rho, phi)
    st.run(steps)
    fo = st.fields()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi)
        s.step(steps)
        fg = s.fields()
    return fo, fg


SHAPES_2D = [(96, 48), (100, 37), (64, 9), (70, 2)]


@pytest.mark.parametrize("shape", SHAPES_2D, ids=[f"{a}x{b}" for a, b in SHAPES_2D])
def test_d2q9_walls_fp64_parity(orc, shape):
    nx, ny = shape
    wl = W.wall_drops(nx, ny, radius=min(12.0, 0.3 * nx), ratio=100.0)
    say("D2Q9 walls FP64", shape)
    fo, fg = run(orc, wl, 200)
    e = {k: rel(fg[k], fo[k]) for k in ("rho", "phi")}
    e["u"] = rel(fg["u"], fo["u"], 1e-14)
    e["mu_rho"] = rel(fg["mu_rho"], fo["mu_rho"], 1e-3)
    print("errors", e, flush=True)
    assert np.isfinite(fo["rho"]).all()
    for k, v in e.items():
        assert v <= 1e-10, (k, v)


SHAPES_3D = [(20, 18, 16), (33, 10, 7), (70, 9, 33)]  # the last: two z-columns of the FP64 collision


@pytest.mark.parametrize("shape", SHAPES_3D, ids=[f"{a}x{b}x{c}" for a, b, c in SHAPES_3D])
def test_d3q27_walls_fp64_parity(orc, shape):
    nx, ny, nz = shape
    wl = W.wall_drops(nx, ny, nz, radius=0.3 * min(nx, 2 * ny), ratio=100.0)
    say("D3Q27 walls FP64", shape)
    fo, fg = run(orc, wl, 40)
    e = {k: rel(fg[k], fo[k]) for k in ("rho", "phi")}
    e["u"] = rel(fg["u"], fo["u"], 1e-14)
    e["mu_rho"] = rel(fg["mu_rho"], fo["mu_rho"], 1e-3)
    print("errors", e, flush=True)
    assert np.isfinite(fo["rho"]).all()
    for k, v in e.items():
        assert v <= 1e-10, (k, v)


def test_d2q9_walls_fp32_mixed(orc):
    wl = W.wall_drops(96, 48, radius=12.0, ratio=100.0)
    say("D2Q9 walls FP32-mixed")
    fo, fg = run(orc, wl, 200, precision=1)
    e = {k: rel(fg[k], fo[k]) for k in ("rho", "phi")}
    e["u"] = rel(fg["u"], fo["u"], 1e-14)
    print("errors", e, flush=True)
    assert e["rho"] <= 1e-5 and e["phi"] <= 1e-5 and e["u"] <= 1e-4, e


@pytest.mark.parametrize("shape", SHAPES_3D, ids=[f"{a}x{b}x{c}" for a, b, c in SHAPES_3D])
def test_d3q27_walls_fp32_mixed(orc, shape):
    """The pair-split FP32 collision with bounce-back on both sides of each
    node (a lane pulling c_i and its partner pulling -c_i)."""
    nx, ny, nz = shape
    wl = W.wall_drops(nx, ny, nz, radius=0.3 * min(nx, 2 * ny), ratio=100.0)
    say("D3Q27 walls FP32-mixed", shape)
    fo, fg = run(orc, wl, 40, precision=1)
    e = {k: rel(fg[k], fo[k]) for k in ("rho", "phi")}
    e["u"] = rel(fg["u"], fo["u"], 1e-14)
    print("errors", e, flush=True)
    assert np.isfinite(fo["rho"]).all()
    assert e["rho"] <= 1e-5 and e["phi"] <= 1e-5 and e["u"] <= 1e-4, e


@pytest.mark.parametrize("lattice", [0, 1])
def test_shear_wave_between_walls(orc, lattice):
    """u_x = U sin(pi (y + 1/2) / ny) in a uniform liquid decays as
    exp(-nu k^2 t); mass is conserved to round-off."""
    import paper_1710_07486_amd as T
    ny, steps = 32, 600
    n = 64 if lattice == 0 else 16
    nz = 1 if lattice == 0 else 8
    po = orc.coexisting_params(10.0, lattice=lattice, nx=n, ny=ny, nz=nz)
    say("shear wave between walls, lattice", lattice)
    U = 1e-3
    prof = U * np.sin(math.pi * (np.arange(ny) + 0.5) / ny)
    rho = np.full((nz, ny, n), po.rho_l)
    phi = np.full((nz, ny, n), po.chi)
    u = np.zeros((3, nz, ny, n))
    u[0] = prof[None, :, None]
    pl = T.Params(lattice=lattice, nx=n, ny=ny, nz=nz, T=po.T, rho_g=po.rho_g, rho_l=po.rho_l, walls=1)
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, u)
        m0 = s.read("rho").sum()
        s.step(steps)
        ux = s.read("ux")[0, :, 0]
        m1 = s.read("rho").sum()
    amp = float((ux * prof).sum() / (prof * prof).sum())
    rate = -math.log(amp) / steps
    theory = po.nu * (math.pi / ny) ** 2
    print("rate", rate, "theory", theory, flush=True)
    assert abs(rate / theory - 1) < 1e-4
    assert abs(m1 / m0 - 1) < 1e-12


@pytest.mark.parametrize("lattice", [0, 1])
def test_walls_reads_between_steps(orc, lattice):
    """Field reads and diagnostics mid-run (which complete the partial
    next-step moments, here with wall rows that take no inbox entries from
    beyond the wall) leave the run unchanged: 5 + read + 7 steps against an
    uninterrupted oracle run of 12."""
    import paper_1710_07486_amd as T
    wl = W.wall_drops(64, 24, radius=10.0, ratio=100.0) if lattice == 0 else \
        W.wall_drops(20, 14, 12, radius=6.0, ratio=100.0)
    say("walls, reads between steps, lattice", lattice)
    po, pl, rho, phi = both(orc, wl)
    st = orc.State(po, rho, phi)
    st.run(12)
    fo = st.fields()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi)
        s.step(5)
        s.read("rho")
        s.diagnostics(check=False)
        s.step(7)
        fg = s.fields()
    for k in ("rho", "phi"):
        assert rel(fg[k], fo[k]) <= 1e-10, k
    assert rel(fg["u"], fo["u"], 1e-14) <= 1e-10


def test_walls_with_peng_robinson(orc):
    """Walls with the Peng-Robinson free energy (density ratio 100)."""
    import paper_1710_07486_amd as T
    wl = W.wall_drops(96, 48, radius=12.0, ratio=100.0)
    say("walls, Peng-Robinson, ratio 100")
    e = dict(eos=2, a=2.0 / 49.0, b=2.0 / 21.0)
    po = orc.coexisting_params(wl.ratio, **wl.physics(), **e)
    for k, v in ANGLES.items():
        setattr(po, k, v)
    rho, phi, _ = W.fields(wl, po.rho_g, po.rho_l)
    pl = T.Params(lattice=0, nx=96, ny=48, nz=1, T=po.T, rho_g=po.rho_g, rho_l=po.rho_l, eos=2, a=po.a, b=po.b,
                  omega=po.omega, lambda1=po.lambda1, lambda2=po.lambda2, lambda3=po.lambda3, kappa1=po.kappa1,
                  kappa2=po.kappa2, kappa3=po.kappa3, chi=po.chi, nu=po.nu, mobility=po.mobility,
                  tau_phi=po.tau_phi, walls=1, **ANGLES)
    st = orc.State(po, rho, phi)
    st.run(200)
    fo = st.fields()
    assert np.isfinite(fo["rho"]).all()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi)
        s.step(200)
        fg = s.fields()
    for k in ("rho", "phi"):
        assert rel(fg[k], fo[k]) <= 1e-10, k


@pytest.mark.parametrize("prec", [0, 1])
def test_liquid_liquid_contact_angle_reaches_the_wall_angle(orc, prec):
    """A liquid-1 cap in liquid 2 on the bottom wall (phase-field interface
    2.8 nodes wide, lambda = kappa / 2; 128 x 64 box, cap radius 20, started
    at 90 degrees): after 80,000 steps it meets the wall within 3 degrees of
    the prescribed 60 and 120 degrees, in FP64 and FP32-mixed storage."""
    import dataclasses
    import paper_1710_07486_amd as T
    from tests import test_oracle_walls as TW
    out = {}
    for th in (60.0, 120.0):
        p, rho, phi = TW.wall_drop(orc, th, nx=128, ny=64, radius=20.0, liquid_liquid=True, phi_only=True)
        p = dataclasses.replace(p, lambda2=0.5 * p.kappa2, lambda3=0.5 * p.kappa3)
        pl = T.Params(lattice=0, precision=prec, nx=p.nx, ny=p.ny, nz=1, T=p.T, rho_g=p.rho_g, rho_l=p.rho_l,
                      lambda1=p.lambda1, lambda2=p.lambda2, lambda3=p.lambda3, kappa1=p.kappa1, kappa2=p.kappa2,
                      kappa3=p.kappa3, chi=p.chi, nu=p.nu, mobility=p.mobility, tau_phi=p.tau_phi, walls=1,
                      theta_rho_lo=p.theta_rho_lo, theta_rho_hi=p.theta_rho_hi, theta_phi_lo=p.theta_phi_lo,
                      theta_phi_hi=p.theta_phi_hi)
        say("liquid-liquid cap", th, "precision", prec)
        with T.Solver(pl) as s:
            s.init_fields(rho, phi)
            s.step(80000)
            out[th] = TW.contact_angle(s.read("phi")[0], -p.chi, p.chi)
    print("liquid-liquid contact angles", out, flush=True)
    for th, a in out.items():
        assert abs(a - th) < 3.0, (th, a)
