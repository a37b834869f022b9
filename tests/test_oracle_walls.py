"""Pins of the oracle's solid walls: halfway bounce-back for f and g and the
geometric wetting condition (the wetting boundary conditions the paper's
outlook names, with the geometric approach among those it cites).

Each check stands on something other than the oracle's own wall code: the
viscous decay rate nu k^2 of a shear wave between no-slip walls (closed
form), exact conservation of mass and phase field, the mirror symmetry that
maps the bottom wall onto the top one, and the response of a drop's contact
angle (measured here by a least-squares circle fit of the mid-value contour,
numpy only) to the prescribed angle: towards it, on the right side of 90
degrees, and closer as the interfaces widen."""
import dataclasses
import math

import numpy as np
import pytest


def shear_wave(orc, lattice, ny, steps):
    n_side = 4
    p = orc.coexisting_params(10.0, lattice=lattice, nx=n_side, ny=ny, nz=n_side if lattice == 1 else 1)
    p = dataclasses.replace(p, walls=1)
    U = 1e-3
    prof = U * np.sin(math.pi * (np.arange(ny) + 0.5) / ny)
    shape = p.shape
    rho = np.full(shape, p.rho_l)
    phi = np.full(shape, p.chi)
    u = np.zeros((3,) + shape)
    u[0] = prof[None, :, None]
    st = orc.State(p, rho, phi, u)
    m0 = st.fields()["rho"].sum()
    st.run(steps)
    f = st.fields()
    ux = f["u"][0][0, :, 0]
    amp = float((ux * prof).sum() / (prof * prof).sum())
    return p, prof, f, ux, amp, m0


@pytest.mark.parametrize("lattice,ny", [(0, 16), (0, 32), (1, 16)])
def test_shear_wave_between_no_slip_walls(orc, lattice, ny):
    """u_x = U sin(pi (y + 1/2) / ny) vanishes on both walls (y = -1/2 and
    ny - 1/2) and decays as exp(-nu k^2 t), k = pi / ny, keeping its shape."""
    steps = 600
    p, prof, f, ux, amp, m0 = shear_wave(orc, lattice, ny, steps)
    rate = -math.log(amp) / steps
    theory = p.nu * (math.pi / ny) ** 2
    assert abs(rate / theory - 1) < 1e-4, (rate, theory)
    assert np.abs(ux / amp - prof).max() < (1e-7 if lattice == 0 else 1e-5) * prof.max()
    assert abs(f["rho"].sum() / m0 - 1) < 1e-12
    # no flow through the walls, nothing along z
    assert np.abs(f["u"][1]).max() < 1e-12 and np.abs(f["u"][2]).max() < 1e-12


def wall_drop(orc, theta_deg, nx=96, ny=48, radius=16.0, start_deg=90.0, kappa=0.1, kappa1=1e-3, top=False,
              liquid_liquid=False, phi_only=False):
    """A liquid-1 cap of the area of a half disc of `radius`, meeting the
    bottom (or top) wall at start_deg, in gas (or in liquid 2)."""
    p = orc.coexisting_params(10.0, lattice=0, nx=nx, ny=ny, nz=1, kappa1=kappa1, kappa2=kappa, kappa3=kappa,
                              lambda2=3.125 * kappa, lambda3=3.125 * kappa)
    th = math.radians(theta_deg)
    w = dict(walls=1, theta_phi_hi=th if top else math.pi / 2, theta_phi_lo=math.pi / 2 if top else th)
    if not phi_only:
        w.update(theta_rho_hi=th if top else math.pi / 2, theta_rho_lo=math.pi / 2 if top else th)
    p = dataclasses.replace(p, **w)
    a0 = math.pi * radius ** 2 / 2
    ts = math.radians(start_deg)
    R = math.sqrt(a0 / (ts - math.sin(ts) * math.cos(ts)))
    yc = -0.5 - R * math.cos(ts)
    yy, xx = np.mgrid[0:ny, 0:nx]
    c = 0.5 * (1 - np.tanh((np.sqrt((xx - nx / 2) ** 2 + (yy - yc) ** 2) - R) / 2.0))
    if top:
        c = c[::-1]
    if liquid_liquid:
        rho, phi = np.full(c.shape, p.rho_l), p.chi * (2 * c - 1)
    else:
        rho, phi = p.rho_g + (p.rho_l - p.rho_g) * c, p.chi * c
    return p, rho[None], phi[None]


def contact_angle(field, lo, hi, ymin=2):
    """Angle (degrees, inside the high phase) at the bottom wall y = -1/2 of
    the circle fitted to the mid-value contour of rows y >= ymin."""
    mid = 0.5 * (lo + hi)
    ny, nx = field.shape
    px, py = [], []
    for x in range(nx):
        col = field[:, x]
        for y in range(ymin, ny - 1):
            if (col[y] - mid) * (col[y + 1] - mid) < 0:
                px.append(x)
                py.append(y + (mid - col[y]) / (col[y + 1] - col[y]))
    for y in range(ymin, ny):
        row = field[y]
        for x in range(nx - 1):
            if (row[x] - mid) * (row[x + 1] - mid) < 0:
                px.append(x + (mid - row[x]) / (row[x + 1] - row[x]))
                py.append(y)
    px, py = np.array(px), np.array(py)
    sol, *_ = np.linalg.lstsq(np.c_[2 * px, 2 * py, np.ones_like(px)], px ** 2 + py ** 2, rcond=None)
    xc, yc, cc = sol
    R = math.sqrt(cc + xc ** 2 + yc ** 2)
    return math.degrees(math.acos(max(-1.0, min(1.0, (-0.5 - yc) / R))))


def test_walls_conserve_mass_and_phase_field(orc):
    p, rho, phi = wall_drop(orc, 60.0, start_deg=70.0)
    st = orc.State(p, rho, phi)
    f0 = st.fields()
    st.run(300)
    f = st.fields()
    assert abs(f["rho"].sum() / f0["rho"].sum() - 1) < 1e-12
    assert abs(f["phi"].sum() / f0["phi"].sum() - 1) < 1e-12


def test_top_wall_mirrors_bottom_wall(orc):
    """The same drop on the top wall is the y-mirror image of the run on the
    bottom wall (u_y changes sign)."""
    out = []
    for top in (False, True):
        p, rho, phi = wall_drop(orc, 60.0, start_deg=70.0, top=top)
        st = orc.State(p, rho, phi)
        st.run(200)
        out.append(st.fields())
    a, b = out
    for k in ("rho", "phi"):
        assert np.abs(a[k] - b[k][:, ::-1]).max() < 1e-11 * np.abs(a[k]).max(), k
    assert np.abs(a["u"][0] - b["u"][0][:, ::-1]).max() < 1e-13
    assert np.abs(a["u"][1] + b["u"][1][:, ::-1]).max() < 1e-13


def test_liquid_liquid_contact_angle_reaches_the_wall_angle(orc):
    """A liquid-1 cap in liquid 2 on the wall (rho uniform, the phase field
    carries the interface, lambda = kappa / 2 so that the interface is
    2.8 nodes wide): started at 90 degrees, its contact line moves by
    Cahn-Hilliard diffusion until the cap meets the wall at the prescribed
    angle, within 3 degrees for 60 and 120 degrees (measured 61.4 and 122.0
    after 30,000 steps on this 80 x 40 box with a cap of radius 14; the same
    cap at 90 degrees stays at 90)."""
    ang = {}
    for th in (60.0, 90.0, 120.0):
        p, rho, phi = wall_drop(orc, th, nx=80, ny=40, radius=14.0, liquid_liquid=True, phi_only=True)
        p = dataclasses.replace(p, lambda2=0.5 * p.kappa2, lambda3=0.5 * p.kappa3)
        st = orc.State(p, rho, phi)
        st.run(30000 if th != 90.0 else 2000)
        ang[th] = contact_angle(st.fields()["phi"][0], -p.chi, p.chi)
    print("liquid-liquid contact angles", ang)
    assert abs(ang[90.0] - 90.0) < 1.0, ang
    assert abs(ang[60.0] - 60.0) < 3.0, ang
    assert abs(ang[120.0] - 120.0) < 3.0, ang


def test_liquid_gas_contact_angle_follows_the_wall_angle(orc):
    """A liquid-1 drop in gas: the relaxed angle lies on the prescribed side
    of 90 degrees, symmetric about 90 for 60 and 120 degrees, and nearer the
    prescribed angle when the interfaces are wider (kappa_1 = 0.03 against
    1e-3).  The geometric condition acts on the density through one ghost
    row, weighted by the small density gradient coefficient against the
    stiff equation of state, and does not reach the prescribed angle for a
    liquid-gas contact line (measured 85 / 95 degrees for 60 / 120 at the
    paper's kappa_1, steady from 3,000 to 100,000 steps and for caps of
    radius 16 and 48; 79 / 101 at a Maxwell ratio of 3)."""
    ang = {}
    for k1 in (1e-3, 3e-2):
        for th in (60.0, 90.0, 120.0):
            p, rho, phi = wall_drop(orc, th, kappa1=k1)
            st = orc.State(p, rho, phi)
            st.run(3000)
            ang[(k1, th)] = contact_angle(st.fields()["rho"][0], p.rho_g, p.rho_l)
    for k1 in (1e-3, 3e-2):
        assert abs(ang[(k1, 90.0)] - 90.0) < 1.0, ang
        assert ang[(k1, 60.0)] < 87.0 and ang[(k1, 120.0)] > 93.0, ang
        assert abs(ang[(k1, 60.0)] + ang[(k1, 120.0)] - 180.0) < 2.0, ang
    assert ang[(3e-2, 60.0)] < ang[(1e-3, 60.0)] - 5.0, ang
    assert ang[(3e-2, 120.0)] > ang[(1e-3, 120.0)] + 5.0, ang
