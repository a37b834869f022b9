"""GPU parity of the HIP path (through the C ABI) with the FP64 oracle.

Metric (per field): max |x_gpu - x_oracle| / max(max |x_oracle|, floor).
Bars: FP64 path <= 1e-10 for rho, phi and u; FP32-mixed path: density and
phase field <= 1e-5, velocity <= 1e-4 relative to the largest velocity (stated
error of the reduced-precision form).  Inputs are seeded synthetic drop
configurations shared by both sides through ``synth``.
"""
import numpy as np
import pytest

from synth import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b, floor=1e-300):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))


def make(orc, wl, precision=0):
    """Oracle params and library params for one workload, plus its fields."""
    import paper_1710_07486_amd as T
    po = orc.workload_params(wl)
    rho, phi, u = W.fields(wl, po.rho_g, po.rho_l)
    nz, ny, nx = wl.shape
    pl = T.Params(lattice=wl.lattice, precision=precision, nx=nx, ny=ny, nz=nz, T=po.T, rho_g=po.rho_g,
                  rho_l=po.rho_l, lambda1=po.lambda1, lambda2=po.lambda2, lambda3=po.lambda3,
                  kappa1=po.kappa1, kappa2=po.kappa2, kappa3=po.kappa3, chi=po.chi, nu=po.nu,
                  mobility=po.mobility, tau_phi=po.tau_phi)
    return po, pl, rho, phi, u


def run_both(orc, wl, steps, precision=0, with_u=True):
    import paper_1710_07486_amd as T
    po, pl, rho, phi, u = make(orc, wl, precision)
    uu = u if (with_u and np.abs(u).max() > 0) else None
    st = orc.State(po, rho, phi, uu)
    st.run(steps)
    fo = st.fields()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, uu)
        s.step(steps)
        fg = s.fields()
    return fo, fg


def check_fp64(fo, fg, tol=FP64_TOL):
    e = {k: rel(fg[k], fo[k]) for k in ("rho", "phi")}
    e["u"] = rel(fg["u"], fo["u"], 1e-14)
    e["mu_rho"] = rel(fg["mu_rho"], fo["mu_rho"], 1e-3)
    e["mu_phi"] = rel(fg["mu_phi"], fo["mu_phi"], 1e-3)
    print("errors", e, flush=True)
    for k, v in e.items():
        assert v <= tol, (k, v)
    return e


def test_lens_128_fp64_full_run(orc):
    """The small lens workload in full: D2Q9 128x128, ratio 10, 1000 steps."""
    wl = W.lens(128, 128, radius=20, ratio=10.0, kappa=0.045, steps=1000)
    say("lens 128^2 D2Q9 FP64 1000 steps")
    fo, fg = run_both(orc, wl, 1000)
    check_fp64(fo, fg)


@pytest.mark.parametrize("shape", [(1, 37, 100), (1, 64, 64), (1, 1, 70), (1, 45, 1)])
def test_d2q9_fp64_ragged_ratio1000(orc, shape):
    nz, ny, nx = shape
    wl = W.lens(nx, ny, radius=max(2.0, min(nx, ny) / 5), ratio=1000.0, kappa=0.1, steps=300)
    for d in wl.drops:
        d["velocity"] = (0.01, -0.005, 0.0)
    say("D2Q9 FP64 ratio 1000", shape)
    fo, fg = run_both(orc, wl, 300)
    check_fp64(fo, fg)


def box_collision(shape, ratio=1000.0, v_rel=0.04, k2=0.1, k3=0.3):
    """Two drops (liquid 1 and 2) approaching along x in a periodic box."""
    nz, ny, nx = shape
    n = min(shape)
    wl = W.collision_3d(n=max(n, 4), radius=max(1.5, n / 6), ratio=ratio, v_rel=v_rel, kappa2=k2, kappa3=k3)
    wl.shape = tuple(shape)
    for d, cx in zip(wl.drops, (nx / 2 - max(n, 4) / 4, nx / 2 + max(n, 4) / 4)):
        d["center"] = (cx, ny / 2, nz / 2)
    return wl


@pytest.mark.parametrize("shape", [(18, 20, 24), (1, 8, 8), (3, 3, 3), (16, 16, 64), (17, 12, 70), (33, 5, 9),
                                   (65, 5, 9), (40, 9, 130)])
def test_d3q27_fp64_collision(orc, shape):
    """The FP64 step against the oracle; the collision walks z-columns of 32
    planes, so the depths cover single short columns (1 to 18 planes), a
    full column and a ragged one of 1 plane (33), and three columns (65);
    130 x 9 x 40 has two columns, three x tiles (the last 2 wide) and three
    y tiles (the last 1 high) at once."""
    wl = box_collision(shape)
    say("D3Q27 FP64 ratio 1000", shape)
    fo, fg = run_both(orc, wl, 60)
    check_fp64(fo, fg)


@pytest.mark.parametrize("precision", [0, 1])
def test_d3q27_long_horizon(orc, precision):
    """1,000 steps of a D3Q27 drop collision at density ratio 1000 (70 x 12 x
    36: two x tiles, the last 6 wide, three y tiles and two z-columns of the
    FP64 collision, the last 4 deep) element by element against the oracle:
    the drops meet and merge (largest speed 0.075 falling to 0.004).  FP64
    within 1e-10; FP32-mixed within its stated bars, 1e-5 for rho and phi
    and 1e-4 of the largest velocity (measured 1.6e-6, 2.3e-6, 9.1e-6)."""
    import paper_1710_07486_amd as T
    wl = wide_box((36, 12, 70))
    say("D3Q27 1000 steps", precision)
    po, pl, rho, phi, u = make(orc, wl, precision)
    st = orc.State(po, rho, phi, u)
    st.run(1000)
    fo = st.fields()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, u)
        s.step(1000)
        fg = s.fields()
    assert np.isfinite(fo["rho"]).all() and fo["rho"].max() > 0.9 * po.rho_l
    if precision == 0:
        check_fp64(fo, fg)
    else:
        e = {"rho": rel(fg["rho"], fo["rho"]), "phi": rel(fg["phi"], fo["phi"]),
             "u": rel(fg["u"], fo["u"], 1e-14),
             "rho_mean": float(np.abs(fg["rho"] - fo["rho"]).mean() / np.abs(fo["rho"]).mean())}
        print("fp32-mixed errors after 1000 steps", e, flush=True)
        assert e["rho"] <= 1e-5 and e["phi"] <= 1e-5 and e["u"] <= 1e-4, e


@pytest.mark.parametrize("lattice", [0, 1])
def test_fp32_mixed_error_vs_oracle(orc, lattice):
    if lattice == 0:
        wl = W.lens(128, 96, radius=16, ratio=1000.0, kappa=0.1)
        steps = 400
    else:
        wl = box_collision((32, 32, 32), k2=0.1, k3=0.1)
        steps = 60
    say("FP32-mixed vs FP64 oracle lattice", lattice)
    fo, fg = run_both(orc, wl, steps, precision=1)
    e = {"rho": rel(fg["rho"], fo["rho"]), "phi": rel(fg["phi"], fo["phi"]),
         "u": rel(fg["u"], fo["u"], 1e-14)}
    gas = fo["rho"] < 2 * fo["rho"].min()
    e["rho_gas_pointwise"] = float(np.abs(fg["rho"][gas] / fo["rho"][gas] - 1).max())
    print("fp32-mixed errors", e, flush=True)
    assert e["rho"] <= 1e-5 and e["phi"] <= 1e-5
    assert e["u"] <= 1e-4


def wide_box(shape, k2=0.1, k3=0.3, v_rel=0.04, ratio=1000.0, walls=0):
    """Two drops approaching along x in a box that spans several tiles of the
    3D kernels in x (64 wide) and y (4 high), with a ragged last tile: the
    drops cross tile edges, so cross-tile moment sums (inboxes) and the
    staged halos of neighbouring tiles all carry interface values."""
    nz, ny, nx = shape
    R = min(5.0, 0.45 * min(ny, nz) + 1.5)
    wl = W.collision_3d(n=16, radius=R, ratio=ratio, v_rel=v_rel, kappa2=k2, kappa3=k3)
    wl.shape = tuple(shape)
    for d, cx in zip(wl.drops, (nx / 2 - R - 2.5, nx / 2 + R + 2.5)):
        d["center"] = (cx, ny / 2 + 0.3, nz / 2 - 0.2)
    if walls:
        wl.walls = 1
    return wl


WIDE = {"fp64": (0, 0, 0), "fp32": (1, 0, 0), "fp64_d3q7": (0, 1, 0), "fp64_walls": (0, 0, 1),
        "fp32_walls": (1, 0, 1)}


@pytest.mark.parametrize("shape", [(9, 13, 200), (7, 10, 130)])
@pytest.mark.parametrize("case", list(WIDE))
def test_d3q27_multi_tile(orc, shape, case):
    """D3Q27 boxes three tiles wide in x and y (200 x 13 x 9, and 130 x 10 x 7
    with two-node ragged last tiles), 200 steps, element by element against
    the oracle: FP64 (full and reduced phase-field lattice, and with wetting
    walls) within 1e-10, FP32-mixed (periodic and with wetting walls) within
    1e-5 (rho, phi) and 1e-4 of the largest velocity (u)."""
    import math
    import paper_1710_07486_amd as T
    precision, glat, walls = WIDE[case]
    wl = wide_box(shape, walls=walls)
    say("D3Q27 multi-tile", case, shape)
    po, pl, rho, phi, u = make(orc, wl, precision)
    po.glattice = pl.glattice = glat
    if walls:
        pl.walls = 1
        ang = dict(theta_rho_lo=math.radians(60.0), theta_phi_lo=math.radians(75.0),
                   theta_rho_hi=math.radians(115.0), theta_phi_hi=math.radians(100.0))
        for key, v in ang.items():
            setattr(po, key, v)
            setattr(pl, key, v)
    steps = 200
    st = orc.State(po, rho, phi, u)
    st.run(steps)
    fo = st.fields()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, u)
        s.step(steps)
        fg = s.fields()
    assert np.isfinite(fo["rho"]).all()
    if precision == 0:
        check_fp64(fo, fg)
    else:
        e = {"rho": rel(fg["rho"], fo["rho"]), "phi": rel(fg["phi"], fo["phi"]),
             "u": rel(fg["u"], fo["u"], 1e-14)}
        print("fp32-mixed multi-tile errors", e, flush=True)
        assert e["rho"] <= 1e-5 and e["phi"] <= 1e-5 and e["u"] <= 1e-4


@pytest.mark.parametrize("case", list(WIDE))
def test_d3q27_rows_wider_than_a_tile(orc, case):
    """A box wider than the 256-node rows of the D3Q27 FP32 collision and
    moment pass tiles (300 x 6 x 5, ragged second tile of 44): one drop
    straddles the tile edge at x = 256 and the other the periodic seam at
    x = 0, 100 steps element by element against the oracle (FP64 forms
    within 1e-10, FP32-mixed within 1e-5 and 1e-4 of the largest velocity)."""
    import math
    import paper_1710_07486_amd as T
    precision, glat, walls = WIDE[case]
    wl = wide_box((5, 6, 300), walls=walls)
    for d, cx in zip(wl.drops, (256.4, 3.6)):
        d["center"] = (cx, 3.3, 2.3)
    say("D3Q27 rows wider than a tile", case)
    po, pl, rho, phi, u = make(orc, wl, precision)
    po.glattice = pl.glattice = glat
    if walls:
        pl.walls = 1
        ang = dict(theta_rho_lo=math.radians(60.0), theta_phi_lo=math.radians(75.0),
                   theta_rho_hi=math.radians(115.0), theta_phi_hi=math.radians(100.0))
        for key, v in ang.items():
            setattr(po, key, v)
            setattr(pl, key, v)
    steps = 100
    st = orc.State(po, rho, phi, u)
    st.run(steps)
    fo = st.fields()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, u)
        s.step(steps)
        fg = s.fields()
    assert np.isfinite(fo["rho"]).all()
    # the drops sit where the tiles meet: the liquid density there
    assert fo["rho"][:, :, 250:263].max() > 0.5 * po.rho_l and fo["rho"][:, :, :8].max() > 0.5 * po.rho_l
    if precision == 0:
        check_fp64(fo, fg)
    else:
        e = {"rho": rel(fg["rho"], fo["rho"]), "phi": rel(fg["phi"], fo["phi"]),
             "u": rel(fg["u"], fo["u"], 1e-14)}
        print("fp32-mixed wide-row errors", e, flush=True)
        assert e["rho"] <= 1e-5 and e["phi"] <= 1e-5 and e["u"] <= 1e-4


DIAG_CASES = {"fp64": (0, 0, 0), "fp32": (1, 0, 0), "fp64_d3q7": (0, 1, 0), "fp64_walls": (0, 0, 1),
              "fp32_walls": (1, 0, 1)}


@pytest.mark.parametrize("case", list(DIAG_CASES))
def test_step_diagnostics_cover_every_plane_3d(orc, case):
    """A diagnosed D3Q27 step reduces over every node: its own diagnostics of
    the starting state (read back without another pass) equal the oracle's
    sums and extremes over that state, and a diagnostic
    pass over the same state, on a 20 x 9 x 70 box whose collisions walk
    several z-columns (the drops straddle the column ends), periodic and
    walled, and with the reduced phase-field lattice."""
    import math
    import paper_1710_07486_amd as T
    precision, glat, walls = DIAG_CASES[case]
    wl = wide_box((70, 9, 20), walls=walls)
    say("D3Q27 step diagnostics", case)
    po, pl, rho, phi, u = make(orc, wl, precision)
    po.glattice = pl.glattice = glat
    if walls:
        pl.walls = 1
        ang = dict(theta_rho_lo=math.radians(60.0), theta_phi_lo=math.radians(75.0),
                   theta_rho_hi=math.radians(115.0), theta_phi_hi=math.radians(100.0))
        for key, v in ang.items():
            setattr(po, key, v)
            setattr(pl, key, v)
    st = orc.State(po, rho, phi, u)
    fo = st.fields()
    # the oracle's totals before its first step: sum rho, sum phi, sum j (3)
    ref = st.run(1, diag=True)[0]
    umax = float(np.sqrt((fo["u"] ** 2).sum(axis=0)).max())
    pl.diag_every = 1
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, u)
        assert s.last_diagnostics()["step"] == -1
        d0 = s.diagnostics()
        s.step(1)
        d = s.last_diagnostics()
    print("step diagnostics", d, "pass", d0, "oracle", ref, umax, flush=True)
    assert d["step"] == 0 and d0["step"] == 0
    assert d["nonfinite"] == 0 and d0["nonfinite"] == 0
    # FP64: the reductions and the oracle agree to round-off; FP32-mixed: the
    # stored deviations round the state at about 1e-8 of the densities
    tol = 1e-12 if precision == 0 else 1e-6
    mass = ref[0]
    for dd in (d, d0):
        assert abs(dd["mass"] / mass - 1) < tol, (dd["mass"], mass)
        assert abs(dd["phi_total"] - ref[1]) < tol * abs(mass)
        assert np.abs(np.array(dd["mom"]) - ref[2:5]).max() < tol * abs(mass)
        assert abs(dd["min_rho"] / fo["rho"].min() - 1) < tol
        assert abs(dd["max_u"] / umax - 1) < (1e-8 if precision == 0 else 1e-4)
        # the stabiliser where a node sits at equilibrium is 0/0 (either value
        # collides alike): its range is checked for sense, not against the oracle
        assert 1.0 < dd["gamma_min"] <= dd["gamma_max"] < 3.0
    # the step's reduction and the pass see the same state (the phase-field
    # total cancels, so it is held to the scale of the mass)
    for key in ("mass", "max_u", "min_rho", "gamma_min", "gamma_max"):
        assert abs(d[key] - d0[key]) <= 1e-12 * abs(d0[key]), key
    assert abs(d["phi_total"] - d0["phi_total"]) <= 1e-12 * abs(mass)


def test_init_rejects_bad_fields(orc):
    import paper_1710_07486_amd as T
    wl = W.lens(32, 32, radius=6, ratio=10.0)
    po, pl, rho, phi, u = make(orc, wl)
    say("init error paths")
    with T.Solver(pl) as s:
        for bad in ("neg", "nan", "u"):
            r, p, uu = rho.copy(), phi.copy(), np.zeros((2,) + rho.shape)
            if bad == "neg":
                r[0, 3, 4] = -1.0
            elif bad == "nan":
                p[0, 5, 5] = np.nan
            else:
                uu[0, 0, 1, 1] = 1.0
            with pytest.raises(T.TelbmError) as e:
                s.init_fields(r, p, uu)
            assert e.value.code == 2  # TELBM_ERR_UNSTABLE
        s.init_fields(rho, phi)
        s.step(3)
        assert s.diagnostics()["nonfinite"] == 0


def test_diagnostics_and_device_read(orc):
    import torch
    import paper_1710_07486_amd as T
    wl = W.lens(96, 64, radius=12, ratio=1000.0, kappa=0.1)
    po, pl, rho, phi, u = make(orc, wl)
    pl.diag_every = 10
    say("diagnostics vs oracle sums")
    st = orc.State(po, rho, phi)
    d_or = st.run(41, diag=True)
    with T.Solver(pl) as s:
        s.init_fields(torch.from_numpy(rho).cuda(), torch.from_numpy(phi).cuda())
        s.step(41)
        s.sync()
        # telbm_diagnostics reports the current state (before step 41)
        d_next = st.run(1, diag=True)
        st.steps -= 1
        d = s.diagnostics()
        assert d["step"] == 41
        ref = d_next[0]
        assert abs(d["mass"] / ref[0] - 1) < 1e-13
        assert abs(d["phi_total"] - ref[1]) < 1e-11 * abs(ref[0])
        assert np.abs(np.array(d["mom"]) - ref[2:5]).max() < 1e-10
        assert d["nonfinite"] == 0 and d["min_rho"] > 0
        assert 1.0 < d["gamma_min"] <= d["gamma_max"] < 3.0
        rd = s.read("rho", device=True)
        assert rd.is_cuda
        assert abs(float(rd.sum()) - ref[0]) < 1e-9 * abs(ref[0])


# (free energy, density ratio).  The van der Waals runs use a small
# attraction a: the density ratio at a given T/T_c does not depend on a, but
# the liquid's dp/drho grows with it (a = 9/49 at ratio 100 gives ~5 against
# c_s^2 = 1/3 and the oracle itself diverges).
EOS_CASES = {"vdw100": (dict(eos=1, a=2.0 / 49.0, b=2.0 / 21.0), 100.0),
             "vdw1000": (dict(eos=1, a=0.5 / 49.0, b=2.0 / 21.0), 1000.0),
             "pr1000": (dict(eos=2, a=2.0 / 49.0, b=2.0 / 21.0), 1000.0)}


@pytest.mark.parametrize("eos", list(EOS_CASES))
@pytest.mark.parametrize("lattice", [0, 1])
def test_other_equations_of_state(orc, eos, lattice):
    """van der Waals and Peng-Robinson free energies at density ratios 100
    and 1000: GPU against oracle, FP64 (D2Q9 lens 96 x 64, 300 steps; D3Q27
    box 16 x 18 x 20, 40 steps)."""
    import paper_1710_07486_amd as T
    e, ratio = EOS_CASES[eos]
    if lattice == 0:
        wl, steps = W.lens(96, 64, radius=12, ratio=ratio, kappa=0.1), 300
    else:
        wl, steps = box_collision((16, 18, 20), ratio=ratio), 40
    say("EOS", eos, "lattice", lattice, wl.shape)
    ph = wl.physics()
    po = orc.coexisting_params(wl.ratio, **ph, **e)
    rho, phi, u = W.fields(wl, po.rho_g, po.rho_l)
    nz, ny, nx = wl.shape
    pl = T.Params(lattice=wl.lattice, nx=nx, ny=ny, nz=nz, T=po.T, rho_g=po.rho_g, rho_l=po.rho_l,
                  eos=e["eos"], a=e["a"], b=e["b"], omega=po.omega, lambda1=po.lambda1, lambda2=po.lambda2,
                  lambda3=po.lambda3, kappa1=po.kappa1, kappa2=po.kappa2, kappa3=po.kappa3, chi=po.chi,
                  nu=po.nu, mobility=po.mobility, tau_phi=po.tau_phi)
    uu = u if np.abs(u).max() > 0 else None
    st = orc.State(po, rho, phi, uu)
    st.run(steps)
    fo = st.fields()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, uu)
        s.step(steps)
        fg = s.fields()
    assert np.isfinite(fo["rho"]).all()
    check_fp64(fo, fg)


@pytest.mark.parametrize("case", ["d2q9_fp64", "d2q9_fp32", "d3q27_fp64", "d3q27_fp32"])
def test_reads_between_steps_leave_the_run_unchanged(orc, case):
    """Reading fields and taking diagnostics mid-run (which complete the
    next-step moments that the step kernels leave as partial sums) must not
    change the run: the state after 5 + read + 7 steps matches an
    uninterrupted oracle run of 12 steps."""
    import paper_1710_07486_amd as T
    lat, prec = (0 if case.startswith("d2q9") else 1), (1 if case.endswith("fp32") else 0)
    wl = W.lens(100, 37, radius=9, ratio=1000.0, kappa=0.1) if lat == 0 else box_collision((18, 20, 24))
    say("reads between steps", case, wl.shape)
    po, pl, rho, phi, u = make(orc, wl, prec)
    uu = u if np.abs(u).max() > 0 else None
    st = orc.State(po, rho, phi, uu)
    st.run(5)
    mid = st.fields()
    st.run(7)
    fo = st.fields()
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, uu)
        s.step(5)
        r5 = s.read("rho")
        s.diagnostics()
        s.step(7)
        fg = s.fields()
    tol = FP64_TOL if prec == 0 else 1e-5
    assert rel(r5, mid["rho"]) <= tol
    for k in ("rho", "phi"):
        assert rel(fg[k], fo[k]) <= tol, (k, rel(fg[k], fo[k]))


def _window(arr, center, r):
    """Periodic window of half-width r around center (z, y, x) of a (.., nz, ny, nx) array."""
    idx = []
    for ax, c in enumerate(center):
        n = arr.shape[-3 + ax]
        if n == 1:
            idx.append(np.array([0]))
        else:
            idx.append((np.arange(c - r, c + r + 1)) % n)
    return arr[..., idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]


FULL_CASES = ["d3q27_256_fp64", "d3q27_256_mixed", "d2q9_1024_fp64", "d2q9_1024_mixed", "d2q9_1024_fp64_reduced",
              "d3q27_256_fp64_reduced", "d2q9_1024_fp64_walls"]


def tile_edge_samples(wl, rng, count):
    """`count` nodes on tile edges of the step kernels (x = 0 or 63 mod 64,
    among them the 256-node rows' ends 0 and 255 mod 256 of the D3Q27 FP32
    tiles; y = 0 or the last row of a 64 x 4 tile in 3D, 64 x 8 in 2D, where
    every row is a 256 x 1 tile's), three in four
    on a drop interface (within 3 nodes of its starting radius, or with walls
    in the wall rows within half a tile of a contact line; in 3D the z
    of such a node is taken on the sphere), the rest anywhere.  In 3D, a
    node on the interface is moved to z = 0 or 15 mod 16 (the potential
    pass's column edges, among them the collision's 32-plane column ends at
    0 and 31 mod 32) when one lies within 2 planes."""
    import math
    nz, ny, nx = wl.shape
    ty = 4 if nz > 1 else 8
    xe = [x for x in range(nx) if x % 64 in (0, 63) or x == nx - 1]
    ye = [y for y in range(ny) if y % ty in (0, ty - 1) or y == ny - 1]
    near = []
    for d in wl.drops:
        c, R = d["center"], d["radius"]
        for X in xe:
            for Y in ye:
                if wl.walls and 3 <= Y <= ny - 4:
                    continue
                rxy = math.hypot(X - c[0], Y - c[1])
                if nz == 1:
                    # wall rows: the contact line and its neighbourhood
                    if abs(rxy - R) < (34 if wl.walls else 3):
                        near.append((0, Y, X))
                elif rxy < R:
                    for sgn in (-1, 1):
                        z = int(round(c[2] + sgn * math.sqrt(R * R - rxy * rxy))) % nz
                        ze = [zz for zz in range(z - 2, z + 3) if zz % 16 in (0, 15)]
                        near.append(((ze[0] if ze else z) % nz, Y, X))
    near = sorted(set(near))
    pick = [near[i] for i in rng.choice(len(near), size=min(len(near), 3 * count // 4), replace=False)]
    out = set(pick)
    while len(out) < count:
        out.add((int(rng.integers(nz)), int(rng.choice(ye)), int(rng.choice(xe))))
    return sorted(out)


@pytest.mark.parametrize("case", FULL_CASES)
def test_full_size_sampled(orc, case):
    """The benchmark's full-size lattices in its launch configuration, checked
    on 64 sampled nodes on tile edges after 6 steps: after k steps a node
    depends on the initial fields within radius 3k + 3, so the oracle on a
    periodic window of half-width 3k + 4 reproduces that node exactly.  With
    walls the window is cut at the walls (and closed by walls beyond the
    dependency radius elsewhere)."""
    import math
    import paper_1710_07486_amd as T
    k = 6
    walls = case.endswith("walls")
    if case.startswith("d3q27"):
        wl = W.collision_3d(256, radius=32, ratio=800.0, v_rel=0.04, kappa2=0.2, kappa3=0.2, lattice_ratio=True)
    elif walls:
        wl = W.wall_drops(1024, 1024, radius=200.0, ratio=1000.0)
        wl.T = W.lattice_ratio_temperature("drops_2d", 0, 1000.0)
    else:
        wl = W.drops_2d(1024, ratio=1000.0, seed=0, lattice_ratio=True)
    precision = 1 if case.endswith("mixed") else 0
    say("full size", case)
    po, pl, rho, phi, u = make(orc, wl, precision)
    if case.endswith("reduced"):
        po.glattice = pl.glattice = 1
    if walls:
        ang = dict(theta_rho_lo=math.radians(60.0), theta_phi_lo=math.radians(70.0),
                   theta_rho_hi=math.radians(120.0), theta_phi_hi=math.radians(100.0))
        for key, v in ang.items():
            setattr(po, key, v)
            setattr(pl, key, v)
        pl.walls = 1
    uu = u if np.abs(u).max() > 0 else None
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, uu)
        s.step(k)
        g = {f: s.read(f) for f in ("rho", "phi", "ux", "uy")}
    rng = np.random.default_rng(7)
    nz, ny, nx = wl.shape
    # the wetting ghost reads the wall row's neighbours along the wall: one
    # more node of reach per step there
    r = 3 * k + 4 + (k if walls else 0)
    pts = tile_edge_samples(wl, rng, 64)
    # absolute tolerances: FP64 1e-10 of the field scale; FP32 storage 1e-5 of it
    scale = {"rho": po.rho_l, "phi": po.chi, "ux": 0.05, "uy": 0.05}
    tol = FP64_TOL if precision == 0 else 1e-5
    worst = {k_: 0.0 for k_ in scale}
    for (z, y, x) in pts:
        wz = 1 if nz == 1 else 2 * r + 1
        ylo, yhi, cy = y - r, y + r, r
        if walls:
            ylo, yhi = max(0, y - r), min(ny - 1, y + r)
            cy = y - ylo
        sub = orc.Params(**{**po.__dict__, "nx": 2 * r + 1, "ny": yhi - ylo + 1, "nz": wz})
        rw = np.ascontiguousarray(_window(rho, (z, y, x), r)[:, (ylo - y + r):(yhi - y + r + 1)])
        pw = np.ascontiguousarray(_window(phi, (z, y, x), r)[:, (ylo - y + r):(yhi - y + r + 1)])
        uw = None if uu is None else np.ascontiguousarray(_window(uu, (z, y, x), r)[..., (ylo - y + r):(yhi - y + r + 1), :])
        st = orc.State(sub, rw, pw, uw)
        st.run(k)
        f = st.fields()
        cz = 0 if nz == 1 else r
        for name, ref in (("rho", f["rho"]), ("phi", f["phi"]), ("ux", f["u"][0]), ("uy", f["u"][1])):
            worst[name] = max(worst[name], abs(g[name][z, y, x] - ref[cz, cy, r]) / scale[name])
    print("sampled max error / scale", case, len(pts), "nodes", worst, flush=True)
    for name, v in worst.items():
        assert v <= tol, (case, name, v)


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_3d_collision_stays_finite_and_conserves_mass(orc, precision):
    """The benchmark's D3Q27 256^3 collision (lattice density ratio 800)
    started at the model's own coexistence densities (oracle 1D relaxation):
    600 steps on the GPU stay finite with bounded velocities, and total mass
    is conserved (FP64 to 1e-12 relative; the FP32 storage form to 1e-7)."""
    import paper_1710_07486_amd as T
    wl = W.collision_3d(256, radius=32, ratio=800.0, v_rel=0.04, kappa2=0.2, kappa3=0.2, lattice_ratio=True)
    po = orc.workload_params(wl)
    pd = orc.Params(**{**po.__dict__, "lattice": 1})
    rg, rl = orc.discrete_coexistence(pd, steps=20000, n=256)
    say("3D 256^3 discrete start", precision, rg, rl)
    rho, phi, u = W.fields(wl, rg, rl)
    nz, ny, nx = wl.shape
    pl = T.Params(lattice=1, precision=precision, nx=nx, ny=ny, nz=nz, T=po.T, rho_g=po.rho_g, rho_l=po.rho_l,
                  lambda1=po.lambda1, lambda2=po.lambda2, lambda3=po.lambda3, kappa1=po.kappa1,
                  kappa2=po.kappa2, kappa3=po.kappa3, chi=po.chi, nu=po.nu, mobility=po.mobility,
                  tau_phi=po.tau_phi, diag_every=50)
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, u)
        d0 = s.diagnostics()
        for _ in range(12):
            s.step(50)
            d = s.diagnostics()
            assert d["nonfinite"] == 0 and d["max_u"] < 0.3 and d["min_rho"] > 0
        tol = 1e-12 if precision == 0 else 1e-7
        print("mass drift", d["mass"] / d0["mass"] - 1, "max_u", d["max_u"], flush=True)
        assert abs(d["mass"] / d0["mass"] - 1) < tol


def test_fp32_mixed_errors_at_equilibrium(orc):
    """The FP32-mixed form against the FP64 path on a relaxing lens at
    density ratio 1000 (D2Q9 256^2, 20,000 steps): density, spurious-current
    magnitude and the lens shape (outline lengths of the liquid-gas and the
    two liquid interfaces, which the three angles fix), each against a bar
    stated below."""
    import paper_1710_07486_amd as T
    from paper_1710_07486_amd.calibrate import discrete_coexistence
    from paper_1710_07486_amd.equilibrium import interface_measures
    wl = W.lens(256, 256, radius=40.0, ratio=1000.0, kappa=0.2, seed=7)
    Tt = T.temperature_for_ratio(1000.0)
    ph = wl.physics()
    base = dict(lattice=0, nx=256, ny=256, nz=1, T=Tt, lambda1=ph["lambda1"], lambda2=ph["lambda2"],
                lambda3=ph["lambda3"], kappa1=ph["kappa1"], kappa2=ph["kappa2"], kappa3=ph["kappa3"])
    rg, rl = discrete_coexistence(T.Params(**base))
    rho, phi, _ = W.fields(wl, rg, rl)
    out = {}
    for prec in (T.FP64, T.FP32_MIXED):
        with T.Solver(T.Params(precision=prec, **base)) as s:
            s.init_fields(rho, phi)
            s.step(20000)
            f = {"rho": s.read("rho"), "phi": s.read("phi"),
                 "u": np.sqrt(s.read("ux") ** 2 + s.read("uy") ** 2)}
            f["shape"] = interface_measures(f["rho"], f["phi"], rg, rl, 5.0)
            out[prec] = f
    a, b = out[T.FP64], out[T.FP32_MIXED]
    e_rho = float(np.abs(b["rho"] - a["rho"]).max() / np.abs(a["rho"]).max())
    sc = (a["rho"] - rg) / (rl - rg)
    co = {}
    for name, mask in (("gas", sc < 0.01), ("liquid", sc > 0.99)):
        m64, m32 = float(np.median(a["rho"][mask])), float(np.median(b["rho"][mask]))
        co[name] = abs(m32 - m64) / m64
    u64, u32 = float(a["u"].max()), float(b["u"].max())
    e_shape = float(np.max(np.abs(b["shape"] - a["shape"]) / a["shape"]))
    say(f"FP32-mixed vs FP64 after 20000 steps: max-norm rho {e_rho:.2e}; coexistence densities gas "
        f"{co['gas']:.2e}, liquid {co['liquid']:.2e}; spurious max|u| {u64:.4e} vs {u32:.4e}; shape {e_shape:.2e}")
    # Bars: the shape (outline lengths) within 1e-4, the bulk densities
    # within the precision form's 1e-5 of the liquid's (the gas's 1e-4 of its
    # own: FP32 rounding of the liquid-scale populations) and the spurious
    # currents within 1 %.  The max-norm density error sits on the
    # interfaces, where it is an interface displacement times the density's
    # slope: its bar follows from the shape bar, a displacement of 1e-4 of
    # the radius at twice the steepest relative slope of the FP64 field.
    gy, gx = np.gradient(a["rho"][0])
    slope = float(np.hypot(gx, gy).max() / np.abs(a["rho"]).max())
    e_rho_bar = 2.0 * 1e-4 * 40.0 * slope
    print("max-norm bar from the shape bar", e_rho_bar, flush=True)
    assert e_shape < 1e-4
    assert e_rho < e_rho_bar
    assert co["gas"] < 1e-4 and co["liquid"] < 1e-5
    assert abs(u32 - u64) < 0.01 * u64
