"""GPU runs of the three-liquid solver (telbm_nl_*) against the oracle's
three-liquid model and against closed forms.

Parity: drops of the three liquids in gas with unequal kappas (so the
mobility matrix is full), D2Q9 with ragged tiles and D3Q27 single- and
multi-tile and across z-columns, every field within 1e-10 of the oracle.  Consistency: the
oracle pin's flat liquid-1 / liquid-3 interface, the GPU within 1e-9 of the
oracle and its absent liquid 2 below the density perturbation.
Neumann angles: a lens of liquid 1 between liquids 2 and 3 (no gas) at
twice the oracle pin's size relaxes to the angles of the closed-form
tensions within the paper's 3 degrees.  Full size: the benchmark's 256^3
three-liquid state on sampled tile-edge nodes within 1e-10 of the field
scales.
"""
import numpy as np
import pytest

from tests.test_oracle_nliquid import _flat13, lens3_fields, lens3_prediction  # noqa: F401
from tests import neumann as NM

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "phi", "psi", "u", "c", "mu", "force")


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b, floor=1e-300):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))


def lib_params(po, lattice, shape):
    import paper_1710_07486_amd as T
    nz, ny, nx = shape
    return T.Params(lattice=lattice, precision=T.FP64, nx=nx, ny=ny, nz=nz, T=po.T, rho_g=po.rho_g, rho_l=po.rho_l,
                    lambda1=po.lambda1, lambda2=po.lambda2, lambda3=po.lambda3, kappa1=po.kappa1, kappa2=po.kappa2,
                    kappa3=po.kappa3, chi=po.chi, nu=po.nu, mobility=po.mobility, tau_phi=po.tau_phi)


def four_phase(shape, po, seed=0):
    """Drops of liquids 1, 2 and 3 in gas (3D: spheres), with a weak seeded
    velocity field so that every term of the step is exercised."""
    nz, ny, nx = shape
    grid = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    z, y, x = grid
    R = 0.2 * min(nx, ny) if nz == 1 else 0.4 * min(ny, nz)
    cs = []
    for cx in (0.2, 0.5, 0.8):
        d = np.sqrt((x - cx * nx) ** 2 + (y - ny / 2 + 0.3) ** 2 + ((z - nz / 2) ** 2 if nz > 1 else 0.0))
        cs.append(0.5 * (1 - np.tanh((d - R) / 2.0)))
    c1, c2, c3 = cs
    rho = po.rho_g + (po.rho_l - po.rho_g) * (c1 + c2 + c3)
    phi = po.chi * (c1 - c2)
    psi = po.chi * c3
    rng = np.random.default_rng(seed)
    u = 0.01 * rng.standard_normal((3,) + shape)
    if nz == 1:
        u[2] = 0.0
    return rho, phi, psi, u


def run_both(orc, po, nl, lattice, shape, steps, fields):
    from paper_1710_07486_amd import nliquid as NL
    rho, phi, psi, u = fields
    st = orc.NLState(po, nl, rho, phi, psi, u)
    st.run(steps)
    fo = st.fields()
    with NL.NLSolver(lib_params(po, lattice, shape), NL.NLParams(lambda4=nl.lambda4, kappa4=nl.kappa4)) as s:
        s.init_fields(rho, phi, psi, u)
        s.step(steps)
        fg = s.fields()
    return fo, fg


def errors(fo, fg):
    e = {}
    for k in FIELDS:
        floor = 1e-14 if k in ("u", "force") else 1e-300
        e[k] = rel(fg[k], fo[k], floor)
    return e


# D3Q27 depths: single short z-columns, and (33) a full 32-plane column with
# a one-plane remainder, so that the column-end sums of (rho, phi) and of psi
# cross between columns
CASES = {"d2q9_100x37": (0, (1, 37, 100), 300), "d3q27_40x18x12": (1, (12, 18, 40), 60),
         "d3q27_200x13x9": (1, (9, 13, 200), 60), "d3q27_20x9x33": (1, (33, 9, 20), 60)}


@pytest.mark.parametrize("case", list(CASES))
def test_three_liquid_parity(orc, case):
    lattice, shape, steps = CASES[case]
    nz, ny, nx = shape
    po = orc.coexisting_params(10.0, lattice=lattice, nx=nx, ny=ny, nz=nz, kappa2=0.03, lambda2=0.09375,
                               kappa3=0.06, lambda3=0.1875)
    nl = orc.NLParams(kappa4=0.05, lambda4=0.15625)
    say("three liquids", case, steps, "steps")
    fo, fg = run_both(orc, po, nl, lattice, shape, steps, four_phase(shape, po))
    assert np.isfinite(fo["rho"]).all()
    assert np.abs(fo["psi"]).max() > 0.2 * po.chi  # liquid 3 present
    e = errors(fo, fg)
    print("errors", e, flush=True)
    for k, v in e.items():
        assert v <= 1e-10, (k, v)


def test_absent_liquid_at_a_liquid_liquid_interface(orc):
    """The oracle pin's flat liquid-1 / liquid-3 interface: the GPU within
    1e-9 of the oracle after 2000 steps (later a net momentum seeded by
    round-off grows, in the two-liquid model too, so that the runs part), and
    its absent liquid 2 below the density perturbation through 10^4 steps."""
    from paper_1710_07486_amd import nliquid as NL
    n = 64
    po = orc.coexisting_params(10.0, nx=n, ny=1, nz=1)
    nl = orc.NLParams(kappa4=2 * po.kappa2, lambda4=2 * po.lambda2)
    rho, phi, psi = _flat13(n, po)
    say("liquid-1 / liquid-3 interface")
    st = orc.NLState(po, nl, rho, phi, psi)
    st.run(2000)
    fo = st.fields()
    worst = 0.0
    with NL.NLSolver(lib_params(po, 0, (1, 1, n)), NL.NLParams(lambda4=nl.lambda4, kappa4=nl.kappa4)) as s:
        s.init_fields(rho, phi, psi)
        for k in range(5):
            s.step(2000)
            fg = s.fields()
            if k == 0:
                e = {key: rel(fg[key], fo[key]) for key in ("rho", "phi", "psi", "c", "mu")}
                print("errors after 2000 steps", e, flush=True)
                for key, v in e.items():
                    assert v <= 1e-9, (key, v)
            cl = 1 - (fg["rho"] - po.rho_l) / (po.rho_g - po.rho_l)
            worst = max(worst, np.abs(fg["c"][1]).max() / np.abs(1 - cl).max())
    print("max |C2| / max |1 - C_L| over 10^4 steps:", worst, flush=True)
    assert worst < 1.0


def test_three_liquid_lens_neumann_angles(orc):
    from paper_1710_07486_amd import nliquid as NL
    k1, k2, k3 = 0.08, 0.1, 0.1
    nx, ny, R = 192, 128, 28.0
    po = orc.coexisting_params(100.0, nx=nx, ny=ny, nz=1, kappa2=k1, lambda2=k1, kappa3=k2, lambda3=k2)
    pred = lens3_prediction(k1, k2, k3)
    band = (ny // 4, ny // 4 + ny * 3 // 8)
    phi, psi = lens3_fields(nx, ny, R, band, po.chi)
    say("three-liquid lens", nx, ny, R)
    with NL.NLSolver(lib_params(po, 0, (1, ny, nx)), NL.NLParams(kappa4=k3, lambda4=k3)) as s:
        s.init_fields(np.full_like(phi, po.rho_l), phi, psi)
        s.step(80000)
        c = np.stack([s.read(k)[0] for k in ("c1", "c2", "c3")])
    ang, fits = NM.measure_angles_c(c[0], c[1], c[2], band[1] - 0.5)
    print("triangle", pred, "lens", ang, "fits", fits, flush=True)
    for a in ang:
        for ph in ("1", "2", "g"):
            assert abs(a[ph] - pred[ph]) < 3.0, (ph, a[ph], pred[ph])


def test_three_liquid_full_size_sampled(orc):
    """The benchmark's three-liquid 256^3 state (the D3Q27 collision of two
    drops, the second one liquid 3) in its launch configuration, checked on
    48 nodes on tile edges after 4 steps: after k steps a node depends on
    the initial fields within radius 3k + 3, so the oracle on a periodic
    window of half-width 3k + 4 reproduces that node exactly."""
    from paper_1710_07486_amd import nliquid as NL
    from synth import workloads as W
    from tests.test_gpu_parity import _window, tile_edge_samples
    k = 4
    wl = W.collision_3d(256, radius=32, ratio=800.0, v_rel=0.04, kappa2=0.2, kappa3=0.2, lattice_ratio=True)
    po = orc.workload_params(wl)
    rho, phi2, u = W.fields(wl, po.rho_g, po.rho_l)
    psi = np.maximum(-phi2, 0.0)
    phi = np.maximum(phi2, 0.0)
    del phi2
    nl = orc.NLParams(lambda4=po.lambda2, kappa4=po.kappa2)
    say("three liquids, full size", wl.shape)
    names = ("rho", "phi", "psi", "ux", "uy", "uz")
    with NL.NLSolver(lib_params(po, 1, wl.shape), NL.NLParams(lambda4=nl.lambda4, kappa4=nl.kappa4)) as s:
        s.init_fields(rho, phi, psi, u)
        s.step(k)
        g = {f: s.read(f) for f in names}
    rng = np.random.default_rng(8)
    r = 3 * k + 4
    pts = tile_edge_samples(wl, rng, 48)
    scale = {"rho": po.rho_l, "phi": po.chi, "psi": po.chi, "ux": 0.05, "uy": 0.05, "uz": 0.05}
    worst = {n: 0.0 for n in names}
    for (z, y, x) in pts:
        sub = orc.Params(**{**po.__dict__, "nx": 2 * r + 1, "ny": 2 * r + 1, "nz": 2 * r + 1})
        win = [np.ascontiguousarray(_window(a, (z, y, x), r)) for a in (rho, phi, psi, u)]
        st = orc.NLState(sub, nl, *win)
        st.run(k)
        f = st.fields()
        ref = {"rho": f["rho"], "phi": f["phi"], "psi": f["psi"], "ux": f["u"][0], "uy": f["u"][1], "uz": f["u"][2]}
        for n in names:
            worst[n] = max(worst[n], abs(g[n][z, y, x] - ref[n][r, r, r]) / scale[n])
    print("sampled max error / scale", len(pts), "nodes", worst, flush=True)
    for n, v in worst.items():
        assert v <= 1e-10, (n, v)
