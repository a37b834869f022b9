"""GPU checks of the batched form: uneven instances advanced together must
match each instance run alone (the node arithmetic is shared; the single D2Q9
solver sums the next step's moments per tile row and completes them at tile
edges, the batch sums them per node, so the two agree to round-off), for
every grid size and across graph replays; every tile shape of the batch gives
the same bits; one instance is checked against the FP64 oracle; the FP32 form
against the FP64 form; members in channels between wetting walls beside
periodic ones match their single runs in every mode and the oracle."""
import numpy as np
import pytest

from synth import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


SIZES = [(48, 40), (64, 64), (37, 50), (100, 30), (70, 71)]


def instances(orc, precision=0, sizes=SIZES):
    import paper_1710_07486_amd as T
    out = []
    rng = np.random.default_rng(5)
    for k, (nx, ny) in enumerate(sizes):
        ratio = float(rng.uniform(100, 1000))
        kap = float(rng.uniform(0.05, 0.2))
        wl = W.lens(nx, ny, radius=min(nx, ny) / 6, ratio=ratio, kappa=kap, seed=100 + k)
        v = float(rng.uniform(0.0, 0.04))
        wl.drops[0]["velocity"] = (v / 2, 0.0, 0.0)
        wl.drops[1]["velocity"] = (-v / 2, 0.0, 0.0)
        po = orc.coexisting_params(wl.ratio, **wl.physics())
        rho, phi, u = W.fields(wl, po.rho_g, po.rho_l)
        pl = T.Params(lattice=0, precision=precision, nx=nx, ny=ny, nz=1, T=po.T, rho_g=po.rho_g, rho_l=po.rho_l,
                      lambda1=po.lambda1, lambda2=po.lambda2, lambda3=po.lambda3, kappa1=po.kappa1,
                      kappa2=po.kappa2, kappa3=po.kappa3, chi=po.chi, nu=po.nu, mobility=po.mobility,
                      tau_phi=po.tau_phi)
        out.append((po, pl, rho, phi, u))
    return out


def run_single(pl, rho, phi, u, steps):
    import paper_1710_07486_amd as T
    with T.Solver(pl) as s:
        s.init_fields(rho, phi, u)
        s.step(steps)
        return {k: s.read(k) for k in ("rho", "phi", "ux", "uy")}


def test_batch_matches_single(orc):
    from paper_1710_07486_amd.batch import Batch
    inst = instances(orc)
    steps = 24  # two graph replays of 10 steps plus 4 eager steps
    say("batch of", len(inst), "vs single solvers")
    singles = [run_single(pl, r, p, u, steps) for (_, pl, r, p, u) in inst]
    with Batch([pl for (_, pl, *_r) in inst]) as b:
        for i, (_, pl, r, p, u) in enumerate(inst):
            b.init_fields(i, r, p, u)
        b.step(steps)
        assert b.steps == steps
        for i in range(len(inst)):
            for k in ("rho", "phi", "ux", "uy"):
                got, ref = b.read(i, k), singles[i][k]
                err = np.abs(got - ref).max() / np.abs(ref).max()
                assert err <= 1e-12, (i, k, err)


def test_batch_tile_shapes_agree(orc):
    from paper_1710_07486_amd.batch import Batch, tile_variants
    inst = instances(orc, sizes=SIZES[:3])
    ref = None
    for v, shape in enumerate(tile_variants()):
        for wg in (1, 3):
            say("tile variant", v, shape, "wg/cu", wg)
            with Batch([pl for (_, pl, *_r) in inst]) as b:
                b.set_tiles(v, wg)
                for i, (_, pl, r, p, u) in enumerate(inst):
                    b.init_fields(i, r, p, u)
                b.step(12)
                res = [b.read(i, "rho") for i in range(len(inst))]
            if ref is None:
                ref = res
            for a, c in zip(res, ref):
                assert np.array_equal(a, c)


def test_batch_instance_vs_oracle(orc):
    from paper_1710_07486_amd.batch import Batch
    inst = instances(orc)
    steps = 40
    say("batch instance 3 vs oracle")
    po, pl, r, p, u = inst[3]
    st = orc.State(po, r, p, u[:2])
    st.run(steps)
    ref = st.fields()
    with Batch([x[1] for x in inst]) as b:
        for i, (_, pl_, r_, p_, u_) in enumerate(inst):
            b.init_fields(i, r_, p_, u_)
        b.step(steps)
        got = b.read(3, "rho")
        gphi = b.read(3, "phi")
    assert np.abs(got - ref["rho"]).max() / np.abs(ref["rho"]).max() < 1e-10
    assert np.abs(gphi - ref["phi"]).max() / np.abs(ref["phi"]).max() < 1e-10


def test_batch_fp32_mixed_vs_fp64(orc):
    from paper_1710_07486_amd.batch import Batch
    i64 = instances(orc, 0)
    i32 = instances(orc, 1)
    steps = 60
    say("batch FP32-mixed vs FP64")
    out = {}
    for tag, inst in (("64", i64), ("32", i32)):
        with Batch([x[1] for x in inst]) as b:
            for i, (_, pl, r, p, u) in enumerate(inst):
                b.init_fields(i, r, p, u)
            b.step(steps)
            out[tag] = [b.read(i, "rho") for i in range(len(inst))]
    errs = [float(np.abs(a - c).max() / np.abs(c).max()) for a, c in zip(out["32"], out["64"])]
    print("per-instance relative density error", errs, flush=True)
    assert max(errs) < 1e-5


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_mixed_equations_of_state(orc, mode):
    """Members with Carnahan-Starling (ratio 100), van der Waals (ratio 100)
    and Peng-Robinson (ratio 1000) free energies in one batch: each matches
    the FP64 oracle run of its own free energy, in every batch mode (the
    one-launch mode runs one launch per free energy present)."""
    import paper_1710_07486_amd as T
    from paper_1710_07486_amd.batch import Batch
    cases = [(dict(eos=0), 100.0, (48, 40)), (dict(eos=1, a=2.0 / 49.0, b=2.0 / 21.0), 100.0, (64, 50)),
             (dict(eos=2, a=2.0 / 49.0, b=2.0 / 21.0), 1000.0, (37, 60))]
    inst = []
    for k, (e, ratio, (nx, ny)) in enumerate(cases):
        wl = W.lens(nx, ny, radius=min(nx, ny) / 6, ratio=ratio, kappa=0.1, seed=200 + k)
        po = orc.coexisting_params(wl.ratio, **wl.physics(), **e)
        rho, phi, u = W.fields(wl, po.rho_g, po.rho_l)
        pl = T.Params(lattice=0, nx=nx, ny=ny, nz=1, T=po.T, rho_g=po.rho_g, rho_l=po.rho_l, eos=po.eos, a=po.a,
                      b=po.b, omega=po.omega, lambda1=po.lambda1, lambda2=po.lambda2, lambda3=po.lambda3,
                      kappa1=po.kappa1, kappa2=po.kappa2, kappa3=po.kappa3, chi=po.chi, nu=po.nu,
                      mobility=po.mobility, tau_phi=po.tau_phi)
        inst.append((po, pl, rho, phi))
    steps = 60
    say("batch with CS, vdW and PR members vs oracle, mode", mode)
    with Batch([x[1] for x in inst]) as b:
        for i, (_, _pl, r, p) in enumerate(inst):
            b.init_fields(i, r, p, None)
        b.set_mode(mode)
        b.step(steps)
        got = [(b.read(i, "rho"), b.read(i, "phi")) for i in range(len(inst))]
    for i, (po, _pl, r, p) in enumerate(inst):
        st = orc.State(po, r, p, None)
        st.run(steps)
        ref = st.fields()
        assert np.isfinite(ref["rho"]).all()
        for g, key in zip(got[i], ("rho", "phi")):
            err = np.abs(g - ref[key]).max() / np.abs(ref[key]).max()
            assert err < 1e-10, (i, key, err)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_fused_mode_matches_single(orc, precision, mode):
    """The fused modes (the single solver's fused step per instance on graph
    branches, or for all instances in one launch) give the single runs'
    results: 4 eager steps then two graph chunks of 10."""
    from paper_1710_07486_amd.batch import Batch
    inst = instances(orc, precision)
    steps = 24
    say("batch fused mode", mode, "vs single solvers, precision", precision)
    singles = [run_single(pl, r, p, u, steps) for (_, pl, r, p, u) in inst]
    with Batch([pl for (_, pl, *_r) in inst]) as b:
        b.set_mode(mode)
        for i, (_, pl, r, p, u) in enumerate(inst):
            b.init_fields(i, r, p, u)
        b.step(4)
        b.step(20)
        for i in range(len(inst)):
            for k in ("rho", "phi", "ux", "uy"):
                got, ref = b.read(i, k), singles[i][k]
                err = np.abs(got - ref).max() / np.abs(ref).max()
                assert err <= 1e-12, (i, k, err)


def test_switching_modes_and_reading_mid_run(orc):
    """Persistent 6 steps, fused per instance 10 (a graph chunk), a read,
    fused in one launch 11, persistent 3: the state carries over and matches
    30 single steps."""
    from paper_1710_07486_amd.batch import Batch
    inst = instances(orc, 0)
    say("batch mode switching")
    singles = [run_single(pl, r, p, u, 30) for (_, pl, r, p, u) in inst]
    with Batch([pl for (_, pl, *_r) in inst]) as b:
        for i, (_, pl, r, p, u) in enumerate(inst):
            b.init_fields(i, r, p, u)
        b.step(6)
        b.set_mode(1)
        b.step(10)
        b.read(2, "rho")
        b.set_mode(2)
        b.step(11)
        b.set_mode(0)
        b.step(3)
        assert b.steps == 30
        for i in range(len(inst)):
            for k in ("rho", "phi", "ux"):
                got, ref = b.read(i, k), singles[i][k]
                err = np.abs(got - ref).max() / np.abs(ref).max()
                assert err <= 1e-12, (i, k, err)


def full_batch():
    """The 64-instance batch workload (sides U{256..1024}, ratio U[100, 1000],
    seed 3) at full size, started at each instance's Maxwell densities:
    FP64 and FP32-mixed parameters, and the initial fields."""
    import dataclasses
    import paper_1710_07486_amd as T
    params, fields = [], []
    for wl in W.batch_instances(64, seed=3, lo=256, hi=1024):
        t = T.temperature_for_ratio(wl.ratio)
        rg, rl, _, _ = T.coexistence(t)
        ph = wl.physics()
        nz, ny, nx = wl.shape
        params.append(T.Params(lattice=0, precision=0, nx=nx, ny=ny, nz=1, T=t, rho_g=rg, rho_l=rl,
                               lambda1=ph["lambda1"], lambda2=ph["lambda2"], lambda3=ph["lambda3"],
                               kappa1=ph["kappa1"], kappa2=ph["kappa2"], kappa3=ph["kappa3"], chi=ph["chi"],
                               nu=ph["nu"], mobility=ph["mobility"], tau_phi=ph["tau_phi"]))
        fields.append(W.fields(wl, rg, rl))
    return params, [dataclasses.replace(p, precision=1) for p in params], fields


SAMPLED = (0, 21, 42, 63)


def test_full_size_batch_modes_fp32_vs_fp64():
    """The full 64-instance workload (27.4 M nodes), 40 steps: the FP64
    batch in the one-launch mode equals single-solver FP64 runs of sampled
    instances to round-off; the FP32-mixed batch, in the persistent and the
    one-launch mode, is within 1e-5 of the FP64 batch for every instance."""
    from paper_1710_07486_amd.batch import Batch
    steps = 40
    say("full-size batch: coexistence temperatures and fields of 64 instances (host, ~30 s)")
    p64, p32, fields = full_batch()
    say("full-size batch, FP64 one-launch mode")
    with Batch(p64) as b:
        for i, (r, ph, u) in enumerate(fields):
            b.init_fields(i, r, ph, u)
        b.set_mode(2)
        b.step(steps)
        ref = [b.read(i, "rho") for i in range(len(p64))]
        phi_ref = {i: b.read(i, "phi") for i in SAMPLED}
    for i in SAMPLED:
        say("single FP64 run of instance", i, p64[i].nx, p64[i].ny)
        single = run_single(p64[i], *fields[i], steps)
        for k, got in (("rho", ref[i]), ("phi", phi_ref[i])):
            err = np.abs(got - single[k]).max() / np.abs(single[k]).max()
            assert err <= 1e-12, (i, k, err)
    for mode in (0, 2):
        say("full-size batch, FP32-mixed, mode", mode)
        with Batch(p32) as b:
            for i, (r, ph, u) in enumerate(fields):
                b.init_fields(i, r, ph, u)
            b.set_mode(mode)
            b.step(steps)
            errs = [float(np.abs(b.read(i, "rho") - ref[i]).max() / np.abs(ref[i]).max()) for i in range(len(p32))]
        print("mode", mode, "max relative density error over instances", max(errs), flush=True)
        assert all(np.isfinite(errs)) and max(errs) < 1e-5, (mode, max(errs))


WALL_ANGLES = [(60.0, 70.0, 120.0, 100.0), (100.0, 110.0, 75.0, 60.0)]


def wall_instances(orc, precision=0):
    """Two periodic lens members and two members in channels between wetting
    walls (caps of both liquids on the walls), each with its own angles."""
    import math
    import paper_1710_07486_amd as T
    out = instances(orc, precision, sizes=[(48, 40), (37, 50)])
    for (nx, ny), ang in zip([(64, 32), (100, 37)], WALL_ANGLES):
        wl = W.wall_drops(nx, ny, radius=min(12.0, 0.3 * nx), ratio=100.0)
        po = orc.coexisting_params(wl.ratio, **wl.physics())
        th = dict(zip(("theta_rho_lo", "theta_phi_lo", "theta_rho_hi", "theta_phi_hi"), map(math.radians, ang)))
        for key, v in th.items():
            setattr(po, key, v)
        po.walls = 1
        rho, phi, u = W.fields(wl, po.rho_g, po.rho_l)
        pl = T.Params(lattice=0, precision=precision, nx=nx, ny=ny, nz=1, T=po.T, rho_g=po.rho_g, rho_l=po.rho_l,
                      lambda1=po.lambda1, lambda2=po.lambda2, lambda3=po.lambda3, kappa1=po.kappa1,
                      kappa2=po.kappa2, kappa3=po.kappa3, chi=po.chi, nu=po.nu, mobility=po.mobility,
                      tau_phi=po.tau_phi, walls=1, **th)
        out.append((po, pl, rho, phi, u))
    return out


@pytest.mark.parametrize("mode,precision", [(0, 0), (1, 0), (2, 0), (1, 1), (2, 1)])
def test_batch_with_walls_matches_single(orc, mode, precision):
    """Members with and without walls in one batch: each equals its single
    run (4 eager steps, then two graph chunks of 10) in every mode."""
    from paper_1710_07486_amd.batch import Batch
    inst = wall_instances(orc, precision)
    steps = 24
    say("batch with walled members, mode", mode, "precision", precision)
    singles = [run_single(pl, r, p, u, steps) for (_, pl, r, p, u) in inst]
    with Batch([pl for (_, pl, *_r) in inst]) as b:
        b.set_mode(mode)
        for i, (_, pl, r, p, u) in enumerate(inst):
            b.init_fields(i, r, p, u)
        b.step(4)
        b.step(20)
        for i in range(len(inst)):
            for k in ("rho", "phi", "ux", "uy"):
                got, ref = b.read(i, k), singles[i][k]
                err = np.abs(got - ref).max() / np.abs(ref).max()
                assert err <= 1e-12, (i, k, err)


@pytest.mark.parametrize("mode", [0, 2])
def test_batch_wall_member_vs_oracle(orc, mode):
    """A walled member of a mixed batch against the FP64 oracle (1e-10)."""
    from paper_1710_07486_amd.batch import Batch
    inst = wall_instances(orc, 0)
    steps = 40
    po, pl, rho, phi, u = inst[3]
    say("batch walled member vs oracle, mode", mode)
    uu = u if np.abs(u).max() > 0 else None
    st = orc.State(po, rho, phi, uu)
    st.run(steps)
    fo = st.fields()
    with Batch([p for (_, p, *_r) in inst]) as b:
        b.set_mode(mode)
        for i, (_, p, r, ph, uv) in enumerate(inst):
            b.init_fields(i, r, ph, uv)
        b.step(steps)
        got = {k: b.read(3, k) for k in ("rho", "phi", "ux")}
    assert np.isfinite(fo["rho"]).all()
    for key, ref in (("rho", fo["rho"]), ("phi", fo["phi"]), ("ux", fo["u"][0])):
        err = np.abs(got[key] - ref).max() / max(np.abs(ref).max(), 1e-14)
        assert err < 1e-10, (key, err)
