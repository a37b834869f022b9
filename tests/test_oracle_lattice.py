"""Pins of the oracle's whole time step against what the continuum equations
(5)-(7) and the free energy (1)-(3) fix: conservation, momentum bookkeeping,
exact fixed points, the Navier-Stokes shear-wave decay rate, the linearised
Cahn-Hilliard growth rate, reflection symmetry, the flat liquid-liquid tanh
profile and the Maxwell coexistence densities.
"""
import numpy as np
import pytest

import synth
from synth import workloads as W


def lens_state(orc, lattice=0, n=32, ratio=10.0, kappa=0.045, seed=0):
    if lattice == 0:
        w = W.lens(n, n, radius=n / 6, ratio=ratio, kappa=kappa, seed=seed)
        u = None
    else:
        w = W.collision_3d(n, radius=n / 6, ratio=ratio, v_rel=0.02, kappa2=kappa, kappa3=kappa, seed=seed)
    p = orc.coexisting_params(w.ratio, **w.physics())
    rho, phi, u = W.fields(w, p.rho_g, p.rho_l)
    return p, orc.State(p, rho, phi, u if lattice else None)


@pytest.mark.parametrize("lattice,n,ratio", [(0, 48, 10.0), (0, 48, 1000.0), (1, 16, 10.0), (1, 16, 1000.0)])
def test_mass_conservation_and_momentum_bookkeeping(orc, lattice, n, ratio):
    p, st = lens_state(orc, lattice, n, ratio)
    steps = 200 if lattice == 0 else 40
    d = st.run(steps, diag=True)
    mass, phit, j, F = d[:, 0], d[:, 1], d[:, 2:5], d[:, 5:8]
    assert np.abs(mass / mass[0] - 1).max() < 1e-13
    assert np.abs(phit - phit[0]).max() < 1e-13 * np.abs(mass[0])
    # sum_x j^{n+1} - sum_x j^n = sum_x F^n (the force is not a divergence discretely)
    jump = j[1:] - j[:-1]
    assert np.abs(jump - F[:-1]).max() < 1e-12 * mass[0]
    assert np.isfinite(d).all()


def test_uniform_states_are_fixed_points(orc):
    for lattice, shape in ((0, (1, 8, 10)), (1, (4, 5, 6))):
        p = orc.coexisting_params(10.0, lattice=lattice, nx=shape[2], ny=shape[1], nz=shape[0])
        for phi0 in (p.chi, -p.chi):
            rho = np.full(shape, p.rho_l)
            phi = np.full(shape, phi0)
            u = np.zeros((3,) + shape)
            u[0] = 0.05
            u[1] = -0.03
            st = orc.State(p, rho, phi, u[:2] if lattice == 0 else u)
            f0, g0 = st.f.copy(), st.g.copy()
            st.run(5)
            assert np.abs(st.f - f0).max() < 1e-14 and np.abs(st.g - g0).max() < 1e-14


@pytest.mark.parametrize("lattice", [0, 1])
def test_shear_wave_decay_rate(orc, lattice):
    """u_x = U sin(2 pi y / L) decays as exp(-nu k^2 t) with nu = (tau - 1/2)/3,
    Navier-Stokes (Eq. 6) at uniform density."""
    L = 64
    shape = (1, L, 4) if lattice == 0 else (2, L, 2)
    nu = 0.1
    p = orc.coexisting_params(10.0, lattice=lattice, nx=shape[2], ny=shape[1], nz=shape[0], nu=nu)
    y = np.arange(L)[None, :, None] * np.ones(shape)
    k = 2 * np.pi / L
    U = 1e-4
    u = np.zeros((3,) + shape)
    u[0] = U * np.sin(k * y)
    st = orc.State(p, np.full(shape, p.rho_l), np.full(shape, p.chi), u if lattice else u[:2])
    st.run(50)  # let the initial (equilibrium-start) layer decay
    a0 = np.sum(st.fields()["u"][0] * np.sin(k * y))
    t = 300
    st.run(t)
    a1 = np.sum(st.fields()["u"][0] * np.sin(k * y))
    rate = -np.log(a1 / a0) / t
    assert abs(rate / (nu * k ** 2) - 1) < 1e-3


def test_linear_cahn_hilliard_growth(orc):
    """phi = eps cos(kx) at rho = rho_l, phi0 = 0 (C1 = C2 = 1/2, the spinodal
    point of the double wells): the linearised Eq. (7) gives
    d phi_k/dt = M s(k) [mu_b'(0) - 2 B s(k)] phi_k with s(k) = 2cos k - 2 and
    mu_b'(0) = -(lambda2 + lambda3)/(8 chi^2)."""
    nx = 128
    p = orc.coexisting_params(10.0, lattice=0, nx=nx, ny=1, nz=1, kappa2=0.3, kappa3=0.3,
                              lambda2=0.9375, lambda3=0.9375, mobility=0.05, tau_phi=1.0)
    A, Bc, D = orc.gradient_coefficients(p)
    x = np.arange(nx)[None, None, :].astype(float)
    for m in (1, 2):
        k = 2 * np.pi * m / nx
        eps = 1e-6
        st = orc.State(p, np.full((1, 1, nx), p.rho_l), eps * np.cos(k * x))
        t = 400
        a0 = np.sum(st.fields()["phi"] * np.cos(k * x))
        st.run(t)
        a1 = np.sum(st.fields()["phi"] * np.cos(k * x))
        s = 2 * np.cos(k) - 2
        mub = -(p.lambda2 + p.lambda3) / (8 * p.chi ** 2)
        want = p.mobility * s * (mub - 2 * Bc * s)
        got = np.log(a1 / a0) / t
        assert abs(got / want - 1) < 1e-2


def test_reflection_symmetry(orc):
    """Mirroring the initial fields in x mirrors the solution and flips u_x."""
    p, st = lens_state(orc, 0, 32, 10.0)
    w = W.lens(32, 32, radius=32 / 6, ratio=10.0, kappa=0.045)
    rho, phi, _ = W.fields(w, p.rho_g, p.rho_l)
    rho2, phi2 = rho[..., ::-1].copy(), phi[..., ::-1].copy()
    st2 = orc.State(p, rho2, phi2)
    st.run(60)
    st2.run(60)
    a, b = st.fields(), st2.fields()
    assert np.abs(a["rho"][..., ::-1] - b["rho"]).max() < 1e-12
    assert np.abs(a["phi"][..., ::-1] - b["phi"]).max() < 1e-12
    assert np.abs(a["u"][0][..., ::-1] + b["u"][0]).max() < 1e-12
    assert np.abs(a["u"][1][..., ::-1] - b["u"][1]).max() < 1e-12


def test_flat_liquid_liquid_interface(orc):
    """With lambda2/kappa2 = lambda3/kappa3 the liquid-liquid interface is
    rho = rho_l and phi = chi tanh(x / W), W = 2 sqrt(kappa/lambda) (continuum).
    Checked at lambda = kappa / 2 (W = 2.83 lattice units), a width the lattice
    resolves; the paper's lambda = 3.125 kappa gives W = 1.13."""
    nx = 128
    kap, lam = 0.2, 0.1
    p = orc.coexisting_params(10.0, lattice=0, nx=nx, ny=1, nz=1, kappa2=kap, kappa3=kap,
                              lambda2=lam, lambda3=lam)
    x = np.arange(nx, dtype=float)
    W0 = 2 * np.sqrt(kap / lam)
    phi0 = p.chi * np.tanh((x - nx / 4) / 3.0) * np.tanh((3 * nx / 4 - x) / 3.0)
    st = orc.State(p, np.full((1, 1, nx), p.rho_l), phi0.reshape(1, 1, nx))
    st.run(3000)
    f = st.fields()
    assert np.abs(f["rho"] - p.rho_l).max() / p.rho_l < 3e-3
    # interface position near nx/4 by linear interpolation of the zero of phi
    ph = f["phi"][0, 0]
    i = int(np.argmin(np.abs(ph[: nx // 2])))
    j = i if ph[i] * ph[i + 1] <= 0 else i - 1
    x0 = j - ph[j] / (ph[j + 1] - ph[j])
    sel = slice(nx // 8, 3 * nx // 8)
    prof = p.chi * np.tanh((x[sel] - x0) / W0)
    assert np.abs(ph[sel] - prof).max() / p.chi < 2e-2


def test_flat_liquid_gas_coexistence(orc):
    """Bulk densities of a flat liquid-gas slab approach the Maxwell densities,
    and more closely as the interface widens (kappa1 up)."""
    nx = 160
    errs = []
    for k1 in (0.003, 0.03):
        p = orc.coexisting_params(10.0, lattice=0, nx=nx, ny=1, nz=1, kappa1=k1, kappa2=0.1,
                                  kappa3=0.1, lambda2=0.3125, lambda3=0.3125)
        x = np.arange(nx, dtype=float)
        c1 = 0.5 * (np.tanh((x - nx / 4) / 3.0) - np.tanh((x - 3 * nx / 4) / 3.0))
        st = orc.State(p, (p.rho_g + (p.rho_l - p.rho_g) * c1).reshape(1, 1, nx), (p.chi * c1).reshape(1, 1, nx))
        st.run(5000)
        f = st.fields()
        errs.append((f["rho"][0, 0, 0] / p.rho_g - 1, f["rho"][0, 0, nx // 2] / p.rho_l - 1))
        assert np.abs(f["u"]).max() < 1e-3
    assert abs(errs[1][1]) < 1e-2 and abs(errs[1][0]) < 3e-2
    assert abs(errs[1][0]) < abs(errs[0][0]) and abs(errs[1][1]) < abs(errs[0][1])


def _slab(orc, p, steps=20000, n=128, width=2.0):
    import dataclasses
    q = dataclasses.replace(p, nx=n, ny=1, nz=1)
    x = np.arange(n, dtype=float)
    c1 = 0.5 * (np.tanh((x - n / 4) / width) - np.tanh((x - 3 * n / 4) / width))
    st = orc.State(q, (p.rho_g + (p.rho_l - p.rho_g) * c1).reshape(1, 1, n), (q.chi * c1).reshape(1, 1, n))
    st.run(steps)
    return st.fields()


def test_coexistence_maxwell_near_critical_and_sharp_interface_offset(orc):
    """Maxwell construction of Eq. (4) (equal pressure, equal chemical
    potential; the paper's coexistence figure): a flat slab of liquid 1 in gas
    with the paper's lambda1 = 0.6, kappa1 = 1e-3 relaxes to the Maxwell
    densities where the lattice resolves the interface, i.e. near the critical
    point (T/T_c = 0.99, 0.98, 0.95 at Maxwell ratios 1.5, 2, 3: measured
    0.02 %, 0.2 %, 0.5 %).  As the ratio grows the interface sharpens to two to
    four nodes and the relaxed gas is denser than the Maxwell gas, by a margin
    that grows with the ratio (measured 2 % at ratio 5, 9 % at 10, x1.7 at 100,
    x3.5 at 1000); the liquid stays within 5 %.  A wrong term in Psi' or in the
    double wells moves the near-critical densities off Maxwell; the growth of
    the offset with the ratio is pinned so that it cannot drift unnoticed."""
    kap = 0.1
    errs = []
    for ratio, tol in ((1.5, 2e-3), (2.0, 3e-3), (3.0, 8e-3), (5.0, 3e-2), (10.0, None), (100.0, None),
                       (1000.0, None)):
        p = orc.coexisting_params(ratio, lattice=0, kappa2=kap, kappa3=kap, lambda2=3.125 * kap,
                                  lambda3=3.125 * kap)
        f = _slab(orc, p)
        rg, rl = f["rho"][0, 0, 0], f["rho"][0, 0, 64]
        eg, el = rg / p.rho_g - 1, rl / p.rho_l - 1
        errs.append(eg)
        assert np.isfinite(f["rho"]).all()
        if tol is not None:
            assert abs(eg) < tol and abs(el) < tol, (ratio, eg, el)
        else:
            assert 0 < eg and abs(el) < 5e-2, (ratio, eg, el)
    assert all(b > a for a, b in zip(errs[1:], errs[2:])), errs
    assert 0.05 < errs[4] < 0.15 and 0.4 < errs[5] < 1.0 and 2.0 < errs[6] < 3.0, errs


@pytest.mark.parametrize("which", ["drops_2d", "collision_3d"])
def test_lattice_ratio_temperatures(orc, which):
    """The stored temperatures of the workloads named by their lattice density
    ratio (synth.workloads.LATTICE_RATIO_T, computed by oracle.lattice_ratio)
    give a relaxed flat slab (256 nodes) with rho_l / rho_g within 1 % of the
    named ratio, at a Maxwell ratio (of the same temperature) several times
    higher."""
    if which == "drops_2d":
        wl = W.drops_2d(1024, ratio=1000.0, seed=0, lattice_ratio=True)
    else:
        wl = W.collision_3d(256, radius=32, ratio=800.0, kappa2=0.2, kappa3=0.2, lattice_ratio=True)
    p = orc.workload_params(wl)
    f = _slab(orc, p, n=256)
    r = f["rho"][0, 0, 128] / f["rho"][0, 0, 0]
    assert abs(r / wl.ratio - 1) < 1e-2, r
    assert p.rho_l / p.rho_g > 5.0 * wl.ratio


def test_laplace_law_scaling(orc):
    """Laplace's law on small 2D drops (the paper's Laplace tests): the
    pressure jump across a relaxed circular drop of liquid 1 in gas, taken
    relative to the jump across a flat interface (with interfaces 2-3 nodes
    wide the bulk pressures on either side of a flat interface differ by a
    discretisation offset), falls as 1/R, and so does the shift of the
    chemical potential above its flat-interface value (Gibbs-Thomson):
    R dp and R dmu agree across radii.  Bulk pressures from the oracle's
    rho mu_rho + phi mu_phi - f_B, pinned by test_bulk_pressure_*."""
    import dataclasses
    base = orc.coexisting_params(10.0, lattice=0, nx=80, ny=80, nz=1, kappa2=0.045, kappa3=0.045,
                                 lambda2=3.125 * 0.045, lambda3=3.125 * 0.045)
    rg, rl = orc.discrete_coexistence(base, steps=10000, n=128)
    q = dataclasses.replace(base, nx=128, ny=1, nz=1)
    x = np.arange(128.0)
    c1 = 0.5 * (np.tanh((x - 32) / 2.0) - np.tanh((x - 96) / 2.0))
    st = orc.State(q, (rg + (rl - rg) * c1).reshape(1, 1, 128), (q.chi * c1).reshape(1, 1, 128))
    st.run(10000)
    f = st.fields()
    dp_flat = (orc.bulk_pressure(q, f["rho"][0, 0, 64], f["phi"][0, 0, 64])
               - orc.bulk_pressure(q, f["rho"][0, 0, 0], f["phi"][0, 0, 0]))
    mu_flat = f["mu_rho"][0, 0, 0]
    N = 80
    yy, xx = np.mgrid[0:N, 0:N]
    rr = np.sqrt((xx - N / 2) ** 2 + (yy - N / 2) ** 2)
    Rdp, Rdmu = [], []
    for R in (14, 18, 24):
        c = 0.5 * (1 - np.tanh((rr - R) / 2.0))
        s = orc.State(base, (rg + (rl - rg) * c).reshape(1, N, N), (base.chi * c).reshape(1, N, N))
        s.run(10000)
        fl = s.fields()
        c0 = N // 2
        ri, pi = fl["rho"][0, c0 - 1:c0 + 2, c0 - 1:c0 + 2].mean(), fl["phi"][0, c0 - 1:c0 + 2, c0 - 1:c0 + 2].mean()
        ro, po = fl["rho"][0, 0:3, 0:3].mean(), fl["phi"][0, 0:3, 0:3].mean()
        dp = orc.bulk_pressure(base, ri, pi) - orc.bulk_pressure(base, ro, po) - dp_flat
        reff = np.sqrt(((fl["rho"][0] - ro) / (ri - ro)).sum() / np.pi)
        assert abs(reff - R) < 2.0
        Rdp.append(dp * reff)
        Rdmu.append((fl["mu_rho"][0, 0, 0] - mu_flat) * reff)
    Rdp, Rdmu = np.array(Rdp), np.array(Rdmu)
    assert np.all(Rdp > 0) and np.all(Rdmu > 0)
    # measured spread 2.6 % (R dp = 0.0939, 0.0963, 0.0944); a 1/R^2 or an
    # R-independent jump would spread these by a factor ~1.7.  The chemical
    # potential still drifts with the slow exchange of mass with the gas.
    assert Rdp.max() / Rdp.min() < 1.05, Rdp
    assert Rdmu.max() / Rdmu.min() < 1.2, Rdmu


def test_bulk_pressure_definition(orc):
    """f_B's derivatives are the bulk chemical potentials, and at the Maxwell
    densities of pure phases the bulk pressures of gas and liquid 1 are equal
    (equal-area rule of the EOS part; the double wells vanish there)."""
    p = orc.coexisting_params(10.0, lattice=0, nx=4, ny=4, nz=1)
    for rho, phi in ((0.8, 0.3), (3.0, -2.0), (5.0, 4.5)):
        h = 1e-6
        dr = (orc.f_bulk(p, rho + h, phi) - orc.f_bulk(p, rho - h, phi)) / (2 * h)
        dq = (orc.f_bulk(p, rho, phi + h) - orc.f_bulk(p, rho, phi - h)) / (2 * h)
        mr, mq = orc.mu_bulk(p, rho, phi)
        assert abs(dr - mr) < 1e-7 and abs(dq - mq) < 1e-7
    pg = orc.bulk_pressure(p, p.rho_g, 0.0)
    pl = orc.bulk_pressure(p, p.rho_l, p.chi)
    assert abs(pl - pg) < 1e-10 * max(1.0, abs(pg))
