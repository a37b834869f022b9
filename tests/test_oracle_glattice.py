"""Pins of the oracle's reduced phase-field lattice (D2Q5 for D2Q9, D3Q7 for
D3Q27: the rest and axis directions, the lattice of g that the paper leaves
open).

Each check stands on what Eq. (7) and the lattice fix, not on the oracle's
own formulas: the equilibrium's zeroth, first and second moments (phi, phi u,
Gamma mu_phi I) summed here, zeros off the axes, exact conservation of phi,
the linearised Cahn-Hilliard growth rate M s(k) [mu_b'(0) - 2 B s(k)]
(s(k) = 2 cos k - 2) along x on both lattices, the flat liquid-liquid tanh
profile, and agreement of a relaxed lens with the full lattice's."""
import numpy as np
import pytest

from synth import workloads as W


def directions(orc, lattice):
    c, _ = orc.lattice_info(lattice)
    return np.asarray(c)


@pytest.mark.parametrize("lattice", [0, 1])
def test_reduced_equilibrium_moments(orc, lattice):
    c = directions(orc, lattice).astype(float)
    axis = np.abs(c).sum(1) == 1
    rng = np.random.default_rng(7)
    for _ in range(10):
        phi, mu, G = rng.uniform(-5, 5), rng.uniform(-1, 1), rng.uniform(0.1, 2)
        u = rng.uniform(-0.1, 0.1, 3)
        if lattice == 0:
            u[2] = 0.0
        g = orc.geq(lattice, phi, mu, G, u, reduced=True)
        assert np.all(g[~axis & (np.abs(c).sum(1) > 0)] == 0.0)
        assert abs(g.sum() - phi) < 1e-13
        assert np.abs((g[:, None] * c).sum(0) - phi * u).max() < 1e-14
        second = np.einsum("i,ia,ib->ab", g, c, c)
        D = 2 if lattice == 0 else 3
        assert np.abs(second[:D, :D] - G * mu * np.eye(D)).max() < 1e-13


@pytest.mark.parametrize("lattice", [0, 1])
def test_reduced_lattice_linear_cahn_hilliard_growth(orc, lattice):
    """As the full-lattice pin: along x the reduced lattice's Laplacian of mu
    is the same three-point stencil, so the rate is unchanged."""
    import dataclasses
    nx = 128
    p = orc.coexisting_params(10.0, lattice=lattice, nx=nx, ny=1, nz=1, kappa2=0.3, kappa3=0.3,
                              lambda2=0.9375, lambda3=0.9375, mobility=0.05, tau_phi=1.0)
    p = dataclasses.replace(p, glattice=1)
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
        assert abs(got / want - 1) < 1e-2, (m, got, want)


def test_reduced_lattice_flat_liquid_liquid_interface(orc):
    """phi = chi tanh(x / W), W = 2 sqrt(kappa / lambda), rho = rho_l."""
    import dataclasses
    nx = 128
    kap, lam = 0.2, 0.1
    p = orc.coexisting_params(10.0, lattice=0, nx=nx, ny=1, nz=1, kappa2=kap, kappa3=kap,
                              lambda2=lam, lambda3=lam)
    p = dataclasses.replace(p, glattice=1)
    x = np.arange(nx, dtype=float)
    W0 = 2 * np.sqrt(kap / lam)
    phi0 = p.chi * np.tanh((x - nx / 4) / 3.0) * np.tanh((3 * nx / 4 - x) / 3.0)
    st = orc.State(p, np.full((1, 1, nx), p.rho_l), phi0.reshape(1, 1, nx))
    st.run(3000)
    f = st.fields()
    assert np.abs(f["rho"] - p.rho_l).max() / p.rho_l < 3e-3
    ph = f["phi"][0, 0]
    i = int(np.argmin(np.abs(ph[: nx // 2])))
    j = i if ph[i] * ph[i + 1] <= 0 else i - 1
    x0 = j - ph[j] / (ph[j + 1] - ph[j])
    sel = slice(nx // 8, 3 * nx // 8)
    prof = p.chi * np.tanh((x[sel] - x0) / W0)
    assert np.abs(ph[sel] - prof).max() / p.chi < 2e-2


@pytest.mark.parametrize("lattice", [0, 1])
def test_reduced_lattice_conserves_phase_field(orc, lattice):
    import dataclasses
    if lattice == 0:
        w = W.lens(48, 48, radius=8.0, ratio=100.0, kappa=0.045)
    else:
        w = W.collision_3d(16, radius=16 / 6, ratio=100.0, v_rel=0.02, kappa2=0.045, kappa3=0.045)
    p = dataclasses.replace(orc.coexisting_params(w.ratio, **w.physics()), glattice=1)
    rho, phi, u = W.fields(w, p.rho_g, p.rho_l)
    st = orc.State(p, rho, phi, u if lattice else None)
    f0 = st.fields()
    st.run(100 if lattice == 0 else 30)
    f = st.fields()
    assert abs(f["phi"].sum() - f0["phi"].sum()) < 1e-11 * np.abs(f0["phi"]).sum()
    assert abs(f["rho"].sum() / f0["rho"].sum() - 1) < 1e-12


def test_reduced_lattice_lens_matches_full_lattice(orc):
    """A relaxed liquid lens (ratio 10) has the same shape on either g
    lattice: the equilibrium is a free-energy minimum, not a property of
    the phase-field velocity set (liquid-1 and liquid-2 areas within 1 %)."""
    import dataclasses
    w = W.lens(64, 64, radius=10.0, ratio=10.0, kappa=0.045)
    out = []
    for gl in (0, 1):
        p = dataclasses.replace(orc.coexisting_params(w.ratio, **w.physics()), glattice=gl)
        rho, phi, _ = W.fields(w, p.rho_g, p.rho_l)
        st = orc.State(p, rho, phi)
        st.run(3000)
        f = st.fields()
        out.append((float((f["c1"] > 0.5).sum()), float((f["c2"] > 0.5).sum())))
    (a1, a2), (b1, b2) = out
    assert abs(b1 / a1 - 1) < 0.01 and abs(b2 / a2 - 1) < 0.01, out
