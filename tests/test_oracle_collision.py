"""Pins of the oracle's node-level kinetics: the entropic equilibrium, the KBC
split and stabiliser gamma, exact-difference forcing, and the phase-field BGK
equilibrium.

References: closed-form moments, the H-theorem characterisation of the
entropic equilibrium (ln(f_i/w_i) affine in c_i), the raw-moment matrix of the
lattice, and the variational definition of gamma (minimiser of the quadratic
entropy estimate), evaluated by scipy.
"""
import itertools

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

LATTICES = [0, 1]


def moments(orc, lattice, f):
    c, _ = orc.lattice_info(lattice)
    out = {}
    for pqr in itertools.product(range(3), repeat=3):
        if lattice == 0 and pqr[2] != 0:
            continue
        out[pqr] = float(np.sum(f * c[:, 0] ** pqr[0] * c[:, 1] ** pqr[1] * c[:, 2] ** pqr[2]))
    return out


def random_state(orc, lattice, rng, amp=0.05, umax=0.3):
    rho = rng.uniform(0.01, 10.0)
    u = rng.uniform(-umax, umax, 3)
    if lattice == 0:
        u[2] = 0.0
    feq = orc.feq(lattice, rho, u)
    f = feq * (1.0 + amp * rng.uniform(-1, 1, feq.size))
    return rho, u, feq, f


@pytest.mark.parametrize("lattice", LATTICES)
def test_lattice_weights(orc, lattice):
    c, w = orc.lattice_info(lattice)
    Q = 9 if lattice == 0 else 27
    assert len(w) == Q and abs(w.sum() - 1) < 1e-15
    assert (c[0] == 0).all()
    assert abs(np.sum(w * c[:, 0] ** 2) - 1 / 3) < 1e-15
    assert abs(np.sum(w * c[:, 0] ** 4) - 1 / 3) < 1e-15
    assert abs(np.sum(w * c[:, 0] ** 2 * c[:, 1] ** 2) - 1 / 9) < 1e-15
    assert sorted(np.unique(np.round(w, 12))) == sorted(np.unique(np.round(
        [4 / 9, 1 / 9, 1 / 36] if lattice == 0 else [8 / 27, 2 / 27, 1 / 54, 1 / 216], 12)))
    # every velocity appears once, opposite pairs present
    assert len({tuple(v) for v in c}) == Q
    assert all(tuple(-v) in {tuple(x) for x in c} for v in c)


@pytest.mark.parametrize("lattice", LATTICES)
def test_entropic_equilibrium_moments(orc, lattice):
    rng = np.random.default_rng(10 + lattice)
    for _ in range(30):
        rho = rng.uniform(0.005, 10.0)
        u = rng.uniform(-0.6, 0.6, 3)
        if lattice == 0:
            u[2] = 0.0
        m = moments(orc, lattice, orc.feq(lattice, rho, u))
        d = 2 if lattice == 0 else 3
        tol = 1e-14 * rho
        assert abs(m[(0, 0, 0)] - rho) < tol
        for a in range(d):
            e = [0, 0, 0]
            e[a] = 1
            assert abs(m[tuple(e)] - rho * u[a]) < tol
            e[a] = 2
            S = np.sqrt(1 + 3 * u[a] ** 2)
            assert abs(m[tuple(e)] - rho * (2 * S - 1) / 3) < tol
        assert abs(m[(1, 1, 0)] - rho * u[0] * u[1]) < tol


@pytest.mark.parametrize("lattice", LATTICES)
def test_entropic_equilibrium_is_h_minimiser(orc, lattice):
    """Stationarity of H = sum f ln(f/w) under mass and momentum constraints:
    ln(feq_i / w_i) must be affine in c_i (Lagrange multipliers)."""
    c, w = orc.lattice_info(lattice)
    d = 2 if lattice == 0 else 3
    rng = np.random.default_rng(20 + lattice)
    for _ in range(10):
        u = rng.uniform(-0.5, 0.5, 3)
        if lattice == 0:
            u[2] = 0
        f = orc.feq(lattice, rng.uniform(0.01, 5), u)
        y = np.log(f / w)
        X = np.column_stack([np.ones(len(w))] + [c[:, a] for a in range(d)])
        coef, *_ = np.linalg.lstsq(X, y, rcond=None)
        assert np.abs(X @ coef - y).max() < 1e-12


@pytest.mark.parametrize("lattice", LATTICES)
def test_kbc_split_carries_deviatoric_moments(orc, lattice):
    rng = np.random.default_rng(30 + lattice)
    d = 2 if lattice == 0 else 3
    for _ in range(20):
        _, _, feq, f = random_state(orc, lattice, rng)
        df = f - feq
        ds, dh = orc.kbc_split(lattice, df)
        assert np.abs(ds + dh - df).max() < 1e-15 * np.abs(f).max() * 10
        ms, mf = moments(orc, lattice, ds), moments(orc, lattice, df)
        tr = sum(mf[tuple(2 if b == a else 0 for b in range(3))] for a in range(d))
        for pqr, v in ms.items():
            order = sum(pqr)
            if order == 2 and max(pqr) == 2:          # diagonal second moments
                assert abs(v - (mf[pqr] - tr / d)) < 1e-14
            elif order == 2:                            # off-diagonal second moments
                assert abs(v - mf[pqr]) < 1e-14
            else:                                       # all other moments vanish
                assert abs(v) < 1e-14


@pytest.mark.parametrize("lattice", LATTICES)
@pytest.mark.parametrize("beta", [0.4995, 0.9, 0.99])
def test_kbc_collision_invariants(orc, lattice, beta):
    rng = np.random.default_rng(40 + lattice)
    d = 2 if lattice == 0 else 3
    for _ in range(10):
        rho, _, _, f = random_state(orc, lattice, rng)
        m = moments(orc, lattice, f)
        u = np.array([m[(1, 0, 0)], m[(0, 1, 0)], m[(0, 0, 1)] if lattice else 0.0]) / m[(0, 0, 0)]
        feq = orc.feq(lattice, m[(0, 0, 0)], u)
        fs, gamma = orc.collide_node(lattice, beta, f)
        ms = moments(orc, lattice, fs)
        # (i) mass and momentum unchanged without force
        for key in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)][: 1 + d]:
            assert abs(ms[key] - m[key]) < 1e-13 * max(1, abs(m[(0, 0, 0)]))
        # (ii) deviatoric second moments of f* - feq are (1 - 2 beta) those of f - feq
        ds0, dh0 = orc.kbc_split(lattice, f - feq)
        ds1, dh1 = orc.kbc_split(lattice, fs - feq)
        assert np.abs(ds1 - (1 - 2 * beta) * ds0).max() < 1e-13 * max(1, np.abs(f).max())
        # (iii) gamma is where the quadratic entropy estimate is stationary: <dh|f*-feq> = 0
        assert abs(np.sum(dh0 * (fs - feq) / feq)) < 1e-12 * max(1e-30, np.sum(dh0 * dh0 / feq)) ** 0.5 * \
            max(1e-30, np.sum((fs - feq) ** 2 / feq)) ** 0.5 + 1e-15
        # ... and a minimum of it, found by a scalar minimiser
        def h2(g):
            post = f - beta * (2 * ds0 + g * dh0)
            return float(np.sum((post - feq) ** 2 / feq))
        best = minimize_scalar(h2, bracket=(0.0, 2.0, 4.0), tol=1e-12).x
        assert abs(best - gamma) < 1e-5


@pytest.mark.parametrize("lattice", LATTICES)
def test_kbc_limits(orc, lattice):
    rng = np.random.default_rng(50 + lattice)
    rho, u, feq, f = random_state(orc, lattice, rng)
    # (v) equilibrium is a fixed point (gamma then only multiplies round-off)
    fs, gamma = orc.collide_node(lattice, 0.7, feq)
    assert np.abs(fs - feq).max() < 1e-15 * rho * 10
    # gamma defaults to the LBGK value 2 when dh vanishes exactly
    z = np.zeros_like(feq)
    assert orc.kbc_gamma(lattice, 0.7, feq, z + 1e-3, z) == 2.0
    # (iv) beta = 1/2 (tau = 1): gamma = 2 and the collision lands on equilibrium (LBGK)
    m = moments(orc, lattice, f)
    um = np.array([m[(1, 0, 0)], m[(0, 1, 0)], m[(0, 0, 1)] if lattice else 0.0]) / m[(0, 0, 0)]
    fs, gamma = orc.collide_node(lattice, 0.5, f)
    assert abs(gamma - 2.0) < 1e-12
    assert np.abs(fs - orc.feq(lattice, m[(0, 0, 0)], um)).max() < 1e-14 * m[(0, 0, 0)]


@pytest.mark.parametrize("lattice", LATTICES)
def test_exact_difference_forcing(orc, lattice):
    rng = np.random.default_rng(60 + lattice)
    d = 2 if lattice == 0 else 3
    for beta in (0.5, 0.8):
        rho, _, _, f = random_state(orc, lattice, rng)
        F = rng.uniform(-0.01, 0.01, 3)
        if lattice == 0:
            F[2] = 0
        fs0, g0 = orc.collide_node(lattice, beta, f)
        fs1, g1 = orc.collide_node(lattice, beta, f, F)
        dm = moments(orc, lattice, fs1 - fs0)
        assert abs(dm[(0, 0, 0)]) < 1e-13
        for a, key in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)][:d]):
            assert abs(dm[key] - F[a]) < 1e-13
        assert g0 == g1  # the stabiliser is computed before the force is added


@pytest.mark.parametrize("lattice", LATTICES)
def test_phase_field_equilibrium_moments(orc, lattice):
    rng = np.random.default_rng(70 + lattice)
    d = 2 if lattice == 0 else 3
    for _ in range(10):
        phi, mu, Gam = rng.uniform(-5, 5), rng.uniform(-0.1, 0.1), rng.uniform(0.2, 2)
        u = rng.uniform(-0.2, 0.2, 3)
        if lattice == 0:
            u[2] = 0
        m = moments(orc, lattice, orc.geq(lattice, phi, mu, Gam, u))
        assert abs(m[(0, 0, 0)] - phi) < 1e-13
        for a in range(d):
            e = [0, 0, 0]
            e[a] = 1
            assert abs(m[tuple(e)] - phi * u[a]) < 1e-13
            for b in range(d):
                e2 = [0, 0, 0]
                e2[a] += 1
                e2[b] += 1
                want = (Gam * mu if a == b else 0.0) + phi * u[a] * u[b]
                assert abs(m[tuple(e2)] - want) < 1e-13
