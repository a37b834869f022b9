"""Pins of the oracle's three-liquid model (the extension to more liquid
components named in the paper's concluding paragraph: one more double well
and one more gradient term, carried by a second phase field psi with
C3 = psi / chi; the reading is stated in oracle/telbm_oracle.c).

- Free energy: the bulk potentials are the derivatives of the bulk energy
  (central differences), the four pure phases are stationary points at one
  bulk pressure, and psi = 0 gives back the two-liquid potentials and energy
  of Eqs. (2)-(3).
- Reduction: with psi = 0 and kappa2 = kappa3 one lattice step equals the
  two-liquid oracle's step (gas present, lambda2 != lambda3, kappa4 apart).
- Mobility: the matrix is symmetric positive definite, diag(1, 1/3) for
  equal kappas, (1, 0) in its first row for kappa2 = kappa3 and any kappa4,
  and it annihilates the absent liquid's flux at a two-liquid
  interface (the consistency property of Boyer-Lapuerta N-phase mobilities);
  the one-mobility-per-order-parameter form does not.
- Consistency on the lattice: at a flat liquid-1 / liquid-3 interface (no
  gas, kappa4 = 2 kappa2, same lambda / kappa), the absent liquid 2 stays
  below the density perturbation 1 - C_L (its only first-order source: the
  map to concentrations is affine in rho) over 10^4 steps; the naive
  mobility exceeds that bound.  At a liquid-gas interface the absent
  liquids of the three-liquid model stay no larger than the absent liquid 2
  of the paper's two-liquid model in the same run.
- Neumann angles: a lens of liquid 1 between liquid 2 (below) and liquid 3
  (above), no gas, relaxes to the angles of the closed-form tensions
  gamma_ab = sqrt((lambda_a + lambda_b)(kappa_a + kappa_b)) / 6 within the
  paper's 3 degrees.
"""
import math

import numpy as np
import pytest

from tests import neumann as NM

RATIO = 10.0


def _params(orc, n=(64, 1, 1), **kw):
    nx, ny, nz = n
    return orc.coexisting_params(RATIO, nx=nx, ny=ny, nz=nz, **kw)


def test_bulk_potentials_are_derivatives_of_the_bulk_energy(orc):
    p = _params(orc, kappa2=0.03, lambda2=0.09, kappa3=0.06, lambda3=0.2)
    nl = orc.NLParams(lambda4=0.3, kappa4=0.05)
    rng = np.random.default_rng(3)
    for _ in range(12):
        x = np.array([rng.uniform(p.rho_g, p.rho_l), rng.uniform(-p.chi, p.chi), rng.uniform(-0.5, 1.2) * p.chi])
        mu = np.array(orc.nl_mu_bulk(p, nl, *x))
        fd = []
        for a in range(3):
            h = 1e-5 * (p.rho_l if a == 0 else p.chi)
            e = np.zeros(3)
            e[a] = h
            fd.append((orc.nl_f_bulk(p, nl, *(x + e)) - orc.nl_f_bulk(p, nl, *(x - e))) / (2 * h))
        assert np.allclose(mu, fd, rtol=1e-6, atol=1e-9), (x, mu, fd)


def test_pure_phases_stationary_at_one_pressure(orc):
    p = _params(orc)
    nl = orc.NLParams(lambda4=0.3, kappa4=0.09)
    phases = {"gas": (p.rho_g, 0.0, 0.0), "1": (p.rho_l, p.chi, 0.0), "2": (p.rho_l, -p.chi, 0.0),
              "3": (p.rho_l, 0.0, p.chi)}
    press = {}
    for k, x in phases.items():
        c = orc.nl_concentrations(p, *x)
        assert all(abs(v - (1.0 if k == str(m + 1) else 0.0)) < 1e-14 for m, v in enumerate(c)), (k, c)
        mu = orc.nl_mu_bulk(p, nl, *x)
        assert abs(mu[1]) < 1e-14 and abs(mu[2]) < 1e-14, (k, mu)
        press[k] = x[0] * mu[0] + x[1] * mu[1] + x[2] * mu[2] - orc.nl_f_bulk(p, nl, *x)
    vals = list(press.values())
    assert max(vals) - min(vals) < 1e-10 * max(1.0, abs(vals[0])), press


def test_psi_zero_gives_the_two_liquid_free_energy(orc):
    p = _params(orc, kappa2=0.03, lambda2=0.09, kappa3=0.06, lambda3=0.2)
    nl = orc.NLParams(lambda4=0.3, kappa4=0.05)
    rng = np.random.default_rng(4)
    for _ in range(10):
        r, ph = rng.uniform(p.rho_g, p.rho_l), rng.uniform(-p.chi, p.chi)
        mu3 = orc.nl_mu_bulk(p, nl, r, ph, 0.0)
        mu2 = orc.mu_bulk(p, r, ph)
        assert abs(mu3[0] - mu2[0]) <= 1e-14 * max(1.0, abs(mu2[0]))
        assert abs(mu3[1] - mu2[1]) <= 1e-14 * max(1.0, abs(mu2[1]))
        assert abs(orc.nl_f_bulk(p, nl, r, ph, 0.0) - orc.f_bulk(p, r, ph)) <= 1e-13 * max(1.0, abs(orc.f_bulk(p, r, ph)))
        c3 = orc.nl_concentrations(p, r, ph, 0.0)
        c2 = orc.concentrations(p, r, ph)
        assert np.allclose(c3[:2], c2, rtol=0, atol=1e-15) and c3[2] == 0.0


def test_psi_zero_step_equals_the_two_liquid_step(orc):
    """Drops of both liquids in gas, lambda2 != lambda3, kappa2 = kappa3 !=
    kappa4: one step of the three-liquid oracle with psi = 0 gives the
    two-liquid oracle's populations f and g (the psi terms vanish, phi's
    mobility is M; the potentials differ only in rounding order)."""
    n = 48
    p = orc.coexisting_params(RATIO, nx=n, ny=n, nz=1, kappa2=0.045, lambda2=0.09, kappa3=0.045, lambda3=0.2)
    nl = orc.NLParams(lambda4=0.3, kappa4=0.09)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    c1 = 0.5 * (1 - np.tanh((np.hypot(x - 14, y - 24) - 8) / 2))
    c2 = 0.5 * (1 - np.tanh((np.hypot(x - 34, y - 24) - 8) / 2))
    rho = (p.rho_g + (p.rho_l - p.rho_g) * (c1 + c2))[None]
    phi = (p.chi * (c1 - c2))[None]
    a = orc.State(p, rho, phi)
    b = orc.NLState(p, nl, rho, phi, np.zeros_like(phi))
    a.run(1)
    b.run(1)
    for pa, pb in ((a.f, b.f), (a.g, b.g)):
        assert np.abs(pa - pb).max() <= 1e-13 * np.abs(pa).max()
    assert np.abs(b.fields()["psi"]).max() < 1e-3  # psi starts diffusing at the gas interfaces


def test_mobility_matrix(orc):
    p = _params(orc)
    m = orc.nl_mobility(p, orc.NLParams(kappa4=p.kappa2))
    assert np.allclose(m, [[1.0, 0.0], [0.0, 1.0 / 3.0]], rtol=0, atol=1e-15)
    m = orc.nl_mobility(p, orc.NLParams(kappa4=3.7 * p.kappa2))
    assert abs(m[0, 0] - 1.0) < 1e-15 and abs(m[0, 1]) < 1e-15 and abs(m[1, 0]) < 1e-15
    chi = p.chi
    # d(C1, C2, C3)/d(phi, psi)
    A = np.array([[0.5, -0.5], [-0.5, -0.5], [0.0, 1.0]]) / chi
    for k2, k3, k4 in ((0.03, 0.06, 0.05), (0.1, 0.02, 0.07), (0.045, 0.045, 0.2)):
        q = orc.coexisting_params(RATIO, kappa2=k2, kappa3=k3)
        mc = orc.nl_mobility(q, orc.NLParams(kappa4=k4))
        assert np.allclose(mc, mc.T, rtol=0, atol=1e-15)
        assert np.all(np.linalg.eigvalsh(mc) > 0)
        MC = A @ mc @ A.T  # concentration mobility (times M)
        assert np.allclose(MC.sum(axis=0), 0.0, atol=1e-15)  # total liquid not diffused
        s = np.array([k2, k3, k4])
        for absent in range(3):
            # chemical potentials of a two-liquid interface with the same
            # lambda / kappa: nu_a / s_a = -nu_b / s_b, nu_absent = 0
            a_, b_ = [i for i in range(3) if i != absent]
            nu = np.zeros(3)
            nu[a_] = s[a_] * 0.7
            nu[b_] = -s[b_] * 0.7
            assert abs((MC @ nu)[absent]) < 1e-15, (absent, MC @ nu)
        naive = A @ np.eye(2) @ A.T
        nu = np.array([0.7 * k2, 0.0, -0.7 * k4])
        assert abs((naive @ nu)[1]) > 1e-5


def _flat13(n, p):
    x = np.arange(n, dtype=float)
    c = 0.5 * (np.tanh((x - n / 4) / 2.0) - np.tanh((x - 3 * n / 4) / 2.0))  # liquid 1 in the middle
    rho = np.full(n, p.rho_l).reshape(1, 1, n)
    return rho, (p.chi * c).reshape(1, 1, n), (p.chi * (1 - c)).reshape(1, 1, n)


@pytest.mark.parametrize("form", [0, 1], ids=["consistent", "naive"])
def test_absent_liquid_at_a_liquid_liquid_interface(orc, form):
    n = 64
    p = _params(orc, n=(n, 1, 1))
    nl = orc.NLParams(kappa4=2 * p.kappa2, lambda4=2 * p.lambda2, mobility_form=form)
    st = orc.NLState(p, nl, *_flat13(n, p))
    worst = 0.0
    for _ in range(5):
        st.run(2000)
        f = st.fields()
        cl = 1 - (f["rho"] - p.rho_l) / (p.rho_g - p.rho_l)
        worst = max(worst, np.abs(f["c"][1]).max() / np.abs(1 - cl).max())
    print("max |C2| / max |1 - C_L|:", worst)
    if form == 0:
        assert worst < 1.0
    else:
        assert worst > 1.0


def test_absent_liquids_at_a_liquid_gas_interface(orc):
    n = 128
    p = _params(orc, n=(n, 1, 1))
    x = np.arange(n, dtype=float)
    c = 0.5 * (np.tanh((x - n / 4) / 2.0) - np.tanh((x - 3 * n / 4) / 2.0))
    rho = (p.rho_g + (p.rho_l - p.rho_g) * c).reshape(1, 1, n)
    phi = (p.chi * c).reshape(1, 1, n)
    three = orc.NLState(p, orc.NLParams(), rho, phi, np.zeros_like(phi))
    two = orc.State(p, rho, phi)
    for _ in range(5):
        three.run(2000)
        two.run(2000)
        f3, f2 = three.fields(), two.fields()
        ref = np.abs(f2["c2"]).max()
        assert np.abs(f3["c"][1]).max() <= ref and np.abs(f3["c"][2]).max() <= ref, (f3["c"].max(), ref)


def lens3_fields(nx, ny, radius, band, chi, width=2.0):
    """(phi, psi) of a liquid-2 band band[0] <= y < band[1] in liquid 3, with
    a liquid-1 disc centred on the band's upper interface at x = nx / 2."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    c1 = 0.5 * (1.0 - np.tanh((np.hypot(x - nx / 2.0, y - (band[1] - 0.5)) - radius) / width))
    c2 = 0.5 * (np.tanh((y - band[0] + 0.5) / width) - np.tanh((y - band[1] + 0.5) / width)) * (1.0 - c1)
    c3 = 1.0 - c1 - c2
    return (chi * (c1 - c2))[None], (chi * c3)[None]


def lens3_prediction(k1, k2, k3):
    g = lambda a, b: math.sqrt((a + b) * (a + b)) / 6.0  # lambda = kappa for every liquid
    return NM.neumann_angles(g(k1, k2), g(k1, k3), g(k2, k3))


def test_three_liquid_lens_neumann_angles(orc):
    k1, k2, k3 = 0.08, 0.1, 0.1
    nx, ny, R = 96, 64, 14.0
    p = orc.coexisting_params(100.0, nx=nx, ny=ny, nz=1, kappa2=k1, lambda2=k1, kappa3=k2, lambda3=k2)
    nl = orc.NLParams(kappa4=k3, lambda4=k3)
    pred = lens3_prediction(k1, k2, k3)
    assert all(95.0 < v < 145.0 for v in pred.values()), pred
    band = (ny // 4, ny // 4 + ny * 3 // 8)
    phi, psi = lens3_fields(nx, ny, R, band, p.chi)
    st = orc.NLState(p, nl, np.full_like(phi, p.rho_l), phi, psi)
    st.run(30000)
    c = st.fields()["c"][:, 0]
    ang, fits = NM.measure_angles_c(c[0], c[1], c[2], band[1] - 0.5)
    print("triangle", pred, "lens", ang, "fits", fits)
    for a in ang:
        for ph in ("1", "2", "g"):
            assert abs(a[ph] - pred[ph]) < 3.0, (ph, a[ph], pred[ph])
