"""Pins of the oracle's van der Waals and Peng-Robinson equations of state
(the alternatives to Carnahan-Starling that the paper names next to Eq. (4)).

Each check stands on something other than the oracle's own formulas: the
textbook pressures typed here from the EOS definitions (not from the
oracle's Psi), the van der Waals critical point in closed form, the
Peng-Robinson critical point solved here from dp/drho = d2p/drho2 = 0 with
mpmath, the relation p = rho Psi' - Psi stated above Eq. (4), derivatives by
mpmath, and the equal-area rule integrated with scipy."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import quad

VDW = dict(kind=1, a=9.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.0)
PR = dict(kind=2, a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344)


def textbook_pressure(e, T, rho, Tc=None):
    """van der Waals: rho RT/(1 - b rho) - a rho^2.  Peng-Robinson:
    rho RT/(1 - b rho) - a alpha(T) rho^2/(1 + 2 b rho - b^2 rho^2) with
    alpha = [1 + m(1 - sqrt(T/Tc))]^2, m = 0.37464 + 1.54226 w - 0.26992 w^2."""
    a, b, R = e["a"], e["b"], e["R"]
    rep = rho * R * T / (1 - b * rho)
    if e["kind"] == 1:
        return rep - a * rho * rho
    w = e["omega"]
    m = 0.37464 + 1.54226 * w - 0.26992 * w * w
    alpha = (1 + m * (1 - mp.sqrt(T / Tc))) ** 2 if Tc is not None else 1.0
    return rep - a * alpha * rho * rho / (1 + 2 * b * rho - b * b * rho * rho)


def _tc(orc, e):
    return orc.eos_critical_temperature(e["kind"], e["a"], e["b"], e["R"], e["omega"])


def test_vdw_critical_point_closed_form(orc):
    Tc, rc = _tc(orc, VDW)
    assert abs(Tc / (8 * VDW["a"] / (27 * VDW["b"] * VDW["R"])) - 1) < 1e-12
    assert abs(rc * 3 * VDW["b"] - 1) < 1e-6


def test_pr_critical_point_from_the_textbook_pressure(orc):
    """Solve dp/drho = d2p/drho2 = 0 of the textbook Peng-Robinson pressure
    (alpha = 1 at T_c) with mpmath; also the textbook constants Z_c = 0.3074,
    b rho_c = 0.2531."""
    mp.mp.dps = 30
    e = PR
    def p(T, r):
        return textbook_pressure(e, T, r)
    def eqs(T, r):
        return [mp.diff(lambda x: p(T, x), r), mp.diff(lambda x: p(T, x), r, 2)]
    T0, r0 = 0.07, 2.6
    sol = mp.findroot(lambda T, r: eqs(T, r), (T0, r0))
    Tc_ref, rc_ref = float(sol[0]), float(sol[1])
    Tc, rc = _tc(orc, e)
    assert abs(Tc / Tc_ref - 1) < 1e-10
    assert abs(rc / rc_ref - 1) < 1e-5
    zc = float(p(Tc_ref, rc_ref)) / (rc_ref * e["R"] * Tc_ref)
    assert abs(zc - 0.3074) < 1e-4
    assert abs(e["b"] * rc_ref - 0.2531) < 1e-4


@pytest.mark.parametrize("e", [VDW, PR], ids=["vdw", "pr"])
def test_psi_gives_the_textbook_pressure_and_its_derivative(orc, e):
    """p = rho Psi' - Psi equals the textbook pressure; Psi' is dPsi/drho."""
    mp.mp.dps = 30
    Tc, _ = _tc(orc, e)
    rng = np.random.default_rng(4)
    k, a, b, R, w = e["kind"], e["a"], e["b"], e["R"], e["omega"]
    for _ in range(20):
        T = float(rng.uniform(0.4, 1.2)) * Tc
        rho = float(rng.uniform(0.01, 0.9)) / b
        C = float(rng.uniform(-1, 1))
        p_orc = rho * orc.eos_psi_prime(k, a, b, R, w, T, C, rho) - orc.eos_psi(k, a, b, R, w, T, C, rho)
        p_ref = float(textbook_pressure(e, T, rho, Tc))
        assert abs(p_orc - p_ref) <= 1e-11 * (abs(p_ref) + rho * R * T)
        d = float(mp.diff(lambda x: orc.eos_psi(k, a, b, R, w, T, C, float(x)), rho, h=1e-6 * rho))
        assert abs(orc.eos_psi_prime(k, a, b, R, w, T, C, rho) - d) < 1e-6 * (1 + abs(d))


@pytest.mark.parametrize("e", [VDW, PR], ids=["vdw", "pr"])
@pytest.mark.parametrize("tr", [0.9, 0.7, 0.6])
def test_maxwell_equal_area(orc, e, tr):
    """The coexisting densities have equal pressure and satisfy the equal-area
    rule in the specific volume v = 1/rho: int_{v_l}^{v_g} p dv = p (v_g - v_l)."""
    Tc, _ = _tc(orc, e)
    T = tr * Tc
    k, a, b, R, w = e["kind"], e["a"], e["b"], e["R"], e["omega"]
    rg, rl, C, psi0 = orc.eos_maxwell(k, T, a, b, R, w)
    assert 0 < rg < rl < 1 / b
    pg = float(textbook_pressure(e, T, rg, Tc))
    pl = float(textbook_pressure(e, T, rl, Tc))
    assert abs(pg - pl) <= 1e-10 * abs(pl) + 1e-14
    area, _ = quad(lambda v: float(textbook_pressure(e, T, 1.0 / v, Tc)), 1.0 / rl, 1.0 / rg,
                   limit=400, epsabs=0, epsrel=1e-12)
    ref = pg * (1.0 / rg - 1.0 / rl)
    assert abs(area - ref) <= 1e-8 * abs(ref)
    # the constants make Psi' vanish at both densities and Psi equal there
    assert abs(orc.eos_psi_prime(k, a, b, R, w, T, C, rg)) < 1e-12
    assert abs(orc.eos_psi_prime(k, a, b, R, w, T, C, rl)) < 1e-10
    assert abs(orc.eos_psi(k, a, b, R, w, T, C, rl) - psi0) < 1e-10 * (1 + abs(psi0))


def test_pr_alpha_is_one_at_the_critical_temperature(orc):
    e = PR
    Tc, _ = _tc(orc, e)
    assert abs(orc.eos_attraction(2, e["a"], e["b"], e["R"], e["omega"], Tc) / e["a"] - 1) < 1e-12
    assert orc.eos_attraction(2, e["a"], e["b"], e["R"], e["omega"], 0.6 * Tc) > e["a"]


@pytest.mark.parametrize("e", [VDW, PR], ids=["vdw", "pr"])
def test_temperature_for_ratio(orc, e):
    k, a, b, R, w = e["kind"], e["a"], e["b"], e["R"], e["omega"]
    T, rg, rl, C, _ = orc.eos_temperature_for_ratio(k, 100.0, a, b, R, w)
    assert abs(rl / rg / 100.0 - 1) < 1e-9
    assert math.isclose(orc.eos_maxwell(k, T, a, b, R, w)[0], rg, rel_tol=1e-12)


@pytest.mark.parametrize("kind", [1, 2], ids=["vdw", "pr"])
def test_flat_slab_approaches_the_maxwell_densities(orc, kind):
    """A flat liquid-gas slab relaxed by the oracle's dynamics with the van der
    Waals or Peng-Robinson free energy (ratio 10) ends at bulk densities near
    the Maxwell ones, and nearer as the interface widens (kappa_1 up): the
    lattice's discretisation error, as for Carnahan-Starling."""
    nx = 160
    errs = []
    for k1 in (0.003, 0.03):
        p = orc.coexisting_params(10.0, lattice=0, nx=nx, ny=1, nz=1, kappa1=k1, kappa2=0.1, kappa3=0.1,
                                  lambda2=0.3125, lambda3=0.3125, eos=kind, a=2.0 / 49.0, b=2.0 / 21.0)
        x = np.arange(nx, dtype=float)
        c1 = 0.5 * (np.tanh((x - nx / 4) / 3.0) - np.tanh((x - 3 * nx / 4) / 3.0))
        st = orc.State(p, (p.rho_g + (p.rho_l - p.rho_g) * c1).reshape(1, 1, nx), (p.chi * c1).reshape(1, 1, nx))
        st.run(5000)
        f = st.fields()
        errs.append((abs(f["rho"][0, 0, 0] / p.rho_g - 1), abs(f["rho"][0, 0, nx // 2] / p.rho_l - 1)))
        assert np.abs(f["u"]).max() < 2e-3
    assert errs[1][1] < 1.2e-2 and errs[1][0] < 5e-2, errs
    assert errs[1][0] < errs[0][0] and errs[1][1] < errs[0][1], errs
