"""Pins of the oracle's free-energy pieces: concentrations (text below Fig. 1),
bulk energy (Eq. 2), interfacial energy and its (rho, phi) rewrite (Eq. 3 and
the expansion after it), and the chemical potentials mu = dF/drho, dF/dphi.

References: the paper's definitions typed into the test (f_B, f_I with
kappas) and mpmath derivatives of them; lattice Fourier symbols in product form.
"""
import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 40


def params(orc, ratio=1000.0, k2=0.1, k3=0.3):
    return orc.coexisting_params(ratio, lattice=0, nx=64, ny=1, nz=1, kappa2=k2, kappa3=k3,
                                 lambda2=3.125 * k2, lambda3=3.125 * k3)


def f_bulk(p, rho, phi):
    """Eq. (2) with Psi_eos of Eq. (4), concentrations from their definitions."""
    rho, phi = mp.mpf(rho), mp.mpf(phi)
    psi = rho * (p.C - p.a * rho - 8 * p.R * p.T * (-6 + p.b * rho) / (-4 + p.b * rho) ** 2
                 + p.R * p.T * mp.log(rho))
    psi0 = p.rho_g * (p.C - p.a * p.rho_g - 8 * p.R * p.T * (-6 + p.b * p.rho_g) / (-4 + p.b * p.rho_g) ** 2
                      + p.R * p.T * mp.log(p.rho_g))
    cg = (rho - p.rho_l) / (p.rho_g - p.rho_l)
    c1 = (1 + phi / p.chi - cg) / 2
    c2 = (1 - phi / p.chi - cg) / 2
    return (p.lambda1 / 2 * (psi - psi0) + p.lambda2 / 2 * c1 ** 2 * (1 - c1) ** 2
            + p.lambda3 / 2 * c2 ** 2 * (1 - c2) ** 2)


def test_concentrations_and_minima(orc):
    p = params(orc)
    for rho, phi, want in ((p.rho_g, 0.0, (0, 0)), (p.rho_l, p.chi, (1, 0)), (p.rho_l, -p.chi, (0, 1))):
        c1, c2 = orc.concentrations(p, rho, phi)
        assert abs(c1 - want[0]) < 1e-14 and abs(c2 - want[1]) < 1e-14
    rng = np.random.default_rng(1)
    for rho, phi in zip(rng.uniform(0.01, 9, 20), rng.uniform(-5, 5, 20)):
        c1, c2 = orc.concentrations(p, rho, phi)
        cg = (rho - p.rho_l) / (p.rho_g - p.rho_l)
        assert abs(cg + c1 + c2 - 1) < 1e-13
    # the three bulk minima of Fig. 1 are stationary points of f_B: mu_bulk = 0 there
    for rho, phi in ((p.rho_g, 0.0), (p.rho_l, p.chi), (p.rho_l, -p.chi)):
        mr, mf = orc.mu_bulk(p, rho, phi)
        assert abs(mr) < 1e-14 and abs(mf) < 1e-14


def test_gradient_coefficients_rewrite(orc):
    """f_I of Eq. (3) with kappa_i equals A|grad rho|^2 + B|grad phi|^2 + D grad rho.grad phi."""
    p = params(orc)
    A, Bc, D = orc.gradient_coefficients(p)
    rng = np.random.default_rng(2)
    dlt = p.rho_g - p.rho_l
    for _ in range(20):
        gr, gp = rng.normal(size=3), rng.normal(size=3)
        gc1 = 0.5 * (gp / p.chi - gr / dlt)
        gc2 = 0.5 * (-gp / p.chi - gr / dlt)
        fi = p.kappa1 / 2 * gr @ gr + p.kappa2 / 2 * gc1 @ gc1 + p.kappa3 / 2 * gc2 @ gc2
        assert abs(A * gr @ gr + Bc * gp @ gp + D * gr @ gp - fi) < 1e-13 * max(1, abs(fi))


@pytest.mark.parametrize("ratio", [10.0, 1000.0])
def test_mu_bulk_is_derivative_of_f_bulk(orc, ratio):
    p = params(orc, ratio)
    rng = np.random.default_rng(3)
    pts = list(zip(rng.uniform(0.5 * p.rho_g, 1.05 * p.rho_l, 12), rng.uniform(-6, 6, 12)))
    pts += [(p.rho_g * 1.3, 0.2), (p.rho_l * 0.9, 4.0)]
    for rho, phi in pts:
        mr, mf = orc.mu_bulk(p, rho, phi)
        dr = mp.diff(lambda x: f_bulk(p, x, phi), mp.mpf(rho))
        dp = mp.diff(lambda y: f_bulk(p, rho, y), mp.mpf(phi))
        assert abs(mr - float(dr)) < 1e-13 * max(1.0, abs(float(dr)))
        assert abs(mf - float(dp)) < 1e-13 * max(1.0, abs(float(dp)))


def laplacian_symbol(k, lattice):
    """6 (prod_alpha (2/3 + cos k_alpha / 3) - 1): the weights factor over axes."""
    d = 2 if lattice == 0 else 3
    return 6.0 * (np.prod([2.0 / 3.0 + np.cos(k[a]) / 3.0 for a in range(d)]) - 1.0)


def gradient_symbol(k, lattice, axis):
    d = 2 if lattice == 0 else 3
    return np.sin(k[axis]) * np.prod([2.0 / 3.0 + np.cos(k[a]) / 3.0 for a in range(d) if a != axis])


@pytest.mark.parametrize("lattice,shape", [(0, (1, 12, 16)), (1, (6, 8, 10))])
def test_stencil_fourier_symbols(orc, lattice, shape):
    nz, ny, nx = shape
    p = orc.Params(lattice=lattice, nx=nx, ny=ny, nz=nz)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for m in ((1, 0, 0), (2, 3, 0), (3, 1, 2), (5, 5, 1)):
        k = np.array([2 * np.pi * m[0] / nx, 2 * np.pi * m[1] / ny, 2 * np.pi * m[2] / nz if nz > 1 else 0.0])
        if lattice == 0:
            k[2] = 0.0
        ph = k[0] * x + k[1] * y + k[2] * z
        lap = orc.laplacian(p, np.cos(ph))
        assert np.abs(lap - laplacian_symbol(k, lattice) * np.cos(ph)).max() < 1e-13
        grad = orc.gradient(p, np.cos(ph))
        for a in range(2 if lattice == 0 else 3):
            assert np.abs(grad[a] + gradient_symbol(k, lattice, a) * np.sin(ph)).max() < 1e-13
    # D2Q9 closed form quoted for the x-wave: 2 cos k - 2
    if lattice == 0:
        kk = 2 * np.pi / nx
        assert abs(laplacian_symbol((kk, 0, 0), 0) - (2 * np.cos(kk) - 2)) < 1e-15


@pytest.mark.parametrize("lattice", [0, 1])
def test_stencils_exact_on_quadratics(orc, lattice):
    shape = (1, 16, 16) if lattice == 0 else (12, 12, 12)
    nz, ny, nx = shape
    p = orc.Params(lattice=lattice, nx=nx, ny=ny, nz=nz)
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    psi = 0.3 * x ** 2 - 0.2 * x * y + 0.1 * y ** 2 + 0.7 * x + (0.05 * z ** 2 + 0.1 * x * z if lattice else 0)
    lap = orc.laplacian(p, psi)
    grad = orc.gradient(p, psi)
    inner = (slice(1, -1) if nz > 1 else slice(None), slice(1, -1), slice(1, -1))
    want_lap = 0.6 + 0.2 + (0.1 if lattice else 0)
    assert np.abs(lap[inner] - want_lap).max() < 1e-11
    assert np.abs(grad[0][inner] - (0.6 * x - 0.2 * y + 0.7 + (0.1 * z if lattice else 0))[inner]).max() < 1e-11
    assert np.abs(grad[1][inner] - (-0.2 * x + 0.2 * y)[inner]).max() < 1e-11


@pytest.mark.parametrize("lattice", [0, 1])
def test_chemical_potential_gradient_terms(orc, lattice):
    """mu_rho - bulk = -2A lap(rho) - D lap(phi) and mu_phi - bulk = -2B lap(phi) - D lap(rho),
    checked on plane waves whose Laplacian the lattice symbol gives exactly."""
    shape = (1, 8, 32) if lattice == 0 else (4, 4, 16)
    nz, ny, nx = shape
    p = orc.coexisting_params(10.0, lattice=lattice, nx=nx, ny=ny, nz=nz, kappa2=0.05, kappa3=0.2,
                              lambda2=3.125 * 0.05, lambda3=3.125 * 0.2)
    A, Bc, D = orc.gradient_coefficients(p)
    x = np.arange(nx)[None, None, :] * np.ones(shape)
    k = 2 * np.pi * 3 / nx
    s = laplacian_symbol((k, 0, 0), lattice)
    er, ep = 0.05, 0.3
    rho = p.rho_l - 0.5 + er * np.cos(k * x)
    phi = 1.0 + ep * np.cos(k * x)
    st = orc.State(p, rho, phi)
    f = st.fields()
    mb = np.array([[orc.mu_bulk(p, r, q) for r, q in zip(rr, qq)] for rr, qq in zip(f["rho"].reshape(-1, nx), f["phi"].reshape(-1, nx))])
    mb = mb.reshape(shape + (2,))
    want_r = -2 * A * s * er * np.cos(k * x) - D * s * ep * np.cos(k * x)
    want_p = -2 * Bc * s * ep * np.cos(k * x) - D * s * er * np.cos(k * x)
    assert np.abs(f["rho"] - rho).max() < 1e-13 and np.abs(f["phi"] - phi).max() < 1e-13
    assert np.abs(f["mu_rho"] - mb[..., 0] - want_r).max() < 1e-13
    assert np.abs(f["mu_phi"] - mb[..., 1] - want_p).max() < 1e-13
