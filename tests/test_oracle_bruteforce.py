"""Brute-force pin of the oracle's whole time step on tiny lattices (4 x 4
D2Q9, 3 x 3 x 3 D3Q27): a second implementation written here from the
method's definitions, with different machinery, must agree with the
oracle to round-off over two steps.

Independent here: lattice tables (tensor products of the D1Q3 set), the
stencils (np.roll sums over the lattice), the entropic equilibrium (the
exponential closed form w_i rho prod (2 - S)[(2u + S)/(1 - u)]^c), the KBC
split (raw-moment matrix of the lattice solved with numpy.linalg instead of
a dual basis), the stabiliser, the forcing, the phase-field BGK and the
streaming.  Shared with the oracle: the bulk chemical potentials and the
f_I coefficients, which have their own pins (mpmath derivatives of the
typed free energy, the f_I rewrite)."""
import itertools

import numpy as np
import pytest

CS2 = 1.0 / 3.0
D1 = [0, 1, -1]          # D1Q3 velocity of index k, the lattice's ordering
W1 = [2 / 3, 1 / 6, 1 / 6]


def lattice(lat):
    D = 2 if lat == 0 else 3
    cs, ws = [], []
    for kz in range(3 if D == 3 else 1):
        for ky in range(3):
            for kx in range(3):
                cs.append((D1[kx], D1[ky], D1[kz] if D == 3 else 0))
                ws.append(W1[kx] * W1[ky] * (W1[kz] if D == 3 else 1.0))
    return np.array(cs), np.array(ws), D


def shift(a, c):
    """a(x + c) on the periodic grid; a has shape (nz, ny, nx)."""
    return np.roll(a, shift=(-c[2], -c[1], -c[0]), axis=(0, 1, 2))


def laplacian(a, C, Wt):
    return 6.0 * sum(w * (shift(a, c) - a) for c, w in zip(C, Wt))


def gradient(a, C, Wt):
    return np.stack([3.0 * sum(w * c[d] * shift(a, c) for c, w in zip(C, Wt)) for d in range(3)])


def feq(rho, u, C, Wt, D):
    """Entropic equilibrium, exponential closed form."""
    out = []
    for c, w in zip(C, Wt):
        v = w * rho
        for d in range(D):
            S = np.sqrt(1.0 + 3.0 * u[d] ** 2)
            v = v * (2.0 - S) * ((2.0 * u[d] + S) / (1.0 - u[d])) ** c[d]
        out.append(v)
    return np.array(out)


def moment_matrix(C, D):
    """Rows: raw moments sum_i c_x^p c_y^q c_z^r, p, q, r in {0, 1, 2}."""
    exps = list(itertools.product(range(3), repeat=D))
    T = np.array([[np.prod([c[d] ** e[d] for d in range(D)]) for c in C] for e in exps], dtype=float)
    return T, exps


def kbc_shear(df, C, D):
    """Shear part: the population whose raw moments are the deviatoric
    second moments of df (trace-free diagonal, off-diagonal pairs) and zero
    otherwise."""
    T, exps = moment_matrix(C, D)
    M = np.tensordot(T, df, axes=(1, 0))
    Ms = np.zeros_like(M)
    diag = [exps.index(tuple(2 if d == a else 0 for d in range(D))) for a in range(D)]
    tr = sum(M[k] for k in diag)
    for k in diag:
        Ms[k] = M[k] - tr / D
    for a in range(D):
        for b in range(a + 1, D):
            k = exps.index(tuple(1 if d in (a, b) else 0 for d in range(D)))
            Ms[k] = M[k]
    flat = Ms.reshape(Ms.shape[0], -1)
    return np.linalg.solve(T, flat).reshape(df.shape)


def step(orc, p, f, g):
    C, Wt, D = lattice(p.lattice)
    rho = f.sum(0)
    phi = g.sum(0)
    j = np.stack([sum(f[i] * C[i][d] for i in range(len(C))) for d in range(3)])
    A, B, Dc = orc.gradient_coefficients(p)
    lr, lp = laplacian(rho, C, Wt), laplacian(phi, C, Wt)
    mub = np.vectorize(lambda r, q: orc.mu_bulk(p, r, q), otypes=[object])(rho, phi)
    mu_r = np.array([[[m[0] for m in row] for row in pl] for pl in mub]) - 2 * A * lr - Dc * lp
    mu_p = np.array([[[m[1] for m in row] for row in pl] for pl in mub]) - 2 * B * lp - Dc * lr
    F = -rho * gradient(mu_r - CS2 * np.log(rho), C, Wt) - phi * gradient(mu_p, C, Wt)
    if D == 2:
        F[2] = 0.0
    tau = 3.0 * p.nu + 0.5
    beta = 1.0 / (2.0 * tau)
    u = j / rho
    du = F / rho
    fe = feq(rho, u, C, Wt, D)
    df = f - fe
    ds = kbc_shear(df, C, D)
    dh = df - ds
    sh = (ds * dh / fe).sum(0)
    hh = (dh * dh / fe).sum(0)
    gam = np.where(hh > 1e-300, 1.0 / beta - (2.0 - 1.0 / beta) * sh / np.where(hh > 1e-300, hh, 1.0), 2.0)
    fstar = f - beta * (2.0 * ds + gam * dh) + (feq(rho, u + du, C, Wt, D) - fe)
    up = (j + 0.5 * F) / rho
    if D == 2:
        up[2] = 0.0
    Gam = p.mobility / (p.tau_phi - 0.5)
    ge = []
    for c, w in zip(C, Wt):
        cu = sum(c[d] * up[d] for d in range(3))
        uu = (up ** 2).sum(0)
        ge.append(w * (Gam * mu_p / CS2 + phi * cu / CS2 + phi * cu ** 2 / (2 * CS2 ** 2) - phi * uu / (2 * CS2)))
    ge = np.array(ge)
    ge[0] = phi - ge[1:].sum(0)
    gstar = g - (g - ge) / p.tau_phi
    # stream: f(x + c) <- f*(x)
    fn = np.array([shift(fstar[i], -C[i]) for i in range(len(C))])
    gn = np.array([shift(gstar[i], -C[i]) for i in range(len(C))])
    return fn, gn


@pytest.mark.parametrize("lat,shape", [(0, (1, 4, 4)), (1, (3, 3, 3))])
def test_whole_step_matches_brute_force(orc, lat, shape):
    nz, ny, nx = shape
    p = orc.coexisting_params(10.0, lattice=lat, nx=nx, ny=ny, nz=nz, kappa2=0.04, kappa3=0.07,
                              lambda2=0.125, lambda3=0.22)
    rng = np.random.default_rng(11 + lat)
    s = rng.uniform(0, 1, size=shape)
    rho0 = p.rho_g + (p.rho_l - p.rho_g) * s
    phi0 = p.chi * s * rng.uniform(-1, 1, size=shape)
    u0 = rng.uniform(-0.03, 0.03, size=(3,) + shape)
    if lat == 0:
        u0[2] = 0.0
    st = orc.State(p, rho0, phi0, u0)
    f, g = st.f.copy(), st.g.copy()
    for _ in range(2):
        f, g = step(orc, p, f, g)
    st.run(2)
    assert np.abs(st.f - f).max() < 1e-12 * np.abs(f).max()
    assert np.abs(st.g - g).max() < 1e-12 * np.abs(g).max()
