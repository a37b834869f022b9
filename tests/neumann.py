"""Liquid-lens geometry for the Neumann-angle checks (test infrastructure).

The paper's lens (Fig. 2): a drop of liquid 1 suspended at the flat
interface between liquid 2 and the gas.  At equilibrium the three interfaces
meet at the triple points at angles fixed by the three tensions (the force
balance stated with Fig. 2: gamma_12 / sin(theta_3) = gamma_2g / sin(theta_2)
= gamma_1g / sin(theta_1)).  Here an angle is labelled by the phase it lies
in; the angle in phase i, opposite the tension gamma_jk of the interface
between the other two phases, has
    cos(theta_i) = (gamma_jk^2 - gamma_ij^2 - gamma_ik^2) / (2 gamma_ij gamma_ik).

`lens_fields` builds the starting state, `measure_angles` fits the relaxed
fields: each interface is the zero set of the difference of the two phases'
concentrations (C_l1, C_l2, C_g from rho and phi as defined in the paper),
points taken by linear interpolation along grid edges, the lens arcs fitted
by least-squares circles and the liquid-2/gas interface by a straight line,
points within `exclude` nodes of the triple points left out.  The triple
points are the intersections of the two arcs; the angles are those between
the tangents there.
"""
from __future__ import annotations

import math

import numpy as np


def neumann_angles(g12: float, g1g: float, g2g: float) -> dict:
    """Angles (degrees) in liquid 1, liquid 2 and gas of the tension triangle."""
    def ang(opp, a, b):
        c = (opp * opp - a * a - b * b) / (2.0 * a * b)
        return math.degrees(math.acos(max(-1.0, min(1.0, c))))
    return {"1": ang(g2g, g1g, g12), "2": ang(g1g, g2g, g12), "g": ang(g12, g1g, g2g)}


def lens_fields(nx, ny, radius, band, rho_g, rho_l, chi, width=2.0):
    """(rho, phi) of shape (1, ny, nx): a liquid-2 band band[0] <= y < band[1]
    with gas elsewhere (periodic), and a disc of liquid 1 of `radius`
    centred on the band's upper interface at x = nx/2."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    yc = band[1] - 0.5
    c1 = 0.5 * (1.0 - np.tanh((np.hypot(x - nx / 2.0, y - yc) - radius) / width))
    c2 = 0.5 * (np.tanh((y - band[0] + 0.5) / width) - np.tanh((y - band[1] + 0.5) / width))
    c2 = c2 * (1.0 - c1)
    liquid = np.clip(c1 + c2, 0.0, 1.0)
    rho = rho_g + (rho_l - rho_g) * liquid
    phi = chi * (c1 - c2)
    return rho[None], phi[None]


def concentrations(rho, phi, rho_g, rho_l, chi):
    cg = (rho - rho_l) / (rho_g - rho_l)
    c1 = 0.5 * (1.0 + phi / chi - cg)
    c2 = 0.5 * (1.0 - phi / chi - cg)
    return c1, c2, cg


def zero_points(f, mask):
    """Linear-interpolated zeros of f along the grid edges where both ends
    are in mask; returns an (n, 2) array of (x, y)."""
    pts = []
    ny, nx = f.shape
    for dy, dx in ((0, 1), (1, 0)):
        a = f[: ny - dy, : nx - dx]
        b = f[dy:, dx:]
        m = (a * b < 0) & mask[: ny - dy, : nx - dx] & mask[dy:, dx:]
        yy, xx = np.nonzero(m)
        t = a[m] / (a[m] - b[m])
        pts.append(np.stack([xx + t * dx, yy + t * dy], axis=1))
    return np.concatenate(pts) if pts else np.zeros((0, 2))


def fit_circle(p):
    """Least-squares circle (algebraic fit, refined by Gauss-Newton on the
    geometric distances): centre (cx, cy) and radius."""
    x, y = p[:, 0], p[:, 1]
    A = np.stack([x, y, np.ones_like(x)], axis=1)
    b = x * x + y * y
    s = np.linalg.lstsq(A, b, rcond=None)[0]
    cx, cy = s[0] / 2, s[1] / 2
    r = math.sqrt(s[2] + cx * cx + cy * cy)
    for _ in range(20):
        dx, dy = x - cx, y - cy
        d = np.hypot(dx, dy)
        J = np.stack([-dx / d, -dy / d, -np.ones_like(d)], axis=1)
        res = d - r
        step = np.linalg.lstsq(J, -res, rcond=None)[0]
        cx, cy, r = cx + step[0], cy + step[1], r + step[2]
        if np.abs(step).max() < 1e-12:
            break
    return np.array([cx, cy]), r


def circle_intersections(c0, r0, c1, r1):
    d = np.linalg.norm(c1 - c0)
    a = (r0 * r0 - r1 * r1 + d * d) / (2 * d)
    h = math.sqrt(max(r0 * r0 - a * a, 0.0))
    m = c0 + a * (c1 - c0) / d
    perp = np.array([-(c1 - c0)[1], (c1 - c0)[0]]) / d
    return m + h * perp, m - h * perp


def _arc_tangent(c, P, pts):
    """Unit tangent of the circle (centre c) at P pointing towards the arc's
    points `pts`."""
    rad = P - c
    t = np.array([-rad[1], rad[0]]) / np.linalg.norm(rad)
    mean = pts.mean(axis=0) - P
    return t if t @ mean > 0 else -t


def _line_tangent(direction, P, pts):
    side = pts - P
    return direction if (side @ direction).mean() > 0 else -direction


def _angle(a, b):
    return math.degrees(math.acos(max(-1.0, min(1.0, float(a @ b)))))


def measure_angles(rho, phi, rho_g, rho_l, chi, band_top, exclude=5.0, thr=0.25):
    """Neumann angles (degrees) of a relaxed lens (2D fields of shape (ny,
    nx)) at both triple points, with the fits used.  `band_top` is the
    nominal y of the liquid-2/gas interface that carries the lens; only the
    points within a quarter of the box height of it are used."""
    c1, c2, cg = concentrations(rho, phi, rho_g, rho_l, chi)
    return measure_angles_c(c1, c2, cg, band_top, exclude, thr)


def measure_angles_c(c1, c2, cg, band_top, exclude=5.0, thr=0.25):
    """measure_angles from the three phases' concentration fields: c1 the
    lens, c2 the phase below the flat interface, cg the phase above it."""
    ny, nx = c1.shape
    yy = np.mgrid[0:ny, 0:nx][0]
    near = np.abs(yy - band_top) < ny / 4
    p1g = zero_points(c1 - cg, near & (c2 < thr))
    p12 = zero_points(c1 - c2, near & (cg < thr))
    p2g = zero_points(c2 - cg, near & (c1 < thr))
    c_1g, r_1g = fit_circle(p1g)
    c_12, r_12 = fit_circle(p12)
    tps = circle_intersections(c_1g, r_1g, c_12, r_12)
    for _ in range(2):
        keep = lambda p: p[np.min([np.linalg.norm(p - t, axis=1) for t in tps], axis=0) > exclude]
        q1g, q12, q2g = keep(p1g), keep(p12), keep(p2g)
        c_1g, r_1g = fit_circle(q1g)
        c_12, r_12 = fit_circle(q12)
        tps = circle_intersections(c_1g, r_1g, c_12, r_12)
    # the liquid-2/gas interface: a straight line (total least squares)
    m = q2g.mean(axis=0)
    _, _, vt = np.linalg.svd(q2g - m)
    d2g = vt[0]
    out = []
    for P in sorted(tps, key=lambda t: t[0]):
        side = q2g[(q2g[:, 0] < P[0]) if P[0] < nx / 2 else (q2g[:, 0] > P[0])]
        # the arcs' points on this triple point's half of the lens
        half = (lambda q: q[(q[:, 0] < nx / 2)] if P[0] < nx / 2 else q[(q[:, 0] >= nx / 2)])
        t1g = _arc_tangent(c_1g, P, half(q1g))
        t12 = _arc_tangent(c_12, P, half(q12))
        t2g = _line_tangent(d2g, P, side)
        out.append({"1": _angle(t1g, t12), "2": _angle(t12, t2g), "g": _angle(t1g, t2g),
                    "point": P.tolist()})
    fits = {"r_1g": r_1g, "r_12": r_12, "c_1g": c_1g.tolist(), "c_12": c_12.tolist(),
            "n_points": [len(q1g), len(q12), len(q2g)]}
    return out, fits
