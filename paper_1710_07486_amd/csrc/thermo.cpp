// thermo.cpp -- host thermodynamics of the equation of state used by the free
// energy (Eq. 4 of arXiv:1710.07486 and the van der Waals / Peng-Robinson
// alternatives): critical point, Maxwell coexistence, temperature for a
// target density ratio.
//
// Written in the packing fraction e = b rho / 4, where the CS pressure is
//   p = (4 R T / b) Z1(e) - (16 a / b^2) e^2,  Z1(e) = e (1 + e + e^2 - e^3)/(1 - e)^3,
// and the chemical potential (Psi' of Eq. 4 with C = 0) is
//   mu(rho) = -2 a rho + R T (ln rho + 1) - 16 R T (12 - b rho)/(b rho - 4)^3.
#include <math.h>

#include "thermo.hpp"

namespace telbm {

static double Z1p(double e) {  // dZ1/de = (1 + 4e + 4e^2 - 4e^3 + e^4)/(1 - e)^4
    const double n = 1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)));
    const double m = 1.0 - e;
    return n / (m * m * m * m);
}

static double Z1pp(double e) {  // d2Z1/de2 = [N'(1 - e) + 4 N]/(1 - e)^5
    const double n = 1.0 + e * (4.0 + e * (4.0 + e * (-4.0 + e)));
    const double np = 4.0 + e * (8.0 + e * (-12.0 + 4.0 * e));
    const double m = 1.0 - e;
    return (np * m + 4.0 * n) / (m * m * m * m * m);
}

double cs_pressure(double a, double b, double R, double T, double rho) {
    const double e = 0.25 * b * rho;
    const double m = 1.0 - e;
    return rho * R * T * (1.0 + e + e * e - e * e * e) / (m * m * m) - a * rho * rho;
}

double cs_mu(double a, double b, double R, double T, double rho) {
    const double d = b * rho - 4.0;
    return -2.0 * a * rho + R * T * (log(rho) + 1.0) - 16.0 * R * T * (12.0 - b * rho) / (d * d * d);
}

// Spinodal temperature as a function of the packing fraction: dp/de = 0.
static double t_spin(double a, double b, double R, double e) { return 8.0 * a * e / (b * R * Z1p(e)); }

bool critical_point(double a, double b, double R, double* Tc, double* rho_c) {
    if (!(a > 0 && b > 0 && R > 0)) return false;
    // e Z1''(e) = Z1'(e) at the critical point; h(e) changes sign once on (0, 1/2)
    double lo = 1e-6, hi = 0.5;
    auto h = [](double e) { return e * Z1pp(e) - Z1p(e); };
    const double hlo = h(lo);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if ((h(mid) < 0) == (hlo < 0)) lo = mid; else hi = mid;
    }
    const double ec = 0.5 * (lo + hi);
    if (Tc) *Tc = t_spin(a, b, R, ec);
    if (rho_c) *rho_c = 4.0 * ec / b;
    return true;
}

// root of f on [lo, hi] with a sign change, by bisection
template <class F>
static double bisect(F f, double lo, double hi, int iters = 300) {
    const bool slo = f(lo) < 0;
    for (int it = 0; it < iters; ++it) {
        const double mid = 0.5 * (lo + hi);
        if ((f(mid) < 0) == slo) lo = mid; else hi = mid;
        if (hi - lo <= 4e-17 * fabs(hi)) break;
    }
    return 0.5 * (lo + hi);
}

bool maxwell(double a, double b, double R, double T, double* rho_g, double* rho_l, double* C, double* Psi0) {
    double Tc, rc;
    if (!critical_point(a, b, R, &Tc, &rc)) return false;
    if (!(T > 0.0 && T < Tc)) return false;
    const double ec = 0.25 * b * rc;
    // spinodal packing fractions bracket the unstable branch
    const double e1 = bisect([&](double e) { return t_spin(a, b, R, e) - T; }, 1e-15, ec);
    const double e2 = bisect([&](double e) { return t_spin(a, b, R, e) - T; }, ec, 1.0 - 1e-12);
    const double s1 = 4.0 * e1 / b, s2 = 4.0 * e2 / b;
    const double mu_s1 = cs_mu(a, b, R, T, s1);
    // For a liquid density y above the liquid spinodal, the gas density x below
    // the gas spinodal with the same chemical potential (mu increases from
    // -inf on the gas branch); the pressure mismatch p(y) - p(x(y)) is shot to zero.
    auto gas_for = [&](double y, bool* ok) {
        const double m = cs_mu(a, b, R, T, y);
        if (m >= mu_s1) { *ok = false; return s1; }
        *ok = true;
        // solve in ln(rho) to cover many decades
        const double lx = bisect([&](double l) { return cs_mu(a, b, R, T, exp(l)) - m; }, -745.0, log(s1));
        return exp(lx);
    };
    auto resid = [&](double y) {
        bool ok;
        const double x = gas_for(y, &ok);
        if (!ok) return -1.0;  // liquid mu above the gas branch: liquid too dilute
        return cs_pressure(a, b, R, T, y) - cs_pressure(a, b, R, T, x);
    };
    // The gas partner exists while mu(y) < mu(s1): up to y* with mu(y*) = mu(s1).
    // The residual is negative at the liquid spinodal and positive just below y*.
    const double ystar = bisect([&](double yv) { return cs_mu(a, b, R, T, yv) - mu_s1; }, s2, 4.0 / b * (1.0 - 1e-9));
    const double y = bisect(resid, s2, ystar * (1.0 - 1e-13), 400);
    bool ok;
    double x = gas_for(y, &ok);
    if (!ok) return false;
    // two Newton polish steps on (ln x, y) for equal mu and p
    double lx = log(x), yy = y;
    for (int it = 0; it < 3; ++it) {
        const double xx = exp(lx);
        const double r1 = cs_mu(a, b, R, T, yy) - cs_mu(a, b, R, T, xx);
        const double r2 = cs_pressure(a, b, R, T, yy) - cs_pressure(a, b, R, T, xx);
        // d mu / d rho = (dp/drho)/rho
        const double h = 1e-7;
        const double dpy = (cs_pressure(a, b, R, T, yy * (1 + h)) - cs_pressure(a, b, R, T, yy * (1 - h))) / (2 * h * yy);
        const double dpx = (cs_pressure(a, b, R, T, xx * (1 + h)) - cs_pressure(a, b, R, T, xx * (1 - h))) / (2 * h * xx);
        // J = [[dmu/dy, -dmu/dlnx], [dp/dy, -dp/dlnx]]
        const double j11 = dpy / yy, j12 = -dpx, j21 = dpy, j22 = -dpx * xx;
        const double det = j11 * j22 - j12 * j21;
        if (!(fabs(det) > 0)) break;
        const double dy = (-r1 * j22 + r2 * j12) / det;
        const double dl = (-r2 * j11 + r1 * j21) / det;
        if (!(isfinite(dy) && isfinite(dl))) break;
        yy += dy;
        lx += dl;
    }
    x = exp(lx);
    const double c = -cs_mu(a, b, R, T, x);
    const double br = b * x;
    *rho_g = x;
    *rho_l = yy;
    if (C) *C = c;
    if (Psi0) *Psi0 = x * (c - a * x - 8.0 * R * T * (br - 6.0) / ((br - 4.0) * (br - 4.0)) + R * T * log(x));
    return isfinite(x) && isfinite(yy) && yy > x;
}

bool temperature_for_ratio(double a, double b, double R, double ratio, double* T) {
    double Tc, rc;
    if (!(ratio > 1.0) || !critical_point(a, b, R, &Tc, &rc)) return false;
    auto lr = [&](double t) {
        double rg, rl;
        if (!maxwell(a, b, R, t, &rg, &rl, nullptr, nullptr)) return -1e300;
        return log(rl / rg) - log(ratio);
    };
    const double t = bisect(lr, 0.05 * Tc, Tc * (1.0 - 1e-9), 200);
    *T = t;
    return isfinite(t);
}

// ---------------------------------------------------------------------------
// van der Waals and Peng-Robinson.  Both read p = rho RT/(1 - b rho) - A g(rho)
// with g = rho^2 (vdW) or rho^2/(1 + 2 b rho - b^2 rho^2) (PR), A = a or
// a alpha(T), alpha = [1 + m(1 - sqrt(T/T_c))]^2, m = 0.37464 + 1.54226 w
// - 0.26992 w^2.  The matching Psi (p = rho Psi' - Psi, C = 0) is
//   rho RT ln(rho/(1 - b rho)) - A rho^2                          (vdW)
//   rho RT ln(rho/(1 - b rho)) - A rho/(2 sqrt2 b) ln[(1 + (1+sqrt2) b rho)
//                                  / (1 + (1-sqrt2) b rho)]        (PR)
// The spinodal dp/drho = 0 reads T = A g'(rho)(1 - b rho)^2 / R =: T_sp(rho);
// the critical point is the maximum of T_sp at alpha = 1.
// ---------------------------------------------------------------------------
namespace {

constexpr double kSqrt2 = 1.41421356237309504880;

double g_att(const EosSpec& e, double rho) {
    const double br = e.b * rho;
    return e.kind == 1 ? rho * rho : rho * rho / (1.0 + 2.0 * br - br * br);
}

double g_att_prime(const EosSpec& e, double rho) {  // dg/drho; PR: 2 rho (1 + b rho)/D^2
    const double br = e.b * rho;
    if (e.kind == 1) return 2.0 * rho;
    const double D = 1.0 + 2.0 * br - br * br;
    return 2.0 * rho * (1.0 + br) / (D * D);
}

double p_cubic(const EosSpec& e, double A, double T, double rho) {
    return rho * e.R * T / (1.0 - e.b * rho) - A * g_att(e, rho);
}

double mu_cubic(const EosSpec& e, double A, double T, double rho) {  // Psi' with C = 0
    const double br = e.b * rho, m = 1.0 - br;
    const double rep = e.R * T * (log(rho / m) + 1.0 / m);
    if (e.kind == 1) return rep - 2.0 * A * rho;
    const double D = 1.0 + 2.0 * br - br * br;
    return rep - A * (log((1.0 + (1.0 + kSqrt2) * br) / (1.0 + (1.0 - kSqrt2) * br)) / (2.0 * kSqrt2 * e.b) + rho / D);
}

double psi_cubic(const EosSpec& e, double A, double T, double rho) {  // Psi with C = 0
    const double br = e.b * rho;
    const double rep = rho * e.R * T * log(rho / (1.0 - br));
    if (e.kind == 1) return rep - A * rho * rho;
    return rep - A * rho / (2.0 * kSqrt2 * e.b) * log((1.0 + (1.0 + kSqrt2) * br) / (1.0 + (1.0 - kSqrt2) * br));
}

double t_sp(const EosSpec& e, double A, double rho) {
    const double m = 1.0 - e.b * rho;
    return A * g_att_prime(e, rho) * m * m / e.R;
}

// Density of the maximum of T_sp (bisection on the sign of its slope).
double t_sp_peak(const EosSpec& e, double A) {
    double lo = 1e-9 / e.b, hi = (1.0 - 1e-9) / e.b;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi), h = 1e-7 * mid;
        if (t_sp(e, A, mid + h) > t_sp(e, A, mid - h)) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

bool cubic_critical(const EosSpec& e, double* Tc, double* rho_c) {
    if (!(e.a > 0 && e.b > 0 && e.R > 0)) return false;
    const double r = t_sp_peak(e, e.a);
    if (Tc) *Tc = t_sp(e, e.a, r);
    if (rho_c) *rho_c = r;
    return true;
}

bool cubic_maxwell(const EosSpec& e, double T, double* rho_g, double* rho_l, double* C, double* Psi0) {
    double Tc;
    if (!cubic_critical(e, &Tc, nullptr) || !(T > 0.0 && T < Tc)) return false;
    const double A = eos_attraction(e, T);
    const double rm = t_sp_peak(e, A);
    if (!(t_sp(e, A, rm) > T)) return false;
    const double top = 1.0 / e.b;
    const double s1 = bisect([&](double r) { return t_sp(e, A, r) - T; }, 1e-300, rm);
    const double s2 = bisect([&](double r) { return T - t_sp(e, A, r); }, rm, top * (1.0 - 1e-14));
    const double mu_s1 = mu_cubic(e, A, T, s1);
    // as for Carnahan-Starling: the gas density with the liquid's chemical
    // potential (mu rises from -inf on the gas branch), then shoot the
    // pressure difference to zero
    auto gas_for = [&](double y, bool* ok) {
        const double m = mu_cubic(e, A, T, y);
        if (m >= mu_s1) { *ok = false; return s1; }
        *ok = true;
        const double lx = bisect([&](double l) { return mu_cubic(e, A, T, exp(l)) - m; }, -745.0, log(s1));
        return exp(lx);
    };
    auto resid = [&](double y) {
        bool ok;
        const double x = gas_for(y, &ok);
        if (!ok) return -1.0;
        return p_cubic(e, A, T, y) - p_cubic(e, A, T, x);
    };
    const double ystar = bisect([&](double yv) { return mu_cubic(e, A, T, yv) - mu_s1; }, s2, top * (1.0 - 1e-12));
    const double y = bisect(resid, s2, ystar * (1.0 - 1e-13), 400);
    bool ok;
    const double x = gas_for(y, &ok);
    if (!ok) return false;
    const double c = -mu_cubic(e, A, T, x);
    *rho_g = x;
    *rho_l = y;
    if (C) *C = c;
    if (Psi0) *Psi0 = psi_cubic(e, A, T, x) + c * x;
    return isfinite(x) && isfinite(y) && y > x;
}

}  // namespace

double eos_attraction(const EosSpec& e, double T) {
    if (e.kind != 2) return e.a;
    double Tc;
    if (!cubic_critical(e, &Tc, nullptr)) return e.a;
    const double m = 0.37464 + 1.54226 * e.omega - 0.26992 * e.omega * e.omega;
    const double s = 1.0 + m * (1.0 - sqrt(T / Tc));
    return e.a * s * s;
}

bool eos_critical_point(const EosSpec& e, double* Tc, double* rho_c) {
    if (e.kind == 0) return critical_point(e.a, e.b, e.R, Tc, rho_c);
    if (e.kind == 2 && !isfinite(e.omega)) return false;
    return (e.kind == 1 || e.kind == 2) && cubic_critical(e, Tc, rho_c);
}

bool eos_maxwell(const EosSpec& e, double T, double* rho_g, double* rho_l, double* C, double* Psi0) {
    if (e.kind == 0) return maxwell(e.a, e.b, e.R, T, rho_g, rho_l, C, Psi0);
    if (e.kind != 1 && e.kind != 2) return false;
    return cubic_maxwell(e, T, rho_g, rho_l, C, Psi0);
}

bool eos_temperature_for_ratio(const EosSpec& e, double ratio, double* T) {
    if (e.kind == 0) return temperature_for_ratio(e.a, e.b, e.R, ratio, T);
    double Tc, rc;
    if (!(ratio > 1.0) || !eos_critical_point(e, &Tc, &rc)) return false;
    auto lr = [&](double t) {
        double rg, rl;
        if (!eos_maxwell(e, t, &rg, &rl, nullptr, nullptr)) return -1e300;
        return log(rl / rg) - log(ratio);
    };
    const double t = bisect(lr, 0.05 * Tc, Tc * (1.0 - 1e-9), 200);
    *T = t;
    return isfinite(t);
}

}  // namespace telbm
