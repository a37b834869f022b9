/*
 * telbm_oracle.c -- plain FP64 CPU oracle for the ternary free-energy
 * entropic lattice Boltzmann update of Woehrwag, Semprebon, Mazloomi,
 * Karlin and Kusumaatmaja, "Ternary free-energy entropic lattice Boltzmann
 * model with high density ratio" (arXiv:1710.07486).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Every lattice-wide quantity is computed in its own full pass, in the order
 * the method defines it: moments -> Laplacians -> chemical potentials ->
 * gradients -> thermodynamic force -> entropic (KBC) collision with
 * exact-difference forcing -> phase-field BGK -> streaming.  Arithmetic is
 * IEEE double; build with -ffp-contract=off so that no multiply-add is fused.
 *
 * Readings of points the paper leaves to its (unavailable) supplement are
 * marked "Reading:" at the place they are used.
 *
 * Parity status: every function here is pinned by the CPU test-suite against
 * closed forms, invariants or independent numerics (see the docstrings of
 * tests/test_oracle_*.py).  None is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Parameters.                                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t lattice;              /* 0: D2Q9, 1: D3Q27                       */
    int32_t nx, ny, nz;           /* periodic box; nz == 1 for D2Q9          */
    double a, b, R, T;            /* EOS constants (Eq. 4 for Carnahan-Starling) */
    double rho_g, rho_l;          /* coexisting gas / liquid densities       */
    double C;                     /* EOS constant C of Eq. (4)               */
    double lambda1, lambda2, lambda3; /* bulk free energy, Eq. (2)           */
    double kappa1, kappa2, kappa3;    /* interfacial free energy, Eq. (3)    */
    double chi;                   /* scale of the phase field phi            */
    double nu;                    /* kinematic viscosity eta/rho             */
    double mobility;              /* M of the Cahn-Hilliard equation (7)     */
    double tau_phi;               /* relaxation time of the phi populations  */
    int32_t eos;                  /* 0 Carnahan-Starling (Eq. 4), 1 van der Waals, 2 Peng-Robinson */
    int32_t pad;
    double omega;                 /* Peng-Robinson acentric factor            */
    int32_t walls;                /* 1: solid walls at y = -1/2 and y = ny - 1/2 */
    int32_t pad2;
    double theta_rho_lo, theta_rho_hi; /* contact angles (radians) of the      */
    double theta_phi_lo, theta_phi_hi; /* rho and phi fields, bottom / top wall */
    int32_t glattice;             /* phase-field lattice: 0 as for f, 1 reduced (D2Q5 / D3Q7) */
    int32_t pad3;
} orc_params;

/* ------------------------------------------------------------------------- */
/* Lattice.  Directions are the tensor product of the D1Q3 set {0,+1,-1} per  */
/* axis: index i = kx + 3 ky + 9 kz with k = 0,1,2 meaning c = 0,+1,-1.      */
/* D2Q9 is the first nine of D3Q27 (kz = 0).  Weights are products of the    */
/* D1Q3 weights 2/3 (c = 0) and 1/6 (c = +-1), which gives 4/9, 1/9, 1/36 in */
/* 2D and 8/27, 2/27, 1/54, 1/216 in 3D.                                     */
/* ------------------------------------------------------------------------- */

static const int K2C[3] = {0, 1, -1};

static int lattice_Q(int lattice) { return lattice == 0 ? 9 : 27; }
static int lattice_D(int lattice) { return lattice == 0 ? 2 : 3; }

static void direction(int i, int c[3])
{
    c[0] = K2C[i % 3];
    c[1] = K2C[(i / 3) % 3];
    c[2] = K2C[i / 9];
}

/* Index of -c_i: negating every component maps k = 1 <-> 2 and keeps 0. */
static int opposite(int i)
{
    static const int NEG[3] = {0, 2, 1};
    return NEG[i % 3] + 3 * NEG[(i / 3) % 3] + 9 * NEG[i / 9];
}

static double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }

/* The D2Q9 weight is the product over two axes only. */
static double weight_lat(int lattice, int i)
{
    int c[3];
    direction(i, c);
    if (lattice == 0) return w1(c[0]) * w1(c[1]);
    return w1(c[0]) * w1(c[1]) * w1(c[2]);
}

int orc_lattice_info(int lattice, int32_t *c_out, double *w_out)
{
    int Q = lattice_Q(lattice);
    for (int i = 0; i < Q; ++i) {
        int c[3];
        direction(i, c);
        c_out[3 * i + 0] = c[0];
        c_out[3 * i + 1] = c[1];
        c_out[3 * i + 2] = c[2];
        w_out[i] = weight_lat(lattice, i);
    }
    return Q;
}

static const double CS2 = 1.0 / 3.0;  /* lattice speed of sound squared */

/* ------------------------------------------------------------------------- */
/* Thermodynamics of the liquid-gas equation of state.  The paper uses the   */
/* Carnahan-Starling EOS, Eq. (4), and names Peng-Robinson and van der Waals */
/* as alternatives.  Psi_eos follows from the EOS pressure through           */
/* p = rho Psi' - Psi (stated above Eq. (4)); each Psi below is that integral */
/* of the textbook pressure, up to the linear term C rho:                    */
/*   van der Waals   p = rho RT/(1 - b rho) - a rho^2                         */
/*     Psi = rho RT ln(rho/(1 - b rho)) - a rho^2 + C rho                     */
/*   Peng-Robinson   p = rho RT/(1 - b rho) - A rho^2/(1 + 2 b rho - b^2 rho^2)*/
/*     Psi = rho RT ln(rho/(1 - b rho))                                       */
/*           - (A rho/(2 sqrt2 b)) ln[(1 + (1+sqrt2) b rho)/(1 + (1-sqrt2) b rho)]*/
/*           + C rho,                                                         */
/*     A = a alpha(T), alpha = [1 + m (1 - sqrt(T/T_c))]^2,                   */
/*     m = 0.37464 + 1.54226 omega - 0.26992 omega^2 (omega: acentric factor).*/
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t kind;       /* 0 Carnahan-Starling, 1 van der Waals, 2 Peng-Robinson */
    double a, b, R, omega;
} orc_eos;

static const double SQRT2 = 1.41421356237309504880;

/* Peng-Robinson critical temperature of a, b, R (alpha = 1 there). */
static double pr_tc(const orc_eos *e);

/* Attraction coefficient at temperature T. */
static double eos_attraction(const orc_eos *e, double T)
{
    if (e->kind != 2) return e->a;
    double m = 0.37464 + 1.54226 * e->omega - 0.26992 * e->omega * e->omega;
    double s = 1.0 + m * (1.0 - sqrt(T / pr_tc(e)));
    return e->a * s * s;
}

/* Psi_eos(rho) with the constant C. */
static double eos_psi_A(const orc_eos *e, double A, double T, double C, double rho)
{
    double a = e->a, b = e->b, RT = e->R * T, br = b * rho;
    if (e->kind == 0)
        return rho * (C - a * rho - 8.0 * RT * (br - 6.0) / ((br - 4.0) * (br - 4.0)) + RT * log(rho));
    double rep = rho * RT * log(rho / (1.0 - br));
    if (e->kind == 1) return rep - A * rho * rho + C * rho;
    return rep - A * rho / (2.0 * SQRT2 * b) * log((1.0 + (1.0 + SQRT2) * br) / (1.0 + (1.0 - SQRT2) * br)) + C * rho;
}

/* d Psi / d rho, differentiated term by term:
 *   CS:  C - 2 a rho + RT (ln rho + 1) - 8RT (b rho - 6)/(b rho - 4)^2
 *          - 8 RT b rho (8 - b rho)/(b rho - 4)^3
 *   vdW: C + RT [ln(rho/(1 - b rho)) + 1/(1 - b rho)] - 2 a rho
 *   PR:  C + RT [ln(rho/(1 - b rho)) + 1/(1 - b rho)]
 *          - (A/(2 sqrt2 b)) ln[...] - A rho/(1 + 2 b rho - b^2 rho^2)        */
static double eos_psi_prime_A(const orc_eos *e, double A, double T, double C, double rho)
{
    double a = e->a, b = e->b, RT = e->R * T, br = b * rho;
    if (e->kind == 0) {
        double d = br - 4.0;
        return C - 2.0 * a * rho + RT * (log(rho) + 1.0) - 8.0 * RT * (br - 6.0) / (d * d)
               - 8.0 * RT * br * (8.0 - br) / (d * d * d);
    }
    double rep = RT * (log(rho / (1.0 - br)) + 1.0 / (1.0 - br));
    if (e->kind == 1) return C + rep - 2.0 * A * rho;
    double D = 1.0 + 2.0 * br - br * br;
    return C + rep - A / (2.0 * SQRT2 * b) * log((1.0 + (1.0 + SQRT2) * br) / (1.0 + (1.0 - SQRT2) * br))
           - A * rho / D;
}

/* Psi'' = T q(rho) - A s(rho): q from the repulsive part (per unit T), s from
 * the attractive part (per unit A).
 *   CS:  q = R/rho - 8 R b (8 - br)/d^3 - 8 R b [(8 - 2 br) d - 3 br (8 - br)]/d^4, s = 2
 *   vdW, PR: q = R [1/rho + b/(1 - br) + b/(1 - br)^2]
 *   vdW: s = 2;  PR: s = 1/D + (1 + br^2)/D^2, D = 1 + 2 br - br^2            */
static double eos_q(const orc_eos *e, double rho)
{
    double b = e->b, R = e->R, br = b * rho;
    if (e->kind == 0) {
        double d = br - 4.0;
        double t1 = -8.0 * R * b * (8.0 - br) / (d * d * d);
        double t2 = -8.0 * R * b * ((8.0 - 2.0 * br) * d - 3.0 * br * (8.0 - br)) / (d * d * d * d);
        return R / rho + t1 + t2;
    }
    double m = 1.0 - br;
    return R * (1.0 / rho + b / m + b / (m * m));
}

static double eos_s(const orc_eos *e, double rho)
{
    if (e->kind != 2) return 2.0;
    double br = e->b * rho, D = 1.0 + 2.0 * br - br * br;
    return 1.0 / D + (1.0 + br * br) / (D * D);
}

static double eos_rho_max(const orc_eos *e) { return e->kind == 0 ? 4.0 / e->b : 1.0 / e->b; }

static double eos_pressure_A(const orc_eos *e, double A, double T, double rho)
{
    return rho * eos_psi_prime_A(e, A, T, 0.0, rho) - eos_psi_A(e, A, T, 0.0, rho);
}

static double eos_dpdrho_A(const orc_eos *e, double A, double T, double rho)
{
    return rho * (T * eos_q(e, rho) - A * eos_s(e, rho));
}

/* Critical point with the attraction a (alpha = 1): the spinodal dp/drho = 0
 * gives T_spin(rho) = a s(rho)/q(rho); the critical point is its maximum
 * (golden-section search on (0, rho_max)).                                  */
static double eos_tc(const orc_eos *e, double *rho_c)
{
    double lo = 1e-6, hi = eos_rho_max(e) * (1.0 - 1e-6);
    const double gr = 0.5 * (sqrt(5.0) - 1.0);
#define TSPIN(r) (e->a * eos_s(e, r) / eos_q(e, r))
    double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
    double f1 = TSPIN(x1), f2 = TSPIN(x2);
    for (int it = 0; it < 300; ++it) {
        if (f1 < f2) {
            lo = x1; x1 = x2; f1 = f2;
            x2 = lo + gr * (hi - lo);
            f2 = TSPIN(x2);
        } else {
            hi = x2; x2 = x1; f2 = f1;
            x1 = hi - gr * (hi - lo);
            f1 = TSPIN(x1);
        }
    }
    double rc = 0.5 * (lo + hi);
    if (rho_c) *rho_c = rc;
    return TSPIN(rc);
#undef TSPIN
}

static double pr_tc(const orc_eos *e) { return eos_tc(e, NULL); }

/* Bisection for p(rho) = P on an interval where p is monotonic increasing. */
static double solve_p(const orc_eos *e, double A, double T, double P, double lo, double hi)
{
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (eos_pressure_A(e, A, T, mid) < P) lo = mid; else hi = mid;
        if (hi - lo <= 1e-17 * hi) break;
    }
    return 0.5 * (lo + hi);
}

/* Root of dp/drho on [lo, hi] where it changes sign. */
static double solve_dp(const orc_eos *e, double A, double T, double lo, double hi)
{
    double flo = eos_dpdrho_A(e, A, T, lo);
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        double fm = eos_dpdrho_A(e, A, T, mid);
        if ((fm > 0) == (flo > 0)) { lo = mid; flo = fm; } else hi = mid;
        if (hi - lo <= 1e-17 * hi) break;
    }
    return 0.5 * (lo + hi);
}

/* Maxwell construction for the coexisting densities at temperature T: the two
 * phases have equal pressure and equal chemical potential Psi' (the common
 * tangent of Psi stated below Eq. (4)).  For a trial pressure P between the
 * spinodal pressures, bisection gives the gas root and the liquid root of
 * p = P; the chemical-potential difference is monotonic in P and is bisected
 * to zero.  Then C = -Psi'_0(rho_g) (Psi'_0: Psi' with C = 0) so that
 * Psi'(rho_g) = Psi'(rho_l) = 0, and Psi0 = Psi(rho_g) = Psi(rho_l), which with
 * that C equals -p_coex.  Returns 0 on success, -1 if T >= T_c.
 * out = {rho_g, rho_l, C, Psi0}.                                            */
static int eos_maxwell(const orc_eos *e, double T, double *out)
{
    double rc;
    double Tc = eos_tc(e, &rc);
    if (!(T > 0.0) || !(T < Tc)) return -1;
    double A = eos_attraction(e, T);
    double rmax = eos_rho_max(e);
    /* spinodals: dp/drho > 0 below rho_s1, < 0 between, > 0 above rho_s2 (at
     * T < T_c the unstable branch brackets the critical density for CS and
     * vdW; for PR alpha(T) > 1 moves it, so search from the maximum of the
     * spinodal curve at this attraction) */
    double lo = 1e-6, hi = rmax * (1.0 - 1e-6);
    const double gr = 0.5 * (sqrt(5.0) - 1.0);
    double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
    double f1 = -eos_dpdrho_A(e, A, T, x1) / x1, f2 = -eos_dpdrho_A(e, A, T, x2) / x2;
    for (int it = 0; it < 300; ++it) {
        if (f1 < f2) { lo = x1; x1 = x2; f1 = f2; x2 = lo + gr * (hi - lo); f2 = -eos_dpdrho_A(e, A, T, x2) / x2; }
        else { hi = x2; x2 = x1; f2 = f1; x1 = hi - gr * (hi - lo); f1 = -eos_dpdrho_A(e, A, T, x1) / x1; }
    }
    double rm = 0.5 * (lo + hi);  /* most unstable density at this T */
    if (!(eos_dpdrho_A(e, A, T, rm) < 0.0)) return -1;
    (void)rc;
    double s1 = solve_dp(e, A, T, 1e-12, rm);
    double s2 = solve_dp(e, A, T, rm, rmax * (1.0 - 1e-12));
    double pmax = eos_pressure_A(e, A, T, s1);
    double pmin = eos_pressure_A(e, A, T, s2);
    double Plo = pmin > 0.0 ? pmin : 0.0, Phi = pmax;
    double rg = 0, rl = 0;
    for (int it = 0; it < 300; ++it) {
        double P = 0.5 * (Plo + Phi);
        rg = solve_p(e, A, T, P, 1e-300, s1);
        rl = solve_p(e, A, T, P, s2, rmax * (1.0 - 1e-15));
        double dmu = eos_psi_prime_A(e, A, T, 0.0, rl) - eos_psi_prime_A(e, A, T, 0.0, rg);
        /* along an isotherm d mu = dp / rho, so d(mu_l - mu_g)/dP =
         * 1/rho_l - 1/rho_g < 0: a positive difference means P is too low */
        if (dmu > 0) Plo = P; else Phi = P;
        if (Phi - Plo <= 1e-17 * Phi) break;
    }
    double C = -eos_psi_prime_A(e, A, T, 0.0, rg);
    out[0] = rg;
    out[1] = rl;
    out[2] = C;
    out[3] = eos_psi_A(e, A, T, C, rg);
    return 0;
}

/* Temperature at which the Maxwell ratio rho_l / rho_g equals `ratio`
 * (the ratio decreases monotonically as T rises to T_c).  Bisection in T.
 * out = {T, rho_g, rho_l, C, Psi0}.                                         */
static int eos_temperature_for_ratio(const orc_eos *e, double ratio, double *out)
{
    if (!(ratio > 1.0)) return -1;
    double Tc = eos_tc(e, NULL);
    double lo = 0.05 * Tc, hi = Tc * (1.0 - 1e-9);
    double m[4];
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (eos_maxwell(e, mid, m) != 0) { hi = mid; continue; }
        if (m[1] / m[0] > ratio) lo = mid; else hi = mid;
        if (hi - lo <= 1e-16 * hi) break;
    }
    out[0] = 0.5 * (lo + hi);
    if (eos_maxwell(e, out[0], m) != 0) return -1;
    out[1] = m[0]; out[2] = m[1]; out[3] = m[2]; out[4] = m[3];
    return 0;
}

/* Exported forms: orc_eos_* take (kind, a, b, R, omega); the unprefixed ones
 * are the Carnahan-Starling EOS of Eq. (4). */
static orc_eos make_eos(int kind, double a, double b, double R, double omega)
{
    orc_eos e = {kind, a, b, R, omega};
    return e;
}

double orc_eos_psi(int kind, double a, double b, double R, double omega, double T, double C, double rho)
{
    orc_eos e = make_eos(kind, a, b, R, omega);
    return eos_psi_A(&e, eos_attraction(&e, T), T, C, rho);
}
double orc_eos_psi_prime(int kind, double a, double b, double R, double omega, double T, double C, double rho)
{
    orc_eos e = make_eos(kind, a, b, R, omega);
    return eos_psi_prime_A(&e, eos_attraction(&e, T), T, C, rho);
}
double orc_eos_pressure(int kind, double a, double b, double R, double omega, double T, double rho)
{
    orc_eos e = make_eos(kind, a, b, R, omega);
    return eos_pressure_A(&e, eos_attraction(&e, T), T, rho);
}
double orc_eos_attraction(int kind, double a, double b, double R, double omega, double T)
{
    orc_eos e = make_eos(kind, a, b, R, omega);
    return eos_attraction(&e, T);
}
double orc_eos_critical_temperature(int kind, double a, double b, double R, double omega, double *rho_c)
{
    orc_eos e = make_eos(kind, a, b, R, omega);
    return eos_tc(&e, rho_c);
}
int orc_eos_maxwell(int kind, double a, double b, double R, double omega, double T, double *out)
{
    orc_eos e = make_eos(kind, a, b, R, omega);
    return eos_maxwell(&e, T, out);
}
int orc_eos_temperature_for_ratio(int kind, double a, double b, double R, double omega, double ratio, double *out)
{
    orc_eos e = make_eos(kind, a, b, R, omega);
    return eos_temperature_for_ratio(&e, ratio, out);
}

double orc_psi_eos(double a, double b, double R, double T, double C, double rho)
{
    return orc_eos_psi(0, a, b, R, 0.0, T, C, rho);
}
double orc_psi_prime(double a, double b, double R, double T, double C, double rho)
{
    return orc_eos_psi_prime(0, a, b, R, 0.0, T, C, rho);
}
double orc_pressure(double a, double b, double R, double T, double rho)
{
    return orc_eos_pressure(0, a, b, R, 0.0, T, rho);
}
double orc_dpdrho(double a, double b, double R, double T, double rho)
{
    orc_eos e = make_eos(0, a, b, R, 0.0);
    return eos_dpdrho_A(&e, a, T, rho);
}
double orc_critical_temperature(double a, double b, double R, double *rho_c)
{
    return orc_eos_critical_temperature(0, a, b, R, 0.0, rho_c);
}
int orc_maxwell(double a, double b, double R, double T, double *out)
{
    return orc_eos_maxwell(0, a, b, R, 0.0, T, out);
}
int orc_temperature_for_ratio(double a, double b, double R, double ratio, double *out)
{
    return orc_eos_temperature_for_ratio(0, a, b, R, 0.0, ratio, out);
}

/* ------------------------------------------------------------------------- */
/* Free energy: concentrations, bulk energy and chemical potentials.         */
/* ------------------------------------------------------------------------- */

/* Concentrations of the two liquids from (rho, phi), as defined in the text
 * below Fig. 1: C_l1 = [1 + phi/chi - (rho - rho_l)/(rho_g - rho_l)]/2 and
 * C_l2 = [1 - phi/chi - (rho - rho_l)/(rho_g - rho_l)]/2.                     */
void orc_concentrations(const orc_params *p, double rho, double phi, double *c1, double *c2)
{
    double cg = (rho - p->rho_l) / (p->rho_g - p->rho_l);
    *c1 = 0.5 * (1.0 + phi / p->chi - cg);
    *c2 = 0.5 * (1.0 - phi / p->chi - cg);
}

/* Coefficients of the interfacial energy rewritten in (rho, phi) (the f_I
 * expansion after Eq. (3)): f_I = A (grad rho)^2 + B (grad phi)^2
 * + D grad rho . grad phi.  out = {A, B, D}.                                 */
void orc_gradient_coefficients(const orc_params *p, double *out)
{
    double dlt = p->rho_g - p->rho_l;
    out[0] = 0.5 * p->kappa1 + (p->kappa2 + p->kappa3) / (8.0 * dlt * dlt);
    out[1] = (p->kappa2 + p->kappa3) / (8.0 * p->chi * p->chi);
    out[2] = (p->kappa3 - p->kappa2) / (4.0 * p->chi * dlt);
}

/* Half the derivative of the double well C^2 (1-C)^2 of Eq. (2). */
static double dwell_half(double c) { return c * (1.0 - c) * (1.0 - 2.0 * c); }

/* Bulk parts of mu_rho = dF/drho and mu_phi = dF/dphi (the definitions after
 * Eq. (7)), from Eq. (2) with the chain rule through C_l1, C_l2:
 *   mu_rho = (lambda1/2) Psi'(rho) - [lambda2 W(C1) + lambda3 W(C2)]/(2 (rho_g - rho_l))
 *   mu_phi = [lambda2 W(C1) - lambda3 W(C2)]/(2 chi)
 * with W(C) = C (1-C)(1-2C).  Reading: no clamping of the concentrations.   */
void orc_mu_bulk(const orc_params *p, double rho, double phi, double *out)
{
    double c1, c2;
    orc_concentrations(p, rho, phi, &c1, &c2);
    double w1v = dwell_half(c1), w2v = dwell_half(c2);
    double dlt = p->rho_g - p->rho_l;
    out[0] = 0.5 * p->lambda1 * orc_eos_psi_prime(p->eos, p->a, p->b, p->R, p->omega, p->T, p->C, rho)
             - (p->lambda2 * w1v + p->lambda3 * w2v) / (2.0 * dlt);
    out[1] = (p->lambda2 * w1v - p->lambda3 * w2v) / (2.0 * p->chi);
}

/* Bulk free-energy density f_B of Eq. (2):
 *   (lambda1/2)(Psi(rho) - Psi0) + (lambda2/2) C1^2 (1-C1)^2 + (lambda3/2) C2^2 (1-C2)^2
 * with Psi0 = Psi(rho_g) (Reading: the constant only shifts the energy).    */
double orc_f_bulk(const orc_params *p, double rho, double phi)
{
    double c1, c2;
    orc_concentrations(p, rho, phi, &c1, &c2);
    double psi = orc_eos_psi(p->eos, p->a, p->b, p->R, p->omega, p->T, p->C, rho);
    double psi0 = orc_eos_psi(p->eos, p->a, p->b, p->R, p->omega, p->T, p->C, p->rho_g);
    double d1 = c1 * (1.0 - c1), d2 = c2 * (1.0 - c2);
    return 0.5 * p->lambda1 * (psi - psi0) + 0.5 * p->lambda2 * d1 * d1 + 0.5 * p->lambda3 * d2 * d2;
}

/* Thermodynamic pressure of a uniform state, rho mu_rho + phi mu_phi - f_B
 * (the bulk part of the pressure tensor stated after Eq. (7)).              */
double orc_bulk_pressure(const orc_params *p, double rho, double phi)
{
    double mu[2];
    orc_mu_bulk(p, rho, phi, mu);
    return rho * mu[0] + phi * mu[1] - orc_f_bulk(p, rho, phi);
}

/* ------------------------------------------------------------------------- */
/* Lattice stencils (Reading: the isotropic stencils with the lattice        */
/* weights; the paper does not state its discretisation).                    */
/*   laplacian psi(x) = (2/cs2) sum_i w_i [psi(x + c_i) - psi(x)]            */
/*   d_alpha psi(x)   = (1/cs2) sum_i w_i c_i,alpha psi(x + c_i)             */
/* ------------------------------------------------------------------------- */

static int64_t node_index(const orc_params *p, int64_t x, int64_t y, int64_t z)
{
    return (z * p->ny + y) * p->nx + x;
}

static int64_t wrap(int64_t v, int64_t n) { v %= n; return v < 0 ? v + n : v; }

static int64_t neighbour(const orc_params *p, int64_t node, const int c[3])
{
    int64_t x = node % p->nx;
    int64_t y = (node / p->nx) % p->ny;
    int64_t z = node / ((int64_t)p->nx * p->ny);
    return node_index(p, wrap(x + c[0], p->nx), wrap(y + c[1], p->ny), wrap(z + c[2], p->nz));
}

static int64_t num_nodes(const orc_params *p) { return (int64_t)p->nx * p->ny * p->nz; }

/* ------------------------------------------------------------------------- */
/* Solid walls (the wetting boundary conditions the paper's outlook names;    */
/* of the approaches it cites, the geometric one).  With walls set, the       */
/* planes y = -1/2 and y = ny - 1/2 are flat solids and the box stays         */
/* periodic in x (and z).  Reading:                                          */
/*  - populations that would stream into a wall return to their node with    */
/*    the opposite velocity (halfway bounce-back), for f and g alike: no     */
/*    slip, no flux of mass or phase field through the wall;                 */
/*  - the stencils see one ghost row beyond each wall.  For rho and phi it   */
/*    holds the geometric wetting condition n.grad psi = -cot(theta)         */
/*    |grad_t psi| (theta measured in the phase where psi is large, n the     */
/*    normal into the fluid), discretised across the wall as                  */
/*      psi(ghost) = psi(wall row) + cot(theta) |grad_t psi(wall row)|        */
/*    with central differences along the wall; for the chemical potentials   */
/*    the ghost repeats the wall row (zero normal gradient, no diffusive     */
/*    flux).  theta = pi/2 makes every ghost a mirror.                        */
/* ------------------------------------------------------------------------- */

enum { GHOST_MIRROR = 0, GHOST_WET_RHO = 1, GHOST_WET_PHI = 2 };

/* psi at node n + c, with the ghost rule `mode` where n + c lies beyond a wall. */
static double stencil_at(const orc_params *p, const double *psi, int64_t n, const int c[3], int mode)
{
    int64_t x = n % p->nx, y = (n / p->nx) % p->ny, z = n / ((int64_t)p->nx * p->ny);
    int64_t yy = y + c[1];
    if (!p->walls || (yy >= 0 && yy < p->ny)) return psi[neighbour(p, n, c)];
    int top = yy >= p->ny;
    int64_t yw = top ? p->ny - 1 : 0;
    int64_t xx = wrap(x + c[0], p->nx), zz = wrap(z + c[2], p->nz);
    double v = psi[node_index(p, xx, yw, zz)];
    if (mode == GHOST_MIRROR) return v;
    double th = mode == GHOST_WET_RHO ? (top ? p->theta_rho_hi : p->theta_rho_lo)
                                      : (top ? p->theta_phi_hi : p->theta_phi_lo);
    double tx = 0.5 * (psi[node_index(p, wrap(xx + 1, p->nx), yw, zz)] - psi[node_index(p, wrap(xx - 1, p->nx), yw, zz)]);
    double tz = 0.0;
    if (p->lattice == 1)
        tz = 0.5 * (psi[node_index(p, xx, yw, wrap(zz + 1, p->nz))] - psi[node_index(p, xx, yw, wrap(zz - 1, p->nz))]);
    return v + cos(th) / sin(th) * sqrt(tx * tx + tz * tz);
}

static void laplacian_mode(const orc_params *p, const double *psi, double *out, int mode)
{
    int Q = lattice_Q(p->lattice);
    int64_t N = num_nodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) {
            int c[3];
            direction(i, c);
            s += weight_lat(p->lattice, i) * (stencil_at(p, psi, n, c, mode) - psi[n]);
        }
        out[n] = (2.0 / CS2) * s;
    }
}

/* out is [3][N]; component z stays 0 on D2Q9. */
static void gradient_mode(const orc_params *p, const double *psi, double *out, int mode)
{
    int Q = lattice_Q(p->lattice);
    int64_t N = num_nodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double s[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            int c[3];
            direction(i, c);
            double v = weight_lat(p->lattice, i) * stencil_at(p, psi, n, c, mode);
            s[0] += v * c[0];
            s[1] += v * c[1];
            s[2] += v * c[2];
        }
        out[n] = s[0] / CS2;
        out[N + n] = s[1] / CS2;
        out[2 * N + n] = s[2] / CS2;
    }
}

/* The lattice operators on a periodic box (walls, if set, act as mirrors). */
void orc_laplacian(const orc_params *p, const double *psi, double *out)
{
    laplacian_mode(p, psi, out, GHOST_MIRROR);
}

void orc_gradient(const orc_params *p, const double *psi, double *out)
{
    gradient_mode(p, psi, out, GHOST_MIRROR);
}

/* ------------------------------------------------------------------------- */
/* Equilibria.                                                               */
/* ------------------------------------------------------------------------- */

/* Reading: the entropic equilibrium of the entropic LBM the paper adopts, in
 * its product form f_i = rho prod_alpha Psi_{c_i,alpha}(u_alpha) over the
 * D1Q3 factors (S = sqrt(1 + 3 u^2)):
 *   Psi_0 = (2/3)(2 - S), Psi_+ = (1/6)(2 - S)(2u + S)/(1 - u),
 *   Psi_- = (1/6)(2 - S)(1 - u)/(2u + S).
 * Defined for |u_alpha| < 1.                                                */
static void d1q3_factors(double u, double psi[3])
{
    double S = sqrt(1.0 + 3.0 * u * u);
    psi[0] = (2.0 / 3.0) * (2.0 - S);
    psi[1] = (1.0 / 6.0) * (2.0 - S) * (2.0 * u + S) / (1.0 - u);
    psi[2] = (1.0 / 6.0) * (2.0 - S) * (1.0 - u) / (2.0 * u + S);
}

void orc_feq(int lattice, double rho, const double *u, double *feq)
{
    int Q = lattice_Q(lattice);
    double px[3], py[3], pz[3];
    d1q3_factors(u[0], px);
    d1q3_factors(u[1], py);
    if (lattice == 1) d1q3_factors(u[2], pz);
    for (int i = 0; i < Q; ++i) {
        int kx = i % 3, ky = (i / 3) % 3, kz = i / 9;
        double v = rho * px[kx] * py[ky];
        if (lattice == 1) v *= pz[kz];
        feq[i] = v;
    }
}

/* Phase-field equilibrium of the standard free-energy BGK scheme for the
 * Cahn-Hilliard equation (7):
 *   geq_i = w_i [Gamma mu_phi / cs2 + phi c_i.u / cs2 + phi (c_i.u)^2/(2 cs2^2)
 *                - phi u^2 / (2 cs2)]      (i != 0)
 *   geq_0 = phi - sum_{i != 0} geq_i.
 * Reading: u is the physical (half-force corrected) velocity.               */
void orc_geq(int lattice, double phi, double mu_phi, double Gamma, const double *u, double *geq)
{
    int Q = lattice_Q(lattice);
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double rest = 0.0;
    for (int i = 1; i < Q; ++i) {
        int c[3];
        direction(i, c);
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        geq[i] = weight_lat(lattice, i) * (Gamma * mu_phi / CS2 + phi * cu / CS2
                                          + phi * cu * cu / (2.0 * CS2 * CS2)
                                          - phi * uu / (2.0 * CS2));
        rest += geq[i];
    }
    geq[0] = phi - rest;
}

/* Reduced phase-field lattice (the paper leaves the lattice of g open): the
 * rest and axis directions of D2Q9 / D3Q27 (D2Q5 / D3Q7), axis weights 1/6
 * so that sum_i w_i c_i c_i = cs2 I as on the full lattice, and the
 * equilibrium to first order in u (a five- or seven-velocity set cannot
 * carry the second-order terms isotropically):
 *   geq_i = w_i [Gamma mu_phi / cs2 + phi c_i.u / cs2] (axis directions),
 *   geq_0 = phi - sum of those, and 0 on the other directions.
 * Its first two moments equal those of the full equilibrium (phi, phi u,
 * Gamma mu_phi I + phi u u without the u u term), so Eq. (7) is recovered
 * with the same mobility M = Gamma (tau_phi - 1/2).                         */
static int axis_direction(int i)
{
    int c[3];
    direction(i, c);
    return abs(c[0]) + abs(c[1]) + abs(c[2]) == 1;
}

void orc_geq_reduced(int lattice, double phi, double mu_phi, double Gamma, const double *u, double *geq)
{
    int Q = lattice_Q(lattice);
    double rest = 0.0;
    for (int i = 1; i < Q; ++i) {
        geq[i] = 0.0;
        if (!axis_direction(i)) continue;
        int c[3];
        direction(i, c);
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        geq[i] = (1.0 / 6.0) * (Gamma * mu_phi / CS2 + phi * cu / CS2);
        rest += geq[i];
    }
    geq[0] = phi - rest;
}

static void geq_of(const orc_params *p, double phi, double mu_phi, double Gamma, const double *u, double *geq)
{
    if (p->glattice) orc_geq_reduced(p->lattice, phi, mu_phi, Gamma, u, geq);
    else orc_geq(p->lattice, phi, mu_phi, Gamma, u, geq);
}

/* ------------------------------------------------------------------------- */
/* KBC entropic collision.                                                   */
/* ------------------------------------------------------------------------- */

/* Dual basis of the D1Q3 raw moments: for populations over c = (0,+1,-1),
 * f(c) = sum_k M_k b_k(c) with M_k = sum_c f(c) c^k, where
 * b_0 = (1, 0, 0), b_1 = (0, 1/2, -1/2) and b_2 = (-1, 1/2, 1/2) on
 * c = (0, +1, -1); sum_c b_k(c) c^m = [k == m] for k, m in {0, 1, 2}.  The
 * D2Q9 / D3Q27 basis is the tensor product over the axes.                  */
static double b0(int c) { return c == 0 ? 1.0 : 0.0; }
static double b1(int c) { return 0.5 * c; }
static double b2(int c) { return c == 0 ? -1.0 : 0.5; }

/* Split the non-equilibrium part df = f - feq into the shear part ds, which
 * carries exactly the deviatoric second-order moments of df, and the rest
 * dh = df - ds.  Reading: the shear subspace s of the KBC scheme is spanned by
 * the traceless second moments (normal-stress differences and off-diagonal
 * stresses); the trace and all higher moments belong to h.                  */
void orc_kbc_split(int lattice, const double *df, double *ds, double *dh)
{
    int Q = lattice_Q(lattice);
    int D = lattice_D(lattice);
    double M[3][3] = {{0}};
    for (int i = 0; i < Q; ++i) {
        int c[3];
        direction(i, c);
        for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb) M[a][bb] += df[i] * c[a] * c[bb];
    }
    double tr = 0.0;
    for (int a = 0; a < D; ++a) tr += M[a][a];
    double dev[3];
    for (int a = 0; a < D; ++a) dev[a] = M[a][a] - tr / D;
    for (int i = 0; i < Q; ++i) {
        int c[3];
        direction(i, c);
        double s;
        if (D == 2) {
            s = dev[0] * b2(c[0]) * b0(c[1])
              + dev[1] * b0(c[0]) * b2(c[1])
              + M[0][1] * b1(c[0]) * b1(c[1]);
        } else {
            s = dev[0] * b2(c[0]) * b0(c[1]) * b0(c[2])
              + dev[1] * b0(c[0]) * b2(c[1]) * b0(c[2])
              + dev[2] * b0(c[0]) * b0(c[1]) * b2(c[2])
              + M[0][1] * b1(c[0]) * b1(c[1]) * b0(c[2])
              + M[0][2] * b1(c[0]) * b0(c[1]) * b1(c[2])
              + M[1][2] * b0(c[0]) * b1(c[1]) * b1(c[2]);
        }
        ds[i] = s;
        dh[i] = df[i] - s;
    }
}

/* Stabiliser gamma of the KBC collision f* = f - beta (2 ds + gamma dh):
 * the minimiser of the quadratic entropy estimate of the post-collision
 * state, gamma = 1/beta - (2 - 1/beta) <ds|dh>/<dh|dh> with the entropic
 * scalar product <X|Y> = sum_i X_i Y_i / feq_i.  Reading: gamma = 2 (the
 * LBGK value) when <dh|dh> vanishes.                                        */
double orc_kbc_gamma(int lattice, double beta, const double *feq, const double *ds, const double *dh)
{
    int Q = lattice_Q(lattice);
    double sh = 0.0, hh = 0.0;
    for (int i = 0; i < Q; ++i) {
        sh += ds[i] * dh[i] / feq[i];
        hh += dh[i] * dh[i] / feq[i];
    }
    if (!(hh > 1e-300)) return 2.0;
    return 1.0 / beta - (2.0 - 1.0 / beta) * sh / hh;
}

/* One node: KBC collision of f about feq(rho, u = j/rho), then the
 * exact-difference forcing term feq(rho, u + F/rho) - feq(rho, u).
 * fstar and gamma are outputs.                                              */
void orc_collide_node(int lattice, double beta, const double *f, const double *force,
                      double *fstar, double *gamma_out)
{
    int Q = lattice_Q(lattice);
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        int c[3];
        direction(i, c);
        rho += f[i];
        j[0] += f[i] * c[0];
        j[1] += f[i] * c[1];
        j[2] += f[i] * c[2];
    }
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    double du[3] = {force[0] / rho, force[1] / rho, force[2] / rho};
    if (lattice == 0) { u[2] = 0.0; du[2] = 0.0; }
    double feq[27], feq2[27], df[27], ds[27], dh[27];
    orc_feq(lattice, rho, u, feq);
    for (int i = 0; i < Q; ++i) df[i] = f[i] - feq[i];
    orc_kbc_split(lattice, df, ds, dh);
    double gamma = orc_kbc_gamma(lattice, beta, feq, ds, dh);
    double u2[3] = {u[0] + du[0], u[1] + du[1], u[2] + du[2]};
    orc_feq(lattice, rho, u2, feq2);
    for (int i = 0; i < Q; ++i)
        fstar[i] = f[i] - beta * (2.0 * ds[i] + gamma * dh[i]) + (feq2[i] - feq[i]);
    if (gamma_out) *gamma_out = gamma;
}

/* ------------------------------------------------------------------------- */
/* Whole-lattice fields and the time step.                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    double *rho, *phi, *j, *lap_rho, *lap_phi, *mu_rho, *mu_phi;
    double *grad_rho, *grad_mu_phi, *force;
} orc_work;

static int work_alloc(orc_work *w, int64_t N)
{
    memset(w, 0, sizeof(*w));
    w->rho = calloc(N, sizeof(double));
    w->phi = calloc(N, sizeof(double));
    w->j = calloc(3 * N, sizeof(double));
    w->lap_rho = calloc(N, sizeof(double));
    w->lap_phi = calloc(N, sizeof(double));
    w->mu_rho = calloc(N, sizeof(double));
    w->mu_phi = calloc(N, sizeof(double));
    w->grad_rho = calloc(3 * N, sizeof(double));
    w->grad_mu_phi = calloc(3 * N, sizeof(double));
    w->force = calloc(3 * N, sizeof(double));
    return (w->rho && w->phi && w->j && w->lap_rho && w->lap_phi && w->mu_rho && w->mu_phi
            && w->grad_rho && w->grad_mu_phi && w->force) ? 0 : -1;
}

static void work_free(orc_work *w)
{
    free(w->rho); free(w->phi); free(w->j); free(w->lap_rho); free(w->lap_phi);
    free(w->mu_rho); free(w->mu_phi); free(w->grad_rho);
    free(w->grad_mu_phi); free(w->force);
}

/* Chemical potentials with their gradient parts (from the f_I rewrite):
 *   mu_rho = bulk - 2 A lap(rho) - D lap(phi)
 *   mu_phi = bulk - 2 B lap(phi) - D lap(rho).                              */
static void chemical_potentials(const orc_params *p, orc_work *w)
{
    int64_t N = num_nodes(p);
    double abd[3];
    orc_gradient_coefficients(p, abd);
    laplacian_mode(p, w->rho, w->lap_rho, GHOST_WET_RHO);
    laplacian_mode(p, w->phi, w->lap_phi, GHOST_WET_PHI);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double mb[2];
        orc_mu_bulk(p, w->rho[n], w->phi[n], mb);
        w->mu_rho[n] = mb[0] - 2.0 * abd[0] * w->lap_rho[n] - abd[2] * w->lap_phi[n];
        w->mu_phi[n] = mb[1] - 2.0 * abd[1] * w->lap_phi[n] - abd[2] * w->lap_rho[n];
    }
}

/* Thermodynamic force on the fluid.  The pressure tensor enters through
 * div P = rho grad mu_rho + phi grad mu_phi (stated after Eq. (7)).  The
 * lattice already carries the ideal pressure cs2 rho, whose chemical
 * potential is cs2 ln rho, so the force added is
 *   F = cs2 grad rho - div P = -rho grad(mu_rho - cs2 ln rho) - phi grad mu_phi.
 * Reading: the gradient is taken of the excess potential mu_rho - cs2 ln rho
 * (the form that stays bounded per unit mass where the gas is thin); the
 * split cs2 grad rho - rho grad mu_rho is identical in the continuum.
 * grad_rho holds the excess potential's gradient.                           */
static void thermodynamic_force(const orc_params *p, orc_work *w)
{
    int64_t N = num_nodes(p);
    double *excess = w->lap_rho;   /* reuse: the Laplacian is no longer needed */
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) excess[n] = w->mu_rho[n] - CS2 * log(w->rho[n]);
    gradient_mode(p, excess, w->grad_rho, GHOST_MIRROR);
    gradient_mode(p, w->mu_phi, w->grad_mu_phi, GHOST_MIRROR);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n)
        for (int a = 0; a < 3; ++a)
            w->force[a * N + n] = -w->rho[n] * w->grad_rho[a * N + n]
                                  - w->phi[n] * w->grad_mu_phi[a * N + n];
}

/* Zeroth and first moments of the (post-streaming) populations. */
static void moments(const orc_params *p, const double *f, const double *g, orc_work *w)
{
    int Q = lattice_Q(p->lattice);
    int64_t N = num_nodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double r = 0.0, ph = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < Q; ++i) {
            int c[3];
            direction(i, c);
            double fi = f[(int64_t)i * N + n];
            r += fi;
            jx += fi * c[0];
            jy += fi * c[1];
            jz += fi * c[2];
            ph += g[(int64_t)i * N + n];
        }
        w->rho[n] = r;
        w->phi[n] = ph;
        w->j[n] = jx;
        w->j[N + n] = jy;
        w->j[2 * N + n] = jz;
    }
}

/* Derived constants: tau = 3 nu + 1/2 (so nu = cs2 (tau - 1/2)),
 * beta = 1/(2 tau), and Gamma = M / (tau_phi - 1/2) so that the phase-field
 * BGK recovers the mobility M of Eq. (7).                                    */
static double beta_of(const orc_params *p) { return 1.0 / (2.0 * (3.0 * p->nu + 0.5)); }
static double gamma_cap_of(const orc_params *p) { return p->mobility / (p->tau_phi - 0.5); }

/* Initial populations.  Reading: f = feq(rho0, u0) and
 * g = geq(phi0, mu_phi(rho0, phi0), u0).  u0 may be NULL (zero velocity).   */
int orc_init(const orc_params *p, const double *rho0, const double *phi0, const double *u0,
             double *f, double *g)
{
    int Q = lattice_Q(p->lattice);
    int64_t N = num_nodes(p);
    orc_work w;
    if (work_alloc(&w, N)) { work_free(&w); return -1; }
    memcpy(w.rho, rho0, N * sizeof(double));
    memcpy(w.phi, phi0, N * sizeof(double));
    chemical_potentials(p, &w);
    double Gam = gamma_cap_of(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double u[3] = {0, 0, 0}, fe[27], ge[27];
        if (u0) { u[0] = u0[n]; u[1] = u0[N + n]; if (p->lattice == 1) u[2] = u0[2 * N + n]; }
        orc_feq(p->lattice, rho0[n], u, fe);
        geq_of(p, phi0[n], w.mu_phi[n], Gam, u, ge);
        for (int i = 0; i < Q; ++i) {
            f[(int64_t)i * N + n] = fe[i];
            g[(int64_t)i * N + n] = ge[i];
        }
    }
    work_free(&w);
    return 0;
}

/* Advance the post-streaming populations f, g (layout [Q][N]) by nsteps time
 * steps.  If diag is not NULL it receives, per step, the totals before the
 * step {sum rho, sum phi, sum j (3), sum F (3)} and the collision's
 * {min gamma, max gamma}: 10 doubles per step.                               */
int orc_run(const orc_params *p, double *f, double *g, int64_t nsteps, double *diag)
{
    int Q = lattice_Q(p->lattice);
    int64_t N = num_nodes(p);
    orc_work w;
    double *fs = malloc((size_t)Q * N * sizeof(double));
    double *gs = malloc((size_t)Q * N * sizeof(double));
    double *gam = malloc((size_t)N * sizeof(double));
    if (work_alloc(&w, N) || !fs || !gs || !gam) {
        work_free(&w); free(fs); free(gs); free(gam);
        return -1;
    }
    const double beta = beta_of(p);
    const double Gam = gamma_cap_of(p);
    const double tau_phi = p->tau_phi;

    for (int64_t step = 0; step < nsteps; ++step) {
        /* 1. rho, j, phi of the post-streaming populations */
        moments(p, f, g, &w);
        /* 2-3. Laplacians and chemical potentials */
        chemical_potentials(p, &w);
        /* 4. gradients and the thermodynamic force */
        thermodynamic_force(p, &w);
        /* 5-9. collisions, node by node */
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            double fn[27], gn[27], fo[27], ge[27], F[3], up[3];
            for (int i = 0; i < Q; ++i) {
                fn[i] = f[(int64_t)i * N + n];
                gn[i] = g[(int64_t)i * N + n];
            }
            F[0] = w.force[n]; F[1] = w.force[N + n]; F[2] = w.force[2 * N + n];
            if (p->lattice == 0) F[2] = 0.0;
            orc_collide_node(p->lattice, beta, fn, F, fo, &gam[n]);
            double r = w.rho[n];
            for (int a = 0; a < 3; ++a) up[a] = (w.j[a * N + n] + 0.5 * F[a]) / r;
            if (p->lattice == 0) up[2] = 0.0;
            geq_of(p, w.phi[n], w.mu_phi[n], Gam, up, ge);
            for (int i = 0; i < Q; ++i) {
                fs[(int64_t)i * N + n] = fo[i];
                gs[(int64_t)i * N + n] = gn[i] - (gn[i] - ge[i]) / tau_phi;
            }
        }
        if (diag) {
            double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, INFINITY, -INFINITY};
            for (int64_t n = 0; n < N; ++n) {
                s[0] += w.rho[n];
                s[1] += w.phi[n];
                for (int a = 0; a < 3; ++a) {
                    s[2 + a] += w.j[a * N + n];
                    s[5 + a] += w.force[a * N + n];
                }
                if (gam[n] < s[8]) s[8] = gam[n];
                if (gam[n] > s[9]) s[9] = gam[n];
            }
            memcpy(diag + 10 * step, s, sizeof(s));
        }
        /* 10. streaming: f(x + c_i, t + 1) = f*(x, t); into a wall: bounce-back,
         * f_{-i}(x, t + 1) = f*_i(x, t) */
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            int64_t y = (n / p->nx) % p->ny;
            for (int i = 0; i < Q; ++i) {
                int c[3];
                direction(i, c);
                int64_t m = n, j = i;
                if (p->walls && (y + c[1] < 0 || y + c[1] >= p->ny)) j = opposite(i);
                else m = neighbour(p, n, c);
                f[j * N + m] = fs[(int64_t)i * N + n];
                g[j * N + m] = gs[(int64_t)i * N + n];
            }
        }
    }
    work_free(&w);
    free(fs); free(gs); free(gam);
    return 0;
}

/* Macroscopic fields of the state held in f, g (post-streaming).  Any output
 * pointer may be NULL.  u is the physical velocity u + F/(2 rho) ([3][N]).   */
int orc_fields(const orc_params *p, const double *f, const double *g,
               double *rho, double *phi, double *u, double *c1, double *c2,
               double *mu_rho, double *mu_phi, double *force)
{
    int64_t N = num_nodes(p);
    orc_work w;
    if (work_alloc(&w, N)) { work_free(&w); return -1; }
    moments(p, f, g, &w);
    chemical_potentials(p, &w);
    thermodynamic_force(p, &w);
    for (int64_t n = 0; n < N; ++n) {
        if (rho) rho[n] = w.rho[n];
        if (phi) phi[n] = w.phi[n];
        if (mu_rho) mu_rho[n] = w.mu_rho[n];
        if (mu_phi) mu_phi[n] = w.mu_phi[n];
        if (c1 || c2) {
            double a1, a2;
            orc_concentrations(p, w.rho[n], w.phi[n], &a1, &a2);
            if (c1) c1[n] = a1;
            if (c2) c2[n] = a2;
        }
        for (int a = 0; a < 3; ++a) {
            double F = (p->lattice == 0 && a == 2) ? 0.0 : w.force[a * N + n];
            if (u) u[a * N + n] = (p->lattice == 0 && a == 2) ? 0.0 : (w.j[a * N + n] + 0.5 * F) / w.rho[n];
            if (force) force[a * N + n] = F;
        }
    }
    work_free(&w);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* More liquid components (the extension named in the paper's concluding     */
/* paragraph: one more double well in f_B and one more gradient term in f_I   */
/* per added liquid).  Here: three liquids and the gas, with a second phase   */
/* field psi.  Reading (the paper gives no equations for it):                 */
/*  - concentrations, with C_L = 1 - C_g the liquid fraction of the text      */
/*    below Fig. 1:                                                          */
/*      C1 = (C_L + phi/chi - psi/chi)/2, C2 = (C_L - phi/chi - psi/chi)/2,  */
/*      C3 = psi/chi,                                                        */
/*    so psi = 0 gives back the two-liquid definitions exactly; the pure     */
/*    phases sit at (rho_g,0,0), (rho_l,chi,0), (rho_l,-chi,0), (rho_l,0,chi); */
/*  - free energy: Eq. (2) plus (lambda4/2) C3^2 (1-C3)^2, Eq. (3) plus       */
/*    (kappa4/2) |grad C3|^2.  With nu_m = lambda_{m+1} W(C_m)                */
/*    - kappa_{m+1} lap C_m (W as in the bulk potentials above) the          */
/*    potentials are the chain rule through C_m:                             */
/*      mu_rho = (lambda1/2) Psi' - kappa1 lap rho - (nu1 + nu2)/(2 (rho_g - rho_l)) */
/*      mu_phi = (nu1 - nu2)/(2 chi),  mu_psi = (2 nu3 - nu1 - nu2)/(2 chi);  */
/*  - force: -rho grad(mu_rho - cs2 ln rho) - phi grad mu_phi - psi grad mu_psi */
/*    (div P with one more order parameter);                                  */
/*  - Cahn-Hilliard equations for phi and psi with a constant 2 x 2 mobility  */
/*    matrix Mt: d_t phi + div(phi u) = lap(Mt_pp mu_phi + Mt_ps mu_psi), and  */
/*    the same for psi.  Mt is the image in (phi, psi) of the concentration   */
/*    mobility of consistent N-phase Cahn-Hilliard models (Boyer & Lapuerta), */
/*      M_C = (M / chi^2) (diag(w) - w w^T / W) / (w1 + w2),                  */
/*      w = (1/kappa2, 1/kappa3, 1/kappa4), W = w1 + w2 + w3,                 */
/*    Mt = A+ M_C A+^T with A+ the pseudo-inverse of d(C1,C2,C3)/d(phi,psi)   */
/*    (rows chi (1,-1,0) and (chi/3)(-1,-1,2)).  At an interface between two  */
/*    liquids with the third absent, M_C sends the absent one's chemical      */
/*    potential combination to zero when lambda_m / kappa_m is the same for   */
/*    every liquid, so an absent liquid does not appear there.  The scale     */
/*    1/(w1 + w2) makes Mt_pp = M and Mt_ps = 0 when kappa2 = kappa3: phi    */
/*    then moves exactly as in the two-liquid model (Mt = M diag(1, 1/3) for */
/*    equal kappas).  mobility_form 1 takes Mt = M I instead (one mobility    */
/*    per order parameter), which is not consistent; it is kept to show that. */
/*  - lattice Boltzmann form: a second set of phase-field populations h for   */
/*    psi with the BGK of g (same tau_phi, same equilibrium with            */
/*    Gamma mu_psi~); the equilibria take the mixed potentials                */
/*    mu_phi~ = (Mt_pp mu_phi + Mt_ps mu_psi)/M and mu_psi~ likewise.         */
/* Periodic boxes on the full phase-field lattice only.                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    double lambda4, kappa4;   /* double well and gradient coefficient of liquid 3 */
    int32_t mobility_form;    /* 0: consistent mobility matrix; 1: M per order parameter */
    int32_t pad;
} orc_nl;

void orc_nl_concentrations(const orc_params *p, double rho, double phi, double psi, double *c)
{
    double cl = 1.0 - (rho - p->rho_l) / (p->rho_g - p->rho_l);
    c[0] = 0.5 * (cl + phi / p->chi - psi / p->chi);
    c[1] = 0.5 * (cl - phi / p->chi - psi / p->chi);
    c[2] = psi / p->chi;
}

/* Mt / M as {pp, ps, sp, ss}; -1 if a kappa is not positive. */
int orc_nl_mobility(const orc_params *p, const orc_nl *nl, double *m)
{
    if (nl->mobility_form == 1) {
        m[0] = 1.0; m[1] = 0.0; m[2] = 0.0; m[3] = 1.0;
        return 0;
    }
    double s[3] = {p->kappa2, p->kappa3, nl->kappa4};
    if (!(s[0] > 0.0 && s[1] > 0.0 && s[2] > 0.0)) return -1;
    double w[3] = {1.0 / s[0], 1.0 / s[1], 1.0 / s[2]};
    double W = w[0] + w[1] + w[2];
    double K[3][3];   /* M_C chi^2 (w1 + w2) / M */
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K[i][j] = (i == j ? w[i] : 0.0) - w[i] * w[j] / W;
    /* rows of A+ divided by chi; the chi^2 of A+ M_C A+^T cancels M_C's */
    double a[2][3] = {{1.0, -1.0, 0.0}, {-1.0 / 3.0, -1.0 / 3.0, 2.0 / 3.0}};
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
            double v = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) v += a[x][i] * K[i][j] * a[y][j];
            m[2 * x + y] = v / (w[0] + w[1]);
        }
    return 0;
}

/* Bulk parts of (mu_rho, mu_phi, mu_psi): the formulas above without the
 * Laplacian terms. */
void orc_nl_mu_bulk(const orc_params *p, const orc_nl *nl, double rho, double phi, double psi, double *out)
{
    double c[3];
    orc_nl_concentrations(p, rho, phi, psi, c);
    double lam[3] = {p->lambda2, p->lambda3, nl->lambda4};
    double nu[3];
    for (int m = 0; m < 3; ++m) nu[m] = lam[m] * dwell_half(c[m]);
    out[0] = 0.5 * p->lambda1 * orc_eos_psi_prime(p->eos, p->a, p->b, p->R, p->omega, p->T, p->C, rho)
             - (nu[0] + nu[1]) / (2.0 * (p->rho_g - p->rho_l));
    out[1] = (nu[0] - nu[1]) / (2.0 * p->chi);
    out[2] = (2.0 * nu[2] - nu[0] - nu[1]) / (2.0 * p->chi);
}

/* Bulk free-energy density: Eq. (2) plus the third liquid's double well. */
double orc_nl_f_bulk(const orc_params *p, const orc_nl *nl, double rho, double phi, double psi)
{
    double c[3];
    orc_nl_concentrations(p, rho, phi, psi, c);
    double psi_e = orc_eos_psi(p->eos, p->a, p->b, p->R, p->omega, p->T, p->C, rho);
    double psi0 = orc_eos_psi(p->eos, p->a, p->b, p->R, p->omega, p->T, p->C, p->rho_g);
    double lam[3] = {p->lambda2, p->lambda3, nl->lambda4};
    double f = 0.5 * p->lambda1 * (psi_e - psi0);
    for (int m = 0; m < 3; ++m) {
        double d = c[m] * (1.0 - c[m]);
        f += 0.5 * lam[m] * d * d;
    }
    return f;
}

typedef struct {
    orc_work w;               /* rho, phi, j, mu_rho, mu_phi, force, ... */
    double *psi, *lap_psi, *mu_psi, *grad_mu_psi;
} orc_nl_work;

static int nl_work_alloc(orc_nl_work *v, int64_t N)
{
    int rc = work_alloc(&v->w, N);
    v->psi = calloc(N, sizeof(double));
    v->lap_psi = calloc(N, sizeof(double));
    v->mu_psi = calloc(N, sizeof(double));
    v->grad_mu_psi = calloc(3 * N, sizeof(double));
    return (rc || !v->psi || !v->lap_psi || !v->mu_psi || !v->grad_mu_psi) ? -1 : 0;
}

static void nl_work_free(orc_nl_work *v)
{
    work_free(&v->w);
    free(v->psi); free(v->lap_psi); free(v->mu_psi); free(v->grad_mu_psi);
}

static void nl_chemical_potentials(const orc_params *p, const orc_nl *nl, orc_nl_work *v)
{
    int64_t N = num_nodes(p);
    orc_work *w = &v->w;
    laplacian_mode(p, w->rho, w->lap_rho, GHOST_MIRROR);
    laplacian_mode(p, w->phi, w->lap_phi, GHOST_MIRROR);
    laplacian_mode(p, v->psi, v->lap_psi, GHOST_MIRROR);
    double lam[3] = {p->lambda2, p->lambda3, nl->lambda4};
    double kap[3] = {p->kappa2, p->kappa3, nl->kappa4};
    double dlt = p->rho_g - p->rho_l, chi = p->chi;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double c[3], lc[3], nu[3];
        orc_nl_concentrations(p, w->rho[n], w->phi[n], v->psi[n], c);
        double lcl = -w->lap_rho[n] / dlt;   /* lap C_L */
        lc[0] = 0.5 * (lcl + w->lap_phi[n] / chi - v->lap_psi[n] / chi);
        lc[1] = 0.5 * (lcl - w->lap_phi[n] / chi - v->lap_psi[n] / chi);
        lc[2] = v->lap_psi[n] / chi;
        for (int m = 0; m < 3; ++m) nu[m] = lam[m] * dwell_half(c[m]) - kap[m] * lc[m];
        w->mu_rho[n] = 0.5 * p->lambda1
                           * orc_eos_psi_prime(p->eos, p->a, p->b, p->R, p->omega, p->T, p->C, w->rho[n])
                       - p->kappa1 * w->lap_rho[n] - (nu[0] + nu[1]) / (2.0 * dlt);
        w->mu_phi[n] = (nu[0] - nu[1]) / (2.0 * chi);
        v->mu_psi[n] = (2.0 * nu[2] - nu[0] - nu[1]) / (2.0 * chi);
    }
}

static void nl_force(const orc_params *p, orc_nl_work *v)
{
    int64_t N = num_nodes(p);
    orc_work *w = &v->w;
    double *excess = w->lap_rho;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) excess[n] = w->mu_rho[n] - CS2 * log(w->rho[n]);
    gradient_mode(p, excess, w->grad_rho, GHOST_MIRROR);
    gradient_mode(p, w->mu_phi, w->grad_mu_phi, GHOST_MIRROR);
    gradient_mode(p, v->mu_psi, v->grad_mu_psi, GHOST_MIRROR);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n)
        for (int a = 0; a < 3; ++a)
            w->force[a * N + n] = -w->rho[n] * w->grad_rho[a * N + n] - w->phi[n] * w->grad_mu_phi[a * N + n]
                                  - v->psi[n] * v->grad_mu_psi[a * N + n];
}

static void nl_moments(const orc_params *p, const double *f, const double *g, const double *h, orc_nl_work *v)
{
    int Q = lattice_Q(p->lattice);
    int64_t N = num_nodes(p);
    moments(p, f, g, &v->w);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += h[(int64_t)i * N + n];
        v->psi[n] = s;
    }
}

static int nl_check(const orc_params *p, const orc_nl *nl, double *m)
{
    if (p->walls || p->glattice) return -2;
    return orc_nl_mobility(p, nl, m) ? -2 : 0;
}

/* Initial populations: f = feq(rho0, u0), g = geq(phi0, mu_phi~, u0),
 * h = geq(psi0, mu_psi~, u0).  u0 may be NULL.  Returns -2 for walls, the
 * reduced phase-field lattice or a non-positive kappa. */
int orc_nl_init(const orc_params *p, const orc_nl *nl, const double *rho0, const double *phi0,
                const double *psi0, const double *u0, double *f, double *g, double *h)
{
    int Q = lattice_Q(p->lattice);
    int64_t N = num_nodes(p);
    double m[4];
    if (nl_check(p, nl, m)) return -2;
    orc_nl_work v;
    if (nl_work_alloc(&v, N)) { nl_work_free(&v); return -1; }
    memcpy(v.w.rho, rho0, N * sizeof(double));
    memcpy(v.w.phi, phi0, N * sizeof(double));
    memcpy(v.psi, psi0, N * sizeof(double));
    nl_chemical_potentials(p, nl, &v);
    double Gam = gamma_cap_of(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double u[3] = {0, 0, 0}, fe[27], ge[27], he[27];
        if (u0) { u[0] = u0[n]; u[1] = u0[N + n]; if (p->lattice == 1) u[2] = u0[2 * N + n]; }
        double mp = m[0] * v.w.mu_phi[n] + m[1] * v.mu_psi[n];
        double ms = m[2] * v.w.mu_phi[n] + m[3] * v.mu_psi[n];
        orc_feq(p->lattice, rho0[n], u, fe);
        orc_geq(p->lattice, phi0[n], mp, Gam, u, ge);
        orc_geq(p->lattice, psi0[n], ms, Gam, u, he);
        for (int i = 0; i < Q; ++i) {
            f[(int64_t)i * N + n] = fe[i];
            g[(int64_t)i * N + n] = ge[i];
            h[(int64_t)i * N + n] = he[i];
        }
    }
    nl_work_free(&v);
    return 0;
}

/* Advance f, g, h (layout [Q][N], post-streaming) by nsteps: moments ->
 * Laplacians and potentials -> gradients and force -> KBC collision of f with
 * exact-difference forcing, BGK of g and h -> streaming. */
int orc_nl_run(const orc_params *p, const orc_nl *nl, double *f, double *g, double *h, int64_t nsteps)
{
    int Q = lattice_Q(p->lattice);
    int64_t N = num_nodes(p);
    double m[4];
    if (nl_check(p, nl, m)) return -2;
    orc_nl_work v;
    double *fs = malloc((size_t)Q * N * sizeof(double));
    double *gs = malloc((size_t)Q * N * sizeof(double));
    double *hs = malloc((size_t)Q * N * sizeof(double));
    if (nl_work_alloc(&v, N) || !fs || !gs || !hs) {
        nl_work_free(&v); free(fs); free(gs); free(hs);
        return -1;
    }
    const double beta = beta_of(p);
    const double Gam = gamma_cap_of(p);
    const double tau_phi = p->tau_phi;
    for (int64_t step = 0; step < nsteps; ++step) {
        nl_moments(p, f, g, h, &v);
        nl_chemical_potentials(p, nl, &v);
        nl_force(p, &v);
        orc_work *w = &v.w;
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            double fn[27], fo[27], ge[27], he[27], F[3], up[3], gam;
            for (int i = 0; i < Q; ++i) fn[i] = f[(int64_t)i * N + n];
            F[0] = w->force[n]; F[1] = w->force[N + n]; F[2] = w->force[2 * N + n];
            if (p->lattice == 0) F[2] = 0.0;
            orc_collide_node(p->lattice, beta, fn, F, fo, &gam);
            double r = w->rho[n];
            for (int a = 0; a < 3; ++a) up[a] = (w->j[a * N + n] + 0.5 * F[a]) / r;
            if (p->lattice == 0) up[2] = 0.0;
            double mp = m[0] * w->mu_phi[n] + m[1] * v.mu_psi[n];
            double ms = m[2] * w->mu_phi[n] + m[3] * v.mu_psi[n];
            orc_geq(p->lattice, w->phi[n], mp, Gam, up, ge);
            orc_geq(p->lattice, v.psi[n], ms, Gam, up, he);
            for (int i = 0; i < Q; ++i) {
                int64_t k = (int64_t)i * N + n;
                fs[k] = fo[i];
                gs[k] = g[k] - (g[k] - ge[i]) / tau_phi;
                hs[k] = h[k] - (h[k] - he[i]) / tau_phi;
            }
        }
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            for (int i = 0; i < Q; ++i) {
                int c[3];
                direction(i, c);
                int64_t mm = neighbour(p, n, c);
                f[(int64_t)i * N + mm] = fs[(int64_t)i * N + n];
                g[(int64_t)i * N + mm] = gs[(int64_t)i * N + n];
                h[(int64_t)i * N + mm] = hs[(int64_t)i * N + n];
            }
        }
    }
    nl_work_free(&v);
    free(fs); free(gs); free(hs);
    return 0;
}

/* Fields of the state (any output may be NULL): rho, phi, psi, u (physical,
 * [3][N]), c ([3][N]: C1, C2, C3), mu ([3][N]: mu_rho, mu_phi, mu_psi),
 * force ([3][N]). */
int orc_nl_fields(const orc_params *p, const orc_nl *nl, const double *f, const double *g, const double *h,
                  double *rho, double *phi, double *psi, double *u, double *c, double *mu, double *force)
{
    int64_t N = num_nodes(p);
    double m[4];
    if (nl_check(p, nl, m)) return -2;
    orc_nl_work v;
    if (nl_work_alloc(&v, N)) { nl_work_free(&v); return -1; }
    nl_moments(p, f, g, h, &v);
    nl_chemical_potentials(p, nl, &v);
    nl_force(p, &v);
    orc_work *w = &v.w;
    for (int64_t n = 0; n < N; ++n) {
        if (rho) rho[n] = w->rho[n];
        if (phi) phi[n] = w->phi[n];
        if (psi) psi[n] = v.psi[n];
        if (c) {
            double cc[3];
            orc_nl_concentrations(p, w->rho[n], w->phi[n], v.psi[n], cc);
            for (int k = 0; k < 3; ++k) c[k * N + n] = cc[k];
        }
        if (mu) {
            mu[n] = w->mu_rho[n];
            mu[N + n] = w->mu_phi[n];
            mu[2 * N + n] = v.mu_psi[n];
        }
        for (int a = 0; a < 3; ++a) {
            double F = (p->lattice == 0 && a == 2) ? 0.0 : w->force[a * N + n];
            if (u) u[a * N + n] = (p->lattice == 0 && a == 2) ? 0.0 : (w->j[a * N + n] + 0.5 * F) / w->rho[n];
            if (force) force[a * N + n] = F;
        }
    }
    nl_work_free(&v);
    return 0;
}
