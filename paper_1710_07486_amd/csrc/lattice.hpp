// lattice.hpp -- velocity sets and per-node arithmetic of the ternary
// free-energy entropic LBM update (arXiv:1710.07486), for gfx950.
//
// Everything here is __device__ inline and templated on the lattice (D2Q9 or
// D3Q27) and on the arithmetic type R (double, or float for the mixed
// precision form), so the single-instance and batched kernels share it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace telbm {

constexpr int kD2Q9 = 0;
constexpr int kD3Q27 = 1;

// Velocity sets: rest first, then opposite pairs (2p-1, 2p) = (c, -c) for
// p = 1..(Q-1)/2, ordered faces, edges, corners.  The pair order lets half a
// wavefront handle each direction's opposite (see node_ops.hpp).
template <int L>
struct Lattice;

template <>
struct Lattice<kD2Q9> {
    static constexpr int D = 2;
    static constexpr int Q = 9;
    static constexpr int c[9][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    static constexpr double w[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
};

template <>
struct Lattice<kD3Q27> {
    static constexpr int D = 3;
    static constexpr int Q = 27;
    static constexpr int c[27][3] = {
        {0, 0, 0},                                                             // rest
        {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},  {0, 0, -1},  // faces
        {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},  {-1, 0, -1},
        {1, 0, -1},  {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1}, {0, -1, 1},  // edges
        {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1},
        {-1, 1, 1},  {1, -1, -1}};                                           // corners
    static constexpr double w[27] = {
        8.0 / 27,
        2.0 / 27,  2.0 / 27,  2.0 / 27,  2.0 / 27,  2.0 / 27,  2.0 / 27,
        1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,
        1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,  1.0 / 54,
        1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216, 1.0 / 216};
};

// Index of -c_i: opposite directions are adjacent pairs (2p-1, 2p).
__host__ __device__ constexpr int opp_dir(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
template <int L>
__host__ __device__ constexpr bool opposites_paired() {
    for (int i = 0; i < Lattice<L>::Q; ++i)
        for (int d = 0; d < 3; ++d)
            if (Lattice<L>::c[opp_dir(i)][d] != -Lattice<L>::c[i][d]) return false;
    return true;
}
static_assert(opposites_paired<kD2Q9>() && opposites_paired<kD3Q27>(), "opposite directions are paired");

// Per-instance constants, precomputed on the host from the parameters.
struct PhysConst {
    // equation of state (Eq. 4) and bulk free energy (Eq. 2)
    double a, b, RT, C;
    double half_lambda1;          // lambda1 / 2
    double lambda2, lambda3;
    double rho_l;
    double inv_delta;             // 1 / (rho_g - rho_l)
    double inv_2delta;            // 1 / (2 (rho_g - rho_l))
    double inv_chi, inv_2chi;
    // gradient terms (f_I rewrite): -2A lap rho - D lap phi, -2B lap phi - D lap rho
    double twoA, twoB, Dc;
    // kinetics
    double beta;                  // 1 / (2 tau), tau = 3 nu + 1/2
    double inv_beta;              // 2 tau
    double omega_phi;             // 1 / tau_phi
    double Gamma;                 // M / (tau_phi - 1/2)
    // equation of state: 0 Carnahan-Starling (Eq. 4), 1 van der Waals, 2 Peng-Robinson;
    // att: attraction a (CS, vdW) or a alpha(T) (PR)
    int eos;
    double att;
    // solid walls at y = -1/2 and y = ny - 1/2 (GridDims::walls): cot of the
    // contact angles of rho and phi at the bottom [0] and top [1] wall
    double cot_rho[2], cot_phi[2];
    // phase-field lattice: 0 as for f, 1 reduced (D2Q5 / D3Q7)
    int glat;
};

// Ghost value of rho or phi beyond a wall (geometric wetting condition): the
// wall-row value v plus cot(theta) times the magnitude of its gradient along
// the wall, from central differences tx (along x) and tz (along z, 0 in 2D).
__device__ __forceinline__ double wet_ghost(double v, double tx, double tz, double cot) {
    return v + cot * sqrt(tx * tx + tz * tz);
}

// Periodic neighbour offsets of one node: off[d][k] is the element offset of
// the neighbour at displacement k-1 along axis d.
struct Nbr {
    int64_t ox[3], oy[3], oz[3];
};

__device__ __forceinline__ Nbr make_nbr(int x, int y, int z, int nx, int ny, int nz) {
    Nbr n;
    const int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    n.ox[1] = 0;
    n.ox[0] = (x == 0 ? (nx - 1) : -1) * sx;
    n.ox[2] = (x == nx - 1 ? -(nx - 1) : 1) * sx;
    n.oy[1] = 0;
    n.oy[0] = (y == 0 ? (int64_t)(ny - 1) : -1) * sy;
    n.oy[2] = (y == ny - 1 ? -(int64_t)(ny - 1) : 1) * sy;
    n.oz[1] = 0;
    n.oz[0] = (z == 0 ? (int64_t)(nz - 1) : -1) * sz;
    n.oz[2] = (z == nz - 1 ? -(int64_t)(nz - 1) : 1) * sz;
    return n;
}

// Element offset of the node at +sign*c_i from the node.
template <int L>
__device__ __forceinline__ int64_t nbr_off(const Nbr& n, int i, int sign) {
    using Lt = Lattice<L>;
    return n.ox[1 + sign * Lt::c[i][0]] + n.oy[1 + sign * Lt::c[i][1]] + n.oz[1 + sign * Lt::c[i][2]];
}

// ---------------------------------------------------------------------------
// Entropic equilibrium in product form.  Per axis, with S = sqrt(1 + 3u^2),
// the D1Q3 factors of the entropic equilibrium simplify without division to
//   psi_0 = (2/3)(2 - S),  psi_+ = (2S - 1 + 3u)/6,  psi_- = (2S - 1 - 3u)/6,
// since (2 - S)(2u + S) = (2S - 1 + 3u)(1 - u).  Relative to the weights:
//   psi_0 / (2/3) - 1 = -(S - 1),  psi_+- / (1/6) - 1 = 2(S - 1) +- 3u,
// with S - 1 = 3u^2 / (1 + S) evaluated without cancellation.
// ---------------------------------------------------------------------------
template <typename R>
struct AxisEq {
    R e[3];      // factor / weight - 1 for c = 0, +1, -1
    R inv[3];    // 1 / factor for c = 0, +1, -1
};

// Reciprocals without the full IEEE division sequence: the hardware estimate,
// refined by Newton steps to full precision in FP64 (one step suffices for
// FP32, whose estimate is accurate to about one ulp).
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = r * (2.0 - x * r);
    r = r * (2.0 - x * r);
    return r;
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// S - 1 = sqrt(1 + 3u^2) - 1.  FP32: 3u^2/(1 + S), free of cancellation, so
// that the equilibrium's deviation from w_i rho keeps its relative precision
// for the deviation storage.  FP64: S - 1 directly; its absolute error is
// one ulp of 1, the rounding the factor (1 + e) carries anyway.
__device__ __forceinline__ double s_minus_1(double u2, double S) { return S - 1.0; }
__device__ __forceinline__ float s_minus_1(float u2, float S) { return 3.0f * u2 * fast_rcp(1.0f + S); }

template <typename R>
__device__ __forceinline__ AxisEq<R> axis_eq(R u, bool want_inv) {
    AxisEq<R> a;
    const R u2 = u * u;
    const R S = sqrt(R(1) + R(3) * u2);
    const R sm1 = s_minus_1(u2, S);
    a.e[0] = -sm1;
    a.e[1] = R(2) * sm1 + R(3) * u;
    a.e[2] = R(2) * sm1 - R(3) * u;
    if (want_inv) {
        // (2S-1+3u)(2S-1-3u) = 5 + 3u^2 - 4S; one reciprocal for the three
        const R twoms = R(1) - sm1;                  // 2 - S
        const R prod = R(5) + R(3) * u2 - R(4) * S;  // > 0 for |u| < 1
        const R inv = fast_rcp(twoms * prod);
        a.inv[0] = R(1.5) * prod * inv;
        a.inv[1] = R(6) * (R(1) + R(2) * sm1 - R(3) * u) * twoms * inv;
        a.inv[2] = R(6) * (R(1) + R(2) * sm1 + R(3) * u) * twoms * inv;
    }
    return a;
}

__device__ __forceinline__ int kidx(int c) { return c == 0 ? 0 : (c > 0 ? 1 : 2); }

// prod_alpha (1 + e_alpha) - 1 for direction i, accurate when the e are small.
template <int L, typename R>
__device__ __forceinline__ R eq_excess(const AxisEq<R>* ax, int i) {
    using Lt = Lattice<L>;
    const R ex = ax[0].e[kidx(Lt::c[i][0])];
    const R ey = ax[1].e[kidx(Lt::c[i][1])];
    R t = ex + ey + ex * ey;
    if (L == kD3Q27) {
        const R ez = ax[2].e[kidx(Lt::c[i][2])];
        t = t + ez * (R(1) + t);
    }
    return t;
}

template <int L, typename R>
__device__ __forceinline__ R eq_inv(const AxisEq<R>* ax, int i) {
    using Lt = Lattice<L>;
    R v = ax[0].inv[kidx(Lt::c[i][0])] * ax[1].inv[kidx(Lt::c[i][1])];
    if (L == kD3Q27) v = v * ax[2].inv[kidx(Lt::c[i][2])];
    return v;
}

// ---------------------------------------------------------------------------
// One collision of the density populations held in registers.  fd[i] holds
// f_i - w_i rho_ref and is overwritten with the post-collision value in the
// same offset form (rho_ref = 0 for absolute populations; the node's own
// density for the FP32 deviation storage).  u = j / rho, du = F / rho.
//
// KBC: df = f - feq; the shear part ds carries exactly the traceless second
// moments of df (normal-stress differences and off-diagonal stresses), the
// rest dh = df - ds.  gamma = 1/beta - (2 - 1/beta) <ds|dh>/<dh|dh> with
// <X|Y> = sum X_i Y_i / feq_i, and gamma = 2 when <dh|dh> = 0.
// f* = f - beta (2 ds + gamma dh) + feq(rho, u + du) - feq(rho, u)
//    = (1 - 2 beta) ds + (1 - beta gamma) dh + feq(rho, u + du)   (offset form).
// The two scalar products and their ratio are accumulated in FP64.  The
// array holds df, then dh, so that one array is live through the passes.
// ---------------------------------------------------------------------------
template <int L, typename R>
__device__ __forceinline__ double collide_f(R* fd, double rho_d, double inv_rho_d, const R* u, const R* du,
                                            R beta, double inv_beta, double rho_ref) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    constexpr int D = Lt::D;
    const R rho = R(rho_d);
    const R drho = R(rho_d - rho_ref);  // rho - rho_ref, formed in FP64 before rounding

    AxisEq<R> ax[3], ax2[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        ax[a] = axis_eq<R>(u[a], true);
        ax2[a] = axis_eq<R>(u[a] + du[a], false);
    }
    if (D == 2) {
        ax[2].e[0] = ax[2].e[1] = ax[2].e[2] = R(0);
        ax[2].inv[0] = ax[2].inv[1] = ax[2].inv[2] = R(1);
        ax2[2] = ax[2];
    }
    // non-equilibrium part df = f - feq (kept in fd) and its second moments
    R mxx = 0, myy = 0, mzz = 0, mxy = 0, mxz = 0, myz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R df = fd[i] - R(Lt::w[i]) * (drho + rho * eq_excess<L, R>(ax, i));
        fd[i] = df;
        const int cx = Lt::c[i][0], cy = Lt::c[i][1], cz = Lt::c[i][2];
        if (cx) mxx += df;
        if (cy) myy += df;
        if (cz) mzz += df;
        if (cx * cy) mxy += (cx * cy > 0) ? df : -df;
        if (cx * cz) mxz += (cx * cz > 0) ? df : -df;
        if (cy * cz) myz += (cy * cz > 0) ? df : -df;
    }
    R dxx, dyy, dzz;
    if (D == 2) {
        dxx = R(0.5) * (mxx - myy);
        dyy = -dxx;
        dzz = 0;
    } else {
        const R tr = (mxx + myy + mzz) * R(1.0 / 3.0);
        dxx = mxx - tr;
        dyy = myy - tr;
        dzz = mzz - tr;
    }
    // shear part: ds_i = sum_pq M_pq b_p(c_ix) b_q(c_iy) b_r(c_iz) over the
    // traceless second moments, with the D1Q3 dual basis b0 = [c == 0],
    // b1 = c/2, b2 = (c == 0 ? -1 : 1/2); only the nonzero terms are formed.
    auto shear = [&](int i) -> R {
        const int cx = Lt::c[i][0], cy = Lt::c[i][1], cz = Lt::c[i][2];
        const int nzc = (cx != 0) + (cy != 0) + (cz != 0);
        if (nzc == 1) return R(0.5) * (cx ? dxx : (cy ? dyy : dzz));
        if (nzc == 2) {
            if (!cz) return R(0.25 * cx * cy) * mxy;
            if (!cy) return R(0.25 * cx * cz) * mxz;
            return R(0.25 * cy * cz) * myz;
        }
        if (nzc == 0) return -(dxx + dyy + dzz);  // zero up to rounding (traceless)
        return R(0);
    };
    const R inv_rho = R(inv_rho_d);
    double sh = 0.0, hh = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R s = shear(i);
        const R dh = fd[i] - s;
        fd[i] = dh;
        const double ifeq = double(inv_rho * eq_inv<L, R>(ax, i));
        sh += double(s) * double(dh) * ifeq;
        hh += double(dh) * double(dh) * ifeq;
    }
    const double gamma = (hh > 1e-300) ? (inv_beta - (2.0 - inv_beta) * sh / hh) : 2.0;
    const R g = R(gamma);
    const R cs = R(1) - R(2) * beta, ch = R(1) - beta * g;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        fd[i] = cs * shear(i) + ch * fd[i] + R(Lt::w[i]) * (drho + rho * eq_excess<L, R>(ax2, i));
    return gamma;
}

// Phase-field BGK (standard free-energy scheme for Eq. 7):
// geq_i = w_i [3 Gamma mu_phi + 3 phi c_i.u + 4.5 phi (c_i.u)^2 - 1.5 phi u^2]
// for i != 0, and geq_0 = phi - sum_{i != 0} geq_i, which in closed form is
// phi - (1 - w_0)(3 Gamma mu_phi - 1.5 phi u^2) - 1.5 phi u^2.
// g* = g + omega_phi (geq - g).  u is the physical velocity.
template <int L, typename R>
__device__ __forceinline__ void collide_g(R* g, R phi, R mu_phi, const R* u, R Gamma, R omega) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R base = R(3) * Gamma * mu_phi - R(1.5) * phi * uu;
    const R g0 = phi - R(1.0 - Lt::w[0]) * base - R(1.5) * phi * uu;
    g[0] = g[0] + omega * (g0 - g[0]);
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const R cu = R(Lt::c[i][0]) * u[0] + R(Lt::c[i][1]) * u[1] + R(Lt::c[i][2]) * u[2];
        const R geq = R(Lt::w[i]) * (base + R(3) * phi * cu + R(4.5) * phi * cu * cu);
        g[i] = g[i] + omega * (geq - g[i]);
    }
}

// Reduced phase-field lattice (RG): the rest and axis directions, the first
// 1 + 2D of the order above (D2Q5 / D3Q7), axis weights 1/6 (sum_i w_i c_i c_i
// = cs2 I as on the full lattice) and the equilibrium to first order in u:
//   geq_i = (1/6)(3 Gamma mu_phi + 3 phi c_i.u) on the axes, geq_0 = phi - sum.
template <int L, bool RG>
struct GLattice {
    static constexpr int Q = RG ? 1 + 2 * Lattice<L>::D : Lattice<L>::Q;
};
template <int L>
__host__ __device__ constexpr bool axes_first() {
    for (int i = 1; i <= 2 * Lattice<L>::D; ++i) {
        int n = 0;
        for (int d = 0; d < 3; ++d) n += Lattice<L>::c[i][d] != 0;
        if (n != 1) return false;
    }
    return true;
}
static_assert(axes_first<kD2Q9>() && axes_first<kD3Q27>(), "axis directions come right after rest");

template <int L, typename R>
__device__ __forceinline__ void collide_g_reduced(R* g, R phi, R mu_phi, const R* u, R Gamma, R omega) {
    constexpr int QG = 1 + 2 * Lattice<L>::D;
    const R half_gm = R(0.5) * Gamma * mu_phi;
    R rest = R(0);
#pragma unroll
    for (int i = 1; i < QG; ++i) {
        const R cu = R(Lattice<L>::c[i][0]) * u[0] + R(Lattice<L>::c[i][1]) * u[1] + R(Lattice<L>::c[i][2]) * u[2];
        const R geq = half_gm + R(0.5) * phi * cu;
        rest += geq;
        g[i] = g[i] + omega * (geq - g[i]);
    }
    g[0] = g[0] + omega * ((phi - rest) - g[0]);
}

template <int L, typename R, bool RG>
__device__ __forceinline__ void collide_g_lat(R* g, R phi, R mu_phi, const R* u, R Gamma, R omega) {
    if constexpr (RG) collide_g_reduced<L, R>(g, phi, mu_phi, u, Gamma, omega);
    else collide_g<L, R>(g, phi, mu_phi, u, Gamma, omega);
}

// Equilibrium populations for initialisation, f in offset form about rho_ref
// (g: GLattice<L, RG>::Q values).
template <int L, typename R, bool RG = false>
__device__ __forceinline__ void equilibria(double rho_d, R phi, R mu_phi, const R* u, R Gamma,
                                           double rho_ref, R* fd, R* g) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    AxisEq<R> ax[3];
#pragma unroll
    for (int a = 0; a < Lt::D; ++a) ax[a] = axis_eq<R>(u[a], false);
    if (Lt::D == 2) ax[2].e[0] = ax[2].e[1] = ax[2].e[2] = R(0);
    const R rho = R(rho_d);
    const R drho = R(rho_d - rho_ref);
#pragma unroll
    for (int i = 0; i < Q; ++i) fd[i] = R(Lt::w[i]) * (drho + rho * eq_excess<L, R>(ax, i));
    for (int i = 0; i < GLattice<L, RG>::Q; ++i) g[i] = R(0);
    collide_g_lat<L, R, RG>(g, phi, mu_phi, u, Gamma, R(1));
}

// Chemical potentials of the free energy (Eqs. 2-4 and the f_I rewrite), in
// FP64.  Returns mu_rho - cs2 ln rho (the excess potential whose gradient
// drives the fluid) in *mu_x and mu_phi in *mu_p; lap_* are lattice
// Laplacians.  Psi' of the equation of state:
//   Carnahan-Starling (Eq. 4): C - 2 a rho + RT (ln rho + 1) - 16 RT (12 - b rho)/(b rho - 4)^3
//   van der Waals:   C + RT [ln(rho/(1 - b rho)) + 1/(1 - b rho)] - 2 a rho
//   Peng-Robinson:   C + RT [ln(rho/(1 - b rho)) + 1/(1 - b rho)]
//                      - A [ln((1 + (1+sqrt2) b rho)/(1 + (1-sqrt2) b rho))/(2 sqrt2 b)
//                           + rho/(1 + 2 b rho - b^2 rho^2)]
// E is the equation of state (0, 1, 2 in the order above), fixed at compile
// time so that the Carnahan-Starling kernels carry none of the other two's
// registers; k.eos must equal E.
template <int E>
__device__ __forceinline__ double eos_psi_prime(const PhysConst& k, double rho, double lr) {
    static_assert(E >= 0 && E <= 2, "equation of state 0..2");
    if constexpr (E == 0) {
        const double d = k.b * rho - 4.0;
        return k.C - 2.0 * k.a * rho + k.RT * (lr + 1.0) - 16.0 * k.RT * (12.0 - k.b * rho) / (d * d * d);
    }
    const double br = k.b * rho, m = 1.0 - br;
    const double rep = k.C + k.RT * (lr - log(m) + 1.0 / m);
    if constexpr (E == 1) return rep - 2.0 * k.att * rho;
    constexpr double s2 = 1.41421356237309504880;
    const double D = 1.0 + 2.0 * br - br * br;
    return rep - k.att * (log((1.0 + (1.0 + s2) * br) / (1.0 + (1.0 - s2) * br)) / (2.0 * s2 * k.b) + rho / D);
}

template <int E>
__device__ __forceinline__ void chem_pot(const PhysConst& k, double rho, double phi, double lap_rho,
                                         double lap_phi, double* mu_x, double* mu_p) {
    const double lr = log(rho);
    const double psi_p = eos_psi_prime<E>(k, rho, lr);
    const double cg = (rho - k.rho_l) * k.inv_delta;
    const double c1 = 0.5 * (1.0 + phi * k.inv_chi - cg);
    const double c2 = 0.5 * (1.0 - phi * k.inv_chi - cg);
    const double w1 = c1 * (1.0 - c1) * (1.0 - 2.0 * c1);
    const double w2 = c2 * (1.0 - c2) * (1.0 - 2.0 * c2);
    const double mu_rho = k.half_lambda1 * psi_p - (k.lambda2 * w1 + k.lambda3 * w2) * k.inv_2delta -
                          k.twoA * lap_rho - k.Dc * lap_phi;
    *mu_x = mu_rho - (1.0 / 3.0) * lr;
    *mu_p = (k.lambda2 * w1 - k.lambda3 * w2) * k.inv_2chi - k.twoB * lap_phi - k.Dc * lap_rho;
}

}  // namespace telbm
