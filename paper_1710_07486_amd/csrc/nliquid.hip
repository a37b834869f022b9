// nliquid.hip -- three liquids and the gas: the extension of the ternary model
// to more liquid components that the paper's concluding paragraph names (one
// more double well in the bulk energy of Eq. 2 and one more gradient term in
// Eq. 3, here with a second phase field psi).  FP64, periodic boxes, D2Q9 and
// D3Q27 with the phase fields on the lattice of f; one node per thread in
// three launches per step (moments, potentials, collision).
//
// The model (phi, psi the phase fields, C_L = 1 - C_g the liquid fraction):
//   C1 = (C_L + phi/chi - psi/chi)/2, C2 = (C_L - phi/chi - psi/chi)/2,
//   C3 = psi/chi,
// so psi = 0 is the two-liquid model of the paper.  With
// nu_m = lambda_{m+1} W(C_m) - kappa_{m+1} lap C_m, W(C) = C (1-C)(1-2C):
//   mu_rho = (lambda1/2) Psi' - kappa1 lap rho - (nu1 + nu2) / (2 (rho_g - rho_l)),
//   mu_phi = (nu1 - nu2)/(2 chi),  mu_psi = (2 nu3 - nu1 - nu2)/(2 chi);
// force -rho grad(mu_rho - cs2 ln rho) - phi grad mu_phi - psi grad mu_psi;
// Cahn-Hilliard for phi and psi with the 2 x 2 mobility matrix m (times M)
// that makes the model consistent at liquid-liquid interfaces (the host
// derives it; telbm_nl_mobility states it): the BGK equilibria of g (phi) and h
// (psi) take Gamma (m_pp mu_phi + m_ps mu_psi) and Gamma (m_sp mu_phi +
// m_ss mu_psi).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "next_sums.hpp"

namespace telbm {

namespace {

constexpr int NBX = 64, NBY = 4;

struct NodeAt {
    int x, y, z;
    int64_t n;
    bool in;
};

__device__ __forceinline__ NodeAt node_at(const GridDims& g) {
    const int bxc = (g.nx + NBX - 1) / NBX, byc = (g.ny + NBY - 1) / NBY;
    const int b = blockIdx.x;
    NodeAt t;
    t.x = (b % bxc) * NBX + threadIdx.x;
    t.y = ((b / bxc) % byc) * NBY + threadIdx.y;
    t.z = b / (bxc * byc);
    t.in = t.x < g.nx && t.y < g.ny && t.z < g.nz;
    t.n = ((int64_t)t.z * g.ny + t.y) * g.nx + t.x;
    return t;
}

unsigned nl_blocks(const GridDims& g) {
    return (unsigned)(((g.nx + NBX - 1) / NBX) * ((g.ny + NBY - 1) / NBY) * g.nz);
}

// pop holds 3 Q slices of N values: f, then g (phi), then h (psi); the state
// is post-collision at the writing node, so the pull of direction i at x
// reads slot x - c_i.
template <int L>
__global__ __launch_bounds__(NBX* NBY) void k_nl_moments(GridDims g, const double* __restrict__ pop,
                                                         double* __restrict__ rho, double* __restrict__ phi,
                                                         double* __restrict__ psi) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    const NodeAt t = node_at(g);
    if (!t.in) return;
    const Nbr nb = make_nbr(t.x, t.y, t.z, g.nx, g.ny, g.nz);
    double r = 0.0, p = 0.0, s = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t m = t.n + nbr_off<L>(nb, i, -1);
        r += pop[(int64_t)i * g.N + m];
        p += pop[(int64_t)(Q + i) * g.N + m];
        s += pop[(int64_t)(2 * Q + i) * g.N + m];
    }
    rho[t.n] = r;
    phi[t.n] = p;
    psi[t.n] = s;
}

// Lattice Laplacian (2/cs2) sum_i w_i (v(x + c_i) - v(x)).
template <int L>
__device__ __forceinline__ double lap(const Nbr& nb, int64_t n, const double* __restrict__ v) {
    using Lt = Lattice<L>;
    const double v0 = v[n];
    double s = 0.0;
#pragma unroll
    for (int i = 1; i < Lt::Q; ++i) s += Lt::w[i] * (v[n + nbr_off<L>(nb, i, +1)] - v0);
    return 6.0 * s;
}

// Potentials of one node from its fields and their lattice Laplacians:
// mx = mu_rho - cs2 ln rho (the excess whose gradient drives the fluid),
// mp = mu_phi, ms = mu_psi.
template <int E>
__device__ __forceinline__ void nl_mu(const PhysConst& k, const NlConst& q, double r, double p, double s, double lr,
                                      double lp, double ls, double& mx, double& mp, double& ms) {
    const double cl = 1.0 - (r - k.rho_l) * k.inv_delta;
    const double lcl = -lr * k.inv_delta;
    const double c[3] = {0.5 * (cl + (p - s) * k.inv_chi), 0.5 * (cl - (p + s) * k.inv_chi), s * k.inv_chi};
    const double lc[3] = {0.5 * (lcl + (lp - ls) * k.inv_chi), 0.5 * (lcl - (lp + ls) * k.inv_chi), ls * k.inv_chi};
    const double lam[3] = {k.lambda2, k.lambda3, q.lambda4};
    const double kap[3] = {q.kappa2, q.kappa3, q.kappa4};
    double nu[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) nu[m] = lam[m] * c[m] * (1.0 - c[m]) * (1.0 - 2.0 * c[m]) - kap[m] * lc[m];
    const double lnr = log(r);
    const double mu_rho = k.half_lambda1 * eos_psi_prime<E>(k, r, lnr) - q.kappa1 * lr - (nu[0] + nu[1]) * k.inv_2delta;
    mx = mu_rho - (1.0 / 3.0) * lnr;
    mp = (nu[0] - nu[1]) * k.inv_2chi;
    ms = (2.0 * nu[2] - nu[0] - nu[1]) * k.inv_2chi;
}

template <int L, int E>
__global__ __launch_bounds__(NBX* NBY) void k_nl_chempot(GridDims g, PhysConst k, NlConst q,
                                                         const double* __restrict__ rho,
                                                         const double* __restrict__ phi,
                                                         const double* __restrict__ psi, double* __restrict__ mux,
                                                         double* __restrict__ mup, double* __restrict__ mus) {
    const NodeAt t = node_at(g);
    if (!t.in) return;
    const Nbr nb = make_nbr(t.x, t.y, t.z, g.nx, g.ny, g.nz);
    const int64_t n = t.n;
    nl_mu<E>(k, q, rho[n], phi[n], psi[n], lap<L>(nb, n, rho), lap<L>(nb, n, phi), lap<L>(nb, n, psi), mux[n],
             mup[n], mus[n]);
}

// D3Q27: the potentials along z-columns from the partial sums the collision
// left (as the two-liquid k_chempot_col<true>): the block walks NCZ planes of
// its BX x BY tile, completes rho, phi, psi of the tile and a one-node x-y
// halo of each plane into LDS (three planes held at a time) and takes the
// Laplacians there, in the lattice order of lap(); the tile's completed
// fields are written too.
constexpr int NCZ = 16;
constexpr int NPX = BX + 2, NPY = BY + 2, NPN = NPX * NPY;

template <int E>
__global__ __launch_bounds__(BX* BY) void k_nl_chempot_col(GridDims g, PhysConst k, NlConst q,
                                                           const double* __restrict__ partA,
                                                           const double* __restrict__ inboxA,
                                                           const double* __restrict__ partB,
                                                           const double* __restrict__ inboxB,
                                                           double* __restrict__ rho, double* __restrict__ phi,
                                                           double* __restrict__ psi, double* __restrict__ mux,
                                                           double* __restrict__ mup, double* __restrict__ mus) {
    using Lt = Lattice<kD3Q27>;
    __shared__ double sr[3][NPN], sp[3][NPN], ss[3][NPN];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + BX - 1) / BX, byc = (g.ny + BY - 1) / BY;
    const int bx = b % bxc, rest = b / bxc, by = rest % byc, bzc = rest / byc;
    const int x0 = bx * BX, y0 = by * BY, z0 = bzc * NCZ;
    const int tid = threadIdx.y * BX + threadIdx.x;
    auto load_plane = [&](int slot, int z) {
        const int zw = wrap_any(z, g.nz);
        for (int e = tid; e < NPN; e += BX * BY) {
            const int gx = wrap_any(x0 - 1 + e % NPX, g.nx), gy = wrap_any(y0 - 1 + e / NPX, g.ny);
            const int64_t n = ((int64_t)zw * g.ny + gy) * g.nx + gx;
            double r, p, s, zero;
            next3_complete(g, partA, inboxA, gx, gy, zw, n, r, p);
            next3_complete<1>(g, partB, inboxB, gx, gy, zw, n, s, zero);
            sr[slot][e] = r;
            sp[slot][e] = p;
            ss[slot][e] = s;
        }
    };
    load_plane(0, z0 - 1);
    load_plane(1, z0);
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    const int c = (threadIdx.y + 1) * NPX + threadIdx.x + 1;
    for (int zz = 0; zz < NCZ; ++zz) {
        const int z = z0 + zz;
        if (z >= g.nz) break;  // uniform over the block
        load_plane((zz + 2) % 3, z + 1);
        __syncthreads();
        const int below = zz % 3, centre = (zz + 1) % 3, above = (zz + 2) % 3;
        if (x < g.nx && y < g.ny) {
            const double r0 = sr[centre][c], p0 = sp[centre][c], s0 = ss[centre][c];
            double lr = 0.0, lp = 0.0, ls = 0.0;
#pragma unroll
            for (int i = 1; i < Lt::Q; ++i) {
                const int sl = Lt::c[i][2] == 0 ? centre : (Lt::c[i][2] > 0 ? above : below);
                const int o = c + Lt::c[i][1] * NPX + Lt::c[i][0];
                lr += Lt::w[i] * (sr[sl][o] - r0);
                lp += Lt::w[i] * (sp[sl][o] - p0);
                ls += Lt::w[i] * (ss[sl][o] - s0);
            }
            const int64_t n = ((int64_t)z * g.ny + y) * g.nx + x;
            nl_mu<E>(k, q, r0, p0, s0, 6.0 * lr, 6.0 * lp, 6.0 * ls, mux[n], mup[n], mus[n]);
            rho[n] = r0;
            phi[n] = p0;
            psi[n] = s0;
        }
        __syncthreads();  // the next plane overwrites the slot just read as `below`
    }
}

// Gradients (1/cs2) sum_i w_i c_i v(x + c_i) of the three potentials.
template <int L>
__device__ __forceinline__ void grads(const Nbr& nb, int64_t n, const double* __restrict__ mux,
                                      const double* __restrict__ mup, const double* __restrict__ mus, double* gx,
                                      double* gp, double* gs) {
    using Lt = Lattice<L>;
#pragma unroll
    for (int d = 0; d < 3; ++d) gx[d] = gp[d] = gs[d] = 0.0;
#pragma unroll
    for (int i = 1; i < Lt::Q; ++i) {
        const int64_t m = n + nbr_off<L>(nb, i, +1);
        const double a = Lt::w[i] * mux[m], b = Lt::w[i] * mup[m], c = Lt::w[i] * mus[m];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (Lt::c[i][d] > 0) { gx[d] += a; gp[d] += b; gs[d] += c; }
            else if (Lt::c[i][d] < 0) { gx[d] -= a; gp[d] -= b; gs[d] -= c; }
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) { gx[d] *= 3.0; gp[d] *= 3.0; gs[d] *= 3.0; }
}

template <int L>
__device__ __forceinline__ void nl_force(const GridDims& g, const Nbr& nb, int64_t n, double r, double p, double s,
                                         const double* __restrict__ mux, const double* __restrict__ mup,
                                         const double* __restrict__ mus, double* F) {
    double gx[3], gp[3], gs[3];
    grads<L>(nb, n, mux, mup, mus, gx, gp, gs);
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = -r * gx[d] - p * gp[d] - s * gs[d];
    if (Lattice<L>::D == 2) F[2] = 0.0;
}

// KBC collision of f with exact-difference forcing, BGK of g and h with the
// mixed potentials, for node (x, y, z): post-collision values stored at the
// node when `active`, and handed to the next-moment sinks (sa: f and g, sb: h;
// NoSink when the moments are taken by a separate pass).
template <int L, typename SA, typename SB>
__device__ __forceinline__ void nl_collide_node(const GridDims& g, const PhysConst& k, const NlConst& q,
                                                const double* __restrict__ src, double* __restrict__ dst,
                                                const double* __restrict__ rho, const double* __restrict__ phi,
                                                const double* __restrict__ psi, const double* __restrict__ mux,
                                                const double* __restrict__ mup, const double* __restrict__ mus,
                                                int x, int y, int z, bool active, SA& sa, SB& sb) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    // 32-bit node offsets from uniform per-array bases, non-temporal
    // population traffic on D3Q27 (ld_pop / st_pop), and the three phases
    // (stencil, f, g and h) kept apart as in the two-liquid collision
    const Nbr32 nb = make_nbr32(x, y, z, g.nx, g.ny, g.nz);
    const uint32_t n = (uint32_t)(((int64_t)z * g.ny + y) * g.nx + x);
    const double r = ld(rho, n), p = ld(phi, n), s = ld(psi, n);
    // the node's phase-field potentials, loaded with its other fields
    const double mp = ld(mup, n), ms = ld(mus, n);
    double F[3];
    {
        // force: gradients (1/cs2) sum_i w_i c_i v(x + c_i) of the three
        // potentials, as grads()
        double gx[3] = {0.0, 0.0, 0.0}, gp[3] = {0.0, 0.0, 0.0}, gs[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const uint32_t m = nbr32<L>(nb, n, i, +1);
            const double a = Lt::w[i] * ld(mux, m), b = Lt::w[i] * ld(mup, m), c = Lt::w[i] * ld(mus, m);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (Lt::c[i][d] > 0) { gx[d] += a; gp[d] += b; gs[d] += c; }
                else if (Lt::c[i][d] < 0) { gx[d] -= a; gp[d] -= b; gs[d] -= c; }
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) F[d] = -r * (3.0 * gx[d]) - p * (3.0 * gp[d]) - s * (3.0 * gs[d]);
        if (Lt::D == 2) F[2] = 0.0;
    }
    phase_fence();
    double f[Q];
    double j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        f[i] = ld_pop<L>(src + (size_t)i * g.N, nbr32<L>(nb, n, i, -1));
#pragma unroll
        for (int d = 0; d < 3; ++d) j[d] += Lt::c[i][d] * f[i];
    }
    const double ir = 1.0 / r;
    double u[3] = {j[0] * ir, j[1] * ir, j[2] * ir}, du[3] = {F[0] * ir, F[1] * ir, F[2] * ir};
    if (Lt::D == 2) u[2] = du[2] = 0.0;
    collide_f<L, double>(f, r, ir, u, du, k.beta, k.inv_beta, 0.0);
    if (active) {
#pragma unroll
        for (int i = 0; i < Q; ++i) st_pop<L>(dst + (size_t)i * g.N, n, f[i]);
    }
    sa.template post_f<L, double>(f, r);
    phase_fence();
    const double up[3] = {u[0] + 0.5 * du[0], u[1] + 0.5 * du[1], u[2] + 0.5 * du[2]};
    double gg[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) gg[i] = ld_pop<L>(src + (size_t)(Q + i) * g.N, nbr32<L>(nb, n, i, -1));
    collide_g<L, double>(gg, p, q.m[0] * mp + q.m[1] * ms, up, k.Gamma, k.omega_phi);
    if (active) {
#pragma unroll
        for (int i = 0; i < Q; ++i) st_pop<L>(dst + (size_t)(Q + i) * g.N, n, gg[i]);
    }
    sa.template post_g<L, double, Q>(gg);
    phase_fence();
#pragma unroll
    for (int i = 0; i < Q; ++i) gg[i] = ld_pop<L>(src + (size_t)(2 * Q + i) * g.N, nbr32<L>(nb, n, i, -1));
    collide_g<L, double>(gg, s, q.m[2] * mp + q.m[3] * ms, up, k.Gamma, k.omega_phi);
    if (active) {
#pragma unroll
        for (int i = 0; i < Q; ++i) st_pop<L>(dst + (size_t)(2 * Q + i) * g.N, n, gg[i]);
    }
    sb.template post_f<L, double>(gg, s);
}

template <int L>
__global__ __launch_bounds__(NBX* NBY) void k_nl_collide(GridDims g, PhysConst k, NlConst q,
                                                         const double* __restrict__ src, double* __restrict__ dst,
                                                         const double* __restrict__ rho,
                                                         const double* __restrict__ phi,
                                                         const double* __restrict__ psi,
                                                         const double* __restrict__ mux,
                                                         const double* __restrict__ mup,
                                                         const double* __restrict__ mus) {
    const NodeAt t = node_at(g);
    if (!t.in) return;
    NoSink a, b;
    nl_collide_node<L>(g, k, q, src, dst, rho, phi, psi, mux, mup, mus, t.x, t.y, t.z, true, a, b);
}

// D3Q27: the collision that also leaves the next step's moments, as the
// two-liquid FP64 collision does (k_collide_next3): the block walks a
// z-column of ZC planes of a BX x BY tile, sums its post-collision values
// for the nodes they stream to, (rho, phi) in one NextSink and psi in a
// one-field one, and accumulates them over the column (next3_col_plane) into
// partA / partB and the neighbouring tiles' inboxes.  Both sinks keep two
// sets of sums, used by alternate planes, so one barrier per plane
// suffices.  The potential pass (k_nl_chempot_col) or k_nl_complete adds
// them up.
__global__ __launch_bounds__(BX* BY) void k_nl_collide_next(GridDims g, PhysConst k, NlConst q,
                                                          const double* __restrict__ src, double* __restrict__ dst,
                                                          const double* __restrict__ rho,
                                                          const double* __restrict__ phi,
                                                          const double* __restrict__ psi,
                                                          const double* __restrict__ mux,
                                                          const double* __restrict__ mup,
                                                          const double* __restrict__ mus, double* __restrict__ partA,
                                                          double* __restrict__ inboxA, double* __restrict__ partB,
                                                          double* __restrict__ inboxB) {
    using SinkA = NextSink<kD3Q27, BY, 2>;
    using SinkB = NextSink<kD3Q27, BY, 1>;
    __shared__ double asum[2][SinkA::SUM], aside[2][SinkA::SIDE], bsum[2][SinkB::SUM], bside[2][SinkB::SIDE];
    __shared__ double aacc[col_acc<2>()], bacc[col_acc<1>()];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + BX - 1) / BX, byc = (g.ny + BY - 1) / BY;
    const int bx = b % bxc, rest = b / bxc, by = rest % byc, bc = rest / byc;
    const int x0 = bx * BX, y0 = by * BY, z0 = bc * ZC, z1 = min(g.nz, z0 + ZC);
    const int W = min(BX, g.nx - x0), H = min(BY, g.ny - y0);
    for (int z = z0; z < z1; ++z) {
        const int sb_ = (z - z0) & 1;  // the set of sums of this plane
        int tx = threadIdx.x, ty = threadIdx.y;
        opaque_thread_index(tx, ty);
        {
            // every lane runs a collision (lanes past a ragged edge on the
            // tile's last node, without stores) so that the sinks' shuffles
            // see whole rows
            const int lx = min(tx, W - 1), ly = min(ty, H - 1);
            const bool active = tx < W && ty < H;
            SinkA sa{asum[sb_], aside[sb_], tx, ty, W, 0};
            SinkB sb{bsum[sb_], bside[sb_], tx, ty, W, 0};
            const GridDims gz = opaque_stride(g);
            nl_collide_node<kD3Q27>(gz, k, q, src, dst, rho, phi, psi, mux, mup, mus, x0 + lx, y0 + ly, z, active,
                                    sa, sb);
        }
        __syncthreads();
        next3_col_plane<false, 2>(g, SinkA{asum[sb_], aside[sb_], 0, 0, W, 0}, aacc, partA, inboxA, x0, y0, W, H, z,
                                  z0, z1, tx, ty);
        next3_col_plane<false, 1>(g, SinkB{bsum[sb_], bside[sb_], 0, 0, W, 0}, bacc, partB, inboxB, x0, y0, W, H, z,
                                  z0, z1, tx, ty);
    }
}

// The moments (rho, phi, psi) of the state k_nl_collide_next left, from its
// partial sums and inbox entries.
__global__ __launch_bounds__(NBX* NBY) void k_nl_complete(GridDims g, const double* __restrict__ partA,
                                                          const double* __restrict__ inboxA,
                                                          const double* __restrict__ partB,
                                                          const double* __restrict__ inboxB,
                                                          double* __restrict__ rho, double* __restrict__ phi,
                                                          double* __restrict__ psi) {
    const NodeAt t = node_at(g);
    if (!t.in) return;
    double r, p, s, zero;
    next3_complete(g, partA, inboxA, t.x, t.y, t.z, t.n, r, p);
    next3_complete<1>(g, partB, inboxB, t.x, t.y, t.z, t.n, s, zero);
    rho[t.n] = r;
    phi[t.n] = p;
    psi[t.n] = s;
}

// Equilibria of the initial fields, written where the first pull reads them
// (slot x - c_i holds direction i of node x).
template <int L>
__global__ __launch_bounds__(NBX* NBY) void k_nl_init(GridDims g, PhysConst k, NlConst q,
                                                      const double* __restrict__ rho, const double* __restrict__ phi,
                                                      const double* __restrict__ psi,
                                                      const double* __restrict__ mup,
                                                      const double* __restrict__ mus,
                                                      const double* __restrict__ u0, double* __restrict__ pop) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    const NodeAt t = node_at(g);
    if (!t.in) return;
    const Nbr nb = make_nbr(t.x, t.y, t.z, g.nx, g.ny, g.nz);
    const int64_t n = t.n;
    double u[3] = {0.0, 0.0, 0.0};
    if (u0) {
        u[0] = u0[n];
        u[1] = u0[g.N + n];
        if (Lt::D == 3) u[2] = u0[2 * g.N + n];
    }
    const double mp = mup[n], ms = mus[n];
    double fd[Q], gg[Q], hh[Q];
    equilibria<L, double, false>(rho[n], phi[n], q.m[0] * mp + q.m[1] * ms, u, k.Gamma, 0.0, fd, gg);
    equilibria<L, double, false>(rho[n], psi[n], q.m[2] * mp + q.m[3] * ms, u, k.Gamma, 0.0, fd, hh);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t m = n + nbr_off<L>(nb, i, -1);
        pop[(int64_t)i * g.N + m] = fd[i];
        pop[(int64_t)(Q + i) * g.N + m] = gg[i];
        pop[(int64_t)(2 * Q + i) * g.N + m] = hh[i];
    }
}

// One field of the current state (moments and potentials already current).
template <int L>
__global__ __launch_bounds__(NBX* NBY) void k_nl_macro(GridDims g, PhysConst k, const double* __restrict__ pop,
                                                       const double* __restrict__ rho,
                                                       const double* __restrict__ phi,
                                                       const double* __restrict__ psi,
                                                       const double* __restrict__ mux,
                                                       const double* __restrict__ mup,
                                                       const double* __restrict__ mus, int field,
                                                       double* __restrict__ out) {
    using Lt = Lattice<L>;
    const NodeAt t = node_at(g);
    if (!t.in) return;
    const Nbr nb = make_nbr(t.x, t.y, t.z, g.nx, g.ny, g.nz);
    const int64_t n = t.n;
    const double r = rho[n], p = phi[n], s = psi[n];
    const double cl = 1.0 - (r - k.rho_l) * k.inv_delta;
    double v = 0.0;
    switch (field) {
        case kNlRho: v = r; break;
        case kNlPhi: v = p; break;
        case kNlPsi: v = s; break;
        case kNlC1: v = 0.5 * (cl + (p - s) * k.inv_chi); break;
        case kNlC2: v = 0.5 * (cl - (p + s) * k.inv_chi); break;
        case kNlC3: v = s * k.inv_chi; break;
        case kNlMuRho: v = mux[n] + (1.0 / 3.0) * log(r); break;
        case kNlMuPhi: v = mup[n]; break;
        case kNlMuPsi: v = mus[n]; break;
        default: {
            double F[3];
            nl_force<L>(g, nb, n, r, p, s, mux, mup, mus, F);
            if (field >= kNlFx) {
                v = F[field - kNlFx];
            } else {
                const int d = field - kNlUx;
                double j = 0.0;
#pragma unroll
                for (int i = 0; i < Lt::Q; ++i)
                    if (Lt::c[i][d]) j += Lt::c[i][d] * pop[(int64_t)i * g.N + n + nbr_off<L>(nb, i, -1)];
                v = (Lt::D == 2 && d == 2) ? 0.0 : (j + 0.5 * F[d]) / r;
            }
        }
    }
    out[n] = v;
}

template <int L>
hipError_t nl_part_t(const NlArgs& a, int part) {
    const dim3 blk(NBX, NBY, 1), grd(nl_blocks(a.g), 1, 1);
    if (part == 0) {
        k_nl_moments<L><<<grd, blk, 0, a.stream>>>(a.g, a.src, a.rho, a.phi, a.psi);
    } else if (part == 1) {
        if (a.k.eos == 0)
            k_nl_chempot<L, 0><<<grd, blk, 0, a.stream>>>(a.g, a.k, a.q, a.rho, a.phi, a.psi, a.mux, a.mup, a.mus);
        else if (a.k.eos == 1)
            k_nl_chempot<L, 1><<<grd, blk, 0, a.stream>>>(a.g, a.k, a.q, a.rho, a.phi, a.psi, a.mux, a.mup, a.mus);
        else
            k_nl_chempot<L, 2><<<grd, blk, 0, a.stream>>>(a.g, a.k, a.q, a.rho, a.phi, a.psi, a.mux, a.mup, a.mus);
    } else if (part == 2) {
        k_nl_collide<L><<<grd, blk, 0, a.stream>>>(a.g, a.k, a.q, a.src, a.dst, a.rho, a.phi, a.psi, a.mux, a.mup,
                                                   a.mus);
    } else if (part == 3) {
        k_nl_init<L><<<grd, blk, 0, a.stream>>>(a.g, a.k, a.q, a.rho, a.phi, a.psi, a.mup, a.mus, a.u0, a.dst);
    } else if (part == 4 && L == kD3Q27) {
        if (!a.partA || !a.inboxA || !a.partB || !a.inboxB) return hipErrorInvalidValue;
        k_nl_collide_next<<<column_blocks(a.g), dim3(BX, BY, 1), 0, a.stream>>>(a.g, a.k, a.q, a.src, a.dst, a.rho, a.phi, a.psi,
                                                                   a.mux, a.mup, a.mus, a.partA, a.inboxA, a.partB,
                                                                   a.inboxB);
    } else if (part == 5 && L == kD3Q27) {
        if (!a.partA || !a.inboxA || !a.partB || !a.inboxB) return hipErrorInvalidValue;
        k_nl_complete<<<grd, blk, 0, a.stream>>>(a.g, a.partA, a.inboxA, a.partB, a.inboxB, a.rho, a.phi, a.psi);
    } else if (part == 6 && L == kD3Q27) {
        if (!a.partA || !a.inboxA || !a.partB || !a.inboxB) return hipErrorInvalidValue;
        const unsigned cb = (unsigned)(((a.g.nx + BX - 1) / BX) * ((a.g.ny + BY - 1) / BY) * ((a.g.nz + NCZ - 1) / NCZ));
#define TELBM_NL_COL(EV)                                                                                          \
    k_nl_chempot_col<EV><<<cb, dim3(BX, BY, 1), 0, a.stream>>>(a.g, a.k, a.q, a.partA, a.inboxA, a.partB, a.inboxB, \
                                                               a.rho, a.phi, a.psi, a.mux, a.mup, a.mus)
        if (a.k.eos == 0) TELBM_NL_COL(0);
        else if (a.k.eos == 1) TELBM_NL_COL(1);
        else TELBM_NL_COL(2);
#undef TELBM_NL_COL
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L>
hipError_t nl_macro_t(const NlArgs& a, int field, double* out) {
    k_nl_macro<L><<<nl_blocks(a.g), dim3(NBX, NBY, 1), 0, a.stream>>>(a.g, a.k, a.src, a.rho, a.phi, a.psi, a.mux,
                                                                       a.mup, a.mus, field, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_nl_part(int lattice, const NlArgs& a, int part) {
    return lattice == kD2Q9 ? nl_part_t<kD2Q9>(a, part) : nl_part_t<kD3Q27>(a, part);
}

hipError_t launch_nl_macro(int lattice, const NlArgs& a, int field, double* out) {
    if (field < 0 || field > kNlFz) return hipErrorInvalidValue;
    return lattice == kD2Q9 ? nl_macro_t<kD2Q9>(a, field, out) : nl_macro_t<kD3Q27>(a, field, out);
}

}  // namespace telbm
