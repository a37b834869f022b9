// kernels.hip -- HIP kernels (gfx950) of the ternary free-energy entropic LBM
// time step (arXiv:1710.07486) and their host-side launchers.
//
// Layout in HBM (structure of arrays, x fastest):
//   populations  pop[k][n], k = 0..Q-1 for f, k = Q..2Q-1 for g;
//                n = (z ny + y) nx + x.  The buffer holds the post-collision
//                values f*(x) of the previous step, so a step pulls
//                f_i(x) = pop[i][x - c_i] (periodic).  FP64: absolute values.
//                FP32: f is stored as the deviation f*_i(x) - w_i rho(x) from
//                the writing node's own density (a collision invariant), and
//                rebuilt on the pull from the FP64 densities of the previous
//                state, so the stored number keeps FP32 relative precision in
//                the dilute gas as well as in the liquid.
//   aux fields   rho[n], phi[n], mux[n] (= mu_rho - cs2 ln rho), mup[n] (mu_phi),
//                all FP64.
//
// One step is three launches: node moments (pull-sum of both population sets),
// chemical potentials (Laplacian stencils over rho, phi), and the fused
// pull -> force -> KBC + exact-difference forcing -> phase-field BGK -> write;
// on D2Q9 the last two are one launch (k_collide_fused2).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "kernels.hpp"
#include "lattice.hpp"
#include "node_ops.hpp"

namespace telbm {

constexpr int BX = 64;   // threads along x: one wavefront spans 64 consecutive nodes
constexpr int BY = 4;    // rows per workgroup
constexpr int NXCD = 8;  // accelerator complex dies of the MI355X

// Workgroups are dispatched to the eight XCDs round robin (block b runs on
// XCD b mod 8).  Remap so that each XCD receives a contiguous range of tiles:
// neighbouring tiles share halo lines in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb / NXCD, r = nb % NXCD;
    const int x = b % NXCD, k = b / NXCD;
    return x * q + (x < r ? x : r) + k;
}

struct Tile {
    int x, y, z;
    bool in;
};

__device__ __forceinline__ Tile tile_coords(const GridDims& g) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + BX - 1) / BX, byc = (g.ny + BY - 1) / BY;
    const int bx = b % bxc;
    const int rest = b / bxc;
    const int by = rest % byc;
    const int bz = rest / byc;
    Tile t;
    t.x = bx * BX + threadIdx.x;
    t.y = by * BY + threadIdx.y;
    t.z = bz;
    t.in = (t.x < g.nx) && (t.y < g.ny) && (t.z < g.nz);
    return t;
}

__device__ __forceinline__ int64_t node_of(const GridDims& g, const Tile& t) {
    return ((int64_t)t.z * g.ny + t.y) * g.nx + t.x;
}

// Block-level reduction of the health diagnostics into partials[block][kDiag]
// (NT threads per block, threadIdx.y rows of BX).
template <int NT = BX * BY>
__device__ void diag_block_reduce(double* vals, double* __restrict__ out) {
    // vals: 0 sum rho, 1 sum phi, 2-4 sum j, 5 max |u|, 6 min rho, 7 min gamma,
    //       8 max gamma, 9 nonfinite count
    __shared__ double red[NT / 64][kDiag];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int v = 0; v < 5; ++v) vals[v] += __shfl_xor(vals[v], off);
        vals[5] = fmax(vals[5], __shfl_xor(vals[5], off));
        vals[6] = fmin(vals[6], __shfl_xor(vals[6], off));
        vals[7] = fmin(vals[7], __shfl_xor(vals[7], off));
        vals[8] = fmax(vals[8], __shfl_xor(vals[8], off));
        vals[9] += __shfl_xor(vals[9], off);
    }
    const int lane = (threadIdx.y * BX + threadIdx.x) & 63;
    const int wave = (threadIdx.y * BX + threadIdx.x) >> 6;
    if (lane == 0) {
#pragma unroll
        for (int v = 0; v < kDiag; ++v) red[wave][v] = vals[v];
    }
    __syncthreads();
    if (wave == 0 && lane < kDiag) {
        double acc = red[0][lane];
        for (int w = 1; w < NT / 64; ++w) {
            const double x = red[w][lane];
            if (lane == 5 || lane == 8) acc = fmax(acc, x);
            else if (lane == 6 || lane == 7) acc = fmin(acc, x);
            else acc += x;
        }
        out[(int64_t)xcd_remap(blockIdx.x, gridDim.x) * kDiag + lane] = acc;
    }
}

// ---------------------------------------------------------------------------
// Kernels of the three phases over one lattice (one node per thread).
// ---------------------------------------------------------------------------
template <int L, typename T>
__global__ __launch_bounds__(BX* BY) void k_moments(GridDims g, const T* __restrict__ pop,
                                                    const double* __restrict__ rho_ref,
                                                    double* __restrict__ rho, double* __restrict__ phi) {
    const Tile t = tile_coords(g);
    if (t.in) node_moments<L, T>(g, pop, rho_ref, rho, phi, t.x, t.y, t.z);
}

template <int L>
__global__ __launch_bounds__(BX* BY) void k_chempot(GridDims g, PhysConst k, const double* __restrict__ rho,
                                                    const double* __restrict__ phi, double* __restrict__ mux,
                                                    double* __restrict__ mup) {
    const Tile t = tile_coords(g);
    if (t.in) node_chempot<L>(g, k, rho, phi, mux, mup, t.x, t.y, t.z);
}

__device__ __forceinline__ int wrap_any(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Chemical potentials of D3Q27 along z-columns: the block walks CZ planes of
// its BX x BY tile, holding three planes of rho and phi (with an x-y halo of
// one node) in LDS and loading one new plane per step, so each plane is
// fetched once per column instead of by every z-neighbour.  The Laplacian
// terms are summed in the lattice order of node_chempot, so the potentials
// are the same numbers.
constexpr int CZ = 8;
constexpr int CPX = BX + 2, CPY = BY + 2, CPN = CPX * CPY;

__global__ __launch_bounds__(BX* BY) void k_chempot_col(GridDims g, PhysConst k, const double* __restrict__ rho,
                                                        const double* __restrict__ phi, double* __restrict__ mux,
                                                        double* __restrict__ mup) {
    using Lt = Lattice<kD3Q27>;
    __shared__ double sr[3][CPN], sp[3][CPN];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + BX - 1) / BX, byc = (g.ny + BY - 1) / BY;
    const int bx = b % bxc, rest = b / bxc, by = rest % byc, bzc = rest / byc;
    const int x0 = bx * BX, y0 = by * BY, z0 = bzc * CZ;
    const int tid = threadIdx.y * BX + threadIdx.x;
    auto load_plane = [&](int slot, int z) {
        const int64_t zo = (int64_t)wrap_any(z, g.nz) * g.ny;
        for (int e = tid; e < CPN; e += BX * BY) {
            const int64_t n = (zo + wrap_any(y0 - 1 + e / CPX, g.ny)) * g.nx + wrap_any(x0 - 1 + e % CPX, g.nx);
            sr[slot][e] = rho[n];
            sp[slot][e] = phi[n];
        }
    };
    load_plane(0, z0 - 1);
    load_plane(1, z0);
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    const int c = (threadIdx.y + 1) * CPX + threadIdx.x + 1;
    for (int zz = 0; zz < CZ; ++zz) {
        const int z = z0 + zz;
        if (z >= g.nz) break;  // uniform over the block
        load_plane((zz + 2) % 3, z + 1);
        __syncthreads();
        const int below = zz % 3, centre = (zz + 1) % 3, above = (zz + 2) % 3;
        if (x < g.nx && y < g.ny) {
            const double r0 = sr[centre][c], p0 = sp[centre][c];
            double lr = 0.0, lp = 0.0;
#pragma unroll
            for (int i = 1; i < Lt::Q; ++i) {
                const int sl = Lt::c[i][2] == 0 ? centre : (Lt::c[i][2] > 0 ? above : below);
                const int o = c + Lt::c[i][1] * CPX + Lt::c[i][0];
                lr += Lt::w[i] * (sr[sl][o] - r0);
                lp += Lt::w[i] * (sp[sl][o] - p0);
            }
            double mx, mp;
            chem_pot(k, r0, p0, 6.0 * lr, 6.0 * lp, &mx, &mp);
            const int64_t n = ((int64_t)z * g.ny + y) * g.nx + x;
            mux[n] = mx;
            mup[n] = mp;
        }
        __syncthreads();  // the next plane overwrites the slot just read as `below`
    }
}

template <int L, typename T>
__global__ __launch_bounds__(BX* BY) void k_collide(GridDims g, PhysConst k, const T* __restrict__ src,
                                                    T* __restrict__ dst, const double* __restrict__ rho_ref,
                                                    const double* __restrict__ rho,
                                                    const double* __restrict__ phi,
                                                    const double* __restrict__ mux,
                                                    const double* __restrict__ mup,
                                                    double* __restrict__ partials, int diag) {
    // the block's tile of BX x BY nodes, two lanes per node
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + BX - 1) / BX, byc = (g.ny + BY - 1) / BY;
    const int bx = b % bxc, rest = b / bxc, by = rest % byc, bz = rest / byc;
    double dv[kDiag] = {0, 0, 0, 0, 0, 0, INFINITY, INFINITY, -INFINITY, 0};
    tile_collide<L, T, BX * BY>(g, k, src, dst, rho_ref, rho, phi, mux, mup, bx * BX, by * BY, bz, BX, BY,
                                     threadIdx.y * BX + threadIdx.x, diag != 0, dv);
    if (diag) diag_block_reduce(dv, partials);
}

// ---------------------------------------------------------------------------
// Fused chemical potentials and collision of the 2D lattice.  The block
// stages the densities and phase field of its BX x FBY tile with a halo of two
// nodes in LDS, computes the chemical potentials of the tile with a halo of
// one node there (the same arithmetic, term for term, as k_chempot), and runs
// the collision of its nodes with the force from those LDS potentials: one
// launch and no potential fields in HBM per step.  (On D3Q27 the potential
// halo of a 64 x 4 tile is 4.6 times the tile, so the 3D step keeps its
// separate stencil pass.)  The tile is 64 x 8 so that the potential halo
// adds 29 % to the tile's potential work rather than 55 % at 64 x 4.
// ---------------------------------------------------------------------------
constexpr int FBY = 8;                      // rows per workgroup of the fused step
constexpr int FHX = BX + 4, FHY = FBY + 4;  // density tile with a halo of 2
constexpr int FMX = BX + 2, FMY = FBY + 2;  // potential tile with a halo of 1

struct LdsAux2 {
    const double* sr;
    const double* sp;
    const double* smx;
    const double* smp;
    int lx, ly;  // the node's position in the tile
    __device__ __forceinline__ double rho0(uint32_t) const { return sr[(ly + 2) * FHX + lx + 2]; }
    __device__ __forceinline__ double phi0(uint32_t) const { return sp[(ly + 2) * FHX + lx + 2]; }
    __device__ __forceinline__ double mup0(uint32_t) const { return smp[(ly + 1) * FMX + lx + 1]; }
    template <int L>
    __device__ __forceinline__ void nbr_mu(const Nbr32&, uint32_t, int i, double& a, double& b) const {
        const int o = (ly + 1 + Lattice<L>::c[i][1]) * FMX + lx + 1 + Lattice<L>::c[i][0];
        a = smx[o];
        b = smp[o];
    }
};

template <typename T>
__global__ __launch_bounds__(BX* FBY) void k_collide_fused2(GridDims g, PhysConst k, const T* __restrict__ src,
                                                           T* __restrict__ dst, const double* __restrict__ rho_ref,
                                                           const double* __restrict__ rho,
                                                           const double* __restrict__ phi,
                                                           double* __restrict__ partials, int diag) {
    using Lt = Lattice<kD2Q9>;
    __shared__ double sr[FHX * FHY], sp[FHX * FHY], smx[FMX * FMY], smp[FMX * FMY];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + BX - 1) / BX, byc = (g.ny + FBY - 1) / FBY;
    const int bx = b % bxc, rest = b / bxc, by = rest % byc, bz = rest / byc;
    const int x0 = bx * BX, y0 = by * FBY;
    const int tid = threadIdx.y * BX + threadIdx.x;
    const int64_t zoff = (int64_t)bz * g.nx * g.ny;
    for (int e = tid; e < FHX * FHY; e += BX * FBY) {
        const int hx = e % FHX, hy = e / FHX;
        const int64_t n = zoff + (int64_t)wrap_any(y0 - 2 + hy, g.ny) * g.nx + wrap_any(x0 - 2 + hx, g.nx);
        sr[e] = rho[n];
        sp[e] = phi[n];
    }
    __syncthreads();
    for (int e = tid; e < FMX * FMY; e += BX * FBY) {
        const int c = (e / FMX + 1) * FHX + e % FMX + 1;
        const double r0 = sr[c], p0 = sp[c];
        double lr = 0.0, lp = 0.0;
#pragma unroll
        for (int i = 1; i < Lt::Q; ++i) {
            const int o = c + Lt::c[i][1] * FHX + Lt::c[i][0];
            lr += Lt::w[i] * (sr[o] - r0);
            lp += Lt::w[i] * (sp[o] - p0);
        }
        double mx, mp;
        chem_pot(k, r0, p0, 6.0 * lr, 6.0 * lp, &mx, &mp);
        smx[e] = mx;
        smp[e] = mp;
    }
    __syncthreads();
    double dv[kDiag] = {0, 0, 0, 0, 0, 0, INFINITY, INFINITY, -INFINITY, 0};
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    if (x < g.nx && y < g.ny) {
        const LdsAux2 aux{sr, sp, smx, smp, (int)threadIdx.x, (int)threadIdx.y};
        node_collide_aux<kD2Q9, T>(g, k, src, dst, rho_ref, aux, x, y, bz, diag != 0, dv);
    }
    if (diag) diag_block_reduce<BX * FBY>(dv, partials);
}

// Deterministic second pass over the block partials (one workgroup).
__global__ __launch_bounds__(256) void k_diag_final(const double* __restrict__ partials, int nblocks,
                                                    double* __restrict__ out) {
    __shared__ double red[256][kDiag];
    double acc[kDiag] = {0, 0, 0, 0, 0, 0, INFINITY, INFINITY, -INFINITY, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        const double* v = partials + (int64_t)b * kDiag;
        for (int j = 0; j < kDiag; ++j) {
            if (j == 5 || j == 8) acc[j] = fmax(acc[j], v[j]);
            else if (j == 6 || j == 7) acc[j] = fmin(acc[j], v[j]);
            else acc[j] += v[j];
        }
    }
    for (int j = 0; j < kDiag; ++j) red[threadIdx.x][j] = acc[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int j = 0; j < kDiag; ++j) {
                const double a = red[threadIdx.x][j], b = red[threadIdx.x + s][j];
                if (j == 5 || j == 8) red[threadIdx.x][j] = fmax(a, b);
                else if (j == 6 || j == 7) red[threadIdx.x][j] = fmin(a, b);
                else red[threadIdx.x][j] = a + b;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < kDiag) out[threadIdx.x] = red[0][threadIdx.x];
}

// ---------------------------------------------------------------------------
// Initialisation: equilibrium populations of (rho0, phi0, u0), written so that
// the next pull sees them at their own node (pop[i][x - c_i] = f_i(x)).
// ---------------------------------------------------------------------------
template <int L, typename T>
__global__ __launch_bounds__(BX* BY) void k_init(GridDims g, PhysConst k, const double* __restrict__ rho,
                                                 const double* __restrict__ phi,
                                                 const double* __restrict__ mup,
                                                 const double* __restrict__ u0, T* __restrict__ pop) {
    using Lt = Lattice<L>;
    using R = T;
    constexpr int Q = Lt::Q;
    const Tile t = tile_coords(g);
    if (!t.in) return;
    const Nbr nb = make_nbr(t.x, t.y, t.z, g.nx, g.ny, g.nz);
    const int64_t n = node_of(g, t);
    R u[3] = {R(0), R(0), R(0)};
    if (u0) {
        u[0] = R(u0[n]);
        u[1] = R(u0[g.N + n]);
        if (Lt::D == 3) u[2] = R(u0[2 * g.N + n]);
    }
    R fd[Q], gg[Q];
    const double r = rho[n];
    equilibria<L, R>(r, R(phi[n]), R(mup[n]), u, R(k.Gamma), Deviation<T>::on ? r : 0.0, fd, gg);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t m = n + nbr_off<L>(nb, i, -1);
        // FP32: the value stored at m is relative to the density held for m
        R v = fd[i];
        if (Deviation<T>::on) v += R(Lt::w[i] * (r - rho[m]));
        pop[(int64_t)i * g.N + m] = v;
        pop[(int64_t)(Q + i) * g.N + m] = gg[i];
    }
}

// Count of nodes whose initial values are unusable.
__global__ void k_check_init(int64_t N, int D, const double* __restrict__ rho, const double* __restrict__ phi,
                             const double* __restrict__ u0, unsigned long long* __restrict__ bad) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    bool b = !(isfinite(rho[n]) && rho[n] > 0.0 && isfinite(phi[n]));
    if (u0) {
        for (int d = 0; d < D; ++d) {
            const double v = u0[(int64_t)d * N + n];
            b = b || !(isfinite(v) && fabs(v) < 1.0);
        }
    }
    if (b) atomicAdd(bad, 1ull);
}

// ---------------------------------------------------------------------------
// Read-out of macroscopic fields of the current state.
// ---------------------------------------------------------------------------
template <int L, typename T>
__global__ __launch_bounds__(BX* BY) void k_macro(GridDims g, PhysConst k, const T* __restrict__ pop,
                                                  const double* __restrict__ rho_ref,
                                                  const double* __restrict__ rho,
                                                  const double* __restrict__ phi,
                                                  const double* __restrict__ mux,
                                                  const double* __restrict__ mup, int field,
                                                  double* __restrict__ out) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    const Tile t = tile_coords(g);
    if (!t.in) return;
    const Nbr nb = make_nbr(t.x, t.y, t.z, g.nx, g.ny, g.nz);
    const int64_t n = node_of(g, t);
    const double r = rho[n], p = phi[n];
    double v = 0.0;
    if (field == kFieldRho) {
        v = r;
    } else if (field == kFieldPhi) {
        v = p;
    } else if (field == kFieldC1 || field == kFieldC2) {
        const double cg = (r - k.rho_l) * k.inv_delta;
        v = 0.5 * (1.0 + (field == kFieldC1 ? 1.0 : -1.0) * p * k.inv_chi - cg);
    } else if (field == kFieldMuRho) {
        v = mux[n] + (1.0 / 3.0) * log(r);
    } else if (field == kFieldMuPhi) {
        v = mup[n];
    } else {
        const int d = (field >= kFieldFx) ? field - kFieldFx : field - kFieldUx;
        double gx[3], gp[3];
        gradient2<L>(nb, n, mux, mup, gx, gp);
        const double F = (Lt::D == 2 && d == 2) ? 0.0 : -r * gx[d] - p * gp[d];
        if (field >= kFieldFx) {
            v = F;
        } else {
            double j = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (Lt::c[i][d] == 0) continue;
                const int64_t m = n + nbr_off<L>(nb, i, -1);
                double fi = double(pop[(int64_t)i * g.N + m]);
                if (Deviation<T>::on) fi += Lt::w[i] * rho_ref[m];
                j += Lt::c[i][d] > 0 ? fi : -fi;
            }
            v = (j + 0.5 * F) / r;
        }
    }
    out[n] = v;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static inline unsigned grid_blocks(const GridDims& g) {
    return (unsigned)(((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY) * g.nz);
}

unsigned collide_blocks(const GridDims& g) { return grid_blocks(g); }

template <int L, typename T>
static hipError_t launch_step_parts(const StepArgs& a, int part) {
    const dim3 blk(BX, BY, 1);
    const dim3 grd(grid_blocks(a.g), 1, 1);
    if (part == 0) {
        k_moments<L, T><<<grd, blk, 0, a.stream>>>(a.g, (const T*)a.src, a.rho_ref, a.rho, a.phi);
    } else if (part == 1) {
        if (L == kD3Q27) {
            const unsigned cb = (unsigned)(((a.g.nx + BX - 1) / BX) * ((a.g.ny + BY - 1) / BY) * ((a.g.nz + CZ - 1) / CZ));
            k_chempot_col<<<cb, blk, 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mux, a.mup);
        } else {
            k_chempot<L><<<grd, blk, 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mux, a.mup);
        }
    } else if (part == 2) {
        k_collide<L, T><<<grd, blk, 0, a.stream>>>(a.g, a.k, (const T*)a.src, (T*)a.dst, a.rho_ref, a.rho,
                                                     a.phi, a.mux, a.mup, a.partials, a.diag);
        if (a.diag) k_diag_final<<<1, 256, 0, a.stream>>>(a.partials, (int)grd.x, a.diag_out);
    } else {
        if (L != kD2Q9) return hipErrorInvalidValue;
        const unsigned fb = (unsigned)(((a.g.nx + BX - 1) / BX) * ((a.g.ny + FBY - 1) / FBY) * a.g.nz);
        k_collide_fused2<T><<<fb, dim3(BX, FBY, 1), 0, a.stream>>>(a.g, a.k, (const T*)a.src, (T*)a.dst, a.rho_ref,
                                                                   a.rho, a.phi, a.partials, a.diag);
        if (a.diag) k_diag_final<<<1, 256, 0, a.stream>>>(a.partials, (int)fb, a.diag_out);
    }
    return hipGetLastError();
}

hipError_t launch_part(int lattice, int precision, const StepArgs& a, int part) {
    if (lattice == kD2Q9)
        return precision ? launch_step_parts<kD2Q9, float>(a, part) : launch_step_parts<kD2Q9, double>(a, part);
    return precision ? launch_step_parts<kD3Q27, float>(a, part) : launch_step_parts<kD3Q27, double>(a, part);
}

template <int L, typename T>
static hipError_t launch_init_t(const StepArgs& a, const double* u0) {
    k_init<L, T><<<grid_blocks(a.g), dim3(BX, BY, 1), 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mup, u0,
                                                                     (T*)a.dst);
    return hipGetLastError();
}

hipError_t launch_init(int lattice, int precision, const StepArgs& a, const double* u0) {
    if (lattice == kD2Q9) return precision ? launch_init_t<kD2Q9, float>(a, u0) : launch_init_t<kD2Q9, double>(a, u0);
    return precision ? launch_init_t<kD3Q27, float>(a, u0) : launch_init_t<kD3Q27, double>(a, u0);
}

hipError_t launch_check_init(const GridDims& g, int D, const double* rho, const double* phi, const double* u0,
                             unsigned long long* bad, hipStream_t s) {
    hipError_t e = hipMemsetAsync(bad, 0, sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((g.N + 255) / 256);
    k_check_init<<<nb, 256, 0, s>>>(g.N, D, rho, phi, u0, bad);
    return hipGetLastError();
}

template <int L, typename T>
static hipError_t launch_macro_t(const StepArgs& a, int field, double* out) {
    k_macro<L, T><<<grid_blocks(a.g), dim3(BX, BY, 1), 0, a.stream>>>(a.g, a.k, (const T*)a.src, a.rho_ref,
                                                                      a.rho, a.phi, a.mux, a.mup, field, out);
    return hipGetLastError();
}

hipError_t launch_macro(int lattice, int precision, const StepArgs& a, int field, double* out) {
    if (lattice == kD2Q9)
        return precision ? launch_macro_t<kD2Q9, float>(a, field, out) : launch_macro_t<kD2Q9, double>(a, field, out);
    return precision ? launch_macro_t<kD3Q27, float>(a, field, out) : launch_macro_t<kD3Q27, double>(a, field, out);
}

}  // namespace telbm
