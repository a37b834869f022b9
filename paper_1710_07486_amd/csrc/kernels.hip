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
//                all FP64.  D2Q9 also keeps per-tile inboxes of next-step
//                moment sums (k_collide_fused2).
//
// D3Q27: one step is three launches: node moments (pull-sum of both population
// sets), chemical potentials (Laplacian stencils over rho, phi), and the fused
// pull -> force -> KBC + exact-difference forcing -> phase-field BGK -> write.
// D2Q9: one launch per step (k_collide_fused2) that also leaves the next
// step's moments; the moment pass runs only after initialisation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "kernels.hpp"
#include "lattice.hpp"
#include "node_ops.hpp"
#include "next_sums.hpp"

namespace telbm {

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
// W: instance for lattices with walls (the periodic instance carries none of
// the wall logic and keeps its registers).

// Planes a collision block walks along z on D3Q27: a node's stencil fields
// on the plane above it are read again by the same block one plane later,
// while they are still in its XCD's L2.  Measured on the FP32 pair split at
// 256^3 (64 x 4 tiles): 2.34 ms at depth 1, 2.29 at 2, 2.30 at 4, 2.34 at 8,
// 2.37 at 16 (deeper columns leave fewer blocks to balance the launch's tail).
constexpr int kCollideDepth = 2;
template <int L>
constexpr int collide_depth() {
    return L == kD3Q27 ? kCollideDepth : 1;
}
// Tile width of the D3Q27 collision and FP32 moment pass blocks (BX BY
// nodes of one plane: 256 x 1).  A pull shifted along x spans one more cache
// line than its row, which the neighbouring tile fetches again: wider tiles
// have fewer such edges.  Measured at 256^3 (FP32 pair split, 64 x 4 ->
// 128 x 2 -> 256 x 1): collision 2.289 -> 2.270 -> 2.231 ms, moment pass
// 0.853 -> 0.833 -> 0.830 ms.
constexpr int kTileW3 = 256;
template <int L>
constexpr int collide_tile_w() {
    return L == kD3Q27 ? kTileW3 : BX;
}
static_assert(BX * BY % kTileW3 == 0, "tiles of BX BY nodes");

template <int L, typename T, bool W, bool RG>
__global__ __launch_bounds__(BX* BY) void k_moments(GridDims g, const T* __restrict__ pop,
                                                    const double* __restrict__ rho_ref,
                                                    double* __restrict__ rho, double* __restrict__ phi) {
    if constexpr (Deviation<T>::on && L == kD3Q27) {
        // FP32 D3Q27 (the moment pass of every step), on MW x MH tiles: the
        // reference densities of the pull sources come from an LDS copy of
        // the tile with a halo of one node in x, y and z instead of 27
        // scattered loads per node
        using Lt = Lattice<L>;
        constexpr int MW = kTileW3, MH = BX * BY / MW;
        constexpr int RX = MW + 2, RY = MH + 2, RP = RX * RY;
        __shared__ double sref[3][RP];
        const int b = xcd_remap(blockIdx.x, gridDim.x);
        const int bxc = (g.nx + MW - 1) / MW, byc = (g.ny + MH - 1) / MH;
        const int x0 = (b % bxc) * MW, y0 = (b / bxc % byc) * MH;
        const int lin = threadIdx.y * BX + threadIdx.x, lx = lin % MW, ly = lin / MW;
        Tile t;
        t.x = x0 + lx;
        t.y = y0 + ly;
        t.z = b / bxc / byc;
        t.in = t.x < g.nx && t.y < g.ny && t.z < g.nz;
        for (int e = lin; e < 3 * RP; e += BX * BY) {
            const int pl = e / RP, q = e % RP;
            auto wr = [](int v, int m) { v %= m; return v < 0 ? v + m : v; };
            const int gx = wr(x0 - 1 + q % RX, g.nx), gy = wr(y0 - 1 + q / RX, g.ny);
            const int gz = wr(t.z - 1 + pl, g.nz);
            sref[pl][q] = rho_ref[((int64_t)gz * g.ny + gy) * g.nx + gx];
        }
        __syncthreads();
        if (!t.in) return;
        const Nbr nb = make_nbr(t.x, t.y, t.z, g.nx, g.ny, g.nz);
        const int64_t n = node_index(g, t.x, t.y, t.z);
        const int c0 = (ly + 1) * RX + lx + 1;
        double r = 0.0, p = 0.0;
#pragma unroll
        for (int i = 0; i < Lt::Q; ++i) {
            const bool bb = W && bounce(g, t.y, Lt::c[i][1]);
            const int64_t m = bb ? n : n + nbr_off<L>(nb, i, -1);
            const int s = bb ? opp_dir(i) : i;
            const double ref = bb ? sref[1][c0] : sref[1 - Lt::c[i][2]][c0 - Lt::c[i][1] * RX - Lt::c[i][0]];
            r += double(pop[(int64_t)s * g.N + m]) + Lt::w[i] * ref;
            if (i < GLattice<L, RG>::Q) p += double(pop[(int64_t)(Lt::Q + s) * g.N + m]);
        }
        rho[n] = r;
        phi[n] = p;
    } else {
        const Tile t = tile_coords(g);
        if (t.in) node_moments<L, T, W, RG>(g, pop, rho_ref, rho, phi, t.x, t.y, t.z);
    }
}

template <int L, int E, bool W>
__global__ __launch_bounds__(BX* BY) void k_chempot(GridDims g, PhysConst k, const double* __restrict__ rho,
                                                    const double* __restrict__ phi, double* __restrict__ mux,
                                                    double* __restrict__ mup) {
    const Tile t = tile_coords(g);
    if (t.in) node_chempot<L, E, W>(g, k, rho, phi, mux, mup, t.x, t.y, t.z);
}

// Chemical potentials of D3Q27 along z-columns: the block walks CZ planes of
// its BX x col_rows tile, holding three planes of rho and phi (with an x-y halo of
// one node) in LDS and loading one new plane per step, so each plane is
// fetched once per column instead of by every z-neighbour.  The Laplacian
// terms are summed in the lattice order of node_chempot, so the potentials
// are the same numbers.
constexpr int CZ = 16;
constexpr int CPX = BX + 2;
// rows of a column's tile: 8 where the pass completes partial sums (their
// halo re-reads cost more per node), else 4
template <bool PART>
constexpr int col_rows() {
    return PART ? 8 : 4;
}

// With PART the densities come as the partial sums and inbox entries that
// the previous D3Q27 FP64 collision (k_collide_next3) left;
// the kernel completes them while staging (see next3_complete) and also writes
// the completed rho, phi of its nodes.  Each thread fetches its entries of
// the plane after next into registers while the block computes a plane
// (four wavefronts per SIMD asked for, so that the registers this holds do
// not cost occupancy).
template <bool PART, int E, bool W>
__global__ __launch_bounds__(BX* col_rows<PART>()) __attribute__((amdgpu_waves_per_eu(4))) void k_chempot_col(GridDims g, PhysConst k, double* __restrict__ rho,
                                                        double* __restrict__ phi, double* __restrict__ mux,
                                                        double* __restrict__ mup, const double* __restrict__ part,
                                                        const double* __restrict__ inbox) {
    using Lt = Lattice<kD3Q27>;
    constexpr int CBY = col_rows<PART>(), CPY = CBY + 2, CPN = CPX * CPY;
    __shared__ double sr[3][CPN], sp[3][CPN];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + BX - 1) / BX, byc = (g.ny + CBY - 1) / CBY;
    const int bx = b % bxc, rest = b / bxc, by = rest % byc, bzc = rest / byc;
    const int x0 = bx * BX, y0 = by * CBY, z0 = bzc * CZ;
    const int tid = threadIdx.y * BX + threadIdx.x;
    // the (completed) densities of node (gx, gy, zw)
    auto get = [&](int gx, int gy, int zw, double& r, double& p) {
        const int64_t n = ((int64_t)zw * g.ny + gy) * g.nx + gx;
        if (PART) {
            next3_complete(g, part, inbox, gx, gy, zw, n, r, p);
        } else {
            r = rho[n];
            p = phi[n];
        }
    };
    // the staged densities of entry e of plane z's tile with its halo
    auto fetch = [&](int e, int z, double& r, double& p) {
        const int zw = wrap_any(z, g.nz);
        const int gx = wrap_any(x0 - 1 + e % CPX, g.nx), yy = y0 - 1 + e / CPX;
        if (W && g.walls && (yy < 0 || yy >= g.ny)) {
            // beyond a wall: the wetting ghost of the wall-row node
            const int top = yy >= g.ny, yw = top ? g.ny - 1 : 0;
            double rxm, pxm, rxp, pxp, rzm, pzm, rzp, pzp;
            get(gx == 0 ? g.nx - 1 : gx - 1, yw, zw, rxm, pxm);
            get(gx + 1 == g.nx ? 0 : gx + 1, yw, zw, rxp, pxp);
            get(gx, yw, zw == 0 ? g.nz - 1 : zw - 1, rzm, pzm);
            get(gx, yw, zw + 1 == g.nz ? 0 : zw + 1, rzp, pzp);
            get(gx, yw, zw, r, p);
            r = wet_ghost(r, 0.5 * (rxp - rxm), 0.5 * (rzp - rzm), k.cot_rho[top]);
            p = wet_ghost(p, 0.5 * (pxp - pxm), 0.5 * (pzp - pzm), k.cot_phi[top]);
        } else {
            get(gx, wrap_any(yy, g.ny), zw, r, p);
        }
    };
    // a plane's entries of this thread (e = tid, tid + BX CBY, ...) travel through
    // registers: fetched a plane ahead, stored to LDS when their slot is free
    constexpr int PER = (CPN + BX * CBY - 1) / (BX * CBY);
    double nr[PER], np[PER];
    auto fetch_plane = [&](int z) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = tid + j * BX * CBY;
            if (e < CPN) fetch(e, z, nr[j], np[j]);
        }
    };
    auto store_plane = [&](int slot) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = tid + j * BX * CBY;
            if (e < CPN) {
                sr[slot][e] = nr[j];
                sp[slot][e] = np[j];
            }
        }
    };
    fetch_plane(z0 - 1);
    store_plane(0);
    fetch_plane(z0);
    store_plane(1);
    fetch_plane(z0 + 1);
    const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
    const int c = (threadIdx.y + 1) * CPX + threadIdx.x + 1;
    for (int zz = 0; zz < CZ; ++zz) {
        const int z = z0 + zz;
        if (z >= g.nz) break;  // uniform over the block
        store_plane((zz + 2) % 3);  // plane z + 1
        __syncthreads();
        // plane z + 2 in flight while plane z is computed
        if (zz + 1 < CZ && z + 1 < g.nz) fetch_plane(z + 2);
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
            chem_pot<E>(k, r0, p0, 6.0 * lr, 6.0 * lp, &mx, &mp);
            const int64_t n = ((int64_t)z * g.ny + y) * g.nx + x;
            mux[n] = mx;
            mup[n] = mp;
            if (PART) {
                rho[n] = r0;
                phi[n] = p0;
            }
        }
        __syncthreads();  // the next plane overwrites the slot just read as `below`
    }
}

template <int L, typename T, bool RG, bool W = false>
__global__ __launch_bounds__(BX* BY) void k_collide(GridDims g, PhysConst k, const T* __restrict__ src,
                                                    T* __restrict__ dst, const double* __restrict__ rho_ref,
                                                    const double* __restrict__ rho,
                                                    const double* __restrict__ phi,
                                                    const double* __restrict__ mux,
                                                    const double* __restrict__ mup,
                                                    double* __restrict__ partials, int diag) {
    // the block's tile of TW x TH nodes over planes [z0, z1) of its z-column
    // (two lanes per node in the pair split)
    constexpr int ZD = collide_depth<L>(), TW = collide_tile_w<L>(), TH = BX * BY / TW;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + TW - 1) / TW, byc = (g.ny + TH - 1) / TH;
    const int bx = b % bxc, rest = b / bxc, by = rest % byc, bc = rest / byc;
    const int z0 = bc * ZD, z1 = min(g.nz, z0 + ZD);
    double dv[kDiag] = {0, 0, 0, 0, 0, 0, INFINITY, INFINITY, -INFINITY, 0};
    for (int z = z0; z < z1; ++z) {
        const GridDims gz = ZD > 1 ? opaque_stride(g) : g;
        tile_collide<L, T, BX * BY, RG, W>(gz, k, src, dst, rho_ref, rho, phi, mux, mup, bx * TW, by * TH, z, TW, TH,
                                         threadIdx.y * BX + threadIdx.x, diag != 0, dv);
    }
    if (diag) diag_block_reduce(dv, partials);
}

// ---------------------------------------------------------------------------
// Fused chemical potentials, collision and next-step densities of the 2D
// lattice.  The block stages the densities and phase field of its BX x FBY
// tile with a halo of two nodes in LDS, computes the chemical potentials of
// the tile with a halo of one node there (the same arithmetic, term for term,
// as k_chempot), and runs the collision of its nodes with the force from those
// LDS potentials: no potential fields in HBM.  (On D3Q27 the potential halo of
// a 64 x 4 tile is 4.6 times the tile, so the 3D step keeps its separate
// stencil pass.)  The tile is 64 x 8 so that the potential halo adds 29 % to
// the tile's potential work rather than 55 % at 64 x 4.
//
// The block also sums the moments of the next step, rho'(x) = sum_i f*_i(x -
// c_i) and phi'(x) = sum_i g*_i(x - c_i), from its own post-collision values
// (the values the pull of the next step reconstructs: in the FP32 form the
// stored deviation plus w_i times the writer's density), over the sources
// that lie in the tile: tile nodes receive these partial sums in rho_next /
// phi_next, and the sums for the one-node ring around the tile go to the
// inboxes of the tiles that own those ring nodes.  The next launch completes
// each staged density with the inbox entries of its node, so a step is one
// launch and the moment pass over all populations runs only after
// initialisation.
//
// Within a wavefront (one tile row of 64 consecutive x) the three directions
// of each row offset c_y are combined with lane shuffles, so a node leaves
// three sums per field in LDS instead of nine values.
// ---------------------------------------------------------------------------
constexpr int FBY = 8;                      // rows per workgroup of the fused step
constexpr int FHX = BX + 4, FHY = FBY + 4;  // density tile with a halo of 2
constexpr int FMX = BX + 2, FMY = FBY + 2;  // potential tile with a halo of 1
constexpr int INBOX = Inbox<FBY>::SIZE;          // the 2D step's tiles

struct LdsAux2 {
    const double* sr;
    const double* sp;
    const double* smx;
    const double* smp;
    const double* sref;  // reference densities of the tile and its halo (FP32 form)
    int lx, ly;  // the node's position in the tile
    template <int L>
    __device__ __forceinline__ double ref(const double*, const Nbr32&, uint32_t, int i, bool bb) const {
        return bb ? sref[(ly + 2) * FHX + lx + 2]
                  : sref[(ly + 2 - Lattice<L>::c[i][1]) * FHX + lx + 2 - Lattice<L>::c[i][0]];
    }
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

// LDS of one fused 2D tile step.
template <typename T>
struct Fused2Lds {
    using Sink = NextSink<kD2Q9, FBY>;
    double sr[FHX * FHY], sp[FHX * FHY], smx[FMX * FMY], smp[FMX * FMY];
    double sref[Deviation<T>::on ? FHX * FHY : 1];
    double nsum[Sink::SUM], nside[Sink::SIDE];
};

// One tile (bx, by) of the fused 2D step: the body of k_collide_fused2, also
// walked over (instance, tile) work lists by the batched form.
template <typename T, int E, bool RG, bool WALL>
__device__ __forceinline__ void fused2_tile(Fused2Lds<T>& sh, const GridDims& g, const PhysConst& k,
                                            const T* __restrict__ src, T* __restrict__ dst,
                                            const double* __restrict__ rho_ref, const double* __restrict__ rho,
                                            const double* __restrict__ phi, const double* __restrict__ inbox_in,
                                            double* __restrict__ rho_next, double* __restrict__ phi_next,
                                            double* __restrict__ inbox_out, double* __restrict__ rho_final,
                                            double* __restrict__ partials, int diag, int bx, int by) {
    using Lt = Lattice<kD2Q9>;
    using Sink = NextSink<kD2Q9, FBY>;
    double* sr = sh.sr;
    double* sp = sh.sp;
    double* smx = sh.smx;
    double* smp = sh.smp;
    double* sref = sh.sref;
    double* nsum = sh.nsum;
    double* nside = sh.nside;
    const int x0 = bx * BX, y0 = by * FBY;
    const int W = min(BX, g.nx - x0), H = min(FBY, g.ny - y0);
    const int tid = threadIdx.y * BX + threadIdx.x;
    // densities of the tile and its halo; partial sums (inbox_in set) are
    // completed with the inbox entries of their nodes
    auto load = [&](int gx, int gy, double& r, double& p) {
        const int64_t n = (int64_t)gy * g.nx + gx;
        r = rho[n];
        p = phi[n];
        if (inbox_in) inbox_complete_fast<FBY>(g, inbox_in, gx, gy, r, p);
    };
    for (int e = tid; e < FHX * FHY; e += BX * FBY) {
        const int hx = e % FHX, hy = e / FHX;
        const int gx = wrap_any(x0 - 2 + hx, g.nx), yy = y0 - 2 + hy;
        double r, p;
        if (WALL && g.walls && (yy < 0 || yy >= g.ny)) {
            // beyond a wall: the wetting ghost of the wall-row node below/above
            const int top = yy >= g.ny, yw = top ? g.ny - 1 : 0;
            double rm, pm, rp, pp;
            load(gx == 0 ? g.nx - 1 : gx - 1, yw, rm, pm);
            load(gx + 1 == g.nx ? 0 : gx + 1, yw, rp, pp);
            load(gx, yw, r, p);
            r = wet_ghost(r, 0.5 * (rp - rm), 0.0, k.cot_rho[top]);
            p = wet_ghost(p, 0.5 * (pp - pm), 0.0, k.cot_phi[top]);
        } else {
            load(gx, wrap_any(yy, g.ny), r, p);
        }
        sr[e] = r;
        sp[e] = p;
        if (Deviation<T>::on) sref[e] = rho_ref[(int64_t)wrap_any(yy, g.ny) * g.nx + gx];
    }
    __syncthreads();
    for (int e = tid; e < FMX * FMY; e += BX * FBY) {
        // beyond a wall the potentials repeat the wall row
        const int yy = y0 - 1 + e / FMX;
        const int my = (WALL && g.walls) ? (yy < 0 ? 1 : (yy == g.ny ? -1 : 0)) : 0;
        const int c = (e / FMX + 1 + my) * FHX + e % FMX + 1;
        const double r0 = sr[c], p0 = sp[c];
        double lr = 0.0, lp = 0.0;
#pragma unroll
        for (int i = 1; i < Lt::Q; ++i) {
            const int o = c + Lt::c[i][1] * FHX + Lt::c[i][0];
            lr += Lt::w[i] * (sr[o] - r0);
            lp += Lt::w[i] * (sp[o] - p0);
        }
        double mx, mp;
        chem_pot<E>(k, r0, p0, 6.0 * lr, 6.0 * lp, &mx, &mp);
        smx[e] = mx;
        smp[e] = mp;
    }
    __syncthreads();
    double dv[kDiag] = {0, 0, 0, 0, 0, 0, INFINITY, INFINITY, -INFINITY, 0};
    {
        // every lane runs a collision (lanes past a ragged edge on the tile's
        // last node, without stores) so that the sink's shuffles see whole rows
        const int lx = min((int)threadIdx.x, W - 1), ly = min((int)threadIdx.y, H - 1);
        const bool active = (int)threadIdx.x < W && (int)threadIdx.y < H;
        const LdsAux2 aux{sr, sp, smx, smp, sref, lx, ly};
        if (rho_final && active) rho_final[(int64_t)(y0 + ly) * g.nx + x0 + lx] = aux.rho0(0);
        const int wy = (WALL && g.walls) ? (y0 + ly == 0 ? -1 : (y0 + ly == g.ny - 1 ? 1 : 0)) : 0;
        Sink sink{nsum, nside, (int)threadIdx.x, (int)threadIdx.y, W, wy};
        node_collide_sink<kD2Q9, T, LdsAux2, Sink, WALL, RG>(g, k, src, dst, rho_ref, aux, x0 + lx, y0 + ly, 0,
                                                             diag != 0, dv, active, sink);
    }
    if (diag) diag_block_reduce<BX * FBY>(dv, partials);
    __syncthreads();
    // next moments of the tile (each thread its own node) and of its ring
    const Sink view{nsum, nside, 0, 0, W, 0};
    if ((int)threadIdx.x < W && (int)threadIdx.y < H) {
        double s0, s1;
        view.gather(threadIdx.x, threadIdx.y, 0, H, s0, s1);
        const int64_t n = (int64_t)(y0 + threadIdx.y) * g.nx + x0 + threadIdx.x;
        rho_next[n] = s0;
        phi_next[n] = s1;
    }
    constexpr int RING2 = 2 * (BX + 2) + 2 * FBY;
    for (int q = tid; q < RING2; q += BX * FBY) {
        int ex, ey;
        if (q < 2 * (BX + 2)) {
            ex = q % (BX + 2) - 1;
            ey = q < BX + 2 ? -1 : H;
            if (ex > W) continue;
        } else {
            const int c = q - 2 * (BX + 2);
            ex = c < FBY ? -1 : W;
            ey = c % FBY;
            if (ey >= H) continue;
        }
        // nothing streams into a wall (those values bounced back in the sink)
        if (WALL && g.walls && ((ey < 0 && y0 == 0) || (ey >= H && y0 + H == g.ny))) continue;
        double s0, s1;
        view.gather(ex, ey, 0, H, s0, s1);
        const int64_t q2 = 2 * inbox_target<FBY>(g, x0, y0, W, H, ex, ey);
        inbox_out[q2] = s0;
        inbox_out[q2 + 1] = s1;
    }
}

template <typename T, int E, bool RG, bool WALL>
__global__ __launch_bounds__(BX* FBY) void k_collide_fused2(GridDims g, PhysConst k, const T* __restrict__ src,
                                                           T* __restrict__ dst, const double* __restrict__ rho_ref,
                                                           const double* __restrict__ rho,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ inbox_in,
                                                           double* __restrict__ rho_next,
                                                           double* __restrict__ phi_next,
                                                           double* __restrict__ inbox_out,
                                                           double* __restrict__ rho_final,
                                                           double* __restrict__ partials, int diag) {
    __shared__ Fused2Lds<T> sh;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + BX - 1) / BX;
    fused2_tile<T, E, RG, WALL>(sh, g, k, src, dst, rho_ref, rho, phi, inbox_in, rho_next, phi_next, inbox_out,
                                rho_final, partials, diag, b % bxc, b / bxc);
}

// The fused 2D step of a batch of lattices in one launch (WB: some of them
// have walls; each instance's own flag decides for it): one
// workgroup per (instance, 64 x 8 tile) item of the work list, consecutive
// items on one XCD.  State: cur (populations), ref (FP32 reference
// densities), fp (densities, phase field and inbox of the current step),
// partial (those densities still to be completed from the inbox).
template <typename T, int E, bool WB>
__global__ __launch_bounds__(BX* FBY) void k_batch_fused2(const FusedDesc* __restrict__ inst,
                                                          const int2* __restrict__ work, int nwork, int cur,
                                                          int ref, int fp, int partial) {
    __shared__ Fused2Lds<T> sh;
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    if (w >= nwork) return;  // uniform over the block
    const int2 it = work[w];
    const FusedDesc& d = inst[it.x];
    const int bxc = (d.g.nx + BX - 1) / BX;
    const bool mixed = Deviation<T>::on;
    fused2_tile<T, E, false, WB>(sh, d.g, d.k, (const T*)d.pop[cur], (T*)d.pop[1 - cur],
                                    mixed ? d.rhob[ref] : nullptr, d.xr[fp], d.xp[fp],
                                    partial ? d.inbox[fp] : nullptr, d.xr[1 - fp], d.xp[1 - fp], d.inbox[1 - fp],
                                    mixed ? d.rhob[1 - ref] : nullptr, nullptr, 0, it.y % bxc, it.y / bxc);
}

template <typename T, bool WB>
static hipError_t launch_batch_fused2_t(int eos, hipStream_t st, const FusedDesc* inst, const int2* work, int nwork,
                                        int cur, int ref, int fp, int partial) {
    const dim3 blk(BX, FBY, 1);
    const int grid = nwork;  // one workgroup per item
    switch (eos) {
        case 0: k_batch_fused2<T, 0, WB><<<grid, blk, 0, st>>>(inst, work, nwork, cur, ref, fp, partial); break;
        case 1: k_batch_fused2<T, 1, WB><<<grid, blk, 0, st>>>(inst, work, nwork, cur, ref, fp, partial); break;
        case 2: k_batch_fused2<T, 2, WB><<<grid, blk, 0, st>>>(inst, work, nwork, cur, ref, fp, partial); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_fused2(int precision, int eos, bool walls, hipStream_t st, const FusedDesc* inst,
                               const int2* work, int nwork, int cur, int ref, int fp, int partial) {
    if (walls)
        return precision ? launch_batch_fused2_t<float, true>(eos, st, inst, work, nwork, cur, ref, fp, partial)
                         : launch_batch_fused2_t<double, true>(eos, st, inst, work, nwork, cur, ref, fp, partial);
    return precision ? launch_batch_fused2_t<float, false>(eos, st, inst, work, nwork, cur, ref, fp, partial)
                     : launch_batch_fused2_t<double, false>(eos, st, inst, work, nwork, cur, ref, fp, partial);
}

int fused_tiles_x(int nx) { return (nx + BX - 1) / BX; }

// Completes partial next-step moments in place with their inbox entries (the
// edge nodes of every tile), before the densities are read outside the fused
// step.  One workgroup per tile, one thread per edge node.
constexpr int FIX_THREADS = 2 * BX + 2 * FBY;

__global__ __launch_bounds__(FIX_THREADS) void k_dens_complete2(GridDims g, double* __restrict__ rho,
                                                                double* __restrict__ phi,
                                                                const double* __restrict__ inbox) {
    const int b = blockIdx.x;
    const int bxc = (g.nx + BX - 1) / BX;
    const int x0 = (b % bxc) * BX, y0 = (b / bxc) * FBY;
    const int W = min(BX, g.nx - x0), H = min(FBY, g.ny - y0);
    const int nrow = H > 1 ? 2 * W : W;
    const int ncol = H > 2 ? (W > 1 ? 2 : 1) * (H - 2) : 0;
    const int t = threadIdx.x;
    if (t >= nrow + ncol) return;
    int lx, ly;
    if (t < W) {
        lx = t;
        ly = 0;
    } else if (t < nrow) {
        lx = t - W;
        ly = H - 1;
    } else if (t - nrow < H - 2) {
        lx = 0;
        ly = 1 + (t - nrow);
    } else {
        lx = W - 1;
        ly = 1 + (t - nrow - (H - 2));
    }
    const int64_t n = (int64_t)(y0 + ly) * g.nx + x0 + lx;
    double r = rho[n], p = phi[n];
    inbox_complete<FBY>(g, inbox, x0 + lx, y0 + ly, r, p);
    rho[n] = r;
    phi[n] = p;
}

// ---------------------------------------------------------------------------
// D3Q27 FP64 collision that also leaves the next step's moments.  The block
// walks a z-column of ZC planes of a BX x BY tile: per plane it runs the
// collision of the tile's nodes and sums their post-collision values for the
// nodes they stream to, with the lane shuffles of NextSink over the nine
// (c_y, c_z) groups, then per target plane z + c_z for the tile and its
// one-node ring.  The sums for the column's own planes accumulate in LDS
// over the three source planes and are stored once a plane is complete: one
// (rho, phi) pair per node (part), plus inbox entries for the tile-edge nodes
// of the neighbouring tiles; only the columns' end planes receive sums from
// the next column (the boundary parts; layout at next3_complete).  The
// chemical-potential pass completes them while it stages the densities
// (k_chempot_col<true>), so the moment pass over all populations is not run.
// ---------------------------------------------------------------------------
// Cache policy of the LDS-DMA loads: non-temporal, as the other population
// loads of the 3D collision.
constexpr int kNonTemporal = 2;

// The phase-field populations pulled by one wavefront's row of the tile: LDS
// row[i BX + d] holds direction i (i < QG, the full or reduced phase-field
// lattice) pulled by node x0 + d of row y in plane z (nodes past a ragged
// edge repeat node W - 1), with the halfway bounce-back of node_collide_sink
// where walls are (a bounced direction reads the node's own slot of -c_i;
// whether it bounces depends on the row only).  Filled by LDS-DMA loads, a
// dword per lane (two loads per direction), so that the fetch of the next
// plane's values holds no registers while the current plane is collided.
template <bool WALL, int QG>
__device__ __forceinline__ void stage_g_row(const GridDims& g, const double* __restrict__ src, double* row, int x0,
                                            int y, int z, int W, int lane) {
    using Lt = Lattice<kD3Q27>;
    constexpr int Q = Lt::Q;
    using GPtr = const __attribute__((address_space(1))) void*;
    using LPtr = __attribute__((address_space(3))) void*;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int x = x0 + min(32 * h + (lane >> 1), W - 1);
        const Nbr32 nb = WALL ? make_nbr32_w(g, x, y, z) : make_nbr32(x, y, z, g.nx, g.ny, g.nz);
        const uint32_t n = (uint32_t)node_index(g, x, y, z);
#pragma unroll
        for (int i = 0; i < QG; ++i) {
            const bool bb = WALL && bounce(g, y, Lt::c[i][1]);
            const uint32_t m = bb ? n : nbr32<kD3Q27>(nb, n, i, -1);
            const char* a = (const char*)(src + (size_t)(Q + (bb ? opp_dir(i) : i)) * g.N) +
                            (uint32_t)(m * 8u + 4u * (lane & 1));
            // lane l fills dword l of the 64 that hold doubles 32 h .. 32 h + 31
            __builtin_amdgcn_global_load_lds((GPtr)a, (LPtr)(row + i * BX + 32 * h), 4, 0, kNonTemporal);
        }
    }
}

// Staging policy of node_collide_sink for the z-column collision: the
// wavefront's row of this plane's values, in LDS.
struct GRowStaged {
    static constexpr bool on = true;
    const double* row;
    int lane;
    __device__ __forceinline__ double pulled(int i) const { return row[i * BX + lane]; }
};

// DIAG: the instance that also reduces the health diagnostics (launched on the
// steps that take them; the other keeps none of their registers).
template <bool WALL, bool RG, bool DIAG>
__global__ __launch_bounds__(BX* BY) void k_collide_next3(GridDims g, PhysConst k, const double* __restrict__ src,
                                                          double* __restrict__ dst, const double* __restrict__ rho,
                                                          const double* __restrict__ phi,
                                                          const double* __restrict__ mux,
                                                          const double* __restrict__ mup, double* __restrict__ part,
                                                          double* __restrict__ inbox, double* __restrict__ partials,
                                                          int diag) {
    using Sink = NextSink<kD3Q27, BY>;
    // two sets of sums, used by alternate planes: a plane's collisions then
    // never overwrite the sums that slower threads still gather from, and one
    // barrier per plane suffices
    __shared__ double nsum[2][Sink::SUM], nside[2][Sink::SIDE], acc[col_acc<2>()];
    // each wavefront's row of pulled phase-field populations is staged one
    // plane ahead (GRowStaged)
    constexpr int QG = GLattice<kD3Q27, RG>::Q;
    __shared__ double gstage[BY * QG * BX];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int bxc = (g.nx + BX - 1) / BX, byc = (g.ny + BY - 1) / BY;
    const int bx = b % bxc, rest = b / bxc, by = rest % byc, bc = rest / byc;
    const int x0 = bx * BX, y0 = by * BY, z0 = bc * ZC, z1 = min(g.nz, z0 + ZC);
    const int W = min(BX, g.nx - x0), H = min(BY, g.ny - y0);
    double dv[kDiag] = {0, 0, 0, 0, 0, 0, INFINITY, INFINITY, -INFINITY, 0};
    const GlobalAux aux{rho, phi, mux, mup};
    // the wavefront's row (uniform over it) and its staging row
    const int wrow = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    double* grow = gstage + wrow * QG * BX;
    stage_g_row<WALL, QG>(g, src, grow, x0, y0 + min(wrow, H - 1), z0, W, threadIdx.x);
    for (int z = z0; z < z1; ++z) {
        int tx = threadIdx.x, ty = threadIdx.y;
        opaque_thread_index(tx, ty);
        {
            // every lane runs a collision (lanes past a ragged edge on the
            // tile's last node, without stores) so that the sink's shuffles
            // see whole rows
            const int lx = min(tx, W - 1), ly = min(ty, H - 1);
            const bool active = tx < W && ty < H;
            const int wy = (WALL && g.walls) ? (y0 + ly == 0 ? -1 : (y0 + ly == g.ny - 1 ? 1 : 0)) : 0;
            const GridDims gz = opaque_stride(g);
            Sink sink{nsum[(z - z0) & 1], nside[(z - z0) & 1], tx, ty, W, wy};
            const GRowStaged st{grow, tx};
            node_collide_sink<kD3Q27, double, GlobalAux, Sink, WALL, RG, GRowStaged>(
                gz, k, src, dst, nullptr, aux, x0 + lx, y0 + ly, z, DIAG, dv, active, sink, st);
        }
        __syncthreads();
        // the next plane's phase-field pulls, staged while this plane's sums
        // are gathered and the next plane's f is collided (issued after the
        // barrier, which would otherwise wait for them; the row's reads of
        // this plane are complete at the barrier)
        if (z + 1 < z1) stage_g_row<WALL, QG>(g, src, grow, x0, y0 + min(wrow, H - 1), z + 1, W, tx);
        next3_col_plane<WALL>(g, Sink{nsum[(z - z0) & 1], nside[(z - z0) & 1], 0, 0, W, 0}, acc, part, inbox, x0,
                              y0, W, H, z, z0, z1, tx, ty);
    }
    if (DIAG) diag_block_reduce(dv, partials);
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
template <int L, typename T, bool RG>
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
    R fd[Q], gg[GLattice<L, RG>::Q];
    const double r = rho[n];
    equilibria<L, R, RG>(r, R(phi[n]), R(mup[n]), u, R(k.Gamma), Deviation<T>::on ? r : 0.0, fd, gg);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // the slot the pull of direction i at this node reads: that of x - c_i,
        // or this node's slot of -c_i where x - c_i lies beyond a wall
        const bool bb = bounce(g, t.y, Lt::c[i][1]);
        const int64_t m = bb ? n : n + nbr_off<L>(nb, i, -1);
        const int s = bb ? opp_dir(i) : i;
        // FP32: the value stored at m is relative to the density held for m
        R v = fd[i];
        if (Deviation<T>::on) v += R(Lt::w[i] * (r - rho[m]));
        pop[(int64_t)s * g.N + m] = v;
        if (i < GLattice<L, RG>::Q) pop[(int64_t)(Q + s) * g.N + m] = gg[i];
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
    const Nbr nb = make_nbr_w(g, t.x, t.y, t.z);
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
                const bool bb = bounce(g, t.y, Lt::c[i][1]);
                const int64_t m = bb ? n : n + nbr_off<L>(nb, i, -1);
                double fi = double(pop[(int64_t)(bb ? opp_dir(i) : i) * g.N + m]);
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

template <int L, typename T>
static inline unsigned moments_grid(const GridDims& g) {
    if (!(Deviation<T>::on && L == kD3Q27)) return grid_blocks(g);
    constexpr int MW = kTileW3, MH = BX * BY / MW;
    return (unsigned)(((g.nx + MW - 1) / MW) * ((g.ny + MH - 1) / MH) * g.nz);
}

template <int L>
static inline unsigned collide_grid(const GridDims& g) {
    constexpr int ZD = collide_depth<L>(), TW = collide_tile_w<L>(), TH = BX * BY / TW;
    return (unsigned)(((g.nx + TW - 1) / TW) * ((g.ny + TH - 1) / TH) * ((g.nz + ZD - 1) / ZD));
}


unsigned fused_tiles(const GridDims& g) { return (unsigned)(((g.nx + BX - 1) / BX) * ((g.ny + FBY - 1) / FBY)); }

size_t inbox_doubles(const GridDims& g) { return (size_t)fused_tiles(g) * INBOX * 2; }

size_t part3_doubles(const GridDims& g, int nf) {
    return nf * ((size_t)g.N + 2 * (size_t)zcols(g.nz) * g.nx * g.ny);
}

size_t inbox3_doubles(const GridDims& g, int nf) {
    return nf * (size_t)(g.nz + 2 * zcols(g.nz)) * (size_t)tiles3(g) * INBOX3;
}

unsigned column_blocks(const GridDims& g) { return (unsigned)(tiles3(g) * zcols(g.nz)); }

// Blocks of the largest launch on this grid that leaves per-block
// diagnostics (the size of the partials buffer): the plain collision of
// either lattice, the z-column collision and the fused 2D step.
unsigned collide_blocks(const GridDims& g) {
    unsigned m = grid_blocks(g);
    for (unsigned v : {collide_grid<kD2Q9>(g), collide_grid<kD3Q27>(g), column_blocks(g), fused_tiles(g)})
        m = v > m ? v : m;
    return m;
}

static inline unsigned col_blocks(const GridDims& g, int rows) {
    return (unsigned)(((g.nx + BX - 1) / BX) * ((g.ny + rows - 1) / rows) * ((g.nz + CZ - 1) / CZ));
}

template <int L, typename T, int E>
static hipError_t launch_step_parts(const StepArgs& a, int part) {
    const dim3 blk(BX, BY, 1);
    const dim3 grd(grid_blocks(a.g), 1, 1);
    const dim3 cgrd(collide_grid<L>(a.g), 1, 1);  // the collision's z-column tiles
    // z-column potential passes: without (0) and with (1) partial sums
    const dim3 cb0(BX, col_rows<false>(), 1), cb1(BX, col_rows<true>(), 1);
    const unsigned cg0 = col_blocks(a.g, col_rows<false>()), cg1 = col_blocks(a.g, col_rows<true>());
    const bool w = a.g.walls != 0, rg = a.k.glat != 0;
    if (part == 0) {
        const dim3 mgrd(moments_grid<L, T>(a.g), 1, 1);
        if (rg) k_moments<L, T, true, true><<<mgrd, blk, 0, a.stream>>>(a.g, (const T*)a.src, a.rho_ref, a.rho, a.phi);
        else if (w) k_moments<L, T, true, false><<<mgrd, blk, 0, a.stream>>>(a.g, (const T*)a.src, a.rho_ref, a.rho, a.phi);
        else k_moments<L, T, false, false><<<mgrd, blk, 0, a.stream>>>(a.g, (const T*)a.src, a.rho_ref, a.rho, a.phi);
    } else if (part == 1) {
        if (L == kD3Q27) {
            if (w)
                k_chempot_col<false, E, true><<<cg0, cb0, 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mux, a.mup,
                                                                         nullptr, nullptr);
            else
                k_chempot_col<false, E, false><<<cg0, cb0, 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mux, a.mup,
                                                                          nullptr, nullptr);
        } else {
            if (w) k_chempot<L, E, true><<<grd, blk, 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mux, a.mup);
            else k_chempot<L, E, false><<<grd, blk, 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mux, a.mup);
        }
    } else if (part == 2) {
        // the pair split (D3Q27 FP32) runs the full phase-field lattice only
        if (rg && L == kD3Q27 && Deviation<T>::on) return hipErrorInvalidValue;
        if (a.diag && cgrd.x > a.partials_blocks) return hipErrorInvalidValue;
#define TELBM_COLLIDE(RGV, WV)                                                                                  \
    k_collide<L, T, RGV, WV><<<cgrd, blk, 0, a.stream>>>(a.g, a.k, (const T*)a.src, (T*)a.dst, a.rho_ref, a.rho,  \
                                                        a.phi, a.mux, a.mup, a.partials, a.diag)
        if (rg) TELBM_COLLIDE(true, false);
        else if constexpr (UsePairs<L, T>::value) {
            // the pair split has an instance with the wall logic (the one-node
            // collision checks walls at run time)
            if (w) TELBM_COLLIDE(false, true);
            else TELBM_COLLIDE(false, false);
        } else TELBM_COLLIDE(false, false);
#undef TELBM_COLLIDE
        if (a.diag) k_diag_final<<<1, 256, 0, a.stream>>>(a.partials, (int)cgrd.x, a.diag_out);
    } else if (part == 3) {
        if (L != kD2Q9 || a.g.nz != 1 || !a.rho_next || !a.phi_next || !a.inbox_out) return hipErrorInvalidValue;
        if (Deviation<T>::on != (a.rho_final != nullptr)) return hipErrorInvalidValue;
        const unsigned fb = fused_tiles(a.g);
        if (a.diag && fb > a.partials_blocks) return hipErrorInvalidValue;
#define TELBM_FUSED2(RGV, WV)                                                                                 \
    k_collide_fused2<T, E, RGV, WV><<<fb, dim3(BX, FBY, 1), 0, a.stream>>>(                                   \
        a.g, a.k, (const T*)a.src, (T*)a.dst, a.rho_ref, a.rho, a.phi, a.inbox_in, a.rho_next, a.phi_next,      \
        a.inbox_out, a.rho_final, a.partials, a.diag)
        if (rg && w) TELBM_FUSED2(true, true);
        else if (rg) TELBM_FUSED2(true, false);
        else if (w) TELBM_FUSED2(false, true);
        else TELBM_FUSED2(false, false);
#undef TELBM_FUSED2
        if (a.diag) k_diag_final<<<1, 256, 0, a.stream>>>(a.partials, (int)fb, a.diag_out);
    } else if (part == 5) {
        if (L != kD3Q27 || !a.part3 || !a.inbox3) return hipErrorInvalidValue;
        if (w)
            k_chempot_col<true, E, true><<<cg1, cb1, 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mux, a.mup,
                                                                    a.part3, a.inbox3);
        else
            k_chempot_col<true, E, false><<<cg1, cb1, 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mux, a.mup,
                                                                     a.part3, a.inbox3);
    } else if (part == 6) {
        if (L != kD3Q27 || Deviation<T>::on || !a.part3 || !a.inbox3) return hipErrorInvalidValue;
        auto* sp = (const double*)a.src;
        auto* dp = (double*)a.dst;
        const unsigned nb3 = column_blocks(a.g);
        if (a.diag && nb3 > a.partials_blocks) return hipErrorInvalidValue;
#define TELBM_NEXT3(WV, RGV, DV)                                                                               \
    k_collide_next3<WV, RGV, DV><<<nb3, blk, 0, a.stream>>>(a.g, a.k, sp, dp, a.rho, a.phi, a.mux, a.mup, a.part3, \
                                                            a.inbox3, a.partials, a.diag)
        if (a.diag) {
            if (w && rg) TELBM_NEXT3(true, true, true);
            else if (w) TELBM_NEXT3(true, false, true);
            else if (rg) TELBM_NEXT3(false, true, true);
            else TELBM_NEXT3(false, false, true);
        } else {
            if (w && rg) TELBM_NEXT3(true, true, false);
            else if (w) TELBM_NEXT3(true, false, false);
            else if (rg) TELBM_NEXT3(false, true, false);
            else TELBM_NEXT3(false, false, false);
        }
#undef TELBM_NEXT3
        if (a.diag) k_diag_final<<<1, 256, 0, a.stream>>>(a.partials, (int)nb3, a.diag_out);
    } else if (part == 4) {
        if (L != kD2Q9 || a.g.nz != 1 || !a.inbox_in) return hipErrorInvalidValue;
        k_dens_complete2<<<fused_tiles(a.g), FIX_THREADS, 0, a.stream>>>(a.g, a.rho, a.phi, a.inbox_in);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int E>
static hipError_t launch_part_e(int lattice, int precision, const StepArgs& a, int part) {
    if (lattice == kD2Q9)
        return precision ? launch_step_parts<kD2Q9, float, E>(a, part) : launch_step_parts<kD2Q9, double, E>(a, part);
    return precision ? launch_step_parts<kD3Q27, float, E>(a, part) : launch_step_parts<kD3Q27, double, E>(a, part);
}

hipError_t launch_part(int lattice, int precision, const StepArgs& a, int part) {
    switch (a.k.eos) {
        case 0: return launch_part_e<0>(lattice, precision, a, part);
        case 1: return launch_part_e<1>(lattice, precision, a, part);
        case 2: return launch_part_e<2>(lattice, precision, a, part);
        default: return hipErrorInvalidValue;
    }
}

template <int L, typename T>
static hipError_t launch_init_t(const StepArgs& a, const double* u0) {
    if (a.k.glat)
        k_init<L, T, true><<<grid_blocks(a.g), dim3(BX, BY, 1), 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mup, u0,
                                                                               (T*)a.dst);
    else
        k_init<L, T, false><<<grid_blocks(a.g), dim3(BX, BY, 1), 0, a.stream>>>(a.g, a.k, a.rho, a.phi, a.mup, u0,
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
