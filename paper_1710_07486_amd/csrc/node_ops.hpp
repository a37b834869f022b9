// node_ops.hpp -- the per-node bodies of the three phases of a time step,
// shared by the single-lattice kernels (kernels.hip) and the batched
// persistent kernels (batch.hip).  Each body handles the node (x, y, z) of
// one periodic lattice described by GridDims / PhysConst and raw pointers.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.hpp"
#include "lattice.hpp"

namespace telbm {

// FP32 populations are deviations from w_i times the writer's density; FP64
// populations are absolute.
template <typename T>
struct Deviation {
    static constexpr bool on = false;
};
template <>
struct Deviation<float> {
    static constexpr bool on = true;
};

__device__ __forceinline__ int64_t node_index(const GridDims& g, int x, int y, int z) {
    return ((int64_t)z * g.ny + y) * g.nx + x;
}

// Solid walls at y = -1/2 and y = ny - 1/2 (g.walls).  A population whose
// pull source x - c_i lies beyond a wall comes back from the node's own slot
// of -c_i (halfway bounce-back); bounce(g, y, cy) says so for c_y = cy.
__device__ __forceinline__ bool bounce(const GridDims& g, int y, int cy) {
    return g.walls && ((cy > 0 && y == 0) || (cy < 0 && y == g.ny - 1));
}
// Stencil neighbour y + cy beyond a wall.
__device__ __forceinline__ bool beyond_wall(const GridDims& g, int y, int cy) {
    return g.walls && ((cy < 0 && y == 0) || (cy > 0 && y == g.ny - 1));
}

// Neighbour offsets that repeat the wall row beyond a wall (the ghost rule of
// the chemical potentials); periodic elsewhere.
__device__ __forceinline__ Nbr make_nbr_w(const GridDims& g, int x, int y, int z) {
    Nbr n = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    if (g.walls) {
        if (y == 0) n.oy[0] = 0;
        if (y == g.ny - 1) n.oy[2] = 0;
    }
    return n;
}

// Wetting ghosts of rho and phi beyond the wall next to the wall-row node
// (xw, yw, zw) (top: the wall at y = ny - 1/2).
template <int L>
__device__ __forceinline__ void wall_ghosts(const GridDims& g, const PhysConst& k, const double* __restrict__ rho,
                                            const double* __restrict__ phi, int xw, int yw, int zw, int top,
                                            double& gr, double& gp) {
    const int64_t c = node_index(g, xw, yw, zw);
    const int64_t ep = node_index(g, xw + 1 == g.nx ? 0 : xw + 1, yw, zw);
    const int64_t em = node_index(g, xw == 0 ? g.nx - 1 : xw - 1, yw, zw);
    const double rx = 0.5 * (rho[ep] - rho[em]), px = 0.5 * (phi[ep] - phi[em]);
    double rz = 0.0, pz = 0.0;
    if (Lattice<L>::D == 3) {
        const int64_t zp = node_index(g, xw, yw, zw + 1 == g.nz ? 0 : zw + 1);
        const int64_t zm = node_index(g, xw, yw, zw == 0 ? g.nz - 1 : zw - 1);
        rz = 0.5 * (rho[zp] - rho[zm]);
        pz = 0.5 * (phi[zp] - phi[zm]);
    }
    gr = wet_ghost(rho[c], rx, rz, k.cot_rho[top]);
    gp = wet_ghost(phi[c], px, pz, k.cot_phi[top]);
}

// Phase 1: rho = sum_i f_i, phi = sum_i g_i of the pulled populations, FP64
// accumulation.  rho_ref: densities the stored f values are relative to.
// W: the lattice may have walls (kernels instantiated without them carry none
// of the wall logic).
template <int L, typename T, bool W = false, bool RG = false>
__device__ __forceinline__ void node_moments(const GridDims& g, const T* __restrict__ pop,
                                             const double* __restrict__ rho_ref, double* __restrict__ rho,
                                             double* __restrict__ phi, int x, int y, int z) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    const int64_t n = node_index(g, x, y, z);
    double r = 0.0, p = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const bool bb = W && bounce(g, y, Lt::c[i][1]);
        const int64_t m = bb ? n : n + nbr_off<L>(nb, i, -1);
        const int s = bb ? opp_dir(i) : i;
        double fi = double(pop[(int64_t)s * g.N + m]);
        if (Deviation<T>::on) fi += Lt::w[i] * rho_ref[m];
        r += fi;
        if (i < GLattice<L, RG>::Q) p += double(pop[(int64_t)(Q + s) * g.N + m]);
    }
    rho[n] = r;
    phi[n] = p;
}

// Phase 2: chemical potentials with the lattice Laplacians
// lap psi(x) = 6 sum_i w_i [psi(x + c_i) - psi(x)].
template <int L, int E, bool W = false>
__device__ __forceinline__ void node_chempot(const GridDims& g, const PhysConst& k, const double* __restrict__ rho,
                                             const double* __restrict__ phi, double* __restrict__ mux,
                                             double* __restrict__ mup, int x, int y, int z) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    const Nbr nb = make_nbr(x, y, z, g.nx, g.ny, g.nz);
    const int64_t n = node_index(g, x, y, z);
    const double r0 = rho[n], p0 = phi[n];
    double lr = 0.0, lp = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        double rm, pm;
        if (W && beyond_wall(g, y, Lt::c[i][1])) {
            const int xw = x + Lt::c[i][0], zw = z + Lt::c[i][2];
            wall_ghosts<L>(g, k, rho, phi, xw < 0 ? g.nx - 1 : (xw == g.nx ? 0 : xw), y,
                           zw < 0 ? g.nz - 1 : (zw == g.nz ? 0 : zw), y != 0, rm, pm);
        } else {
            const int64_t m = n + nbr_off<L>(nb, i, +1);
            rm = rho[m];
            pm = phi[m];
        }
        lr += Lt::w[i] * (rm - r0);
        lp += Lt::w[i] * (pm - p0);
    }
    double mx, mp;
    chem_pot<E>(k, r0, p0, 6.0 * lr, 6.0 * lp, &mx, &mp);
    mux[n] = mx;
    mup[n] = mp;
}

// Isotropic gradient grad psi(x) = 3 sum_i w_i c_i psi(x + c_i) of two fields.
template <int L>
__device__ __forceinline__ void gradient2(const Nbr& nb, int64_t n, const double* __restrict__ a,
                                          const double* __restrict__ b, double* ga, double* gb) {
    using Lt = Lattice<L>;
    constexpr int Q = Lt::Q;
    ga[0] = ga[1] = ga[2] = 0.0;
    gb[0] = gb[1] = gb[2] = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int64_t m = n + nbr_off<L>(nb, i, +1);
        const double va = Lt::w[i] * a[m], vb = Lt::w[i] * b[m];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (Lt::c[i][d] > 0) {
                ga[d] += va;
                gb[d] += vb;
            } else if (Lt::c[i][d] < 0) {
                ga[d] -= va;
                gb[d] -= vb;
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ga[d] *= 3.0;
        gb[d] *= 3.0;
    }
}

// Compiler fence between the sub-phases of the collision kernel: memory
// operations are not moved across it, so the loads of one sub-phase are not
// hoisted into the live range of the previous one.
__device__ __forceinline__ void phase_fence() { asm volatile("" ::: "memory"); }

// 32-bit periodic neighbour offsets (node counts below 2^31 per lattice): the
// pulls then address a uniform per-direction base plus a 32-bit lane offset.
struct Nbr32 {
    int32_t ox[3], oy[3], oz[3];
};

__device__ __forceinline__ Nbr32 make_nbr32(int x, int y, int z, int nx, int ny, int nz) {
    Nbr32 n;
    const int32_t sy = nx, sz = nx * ny;
    n.ox[1] = 0;
    n.ox[0] = x == 0 ? nx - 1 : -1;
    n.ox[2] = x == nx - 1 ? -(nx - 1) : 1;
    n.oy[1] = 0;
    n.oy[0] = (y == 0 ? ny - 1 : -1) * sy;
    n.oy[2] = (y == ny - 1 ? -(ny - 1) : 1) * sy;
    n.oz[1] = 0;
    n.oz[0] = (z == 0 ? nz - 1 : -1) * sz;
    n.oz[2] = (z == nz - 1 ? -(nz - 1) : 1) * sz;
    return n;
}

// The same with the wall row repeated beyond a wall (walls set): potentials
// read there take the ghost rule of the chemical potentials, and the pulls of
// bounced directions address the node's own row (read from the slot of -c_i).
__device__ __forceinline__ Nbr32 make_nbr32_w(const GridDims& g, int x, int y, int z) {
    Nbr32 n = make_nbr32(x, y, z, g.nx, g.ny, g.nz);
    if (g.walls) {
        if (y == 0) n.oy[0] = 0;
        if (y == g.ny - 1) n.oy[2] = 0;
    }
    return n;
}

template <int L>
__device__ __forceinline__ uint32_t nbr32(const Nbr32& nb, uint32_t n, int i, int sign) {
    using Lt = Lattice<L>;
    return n + nb.ox[1 + sign * Lt::c[i][0]] + nb.oy[1 + sign * Lt::c[i][1]] + nb.oz[1 + sign * Lt::c[i][2]];
}

// Element m of the array at `base`, addressed as a uniform base plus a 32-bit
// byte offset (the host guarantees every per-direction slice is < 4 GiB), so
// that the load takes its base from scalar registers.
template <typename T>
__device__ __forceinline__ T ld(const T* __restrict__ base, uint32_t m) {
    return *(const T*)((const char*)base + (uint32_t)(m * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st(T* __restrict__ base, uint32_t m, T v) {
    *(T*)((char*)base + (uint32_t)(m * (uint32_t)sizeof(T))) = v;
}

// Population traffic of the collision.  On D3Q27 the populations (7 GB per
// copy at 256^3 in FP64) stream through once per step, far beyond the L2 and
// the 256 MB last-level cache: non-temporal hints keep them from evicting the
// stencil fields (measured: collision 3.65 -> 3.39 ms at 256^3 FP64).  A 2D
// lattice of a million nodes fits in the last-level cache between the moments
// and collision passes, so there the hints would cost (measured: 2D step
// 91 -> 98 us).
template <int L>
struct StreamPops {
    static constexpr bool value = (L == kD3Q27);
};
template <int L, typename T>
__device__ __forceinline__ T ld_pop(const T* __restrict__ base, uint32_t m) {
    const T* a = (const T*)((const char*)base + (uint32_t)(m * (uint32_t)sizeof(T)));
    if (StreamPops<L>::value) return __builtin_nontemporal_load(a);
    return *a;
}
template <int L, typename T>
__device__ __forceinline__ void st_pop(T* __restrict__ base, uint32_t m, T v) {
    T* a = (T*)((char*)base + (uint32_t)(m * (uint32_t)sizeof(T)));
    if (StreamPops<L>::value) __builtin_nontemporal_store(v, a);
    else *a = v;
}

// Where the collision reads its node's density, phase field and mu_phi, and
// the potentials of its neighbours for the force: the aux fields in global
// memory (GlobalAux) or a workgroup's LDS tile (the fused 2D step).
struct GlobalAux {
    const double* __restrict__ rho;
    const double* __restrict__ phi;
    const double* __restrict__ mux;
    const double* __restrict__ mup;
    __device__ __forceinline__ double rho0(uint32_t n) const { return ld(rho, n); }
    __device__ __forceinline__ double phi0(uint32_t n) const { return ld(phi, n); }
    __device__ __forceinline__ double mup0(uint32_t n) const { return ld(mup, n); }
    template <int L>
    __device__ __forceinline__ void nbr_mu(const Nbr32& nb, uint32_t n, int i, double& a, double& b) const {
        const uint32_t m = nbr32<L>(nb, n, i, +1);
        a = ld(mux, m);
        b = ld(mup, m);
    }
    // reference density of the pull source of direction i (FP32 form)
    template <int L>
    __device__ __forceinline__ double ref(const double* rho_ref, const Nbr32& nb, uint32_t n, int i, bool bb) const {
        return ld(rho_ref, bb ? n : nbr32<L>(nb, n, i, -1));
    }
};

// Receiver of a node's post-collision populations, called right after they
// are stored (post_f with the node's density, post_g).  NoSink: none.
struct NoSink {
    template <int L, typename R>
    __device__ __forceinline__ void post_f(const R*, double) {}
    template <int L, typename R, int QG>
    __device__ __forceinline__ void post_g(const R*) {}
};

// Where the collision takes the phase-field populations it pulls: global
// memory (NoGPrefetch), or a policy with on = true whose pulled(i) returns
// direction i of the node (the z-column collision stages them in LDS ahead
// of the plane).
struct NoGPrefetch {
    static constexpr bool on = false;
    __device__ __forceinline__ double pulled(int) const { return 0.0; }
};

// Adds one node's diagnostics to a thread's running values over the nodes it
// has collided (the collisions below merge, so that a thread may collide any
// number of nodes): sums of mass, phase field and momentum, the largest
// speed, the smallest density, the range of the stabiliser and the count of
// non-finite nodes.  A thread starts from {0, 0, 0, 0, 0, 0, +inf, +inf,
// -inf, 0}.
__device__ __forceinline__ void diag_merge(double* dv, const double* d1) {
    for (int v = 0; v < 5; ++v) dv[v] += d1[v];
    dv[5] = fmax(dv[5], d1[5]);
    dv[6] = fmin(dv[6], d1[6]);
    dv[7] = fmin(dv[7], d1[7]);
    dv[8] = fmax(dv[8], d1[8]);
    dv[9] += d1[9];
}

// Phase 3: pull f, g; force from the excess potentials; KBC with
// exact-difference forcing; phase-field BGK; write the node's own slots.
// If diag, the node's {rho, phi, j (3), |u_phys|, rho, gamma, gamma, bad} are
// merged into dv (diag_merge).
// The three sub-phases (stencil, f, g) are kept apart by scheduling barriers
// so that their loads do not all become live at once.  With active false the
// node is computed but nothing is stored or reported (lanes past a ragged
// edge that run on a clamped node so that the sink sees a full wavefront).
// W false: the lattice has no walls (the kernel carries none of their logic).
// RG: the phase field lives on the reduced lattice (GLattice).  GPF: where
// the pulled phase-field populations come from (a staging policy holds them
// with the bounce-back of bounced directions applied; FP64 only).
template <int L, typename T, typename AUX, typename SINK, bool W = true, bool RG = false,
          typename GPF = NoGPrefetch>
__device__ __forceinline__ void node_collide_sink(const GridDims& g, const PhysConst& k, const T* __restrict__ src,
                                                  T* __restrict__ dst, const double* __restrict__ rho_ref,
                                                  const AUX& aux, int x, int y, int z, bool diag, double* dv,
                                                  bool active, SINK& sink, const GPF& gpf = GPF{}) {
    static_assert(!GPF::on || sizeof(T) == 8, "staged phase-field pulls: FP64");
    using Lt = Lattice<L>;
    using R = T;
    constexpr int Q = Lt::Q;
    const Nbr32 nb = W ? make_nbr32_w(g, x, y, z) : make_nbr32(x, y, z, g.nx, g.ny, g.nz);
    const uint32_t n = (uint32_t)node_index(g, x, y, z);
    const double r = aux.rho0(n), p = aux.phi0(n);
    // mu_phi of the node (for the phase-field collision), with its other
    // fields: loaded later, its wait could also cover a staging policy's loads
    const double mphi = aux.mup0(n);

    // force from the isotropic gradients of the two potentials
    double gx[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        double ma, mb;
        aux.template nbr_mu<L>(nb, n, i, ma, mb);
        const double va = Lt::w[i] * ma, vb = Lt::w[i] * mb;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (Lt::c[i][d] > 0) {
                gx[d] += va;
                gp[d] += vb;
            } else if (Lt::c[i][d] < 0) {
                gx[d] -= va;
                gp[d] -= vb;
            }
        }
    }
    double F[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = -r * 3.0 * gx[d] - p * 3.0 * gp[d];
    phase_fence();

    // pull f (offset form about this node's density in the FP32 form)
    R f[Q];
    R jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // a bounced direction reads the node's own slot of -c_i (its address
        // below is the node itself: the wall row repeats beyond the wall)
        const bool bb = W && bounce(g, y, Lt::c[i][1]);
        const uint32_t m = nbr32<L>(nb, n, i, -1);
        R v = bb ? ld_pop<L>(src + (size_t)opp_dir(i) * g.N, n) : ld_pop<L>(src + (size_t)i * g.N, m);
        if (Deviation<T>::on) v += R(Lt::w[i] * (aux.template ref<L>(rho_ref, nb, n, i, bb) - r));
        f[i] = v;
        if (Lt::c[i][0]) jx += Lt::c[i][0] > 0 ? v : -v;
        if (Lt::c[i][1]) jy += Lt::c[i][1] > 0 ? v : -v;
        if (Lt::c[i][2]) jz += Lt::c[i][2] > 0 ? v : -v;
    }
    const double ir = 1.0 / r;
    R u[3] = {R(double(jx) * ir), R(double(jy) * ir), R(double(jz) * ir)};
    R du[3] = {R(F[0] * ir), R(F[1] * ir), R(F[2] * ir)};
    if (Lt::D == 2) u[2] = du[2] = R(0);
    const double gam = collide_f<L, R>(f, r, ir, u, du, R(k.beta), k.inv_beta, Deviation<T>::on ? r : 0.0);
    if (active) {
#pragma unroll
        for (int i = 0; i < Q; ++i) st_pop<L>(dst + (size_t)i * g.N, n, f[i]);
    }
    sink.template post_f<L, R>(f, r);
    phase_fence();

    constexpr int QG = GLattice<L, RG>::Q;
    R gg[QG];
    if constexpr (GPF::on) {
#pragma unroll
        for (int i = 0; i < QG; ++i) gg[i] = R(gpf.pulled(i));
    } else {
#pragma unroll
        for (int i = 0; i < QG; ++i)
            gg[i] = (W && bounce(g, y, Lt::c[i][1])) ? ld_pop<L>(src + (size_t)(Q + opp_dir(i)) * g.N, n)
                                              : ld_pop<L>(src + (size_t)(Q + i) * g.N, nbr32<L>(nb, n, i, -1));
    }
    R up[3] = {u[0] + R(0.5) * du[0], u[1] + R(0.5) * du[1], u[2] + R(0.5) * du[2]};
    collide_g_lat<L, R, RG>(gg, R(p), R(mphi), up, R(k.Gamma), R(k.omega_phi));
    if (active) {
#pragma unroll
        for (int i = 0; i < QG; ++i) st_pop<L>(dst + (size_t)(Q + i) * g.N, n, gg[i]);
    }
    sink.template post_g<L, R, QG>(gg);

    if (diag && active) {
        const double ux = double(jx) * ir + 0.5 * F[0] * ir;
        const double uy = double(jy) * ir + 0.5 * F[1] * ir;
        const double uz = double(jz) * ir + 0.5 * F[2] * ir;
        const double um = sqrt(ux * ux + uy * uy + uz * uz);
        const bool bad = !(isfinite(r) && isfinite(p) && isfinite(um)) || !(r > 0.0);
        const double d1[kDiag] = {r, p, double(jx), double(jy), double(jz), bad ? INFINITY : um,
                                  r, gam, gam, bad ? 1.0 : 0.0};
        diag_merge(dv, d1);
    }
}

template <int L, typename T, typename AUX, bool RG = false>
__device__ __forceinline__ void node_collide_aux(const GridDims& g, const PhysConst& k, const T* __restrict__ src,
                                                 T* __restrict__ dst, const double* __restrict__ rho_ref,
                                                 const AUX& aux, int x, int y, int z, bool diag, double* dv) {
    NoSink none;
    node_collide_sink<L, T, AUX, NoSink, true, RG>(g, k, src, dst, rho_ref, aux, x, y, z, diag, dv, true, none);
}

template <int L, typename T, bool RG = false>
__device__ __forceinline__ void node_collide(const GridDims& g, const PhysConst& k, const T* __restrict__ src,
                                             T* __restrict__ dst, const double* __restrict__ rho_ref,
                                             const double* __restrict__ rho, const double* __restrict__ phi,
                                             const double* __restrict__ mux, const double* __restrict__ mup,
                                             int x, int y, int z, bool diag, double* dv) {
    const GlobalAux aux{rho, phi, mux, mup};
    node_collide_aux<L, T, GlobalAux, RG>(g, k, src, dst, rho_ref, aux, x, y, z, diag, dv);
}

// ---------------------------------------------------------------------------
// Collision with the work of one node split over two lanes l and l ^ 32 of a
// wavefront.  The directions come in opposite pairs (2p-1, 2p) = (c, -c);
// side A (lanes 0-31) takes c_{2p-1} and the rest population, side B (lanes
// 32-63) takes c_{2p}.  Side B works in the mirrored frame x -> -x: the
// entropic factors satisfy psi_-(u) = psi_+(-u) and the phase-field
// equilibrium is even in (c, u) -> (-c, -u), so side B runs the same
// instructions with u -> -u on the opposite populations.  Odd partial sums
// (momentum, gradients) combine as A - B, even ones (second moments, the
// entropic scalar products) as A + B, each with one cross-half exchange.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double xhalf(double v) { return __shfl_xor(v, 32); }
__device__ __forceinline__ float xhalf(float v) { return __shfl_xor(v, 32); }

// W: the lattice may have walls (halfway bounce-back as in node_collide_sink:
// a pull whose source lies beyond a wall reads the node's own slot of the
// opposite direction; the potentials beyond a wall repeat the wall row).
template <int L, typename T, bool W = false>
__device__ __forceinline__ void node_collide_pair(const GridDims& g, const PhysConst& k, const T* __restrict__ src,
                                                  T* __restrict__ dst, const double* __restrict__ rho_ref,
                                                  const double* __restrict__ rho, const double* __restrict__ phi,
                                                  const double* __restrict__ mux, const double* __restrict__ mup,
                                                  int x, int y, int z, int side, bool diag, double* dv) {
    using Lt = Lattice<L>;
    using R = T;
    constexpr int Q = Lt::Q;
    constexpr int NP = (Q - 1) / 2;
    constexpr int D = Lt::D;
    const bool B = side != 0;
    Nbr32 nb = W ? make_nbr32_w(g, x, y, z) : make_nbr32(x, y, z, g.nx, g.ny, g.nz);
    if (B) {  // this side's frame is mirrored: +c here is -c on the lattice
        int32_t t;
        t = nb.ox[0]; nb.ox[0] = nb.ox[2]; nb.ox[2] = t;
        t = nb.oy[0]; nb.oy[0] = nb.oy[2]; nb.oy[2] = t;
        t = nb.oz[0]; nb.oz[0] = nb.oz[2]; nb.oz[2] = t;
    }
    const uint32_t n = (uint32_t)node_index(g, x, y, z);
    const uint32_t soff = B ? (uint32_t)g.N : 0u;  // side B addresses direction 2p, the next array
    const double r = ld(rho, n), p = ld(phi, n);

    // gradients of the two potentials (frame components)
    double gx[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
#pragma unroll
    for (int q = 1; q <= NP; ++q) {
        const int i = 2 * q - 1;
        const uint32_t m = nbr32<L>(nb, n, i, +1);
        const double va = Lt::w[i] * ld(mux, m), vb = Lt::w[i] * ld(mup, m);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (Lt::c[i][d] > 0) {
                gx[d] += va;
                gp[d] += vb;
            } else if (Lt::c[i][d] < 0) {
                gx[d] -= va;
                gp[d] -= vb;
            }
        }
    }
    double F[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double ga = 3.0 * (gx[d] - xhalf(gx[d]));
        const double gb = 3.0 * (gp[d] - xhalf(gp[d]));
        F[d] = -r * ga - p * gb;
    }
    phase_fence();

    // pull f: side A directions 2p-1 at x - c, side B directions 2p at x + c
    R f[NP];
    R f0 = ld_pop<L>(src, n);
    if (Deviation<T>::on) f0 += R(Lt::w[0] * (ld(rho_ref, n) - r));
    R jx = 0, jy = 0, jz = 0;
    double P[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int q = 1; q <= NP; ++q) {
        const int i = 2 * q - 1;
        const uint32_t m = nbr32<L>(nb, n, i, -1);
        // this side's lattice direction is c_i (A) or -c_i (B); bounced, it
        // reads the node's own slot of the other one
        const bool bb = W && bounce(g, y, B ? -Lt::c[i][1] : Lt::c[i][1]);
        R v = bb ? ld_pop<L>(src + (size_t)i * g.N, (B ? 0u : (uint32_t)g.N) + n)
                 : ld_pop<L>(src + (size_t)i * g.N, soff + m);
        if (Deviation<T>::on) v += R(Lt::w[i] * (ld(rho_ref, bb ? n : m) - r));
        f[q - 1] = v;
        const int cx = Lt::c[i][0], cy = Lt::c[i][1], cz = Lt::c[i][2];
        if (cx) jx += cx > 0 ? v : -v;
        if (cy) jy += cy > 0 ? v : -v;
        if (cz) jz += cz > 0 ? v : -v;
        const double fd = double(v);
        if (cx) P[0] += fd;
        if (cy) P[1] += fd;
        if (cz) P[2] += fd;
        if (cx * cy) P[3] += cx * cy > 0 ? fd : -fd;
        if (cx * cz) P[4] += cx * cz > 0 ? fd : -fd;
        if (cy * cz) P[5] += cy * cz > 0 ? fd : -fd;
    }
    jx = jx - xhalf(jx);
    jy = jy - xhalf(jy);
    jz = jz - xhalf(jz);
#pragma unroll
    for (int a = 0; a < 6; ++a) P[a] += xhalf(P[a]);
    const double ir = 1.0 / r;
    R u[3] = {R(double(jx) * ir), R(double(jy) * ir), R(double(jz) * ir)};
    R du[3] = {R(F[0] * ir), R(F[1] * ir), R(F[2] * ir)};
    if (D == 2) u[2] = du[2] = R(0);

    // KBC with exact-difference forcing (see collide_f in lattice.hpp)
    const R rr = R(r);
    const double rho_off = Deviation<T>::on ? r : 0.0;
    const R drho = R(r - rho_off);
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
    double mm[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double sm1 = a < D ? double(-ax[a].e[0]) : 0.0;  // S_a - 1
        mm[a] = P[a] - (2.0 * r * sm1 + (r - rho_off)) * (1.0 / 3.0);
    }
    mm[3] = P[3] - r * double(u[0]) * double(u[1]);
    mm[4] = P[4] - r * double(u[0]) * double(u[2]);
    mm[5] = P[5] - r * double(u[1]) * double(u[2]);
    R dxx, dyy, dzz;
    if (D == 2) {
        dxx = R(0.5 * (mm[0] - mm[1]));
        dyy = -dxx;
        dzz = 0;
    } else {
        const double tr = (mm[0] + mm[1] + mm[2]) * (1.0 / 3.0);
        dxx = R(mm[0] - tr);
        dyy = R(mm[1] - tr);
        dzz = R(mm[2] - tr);
    }
    const R mxy = R(mm[3]), mxz = R(mm[4]), myz = R(mm[5]);
    auto shear = [&](int i) -> R {
        const int cx = Lt::c[i][0], cy = Lt::c[i][1], cz = Lt::c[i][2];
        const int nzc = (cx != 0) + (cy != 0) + (cz != 0);
        if (nzc == 1) return R(0.5) * (cx ? dxx : (cy ? dyy : dzz));
        if (nzc == 2) {
            if (!cz) return R(0.25 * cx * cy) * mxy;
            if (!cy) return R(0.25 * cx * cz) * mxz;
            return R(0.25 * cy * cz) * myz;
        }
        if (nzc == 0) return -(dxx + dyy + dzz);
        return R(0);
    };
    const R inv_rho = R(ir);
    double sh = 0.0, hh = 0.0;
#pragma unroll
    for (int q = 1; q <= NP; ++q) {
        const int i = 2 * q - 1;
        const R s = shear(i);
        const R dh = f[q - 1] - R(Lt::w[i]) * (drho + rr * eq_excess<L, R>(ax, i)) - s;
        f[q - 1] = dh;
        const double ifeq = double(inv_rho * eq_inv<L, R>(ax, i));
        sh += double(s) * double(dh) * ifeq;
        hh += double(dh) * double(dh) * ifeq;
    }
    const R s0 = shear(0);
    const R dh0 = f0 - R(Lt::w[0]) * (drho + rr * eq_excess<L, R>(ax, 0)) - s0;
    if (!B) {
        const double ifeq0 = double(inv_rho * eq_inv<L, R>(ax, 0));
        sh += double(s0) * double(dh0) * ifeq0;
        hh += double(dh0) * double(dh0) * ifeq0;
    }
    sh += xhalf(sh);
    hh += xhalf(hh);
    const double gam = (hh > 1e-300) ? (k.inv_beta - (2.0 - k.inv_beta) * sh / hh) : 2.0;
    const R beta = R(k.beta);
    const R cs = R(1) - R(2) * beta, ch = R(1) - beta * R(gam);
#pragma unroll
    for (int q = 1; q <= NP; ++q) {
        const int i = 2 * q - 1;
        const R v = cs * shear(i) + ch * f[q - 1] + R(Lt::w[i]) * (drho + rr * eq_excess<L, R>(ax2, i));
        st_pop<L>(dst + (size_t)i * g.N, soff + n, v);
    }
    if (!B) st_pop<L>(dst, n, cs * s0 + ch * dh0 + R(Lt::w[0]) * (drho + rr * eq_excess<L, R>(ax2, 0)));
    phase_fence();

    // phase-field BGK on the same split (geq is even in (c, u) -> (-c, -u))
    R up[3] = {u[0] + R(0.5) * du[0], u[1] + R(0.5) * du[1], u[2] + R(0.5) * du[2]};
    const R ph = R(p), om = R(k.omega_phi);
    const R uu = up[0] * up[0] + up[1] * up[1] + up[2] * up[2];
    const R base = R(3) * R(k.Gamma) * R(ld(mup, n)) - R(1.5) * ph * uu;
#pragma unroll
    for (int q = 1; q <= NP; ++q) {
        const int i = 2 * q - 1;
        const bool bb = W && bounce(g, y, B ? -Lt::c[i][1] : Lt::c[i][1]);
        const R gi = bb ? ld_pop<L>(src + (size_t)(Q + i) * g.N, (B ? 0u : (uint32_t)g.N) + n)
                        : ld_pop<L>(src + (size_t)(Q + i) * g.N, soff + nbr32<L>(nb, n, i, -1));
        const R cu = R(Lt::c[i][0]) * up[0] + R(Lt::c[i][1]) * up[1] + R(Lt::c[i][2]) * up[2];
        const R geq = R(Lt::w[i]) * (base + R(3) * ph * cu + R(4.5) * ph * cu * cu);
        st_pop<L>(dst + (size_t)(Q + i) * g.N, soff + n, gi + om * (geq - gi));
    }
    if (!B) {
        const R g0 = ld_pop<L>(src + (size_t)Q * g.N, n);
        const R geq0 = ph - R(1.0 - Lt::w[0]) * base - R(1.5) * ph * uu;
        st_pop<L>(dst + (size_t)Q * g.N, n, g0 + om * (geq0 - g0));
    }

    if (diag && !B) {
        const double ux = double(jx) * ir + 0.5 * F[0] * ir;
        const double uy = double(jy) * ir + 0.5 * F[1] * ir;
        const double uz = double(jz) * ir + 0.5 * F[2] * ir;
        const double um = sqrt(ux * ux + uy * uy + uz * uz);
        const bool bad = !(isfinite(r) && isfinite(p) && isfinite(um)) || !(r > 0.0);
        const double d1[kDiag] = {r, p, double(jx), double(jy), double(jz), bad ? INFINITY : um,
                                  r, gam, gam, bad ? 1.0 : 0.0};
        diag_merge(dv, d1);
    }
}

// All nodes of a tile of TW x TH nodes at (x0, y0, z), processed by a block
// of NT threads with the two sides of each node on lanes l and l ^ 32.
template <int L, typename T, int NT, bool W = false>
__device__ __forceinline__ void tile_collide_pair(const GridDims& g, const PhysConst& k, const T* __restrict__ src,
                                                  T* __restrict__ dst, const double* __restrict__ rho_ref,
                                                  const double* __restrict__ rho, const double* __restrict__ phi,
                                                  const double* __restrict__ mux, const double* __restrict__ mup,
                                                  int x0, int y0, int z, int TW, int TH, int tid, bool diag,
                                                  double* dv) {
    const int lane = tid & 63, wave = tid >> 6;
    const int side = lane >> 5;
    for (int base = 0; base < TW * TH; base += NT / 2) {
        const int kk = base + wave * 32 + (lane & 31);
        const int x = x0 + kk % TW, y = y0 + kk / TW;
        if (kk < TW * TH && x < g.nx && y < g.ny && z < g.nz) {
            node_collide_pair<L, T, W>(g, k, src, dst, rho_ref, rho, phi, mux, mup, x, y, z, side, diag, dv);
        }
    }
}

// Whether the collision of this lattice and storage type runs two lanes per
// node (pair split) or one: the split halves the per-lane registers but
// repeats the per-node square roots and reciprocals on both halves, which pays
// off where registers limit occupancy most (D3Q27 with FP32 storage).
template <int L, typename T>
struct UsePairs {
    static constexpr bool value = (L == kD3Q27) && Deviation<T>::on;
};

// All nodes of a tile of TW x TH nodes at (x0, y0, z) with the block's NT
// threads, in the collision form UsePairs selects.
// RG: reduced phase-field lattice (one node per lane; the pair split runs the
// full lattice only).
template <int L, typename T, int NT, bool RG = false, bool W = false>
__device__ __forceinline__ void tile_collide(const GridDims& g, const PhysConst& k, const T* __restrict__ src,
                                             T* __restrict__ dst, const double* __restrict__ rho_ref,
                                             const double* __restrict__ rho, const double* __restrict__ phi,
                                             const double* __restrict__ mux, const double* __restrict__ mup,
                                             int x0, int y0, int z, int TW, int TH, int tid, bool diag, double* dv) {
    if constexpr (UsePairs<L, T>::value && !RG) {
        tile_collide_pair<L, T, NT, W>(g, k, src, dst, rho_ref, rho, phi, mux, mup, x0, y0, z, TW, TH, tid, diag, dv);
        return;
    }
    for (int kk = tid; kk < TW * TH; kk += NT) {
        const int x = x0 + kk % TW, y = y0 + kk / TW;
        if (x < g.nx && y < g.ny && z < g.nz)
            node_collide<L, T, RG>(g, k, src, dst, rho_ref, rho, phi, mux, mup, x, y, z, diag, dv);
    }
}

}  // namespace telbm
