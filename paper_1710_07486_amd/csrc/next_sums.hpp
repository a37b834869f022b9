// next_sums.hpp -- tiling constants and the next-step moment sums that a
// collision leaves for the following step (the tile sums of NextSink, the
// per-plane partial sums and the inboxes of the neighbouring tiles), shared by
// the two-liquid kernels (kernels.hip) and the three-liquid ones (nliquid.hip).
#pragma once

#include <hip/hip_runtime.h>
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

__device__ __forceinline__ int wrap_any(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Inbox of a BX x TH tile: sums of next-step moments that neighbouring tiles
// hold for its edge nodes, (rho, phi) pairs.  Slots: bottom row from the tile
// below, top row from the tile above, left and right columns from the side
// tiles, then the four corners from the diagonal tiles (bottom-left,
// bottom-right, top-left, top-right).
template <int TH>
struct Inbox {
    static constexpr int DOWN = 0, UP = BX, LEFT = 2 * BX, RIGHT = 2 * BX + TH, CORNER = 2 * BX + 2 * TH;
    static constexpr int SIZE = CORNER + 4;
};

// Tile (of the BX x TH tiling of an x-y plane) of a node and its place in it.
struct TilePos {
    int tile, lx, ly, W, H;
};
template <int TH>
__device__ __forceinline__ TilePos tile_pos(const GridDims& g, int gx, int gy) {
    const int bxc = (g.nx + BX - 1) / BX;
    const int tbx = gx / BX, tby = gy / TH;
    TilePos t;
    t.tile = tby * bxc + tbx;
    t.lx = gx - tbx * BX;
    t.ly = gy - tby * TH;
    t.W = min(BX, g.nx - tbx * BX);
    t.H = min(TH, g.ny - tby * TH);
    return t;
}

// Add the inbox entries of node (gx, gy) to its tile's partial sums (r, p),
// in a fixed order.  `in` is the inbox array of the node's plane, NF fields
// per slot ((r, p) pairs, or r alone with NF = 1, p then untouched).
template <int TH, int NF = 2>
__device__ __forceinline__ void inbox_complete(const GridDims& g, const double* __restrict__ in, int gx, int gy,
                                               double& r, double& p) {
    using I = Inbox<TH>;
    const TilePos t = tile_pos<TH>(g, gx, gy);
    // a tile edge on a wall receives nothing from beyond it
    const bool x0 = t.lx == 0, x1 = t.lx == t.W - 1;
    const bool y0 = t.ly == 0 && !(g.walls && gy == 0), y1 = t.ly == t.H - 1 && !(g.walls && gy == g.ny - 1);
    if (!(x0 || x1 || y0 || y1)) return;
    const double* b = in + (int64_t)t.tile * I::SIZE * NF;
    auto add = [&](int slot) {
        r += b[NF * slot];
        if (NF == 2) p += b[NF * slot + 1];
    };
    if (y0) add(I::DOWN + t.lx);
    if (y1) add(I::UP + t.lx);
    if (x0) add(I::LEFT + t.ly);
    if (x1) add(I::RIGHT + t.ly);
    if (x0 && y0) add(I::CORNER + 0);
    if (x1 && y0) add(I::CORNER + 1);
    if (x0 && y1) add(I::CORNER + 2);
    if (x1 && y1) add(I::CORNER + 3);
}

// The same completion with the entries loaded together: a node of a tile at
// least two nodes wide and high has at most one entry from each of a vertical
// side, a horizontal side and a corner, taken in the order of inbox_complete;
// the three loads are issued unconditionally (a missing entry reads the
// tile's first slot and is not added).  Narrower tiles use inbox_complete.
template <int TH, int NF = 2>
__device__ __forceinline__ void inbox_complete_fast(const GridDims& g, const double* __restrict__ in, int gx,
                                                    int gy, double& r, double& p) {
    using I = Inbox<TH>;
    const TilePos t = tile_pos<TH>(g, gx, gy);
    const bool x0 = t.lx == 0, x1 = t.lx == t.W - 1;
    const bool y0 = t.ly == 0 && !(g.walls && gy == 0), y1 = t.ly == t.H - 1 && !(g.walls && gy == g.ny - 1);
    if (!(x0 || x1 || y0 || y1)) return;
    if (t.W < 2 || t.H < 2) {
        inbox_complete<TH, NF>(g, in, gx, gy, r, p);
        return;
    }
    const bool hv = y0 || y1, hh = x0 || x1, hc = hv && hh;
    const int sv = hv ? (y0 ? I::DOWN : I::UP) + t.lx : 0;
    const int sh = hh ? (x0 ? I::LEFT : I::RIGHT) + t.ly : 0;
    const int sc = hc ? I::CORNER + (x1 ? 1 : 0) + (y1 ? 2 : 0) : 0;
    if (NF == 1) {
        const double* b = in + (int64_t)t.tile * I::SIZE;
        const double v = b[sv], h = b[sh], c = b[sc];
        if (hv) r += v;
        if (hh) r += h;
        if (hc) r += c;
        return;
    }
    const double2* b = reinterpret_cast<const double2*>(in) + (int64_t)t.tile * I::SIZE;
    const double2 v = b[sv], h = b[sh], c = b[sc];
    if (hv) {
        r += v.x;
        p += v.y;
    }
    if (hh) {
        r += h.x;
        p += h.y;
    }
    if (hc) {
        r += c.x;
        p += c.y;
    }
}

// Inbox slot (in the owning tile of the same plane) that receives the ring
// position (ex, ey) of a W x H tile at (x0, y0).  Returns the slot's index in
// the plane's inbox array.
template <int TH>
__device__ __forceinline__ int64_t inbox_target(const GridDims& g, int x0, int y0, int W, int H, int ex, int ey) {
    using I = Inbox<TH>;
    int tx = x0 + ex, ty = y0 + ey;
    tx += tx < 0 ? g.nx : (tx >= g.nx ? -g.nx : 0);
    ty += ty < 0 ? g.ny : (ty >= g.ny ? -g.ny : 0);
    const TilePos t = tile_pos<TH>(g, tx, ty);
    // where the sending tile lies as seen from the receiving node
    const int dx = ex < 0 ? 1 : (ex >= W ? -1 : 0);
    const int dy = ey < 0 ? 1 : (ey >= H ? -1 : 0);
    int slot;
    if (dx == 0) slot = (dy > 0 ? I::UP : I::DOWN) + t.lx;
    else if (dy == 0) slot = (dx > 0 ? I::RIGHT : I::LEFT) + t.ly;
    else slot = I::CORNER + (dx > 0 ? 1 : 0) + (dy > 0 ? 2 : 0);
    return (int64_t)t.tile * I::SIZE + slot;
}

// Index of the lattice direction (cx, cy, cz), and the offset of D1Q3 index k
// (0, +1, -1 for k = 0, 1, 2).
template <int L>
__host__ __device__ constexpr int lat_dir(int cx, int cy, int cz) {
    for (int i = 0; i < Lattice<L>::Q; ++i)
        if (Lattice<L>::c[i][0] == cx && Lattice<L>::c[i][1] == cy && Lattice<L>::c[i][2] == cz) return i;
    return -1;
}
__host__ __device__ constexpr int row_offset(int ky) { return ky == 0 ? 0 : (ky == 1 ? 1 : -1); }
template <int L>
__host__ __device__ constexpr bool all_dirs_present() {
    for (int kz = 0; kz < (Lattice<L>::D == 3 ? 3 : 1); ++kz)
        for (int ky = 0; ky < 3; ++ky)
            for (int kx = 0; kx < 3; ++kx)
                if (lat_dir<L>(row_offset(kx), row_offset(ky), row_offset(kz)) < 0) return false;
    return true;
}
static_assert(all_dirs_present<kD2Q9>() && all_dirs_present<kD3Q27>(), "every lattice direction present");

// Per-row partial sums of the next moments in a BX x TH tile.  Group
// gi = ky + 3 kz holds the directions with c_y = row_offset(ky), c_z =
// row_offset(kz) (D2Q9: kz = 0 only).  For group gi the node at lane l leaves
//   S_gi(l) = v(0, c_y, c_z)(l) + v(+1, c_y, c_z)(l - 1) + v(-1, c_y, c_z)(l + 1)
// (terms from lanes of the tile only) in sum[field][gi][ly][l], and the
// values that leave the tile sideways, v(-1, .) of lane 0 and v(+1, .) of the
// last lane, in side[field][0 / 1][gi][ly].
template <int L, int TH, int NF = 2>
struct NextSink {
    static constexpr int NG = Lattice<L>::D == 3 ? 9 : 3;
    static constexpr int SUM = NF * NG * TH * BX, SIDE = NF * 2 * NG * TH;
    double* sum;
    double* side;
    int lx, ly, W;
    // c_y of the directions that stream into a wall from this node's row (-1
    // on the bottom wall row, +1 on the top one, 0 elsewhere; uniform over a
    // wavefront): they bounce back to the node itself, so their values join
    // the node's own target (group c_y = c_z = 0)
    int wall_cy;
    __device__ __forceinline__ void put(int field, const double* v) {
        double back = 0.0;
        if (wall_cy != 0) {
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                const int cy = row_offset(gi % 3), cz = row_offset(gi / 3);
                if (cy != wall_cy) continue;
                back += v[lat_dir<L>(0, cy, cz)] + v[lat_dir<L>(1, cy, cz)] + v[lat_dir<L>(-1, cy, cz)];
            }
        }
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            const int cy = row_offset(gi % 3), cz = row_offset(gi / 3);
            const double a = v[lat_dir<L>(0, cy, cz)], b = v[lat_dir<L>(1, cy, cz)], c = v[lat_dir<L>(-1, cy, cz)];
            const double bl = __shfl_up(b, 1);
            const double cr = __shfl_down(c, 1);
            double t = a;
            if (lx >= 1) t += bl;
            if (lx + 1 < W) t += cr;
            if (cy == 0 && cz == 0) t += back;
            sum[((field * NG + gi) * TH + ly) * BX + lx] = t;
            if (lx == 0) side[((field * 2 + 0) * NG + gi) * TH + ly] = c;
            if (lx == W - 1) side[((field * 2 + 1) * NG + gi) * TH + ly] = b;
        }
    }
    template <int L2, typename R>
    __device__ __forceinline__ void post_f(const R* f, double r) {
        using Lt = Lattice<L>;
        double v[Lt::Q];
#pragma unroll
        for (int i = 0; i < Lt::Q; ++i) {
            v[i] = double(f[i]);
            if (Deviation<R>::on) v[i] += Lt::w[i] * r;
        }
        put(0, v);
    }
    template <int L2, typename R, int QG>
    __device__ __forceinline__ void post_g(const R* gg) {
        static_assert(NF == 2, "the phase field is the second field");
        // a reduced phase-field lattice has no populations beyond its QG
        double v[Lattice<L>::Q];
#pragma unroll
        for (int i = 0; i < Lattice<L>::Q; ++i) v[i] = i < QG ? double(gg[i]) : 0.0;
        put(1, v);
    }
    // sum over the tile's sources for target (ex, ey) of the ring-extended
    // tile, in the target plane offset by c_z = row_offset(kz)
    __device__ __forceinline__ void gather(int ex, int ey, int kz, int H, double& s0, double& s1) const {
        s0 = 0.0;
        s1 = 0.0;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int gi = ky + 3 * kz;
            const int sy = ey - row_offset(ky);
            if (sy < 0 || sy >= H) continue;
            if (ex < 0) {
                s0 += side[((0 * 2 + 0) * NG + gi) * TH + sy];
                if (NF == 2) s1 += side[((1 * 2 + 0) * NG + gi) * TH + sy];
            } else if (ex >= W) {
                s0 += side[((0 * 2 + 1) * NG + gi) * TH + sy];
                if (NF == 2) s1 += side[((1 * 2 + 1) * NG + gi) * TH + sy];
            } else {
                s0 += sum[((0 * NG + gi) * TH + sy) * BX + ex];
                if (NF == 2) s1 += sum[((1 * NG + gi) * TH + sy) * BX + ex];
            }
        }
    }
};

constexpr int INBOX3 = Inbox<BY>::SIZE;

// D3Q27 collisions that leave the next moments walk z-columns of ZC planes of
// their tile (column c holds planes [c ZC, min(nz, (c + 1) ZC))), so that the
// sums for a node from the three source planes above, at and below it meet
// in the block that owns the node's column; only a column's first and last
// planes receive sums from a neighbouring column.  Buffers (NF doubles per
// entry: (rho, phi) pairs, or one field; nch = zcols(nz) columns, `plane` =
// nx ny):
//   part:  [N] sums from the node's own column, then [nch][plane] sums for
//          each column's first plane from the plane below it, then
//          [nch][plane] sums for each column's last plane from the plane
//          above it (periodic in z);
//   inbox: the tile inboxes (INBOX3 slots per tile) of the same three parts,
//          [nz][tiles], [nch][tiles], [nch][tiles].
constexpr int ZC = kZc;

__host__ __device__ __forceinline__ int zcols(int nz) { return (nz + ZC - 1) / ZC; }

__host__ __device__ __forceinline__ int64_t tiles3(const GridDims& g) {
    return (int64_t)((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY);
}

// Entry e of a buffer of NF-field entries (p = 0 with one field).
template <int NF>
__device__ __forceinline__ void entry_get(const double* __restrict__ buf, int64_t e, double& r, double& p) {
    if (NF == 2) {
        const double2 a = reinterpret_cast<const double2*>(buf)[e];
        r = a.x;
        p = a.y;
    } else {
        r = buf[e];
        p = 0.0;
    }
}
template <int NF>
__device__ __forceinline__ void entry_put(double* __restrict__ buf, int64_t e, double r, double p) {
    if (NF == 2) reinterpret_cast<double2*>(buf)[e] = make_double2(r, p);
    else buf[e] = r;
}

// Completed next-step moments (r, p) of node (gx, gy, z), index n: the
// column's own sum and inbox entries, plus those from the neighbouring
// columns at a column's first and last plane (p = 0 with one field).
template <int NF = 2>
__device__ __forceinline__ void next3_complete(const GridDims& g, const double* __restrict__ part,
                                               const double* __restrict__ inbox, int gx, int gy, int z, int64_t n,
                                               double& r, double& p) {
    const int64_t plane = (int64_t)g.nx * g.ny, xy = (int64_t)gy * g.nx + gx;
    const int64_t box = tiles3(g) * INBOX3 * NF;  // doubles of one plane's inboxes
    const int nch = zcols(g.nz), c = z / ZC;
    const bool first = z == c * ZC, last = z == min(g.nz, (c + 1) * ZC) - 1;
    entry_get<NF>(part, n, r, p);
    inbox_complete_fast<BY, NF>(g, inbox + (int64_t)z * box, gx, gy, r, p);
    if (first) {
        double br, bp;
        entry_get<NF>(part, g.N + c * plane + xy, br, bp);
        r += br;
        p += bp;
        inbox_complete_fast<BY, NF>(g, inbox + ((int64_t)g.nz + c) * box, gx, gy, r, p);
    }
    if (last) {
        double br, bp;
        entry_get<NF>(part, g.N + (nch + c) * plane + xy, br, bp);
        r += br;
        p += bp;
        inbox_complete_fast<BY, NF>(g, inbox + ((int64_t)g.nz + nch + c) * box, gx, gy, r, p);
    }
}

// Ring position q (0 <= q < RING3) of a W x H tile: the rows below and above
// the tile (x from -1 to W), then the left and right columns; false where
// the position lies beyond a ragged tile's edge.
constexpr int RING3 = 2 * (BX + 2) + 2 * BY;
__device__ __forceinline__ bool ring_at(int q, int W, int H, int& ex, int& ey) {
    if (q < 2 * (BX + 2)) {
        ex = q % (BX + 2) - 1;
        ey = q < BX + 2 ? -1 : H;
        return ex <= W;
    }
    const int c = q - 2 * (BX + 2);
    ex = c < BY ? -1 : W;
    ey = c % BY;
    return ey < H;
}

// Running sums of a column walk, in LDS: [3 target-plane slots][NF fields]
// [the tile's BX BY nodes, then its RING3 ring positions].
constexpr int COL_NE = BX * BY + RING3;
template <int NF>
constexpr int col_acc() {
    return 3 * NF * COL_NE;
}

// Make the thread's index in its block (tx, ty) values the compiler cannot
// take for loop invariants: a plane loop around a collision that needs every
// register would otherwise keep the per-lane index arithmetic of its body
// live through the collision, and the collision then issues its loads one by
// one.
__device__ __forceinline__ void opaque_thread_index(int& tx, int& ty) {
    asm volatile("" : "+v"(tx), "+v"(ty));
}

// The same for the lattice size N, the stride of the population arrays: the
// per-direction bases src + i N held through the loop would not fit the
// scalar registers.
__device__ __forceinline__ GridDims opaque_stride(GridDims g) {
    asm volatile("" : "+s"(g.N));
    return g;
}

// After the collisions of source plane z of the column [z0, z1) have put
// their values in `view`'s sums (and a barrier): the block takes every item
// (a tile node or ring position, and a target plane z + c_z), each thread its
// own tile node's three and ring items tid, tid + BX BY.  A target plane
// outside the column receives its sum in that column's boundary part; one
// inside it accumulates in `acc` over the source planes z - 1, z, z + 1,
// started by the first (the plane below it, or its own at the column's first
// plane) and stored by the thread of the last (the plane above it, or its own
// at the column's last plane).  An entry of `acc` written in one plane and
// read in another may belong to different threads: the barrier between the
// planes orders them.  Blocks of BX x BY threads; (tx, ty) is the thread's
// index in the block.
template <bool WALL, int NF = 2>
__device__ __forceinline__ void next3_col_plane(const GridDims& g, const NextSink<kD3Q27, BY, NF>& view,
                                                double* __restrict__ acc, double* __restrict__ part,
                                                double* __restrict__ inbox, int x0, int y0, int W, int H, int z,
                                                int z0, int z1, int tx, int ty) {
    const int64_t tiles = tiles3(g), plane = (int64_t)g.nx * g.ny;
    const int nch = zcols(g.nz), c = z0 / ZC;
    const int below = c == 0 ? nch - 1 : c - 1, above = c + 1 == nch ? 0 : c + 1;
    // one item: position (ex, ey) of the ring-extended tile (ring: inbox
    // slot `where` of the receiving tile; else node `where` of the plane),
    // target plane offset row_offset(kz), running sum `slot` of acc
    auto item = [&](bool ring, int64_t where, int slot, int ex, int ey, int kz) {
        double s0, s1;
        view.gather(ex, ey, kz, H, s0, s1);
        auto put = [&](int64_t part_plane, double a0, double a1) {
            if (ring) entry_put<NF>(inbox, part_plane * tiles * INBOX3 + where, a0, a1);
            else entry_put<NF>(part, part_plane * plane + where, a0, a1);
        };
        const int dz = row_offset(kz), t = z + dz;
        if (t < z0) {
            put(g.nz + nch + below, s0, s1);  // the last plane of the column below (periodic)
        } else if (t >= z1) {
            put(g.nz + above, s0, s1);  // the first plane of the column above (periodic)
        } else {
            double* a = acc + ((t - z0) % 3) * NF * COL_NE + slot;
            if (dz == 1) {
                a[0] = s0;
                if (NF == 2) a[COL_NE] = s1;
            } else if (dz == 0) {
                if (z != z0) {
                    s0 += a[0];
                    if (NF == 2) s1 += a[COL_NE];
                }
                if (z == z1 - 1) {
                    put(t, s0, s1);
                } else {
                    a[0] = s0;
                    if (NF == 2) a[COL_NE] = s1;
                }
            } else {
                put(t, a[0] + s0, NF == 2 ? a[COL_NE] + s1 : 0.0);
            }
        }
    };
    const int tid = ty * BX + tx;
    if (tx < W && ty < H) {
        const int64_t xy = (int64_t)(y0 + ty) * g.nx + x0 + tx;
#pragma unroll
        for (int kz = 0; kz < 3; ++kz) item(false, xy, tid, tx, ty, kz);
    }
    for (int e = tid; e < 3 * RING3; e += BX * BY) {
        const int kz = e / RING3, q = e % RING3;
        int ex, ey;
        if (!ring_at(q, W, H, ex, ey)) continue;
        // nothing streams into a wall (those values bounced back in the sink)
        if (WALL && g.walls && ((ey < 0 && y0 == 0) || (ey >= H && y0 + H == g.ny))) continue;
        item(true, inbox_target<BY>(g, x0, y0, W, H, ex, ey), BX * BY + q, ex, ey, kz);
    }
}

}  // namespace telbm
