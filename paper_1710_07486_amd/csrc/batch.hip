// batch.hip -- batched form of the time step: many periodic lattices of
// uneven size and parameters advanced together.
//
// Each phase of a step (moments, chemical potentials, collision) is one
// persistent launch over a work list of (instance, tile) items covering every
// instance; the descriptors (sizes, constants, pointers) live in device
// memory.  Each XCD works through a contiguous range of the list so that
// neighbouring tiles share its L2.  Steps are replayed from hipGraphs that
// capture an even number of steps (so the ping-pong parity returns to its
// start).  The tile shape is a template parameter chosen at run time
// (telbm_batch_set_tiles, driven by the autotuner in autotune.py).
//
// D2Q9 batches have two more modes (telbm_batch_set_mode) that take the
// single solver's fused one-launch step (potentials, collision and
// next-step moment sums with tile inboxes): mode 1 launches it per instance,
// captured into the graphs on a few parallel branches (instance i on branch
// i mod kBranches); mode 2 runs it for all instances in one launch over an
// (instance, 64 x 8 tile) work list (one launch per equation of state
// present).  All modes share the state at a step boundary (populations, and
// for the FP32 form the reference densities rhob[ref]); the fused modes add
// per-instance partial densities, phase field and inboxes, rebuilt from the
// populations whenever they are entered.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/telbm.h"
#include "kernels.hpp"
#include "lattice.hpp"
#include "node_ops.hpp"
#include "thermo.hpp"

namespace telbm {

struct InstDesc {
    GridDims g;
    PhysConst k;
    void* pop[2];
    double* rhob[2];
    double *phi, *mux, *mup;
    int bxc, byc;  // tiles along x and y for the current tile shape
    // fused mode (D2Q9): current / next partial densities and phase field,
    // and the two inbox arrays
    double *xr[2], *xp[2], *inbox[2];
};

constexpr int kBranches = 4;  // parallel graph branches of the fused mode

struct TileShape {
    int bx, by;
};
constexpr TileShape kShapes[] = {{64, 1}, {64, 2}, {64, 4}, {64, 8}, {32, 8}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// WB: some member has walls (the instance for that case; members without
// walls take no wall branch, since every check reads the member's own flag).
template <int L, typename T, int TBX, int TBY, int PHASE, bool WB>
__global__ __launch_bounds__(TBX* TBY) void kb_phase(const InstDesc* __restrict__ inst,
                                                     const int2* __restrict__ work, int nwork, int cur,
                                                     int ref) {
    constexpr int NX = 8;  // XCDs
    const int G = gridDim.x;
    const int xcd = blockIdx.x % NX, j = blockIdx.x / NX;
    const int wgs = (G - xcd + NX - 1) / NX;  // workgroups resident on this XCD
    const int q = nwork / NX, rem = nwork % NX;
    const int lo = xcd * q + (xcd < rem ? xcd : rem);
    const int hi = lo + q + (xcd < rem ? 1 : 0);
    for (int w = lo + j; w < hi; w += wgs) {
        const int2 it = work[w];
        const InstDesc& d = inst[it.x];
        const int bx = it.y % d.bxc;
        const int rest = it.y / d.bxc;
        const int by = rest % d.byc;
        const int bz = rest / d.byc;
        const bool dev = Deviation<T>::on;
        double* rho = dev ? d.rhob[1 - ref] : d.rhob[0];
        const double* rho_ref = dev ? d.rhob[ref] : nullptr;
        if (PHASE == 2) {
            // two lanes per node (uniform control flow for the lane exchange)
            double dv[kDiag];
            tile_collide<L, T, TBX * TBY, false, WB>(d.g, d.k, (const T*)d.pop[cur], (T*)d.pop[1 - cur], rho_ref, rho,
                                               d.phi, d.mux, d.mup, bx * TBX, by * TBY, bz, TBX, TBY,
                                               threadIdx.y * TBX + threadIdx.x, false, dv);
            continue;
        }
        const int x = bx * TBX + threadIdx.x, y = by * TBY + threadIdx.y, z = bz;
        if (x >= d.g.nx || y >= d.g.ny || z >= d.g.nz) continue;
        if (PHASE == 0) {
            node_moments<L, T, WB>(d.g, (const T*)d.pop[cur], rho_ref, rho, d.phi, x, y, z);
        } else {
            // the members may differ in their equation of state
            if (d.k.eos == 0) node_chempot<L, 0, WB>(d.g, d.k, rho, d.phi, d.mux, d.mup, x, y, z);
            else if (d.k.eos == 1) node_chempot<L, 1, WB>(d.g, d.k, rho, d.phi, d.mux, d.mup, x, y, z);
            else node_chempot<L, 2, WB>(d.g, d.k, rho, d.phi, d.mux, d.mup, x, y, z);
        }
    }
}

template <int L, typename T, int S, bool WB>
static void launch_shape_w(int phase, int grid, hipStream_t st, const InstDesc* inst, const int2* work, int nwork,
                           int cur, int ref) {
    constexpr int TBX = kShapes[S].bx, TBY = kShapes[S].by;
    const dim3 blk(TBX, TBY, 1);
    if (phase == 0) kb_phase<L, T, TBX, TBY, 0, WB><<<grid, blk, 0, st>>>(inst, work, nwork, cur, ref);
    else if (phase == 1) kb_phase<L, T, TBX, TBY, 1, WB><<<grid, blk, 0, st>>>(inst, work, nwork, cur, ref);
    else kb_phase<L, T, TBX, TBY, 2, WB><<<grid, blk, 0, st>>>(inst, work, nwork, cur, ref);
}

template <int L, typename T, int S>
static hipError_t launch_shape(int phase, int grid, hipStream_t st, const InstDesc* inst, const int2* work,
                               int nwork, int cur, int ref, bool walls) {
    if (walls) launch_shape_w<L, T, S, true>(phase, grid, st, inst, work, nwork, cur, ref);
    else launch_shape_w<L, T, S, false>(phase, grid, st, inst, work, nwork, cur, ref);
    return hipGetLastError();
}

template <int L, typename T>
static hipError_t launch_batch_lt(int shape, int phase, int grid, hipStream_t st, const InstDesc* inst,
                                  const int2* work, int nwork, int cur, int ref, bool walls) {
    switch (shape) {
        case 0: return launch_shape<L, T, 0>(phase, grid, st, inst, work, nwork, cur, ref, walls);
        case 1: return launch_shape<L, T, 1>(phase, grid, st, inst, work, nwork, cur, ref, walls);
        case 2: return launch_shape<L, T, 2>(phase, grid, st, inst, work, nwork, cur, ref, walls);
        case 3: return launch_shape<L, T, 3>(phase, grid, st, inst, work, nwork, cur, ref, walls);
        default: return launch_shape<L, T, 4>(phase, grid, st, inst, work, nwork, cur, ref, walls);
    }
}

static hipError_t launch_batch(int lattice, int precision, int shape, int phase, int grid, hipStream_t st,
                               const InstDesc* inst, const int2* work, int nwork, int cur, int ref, bool walls) {
    if (lattice == kD2Q9)
        return precision ? launch_batch_lt<kD2Q9, float>(shape, phase, grid, st, inst, work, nwork, cur, ref, walls)
                         : launch_batch_lt<kD2Q9, double>(shape, phase, grid, st, inst, work, nwork, cur, ref, walls);
    return precision ? launch_batch_lt<kD3Q27, float>(shape, phase, grid, st, inst, work, nwork, cur, ref, walls)
                     : launch_batch_lt<kD3Q27, double>(shape, phase, grid, st, inst, work, nwork, cur, ref, walls);
}

}  // namespace telbm

using namespace telbm;

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct telbm_batch {
    int count;
    int lattice, precision;
    bool walls;  // some member has walls
    std::vector<telbm_params> p;
    std::vector<InstDesc> desc;  // host copy
    InstDesc* desc_dev;
    int2* work_dev;
    size_t work_cap;  // capacity in items
    int nwork;
    int shape, wg_per_cu, cus;
    hipStream_t stream;
    hipStream_t cap;  // internal stream for graph capture
    int cur, ref;
    int64_t steps;
    int chunk;  // steps per captured graph (even)
    std::map<std::tuple<int, int, int, int, int, int>, hipGraphExec_t> graphs;  // (mode, shape, wg, chunk, cur, ref)
    std::string err;
    // mode 0 (persistent three-phase), 1 (fused per instance) or 2 (fused,
    // one launch); whether xr[fp], xp[fp] hold the current densities and
    // phase field (fvalid) and whether they are partial sums still to be
    // completed from inbox[fp] (fpartial)
    int mode;
    FusedDesc* fdesc_dev;  // mode 2: per-instance pointers
    int2* fwork_dev;       // mode 2: (instance, tile) items grouped by equation of state
    int fwork_off[3], fwork_cnt[3];
    int fp;
    bool fvalid, fpartial;
    hipStream_t br[kBranches];  // capture branches
    hipEvent_t fork, join[kBranches];
};

namespace {

constexpr size_t kAlignB = 256;
size_t al(size_t v) { return (v + kAlignB - 1) & ~(kAlignB - 1); }

int bfail(telbm_batch* b, int code, const std::string& m) {
    if (b) b->err = m;
    return code;
}

size_t fused_extra_bytes(const telbm_params& p) {
    if (p.lattice != TELBM_D2Q9) return 0;
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    GridDims g{p.nx, p.ny, p.nz, 0, (int64_t)N};
    return 4 * al(N * sizeof(double)) + 2 * al(inbox_doubles(g) * sizeof(double));
}

size_t inst_bytes(const telbm_params& p) {
    const int Q = p.lattice == TELBM_D2Q9 ? 9 : 27;
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    const size_t s = p.precision == TELBM_FP32_MIXED ? 4 : 8;
    return 2 * al(2 * Q * N * s) + 5 * al(N * sizeof(double)) + fused_extra_bytes(p);
}

// (instance, 64 x 8 tile) items of the fused one-launch mode (D2Q9 only)
size_t fused_items(const telbm_params* p, int count) {
    size_t t = 0;
    for (int i = 0; i < count; ++i)
        if (p[i].lattice == TELBM_D2Q9) t += (size_t)fused_tiles_x(p[i].nx) * ((p[i].ny + 7) / 8);
    return t;
}

size_t max_tiles(const telbm_params* p, int count) {
    size_t best = 0;
    for (int v = 0; v < kNumShapes; ++v) {
        size_t t = 0;
        for (int i = 0; i < count; ++i)
            t += (size_t)((p[i].nx + kShapes[v].bx - 1) / kShapes[v].bx) *
                 ((p[i].ny + kShapes[v].by - 1) / kShapes[v].by) * p[i].nz;
        best = t > best ? t : best;
    }
    return best;
}

int check_params(const telbm_params* p, int count, std::string* why) {
    if (!p || count < 1) {
        *why = "need at least one instance";
        return TELBM_ERR_INVAL;
    }
    for (int i = 0; i < count; ++i) {
        if (p[i].lattice != p[0].lattice || p[i].precision != p[0].precision) {
            *why = "all instances of a batch share lattice and precision";
            return TELBM_ERR_INVAL;
        }
        if (p[i].glattice) {
            *why = "the batched form runs the full phase-field lattice only (instance " + std::to_string(i) + ")";
            return TELBM_ERR_INVAL;
        }
        size_t b;
        const int rc = telbm_required_bytes(&p[i], &b);
        if (rc) {
            *why = "instance " + std::to_string(i) + " has invalid parameters";
            return rc;
        }
    }
    return TELBM_OK;
}

PhysConst physconst(const telbm_params& p, double rg, double rl, double C) {
    PhysConst k{};
    k.a = p.a;
    k.b = p.b;
    k.RT = p.R * p.T;
    k.C = C;
    k.half_lambda1 = 0.5 * p.lambda1;
    k.lambda2 = p.lambda2;
    k.lambda3 = p.lambda3;
    k.rho_l = rl;
    const double dlt = rg - rl;
    k.inv_delta = 1.0 / dlt;
    k.inv_2delta = 1.0 / (2.0 * dlt);
    k.inv_chi = 1.0 / p.chi;
    k.inv_2chi = 1.0 / (2.0 * p.chi);
    k.twoA = 2.0 * (0.5 * p.kappa1 + (p.kappa2 + p.kappa3) / (8.0 * dlt * dlt));
    k.twoB = 2.0 * ((p.kappa2 + p.kappa3) / (8.0 * p.chi * p.chi));
    k.Dc = (p.kappa3 - p.kappa2) / (4.0 * p.chi * dlt);
    k.beta = 1.0 / (2.0 * (3.0 * p.nu + 0.5));
    k.inv_beta = 2.0 * (3.0 * p.nu + 0.5);
    k.omega_phi = 1.0 / p.tau_phi;
    k.Gamma = p.mobility / (p.tau_phi - 0.5);
    k.eos = p.eos;
    k.att = eos_attraction(eos_of(p), p.T);
    if (p.walls) {
        k.cot_rho[0] = cos(p.theta_rho_lo) / sin(p.theta_rho_lo);
        k.cot_rho[1] = cos(p.theta_rho_hi) / sin(p.theta_rho_hi);
        k.cot_phi[0] = cos(p.theta_phi_lo) / sin(p.theta_phi_lo);
        k.cot_phi[1] = cos(p.theta_phi_hi) / sin(p.theta_phi_hi);
    }
    return k;
}

int build_work(telbm_batch* b) {
    std::vector<int2> work;
    const TileShape sh = kShapes[b->shape];
    for (int i = 0; i < b->count; ++i) {
        InstDesc& d = b->desc[i];
        d.bxc = (d.g.nx + sh.bx - 1) / sh.bx;
        d.byc = (d.g.ny + sh.by - 1) / sh.by;
        const int nt = d.bxc * d.byc * d.g.nz;
        for (int t = 0; t < nt; ++t) work.push_back(make_int2(i, t));
    }
    if (work.size() > b->work_cap) return bfail(b, TELBM_ERR_NOMEM, "work list capacity");
    b->nwork = (int)work.size();
    hipError_t e = hipMemcpyAsync(b->work_dev, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->desc_dev, b->desc.data(), b->count * sizeof(InstDesc), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, std::string("descriptor upload: ") + hipGetErrorString(e));
    return TELBM_OK;
}

// Descriptors and the equation-of-state-grouped work list of mode 2.
int build_fused(telbm_batch* b) {
    std::vector<FusedDesc> fd(b->count);
    std::vector<int2> work;
    for (int i = 0; i < b->count; ++i) {
        const InstDesc& d = b->desc[i];
        FusedDesc& f = fd[i];
        f.g = d.g;
        f.k = d.k;
        for (int j = 0; j < 2; ++j) {
            f.pop[j] = d.pop[j];
            f.rhob[j] = d.rhob[j];
            f.xr[j] = d.xr[j];
            f.xp[j] = d.xp[j];
            f.inbox[j] = d.inbox[j];
        }
    }
    for (int e = 0; e < 3; ++e) {
        b->fwork_off[e] = (int)work.size();
        for (int i = 0; i < b->count; ++i) {
            if (b->desc[i].k.eos != e) continue;
            const int nt = fused_tiles_x(b->desc[i].g.nx) * ((b->desc[i].g.ny + 7) / 8);
            for (int t = 0; t < nt; ++t) work.push_back(make_int2(i, t));
        }
        b->fwork_cnt[e] = (int)work.size() - b->fwork_off[e];
    }
    hipError_t e = hipMemcpyAsync(b->fdesc_dev, fd.data(), b->count * sizeof(FusedDesc), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess && !work.empty())
        e = hipMemcpyAsync(b->fwork_dev, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, std::string("fused work list: ") + hipGetErrorString(e));
    return TELBM_OK;
}

// One step of every instance in mode 2 (one launch per equation of state).
hipError_t fused_launches(telbm_batch* b, hipStream_t st, int cur, int ref, int fp, bool partial) {
    for (int e = 0; e < 3; ++e) {
        if (b->fwork_cnt[e] == 0) continue;
        hipError_t r = launch_batch_fused2(b->precision, e, b->walls, st, b->fdesc_dev,
                                           b->fwork_dev + b->fwork_off[e], b->fwork_cnt[e], cur, ref, fp,
                                           partial ? 1 : 0);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

void drop_graphs(telbm_batch* b) {
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
}

hipError_t enqueue_step(telbm_batch* b, hipStream_t st, int cur, int ref) {
    const int grid = b->cus * b->wg_per_cu;
    for (int phase = 0; phase < 3; ++phase) {
        hipError_t e = launch_batch(b->lattice, b->precision, b->shape, phase, grid, st, b->desc_dev, b->work_dev,
                                    b->nwork, cur, ref, b->walls);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void advance(telbm_batch* b) {
    b->cur = 1 - b->cur;
    if (b->precision == TELBM_FP32_MIXED) b->ref = 1 - b->ref;
    b->steps += 1;
    if (b->mode != 0) {
        b->fp = 1 - b->fp;
        b->fpartial = true;
    } else {
        b->fvalid = false;
    }
}

// One fused step of instance i on stream st, from state (cur, ref, fp); the
// densities of the first step after entering the mode are complete
// (partial false).
hipError_t fused_step(telbm_batch* b, int i, hipStream_t st, int cur, int ref, int fp, bool partial) {
    const InstDesc& d = b->desc[i];
    const bool mixed = b->precision == TELBM_FP32_MIXED;
    StepArgs a{};
    a.g = d.g;
    a.k = d.k;
    a.src = d.pop[cur];
    a.dst = d.pop[1 - cur];
    a.rho_ref = mixed ? d.rhob[ref] : nullptr;
    a.rho = d.xr[fp];
    a.phi = d.xp[fp];
    a.inbox_in = partial ? d.inbox[fp] : nullptr;
    a.rho_next = d.xr[1 - fp];
    a.phi_next = d.xp[1 - fp];
    a.inbox_out = d.inbox[1 - fp];
    a.rho_final = mixed ? d.rhob[1 - ref] : nullptr;
    a.diag = 0;
    a.stream = st;
    return launch_part(b->lattice, b->precision, a, 3);
}

// Enter the fused mode: the current densities and phase field of every
// instance from its populations (relative to rhob[ref] in the FP32 form).
hipError_t fused_enter(telbm_batch* b) {
    const bool mixed = b->precision == TELBM_FP32_MIXED;
    for (int i = 0; i < b->count; ++i) {
        const InstDesc& d = b->desc[i];
        StepArgs a{};
        a.g = d.g;
        a.k = d.k;
        a.src = d.pop[b->cur];
        a.rho_ref = mixed ? d.rhob[b->ref] : nullptr;
        a.rho = d.xr[b->fp];
        a.phi = d.xp[b->fp];
        a.stream = b->stream;
        hipError_t e = launch_part(b->lattice, b->precision, a, 0);
        if (e != hipSuccess) return e;
    }
    b->fvalid = true;
    b->fpartial = false;
    return hipSuccess;
}

StepArgs inst_args(telbm_batch* b, int i, bool init) {
    const InstDesc& d = b->desc[i];
    const bool mixed = b->precision == TELBM_FP32_MIXED;
    StepArgs a{};
    a.g = d.g;
    a.k = d.k;
    a.src = d.pop[b->cur];
    a.dst = d.pop[b->cur];
    // initial fields are written into the state's own reference density
    a.rho = mixed ? (init ? d.rhob[b->ref] : d.rhob[1 - b->ref]) : d.rhob[0];
    a.rho_ref = mixed ? d.rhob[b->ref] : nullptr;
    a.phi = d.phi;
    a.mux = d.mux;
    a.mup = d.mup;
    a.stream = b->stream;
    return a;
}

}  // namespace

extern "C" {

int telbm_batch_required_bytes(const telbm_params* p, int count, size_t* bytes) {
    std::string why;
    if (!bytes) return TELBM_ERR_INVAL;
    int rc = check_params(p, count, &why);
    if (rc) return rc;
    size_t total = al(count * sizeof(InstDesc)) + al(max_tiles(p, count) * sizeof(int2)) + al(sizeof(unsigned long long));
    total += al(count * sizeof(FusedDesc)) + al(fused_items(p, count) * sizeof(int2));
    for (int i = 0; i < count; ++i) total += inst_bytes(p[i]);
    *bytes = total;
    return TELBM_OK;
}

int telbm_batch_create(const telbm_params* p, int count, void* arena, size_t bytes, telbm_batch** out) {
    if (!out) return TELBM_ERR_INVAL;
    *out = nullptr;
    size_t need;
    int rc = telbm_batch_required_bytes(p, count, &need);
    if (rc) return rc;
    if (!arena || ((uintptr_t)arena % kAlignB) != 0) return TELBM_ERR_INVAL;
    if (bytes < need) return TELBM_ERR_NOMEM;
    telbm_batch* b = new (std::nothrow) telbm_batch();
    if (!b) return TELBM_ERR_NOMEM;
    b->count = count;
    b->lattice = p[0].lattice;
    b->precision = p[0].precision;
    b->walls = false;
    for (int i = 0; i < count; ++i) b->walls = b->walls || p[i].walls != 0;
    b->p.assign(p, p + count);
    b->desc.resize(count);
    char* a = (char*)arena;
    size_t o = 0;
    b->desc_dev = (InstDesc*)(a + o);
    o += al(count * sizeof(InstDesc));
    b->work_cap = max_tiles(p, count);
    b->work_dev = (int2*)(a + o);
    o += al(b->work_cap * sizeof(int2));
    o += al(sizeof(unsigned long long));
    b->fdesc_dev = (FusedDesc*)(a + o);
    o += al(count * sizeof(FusedDesc));
    b->fwork_dev = (int2*)(a + o);
    o += al(fused_items(p, count) * sizeof(int2));
    for (int i = 0; i < count; ++i) {
        const telbm_params& q = p[i];
        double mg, ml, C, psi0;
        if (!eos_maxwell(eos_of(q), q.T, &mg, &ml, &C, &psi0)) {
            delete b;
            return TELBM_ERR_INVAL;
        }
        double rg = q.rho_g, rl = q.rho_l;
        if (rg == 0.0 && rl == 0.0) {
            rg = mg;
            rl = ml;
        }
        b->p[i].rho_g = rg;
        b->p[i].rho_l = rl;
        InstDesc& d = b->desc[i];
        const int Q = q.lattice == TELBM_D2Q9 ? 9 : 27;
        const int64_t N = (int64_t)q.nx * q.ny * q.nz;
        const size_t s = q.precision == TELBM_FP32_MIXED ? 4 : 8;
        d.g = GridDims{q.nx, q.ny, q.nz, q.walls, N};
        d.k = physconst(q, rg, rl, C);
        d.pop[0] = a + o;
        o += al(2 * Q * N * s);
        d.pop[1] = a + o;
        o += al(2 * Q * N * s);
        d.rhob[0] = (double*)(a + o);
        o += al(N * sizeof(double));
        d.rhob[1] = (double*)(a + o);
        o += al(N * sizeof(double));
        d.phi = (double*)(a + o);
        o += al(N * sizeof(double));
        d.mux = (double*)(a + o);
        o += al(N * sizeof(double));
        d.mup = (double*)(a + o);
        o += al(N * sizeof(double));
        for (int j = 0; j < 2; ++j) d.xr[j] = d.xp[j] = d.inbox[j] = nullptr;
        if (q.lattice == TELBM_D2Q9) {
            for (int j = 0; j < 2; ++j) {
                d.xr[j] = (double*)(a + o);
                o += al(N * sizeof(double));
                d.xp[j] = (double*)(a + o);
                o += al(N * sizeof(double));
                d.inbox[j] = (double*)(a + o);
                o += al(inbox_doubles(d.g) * sizeof(double));
            }
        }
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || b->cus < 1)
        b->cus = 256;
    b->shape = 2;
    b->wg_per_cu = 4;
    b->stream = nullptr;
    b->cur = 0;
    b->ref = 0;
    b->steps = 0;
    b->chunk = 10;
    b->mode = 0;
    b->fp = 0;
    b->fvalid = b->fpartial = false;
    bool ok = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess;
    for (int j = 0; j < kBranches; ++j) {
        b->br[j] = nullptr;
        b->join[j] = nullptr;
    }
    b->fork = nullptr;
    ok = ok && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int j = 0; j < kBranches && ok; ++j)
        ok = hipStreamCreateWithFlags(&b->br[j], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->join[j], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        for (int j = 0; j < kBranches; ++j) {
            if (b->br[j]) (void)hipStreamDestroy(b->br[j]);
            if (b->join[j]) (void)hipEventDestroy(b->join[j]);
        }
        if (b->fork) (void)hipEventDestroy(b->fork);
        if (b->cap) (void)hipStreamDestroy(b->cap);
        delete b;
        return TELBM_ERR_DEVICE;
    }
    rc = build_work(b);
    if (rc == TELBM_OK && b->lattice == TELBM_D2Q9) rc = build_fused(b);
    if (rc) {
        (void)telbm_batch_destroy(b);
        return rc;
    }
    *out = b;
    return TELBM_OK;
}

int telbm_batch_set_mode(telbm_batch* b, int mode) {
    if (!b || mode < 0 || mode > 2) return TELBM_ERR_INVAL;
    if (mode != 0 && b->lattice != TELBM_D2Q9) return bfail(b, TELBM_ERR_INVAL, "the fused modes are for D2Q9 batches");
    b->mode = mode;
    if (mode == 0) b->fvalid = false;
    return TELBM_OK;
}

int telbm_batch_set_stream(telbm_batch* b, void* stream) {
    if (!b) return TELBM_ERR_INVAL;
    b->stream = (hipStream_t)stream;
    return TELBM_OK;
}

int telbm_batch_tile_variants(int* count) {
    if (!count) return TELBM_ERR_INVAL;
    *count = kNumShapes;
    return TELBM_OK;
}

int telbm_batch_tile_shape(int variant, int* bx, int* by) {
    if (variant < 0 || variant >= kNumShapes || !bx || !by) return TELBM_ERR_INVAL;
    *bx = kShapes[variant].bx;
    *by = kShapes[variant].by;
    return TELBM_OK;
}

int telbm_batch_set_tiles(telbm_batch* b, int variant, int wg_per_cu) {
    if (!b || variant < 0 || variant >= kNumShapes || wg_per_cu < 1 || wg_per_cu > 64) return TELBM_ERR_INVAL;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, hipGetErrorString(e));
    b->shape = variant;
    b->wg_per_cu = wg_per_cu;
    drop_graphs(b);
    return build_work(b);
}

int telbm_batch_set_graph_steps(telbm_batch* b, int steps_per_graph) {
    if (!b || steps_per_graph < 0 || (steps_per_graph % 2) != 0) return TELBM_ERR_INVAL;
    b->chunk = steps_per_graph;
    return TELBM_OK;
}

int telbm_batch_init_fields(telbm_batch* b, int idx, const double* rho, const double* phi, const double* u,
                            int on_device) {
    if (!b || idx < 0 || idx >= b->count || !rho || !phi) return TELBM_ERR_INVAL;
    const InstDesc& d = b->desc[idx];
    const int64_t N = d.g.N;
    const int D = b->lattice == TELBM_D2Q9 ? 2 : 3;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    StepArgs a = inst_args(b, idx, true);
    double* u_dev = u ? (double*)d.pop[1 - b->cur] : nullptr;
    unsigned long long* bad =
        (unsigned long long*)((char*)b->work_dev + al(b->work_cap * sizeof(int2)));
    hipError_t e = hipMemcpyAsync(a.rho, rho, N * sizeof(double), kind, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d.phi, phi, N * sizeof(double), kind, b->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u_dev, u, (size_t)D * N * sizeof(double), kind, b->stream);
    if (e == hipSuccess) e = launch_check_init(d.g, D, a.rho, d.phi, u_dev, bad, b->stream);
    unsigned long long nbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, std::string("init: ") + hipGetErrorString(e));
    if (nbad) return bfail(b, TELBM_ERR_UNSTABLE, "unusable initial values");
    e = launch_part(b->lattice, b->precision, a, 1);
    if (e == hipSuccess) e = launch_init(b->lattice, b->precision, a, u_dev);
    if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, std::string("init launch: ") + hipGetErrorString(e));
    return TELBM_OK;
}

int fused_steps(telbm_batch* b, int64_t n) {
    while (n > 0) {
        if (!b->fvalid) {
            hipError_t e = fused_enter(b);
            if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, std::string("fused enter: ") + hipGetErrorString(e));
        }
        if (b->fpartial && b->chunk > 0 && n >= b->chunk) {
            auto key = std::make_tuple(b->mode, 0, 0, b->chunk, b->cur, b->ref * 2 + b->fp);
            auto it = b->graphs.find(key);
            if (it == b->graphs.end() && b->mode == 2) {
                hipGraph_t g;
                hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
                int cur = b->cur, ref = b->ref, fp = b->fp;
                for (int s = 0; s < b->chunk && e == hipSuccess; ++s) {
                    e = fused_launches(b, b->cap, cur, ref, fp, true);
                    cur = 1 - cur;
                    fp = 1 - fp;
                    if (b->precision == TELBM_FP32_MIXED) ref = 1 - ref;
                }
                hipError_t e2 = hipStreamEndCapture(b->cap, &g);
                if (e != hipSuccess || e2 != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, "graph capture failed");
                hipGraphExec_t ex;
                e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, "graph instantiate failed");
                it = b->graphs.emplace(key, ex).first;
            } else if (it == b->graphs.end()) {
                // the chunk's steps on kBranches parallel branches (instance i
                // on branch i mod kBranches), forked from and joined to b->cap
                hipGraph_t g;
                hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) e = hipEventRecord(b->fork, b->cap);
                for (int j = 0; j < kBranches && e == hipSuccess; ++j) e = hipStreamWaitEvent(b->br[j], b->fork, 0);
                int cur = b->cur, ref = b->ref, fp = b->fp;
                for (int s = 0; s < b->chunk && e == hipSuccess; ++s) {
                    for (int i = 0; i < b->count && e == hipSuccess; ++i)
                        e = fused_step(b, i, b->br[i % kBranches], cur, ref, fp, true);
                    cur = 1 - cur;
                    fp = 1 - fp;
                    if (b->precision == TELBM_FP32_MIXED) ref = 1 - ref;
                }
                for (int j = 0; j < kBranches && e == hipSuccess; ++j) e = hipEventRecord(b->join[j], b->br[j]);
                for (int j = 0; j < kBranches && e == hipSuccess; ++j) e = hipStreamWaitEvent(b->cap, b->join[j], 0);
                hipError_t e2 = hipStreamEndCapture(b->cap, &g);
                if (e != hipSuccess || e2 != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, "graph capture failed");
                hipGraphExec_t ex;
                e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, "graph instantiate failed");
                it = b->graphs.emplace(key, ex).first;
            }
            hipError_t e = hipGraphLaunch(it->second, b->stream);
            if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
            for (int s = 0; s < b->chunk; ++s) advance(b);
            n -= b->chunk;
        } else {
            if (b->mode == 2) {
                hipError_t e = fused_launches(b, b->stream, b->cur, b->ref, b->fp, b->fpartial);
                if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, std::string("fused step: ") + hipGetErrorString(e));
            } else {
                for (int i = 0; i < b->count; ++i) {
                    hipError_t e = fused_step(b, i, b->stream, b->cur, b->ref, b->fp, b->fpartial);
                    if (e != hipSuccess)
                        return bfail(b, TELBM_ERR_DEVICE, std::string("fused step: ") + hipGetErrorString(e));
                }
            }
            advance(b);
            n -= 1;
        }
    }
    return TELBM_OK;
}

int telbm_batch_step(telbm_batch* b, int64_t n) {
    if (!b || n < 0) return TELBM_ERR_INVAL;
    if (b->mode != 0) return fused_steps(b, n);
    while (n > 0) {
        if (b->chunk > 0 && n >= b->chunk) {
            auto key = std::make_tuple(0, b->shape, b->wg_per_cu, b->chunk, b->cur, b->ref);
            auto it = b->graphs.find(key);
            if (it == b->graphs.end()) {
                hipGraph_t g;
                hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
                int cur = b->cur, ref = b->ref;
                for (int s = 0; s < b->chunk && e == hipSuccess; ++s) {
                    e = enqueue_step(b, b->cap, cur, ref);
                    cur = 1 - cur;
                    if (b->precision == TELBM_FP32_MIXED) ref = 1 - ref;
                }
                hipError_t e2 = hipStreamEndCapture(b->cap, &g);
                if (e != hipSuccess || e2 != hipSuccess)
                    return bfail(b, TELBM_ERR_DEVICE, "graph capture failed");
                hipGraphExec_t ex;
                e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, "graph instantiate failed");
                it = b->graphs.emplace(key, ex).first;
            }
            hipError_t e = hipGraphLaunch(it->second, b->stream);
            if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
            for (int s = 0; s < b->chunk; ++s) advance(b);
            n -= b->chunk;
        } else {
            hipError_t e = enqueue_step(b, b->stream, b->cur, b->ref);
            if (e != hipSuccess) return bfail(b, TELBM_ERR_DEVICE, std::string("batch step: ") + hipGetErrorString(e));
            advance(b);
            n -= 1;
        }
    }
    return TELBM_OK;
}

int telbm_batch_sync(telbm_batch* b) {
    if (!b) return TELBM_ERR_INVAL;
    hipError_t e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? TELBM_OK : bfail(b, TELBM_ERR_DEVICE, hipGetErrorString(e));
}

int telbm_batch_read(telbm_batch* b, int idx, int field, double* out, int on_device) {
    if (!b || idx < 0 || idx >= b->count || !out || field < 0 || field > kFieldFz) return TELBM_ERR_INVAL;
    const InstDesc& d = b->desc[idx];
    StepArgs a = inst_args(b, idx, false);
    hipError_t e = launch_part(b->lattice, b->precision, a, 0);
    if (e == hipSuccess) e = launch_part(b->lattice, b->precision, a, 1);
    double* dst = on_device ? out : (double*)d.pop[1 - b->cur];
    if (e == hipSuccess) e = launch_macro(b->lattice, b->precision, a, field, dst);
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(out, dst, d.g.N * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e == hipSuccess ? TELBM_OK : bfail(b, TELBM_ERR_DEVICE, std::string("batch read: ") + hipGetErrorString(e));
}

int telbm_batch_step_count(const telbm_batch* b, int64_t* steps) {
    if (!b || !steps) return TELBM_ERR_INVAL;
    *steps = b->steps;
    return TELBM_OK;
}

int telbm_batch_destroy(telbm_batch* b) {
    if (!b) return TELBM_ERR_INVAL;
    (void)hipStreamSynchronize(b->stream);
    for (int j = 0; j < kBranches; ++j)
        if (b->br[j]) (void)hipStreamSynchronize(b->br[j]);
    drop_graphs(b);
    for (int j = 0; j < kBranches; ++j) {
        if (b->br[j]) (void)hipStreamDestroy(b->br[j]);
        if (b->join[j]) (void)hipEventDestroy(b->join[j]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return TELBM_OK;
}

const char* telbm_batch_last_error(const telbm_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
