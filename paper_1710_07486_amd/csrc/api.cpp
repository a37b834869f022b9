// api.cpp -- the C ABI of include/telbm.h: parameter validation, arena
// layout, state machine of the time stepping, read-out and diagnostics.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/telbm.h"
#include "kernels.hpp"
#include "thermo.hpp"

using namespace telbm;

struct telbm_solver {
    telbm_params p;
    PhysConst k;
    GridDims g;
    int Q;
    size_t pop_bytes;  // bytes of one population buffer
    char* arena;
    size_t arena_bytes;
    void* pop[2];
    // Density slots.  rhob[dsl], phib[psl]: moments of the current state (when
    // dens_valid; partial tile sums completed by inbox[isl] when dens_partial).
    // FP32 form: the stored f values are relative to rhob[ref].  The fused
    // D2Q9 step writes the next partial moments into free slots and the other
    // inbox, and (FP32 form) the completed current densities, the next
    // reference, into a fourth density slot.
    double* rhob[4];
    double* phib[2];
    double* inbox[2];
    double *part3, *inbox3;  // D3Q27 FP64: partial next-step moments and their inbox
    double *mux, *mup, *partials, *diag_dev;
    unsigned long long* bad;
    double diag_host[16];  // host copy of the diagnostics (pageable; 80 bytes)
    hipStream_t stream;
    int cur;             // pop[cur] holds the state
    int ref;             // FP32 form: the state's f values are relative to rhob[ref]
    int dsl, psl, isl;   // slots of the current moments and of their inbox
    bool dens_partial;   // D2Q9: rhob[dsl] / phib[psl] hold tile sums to complete;
                         // D3Q27 FP64: part3 / inbox3 hold the current moments
    bool aux_valid;      // rho/phi/mux/mup belong to the current state
    bool dens_valid;     // rho/phi belong to the current state
    int64_t steps;
    int64_t diag_step;   // step of the last diagnostics enqueued (-1: none)
    bool diag_unread;
    telbm_diag last;
    std::string err;
};

// Three liquids and the gas (nliquid.hip).
struct telbm_nl {
    telbm_params p;
    telbm_nl_params q;
    NlArgs a;           // constants and buffers; src / dst set per launch
    void* pop[2];
    int cur;            // pop[cur] holds the state
    bool aux_valid;     // rho, phi, psi and the potentials belong to the state
    bool partial;       // D3Q27: the state's moments are held as partial sums (a.partA ...)
    int64_t steps;
    std::string err;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int fail(telbm_solver* s, int code, const std::string& msg) {
    if (s) s->err = msg;
    return code;
}

int hip_fail(telbm_solver* s, hipError_t e, const char* where) {
    return fail(s, TELBM_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

struct Layout {
    size_t pop, aux, inbox, part3, inbox3, partials, diag, bad, total;
    int n_rho, n_phi, n_inbox;
    size_t o_pop0, o_pop1, o_rho[4], o_phi[2], o_inbox[2], o_part3, o_inbox3, o_mux, o_mup, o_part, o_diag, o_bad;
};

// Population values per node: f on the lattice, g on the full or reduced one.
int pops_per_node(const telbm_params& p) {
    const int Q = p.lattice == TELBM_D2Q9 ? 9 : 27;
    const int QG = p.glattice ? (p.lattice == TELBM_D2Q9 ? 5 : 7) : Q;
    return Q + QG;
}

Layout layout_of(const telbm_params& p) {
    const int64_t N = (int64_t)p.nx * p.ny * p.nz;
    const size_t s = p.precision == TELBM_FP32_MIXED ? 4 : 8;
    GridDims g{p.nx, p.ny, p.nz, 0, N};
    Layout L{};
    L.pop = align_up((size_t)pops_per_node(p) * N * s);
    L.aux = align_up((size_t)N * sizeof(double));
    // D2Q9 (fused step): current and next moments, FP32 form also the
    // reference and next reference densities; two inboxes
    const bool fz = p.lattice == TELBM_D2Q9;
    L.n_rho = fz && p.precision == TELBM_FP32_MIXED ? 4 : 2;
    L.n_phi = fz ? 2 : 1;
    L.n_inbox = fz ? 2 : 0;
    L.inbox = fz ? align_up(inbox_doubles(g) * sizeof(double)) : 0;
    // D3Q27 FP64: partial next-step moments and their inboxes
    const bool next3 = !fz && p.precision == TELBM_FP64;
    L.part3 = next3 ? align_up(part3_doubles(g, 2) * sizeof(double)) : 0;
    L.inbox3 = next3 ? align_up(inbox3_doubles(g, 2) * sizeof(double)) : 0;
    L.partials = align_up((size_t)collide_blocks(g) * kDiag * sizeof(double));
    L.diag = align_up(16 * sizeof(double));
    L.bad = align_up(sizeof(unsigned long long));
    size_t o = 0;
    L.o_pop0 = o; o += L.pop;
    L.o_pop1 = o; o += L.pop;
    for (int i = 0; i < L.n_rho; ++i) { L.o_rho[i] = o; o += L.aux; }
    for (int i = 0; i < L.n_phi; ++i) { L.o_phi[i] = o; o += L.aux; }
    for (int i = 0; i < L.n_inbox; ++i) { L.o_inbox[i] = o; o += L.inbox; }
    L.o_part3 = o; o += L.part3;
    L.o_inbox3 = o; o += L.inbox3;
    L.o_mux = o; o += L.aux;
    L.o_mup = o; o += L.aux;
    L.o_part = o; o += L.partials;
    L.o_diag = o; o += L.diag;
    L.o_bad = o; o += L.bad;
    L.total = o;
    return L;
}

int validate(const telbm_params* p, std::string* why) {
    if (!p) { *why = "null params"; return TELBM_ERR_INVAL; }
    if (p->lattice != TELBM_D2Q9 && p->lattice != TELBM_D3Q27) { *why = "lattice must be D2Q9 or D3Q27"; return TELBM_ERR_INVAL; }
    if (p->precision != TELBM_FP64 && p->precision != TELBM_FP32_MIXED) { *why = "unknown precision"; return TELBM_ERR_INVAL; }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) { *why = "sizes must be >= 1"; return TELBM_ERR_INVAL; }
    if (p->lattice == TELBM_D2Q9 && p->nz != 1) { *why = "D2Q9 needs nz == 1"; return TELBM_ERR_INVAL; }
    // The kernels address each per-direction population slice and each FP64
    // field with 32-bit byte offsets and 32-bit node indices, so an FP64
    // slice (N * 8 bytes) must stay below 4 GiB: N < 2^29 nodes.
    const double N = (double)p->nx * p->ny * p->nz;
    if (N * 8.0 >= 4294967296.0) {
        *why = "lattice too large: at most 2^29 - 1 nodes (32-bit byte offsets of the FP64 slices)";
        return TELBM_ERR_INVAL;
    }
    if (p->eos < TELBM_EOS_CS || p->eos > TELBM_EOS_PR) { *why = "unknown equation of state"; return TELBM_ERR_INVAL; }
    if (p->eos == TELBM_EOS_PR && !isfinite(p->omega)) { *why = "omega must be finite"; return TELBM_ERR_INVAL; }
    if (p->walls != 0 && p->walls != 1) { *why = "walls must be 0 or 1"; return TELBM_ERR_INVAL; }
    if (p->glattice != 0 && p->glattice != 1) { *why = "glattice must be 0 or 1"; return TELBM_ERR_INVAL; }
    if (p->glattice && p->lattice == TELBM_D3Q27 && p->precision == TELBM_FP32_MIXED) {
        *why = "the reduced phase-field lattice is not available for D3Q27 in the FP32-mixed form";
        return TELBM_ERR_INVAL;
    }
    if (p->walls) {
        if (p->ny < 2) { *why = "walls need ny >= 2"; return TELBM_ERR_INVAL; }
        for (double t : {p->theta_rho_lo, p->theta_rho_hi, p->theta_phi_lo, p->theta_phi_hi})
            if (!(t > 0.0 && t < M_PI)) { *why = "contact angles must lie in (0, pi)"; return TELBM_ERR_INVAL; }
    }
    double Tc;
    if (!eos_critical_point(eos_of(*p), &Tc, nullptr)) { *why = "a, b, R must be positive"; return TELBM_ERR_INVAL; }
    if (!(p->T > 0.0 && p->T < Tc)) { *why = "T must lie in (0, T_c)"; return TELBM_ERR_INVAL; }
    if (!(p->nu > 0.0) || !isfinite(p->nu)) { *why = "nu must be positive"; return TELBM_ERR_INVAL; }
    if (!(p->tau_phi > 0.5) || !isfinite(p->tau_phi)) { *why = "tau_phi must exceed 1/2"; return TELBM_ERR_INVAL; }
    if (!(p->chi != 0.0) || !isfinite(p->chi)) { *why = "chi must be non-zero"; return TELBM_ERR_INVAL; }
    if (!(p->mobility >= 0.0)) { *why = "mobility must be non-negative"; return TELBM_ERR_INVAL; }
    const bool given = p->rho_g != 0.0 || p->rho_l != 0.0;
    if (given && !(p->rho_l > p->rho_g && p->rho_g > 0.0)) { *why = "need rho_l > rho_g > 0"; return TELBM_ERR_INVAL; }
    const double vals[] = {p->lambda1, p->lambda2, p->lambda3, p->kappa1, p->kappa2, p->kappa3, p->rho_ref};
    for (double v : vals)
        if (!isfinite(v)) { *why = "non-finite free-energy parameter"; return TELBM_ERR_INVAL; }
    return TELBM_OK;
}

// Derived constants of the free energy and the kinetics.
PhysConst derive(const telbm_params& p, double rho_g, double rho_l, double C) {
    PhysConst k{};
    k.a = p.a;
    k.b = p.b;
    k.RT = p.R * p.T;
    k.C = C;
    k.half_lambda1 = 0.5 * p.lambda1;
    k.lambda2 = p.lambda2;
    k.lambda3 = p.lambda3;
    k.rho_l = rho_l;
    const double dlt = rho_g - rho_l;
    k.inv_delta = 1.0 / dlt;
    k.inv_2delta = 1.0 / (2.0 * dlt);
    k.inv_chi = 1.0 / p.chi;
    k.inv_2chi = 1.0 / (2.0 * p.chi);
    const double A = 0.5 * p.kappa1 + (p.kappa2 + p.kappa3) / (8.0 * dlt * dlt);
    const double B = (p.kappa2 + p.kappa3) / (8.0 * p.chi * p.chi);
    const double D = (p.kappa3 - p.kappa2) / (4.0 * p.chi * dlt);
    k.twoA = 2.0 * A;
    k.twoB = 2.0 * B;
    k.Dc = D;
    const double tau = 3.0 * p.nu + 0.5;
    k.beta = 1.0 / (2.0 * tau);
    k.inv_beta = 2.0 * tau;
    k.omega_phi = 1.0 / p.tau_phi;
    k.Gamma = p.mobility / (p.tau_phi - 0.5);
    k.eos = p.eos;
    k.att = eos_attraction(eos_of(p), p.T);
    k.glat = p.glattice;
    if (p.walls) {
        k.cot_rho[0] = cos(p.theta_rho_lo) / sin(p.theta_rho_lo);
        k.cot_rho[1] = cos(p.theta_rho_hi) / sin(p.theta_rho_hi);
        k.cot_phi[0] = cos(p.theta_phi_lo) / sin(p.theta_phi_lo);
        k.cot_phi[1] = cos(p.theta_phi_hi) / sin(p.theta_phi_hi);
    }
    return k;
}

bool mixed(const telbm_solver* s) { return s->p.precision == TELBM_FP32_MIXED; }
bool fused(const telbm_solver* s) { return s->p.lattice == TELBM_D2Q9; }
// D3Q27 FP64: the collision leaves the next moments as partial sums
bool next3(const telbm_solver* s) { return s->p.lattice == TELBM_D3Q27 && !mixed(s); }

// A density slot other than `a`.
int other_slot(const telbm_solver* s, int a) { return fused(s) && mixed(s) ? (a + 1) % 4 : 1 - a; }

// Free density slots of the fused step: k = 0 receives the next partial
// moments, k = 1 (FP32 form) the completed current densities.  Neither is the
// current slot or the reference.
int free_slot(const telbm_solver* s, int k) {
    if (!mixed(s)) return 1 - s->dsl;
    for (int i = 0; i < 4; ++i)
        if (i != s->dsl && i != s->ref && k-- == 0) return i;
    return -1;
}

// Density field that the moment kernel fills for the current state.
double* density_out(telbm_solver* s) { return s->rhob[s->dsl]; }

StepArgs args_of(telbm_solver* s, bool forward) {
    StepArgs a{};
    a.g = s->g;
    a.k = s->k;
    a.src = s->pop[s->cur];
    a.dst = forward ? s->pop[1 - s->cur] : s->pop[s->cur];
    a.rho_ref = mixed(s) ? s->rhob[s->ref] : nullptr;
    a.rho = density_out(s);
    a.phi = s->phib[s->psl];
    if (fused(s)) {
        a.inbox_in = s->dens_partial ? s->inbox[s->isl] : nullptr;
        a.rho_next = s->rhob[free_slot(s, 0)];
        a.phi_next = s->phib[1 - s->psl];
        a.inbox_out = s->inbox[1 - s->isl];
        a.rho_final = mixed(s) ? s->rhob[free_slot(s, 1)] : nullptr;
    }
    a.mux = s->mux;
    a.mup = s->mup;
    a.part3 = s->part3;
    a.inbox3 = s->inbox3;
    a.partials = s->partials;
    a.partials_blocks = collide_blocks(s->g);
    a.diag_out = s->diag_dev;
    a.diag = 0;
    a.stream = s->stream;
    return a;
}

// Optional per-launch event timing (telbm_time_kernels).
struct Timing {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    size_t used = 0;
    std::vector<int> kind;
};

hipError_t timed_launch(telbm_solver* s, const StepArgs& a, int part, Timing* t) {
    if (!t) return launch_part(s->p.lattice, s->p.precision, a, part);
    if (t->used >= t->pool.size()) return hipErrorInvalidValue;
    auto& ev = t->pool[t->used++];
    hipError_t e = hipEventRecord(ev.first, s->stream);
    if (e == hipSuccess) e = launch_part(s->p.lattice, s->p.precision, a, part);
    if (e == hipSuccess) e = hipEventRecord(ev.second, s->stream);
    // fused 2D launch and the 3D collision with next sums: collision; 2D
    // completion: moments; completing 3D potential pass: potentials
    t->kind.push_back(part == 3 || part == 6 ? 2 : part == 4 ? 0 : part == 5 ? 1 : part);
    return e;
}

// Bring the densities (moments) to the current state; partial tile sums are
// kept (the fused step completes them) unless `complete`.
int ensure_dens(telbm_solver* s, Timing* t = nullptr, bool complete = true) {
    if (s->dens_valid) {
        if (!s->dens_partial || !complete) return TELBM_OK;
        // D3Q27: the completing pass also computes the chemical potentials
        StepArgs a = args_of(s, false);
        hipError_t e = timed_launch(s, a, fused(s) ? 4 : 5, t);
        if (e != hipSuccess) return hip_fail(s, e, "moment completion launch");
        s->dens_partial = false;
        if (!fused(s)) s->aux_valid = true;
        return TELBM_OK;
    }
    StepArgs a = args_of(s, false);
    hipError_t e = timed_launch(s, a, 0, t);
    if (e != hipSuccess) return hip_fail(s, e, "moment launch");
    s->dens_valid = true;
    s->dens_partial = false;
    return TELBM_OK;
}

// Bring the aux fields to the current state (moments + chemical potentials).
int ensure_aux(telbm_solver* s, Timing* t = nullptr) {
    if (s->aux_valid) return TELBM_OK;
    int rc = ensure_dens(s, t);
    if (rc) return rc;
    if (s->aux_valid) return TELBM_OK;  // completed together with the potentials
    StepArgs a = args_of(s, false);
    hipError_t e = timed_launch(s, a, 1, t);
    if (e != hipSuccess) return hip_fail(s, e, "chemical-potential launch");
    s->aux_valid = true;
    return TELBM_OK;
}

int consume_diag(telbm_solver* s) {
    if (!s->diag_unread) return TELBM_OK;
    hipError_t e = hipMemcpyAsync(s->diag_host, s->diag_dev, kDiag * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "diagnostics copy");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "stream synchronise");
    const double* d = s->diag_host;
    telbm_diag& o = s->last;
    o.step = s->diag_step;
    o.mass = d[0];
    o.phi_total = d[1];
    o.mom[0] = d[2];
    o.mom[1] = d[3];
    o.mom[2] = d[4];
    o.max_u = d[5];
    o.min_rho = d[6];
    o.gamma_min = d[7];
    o.gamma_max = d[8];
    o.nonfinite = (int64_t)d[9];
    s->diag_unread = false;
    return TELBM_OK;
}

bool unstable(const telbm_diag& d) {
    return d.nonfinite > 0 || !(d.min_rho > 0.0) || !(d.max_u < 1.0) || !isfinite(d.mass);
}

// One time step.
// On D2Q9 one launch computes the chemical potentials, the collision and the
// next state's moments (as tile sums plus inbox entries, completed by the
// next launch), so the moment pass runs only after initialisation.
int one_step(telbm_solver* s, bool diag, Timing* t = nullptr) {
    const bool fz = fused(s);
    int rc = fz ? ensure_dens(s, t, false) : ensure_aux(s, t);
    if (rc) return rc;
    StepArgs a = args_of(s, true);
    a.diag = diag ? 1 : 0;
    hipError_t e = timed_launch(s, a, fz ? 3 : (next3(s) ? 6 : 2), t);
    if (e != hipSuccess) return hip_fail(s, e, "collision launch");
    s->cur = 1 - s->cur;
    if (fz) {
        const int nxt = free_slot(s, 0), fin = free_slot(s, 1);
        s->dsl = nxt;
        s->psl = 1 - s->psl;
        s->isl = 1 - s->isl;
        s->dens_partial = true;
        if (mixed(s)) s->ref = fin;  // the new state is relative to the completed densities
    } else if (mixed(s)) {
        s->ref = s->dsl;  // the new state is relative to the density just used
        s->dsl = other_slot(s, s->dsl);
    }
    s->aux_valid = false;
    s->dens_valid = fz || next3(s);
    if (next3(s)) s->dens_partial = true;
    if (diag) {
        s->diag_step = s->steps;
        s->diag_unread = true;
    }
    s->steps += 1;
    return TELBM_OK;
}

constexpr int kKinds = 3;
const char* kKernelNames[kKinds] = {"moments", "chemical_potentials", "collide"};

// -- three liquids ------------------------------------------------------------

// Mobility matrix / M in closed form (the header states it).
bool nl_mobility(const telbm_params& p, const telbm_nl_params& q, double* m) {
    if (!(p.kappa2 > 0.0 && p.kappa3 > 0.0 && q.kappa4 > 0.0)) return false;
    const double w1 = 1.0 / p.kappa2, w2 = 1.0 / p.kappa3, w3 = 1.0 / q.kappa4;
    const double W = w1 + w2 + w3, s = 1.0 / (W * (w1 + w2));
    m[0] = s * (4.0 * w1 * w2 + (w1 + w2) * w3);
    m[1] = m[2] = s * w3 * (w2 - w1);
    m[3] = w3 / W;
    return true;
}

int nl_validate(const telbm_params* p, const telbm_nl_params* q, std::string* why) {
    int rc = validate(p, why);
    if (rc) return rc;
    if (!q) { *why = "null third-liquid params"; return TELBM_ERR_INVAL; }
    if (p->precision != TELBM_FP64) { *why = "three liquids: FP64 only"; return TELBM_ERR_INVAL; }
    if (p->walls || p->glattice) { *why = "three liquids: periodic boxes on the full lattice only"; return TELBM_ERR_INVAL; }
    if (!isfinite(q->lambda4) || !isfinite(q->kappa4)) { *why = "non-finite lambda4 / kappa4"; return TELBM_ERR_INVAL; }
    double m[4];
    if (!nl_mobility(*p, *q, m)) { *why = "three liquids: kappa2, kappa3, kappa4 must be positive"; return TELBM_ERR_INVAL; }
    return TELBM_OK;
}

struct NlLayout {
    size_t pop, aux, partA, inboxA, partB, inboxB, total;
};

// Two population buffers of 3 Q N doubles, six N-double fields and, for
// D3Q27, the partial next-step moments with their inboxes: (rho, phi) pairs
// (A) and psi (B).
NlLayout nl_layout(const telbm_params& p) {
    const int64_t N = (int64_t)p.nx * p.ny * p.nz;
    const int Q = p.lattice == TELBM_D2Q9 ? 9 : 27;
    const GridDims g{p.nx, p.ny, p.nz, 0, N};
    NlLayout L;
    L.pop = align_up((size_t)3 * Q * N * sizeof(double));
    L.aux = align_up((size_t)N * sizeof(double));
    const bool d3 = p.lattice == TELBM_D3Q27;
    L.partA = d3 ? align_up(part3_doubles(g, 2) * sizeof(double)) : 0;
    L.inboxA = d3 ? align_up(inbox3_doubles(g, 2) * sizeof(double)) : 0;
    L.partB = d3 ? align_up(part3_doubles(g, 1) * sizeof(double)) : 0;
    L.inboxB = d3 ? align_up(inbox3_doubles(g, 1) * sizeof(double)) : 0;
    L.total = 2 * L.pop + 6 * L.aux + L.partA + L.inboxA + L.partB + L.inboxB;
    return L;
}

int nl_fail(telbm_nl* s, int code, const std::string& msg) {
    s->err = msg;
    return code;
}

hipError_t nl_launch(telbm_nl* s, int part) {
    NlArgs a = s->a;
    a.src = (const double*)s->pop[s->cur];
    a.dst = (double*)s->pop[part == 3 ? s->cur : 1 - s->cur];  // part 3 writes the state itself
    return launch_nl_part(s->p.lattice, a, part);
}

// Moments (completed from the partial sums the last D3Q27 collision left, or
// pulled from the populations) and potentials of the current state.
int nl_ensure_aux(telbm_nl* s) {
    if (s->aux_valid) return TELBM_OK;
    // partial sums (D3Q27): completion and potentials in one column pass
    hipError_t e = s->partial ? nl_launch(s, 6) : nl_launch(s, 0);
    if (e == hipSuccess && !s->partial) e = nl_launch(s, 1);
    if (e != hipSuccess) return nl_fail(s, TELBM_ERR_DEVICE, std::string("three-liquid launch: ") + hipGetErrorString(e));
    s->aux_valid = true;
    s->partial = false;
    return TELBM_OK;
}

}  // namespace

extern "C" {

const char* telbm_version(void) { return "telbm 0.1 (gfx950)"; }

int telbm_critical_temperature(double a, double b, double R, double* T_c) {
    if (!T_c) return TELBM_ERR_INVAL;
    return critical_point(a, b, R, T_c, nullptr) ? TELBM_OK : TELBM_ERR_INVAL;
}

int telbm_coexistence(double a, double b, double R, double T, double* rho_g, double* rho_l, double* C,
                      double* Psi0) {
    if (!rho_g || !rho_l) return TELBM_ERR_INVAL;
    double c = 0, p0 = 0;
    if (!maxwell(a, b, R, T, rho_g, rho_l, &c, &p0)) return TELBM_ERR_INVAL;
    if (C) *C = c;
    if (Psi0) *Psi0 = p0;
    return TELBM_OK;
}

int telbm_temperature_for_ratio(double a, double b, double R, double ratio, double* T) {
    if (!T) return TELBM_ERR_INVAL;
    return temperature_for_ratio(a, b, R, ratio, T) ? TELBM_OK : TELBM_ERR_INVAL;
}

int telbm_eos_critical_temperature(int eos, double a, double b, double R, double omega, double* T_c) {
    if (!T_c) return TELBM_ERR_INVAL;
    return eos_critical_point(EosSpec{eos, a, b, R, omega}, T_c, nullptr) ? TELBM_OK : TELBM_ERR_INVAL;
}

int telbm_eos_coexistence(int eos, double a, double b, double R, double omega, double T, double* rho_g,
                          double* rho_l, double* C, double* Psi0) {
    if (!rho_g || !rho_l) return TELBM_ERR_INVAL;
    double c = 0, p0 = 0;
    if (!eos_maxwell(EosSpec{eos, a, b, R, omega}, T, rho_g, rho_l, &c, &p0)) return TELBM_ERR_INVAL;
    if (C) *C = c;
    if (Psi0) *Psi0 = p0;
    return TELBM_OK;
}

int telbm_eos_temperature_for_ratio(int eos, double a, double b, double R, double omega, double ratio, double* T) {
    if (!T) return TELBM_ERR_INVAL;
    return eos_temperature_for_ratio(EosSpec{eos, a, b, R, omega}, ratio, T) ? TELBM_OK : TELBM_ERR_INVAL;
}

int telbm_required_bytes(const telbm_params* p, size_t* bytes) {
    std::string why;
    if (!bytes) return TELBM_ERR_INVAL;
    int rc = validate(p, &why);
    if (rc) return rc;
    *bytes = layout_of(*p).total;
    return TELBM_OK;
}

int telbm_create(const telbm_params* p, void* device_arena, size_t bytes, telbm_solver** out) {
    if (!out) return TELBM_ERR_INVAL;
    *out = nullptr;
    std::string why;
    int rc = validate(p, &why);
    if (rc) return rc;
    const Layout L = layout_of(*p);
    if (!device_arena || ((uintptr_t)device_arena % kAlign) != 0) return TELBM_ERR_INVAL;
    if (bytes < L.total) return TELBM_ERR_NOMEM;
    double rg = p->rho_g, rl = p->rho_l, C = 0.0, psi0 = 0.0;
    double mg, ml;
    if (!eos_maxwell(eos_of(*p), p->T, &mg, &ml, &C, &psi0)) return TELBM_ERR_INVAL;
    if (rg == 0.0 && rl == 0.0) {
        rg = mg;
        rl = ml;
    }
    telbm_solver* s = new (std::nothrow) telbm_solver();
    if (!s) return TELBM_ERR_NOMEM;
    s->p = *p;
    s->p.rho_g = rg;
    s->p.rho_l = rl;
    s->k = derive(*p, rg, rl, C);
    s->Q = p->lattice == TELBM_D2Q9 ? 9 : 27;
    s->g = GridDims{p->nx, p->ny, p->nz, p->walls, (int64_t)p->nx * p->ny * p->nz};
    s->pop_bytes = L.pop;
    s->arena = (char*)device_arena;
    s->arena_bytes = bytes;
    s->pop[0] = s->arena + L.o_pop0;
    s->pop[1] = s->arena + L.o_pop1;
    for (int i = 0; i < 4; ++i) s->rhob[i] = i < L.n_rho ? (double*)(s->arena + L.o_rho[i]) : nullptr;
    for (int i = 0; i < 2; ++i) s->phib[i] = (double*)(s->arena + L.o_phi[i < L.n_phi ? i : 0]);
    for (int i = 0; i < 2; ++i) s->inbox[i] = i < L.n_inbox ? (double*)(s->arena + L.o_inbox[i]) : nullptr;
    s->part3 = L.part3 ? (double*)(s->arena + L.o_part3) : nullptr;
    s->inbox3 = L.inbox3 ? (double*)(s->arena + L.o_inbox3) : nullptr;
    s->mux = (double*)(s->arena + L.o_mux);
    s->mup = (double*)(s->arena + L.o_mup);
    s->partials = (double*)(s->arena + L.o_part);
    s->diag_dev = (double*)(s->arena + L.o_diag);
    s->bad = (unsigned long long*)(s->arena + L.o_bad);
    s->stream = nullptr;
    s->cur = 0;
    s->ref = 0;
    s->dsl = mixed(s) ? 1 : 0;
    s->psl = 0;
    s->isl = 0;
    s->dens_partial = false;
    s->aux_valid = false;
    s->dens_valid = false;
    s->steps = 0;
    s->diag_step = -1;
    s->diag_unread = false;
    memset(&s->last, 0, sizeof(s->last));
    s->last.step = -1;
    *out = s;
    return TELBM_OK;
}

int telbm_set_stream(telbm_solver* s, void* stream) {
    if (!s) return TELBM_ERR_INVAL;
    s->stream = (hipStream_t)stream;
    return TELBM_OK;
}

int telbm_init_fields(telbm_solver* s, const double* rho, const double* phi, const double* u, int on_device) {
    if (!s) return TELBM_ERR_INVAL;
    if (!rho || !phi) return fail(s, TELBM_ERR_INVAL, "rho and phi are required");
    const int64_t N = s->g.N;
    const int D = s->p.lattice == TELBM_D2Q9 ? 2 : 3;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    // stage: rho, phi into the aux fields, u into the spare population buffer
    double* u_dev = u ? (double*)s->pop[1 - s->cur] : nullptr;
    double* rho_dev = density_out(s);
    double* phi_dev = s->phib[s->psl];
    hipError_t e = hipMemcpyAsync(rho_dev, rho, N * sizeof(double), kind, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(phi_dev, phi, N * sizeof(double), kind, s->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u_dev, u, (size_t)D * N * sizeof(double), kind, s->stream);
    if (e == hipSuccess) e = launch_check_init(s->g, D, rho_dev, phi_dev, u_dev, s->bad, s->stream);
    unsigned long long bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(s->diag_host, s->bad, sizeof(bad), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "init staging");
    memcpy(&bad, s->diag_host, sizeof(bad));
    s->aux_valid = false;
    s->dens_valid = false;
    s->dens_partial = false;
    if (bad) return fail(s, TELBM_ERR_UNSTABLE, std::to_string(bad) + " nodes with rho <= 0, |u| >= 1 or non-finite values");
    // mu_phi of the initial fields, then the equilibria into the state buffer
    StepArgs a = args_of(s, false);
    e = launch_part(s->p.lattice, s->p.precision, a, 1);
    if (e == hipSuccess) e = launch_init(s->p.lattice, s->p.precision, a, u_dev);
    if (e != hipSuccess) return hip_fail(s, e, "init launch");
    // FP32 form: the initial populations are relative to the initial density
    if (mixed(s)) {
        s->ref = s->dsl;
        s->dsl = other_slot(s, s->ref);
    }
    s->steps = 0;
    s->diag_step = -1;
    s->diag_unread = false;
    s->last.step = -1;
    return TELBM_OK;
}

int telbm_step(telbm_solver* s, int64_t n) {
    if (!s || n < 0) return TELBM_ERR_INVAL;
    for (int64_t i = 0; i < n; ++i) {
        const bool diag = s->p.diag_every > 0 && (s->steps % s->p.diag_every) == 0;
        int rc = one_step(s, diag);
        if (rc) return rc;
    }
    return TELBM_OK;
}

int telbm_sync(telbm_solver* s) {
    if (!s) return TELBM_ERR_INVAL;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "stream synchronise");
    int rc = consume_diag(s);
    if (rc) return rc;
    if (s->last.step >= 0 && unstable(s->last)) return fail(s, TELBM_ERR_UNSTABLE, "unstable state detected");
    return TELBM_OK;
}

int telbm_read(telbm_solver* s, int field, double* out, int on_device) {
    if (!s || !out) return TELBM_ERR_INVAL;
    if (field < 0 || field > kFieldFz) return fail(s, TELBM_ERR_INVAL, "unknown field");
    int rc = ensure_aux(s);
    if (rc) return rc;
    StepArgs a = args_of(s, false);
    double* dst = on_device ? out : (double*)s->pop[1 - s->cur];
    hipError_t e = launch_macro(s->p.lattice, s->p.precision, a, field, dst);
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(out, dst, s->g.N * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "read");
    return telbm_sync(s);
}

int telbm_diagnostics(telbm_solver* s, telbm_diag* out) {
    if (!s || !out) return TELBM_ERR_INVAL;
    if (s->diag_step != s->steps) {
        // diagnostic pass over the current state: a collision into the spare
        // buffer with the diagnostics on; the state itself is not advanced
        int rc = ensure_aux(s);
        if (rc) return rc;
        StepArgs a = args_of(s, true);
        a.diag = 1;
        hipError_t e = launch_part(s->p.lattice, s->p.precision, a, 2);
        if (e != hipSuccess) return hip_fail(s, e, "diagnostic launch");
        s->diag_step = s->steps;
        s->diag_unread = true;
    }
    int rc = telbm_sync(s);
    *out = s->last;
    return rc;
}

int telbm_last_diagnostics(telbm_solver* s, telbm_diag* out) {
    if (!s || !out) return TELBM_ERR_INVAL;
    int rc = telbm_sync(s);
    *out = s->last;
    return rc;
}

int telbm_step_count(const telbm_solver* s, int64_t* steps) {
    if (!s || !steps) return TELBM_ERR_INVAL;
    *steps = s->steps;
    return TELBM_OK;
}

int telbm_time_kernels(telbm_solver* s, int64_t n, double* ms, int* kinds) {
    if (!s || !ms || !kinds || n < 1) return TELBM_ERR_INVAL;
    Timing t;
    t.pool.resize(3 * n);
    int rc = TELBM_OK;
    size_t made = 0;
    for (auto& pr : t.pool) {
        if (hipEventCreate(&pr.first) != hipSuccess) { rc = fail(s, TELBM_ERR_DEVICE, "event create"); break; }
        if (hipEventCreate(&pr.second) != hipSuccess) { (void)hipEventDestroy(pr.first); rc = fail(s, TELBM_ERR_DEVICE, "event create"); break; }
        ++made;
    }
    for (int64_t i = 0; i < n && rc == TELBM_OK; ++i) {
        const bool diag = s->p.diag_every > 0 && (s->steps % s->p.diag_every) == 0;
        rc = one_step(s, diag, &t);
    }
    if (rc == TELBM_OK) {
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) rc = hip_fail(s, e, "timed synchronise");
    }
    if (rc == TELBM_OK) {
        double sum[kKinds] = {0, 0, 0};
        int cnt[kKinds] = {0, 0, 0};
        for (size_t i = 0; i < t.used; ++i) {
            float ms1 = 0.f;
            if (hipEventElapsedTime(&ms1, t.pool[i].first, t.pool[i].second) != hipSuccess) continue;
            sum[t.kind[i]] += ms1;
            cnt[t.kind[i]] += 1;
        }
        for (int k = 0; k < kKinds; ++k) ms[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
        // the whole timed span per step: first launch's start event to the
        // last launch's end event, on the solver's stream
        float span = 0.f;
        ms[kKinds] = 0.0;
        if (t.used > 0 && hipEventElapsedTime(&span, t.pool[0].first, t.pool[t.used - 1].second) == hipSuccess)
            ms[kKinds] = span / (double)n;
        *kinds = kKinds;
    }
    for (size_t i = 0; i < made; ++i) {
        (void)hipEventDestroy(t.pool[i].first);
        (void)hipEventDestroy(t.pool[i].second);
    }
    return rc;
}

const char* telbm_kernel_name(const telbm_solver* s, int kind) {
    (void)s;
    if (kind < 0 || kind >= kKinds) return "";
    return kKernelNames[kind];
}

double telbm_algorithmic_bytes_per_update(const telbm_solver* s) {
    if (!s) return 0.0;
    const double b = s->p.precision == TELBM_FP32_MIXED ? 4.0 : 8.0;
    return 2.0 * pops_per_node(s->p) * b;
}

int telbm_destroy(telbm_solver* s) {
    if (!s) return TELBM_ERR_INVAL;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    delete s;
    return TELBM_OK;
}

const char* telbm_last_error(const telbm_solver* s) {
    if (!s) return "null solver";
    return s->err.c_str();
}

int telbm_nl_mobility(const telbm_params* p, const telbm_nl_params* q, double* m) {
    if (!p || !q || !m) return TELBM_ERR_INVAL;
    return nl_mobility(*p, *q, m) ? TELBM_OK : TELBM_ERR_INVAL;
}

int telbm_nl_required_bytes(const telbm_params* p, const telbm_nl_params* q, size_t* bytes) {
    std::string why;
    if (!bytes) return TELBM_ERR_INVAL;
    int rc = nl_validate(p, q, &why);
    if (rc) return rc;
    *bytes = nl_layout(*p).total;
    return TELBM_OK;
}

int telbm_nl_create(const telbm_params* p, const telbm_nl_params* q, void* device_arena, size_t bytes,
                    telbm_nl** out) {
    if (!out) return TELBM_ERR_INVAL;
    *out = nullptr;
    std::string why;
    int rc = nl_validate(p, q, &why);
    if (rc) return rc;
    const NlLayout L = nl_layout(*p);
    if (!device_arena || ((uintptr_t)device_arena % kAlign) != 0) return TELBM_ERR_INVAL;
    if (bytes < L.total) return TELBM_ERR_NOMEM;
    double rg = p->rho_g, rl = p->rho_l, C = 0.0, psi0 = 0.0, mg, ml;
    if (!eos_maxwell(eos_of(*p), p->T, &mg, &ml, &C, &psi0)) return TELBM_ERR_INVAL;
    if (rg == 0.0 && rl == 0.0) {
        rg = mg;
        rl = ml;
    }
    telbm_nl* s = new (std::nothrow) telbm_nl();
    if (!s) return TELBM_ERR_NOMEM;
    s->p = *p;
    s->p.rho_g = rg;
    s->p.rho_l = rl;
    s->q = *q;
    NlArgs& a = s->a;
    a.g = GridDims{p->nx, p->ny, p->nz, 0, (int64_t)p->nx * p->ny * p->nz};
    a.k = derive(*p, rg, rl, C);
    a.q.kappa1 = p->kappa1;
    a.q.kappa2 = p->kappa2;
    a.q.kappa3 = p->kappa3;
    a.q.kappa4 = q->kappa4;
    a.q.lambda4 = q->lambda4;
    nl_mobility(*p, *q, a.q.m);
    char* base = (char*)device_arena;
    s->pop[0] = base;
    s->pop[1] = base + L.pop;
    double** f[6] = {&a.rho, &a.phi, &a.psi, &a.mux, &a.mup, &a.mus};
    for (int i = 0; i < 6; ++i) *f[i] = (double*)(base + 2 * L.pop + i * L.aux);
    char* nx = base + 2 * L.pop + 6 * L.aux;
    a.partA = L.partA ? (double*)nx : nullptr;
    a.inboxA = L.partA ? (double*)(nx + L.partA) : nullptr;
    a.partB = L.partA ? (double*)(nx + L.partA + L.inboxA) : nullptr;
    a.inboxB = L.partA ? (double*)(nx + L.partA + L.inboxA + L.partB) : nullptr;
    a.u0 = nullptr;
    a.stream = nullptr;
    s->cur = 0;
    s->aux_valid = false;
    s->partial = false;
    s->steps = 0;
    *out = s;
    return TELBM_OK;
}

int telbm_nl_set_stream(telbm_nl* s, void* stream) {
    if (!s) return TELBM_ERR_INVAL;
    s->a.stream = (hipStream_t)stream;
    return TELBM_OK;
}

int telbm_nl_init_fields(telbm_nl* s, const double* rho, const double* phi, const double* psi, const double* u,
                         int on_device) {
    if (!s) return TELBM_ERR_INVAL;
    if (!rho || !phi || !psi) return nl_fail(s, TELBM_ERR_INVAL, "rho, phi and psi are required");
    NlArgs& a = s->a;
    const int64_t N = a.g.N;
    const int D = s->p.lattice == TELBM_D2Q9 ? 2 : 3;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    // u is staged in the spare population buffer, the check count in mux
    double* u_dev = u ? (double*)s->pop[1 - s->cur] : nullptr;
    auto* bad = (unsigned long long*)a.mux;
    hipError_t e = hipMemcpyAsync(a.rho, rho, N * sizeof(double), kind, a.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(a.phi, phi, N * sizeof(double), kind, a.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(a.psi, psi, N * sizeof(double), kind, a.stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u_dev, u, (size_t)D * N * sizeof(double), kind, a.stream);
    if (e == hipSuccess) e = launch_check_init(a.g, D, a.rho, a.phi, u_dev, bad, a.stream);
    unsigned long long nbad[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(&nbad[0], bad, sizeof(nbad[0]), hipMemcpyDeviceToHost, a.stream);
    if (e == hipSuccess) e = launch_check_init(a.g, D, a.rho, a.psi, nullptr, bad, a.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&nbad[1], bad, sizeof(nbad[1]), hipMemcpyDeviceToHost, a.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(a.stream);
    if (e != hipSuccess) return nl_fail(s, TELBM_ERR_DEVICE, std::string("init staging: ") + hipGetErrorString(e));
    s->aux_valid = false;
    s->partial = false;
    if (nbad[0] || nbad[1])
        return nl_fail(s, TELBM_ERR_UNSTABLE, std::to_string(nbad[0] + nbad[1]) + " nodes with unusable initial values");
    // potentials of the initial fields, then the equilibria into pop[cur]
    a.u0 = u_dev;
    e = nl_launch(s, 1);
    if (e == hipSuccess) e = nl_launch(s, 3);
    a.u0 = nullptr;
    if (e != hipSuccess) return nl_fail(s, TELBM_ERR_DEVICE, std::string("init launch: ") + hipGetErrorString(e));
    s->aux_valid = false;
    s->partial = false;
    s->steps = 0;
    return TELBM_OK;
}

int telbm_nl_step(telbm_nl* s, int64_t n) {
    if (!s || n < 0) return TELBM_ERR_INVAL;
    for (int64_t i = 0; i < n; ++i) {
        int rc = nl_ensure_aux(s);
        if (rc) return rc;
        // D3Q27: the collision also leaves the next moments (no moment pass)
        const bool d3 = s->p.lattice == TELBM_D3Q27;
        hipError_t e = nl_launch(s, d3 ? 4 : 2);
        if (e != hipSuccess) return nl_fail(s, TELBM_ERR_DEVICE, std::string("collision launch: ") + hipGetErrorString(e));
        s->cur = 1 - s->cur;
        s->aux_valid = false;
        s->partial = d3;
        s->steps += 1;
    }
    return TELBM_OK;
}

int telbm_nl_read(telbm_nl* s, int field, double* out, int on_device) {
    if (!s || !out) return TELBM_ERR_INVAL;
    if (field < 0 || field > kNlFz) return nl_fail(s, TELBM_ERR_INVAL, "unknown field");
    int rc = nl_ensure_aux(s);
    if (rc) return rc;
    NlArgs a = s->a;
    a.src = (const double*)s->pop[s->cur];
    double* dst = on_device ? out : (double*)s->pop[1 - s->cur];
    hipError_t e = launch_nl_macro(s->p.lattice, a, field, dst);
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(out, dst, a.g.N * sizeof(double), hipMemcpyDeviceToHost, a.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(a.stream);
    if (e != hipSuccess) return nl_fail(s, TELBM_ERR_DEVICE, std::string("read: ") + hipGetErrorString(e));
    return TELBM_OK;
}

int telbm_nl_step_count(const telbm_nl* s, int64_t* steps) {
    if (!s || !steps) return TELBM_ERR_INVAL;
    *steps = s->steps;
    return TELBM_OK;
}

int telbm_nl_destroy(telbm_nl* s) {
    if (!s) return TELBM_ERR_INVAL;
    if (s->a.stream) (void)hipStreamSynchronize(s->a.stream);
    else (void)hipDeviceSynchronize();
    delete s;
    return TELBM_OK;
}

const char* telbm_nl_last_error(const telbm_nl* s) {
    if (!s) return "null solver";
    return s->err.c_str();
}

}  // extern "C"
