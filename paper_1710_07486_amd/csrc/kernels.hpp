// kernels.hpp -- internal interface between the C ABI (api.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace telbm {

constexpr int kDiag = 10;  // sum rho, sum phi, sum j (3), max |u|, min rho, min/max gamma, nonfinite

// field codes, equal to the TELBM_FIELD_* values of the ABI
constexpr int kFieldRho = 0, kFieldPhi = 1, kFieldUx = 2, kFieldUy = 3, kFieldUz = 4, kFieldC1 = 5,
              kFieldC2 = 6, kFieldMuRho = 7, kFieldMuPhi = 8, kFieldFx = 9, kFieldFy = 10, kFieldFz = 11;

struct GridDims {
    int nx, ny, nz;
    int walls;  // 1: solid walls at y = -1/2 and y = ny - 1/2 (x, z stay periodic)
    int64_t N;
};

struct StepArgs {
    GridDims g;
    PhysConst k;
    const void* src;     // populations holding the current state
    void* dst;           // populations receiving the next state
    const double* rho_ref;  // density the stored f values are relative to (FP32 form)
    double *rho, *phi, *mux, *mup;
    // D2Q9 fused step (part 3): rho / phi may be partial sums completed from
    // inbox_in (null: complete); the step leaves the next state's partial
    // moments in rho_next / phi_next and their inbox entries in inbox_out;
    // FP32 form: the completed densities (the new reference) in rho_final.
    // Part 4 completes rho / phi in place from inbox_in.
    const double* inbox_in;
    double *rho_next, *phi_next, *inbox_out, *rho_final;
    // D3Q27 FP64: next-step moments as partial sums (part3_doubles: the sums
    // of each node's own z-column and of the neighbouring columns at column
    // ends) and their inbox entries (part 6 writes, part 5 completes them
    // while computing the chemical potentials)
    double *part3, *inbox3;
    double* partials;    // per-block diagnostic partials
    unsigned partials_blocks;  // blocks the partials hold (kDiag doubles each)
    double* diag_out;    // final diagnostics (kDiag doubles)
    int diag;
    hipStream_t stream;
};

// Per-instance pointers of the batched fused 2D step (k_batch_fused2).
struct FusedDesc {
    GridDims g;
    PhysConst k;
    void* pop[2];
    double* rhob[2];            // FP32 form: reference / completed densities
    double *xr[2], *xp[2];      // current / next (partial) densities and phase field
    double* inbox[2];
};

// One launch of the fused 2D step over an (instance, tile) work list (tile
// index = by * fused_tiles_x(nx) + bx on 64 x 8 tiles, one workgroup per
// item) whose instances all have the equation of state `eos`; `walls`: some
// instance has walls (the kernel instance with the wall logic).
hipError_t launch_batch_fused2(int precision, int eos, bool walls, hipStream_t st, const FusedDesc* inst,
                               const int2* work, int nwork, int cur, int ref, int fp, int partial);
int fused_tiles_x(int nx);

unsigned collide_blocks(const GridDims& g);
unsigned fused_tiles(const GridDims& g);        // D2Q9 tiles of the fused step
size_t inbox_doubles(const GridDims& g);        // size of one inbox array
// D3Q27 collisions that leave the next moments walk z-columns of kZc planes
// per workgroup.  Sizes of the partial sums and their inboxes (nf fields per
// entry: 2 for (rho, phi) pairs, 1 for psi alone), and the workgroups of such
// a collision.
constexpr int kZc = 32;
size_t part3_doubles(const GridDims& g, int nf);
size_t inbox3_doubles(const GridDims& g, int nf);
unsigned column_blocks(const GridDims& g);

// part 0: moments, 1: chemical potentials, 2: collision (+ diagnostics);
// D2Q9 only: 3: fused potentials + collision + tile sums of the next moments,
// 4: completion of partial moments at the tile edges; D3Q27 only: 5: chemical
// potentials completing the partial moments, 6: FP64 collision + partial
// sums of the next moments
hipError_t launch_part(int lattice, int precision, const StepArgs& a, int part);
hipError_t launch_init(int lattice, int precision, const StepArgs& a, const double* u0);
hipError_t launch_check_init(const GridDims& g, int D, const double* rho, const double* phi, const double* u0,
                             unsigned long long* bad, hipStream_t s);
hipError_t launch_macro(int lattice, int precision, const StepArgs& a, int field, double* out);

// Three liquids and the gas (nliquid.hip): constants beyond PhysConst, the
// step's buffers, and the field codes of its read-out (the TELBM_NL_FIELD_*
// values of the ABI).
struct NlConst {
    double kappa1, kappa2, kappa3, kappa4;  // gradient coefficients of rho and the three liquids
    double lambda4;                         // double well of liquid 3
    double m[4];                            // mobility matrix / M: pp, ps, sp, ss
};

struct NlArgs {
    GridDims g;
    PhysConst k;
    NlConst q;
    const double* src;  // populations of the state: f, g (phi), h (psi), 3 Q slices of N
    double* dst;        // populations receiving the next state (part 3: the initial state)
    double *rho, *phi, *psi, *mux, *mup, *mus;
    const double* u0;   // part 3: initial velocity ([D][N]) or null
    // D3Q27: next-step moments as partial sums, (rho, phi) pairs in partA
    // and psi in partB (part3_doubles with 2 and 1 fields), with their
    // inboxes (inbox3_doubles likewise): part 4 writes them, parts 5 and 6
    // complete them
    double *partA, *inboxA, *partB, *inboxB;
    hipStream_t stream;
};

constexpr int kNlRho = 0, kNlPhi = 1, kNlPsi = 2, kNlUx = 3, kNlUy = 4, kNlUz = 5, kNlC1 = 6, kNlC2 = 7,
              kNlC3 = 8, kNlMuRho = 9, kNlMuPhi = 10, kNlMuPsi = 11, kNlFx = 12, kNlFy = 13, kNlFz = 14;

// part 0: moments (rho, phi, psi), 1: potentials, 2: collision src -> dst,
// 3: equilibria of (rho, phi, psi, u0) into dst (potentials current);
// D3Q27 only: 4: collision src -> dst that also leaves the next moments as
// partial sums, 5: completion of those into rho, phi, psi, 6: completion and
// potentials in one z-column pass.
hipError_t launch_nl_part(int lattice, const NlArgs& a, int part);
hipError_t launch_nl_macro(int lattice, const NlArgs& a, int field, double* out);

}  // namespace telbm
