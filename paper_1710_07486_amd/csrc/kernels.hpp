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
    int pad;
    int64_t N;
};

struct StepArgs {
    GridDims g;
    PhysConst k;
    const void* src;     // populations holding the current state
    void* dst;           // populations receiving the next state
    const double* rho_ref;  // density the stored f values are relative to (FP32 form)
    double *rho, *phi, *mux, *mup;
    double* partials;    // per-block diagnostic partials
    double* diag_out;    // final diagnostics (kDiag doubles)
    int diag;
    hipStream_t stream;
};

unsigned collide_blocks(const GridDims& g);

// part 0: moments, 1: chemical potentials, 2: collision (+ diagnostics)
hipError_t launch_part(int lattice, int precision, const StepArgs& a, int part);
hipError_t launch_init(int lattice, int precision, const StepArgs& a, const double* u0);
hipError_t launch_check_init(const GridDims& g, int D, const double* rho, const double* phi, const double* u0,
                             unsigned long long* bad, hipStream_t s);
hipError_t launch_macro(int lattice, int precision, const StepArgs& a, int field, double* out);

}  // namespace telbm
