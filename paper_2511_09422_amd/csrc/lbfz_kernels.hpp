// lbfz_kernels.hpp -- launch interface between the C ABI and the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbfz_common.hpp"

namespace lbfz {

// Buffers of one step.  src/dst: population buffers; p, u: double-buffered
// previous-time-level fields read through stencils; fs, phiP, CP: pointwise
// previous-time-level fields updated in place.  DRY launches evaluate the
// macroscopic fields of the current time level into out[] (any entry may be
// null) and per-tile totals into tot_part[tile * 8 + k].
struct StepArgs {
  const float* src;
  float* dst;
  const float* p_old;
  float* p_new;
  const float* u_old;  // [dim][N]
  float* u_new;
  float* fs;
  float* phiP;
  float* CP;
  const uint8_t* mask;  // 3D obstacle mask or null
  double* mpc_part;     // [ntiles]
  float* out[9];
  double* tot_part;     // [ntiles][8]
};
using Step2DArgs = StepArgs;

struct StateArgs {
  float *pA, *pB, *uA, *uB, *fs, *phiP, *CP;
};

int tiles2d(int nx, int ny, int* nbx, int* nby);
hipError_t launch_init2d(const KParams& P, const double* phi, const double* T, const double* C,
                         float* pop, const StateArgs& S, hipStream_t st);
hipError_t launch_step2d(const KParams& P, const StepArgs& A, bool dry, hipStream_t st);

int tiles3d(int nx, int ny, int nz, int seg, int* nbx, int* nby, int* nbz);
size_t lds3d_bytes();
hipError_t launch_init3d(const KParams& P, const double* phi, const double* T, const double* C,
                         const uint8_t* mask, float* popA, float* popB, const StateArgs& S,
                         hipStream_t st);
hipError_t launch_step3d(const KParams& P, const StepArgs& A, int seg, bool dry, hipStream_t st);

}  // namespace lbfz
