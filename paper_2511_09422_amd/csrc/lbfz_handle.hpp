// lbfz_handle.hpp -- the solver handle behind the C ABI (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbfz.h"
#include "lbfz_common.hpp"
#include "lbfz_kernels.hpp"

struct lbfz_handle {
  lbfz_params prm;
  lbfz::KParams kp;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  int storage;
  float* pop[2];
  float* p[3];     // FP32: two levels; 16-bit: three (p_ref)
  float* u[2];
  float* fs;       // 2D
  float* phiP[2];  // 2D; FP32: [1] == [0] (updated in place)
  float* CP[2];
  float* T[2];     // 2D 16-bit only
  float* cf[2];    // 3D closure fields (phi, T, C, f_s, div u planes) per level
  bool narrow;     // 16-bit population storage
  double* mpc_part;
  double* tot_part;
  double* red;
  float* stage;
  uint8_t* mask;
  int cur;
  int64_t step;
  int ntiles;
  int npop;
};

namespace lbfz {
// Buffers of the next step of h from its current level.
StepArgs base_args(lbfz_handle* h);
// One step (dry: fields / totals only) of h on its stream.
hipError_t launch_step(lbfz_handle* h, const StepArgs& a, bool dry);
// The equilibrium restart of a 2D FP32-storage grid from device fields
// (lbfz_restart_fields) as a job of a batched launch; LBFZ_EUNSUPPORTED for
// 3D or 16-bit storage (their restart needs the per-grid import pass).
int restart_job(lbfz_handle* h, const float* const* d_fields, EquilJob* job);
}  // namespace lbfz
