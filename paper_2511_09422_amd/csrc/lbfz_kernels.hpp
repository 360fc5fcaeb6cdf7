// lbfz_kernels.hpp -- launch interface between the C ABI and the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbfz_common.hpp"

namespace lbfz {

// Buffers of one step.  src/dst: population buffers; p, u: double-buffered
// previous-time-level fields read through stencils; fs: pointwise
// previous-time-level f_s updated in place; phiP, CP: previous-level phi and C
// (FP32 storage: one buffer, old == new, updated in place; 16-bit storage:
// double-buffered, they are also the populations' decode references, as are
// T and p_ref, the pressure two levels back).  DRY launches evaluate the
// macroscopic fields of the current time level into out[] (any entry may be
// null) and per-tile totals into tot_part[tile * 8 + k].
struct StepArgs {
  const float* src;
  float* dst;
  const float* p_old;
  float* p_new;
  const float* p_ref;  // 16-bit storage only
  const float* u_old;  // [dim][ps]
  float* u_new;
  float* fs;
  const float* phiP_old;
  float* phiP_new;
  const float* CP_old;
  float* CP_new;
  const float* T_old;  // 16-bit storage only
  float* T_new;
  const float* cf_old;  // 3D closure fields phi, T, C, f_s, div u [5][ps]: previous level
  float* cf_new;        //   and this level
  const uint8_t* mask;  // 3D obstacle mask or null
  double* mpc_part;     // [ntiles]
  float* out[9];
  double* tot_part;     // [ntiles][8]
  int rev;              // 2D: walk the tiles in reverse (odd steps)
};

// Buffers the initial state is written to (pop: the buffer the first step
// reads; pC: 16-bit storage only; TA: 16-bit 2D and 3D; DA: 3D only).
struct StateArgs {
  float *pA, *pB, *pC, *uA, *uB, *fs, *phiA, *CA, *TA, *DA;
};

// One grid of the batched sweep: its kernel parameters and the buffers of
// each step parity slot (2 slots with FP32 storage, 6 with 16-bit storage,
// whose pressure is triple-buffered).
struct BatchCase {
  KParams P;
  StepArgs A[6];
};

int tiles2d(int nx, int ny, int* nbx, int* nby, int ty = 0);
size_t pop_bytes2d(int storage, size_t ps);
hipError_t launch_init2d(const KParams& P, int storage, const double* phi, const double* T,
                         const double* C, float* pop, const StateArgs& S, hipStream_t st);
hipError_t launch_step2d(const KParams& P, int storage, const StepArgs& A, bool dry,
                         hipStream_t st);
hipError_t launch_step2d_batch(int storage, int ty, const BatchCase* cases, const int2* work,
                               int nwork, int grid, int slot, hipStream_t st);
hipError_t launch_fields2d_batch(int storage, int ty, const BatchCase* cases, const int2* work,
                                 int nwork, int slot, float* dst, long case_stride,
                                 uint32_t mask, hipStream_t st);
hipError_t launch_export2d(const KParams& P, int storage, const StepArgs& A, float* dst,
                           hipStream_t st);
hipError_t launch_import2d(const KParams& P, int storage, const StepArgs& A, const float* src,
                           hipStream_t st);

// Macroscopic fields of a 2D restart (device FP32 planes of N values) and the
// 30 raw state planes it writes (the exported layout).
struct EquilFields {
  const float *phi, *fl, *T, *C, *ux, *uy, *p;
};
struct StatePlanes {
  float* p[30];
};
hipError_t launch_equil2d(const KParams& P, const EquilFields& F, const StatePlanes& S,
                          hipStream_t st);
// One grid of a batched restart: its parameters, fields and state planes.
struct EquilJob {
  KParams P;
  EquilFields F;
  StatePlanes S;
};
// The restarts of njobs grids (jobs: a device table) in one launch.
hipError_t launch_equil2d_batch(const EquilJob* jobs, int njobs, long max_n, hipStream_t st);

int tiles3d(int nx, int ny, int nz, int storage, int* nbx, int* nby, int* nbz);
size_t pop_bytes3d(int storage, size_t ps);
hipError_t launch_init3d(const KParams& P, int storage, const double* phi, const double* T,
                         const double* C, const uint8_t* mask, float* popA, float* popB,
                         const StateArgs& S, hipStream_t st);
hipError_t launch_step3d(const KParams& P, int storage, const StepArgs& A, bool dry,
                         hipStream_t st);
hipError_t launch_export3d(const KParams& P, int storage, const StepArgs& A, float* dst,
                           hipStream_t st);
hipError_t launch_import3d(const KParams& P, int storage, const StepArgs& A, const float* src,
                           hipStream_t st);

}  // namespace lbfz
