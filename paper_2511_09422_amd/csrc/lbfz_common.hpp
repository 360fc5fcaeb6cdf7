// lbfz_common.hpp -- device-side parameters and pointwise physics shared by
// the 2D and 3D step kernels of the coupled LB freezing scheme
// (arXiv 2511.09422, Sec. 2-3).  FP32 arithmetic; FP64 only in reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbfz.h"

namespace lbfz {

constexpr float kCs2 = 1.0f / 3.0f;
constexpr float kInvCs2 = 3.0f;

// Kernel parameter block: every constant the step needs, derived once on the
// host from lbfz_params and passed by value.
struct KParams {
  int nx, ny, nz, N;
  int ps;  // stride between the planes of one array (elements), >= N
  int walls, tlo_dir, thi_dir, st_mode;
  int nblk_x, nblk_y, nblk_z, nblk;  // tile grid (logical)
  // property end members (end of Sec. 2)
  float rho_l, rho_g, rho_s, cp_l, cp_s, cp_g;
  float rc_l, rc_s, rc_g;  // rho * c_p of each phase
  float rhoc_ref, rho_l_latent, T_sol, T_liq;
  float ratio;  // 1 - rho_s / rho_l (Eq. NS1)
  // relaxation (Sec. 3.1-3.4)
  // tau_gp = tau_g - 1/2: the weight of G_0 in the pressure (Sec. 3.2; the
  // first-order non-equilibrium part of the rest population); wg = 1 - 1/(2 tau)
  float tau_gp, itau_g, wg;
  float itau_f, wf;
  float itau_a, itau_s, ws;  // enthalpy TRT: antisymmetric / symmetric
  float Dl, Ds, k_p;
  // interface and forces (Sec. 2, Eq. Fs)
  float alpha, ieps2, isq;  // isq = 1/(sqrt(2) eps)
  float sigma0, sigma_T, sigma_c, T_ref, c_ref;
  float bfx, bfy, bfz;
  // walls
  float T_lo, T_hi, T_lo_amp, kwall;  // kwall = 2 pi / nx
};

__device__ __forceinline__ float clamp01(float v) { return fminf(fmaxf(v, 0.0f), 1.0f); }

// Property interpolation, end of Sec. 2.
__device__ __forceinline__ float interp(float phi, float fs, float zl, float zg, float zs) {
  return 0.5f * phi * (zl - zg) + fs * (zs - zl) + 0.5f * (zl + zg);
}

// Reciprocal by the hardware instruction (about 1 ulp); the scheme's
// denominators are all O(0.1 .. 10), far from the denormal and overflow range.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Enthalpy -> (T, f_s) map of Eq. (Hfl) with the heat capacities and the
// latent heat weighted by the phase-change-material fraction psi; f_s =
// psi (1 - f_l).  At psi = 1 this is Eq. (Hfl).  The three branches share one
// reciprocal (solid: E / rcs, liquid: (E - El) / rcl, mushy: (E - Es) / d).
__device__ __forceinline__ void enthalpy_map(const KParams& P, float E, float psi, float& T,
                                             float& fs) {
  const float rcs = psi * P.rc_s + (1.0f - psi) * P.rc_g;
  const float rcl = psi * P.rc_l + (1.0f - psi) * P.rc_g;
  const float Es = rcs * P.T_sol;
  const float El = rcl * P.T_liq + psi * P.rho_l_latent;
  const bool below = E < Es, above = E > El;
  const float d = El - Es;
  const bool flat = d <= 1e-12f * fmaxf(1.0f, fabsf(E));  // pure substance, no latent heat
  const float den = below ? rcs : (above ? rcl : (flat ? 1.0f : d));
  const float q = (below ? E : (above ? E - El : E - Es)) * frcp(den);
  const float fl = below ? 0.0f : (above ? 1.0f : (flat ? 1.0f : q));
  T = below ? q : (above ? P.T_liq + q : P.T_sol + fl * (P.T_liq - P.T_sol));
  fs = psi * (1.0f - fl);
}

// Pointwise closure of one node from its raw moments (Sec. 3.1, 3.3, Eq. NS1):
// phi from phi0 and div u, then one predictor and one corrector of the
// implicit enthalpy moment.  Outputs phi, T, f_s and the enthalpy source Q.
struct Closure {
  float phi, T, fs, E, Q;
};

__device__ __forceinline__ Closure closure(const KParams& P, float phi0, float E0, float D) {
  Closure c;
  const float psi = clamp01(0.5f * (1.0f + phi0));
  // correctly rounded: the phase-field budget sum f(n+1) - sum f(n) = phi D
  // holds only through phi0 = phi (1 - D / 2), and a biased quotient would
  // accumulate in it
  c.phi = phi0 / (1.0f - 0.5f * D);
  float T0, fs0;
  enthalpy_map(P, E0, psi, T0, fs0);
  const float rc0 = interp(c.phi, fs0, P.rho_l, P.rho_g, P.rho_s) *
                    interp(c.phi, fs0, P.cp_l, P.cp_g, P.cp_s);
  c.Q = rc0 * T0 * D;
  c.E = E0 + 0.5f * c.Q;
  enthalpy_map(P, c.E, psi, c.T, c.fs);
  return c;
}

// Wave64 + block reduction of doubles into lds scratch (blockDim.x threads).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sred) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sred[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += sred[w];
  }
  return s;  // valid on thread 0
}

// 2D population planes of a direction with an x component are stored shifted
// by -c_x nodes: node m's population i sits at element m - c_x,i of its
// plane.  A push-streamed write from node x to x + c_i then lands at flat
// element x + c_y,i nx -- a wave's 64 writes fill aligned cache lines -- and
// the misalignment moves to the reads of the next step, which the caches
// absorb (FP32 step 217 -> 209 us at 2048^2).  The planes' padding holds the
// one element a plane reaches past either end.  The 3D step keeps its planes
// unshifted: shifted, its FP32 step was no faster and its 16-bit step slower
// (its reads are the critical path).
constexpr int kXS = 1;
// A 2D population set's buffer descriptor starts this many bytes before its
// first plane, so that the (unsigned) plane offsets stay positive for a
// first plane shifted by -1 element.
constexpr uint32_t kSetPad = 256;

// Word 3 of a CDNA buffer descriptor: 32-bit data format, no swizzle.
constexpr int kBufWord3 = 0x00020000;

// Buffer descriptor of `bytes` bytes at `base`; accesses through it are one
// buffer instruction each: descriptor and plane offset wave-uniform (scalar
// registers), the lane supplies only a 32-bit byte offset.  Offsets outside
// the range read 0 and write nothing.
using rsrc_t = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ rsrc_t rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           kBufWord3);
}
// Cache policy of the loads and stores: stores carry the non-temporal hint
// (every plane a step writes is read only by the next step, after the whole
// grid has streamed through the caches; 2048^2 FP32 step 208 -> 200 us),
// loads the default policy (non-temporal loads lose the reuse of the halo
// rows between neighbouring tiles: 254 us).  The values are the cache-policy
// operand of the buffer instructions: 0 default, 2 non-temporal.
constexpr int kLdPolicy = 0;
constexpr int kStPolicy = 2;
__device__ __forceinline__ float ld(rsrc_t r, uint32_t off, uint32_t soff = 0) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, (int)soff,
                                                                          kLdPolicy));
}
__device__ __forceinline__ void st(rsrc_t r, uint32_t off, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, (int)soff,
                                        kStPolicy);
}
// Stores with the default cache policy: the 3D step's (its two launches read
// the closure fields back at once, and its population writes measured
// slower with the hint: 1.80 -> 1.89 ms at 256^3).
__device__ __forceinline__ void st_keep(rsrc_t r, uint32_t off, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, (int)soff, 0);
}
__device__ __forceinline__ void st16_keep(rsrc_t r, uint32_t off, uint32_t soff, uint16_t v) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)off, (int)soff, 0);
}
__device__ __forceinline__ uint16_t ld16(rsrc_t r, uint32_t off, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, (int)soff, kLdPolicy);
}
__device__ __forceinline__ uint8_t ld8(rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
}
__device__ __forceinline__ void st16(rsrc_t r, uint32_t off, uint32_t soff, uint16_t v) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)off, (int)soff, kStPolicy);
}

// 16-bit storage: offsets from the reference are scaled by these powers of two
// (exact) so that typical offsets sit in the FP16 normal range.
constexpr float SC_F = 256.0f, SC_G = 16384.0f, SC_H = 1024.0f, SC_L = 4096.0f;

// 16-bit storage formats: round to nearest even either way.
template <int ST>
__device__ __forceinline__ float dec16(uint16_t b) {
  if constexpr (ST == LBFZ_STORE_F16)
    return (float)__builtin_bit_cast(_Float16, b);
  else
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}
template <int ST>
__device__ __forceinline__ uint16_t enc16(float v) {
  if constexpr (ST == LBFZ_STORE_F16)
    return __builtin_bit_cast(uint16_t, (_Float16)v);
  else
    return __builtin_bit_cast(uint16_t, (__bf16)v);
}

// Periodic image of v in [-n, 2n); positions beyond that (staged only by
// partial tiles, never read for a node of the grid) are clamped into it.
__device__ __forceinline__ int wrap_near(int v, int n) {
  return v < 0 ? v + n : (v >= n ? min(v - n, n - 1) : v);
}

// Map a hardware block index to a logical tile index so that each of the 8
// XCDs (blocks are dealt round-robin to them) works on one contiguous band of
// tiles and the halo rows it re-reads stay in its own L2.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
  const int per = nblk >> 3;
  if (per == 0 || (nblk & 7)) return b;
  return (b & 7) * per + (b >> 3);
}
// The same bands, each walked from its last tile to its first.  A launch that
// follows one walked forward starts on the tiles whose data the previous
// launch touched last, while part of it is still in the memory-side cache
// (bit-identical results: tiles are independent and per-tile partial sums are
// indexed by tile).
__device__ __forceinline__ int xcd_tile_rev(int b, int nblk) {
  const int per = nblk >> 3;
  if (per == 0 || (nblk & 7)) return nblk - 1 - b;
  return (b & 7) * per + (per - 1 - (b >> 3));
}

}  // namespace lbfz
