// lbfz_3d.hip -- 3D step of the coupled LB freezing scheme (arXiv
// 2511.09422, Sec. 3) for gfx950: D3Q19 flow g, D3Q7 phase field f, enthalpy
// h (TRT) and solute l; walls on z, periodic x and y; optional obstacle mask
// (bounce-back for f, g, l; h conducts through it).
//
// Two launches per step, each one node per thread on tiles of 64 x TY x TZ
// nodes, one x row per wave (closure: FP32 storage 64 x 4 x 4, 16-bit
// 64 x 4 x 2; collision: 64 x 1 x 4, 64 x 4 x 1):
//   k_close3d    the pointwise closure of every node -- phi, T, C, f_s from
//                its f, h, l populations and div u^{n-1} from a velocity ring
//                staged in LDS -- into the closure-field buffer of the level;
//   k_collide3d  stencils of phi, T, C, f_s and p^{n-1} from the tile and
//                its 1-ring staged in LDS, forces, velocity, pressure, the four
//                collisions and push streaming into the other population
//                buffer.
// The closure-field buffers (phi, T, C, f_s, div u) are double-buffered: the
// previous level's buffer is the scheme's previous-level state (f_s^{n-1},
// phi^{n-1}, C^{n-1}) and, with 16-bit storage, the populations' decode
// references.  Compared with one fused launch (the closure of the halo
// recomputed per tile), the split re-reads the f, h, l populations once
// (+76 B) and moves the closure fields through HBM (+36 B), in exchange for
// full occupancy and one memory round trip per launch.
//
// Population storage (template parameter ST):
//   F32   40 FP32 planes: f 0..6, g 7..25, h 26..32, l 33..39 (with the D3Q7
//         weights the rest components of f and l are identically zero: those
//         planes are never read or written).
//   F16 / BF16  FP32 rest planes g0, h0, then 36 16-bit moving planes (f1..6,
//         g1..18, h1..6, l1..6) stored as offsets (v - w_i r) S from the
//         reference moments of the node they sit at, as in the 2D step.
#include <type_traits>

#include "../../include/lbfz.h"
#include "lbfz_common.hpp"
#include "lbfz_kernels.hpp"

namespace lbfz {

namespace {

// Tile of one block of the collide launch: 64 x TY x TZ nodes, one x row per
// wave, 256 threads.
// A tile that spans several z planes re-reads fewer ring planes per node
// (2 / TZ) from beyond the L2; at 256^3 FP32 storage runs fastest with
// 64 x 1 x 4 tiles (step 1.719 ms; 64 x 2 x 2: 1.741, 64 x 4 x 1: 1.774),
// 16-bit storage with 64 x 4 x 1 (1.254 ms; 64 x 2 x 2: 1.268, 64 x 1 x 4:
// 1.258), the closure launch on its own tiles in every case.
constexpr int TX = 64, NT = 256, HX = TX + 2;
template <int ST>
struct G3 {
  static constexpr int TY = ST == LBFZ_STORE_F32 ? 1 : 4;
  static constexpr int TZ = NT / (TX * TY);
  static constexpr int HY = TY + 2, HZ = TZ + 2;  // tile + 1-ring
  static constexpr int HP = HX * HY;              // ring slots per plane
  static constexpr int RS = HZ * HP;              // ring slots
  static constexpr int RIT = (RS + NT - 1) / NT;  // ring slots per thread
  static_assert(TX * TY * TZ == NT, "tile shape");
};
// Tiles of the closure launch.  It holds few registers, so it takes larger
// blocks (1024 / 512 threads), which re-read fewer velocity-ring slots per
// node (2.3 / 2.6 against 4.6 / 4.1 on 64 x 1 x 4 / 64 x 2 x 2 tiles): 256^3
// step 1.750 -> 1.717 ms (FP32), 1.295 -> 1.269 ms (16-bit, both launches on
// 64 x 2 x 2 before), results bit-identical (the closure is pointwise but
// for the ring).
template <int ST>
struct GC3 {
  static constexpr int TY = 4, TZ = ST == LBFZ_STORE_F32 ? 4 : 2;
  static constexpr int NT = TX * TY * TZ;
  static constexpr int HY = TY + 2, HZ = TZ + 2;
  static constexpr int HP = HX * HY;
  static constexpr int RS = HZ * HP;
  static constexpr int RIT = (RS + NT - 1) / NT;
};

constexpr int PF = 0, PG = 7, PH = 26, PL = 33;  // FP32 layout
// 16-bit layout: FP32 rest planes, then the first 16-bit plane of each set
constexpr int R_G0 = 0, R_H0 = 1;
constexpr int M_F = 0, M_G = 6, M_H = 24, M_L = 30, M_N = 36;
// closure-field planes
enum { CF_PHI = 0, CF_T = 1, CF_C = 2, CF_FS = 3, CF_D = 4, CF_N = 5 };

// D3Q19; the first seven are D3Q7
constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
constexpr float W19[19] = {1.f / 3,  1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18,
                           1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                           1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
constexpr float W7 = 1.f / 6;
// D3Q7 weights of the phase-field and solute equilibria and sources: 1/6
// rounded up on the x and y links and one ulp below that on the z links, so
// that the six sum to exactly one in FP32 (2 (2 fl(1/6) + lo) = 1; six
// fl(1/6) sum to 1 + 3e-8, and these sets have no rest population to take
// the difference, so their equilibria would make phase-field and solute
// mass at that rate every step).  The initial populations and the 16-bit
// offsets' references keep W7 (any consistent reference serves; the first
// collision relaxes the initial state onto these equilibria), and so does
// the enthalpy set (its rest equilibrium is the complement of the moving
// ones).
constexpr float W7A[7] = {0.0f, 1.f / 6, 1.f / 6, 1.f / 6, 1.f / 6, 0.1666666567325592f,
                          0.1666666567325592f};

// Wall-normal (z) plane -> stored plane.  ghost: 0 inside, -1 below the low
// wall, +1 above the high wall (a ghost takes its mirror plane).
__device__ __forceinline__ int map_z(const KParams& P, int k, int& ghost) {
  ghost = 0;
  if (!P.walls) return wrap_near(k, P.nz);
  if (k < 0) {
    ghost = -1;
    k = -1 - k;
  } else if (k >= P.nz) {
    ghost = 1;
    k = 2 * P.nz - 1 - k;
  }
  return min(max(k, 0), P.nz - 1);
}

__device__ __forceinline__ uint32_t node3(const KParams& P, int x, int y, int z) {
  return (((uint32_t)z * (uint32_t)P.ny + (uint32_t)y) * (uint32_t)P.nx + (uint32_t)x) * 4u;
}

// Ring slot s (0 <= s < RS) -> (plane 0..HZ-1, row 0..HY-1, column 0..HX-1).
template <int HP>
__device__ __forceinline__ void ring_pos(int s, int& pz, int& ly, int& lx) {
  pz = s / HP;
  const int r = s - pz * HP;
  ly = r / HX;
  lx = r - ly * HX;
}

struct Bufs3 {
  rsrc_t f, g, h, l, rest;       // source populations
  rsrc_t df, dg, dh, dl, drest;  // destination populations
  rsrc_t cfo, cfn;               // closure fields, previous / this level (CF_N planes)
  rsrc_t p_old, p_ref, u_old, mask;
  uint32_t pb, hb;
};

template <int ST>
__device__ __forceinline__ Bufs3 make_bufs3(const KParams& P, const StepArgs& A) {
  Bufs3 B;
  const long PS = P.ps;
  B.pb = (uint32_t)PS * 4u;
  B.hb = (uint32_t)PS * 2u;
  if constexpr (ST == LBFZ_STORE_F32) {
    B.f = rsrc(A.src + PF * PS, 7 * B.pb);
    B.g = rsrc(A.src + PG * PS, 19 * B.pb);
    B.h = rsrc(A.src + PH * PS, 7 * B.pb);
    B.l = rsrc(A.src + PL * PS, 7 * B.pb);
    B.df = rsrc(A.dst + PF * PS, 7 * B.pb);
    B.dg = rsrc(A.dst + PG * PS, 19 * B.pb);
    B.dh = rsrc(A.dst + PH * PS, 7 * B.pb);
    B.dl = rsrc(A.dst + PL * PS, 7 * B.pb);
  } else {
    const uint16_t* s16 = reinterpret_cast<const uint16_t*>(A.src + 2 * PS);
    const uint16_t* d16 = reinterpret_cast<const uint16_t*>(A.dst + 2 * PS);
    B.rest = rsrc(A.src, 2 * B.pb);
    B.drest = rsrc(A.dst, 2 * B.pb);
    B.f = rsrc(s16 + M_F * PS, 6 * B.hb);
    B.g = rsrc(s16 + M_G * PS, 18 * B.hb);
    B.h = rsrc(s16 + M_H * PS, 6 * B.hb);
    B.l = rsrc(s16 + M_L * PS, 6 * B.hb);
    B.df = rsrc(d16 + M_F * PS, 6 * B.hb);
    B.dg = rsrc(d16 + M_G * PS, 18 * B.hb);
    B.dh = rsrc(d16 + M_H * PS, 6 * B.hb);
    B.dl = rsrc(d16 + M_L * PS, 6 * B.hb);
    B.p_ref = rsrc(A.p_ref, B.pb);
  }
  B.cfo = rsrc(A.cf_old, CF_N * B.pb);
  B.cfn = rsrc(A.cf_new, CF_N * B.pb);
  B.p_old = rsrc(A.p_old, B.pb);
  B.u_old = rsrc(A.u_old, 3 * B.pb);
  B.mask = rsrc(A.mask, A.mask ? (uint32_t)P.N : 0u);
  return B;
}

// f (links 1..6), h (0..6), l (1..6) of the node at byte offset o; f[0] = l[0]
// = 0.  16-bit: decoded against the previous level's closure fields.
template <int ST>
__device__ __forceinline__ void load_fhl3(const KParams& P, const Bufs3& B, uint32_t o, float* f,
                                          float* h, float* l) {
  f[0] = 0.0f;
  l[0] = 0.0f;
  if constexpr (ST == LBFZ_STORE_F32) {
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      if (i) f[i] = ld(B.f, o, i * B.pb);
      h[i] = ld(B.h, o, i * B.pb);
      if (i) l[i] = ld(B.l, o, i * B.pb);
    }
  } else {
    const uint32_t o2 = o >> 1;
    const float rf = W7 * ld(B.cfo, o, CF_PHI * B.pb);
    const float rh = W7 * P.rhoc_ref * ld(B.cfo, o, CF_T * B.pb);
    const float rl = W7 * ld(B.cfo, o, CF_C * B.pb);
    h[0] = ld(B.rest, o, R_H0 * B.pb);
#pragma unroll
    for (int i = 1; i < 7; ++i) {
      f[i] = fmaf(dec16<ST>(ld16(B.f, o2, (i - 1) * B.hb)), 1.0f / SC_F, rf);
      h[i] = fmaf(dec16<ST>(ld16(B.h, o2, (i - 1) * B.hb)), 1.0f / SC_H, rh);
      l[i] = fmaf(dec16<ST>(ld16(B.l, o2, (i - 1) * B.hb)), 1.0f / SC_L, rl);
    }
  }
}

template <int ST>
__device__ __forceinline__ void load_g3(const Bufs3& B, uint32_t o, float* g) {
  if constexpr (ST == LBFZ_STORE_F32) {
#pragma unroll
    for (int i = 0; i < 19; ++i) g[i] = ld(B.g, o, i * B.pb);
  } else {
    const uint32_t o2 = o >> 1;
    const float p3 = 3.0f * ld(B.p_ref, o);
    g[0] = ld(B.rest, o, R_G0 * B.pb);
#pragma unroll
    for (int i = 1; i < 19; ++i)
      g[i] = fmaf(dec16<ST>(ld16(B.g, o2, (i - 1) * B.hb)), 1.0f / SC_G, W19[i] * p3);
  }
}

// Tile of a block: (x0, y0, z) in XCD-aware order (rev: each band walked
// backwards); one row per wave.
struct Tile3 {
  int tile, x0, y0, z0, tx, ty, tz, gx, gy, z;  // z: own plane, clamped into the grid
  bool valid;
};
template <int TY, int TZ>
__device__ __forceinline__ Tile3 tile3(const KParams& P, bool rev) {
  Tile3 t;
  t.tile = rev ? xcd_tile_rev(blockIdx.x, P.nblk) : xcd_tile(blockIdx.x, P.nblk);
  const int txy = P.nblk_x * P.nblk_y;
  const int bz = t.tile / txy;
  const int r = t.tile - bz * txy;
  t.x0 = (r % P.nblk_x) * TX;
  t.y0 = (r / P.nblk_x) * TY;
  t.z0 = bz * TZ;
  t.tx = threadIdx.x & (TX - 1);
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // wave = x row
  t.ty = w % TY;
  t.tz = w / TY;
  t.gx = t.x0 + t.tx;
  t.gy = t.y0 + t.ty;
  t.valid = t.gx < P.nx && t.gy < P.ny && t.z0 + t.tz < P.nz;
  t.z = min(t.z0 + t.tz, P.nz - 1);
  return t;
}

// ---------------------------------------------------------------------------
// Closure: phi, T, C, f_s and div u^{n-1} of every node (Sec. 3.1, 3.3, Eq. NS1).
template <int ST>
__global__ __launch_bounds__(GC3<ST>::NT) void k_close3d(KParams P, StepArgs A) {
  using G = GC3<ST>;
  constexpr int HP = G::HP, RS = G::RS, RIT = G::RIT, NT = G::NT;
  __shared__ float s_u[3][RS];  // previous velocity on the tile + 1-ring
  __shared__ uint8_t s_m[RS];   // obstacle mask on the ring (ghost planes: 0)
  const Tile3 t = tile3<G::TY, G::TZ>(P, false);
  const Bufs3 B = make_bufs3<ST>(P, A);
  const uint32_t PB = B.pb;
  const int omx = wrap_near(t.gx, P.nx), omy = wrap_near(t.gy, P.ny);
  const uint32_t on = node3(P, omx, omy, t.z);
  float f[7], h[7], l[7];
  load_fhl3<ST>(P, B, on, f, h, l);
  const bool ob = A.mask && ld8(B.mask, on >> 2);
  // velocity ring: every load is issued before the first is stored
  float v[RIT][3], sg[RIT];
  uint8_t mk[RIT];
#pragma unroll
  for (int j = 0; j < RIT; ++j) {
    const int s = min((int)threadIdx.x + j * NT, RS - 1);
    int pz, ly, lx, ghost;
    ring_pos<HP>(s, pz, ly, lx);
    const int kz = map_z(P, t.z0 - 1 + pz, ghost);
    const uint32_t o =
        node3(P, wrap_near(t.x0 + lx - 1, P.nx), wrap_near(t.y0 + ly - 1, P.ny), kz);
    sg[j] = ghost ? -1.0f : 1.0f;  // no-slip walls: negated mirror
#pragma unroll
    for (int a = 0; a < 3; ++a) v[j][a] = ld(B.u_old, o, a * PB);
    mk[j] = (A.mask && !ghost) ? ld8(B.mask, o >> 2) : (uint8_t)0;
  }
#pragma unroll
  for (int j = 0; j < RIT; ++j) {
    const int s = (int)threadIdx.x + j * NT;
    if (s < RS) {
#pragma unroll
      for (int a = 0; a < 3; ++a) s_u[a][s] = sg[j] * v[j][a];
      s_m[s] = mk[j];
    }
  }
  __syncthreads();
  if (!t.valid) return;
  float phi0 = 0.f, E0 = 0.f, C = 0.f;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    phi0 += f[i];
    E0 += h[i];
    C += l[i];
  }
  float phi, T, fs, D;
  if (ob) {
    enthalpy_map(P, E0, 0.0f, T, fs);
    phi = -1.0f;
    C = 0.0f;
    fs = 0.0f;
    D = 0.0f;
  } else {
    // div u^{n-1}: D3Q19 isotropic gradient; obstacle neighbours give -u(centre)
    const int c = (t.tz + 1) * HP + (t.ty + 1) * HX + (t.tx + 1);
    float acc = 0.0f;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      const int q = c + CZ[i] * HP + CY[i] * HX + CX[i];
      const bool nob = s_m[q] != 0;
      float w = 0.0f;
      if (CX[i]) w += CX[i] * (nob ? -s_u[0][c] : s_u[0][q]);
      if (CY[i]) w += CY[i] * (nob ? -s_u[1][c] : s_u[1][q]);
      if (CZ[i]) w += CZ[i] * (nob ? -s_u[2][c] : s_u[2][q]);
      acc += W19[i] * w;
    }
    D = acc * kInvCs2;
    const Closure cl = closure(P, phi0, E0, D);
    phi = cl.phi;
    T = cl.T;
    fs = cl.fs;
  }
  st_keep(B.cfn, on, CF_PHI * PB, phi);
  st_keep(B.cfn, on, CF_T * PB, T);
  st_keep(B.cfn, on, CF_C * PB, C);
  st_keep(B.cfn, on, CF_FS * PB, fs);
  st_keep(B.cfn, on, CF_D * PB, D);
}

// ---------------------------------------------------------------------------
// Collision and streaming (Sec. 3.1-3.4, walls Sec. 4.5).
template <bool DRY, int ST>
__global__ __launch_bounds__(NT) void k_collide3d(KParams P, StepArgs A) {
  using G = G3<ST>;
  constexpr int HP = G::HP, RS = G::RS, RIT = G::RIT;
  __shared__ float s_c[5][RS];  // phi, T, C, f_s, p^{n-1} on the tile + 1-ring
  __shared__ uint8_t s_m[RS];
  __shared__ double s_red[NT / 64];
  // the tiles in reverse: the collision starts where the closure launch
  // ended, and the next closure where this launch ends
  const Tile3 t = tile3<G::TY, G::TZ>(P, true);
  const Bufs3 B = make_bufs3<ST>(P, A);
  const uint32_t PB = B.pb, HB = B.hb, NB = (uint32_t)P.N * 4u;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int omx = wrap_near(t.gx, nx), omy = wrap_near(t.gy, ny);
  const uint32_t on = node3(P, omx, omy, t.z);
  // every global load of the block before the barrier
  float g[19], f[7], h[7], l[7];
  load_g3<ST>(B, on, g);
  load_fhl3<ST>(P, B, on, f, h, l);
  const float D = ld(B.cfn, on, CF_D * PB);
  const float fs_prev = ld(B.cfo, on, CF_FS * PB);
  const float phiP = ld(B.cfo, on, CF_PHI * PB), CP = ld(B.cfo, on, CF_C * PB);
  const float up0 = ld(B.u_old, on), up1 = ld(B.u_old, on, PB), up2 = ld(B.u_old, on, 2 * PB);
  float rv[RIT][5];
  uint8_t rmk[RIT];
  int rgh[RIT], rgx[RIT];
#pragma unroll
  for (int j = 0; j < RIT; ++j) {
    const int s = min((int)threadIdx.x + j * NT, RS - 1);
    int pz, ly, lx, ghost;
    ring_pos<HP>(s, pz, ly, lx);
    const int kz = map_z(P, t.z0 - 1 + pz, ghost);
    const int mx = wrap_near(t.x0 + lx - 1, nx);
    const uint32_t o = node3(P, mx, wrap_near(t.y0 + ly - 1, ny), kz);
#pragma unroll
    for (int q = 0; q < 4; ++q) rv[j][q] = ld(B.cfn, o, q * PB);
    rv[j][4] = ld(B.p_old, o);
    rmk[j] = (A.mask && !ghost) ? ld8(B.mask, o >> 2) : (uint8_t)0;
    rgh[j] = ghost;
    rgx[j] = mx;
  }
#pragma unroll
  for (int j = 0; j < RIT; ++j) {
    const int s = (int)threadIdx.x + j * NT;
    if (s < RS) {
      float T = rv[j][1];
      // a ghost plane beyond a wall mirrors the adjacent plane; T by the wall rule
      if (rgh[j] < 0 && P.tlo_dir)
        T = 2.0f * (P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)rgx[j])) - T;
      if (rgh[j] > 0 && P.thi_dir) T = 2.0f * P.T_hi - T;
      s_c[0][s] = rv[j][0];
      s_c[1][s] = T;
      s_c[2][s] = rv[j][2];
      s_c[3][s] = rv[j][3];
      s_c[4][s] = rv[j][4];
      s_m[s] = rmk[j];
    }
  }
  __syncthreads();

  const int c = (t.tz + 1) * HP + (t.ty + 1) * HX + (t.tx + 1);  // own ring slot
  const bool valid = t.valid;
  const bool ob = s_m[c] != 0;
  double mpc_acc = 0.0;
  double tot[6] = {0, 0, 0, 0, 0, 0};
  // obstacle neighbours as a bit set (bit i for link i)
  uint32_t obm = 0;
  if (A.mask) {
#pragma unroll
    for (int i = 1; i < 19; ++i)
      obm |= s_m[c + CZ[i] * HP + CY[i] * HX + CX[i]] ? (1u << i) : 0u;
  }
  // stencil neighbour value; kind 0 fields take the centre value at an obstacle
  auto nb = [&](int fld, int i, bool kind0) -> float {
    if (kind0 && (obm >> i & 1u)) return s_c[fld][c];
    return s_c[fld][c + CZ[i] * HP + CY[i] * HX + CX[i]];
  };
  // the same with the obstacle tests compiled in (obs true) or out (false)
  auto nbT = [&](auto obs, int fld, int i, bool kind0) -> float {
    if constexpr (decltype(obs)::value) {
      if (kind0 && (obm >> i & 1u)) return s_c[fld][c];
    }
    return s_c[fld][c + CZ[i] * HP + CY[i] * HX + CX[i]];
  };
  // field of the node link i streams to (16-bit encoding references)
  auto tref = [&](int fld, int i) -> float {
    return s_c[fld][c + CZ[i] * HP + CY[i] * HX + CX[i]];
  };
  const float phi = s_c[0][c], T = s_c[1][c], C = s_c[2][c], fs = s_c[3][c];
  float E0 = 0.f, phi0 = 0.f;
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    phi0 += f[i];
    E0 += h[i];
  }
  // Link targets: x, y periodic; z periodic or closed by the walls.  Plane
  // and row offsets are wave-uniform, column offsets per lane.
  const bool zlo = P.walls && t.z == 0, zhi = P.walls && t.z == nz - 1;
  const int zm = t.z == 0 ? nz - 1 : t.z - 1, zp = t.z == nz - 1 ? 0 : t.z + 1;
  const int ym = omy == 0 ? ny - 1 : omy - 1, yp = omy == ny - 1 ? 0 : omy + 1;
  const uint32_t plb[3] = {(uint32_t)zm * (uint32_t)ny, (uint32_t)t.z * (uint32_t)ny,
                           (uint32_t)zp * (uint32_t)ny};
  const uint32_t rwb[3] = {(uint32_t)ym, (uint32_t)omy, (uint32_t)yp};
  const uint32_t colb[3] = {(uint32_t)(omx == 0 ? nx - 1 : omx - 1) * 4u, (uint32_t)omx * 4u,
                            (uint32_t)(omx == nx - 1 ? 0 : omx + 1) * 4u};
  auto target = [&](int i) -> uint32_t {
    return (plb[CZ[i] + 1] + rwb[CY[i] + 1]) * (uint32_t)nx * 4u + colb[CX[i] + 1];
  };
  // 0 stream, 1 wall (bounce-back; anti-bounce-back for h at a Dirichlet
  // wall), 2 obstacle (bounce-back for f, g, l; h streams into it)
  auto kind = [&](int i) -> int {
    if ((CZ[i] < 0 && zlo) || (CZ[i] > 0 && zhi)) return 1;
    return (obm >> i & 1u) ? 2 : 0;
  };
  auto kindT = [&](auto obs, int i) -> int {
    if ((CZ[i] < 0 && zlo) || (CZ[i] > 0 && zhi)) return 1;
    if constexpr (decltype(obs)::value) return (obm >> i & 1u) ? 2 : 0;
    return 0;
  };
  // store value v of moving slot `slot` of a set at byte offset off; 16-bit:
  // against the reference refw = w_i r of the node it is stored at
  auto put = [&](rsrc_t set, uint32_t off, int slot, float v, float refw, float scale) {
    if constexpr (ST == LBFZ_STORE_F32)
      st_keep(set, off, slot * PB, v);
    else
      st16_keep(set, off >> 1, (slot - 1) * HB, enc16<ST>((v - refw) * scale));
  };
  auto put_rest = [&](rsrc_t set, int slot32, int slot16, float v) {
    if constexpr (ST == LBFZ_STORE_F32)
      st_keep(set, on, slot32 * PB, v);
    else
      st_keep(B.drest, on, slot16 * PB, v);
  };
  const float href_w = W7 * P.rhoc_ref;

  if (valid && ob) {
    // obstacle: enthalpy at rest without source (pure conduction)
    float heq[7];
    heq[0] = E0;
#pragma unroll
    for (int i = 1; i < 7; ++i) {
      heq[i] = W7 * P.rhoc_ref * T;
      heq[0] -= heq[i];
    }
    if (DRY) {
      float* const* o = A.out;
      if (o[0]) st_keep(rsrc(o[0], NB), on, 0, -1.0f);
      if (o[1]) st_keep(rsrc(o[1], NB), on, 0, 1.0f);
      if (o[2]) st_keep(rsrc(o[2], NB), on, 0, T);
      if (o[3]) st_keep(rsrc(o[3], NB), on, 0, 0.0f);
      if (o[4]) st_keep(rsrc(o[4], NB), on, 0, 0.0f);
      if (o[5]) st_keep(rsrc(o[5], NB), on, 0, 0.0f);
      if (o[6]) st_keep(rsrc(o[6], NB), on, 0, 0.0f);
      if (o[7]) st_keep(rsrc(o[7], NB), on, 0, 0.0f);
      if (o[8]) st_keep(rsrc(o[8], NB), on, 0, P.rho_g);
      double dh = 0.0;
      float sh = 0.f;
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        dh += (double)h[i];
        sh += h[i];
      }
      tot[2] += dh;
      if (!isfinite(sh)) tot[5] += 1.0;
    } else {
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        const int o = OPP[i];
        const float hs = 0.5f * (h[i] + h[o]), ha = 0.5f * (h[i] - h[o]);
        const float es = 0.5f * (heq[i] + heq[o]), ea = 0.5f * (heq[i] - heq[o]);
        const float hp = h[i] - (hs - es) * P.itau_s - (ha - ea) * P.itau_a;
        if (i == 0) {
          put_rest(B.dh, 0, R_H0, hp);
        } else if (kind(i) == 1) {
          float hv = hp;
          if (CZ[i] < 0 && P.tlo_dir)
            hv = -hv + 2.0f * W7 * P.rhoc_ref *
                           (P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)t.gx));
          if (CZ[i] > 0 && P.thi_dir) hv = -hv + 2.0f * W7 * P.rhoc_ref * P.T_hi;
          put(B.dh, on, o, hv, href_w * T, SC_H);
        } else {
          put(B.dh, target(i), i, hp, href_w * tref(1, i), SC_H);
        }
      }
      st_keep(rsrc(A.p_new, PB), on, 0, 0.0f);
      const rsrc_t r_un = rsrc(A.u_new, 3 * PB);
      st_keep(r_un, on, 0, 0.0f);
      st_keep(r_un, on, PB, 0.0f);
      st_keep(r_un, on, 2 * PB, 0.0f);
    }
  } else if (valid) {
    // the collision of a fluid node.  16-bit storage (bound by instruction
    // issue): a wave none of whose nodes has an obstacle neighbour (nearly
    // all of them) runs it without the per-link obstacle tests (1.383 ->
    // 1.302 ms per 256^3 step); FP32 storage (bound by memory) keeps one
    // copy of the code
    auto body = [&](auto obs) {
      // stencils (isotropic D3Q19 gradient / Laplacian), one field per pass
      float gp[3], gT[3], gC[3], gf[3], gP[3], lap = 0.f;
      auto grad = [&](int fld, bool kind0, float* gr) {
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int i = 1; i < 19; ++i) {
          const float v = nbT(obs, fld, i, kind0) * (W19[i] * kInvCs2);
          if (CX[i]) a0 += CX[i] * v;
          if (CY[i]) a1 += CY[i] * v;
          if (CZ[i]) a2 += CZ[i] * v;
        }
        gr[0] = a0;
        gr[1] = a1;
        gr[2] = a2;
      };
      grad(0, true, gp);
#pragma unroll
      for (int i = 1; i < 19; ++i) lap += 2.0f * W19[i] * kInvCs2 * (nbT(obs, 0, i, true) - phi);
      grad(1, false, gT);
      grad(2, true, gC);
      grad(3, true, gf);
      grad(4, true, gP);
      // forces, velocity, pressure (Sec. 3.2, Eq. Fs)
      float grho[3], F[3], nv[3], gsig[3];
      const float g2 = gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2];
      // 1 / max(|grad phi|, 1e-6): n regularised in the bulk
      const float inv_ng = __builtin_amdgcn_rsqf(fmaxf(g2, 1e-12f));
      const float mu = phi * (phi * phi - 1.0f) * P.ieps2 - lap;
      const float sig = P.sigma0 + P.sigma_T * (T - P.T_ref) + P.sigma_c * (C - P.c_ref);
      const float wst = P.st_mode == 0 ? (1.0f - fs) : 1.0f;
      const float bf[3] = {P.bfx, P.bfy, P.bfz};
      float gsdp = 0.f;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        grho[a] = 0.5f * (P.rho_l - P.rho_g) * gp[a] + (P.rho_s - P.rho_l) * gf[a];
        nv[a] = gp[a] * inv_ng;
        gsig[a] = P.sigma_T * gT[a] + P.sigma_c * gC[a];
        gsdp += gsig[a] * gp[a];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
        F[a] = wst * P.alpha * (sig * mu * gp[a] + g2 * gsig[a] - gsdp * gp[a]) + bf[a];
      const float rho = interp(phi, fs, P.rho_l, P.rho_g, P.rho_s);
      const float rcp = rho * interp(phi, fs, P.cp_l, P.cp_g, P.cp_s);
      float mom[3] = {0, 0, 0};
#pragma unroll
      for (int i = 1; i < 19; ++i) {
        mom[0] += CX[i] * g[i];
        mom[1] += CY[i] * g[i];
        mom[2] += CZ[i] * g[i];
      }
      const float irho = frcp(rho);
      float u[3], fd[3], Ft[3], Ff[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float us_ = (mom[a] + 0.5f * F[a]) * irho;
        fd[a] = -fs * us_;
        u[a] = us_ + 0.5f * fd[a];
      }
      const float mdot = P.ratio * (fs - fs_prev);
      const float S_ = rho * mdot + u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        Ft[a] = F[a] - gP[a] + kCs2 * grho[a];
        Ff[a] = F[a] + rho * fd[a];
      }
      const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      const float uFt = u[0] * Ft[0] + u[1] * Ft[1] + u[2] * Ft[2];
      // G_i (Sec. 3.2), computed where it is used, to keep no array of them
      // live.  The rest component G_0 = w_0 (S - u.Ft / cs^2): with sum_i w_i c_i
      // = 0 and sum_i w_i c_i c_i = cs^2 I it is what the moving ones leave of
      // S (sum G = S), without evaluating them twice (the 16-bit collision
      // is bound by instruction issue)
      auto Gi = [&](int i) -> float {
        const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        const float cFt = CX[i] * Ft[0] + CY[i] * Ft[1] + CZ[i] * Ft[2];
        const float cFf = CX[i] * Ff[0] + CY[i] * Ff[1] + CZ[i] * Ff[2];
        return W19[i] * (S_ + kInvCs2 * cFf + 9.0f * (cu * cFt) - 3.0f * uFt);
      };
      const float G0 = W19[0] * (S_ - 3.0f * uFt);
      float sum_nz = 0.f;
#pragma unroll
      for (int i = 1; i < 19; ++i) sum_nz += g[i];
      const float srest = W19[0] * (-1.5f * uu);
      const float pn =
          (kCs2 / (1.0f - W19[0])) * (sum_nz + 0.5f * S_ + P.tau_gp * G0 + rho * srest);
      if (DRY) {
        float* const* o = A.out;
        if (o[0]) st_keep(rsrc(o[0], NB), on, 0, phi);
        if (o[1]) st_keep(rsrc(o[1], NB), on, 0, 1.0f - fs);
        if (o[2]) st_keep(rsrc(o[2], NB), on, 0, T);
        if (o[3]) st_keep(rsrc(o[3], NB), on, 0, C);
        if (o[4]) st_keep(rsrc(o[4], NB), on, 0, u[0]);
        if (o[5]) st_keep(rsrc(o[5], NB), on, 0, u[1]);
        if (o[6]) st_keep(rsrc(o[6], NB), on, 0, u[2]);
        if (o[7]) st_keep(rsrc(o[7], NB), on, 0, pn);
        if (o[8]) st_keep(rsrc(o[8], NB), on, 0, rho);
        double df = 0, dh = 0, dl = 0;
        bool bad = !isfinite(phi) || !isfinite(T) || !isfinite(pn) || !isfinite(uu);
#pragma unroll
        for (int i = 0; i < 7; ++i) {
          df += (double)f[i];
          dh += (double)h[i];
          dl += (double)l[i];
        }
        bad = bad || !isfinite(df) || !isfinite(dh) || !isfinite(dl);
        tot[0] += df;
        tot[1] += dl;
        tot[2] += dh;
        tot[3] += (double)fs;
        tot[4] += (double)clamp01(0.5f * (1.0f + phi));
        tot[5] += bad ? 1.0 : 0.0;
      } else {
        // E and Q of the own node: the closure again, from the same inputs
        const Closure cl = closure(P, phi0, E0, D);
        mpc_acc += (double)phi * (double)D;
        // flow BGK (Sec. 3.2)
        float geq_sum = 0.f;
#pragma unroll
        for (int i = 1; i < 19; ++i) {
          const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
          const float geq =
              pn * kInvCs2 * W19[i] + rho * W19[i] * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
          geq_sum += geq;
          const float post = g[i] - (g[i] - geq) * P.itau_g + P.wg * Gi(i);
          if (kindT(obs, i))
            put(B.dg, on, OPP[i], post, W19[i] * (3.0f * s_c[4][c]), SC_G);
          else
            put(B.dg, target(i), i, post, W19[i] * (3.0f * tref(4, i)), SC_G);
        }
        put_rest(B.dg, 0, R_G0, g[0] - (g[0] + geq_sum) * P.itau_g + P.wg * G0);
        // phase field BGK (Sec. 3.1); the D3Q7 rest component is zero
        {
          const float cf = kCs2 * (1.0f - phi * phi) * P.isq;
          const float B0 = (phi * u[0] - phiP * up0) + cf * nv[0];
          const float B1 = (phi * u[1] - phiP * up1) + cf * nv[1];
          const float B2 = (phi * u[2] - phiP * up2) + cf * nv[2];
#pragma unroll
          for (int i = 1; i < 7; ++i) {
            const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
            const float cB = CX[i] * B0 + CY[i] * B1 + CZ[i] * B2;
            const float Fi = W7A[i] * (kInvCs2 * cB + phi * D);
            const float feq = W7A[i] * phi * (1.0f + kInvCs2 * cu);
            const float post = f[i] - (f[i] - feq) * P.itau_f + P.wf * Fi;
            if (kindT(obs, i))
              put(B.df, on, OPP[i], post, W7 * phi, SC_F);
            else
              put(B.df, target(i), i, post, W7 * tref(0, i), SC_F);
          }
        }
        // enthalpy TRT (Sec. 3.3)
        {
          float heq[7];
          const float rT = P.rhoc_ref * T, cT = rcp * T;
          heq[0] = cl.E;
#pragma unroll
          for (int i = 1; i < 7; ++i) {
            const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
            heq[i] = W7 * (rT + cT * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
            heq[0] -= heq[i];
          }
          const float hq = W7 * cl.Q, hq0 = cl.Q - 6.0f * hq;
#pragma unroll
          for (int i = 0; i < 7; ++i) {
            const int o = OPP[i];
            const float hs = 0.5f * (h[i] + h[o]), ha = 0.5f * (h[i] - h[o]);
            const float es = 0.5f * (heq[i] + heq[o]), ea = 0.5f * (heq[i] - heq[o]);
            const float post = h[i] - (hs - es) * P.itau_s - (ha - ea) * P.itau_a +
                               P.ws * (i == 0 ? hq0 : hq);
            if (i == 0) {
              put_rest(B.dh, 0, R_H0, post);
            } else if (kindT(obs, i) == 1) {
              float hv = post;
              if (CZ[i] < 0 && P.tlo_dir)
                hv = -hv + 2.0f * W7 * P.rhoc_ref *
                               (P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)t.gx));
              if (CZ[i] > 0 && P.thi_dir) hv = -hv + 2.0f * W7 * P.rhoc_ref * P.T_hi;
              put(B.dh, on, o, hv, href_w * T, SC_H);
            } else {
              put(B.dh, target(i), i, post, href_w * tref(1, i), SC_H);
            }
          }
        }
        // solute BGK (Sec. 3.4)
        {
          const float keff = 1.0f - fs * (1.0f - P.k_p);
          const float De = fs * P.k_p * P.Ds + (1.0f - fs) * P.Dl;
          const float ikeff = frcp(keff);
          const float itau_l = frcp(3.0f * De * ikeff + 0.5f), wl = 1.0f - 0.5f * itau_l;
          const float cr = (1.0f - phi) * C * P.isq, ck = (P.k_p - 1.0f) * C * ikeff;
          const float L0 = (C * u[0] - CP * up0) + kCs2 * (cr * nv[0] + ck * gf[0]);
          const float L1 = (C * u[1] - CP * up1) + kCs2 * (cr * nv[1] + ck * gf[1]);
          const float L2 = (C * u[2] - CP * up2) + kCs2 * (cr * nv[2] + ck * gf[2]);
#pragma unroll
          for (int i = 1; i < 7; ++i) {
            const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
            const float cL = CX[i] * L0 + CY[i] * L1 + CZ[i] * L2;
            const float leq = W7A[i] * C * (1.0f + kInvCs2 * cu);
            const float post = l[i] - (l[i] - leq) * itau_l + wl * W7A[i] * kInvCs2 * cL;
            if (kindT(obs, i))
              put(B.dl, on, OPP[i], post, W7 * C, SC_L);
            else
              put(B.dl, target(i), i, post, W7 * tref(2, i), SC_L);
          }
        }
        st_keep(rsrc(A.p_new, PB), on, 0, pn);
        const rsrc_t r_un = rsrc(A.u_new, 3 * PB);
        st_keep(r_un, on, 0, u[0]);
        st_keep(r_un, on, PB, u[1]);
        st_keep(r_un, on, 2 * PB, u[2]);
      }
    };
    if (ST == LBFZ_STORE_F32 || __builtin_amdgcn_ballot_w64(obm != 0u) != 0)
      body(std::true_type{});
    else
      body(std::false_type{});
  }
  // per-tile FP64 reductions
  if (DRY) {
    if (A.tot_part) {
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const double s = block_sum<NT>(tot[q], s_red);
        if (threadIdx.x == 0) A.tot_part[(long)t.tile * 8 + q] = s;
      }
    }
  } else {
    const double s = block_sum<NT>(mpc_acc, s_red);
    if (threadIdx.x == 0) A.mpc_part[t.tile] += s;
  }
}

// Equilibrium populations of the initial fields (u = 0, p = 0), the
// previous-level closure fields (phi, T, C; f_s = 0, div u = 0) and zero
// pressure and velocity.  The second population buffer is cleared: obstacle
// slots and the zero rest slots of f and l are never written by a step.
template <int ST>
__global__ __launch_bounds__(256) void k_init3d(KParams P, const double* __restrict__ phi_in,
                                                const double* __restrict__ T_in,
                                                const double* __restrict__ C_in,
                                                const uint8_t* __restrict__ mask,
                                                float* __restrict__ popA,
                                                float* __restrict__ popB, StateArgs S) {
  // no contraction into fused multiply-adds in this kernel: its FP32 and
  // 16-bit instantiations must round alike (their initial states are equal
  // bit for bit)
#pragma clang fp contract(off)
  const long N = P.N, PS = P.ps;
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < N;
       n += (long)gridDim.x * blockDim.x) {
    const bool ob = mask && mask[n];
    const float phi = ob ? -1.0f : (float)phi_in[n];
    const float T = (float)T_in[n], C = ob ? 0.0f : (float)C_in[n];
    const float psi = clamp01(0.5f * (1.0f + phi));
    const float rcl = psi * P.rc_l + (1.0f - psi) * P.rc_g;
    const float E = rcl * T + psi * P.rho_l_latent;
    const float hw = W7 * P.rhoc_ref * T;
    float h0 = E;
#pragma unroll
    for (int i = 1; i < 7; ++i) h0 -= hw;
    if constexpr (ST == LBFZ_STORE_F32) {
#pragma unroll
      for (int i = 1; i < 7; ++i) {
        popA[(PH + i) * PS + n] = hw;
        popA[(PF + i) * PS + n] = ob ? 0.0f : W7 * phi;
        popA[(PL + i) * PS + n] = ob ? 0.0f : W7 * C;
      }
      popA[(PH + 0) * PS + n] = h0;
      popA[(PF + 0) * PS + n] = 0.0f;
      popA[(PL + 0) * PS + n] = 0.0f;
#pragma unroll
      for (int i = 0; i < 19; ++i) popA[(PG + i) * PS + n] = 0.0f;
#pragma unroll
      for (int q = 0; q < 40; ++q) popB[q * PS + n] = 0.0f;
    } else {
      // every moving population at its reference (offset 0); obstacle f and l
      // slots are never read for the step
      popA[R_G0 * PS + n] = 0.0f;
      popA[R_H0 * PS + n] = h0;
      popB[R_G0 * PS + n] = 0.0f;
      popB[R_H0 * PS + n] = 0.0f;
      uint16_t* a16 = reinterpret_cast<uint16_t*>(popA + 2 * PS);
      uint16_t* b16 = reinterpret_cast<uint16_t*>(popB + 2 * PS);
#pragma unroll
      for (int j = 0; j < M_N; ++j) {
        a16[j * PS + n] = enc16<ST>(0.0f);
        b16[j * PS + n] = enc16<ST>(0.0f);
      }
      S.pC[n] = 0.f;
    }
    S.pA[n] = S.pB[n] = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) S.uA[a * PS + n] = S.uB[a * PS + n] = 0.f;
    // previous-level closure fields
    S.phiA[n] = phi;
    S.TA[n] = T;
    S.CA[n] = C;
    S.fs[n] = 0.f;
    S.DA[n] = 0.f;
  }
}

// 16-bit forms: populations of the current level decoded into FP32 planes in
// the 40-plane state order, dst[q * N + n].  (g at an obstacle decodes to its
// stored zero: its reference, p, is zero there.)
template <int ST>
__global__ __launch_bounds__(256) void k_export3d(KParams P, StepArgs A, float* __restrict__ dst) {
  const long N = P.N;
  const Bufs3 B = make_bufs3<ST>(P, A);
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < N;
       n += (long)gridDim.x * blockDim.x) {
    const uint32_t o = (uint32_t)n * 4u;
    float f[7], h[7], l[7], g[19];
    load_fhl3<ST>(P, B, o, f, h, l);
    load_g3<ST>(B, o, g);
    // obstacle f, l slots are never written by a step; they read as zero, as
    // with FP32 storage
    const bool ob = A.mask && A.mask[n];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      if (ob) f[i] = l[i] = 0.0f;
      dst[(PF + i) * N + n] = f[i];
      dst[(PH + i) * N + n] = h[i];
      dst[(PL + i) * N + n] = l[i];
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) dst[(PG + i) * N + n] = g[i];
  }
}

// 16-bit forms: encode FP32 populations src[q * N + n] (state order) into
// A.dst against phi, C of A.cf_old (imported), p of A.p_ref and T from the
// enthalpy map of the imported populations, stored into A.cf_old's T plane.
template <int ST>
__global__ __launch_bounds__(256) void k_import3d(KParams P, StepArgs A,
                                                  const float* __restrict__ src) {
  const long N = P.N, PS = P.ps;
  float* cfo = const_cast<float*>(A.cf_old);
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < N;
       n += (long)gridDim.x * blockDim.x) {
    float phi0 = 0.f, E = 0.f;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      phi0 += src[(PF + i) * N + n];
      E += src[(PH + i) * N + n];
    }
    float T, fs;
    enthalpy_map(P, E, clamp01(0.5f * (1.0f + phi0)), T, fs);
    cfo[CF_T * PS + n] = T;
    const float rf = W7 * cfo[CF_PHI * PS + n], rl = W7 * cfo[CF_C * PS + n];
    const float rh = W7 * P.rhoc_ref * T, p3 = 3.0f * A.p_ref[n];
    A.dst[R_G0 * PS + n] = src[PG * N + n];
    A.dst[R_H0 * PS + n] = src[PH * N + n];
    uint16_t* m16 = reinterpret_cast<uint16_t*>(A.dst + 2 * PS);
#pragma unroll
    for (int i = 1; i < 7; ++i) {
      m16[(M_F + i - 1) * PS + n] = enc16<ST>((src[(PF + i) * N + n] - rf) * SC_F);
      m16[(M_H + i - 1) * PS + n] = enc16<ST>((src[(PH + i) * N + n] - rh) * SC_H);
      m16[(M_L + i - 1) * PS + n] = enc16<ST>((src[(PL + i) * N + n] - rl) * SC_L);
    }
#pragma unroll
    for (int i = 1; i < 19; ++i)
      m16[(M_G + i - 1) * PS + n] = enc16<ST>((src[(PG + i) * N + n] - W19[i] * p3) * SC_G);
  }
}

int grid3(long N) { return (int)std::min<long>((N + 255) / 256, 65536); }

template <int ST>
void launch_step3d_st(const KParams& P, const StepArgs& A, bool dry, hipStream_t st) {
  {
    // the closure launch's own tiles: the same x columns, its own y and z blocks
    using G = GC3<ST>;
    KParams Pc = P;
    Pc.nblk_y = (P.ny + G::TY - 1) / G::TY;
    Pc.nblk_z = (P.nz + G::TZ - 1) / G::TZ;
    Pc.nblk = Pc.nblk_x * Pc.nblk_y * Pc.nblk_z;
    hipLaunchKernelGGL((k_close3d<ST>), dim3(Pc.nblk), dim3(G::NT), 0, st, Pc, A);
  }
  if (dry)
    hipLaunchKernelGGL((k_collide3d<true, ST>), dim3(P.nblk), dim3(NT), 0, st, P, A);
  else
    hipLaunchKernelGGL((k_collide3d<false, ST>), dim3(P.nblk), dim3(NT), 0, st, P, A);
}

}  // namespace

int tiles3d(int nx, int ny, int nz, int storage, int* nbx, int* nby, int* nbz) {
  const int ty = storage == LBFZ_STORE_F32 ? G3<LBFZ_STORE_F32>::TY : G3<LBFZ_STORE_F16>::TY;
  const int tz = storage == LBFZ_STORE_F32 ? G3<LBFZ_STORE_F32>::TZ : G3<LBFZ_STORE_F16>::TZ;
  *nbx = (nx + TX - 1) / TX;
  *nby = (ny + ty - 1) / ty;
  *nbz = (nz + tz - 1) / tz;
  return (*nbx) * (*nby) * (*nbz);
}

size_t pop_bytes3d(int storage, size_t ps) {
  return storage == LBFZ_STORE_F32 ? 40 * ps * sizeof(float)
                                   : 2 * ps * sizeof(float) + M_N * ps * sizeof(uint16_t);
}

hipError_t launch_init3d(const KParams& P, int storage, const double* phi, const double* T,
                         const double* C, const uint8_t* mask, float* popA, float* popB,
                         const StateArgs& S, hipStream_t st) {
  const int blocks = grid3(P.N);
  switch (storage) {
    case LBFZ_STORE_F32:
      hipLaunchKernelGGL(k_init3d<LBFZ_STORE_F32>, dim3(blocks), dim3(256), 0, st, P, phi, T, C,
                         mask, popA, popB, S);
      break;
    case LBFZ_STORE_F16:
      hipLaunchKernelGGL(k_init3d<LBFZ_STORE_F16>, dim3(blocks), dim3(256), 0, st, P, phi, T, C,
                         mask, popA, popB, S);
      break;
    default:
      hipLaunchKernelGGL(k_init3d<LBFZ_STORE_BF16>, dim3(blocks), dim3(256), 0, st, P, phi, T,
                         C, mask, popA, popB, S);
  }
  return hipGetLastError();
}

hipError_t launch_step3d(const KParams& P, int storage, const StepArgs& A, bool dry,
                         hipStream_t st) {
  switch (storage) {
    case LBFZ_STORE_F32: launch_step3d_st<LBFZ_STORE_F32>(P, A, dry, st); break;
    case LBFZ_STORE_F16: launch_step3d_st<LBFZ_STORE_F16>(P, A, dry, st); break;
    default: launch_step3d_st<LBFZ_STORE_BF16>(P, A, dry, st);
  }
  return hipGetLastError();
}

hipError_t launch_export3d(const KParams& P, int storage, const StepArgs& A, float* dst,
                           hipStream_t st) {
  const int blocks = grid3(P.N);
  if (storage == LBFZ_STORE_F16)
    hipLaunchKernelGGL(k_export3d<LBFZ_STORE_F16>, dim3(blocks), dim3(256), 0, st, P, A, dst);
  else
    hipLaunchKernelGGL(k_export3d<LBFZ_STORE_BF16>, dim3(blocks), dim3(256), 0, st, P, A, dst);
  return hipGetLastError();
}

hipError_t launch_import3d(const KParams& P, int storage, const StepArgs& A, const float* src,
                           hipStream_t st) {
  const int blocks = grid3(P.N);
  if (storage == LBFZ_STORE_F16)
    hipLaunchKernelGGL(k_import3d<LBFZ_STORE_F16>, dim3(blocks), dim3(256), 0, st, P, A, src);
  else
    hipLaunchKernelGGL(k_import3d<LBFZ_STORE_BF16>, dim3(blocks), dim3(256), 0, st, P, A, src);
  return hipGetLastError();
}

}  // namespace lbfz
