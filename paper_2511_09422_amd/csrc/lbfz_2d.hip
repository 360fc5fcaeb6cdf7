// lbfz_2d.hip -- fused 2D step of the coupled LB freezing scheme
// (arXiv 2511.09422, Sec. 3) for gfx950: D2Q9 flow g, D2Q5 phase field f,
// enthalpy h (TRT) and solute l.
//
// One kernel launch = one time step.  A step reads population buffer A at
// each node's own location and pushes post-collision values along their
// links into buffer B (half-way bounce-back / anti-bounce-back at walls).
// Each 64 x TY tile (one row per wave) stages in LDS
//   - the previous velocity on the tile + 2 ring   (div u for the closure),
//   - phi, T, C, f_s of the tile + 1 ring, computed from that ring's own
//     populations (the pointwise closure, evaluated redundantly on the ring
//     by the first ceil(ring / 64) waves only),
//   - the previous pressure on the tile + 1 ring,
// and then every thread owns one node: stencils, forces, velocity, pressure,
// four collisions and the streaming writes.  Reads and writes each touch every
// population once.
//
// Population storage (template parameter ST):
//   F32   24 FP32 planes, plane q at q * ps floats: f 0..4, g 5..13, h 14..18,
//         l 19..23.  240 B per node update.
//   F16 / BF16  the four rest populations stay FP32 (planes 0..3: f0, g0, h0,
//         l0; they carry most of each conserved sum), the 20 moving ones are
//         16-bit planes after them (f1..4, g1..8, h1..4, l1..4).  A moving
//         population is stored as (v - w_i r) * S of the node it sits at,
//         with r the node's reference moment from the step that wrote it --
//         phi for f, 3 p (= p / cs^2) for g, (rho c)_ref T for h, C for l --
//         and a power-of-two scale S per set that keeps the offsets in the
//         FP16 normal range.  The writer takes the target's references from
//         the LDS ring (phi, T, C of this step, p of the previous one); the
//         reader decodes with the same values from the time-level fields,
//         which are double-buffered (p: triple) so that a ring read never
//         races the owner's update.  172 B per node update.
//
// The step is bound by vector-ALU issue as much as by HBM, so addressing is
// kept off the vector units: buffer descriptors and the tile row are
// wave-uniform (scalar registers), a lane carries only a 32-bit byte offset,
// and every load or store is one instruction.
#include "../../include/lbfz.h"
#include "lbfz_common.hpp"
#include "lbfz_kernels.hpp"

namespace lbfz {

namespace {

// Tile geometry: 64 x TY nodes, one row per wave; TY is a template parameter
// of the step (4 for the single-grid solver; the batched sweep chooses).
constexpr int TX = 64;
constexpr int HX = TX + 2;  // closure ring width
constexpr int UX = TX + 4;  // velocity ring width
template <int TY>
struct Geo {
  static constexpr int NT = TX * TY;
  static constexpr int HY = TY + 2, UY = TY + 4;
  static constexpr int RING = 2 * HX + 2 * TY;
  static_assert(RING <= NT, "every ring slot needs a thread");
};
constexpr int TY_DEFAULT = 4;

constexpr int PF = 0, PG = 5, PH = 14, PL = 19;  // FP32 layout: first plane of each set
enum { SF = 0, SG = 1, SH = 2, SL = 3 };         // set index (16-bit layout: rest plane)

// D2Q9 (first five = D2Q5)
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr float W9[9] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                         1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
constexpr float W5[5] = {1.f / 3, 1.f / 6, 1.f / 6, 1.f / 6, 1.f / 6};

// Descriptors of one step.  F32: population sets incl. rest (plane i of a set
// at byte offset i * pb).  16-bit: rest = the four FP32 rest planes, f/g/h/l =
// the moving 16-bit planes of each set (plane i - 1 at (i - 1) * hb).
struct Bufs {
  rsrc_t f, g, h, l, rest;       // source
  rsrc_t df, dg, dh, dl, drest;  // destination
  rsrc_t p_old, u_old;           // u_old: x plane, then y plane
  rsrc_t phiO, CO, TO, pR;       // 16-bit: decode references of the source
  uint32_t pb, hb;               // FP32 / 16-bit plane bytes
};

template <int ST>
__device__ __forceinline__ Bufs make_bufs(const KParams& P, const StepArgs& A) {
  Bufs B;
  const long PS = P.ps;
  B.pb = (uint32_t)PS * 4u;
  B.hb = (uint32_t)PS * 2u;
  // population sets: descriptors from kSetPad bytes before the first plane
  auto set = [](const void* first, uint32_t bytes) {
    return rsrc(static_cast<const char*>(first) - kSetPad, bytes + kSetPad);
  };
  if constexpr (ST == LBFZ_STORE_F32) {
    B.f = set(A.src + PF * PS, 5 * B.pb);
    B.g = set(A.src + PG * PS, 9 * B.pb);
    B.h = set(A.src + PH * PS, 5 * B.pb);
    B.l = set(A.src + PL * PS, 5 * B.pb);
    B.df = set(A.dst + PF * PS, 5 * B.pb);
    B.dg = set(A.dst + PG * PS, 9 * B.pb);
    B.dh = set(A.dst + PH * PS, 5 * B.pb);
    B.dl = set(A.dst + PL * PS, 5 * B.pb);
  } else {
    const uint16_t* s16 = reinterpret_cast<const uint16_t*>(A.src + 4 * PS);
    const uint16_t* d16 = reinterpret_cast<const uint16_t*>(A.dst + 4 * PS);
    B.rest = rsrc(A.src, 4 * B.pb);
    B.f = set(s16, 4 * B.hb);
    B.g = set(s16 + 4 * PS, 8 * B.hb);
    B.h = set(s16 + 12 * PS, 4 * B.hb);
    B.l = set(s16 + 16 * PS, 4 * B.hb);
    B.drest = rsrc(A.dst, 4 * B.pb);
    B.df = set(d16, 4 * B.hb);
    B.dg = set(d16 + 4 * PS, 8 * B.hb);
    B.dh = set(d16 + 12 * PS, 4 * B.hb);
    B.dl = set(d16 + 16 * PS, 4 * B.hb);
    B.phiO = rsrc(A.phiP_old, B.pb);
    B.CO = rsrc(A.CP_old, B.pb);
    B.TO = rsrc(A.T_old, B.pb);
    B.pR = rsrc(A.p_ref, B.pb);
  }
  B.p_old = rsrc(A.p_old, B.pb);
  B.u_old = rsrc(A.u_old, 2 * B.pb);
  return B;
}

// Plane byte offsets within a population set's descriptor for direction i:
// FP32 sets hold directions 0.., 16-bit sets 1.. (the rest populations are
// FP32 planes of their own); both shifted by -c_x (kXS).
__device__ __forceinline__ uint32_t off32(const Bufs& B, int i) {
  return kSetPad + (uint32_t)i * B.pb - kXS * CX[i] * 4;
}
__device__ __forceinline__ uint32_t off16(const Bufs& B, int i) {
  return kSetPad + (uint32_t)(i - 1) * B.hb - kXS * CX[i] * 2;
}

// Wall-normal (y) coordinate -> stored row.  side: 0 inside, -1 ghost below
// the low wall, +1 ghost above the high wall; a ghost takes its mirror row.
__device__ __forceinline__ int map_y(int g, int n, int walls, int& side) {
  side = 0;
  if (!walls) return wrap_near(g, n);
  if (g < 0) {
    side = -1;
    g = -1 - g;
  } else if (g >= n) {
    side = 1;
    g = 2 * n - 1 - g;
  }
  return min(max(g, 0), n - 1);
}

__device__ __forceinline__ uint32_t node_off(int mx, int my, int nx) {
  return ((uint32_t)my * (uint32_t)nx + (uint32_t)mx) * 4u;
}

// f, h, l populations of the node at byte offset o (FP32 units).
template <int ST>
__device__ __forceinline__ void load_fhl(const KParams& P, const Bufs& B, uint32_t o, float* f,
                                         float* h, float* l) {
  if constexpr (ST == LBFZ_STORE_F32) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      f[i] = ld(B.f, o, off32(B, i));
      h[i] = ld(B.h, o, off32(B, i));
      l[i] = ld(B.l, o, off32(B, i));
    }
  } else {
    const uint32_t o2 = o >> 1;
    const float rf = W5[1] * ld(B.phiO, o), rh = W5[1] * P.rhoc_ref * ld(B.TO, o),
                rl = W5[1] * ld(B.CO, o);
    f[0] = ld(B.rest, o, SF * B.pb);
    h[0] = ld(B.rest, o, SH * B.pb);
    l[0] = ld(B.rest, o, SL * B.pb);
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      f[i] = fmaf(dec16<ST>(ld16(B.f, o2, off16(B, i))), 1.0f / SC_F, rf);
      h[i] = fmaf(dec16<ST>(ld16(B.h, o2, off16(B, i))), 1.0f / SC_H, rh);
      l[i] = fmaf(dec16<ST>(ld16(B.l, o2, off16(B, i))), 1.0f / SC_L, rl);
    }
  }
}

template <int ST>
__device__ __forceinline__ void load_g(const Bufs& B, uint32_t o, float* g) {
  if constexpr (ST == LBFZ_STORE_F32) {
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = ld(B.g, o, off32(B, i));
  } else {
    const uint32_t o2 = o >> 1;
    const float p3 = 3.0f * ld(B.pR, o);
    g[0] = ld(B.rest, o, SG * B.pb);
#pragma unroll
    for (int i = 1; i < 9; ++i)
      g[i] = fmaf(dec16<ST>(ld16(B.g, o2, off16(B, i))), 1.0f / SC_G, W9[i] * p3);
  }
}

struct Slot {
  float phi, T, C, fs, p;
};

// Raw inputs of one closure slot: its f, h, l populations and p^{n-1}.
struct Raw {
  float f[5], h[5], l[5], p;
};

template <int ST>
__device__ __forceinline__ void load_raw(const KParams& P, const Bufs& B, uint32_t o, Raw& r) {
  load_fhl<ST>(P, B, o, r.f, r.h, r.l);
  r.p = ld(B.p_old, o);
}

// Closure of the node (mx, my) staged in closure-ring slot (lx, ly), from its
// raw inputs and div u^{n-1} on the velocity ring.  A ghost slot (side != 0)
// holds the mirror node with the wall's temperature transform.
template <int UY>
__device__ __forceinline__ Slot close_slot(const KParams& P, const Raw& r, int y0, int mx,
                                           int my, int side, int lx, int ly, float (*s_ux)[UX],
                                           float (*s_uy)[UX], float& Dout, Closure& cout) {
  float phi0 = 0.f, E0 = 0.f, C = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    phi0 += r.f[i];
    E0 += r.h[i];
    C += r.l[i];
  }
  // velocity-ring position of the source node
  const int ux = lx + 1;
  int uy = side == 0 ? ly + 1 : my - y0 + 2;
  uy = min(max(uy, 1), UY - 2);
  // div u^{n-1} by the isotropic gradient (D2Q9 weights / cs^2)
  const float dux = (1.f / 3.f) * (s_ux[uy][ux + 1] - s_ux[uy][ux - 1]) +
                    (1.f / 12.f) * (s_ux[uy + 1][ux + 1] + s_ux[uy - 1][ux + 1] -
                                    s_ux[uy + 1][ux - 1] - s_ux[uy - 1][ux - 1]);
  const float duy = (1.f / 3.f) * (s_uy[uy + 1][ux] - s_uy[uy - 1][ux]) +
                    (1.f / 12.f) * (s_uy[uy + 1][ux + 1] + s_uy[uy + 1][ux - 1] -
                                    s_uy[uy - 1][ux + 1] - s_uy[uy - 1][ux - 1]);
  const float D = dux + duy;
  Dout = D;
  const Closure c = closure(P, phi0, E0, D);
  cout = c;
  Slot s;
  s.phi = c.phi;
  s.C = C;
  s.fs = c.fs;
  s.p = r.p;
  float T = c.T;
  if (side < 0 && P.tlo_dir) T = 2.0f * (P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)mx)) - T;
  if (side > 0 && P.thi_dir) T = 2.0f * P.T_hi - T;
  s.T = T;
  return s;
}

// One tile of one step (the body of the single-grid and the batched kernels).
template <bool DRY, int ST, int TY>
__device__ __forceinline__ void step2d_tile(const KParams& P, const StepArgs& A, const int tile) {
  constexpr int NT = Geo<TY>::NT, HY = Geo<TY>::HY, UY = Geo<TY>::UY, RING = Geo<TY>::RING;
  __shared__ float s_ux[UY][UX], s_uy[UY][UX];
  __shared__ float s_phi[HY][HX], s_T[HY][HX], s_C[HY][HX], s_fs[HY][HX], s_p[HY][HX];
  __shared__ double s_red[NT / 64];

  const int bx = tile % P.nblk_x, by = tile / P.nblk_x;
  const int x0 = bx * TX, y0 = by * TY;
  const int tid = threadIdx.x, tx = tid & (TX - 1);
  const int ty = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform row
  const int nx = P.nx, ny = P.ny;
  const Bufs B = make_bufs<ST>(P, A);
  const uint32_t PB = B.pb, HB = B.hb, NB = (uint32_t)P.N * 4u;  // plane / output bytes
  const int gx = x0 + tx, gy = y0 + ty;
  const bool valid = gx < nx && gy < ny;
  // own slot; lanes of a partial tile outside the grid stage the periodic
  // image or wall mirror that the ring of the last nodes of the grid needs
  int oside;
  const int omx = wrap_near(gx, nx);
  const int omy = map_y(gy, ny, P.walls, oside);
  const uint32_t on = node_off(omx, omy, nx);
  // Every global load of the block -- own node and its ring slot -- is issued
  // before the first barrier, so a block waits for memory once.
  float g[9];
  load_g<ST>(B, on, g);
  const rsrc_t r_fs = rsrc(A.fs, PB);
  const float fs_prev = ld(r_fs, on);
  const float phiP = ld(rsrc(A.phiP_old, PB), on), CP = ld(rsrc(A.CP_old, PB), on);
  Raw own;
  load_raw<ST>(P, B, on, own);
  // 1. previous velocity on tile + 2 ring; no-slip ghosts are negated mirrors.
  // All of a thread's slots are loaded before the first is stored.
  constexpr int UN = UX * UY, UIT = (UN + NT - 1) / NT;
  float vx[UIT], vy[UIT], sg[UIT];
#pragma unroll
  for (int k = 0; k < UIT; ++k) {
    const int s = min(tid + k * NT, UN - 1);
    const int lx = s % UX, ly = s / UX;
    int side;
    const int my = map_y(y0 + ly - 2, ny, P.walls, side);
    const uint32_t o = node_off(wrap_near(x0 + lx - 2, nx), my, nx);
    sg[k] = side ? -1.0f : 1.0f;
    vx[k] = ld(B.u_old, o);
    vy[k] = ld(B.u_old, o, PB);
  }
  // ring slots go to the first threads, so only ceil(RING / 64) waves run the
  // extra closure
  const bool has_ring = tid < RING;
  int rlx = 0, rly = 0, rmx = 0, rmy = 0, rside = 0;
  Raw ring;
  if (has_ring) {
    if (tid < HX) {
      rlx = tid;
      rly = 0;
    } else if (tid < 2 * HX) {
      rlx = tid - HX;
      rly = HY - 1;
    } else if (tid < 2 * HX + TY) {
      rlx = 0;
      rly = tid - 2 * HX + 1;
    } else {
      rlx = HX - 1;
      rly = tid - 2 * HX - TY + 1;
    }
    rmy = map_y(y0 + rly - 1, ny, P.walls, rside);
    rmx = wrap_near(x0 + rlx - 1, nx);
    load_raw<ST>(P, B, node_off(rmx, rmy, nx), ring);
  }

#pragma unroll
  for (int k = 0; k < UIT; ++k) {
    const int s = tid + k * NT;
    if (s < UN) {
      s_ux[s / UX][s % UX] = sg[k] * vx[k];
      s_uy[s / UX][s % UX] = sg[k] * vy[k];
    }
  }
  __syncthreads();

  // 2. closure on tile + 1 ring
  float D;
  Closure cl;
  {
    const Slot s =
        close_slot<UY>(P, own, y0, omx, omy, oside, tx + 1, ty + 1, s_ux, s_uy, D, cl);
    s_phi[ty + 1][tx + 1] = s.phi;
    s_T[ty + 1][tx + 1] = s.T;
    s_C[ty + 1][tx + 1] = s.C;
    s_fs[ty + 1][tx + 1] = s.fs;
    s_p[ty + 1][tx + 1] = s.p;
  }
  if (has_ring) {
    float D2;
    Closure c2;
    const Slot s =
        close_slot<UY>(P, ring, y0, rmx, rmy, rside, rlx, rly, s_ux, s_uy, D2, c2);
    s_phi[rly][rlx] = s.phi;
    s_T[rly][rlx] = s.T;
    s_C[rly][rlx] = s.C;
    s_fs[rly][rlx] = s.fs;
    s_p[rly][rlx] = s.p;
  }
  __syncthreads();
  const float* f = own.f;
  const float* h = own.h;
  const float* l = own.l;

  const int cx = tx + 1, cy = ty + 1;

  // 3. stencils (isotropic D2Q9 gradient / Laplacian)
#define GRADX(a)                                                          \
  ((1.f / 3.f) * (a[cy][cx + 1] - a[cy][cx - 1]) +                        \
   (1.f / 12.f) * (a[cy + 1][cx + 1] + a[cy - 1][cx + 1] - a[cy + 1][cx - 1] - \
                   a[cy - 1][cx - 1]))
#define GRADY(a)                                                          \
  ((1.f / 3.f) * (a[cy + 1][cx] - a[cy - 1][cx]) +                        \
   (1.f / 12.f) * (a[cy + 1][cx + 1] + a[cy + 1][cx - 1] - a[cy - 1][cx + 1] - \
                   a[cy - 1][cx - 1]))
  const float phi = s_phi[cy][cx], T = s_T[cy][cx], C = s_C[cy][cx], fs = s_fs[cy][cx];
  const float gpx = GRADX(s_phi), gpy = GRADY(s_phi);
  const float gTx = GRADX(s_T), gTy = GRADY(s_T);
  const float gCx = GRADX(s_C), gCy = GRADY(s_C);
  const float gfx = GRADX(s_fs), gfy = GRADY(s_fs);
  const float gPx = GRADX(s_p), gPy = GRADY(s_p);
  const float lap = (2.f / 3.f) * (s_phi[cy][cx + 1] + s_phi[cy][cx - 1] + s_phi[cy + 1][cx] +
                                   s_phi[cy - 1][cx]) +
                    (1.f / 6.f) * (s_phi[cy + 1][cx + 1] + s_phi[cy + 1][cx - 1] +
                                   s_phi[cy - 1][cx + 1] + s_phi[cy - 1][cx - 1]) -
                    (10.f / 3.f) * phi;
#undef GRADX
#undef GRADY

  // 4. interface force (Eq. Fs), velocity with solid drag, pressure (Sec. 3.2)
  const float grx = 0.5f * (P.rho_l - P.rho_g) * gpx + (P.rho_s - P.rho_l) * gfx;
  const float gry = 0.5f * (P.rho_l - P.rho_g) * gpy + (P.rho_s - P.rho_l) * gfy;
  const float g2 = gpx * gpx + gpy * gpy;
  // 1 / max(|grad phi|, 1e-6): n regularised in the bulk
  const float inv_ng = __builtin_amdgcn_rsqf(fmaxf(g2, 1e-12f));
  const float nvx = gpx * inv_ng, nvy = gpy * inv_ng;
  const float mu = phi * (phi * phi - 1.0f) * P.ieps2 - lap;
  const float sig = P.sigma0 + P.sigma_T * (T - P.T_ref) + P.sigma_c * (C - P.c_ref);
  const float gsx = P.sigma_T * gTx + P.sigma_c * gCx;
  const float gsy = P.sigma_T * gTy + P.sigma_c * gCy;
  const float gsdp = gsx * gpx + gsy * gpy;
  const float wst = P.st_mode == 0 ? (1.0f - fs) : 1.0f;
  const float Fx = wst * P.alpha * (sig * mu * gpx + g2 * gsx - gsdp * gpx) + P.bfx;
  const float Fy = wst * P.alpha * (sig * mu * gpy + g2 * gsy - gsdp * gpy) + P.bfy;

  const float rho = interp(phi, fs, P.rho_l, P.rho_g, P.rho_s);
  const float rcp = rho * interp(phi, fs, P.cp_l, P.cp_g, P.cp_s);
  const float momx = g[1] - g[3] + g[5] - g[6] - g[7] + g[8];
  const float momy = g[2] - g[4] + g[5] + g[6] - g[7] - g[8];
  const float irho = frcp(rho);
  const float usx = (momx + 0.5f * Fx) * irho, usy = (momy + 0.5f * Fy) * irho;
  const float fdx = -fs * usx, fdy = -fs * usy;
  const float ux = usx + 0.5f * fdx, uy = usy + 0.5f * fdy;
  const float mdot = P.ratio * (fs - fs_prev);
  const float S = rho * mdot + ux * grx + uy * gry;
  const float Ftx = Fx - gPx + kCs2 * grx, Fty = Fy - gPy + kCs2 * gry;
  const float Ffx = Fx + rho * fdx, Ffy = Fy + rho * fdy;
  const float uu = ux * ux + uy * uy;
  const float uFt = ux * Ftx + uy * Fty;
  // Rest components of every equilibrium and source below are taken as the
  // complement of the moving ones, so that the FP32-rounded weights cannot
  // bias the conserved sums (sum G = S, sum g_eq = 0, sum f_eq = phi, ...).
  float G[9];
  G[0] = S;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const float cu = CX[i] * ux + CY[i] * uy;
    const float cFt = CX[i] * Ftx + CY[i] * Fty;
    const float cFf = CX[i] * Ffx + CY[i] * Ffy;
    // (u Ft + Ft u):(c c - cs2 I) / (2 cs2^2) = 9 (c.u)(c.Ft) - 3 u.Ft
    G[i] = W9[i] * (S + kInvCs2 * cFf + 9.0f * (cu * cFt) - 3.0f * uFt);
    G[0] -= G[i];
  }
  float sum_nz = 0.f;
#pragma unroll
  for (int i = 1; i < 9; ++i) sum_nz += g[i];
  const float s0 = W9[0] * (-1.5f * uu);
  const float pn = (kCs2 / (1.0f - W9[0])) * (sum_nz + 0.5f * S + P.tau_gp * G[0] + rho * s0);

  if (DRY) {
    if (valid) {
      float* const* o = A.out;
      if (o[0]) st(rsrc(o[0], NB), on, 0, phi);
      if (o[1]) st(rsrc(o[1], NB), on, 0, 1.0f - fs);
      if (o[2]) st(rsrc(o[2], NB), on, 0, T);
      if (o[3]) st(rsrc(o[3], NB), on, 0, C);
      if (o[4]) st(rsrc(o[4], NB), on, 0, ux);
      if (o[5]) st(rsrc(o[5], NB), on, 0, uy);
      if (o[6]) st(rsrc(o[6], NB), on, 0, 0.0f);
      if (o[7]) st(rsrc(o[7], NB), on, 0, pn);
      if (o[8]) st(rsrc(o[8], NB), on, 0, rho);
    }
    if (A.tot_part) {
      double vals[6] = {0, 0, 0, 0, 0, 0};
      if (valid) {
        float sf = 0.f, sh = 0.f, sl = 0.f;
        bool bad = false;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          sf += f[i];
          sh += h[i];
          sl += l[i];
        }
        bad = !isfinite(sf) || !isfinite(sh) || !isfinite(sl) || !isfinite(phi) ||
              !isfinite(T) || !isfinite(ux) || !isfinite(uy) || !isfinite(pn);
#pragma unroll
        for (int i = 0; i < 9; ++i) bad = bad || !isfinite(g[i]);
        double df = 0, dh = 0, dl = 0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
          df += (double)f[i];
          dh += (double)h[i];
          dl += (double)l[i];
        }
        vals[0] = df;
        vals[1] = dl;
        vals[2] = dh;
        vals[3] = (double)fs;
        vals[4] = (double)clamp01(0.5f * (1.0f + phi));
        vals[5] = bad ? 1.0 : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double s = block_sum<NT>(vals[k], s_red);
        if (tid == 0) A.tot_part[(long)tile * 8 + k] = s;
      }
    }
    return;
  }

  // 5. collisions, each post-collision population pushed along its link as
  // soon as it is computed (no arrays of post-collision values stay live).
  // A link across a wall is closed by half-way bounce-back into the opposite
  // slot of the same node; h at a Dirichlet wall by anti-bounce-back.
  // Link targets: x periodic; y periodic, or closed by the walls.  Row
  // offsets are wave-uniform, column offsets per lane.
  const bool wlo = P.walls && gy == 0, whi = P.walls && gy == ny - 1;
  const int rm = gy == 0 ? ny - 1 : gy - 1, rp = gy == ny - 1 ? 0 : gy + 1;
  const uint32_t rowb[3] = {(uint32_t)rm * (uint32_t)nx * 4u, (uint32_t)gy * (uint32_t)nx * 4u,
                            (uint32_t)rp * (uint32_t)nx * 4u};
  const uint32_t colb[3] = {(uint32_t)(omx == 0 ? nx - 1 : omx - 1) * 4u, (uint32_t)omx * 4u,
                            (uint32_t)(omx == nx - 1 ? 0 : omx + 1) * 4u};
  auto walled = [&](int i) { return (CY[i] < 0 && wlo) || (CY[i] > 0 && whi); };
  // Store post-collision value v of link i (> 0) of a set at the node it
  // streams to.  16-bit: encoded against w_i r of that node, where ref(dy, dx)
  // reads w_i r from the LDS ring.
  auto push = [&](rsrc_t set, int i, float v, float scale, auto ref) {
    if constexpr (ST == LBFZ_STORE_F32) {
      if (walled(i))
        st(set, on, off32(B, OPP[i]), v);  // half-way bounce-back
      else
        st(set, rowb[CY[i] + 1] + colb[CX[i] + 1], off32(B, i), v);
    } else {
      if (walled(i)) {
        st16(set, on >> 1, off16(B, OPP[i]), enc16<ST>((v - ref(0, 0)) * scale));
      } else {
        st16(set, (rowb[CY[i] + 1] + colb[CX[i] + 1]) >> 1, off16(B, i),
             enc16<ST>((v - ref(CY[i], CX[i])) * scale));
      }
    }
  };
  // rest population of set k at the own node
  auto put_rest = [&](rsrc_t set, int k, float v) {
    if constexpr (ST == LBFZ_STORE_F32)
      st(set, on, kSetPad, v);
    else
      st(B.drest, on, k * PB, v);
  };
  // flow BGK (Sec. 3.2)
  if (valid) {
    float geq_sum = 0.0f;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const float cu = CX[i] * ux + CY[i] * uy;
      const float si = W9[i] * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
      const float geq = pn * kInvCs2 * W9[i] + rho * si;
      geq_sum += geq;
      push(B.dg, i, g[i] - (g[i] - geq) * P.itau_g + P.wg * G[i], SC_G,
           [&](int dy, int dx) { return W9[i] * (3.0f * s_p[cy + dy][cx + dx]); });
    }
    put_rest(B.dg, SG, g[0] - (g[0] + geq_sum) * P.itau_g + P.wg * G[0]);
  }
  // phase field BGK (Sec. 3.1)
  const float upx = s_ux[ty + 2][tx + 2], upy = s_uy[ty + 2][tx + 2];
  if (valid) {
    const float cf = kCs2 * (1.0f - phi * phi) * P.isq;
    const float Bx = (phi * ux - phiP * upx) + cf * nvx;
    const float By = (phi * uy - phiP * upy) + cf * nvy;
    float feq_sum = 0.0f, F_sum = 0.0f;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const float cu = CX[i] * ux + CY[i] * uy;
      const float Fi = W5[i] * (kInvCs2 * (CX[i] * Bx + CY[i] * By) + phi * D);
      const float feq = W5[i] * phi * (1.0f + kInvCs2 * cu);
      feq_sum += feq;
      F_sum += Fi;
      push(B.df, i, f[i] - (f[i] - feq) * P.itau_f + P.wf * Fi, SC_F,
           [&](int dy, int dx) { return W5[1] * s_phi[cy + dy][cx + dx]; });
    }
    put_rest(B.df, SF, f[0] - (f[0] - (phi - feq_sum)) * P.itau_f + P.wf * (phi * D - F_sum));
  }
  // enthalpy TRT (Sec. 3.3); E and Q from the closure of the own node
  if (valid) {
    float heq[5];
    const float rT = P.rhoc_ref * T, cT = rcp * T;
    heq[0] = cl.E;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const float cu = CX[i] * ux + CY[i] * uy;
      heq[i] = W5[i] * (rT + cT * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
      heq[0] -= heq[i];
    }
    const float hq = W5[1] * cl.Q, hq0 = cl.Q - 4.0f * hq;
    const float href_w = W5[1] * P.rhoc_ref;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const int o = OPP[i];
      const float hs = 0.5f * (h[i] + h[o]), ha = 0.5f * (h[i] - h[o]);
      const float es = 0.5f * (heq[i] + heq[o]), ea = 0.5f * (heq[i] - heq[o]);
      const float v = h[i] - (hs - es) * P.itau_s - (ha - ea) * P.itau_a +
                      P.ws * (i == 0 ? hq0 : hq);
      if (i == 0) {
        put_rest(B.dh, SH, v);
      } else if (walled(i) && ((CY[i] < 0 && P.tlo_dir) || (CY[i] > 0 && P.thi_dir))) {
        const float Tw = CY[i] < 0 ? P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)gx) : P.T_hi;
        const float hv = -v + 2.0f * W5[o] * P.rhoc_ref * Tw;  // anti-bounce-back
        if constexpr (ST == LBFZ_STORE_F32)
          st(B.dh, on, off32(B, o), hv);
        else
          st16(B.dh, on >> 1, off16(B, o), enc16<ST>((hv - href_w * T) * SC_H));
      } else {
        push(B.dh, i, v, SC_H, [&](int dy, int dx) { return href_w * s_T[cy + dy][cx + dx]; });
      }
    }
  }
  // solute BGK (Sec. 3.4)
  if (valid) {
    const float keff = 1.0f - fs * (1.0f - P.k_p);
    const float De = fs * P.k_p * P.Ds + (1.0f - fs) * P.Dl;
    const float ikeff = frcp(keff);
    const float tau_l = 3.0f * De * ikeff + 0.5f;  // D_e / (cs2 k_eff) + 1/2
    const float itau_l = frcp(tau_l), wl = 1.0f - 0.5f * itau_l;
    const float cr = (1.0f - phi) * C * P.isq, ck = (P.k_p - 1.0f) * C * ikeff;
    const float Lx = (C * ux - CP * upx) + kCs2 * (cr * nvx + ck * gfx);
    const float Ly = (C * uy - CP * upy) + kCs2 * (cr * nvy + ck * gfy);
    float leq_sum = 0.0f;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const float cu = CX[i] * ux + CY[i] * uy;
      const float Li = W5[i] * kInvCs2 * (CX[i] * Lx + CY[i] * Ly);
      const float leq = W5[i] * C * (1.0f + kInvCs2 * cu);
      leq_sum += leq;
      push(B.dl, i, l[i] - (l[i] - leq) * itau_l + wl * Li, SC_L,
           [&](int dy, int dx) { return W5[1] * s_C[cy + dy][cx + dx]; });
    }
    put_rest(B.dl, SL, l[0] - (l[0] - (C - leq_sum)) * itau_l);
  }

  // 6. the time-level state (16-bit: phi, C, T are also the decode references
  // of the populations just written)
  if (valid) {
    st(rsrc(A.p_new, PB), on, 0, pn);
    const rsrc_t r_un = rsrc(A.u_new, 2 * PB);
    st(r_un, on, 0, ux);
    st(r_un, on, PB, uy);
    st(r_fs, on, 0, fs);
    st(rsrc(A.phiP_new, PB), on, 0, phi);
    st(rsrc(A.CP_new, PB), on, 0, C);
    if constexpr (ST != LBFZ_STORE_F32) st(rsrc(A.T_new, PB), on, 0, T);
  }
  // phase-field source budget: sum of phi div u over the tile, FP64
  const double s = block_sum<NT>(valid ? (double)phi * (double)D : 0.0, s_red);
  if (tid == 0) A.mpc_part[tile] += s;
}

template <bool DRY, int ST, int TY>
__global__ __launch_bounds__(Geo<TY>::NT) void k_step2d(KParams P, StepArgs A) {
  // consecutive steps walk the tiles in opposite directions
  step2d_tile<DRY, ST, TY>(
      P, A, A.rev ? xcd_tile_rev(blockIdx.x, P.nblk) : xcd_tile(blockIdx.x, P.nblk));
}

// Batched sweep: every (case, tile) of one step of many grids in one launch.
// Work item e = (case, tile) comes from a table built on the host (in an
// XCD-aware order), with the case's parameters and the buffers of step
// parity `slot` read from the case table (wave-uniform: scalar loads).  One
// block per item, or a persistent grid whose blocks process items
// blockIdx.x, blockIdx.x + gridDim.x, ...: the loop holds 37 more VGPRs (122
// against 85: 4 waves per SIMD instead of 5), so the one-item form is a
// kernel of its own.
template <int ST, int TY>
__global__ __launch_bounds__(Geo<TY>::NT) void k_step2d_batch(
    const BatchCase* __restrict__ cases, const int2* __restrict__ work, int nwork, int slot) {
  for (int e = blockIdx.x; e < nwork; e += gridDim.x) {
    const int2 w = work[e];
    const int c = __builtin_amdgcn_readfirstlane(w.x);
    const int tile = __builtin_amdgcn_readfirstlane(w.y);
    step2d_tile<false, ST, TY>(cases[c].P, cases[c].A[slot], tile);
    __syncthreads();  // LDS is reused by the next item
  }
}
template <int ST, int TY>
__global__ __launch_bounds__(Geo<TY>::NT) void k_step2d_batch1(
    const BatchCase* __restrict__ cases, const int2* __restrict__ work, int slot) {
  const int2 w = work[blockIdx.x];
  const int c = __builtin_amdgcn_readfirstlane(w.x);
  const int tile = __builtin_amdgcn_readfirstlane(w.y);
  step2d_tile<false, ST, TY>(cases[c].P, cases[c].A[slot], tile);
}

// Fields of many grids in one launch: the dry pass (the step's closure, forces
// and velocity, no collision) over the same (case, tile) items, one block per
// item, the fields selected by `mask` (bit k: field k of lbfz_fields) written
// to grid c's slice dst + c * case_stride, one plane of N_c values per
// selected field in the order of the bits.
template <int ST, int TY>
__global__ __launch_bounds__(Geo<TY>::NT) void k_fields2d_batch(
    const BatchCase* __restrict__ cases, const int2* __restrict__ work, int slot,
    float* __restrict__ dst, long case_stride, uint32_t mask) {
  {
    const int e = blockIdx.x;
    const int2 w = work[e];
    const int c = __builtin_amdgcn_readfirstlane(w.x);
    const int tile = __builtin_amdgcn_readfirstlane(w.y);
    StepArgs A = cases[c].A[slot];
    const long N = cases[c].P.N;
    float* base = dst + (long)c * case_stride;
    int r = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      A.out[k] = ((mask >> k) & 1u) ? base + (long)r * N : nullptr;
      r += (mask >> k) & 1u;
    }
    A.tot_part = nullptr;
    step2d_tile<true, ST, TY>(cases[c].P, A, tile);
  }
}

// Equilibrium populations of the initial fields (u = 0, p = 0) and the zero
// previous-level state.  16-bit: every moving population sits exactly at its
// reference (offset 0), and the references phi, C, T are stored.
template <int ST>
__global__ __launch_bounds__(256) void k_init2d(KParams P, const double* __restrict__ phi_in,
                                                const double* __restrict__ T_in,
                                                const double* __restrict__ C_in,
                                                float* __restrict__ pop, StateArgs S) {
  const long N = P.N, PS = P.ps;
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < N;
       n += (long)gridDim.x * blockDim.x) {
    const float phi = (float)phi_in[n], T = (float)T_in[n], C = (float)C_in[n];
    const float psi = clamp01(0.5f * (1.0f + phi));
    const float rcl = psi * P.rc_l + (1.0f - psi) * P.rc_g;
    const float E = rcl * T + psi * P.rho_l_latent;
    float h0 = E, f0 = phi, l0 = C;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      h0 -= W5[i] * P.rhoc_ref * T;
      f0 -= W5[i] * phi;
      l0 -= W5[i] * C;
    }
    if constexpr (ST == LBFZ_STORE_F32) {
#pragma unroll
      for (int i = 1; i < 5; ++i) {
        const long m = n - kXS * CX[i];  // shifted plane position of node n
        pop[(PH + i) * PS + m] = W5[i] * P.rhoc_ref * T;
        pop[(PF + i) * PS + m] = W5[i] * phi;
        pop[(PL + i) * PS + m] = W5[i] * C;
      }
      pop[(PH + 0) * PS + n] = h0;
      pop[(PF + 0) * PS + n] = f0;
      pop[(PL + 0) * PS + n] = l0;
#pragma unroll
      for (int i = 0; i < 9; ++i) pop[(PG + i) * PS + n - kXS * CX[i]] = 0.0f;
      S.phiA[n] = 0.f;
      S.CA[n] = 0.f;
    } else {
      pop[SF * PS + n] = f0;
      pop[SG * PS + n] = 0.0f;
      pop[SH * PS + n] = h0;
      pop[SL * PS + n] = l0;
      uint16_t* m16 = reinterpret_cast<uint16_t*>(pop + 4 * PS);
#pragma unroll
      for (int j = 0; j < 20; ++j) {
        const int i = j < 4 ? j + 1 : (j < 12 ? j - 3 : (j < 16 ? j - 11 : j - 15));
        m16[j * PS + n - kXS * CX[i]] = enc16<ST>(0.0f);
      }
      // decode references of the step that reads these populations
      S.phiA[n] = phi;
      S.CA[n] = C;
      S.TA[n] = T;
      S.pC[n] = 0.f;
    }
    S.pA[n] = 0.f;
    S.pB[n] = 0.f;
    S.uA[n] = S.uA[PS + n] = 0.f;
    S.uB[n] = S.uB[PS + n] = 0.f;
    S.fs[n] = 0.f;
  }
}

// 16-bit forms: populations of the current level decoded to FP32 planes
// (state order) in dst[q * N + n], q < 24.
template <int ST>
__global__ __launch_bounds__(256) void k_export2d(KParams P, StepArgs A, float* __restrict__ dst) {
  const long N = P.N;
  const Bufs B = make_bufs<ST>(P, A);
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < N;
       n += (long)gridDim.x * blockDim.x) {
    const uint32_t o = (uint32_t)n * 4u;
    float f[5], h[5], l[5], g[9];
    load_fhl<ST>(P, B, o, f, h, l);
    load_g<ST>(B, o, g);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      dst[(PF + i) * N + n] = f[i];
      dst[(PH + i) * N + n] = h[i];
      dst[(PL + i) * N + n] = l[i];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) dst[(PG + i) * N + n] = g[i];
  }
}

// 16-bit forms: encode FP32 populations src[q * N + n] (state order) into the
// buffer A.dst with the references phi = A.phiP_old, C = A.CP_old, p =
// A.p_ref (all already imported) and T from the enthalpy map of the imported
// populations, which is stored in A.T_new.
template <int ST>
__global__ __launch_bounds__(256) void k_import2d(KParams P, StepArgs A,
                                                  const float* __restrict__ src) {
  const long N = P.N, PS = P.ps;
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < N;
       n += (long)gridDim.x * blockDim.x) {
    float f[5], h[5], l[5], g[9];
    float phi0 = 0.f, E = 0.f;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      f[i] = src[(PF + i) * N + n];
      h[i] = src[(PH + i) * N + n];
      l[i] = src[(PL + i) * N + n];
      phi0 += f[i];
      E += h[i];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) g[i] = src[(PG + i) * N + n];
    float T, fs;
    enthalpy_map(P, E, clamp01(0.5f * (1.0f + phi0)), T, fs);
    A.T_new[n] = T;
    const float rf = W5[1] * A.phiP_old[n], rl = W5[1] * A.CP_old[n];
    const float rh = W5[1] * P.rhoc_ref * T, p3 = 3.0f * A.p_ref[n];
    A.dst[SF * PS + n] = f[0];
    A.dst[SG * PS + n] = g[0];
    A.dst[SH * PS + n] = h[0];
    A.dst[SL * PS + n] = l[0];
    uint16_t* m16 = reinterpret_cast<uint16_t*>(A.dst + 4 * PS);
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const long m = n - kXS * CX[i];
      m16[(i - 1) * PS + m] = enc16<ST>((f[i] - rf) * SC_F);
      m16[(12 + i - 1) * PS + m] = enc16<ST>((h[i] - rh) * SC_H);
      m16[(16 + i - 1) * PS + m] = enc16<ST>((l[i] - rl) * SC_L);
    }
#pragma unroll
    for (int i = 1; i < 9; ++i)
      m16[(4 + i - 1) * PS + n - kXS * CX[i]] = enc16<ST>((g[i] - W9[i] * p3) * SC_G);
  }
}

// Equilibrium state of given macroscopic fields (restart from fields, e.g. a
// surrogate's prediction): the raw state planes of the exported layout --
// populations f, g, h, l at their equilibria of Sec. 3.1 - 3.4 for (phi, u),
// (p, rho, u), (E, T, u), (C, u), then the previous level's f_s, p, u, phi, C
// set to the same fields.  The liquid fraction comes as exported, 1 - f_s
// with f_s = psi (1 - f_l) <= psi; the enthalpy is the inverse of the
// enthalpy map written as sensible heat below the solidus, latent heat by
// the liquid fraction, sensible heat above the liquidus,
//   E = rc_s min(T, T_sol) + f_l (E_l - E_s) + rc_l max(T - T_liq, 0),
// which equals the map's E on each branch and, unlike a choice of branch by
// f_l or T alone, stays well-behaved for fields slightly off the map (a
// pure substance's mushy band is the single temperature T_m).  The flow's
// momentum is rho u / (1 - f_s / 2) (the solid drag's half-step undone, the
// interface force's half-step left out).  Non-equilibrium parts are zero.
__device__ __forceinline__ void equil_node(const KParams& P, const EquilFields& F,
                                           const StatePlanes& S, long n) {
  {
    const float phi = F.phi[n], T = F.T[n], C = F.C[n];
    const float ux = F.ux[n], uy = F.uy[n], p = F.p[n];
    const float psi = clamp01(0.5f * (1.0f + phi));
    const float fs = fminf(fmaxf(1.0f - F.fl[n], 0.0f), psi);
    const float fl = psi > 0.0f ? clamp01(1.0f - fs / psi) : 1.0f;
    const float rcs = psi * P.rc_s + (1.0f - psi) * P.rc_g;
    const float rcl = psi * P.rc_l + (1.0f - psi) * P.rc_g;
    const float Es = rcs * P.T_sol, El = rcl * P.T_liq + psi * P.rho_l_latent;
    const float E = rcs * fminf(T, P.T_sol) + fl * (El - Es) + rcl * fmaxf(T - P.T_liq, 0.0f);
    const float rho = interp(phi, fs, P.rho_l, P.rho_g, P.rho_s);
    const float rcp = rho * interp(phi, fs, P.cp_l, P.cp_g, P.cp_s);
    const float uu = ux * ux + uy * uy;
    float f0 = phi, h0 = E, l0 = C;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const float cu = CX[i] * ux + CY[i] * uy;
      const float fi = W5[i] * phi * (1.0f + kInvCs2 * cu);
      const float hi = W5[i] * (P.rhoc_ref * T + rcp * T * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
      const float li = W5[i] * C * (1.0f + kInvCs2 * cu);
      S.p[PF + i][n] = fi;
      S.p[PH + i][n] = hi;
      S.p[PL + i][n] = li;
      f0 -= fi;
      h0 -= hi;
      l0 -= li;
    }
    S.p[PF][n] = f0;
    S.p[PH][n] = h0;
    S.p[PL][n] = l0;
    const float dr = 1.0f / (1.0f - 0.5f * fs);
    const float vx = ux * dr, vy = uy * dr, vv = vx * vx + vy * vy;
    float g0 = 0.0f;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const float cu = CX[i] * vx + CY[i] * vy;
      const float gi = p * kInvCs2 * W9[i] + rho * W9[i] * (3.0f * cu + 4.5f * cu * cu - 1.5f * vv);
      S.p[PG + i][n] = gi;
      g0 -= gi;
    }
    S.p[PG][n] = g0;
    // previous level: f_s, p, u_x, u_y, phi, C
    S.p[24][n] = fs;
    S.p[25][n] = p;
    S.p[26][n] = ux;
    S.p[27][n] = uy;
    S.p[28][n] = phi;
    S.p[29][n] = C;
  }
}

__global__ __launch_bounds__(256) void k_equil2d(KParams P, EquilFields F, StatePlanes S) {
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < P.N;
       n += (long)gridDim.x * blockDim.x)
    equil_node(P, F, S, n);
}

// Batched restart: grid blockIdx.y of the job table, nodes strided over
// blockIdx.x (the job is read by every thread from the same address).
__global__ __launch_bounds__(256) void k_equil2d_batch(const EquilJob* __restrict__ jobs) {
  const EquilJob& J = jobs[blockIdx.y];
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < J.P.N;
       n += (long)gridDim.x * blockDim.x)
    equil_node(J.P, J.F, J.S, n);
}

int grid_of(long N) { return (int)std::min<long>((N + 255) / 256, 65536); }

}  // namespace

int tiles2d(int nx, int ny, int* nbx, int* nby, int ty) {
  if (ty <= 0) ty = TY_DEFAULT;
  *nbx = (nx + TX - 1) / TX;
  *nby = (ny + ty - 1) / ty;
  return (*nbx) * (*nby);
}

size_t pop_bytes2d(int storage, size_t ps) {
  return storage == LBFZ_STORE_F32 ? 24 * ps * sizeof(float)
                                   : 4 * ps * sizeof(float) + 20 * ps * sizeof(uint16_t);
}

hipError_t launch_init2d(const KParams& P, int storage, const double* phi, const double* T,
                         const double* C, float* pop, const StateArgs& S, hipStream_t st) {
  const int blocks = grid_of(P.N);
  switch (storage) {
    case LBFZ_STORE_F32:
      hipLaunchKernelGGL(k_init2d<LBFZ_STORE_F32>, dim3(blocks), dim3(256), 0, st, P, phi, T,
                         C, pop, S);
      break;
    case LBFZ_STORE_F16:
      hipLaunchKernelGGL(k_init2d<LBFZ_STORE_F16>, dim3(blocks), dim3(256), 0, st, P, phi, T,
                         C, pop, S);
      break;
    default:
      hipLaunchKernelGGL(k_init2d<LBFZ_STORE_BF16>, dim3(blocks), dim3(256), 0, st, P, phi, T,
                         C, pop, S);
  }
  return hipGetLastError();
}

template <int ST>
static void launch_step2d_st(const KParams& P, const StepArgs& A, bool dry, hipStream_t st) {
  constexpr int NT = Geo<TY_DEFAULT>::NT;
  if (dry)
    hipLaunchKernelGGL((k_step2d<true, ST, TY_DEFAULT>), dim3(P.nblk), dim3(NT), 0, st, P, A);
  else
    hipLaunchKernelGGL((k_step2d<false, ST, TY_DEFAULT>), dim3(P.nblk), dim3(NT), 0, st, P, A);
}

template <int ST, int TY>
static void launch_batch_st(const BatchCase* cases, const int2* work, int nwork, int grid,
                            int slot, hipStream_t st) {
  if (grid >= nwork)
    hipLaunchKernelGGL((k_step2d_batch1<ST, TY>), dim3(nwork), dim3(Geo<TY>::NT), 0, st, cases,
                       work, slot);
  else
    hipLaunchKernelGGL((k_step2d_batch<ST, TY>), dim3(grid), dim3(Geo<TY>::NT), 0, st, cases,
                       work, nwork, slot);
}

hipError_t launch_step2d(const KParams& P, int storage, const StepArgs& A, bool dry,
                         hipStream_t st) {
  switch (storage) {
    case LBFZ_STORE_F32: launch_step2d_st<LBFZ_STORE_F32>(P, A, dry, st); break;
    case LBFZ_STORE_F16: launch_step2d_st<LBFZ_STORE_F16>(P, A, dry, st); break;
    default: launch_step2d_st<LBFZ_STORE_BF16>(P, A, dry, st);
  }
  return hipGetLastError();
}

hipError_t launch_step2d_batch(int storage, int ty, const BatchCase* cases, const int2* work,
                               int nwork, int grid, int slot, hipStream_t st) {
  if (nwork <= 0) return hipSuccess;
  if (grid <= 0 || grid > nwork) grid = nwork;
  switch (storage * 16 + ty) {
    case LBFZ_STORE_F32 * 16 + 4: launch_batch_st<LBFZ_STORE_F32, 4>(cases, work, nwork, grid, slot, st); break;
    case LBFZ_STORE_F32 * 16 + 8: launch_batch_st<LBFZ_STORE_F32, 8>(cases, work, nwork, grid, slot, st); break;
    case LBFZ_STORE_F16 * 16 + 4: launch_batch_st<LBFZ_STORE_F16, 4>(cases, work, nwork, grid, slot, st); break;
    case LBFZ_STORE_F16 * 16 + 8: launch_batch_st<LBFZ_STORE_F16, 8>(cases, work, nwork, grid, slot, st); break;
    case LBFZ_STORE_BF16 * 16 + 4: launch_batch_st<LBFZ_STORE_BF16, 4>(cases, work, nwork, grid, slot, st); break;
    case LBFZ_STORE_BF16 * 16 + 8: launch_batch_st<LBFZ_STORE_BF16, 8>(cases, work, nwork, grid, slot, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int ST, int TY>
static void launch_fields_batch_st(const BatchCase* cases, const int2* work, int nwork, int slot,
                                   float* dst, long case_stride, uint32_t mask, hipStream_t st) {
  hipLaunchKernelGGL((k_fields2d_batch<ST, TY>), dim3(nwork), dim3(Geo<TY>::NT), 0, st, cases,
                     work, slot, dst, case_stride, mask);
}

hipError_t launch_fields2d_batch(int storage, int ty, const BatchCase* cases, const int2* work,
                                 int nwork, int slot, float* dst, long case_stride,
                                 uint32_t mask, hipStream_t st) {
  if (nwork <= 0) return hipSuccess;
  switch (storage * 16 + ty) {
    case LBFZ_STORE_F32 * 16 + 4: launch_fields_batch_st<LBFZ_STORE_F32, 4>(cases, work, nwork, slot, dst, case_stride, mask, st); break;
    case LBFZ_STORE_F32 * 16 + 8: launch_fields_batch_st<LBFZ_STORE_F32, 8>(cases, work, nwork, slot, dst, case_stride, mask, st); break;
    case LBFZ_STORE_F16 * 16 + 4: launch_fields_batch_st<LBFZ_STORE_F16, 4>(cases, work, nwork, slot, dst, case_stride, mask, st); break;
    case LBFZ_STORE_F16 * 16 + 8: launch_fields_batch_st<LBFZ_STORE_F16, 8>(cases, work, nwork, slot, dst, case_stride, mask, st); break;
    case LBFZ_STORE_BF16 * 16 + 4: launch_fields_batch_st<LBFZ_STORE_BF16, 4>(cases, work, nwork, slot, dst, case_stride, mask, st); break;
    case LBFZ_STORE_BF16 * 16 + 8: launch_fields_batch_st<LBFZ_STORE_BF16, 8>(cases, work, nwork, slot, dst, case_stride, mask, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_export2d(const KParams& P, int storage, const StepArgs& A, float* dst,
                           hipStream_t st) {
  const int blocks = grid_of(P.N);
  if (storage == LBFZ_STORE_F16)
    hipLaunchKernelGGL(k_export2d<LBFZ_STORE_F16>, dim3(blocks), dim3(256), 0, st, P, A, dst);
  else
    hipLaunchKernelGGL(k_export2d<LBFZ_STORE_BF16>, dim3(blocks), dim3(256), 0, st, P, A, dst);
  return hipGetLastError();
}

hipError_t launch_import2d(const KParams& P, int storage, const StepArgs& A, const float* src,
                           hipStream_t st) {
  const int blocks = grid_of(P.N);
  if (storage == LBFZ_STORE_F16)
    hipLaunchKernelGGL(k_import2d<LBFZ_STORE_F16>, dim3(blocks), dim3(256), 0, st, P, A, src);
  else
    hipLaunchKernelGGL(k_import2d<LBFZ_STORE_BF16>, dim3(blocks), dim3(256), 0, st, P, A, src);
  return hipGetLastError();
}

hipError_t launch_equil2d(const KParams& P, const EquilFields& F, const StatePlanes& S,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_equil2d, dim3(grid_of(P.N)), dim3(256), 0, st, P, F, S);
  return hipGetLastError();
}

hipError_t launch_equil2d_batch(const EquilJob* jobs, int njobs, long max_n, hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  const int bx = (int)std::min<long>((max_n + 255) / 256, std::max(1L, 8192L / njobs));
  hipLaunchKernelGGL(k_equil2d_batch, dim3(bx, njobs), dim3(256), 0, st, jobs);
  return hipGetLastError();
}

}  // namespace lbfz
