// lbfz_2d.hip -- fused 2D step of the coupled LB freezing scheme
// (arXiv 2511.09422, Sec. 3) for gfx950: D2Q9 flow g, D2Q5 phase field f,
// enthalpy h (TRT) and solute l.
//
// One kernel launch = one time step.  Populations live in two SoA buffers
// (plane q of N floats each: f 0..4, g 5..13, h 14..18, l 19..23); a step
// reads buffer A at each node's own location and pushes post-collision values
// along their links into buffer B (half-way bounce-back / anti-bounce-back at
// walls).  Each 64x4 tile stages in LDS
//   - the previous velocity on the tile + 2 ring   (div u for the closure),
//   - phi, T, C, f_s of the tile + 1 ring, computed from that ring's own
//     populations (the pointwise closure, evaluated redundantly on the ring),
//   - the previous pressure on the tile + 1 ring,
// and then every thread owns one node: stencils, forces, velocity, pressure,
// four collisions and the streaming writes.  Reads and writes each touch every
// population once, so HBM traffic is the algorithmic 240 B per node update.
#include "lbfz_common.hpp"
#include "lbfz_kernels.hpp"

namespace lbfz {

namespace {

#ifndef LBFZ_TY
#define LBFZ_TY 4
#endif
constexpr int TX = 64, TY = LBFZ_TY, NT = TX * TY;
constexpr int HX = TX + 2, HY = TY + 2;  // closure ring
constexpr int UX = TX + 4, UY = TY + 4;  // velocity ring
constexpr int RING = 2 * HX + 2 * TY;
static_assert(RING <= NT, "every ring slot needs a thread");

constexpr int PF = 0, PG = 5, PH = 14, PL = 19;

// D2Q9 (first five = D2Q5)
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr float W9[9] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                         1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
constexpr float W5[5] = {1.f / 3, 1.f / 6, 1.f / 6, 1.f / 6, 1.f / 6};

__device__ __forceinline__ int wrapc(int v, int n) {
  return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Map a wall-axis coordinate to the node whose value its slot holds.
// side: 0 inside, -1 ghost below the low wall, +1 ghost above the high wall.
__device__ __forceinline__ int map_axis(int g, int n, int walls, int& side) {
  side = 0;
  if (walls) {
    if (g < 0) {
      side = -1;
      g = -1 - g;
    } else if (g >= n) {
      side = 1;
      g = 2 * n - 1 - g;
    }
    g = min(max(g, 0), n - 1);
  } else {
    g = ((g % n) + n) % n;
  }
  return g;
}

__device__ __forceinline__ int map_periodic(int g, int n) { return ((g % n) + n) % n; }

struct Slot {
  float phi, T, C, fs, p;
};

// Closure of the node staged in ring slot (lx, ly) (closure-ring coordinates).
// Returns the slot values; pops of the source node are returned in f/h/l.
__device__ __forceinline__ Slot eval_slot(const KParams& P, const float* __restrict__ src,
                                          const float* __restrict__ p_old, int x0, int y0,
                                          int lx, int ly, float (*s_ux)[UX],
                                          float (*s_uy)[UX], float* f, float* h, float* l,
                                          float& Dout, Closure& cout) {
  const int nx = P.nx, ny = P.ny;
  const long N = P.N;
  const int mx = map_periodic(x0 + lx - 1, nx);
  int side;
  const int my = map_axis(y0 + ly - 1, ny, P.walls, side);
  const int n = my * nx + mx;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    f[i] = src[(PF + i) * N + n];
    h[i] = src[(PH + i) * N + n];
    l[i] = src[(PL + i) * N + n];
  }
  float phi0 = 0.f, E0 = 0.f, C = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    phi0 += f[i];
    E0 += h[i];
    C += l[i];
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
  s.p = p_old[n];
  float T = c.T;
  if (side < 0 && P.tlo_dir) T = 2.0f * (P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)mx)) - T;
  if (side > 0 && P.thi_dir) T = 2.0f * P.T_hi - T;
  s.T = T;
  return s;
}

#ifdef LBFZ_WPE
#define LBFZ_OCC __attribute__((amdgpu_waves_per_eu(LBFZ_WPE, 8)))
#else
#define LBFZ_OCC
#endif

template <bool DRY>
__global__ __launch_bounds__(NT) LBFZ_OCC void k_step2d(KParams P, Step2DArgs A) {
  __shared__ float s_ux[UY][UX], s_uy[UY][UX];
  __shared__ float s_phi[HY][HX], s_T[HY][HX], s_C[HY][HX], s_fs[HY][HX], s_p[HY][HX];
  __shared__ double s_red[NT / 64];

  const int tile = xcd_tile(blockIdx.x, P.nblk);
  const int bx = tile % P.nblk_x, by = tile / P.nblk_x;
  const int x0 = bx * TX, y0 = by * TY;
  const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
  const int nx = P.nx, ny = P.ny;
  const long N = P.N;
  const float* __restrict__ src = A.src;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool valid = gx < nx && gy < ny;
  const int n = valid ? gy * nx + gx : 0;
  // own-node loads that do not depend on the LDS phases are issued first
  float g[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) g[i] = src[(PG + i) * N + n];
  const float fs_prev = A.fs[n];
  const float phiP = A.phiP[n], CP = A.CP[n];

  // 1. previous velocity on tile + 2 ring; no-slip ghosts are negated mirrors
  for (int s = tid; s < UX * UY; s += NT) {
    const int lx = s % UX, ly = s / UX;
    const int gx = map_periodic(x0 + lx - 2, nx);
    int side;
    const int gy = map_axis(y0 + ly - 2, ny, P.walls, side);
    const int n = gy * nx + gx;
    const float sg = side ? -1.0f : 1.0f;
    s_ux[ly][lx] = sg * A.u_old[n];
    s_uy[ly][lx] = sg * A.u_old[N + n];
  }
  __syncthreads();

  // 2. closure on tile + 1 ring: own slot first (pops kept in registers)
  float f[5], h[5], l[5], D;
  Closure cl;
  {
    const Slot s = eval_slot(P, src, A.p_old, x0, y0, tx + 1, ty + 1, s_ux, s_uy, f, h, l, D,
                             cl);
    s_phi[ty + 1][tx + 1] = s.phi;
    s_T[ty + 1][tx + 1] = s.T;
    s_C[ty + 1][tx + 1] = s.C;
    s_fs[ty + 1][tx + 1] = s.fs;
    s_p[ty + 1][tx + 1] = s.p;
  }
  // ring slots are dealt to the waves in turn (slot r -> lane r / NW of wave
  // r % NW) so that every wave carries an equal share of the extra closures
  constexpr int NW = NT / 64;
  const int rslot = (tid & 63) * NW + (tid >> 6);
  if (rslot < RING) {
    int lx, ly;
    if (rslot < HX) {
      lx = rslot;
      ly = 0;
    } else if (rslot < 2 * HX) {
      lx = rslot - HX;
      ly = HY - 1;
    } else if (rslot < 2 * HX + TY) {
      lx = 0;
      ly = rslot - 2 * HX + 1;
    } else {
      lx = HX - 1;
      ly = rslot - 2 * HX - TY + 1;
    }
    float f2[5], h2[5], l2[5], D2;
    Closure c2;
    const Slot s = eval_slot(P, src, A.p_old, x0, y0, lx, ly, s_ux, s_uy, f2, h2, l2, D2, c2);
    s_phi[ly][lx] = s.phi;
    s_T[ly][lx] = s.T;
    s_C[ly][lx] = s.C;
    s_fs[ly][lx] = s.fs;
    s_p[ly][lx] = s.p;
  }
  __syncthreads();

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
  const float ng = sqrtf(g2);
  const float inv_ng = 1.0f / fmaxf(ng, 1e-6f);  // n regularised in the bulk
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
  const float irho = 1.0f / rho;
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
  const float pn = (kCs2 / (1.0f - W9[0])) * (sum_nz + 0.5f * S + P.tau_g * G[0] + rho * s0);

  if (DRY) {
    if (valid) {
      float* const* o = A.out;
      if (o[0]) o[0][n] = phi;
      if (o[1]) o[1][n] = 1.0f - fs;
      if (o[2]) o[2][n] = T;
      if (o[3]) o[3][n] = C;
      if (o[4]) o[4][n] = ux;
      if (o[5]) o[5][n] = uy;
      if (o[6]) o[6][n] = 0.0f;
      if (o[7]) o[7][n] = pn;
      if (o[8]) o[8][n] = rho;
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
  float* __restrict__ dst = A.dst;
  auto target = [&](int i, int& m) -> bool {  // true: the link leaves through a wall
    const int ty2 = gy + CY[i];
    if (P.walls && (ty2 < 0 || ty2 >= ny)) return true;
    m = wrapc(ty2, ny) * nx + wrapc(gx + CX[i], nx);
    return false;
  };
  auto push = [&](int base, int i, float v) {
    int m = n;
    if (target(i, m))
      dst[(base + OPP[i]) * N + n] = v;
    else
      dst[(base + i) * N + m] = v;
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
      push(PG, i, g[i] - (g[i] - geq) * P.itau_g + P.wg * G[i]);
    }
    dst[(PG + 0) * N + n] = g[0] - (g[0] + geq_sum) * P.itau_g + P.wg * G[0];
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
      push(PF, i, f[i] - (f[i] - feq) * P.itau_f + P.wf * Fi);
    }
    dst[(PF + 0) * N + n] =
        f[0] - (f[0] - (phi - feq_sum)) * P.itau_f + P.wf * (phi * D - F_sum);
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
    const float Tw_lo = P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)gx);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const int o = OPP[i];
      const float hs = 0.5f * (h[i] + h[o]), ha = 0.5f * (h[i] - h[o]);
      const float es = 0.5f * (heq[i] + heq[o]), ea = 0.5f * (heq[i] - heq[o]);
      const float v = h[i] - (hs - es) * P.itau_s - (ha - ea) * P.itau_a +
                      P.ws * (i == 0 ? hq0 : hq);
      int m = n;
      if (target(i, m)) {
        const int ty2 = gy + CY[i];
        float hv = v;
        if (ty2 < 0 && P.tlo_dir) hv = -hv + 2.0f * W5[o] * P.rhoc_ref * Tw_lo;
        if (ty2 >= ny && P.thi_dir) hv = -hv + 2.0f * W5[o] * P.rhoc_ref * P.T_hi;
        dst[(PH + o) * N + n] = hv;
      } else {
        dst[(PH + i) * N + m] = v;
      }
    }
  }
  // solute BGK (Sec. 3.4)
  if (valid) {
    const float keff = 1.0f - fs * (1.0f - P.k_p);
    const float De = fs * P.k_p * P.Ds + (1.0f - fs) * P.Dl;
    const float tau_l = De / (kCs2 * keff) + 0.5f;
    const float itau_l = 1.0f / tau_l, wl = 1.0f - 0.5f * itau_l;
    const float cr = (1.0f - phi) * C * P.isq, ck = (P.k_p - 1.0f) * C / keff;
    const float Lx = (C * ux - CP * upx) + kCs2 * (cr * nvx + ck * gfx);
    const float Ly = (C * uy - CP * upy) + kCs2 * (cr * nvy + ck * gfy);
    float leq_sum = 0.0f;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const float cu = CX[i] * ux + CY[i] * uy;
      const float Li = W5[i] * kInvCs2 * (CX[i] * Lx + CY[i] * Ly);
      const float leq = W5[i] * C * (1.0f + kInvCs2 * cu);
      leq_sum += leq;
      push(PL, i, l[i] - (l[i] - leq) * itau_l + wl * Li);
    }
    dst[(PL + 0) * N + n] = l[0] - (l[0] - (C - leq_sum)) * itau_l;
  }

  // 6. the time-level state
  if (valid) {
    A.p_new[n] = pn;
    A.u_new[n] = ux;
    A.u_new[N + n] = uy;
    A.fs[n] = fs;
    A.phiP[n] = phi;
    A.CP[n] = C;
  }
  // phase-field source budget: sum of phi div u over the tile, FP64
  const double s = block_sum<NT>(valid ? (double)phi * (double)D : 0.0, s_red);
  if (tid == 0) A.mpc_part[tile] += s;
}

__global__ __launch_bounds__(256) void k_init2d(KParams P, const double* __restrict__ phi_in,
                                                const double* __restrict__ T_in,
                                                const double* __restrict__ C_in,
                                                float* __restrict__ pop, StateArgs S) {
  const long N = P.N;
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < N;
       n += (long)gridDim.x * blockDim.x) {
    const float phi = (float)phi_in[n], T = (float)T_in[n], C = (float)C_in[n];
    const float psi = clamp01(0.5f * (1.0f + phi));
    const float rcl = psi * P.rc_l + (1.0f - psi) * P.rc_g;
    const float E = rcl * T + psi * P.rho_l_latent;
    float h0 = E, f0 = phi, l0 = C;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      pop[(PH + i) * N + n] = W5[i] * P.rhoc_ref * T;
      pop[(PF + i) * N + n] = W5[i] * phi;
      pop[(PL + i) * N + n] = W5[i] * C;
      h0 -= W5[i] * P.rhoc_ref * T;
      f0 -= W5[i] * phi;
      l0 -= W5[i] * C;
    }
    pop[(PH + 0) * N + n] = h0;
    pop[(PF + 0) * N + n] = f0;
    pop[(PL + 0) * N + n] = l0;
#pragma unroll
    for (int i = 0; i < 9; ++i) pop[(PG + i) * N + n] = 0.0f;
    S.pA[n] = 0.f;
    S.pB[n] = 0.f;
    S.uA[n] = S.uA[N + n] = 0.f;
    S.uB[n] = S.uB[N + n] = 0.f;
    S.fs[n] = 0.f;
    S.phiP[n] = 0.f;
    S.CP[n] = 0.f;
  }
}

}  // namespace

int tiles2d(int nx, int ny, int* nbx, int* nby) {
  *nbx = (nx + TX - 1) / TX;
  *nby = (ny + TY - 1) / TY;
  return (*nbx) * (*nby);
}

hipError_t launch_init2d(const KParams& P, const double* phi, const double* T, const double* C,
                         float* pop, const StateArgs& S, hipStream_t st) {
  const int blocks = (int)std::min<long>((P.N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_init2d, dim3(blocks), dim3(256), 0, st, P, phi, T, C, pop, S);
  return hipGetLastError();
}

hipError_t launch_step2d(const KParams& P, const Step2DArgs& A, bool dry, hipStream_t st) {
  if (dry)
    hipLaunchKernelGGL(k_step2d<true>, dim3(P.nblk), dim3(NT), 0, st, P, A);
  else
    hipLaunchKernelGGL(k_step2d<false>, dim3(P.nblk), dim3(NT), 0, st, P, A);
  return hipGetLastError();
}

}  // namespace lbfz
