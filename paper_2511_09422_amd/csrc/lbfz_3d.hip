// lbfz_3d.hip -- fused 3D step of the coupled LB freezing scheme
// (arXiv 2511.09422, Sec. 3) for gfx950: D3Q19 flow g, D3Q7 phase field f,
// enthalpy h (TRT) and solute l, walls on z, periodic x and y, optional
// obstacle mask (bounce-back for f, g, l; h conducts through it).
//
// Populations: two SoA buffers of 40 planes (f 0..6, g 7..25, h 26..32,
// l 33..39), push streaming from A into B.  With D3Q7 weights (0, 1/6 x 6)
// the rest components of f and l are identically zero and are never read or
// written.
//
// Each block owns a 32x8 xy tile and marches up a segment of z planes,
// keeping rolling LDS windows of three planes of the previous velocity (xy
// ring 2, for div u of the closure ring) and three planes of the closure
// fields phi, T, C, f_s and the previous pressure (xy ring 1).  Per plane:
// load velocity plane k+2, close plane k+1, collide plane k.  The closure of
// a node is evaluated once per segment (plus the xy ring and two planes at
// the segment ends), every population is read once and written once.
#include "lbfz_common.hpp"
#include "lbfz_kernels.hpp"

namespace lbfz {

namespace {

constexpr int TX = 32, TY = 8, NT = TX * TY;
constexpr int HX = TX + 2, HY = TY + 2;  // closure ring
constexpr int UX = TX + 4, UY = TY + 4;  // velocity ring
constexpr int HS = HX * HY, US = UX * UY;
constexpr int NF = 8;                    // phi, T, C, f_s, p, div u, E, Q

constexpr int PF = 0, PG = 7, PH = 26, PL = 33;

// D3Q19; the first seven are D3Q7
constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
constexpr float W19[19] = {1.f / 3,  1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18, 1.f / 18,
                           1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36,
                           1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
constexpr float W7 = 1.f / 6;

__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ __forceinline__ int wrapm(int v, int n) { return ((v % n) + n) % n; }

struct LDS3 {
  float u[3][3][US];      // [plane slot][component][uy*UX+ux]
  uint8_t mk[3][US];      // obstacle mask on the velocity ring
  float c[3][NF][HS];     // [plane slot][field][hy*HX+hx]
  uint8_t cm[3][HS];      // obstacle mask on the closure ring
  double red[NT / 64];
};

// Map plane index k to a stored plane (walls on z: mirror, flagged ghost).
__device__ __forceinline__ int map_plane(const KParams& P, int k, int& ghost) {
  ghost = 0;
  if (P.walls) {
    if (k < 0) {
      ghost = -1;
      k = -1 - k;
    } else if (k >= P.nz) {
      ghost = 1;
      k = 2 * P.nz - 1 - k;
    }
    return min(max(k, 0), P.nz - 1);
  }
  return wrapm(k, P.nz);
}

// Stage velocity plane k (tile + 2 ring) and its mask into slot k % 3.
__device__ __forceinline__ void load_u_plane(const KParams& P, const StepArgs& A, LDS3& S, int x0,
                                             int y0, int k) {
  const long N = P.N, PS = P.ps;
  int ghost;
  const int kz = map_plane(P, k, ghost);
  const int slot = wrapm(k, 3);
  const float sg = ghost ? -1.0f : 1.0f;
  for (int s = threadIdx.x; s < US; s += NT) {
    const int lx = s % UX, ly = s / UX;
    const int gx = wrapm(x0 + lx - 2, P.nx), gy = wrapm(y0 + ly - 2, P.ny);
    const long n = ((long)kz * P.ny + gy) * P.nx + gx;
    const uint8_t m = A.mask ? A.mask[n] : (uint8_t)0;
    S.mk[slot][s] = ghost ? (uint8_t)0 : m;
    S.u[slot][0][s] = sg * A.u_old[n];
    S.u[slot][1][s] = sg * A.u_old[PS + n];
    S.u[slot][2][s] = sg * A.u_old[2 * PS + n];
  }
}

// Closure of plane k (tile + 1 ring) into slot k % 3.  Ghost planes beyond a
// wall copy the adjacent plane (already closed) with the wall rule for T.
__device__ __forceinline__ void close_plane(const KParams& P, const StepArgs& A, LDS3& S, int x0,
                                            int y0, int k) {
  const long N = P.N, PS = P.ps;
  const int slot = wrapm(k, 3);
  int ghost;
  const int kz = map_plane(P, k, ghost);
  if (ghost) {
    const int src = wrapm(ghost < 0 ? k + 1 : k - 1, 3);
    for (int s = threadIdx.x; s < HS; s += NT) {
      const int lx = s % HX;
      const int gx = wrapm(x0 + lx - 1, P.nx);
#pragma unroll
      for (int f = 0; f < NF; ++f) S.c[slot][f][s] = S.c[src][f][s];
      S.cm[slot][s] = 0;
      float T = S.c[src][1][s];
      if (ghost < 0 && P.tlo_dir) T = 2.0f * (P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)gx)) - T;
      if (ghost > 0 && P.thi_dir) T = 2.0f * P.T_hi - T;
      S.c[slot][1][s] = T;
    }
    return;
  }
  const int um = wrapm(k - 1, 3), u0 = slot, up = wrapm(k + 1, 3);
  for (int s = threadIdx.x; s < HS; s += NT) {
    const int lx = s % HX, ly = s / HX;
    const int gx = wrapm(x0 + lx - 1, P.nx), gy = wrapm(y0 + ly - 1, P.ny);
    const long n = ((long)kz * P.ny + gy) * P.nx + gx;
    const int us = (ly + 1) * UX + (lx + 1);  // velocity-ring index of this node
    float phi0 = 0.f, E0 = 0.f, C = 0.f;
#pragma unroll
    for (int i = 1; i < 7; ++i) {
      phi0 += A.src[(PF + i) * PS + n];
      C += A.src[(PL + i) * PS + n];
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) E0 += A.src[(PH + i) * PS + n];
    S.cm[slot][s] = S.mk[u0][us];
    if (S.mk[u0][us]) {
      float T, fs;
      enthalpy_map(P, E0, 0.0f, T, fs);
      S.c[slot][0][s] = -1.0f;
      S.c[slot][1][s] = T;
      S.c[slot][2][s] = 0.0f;
      S.c[slot][3][s] = 0.0f;
      S.c[slot][4][s] = 0.0f;
      S.c[slot][5][s] = 0.0f;
      S.c[slot][6][s] = E0;
      S.c[slot][7][s] = 0.0f;
      continue;
    }
    // div u^{n-1}: D3Q19 isotropic gradient, obstacle neighbours give -u(centre)
    float D = 0.0f;
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      const int pl = CZ[i] < 0 ? um : (CZ[i] > 0 ? up : u0);
      const int t = us + CY[i] * UX + CX[i];
      const bool ob = S.mk[pl][t] != 0;
      float v = 0.0f;
      if (CX[i]) v += CX[i] * (ob ? -S.u[u0][0][us] : S.u[pl][0][t]);
      if (CY[i]) v += CY[i] * (ob ? -S.u[u0][1][us] : S.u[pl][1][t]);
      if (CZ[i]) v += CZ[i] * (ob ? -S.u[u0][2][us] : S.u[pl][2][t]);
      D += W19[i] * v;
    }
    D *= kInvCs2;
    const Closure cl = closure(P, phi0, E0, D);
    S.c[slot][0][s] = cl.phi;
    S.c[slot][1][s] = cl.T;
    S.c[slot][2][s] = C;
    S.c[slot][3][s] = cl.fs;
    S.c[slot][4][s] = A.p_old[n];
    S.c[slot][5][s] = D;
    S.c[slot][6][s] = cl.E;
    S.c[slot][7][s] = cl.Q;
  }
}

template <bool DRY>
__global__ __launch_bounds__(NT) void k_step3d(KParams P, StepArgs A, int seg) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  LDS3& S = *reinterpret_cast<LDS3*>(lds_raw);
  const int tiles_xy = P.nblk_x * P.nblk_y;
  const int tile = xcd_tile(blockIdx.x, P.nblk);
  const int zt = tile / tiles_xy, rxy = tile % tiles_xy;
  const int x0 = (rxy % P.nblk_x) * TX, y0 = (rxy / P.nblk_x) * TY;
  const int z0 = zt * seg, z1 = min(z0 + seg, P.nz);
  const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool inxy = gx < P.nx && gy < P.ny;
  const long N = P.N, PS = P.ps;
  const int nx = P.nx, ny = P.ny, nz = P.nz;

  // prologue: closure planes z0-1 and z0 (velocity planes z0-2 .. z0+1)
  load_u_plane(P, A, S, x0, y0, z0 - 1);
  load_u_plane(P, A, S, x0, y0, z0);
  load_u_plane(P, A, S, x0, y0, z0 + 1);
  __syncthreads();
  int gh;
  map_plane(P, z0 - 1, gh);
  if (gh) {
    close_plane(P, A, S, x0, y0, z0);
    __syncthreads();
    close_plane(P, A, S, x0, y0, z0 - 1);
  } else {
    close_plane(P, A, S, x0, y0, z0);
    __syncthreads();
    load_u_plane(P, A, S, x0, y0, z0 - 2);  // slot of z0+1, restored below
    __syncthreads();
    close_plane(P, A, S, x0, y0, z0 - 1);
    __syncthreads();
    load_u_plane(P, A, S, x0, y0, z0 + 1);
  }
  __syncthreads();

  double mpc_acc = 0.0;
  double tot[6] = {0, 0, 0, 0, 0, 0};
  const int cs = (ty + 1) * HX + (tx + 1);  // closure-ring index of the own node
  const int us = (ty + 2) * UX + (tx + 2);  // velocity-ring index of the own node

  for (int k = z0; k < z1; ++k) {
    // A. velocity plane k+2, B. closure of plane k+1
    load_u_plane(P, A, S, x0, y0, k + 2);
    __syncthreads();
    close_plane(P, A, S, x0, y0, k + 1);
    __syncthreads();
    // C. collide plane k
    const int sm = wrapm(k - 1, 3), s0 = wrapm(k, 3), sp = wrapm(k + 1, 3);
    const bool valid = inxy;
    const long n = ((long)k * ny + (inxy ? gy : 0)) * nx + (inxy ? gx : 0);
    const bool ob = S.cm[s0][cs] != 0;
    if (valid) {
      // stencil neighbour value with the obstacle rule (kind 0 -> centre)
      // obstacle neighbours as a bit set (bit i for link i), so the stencils
      // below read the mask once; without a mask it stays zero
      uint32_t obm = 0;
      if (A.mask) {
#pragma unroll
        for (int i = 1; i < 19; ++i) {
          const int pl = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
          obm |= S.cm[pl][cs + CY[i] * HX + CX[i]] ? (1u << i) : 0u;
        }
      }
      auto nb = [&](int f, int i, bool kind0) -> float {
        const int pl = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
        const int t = cs + CY[i] * HX + CX[i];
        if (kind0 && (obm >> i & 1u)) return S.c[s0][f][cs];
        return S.c[pl][f][t];
      };
      const float phi = S.c[s0][0][cs], T = S.c[s0][1][cs], C = S.c[s0][2][cs];
      const float fs = S.c[s0][3][cs];
      if (ob) {
        // obstacle: enthalpy at rest without source (pure conduction)
        float h[7];
#pragma unroll
        for (int i = 0; i < 7; ++i) h[i] = A.src[(PH + i) * PS + n];
        const float E = S.c[s0][6][cs];
        float heq[7];
        heq[0] = E;
#pragma unroll
        for (int i = 1; i < 7; ++i) {
          heq[i] = W7 * P.rhoc_ref * T;
          heq[0] -= heq[i];
        }
        if (DRY) {
          float* const* o = A.out;
          if (o[0]) o[0][n] = -1.0f;
          if (o[1]) o[1][n] = 1.0f;
          if (o[2]) o[2][n] = T;
          if (o[3]) o[3][n] = 0.0f;
          if (o[4]) o[4][n] = 0.0f;
          if (o[5]) o[5][n] = 0.0f;
          if (o[6]) o[6][n] = 0.0f;
          if (o[7]) o[7][n] = 0.0f;
          if (o[8]) o[8][n] = P.rho_g;
          tot[2] += (double)h[0] + h[1] + h[2] + h[3] + h[4] + h[5] + h[6];
          float s = 0.f;
#pragma unroll
          for (int i = 0; i < 7; ++i) s += h[i];
          if (!isfinite(s)) tot[5] += 1.0;
        } else {
#pragma unroll
          for (int i = 0; i < 7; ++i) {
            const int o = OPP[i];
            const float hs = 0.5f * (h[i] + h[o]), ha = 0.5f * (h[i] - h[o]);
            const float es = 0.5f * (heq[i] + heq[o]), ea = 0.5f * (heq[i] - heq[o]);
            const float hp = h[i] - (hs - es) * P.itau_s - (ha - ea) * P.itau_a;
            const int tz = k + CZ[i];
            if (P.walls && (tz < 0 || tz >= nz)) {
              float hv = hp;
              if (tz < 0 && P.tlo_dir)
                hv = -hv + 2.0f * W7 * P.rhoc_ref * (P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)gx));
              if (tz >= nz && P.thi_dir) hv = -hv + 2.0f * W7 * P.rhoc_ref * P.T_hi;
              A.dst[(PH + o) * PS + n] = hv;
            } else {
              const long m = ((long)wrapc(tz, nz) * ny + wrapc(gy + CY[i], ny)) * nx +
                             wrapc(gx + CX[i], nx);
              A.dst[(PH + i) * PS + m] = hp;
            }
          }
          A.p_new[n] = 0.f;
          A.u_new[n] = A.u_new[PS + n] = A.u_new[2 * PS + n] = 0.f;
          A.fs[n] = 0.f;
          A.phiP_new[n] = -1.f;
          A.CP_new[n] = 0.f;
        }
      } else {
        // stencils (isotropic D3Q19 gradient / Laplacian), one field per pass so
        // that few LDS values are in flight at once
        float gp[3], gT[3], gC[3], gf[3], gP[3], lap = 0.f;
        auto grad = [&](int fld, bool kind0, float* gr) {
          float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
          for (int i = 1; i < 19; ++i) {
            const float v = nb(fld, i, kind0) * (W19[i] * kInvCs2);
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
        for (int i = 1; i < 19; ++i) lap += 2.0f * W19[i] * kInvCs2 * (nb(0, i, true) - phi);
        __builtin_amdgcn_sched_barrier(0);
        grad(1, false, gT);
        __builtin_amdgcn_sched_barrier(0);
        grad(2, true, gC);
        __builtin_amdgcn_sched_barrier(0);
        grad(3, true, gf);
        __builtin_amdgcn_sched_barrier(0);
        grad(4, true, gP);
        __builtin_amdgcn_sched_barrier(0);
        float g[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) g[i] = A.src[(PG + i) * PS + n];
        // forces, velocity, pressure (Sec. 3.2, Eq. Fs)
        float grho[3], F[3], nv[3], gsig[3];
        const float g2 = gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2];
        const float ng = sqrtf(g2);
        const float inv_ng = 1.0f / fmaxf(ng, 1e-6f);  // n regularised in the bulk
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
        const float irho = 1.0f / rho;
        float u[3], fd[3], Ft[3], Ff[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float us_ = (mom[a] + 0.5f * F[a]) * irho;
          fd[a] = -fs * us_;
          u[a] = us_ + 0.5f * fd[a];
        }
        const float fs_prev = A.fs[n];
        const float mdot = P.ratio * (fs - fs_prev);
        const float S_ = rho * mdot + u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          Ft[a] = F[a] - gP[a] + kCs2 * grho[a];
          Ff[a] = F[a] + rho * fd[a];
        }
        const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const float uFt = u[0] * Ft[0] + u[1] * Ft[1] + u[2] * Ft[2];
        // G_i (Sec. 3.2); its rest component is the complement of the moving
        // ones so that sum G = S exactly.  The moving ones are recomputed where
        // they are used, to keep no array of them live.
        auto Gi = [&](int i) -> float {
          const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
          const float cFt = CX[i] * Ft[0] + CY[i] * Ft[1] + CZ[i] * Ft[2];
          const float cFf = CX[i] * Ff[0] + CY[i] * Ff[1] + CZ[i] * Ff[2];
          return W19[i] * (S_ + kInvCs2 * cFf + 9.0f * (cu * cFt) - 3.0f * uFt);
        };
        float G0 = S_;
#pragma unroll
        for (int i = 1; i < 19; ++i) G0 -= Gi(i);
        float sum_nz = 0.f;
#pragma unroll
        for (int i = 1; i < 19; ++i) sum_nz += g[i];
        const float srest = W19[0] * (-1.5f * uu);
        const float pn =
            (kCs2 / (1.0f - W19[0])) * (sum_nz + 0.5f * S_ + P.tau_g * G0 + rho * srest);
        if (DRY) {
          float* const* o = A.out;
          if (o[0]) o[0][n] = phi;
          if (o[1]) o[1][n] = 1.0f - fs;
          if (o[2]) o[2][n] = T;
          if (o[3]) o[3][n] = C;
          if (o[4]) o[4][n] = u[0];
          if (o[5]) o[5][n] = u[1];
          if (o[6]) o[6][n] = u[2];
          if (o[7]) o[7][n] = pn;
          if (o[8]) o[8][n] = rho;
          double df = 0, dh = 0, dl = 0;
          bool bad = !isfinite(phi) || !isfinite(T) || !isfinite(pn) || !isfinite(uu);
#pragma unroll
          for (int i = 0; i < 7; ++i) {
            if (i) df += (double)A.src[(PF + i) * PS + n];
            dh += (double)A.src[(PH + i) * PS + n];
            if (i) dl += (double)A.src[(PL + i) * PS + n];
          }
          bad = bad || !isfinite(df) || !isfinite(dh) || !isfinite(dl);
          tot[0] += df;
          tot[1] += dl;
          tot[2] += dh;
          tot[3] += (double)fs;
          tot[4] += (double)clamp01(0.5f * (1.0f + phi));
          tot[5] += bad ? 1.0 : 0.0;
        } else {
          // div u, E and Q of the own node from its closure
          const float Dr = S.c[s0][5][cs];
          const float clE = S.c[s0][6][cs], clQ = S.c[s0][7][cs];
          mpc_acc += (double)phi * (double)Dr;
          // Each post-collision population is computed and pushed along its
          // link at once.  Link kinds: 0 stream to m, 1 wall (bounce-back, or
          // anti-bounce-back for h at a Dirichlet wall), 2 obstacle (bounce-back
          // for f, g, l; h streams into it).
          auto link = [&](int i, long& m) -> int {
            const int tz = k + CZ[i];
            if (P.walls && (tz < 0 || tz >= nz)) return 1;
            const int pl = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
            m = ((long)wrapc(tz, nz) * ny + wrapc(gy + CY[i], ny)) * nx + wrapc(gx + CX[i], nx);
            return S.cm[pl][cs + CY[i] * HX + CX[i]] ? 2 : 0;
          };
          // flow BGK (Sec. 3.2)
          float geq_sum = 0.f;
#pragma unroll
          for (int i = 1; i < 19; ++i) {
            const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
            const float geq = pn * kInvCs2 * W19[i] + rho * W19[i] * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
            geq_sum += geq;
            const float post = g[i] - (g[i] - geq) * P.itau_g + P.wg * Gi(i);
            long m = n;
            if (link(i, m)) A.dst[(PG + OPP[i]) * PS + n] = post;
            else A.dst[(PG + i) * PS + m] = post;
          }
          A.dst[(PG + 0) * PS + n] = g[0] - (g[0] + geq_sum) * P.itau_g + P.wg * G0;
          __builtin_amdgcn_sched_barrier(0);
          // phase field BGK (Sec. 3.1); the D3Q7 rest component is zero
          float f[7];
          f[0] = 0.f;
#pragma unroll
          for (int i = 1; i < 7; ++i) f[i] = A.src[(PF + i) * PS + n];
          const float up0 = A.u_old[n], up1 = A.u_old[PS + n], up2 = A.u_old[2 * PS + n];
          const float phiP = A.phiP_old[n], CP = A.CP_old[n];
          {
            const float cf = kCs2 * (1.0f - phi * phi) * P.isq;
            const float B0 = (phi * u[0] - phiP * up0) + cf * nv[0];
            const float B1 = (phi * u[1] - phiP * up1) + cf * nv[1];
            const float B2 = (phi * u[2] - phiP * up2) + cf * nv[2];
#pragma unroll
            for (int i = 1; i < 7; ++i) {
              const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
              const float cB = CX[i] * B0 + CY[i] * B1 + CZ[i] * B2;
              const float Fi = W7 * (kInvCs2 * cB + phi * Dr);
              const float feq = W7 * phi * (1.0f + kInvCs2 * cu);
              const float post = f[i] - (f[i] - feq) * P.itau_f + P.wf * Fi;
              long m = n;
              if (link(i, m)) A.dst[(PF + OPP[i]) * PS + n] = post;
              else A.dst[(PF + i) * PS + m] = post;
            }
          }
          __builtin_amdgcn_sched_barrier(0);
          // enthalpy TRT (Sec. 3.3)
          {
            float h[7];
#pragma unroll
            for (int i = 0; i < 7; ++i) h[i] = A.src[(PH + i) * PS + n];
            float heq[7];
            const float rT = P.rhoc_ref * T, cT = rcp * T;
            heq[0] = clE;
#pragma unroll
            for (int i = 1; i < 7; ++i) {
              const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
              heq[i] = W7 * (rT + cT * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
              heq[0] -= heq[i];
            }
            const float hq = W7 * clQ, hq0 = clQ - 6.0f * hq;
            const float Tw_lo = P.T_lo + P.T_lo_amp * cosf(P.kwall * (float)gx);
#pragma unroll
            for (int i = 0; i < 7; ++i) {
              const int o = OPP[i];
              const float hs = 0.5f * (h[i] + h[o]), ha = 0.5f * (h[i] - h[o]);
              const float es = 0.5f * (heq[i] + heq[o]), ea = 0.5f * (heq[i] - heq[o]);
              const float post = h[i] - (hs - es) * P.itau_s - (ha - ea) * P.itau_a +
                                 P.ws * (i == 0 ? hq0 : hq);
              long m = n;
              if (link(i, m) == 1) {
                float hv = post;
                const int tz = k + CZ[i];
                if (tz < 0 && P.tlo_dir) hv = -hv + 2.0f * W7 * P.rhoc_ref * Tw_lo;
                if (tz >= nz && P.thi_dir) hv = -hv + 2.0f * W7 * P.rhoc_ref * P.T_hi;
                A.dst[(PH + o) * PS + n] = hv;
              } else {
                A.dst[(PH + i) * PS + m] = post;
              }
            }
          }
          __builtin_amdgcn_sched_barrier(0);
          // solute BGK (Sec. 3.4)
          {
            float l[7];
            l[0] = 0.f;
#pragma unroll
            for (int i = 1; i < 7; ++i) l[i] = A.src[(PL + i) * PS + n];
            const float keff = 1.0f - fs * (1.0f - P.k_p);
            const float De = fs * P.k_p * P.Ds + (1.0f - fs) * P.Dl;
            const float itau_l = 1.0f / (De / (kCs2 * keff) + 0.5f), wl = 1.0f - 0.5f * itau_l;
            const float cr = (1.0f - phi) * C * P.isq, ck = (P.k_p - 1.0f) * C / keff;
            const float L0 = (C * u[0] - CP * up0) + kCs2 * (cr * nv[0] + ck * gf[0]);
            const float L1 = (C * u[1] - CP * up1) + kCs2 * (cr * nv[1] + ck * gf[1]);
            const float L2 = (C * u[2] - CP * up2) + kCs2 * (cr * nv[2] + ck * gf[2]);
#pragma unroll
            for (int i = 1; i < 7; ++i) {
              const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
              const float cL = CX[i] * L0 + CY[i] * L1 + CZ[i] * L2;
              const float leq = W7 * C * (1.0f + kInvCs2 * cu);
              const float post = l[i] - (l[i] - leq) * itau_l + wl * W7 * kInvCs2 * cL;
              long m = n;
              if (link(i, m)) A.dst[(PL + OPP[i]) * PS + n] = post;
              else A.dst[(PL + i) * PS + m] = post;
            }
          }
          A.p_new[n] = pn;
          A.u_new[n] = u[0];
          A.u_new[PS + n] = u[1];
          A.u_new[2 * PS + n] = u[2];
          A.fs[n] = fs;
          A.phiP_new[n] = phi;
          A.CP_new[n] = C;
        }
      }
    }
  }
  // per-tile FP64 reductions
  if (DRY) {
    if (A.tot_part) {
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const double s = block_sum<NT>(tot[q], S.red);
        if (tid == 0) A.tot_part[(long)tile * 8 + q] = s;
      }
    }
  } else {
    const double s = block_sum<NT>(mpc_acc, S.red);
    if (tid == 0) A.mpc_part[tile] += s;
  }
}

__global__ __launch_bounds__(256) void k_init3d(KParams P, const double* __restrict__ phi_in,
                                                const double* __restrict__ T_in,
                                                const double* __restrict__ C_in,
                                                const uint8_t* __restrict__ mask,
                                                float* __restrict__ popA,
                                                float* __restrict__ popB, StateArgs S) {
  const long N = P.N, PS = P.ps;
  for (long n = blockIdx.x * (long)blockDim.x + threadIdx.x; n < N;
       n += (long)gridDim.x * blockDim.x) {
    const bool ob = mask && mask[n];
    const float phi = ob ? -1.0f : (float)phi_in[n];
    const float T = (float)T_in[n], C = ob ? 0.0f : (float)C_in[n];
    const float psi = clamp01(0.5f * (1.0f + phi));
    const float rcl = psi * P.rc_l + (1.0f - psi) * P.rc_g;
    const float E = rcl * T + psi * P.rho_l_latent;
    float h0 = E;
#pragma unroll
    for (int i = 1; i < 7; ++i) {
      popA[(PH + i) * PS + n] = W7 * P.rhoc_ref * T;
      popA[(PF + i) * PS + n] = ob ? 0.0f : W7 * phi;
      popA[(PL + i) * PS + n] = ob ? 0.0f : W7 * C;
      h0 -= W7 * P.rhoc_ref * T;
    }
    popA[(PH + 0) * PS + n] = h0;
    popA[(PF + 0) * PS + n] = 0.0f;
    popA[(PL + 0) * PS + n] = 0.0f;
#pragma unroll
    for (int i = 0; i < 19; ++i) popA[(PG + i) * PS + n] = 0.0f;
    // the other buffer: obstacle and rest slots are never written by a step
#pragma unroll
    for (int q = 0; q < 40; ++q) popB[q * PS + n] = 0.0f;
    S.pA[n] = S.pB[n] = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) S.uA[a * PS + n] = S.uB[a * PS + n] = 0.f;
    S.fs[n] = 0.f;
    S.phiA[n] = 0.f;
    S.CA[n] = 0.f;
  }
}

}  // namespace

int tiles3d(int nx, int ny, int nz, int seg, int* nbx, int* nby, int* nbz) {
  *nbx = (nx + TX - 1) / TX;
  *nby = (ny + TY - 1) / TY;
  *nbz = (nz + seg - 1) / seg;
  return (*nbx) * (*nby) * (*nbz);
}

size_t lds3d_bytes() { return sizeof(LDS3); }

hipError_t launch_init3d(const KParams& P, const double* phi, const double* T, const double* C,
                         const uint8_t* mask, float* popA, float* popB, const StateArgs& S,
                         hipStream_t st) {
  const int blocks = (int)std::min<long>((P.N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_init3d, dim3(blocks), dim3(256), 0, st, P, phi, T, C, mask, popA, popB,
                     S);
  return hipGetLastError();
}

hipError_t launch_step3d(const KParams& P, const StepArgs& A, int seg, bool dry, hipStream_t st) {
  const size_t lds = sizeof(LDS3);
  if (dry)
    hipLaunchKernelGGL(k_step3d<true>, dim3(P.nblk), dim3(NT), lds, st, P, A, seg);
  else
    hipLaunchKernelGGL(k_step3d<false>, dim3(P.nblk), dim3(NT), lds, st, P, A, seg);
  return hipGetLastError();
}

}  // namespace lbfz
