// lbfz_api.hip -- the C ABI declared in include/lbfz.h: parameter checks,
// workspace layout, launches on the caller's stream, FP64 fixed-order
// reductions for the conservation totals.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbfz.h"
#include "lbfz_common.hpp"
#include "lbfz_handle.hpp"
#include "lbfz_kernels.hpp"

using namespace lbfz;


namespace {

struct Layout {
  size_t pop, p, u, scal, mpc, tot, red, stage, mask, total;
  int np, nscal;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Elements between consecutive planes of a population or velocity array: the
// node count rounded up to 64 plus a skew of 4 KiB + 256 B, so that the planes
// of one node do not all start on the same HBM channel and bank.
constexpr size_t kPlanePad = 1088;
size_t plane_stride(size_t N) { return ((N + 63) / 64) * 64 + kPlanePad; }

bool valid_params(const lbfz_params* p) {
  if (!p) return false;
  if (p->dim != 2 && p->dim != 3) return false;
  if (p->nx < 2 || p->ny < 2) return false;
  if (p->dim == 2 && p->nz != 1) return false;
  if (p->dim == 3 && p->nz < 2) return false;
  if ((long long)p->nx * p->ny * p->nz > (1ll << 26)) return false;
  // Every global access goes through a buffer descriptor with a 32-bit byte
  // range and 32-bit offsets; the widest one spans a whole population set
  // (the flow set: 19 planes of 4 bytes in 3D FP32, 18 of 2 bytes in 3D
  // 16-bit storage, 9 of 4 bytes in 2D) plus the set's leading pad, so that
  // span must stay below 2^32 bytes.
  {
    const long long N = (long long)p->nx * p->ny * p->nz;
    const long long ps = (long long)plane_stride((size_t)N);
    const long long widest =
        p->dim == 3 ? (p->storage == LBFZ_STORE_F32 ? 19 * 4 : 18 * 2) : 9 * 4;
    if (widest * ps + 4096 >= (1ll << 32)) return false;
  }
  if (!(p->tau_phi > 0.5 && p->tau_h > 0.5 && p->tau_c > 0.5 && p->nu > 0.0)) return false;
  if (!(p->eps > 0.0 && p->rhoc_ref > 0.0)) return false;
  if (!(p->rho_l > 0 && p->rho_g > 0 && p->rho_s > 0)) return false;
  if (!(p->cp_l > 0 && p->cp_s > 0 && p->cp_g > 0)) return false;
  if (p->contact_angle_deg != 90) return false;
  if (p->walls != 0 && p->walls != 1) return false;
  if (p->surface_tension_mode != 0 && p->surface_tension_mode != 1) return false;
  if (!(p->k_p > 0.0 && p->Ds_over_Dl >= 0.0)) return false;
  return true;
}

int check_support(const lbfz_params* p) {
  if (!p) return LBFZ_OK;
  if (p->storage != LBFZ_STORE_F32 && p->storage != LBFZ_STORE_F16 &&
      p->storage != LBFZ_STORE_BF16)
    return LBFZ_EINVAL;
  return LBFZ_OK;
}

int npop_of(const lbfz_params* p) { return p->dim == 3 ? 40 : 24; }

int tiles_of(const lbfz_params* p, int* nbx, int* nby, int* nbz) {
  if (p->dim == 3) return tiles3d(p->nx, p->ny, p->nz, p->storage, nbx, nby, nbz);
  *nbz = 1;
  return tiles2d(p->nx, p->ny, nbx, nby);
}

Layout layout(const lbfz_params* p, int ntiles, int npop) {
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  const size_t ps = plane_stride(N);
  Layout L;
  const bool narrow = p->storage != LBFZ_STORE_F32;
  L.pop = align256(p->dim == 2 ? pop_bytes2d(p->storage, ps) : pop_bytes3d(p->storage, ps));
  L.p = align256(ps * sizeof(float));
  L.u = align256(ps * p->dim * sizeof(float));
  L.scal = align256(ps * sizeof(float));
  L.np = narrow ? 3 : 2;
  // 2D: fs, phi x2, C x2, T x2 (16-bit) | fs, phi, C (FP32); 3D: two levels of
  // the five closure-field planes
  L.nscal = p->dim == 3 ? 10 : (narrow ? 7 : 3);
  L.mpc = align256((size_t)ntiles * sizeof(double));
  L.tot = align256((size_t)ntiles * 8 * sizeof(double));
  L.red = 256;
  L.stage = align256(std::max(N * LBFZ_NFIELDS * sizeof(float), N * 3 * sizeof(double)));
  if (narrow) L.stage = std::max(L.stage, align256(N * npop * sizeof(float)));
  L.mask = p->dim == 3 ? align256(N) : 0;
  L.total = 2 * L.pop + L.np * L.p + 2 * L.u + L.nscal * L.scal + L.mpc + L.tot + L.red +
            L.stage + L.mask;
  return L;
}

KParams make_kparams(const lbfz_params* p, int nbx, int nby, int nbz) {
  KParams k;
  std::memset(&k, 0, sizeof(k));
  k.nx = p->nx;
  k.ny = p->ny;
  k.nz = p->nz;
  k.N = p->nx * p->ny * p->nz;
  k.ps = (int)plane_stride((size_t)k.N);
  k.walls = p->walls;
  k.tlo_dir = p->t_lo_dirichlet;
  k.thi_dir = p->t_hi_dirichlet;
  k.st_mode = p->surface_tension_mode;
  k.nblk_x = nbx;
  k.nblk_y = nby;
  k.nblk_z = nbz;
  k.nblk = nbx * nby * nbz;
  k.rho_l = (float)p->rho_l;
  k.rho_g = (float)p->rho_g;
  k.rho_s = (float)p->rho_s;
  k.cp_l = (float)p->cp_l;
  k.cp_s = (float)p->cp_s;
  k.cp_g = (float)p->cp_g;
  k.rc_l = (float)(p->rho_l * p->cp_l);
  k.rc_s = (float)(p->rho_s * p->cp_s);
  k.rc_g = (float)(p->rho_g * p->cp_g);
  k.rhoc_ref = (float)p->rhoc_ref;
  k.rho_l_latent = (float)(p->rho_l * p->latent);
  k.T_sol = (float)p->T_sol;
  k.T_liq = (float)p->T_liq;
  k.ratio = (float)(1.0 - p->rho_s / p->rho_l);
  const double cs2 = 1.0 / 3.0;
  const double tau_g = p->nu / cs2 + 0.5;
  k.tau_gp = (float)(tau_g - 0.5);
  k.itau_g = (float)(1.0 / tau_g);
  k.wg = (float)(1.0 - 0.5 / tau_g);
  k.itau_f = (float)(1.0 / p->tau_phi);
  k.wf = (float)(1.0 - 0.5 / p->tau_phi);
  const double tau_a = p->tau_h, tau_s = tau_a / (2.0 * tau_a - 1.0);  // 1/ts + 1/ta = 2
  k.itau_a = (float)(1.0 / tau_a);
  k.itau_s = (float)(1.0 / tau_s);
  k.ws = (float)(1.0 - 0.5 / tau_s);
  const double Dl = cs2 * (p->tau_c - 0.5);
  k.Dl = (float)Dl;
  k.Ds = (float)(p->Ds_over_Dl * Dl);
  k.k_p = (float)p->k_p;
  k.alpha = (float)(3.0 * std::sqrt(2.0) * p->eps / 4.0);
  k.ieps2 = (float)(1.0 / (p->eps * p->eps));
  k.isq = (float)(1.0 / (std::sqrt(2.0) * p->eps));
  k.sigma0 = (float)p->sigma0;
  k.sigma_T = (float)p->sigma_T;
  k.sigma_c = (float)p->sigma_c;
  k.T_ref = (float)p->T_ref;
  k.c_ref = (float)p->c_ref;
  k.bfx = (float)p->body_force[0];
  k.bfy = (float)p->body_force[1];
  k.bfz = (float)p->body_force[2];
  k.T_lo = (float)p->T_lo;
  k.T_hi = (float)p->T_hi;
  k.T_lo_amp = (float)p->T_lo_amp;
  k.kwall = (float)(2.0 * M_PI / p->nx);
  return k;
}

__global__ void k_zero_f64(double* a, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    a[i] = 0.0;
}

// Fixed-order FP64 reduction of the per-tile totals (6 values) and the
// per-tile phase-field source accumulators into out[0..6].
__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ tot,
                                                const double* __restrict__ mpc, int ntiles,
                                                double* __restrict__ out) {
  __shared__ double sm[256];
  for (int k = 0; k < 7; ++k) {
    double s = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += 256) s += k < 6 ? tot[(long)t * 8 + k] : mpc[t];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sm[0];
    __syncthreads();
  }
}

#define HIPCHK(x)                        \
  do {                                   \
    if ((x) != hipSuccess) return LBFZ_EHIP; \
  } while (0)

}  // namespace

namespace lbfz {

hipError_t launch_step(lbfz_handle* h, const StepArgs& a, bool dry) {
  if (h->prm.dim == 3) return launch_step3d(h->kp, h->storage, a, dry, h->stream);
  return launch_step2d(h->kp, h->storage, a, dry, h->stream);
}

// Buffers of the next step from the current level.  16-bit storage: the
// pressure of step s is written to p[s % 3], so the step reads p[(s + 2) % 3]
// (previous level) and decodes g with p[(s + 1) % 3] (two levels back).
StepArgs base_args(lbfz_handle* h) {
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  const int c = h->cur;
  a.src = h->pop[c];
  a.dst = h->pop[1 - c];
  if (h->narrow) {
    const int s3 = (int)(h->step % 3);
    a.p_new = h->p[s3];
    a.p_old = h->p[(s3 + 2) % 3];
    a.p_ref = h->p[(s3 + 1) % 3];
    a.T_old = h->T[c];
    a.T_new = h->T[1 - c];
  } else {
    a.p_old = h->p[c];
    a.p_new = h->p[1 - c];
  }
  a.u_old = h->u[c];
  a.u_new = h->u[1 - c];
  if (h->prm.dim == 3) {
    a.cf_old = h->cf[c];
    a.cf_new = h->cf[1 - c];
  } else {
    a.fs = h->fs;
    a.phiP_old = h->phiP[c];
    a.phiP_new = h->phiP[1 - c];
    a.CP_old = h->CP[c];
    a.CP_new = h->CP[1 - c];
  }
  a.mask = h->mask;
  a.mpc_part = h->mpc_part;
  a.rev = (int)(h->step & 1);
  return a;
}

}  // namespace lbfz

extern "C" {

int lbfz_workspace_bytes(const lbfz_params* p, size_t* bytes) {
  if (!bytes || !valid_params(p)) return LBFZ_EINVAL;
  const int sup = check_support(p);
  if (sup != LBFZ_OK) return sup;
  int nbx, nby, nbz;
  const int nt = tiles_of(p, &nbx, &nby, &nbz);
  *bytes = layout(p, nt, npop_of(p)).total;
  return LBFZ_OK;
}

int lbfz_create(const lbfz_params* p, const double* phi, const double* T, const double* C,
                const uint8_t* mask, void* d_workspace, size_t ws_bytes, void* stream,
                lbfz_handle** out) {
  if (!out) return LBFZ_EINVAL;
  *out = nullptr;
  const int sup = check_support(p);
  if (sup != LBFZ_OK) return sup;
  if (!valid_params(p) || !phi || !T || !C || !d_workspace) return LBFZ_EINVAL;
  if (mask && p->dim == 2) return LBFZ_EINVAL;
  if (((uintptr_t)d_workspace & 255) != 0) return LBFZ_ENOMEM;
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  for (size_t n = 0; n < N; ++n)
    if (!std::isfinite(phi[n]) || !std::isfinite(T[n]) || !std::isfinite(C[n]))
      return LBFZ_ENONFINITE;
  int nbx, nby, nbz;
  const int ntiles = tiles_of(p, &nbx, &nby, &nbz);
  const int npop = npop_of(p);
  const Layout L = layout(p, ntiles, npop);
  if (ws_bytes < L.total) return LBFZ_ENOMEM;

  lbfz_handle* h = new (std::nothrow) lbfz_handle;
  if (!h) return LBFZ_ENOMEM;
  std::memset(h, 0, sizeof(*h));
  h->prm = *p;
  h->kp = make_kparams(p, nbx, nby, nbz);
  h->stream = (hipStream_t)stream;
  h->ws = (char*)d_workspace;
  h->ws_bytes = ws_bytes;
  h->ntiles = ntiles;
  h->npop = npop;
  h->storage = p->storage;
  h->narrow = p->storage != LBFZ_STORE_F32;
  char* q = h->ws;
  h->pop[0] = (float*)q; q += L.pop;
  h->pop[1] = (float*)q; q += L.pop;
  for (int k = 0; k < L.np; ++k) {
    h->p[k] = (float*)q;
    q += L.p;
  }
  h->u[0] = (float*)q; q += L.u;
  h->u[1] = (float*)q; q += L.u;
  const size_t ps = (size_t)h->kp.ps;
  if (p->dim == 3) {
    h->cf[0] = (float*)q;
    h->cf[1] = h->cf[0] + 5 * ps;
    q += 10 * L.scal;
  } else {
    h->fs = (float*)q; q += L.scal;
    h->phiP[0] = (float*)q; q += L.scal;
    h->CP[0] = (float*)q; q += L.scal;
    if (h->narrow) {
      h->phiP[1] = (float*)q; q += L.scal;
      h->CP[1] = (float*)q; q += L.scal;
      h->T[0] = (float*)q; q += L.scal;
      h->T[1] = (float*)q; q += L.scal;
    } else {
      h->phiP[1] = h->phiP[0];
      h->CP[1] = h->CP[0];
    }
  }
  h->mpc_part = (double*)q; q += L.mpc;
  h->tot_part = (double*)q; q += L.tot;
  h->red = (double*)q; q += L.red;
  h->stage = (float*)q; q += L.stage;
  h->mask = p->dim == 3 && mask ? (uint8_t*)q : nullptr;
  q += L.mask;
  h->cur = 0;
  h->step = 0;

  double* st = (double*)h->stage;
  int rc = LBFZ_OK;
  do {
    if (hipMemcpyAsync(st, phi, N * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(st + N, T, N * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess ||
        hipMemcpyAsync(st + 2 * N, C, N * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
            hipSuccess) {
      rc = LBFZ_EHIP;
      break;
    }
    StateArgs S{h->p[0], h->p[1], h->narrow ? h->p[2] : nullptr, h->u[0], h->u[1], h->fs,
                h->phiP[0], h->CP[0], h->narrow ? h->T[0] : nullptr, nullptr};
    if (p->dim == 3) {  // previous-level closure fields: phi, T, C, f_s, div u
      S.phiA = h->cf[0];
      S.TA = h->cf[0] + ps;
      S.CA = h->cf[0] + 2 * ps;
      S.fs = h->cf[0] + 3 * ps;
      S.DA = h->cf[0] + 4 * ps;
    }
    if (h->mask &&
        hipMemcpyAsync(h->mask, mask, N, hipMemcpyHostToDevice, h->stream) != hipSuccess) {
      rc = LBFZ_EHIP;
      break;
    }
    const hipError_t e = p->dim == 3 ? launch_init3d(h->kp, h->storage, st, st + N, st + 2 * N,
                                                     h->mask, h->pop[0], h->pop[1], S, h->stream)
                                     : launch_init2d(h->kp, h->storage, st, st + N, st + 2 * N,
                                                     h->pop[0], S, h->stream);
    if (e != hipSuccess) {
      rc = LBFZ_EHIP;
      break;
    }
    hipLaunchKernelGGL(k_zero_f64, dim3(64), dim3(256), 0, h->stream, h->mpc_part, ntiles);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
      rc = LBFZ_EHIP;
  } while (0);
  if (rc != LBFZ_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return LBFZ_OK;
}

int lbfz_step(lbfz_handle* h, int64_t nsteps) {
  if (!h || nsteps < 0) return LBFZ_EINVAL;
  for (int64_t k = 0; k < nsteps; ++k) {
    StepArgs a = base_args(h);
    HIPCHK(launch_step(h, a, false));
    h->cur ^= 1;
    h->step += 1;
  }
  return LBFZ_OK;
}

int lbfz_fields(lbfz_handle* h, uint32_t field_mask, float* const* dst, int dst_is_device) {
  if (!h || !dst) return LBFZ_EINVAL;
  const size_t N = (size_t)h->kp.N;
  StepArgs a = base_args(h);
  for (int k = 0; k < LBFZ_NFIELDS; ++k) {
    a.out[k] = nullptr;
    if (field_mask & (1u << k)) {
      if (!dst[k]) return LBFZ_EINVAL;
      a.out[k] = dst_is_device ? dst[k] : h->stage + (size_t)k * N;
    }
  }
  HIPCHK(launch_step(h, a, true));
  if (!dst_is_device) {
    for (int k = 0; k < LBFZ_NFIELDS; ++k)
      if (field_mask & (1u << k))
        HIPCHK(hipMemcpyAsync(dst[k], h->stage + (size_t)k * N, N * sizeof(float),
                              hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  return LBFZ_OK;
}

int lbfz_totals(lbfz_handle* h, lbfz_totals_t* out) {
  if (!h || !out) return LBFZ_EINVAL;
  StepArgs a = base_args(h);
  for (int k = 0; k < LBFZ_NFIELDS; ++k) a.out[k] = nullptr;
  a.tot_part = h->tot_part;
  HIPCHK(launch_step(h, a, true));
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, h->stream, h->tot_part, h->mpc_part,
                     h->ntiles, h->red);
  HIPCHK(hipGetLastError());
  double r[8];
  HIPCHK(hipMemcpyAsync(r, h->red, 7 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  out->sum_f = r[0];
  out->sum_l = r[1];
  out->sum_h = r[2];
  out->vol_solid = r[3];
  out->vol_sl = r[4];
  out->nonfinite = (int64_t)std::llround(r[5]);
  out->mpc = r[6];
  out->step = h->step;
  return LBFZ_OK;
}

namespace {
// Device planes of the exported state, in the documented order.  16-bit
// storage: the population planes are the FP32 decode in the stage buffer.
int state_planes(lbfz_handle* h, std::vector<float*>& planes) {
  const size_t ps = (size_t)h->kp.ps, N = (size_t)h->kp.N;
  planes.clear();
  if (h->narrow) {
    for (int q = 0; q < h->npop; ++q) planes.push_back(h->stage + q * N);
  } else {
    float* pop = h->pop[h->cur];
    // 2D planes of a direction with an x component are stored shifted by
    // -c_x (direction order as documented for the state layout)
    static const int kCx9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    for (int q = 0; q < h->npop; ++q) {
      int cx = 0;
      if (h->prm.dim == 2) {
        const int i = q < 5 ? q : (q < 14 ? q - 5 : (q < 19 ? q - 14 : q - 19));
        cx = kXS * kCx9[i];
      }
      planes.push_back(pop + q * ps - cx);
    }
  }
  float* cf = h->cf[h->cur];
  planes.push_back(h->prm.dim == 3 ? cf + 3 * ps : h->fs);
  planes.push_back(h->narrow ? h->p[(h->step + 2) % 3] : h->p[h->cur]);
  for (int a = 0; a < h->prm.dim; ++a) planes.push_back(h->u[h->cur] + a * ps);
  planes.push_back(h->prm.dim == 3 ? cf : h->phiP[h->cur]);
  planes.push_back(h->prm.dim == 3 ? cf + 2 * ps : h->CP[h->cur]);
  return (int)planes.size();
}
}  // namespace

int lbfz_state_floats(lbfz_handle* h, size_t* nfloats) {
  if (!h || !nfloats) return LBFZ_EINVAL;
  std::vector<float*> planes;
  *nfloats = (size_t)state_planes(h, planes) * (size_t)h->kp.N;
  return LBFZ_OK;
}

int lbfz_get_state(lbfz_handle* h, float* host_dst) {
  if (!h || !host_dst) return LBFZ_EINVAL;
  const size_t N = (size_t)h->kp.N;
  std::vector<float*> planes;
  const int np = state_planes(h, planes);
  if (h->narrow)
    HIPCHK(h->prm.dim == 3
               ? launch_export3d(h->kp, h->storage, base_args(h), h->stage, h->stream)
               : launch_export2d(h->kp, h->storage, base_args(h), h->stage, h->stream));
  for (int k = 0; k < np; ++k)
    HIPCHK(hipMemcpyAsync(host_dst + k * N, planes[k], N * sizeof(float), hipMemcpyDeviceToHost,
                          h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBFZ_OK;
}

namespace {
// 16-bit storage: encode the raw state planes (stage buffer and previous-level
// planes) into the populations, against the imported phi, C and p (p doubles
// as the g reference).  Asynchronous.
int import_narrow(lbfz_handle* h) {
  const size_t N = (size_t)h->kp.N;
  StepArgs a = base_args(h);
  HIPCHK(hipMemcpyAsync((void*)a.p_ref, a.p_old, N * sizeof(float), hipMemcpyDeviceToDevice,
                        h->stream));
  a.dst = h->pop[h->cur];
  if (h->prm.dim == 3) {
    HIPCHK(launch_import3d(h->kp, h->storage, a, h->stage, h->stream));
  } else {
    a.T_new = h->T[h->cur];
    HIPCHK(launch_import2d(h->kp, h->storage, a, h->stage, h->stream));
  }
  return LBFZ_OK;
}
}  // namespace

int lbfz_set_state(lbfz_handle* h, const float* host_src) {
  if (!h || !host_src) return LBFZ_EINVAL;
  const size_t N = (size_t)h->kp.N;
  std::vector<float*> planes;
  const int np = state_planes(h, planes);
  for (int k = 0; k < np; ++k)
    HIPCHK(hipMemcpyAsync(planes[k], host_src + k * N, N * sizeof(float), hipMemcpyHostToDevice,
                          h->stream));
  if (h->narrow) {
    const int rc = import_narrow(h);
    if (rc != LBFZ_OK) return rc;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return LBFZ_OK;
}

}  // extern "C"

namespace lbfz {
int restart_job(lbfz_handle* h, const float* const* d_fields, EquilJob* job) {
  if (!h || !d_fields || !job) return LBFZ_EINVAL;
  for (int k = 0; k < 7; ++k)
    if (!d_fields[k]) return LBFZ_EINVAL;
  if (h->prm.dim != 2 || h->narrow) return LBFZ_EUNSUPPORTED;
  std::vector<float*> planes;
  if (state_planes(h, planes) != 30) return LBFZ_EUNSUPPORTED;
  job->P = h->kp;
  job->F = EquilFields{d_fields[0], d_fields[1], d_fields[2], d_fields[3],
                       d_fields[4], d_fields[5], d_fields[6]};
  for (int k = 0; k < 30; ++k) job->S.p[k] = planes[k];
  return LBFZ_OK;
}
}  // namespace lbfz

extern "C" {

int lbfz_restart_fields(lbfz_handle* h, const float* const* d_fields) {
  if (!h || !d_fields) return LBFZ_EINVAL;
  for (int k = 0; k < 7; ++k)
    if (!d_fields[k]) return LBFZ_EINVAL;
  if (h->prm.dim != 2) return LBFZ_EUNSUPPORTED;
  std::vector<float*> planes;
  if (state_planes(h, planes) != 30) return LBFZ_EUNSUPPORTED;
  EquilFields F{d_fields[0], d_fields[1], d_fields[2], d_fields[3],
                d_fields[4], d_fields[5], d_fields[6]};
  StatePlanes S;
  for (int k = 0; k < 30; ++k) S.p[k] = planes[k];
  HIPCHK(launch_equil2d(h->kp, F, S, h->stream));
  if (h->narrow) return import_narrow(h);
  return LBFZ_OK;
}

int lbfz_sync(lbfz_handle* h) {
  if (!h) return LBFZ_EINVAL;
  return hipStreamSynchronize(h->stream) == hipSuccess ? LBFZ_OK : LBFZ_EHIP;
}

void lbfz_destroy(lbfz_handle* h) { delete h; }

const char* lbfz_strerror(int code) {
  switch (code) {
    case LBFZ_OK: return "ok";
    case LBFZ_EINVAL: return "invalid argument or parameter";
    case LBFZ_ENOMEM: return "device workspace too small or misaligned";
    case LBFZ_EHIP: return "HIP runtime error";
    case LBFZ_ENONFINITE: return "non-finite input field";
    case LBFZ_EUNSUPPORTED: return "configuration not supported by this library";
    default: return "unknown error";
  }
}

}  // extern "C"
