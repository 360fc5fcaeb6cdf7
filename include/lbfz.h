/*
 * lbfz.h -- C ABI of the MI355X (gfx950) coupled lattice Boltzmann freezing
 * step: one time step of the diffuse-interface scheme of Huang, Chai, Liu,
 * Huang, "Diffuse-interface modeling and simulation of the freezing of binary
 * fluids with the Marangoni effect" (arXiv 2511.09422), Sec. 3:
 *   - conservative Allen-Cahn phase field f (BGK, D2Q5 / D3Q7), Sec. 3.1;
 *   - pressure-based flow g with the phase-change mass source (BGK,
 *     D2Q9 / D3Q19), capillary + Marangoni force (Eq. Fs) and solid drag,
 *     Sec. 3.2;
 *   - total enthalpy h (TRT, D2Q5 / D3Q7) with the enthalpy -> (T, f_l) map of
 *     Eq. (Hfl), Sec. 3.3;
 *   - constrained solute l (BGK, D2Q5 / D3Q7) with the pseudo-potential
 *     rejection flux, Sec. 3.4;
 *   - isotropic gradient / Laplacian stencils, end of Sec. 3.4;
 *   - half-way bounce-back and anti-bounce-back walls, Sec. 4.5.
 *
 * Conventions (all calls):
 *   - Lattice units, dx = dt = 1, cs^2 = 1/3.
 *   - Scalar fields are C-order [nz][ny][nx] (2D: nz = 1).  With walls != 0
 *     the last axis (y in 2D, z in 3D) is bounded by walls at -1/2 and n-1/2
 *     (cell-centred nodes); every other axis is periodic.
 *   - Device memory: the library never allocates.  The caller provides one
 *     device workspace of at least lbfz_workspace_bytes() bytes (256-byte
 *     aligned) and a HIP stream (passed as void*, NULL = default stream); the
 *     handle keeps both until lbfz_destroy.  The handle itself is host memory
 *     owned by the library.
 *   - All device work is enqueued on that stream.  lbfz_step does not
 *     synchronise; lbfz_fields (to host) and lbfz_totals synchronise it.
 *   - One handle per stream; a handle is not thread-safe.
 *   - Every int-returning call returns LBFZ_OK (0) or a negative LBFZ_E* code;
 *     nothing aborts and no C++ exception crosses the ABI.
 */
#ifndef LBFZ_H
#define LBFZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBFZ_OK = 0,
  LBFZ_EINVAL = -1,     /* bad argument or parameter (tau <= 1/2, sizes, ...) */
  LBFZ_ENOMEM = -2,     /* workspace too small or misaligned                 */
  LBFZ_EHIP = -3,       /* a HIP runtime call failed                         */
  LBFZ_ENONFINITE = -4, /* non-finite input field                            */
  LBFZ_EUNSUPPORTED = -5
};

/* Population storage of the step. */
enum { LBFZ_STORE_F32 = 0, LBFZ_STORE_F16 = 1, LBFZ_STORE_BF16 = 2 };

/* Field selector bits for lbfz_fields. */
enum {
  LBFZ_PHI = 1u << 0, /* order parameter phi (Sec. 3.1 moment)              */
  LBFZ_FL = 1u << 1,  /* liquid fraction reported as 1 - f_s                */
  LBFZ_T = 1u << 2,   /* temperature (Eq. Hfl)                              */
  LBFZ_C = 1u << 3,   /* solute concentration (Sec. 3.4 moment)             */
  LBFZ_UX = 1u << 4,  /* velocity (Sec. 3.2, corrected by the solid drag)   */
  LBFZ_UY = 1u << 5,
  LBFZ_UZ = 1u << 6,
  LBFZ_P = 1u << 7,   /* pressure (Sec. 3.2)                                */
  LBFZ_RHO = 1u << 8  /* interpolated density (end of Sec. 2)               */
};
#define LBFZ_NFIELDS 9

/* Physical and numerical parameters (lattice units).  Sec. references are
 * to the paper. */
typedef struct lbfz_params {
  int32_t dim, nx, ny, nz;       /* dim 2 or 3; nz = 1 in 2D                   */
  int32_t walls;                 /* 0 all periodic; 1 walls on the last axis   */
  int32_t t_lo_dirichlet;        /* low wall: 1 Dirichlet T (anti-bounce-back), 0 adiabatic */
  int32_t t_hi_dirichlet;        /* high wall: same                            */
  int32_t surface_tension_mode;  /* 0: (1 - f_s) F_s (Sec. 4.5), 1: F_s        */
  int32_t storage;               /* LBFZ_STORE_*                               */
  int32_t contact_angle_deg;     /* wetting: only 90 is supported              */
  double rho_l, rho_g, rho_s;    /* end-member densities (end of Sec. 2)       */
  double nu;                     /* kinematic viscosity, tau_g = nu/cs^2 + 1/2 */
  double tau_phi;                /* phase field: mobility M = cs^2 (tau - 1/2) */
  double tau_h;                  /* enthalpy antisymmetric tau; lambda = (rho C)_ref cs^2 (tau - 1/2) */
  double tau_c;                  /* solute: D_l = cs^2 (tau - 1/2)             */
  double eps;                    /* interface thickness parameter (Eq. 3)      */
  double sigma0, sigma_T, sigma_c, T_ref, c_ref; /* linear equation of state (Sec. 2) */
  double cp_l, cp_s, cp_g;       /* specific heats                             */
  double rhoc_ref;               /* (rho C_p)_ref of the enthalpy equilibrium  */
  double latent, T_sol, T_liq;   /* latent heat, solidus, liquidus (Eq. Hfl)   */
  double k_p, Ds_over_Dl;        /* partition coefficient, D_s / D_l (Eq. c)   */
  double T_lo, T_hi, T_lo_amp;   /* wall T; low wall T_lo + T_lo_amp cos(2 pi x / nx) */
  double body_force[3];          /* F_b                                        */
} lbfz_params;

typedef struct lbfz_totals_t {
  double sum_f;     /* sum over nodes and directions of f (phase field)        */
  double sum_l;     /* sum of l (solute)                                       */
  double sum_h;     /* sum of h (enthalpy)                                     */
  double mpc;       /* accumulated sum over steps and nodes of phi div u: the
                       phase-field source, so sum_f - sum_f(0) - mpc = 0      */
  double vol_solid; /* sum of f_s at the current time level                    */
  double vol_sl;    /* sum of clamp((1 + phi) / 2, 0, 1)                       */
  int64_t step;     /* steps taken                                             */
  int64_t nonfinite;/* nodes with a non-finite population or field             */
} lbfz_totals_t;

typedef struct lbfz_handle lbfz_handle;

/* Bytes of device workspace the configuration needs (>= 256-byte aligned
 * base required).  Errors: LBFZ_EINVAL for invalid parameters. */
int lbfz_workspace_bytes(const lbfz_params* p, size_t* bytes);

/* Create a solver state from initial host fields (FP64, C-order, N values
 * each): phi, T, C, and an optional uint8 obstacle mask (3D only, NULL for
 * none; nonzero = obstacle).  u = 0, p = 0, f_l = 1 and every population at
 * its equilibrium (Sec. 3).  d_workspace / ws_bytes: caller-owned device
 * memory; stream: a hipStream_t or NULL.  Synchronises the stream once.
 * Errors: LBFZ_EINVAL (parameters: tau <= 1/2, eps <= 0, dims, contact angle
 * != 90, mask in 2D), LBFZ_ENOMEM (workspace), LBFZ_ENONFINITE (inputs),
 * LBFZ_EHIP. */
int lbfz_create(const lbfz_params* p, const double* phi, const double* T, const double* C,
                const uint8_t* mask, void* d_workspace, size_t ws_bytes, void* stream,
                lbfz_handle** out);

/* Advance nsteps >= 0 time steps (Sec. 3: closure, stencils, forces, the four
 * collisions, streaming).  Asynchronous on the handle's stream. */
int lbfz_step(lbfz_handle* h, int64_t nsteps);

/* Macroscopic fields at the current time level, FP32, N values each, for every
 * bit set in field_mask (bit k -> dst[k]; dst entries of unset bits are
 * ignored).  dst_is_device != 0: dst are device pointers (asynchronous);
 * else host pointers (synchronises). */
int lbfz_fields(lbfz_handle* h, uint32_t field_mask, float* const* dst, int dst_is_device);

/* Conservation totals at the current time level (FP64 reductions in a fixed
 * order, so repeated calls agree bit for bit).  Synchronises the stream. */
int lbfz_totals(lbfz_handle* h, lbfz_totals_t* out);

/* Raw solver state, for checkpoint / restart and for step-by-step checks:
 * FP32 planes of N values, in this order: the populations of the current
 * time level (f: Q_s planes, g: Q_g, h: Q_s, l: Q_s; D2Q5/D2Q9 order
 * (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1); D3Q7/D3Q19 order
 * rest, +x, -x, +y, -y, +z, -z, then the 12 edge links (+-x+-y, +-x+-z,
 * +-y+-z)), then the previous time level's f_s, p, u (dim planes), phi, C.
 * 2D: 30 planes, 3D: 47 planes.  lbfz_state_floats gives the count; get and
 * set copy to / from host memory and synchronise the stream.  The phase-field
 * source accumulator and the step counter are not part of the state. */
int lbfz_state_floats(lbfz_handle* h, size_t* nfloats);
int lbfz_get_state(lbfz_handle* h, float* host_dst);
int lbfz_set_state(lbfz_handle* h, const float* host_src);

/* Restart from macroscopic fields (2D): replace the state at the current time
 * level by the equilibrium one of the given fields -- d_fields[0..6]: device
 * FP32 planes of N values, phi, f_l, T, C, u_x, u_y, p.  Populations f, g, h,
 * l take their equilibria (Sec. 3.1 - 3.4) of (phi, u), (p, rho, u), (E, T,
 * u), (C, u) with E the enthalpy of (T, f_l) (the inverse of the enthalpy
 * map: sensible heat below the solidus, latent heat by the liquid fraction,
 * sensible heat above the liquidus); the previous level's f_s, p, u, phi, C
 * take the same fields.  Non-equilibrium parts (and the interface force's
 * half-step in the momentum) are dropped, so a restart from a solver's own
 * fields is close to, not equal to, continuing it.  Asynchronous on the
 * handle's stream.  f_l is taken as lbfz_fields exports it (1 - f_s, so 1 in
 * the gas).  Errors: LBFZ_EINVAL (NULL), LBFZ_EUNSUPPORTED (3D). */
int lbfz_restart_fields(lbfz_handle* h, const float* const* d_fields);

/* ------------------------------------------------------------------------
 * Batched sweep: many independent 2D grids (the parameter sweep of Sec. 5's
 * study, each grid a complete solver state with its own parameters, size,
 * buffers and totals) advanced in lockstep.  One batch step is one launch
 * over a single table of (grid, tile) work items that spans every grid,
 * whatever its size, replayed from a captured HIP graph (one kernel node per
 * step).  Results are those of the same grids stepped one by one (the
 * per-node arithmetic is identical).  Grids of equal size form a group, which
 * is only reported (lbfz_batch_group_config).
 * ------------------------------------------------------------------------ */
typedef struct lbfz_batch lbfz_batch;

/* Device workspace for ncases grids (params[i]: dim 2, one storage form for
 * all).  Errors: LBFZ_EINVAL. */
int lbfz_batch_workspace_bytes(int32_t ncases, const lbfz_params* params, size_t* bytes);

/* Create the grids from host FP64 initial fields phi[i], T[i], C[i] (as
 * lbfz_create), their work tables and case table in the caller's workspace.
 * Creates one internal HIP stream (default priority) used only to capture
 * graphs; all work runs on `stream`.  Synchronises the stream.  Errors as
 * lbfz_create, plus LBFZ_EINVAL for mixed storage or dim != 2. */
int lbfz_batch_create(int32_t ncases, const lbfz_params* params, const double* const* phi,
                      const double* const* T, const double* const* C, void* d_workspace,
                      size_t ws_bytes, void* stream, lbfz_batch** out);

/* Autotuner: time each candidate configuration of the whole batch step
 * (tile height 4 or 8 rows, i.e. 4 or 8 waves per block; one block per work
 * item, or a persistent grid of 2, 4 or 8 blocks per CU walking the work
 * table) over trial_steps steps and keep the fastest.  The trial steps are
 * real steps of every selected grid (8 * trial_steps in all).  Synchronises. */
int lbfz_batch_tune(lbfz_batch* b, int32_t trial_steps);

/* Advance every grid by nsteps (asynchronous on the stream). */
int lbfz_batch_step(lbfz_batch* b, int64_t nsteps);

/* The same with plain launches, one grid after the other (the reference the
 * batched step is measured against). */
int lbfz_batch_step_sequential(lbfz_batch* b, int64_t nsteps);

/* Number of groups (grids of equal size), and one group's size and count with
 * the batch's launch configuration (any output may be NULL). */
int lbfz_batch_groups(lbfz_batch* b);
int lbfz_batch_group_config(lbfz_batch* b, int32_t group, int32_t* nx, int32_t* ny,
                            int32_t* ncases, int32_t* tile_rows, int32_t* grid_blocks);

/* Fields and totals of grid i, as lbfz_fields / lbfz_totals.  LBFZ_EINVAL
 * for a stale grid (see lbfz_batch_select). */
int lbfz_batch_fields(lbfz_batch* b, int32_t i, uint32_t field_mask, float* const* dst,
                      int dst_is_device);
int lbfz_batch_totals(lbfz_batch* b, int32_t i, lbfz_totals_t* out);

/* The fields of every grid into one device buffer (asynchronous): grid i's
 * fields of the set bits of field_mask (bit order), one plane of its N
 * values after the other, from d_dst + i * case_stride (floats; case_stride
 * >= the number of set bits times the largest N).  One launch over every
 * grid's tiles; the values agree with lbfz_batch_fields up to FP32
 * rounding (the batched kernel forms its fused multiply-adds differently).
 * LBFZ_EINVAL if a grid is stale, LBFZ_EHIP if a launch fails. */
int lbfz_batch_fields_all(lbfz_batch* b, uint32_t field_mask, float* d_dst, int64_t case_stride);

/* Subset stepping (the LB fallback of a screened sweep): later steps advance
 * only the n grids listed in idx (n = 0: all grids again).  A grid left out
 * while the others step becomes stale -- its state no longer matches the
 * batch's time level -- until lbfz_batch_restart_fields gives it one; stepping
 * a selection that holds a stale grid, or reading a stale grid, is
 * LBFZ_EINVAL.  The autotuner times the selected grids.  Synchronises the
 * stream (uploads the work tables); a subset is stepped with plain launches,
 * the full selection with its captured graph. */
int lbfz_batch_select(lbfz_batch* b, int32_t n, const int32_t* idx);

/* lbfz_restart_fields for grid i at the batch's time level; clears its stale
 * mark.  Asynchronous. */
int lbfz_batch_restart_fields(lbfz_batch* b, int32_t i, const float* const* d_fields);

/* The same for the n grids idx[0 .. n-1]: field m of grid i at d_fields[m] +
 * i * case_stride[m] (floats; m < 7, order as lbfz_restart_fields).  FP32
 * storage: one launch for all n grids from a job table uploaded by this
 * call, which then synchronises the stream; 16-bit storage: one restart (and
 * its encoding pass) per grid, asynchronous. */
int lbfz_batch_restart_many(lbfz_batch* b, int32_t n, const int32_t* idx,
                            const float* const* d_fields, const int64_t* case_stride);

/* Release the grids, graphs and the capture stream (not the workspace). */
void lbfz_batch_destroy(lbfz_batch* b);

/* Device-to-device copy of `bytes` bytes (a multiple of 16; both pointers
 * 16-byte aligned; the ranges must not overlap): a streaming kernel that
 * reads and writes every byte once, as one time step reads and writes the
 * solver state once.  It is the memory-system ceiling the step's bandwidth is
 * measured against.  Asynchronous on `stream` (a hipStream_t or NULL).
 * Errors: LBFZ_EINVAL (NULL or misaligned pointer, size not a multiple of
 * 16), LBFZ_EHIP. */
int lbfz_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/* The memory pattern of one 2D FP32 step of an nx x ny grid without its
 * arithmetic: for every node, the 30 FP32 planes a node update reads (24
 * populations and 6 previous-level fields; plane k of src at k *
 * plane_stride floats) are read at the node and written into the same plane
 * of dst one row down, in place or one row up (k mod 3; y periodic), as the
 * step's pushed populations land on their target rows.  The bandwidth of
 * this kernel, beside lbfz_stream_copy's, bounds what the step's access
 * pattern can reach.  Both buffers hold 30 planes, device memory, not
 * overlapping; asynchronous on `stream`.  Errors: LBFZ_EINVAL (NULL pointer,
 * empty grid, plane_stride below nx * ny), LBFZ_EHIP. */
int lbfz_stream_planes(float* dst, const float* src, int nx, int ny, long plane_stride,
                       void* stream);

/* The memory pattern of one launch of the 3D FP32 step of an nx x ny x nz
 * grid without its arithmetic: for every node, planes 0 .. nread - 1 of src
 * (plane k at k * plane_stride floats) are read at the node, and planes 0 ..
 * nwrite - 1 of dst are written: plane k < 38 at the node displaced by D3Q19
 * direction k mod 19 (the step pushes its populations to the nodes they
 * stream to; x, y and z periodic here), planes from 38 on in place, each
 * with the value read from the same plane.  (nread, nwrite) is one of the
 * step's two launches: (22, 5) for the closure launch, (50, 42) for the
 * collision launch.  Device buffers of nread and nwrite planes, not
 * overlapping; asynchronous on `stream`.  Errors: LBFZ_EINVAL (NULL pointer,
 * empty grid, another (nread, nwrite), plane_stride below nx * ny * nz),
 * LBFZ_EHIP. */
int lbfz_stream_planes3d(float* dst, const float* src, int nx, int ny, int nz, long plane_stride,
                         int nread, int nwrite, void* stream);

/* Blocks until the handle's stream is idle. */
int lbfz_sync(lbfz_handle* h);

/* Release the handle (not the workspace or the stream, which the caller owns). */
void lbfz_destroy(lbfz_handle* h);

/* Static text for an error code. */
const char* lbfz_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* LBFZ_H */
