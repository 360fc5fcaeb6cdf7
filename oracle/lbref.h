/*
 * lbref.h -- FP64 CPU oracle of one time step of the coupled lattice
 * Boltzmann freezing scheme (Huang, Chai, Liu, Huang, "Diffuse-interface
 * modeling and simulation of the freezing of binary fluids with the
 * Marangoni effect", arXiv 2511.09422, Sec. 2 and Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the independent checker of the
 * GPU path: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no source, header, table or helper
 * with the HIP library, and the HIP library never calls it.
 *
 * Everything is plain FP64 on two population arrays with pull streaming; the
 * order of operations follows the paper's Sec. 3 (closure, gradients, forces,
 * collisions, streaming).  Lattice units throughout: dx = dt = 1, cs^2 = 1/3.
 *
 * Layout: scalar fields are C-order [nz][ny][nx] (2D: nz = 1).  The wall axis
 * (when walls != 0) is the last axis: y in 2D, z in 3D; the other axes are
 * periodic.  Nodes are cell-centred: node j sits at coordinate j, the low wall
 * at -1/2 and the high wall at n-1/2.
 *
 * Errors: every int-returning call returns 0 on success or a negative code
 * (-1 invalid argument, -2 out of memory).  No call aborts.
 */
#ifndef LBREF_H
#define LBREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbref_params {
  int32_t dim, nx, ny, nz;        /* 2 or 3; nz = 1 in 2D                      */
  int32_t walls;                  /* 0: all axes periodic; 1: walls on last axis */
  int32_t t_lo_dirichlet;         /* low wall: 1 Dirichlet T (anti-bounce-back), 0 adiabatic */
  int32_t t_hi_dirichlet;         /* high wall: same                              */
  int32_t surface_tension_mode;   /* 0: (1 - f_s) F_s (Sec. 4.5), 1: F_s          */
  int32_t threads;                /* OpenMP threads for node loops (>= 1)         */
  double rho_l, rho_g, rho_s;     /* end-member densities (property interpolation) */
  double nu;                      /* kinematic viscosity, tau_g = nu/cs2 + 1/2    */
  double tau_phi;                 /* phase-field relaxation time (mobility M)     */
  double tau_h;                   /* antisymmetric enthalpy relaxation time       */
  double tau_c;                   /* solute relaxation time for the liquid D_l    */
  double eps;                     /* interface thickness parameter epsilon        */
  double sigma0, sigma_T, sigma_c, T_ref, c_ref;   /* linear equation of state  */
  double cp_l, cp_s, cp_g;        /* specific heats                               */
  double rhoc_ref;                /* constant (rho C_p)_ref of the enthalpy LB    */
  double latent, T_sol, T_liq;    /* latent heat, solidus, liquidus               */
  double k_p, Ds_over_Dl;         /* partition coefficient, D_s / D_l             */
  double T_lo, T_hi, T_lo_amp;    /* wall temperatures; low wall T_lo + amp cos(2 pi x / nx) */
  double body_force[3];           /* F_b                                          */
} lbref_params;

typedef struct lbref_state lbref_state;

/* Initial macroscopic fields phi, T, C (FP64, C-order), optional obstacle
 * mask (uint8, nonzero = obstacle).  u = 0, p = 0, f_l = 1 everywhere. */
int  lbref_create(const lbref_params* p, const double* phi, const double* T,
                  const double* C, const uint8_t* mask, lbref_state** out);
void lbref_destroy(lbref_state* s);
int  lbref_step(lbref_state* s, int64_t nsteps);

/* Macroscopic fields at the current time level (a dry evaluation of the
 * closure, gradients and forces; populations are not touched).  Any pointer
 * may be NULL.  Obstacle nodes report phi = -1, u = 0, p = 0, C = 0. */
int  lbref_fields(lbref_state* s, double* phi, double* fl, double* T, double* C,
                  double* ux, double* uy, double* uz, double* p, double* rho);

/* out[0..8] = sum_f, sum_l, sum_h, M_pc (accumulated sum phi div u),
 * vol_solid (sum f_s), vol_sl (sum clamp((1+phi)/2)), step, nonfinite-node
 * count, accumulated sum of the enthalpy source Q. */
int  lbref_totals(lbref_state* s, double out[9]);
/* Lattice tables: which 1 = flow lattice, else the scalar lattice.
 * c: [q][3] ints, w: [q] doubles, opp: [q] ints.  Returns q. */
int  lbref_lattice(int dim, int which, int* c, double* w, int* opp);

/* Raw access for tests and checkpoints.  which: 0 f, 1 g, 2 h, 3 l; the
 * array is [q][nz][ny][nx].  State scalars of time level n-1: 0 f_s, 1 p,
 * 2..4 u components, 5 phi, 6 C. */
int  lbref_get_pops(lbref_state* s, int which, double* dst);
int  lbref_set_pops(lbref_state* s, int which, const double* src);
int  lbref_get_state(lbref_state* s, int which, double* dst);
int  lbref_set_state(lbref_state* s, int which, const double* src);
int  lbref_q(int dim, int which);

/* Pointwise pieces exposed for the moment-identity and stencil pins. */
void lbref_enthalpy_map(const lbref_params* p, double E, double psi,
                        double* T, double* fl, double* fs);
void lbref_feq_g(int dim, double pr, double rho, const double* u, double* out);
void lbref_src_g(int dim, double S, const double* Ff, const double* u,
                 const double* Ft, double* out);
void lbref_heq(const lbref_params* p, double E, double T, double rhocp,
               const double* u, double* out);
void lbref_grad_lap(const lbref_params* p, const double* field, int kind,
                    double* grad /* [3][N] */, double* lap /* [N] or NULL */);

#ifdef __cplusplus
}
#endif
#endif
