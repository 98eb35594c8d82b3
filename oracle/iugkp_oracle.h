/*
 * iugkp_oracle.h -- plain single-threaded FP64 CPU oracle for the implicit
 * unified gas-kinetic particle (IUGKP) steady gray phonon BTE iteration.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes (paper: Liu, Yang, Zhang, Ji, Xu, "Implicit unified gas
 * kinetic particle method for steady-state solution of multiscale phonon
 * transport", arXiv 2506.09465):
 *   - Sec. 2, linearised gray BGK model: e_eq = C (T - T_ref) / 4 pi,
 *     E = integral of e over the sphere, T = E / C + T_ref;
 *   - Sec. 3.1, one iteration = resample every particle from its cell's
 *     equilibrium, fly an exponential free path lambda = -u tau ln(eta),
 *     count the energy deposited per cell (eq. for W_i as a sum of particle
 *     weights);
 *   - Sec. 3.2, spatially varying tau: a common time scale tau_min, candidate
 *     collisions with free path -u tau_min ln(eta), accepted as real with
 *     probability sigma(x)/sigma_max = tau_min/tau(x), total tally W (null +
 *     real) and real tally W^h, re-emission from W^h;
 *   - Sec. 3.3, inexact Newton with the diffusion-type operator
 *     div(-kappa grad dT) on the energy residual between iterations;
 *   - beyond the paper: a volumetric heat source (extra isotropic emission
 *     S V tau_min per cell and iteration) and the adjoint of the steady state
 *     with respect to the wall temperatures and the source (orc_adjoint).
 * Every point the paper leaves open is fixed by a reading stated next to the
 * function that implements it.
 */
#ifndef IUGKP_ORACLE_H
#define IUGKP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_W_NOT_CONVERGED = 1,
  ORC_E_INVALID_ARG = -1,
  ORC_E_NOMEM = -2,
  ORC_E_FIXED_OVERFLOW = -4,
  ORC_E_NONFINITE = -5,
  ORC_E_CG_BREAKDOWN = -6,
  ORC_E_CG_NOT_CONVERGED = -7,
  ORC_E_DIVERGED = -8
};

enum { ORC_RNG_FRESH = 0, ORC_RNG_CRN = 1 };
enum { ORC_FACES_OFF = 0, ORC_FACES_EVERY = 1, ORC_FACES_FINAL = 2 };

typedef struct orc_problem {
  int dim;              /* 1 or 2 */
  int nx, ny;           /* cells; ny == 1 in 1D */
  double dx, dy;        /* cell sizes; dy == 1 in 1D (unit area) */
  double t_ref, cv, vg; /* reference temperature, volumetric heat capacity, |V_g| */
  const double *tau;    /* [nx*ny] relaxation time per cell, c = ix + nx*iy */
  const double *wall_T; /* [n_b] wall temperatures: left rows, right rows, bottom cols, top cols */
  const double *T_init; /* [nx*ny] initial temperature or NULL (-> t_ref) */
  const double *diff_x; /* [nx*ny] per-iteration diffusion coefficient along x (Newton), or NULL */
  const double *diff_y; /* [nx*ny] along y (2D Newton), or NULL */
  const double *source; /* [nx*ny] volumetric heat source S (energy per volume and time), or NULL */
  int n_bands;          /* 0 or 1: gray (cv, vg, tau as above); >= 2: frequency bands (orc_bands_*) */
  const double *band_C; /* [n_bands] heat capacity per band (the total replaces cv) */
  const double *band_vg;/* [n_bands] group speed per band (replaces vg); tau is then [n_bands][nx*ny] */
} orc_problem;

typedef struct orc_options {
  uint64_t seed;
  uint64_t particles_per_iter;
  int rng_mode;         /* ORC_RNG_FRESH: Philox slot = iteration; ORC_RNG_CRN: slot = rng_epoch */
  uint32_t rng_epoch;
  int max_iters;
  double res_tol;
  int newton;           /* 0/1 */
  double cg_tol;
  int cg_max_iters;
  int tally_faces;      /* ORC_FACES_* */
  int avg_iters;
  int estimator;        /* ORC_EST_ANALOG: sampled collision points; ORC_EST_EXPECTED: the
                           expected deposits along each ray (gray emitter scheme only) */
  int cg_precond;       /* ORC_PRECOND_NONE: plain CG; ORC_PRECOND_MG: multigrid V-cycle PCG */
} orc_options;

enum { ORC_PRECOND_NONE = 0, ORC_PRECOND_MG = 1 };

enum { ORC_EST_ANALOG = 0, ORC_EST_EXPECTED = 1 };

typedef struct orc_info {
  uint32_t iter;        /* iterations done */
  int F;                /* fixed-point exponent */
  uint64_t n_per_emitter;
  int n_cells, n_bfaces, n_emitters;
  double tau_min, lam_min;
  double d0, res;       /* first-iteration update norm, last relative residual */
  uint64_t flights, segments, crossings;         /* last iteration */
  uint64_t tot_flights, tot_segments, tot_crossings;
  int cg_iters_last, cg_iters_total;
} orc_info;

typedef struct orc_state orc_state;

/* ---- building blocks (exported for unit tests) ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u53(uint32_t hi, uint32_t lo);
double orc_log(double x);
double orc_cos2pi(double u);
double orc_expm(double T);   /* exp(-T) for T >= 0 from + - * / (0 beyond T = 700) */
void orc_philox_batch(const uint32_t *ctr, uint64_t n, uint32_t k0, uint32_t k1, uint32_t *out);
/* op: 0 log, 1 cos(2 pi x), 2 sqrt, 3 x / y, 4 (double) of the int64 bits of x,
 * 5 rint(ldexp(x, (int) y)) stored as int64 bits, 6 exp(-x) (orc_expm) */
void orc_math_batch(int op, const double *x, const double *y, double *out, uint64_t n);
int64_t orc_split_weight(int64_t G, uint64_t n, uint64_t k);
double orc_tree_sum(const double *v, uint64_t n);
int orc_fixed_exponent(const orc_problem *p, double *tau_min_out);

/* One ray, recorded: march from (x0,y0) in cell (ix,iy) along (sx,sy) a length
 * ell (no null collisions).  events[3*i] = axis (0 x, 1 y), [3*i+1] = face
 * index in its tally array, [3*i+2] = sign.  Returns the number of crossings;
 * *end_kind = 0 stopped in cell *end_cell, 1 absorbed by boundary face *end_cell. */
int orc_trace_ray(const orc_problem *p, double x0, double y0, int ix, int iy, double sx,
                  double sy, double ell, int32_t *events, int max_events, int *end_kind,
                  int *end_cell);

/* Unpreconditioned CG on the Newton operator assembled from diff_x/diff_y. */
int orc_newton_operator(const orc_problem *p, double *gx, double *gy, double *diag);
int orc_cg(const orc_problem *p, const double *gx, const double *gy, const double *diag,
           const double *b, double *x, double tol, int max_iters, int *iters_out);
/* The same system by CG preconditioned with one multigrid V-cycle (reading R19). */
int orc_pcg_mg(const orc_problem *p, const double *gx, const double *gy, const double *diag,
               const double *b, double *x, double tol, int max_iters, int *iters_out);
/* x = M b, the V-cycle preconditioner alone. */
int orc_mg_precondition(const orc_problem *p, const double *gx, const double *gy,
                        const double *diag, const double *b, double *x);
/* Number of levels of the hierarchy and the mesh of level k (nx, ny). */
int orc_mg_levels(const orc_problem *p, int *nx_out, int *ny_out, int max_levels);

/* ---- the iteration ---- */
int orc_create(const orc_problem *p, const orc_options *o, orc_state **out);
void orc_destroy(orc_state *s);
int orc_step(orc_state *s, int n_iters, int faces);
int orc_solve(orc_state *s, double *T_out, double *qx_out, double *qy_out);
void orc_get_info(const orc_state *s, orc_info *info);
void orc_get_tallies(const orc_state *s, int64_t *D, int64_t *W, int64_t *Phix, int64_t *Phiy,
                     int64_t *B);
void orc_get_E(const orc_state *s, double *E);
void orc_get_G(const orc_state *s, int64_t *G);
void orc_get_residuals(const orc_state *s, double *res, int max_n);
int orc_set_state(orc_state *s, uint32_t iter, double d0, const double *E, const int64_t *G);

/* Adjoint of the steady state (uniform relaxation time, common random numbers):
 * given dL/dT per cell, the gradient of L with respect to every wall face's
 * temperature (grad_wall [n_b]) and every cell's source (grad_source [nc]),
 * for the particle paths of slot rng_epoch.  Iterates to a relative change
 * below tol (at most max_iters passes), with the forward solve's diffusion
 * correction when the state was created with newton.  *iters_out = passes. */
int orc_adjoint(orc_state *s, const double *dLdT, double *grad_wall, double *grad_source,
                int max_iters, double tol, int *iters_out);

/* ---- frequency bands (beyond the paper's gray model) ----
 * K bands with heat capacity C_k, group speed v_k and relaxation time
 * tau_k(c).  Band k uses its own common time scale tau*_k = min_c tau_k(c)
 * (candidate path v_k tau*_k, acceptance tau*_k / tau_k(c)); emitters are
 * (band, cell or wall face), counter index k (nc + nb) + emitter.  One
 * iteration: every band flies its emitters; per cell the absorbed rate
 * R = sum_k D_k 2^-F / tau*_k (+ S V) is re-emitted over the bands as the
 * equilibrium spectrum, G_k = tau*_k (C_k / tau_k) / (sum_j C_j / tau_j) R
 * (pseudo-temperature); the energy density is E = sum_k W_k 2^-F / V and
 * T = t_ref + E / sum_k C_k; walls emit C_k (T_w - t_ref) v_k tau*_k A / 4;
 * the heat flux is sum_k Phi_k 2^-F / tau*_k / A.  No Newton step. */
typedef struct orc_bands orc_bands;
int orc_bands_create(const orc_problem *p, const orc_options *o, orc_bands **out);
void orc_bands_destroy(orc_bands *s);
int orc_bands_step(orc_bands *s, int n_iters, int faces);
int orc_bands_solve(orc_bands *s, double *T_out, double *qx_out, double *qy_out);
void orc_bands_get_info(const orc_bands *s, orc_info *info);
void orc_bands_get_E(const orc_bands *s, double *E);
/* band k's tallies of the last iteration and its emitter energies for the next */
void orc_bands_get_band(const orc_bands *s, int k, int64_t *D, int64_t *W, int64_t *Phix,
                        int64_t *Phiy, int64_t *B, int64_t *G);

/* ---- persistent particles: the paper's variable-tau iteration (Sec. 3.2
 * steps (1)-(6)) with a fixed particle population ----
 * N = max(1, particles_per_iter / (cells + wall faces)) particles per cell
 * are created in equilibrium (weight: the cell's energy E V split over its N
 * particles, uniform position, isotropic direction), and N per wall face as
 * if just absorbed there (they carry the face's first emission); the
 * population is kept from iteration to iteration (particle c N + k of cell
 * c, (cells + b) N + k of wall face b).  Each iteration every particle flies one candidate path on the
 * common time scale tau_min: a real-collision particle is first resampled
 * from its cell's equilibrium (uniform point of the cell, isotropic
 * direction) with the weight w_c of its cell, a particle absorbed by
 * a wall face is re-emitted from that face (uniform point, cosine law) with
 * the face's weight w_b, a null-collision particle keeps its position,
 * direction and weight.  At the end of its path it is absorbed by a wall or
 * adds its weight to W of the cell it reached and is accepted as real with
 * probability tau_min / tau (then also to W^h and the count N_rc).  Then
 * E = W / V, and the real particles of cell c share W^h_c + S V tau_min plus
 * the cell's carried remainder: w_c = floor(. / N_rc), the remainder carried
 * to the next iteration (all of it when N_rc = 0); likewise wall face b
 * shares its emission E_w lambda_min A / 4 plus its carried remainder over
 * the N_b particles it absorbed.  Counter of particle p's draw d in an
 * iteration with slot s: (d, p, 0xffffffff, s); creation uses slot
 * 0xffffffff; d = 0 position, 1 direction, 2 (free path, acceptance).
 * Particle kinds: 0 null (moves on), 1 real (resampled in its cell),
 * 2 absorbed by a wall face (re-emitted from it); loc = cell or wall face. */
typedef struct orc_persist orc_persist;
int orc_persist_create(const orc_problem *p, const orc_options *o, orc_persist **out);
void orc_persist_destroy(orc_persist *s);
int orc_persist_step(orc_persist *s, int n_iters, int faces);
int orc_persist_solve(orc_persist *s, double *T_out, double *qx_out, double *qy_out);
void orc_persist_get_info(const orc_persist *s, orc_info *info);
void orc_persist_get_E(const orc_persist *s, double *E);
uint64_t orc_persist_count(const orc_persist *s);
/* particle state (any pointer may be NULL) */
void orc_persist_get_particles(const orc_persist *s, double *x, double *y, double *sx, double *sy,
                               int64_t *q, int32_t *kind, int32_t *loc);
/* tallies of the last iteration: W, W^h and N_rc per cell, face fluxes, wall
 * absorption B and count N_b; next weights and carried remainders */
void orc_persist_get_tallies(const orc_persist *s, int64_t *W, int64_t *Wh, uint32_t *Nrc,
                             int64_t *Phix, int64_t *Phiy, int64_t *B, uint32_t *Nb);
void orc_persist_get_shares(const orc_persist *s, int64_t *wc, int64_t *rc, int64_t *wb,
                            int64_t *rb);

#ifdef __cplusplus
}
#endif
#endif
