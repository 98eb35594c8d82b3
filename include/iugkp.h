/*
 * iugkp.h -- C ABI of the MI355X (gfx950) implicit unified gas-kinetic
 * particle (IUGKP) solver for the steady linearised gray phonon BTE.
 *
 * Method: Liu, Yang, Zhang, Ji, Xu, "Implicit unified gas kinetic particle
 * method for steady-state solution of multiscale phonon transport",
 * arXiv 2506.09465.
 *   Sec. 2   model: V_g . grad e = (e_eq - e) / tau, e_eq = C (T - T_ref) / 4 pi,
 *            E = integral of e over the sphere, T = E / C + T_ref, q = integral of V_g e.
 *   Sec. 3.1 iteration for constant tau: resample every particle from its
 *            cell's equilibrium, fly the exponential free path
 *            lambda = -|V_g| tau ln(eta), count the energy that lands in each cell.
 *   Sec. 3.2 variable tau: common time scale tau_min, candidate collisions
 *            accepted with probability tau_min / tau(x) (null collisions); the
 *            macroscopic energy from all candidates (W), re-emission from the
 *            real ones (W^h).
 *   Sec. 3.3 inexact Newton: a diffusion-type linear operator on the energy
 *            change between iterations predicts the next equilibrium.
 *
 * Conventions shared by every call
 *   - Uniform Cartesian mesh, cell c = ix + nx * iy, sizes dx, dy (1D: ny = 1,
 *     dy = 1, unit face area).
 *   - Wall faces b = 0 .. n_b-1 in the order: left wall rows (ny), right wall
 *     rows (ny), bottom wall columns (nx), top wall columns (nx); 1D has the
 *     two end walls only (n_b = 2).
 *   - Emitters: the n_cells cells then the n_b wall faces; every emitter emits
 *     the same number N = max(1, particles_per_iter / (n_cells + n_b)) of
 *     particles per iteration.
 *   - Face arrays: x-faces [ny][nx+1] (face k of row iy at index iy*(nx+1)+k),
 *     y-faces [ny+1][nx] (face k of column ix at index k*nx+ix); 1D has no
 *     y-faces.
 *   - Energies are int64 fixed-point numbers with scale 2^F; tallies are exact
 *     integer sums, identical for any launch shape or order.
 *   - Every entry point returns IUGKP_OK (0) on success, a negative error code
 *     on failure (nothing is written to outputs then), or the positive warning
 *     IUGKP_W_NOT_CONVERGED (outputs written).  iugkp_last_error() gives a
 *     message for the last failing call on the calling thread.
 *   - A handle is not thread-safe; distinct handles may be used concurrently.
 *   - All device work is issued on the HIP stream given at creation; calls
 *     returning host data synchronise that stream.
 */
#ifndef IUGKP_H
#define IUGKP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IUGKP_OK 0
#define IUGKP_W_NOT_CONVERGED 1
#define IUGKP_E_INVALID_ARG (-1)
#define IUGKP_E_NOMEM (-2)
#define IUGKP_E_DEVICE (-3)
#define IUGKP_E_FIXED_OVERFLOW (-4)
#define IUGKP_E_NONFINITE (-5)
#define IUGKP_E_CG_BREAKDOWN (-6)
#define IUGKP_E_CG_NOT_CONVERGED (-7)
#define IUGKP_E_DIVERGED (-8)

/* where caller arrays live */
#define IUGKP_MEM_HOST 0
#define IUGKP_MEM_DEVICE 1

/* Philox slot per iteration: FRESH = iteration index, CRN = rng_epoch (fixed) */
#define IUGKP_RNG_FRESH 0
#define IUGKP_RNG_CRN 1

/* face (heat-flux) tallies: never, every iteration, or only in the output iteration(s) */
#define IUGKP_FACES_OFF 0
#define IUGKP_FACES_EVERY 1
#define IUGKP_FACES_FINAL 2

typedef struct iugkp_problem {
  int dim;              /* 1 or 2 */
  int nx, ny;           /* cell counts, ny == 1 in 1D, nx * ny <= 2^24 */
  double dx, dy;        /* cell sizes (> 0); dy is the unit face area in 1D */
  double t_ref;         /* reference temperature of the linearisation (Sec. 2) */
  double cv;            /* volumetric heat capacity C (> 0) */
  double vg;            /* group velocity magnitude |V_g| (> 0) */
  const double *tau;    /* [n_cells] relaxation time (> 0, finite, max/min <= 1e6) */
  const double *wall_T; /* [n_b] wall temperatures */
  const double *T_init; /* [n_cells] initial temperature, or NULL for t_ref everywhere */
  const double *diff_x; /* [n_cells] Newton diffusion coefficient along x per iteration, or
                           NULL: the library uses D_eff(|V_g| tau_c, dx) (iugkp_d_eff) */
  const double *diff_y; /* [n_cells] the same along y (2D), or NULL */
  int mem_kind;         /* IUGKP_MEM_HOST or IUGKP_MEM_DEVICE for the arrays above and below */
  const double *source; /* [n_cells] volumetric heat source S (energy per volume and time), or
                           NULL.  Each cell emits S V tau_min more per iteration, isotropically
                           from uniform positions like its equilibrium emission (an addition to
                           the gray model of Sec. 2-3) */
  int n_bands;          /* 0 or 1: the gray model (Sec. 2).  K >= 2: K frequency bands (an
                           extension of the gray model): tau is then [K][n_cells] (band-major),
                           band k carries heat capacity band_C[k] and group velocity
                           band_vg[k] (cv and vg are not used), its own candidate time
                           tau*_k = min_c tau_k(c), free path band_vg[k] tau*_k and acceptance
                           tau*_k / tau_k(c).  Every cell re-emits its absorbed rate
                           R = sum_k D_k / tau*_k (+ S V) over the bands with the equilibrium
                           spectrum, band k taking the share (C_k / tau_k) / sum_j (C_j / tau_j),
                           emission G_k = tau*_k share_k R; the energy density is
                           E = sum_k W_k / V and T = t_ref + E / sum_k C_k.  Walls emit
                           C_k (T_w - t_ref) lambda*_k A / 4 in band k.  Every emitter of
                           every band flies N = max(1, particles_per_iter / (K (n_cells + n_b)))
                           particles, band k's with emitter index k (n_cells + n_b) + e in the
                           Philox counter.  No Newton correction and no output averaging; not
                           for batches or the adjoint */
  const double *band_C; /* [n_bands] band heat capacities (> 0), n_bands >= 2 only */
  const double *band_vg;/* [n_bands] band group velocities (> 0), n_bands >= 2 only */
} iugkp_problem;

typedef struct iugkp_options {
  uint64_t seed;                /* Philox key = (seed low 32 bits, seed high 32 bits) */
  uint64_t particles_per_iter;  /* requested particles per iteration (>= 1) */
  int rng_mode;                 /* IUGKP_RNG_FRESH or IUGKP_RNG_CRN */
  uint32_t rng_epoch;           /* slot used in CRN mode */
  int max_iters;                /* iteration cap of iugkp_solve (>= 0) */
  double res_tol;               /* stop when ||E^{n+1}-E^n|| / ||E^1-E^0|| < res_tol */
  int newton;                   /* 0/1: inexact-Newton (diffusion) correction, Sec. 3.3 */
  double cg_tol;                /* CG stop: ||r||^2 <= cg_tol^2 ||b||^2 */
  int cg_max_iters;             /* CG iteration cap per Newton step (>= 1 if newton) */
  int tally_faces;              /* IUGKP_FACES_* */
  int avg_iters;                /* iterations averaged for the outputs after stopping (>= 0) */
  int block_size;               /* transport kernel workgroup size: 0 (= 256), 64..1024 */
  int march;                    /* single solves on 2D meshes: 0 automatic (row stripes for
                                   face-tallied iterations with long free paths, tiles
                                   otherwise; see iugkp_march_tuning), 1 emitter tiles, 2 row
                                   stripes (also for the expected-value estimator, with or
                                   without face tallies), 3 row stripes with the y faces cut
                                   into pieces (without null collisions; else as 2).
                                   Persistent scheme: the y faces of face-tallied moves by a
                                   row-stripe pass (2 or 3, or 0 with long free paths) or as
                                   global atomics in the move (1).  Frequency bands: bands
                                   whose free paths reach half the domain's height run their
                                   face-tallied iterations by row stripes unless march is 1.
                                   The result does not depend on it */
  int cg_waves;                 /* single solves: 256-cell tree blocks per CG workgroup, 0
                                   (= 8) or 1..12 with the CG state in registers, -1..-12 with
                                   it in global memory (with IUGKP_PRECOND_MG: |cg_waves|
                                   wavefronts per workgroup); the result does not depend on
                                   it */
  int scheme;                   /* IUGKP_SCHEME_EMITTERS (0): every emitter flies N fresh
                                   particles per iteration, null collisions followed within
                                   the iteration.  IUGKP_SCHEME_PERSISTENT (1): the variable-tau
                                   iteration of Sec. 3.2 steps (1)-(6) with a fixed population
                                   of N = max(1, particles_per_iter / (n_cells + n_b))
                                   particles per cell and per wall face, kept between
                                   iterations: each iteration every particle flies one
                                   candidate path on the common time scale tau_min; a
                                   real-collision particle is first resampled from its cell's
                                   equilibrium (uniform point, isotropic direction) with the
                                   cell's share w_c = floor((W^h_c + S V tau_min + r_c) /
                                   N_rc), the remainder r_c carried to the next iteration (all
                                   of it when N_rc = 0); a particle absorbed by a wall face is
                                   re-emitted from it (uniform point, cosine law) with the
                                   face's share of its emission E_w lambda_min A / 4 plus its
                                   carried remainder; a null particle keeps position, direction
                                   and weight.  E = W / V (all candidates).  Particle p's draw
                                   d uses the counter (d, p, 0xffffffff, slot), creation slot
                                   0xffffffff.  Gray single solves without the Newton step
                                   only.  Tallies: D = W^h (real collisions), W, faces, B */
  int estimator;                /* IUGKP_EST_ANALOG (0): each particle ends at sampled
                                   candidate points.  IUGKP_EST_EXPECTED (1, emitter scheme,
                                   gray): variance reduction by the expected deposits along
                                   each ray (the particle form of the CDF-weighted sum of
                                   Sec. 2): no free path is drawn; with optical depth T along
                                   the ray (T += chord tau_min / (lambda_min tau_c)) and the
                                   rounded surviving weight S(T) = rint(q exp(-T)), a cell's
                                   chord from T_a to T_b receives D += S(T_a) - S(T_b) (exactly
                                   conserved) and, with null collisions, the expected
                                   candidates W += rint(q (exp(-T_a) - exp(-T_b)) / ratio_c);
                                   crossed faces carry S, a wall face absorbs it; the ray ends
                                   where S reaches 0.  exp is the library's own (+ - * / and
                                   exact scaling), bitwise reproducible */
  int own_stream;               /* 0: work is issued on the stream given to iugkp_create.
                                   1: the handle creates a stream of its own (default priority,
                                   ordered with the null stream) and destroys it with the
                                   handle; the stream argument is ignored.  Handles with their
                                   own streams advance concurrently under iugkp_step_group */
  int cg_precond;               /* linear solver of the Newton step (Sec. 3.3 leaves it open):
                                   IUGKP_PRECOND_NONE (0) plain CG; IUGKP_PRECOND_MG (1), single
                                   solves only: CG preconditioned with one multigrid V-cycle
                                   (2x2 aggregation down to one cell, Galerkin coarse
                                   operators, two damped Jacobi sweeps with weight 0.8 before
                                   and after the coarse correction scaled by 1.8, the one-cell
                                   level solved exactly).  Both stop at the same rule */
} iugkp_options;

enum { IUGKP_PRECOND_NONE = 0, IUGKP_PRECOND_MG = 1 };

enum { IUGKP_SCHEME_EMITTERS = 0, IUGKP_SCHEME_PERSISTENT = 1 };
enum { IUGKP_EST_ANALOG = 0, IUGKP_EST_EXPECTED = 1 };

typedef struct iugkp_stats {
  int iters;                    /* iterations done since creation (or the restored state) */
  double res;                   /* last relative update norm */
  uint64_t flights;             /* particles flown in the last iteration (weight != 0) */
  uint64_t segments;            /* free-path segments in the last iteration */
  uint64_t crossings;           /* face crossings in the last iteration */
  uint64_t tot_flights, tot_segments, tot_crossings;
  double ms_march, ms_update, ms_cg;  /* accumulated GPU time per phase (HIP events) */
  int cg_iters_last, cg_iters_total;
  int fixed_point_F;            /* fixed-point exponent */
  uint64_t n_per_emitter;       /* N */
  int n_emitters;
  int status;                   /* result of the solve: IUGKP_OK, IUGKP_W_NOT_CONVERGED or an
                                   error code (per instance in a batch) */
} iugkp_stats;

typedef struct iugkp_handle iugkp_handle;
typedef struct iugkp_batch iugkp_batch;

/* Create a solver for one problem.  Copies every problem array into library-owned
 * device memory (the caller may free its arrays on return), computes the
 * fixed-point exponent F = 62 - ceil(log2 B), B = 4 max|E| (sum of cell volumes
 * + lambda_min (sum of wall areas) / 4), the wall emission energies
 * E_w lambda_min A / 4 (cosine-law black walls) and the initial cell emission.
 * stream: a hipStream_t (NULL = default stream).
 * Errors: INVALID_ARG (bad sizes, tau <= 0 or not finite, NULL arrays, Newton
 * options out of range), NOMEM, DEVICE, FIXED_OVERFLOW. */
int iugkp_create(const iugkp_problem *problem, const iugkp_options *options, void *stream,
                 iugkp_handle **out);

void iugkp_destroy(iugkp_handle *h);

/* Run n_iters iterations (Sec. 3.1 steps (1)-(3) / Sec. 3.2 steps (1)-(6), then
 * the macroscopic update and, if enabled, the Newton correction of Sec. 3.3).
 * Face tallies are taken when tally_faces == IUGKP_FACES_EVERY.
 * Errors: FIXED_OVERFLOW, NONFINITE, CG_BREAKDOWN, CG_NOT_CONVERGED, DIVERGED, DEVICE. */
int iugkp_step(iugkp_handle *h, int n_iters);

/* n_iters iterations of each of n distinct handles.  Every handle's
 * iterations run back to back on its stream; the host enqueues a handle's
 * next iteration as soon as its previous one has completed, without waiting
 * for the others, so independent problems on their own streams overlap on
 * the GPU (one's Newton CG with another's particle step).  Each handle takes
 * its own tally_faces mode, as iugkp_step.  After the first error no new
 * iteration is started (those in flight are completed) and that error is
 * returned; the results of each handle equal those of iugkp_step. */
int iugkp_step_group(iugkp_handle *const *hs, int n, int n_iters);

/* Same with the face tallies forced on (faces = 1) or off (faces = 0). */
int iugkp_step_faces(iugkp_handle *h, int n_iters, int faces);

/* Iterate until res < res_tol or max_iters, then produce the outputs: with
 * avg_iters > 0 the mean of that many further iterations, otherwise the last
 * state (plus one face-tally iteration in FACES_FINAL mode).
 *   T_out  [n_cells]            T = t_ref + E / cv
 *   qx_out [ny*(nx+1)] or NULL  x heat flux per face (energy / (area * tau_min))
 *   qy_out [(ny+1)*nx] or NULL  y heat flux per face (2D)
 * Output arrays are caller-owned, in the problem's mem_kind.
 * Returns OK, W_NOT_CONVERGED, or an error as iugkp_step. */
int iugkp_solve(iugkp_handle *h, double *T_out, double *qx_out, double *qy_out,
                iugkp_stats *stats);

/* Tallies of the last iteration (int64, exact): D = real-collision energy per
 * cell (W^h), W = all candidate-collision energy per cell, Phi_x / Phi_y = net
 * energy through each face along +x / +y, B = energy absorbed per wall face.
 * Any pointer may be NULL.  Arrays in the problem's mem_kind.  For a problem of K
 * frequency bands every array holds K consecutive per-band blocks (band-major). */
int iugkp_get_tallies(iugkp_handle *h, int64_t *D, int64_t *W, int64_t *Phi_x,
                      int64_t *Phi_y, int64_t *B);

/* Resumable state: iteration count, first-iteration update norm, E^n [n_cells]
 * and the next emission energies G [n_cells + n_b] (int64; [K][n_cells + n_b]
 * for K frequency bands; the shares w_c then w_b for the persistent scheme,
 * whose state is its population: set_state refuses it).  set_state restores
 * it (resume is bitwise identical to an uninterrupted run).  Arrays in the
 * problem's mem_kind. */
int iugkp_get_state(iugkp_handle *h, uint32_t *iter, double *d0, double *E, int64_t *G);
int iugkp_set_state(iugkp_handle *h, uint32_t iter, double d0, const double *E,
                    const int64_t *G);

/* Persistent population (scheme IUGKP_SCHEME_PERSISTENT): the particles'
 * position x, y, direction sx, sy, weight q (int64, 2^F units), kind (0 null,
 * 1 real collision, 2 absorbed by a wall face) and location (cell c = ix + nx iy,
 * or wall face) after the last iteration, n = N (n_cells + n_b) entries each
 * (particle c N + k of cell c, (n_cells + b) N + k of wall face b at creation);
 * any pointer may be NULL.  Arrays in the problem's mem_kind.  Returns
 * IUGKP_E_INVALID_ARG for the emitter scheme. */
int iugkp_get_particles(iugkp_handle *h, double *x, double *y, double *sx, double *sy,
                        int64_t *q, int32_t *kind, int32_t *loc);

/* Persistent population: real collisions per cell N_rc [n_cells] and
 * absorptions per wall face N_b [n_b] (uint32) of the last iteration, and the
 * shares and carried remainders for the next one: w_c, r_c [n_cells],
 * w_b, r_b [n_b] (int64).  Any pointer may be NULL.  Arrays in the problem's
 * mem_kind. */
int iugkp_get_shares(iugkp_handle *h, uint32_t *n_rc, uint32_t *n_b, int64_t *w_c, int64_t *r_c,
                     int64_t *w_b, int64_t *r_b);

/* Relative residual history (host array, up to max_n entries); returns the count. */
int iugkp_get_residuals(iugkp_handle *h, double *res, int max_n);

int iugkp_get_stats(iugkp_handle *h, iugkp_stats *stats);

/* The particle step's form for the face-tallied iterations (the A4 march of
 * Sec. 3.1; how it is run is an implementation choice, not the paper's): 0 =
 * emitter tiles of 256 threads, 1 = emitter tiles of 512 threads, 2 = row
 * stripes, 3 = row stripes with the y faces in pieces (without null
 * collisions); -1 while the handle still measures them.  A 2D gray single solve
 * with the automatic march and the default block size times one face-tallied
 * iteration in each form (after an untimed first one) and keeps the fastest;
 * later handles of the same mesh, particles per emitter, null-collision
 * setting and free path in cells (to half an octave) start with it.  Every
 * form gives the same tallies bit for bit.  ms (NULL or host float[4]): the
 * measured particle-step milliseconds per form, -1 where not measured.
 * Returns 0, or IUGKP_E_INVALID_ARG for a NULL handle. */
int iugkp_march_tuning(iugkp_handle *h, int *form, float *ms);

/* Adjoint of the steady state reached by this handle (an addition to the
 * paper, which has no adjoint): given dL/dT per cell for a loss L(T), the
 * gradient of L with respect to every wall face's temperature and every
 * cell's source S.  Needs rng_mode CRN (the particle paths of slot rng_epoch)
 * and a uniform relaxation time; at most 65536 particles per emitter.
 * With fixed counters one iteration is linear in the emission energies,
 *   D = T_cc G_cells + T_cw G_walls   (T_xe = share of emitter e's particles
 *                                      ending in cell x),
 * so with psi = (I - T_cc^T)^-1 dL/dD the gradients are T_cc^T psi (source)
 * and T_cw^T psi (walls), chained through G_src = 2^F S V tau_min and
 * G_f = 2^F C (T_f - t_ref) lambda_min A_f / 4.  T^T psi at an emitter is the
 * mean of psi over the cells where its particles end: the forward paths
 * traced again and used in reverse.  psi is iterated as psi <- T^T psi + u
 * (with the handle's diffusion correction when newton is on) until the
 * relative change ||psi' - psi|| / ||first change|| < tol, at most max_iters
 * passes.  dLdT [n_cells] is read and grad_wall [n_b], grad_source [n_cells]
 * (either may be NULL) are written in the problem's mem_kind; *iters_out
 * (optional) = passes.  Returns IUGKP_OK, IUGKP_W_NOT_CONVERGED (gradients
 * written from the last psi), or an error: INVALID_ARG (arguments, FRESH
 * mode, varying tau, N > 65536), NOMEM, DEVICE, CG_BREAKDOWN,
 * CG_NOT_CONVERGED, NONFINITE.  Enqueued on the handle's stream and
 * synchronised before returning. */
int iugkp_adjoint(iugkp_handle *h, const double *dLdT, double *grad_wall, double *grad_source,
                  int max_iters, double tol, int *iters_out);

/* Per-iteration diffusion coefficient of the flat-cell kernel used by the Newton
 * operator when none is given: half the second moment of one cell-to-cell jump,
 * D_eff = (lam delta / 2) (1/2 + 2 sum_{j>=1} E_3(j delta / lam)); tends to
 * lam^2 / 3 for lam >> delta and lam delta / 4 for lam << delta.  Host function. */
double iugkp_d_eff(double lam, double delta);

/* The increment equation of the Newton step (Sec. 3.3: the diffusion-type
 * operator div(-kappa grad dT) applied to the energy increment), solved on its
 * own: A x = b with A the conservative 3-point (1D) or 5-point (2D) operator
 * -div(D grad) of the nx x ny mesh (cell c = ix + nx iy, sizes dx, dy),
 * harmonic-mean face conductances 2 D_a D_b / (D_a + D_b) / delta^2 and Robin
 * walls D / (delta (delta / 2 + 2 lambda / 3)) with lambda = vg tau, in the
 * per-iteration units of iugkp_solve.  Plain FP64 CG from x = 0 (single
 * reduction form of Chronopoulos and Gear, dot products in the fixed order of
 * blocks of 256), stopped when (r, r) <= tol^2 (b, b) or after max_iters
 * iterations: the same iterates, bit for bit, as the CG inside iugkp_step.
 * tau, D_x, D_y (2D only; NULL in 1D), b: [nx ny] device arrays, read only;
 * x: [nx ny] device array, written.  *iters_out (optional, host) = CG
 * iterations.  Work is issued on `stream` and completed before return; the
 * library allocates its scratch (operator, CG vectors, partials) for the call
 * and frees it before returning.  Returns IUGKP_OK, INVALID_ARG, NOMEM, DEVICE,
 * CG_BREAKDOWN or CG_NOT_CONVERGED (x then holds the last iterate). */
int iugkp_diffusion_solve(int dim, int nx, int ny, double dx, double dy, double vg,
                          const double *tau, const double *D_x, const double *D_y,
                          const double *b, double *x, double tol, int max_iters, int *iters_out,
                          void *stream);

/* iugkp_diffusion_solve without any allocation, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid it).  Same arguments, results (bit for bit) and
 * errors as iugkp_diffusion_solve; its scratch is a fixed 8 MiB array in
 * device memory, one per GPU, held until the process ends (enough for 65536
 * cells; a mesh whose scratch does not fit returns IUGKP_E_INVALID_ARG before
 * any device work).  It calls no hipMalloc, hipFree or other allocating
 * routine.  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (other threads, or other streams before this one's work is
 * complete) race; the call completes its work before returning. */
int iugkp_diffusion_solve_noalloc(int dim, int nx, int ny, double dx, double dy, double vg,
                                  const double *tau, const double *D_x, const double *D_y,
                                  const double *b, double *x, double tol, int max_iters,
                                  int *iters_out, void *stream);

/* Batched solves: n independent problems advanced together, one launch per phase
 * for all of them (the particle step over the emitter tiles of every instance,
 * one workgroup per instance for the Newton CG), the per-iteration sequence
 * captured once in a HIP graph on a stream of the batch's own (ordered after
 * `stream` with events) and replayed until every instance is done.  Every
 * instance's results are bitwise those of iugkp_solve on the same problem and
 * options, including the iteration at which it stops or fails.  All problems
 * must use the same mem_kind; outputs per instance as iugkp_solve (T_out[i]
 * required, qx_out[i], qy_out[i] may be NULL; qx_out, qy_out, stats may be NULL,
 * stats otherwise an array of n).  iugkp_batch_solve may be called once per batch;
 * it returns the most severe per-instance status (the most negative error, else
 * IUGKP_W_NOT_CONVERGED, else IUGKP_OK); outputs are written for every instance
 * that did not fail, and stats[i].status holds each instance's own status. */
int iugkp_batch_create(const iugkp_problem *const *problems,
                       const iugkp_options *const *options, int n, void *stream,
                       iugkp_batch **out);
int iugkp_batch_solve(iugkp_batch *b, double *const *T_out, double *const *qx_out,
                      double *const *qy_out, iugkp_stats *stats);
void iugkp_batch_destroy(iugkp_batch *b);
/* Tile edges of a batch's particle step (cells per side of an emitter tile,
 * 8 or 16; the A4 march of Sec. 3.1 run over every instance's tiles in one
 * launch): edges (host int[n]) receives each instance's.  An instance whose
 * class (mesh, particles per emitter, null collisions, free path in cells to
 * half an octave) no earlier batch of the process measured runs its second
 * replay with 8 and its third with 16, the device timing each workgroup, and
 * keeps the edge with the smaller device time per flight; the process keeps
 * the choice for the class.  The tallies do not depend on the tiles.
 * Returns 0, or IUGKP_E_INVALID_ARG for NULL arguments. */
int iugkp_batch_tiles(iugkp_batch *b, int *edges);

/* The autotuner of the batch's multigrid CG pool.  Before every replay the
 * library picks each multigrid instance's group of workgroups from a model of
 * one CG iteration, per_iter_us + per_cell_us * cells / group microseconds,
 * fitted to the measured duration of every multigrid job so far in this
 * process (the fit is kept for later batches); results do not depend on the
 * groups.  Writes the current fit (either pointer may be NULL) and, when
 * groups is not NULL, groups[i] = the group size of instance i in the last
 * replay (0 without a Newton step; plain-CG instances keep their fixed group).
 * Host pointers.  Returns IUGKP_OK or IUGKP_E_INVALID_ARG. */
int iugkp_batch_tuning(iugkp_batch *b, double *per_iter_us, double *per_cell_us, int *groups);

const char *iugkp_strerror(int code);
const char *iugkp_last_error(void);

/* ---- device building blocks, exposed for bitwise verification ----
 * All pointers are device pointers; work is issued on `stream` and completed
 * before return.
 * iugkp_dev_philox: out[4i..4i+3] = Philox4x32-10(counter = ctr[4i..4i+3], key). */
int iugkp_dev_philox(const uint32_t *ctr, uint32_t key0, uint32_t key1, uint32_t *out,
                     int64_t n, void *stream);
/* iugkp_dev_math: op 0 = log(x), 1 = cos(2 pi x) for x in [0,1), 2 = sqrt(x),
 * 3 = x / y, 4 = (double) of the int64 bits of x, 5 = rint(ldexp(x, k)) as int64 bits
 * with k = (int)y, 6 = exp(-x) for x >= 0 (the expected-value estimator's);
 * out[i] = op(x[i], y[i]). */
int iugkp_dev_math(int op, const double *x, const double *y, double *out, int64_t n,
                   void *stream);
/* iugkp_dev_segments: the closed-form segment walk used when no face is tallied,
 * on a dim/nx/ny/dx/dy mesh.  rays[7i..7i+6] = x0, y0, ix, iy (cell of the start
 * point, as doubles), sx, sy, ell; out[3i..3i+2] = 1 if a boundary face absorbs
 * the segment else 0, that face's wall index or the final cell ix + nx iy, and
 * the number of faces crossed (the wall face included). */
/* iugkp_dev_atomics: the tally-throughput ceilings the particle step is held
 * against.  n_threads (a multiple of 256) threads each add 1 to per_thread
 * pseudo-random int64 words: of a global array of n_words (lds = 0; 4096 <=
 * n_words <= 2^28, allocated here) or of a 4096-word LDS array per workgroup
 * (lds = 1).  *ms_out = the second of two identical launches (HIP events);
 * the rate is n_threads * per_thread / ms. */
int iugkp_dev_atomics(int lds, int64_t n_words, int64_t per_thread, int64_t n_threads,
                      double *ms_out, void *stream);

int iugkp_dev_segments(int dim, int nx, int ny, double dx, double dy, const double *rays,
                       int64_t n, int64_t *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif
