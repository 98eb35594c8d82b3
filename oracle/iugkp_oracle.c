/*
 * iugkp_oracle.c -- plain single-threaded FP64 CPU oracle of the IUGKP
 * steady gray phonon iteration (arXiv 2506.09465, Sections 2 and 3).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  It shares no code with the HIP library.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fPIC -shared.
 * Every floating-point operation is a plain IEEE-754 binary64 operation in
 * round-to-nearest-even, written in the order that the readings below fix.
 *
 * Readings of points the paper leaves open (each is a fixed rule here):
 *  R1 Walls are black, diffusely emitting equilibrium walls (the boundary
 *     distribution is an equilibrium, Sec. 2).  A wall face of area A at
 *     energy E_w emits E_w * lambda_min * A / 4 per iteration (the hemispherical
 *     flux E_w |V_g| / 4 times the common time scale tau_min), with
 *     cosine-law (Lambertian) directions: cosine to the inward normal sqrt(u).
 *  R2 Directions are 3D unit vectors (Sec. 2); in 1D and 2D the particle
 *     moves along the in-plane projection, the free path is the 3D length.
 *  R3 Stateless emitters: every cell and every wall face emits the same
 *     number N of particles per iteration from fresh samples (Sec. 3.1 steps
 *     (1)-(3) resample every particle from the local equilibrium).
 *  R4 Null collisions (Sec. 3.2) are followed in the same iteration (delta
 *     tracking): a rejected candidate tallies W and flies on from where it
 *     stopped with a new free path; the accepted one tallies both W and W^h.
 *     The macroscopic energy comes from W, re-emission from W^h (= D here).
 *  R5 Energies are int64 fixed-point numbers with scale 2^F; each emitter's
 *     integer energy is split over its N particles with an exact remainder,
 *     so every tally is an exact, order-independent integer sum.
 *  R6 Newton (Sec. 3.3) is read as E^{n+1} = E^{n+1/2} + A^{-1}(E^{n+1/2} - E^n),
 *     A the conservative 3/5-point discretisation of -div(D grad .) with
 *     Robin wall terms, D per cell given as problem data.
 *  R7 Residual: res_n = ||E^{n+1} - E^n||_2 / ||E^1 - E^0||_2.
 *  R19 The paper leaves the linear solver of the Newton step open.  Besides
 *     plain CG, A is solved by CG preconditioned with one multigrid V-cycle:
 *     cell-centred 2x2 (2 in 1D) aggregation down to one cell, piecewise
 *     constant transfers, the Galerkin coarse operator (again a 3/5-point
 *     operator: a coarse face sums the fine faces it covers), two damped
 *     Jacobi sweeps (omega 0.8) before and after the coarse correction, the
 *     correction scaled by 1.8, the one-cell level solved exactly.
 */
#include "iugkp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_SEGMENTS (1u << 20)   /* a flight's last allowed segment always ends real */
#define ORC_TWO62 4611686018427387904.0

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11.  Ten rounds of the 4x32 Philox S-box with the    */
/* published multipliers and Weyl key increments.                            */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform on [0,1): the top 27 bits of hi and top 26 bits of lo. */
double orc_u53(uint32_t hi, uint32_t lo)
{
  uint64_t m = ((uint64_t)(hi >> 5) << 26) | (uint64_t)(lo >> 6);
  return (double)m * 0x1p-53;
}

/* Draw d of particle k of emitter e in Philox slot s:
 * counter = (d, k, e, s), key = (seed low word, seed high word). */
static void orc_draw(uint64_t seed, uint32_t slot, uint32_t e, uint32_t k, uint32_t d,
                     double *u0, double *u1)
{
  uint32_t ctr[4] = {d, k, e, slot};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  *u0 = orc_u53(o[0], o[1]);
  *u1 = orc_u53(o[2], o[3]);
}

/* ------------------------------------------------------------------------ */
/* Natural logarithm from + - * / only (so that it is reproducible bit for   */
/* bit): x = m 2^e with m in (sqrt(2)/2, sqrt(2)], f = m - 1 (exact),        */
/* s = f / (2 + f), ln m = 2 atanh(s) = f - s (f - R) with                   */
/* R = 2 (z/3 + z^2/5 + ... + z^10/21), z = s^2 (the atanh Taylor series;    */
/* 2s = f - f s).  ln 2 is split in a high part with trailing zero bits and  */
/* a low part (Cody-Waite).  Defined for finite normal x > 0.                */
/* ------------------------------------------------------------------------ */
double orc_log(double x)
{
  const double ln2_hi = 6.93147180369123816490e-01;
  const double ln2_lo = 1.90821492927058770002e-10;
  const double sqrt2 = 1.41421356237309504880;
  uint64_t bits;
  memcpy(&bits, &x, sizeof bits);
  int e = (int)((bits >> 52) & 0x7ffu) - 1023;
  uint64_t mbits = (bits & 0x000fffffffffffffull) | (0x3ffull << 52);
  double m;
  memcpy(&m, &mbits, sizeof m);            /* m in [1, 2) */
  if (m > sqrt2) {
    m = m * 0.5;
    e = e + 1;
  }
  double f = m - 1.0;
  double s = f / (2.0 + f);
  double z = s * s;
  double R = 2.0 / 21.0;
  R = R * z + 2.0 / 19.0;
  R = R * z + 2.0 / 17.0;
  R = R * z + 2.0 / 15.0;
  R = R * z + 2.0 / 13.0;
  R = R * z + 2.0 / 11.0;
  R = R * z + 2.0 / 9.0;
  R = R * z + 2.0 / 7.0;
  R = R * z + 2.0 / 5.0;
  R = R * z + 2.0 / 3.0;
  R = R * z;
  double corr = s * (f - R);
  double de = (double)e;
  return de * ln2_hi + ((de * ln2_lo - corr) + f);
}

/* ------------------------------------------------------------------------ */
/* exp(-T), T >= 0, from + - * / and exact scaling: T = k ln2 + r with       */
/* k = rint(T / ln2), r = (T - k ln2_hi) - k ln2_lo (Cody-Waite, ln2_hi with */
/* trailing zero bits so k ln2_hi is exact), |r| <= ln2 / 2; exp(-r) by its  */
/* Taylor polynomial to degree 14 in Horner form (truncation below 2^-60),   */
/* scaled by 2^-k.  Returns 0 for T > 700 (far below any weight's unit).     */
/* ------------------------------------------------------------------------ */
double orc_expm(double T)
{
  const double ln2_hi = 6.93147180369123816490e-01;
  const double ln2_lo = 1.90821492927058770002e-10;
  const double inv_ln2 = 1.44269504088896338700e+00;
  if (T > 700.0) return 0.0;
  double kd = rint(T * inv_ln2);
  double r = (T - kd * ln2_hi) - kd * ln2_lo;
  double x = -r;
  double p = 1.0 / 87178291200.0;          /* 1/14! */
  p = p * x + 1.0 / 6227020800.0;
  p = p * x + 1.0 / 479001600.0;
  p = p * x + 1.0 / 39916800.0;
  p = p * x + 1.0 / 3628800.0;
  p = p * x + 1.0 / 362880.0;
  p = p * x + 1.0 / 40320.0;
  p = p * x + 1.0 / 5040.0;
  p = p * x + 1.0 / 720.0;
  p = p * x + 1.0 / 120.0;
  p = p * x + 1.0 / 24.0;
  p = p * x + 1.0 / 6.0;
  p = p * x + 0.5;
  p = p * x + 1.0;
  p = p * x + 1.0;
  return ldexp(p, -(int)kd);
}

/* ------------------------------------------------------------------------ */
/* cos(2 pi u) for u in [0, 1): exact quarter-turn reduction t = 4u,         */
/* q = floor(t), f = t - q, fold f > 1/2 to 1 - f, then Taylor polynomials   */
/* of sin and cos on [0, pi/4] (to x^19 and x^18).                           */
/* ------------------------------------------------------------------------ */
double orc_cos2pi(double u)
{
  const double half_pi = 1.57079632679489661923;
  double t = 4.0 * u;
  int q = (int)t;
  double f = t - (double)q;
  int folded = 0;
  double g = f;
  if (f > 0.5) {
    g = 1.0 - f;
    folded = 1;
  }
  double x = half_pi * g;
  double z = x * x;
  double c = -1.0 / 6402373705728000.0;        /* -1/18! */
  c = c * z + 1.0 / 20922789888000.0;          /*  1/16! */
  c = c * z - 1.0 / 87178291200.0;             /* -1/14! */
  c = c * z + 1.0 / 479001600.0;               /*  1/12! */
  c = c * z - 1.0 / 3628800.0;                 /* -1/10! */
  c = c * z + 1.0 / 40320.0;                   /*  1/8!  */
  c = c * z - 1.0 / 720.0;                     /* -1/6!  */
  c = c * z + 1.0 / 24.0;                      /*  1/4!  */
  c = c * z - 1.0 / 2.0;                       /* -1/2!  */
  c = c * z + 1.0;
  double s = -1.0 / 121645100408832000.0;      /* -1/19! */
  s = s * z + 1.0 / 355687428096000.0;         /*  1/17! */
  s = s * z - 1.0 / 1307674368000.0;           /* -1/15! */
  s = s * z + 1.0 / 6227020800.0;              /*  1/13! */
  s = s * z - 1.0 / 39916800.0;                /* -1/11! */
  s = s * z + 1.0 / 362880.0;                  /*  1/9!  */
  s = s * z - 1.0 / 5040.0;                    /* -1/7!  */
  s = s * z + 1.0 / 120.0;                     /*  1/5!  */
  s = s * z - 1.0 / 6.0;                       /* -1/3!  */
  s = s * z + 1.0;
  s = x * s;
  /* cos(f pi/2) and sin(f pi/2) */
  double cf = folded ? s : c;
  double sf = folded ? c : s;
  switch (q) {
    case 0: return cf;
    case 1: return -sf;
    case 2: return -cf;
    default: return sf;
  }
}

/* Vectorised probes of the building blocks (for element-wise comparisons). */
void orc_philox_batch(const uint32_t *ctr, uint64_t n, uint32_t k0, uint32_t k1, uint32_t *out)
{
  uint32_t key[2] = {k0, k1};
  for (uint64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

void orc_math_batch(int op, const double *x, const double *y, double *out, uint64_t n)
{
  for (uint64_t i = 0; i < n; ++i) {
    switch (op) {
      case 0: out[i] = orc_log(x[i]); break;
      case 1: out[i] = orc_cos2pi(x[i]); break;
      case 2: out[i] = sqrt(x[i]); break;
      case 3: out[i] = x[i] / y[i]; break;
      case 4: {
        int64_t v;
        memcpy(&v, &x[i], 8);
        out[i] = (double)v;
        break;
      }
      case 5: {
        int64_t v = (int64_t)rint(ldexp(x[i], (int)y[i]));
        memcpy(&out[i], &v, 8);
        break;
      }
      case 6: out[i] = orc_expm(x[i]); break;
      default: out[i] = 0.0;
    }
  }
}

/* Particle k's share of an emitter's integer energy G over n particles:
 * floor(G/n) plus one for the first (G - n floor(G/n)) particles. */
int64_t orc_split_weight(int64_t G, uint64_t n, uint64_t k)
{
  int64_t nn = (int64_t)n;
  int64_t base = G / nn;
  if ((G % nn) != 0 && G < 0) base -= 1;
  int64_t rem = G - base * nn;
  return base + ((int64_t)k < rem ? 1 : 0);
}

/* Fixed-order sum: zero-padded blocks of 256 in index order, each reduced by
 * halving strides (v[i] += v[i+s], s = 128, 64, ..., 1); the block sums are
 * reduced the same way, recursively, until one value is left. */
static double orc_tree256(const double *v, uint64_t n)
{
  double buf[256];
  for (uint64_t i = 0; i < 256; ++i) buf[i] = (i < n) ? v[i] : 0.0;
  for (int s = 128; s >= 1; s /= 2)
    for (int i = 0; i < s; ++i) buf[i] = buf[i] + buf[i + s];
  return buf[0];
}

double orc_tree_sum(const double *v, uint64_t n)
{
  if (n == 0) return 0.0;
  uint64_t nb = (n + 255) / 256;
  double *part = (double *)malloc(nb * sizeof(double));
  for (uint64_t b = 0; b < nb; ++b) {
    uint64_t len = n - 256 * b;
    if (len > 256) len = 256;
    part[b] = orc_tree256(v + 256 * b, len);
  }
  double r = (nb == 1) ? part[0] : orc_tree_sum(part, nb);
  free(part);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Problem set-up                                                            */
/* ------------------------------------------------------------------------ */
static int orc_nb(const orc_problem *p) { return 2 * p->ny + (p->dim == 2 ? 2 * p->nx : 0); }

static int orc_validate(const orc_problem *p)
{
  if (!p || !p->tau || !p->wall_T) return ORC_E_INVALID_ARG;
  if (p->dim != 1 && p->dim != 2) return ORC_E_INVALID_ARG;
  if (p->nx < 1 || p->ny < 1 || (p->dim == 1 && p->ny != 1)) return ORC_E_INVALID_ARG;
  if (!(p->dx > 0.0) || !(p->dy > 0.0) || !isfinite(p->dx) || !isfinite(p->dy))
    return ORC_E_INVALID_ARG;
  if (!(p->cv > 0.0) || !(p->vg > 0.0) || !isfinite(p->cv) || !isfinite(p->vg) ||
      !isfinite(p->t_ref))
    return ORC_E_INVALID_ARG;
  int nc = p->nx * p->ny;
  double tmin = INFINITY, tmax = 0.0;
  for (int c = 0; c < nc; ++c) {
    if (!(p->tau[c] > 0.0) || !isfinite(p->tau[c])) return ORC_E_INVALID_ARG;
    if (p->tau[c] < tmin) tmin = p->tau[c];
    if (p->tau[c] > tmax) tmax = p->tau[c];
  }
  if (tmax > 1e6 * tmin) return ORC_E_INVALID_ARG;
  for (int b = 0; b < orc_nb(p); ++b)
    if (!isfinite(p->wall_T[b])) return ORC_E_INVALID_ARG;
  if (p->T_init)
    for (int c = 0; c < nc; ++c)
      if (!isfinite(p->T_init[c])) return ORC_E_INVALID_ARG;
  if (p->source)
    for (int c = 0; c < nc; ++c)
      if (!isfinite(p->source[c])) return ORC_E_INVALID_ARG;
  return ORC_OK;
}

/* Scale exponent F = 62 - ceil(log2 B) with
 * B = 4 max(|E_wall|, |E_0|) (sum of cell volumes + lambda_min * (sum of wall areas) / 4),
 * the bound on one iteration's total |emission| times a safety factor 4.
 * With a volumetric source the energy level is raised by at most about
 * S_max tau_min times the number of iterations energy stays in the domain,
 * bounded by 1 + 3 (L / lambda_min)^2 (L the longer side): B uses
 * max(|E_wall|, |E_0|) + S_max tau_min (1 + 3 (L / lambda_min)^2) instead. */
int orc_fixed_exponent(const orc_problem *p, double *tau_min_out)
{
  int nc = p->nx * p->ny;
  double tmin = p->tau[0];
  for (int c = 1; c < nc; ++c)
    if (p->tau[c] < tmin) tmin = p->tau[c];
  if (tau_min_out) *tau_min_out = tmin;
  double lam_min = p->vg * tmin;
  double maxabs = 0.0;
  for (int b = 0; b < orc_nb(p); ++b) {
    double ew = fabs(p->cv * (p->wall_T[b] - p->t_ref));
    if (ew > maxabs) maxabs = ew;
  }
  if (p->T_init)
    for (int c = 0; c < nc; ++c) {
      double e0 = fabs(p->cv * (p->T_init[c] - p->t_ref));
      if (e0 > maxabs) maxabs = e0;
    }
  double vol = (double)nc * (p->dx * p->dy);
  double area = (p->dim == 2) ? ((2.0 * (double)p->ny) * p->dy + (2.0 * (double)p->nx) * p->dx)
                              : 2.0;
  double total = vol + (lam_min * area) / 4.0;
  double B = (4.0 * maxabs) * total;
  double smax = 0.0;
  if (p->source)
    for (int c = 0; c < nc; ++c)
      if (fabs(p->source[c]) > smax) smax = fabs(p->source[c]);
  if (smax > 0.0) {
    double L = (double)p->nx * p->dx;
    if (p->dim == 2 && (double)p->ny * p->dy > L) L = (double)p->ny * p->dy;
    double rl = L / lam_min;
    double esrc = (smax * tmin) * (1.0 + 3.0 * (rl * rl));
    B = (4.0 * (maxabs + esrc)) * total;
  }
  if (!(B > 0.0)) return 62;
  int e;
  double m = frexp(B, &e);          /* B = m 2^e, m in [0.5, 1) */
  int ceil_log2 = (m == 0.5) ? e - 1 : e;
  return 62 - ceil_log2;
}

/* ------------------------------------------------------------------------ */
/* State                                                                     */
/* ------------------------------------------------------------------------ */
struct orc_state {
  orc_problem p;
  orc_options o;
  double *tau, *wall_T, *diff_x, *diff_y;
  int nc, nb, ne, nfx, nfy;
  uint64_t N;
  int F;
  double tau_min, lam_min, V;
  double *ratio;       /* tau_min / tau_c */
  double *source;      /* volumetric source per cell or NULL */
  int64_t *Gs;         /* its emission per iteration, fixed point */
  double *E;           /* E^n */
  double *E_half;      /* W / V of the last iteration */
  int64_t *G;          /* emission energies of the next iteration, per emitter */
  int64_t *D, *W, *Phix, *Phiy, *B;
  double *gx, *gy, *diag;
  int has_null;        /* some tau_c > tau_min */
  uint32_t iter;
  double d0, res;
  double res_p1, res_p2;   /* residuals of the two preceding iterations (+inf: none) */
  double *res_hist;
  int res_cap;
  uint64_t flights, segments, crossings, tot_flights, tot_segments, tot_crossings;
  int cg_last, cg_total;
};

typedef struct {
  int64_t *D, *W, *Phix, *Phiy, *B;
  int end;             /* where the last particle ended: cell, or -1 - wall face */
  int faces;
  uint64_t crossings;
  int32_t *events;     /* optional crossing log */
  int n_events, max_events;
  int bad;             /* an expected-candidate deposit beyond the 2^62 range */
} orc_tally;

/* int64 of round-to-nearest-even(ldexp(v, F)); returns 0 and sets *ok = 0 on overflow. */
static int64_t orc_to_fixed(double v, int F, int *ok)
{
  double s = ldexp(v, F);
  if (!(fabs(s) <= ORC_TWO62)) {
    *ok = 0;
    return 0;
  }
  return (int64_t)rint(s);
}

/* a + b for |a|, |b| <= 2^62 without signed overflow; *ok = 0 if |a + b| > 2^62 */
static int64_t orc_add(int64_t a, int64_t b, int *ok)
{
  int64_t r = (int64_t)((uint64_t)a + (uint64_t)b);
  if (r > ((int64_t)1 << 62) || r < -((int64_t)1 << 62)) *ok = 0;
  return r;
}

static int orc_check_budget(const int64_t *G, int n)
{
  uint64_t acc = 0;
  const uint64_t lim = (uint64_t)1 << 62;
  for (int i = 0; i < n; ++i) {
    uint64_t a = (G[i] < 0) ? (uint64_t)0 - (uint64_t)G[i] : (uint64_t)G[i];
    if (a > lim) return 0;
    acc += a;
    if (acc > lim) return 0;
  }
  return 1;
}

/* Newton operator (reading R6): face conductances and diagonal.
 * Interior face between cells a|b: H(D_a, D_b) / d^2, H the harmonic mean;
 * wall face of cell c: D_c / (d (d/2 + 2 lambda_c / 3)), lambda_c = |V_g| tau_c
 * (extrapolated wall distance 2 lambda / 3). */
int orc_newton_operator(const orc_problem *p, double *gx, double *gy, double *diag)
{
  int nx = p->nx, ny = p->ny;
  if (!p->diff_x || (p->dim == 2 && !p->diff_y)) return ORC_E_INVALID_ARG;
  for (int iy = 0; iy < ny; ++iy)
    for (int kx = 0; kx <= nx; ++kx) {
      double g;
      if (kx == 0 || kx == nx) {
        int c = iy * nx + (kx == 0 ? 0 : nx - 1);
        double lam = p->vg * p->tau[c];
        double den = p->dx * (p->dx / 2.0 + (2.0 * lam) / 3.0);
        g = p->diff_x[c] / den;
      } else {
        double a = p->diff_x[iy * nx + kx - 1], b = p->diff_x[iy * nx + kx];
        double h = ((2.0 * a) * b) / (a + b);
        g = h / (p->dx * p->dx);
      }
      gx[iy * (nx + 1) + kx] = g;
    }
  if (p->dim == 2)
    for (int ky = 0; ky <= ny; ++ky)
      for (int ix = 0; ix < nx; ++ix) {
        double g;
        if (ky == 0 || ky == ny) {
          int c = (ky == 0 ? 0 : ny - 1) * nx + ix;
          double lam = p->vg * p->tau[c];
          double den = p->dy * (p->dy / 2.0 + (2.0 * lam) / 3.0);
          g = p->diff_y[c] / den;
        } else {
          double a = p->diff_y[(ky - 1) * nx + ix], b = p->diff_y[ky * nx + ix];
          double h = ((2.0 * a) * b) / (a + b);
          g = h / (p->dy * p->dy);
        }
        gy[ky * nx + ix] = g;
      }
  for (int iy = 0; iy < ny; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      double d = gx[iy * (nx + 1) + ix] + gx[iy * (nx + 1) + ix + 1];
      if (p->dim == 2) {
        d = d + gy[iy * nx + ix];
        d = d + gy[(iy + 1) * nx + ix];
      }
      diag[iy * nx + ix] = d;
    }
  return ORC_OK;
}

static void orc_apply(const orc_problem *p, const double *gx, const double *gy,
                      const double *diag, const double *x, double *y)
{
  int nx = p->nx, ny = p->ny;
  for (int iy = 0; iy < ny; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      int c = iy * nx + ix;
      double acc = diag[c] * x[c];
      if (ix > 0) acc = acc - gx[iy * (nx + 1) + ix] * x[c - 1];
      if (ix < nx - 1) acc = acc - gx[iy * (nx + 1) + ix + 1] * x[c + 1];
      if (p->dim == 2) {
        if (iy > 0) acc = acc - gy[iy * nx + ix] * x[c - nx];
        if (iy < ny - 1) acc = acc - gy[(iy + 1) * nx + ix] * x[c + nx];
      }
      y[c] = acc;
    }
}

static double orc_dot(const double *a, const double *b, int n, double *tmp)
{
  for (int i = 0; i < n; ++i) tmp[i] = a[i] * b[i];
  return orc_tree_sum(tmp, (uint64_t)n);
}

/* Conjugate gradients in the single-reduction form of Chronopoulos and Gear
 * (J. Comput. Appl. Math. 25, 1989): with w = A r and s = A p carried by
 * recurrence, both inner products of an iteration, (r, r) and (w, r), come
 * from the same vectors, so one global reduction per iteration suffices.
 *   x = 0, r = b, w = A r, gamma = (r, r), delta = (w, r), alpha = gamma / delta
 *   repeat: p = r + beta p, s = w + beta s (p = r, s = w the first time)
 *           x = x + alpha p, r = r - alpha s, w = A r
 *           gamma' = (r, r), delta = (w, r); stop if gamma' <= tol^2 (b, b)
 *           beta = gamma' / gamma, alpha = gamma' / (delta - beta gamma' / alpha)
 * In exact arithmetic the iterates are those of Hestenes-Stiefel CG. */
int orc_cg(const orc_problem *p, const double *gx, const double *gy, const double *diag,
           const double *b, double *x, double tol, int max_iters, int *iters_out)
{
  int n = p->nx * p->ny;
  double *r = (double *)malloc(sizeof(double) * n);
  double *w = (double *)malloc(sizeof(double) * n);
  double *pp = (double *)malloc(sizeof(double) * n);
  double *sv = (double *)malloc(sizeof(double) * n);
  double *tmp = (double *)malloc(sizeof(double) * n);
  for (int i = 0; i < n; ++i) {
    x[i] = 0.0;
    r[i] = b[i];
  }
  orc_apply(p, gx, gy, diag, r, w);
  double gamma = orc_dot(r, r, n, tmp);
  double delta = orc_dot(w, r, n, tmp);
  double thr = (tol * tol) * gamma;
  int it = 0, rc = ORC_OK, done = (gamma == 0.0);
  double alpha = 0.0, beta = 0.0;
  if (!done) {
    if (!(delta > 0.0)) rc = ORC_E_CG_BREAKDOWN;
    else alpha = gamma / delta;
  }
  while (!done && rc == ORC_OK && it < max_iters) {
    for (int i = 0; i < n; ++i) {
      pp[i] = (it == 0) ? r[i] : r[i] + beta * pp[i];
      sv[i] = (it == 0) ? w[i] : w[i] + beta * sv[i];
      x[i] = x[i] + alpha * pp[i];
      r[i] = r[i] - alpha * sv[i];
    }
    orc_apply(p, gx, gy, diag, r, w);
    double gamma_new = orc_dot(r, r, n, tmp);
    delta = orc_dot(w, r, n, tmp);
    ++it;
    if (gamma_new <= thr) {
      done = 1;
      break;
    }
    beta = gamma_new / gamma;
    double t = beta * gamma_new;
    t = t / alpha;
    double den = delta - t;
    if (!(den > 0.0)) {
      rc = ORC_E_CG_BREAKDOWN;
      break;
    }
    alpha = gamma_new / den;
    gamma = gamma_new;
  }
  if (rc == ORC_OK && !done) rc = ORC_E_CG_NOT_CONVERGED;
  if (iters_out) *iters_out = it;
  free(r);
  free(w);
  free(pp);
  free(sv);
  free(tmp);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Multigrid V-cycle preconditioner (reading R19).                          */
/* Level k+1 aggregates 2x2 cells of level k (NX = ceil(nx/2), NY =          */
/* ceil(ny/2)); with P the piecewise-constant prolongation, the Galerkin     */
/* operator P^T A P keeps the 3/5-point form: the coarse face between two    */
/* aggregates carries the sum of the fine faces between them (a wall face the */
/* sum of the fine wall faces), and the diagonal is again the sum of the     */
/* cell's four faces.  The V-cycle is symmetric (the same sweeps before and  */
/* after the correction, R = P^T), so M is a valid CG preconditioner.        */
/* ------------------------------------------------------------------------ */
#define ORC_MG_OMEGA 0.8
#define ORC_MG_SCALE 1.8
#define ORC_MG_MAX_LEVELS 64

typedef struct {
  int nx, ny, has_y;
  const double *gx, *gy, *diag;
  double *own[3];   /* coarse levels: the arrays allocated here */
} orc_mg_level;

typedef struct {
  int L;
  orc_mg_level lv[ORC_MG_MAX_LEVELS];
} orc_mg;

static void orc_mg_free(orc_mg *h)
{
  for (int k = 0; k < h->L; ++k)
    for (int j = 0; j < 3; ++j) free(h->lv[k].own[j]);
}

static void orc_mg_build(const orc_problem *p, const double *gx, const double *gy,
                         const double *diag, orc_mg *h)
{
  memset(h, 0, sizeof(*h));
  h->L = 1;
  h->lv[0].nx = p->nx;
  h->lv[0].ny = p->ny;
  h->lv[0].has_y = (p->dim == 2);
  h->lv[0].gx = gx;
  h->lv[0].gy = gy;
  h->lv[0].diag = diag;
  while (!(h->lv[h->L - 1].nx == 1 && h->lv[h->L - 1].ny == 1)) {
    const orc_mg_level *f = &h->lv[h->L - 1];
    orc_mg_level *c = &h->lv[h->L];
    const int nx = f->nx, ny = f->ny, NX = (nx + 1) / 2, NY = (ny + 1) / 2;
    c->nx = NX;
    c->ny = NY;
    c->has_y = f->has_y;
    double *Gx = (double *)malloc(sizeof(double) * (size_t)NY * (NX + 1));
    double *Gy = c->has_y ? (double *)malloc(sizeof(double) * (size_t)(NY + 1) * NX) : NULL;
    double *Dg = (double *)malloc(sizeof(double) * (size_t)NY * NX);
    for (int J = 0; J < NY; ++J)
      for (int K = 0; K <= NX; ++K) {
        const int k = (2 * K < nx) ? 2 * K : nx;   /* the fine face under coarse face K */
        const double a = f->gx[(2 * J) * (nx + 1) + k];
        const double b = (2 * J + 1 < ny) ? f->gx[(2 * J + 1) * (nx + 1) + k] : 0.0;
        Gx[J * (NX + 1) + K] = a + b;
      }
    if (c->has_y)
      for (int K = 0; K <= NY; ++K)
        for (int I = 0; I < NX; ++I) {
          const int k = (2 * K < ny) ? 2 * K : ny;
          const double a = f->gy[k * nx + 2 * I];
          const double b = (2 * I + 1 < nx) ? f->gy[k * nx + 2 * I + 1] : 0.0;
          Gy[K * NX + I] = a + b;
        }
    for (int J = 0; J < NY; ++J)
      for (int I = 0; I < NX; ++I) {
        double d = Gx[J * (NX + 1) + I] + Gx[J * (NX + 1) + I + 1];
        if (c->has_y) {
          d = d + Gy[J * NX + I];
          d = d + Gy[(J + 1) * NX + I];
        }
        Dg[J * NX + I] = d;
      }
    c->gx = c->own[0] = Gx;
    c->gy = c->own[1] = Gy;
    c->diag = c->own[2] = Dg;
    h->L += 1;
  }
}

/* (A_k v)_c in the order diag v_c - g_l v_{c-1} - g_r v_{c+1} - g_dn v_{c-nx}
 * - g_up v_{c+nx}, absent neighbours skipped (the fine operator's order). */
static double orc_mg_apply(const orc_mg_level *l, const double *v, int c)
{
  const int nx = l->nx, ny = l->ny, iy = c / nx, ix = c - iy * nx;
  double acc = l->diag[c] * v[c];
  if (ix > 0) acc = acc - l->gx[iy * (nx + 1) + ix] * v[c - 1];
  if (ix < nx - 1) acc = acc - l->gx[iy * (nx + 1) + ix + 1] * v[c + 1];
  if (iy > 0) acc = acc - l->gy[iy * nx + ix] * v[c - nx];
  if (iy < ny - 1) acc = acc - l->gy[(iy + 1) * nx + ix] * v[c + nx];
  return acc;
}

/* one damped Jacobi sweep y = x + omega (b - A x) / diag */
static void orc_mg_sweep(const orc_mg_level *l, const double *b, const double *x, double *y)
{
  const int n = l->nx * l->ny;
  for (int c = 0; c < n; ++c) {
    const double t = b[c] - orc_mg_apply(l, x, c);
    y[c] = x[c] + (ORC_MG_OMEGA * t) / l->diag[c];
  }
}

/* x = V-cycle of level k applied to b (zero initial guess) */
static void orc_mg_vcycle(const orc_mg *h, int k, const double *b, double *x)
{
  const orc_mg_level *l = &h->lv[k];
  const int nx = l->nx, ny = l->ny, n = nx * ny;
  if (k == h->L - 1) {                       /* one cell: exact */
    x[0] = b[0] / l->diag[0];
    return;
  }
  const orc_mg_level *cl = &h->lv[k + 1];
  const int NX = cl->nx, NY = cl->ny, N = NX * NY;
  double *x0 = (double *)calloc((size_t)n, sizeof(double));
  double *x1 = (double *)malloc(sizeof(double) * (size_t)n);
  double *res = (double *)malloc(sizeof(double) * (size_t)n);
  double *B = (double *)malloc(sizeof(double) * (size_t)N);
  double *e = (double *)malloc(sizeof(double) * (size_t)N);
  orc_mg_sweep(l, b, x0, x1);                /* pre-smoothing: x0 = 0 -> x1 -> x0 */
  orc_mg_sweep(l, b, x1, x0);
  for (int c = 0; c < n; ++c) res[c] = b[c] - orc_mg_apply(l, x0, c);
  /* restriction R = P^T: an aggregate sums its children's residuals,
   * (r(2I,2J) + r(2I+1,2J)) + (r(2I,2J+1) + r(2I+1,2J+1)), absent children 0 */
  for (int J = 0; J < NY; ++J)
    for (int I = 0; I < NX; ++I) {
      double q[4];
      for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) {
          const int ix = 2 * I + i, iy = 2 * J + j;
          q[2 * j + i] = (ix < nx && iy < ny) ? res[iy * nx + ix] : 0.0;
        }
      B[J * NX + I] = (q[0] + q[1]) + (q[2] + q[3]);
    }
  orc_mg_vcycle(h, k + 1, B, e);
  /* scaled coarse correction, then post-smoothing */
  for (int c = 0; c < n; ++c) {
    const int iy = c / nx, ix = c - iy * nx;
    x1[c] = x0[c] + ORC_MG_SCALE * e[(iy / 2) * NX + ix / 2];
  }
  orc_mg_sweep(l, b, x1, x0);
  orc_mg_sweep(l, b, x0, x);
  free(x0);
  free(x1);
  free(res);
  free(B);
  free(e);
}

int orc_mg_precondition(const orc_problem *p, const double *gx, const double *gy,
                        const double *diag, const double *b, double *x)
{
  orc_mg h;
  orc_mg_build(p, gx, gy, diag, &h);
  orc_mg_vcycle(&h, 0, b, x);
  orc_mg_free(&h);
  return ORC_OK;
}

int orc_mg_levels(const orc_problem *p, int *nx_out, int *ny_out, int max_levels)
{
  int nx = p->nx, ny = p->ny, L = 0;
  for (;;) {
    if (L < max_levels) {
      nx_out[L] = nx;
      ny_out[L] = ny;
    }
    ++L;
    if (nx == 1 && ny == 1) break;
    nx = (nx + 1) / 2;
    ny = (ny + 1) / 2;
  }
  return L;
}

/* Preconditioned CG in the single-reduction form (Chronopoulos and Gear) with
 * u = M r, w = A u and s = A p carried by recurrence; one reduction of the
 * three products (r, u), (w, u), (r, r) per iteration.
 *   x = 0, r = b, u = M r, w = A u, gamma = (r, u), delta = (w, u),
 *   alpha = gamma / delta
 *   repeat: p = u + beta p, s = w + beta s (p = u, s = w the first time)
 *           x = x + alpha p, r = r - alpha s, u = M r, w = A u
 *           gamma' = (r, u), delta = (w, u), rho = (r, r); stop if rho <= tol^2 (b, b)
 *           beta = gamma' / gamma, alpha = gamma' / (delta - beta gamma' / alpha)
 * In exact arithmetic the iterates are those of preconditioned CG. */
int orc_pcg_mg(const orc_problem *p, const double *gx, const double *gy, const double *diag,
               const double *b, double *x, double tol, int max_iters, int *iters_out)
{
  const int n = p->nx * p->ny;
  orc_mg h;
  orc_mg_build(p, gx, gy, diag, &h);
  const orc_mg_level *l0 = &h.lv[0];
  double *r = (double *)malloc(sizeof(double) * n);
  double *u = (double *)malloc(sizeof(double) * n);
  double *w = (double *)malloc(sizeof(double) * n);
  double *pp = (double *)malloc(sizeof(double) * n);
  double *sv = (double *)malloc(sizeof(double) * n);
  double *tmp = (double *)malloc(sizeof(double) * n);
  for (int i = 0; i < n; ++i) {
    x[i] = 0.0;
    r[i] = b[i];
  }
  const double rho0 = orc_dot(r, r, n, tmp);
  const double thr = (tol * tol) * rho0;
  int it = 0, rc = ORC_OK, done = (rho0 == 0.0);
  double alpha = 0.0, beta = 0.0, gamma = 0.0, delta = 0.0;
  if (!done) {
    orc_mg_vcycle(&h, 0, r, u);
    for (int c = 0; c < n; ++c) w[c] = orc_mg_apply(l0, u, c);
    gamma = orc_dot(r, u, n, tmp);
    delta = orc_dot(w, u, n, tmp);
    if (!(delta > 0.0)) rc = ORC_E_CG_BREAKDOWN;
    else alpha = gamma / delta;
  }
  while (!done && rc == ORC_OK && it < max_iters) {
    for (int i = 0; i < n; ++i) {
      pp[i] = (it == 0) ? u[i] : u[i] + beta * pp[i];
      sv[i] = (it == 0) ? w[i] : w[i] + beta * sv[i];
      x[i] = x[i] + alpha * pp[i];
      r[i] = r[i] - alpha * sv[i];
    }
    orc_mg_vcycle(&h, 0, r, u);
    for (int c = 0; c < n; ++c) w[c] = orc_mg_apply(l0, u, c);
    const double gamma_new = orc_dot(r, u, n, tmp);
    delta = orc_dot(w, u, n, tmp);
    const double rho = orc_dot(r, r, n, tmp);
    ++it;
    if (rho <= thr) {
      done = 1;
      break;
    }
    beta = gamma_new / gamma;
    double t = beta * gamma_new;
    t = t / alpha;
    const double den = delta - t;
    if (!(den > 0.0)) {
      rc = ORC_E_CG_BREAKDOWN;
      break;
    }
    alpha = gamma_new / den;
    gamma = gamma_new;
  }
  if (rc == ORC_OK && !done) rc = ORC_E_CG_NOT_CONVERGED;
  if (iters_out) *iters_out = it;
  free(r);
  free(u);
  free(w);
  free(pp);
  free(sv);
  free(tmp);
  orc_mg_free(&h);
  return rc;
}

/* The Newton step's linear solve with the configured preconditioner. */
static int orc_newton_solve(const orc_problem *p, const orc_options *o, const double *gx,
                            const double *gy, const double *diag, const double *b, double *x,
                            int *iters_out)
{
  if (o->cg_precond == ORC_PRECOND_MG)
    return orc_pcg_mg(p, gx, gy, diag, b, x, o->cg_tol, o->cg_max_iters, iters_out);
  return orc_cg(p, gx, gy, diag, b, x, o->cg_tol, o->cg_max_iters, iters_out);
}

void orc_destroy(orc_state *s)
{
  if (!s) return;
  free(s->tau); free(s->wall_T); free(s->diff_x); free(s->diff_y);
  free(s->ratio); free(s->E); free(s->E_half); free(s->G);
  free(s->D); free(s->W); free(s->Phix); free(s->Phiy); free(s->B);
  free(s->gx); free(s->gy); free(s->diag); free(s->res_hist);
  free(s->source); free(s->Gs);
  free(s);
}

static double *orc_dup(const double *a, int n)
{
  if (!a) return NULL;
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  memcpy(r, a, sizeof(double) * (size_t)n);
  return r;
}

int orc_create(const orc_problem *p, const orc_options *o, orc_state **out)
{
  *out = NULL;
  int rc = orc_validate(p);
  if (rc) return rc;
  if (p->n_bands > 1) return ORC_E_INVALID_ARG;   /* bands: orc_bands_create */
  if (!o || o->particles_per_iter < 1 || o->max_iters < 0 || o->avg_iters < 0 ||
      (o->estimator != ORC_EST_ANALOG && o->estimator != ORC_EST_EXPECTED) ||
      (o->cg_precond != ORC_PRECOND_NONE && o->cg_precond != ORC_PRECOND_MG))
    return ORC_E_INVALID_ARG;
  if (o->newton && (!p->diff_x || (p->dim == 2 && !p->diff_y) || !(o->cg_tol > 0.0) ||
                    o->cg_max_iters < 1))
    return ORC_E_INVALID_ARG;
  orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
  s->p = *p;
  s->o = *o;
  s->nc = p->nx * p->ny;
  s->nb = orc_nb(p);
  s->ne = s->nc + s->nb;
  s->nfx = p->ny * (p->nx + 1);
  s->nfy = (p->dim == 2) ? (p->ny + 1) * p->nx : 0;
  s->tau = orc_dup(p->tau, s->nc);
  s->wall_T = orc_dup(p->wall_T, s->nb);
  s->diff_x = orc_dup(p->diff_x, s->nc);
  s->diff_y = orc_dup(p->diff_y, s->nc);
  s->p.tau = s->tau;
  s->p.wall_T = s->wall_T;
  s->p.diff_x = s->diff_x;
  s->p.diff_y = s->diff_y;
  s->p.T_init = NULL;
  s->source = orc_dup(p->source, s->nc);
  s->p.source = s->source;
  s->N = o->particles_per_iter / (uint64_t)s->ne;
  if (s->N < 1) s->N = 1;
  s->F = orc_fixed_exponent(p, &s->tau_min);
  s->lam_min = p->vg * s->tau_min;
  s->V = p->dx * p->dy;
  s->ratio = (double *)malloc(sizeof(double) * s->nc);
  s->E = (double *)malloc(sizeof(double) * s->nc);
  s->E_half = (double *)calloc((size_t)s->nc, sizeof(double));
  s->G = (int64_t *)calloc((size_t)s->ne, sizeof(int64_t));
  s->D = (int64_t *)calloc((size_t)s->nc, sizeof(int64_t));
  s->W = (int64_t *)calloc((size_t)s->nc, sizeof(int64_t));
  s->Phix = (int64_t *)calloc((size_t)s->nfx, sizeof(int64_t));
  s->Phiy = (int64_t *)calloc((size_t)(s->nfy ? s->nfy : 1), sizeof(int64_t));
  s->B = (int64_t *)calloc((size_t)s->nb, sizeof(int64_t));
  s->res_cap = o->max_iters + o->avg_iters + 8;
  s->res_hist = (double *)calloc((size_t)s->res_cap, sizeof(double));
  s->res_p1 = s->res_p2 = HUGE_VAL;
  for (int c = 0; c < s->nc; ++c) {
    s->ratio[c] = s->tau_min / s->tau[c];
    if (s->ratio[c] != 1.0) s->has_null = 1;
    double T0 = p->T_init ? p->T_init[c] : p->t_ref;
    s->E[c] = p->cv * (T0 - p->t_ref);
  }
  int ok = 1;
  /* source emission per iteration: S V tau_min */
  s->Gs = (int64_t *)calloc((size_t)s->nc, sizeof(int64_t));
  if (s->source)
    for (int c = 0; c < s->nc; ++c)
      s->Gs[c] = orc_to_fixed((s->source[c] * s->V) * s->tau_min, s->F, &ok);
  /* cell emission: (E V) tau_min/tau (Sec. 3.2, candidate rate tau_min), plus the source */
  for (int c = 0; c < s->nc; ++c)
    s->G[c] = orc_add(orc_to_fixed((s->E[c] * s->V) * s->ratio[c], s->F, &ok), s->Gs[c], &ok);
  /* wall emission, reading R1 */
  for (int b = 0; b < s->nb; ++b) {
    double A = (b < 2 * p->ny) ? p->dy : p->dx;
    double ew = p->cv * (s->wall_T[b] - p->t_ref);
    s->G[s->nc + b] = orc_to_fixed((ew * (s->lam_min * A)) / 4.0, s->F, &ok);
  }
  if (!ok || !orc_check_budget(s->G, s->ne)) {
    orc_destroy(s);
    return ORC_E_FIXED_OVERFLOW;
  }
  if (o->newton) {
    s->gx = (double *)malloc(sizeof(double) * s->nfx);
    s->gy = (double *)malloc(sizeof(double) * (s->nfy ? s->nfy : 1));
    s->diag = (double *)malloc(sizeof(double) * s->nc);
    orc_newton_operator(&s->p, s->gx, s->gy, s->diag);
  }
  *out = s;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The flight of one particle (Sec. 3.1 step (2), Sec. 3.2 steps (3)-(6))    */
/* ------------------------------------------------------------------------ */

/* March one straight segment of length ell from (x0,y0) in cell (*ix,*iy).
 * Next x-face k (k = ix+1 moving +x, k = ix moving -x) is reached at
 * t = (k dx - x0) * (1/sx); likewise y.  The earlier face is crossed while
 * t < ell (strict); at equal t the x-face goes first.  Crossing a boundary
 * face absorbs the particle.  Returns 1 if absorbed (b index in *bface). */
static int orc_march(const orc_problem *p, double x0, double y0, int *ix, int *iy, double sx,
                     double sy, double inv_sx, double inv_sy, double ell, int64_t q,
                     orc_tally *t, int *bface)
{
  int nx = p->nx, ny = p->ny;
  int stepx = (sx > 0.0) ? 1 : ((sx < 0.0) ? -1 : 0);
  int stepy = (sy > 0.0) ? 1 : ((sy < 0.0) ? -1 : 0);
  int kx = (stepx > 0) ? *ix + 1 : *ix;
  int ky = (stepy > 0) ? *iy + 1 : *iy;
  for (;;) {
    double tx = stepx ? ((double)kx * p->dx - x0) * inv_sx : INFINITY;
    double ty = stepy ? ((double)ky * p->dy - y0) * inv_sy : INFINITY;
    int axis_x = (tx <= ty);
    double tt = axis_x ? tx : ty;
    if (!(tt < ell)) return 0;
    t->crossings++;
    if (axis_x) {
      int f = *iy * (nx + 1) + kx;
      if (t->faces) t->Phix[f] += (stepx > 0) ? q : -q;
      if (t->events && t->n_events < t->max_events) {
        t->events[3 * t->n_events] = 0;
        t->events[3 * t->n_events + 1] = f;
        t->events[3 * t->n_events + 2] = stepx;
        t->n_events++;
      }
      if (kx == 0 || kx == nx) {
        *bface = (kx == 0) ? *iy : ny + *iy;
        return 1;
      }
      *ix += stepx;
      kx += stepx;
    } else {
      int f = ky * nx + *ix;
      if (t->faces) t->Phiy[f] += (stepy > 0) ? q : -q;
      if (t->events && t->n_events < t->max_events) {
        t->events[3 * t->n_events] = 1;
        t->events[3 * t->n_events + 1] = f;
        t->events[3 * t->n_events + 2] = stepy;
        t->n_events++;
      }
      if (ky == 0 || ky == ny) {
        *bface = (ky == 0) ? 2 * ny + *ix : 2 * ny + nx + *ix;
        return 1;
      }
      *iy += stepy;
      ky += stepy;
    }
  }
}

static double orc_clamp(double v, double lo, double hi)
{
  if (v < lo) return lo;
  if (v > hi) return hi;
  return v;
}

/* What a flight needs besides its counters: the mesh, the seed, the candidate
 * mean free path |V_g| tau* of its band, the acceptance tau* / tau per cell,
 * and the offset of the band's emitters in the Philox counter (0 when gray). */
typedef struct {
  const orc_problem *p;
  int nc;
  uint64_t seed;
  double lam;
  const double *ratio;
  uint32_t e_off;
  int has_null;          /* some tau_c > tau_min: W tallied apart from D */
} orc_flyctx;

static orc_flyctx orc_gray_ctx(const orc_state *s)
{
  orc_flyctx f = {&s->p, s->nc, s->o.seed, s->lam_min, s->ratio, 0u, s->has_null};
  return f;
}

/* Fly particle k of emitter e carrying q (q != 0). */
static void orc_fly(const orc_flyctx *f, uint32_t slot, int e, uint32_t k, int64_t q, orc_tally *t,
                    uint64_t *segs)
{
  const orc_problem *p = f->p;
  int nx = p->nx, ny = p->ny;
  uint32_t ec = (uint32_t)e + f->e_off;
  double ua, ub, uc, ud;
  orc_draw(f->seed, slot, ec, k, 0u, &ua, &ub);
  orc_draw(f->seed, slot, ec, k, 1u, &uc, &ud);
  int ix, iy;
  double x0, y0, sx, sy;
  if (e < f->nc) {
    /* equilibrium emission from a cell: uniform position, isotropic 3D direction */
    ix = e % nx;
    iy = e / nx;
    x0 = ((double)ix + ua) * p->dx;
    y0 = ((double)iy + ub) * p->dy;
    double mu = 2.0 * uc - 1.0;
    sx = mu;
    sy = (p->dim == 2) ? sqrt((1.0 - mu) * (1.0 + mu)) * orc_cos2pi(ud) : 0.0;
  } else {
    /* wall emission (reading R1): cosine-law direction into the domain */
    int b = e - f->nc;
    double cn = sqrt(uc);
    double tg = (p->dim == 2) ? sqrt((1.0 - cn) * (1.0 + cn)) * orc_cos2pi(ud) : 0.0;
    if (b < ny) {                       /* left wall, row b */
      ix = 0; iy = b;
      x0 = 0.0; y0 = ((double)iy + ua) * p->dy;
      sx = cn; sy = tg;
    } else if (b < 2 * ny) {            /* right wall */
      ix = nx - 1; iy = b - ny;
      x0 = (double)nx * p->dx; y0 = ((double)iy + ua) * p->dy;
      sx = -cn; sy = tg;
    } else if (b < 2 * ny + nx) {       /* bottom wall, column */
      ix = b - 2 * ny; iy = 0;
      x0 = ((double)ix + ua) * p->dx; y0 = 0.0;
      sx = tg; sy = cn;
    } else {                            /* top wall */
      ix = b - 2 * ny - nx; iy = ny - 1;
      x0 = ((double)ix + ua) * p->dx; y0 = (double)ny * p->dy;
      sx = tg; sy = -cn;
    }
  }
  double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
  double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
  for (uint32_t j = 0;; ++j) {
    double ulen, uacc;
    orc_draw(f->seed, slot, ec, k, 2u + j, &ulen, &uacc);
    /* candidate free path on the common time scale: -|V_g| tau_min ln(eta) */
    double ell = -(f->lam * orc_log(1.0 - ulen));
    (*segs)++;
    int bface = -1;
    if (orc_march(p, x0, y0, &ix, &iy, sx, sy, inv_sx, inv_sy, ell, q, t, &bface)) {
      t->B[bface] += q;
      t->end = -1 - bface;
      return;
    }
    int c = ix + nx * iy;
    t->W[c] += q;
    /* accept as a real collision with probability sigma/sigma_max = tau_min/tau */
    if (uacc < f->ratio[c] || j == ORC_MAX_SEGMENTS - 1) {
      t->D[c] += q;
      t->end = c;
      return;
    }
    /* null collision: same direction, new free path from the stopping point */
    x0 = orc_clamp(x0 + ell * sx, (double)ix * p->dx, (double)(ix + 1) * p->dx);
    if (p->dim == 2) y0 = orc_clamp(y0 + ell * sy, (double)iy * p->dy, (double)(iy + 1) * p->dy);
  }
}

/* Expected-value flight of particle k of emitter e carrying q (variance
 * reduction; the expectation of the analog flight above).  Same start and
 * direction; no free path is drawn.  The ray is followed cell by cell; with
 * optical depth T(s) = sum of chord * tau_min / (lambda_min tau_c) the
 * rounded surviving weight is S(T) = rint(q exp(-T)).  A cell's chord from
 * depth T_a to T_b deposits D += S(T_a) - S(T_b) (the real collisions, exactly
 * conserved) and, with null collisions, the expected candidates
 * W += rint(q (exp(-T_a) - exp(-T_b)) / ratio_c) (W = D without them); a
 * crossed face carries S at the face, a wall face absorbs it.  The ray ends
 * at the first face where S has reached 0, and a ray with no direction
 * leaves all of q in its cell. */
static int64_t orc_cand(double v, double ratio, orc_tally *t)
{
  double x = v / ratio;
  if (!(fabs(x) <= ORC_TWO62)) {
    t->bad = 1;
    return 0;
  }
  return (int64_t)rint(x);
}

static void orc_fly_expected(const orc_flyctx *f, uint32_t slot, int e, uint32_t k, int64_t q,
                             orc_tally *t, uint64_t *segs)
{
  const orc_problem *p = f->p;
  int nx = p->nx, ny = p->ny;
  uint32_t ec = (uint32_t)e + f->e_off;
  double ua, ub, uc, ud;
  orc_draw(f->seed, slot, ec, k, 0u, &ua, &ub);
  orc_draw(f->seed, slot, ec, k, 1u, &uc, &ud);
  int ix, iy;
  double x0, y0, sx, sy;
  if (e < f->nc) {
    ix = e % nx;
    iy = e / nx;
    x0 = ((double)ix + ua) * p->dx;
    y0 = ((double)iy + ub) * p->dy;
    double mu = 2.0 * uc - 1.0;
    sx = mu;
    sy = (p->dim == 2) ? sqrt((1.0 - mu) * (1.0 + mu)) * orc_cos2pi(ud) : 0.0;
  } else {
    int b = e - f->nc;
    double cn = sqrt(uc);
    double tg = (p->dim == 2) ? sqrt((1.0 - cn) * (1.0 + cn)) * orc_cos2pi(ud) : 0.0;
    if (b < ny) {
      ix = 0; iy = b;
      x0 = 0.0; y0 = ((double)iy + ua) * p->dy;
      sx = cn; sy = tg;
    } else if (b < 2 * ny) {
      ix = nx - 1; iy = b - ny;
      x0 = (double)nx * p->dx; y0 = ((double)iy + ua) * p->dy;
      sx = -cn; sy = tg;
    } else if (b < 2 * ny + nx) {
      ix = b - 2 * ny; iy = 0;
      x0 = ((double)ix + ua) * p->dx; y0 = 0.0;
      sx = tg; sy = cn;
    } else {
      ix = b - 2 * ny - nx; iy = ny - 1;
      x0 = ((double)ix + ua) * p->dx; y0 = (double)ny * p->dy;
      sx = tg; sy = -cn;
    }
  }
  (*segs)++;
  double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
  double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
  int stepx = (sx > 0.0) ? 1 : ((sx < 0.0) ? -1 : 0);
  int stepy = (sy > 0.0) ? 1 : ((sy < 0.0) ? -1 : 0);
  int kx = (stepx > 0) ? ix + 1 : ix;
  int ky = (stepy > 0) ? iy + 1 : iy;
  double T = 0.0, surv = 1.0, tprev = 0.0;
  int64_t S = q;
  const double qd = (double)q;
  for (;;) {
    int c = ix + nx * iy;
    double tx = stepx ? ((double)kx * p->dx - x0) * inv_sx : INFINITY;
    double ty = stepy ? ((double)ky * p->dy - y0) * inv_sy : INFINITY;
    int axis_x = (tx <= ty);
    double tt = axis_x ? tx : ty;
    if (!(tt < INFINITY)) {            /* no direction: everything stays here */
      t->D[c] += S;
      t->W[c] += f->has_null ? orc_cand(qd * surv, f->ratio[c], t) : S;
      t->end = c;
      return;
    }
    double Tn = T + (tt - tprev) * (f->ratio[c] / f->lam);
    double sn = orc_expm(Tn);
    int64_t Sn = (int64_t)rint(qd * sn);
    t->D[c] += S - Sn;
    t->W[c] += f->has_null ? orc_cand(qd * (surv - sn), f->ratio[c], t) : S - Sn;
    T = Tn;
    surv = sn;
    S = Sn;
    tprev = tt;
    if (S == 0) {
      t->end = c;
      return;
    }
    t->crossings++;
    if (axis_x) {
      if (t->faces) t->Phix[iy * (nx + 1) + kx] += (stepx > 0) ? S : -S;
      if (kx == 0 || kx == nx) {
        int b = (kx == 0) ? iy : ny + iy;
        t->B[b] += S;
        t->end = -1 - b;
        return;
      }
      ix += stepx;
      kx += stepx;
    } else {
      if (t->faces) t->Phiy[ky * nx + ix] += (stepy > 0) ? S : -S;
      if (ky == 0 || ky == ny) {
        int b = (ky == 0) ? 2 * ny + ix : 2 * ny + nx + ix;
        t->B[b] += S;
        t->end = -1 - b;
        return;
      }
      iy += stepy;
      ky += stepy;
    }
  }
}

int orc_trace_ray(const orc_problem *p, double x0, double y0, int ix, int iy, double sx,
                  double sy, double ell, int32_t *events, int max_events, int *end_kind,
                  int *end_cell)
{
  orc_tally t;
  memset(&t, 0, sizeof t);
  t.events = events;
  t.max_events = max_events;
  double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
  double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
  int b = -1;
  int absorbed = orc_march(p, x0, y0, &ix, &iy, sx, sy, inv_sx, inv_sy, ell, 1, &t, &b);
  *end_kind = absorbed;
  *end_cell = absorbed ? b : ix + p->nx * iy;
  return t.n_events;
}

/* One iteration (Sec. 3.1 steps (1)-(3); Sec. 3.2 steps (1)-(6); Sec. 3.3). */
static int orc_iterate(orc_state *s, int faces)
{
  const orc_problem *p = &s->p;
  uint32_t slot = (s->o.rng_mode == ORC_RNG_CRN) ? s->o.rng_epoch : s->iter;
  memset(s->D, 0, sizeof(int64_t) * s->nc);
  memset(s->W, 0, sizeof(int64_t) * s->nc);
  memset(s->Phix, 0, sizeof(int64_t) * s->nfx);
  if (s->nfy) memset(s->Phiy, 0, sizeof(int64_t) * s->nfy);
  memset(s->B, 0, sizeof(int64_t) * s->nb);
  orc_tally t;
  memset(&t, 0, sizeof t);
  t.D = s->D; t.W = s->W; t.Phix = s->Phix; t.Phiy = s->Phiy; t.B = s->B;
  t.faces = faces;
  if (faces) {
    /* every wall particle enters through its wall face: inward crossing of G_f */
    int nx = p->nx, ny = p->ny;
    for (int b = 0; b < s->nb; ++b) {
      int64_t g = s->G[s->nc + b];
      if (b < ny) s->Phix[b * (nx + 1)] += g;
      else if (b < 2 * ny) s->Phix[(b - ny) * (nx + 1) + nx] -= g;
      else if (b < 2 * ny + nx) s->Phiy[b - 2 * ny] += g;
      else s->Phiy[ny * nx + (b - 2 * ny - nx)] -= g;
    }
  }
  uint64_t flights = 0, segs = 0;
  const orc_flyctx fc = orc_gray_ctx(s);
  for (int e = 0; e < s->ne; ++e)
    for (uint64_t k = 0; k < s->N; ++k) {
      int64_t q = orc_split_weight(s->G[e], s->N, k);
      if (q == 0) continue;
      flights++;
      if (s->o.estimator == ORC_EST_EXPECTED)
        orc_fly_expected(&fc, slot, e, (uint32_t)k, q, &t, &segs);
      else
        orc_fly(&fc, slot, e, (uint32_t)k, q, &t, &segs);
    }
  s->flights = flights;
  s->segments = segs;
  s->crossings = t.crossings;
  s->tot_flights += flights;
  s->tot_segments += segs;
  s->tot_crossings += t.crossings;

  /* macroscopic update: E^{n+1/2} from the total tally W */
  double *E_new = (double *)malloc(sizeof(double) * s->nc);
  double *tmp = (double *)malloc(sizeof(double) * s->nc);
  for (int c = 0; c < s->nc; ++c) s->E_half[c] = ldexp((double)s->W[c], -s->F) / s->V;
  int rc = ORC_OK;
  int ok = !t.bad;
  if (s->o.newton) {
    double *r = (double *)malloc(sizeof(double) * s->nc);
    double *x = (double *)malloc(sizeof(double) * s->nc);
    for (int c = 0; c < s->nc; ++c) r[c] = s->E_half[c] - s->E[c];
    int its = 0;
    rc = orc_newton_solve(p, &s->o, s->gx, s->gy, s->diag, r, x, &its);
    s->cg_last = its;
    s->cg_total += its;
    for (int c = 0; c < s->nc; ++c) E_new[c] = s->E_half[c] + x[c];
    for (int c = 0; c < s->nc; ++c)
      s->G[c] = orc_add(orc_to_fixed((E_new[c] * s->V) * s->ratio[c], s->F, &ok), s->Gs[c], &ok);
    free(r);
    free(x);
  } else {
    for (int c = 0; c < s->nc; ++c) E_new[c] = s->E_half[c];
    for (int c = 0; c < s->nc; ++c) s->G[c] = orc_add(s->D[c], s->Gs[c], &ok);   /* re-emit W^h */
  }
  for (int c = 0; c < s->nc; ++c) {
    double d = E_new[c] - s->E[c];
    tmp[c] = d * d;
  }
  double dn = sqrt(orc_tree_sum(tmp, (uint64_t)s->nc));
  if (s->iter == 0) s->d0 = dn;
  s->res = (s->d0 > 0.0) ? dn / s->d0 : 0.0;
  for (int c = 0; c < s->nc; ++c) {
    if (!isfinite(E_new[c]) && rc == ORC_OK) rc = ORC_E_NONFINITE;
    s->E[c] = E_new[c];
  }
  if ((int)s->iter < s->res_cap) s->res_hist[s->iter] = s->res;
  s->iter++;
  free(E_new);
  free(tmp);
  int over = (!ok || !orc_check_budget(s->G, s->ne));
  /* Growth rule of the Newton iteration (reading R6): the update has grown
   * beyond the first one (res > 1) and either the next emission left the
   * fixed-point range or, with common random numbers (one fixed map, so a
   * rise is the map's and not sampling noise), the residual rose in two
   * consecutive iterations. */
  int grew = s->o.newton && s->res > 1.0 &&
             (over || (s->o.rng_mode == ORC_RNG_CRN && s->res > s->res_p1 &&
                       s->res_p1 > s->res_p2));
  s->res_p2 = s->res_p1;
  s->res_p1 = s->res;
  if (rc == ORC_OK && grew) rc = ORC_E_DIVERGED;
  if (rc == ORC_OK && over) rc = ORC_E_FIXED_OVERFLOW;
  if (rc == ORC_OK && s->iter > 1 && s->res > 1e3) rc = ORC_E_DIVERGED;
  return rc;
}

int orc_step(orc_state *s, int n_iters, int faces)
{
  for (int i = 0; i < n_iters; ++i) {
    int rc = orc_iterate(s, faces);
    if (rc) return rc;
  }
  return ORC_OK;
}

int orc_solve(orc_state *s, double *T_out, double *qx_out, double *qy_out)
{
  const orc_problem *p = &s->p;
  int faces_each = (s->o.tally_faces == ORC_FACES_EVERY);
  int converged = 0, rc;
  while ((int)s->iter < s->o.max_iters) {
    rc = orc_iterate(s, faces_each);
    if (rc) return rc;
    if (s->res < s->o.res_tol) {
      converged = 1;
      break;
    }
  }
  int faces_out = (s->o.tally_faces != ORC_FACES_OFF);
  double *Eo = (double *)calloc((size_t)s->nc, sizeof(double));
  double *fx = (double *)calloc((size_t)s->nfx, sizeof(double));
  double *fy = (double *)calloc((size_t)(s->nfy ? s->nfy : 1), sizeof(double));
  if (s->o.avg_iters > 0) {
    for (int a = 0; a < s->o.avg_iters; ++a) {
      rc = orc_iterate(s, faces_out);
      if (rc) { free(Eo); free(fx); free(fy); return rc; }
      for (int c = 0; c < s->nc; ++c) Eo[c] = Eo[c] + s->E[c];
      for (int f = 0; f < s->nfx; ++f) fx[f] = fx[f] + ldexp((double)s->Phix[f], -s->F);
      for (int f = 0; f < s->nfy; ++f) fy[f] = fy[f] + ldexp((double)s->Phiy[f], -s->F);
    }
    double na = (double)s->o.avg_iters;
    for (int c = 0; c < s->nc; ++c) Eo[c] = Eo[c] / na;
    for (int f = 0; f < s->nfx; ++f) fx[f] = fx[f] / na;
    for (int f = 0; f < s->nfy; ++f) fy[f] = fy[f] / na;
  } else {
    if (s->o.tally_faces == ORC_FACES_FINAL) {
      rc = orc_iterate(s, 1);
      if (rc) { free(Eo); free(fx); free(fy); return rc; }
    }
    for (int c = 0; c < s->nc; ++c) Eo[c] = s->E[c];
    for (int f = 0; f < s->nfx; ++f) fx[f] = ldexp((double)s->Phix[f], -s->F);
    for (int f = 0; f < s->nfy; ++f) fy[f] = ldexp((double)s->Phiy[f], -s->F);
  }
  if (T_out)
    for (int c = 0; c < s->nc; ++c) T_out[c] = p->t_ref + Eo[c] / p->cv;
  if (qx_out) {
    double den = p->dy * s->tau_min;
    for (int f = 0; f < s->nfx; ++f) qx_out[f] = faces_out ? fx[f] / den : 0.0;
  }
  if (qy_out && s->nfy) {
    double den = p->dx * s->tau_min;
    for (int f = 0; f < s->nfy; ++f) qy_out[f] = faces_out ? fy[f] / den : 0.0;
  }
  free(Eo);
  free(fx);
  free(fy);
  return converged ? ORC_OK : ORC_W_NOT_CONVERGED;
}

void orc_get_info(const orc_state *s, orc_info *info)
{
  info->iter = s->iter;
  info->F = s->F;
  info->n_per_emitter = s->N;
  info->n_cells = s->nc;
  info->n_bfaces = s->nb;
  info->n_emitters = s->ne;
  info->tau_min = s->tau_min;
  info->lam_min = s->lam_min;
  info->d0 = s->d0;
  info->res = s->res;
  info->flights = s->flights;
  info->segments = s->segments;
  info->crossings = s->crossings;
  info->tot_flights = s->tot_flights;
  info->tot_segments = s->tot_segments;
  info->tot_crossings = s->tot_crossings;
  info->cg_iters_last = s->cg_last;
  info->cg_iters_total = s->cg_total;
}

void orc_get_tallies(const orc_state *s, int64_t *D, int64_t *W, int64_t *Phix, int64_t *Phiy,
                     int64_t *B)
{
  if (D) memcpy(D, s->D, sizeof(int64_t) * s->nc);
  if (W) memcpy(W, s->W, sizeof(int64_t) * s->nc);
  if (Phix) memcpy(Phix, s->Phix, sizeof(int64_t) * s->nfx);
  if (Phiy && s->nfy) memcpy(Phiy, s->Phiy, sizeof(int64_t) * s->nfy);
  if (B) memcpy(B, s->B, sizeof(int64_t) * s->nb);
}

void orc_get_E(const orc_state *s, double *E) { memcpy(E, s->E, sizeof(double) * s->nc); }

void orc_get_G(const orc_state *s, int64_t *G) { memcpy(G, s->G, sizeof(int64_t) * s->ne); }

void orc_get_residuals(const orc_state *s, double *res, int max_n)
{
  for (int i = 0; i < max_n && i < s->res_cap; ++i) res[i] = s->res_hist[i];
}

int orc_set_state(orc_state *s, uint32_t iter, double d0, const double *E, const int64_t *G)
{
  s->iter = iter;
  s->d0 = d0;
  s->res_p1 = s->res_p2 = HUGE_VAL;
  memcpy(s->E, E, sizeof(double) * s->nc);
  memcpy(s->G, G, sizeof(int64_t) * s->ne);
  return orc_check_budget(s->G, s->ne) ? ORC_OK : ORC_E_FIXED_OVERFLOW;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the steady state                                               */
/* ------------------------------------------------------------------------ */
/* With a uniform relaxation time every candidate collision is real, and with
 * common random numbers the particle paths depend only on their counters, not
 * on the weights: one iteration is the linear map
 *   D = T_cc G_cells + T_cw G_walls,   T_xe = (1/N) #{k : particle (e,k) ends in x},
 * and re-emission G_cells = D + G_src gives the steady state
 *   D* = (I - T_cc)^-1 (T_cc G_src + T_cw G_walls),  T = t_ref + ldexp(D*, -F) / (V C).
 * For a loss L(T), with u = dL/dD* and psi = (I - T_cc^T)^-1 u,
 *   dL/dG_src = T_cc^T psi,  dL/dG_walls = T_cw^T psi.
 * (T^T psi)_e is the mean of psi over the cells where emitter e's N particles
 * end: the same paths used in reverse.  psi is the fixed point of
 * psi <- T^T psi + u, each pass optionally followed by the diffusion
 * correction of the forward solve (same operator, same CG).  Chain rule to
 * the inputs: G_src = ldexp(S V tau_min, F), G_f = ldexp(C (T_f - t_ref)
 * lambda_min A_f / 4, F). */
static void orc_gather(const orc_state *s, const int32_t *end, const double *psi, double *vals,
                       double *g)
{
  uint64_t N = s->N;
  for (int e = 0; e < s->ne; ++e) {
    for (uint64_t k = 0; k < N; ++k) {
      int32_t a = end[(uint64_t)e * N + k];
      vals[k] = (a >= 0) ? psi[a] : 0.0;
    }
    g[e] = orc_tree_sum(vals, N) / (double)N;
  }
}

int orc_adjoint(orc_state *s, const double *dLdT, double *grad_wall, double *grad_source,
                int max_iters, double tol, int *iters_out)
{
  const orc_problem *p = &s->p;
  if (iters_out) *iters_out = 0;
  if (s->o.rng_mode != ORC_RNG_CRN || s->o.estimator != ORC_EST_ANALOG || max_iters < 1 ||
      !(tol >= 0.0) || !dLdT)
    return ORC_E_INVALID_ARG;
  for (int c = 0; c < s->nc; ++c)
    if (s->ratio[c] != 1.0 || !isfinite(dLdT[c])) return ORC_E_INVALID_ARG;
  int nc = s->nc, ne = s->ne;
  uint64_t N = s->N;
  uint32_t slot = s->o.rng_epoch;
  /* where every particle ends (the weight does not change the path) */
  int32_t *end = (int32_t *)malloc(sizeof(int32_t) * (size_t)ne * N);
  int64_t *sD = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  int64_t *sW = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  int64_t *sB = (int64_t *)calloc((size_t)s->nb, sizeof(int64_t));
  orc_tally t;
  memset(&t, 0, sizeof t);
  t.D = sD; t.W = sW; t.B = sB; t.faces = 0;
  uint64_t segs = 0;
  const orc_flyctx fc = orc_gray_ctx(s);
  for (int e = 0; e < ne; ++e)
    for (uint64_t k = 0; k < N; ++k) {
      orc_fly(&fc, slot, e, (uint32_t)k, 1, &t, &segs);
      end[(uint64_t)e * N + k] = (t.end >= 0) ? t.end : -1;
    }
  double *u = (double *)malloc(sizeof(double) * nc);
  double *psi = (double *)malloc(sizeof(double) * nc);
  double *half = (double *)malloc(sizeof(double) * nc);
  double *nw = (double *)malloc(sizeof(double) * nc);
  double *tmp = (double *)malloc(sizeof(double) * nc);
  double *r = (double *)malloc(sizeof(double) * nc);
  double *x = (double *)malloc(sizeof(double) * nc);
  double *vals = (double *)malloc(sizeof(double) * N);
  double *g = (double *)malloc(sizeof(double) * ne);
  /* u = dL/dD* since T_c = t_ref + ldexp(D_c, -F) / V / C */
  for (int c = 0; c < nc; ++c) u[c] = ldexp((dLdT[c] / p->cv) / s->V, -s->F);
  for (int c = 0; c < nc; ++c) psi[c] = u[c];
  int rc = ORC_W_NOT_CONVERGED, passes = 0;
  double d0 = 0.0;
  for (int m = 0; m < max_iters; ++m) {
    orc_gather(s, end, psi, vals, g);
    for (int c = 0; c < nc; ++c) half[c] = g[c] + u[c];
    if (s->o.newton) {
      for (int c = 0; c < nc; ++c) r[c] = half[c] - psi[c];
      int its = 0;
      int crc = orc_newton_solve(p, &s->o, s->gx, s->gy, s->diag, r, x, &its);
      if (crc) {
        rc = crc;
        break;
      }
      for (int c = 0; c < nc; ++c) nw[c] = half[c] + x[c];
    } else {
      for (int c = 0; c < nc; ++c) nw[c] = half[c];
    }
    for (int c = 0; c < nc; ++c) {
      double d = nw[c] - psi[c];
      tmp[c] = d * d;
    }
    double dn = sqrt(orc_tree_sum(tmp, (uint64_t)nc));
    if (m == 0) d0 = dn;
    double res = (d0 > 0.0) ? dn / d0 : 0.0;
    for (int c = 0; c < nc; ++c) psi[c] = nw[c];
    passes = m + 1;
    if (!isfinite(res)) {
      rc = ORC_E_NONFINITE;
      break;
    }
    if (res < tol) {
      rc = ORC_OK;
      break;
    }
  }
  if (rc >= 0) {
    orc_gather(s, end, psi, vals, g);
    double fs = ldexp(s->V * s->tau_min, s->F);
    if (grad_source)
      for (int c = 0; c < nc; ++c) grad_source[c] = g[c] * fs;
    if (grad_wall)
      for (int b = 0; b < s->nb; ++b) {
        double A = (b < 2 * p->ny) ? p->dy : p->dx;
        grad_wall[b] = g[nc + b] * ldexp((p->cv * (s->lam_min * A)) / 4.0, s->F);
      }
  }
  if (iters_out) *iters_out = passes;
  free(end); free(sD); free(sW); free(sB);
  free(u); free(psi); free(half); free(nw); free(tmp); free(r); free(x); free(vals); free(g);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Frequency bands (beyond the paper's gray model)                           */
/* ------------------------------------------------------------------------ */
struct orc_bands {
  orc_problem p;
  orc_options o;
  int K, nc, nb, ne, nfx, nfy;
  uint64_t N;
  int F;
  double V, Ctot;
  double *tau, *wall_T, *source, *bC, *bv;   /* copies; tau [K][nc] */
  double *ts, *lam;                          /* [K] tau*_k, v_k tau*_k */
  double *ratio;                             /* [K][nc] tau*_k / tau_k(c) */
  double *den;                               /* [nc] sum_k C_k / tau_k(c) */
  double *E;                                 /* energy density */
  int64_t *G, *D, *W, *Phix, *Phiy, *B;      /* [K][ne], [K][nc] x2, [K][nfx], [K][nfy], [K][nb] */
  uint32_t iter;
  double d0, res;
  uint64_t flights, segments, crossings, tot_flights, tot_segments, tot_crossings;
};

void orc_bands_destroy(orc_bands *s)
{
  if (!s) return;
  free(s->tau); free(s->wall_T); free(s->source); free(s->bC); free(s->bv);
  free(s->ts); free(s->lam); free(s->ratio); free(s->den); free(s->E);
  free(s->G); free(s->D); free(s->W); free(s->Phix); free(s->Phiy); free(s->B);
  free(s);
}

/* next emission of cell c for every band from the absorbed rate R */
static void orc_bands_emit(orc_bands *s, int c, double R, int *ok)
{
  for (int k = 0; k < s->K; ++k) {
    const double pk = (s->bC[k] / s->tau[(size_t)k * s->nc + c]) / s->den[c];
    s->G[(size_t)k * s->ne + c] = orc_to_fixed((s->ts[k] * pk) * R, s->F, ok);
  }
}

int orc_bands_create(const orc_problem *p, const orc_options *o, orc_bands **out)
{
  *out = NULL;
  if (!p || p->n_bands < 2 || !p->band_C || !p->band_vg || !p->tau || !p->wall_T)
    return ORC_E_INVALID_ARG;
  if (p->dim != 1 && p->dim != 2) return ORC_E_INVALID_ARG;
  if (p->nx < 1 || p->ny < 1 || (p->dim == 1 && p->ny != 1)) return ORC_E_INVALID_ARG;
  if (!(p->dx > 0.0) || !(p->dy > 0.0) || !isfinite(p->dx) || !isfinite(p->dy) ||
      !isfinite(p->t_ref))
    return ORC_E_INVALID_ARG;
  if (!o || o->particles_per_iter < 1 || o->max_iters < 0 || o->avg_iters != 0 || o->newton ||
      o->estimator != ORC_EST_ANALOG)
    return ORC_E_INVALID_ARG;
  const int K = p->n_bands, nc = p->nx * p->ny, nb = orc_nb(p);
  for (int k = 0; k < K; ++k)
    if (!(p->band_C[k] > 0.0) || !isfinite(p->band_C[k]) || !(p->band_vg[k] > 0.0) ||
        !isfinite(p->band_vg[k]))
      return ORC_E_INVALID_ARG;
  for (int k = 0; k < K; ++k) {
    double tmin = INFINITY, tmax = 0.0;
    for (int c = 0; c < nc; ++c) {
      const double t = p->tau[(size_t)k * nc + c];
      if (!(t > 0.0) || !isfinite(t)) return ORC_E_INVALID_ARG;
      if (t < tmin) tmin = t;
      if (t > tmax) tmax = t;
    }
    if (tmax > 1e6 * tmin) return ORC_E_INVALID_ARG;
  }
  for (int b = 0; b < nb; ++b)
    if (!isfinite(p->wall_T[b])) return ORC_E_INVALID_ARG;
  if (p->T_init)
    for (int c = 0; c < nc; ++c)
      if (!isfinite(p->T_init[c])) return ORC_E_INVALID_ARG;
  if (p->source)
    for (int c = 0; c < nc; ++c)
      if (!isfinite(p->source[c])) return ORC_E_INVALID_ARG;

  orc_bands *s = (orc_bands *)calloc(1, sizeof(orc_bands));
  s->p = *p;
  s->o = *o;
  s->K = K;
  s->nc = nc;
  s->nb = nb;
  s->ne = nc + nb;
  s->nfx = p->ny * (p->nx + 1);
  s->nfy = (p->dim == 2) ? (p->ny + 1) * p->nx : 0;
  s->tau = orc_dup(p->tau, K * nc);
  s->wall_T = orc_dup(p->wall_T, nb);
  s->source = orc_dup(p->source, nc);
  s->bC = orc_dup(p->band_C, K);
  s->bv = orc_dup(p->band_vg, K);
  s->p.tau = s->tau;
  s->p.wall_T = s->wall_T;
  s->p.source = s->source;
  s->p.band_C = s->bC;
  s->p.band_vg = s->bv;
  s->p.T_init = NULL;
  s->p.diff_x = s->p.diff_y = NULL;
  s->N = o->particles_per_iter / ((uint64_t)s->ne * (uint64_t)K);
  if (s->N < 1) s->N = 1;
  s->V = p->dx * p->dy;
  s->ts = (double *)malloc(sizeof(double) * K);
  s->lam = (double *)malloc(sizeof(double) * K);
  s->ratio = (double *)malloc(sizeof(double) * (size_t)K * nc);
  s->den = (double *)calloc((size_t)nc, sizeof(double));
  s->Ctot = 0.0;
  for (int k = 0; k < K; ++k) {
    double tmin = p->tau[(size_t)k * nc];
    for (int c = 1; c < nc; ++c)
      if (p->tau[(size_t)k * nc + c] < tmin) tmin = p->tau[(size_t)k * nc + c];
    s->ts[k] = tmin;
    s->lam[k] = p->band_vg[k] * tmin;
    for (int c = 0; c < nc; ++c) s->ratio[(size_t)k * nc + c] = tmin / p->tau[(size_t)k * nc + c];
    s->Ctot = s->Ctot + p->band_C[k];
  }
  for (int c = 0; c < nc; ++c)
    for (int k = 0; k < K; ++k) s->den[c] = s->den[c] + p->band_C[k] / p->tau[(size_t)k * nc + c];
  /* fixed-point scale: as the gray budget with the band sums (emission of the
     cells <= C dT V per iteration, walls <= dT sum_k C_k lambda*_k A / 4), plus
     the source's energy density S_max times the longest residence time of a
     band, max_k tau*_k (1 + 3 (L / lambda*_k)^2) (the gray bound per band) */
  double dT = 0.0;
  for (int b = 0; b < nb; ++b)
    if (fabs(p->wall_T[b] - p->t_ref) > dT) dT = fabs(p->wall_T[b] - p->t_ref);
  if (p->T_init)
    for (int c = 0; c < nc; ++c)
      if (fabs(p->T_init[c] - p->t_ref) > dT) dT = fabs(p->T_init[c] - p->t_ref);
  double lam_sum = 0.0;
  for (int k = 0; k < K; ++k) lam_sum = lam_sum + p->band_C[k] * s->lam[k];
  const double vol = (double)nc * s->V;
  const double area = (p->dim == 2) ? ((2.0 * (double)p->ny) * p->dy + (2.0 * (double)p->nx) * p->dx)
                                    : 2.0;
  double esrc = 0.0;
  if (p->source) {
    double smax = 0.0;
    for (int c = 0; c < nc; ++c)
      if (fabs(p->source[c]) > smax) smax = fabs(p->source[c]);
    double L = (double)p->nx * p->dx;
    if (p->dim == 2 && (double)p->ny * p->dy > L) L = (double)p->ny * p->dy;
    double res_hi = 0.0;
    for (int k = 0; k < K; ++k) {
      const double rl = L / s->lam[k];
      const double r = s->ts[k] * (1.0 + 3.0 * (rl * rl));
      if (r > res_hi) res_hi = r;
    }
    esrc = smax * res_hi;
  }
  const double Bb = 4.0 * ((dT * s->Ctot + esrc) * vol + (dT * lam_sum * area) / 4.0);
  if (Bb > 0.0) {
    int ex;
    double m = frexp(Bb, &ex);
    s->F = 62 - ((m == 0.5) ? ex - 1 : ex);
  } else {
    s->F = 62;
  }
  s->E = (double *)calloc((size_t)nc, sizeof(double));
  s->G = (int64_t *)calloc((size_t)K * s->ne, sizeof(int64_t));
  s->D = (int64_t *)calloc((size_t)K * nc, sizeof(int64_t));
  s->W = (int64_t *)calloc((size_t)K * nc, sizeof(int64_t));
  s->Phix = (int64_t *)calloc((size_t)K * s->nfx, sizeof(int64_t));
  s->Phiy = (int64_t *)calloc((size_t)K * (s->nfy ? s->nfy : 1), sizeof(int64_t));
  s->B = (int64_t *)calloc((size_t)K * nb, sizeof(int64_t));
  int ok = 1;
  /* start in equilibrium at T_init: absorbed rate (T0 - t_ref) V sum_k C_k / tau_k, plus S V */
  for (int c = 0; c < nc; ++c) {
    const double T0 = p->T_init ? p->T_init[c] : p->t_ref;
    s->E[c] = s->Ctot * (T0 - p->t_ref);
    double R = ((T0 - p->t_ref) * s->V) * s->den[c];
    if (s->source) R = R + s->source[c] * s->V;
    orc_bands_emit(s, c, R, &ok);
  }
  for (int k = 0; k < K; ++k)
    for (int b = 0; b < nb; ++b) {
      const double A = (b < 2 * p->ny) ? p->dy : p->dx;
      s->G[(size_t)k * s->ne + nc + b] =
          orc_to_fixed(((p->band_C[k] * (s->wall_T[b] - p->t_ref)) * (s->lam[k] * A)) / 4.0, s->F, &ok);
    }
  if (!ok || !orc_check_budget(s->G, K * s->ne)) {
    orc_bands_destroy(s);
    return ORC_E_FIXED_OVERFLOW;
  }
  *out = s;
  return ORC_OK;
}

static int orc_bands_iterate(orc_bands *s, int faces)
{
  const orc_problem *p = &s->p;
  const int K = s->K, nc = s->nc, ne = s->ne, nb = s->nb;
  uint32_t slot = (s->o.rng_mode == ORC_RNG_CRN) ? s->o.rng_epoch : s->iter;
  memset(s->D, 0, sizeof(int64_t) * (size_t)K * nc);
  memset(s->W, 0, sizeof(int64_t) * (size_t)K * nc);
  memset(s->Phix, 0, sizeof(int64_t) * (size_t)K * s->nfx);
  if (s->nfy) memset(s->Phiy, 0, sizeof(int64_t) * (size_t)K * s->nfy);
  memset(s->B, 0, sizeof(int64_t) * (size_t)K * nb);
  uint64_t flights = 0, segs = 0, cross = 0;
  for (int k = 0; k < K; ++k) {
    orc_tally t;
    memset(&t, 0, sizeof t);
    t.D = s->D + (size_t)k * nc;
    t.W = s->W + (size_t)k * nc;
    t.Phix = s->Phix + (size_t)k * s->nfx;
    t.Phiy = s->Phiy + (size_t)k * (s->nfy ? s->nfy : 0);
    t.B = s->B + (size_t)k * nb;
    t.faces = faces;
    const int64_t *G = s->G + (size_t)k * ne;
    if (faces) {
      int nx = p->nx, ny = p->ny;
      for (int b = 0; b < nb; ++b) {
        int64_t g = G[nc + b];
        if (b < ny) t.Phix[b * (nx + 1)] += g;
        else if (b < 2 * ny) t.Phix[(b - ny) * (nx + 1) + nx] -= g;
        else if (b < 2 * ny + nx) t.Phiy[b - 2 * ny] += g;
        else t.Phiy[ny * nx + (b - 2 * ny - nx)] -= g;
      }
    }
    orc_flyctx fc = {p, nc, s->o.seed, s->lam[k], s->ratio + (size_t)k * nc, (uint32_t)(k * ne)};
    for (int e = 0; e < ne; ++e)
      for (uint64_t i = 0; i < s->N; ++i) {
        int64_t q = orc_split_weight(G[e], s->N, i);
        if (q == 0) continue;
        flights++;
        orc_fly(&fc, slot, e, (uint32_t)i, q, &t, &segs);
      }
    cross += t.crossings;
  }
  s->flights = flights;
  s->segments = segs;
  s->crossings = cross;
  s->tot_flights += flights;
  s->tot_segments += segs;
  s->tot_crossings += cross;
  /* energy density from the candidate tallies, re-emission of the absorbed rate */
  double *tmp = (double *)malloc(sizeof(double) * nc);
  int ok = 1, rc = ORC_OK;
  for (int c = 0; c < nc; ++c) {
    double R = 0.0, Wsum = 0.0;
    for (int k = 0; k < K; ++k) {
      R = R + ldexp((double)s->D[(size_t)k * nc + c], -s->F) / s->ts[k];
      Wsum = Wsum + ldexp((double)s->W[(size_t)k * nc + c], -s->F);
    }
    if (s->source) R = R + s->source[c] * s->V;
    const double En = Wsum / s->V;
    const double d = En - s->E[c];
    tmp[c] = d * d;
    if (!isfinite(En)) rc = ORC_E_NONFINITE;
    s->E[c] = En;
    orc_bands_emit(s, c, R, &ok);
  }
  double dn = sqrt(orc_tree_sum(tmp, (uint64_t)nc));
  free(tmp);
  if (s->iter == 0) s->d0 = dn;
  s->res = (s->d0 > 0.0) ? dn / s->d0 : 0.0;
  s->iter++;
  if (rc == ORC_OK && (!ok || !orc_check_budget(s->G, K * ne))) rc = ORC_E_FIXED_OVERFLOW;
  if (rc == ORC_OK && s->iter > 1 && s->res > 1e3) rc = ORC_E_DIVERGED;
  return rc;
}

int orc_bands_step(orc_bands *s, int n_iters, int faces)
{
  for (int i = 0; i < n_iters; ++i) {
    int rc = orc_bands_iterate(s, faces);
    if (rc) return rc;
  }
  return ORC_OK;
}

int orc_bands_solve(orc_bands *s, double *T_out, double *qx_out, double *qy_out)
{
  const orc_problem *p = &s->p;
  int faces_each = (s->o.tally_faces == ORC_FACES_EVERY);
  int converged = 0, rc;
  while ((int)s->iter < s->o.max_iters) {
    rc = orc_bands_iterate(s, faces_each);
    if (rc) return rc;
    if (s->res < s->o.res_tol) {
      converged = 1;
      break;
    }
  }
  if (s->o.tally_faces == ORC_FACES_FINAL) {
    rc = orc_bands_iterate(s, 1);
    if (rc) return rc;
  }
  int faces_out = (s->o.tally_faces != ORC_FACES_OFF);
  if (T_out)
    for (int c = 0; c < s->nc; ++c) T_out[c] = p->t_ref + s->E[c] / s->Ctot;
  if (qx_out)
    for (int f = 0; f < s->nfx; ++f) {
      double v = 0.0;
      for (int k = 0; k < s->K; ++k)
        v = v + ldexp((double)s->Phix[(size_t)k * s->nfx + f], -s->F) / s->ts[k];
      qx_out[f] = faces_out ? v / p->dy : 0.0;
    }
  if (qy_out && s->nfy)
    for (int f = 0; f < s->nfy; ++f) {
      double v = 0.0;
      for (int k = 0; k < s->K; ++k)
        v = v + ldexp((double)s->Phiy[(size_t)k * s->nfy + f], -s->F) / s->ts[k];
      qy_out[f] = faces_out ? v / p->dx : 0.0;
    }
  return converged ? ORC_OK : ORC_W_NOT_CONVERGED;
}

void orc_bands_get_info(const orc_bands *s, orc_info *info)
{
  memset(info, 0, sizeof *info);
  info->iter = s->iter;
  info->F = s->F;
  info->n_per_emitter = s->N;
  info->n_cells = s->nc;
  info->n_bfaces = s->nb;
  info->n_emitters = s->ne * s->K;
  info->tau_min = s->ts[0];
  info->lam_min = s->lam[0];
  info->d0 = s->d0;
  info->res = s->res;
  info->flights = s->flights;
  info->segments = s->segments;
  info->crossings = s->crossings;
  info->tot_flights = s->tot_flights;
  info->tot_segments = s->tot_segments;
  info->tot_crossings = s->tot_crossings;
}

void orc_bands_get_E(const orc_bands *s, double *E) { memcpy(E, s->E, sizeof(double) * s->nc); }

void orc_bands_get_band(const orc_bands *s, int k, int64_t *D, int64_t *W, int64_t *Phix,
                        int64_t *Phiy, int64_t *B, int64_t *G)
{
  if (k < 0 || k >= s->K) return;
  if (D) memcpy(D, s->D + (size_t)k * s->nc, sizeof(int64_t) * s->nc);
  if (W) memcpy(W, s->W + (size_t)k * s->nc, sizeof(int64_t) * s->nc);
  if (Phix) memcpy(Phix, s->Phix + (size_t)k * s->nfx, sizeof(int64_t) * s->nfx);
  if (Phiy && s->nfy) memcpy(Phiy, s->Phiy + (size_t)k * s->nfy, sizeof(int64_t) * s->nfy);
  if (B) memcpy(B, s->B + (size_t)k * s->nb, sizeof(int64_t) * s->nb);
  if (G) memcpy(G, s->G + (size_t)k * s->ne, sizeof(int64_t) * s->ne);
}

/* ------------------------------------------------------------------------ */
/* Persistent particles: the variable-tau iteration of Sec. 3.2, steps       */
/* (1)-(6), with a fixed population kept between iterations                  */
/* ------------------------------------------------------------------------ */
enum { ORC_P_NULL = 0, ORC_P_REAL = 1, ORC_P_WALL = 2 };
#define ORC_P_STREAM 0xFFFFFFFFu   /* emitter word of every persistent draw */
#define ORC_P_CREATE 0xFFFFFFFFu   /* slot of the creation draws */

struct orc_persist {
  orc_problem p;
  orc_options o;
  int nc, nb, nfx, nfy;
  uint64_t n, N;
  int F;
  double V, tau_min, lam_min;
  double *tau, *wall_T, *source, *ratio, *E;
  int64_t *Gw, *Gs;                 /* per iteration: wall emission [nb], source [nc] */
  double *x, *y, *sx, *sy;          /* particles */
  int64_t *q;
  int32_t *kind, *loc;
  int64_t *W, *Wh, *Phix, *Phiy, *B;
  uint32_t *Nrc, *Nb;
  int64_t *wc, *rc, *wb, *rb;       /* next weights, carried remainders */
  uint32_t iter;
  double d0, res;
  uint64_t flights, segments, crossings, tot_flights, tot_segments, tot_crossings;
};

void orc_persist_destroy(orc_persist *s)
{
  if (!s) return;
  free(s->tau); free(s->wall_T); free(s->source); free(s->ratio); free(s->E);
  free(s->Gw); free(s->Gs);
  free(s->x); free(s->y); free(s->sx); free(s->sy); free(s->q); free(s->kind); free(s->loc);
  free(s->W); free(s->Wh); free(s->Phix); free(s->Phiy); free(s->B); free(s->Nrc); free(s->Nb);
  free(s->wc); free(s->rc); free(s->wb); free(s->rb);
  free(s);
}

/* a = w n + r with 0 <= r < n (n > 0) */
static void orc_share(int64_t a, uint32_t n, int64_t *w, int64_t *r)
{
  int64_t nn = (int64_t)n;
  int64_t b = a / nn;
  if ((a % nn) != 0 && a < 0) b -= 1;
  *w = b;
  *r = a - b * nn;
}

static uint64_t orc_abs64(int64_t v) { return (v < 0) ? (uint64_t)0 - (uint64_t)v : (uint64_t)v; }

/* isotropic 3D direction, projected on the plane (as a cell's emission) */
static void orc_iso_dir(const orc_problem *p, double uc, double ud, double *sx, double *sy)
{
  double mu = 2.0 * uc - 1.0;
  *sx = mu;
  *sy = (p->dim == 2) ? sqrt((1.0 - mu) * (1.0 + mu)) * orc_cos2pi(ud) : 0.0;
}

int orc_persist_create(const orc_problem *p, const orc_options *o, orc_persist **out)
{
  *out = NULL;
  int rc = orc_validate(p);
  if (rc) return rc;
  if (p->n_bands > 1 || !o || o->particles_per_iter < 1 || o->max_iters < 0 ||
      o->avg_iters < 0 || o->newton || o->estimator != ORC_EST_ANALOG)
    return ORC_E_INVALID_ARG;
  const int nc = p->nx * p->ny, nb = orc_nb(p);
  uint64_t N = o->particles_per_iter / (uint64_t)(nc + nb);
  if (N < 1) N = 1;
  if (N * (uint64_t)(nc + nb) > 0xFFFFFFFEull) return ORC_E_INVALID_ARG;
  orc_persist *s = (orc_persist *)calloc(1, sizeof(orc_persist));
  s->p = *p;
  s->o = *o;
  s->nc = nc;
  s->nb = nb;
  s->nfx = p->ny * (p->nx + 1);
  s->nfy = (p->dim == 2) ? (p->ny + 1) * p->nx : 0;
  s->N = N;
  s->n = N * (uint64_t)(nc + nb);
  s->tau = orc_dup(p->tau, nc);
  s->wall_T = orc_dup(p->wall_T, nb);
  s->source = orc_dup(p->source, nc);
  s->p.tau = s->tau;
  s->p.wall_T = s->wall_T;
  s->p.source = s->source;
  s->p.T_init = NULL;
  s->p.diff_x = s->p.diff_y = NULL;
  s->F = orc_fixed_exponent(p, &s->tau_min);
  s->lam_min = p->vg * s->tau_min;
  s->V = p->dx * p->dy;
  s->ratio = (double *)malloc(sizeof(double) * nc);
  s->E = (double *)malloc(sizeof(double) * nc);
  s->Gw = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
  s->Gs = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  s->x = (double *)malloc(sizeof(double) * s->n);
  s->y = (double *)malloc(sizeof(double) * s->n);
  s->sx = (double *)malloc(sizeof(double) * s->n);
  s->sy = (double *)malloc(sizeof(double) * s->n);
  s->q = (int64_t *)malloc(sizeof(int64_t) * s->n);
  s->kind = (int32_t *)malloc(sizeof(int32_t) * s->n);
  s->loc = (int32_t *)malloc(sizeof(int32_t) * s->n);
  s->W = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  s->Wh = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  s->Nrc = (uint32_t *)calloc((size_t)nc, sizeof(uint32_t));
  s->Phix = (int64_t *)calloc((size_t)s->nfx, sizeof(int64_t));
  s->Phiy = (int64_t *)calloc((size_t)(s->nfy ? s->nfy : 1), sizeof(int64_t));
  s->B = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
  s->Nb = (uint32_t *)calloc((size_t)nb, sizeof(uint32_t));
  s->wc = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  s->rc = (int64_t *)calloc((size_t)nc, sizeof(int64_t));
  s->wb = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
  s->rb = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
  int ok = 1;
  for (int c = 0; c < nc; ++c) {
    s->ratio[c] = s->tau_min / s->tau[c];
    double T0 = p->T_init ? p->T_init[c] : p->t_ref;
    s->E[c] = p->cv * (T0 - p->t_ref);
    if (s->source) s->Gs[c] = orc_to_fixed((s->source[c] * s->V) * s->tau_min, s->F, &ok);
  }
  for (int b = 0; b < nb; ++b) {
    double A = (b < 2 * p->ny) ? p->dy : p->dx;
    double ew = p->cv * (s->wall_T[b] - p->t_ref);
    s->Gw[b] = orc_to_fixed((ew * (s->lam_min * A)) / 4.0, s->F, &ok);
  }
  /* step (1): N particles per cell in the local equilibrium, the cell's energy
     E V split over them, uniform positions and isotropic directions */
  uint64_t acc = 0;
  for (int c = 0; c < nc; ++c) {
    int ix = c % p->nx, iy = c / p->nx;
    int64_t G0 = orc_to_fixed(s->E[c] * s->V, s->F, &ok);
    for (uint64_t k = 0; k < N; ++k) {
      uint64_t i = (uint64_t)c * N + k;
      double ua, ub, uc, ud;
      orc_draw(o->seed, ORC_P_CREATE, ORC_P_STREAM, (uint32_t)i, 0u, &ua, &ub);
      orc_draw(o->seed, ORC_P_CREATE, ORC_P_STREAM, (uint32_t)i, 1u, &uc, &ud);
      s->x[i] = ((double)ix + ua) * p->dx;
      s->y[i] = ((double)iy + ub) * p->dy;
      orc_iso_dir(p, uc, ud, &s->sx[i], &s->sy[i]);
      s->q[i] = orc_split_weight(G0, N, k);
      s->kind[i] = ORC_P_NULL;
      s->loc[i] = c;
      acc += orc_abs64(s->q[i]);
      if (acc > ((uint64_t)1 << 62)) ok = 0;
    }
  }
  /* N particles per wall face, as if absorbed there: they carry the faces'
     first emission */
  for (int b = 0; b < nb; ++b) {
    for (uint64_t k = 0; k < N; ++k) {
      uint64_t i = (uint64_t)(nc + b) * N + k;
      s->x[i] = s->y[i] = s->sx[i] = s->sy[i] = 0.0;
      s->q[i] = 0;
      s->kind[i] = ORC_P_WALL;
      s->loc[i] = b;
    }
    orc_share(s->Gw[b], (uint32_t)N, &s->wb[b], &s->rb[b]);
    uint64_t a = orc_abs64(s->wb[b]) * N + orc_abs64(s->rb[b]);
    acc += a;
    if (acc > ((uint64_t)1 << 62)) ok = 0;
  }
  if (!ok) {
    orc_persist_destroy(s);
    return ORC_E_FIXED_OVERFLOW;
  }
  *out = s;
  return ORC_OK;
}

static int orc_persist_iterate(orc_persist *s, int faces)
{
  const orc_problem *p = &s->p;
  const int nx = p->nx, ny = p->ny, nc = s->nc, nb = s->nb;
  uint32_t slot = (s->o.rng_mode == ORC_RNG_CRN) ? s->o.rng_epoch : s->iter;
  memset(s->W, 0, sizeof(int64_t) * nc);
  memset(s->Wh, 0, sizeof(int64_t) * nc);
  memset(s->Nrc, 0, sizeof(uint32_t) * nc);
  memset(s->Phix, 0, sizeof(int64_t) * s->nfx);
  if (s->nfy) memset(s->Phiy, 0, sizeof(int64_t) * s->nfy);
  memset(s->B, 0, sizeof(int64_t) * nb);
  memset(s->Nb, 0, sizeof(uint32_t) * nb);
  orc_tally t;
  memset(&t, 0, sizeof t);
  t.Phix = s->Phix;
  t.Phiy = s->Phiy;
  t.faces = faces;
  uint64_t flights = 0, nul = 0;
  int ok = 1;
  for (uint64_t i = 0; i < s->n; ++i) {
    int ix, iy;
    if (s->kind[i] == ORC_P_REAL) {
      /* step (2): real collision -> resampled from the cell's equilibrium:
         uniform point of the cell, isotropic direction, the cell's share */
      int c = s->loc[i];
      double ua, ub, uc, ud;
      orc_draw(s->o.seed, slot, ORC_P_STREAM, (uint32_t)i, 0u, &ua, &ub);
      orc_draw(s->o.seed, slot, ORC_P_STREAM, (uint32_t)i, 1u, &uc, &ud);
      ix = c % nx;
      iy = c / nx;
      s->x[i] = ((double)ix + ua) * p->dx;
      s->y[i] = ((double)iy + ub) * p->dy;
      orc_iso_dir(p, uc, ud, &s->sx[i], &s->sy[i]);
      s->q[i] = s->wc[c];
    } else if (s->kind[i] == ORC_P_WALL) {
      /* absorbed by a black wall face: re-emitted from it (reading R1) */
      int b = s->loc[i];
      double ua, ub, uc, ud;
      orc_draw(s->o.seed, slot, ORC_P_STREAM, (uint32_t)i, 0u, &ua, &ub);
      orc_draw(s->o.seed, slot, ORC_P_STREAM, (uint32_t)i, 1u, &uc, &ud);
      double cn = sqrt(uc);
      double tg = (p->dim == 2) ? sqrt((1.0 - cn) * (1.0 + cn)) * orc_cos2pi(ud) : 0.0;
      int64_t w = s->wb[b];
      s->q[i] = w;
      if (b < ny) {
        ix = 0; iy = b;
        s->x[i] = 0.0; s->y[i] = ((double)iy + ua) * p->dy;
        s->sx[i] = cn; s->sy[i] = tg;
        if (faces) s->Phix[iy * (nx + 1)] += w;
      } else if (b < 2 * ny) {
        ix = nx - 1; iy = b - ny;
        s->x[i] = (double)nx * p->dx; s->y[i] = ((double)iy + ua) * p->dy;
        s->sx[i] = -cn; s->sy[i] = tg;
        if (faces) s->Phix[iy * (nx + 1) + nx] -= w;
      } else if (b < 2 * ny + nx) {
        ix = b - 2 * ny; iy = 0;
        s->x[i] = ((double)ix + ua) * p->dx; s->y[i] = 0.0;
        s->sx[i] = tg; s->sy[i] = cn;
        if (faces) s->Phiy[ix] += w;
      } else {
        ix = b - 2 * ny - nx; iy = ny - 1;
        s->x[i] = ((double)ix + ua) * p->dx; s->y[i] = (double)ny * p->dy;
        s->sx[i] = tg; s->sy[i] = -cn;
        if (faces) s->Phiy[ny * nx + ix] -= w;
      }
    } else {
      /* null collision: same position, direction and weight (step (6)) */
      int c = s->loc[i];
      ix = c % nx;
      iy = c / nx;
    }
    int64_t q = s->q[i];
    if (q != 0) flights++;
    /* step (3): one candidate path on the common time scale */
    double ulen, uacc;
    orc_draw(s->o.seed, slot, ORC_P_STREAM, (uint32_t)i, 2u, &ulen, &uacc);
    double ell = -(s->lam_min * orc_log(1.0 - ulen));
    double sx = s->sx[i], sy = s->sy[i];
    double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
    double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
    int bface = -1;
    if (orc_march(p, s->x[i], s->y[i], &ix, &iy, sx, sy, inv_sx, inv_sy, ell, q, &t, &bface)) {
      s->B[bface] += q;
      s->Nb[bface] += 1u;
      s->kind[i] = ORC_P_WALL;
      s->loc[i] = bface;
      continue;
    }
    /* steps (4)-(5): candidate collision, accepted with probability tau_min / tau */
    int c = ix + nx * iy;
    s->W[c] += q;
    s->x[i] = orc_clamp(s->x[i] + ell * sx, (double)ix * p->dx, (double)(ix + 1) * p->dx);
    if (p->dim == 2)
      s->y[i] = orc_clamp(s->y[i] + ell * sy, (double)iy * p->dy, (double)(iy + 1) * p->dy);
    s->loc[i] = c;
    if (uacc < s->ratio[c]) {
      s->Wh[c] += q;
      s->Nrc[c] += 1u;
      s->kind[i] = ORC_P_REAL;
    } else {
      s->kind[i] = ORC_P_NULL;
      nul += orc_abs64(q);
      if (nul > ((uint64_t)1 << 62)) nul = ((uint64_t)1 << 62) + 1;
    }
  }
  s->flights = flights;
  s->segments = s->n;
  s->crossings = t.crossings;
  s->tot_flights += flights;
  s->tot_segments += s->n;
  s->tot_crossings += t.crossings;
  /* E = W / V; shares of the real particles and of the walls for the next iteration */
  double *tmp = (double *)malloc(sizeof(double) * nc);
  int rc = ORC_OK;
  uint64_t acc = nul;
  const uint64_t cap = ((uint64_t)1 << 62) + 1;
  for (int c = 0; c < nc; ++c) {
    double En = ldexp((double)s->W[c], -s->F) / s->V;
    double d = En - s->E[c];
    tmp[c] = d * d;
    if (!isfinite(En)) rc = ORC_E_NONFINITE;
    s->E[c] = En;
    int64_t avail = orc_add(orc_add(s->Wh[c], s->Gs[c], &ok), s->rc[c], &ok);
    if (s->Nrc[c] > 0) {
      orc_share(avail, s->Nrc[c], &s->wc[c], &s->rc[c]);
    } else {
      s->wc[c] = 0;
      s->rc[c] = avail;
    }
    uint64_t a = orc_abs64(s->wc[c]) * (uint64_t)s->Nrc[c] + orc_abs64(s->rc[c]);
    acc = (acc + a > cap) ? cap : acc + a;
  }
  for (int b = 0; b < nb; ++b) {
    int64_t avail = orc_add(s->Gw[b], s->rb[b], &ok);
    if (s->Nb[b] > 0) {
      orc_share(avail, s->Nb[b], &s->wb[b], &s->rb[b]);
    } else {
      s->wb[b] = 0;
      s->rb[b] = avail;
    }
    uint64_t a = orc_abs64(s->wb[b]) * (uint64_t)s->Nb[b] + orc_abs64(s->rb[b]);
    acc = (acc + a > cap) ? cap : acc + a;
  }
  double dn = sqrt(orc_tree_sum(tmp, (uint64_t)nc));
  free(tmp);
  if (s->iter == 0) s->d0 = dn;
  s->res = (s->d0 > 0.0) ? dn / s->d0 : 0.0;
  s->iter++;
  if (rc == ORC_OK && (!ok || acc > ((uint64_t)1 << 62))) rc = ORC_E_FIXED_OVERFLOW;
  if (rc == ORC_OK && s->iter > 1 && s->res > 1e3) rc = ORC_E_DIVERGED;
  return rc;
}

int orc_persist_step(orc_persist *s, int n_iters, int faces)
{
  for (int i = 0; i < n_iters; ++i) {
    int rc = orc_persist_iterate(s, faces);
    if (rc) return rc;
  }
  return ORC_OK;
}

int orc_persist_solve(orc_persist *s, double *T_out, double *qx_out, double *qy_out)
{
  const orc_problem *p = &s->p;
  int faces_each = (s->o.tally_faces == ORC_FACES_EVERY);
  int faces_out = (s->o.tally_faces != ORC_FACES_OFF);
  int converged = 0, rc;
  while ((int)s->iter < s->o.max_iters) {
    rc = orc_persist_iterate(s, faces_each);
    if (rc) return rc;
    if (s->res < s->o.res_tol) {
      converged = 1;
      break;
    }
  }
  double *Eo = (double *)calloc((size_t)s->nc, sizeof(double));
  double *fx = (double *)calloc((size_t)s->nfx, sizeof(double));
  double *fy = (double *)calloc((size_t)(s->nfy ? s->nfy : 1), sizeof(double));
  if (s->o.avg_iters > 0) {
    for (int a = 0; a < s->o.avg_iters; ++a) {
      rc = orc_persist_iterate(s, faces_out);
      if (rc) { free(Eo); free(fx); free(fy); return rc; }
      for (int c = 0; c < s->nc; ++c) Eo[c] = Eo[c] + s->E[c];
      for (int f = 0; f < s->nfx; ++f) fx[f] = fx[f] + ldexp((double)s->Phix[f], -s->F);
      for (int f = 0; f < s->nfy; ++f) fy[f] = fy[f] + ldexp((double)s->Phiy[f], -s->F);
    }
    double na = (double)s->o.avg_iters;
    for (int c = 0; c < s->nc; ++c) Eo[c] = Eo[c] / na;
    for (int f = 0; f < s->nfx; ++f) fx[f] = fx[f] / na;
    for (int f = 0; f < s->nfy; ++f) fy[f] = fy[f] / na;
  } else {
    if (s->o.tally_faces == ORC_FACES_FINAL) {
      rc = orc_persist_iterate(s, 1);
      if (rc) { free(Eo); free(fx); free(fy); return rc; }
    }
    for (int c = 0; c < s->nc; ++c) Eo[c] = s->E[c];
    for (int f = 0; f < s->nfx; ++f) fx[f] = ldexp((double)s->Phix[f], -s->F);
    for (int f = 0; f < s->nfy; ++f) fy[f] = ldexp((double)s->Phiy[f], -s->F);
  }
  if (T_out)
    for (int c = 0; c < s->nc; ++c) T_out[c] = p->t_ref + Eo[c] / p->cv;
  if (qx_out) {
    double den = p->dy * s->tau_min;
    for (int f = 0; f < s->nfx; ++f) qx_out[f] = faces_out ? fx[f] / den : 0.0;
  }
  if (qy_out && s->nfy) {
    double den = p->dx * s->tau_min;
    for (int f = 0; f < s->nfy; ++f) qy_out[f] = faces_out ? fy[f] / den : 0.0;
  }
  free(Eo);
  free(fx);
  free(fy);
  return converged ? ORC_OK : ORC_W_NOT_CONVERGED;
}

void orc_persist_get_info(const orc_persist *s, orc_info *info)
{
  memset(info, 0, sizeof *info);
  info->iter = s->iter;
  info->F = s->F;
  info->n_per_emitter = s->N;
  info->n_cells = s->nc;
  info->n_bfaces = s->nb;
  info->n_emitters = s->nc;
  info->tau_min = s->tau_min;
  info->lam_min = s->lam_min;
  info->d0 = s->d0;
  info->res = s->res;
  info->flights = s->flights;
  info->segments = s->segments;
  info->crossings = s->crossings;
  info->tot_flights = s->tot_flights;
  info->tot_segments = s->tot_segments;
  info->tot_crossings = s->tot_crossings;
}

void orc_persist_get_E(const orc_persist *s, double *E) { memcpy(E, s->E, sizeof(double) * s->nc); }

uint64_t orc_persist_count(const orc_persist *s) { return s->n; }

void orc_persist_get_particles(const orc_persist *s, double *x, double *y, double *sx, double *sy,
                               int64_t *q, int32_t *kind, int32_t *loc)
{
  if (x) memcpy(x, s->x, sizeof(double) * s->n);
  if (y) memcpy(y, s->y, sizeof(double) * s->n);
  if (sx) memcpy(sx, s->sx, sizeof(double) * s->n);
  if (sy) memcpy(sy, s->sy, sizeof(double) * s->n);
  if (q) memcpy(q, s->q, sizeof(int64_t) * s->n);
  if (kind) memcpy(kind, s->kind, sizeof(int32_t) * s->n);
  if (loc) memcpy(loc, s->loc, sizeof(int32_t) * s->n);
}

void orc_persist_get_tallies(const orc_persist *s, int64_t *W, int64_t *Wh, uint32_t *Nrc,
                             int64_t *Phix, int64_t *Phiy, int64_t *B, uint32_t *Nb)
{
  if (W) memcpy(W, s->W, sizeof(int64_t) * s->nc);
  if (Wh) memcpy(Wh, s->Wh, sizeof(int64_t) * s->nc);
  if (Nrc) memcpy(Nrc, s->Nrc, sizeof(uint32_t) * s->nc);
  if (Phix) memcpy(Phix, s->Phix, sizeof(int64_t) * s->nfx);
  if (Phiy && s->nfy) memcpy(Phiy, s->Phiy, sizeof(int64_t) * s->nfy);
  if (B) memcpy(B, s->B, sizeof(int64_t) * s->nb);
  if (Nb) memcpy(Nb, s->Nb, sizeof(uint32_t) * s->nb);
}

void orc_persist_get_shares(const orc_persist *s, int64_t *wc, int64_t *rc, int64_t *wb,
                            int64_t *rb)
{
  if (wc) memcpy(wc, s->wc, sizeof(int64_t) * s->nc);
  if (rc) memcpy(rc, s->rc, sizeof(int64_t) * s->nc);
  if (wb) memcpy(wb, s->wb, sizeof(int64_t) * s->nb);
  if (rb) memcpy(rb, s->rb, sizeof(int64_t) * s->nb);
}
