// kernels.hpp -- gfx950 kernels of one IUGKP iteration.
//
//   prepare_kernel   zero the tallies, split every emitter's integer energy over
//                    its N particles (floor + remainder), put the wall emission on
//                    the wall faces
//   march_kernel     Sec. 3.1 step (2) / Sec. 3.2 steps (3)-(5): sample, fly, tally
//   update kernels   Sec. 3.1 step (3) / Sec. 3.3: E^{n+1/2} = W / V, Newton RHS,
//                    next emission, squared update per cell, fixed-order partials
//   finish_kernel    fixed-order totals -> relative residual, status flags
//   newton_operator_kernel / cg_kernel   the diffusion correction of Sec. 3.3
//
// Reductions that feed floating-point results use one fixed order: blocks of 256
// consecutive values (zero-padded), each reduced by halving strides
// (v[i] += v[i + s], s = 128 ... 1); the block sums are reduced the same way.
// Integer tallies use 64-bit atomics: exact, so any order gives the same bits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "device_core.hpp"

namespace iugkp {

constexpr int kTree = 256;                       // fixed reduction block
constexpr uint32_t kMaxSegments = 1u << 20;      // last allowed segment always ends real
constexpr unsigned long long kBudgetCap = (1ull << 62) + 1ull;

struct Mesh {
  int dim, nx, ny;
  int n_cells, n_b, n_emit;
  int n_fx, n_fy;
  double dx, dy;
};

// Device-side scalars of one solve: the last iteration's counters and norms,
// and the iteration control used when a batch advances on its own.
struct DevScalars {
  unsigned long long flights, segments, crossings;
  unsigned long long tot_flights, tot_segments, tot_crossings;
  unsigned long long gsum;      // saturating sum of |G| (Newton emission budget)
  double dn, d0, res;
  double res_p1, res_p2;        // residuals of the two preceding iterations (+inf: none)
  int grew;                     // the Newton iteration's growth rule fired this iteration
  int flags;                    // bit 0: non-finite energy, bit 1: fixed-point overflow
  int cg_iters, cg_status, cg_iters_total;
  unsigned long long cg_t0, cg_t1;   // device wall clock at the multigrid CG's start and end
  unsigned int iter;            // iterations done
  int state;                    // 0 iterating, 1 output iterations, 2 done
  int out_left;                 // output iterations still to run (state 1)
  int faces_now;                // face tallies in the next iteration
  int acc_mode;                 // last iteration feeds the outputs: 0 no, 1 add, 2 restart
  int converged;
  int err;                      // first error of the solve (negative code) or 0
};

// A persistent particle's straight path of one move, kept for the row-stripe
// pass of its y-face tallies: start point, direction (s_x and the two
// reciprocals of the walk), weight, start cell (column | row << 16) and the
// number of y faces crossed.
struct PFace {
  double x0, y0, sx, inv_sx, inv_sy;
  long long q;
  uint32_t cell, nyp;
};

// Everything the per-iteration kernels need about one problem instance.
struct Inst {
  Mesh m;
  double lam_min, V, t_ref, cv, tau_min, res_tol, tol2;
  int F;
  uint32_t N, key0, key1, epoch;
  int crn, has_null, newton, faces_each, faces_out, final_iter, avg_iters, max_iters, cg_max;
  int WX, WY, lds_walls;
  const double *ratio;
  double *E, *E_half, *rhs;
  long long *G, *base;
  uint32_t *rem;
  long long *D, *W, *Phix, *Phiy, *dB, *B;
  double *part;                 // squared-update partials [ceil(n_emit / 256)]
  unsigned long long *gpart;    // |G| budget partials
  const double *gx, *gy, *diag;
  double *cg_x, *cg_r, *cg_w, *cg_p, *cg_s, *cg_part;   // CG state (global-memory layout)
  double *cg_pub, *cg_mpart;                            // published rows, partials
  unsigned int *cg_barrier;                             // [2] barrier of the instance's group
  double *acc_E, *acc_x, *acc_y;
  const long long *Gs;          // per-cell source emission per iteration, or null
  int estimator;                // 0 sampled collision points, 1 expected deposits along the ray
  uint32_t e_off;               // emitter offset in the Philox counter (frequency band k: k (nc + nb))
  int n_bands;                  // > 1: the coordinating instance of a multi-band problem
  unsigned long long wall_budget;   // saturating sum of |G| over the wall emitters
  // persistent particles (one population kept between iterations)
  int persist;
  unsigned int n_part;          // population: N per cell, then N per wall face
  double *px, *py, *psx, *psy;  // position, direction
  long long *pq;                // weight
  uint32_t *plk;                // location | kind << 30 (kind 0 null, 1 real, 2 wall)
  uint32_t *Nrc, *Nb;           // real collisions per cell, absorptions per wall face
  long long *wc, *rc, *wb, *rb; // next weights and carried remainders (cells, wall faces)
  const long long *Gw;          // wall emission per iteration
  long long *pstart;            // energy starting this iteration's paths in each cell
  long long *pein;              // energy re-emitted this iteration by each wall face
  PFace *pf;                    // row-stripe face pass: each move's path, and its crossed
  uint32_t *pkey;               //   y faces' range (first | last << 16; kNoFaces if none)
  unsigned long long *npart;    // per move workgroup: saturating sum of |q| over null particles
  int n_npart, n_gpart;
  DevScalars *sc;
};

// a + b for |a|, |b| <= 2^62 (two's complement, no overflow trap); sets
// *bad when |a + b| exceeds the 2^62 budget
__device__ __forceinline__ long long add_budget(long long a, long long b, int *bad)
{
  const long long r = static_cast<long long>(static_cast<unsigned long long>(a) +
                                             static_cast<unsigned long long>(b));
  if (r > (1ll << 62) || r < -(1ll << 62)) *bad = 1;
  return r;
}

// ---------------------------------------------------------------------------
// Fixed-order tree over 256 values held by 256 consecutive threads (one
// "slice"; a workgroup may hold several slices).  Levels s = 128 and 64 go
// through LDS, the last six (s = 32 .. 1) inside the first wavefront of the
// slice with shuffles; every level adds v[i] + v[i + s], exactly the pairs and
// the operand order of the reference tree.  Returns the sum in the slice's
// thread 0 (other threads: unspecified).  All threads of the workgroup call it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double slice_tree256(double v, double *lds)
{
  const int t = threadIdx.x & (kTree - 1);
  double *sl = lds + (threadIdx.x - t);
  sl[t] = v;
  __syncthreads();
  if (t < 128) sl[t] = sl[t] + sl[t + 128];
  __syncthreads();
  double r = 0.0;
  if (t < 64) {
    r = sl[t] + sl[t + 64];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) r = r + __shfl_down(r, s, 64);
  }
  __syncthreads();
  return r;
}

// Whole-workgroup version for 256-wide workgroups: result broadcast to all threads.
__device__ __forceinline__ double block_tree256(double v, double *lds)
{
  const double r = slice_tree256(v, lds);
  if (threadIdx.x == 0) lds[0] = r;
  __syncthreads();
  const double out = lds[0];
  __syncthreads();
  return out;
}

// Reduce n (<= 65536) block sums with the same tree (two levels at most);
// blockDim.x >= 256, all threads call it, all get the result.  lds needs
// blockDim.x doubles, lds2 256.
__device__ double tree_all(const double *part, int n, double *lds, double *lds2)
{
  const int nb = (n + kTree - 1) / kTree;
  const int slices = blockDim.x / kTree;
  const int sl = threadIdx.x / kTree, t = threadIdx.x & (kTree - 1);
  for (int b0 = 0; b0 < nb; b0 += slices) {
    const int b = b0 + sl;
    const int i = b * kTree + t;
    const double v = (b < nb && i < n) ? part[i] : 0.0;
    const double r = slice_tree256(v, lds);
    if (t == 0 && b < nb) lds2[b] = r;
  }
  __syncthreads();
  double out;
  if (nb == 1) {
    out = lds2[0];
  } else {
    const double v = (threadIdx.x < nb) ? lds2[threadIdx.x] : 0.0;
    const double r = slice_tree256(threadIdx.x < kTree ? v : 0.0, lds);
    if (threadIdx.x == 0) lds2[0] = r;
    __syncthreads();
    out = lds2[0];
  }
  __syncthreads();
  return out;
}

// ---------------------------------------------------------------------------
// prepare: zero tallies, per-emitter split, wall emission on the wall faces.
// Grid (x: elements, y: instance).  faces_mode >= 0 forces the face tallies,
// -1 takes them from the instance's iteration control; with `batch` set,
// finished instances are skipped.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool inst_idle(const Inst &in, int batch)
{
  return batch && in.sc->state == 2;
}

__device__ __forceinline__ int inst_faces(const Inst &in, int faces_mode)
{
  return faces_mode >= 0 ? faces_mode : in.sc->faces_now;
}

__global__ void prepare_kernel(const Inst *__restrict__ insts, int faces_mode, int batch)
{
  const Inst &in = insts[blockIdx.y];
  if (inst_idle(in, batch)) return;
  const Mesh &m = in.m;
  const int faces = inst_faces(in, faces_mode);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    in.sc->flights = 0;
    in.sc->segments = 0;
    in.sc->crossings = 0;
    in.sc->gsum = 0;
    in.sc->flags = 0;
  }
  if (i < m.n_cells) {
    in.D[i] = 0;
    in.W[i] = 0;
  }
  if (i < m.n_b) in.B[i] = 0;
  if (i < m.n_emit) {
    // floor division of a signed energy by N with a non-negative remainder
    const long long g = in.G[i];
    const long long n = static_cast<long long>(in.N);
    long long b = g / n;
    if (g % n != 0 && g < 0) b -= 1;
    in.base[i] = b;
    in.rem[i] = static_cast<uint32_t>(g - b * n);
  }
  if (i < m.n_fx) in.Phix[i] = 0;   // rebuilt from the balance when faces are on
  if (m.dim == 2 && i < (m.ny + 2) * m.nx) in.dB[i] = 0;
  if (i < m.n_fy) {
    long long v = 0;
    if (faces) {
      const int k = i / m.nx, col = i - k * m.nx;
      if (k == 0) v = in.G[m.n_cells + 2 * m.ny + col];
      else if (k == m.ny) v = -in.G[m.n_cells + 2 * m.ny + m.nx + col];
    }
    in.Phiy[i] = v;
  }
}

// ---------------------------------------------------------------------------
// The particle step.
//
// Work decomposition: workgroup = one emitter tile (a TX x TY block of cells, or
// a segment of one wall) and all N particles of its emitters; particle p of the
// tile belongs to emitter p mod n_e (emitters run fastest, so the lanes of a
// wavefront start in different cells) and has index k = p / n_e within it.
// Each lane flies its particles one after the other, which evens out the
// lanes' total work.
//
// Tallies: the workgroup keeps the cell tallies (D, W), the y-face tallies and
// the column-run differences of a window of cells around its tile in LDS
// (64-bit LDS atomics), and flushes the window with row-contiguous (coalesced)
// global atomics at the end; events outside the window go to global atomics.
// x-face tallies are not taken at all: they follow exactly from the per-cell
// identity  net face inflow = D - G  (reconstruct_faces_kernel).  For steep
// segments the y-faces crossed inside one column form a run [lo, hi]; it is
// recorded as +q at lo and -q at hi + 1 of a per-column difference array,
// two updates instead of one per face.
// ---------------------------------------------------------------------------
struct TileDesc {
  int inst;        // instance of the batch
  int kind;        // 0 = cell tile, 1 = wall segment
  int x0, y0;      // cell tile: first cell; wall segment: first wall index in x0
  int ex, ey;      // cell tile: extent; wall segment: face count in ex
  int wx0, wy0;    // window origin (cells)
};

__device__ __forceinline__ void atom_add(long long *a, long long v)
{
  atomicAdd(reinterpret_cast<unsigned long long *>(a), static_cast<unsigned long long>(v));
}

__device__ __forceinline__ double clamp_to(double v, double lo, double hi)
{
  return (v < lo) ? lo : ((v > hi) ? hi : v);
}

struct Window {
  long long *D, *W, *By, *dB, *B;   // LDS arrays
  int wx0, wy0, WX, WY;
};

// LDS layout of one window: D [WY][WX], W [WY][WX] (null collisions only),
// By [WY+1][WX], dB [WY+2][WX], B [n_b] (if kept in LDS).
__host__ __device__ inline size_t window_words(int WX, int WY, int has_null, int lds_walls, int n_b)
{
  return static_cast<size_t>(WX) * WY * (has_null ? 2 : 1) + static_cast<size_t>(WX) * (WY + 1) +
         static_cast<size_t>(WX) * (WY + 2) + (lds_walls ? n_b : 0);
}

// The flight of particle k of emitter e carrying q: sampling (start point,
// direction), free paths on the common time scale, the DDA walk through the
// uniform grid and the candidate/real collision decisions.  The tallies are
// callbacks, so the particle step and the adjoint's path tracing share one
// definition of the path:
//   add_diff(k, ix, v)   column-run difference of y-faces in column ix
//   add_yface(ky, ix, v) one y-face crossing
//   add_wall(b, q)       absorbed by boundary face b
//   add_cand(ix, iy, q)  candidate collision (null-collision runs only)
//   add_real(ix, iy, q)  real collision (deposit)
// Number of faces j = 0..jmax of the sequence k(j) = k0 + j st reached before
// T: t(j) = (k(j) d - p0) * inv < T (STRICT) or <= T.  t(j) is the walk's own
// expression and is non-decreasing in j (each rounding step is monotone), so
// the faces reached form a prefix and a binary search finds its length.
template <bool STRICT>
__device__ __forceinline__ int faces_before(int k0, int st, int jmax, double d, double p0,
                                            double inv, double T)
{
  int lo = 0, hi = jmax + 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const double t = (static_cast<double>(k0 + mid * st) * d - p0) * inv;
    if (STRICT ? (t < T) : (t <= T)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The same count, estimated from the coordinate reached at T (direction
// component from the hardware's approximate reciprocal of inv: an estimate
// only) and checked against the walk's own times t(lo - 1) and t(lo); a miss
// (a crossing within rounding of a face, or a poor estimate) falls back to the
// search, so the result is always faces_before's.
template <bool STRICT>
__device__ __forceinline__ int faces_before_near(int k0, int st, int jmax, double d, double inv_d,
                                                 double p0, double inv, double T)
{
  const double pos = p0 + T * __builtin_amdgcn_rcp(inv);
  const double jr = (st > 0) ? pos * inv_d - static_cast<double>(k0)
                             : static_cast<double>(k0) - pos * inv_d;
  int lo;
  if (!(jr < static_cast<double>(jmax))) lo = jmax + 1;
  else if (!(jr >= 0.0)) lo = 0;
  else lo = static_cast<int>(floor(jr)) + 1;
  // (t at an index outside [0, jmax] is plain arithmetic, its result unused)
  auto t = [&](int j) { return (static_cast<double>(k0 + j * st) * d - p0) * inv; };
  auto before = [&](double tj) { return STRICT ? (tj < T) : (tj <= T); };
  const bool ok = (lo == 0 || before(t(lo - 1))) && (lo > jmax || !before(t(lo)));
  return ok ? lo : faces_before<STRICT>(k0, st, jmax, d, p0, inv, T);
}

// The walk of one segment of length ell from (x0, y0) in cell (ix, iy) with
// no face tallies, in closed form (segment_end also returns the x and y faces
// crossed, nxp and nyp, a crossed wall face included).  Crossings before ell in each direction are
// prefixes of the face sequences (faces_before); the walk ends at the first
// wall face in time order (x first on ties) or in the cell reached after all
// crossings.  Same final cell, wall face (bface, else left at -1) and crossing
// count as the face-by-face walk.  kx, ky: the first faces ahead.
__device__ __forceinline__ void segment_end(const Mesh &m, double x0, double y0, int &ix, int &iy,
                                            int stx, int sty, double inv_sx, double inv_sy, int kx,
                                            int ky, double ell, int &bface, int &nxp, int &nyp)
{
  const int jwx = (stx > 0) ? m.nx - kx : kx;   // position of the x wall in the sequence
  const int jwy = (sty > 0) ? m.ny - ky : ky;
  // (approximate reciprocals: they only feed the estimates)
  const double inv_dx = __builtin_amdgcn_rcp(m.dx), inv_dy = __builtin_amdgcn_rcp(m.dy);
  const int nxc = stx ? faces_before_near<true>(kx, stx, jwx, m.dx, inv_dx, x0, inv_sx, ell) : 0;
  const int nyc = sty ? faces_before_near<true>(ky, sty, jwy, m.dy, inv_dy, y0, inv_sy, ell) : 0;
  const bool wx = stx && nxc > jwx, wy = sty && nyc > jwy;
  if (wx || wy) {
    const int kwx = kx + jwx * stx, kwy = ky + jwy * sty;
    const double Tx = wx ? (static_cast<double>(kwx) * m.dx - x0) * inv_sx : INFINITY;
    const double Ty = wy ? (static_cast<double>(kwy) * m.dy - y0) * inv_sy : INFINITY;
    if (wx && Tx <= Ty) {
      const int nb = sty ? faces_before_near<true>(ky, sty, jwy, m.dy, inv_dy, y0, inv_sy, Tx) : 0;
      iy += sty * nb;
      nxp = jwx + 1;
      nyp = nb;
      bface = (kwx == 0) ? iy : m.ny + iy;
    } else {
      const int nb = stx ? faces_before_near<false>(kx, stx, jwx, m.dx, inv_dx, x0, inv_sx, Ty) : 0;
      ix += stx * nb;
      nxp = nb;
      nyp = jwy + 1;
      bface = (kwy == 0) ? 2 * m.ny + ix : 2 * m.ny + m.nx + ix;
    }
  } else {
    ix += stx * nxc;
    iy += sty * nyc;
    nxp = nxc;
    nyp = nyc;
  }
}

__device__ __forceinline__ void segment_jump(const Mesh &m, double x0, double y0, int &ix, int &iy,
                                             int stx, int sty, double inv_sx, double inv_sy, int kx,
                                             int ky, double ell, int &bface,
                                             unsigned long long &n_cross)
{
  int nxp = 0, nyp = 0;
  segment_end(m, x0, y0, ix, iy, stx, sty, inv_sx, inv_sy, kx, ky, ell, bface, nxp, nyp);
  n_cross += static_cast<unsigned long long>(nxp + nyp);
}

// A segment expected to cross more faces than this is resolved in closed form
// when no face is tallied (same outcome as the walk, see fly()).
constexpr double kJumpMinFaces = 6.0;
// idle lanes of a wavefront that start new particles together (tile march
// with null collisions), and the particles per lane of a tile from which the
// lanes refill at all (below it each lane flies its few particles in turn)
constexpr int kRefillLanes = 32;
constexpr uint32_t kRefillMinPer = 4;

struct FlyIn {
  Mesh m;
  double lam_min;
  uint32_t slot, key0, key1;
  int faces, has_null;
  const double *ratio;
  uint32_t e_off;        // added to the emitter index in the Philox counter
};

// Start point and direction of particle k of emitter e: a uniform point of the
// cell and an isotropic 3D direction projected on the plane (cell emitters),
// or a uniform point of the wall face and a cosine-law direction into the
// domain (wall emitters).
__device__ __forceinline__ void sample_particle(const FlyIn &a, uint32_t e, uint32_t k, int &ix,
                                                int &iy, double &x0, double &y0, double &sx,
                                                double &sy)
{
  const Mesh &m = a.m;
  const double2 uab = draw2(0u, k, e + a.e_off, a.slot, a.key0, a.key1);
  const double2 ucd = draw2(1u, k, e + a.e_off, a.slot, a.key0, a.key1);
  if (e < static_cast<uint32_t>(m.n_cells)) {
    // isotropic emission from a uniformly sampled point of the cell
    iy = static_cast<int>(e) / m.nx;
    ix = static_cast<int>(e) - iy * m.nx;
    x0 = (static_cast<double>(ix) + uab.x) * m.dx;
    y0 = (static_cast<double>(iy) + uab.y) * m.dy;
    const double mu = 2.0 * ucd.x - 1.0;
    sx = mu;
    sy = (m.dim == 2) ? sqrt((1.0 - mu) * (1.0 + mu)) * cos2pi_own(ucd.y) : 0.0;
  } else {
    // cosine-law emission from a black wall face into the domain
    const int b = static_cast<int>(e) - m.n_cells;
    const double cn = sqrt(ucd.x);
    const double tg = (m.dim == 2) ? sqrt((1.0 - cn) * (1.0 + cn)) * cos2pi_own(ucd.y) : 0.0;
    if (b < m.ny) {
      ix = 0; iy = b;
      x0 = 0.0; y0 = (static_cast<double>(iy) + uab.x) * m.dy;
      sx = cn; sy = tg;
    } else if (b < 2 * m.ny) {
      ix = m.nx - 1; iy = b - m.ny;
      x0 = static_cast<double>(m.nx) * m.dx; y0 = (static_cast<double>(iy) + uab.x) * m.dy;
      sx = -cn; sy = tg;
    } else if (b < 2 * m.ny + m.nx) {
      ix = b - 2 * m.ny; iy = 0;
      x0 = (static_cast<double>(ix) + uab.x) * m.dx; y0 = 0.0;
      sx = tg; sy = cn;
    } else {
      ix = b - 2 * m.ny - m.nx; iy = m.ny - 1;
      x0 = (static_cast<double>(ix) + uab.x) * m.dx; y0 = static_cast<double>(m.ny) * m.dy;
      sx = tg; sy = -cn;
    }
  }
}

// An analog flight's state between two segments: fly() runs one to its end,
// the tile march's lanes with null collisions run theirs a segment at a time
// and take the next particle when one ends.
struct Flight {
  uint32_t e, k, j;
  long long q, qy;
  int ix, iy, stx, sty;
  double x0, y0, sx, sy, inv_sx, inv_sy;
  bool runs;
  // the open run of y faces in the current column (first and last face, or
  // run_a = -1): it stays open across null collisions, which keep the
  // direction and the column
  int run_a, run_b;
  // pending candidate tallies: n candidates of weight q in cell (cand_x, cand_y)
  int cand_x, cand_y;
  long long cand_n;
};

__device__ __forceinline__ void flight_start(const FlyIn &a, uint32_t e, uint32_t k, long long q,
                                             Flight &f)
{
  sample_particle(a, e, k, f.ix, f.iy, f.x0, f.y0, f.sx, f.sy);
  f.e = e;
  f.k = k;
  f.j = 0;
  f.q = q;
  f.inv_sx = (f.sx != 0.0) ? 1.0 / f.sx : 0.0;
  f.inv_sy = (f.sy != 0.0) ? 1.0 / f.sy : 0.0;
  f.stx = (f.sx > 0.0) ? 1 : ((f.sx < 0.0) ? -1 : 0);
  f.sty = (f.sy > 0.0) ? 1 : ((f.sy < 0.0) ? -1 : 0);
  f.qy = (f.sty > 0) ? q : -q;
  // steep flights record their y-faces as runs per column
  f.runs = a.faces && (fabs(f.sy) > 2.0 * fabs(f.sx));
  f.run_a = -1;
  f.run_b = -1;
  f.cand_x = -1;
  f.cand_y = -1;
  f.cand_n = 0;
}

// The flight's next segment and its tallies: true after a null collision
// (another segment follows), false when the flight ended (its pending
// candidates tallied).
template <class Diff, class YFace, class Wall, class Cand, class Real>
__device__ __forceinline__ bool flight_segment(const FlyIn &a, Flight &f, Diff &&add_diff,
                                               YFace &&add_yface, Wall &&add_wall, Cand &&add_cand,
                                               Real &&add_real, unsigned long long &n_seg,
                                               unsigned long long &n_cross)
{
  const Mesh &m = a.m;
  // n q modulo 2^64, the same bits as n separate integer additions
  auto times = [](long long v, long long n) {
    return static_cast<long long>(static_cast<unsigned long long>(v) * static_cast<unsigned long long>(n));
  };
  const uint32_t j = f.j;
  const double2 us = draw2(2u + j, f.k, f.e + a.e_off, a.slot, a.key0, a.key1);
  // candidate free path on the common time scale tau_min: -|V_g| tau_min ln(eta)
  const double ell = -(a.lam_min * log_own(1.0 - us.x));
  ++n_seg;
  const int stx = f.stx, sty = f.sty;
  int ix = f.ix, iy = f.iy;
  int kx = (stx > 0) ? ix + 1 : ix;
  int ky = (sty > 0) ? iy + 1 : iy;
  int bface = -1;
  int run_a = f.run_a, run_b = f.run_b;   // first and last y-face of the open run
  if (!a.faces && ell * (fabs(f.sx) / m.dx + fabs(f.sy) / m.dy) > kJumpMinFaces) {
    segment_jump(m, f.x0, f.y0, ix, iy, stx, sty, f.inv_sx, f.inv_sy, kx, ky, ell, bface, n_cross);
  } else
  for (;;) {
    const double tx = stx ? (static_cast<double>(kx) * m.dx - f.x0) * f.inv_sx : INFINITY;
    const double ty = sty ? (static_cast<double>(ky) * m.dy - f.y0) * f.inv_sy : INFINITY;
    const bool along_x = tx <= ty;
    const double tt = along_x ? tx : ty;
    if (!(tt < ell)) break;
    ++n_cross;
    if (along_x) {
      if (run_a >= 0) {
        add_diff(min(run_a, run_b), ix, f.qy);
        add_diff(max(run_a, run_b) + 1, ix, -f.qy);
        run_a = -1;
      }
      if (kx == 0 || kx == m.nx) {
        bface = (kx == 0) ? iy : m.ny + iy;
        break;
      }
      ix += stx;
      kx += stx;
    } else {
      if (f.runs) {
        if (run_a < 0) run_a = ky;
        run_b = ky;
      } else if (a.faces) {
        add_yface(ky, ix, f.qy);
      }
      if (ky == 0 || ky == m.ny) {
        bface = (ky == 0) ? 2 * m.ny + ix : 2 * m.ny + m.nx + ix;
        break;
      }
      iy += sty;
      ky += sty;
    }
  }
  f.ix = ix;
  f.iy = iy;
  bool more = false;
  if (bface >= 0) {
    add_wall(bface, f.q);
  } else if (!a.has_null) {
    add_real(ix, iy, f.q);   // every candidate is real: W == D
  } else {
    // candidates in the same cell one after the other are tallied together
    if (ix == f.cand_x && iy == f.cand_y) {
      ++f.cand_n;
    } else {
      if (f.cand_n) add_cand(f.cand_x, f.cand_y, times(f.q, f.cand_n));
      f.cand_x = ix;
      f.cand_y = iy;
      f.cand_n = 1;
    }
    // accept with probability sigma / sigma_max = tau_min / tau_c
    const int c = ix + m.nx * iy;
    if (us.y < a.ratio[c] || j == kMaxSegments - 1) {
      add_real(ix, iy, f.q);
    } else {
      // null collision: keep the direction, restart from the stopping point
      f.x0 = clamp_to(f.x0 + ell * f.sx, static_cast<double>(ix) * m.dx,
                      static_cast<double>(ix + 1) * m.dx);
      if (m.dim == 2)
        f.y0 = clamp_to(f.y0 + ell * f.sy, static_cast<double>(iy) * m.dy,
                        static_cast<double>(iy + 1) * m.dy);
      f.j = j + 1;
      more = true;
    }
  }
  if (!more && f.cand_n) add_cand(f.cand_x, f.cand_y, times(f.q, f.cand_n));
  // the run stays open into the next segment (same column, the next face)
  if (!more && run_a >= 0) {
    add_diff(min(run_a, run_b), ix, f.qy);
    add_diff(max(run_a, run_b) + 1, ix, -f.qy);
    run_a = -1;
  }
  f.run_a = run_a;
  f.run_b = run_b;
  return more;
}

template <class Diff, class YFace, class Wall, class Cand, class Real>
__device__ __forceinline__ void fly(const FlyIn &a, uint32_t e, uint32_t k, long long q,
                                    Diff &&add_diff, YFace &&add_yface, Wall &&add_wall,
                                    Cand &&add_cand, Real &&add_real, unsigned long long &n_seg,
                                    unsigned long long &n_cross)
{
  Flight f;
  flight_start(a, e, k, q, f);
  while (flight_segment(a, f, add_diff, add_yface, add_wall, add_cand, add_real, n_seg, n_cross)) {
  }
}

// Expected-value flight of particle k of emitter e carrying q (variance
// reduction; the expectation of fly()).  Same start and direction, no free
// path: the ray is followed cell by cell with optical depth
// T += chord tau_min / (lambda_min tau_c); with S(T) = rint(q exp(-T)) a
// cell's chord from T_a to T_b deposits S(T_a) - S(T_b) as real collisions
// (exactly conserved) and, with null collisions, the expected candidates
// rint(q (exp(-T_a) - exp(-T_b)) / ratio_c); a crossed face carries S, a wall
// face absorbs it; the ray ends at the first face where S is 0.  A candidate
// deposit beyond 2^62 sets `bad`.
template <class YFace, class Wall, class Cand, class Real>
__device__ __forceinline__ void fly_expected(const FlyIn &a, uint32_t e, uint32_t k, long long q,
                                             YFace &&add_yface, Wall &&add_wall, Cand &&add_cand,
                                             Real &&add_real, unsigned long long &n_seg,
                                             unsigned long long &n_cross, int &bad)
{
  const Mesh &m = a.m;
  int ix, iy;
  double x0, y0, sx, sy;
  sample_particle(a, e, k, ix, iy, x0, y0, sx, sy);
  ++n_seg;
  const double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
  const double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
  const int stx = (sx > 0.0) ? 1 : ((sx < 0.0) ? -1 : 0);
  const int sty = (sy > 0.0) ? 1 : ((sy < 0.0) ? -1 : 0);
  int kx = (stx > 0) ? ix + 1 : ix;
  int ky = (sty > 0) ? iy + 1 : iy;
  const double qd = static_cast<double>(q);
  double T = 0.0, surv = 1.0, tprev = 0.0;
  long long S = q;
  const double inv_lam = 1.0 / a.lam_min;   // = ratio / lambda_min where ratio is 1
  auto cand = [&](int cx, int cy, double v, double ratio) {
    const double x = v / ratio;
    if (!(fabs(x) <= 4611686018427387904.0)) {
      bad = 1;
      return;
    }
    const long long w = static_cast<long long>(rint(x));
    if (w) add_cand(cx, cy, w);
  };
  for (;;) {
    const int c = ix + m.nx * iy;
    const double tx = stx ? (static_cast<double>(kx) * m.dx - x0) * inv_sx : INFINITY;
    const double ty = sty ? (static_cast<double>(ky) * m.dy - y0) * inv_sy : INFINITY;
    const bool along_x = tx <= ty;
    const double tt = along_x ? tx : ty;
    if (!(tt < INFINITY)) {
      if (S) add_real(ix, iy, S);
      if (a.has_null) cand(ix, iy, qd * surv, a.ratio[c]);
      return;
    }
    const double ratio = a.has_null ? a.ratio[c] : 1.0;
    const double Tn = T + (tt - tprev) * (a.has_null ? ratio / a.lam_min : inv_lam);
    const double sn = expm_own(Tn);
    const long long Sn = static_cast<long long>(rint(qd * sn));
    if (S != Sn) add_real(ix, iy, S - Sn);
    if (a.has_null) cand(ix, iy, qd * (surv - sn), ratio);
    T = Tn;
    surv = sn;
    S = Sn;
    tprev = tt;
    if (S == 0) return;
    ++n_cross;
    if (along_x) {
      if (kx == 0 || kx == m.nx) {
        add_wall((kx == 0) ? iy : m.ny + iy, S);
        return;
      }
      ix += stx;
      kx += stx;
    } else {
      if (a.faces) add_yface(ky, ix, sty > 0 ? S : -S);
      if (ky == 0 || ky == m.ny) {
        add_wall((ky == 0) ? 2 * m.ny + ix : 2 * m.ny + m.nx + ix, S);
        return;
      }
      iy += sty;
      ky += sty;
    }
  }
}

// EV: also the expected-value flights of instances that ask for them (a
// separate instantiation, so the analog kernel keeps its register budget).
template <int BS, bool EV>
__global__ __launch_bounds__(BS) void march_kernel(const Inst *__restrict__ insts,
                                                   const TileDesc *__restrict__ tiles,
                                                   int faces_mode, int batch,
                                                   unsigned long long *__restrict__ clk)
{
  extern __shared__ long long lds_words[];
  __shared__ unsigned long long s_cnt[3];
  __shared__ uint32_t s_next;          // the tile's next unclaimed particle (null collisions)
  const TileDesc td = tiles[blockIdx.x];
  const Inst &in = insts[td.inst];
  if (inst_idle(in, batch)) return;
  // (clk: the workgroup's start and end on the device clock and its flights,
  // for the batch's tile-size choice)
  const unsigned long long t_start = clk ? static_cast<unsigned long long>(wall_clock64()) : 0ull;
  struct {
    Mesh m;
    double lam_min;
    uint32_t N, slot, key0, key1;
    int faces, has_null;
    const long long *base;
    const uint32_t *rem;
    const double *ratio;
    long long *D, *W, *Phiy, *dB, *B;
    DevScalars *sc;
  } a = {in.m, in.lam_min, in.N, in.crn ? in.epoch : in.sc->iter, in.key0, in.key1,
         inst_faces(in, faces_mode), in.has_null, in.base, in.rem, in.ratio, in.D, in.W,
         in.Phiy, in.dB, in.B, in.sc};
  const Mesh &m = a.m;
  Window win;
  win.WX = in.WX;
  win.WY = in.WY;
  win.wx0 = td.wx0;
  win.wy0 = td.wy0;
  {
    long long *p = lds_words;
    win.D = p;
    p += win.WX * win.WY;
    win.W = a.has_null ? p : nullptr;
    if (a.has_null) p += win.WX * win.WY;
    win.By = p;
    p += win.WX * (win.WY + 1);
    win.dB = p;
    p += win.WX * (win.WY + 2);
    win.B = in.lds_walls ? p : nullptr;
  }
  const int nwords = static_cast<int>(window_words(win.WX, win.WY, a.has_null, in.lds_walls, m.n_b));
  for (int i = threadIdx.x; i < nwords; i += BS) lds_words[i] = 0;
  if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_next = 0;
  __syncthreads();

  auto add_cell = [&](long long *lds_arr, long long *glob, int ix, int iy, long long v) {
    const unsigned lx = static_cast<unsigned>(ix - win.wx0), ly = static_cast<unsigned>(iy - win.wy0);
    if (lx < static_cast<unsigned>(win.WX) && ly < static_cast<unsigned>(win.WY))
      atomicAdd(reinterpret_cast<unsigned long long *>(&lds_arr[ly * win.WX + lx]),
                static_cast<unsigned long long>(v));
    else
      atom_add(&glob[iy * m.nx + ix], v);
  };
  auto add_yface = [&](int ky, int ix, long long v) {
    const unsigned lx = static_cast<unsigned>(ix - win.wx0), ly = static_cast<unsigned>(ky - win.wy0);
    if (lx < static_cast<unsigned>(win.WX) && ly <= static_cast<unsigned>(win.WY))
      atomicAdd(reinterpret_cast<unsigned long long *>(&win.By[ly * win.WX + lx]),
                static_cast<unsigned long long>(v));
    else
      atom_add(&a.Phiy[ky * m.nx + ix], v);
  };
  auto add_diff = [&](int k, int ix, long long v) {
    const unsigned lx = static_cast<unsigned>(ix - win.wx0), ly = static_cast<unsigned>(k - win.wy0);
    if (lx < static_cast<unsigned>(win.WX) && ly <= static_cast<unsigned>(win.WY + 1))
      atomicAdd(reinterpret_cast<unsigned long long *>(&win.dB[ly * win.WX + lx]),
                static_cast<unsigned long long>(v));
    else
      atom_add(&a.dB[k * m.nx + ix], v);
  };
  auto add_wall = [&](int b, long long v) {
    if (win.B)
      atomicAdd(reinterpret_cast<unsigned long long *>(&win.B[b]), static_cast<unsigned long long>(v));
    else
      atom_add(&a.B[b], v);
  };

  const FlyIn fa = {a.m, a.lam_min, a.slot, a.key0, a.key1, a.faces, a.has_null, a.ratio, in.e_off};
  const int n_e = (td.kind == 0) ? td.ex * td.ey : td.ex;
  const uint32_t P = static_cast<uint32_t>(n_e) * a.N;
  unsigned long long n_fl = 0, n_seg = 0, n_cross = 0;
  int bad = 0;
  // particle p of the tile: emitter (tile order) fastest
  auto emitter_of = [&](uint32_t p, uint32_t &e, uint32_t &k) {
    const uint32_t ei = p % static_cast<uint32_t>(n_e);
    k = p / static_cast<uint32_t>(n_e);
    if (td.kind == 0) {
      const int ty = static_cast<int>(ei) / td.ex;
      e = static_cast<uint32_t>((td.y0 + ty) * m.nx + td.x0 + (static_cast<int>(ei) - ty * td.ex));
    } else {
      e = static_cast<uint32_t>(m.n_cells + td.x0) + ei;
    }
  };
  auto add_w = [&](int cx, int cy, long long v) { add_cell(win.W, a.W, cx, cy, v); };
  auto add_d = [&](int cx, int cy, long long v) { add_cell(win.D, a.D, cx, cy, v); };
  if (!(EV && in.estimator) && a.has_null && P >= kRefillMinPer * BS) {
    // Null collisions make a flight a chain of segments of geometric length:
    // each lane runs its flight a segment per trip, and the idle lanes of a
    // wavefront claim the tile's next particles (one LDS atomic per
    // wavefront) once kRefillLanes of them are idle (or no lane is busy), so
    // that a wavefront is not held by its longest chain and the sampling of
    // new particles runs once for many lanes.
    const int lane = static_cast<int>(threadIdx.x & 63);
    Flight f;
    bool live = false, done = false;
    for (;;) {
      const unsigned long long busy = __ballot(live);
      const unsigned long long idle = __ballot(!live && !done);
      if (!busy && !idle) break;
      if (!live && !done && (__popcll(idle) >= kRefillLanes || !busy)) {
        bool got = false;
        for (;;) {
          const unsigned long long want = __ballot(true);
          const int lead = __ffsll(static_cast<long long>(want)) - 1;
          uint32_t first = 0;
          if (lane == lead) first = atomicAdd(&s_next, static_cast<uint32_t>(__popcll(want)));
          first = static_cast<uint32_t>(__shfl(static_cast<int>(first), lead, 64));
          const uint32_t p = first + static_cast<uint32_t>(__popcll(want & ((1ull << lane) - 1ull)));
          if (p >= P) break;
          uint32_t e, k;
          emitter_of(p, e, k);
          const long long q = a.base[e] + ((k < a.rem[e]) ? 1 : 0);
          if (q == 0) continue;
          flight_start(fa, e, k, q, f);
          got = true;
          break;
        }
        if (got) {
          ++n_fl;
          live = true;
        } else {
          done = true;
        }
      }
      if (live) live = flight_segment(fa, f, add_diff, add_yface, add_wall, add_w, add_d, n_seg, n_cross);
    }
  } else
  for (uint32_t p = threadIdx.x; p < P; p += BS) {
    uint32_t e, k;
    emitter_of(p, e, k);
    const long long q = a.base[e] + ((k < a.rem[e]) ? 1 : 0);
    if (q == 0) continue;
    ++n_fl;
    if (EV && in.estimator)
      fly_expected(fa, e, k, q, add_yface, add_wall, add_w, add_d, n_seg, n_cross, bad);
    else
      fly(fa, e, k, q, add_diff, add_yface, add_wall, add_w, add_d, n_seg, n_cross);
  }
  if (bad) atomicOr(&a.sc->flags, 2);
  if (n_fl) {
    atomicAdd(&s_cnt[0], n_fl);
    atomicAdd(&s_cnt[1], n_seg);
    atomicAdd(&s_cnt[2], n_cross);
  }
  __syncthreads();
  // flush the window: row-contiguous, so neighbouring lanes update one cache line
  auto flush = [&](const long long *src, long long *dst, int rows, int row0, int nrows_glob) {
    for (int i = threadIdx.x; i < rows * win.WX; i += BS) {
      const long long v = src[i];
      if (v == 0) continue;
      const int ly = i / win.WX, lx = i - ly * win.WX;
      const int gx = win.wx0 + lx, gy = row0 + ly;
      if (gx >= 0 && gx < m.nx && gy >= 0 && gy < nrows_glob) atom_add(&dst[gy * m.nx + gx], v);
    }
  };
  flush(win.D, a.D, win.WY, win.wy0, m.ny);
  if (a.has_null) flush(win.W, a.W, win.WY, win.wy0, m.ny);
  if (a.faces && m.dim == 2) {
    flush(win.By, a.Phiy, win.WY + 1, win.wy0, m.ny + 1);
    flush(win.dB, a.dB, win.WY + 2, win.wy0, m.ny + 2);
  }
  if (win.B)
    for (int b = threadIdx.x; b < m.n_b; b += BS)
      if (win.B[b]) atom_add(&a.B[b], win.B[b]);
  if (threadIdx.x == 0 && s_cnt[0]) {
    atomicAdd(&a.sc->flights, s_cnt[0]);
    atomicAdd(&a.sc->segments, s_cnt[1]);
    atomicAdd(&a.sc->crossings, s_cnt[2]);
  }
  if (clk) {
    __syncthreads();
    if (threadIdx.x == 0) {
      clk[3 * blockIdx.x] = t_start;
      clk[3 * blockIdx.x + 1] = static_cast<unsigned long long>(wall_clock64());
      clk[3 * blockIdx.x + 2] = s_cnt[0];
    }
  }
}

// Number of faces j <= jmax of the sequence k(j) = k0 + j st with
// t(j) = (k(j) d - p0) * inv <= T, given that the first cnt are: galloping
// from cnt, then bisection (t is non-decreasing in j).
__device__ __attribute__((noinline)) int faces_upto_from(int cnt, int k0, int st, int jmax,
                                                        double d, double p0, double inv, double T)
{
  int lo = cnt, hi = jmax + 1, step = 1;
  for (;;) {
    const int probe = lo + step - 1;
    if (probe > jmax) break;
    const double t = (static_cast<double>(k0 + probe * st) * d - p0) * inv;
    if (!(t <= T)) {
      hi = probe;
      break;
    }
    lo = probe + 1;
    step <<= 1;
  }
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const double t = (static_cast<double>(k0 + mid * st) * d - p0) * inv;
    if (t <= T) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The same count, estimated from the coordinate reached at T, pos = p0 + T s
// (faces at or before pos: floor(pos / d - k0) + 1 for st > 0,
// floor(k0 - pos / d) + 1 for st < 0) and checked against the walk's own
// times: the estimate c is the count when t(c - 1) <= T (or c = cnt) and
// t(c) > T (or c > jmax).  Rounding in the estimate and in the walk's
// comparisons place the crossing point within a few units in the last place
// of a coordinate, so a miss is rare; it is settled by the search above
// (kept out of line).  No loop on the common path: a loop there costs the
// whole wavefront its slowest lane's trip count at every crossing.
__device__ __forceinline__ int faces_upto_near(int cnt, int k0, int st, int jmax, double d,
                                               double inv_d, double p0, double inv, double s,
                                               double T)
{
  const double pos = p0 + T * s;
  const double jr = (st > 0) ? pos * inv_d - static_cast<double>(k0)
                             : static_cast<double>(k0) - pos * inv_d;
  int lo;
  if (!(jr < static_cast<double>(jmax))) lo = jmax + 1;
  else if (!(jr >= static_cast<double>(cnt))) lo = cnt;
  else lo = static_cast<int>(floor(jr)) + 1;
  // (t at an index outside [0, jmax] is plain arithmetic, its result unused)
  auto t = [&](int j) { return (static_cast<double>(k0 + j * st) * d - p0) * inv; };
  const double ta = t(lo - 1), tb = t(lo);
  const bool ok = (lo == cnt || ta <= T) && (lo > jmax || !(tb <= T));
  return ok ? lo : faces_upto_from(cnt, k0, st, jmax, d, p0, inv, T);
}

// ---------------------------------------------------------------------------
// The particle step with face tallies for long free paths, by row stripes.
// Workgroup (chunk c, stripe s) keeps in LDS the y-face tallies of faces
// [r0, r1f) (the last stripe also owns face ny) and the wall tallies, and
// runs every particle of its chunk: start and first segment from the
// records sampled once for all stripes (stripe_presample_kernel), later
// segments' ends in closed form (segment_end), then only the y faces it
// crosses inside the stripe, each in the column reached by the
// x faces crossed first (x first on ties, as in the walk).  A particle's
// deposits, wall absorption and counters go to the stripe holding the row
// where that event happens; the deposits (one per particle, one W per null
// segment) go straight to global memory, which leaves the LDS to the y faces
// and so roughly halves the number of stripes that read each particle.  All
// tallies are integer sums, so the result is the tile kernel's bit for bit.
// Each lane runs a small state machine, one trip per segment (an idle lane
// takes its next particle; then the segment's owned y-face crossings and its
// end), so a lane with a long flight holds the others of its wavefront for
// one segment at a time.
// ---------------------------------------------------------------------------
// Every particle's start and first segment, sampled once per iteration for
// all row stripes: weight, start point and direction, start and end cells
// (16-bit columns and rows), the wall face that absorbs the segment or -1,
// the y faces and all faces it crosses, and the particle's place in the
// enumeration (its random-number counters); with null collisions also the
// free path and the acceptance draw.  64 bytes, or 80 with null collisions.
// The records are binned by start stripe and direction of travel: start
// stripe t owns K sub-bins of slots, sub-bin k for the particles that pre-pass
// blocks k, k + K, ... sample (the host counts them exactly), each filled from
// the front by the particles whose rows stay inside the stripe and from the
// back by those that leave it.  A stripe reads the particles that start in it
// without a check, and only the other stripes' leavers against its rows.  A
// block claims its slots of a bin with one atomic; the K sub-bins spread
// those atomics over K counters per bin (one counter per bin took 3.5 ms per
// launch to serialise the claims of 1e7 particles).
struct alignas(16) PRec {
  long long q;
  double x0, y0, sx, sy;
  uint32_t cell, cell_e;     // ix | iy << 16, ixe | iye << 16
  int bface;
  uint32_t nyp, ncross, pc;
};
struct alignas(16) PRecN {   // with null collisions
  PRec c;
  double ell, uacc;
};
static_assert(sizeof(PRec) == 64 && sizeof(PRecN) == 80, "record sizes");
// and, beside a leaver's record, the rows that stripes must run the particle
// in (lo, hi): the rows of a first segment that is the whole flight (up to the
// wall for an absorption on a y wall), or with null collisions every row in
// its direction of travel, as two 16-bit rows (lo in the high half).  A
// stripe reads these 4 bytes to skip another stripe's leaver that does not
// reach its rows, not the whole record.
constexpr int kStripeSegMax = 1024;   // (S + 1) K segments at most (the march's segment table)
constexpr int kStripeBinMax = 64;     // bins (start stripe, direction) of a pre-pass block
constexpr int kPresampleBlock = 1024; // pre-pass threads per block,
constexpr int kPresamplePer = 1;      // particles per thread
struct StripeRec {
  void *r;                   // PRec, or PRecN with null collisions [particles]
  uint32_t *key;             // [particles]
  uint32_t *cnt;             // [S K][2]: per sub-bin, records filled from the front, from the back
  const uint32_t *base;      // [S K + 1]: first slot of sub-bin t K + k
  int R, S, K;               // rows per stripe, stripes, sub-bins per stripe
};
__device__ __forceinline__ uint32_t row_range(int lo, int hi)
{
  return (static_cast<uint32_t>(lo) << 16) | static_cast<uint32_t>(hi);
}

// (dynamic LDS: the block's records, sorted by bin, then their slots)
template <int BS, bool NUL>
__global__ __launch_bounds__(BS) void stripe_presample_kernel(const Inst *__restrict__ insts,
                                                              StripeRec rec)
{
  using Rec = typename std::conditional<NUL, PRecN, PRec>::type;
  constexpr int kWords = static_cast<int>(sizeof(Rec) / sizeof(uint4));
  static_assert(sizeof(Rec) % sizeof(uint4) == 0, "records are whole 16-byte words");
  static_assert(kPresamplePer == 1, "one particle per thread");
  extern __shared__ uint4 srec[];                                   // [BS][kWords]
  uint32_t *const s_dst = reinterpret_cast<uint32_t *>(srec + BS * kWords);   // [BS]
  __shared__ uint32_t s_n[kStripeBinMax], s_g[kStripeBinMax], s_off[kStripeBinMax + 1];
  const Inst &in = insts[0];
  const Mesh &m = in.m;
  const FlyIn fa = {m, in.lam_min, in.crn ? in.epoch : in.sc->iter, in.key0, in.key1, 1,
                    in.has_null, in.ratio, in.e_off};
  const unsigned long long n_emit = static_cast<unsigned long long>(m.n_emit);
  const unsigned long long total = n_emit * in.N;
  const int nbin = 2 * rec.S, k = static_cast<int>(blockIdx.x % static_cast<unsigned>(rec.K));
  for (int b = threadIdx.x; b < nbin; b += BS) s_n[b] = 0;
  __syncthreads();
  Rec rc_out;
  PRec &out = *reinterpret_cast<PRec *>(&rc_out);     // (the common part comes first)
  uint32_t key = 0, rank = 0;
  int bin = -1;
  const int lane = static_cast<int>(threadIdx.x & 63);
  const unsigned long long pc = static_cast<unsigned long long>(blockIdx.x) * BS + threadIdx.x;
  if (pc < total) {
    // (32-bit: the planner keeps the particles below 2^32)
    const uint32_t pc32 = static_cast<uint32_t>(pc), ne32 = static_cast<uint32_t>(n_emit);
    const uint32_t kk = pc32 / ne32;
    const uint32_t e = pc32 - kk * ne32;
    const long long q = in.base[e] + ((kk < in.rem[e]) ? 1 : 0);
    if (q != 0) {
      int ix = 0, iy = 0;
      double x0 = 0.0, y0 = 0.0, sx = 0.0, sy = 0.0;
      sample_particle(fa, e, kk, ix, iy, x0, y0, sx, sy);
      const double2 us = draw2(2u, kk, e + fa.e_off, fa.slot, fa.key0, fa.key1);
      const double ell = -(fa.lam_min * log_own(1.0 - us.x));
      const double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
      const double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
      const int stx = (sx > 0.0) ? 1 : ((sx < 0.0) ? -1 : 0);
      const int sty = (sy > 0.0) ? 1 : ((sy < 0.0) ? -1 : 0);
      const int kx0 = (stx > 0) ? ix + 1 : ix;
      const int ky0 = (sty > 0) ? iy + 1 : iy;
      int ixe = ix, iye = iy, bface = -1, nxp = 0, nyp = 0;
      segment_end(m, x0, y0, ixe, iye, stx, sty, inv_sx, inv_sy, kx0, ky0, ell, bface, nxp, nyp);
      out.q = q;
      out.x0 = x0;
      out.y0 = y0;
      out.sx = sx;
      out.sy = sy;
      out.cell = static_cast<uint32_t>(ix) | (static_cast<uint32_t>(iy) << 16);
      out.cell_e = static_cast<uint32_t>(ixe) | (static_cast<uint32_t>(iye) << 16);
      out.bface = bface;
      out.nyp = static_cast<uint32_t>(nyp);
      out.ncross = static_cast<uint32_t>(nxp + nyp);
      out.pc = static_cast<uint32_t>(pc);
      if constexpr (NUL) {
        rc_out.ell = ell;
        rc_out.uacc = us.y;
      }
      int lo = min(iy, iye), hi = max(iy, iye);
      if (fa.has_null) {
        lo = (sty < 0) ? 0 : iy;
        hi = (sty > 0) ? m.ny - 1 : iy;
      } else if (bface >= 2 * m.ny) {
        if (sty > 0) hi = m.ny - 1;
        else lo = 0;
      }
      key = row_range(lo, hi);
      bin = 2 * (iy / rec.R) + ((lo / rec.R != hi / rec.R) ? 1 : 0);
    }
  }
  // the particle's rank in its bin within the block: one LDS atomic per bin
  // and wavefront
  unsigned long long pending = __ballot(bin >= 0);
  while (pending) {
    const int lead = __ffsll(static_cast<long long>(pending)) - 1;
    const int bl = __shfl(bin, lead, 64);
    const unsigned long long mine = __ballot(bin == bl);
    uint32_t first = 0;
    if (lane == lead) first = atomicAdd(&s_n[bl], static_cast<uint32_t>(__popcll(mine)));
    first = static_cast<uint32_t>(__shfl(static_cast<int>(first), lead, 64));
    if ((mine >> lane) & 1ull)
      rank = first + static_cast<uint32_t>(__popcll(mine & ((1ull << lane) - 1ull)));
    pending &= ~mine;
  }
  __syncthreads();
  // the block's slots (one atomic per bin on sub-bin k's counter) and the
  // bins' places in the block's sorted records (a scan by wavefront 0)
  for (int b = threadIdx.x; b < nbin; b += BS)
    s_g[b] = s_n[b] ? atomicAdd(&rec.cnt[2 * ((b >> 1) * rec.K + k) + (b & 1)], s_n[b]) : 0u;
  if (threadIdx.x < 64) {
    const uint32_t v = (lane < nbin) ? s_n[lane] : 0u;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), d, 64));
      if (lane >= d) incl += o;
    }
    s_off[lane] = incl - v;
    if (lane == 63) s_off[64] = incl;
  }
  __syncthreads();
  if (bin >= 0) {
    const int sb = (bin >> 1) * rec.K + k;
    const uint32_t r = s_g[bin] + rank;
    const uint32_t slot = (bin & 1) ? rec.base[sb + 1] - 1u - r : rec.base[sb] + r;
    const uint32_t j = s_off[bin] + rank;
    const uint4 *src = reinterpret_cast<const uint4 *>(&rc_out);
#pragma unroll
    for (int i = 0; i < kWords; ++i) srec[j * kWords + i] = src[i];
    s_dst[j] = slot;
    if (bin & 1) rec.key[slot] = key;
  }
  __syncthreads();
  // out as 16-byte words, consecutive threads on consecutive words of the
  // sorted records (the runs of one bin are consecutive slots)
  const int nw = static_cast<int>(s_off[64]) * kWords;
  Rec *const dst = static_cast<Rec *>(rec.r);
  for (int i = threadIdx.x; i < nw; i += BS) {
    const int j = i / kWords, w = i - j * kWords;
    reinterpret_cast<uint4 *>(dst + s_dst[j])[w] = srec[i];
  }
}

// The segment table of a stripe's candidates (one thread per segment):
// segment i < 2K is this stripe's sub-bin i / 2, its front (stayers) or back
// (leavers); then, for each other stripe in order, its K sub-bins' leavers.
// s_slot: the first slot of each; s_pre: their starts in one running count
// (a workgroup scan of the counts), s_pre[(S + 1) K] the total.  Ends with a
// barrier.
template <int BS>
__device__ __forceinline__ void stripe_segment_table(const StripeRec &rec, uint32_t *s_pre,
                                                     uint32_t *s_slot, uint32_t *s_wsum)
{
  static_assert(BS >= kStripeSegMax, "one thread per segment");
  const int K = rec.K, nseg = (rec.S + 1) * K, nown = 2 * K;
  {
    const int sb = static_cast<int>(blockIdx.y);
    const int i = static_cast<int>(threadIdx.x);
    uint32_t cnt = 0, first = 0;
    if (i < nseg) {
      int t, kb, back;
      if (i < nown) {
        t = sb;
        kb = i >> 1;
        back = i & 1;
      } else {
        const int j = i - nown;
        t = j / K;
        kb = j - t * K;
        if (t >= sb) ++t;
        back = 1;
      }
      const int sub = t * K + kb;
      cnt = rec.cnt[2 * sub + back];
      first = back ? rec.base[sub + 1] - cnt : rec.base[sub];
      s_slot[i] = first;
    }
    // exclusive scan of the counts over the workgroup (BS >= nseg)
    const int lane = i & 63, w = i >> 6;
    uint32_t incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), d, 64));
      if (lane >= d) incl += o;
    }
    if (lane == 63) s_wsum[w] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int v = 0; v < w; ++v) off += s_wsum[v];
    if (i < nseg) s_pre[i] = off + incl - cnt;
    if (i == nseg - 1) s_pre[nseg] = off + incl;
  }
  __syncthreads();
}

template <int BS>
__global__ __launch_bounds__(BS) void march_stripes_kernel(const Inst *__restrict__ insts, int R,
                                                           int chunks, StripeRec rec)
{
  extern __shared__ long long lds_words[];
  __shared__ unsigned long long s_cnt[3];
  // the stripe's candidates as segments of slots: its own stayers, its own
  // leavers, then every other start stripe's leavers (checked against the
  // rows); s_pre: their starts in one running count
  static_assert(BS >= kStripeSegMax, "one thread per segment");
  __shared__ uint32_t s_pre[kStripeSegMax + 1], s_slot[kStripeSegMax];
  __shared__ uint32_t s_wsum[BS / 64];
  const Inst &in = insts[0];
  // (the mesh and the tally pointers in registers: reloaded inside the state
  // machine, each load would also wait for the lane's pending LDS atomics)
  const Mesh m = in.m;
  long long *const gD = in.D, *const gW = in.W, *const gB = in.B, *const gPhiy = in.Phiy;
  const bool lds_walls = in.lds_walls != 0;
  const int nx = m.nx;
  const int r0 = static_cast<int>(blockIdx.y) * R, r1 = min(r0 + R, m.ny);
  const int r1f = (r1 == m.ny) ? m.ny + 1 : r1;
  const int nface = r1f - r0;
  long long *By = lds_words;                                  // [nface][nx]
  long long *Bl = By + nface * nx;                            // [n_b] when lds_walls
  const int nwords = nface * nx + (lds_walls ? m.n_b : 0);
  for (int i = threadIdx.x; i < nwords; i += BS) lds_words[i] = 0;
  if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
  // the candidates: segments of slots (this stripe's stayers and leavers, then
  // the other stripes' leavers), their starts in one running count
  const int K = rec.K, nseg = (rec.S + 1) * K, nown = 2 * K;
  stripe_segment_table<BS>(rec, s_pre, s_slot, s_wsum);
  auto lds_add = [](long long *p, long long v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
  };

  const FlyIn fa = {m, in.lam_min, in.crn ? in.epoch : in.sc->iter, in.key0, in.key1, 1,
                    in.has_null, in.ratio, in.e_off};
  const unsigned long long n_emit = static_cast<unsigned long long>(m.n_emit);
  const uint32_t V = s_pre[nseg];
  const uint32_t vb = static_cast<uint32_t>(static_cast<unsigned long long>(V) * blockIdx.x / chunks);
  const uint32_t ve = static_cast<uint32_t>(static_cast<unsigned long long>(V) * (blockIdx.x + 1) / chunks);
  unsigned long long n_fl = 0, n_seg = 0, n_cross = 0;
  const double inv_dx = 1.0 / m.dx;       // (only to estimate a face count)
  // the lane's next candidate, located (segment, slot) and, for another
  // stripe's leaver, its row range loaded, one particle ahead
  uint32_t vnext = vb + threadIdx.x;
  int sg = 0;
  uint32_t nslot = 0, nkey = 0;
  bool nchk = false;
  auto locate = [&](uint32_t v) {
    while (sg + 1 < nseg && v >= s_pre[sg + 1]) ++sg;
    nslot = s_slot[sg] + (v - s_pre[sg]);
    nchk = sg >= nown;
    nkey = nchk ? rec.key[nslot] : 0u;
  };
  if (vnext < ve) locate(vnext);

  // the lane's particle
  bool live = false;
  uint32_t e = 0, kk = 0, j = 0;
  long long q = 0, qy = 0;
  int ix = 0, iy = 0, stx = 0, sty = 0;
  double x0 = 0.0, y0 = 0.0, sx = 0.0, sy = 0.0, inv_sx = 0.0, inv_sy = 0.0;
  unsigned p_seg = 0, p_cross = 0;
  // its current segment
  double ell = 0.0, uacc = 0.0;
  int kx0 = 0, ky0 = 0, ixs = 0, jwx = 0, k = 0, k_end = 0, cnt = 0, ixe = 0, iye = 0, bface = -1;

  auto draw_path = [&]() {
    const double2 us = draw2(2u + j, kk, e + fa.e_off, fa.slot, fa.key0, fa.key1);
    ell = -(fa.lam_min * log_own(1.0 - us.x));
    uacc = us.y;
  };
  // a segment from (x0, y0) in cell (ix, iy): its first faces; then, given the
  // y faces it crosses, those this stripe owns
  auto segment_faces = [&]() {
    kx0 = (stx > 0) ? ix + 1 : ix;
    ky0 = (sty > 0) ? iy + 1 : iy;
    ixs = ix;
    jwx = (stx > 0) ? nx - kx0 : kx0;
  };
  auto owned_faces = [&](int nyp) {
    // the crossed y faces ky0 + k sty (k < nyp) that this stripe owns
    if (sty > 0) {
      k = max(0, r0 - ky0);
      k_end = min(nyp, r1f - ky0);
    } else if (sty < 0) {
      k = max(0, ky0 - r1f + 1);
      k_end = min(nyp, ky0 - r0 + 1);
    } else {
      k = 0;
      k_end = 0;
    }
    cnt = 0;
  };
  auto start_segment = [&]() {      // a later segment (after a null collision)
    ++p_seg;
    segment_faces();
    ixe = ix;
    iye = iy;
    bface = -1;
    int nxp = 0, nyp = 0;
    segment_end(m, x0, y0, ixe, iye, stx, sty, inv_sx, inv_sy, kx0, ky0, ell, bface, nxp, nyp);
    p_cross += static_cast<unsigned>(nxp + nyp);
    owned_faces(nyp);
  };
  auto owned = [&](int row) { return row >= r0 && row < r1; };
  auto retire = [&]() {          // the particle ended in row iye of this stripe
    ++n_fl;
    n_seg += p_seg;
    n_cross += p_cross;
  };

  for (;;) {
    if (!live) {
      bool got = false;
      uint32_t slot = 0;
      while (vnext < ve) {
        slot = nslot;
        const uint32_t key = nkey;
        const bool chk = nchk;
        vnext += BS;
        if (vnext < ve) locate(vnext);
        // another stripe's leaver that cannot reach these rows has nothing here
        if (chk && (static_cast<int>(key & 0xffffu) < r0 || static_cast<int>(key >> 16) >= r1))
          continue;
        got = true;
        break;
      }
      if (!got) break;
      // (the record's common part comes first in both forms)
      const unsigned char *rb = static_cast<const unsigned char *>(rec.r) +
                                static_cast<size_t>(slot) * (fa.has_null ? sizeof(PRecN) : sizeof(PRec));
      const PRec &rp = *reinterpret_cast<const PRec *>(rb);
      const uint32_t pc = rp.pc, ne32 = static_cast<uint32_t>(n_emit);
      kk = pc / ne32;
      e = pc - kk * ne32;
      q = rp.q;
      const uint32_t cs = rp.cell, ce = rp.cell_e;
      ix = static_cast<int>(cs & 0xffffu);
      iy = static_cast<int>(cs >> 16);
      ixe = static_cast<int>(ce & 0xffffu);
      iye = static_cast<int>(ce >> 16);
      sy = rp.sy;
      sty = (sy > 0.0) ? 1 : ((sy < 0.0) ? -1 : 0);
      x0 = rp.x0;
      y0 = rp.y0;
      sx = rp.sx;
      if (fa.has_null) {
        const PRecN &rn = *reinterpret_cast<const PRecN *>(rb);
        ell = rn.ell;
        uacc = rn.uacc;
      }
      bface = rp.bface;
      const int nyp = static_cast<int>(rp.nyp);
      inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
      inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
      stx = (sx > 0.0) ? 1 : ((sx < 0.0) ? -1 : 0);
      qy = (sty > 0) ? q : -q;
      j = 0;
      p_seg = 1;
      p_cross = static_cast<unsigned>(rp.ncross);
      live = true;
      segment_faces();
      owned_faces(nyp);
    }
    {
      // all the segment's owned y-face crossings, each in the column reached
      // by the x faces before it, in one trip through the state machine
      // (one trip per crossing cost a fifth more)
      for (; k < k_end; ++k) {
        const int kyk = ky0 + k * sty;
        const double ty = (static_cast<double>(kyk) * m.dy - y0) * inv_sy;
        if (stx) cnt = faces_upto_near(cnt, kx0, stx, jwx, m.dx, inv_dx, x0, inv_sx, sx, ty);
        lds_add(&By[(kyk - r0) * nx + ixs + stx * cnt], qy);
      }
    }
    // the segment's end (in the same trip)
    if (bface >= 0) {
      if (owned(iye)) {
        if (!lds_walls) atom_add(&gB[bface], q);
        else lds_add(&Bl[bface], q);
        retire();
      }
      live = false;
      continue;
    }
    const int c = ixe + nx * iye;
    if (!fa.has_null) {
      if (owned(iye)) {
        atom_add(&gD[c], q);
        retire();
      }
      live = false;
      continue;
    }
    if (owned(iye)) atom_add(&gW[c], q);
    if (uacc < fa.ratio[c] || j == kMaxSegments - 1) {
      if (owned(iye)) {
        atom_add(&gD[c], q);
        retire();
      }
      live = false;
      continue;
    }
    // null collision: same direction, new free path from the stopping point
    x0 = clamp_to(x0 + ell * sx, static_cast<double>(ixe) * m.dx,
                  static_cast<double>(ixe + 1) * m.dx);
    y0 = clamp_to(y0 + ell * sy, static_cast<double>(iye) * m.dy,
                  static_cast<double>(iye + 1) * m.dy);
    ix = ixe;
    iy = iye;
    ++j;
    draw_path();
    start_segment();
  }
  if (n_fl) {
    atomicAdd(&s_cnt[0], n_fl);
    atomicAdd(&s_cnt[1], n_seg);
    atomicAdd(&s_cnt[2], n_cross);
  }
  __syncthreads();
  // row-contiguous flush
  for (int i = threadIdx.x; i < nface * nx; i += BS)
    if (By[i]) atom_add(&gPhiy[r0 * nx + i], By[i]);
  if (lds_walls)
    for (int b = threadIdx.x; b < m.n_b; b += BS)
      if (Bl[b]) atom_add(&gB[b], Bl[b]);
  if (threadIdx.x == 0 && s_cnt[0]) {
    atomicAdd(&in.sc->flights, s_cnt[0]);
    atomicAdd(&in.sc->segments, s_cnt[1]);
    atomicAdd(&in.sc->crossings, s_cnt[2]);
  }
}

// ---------------------------------------------------------------------------
// The same particle step for flights without null collisions (each record's
// first segment is the whole flight), with the y-face work cut into pieces:
// workgroup (chunk c, stripe s) takes its candidates kStripeScan at a time,
// one per thread: a candidate that meets the stripe tallies its end (deposit
// or wall absorption, and the counters) if that happens in the stripe's rows,
// and is listed with its number of pieces, at most kStripePiece consecutive
// owned y faces each; a workgroup prefix sum numbers the pieces and every lane
// takes one (a binary search finds its particle), so the lanes of a wavefront
// do nearly equal work whatever the spread of path lengths (with one
// particle per lane they waited for the longest: 28% / 52% / 61% VALU lane
// utilisation at Kn 0.1 / 1 / 10 on the 256^2 cavity).  Each crossing is
// tallied in the column reached by the x faces before it, from its own time
// (faces_upto_near), so a piece needs no earlier crossing of its particle.
// Each thread loads its next round's candidate (slot and row range, then the
// record once the range lets it in) and the record of its next piece while
// the current work runs: with one workgroup per CU (the stripe's tallies fill
// the LDS) nothing else hides those loads behind the rounds' barriers.
// Integer sums: the same tallies as the tile kernel, bit for bit.
// ---------------------------------------------------------------------------
constexpr int kStripeScan = 1024;
constexpr int kStripePiece = 16;

template <int BS>
__global__ __launch_bounds__(BS) void march_stripes_pieces_kernel(const Inst *__restrict__ insts,
                                                                  int R, int chunks, StripeRec rec)
{
  static_assert(BS == kStripeScan, "one candidate per thread per round");
  extern __shared__ long long lds_words[];
  __shared__ unsigned long long s_cnt[3];
  __shared__ uint32_t s_pre[kStripeSegMax + 1], s_slot[kStripeSegMax];
  __shared__ uint32_t s_wsum[BS / 64];
  __shared__ uint32_t s_list[kStripeScan], s_ppre[kStripeScan + 1];
  __shared__ uint32_t s_n;
  const Inst &in = insts[0];
  const Mesh m = in.m;
  long long *const gD = in.D, *const gB = in.B, *const gPhiy = in.Phiy;
  const bool lds_walls = in.lds_walls != 0;
  const int nx = m.nx;
  const int r0 = static_cast<int>(blockIdx.y) * R, r1 = min(r0 + R, m.ny);
  const int r1f = (r1 == m.ny) ? m.ny + 1 : r1;
  const int nface = r1f - r0;
  long long *By = lds_words;                                  // [nface][nx]
  long long *Bl = By + nface * nx;                            // [n_b] when lds_walls
  const int nwords = nface * nx + (lds_walls ? m.n_b : 0);
  for (int i = threadIdx.x; i < nwords; i += BS) lds_words[i] = 0;
  if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
  const int K = rec.K, nseg = (rec.S + 1) * K, nown = 2 * K;
  stripe_segment_table<BS>(rec, s_pre, s_slot, s_wsum);
  auto lds_add = [](long long *p, long long v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
  };
  const uint32_t V = s_pre[nseg];
  const uint32_t vb = static_cast<uint32_t>(static_cast<unsigned long long>(V) * blockIdx.x / chunks);
  const uint32_t ve = static_cast<uint32_t>(static_cast<unsigned long long>(V) * (blockIdx.x + 1) / chunks);
  const double inv_dx = 1.0 / m.dx;       // (only to estimate a face count)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const PRec *const recs = static_cast<const PRec *>(rec.r);
  // the owned crossed y faces of a record: first face and count (0: none)
  auto owned_faces = [&](uint32_t cell, double sy, uint32_t nyp, int &f_lo) {
    if (nyp == 0u) return 0;
    const int sty = (sy > 0.0) ? 1 : -1;
    const int iy = static_cast<int>(cell >> 16);
    const int ky0 = (sty > 0) ? iy + 1 : iy;
    const int kl = ky0 + (static_cast<int>(nyp) - 1) * sty;
    f_lo = max(min(ky0, kl), r0);
    return max(0, min(max(ky0, kl), r1f - 1) - f_lo + 1);
  };
  unsigned long long n_fl = 0, n_cross = 0;
  // the thread's candidate of the next round, loaded while the current
  // round's pieces run: its slot, row range (another stripe's leaver) and
  // record (whether or not the range lets it in)
  int sg = 0;
  uint32_t c_slot = 0, c_key = 0;
  bool c_valid = false, c_foreign = false;
  PRec c_rec{};
  auto fetch = [&](unsigned long long vv) {   // the slot and row range
    c_valid = vv < ve;
    if (!c_valid) return;
    const uint32_t v = static_cast<uint32_t>(vv);
    while (sg + 1 < nseg && v >= s_pre[sg + 1]) ++sg;
    c_slot = s_slot[sg] + (v - s_pre[sg]);
    c_foreign = sg >= nown;
    c_key = c_foreign ? rec.key[c_slot] : 0u;
  };
  // (another stripe's leaver enters only if it reaches these rows)
  auto accepted = [&]() {
    return c_valid &&
           !(c_foreign && (static_cast<int>(c_key & 0xffffu) < r0 || static_cast<int>(c_key >> 16) >= r1));
  };
  auto fetch_rec = [&]() {                     // the record, if the candidate enters
    if (accepted()) c_rec = recs[c_slot];
  };
  // a piece's particle: what its crossings need
  struct Piece {
    double x0, y0, sx, sy;
    long long q;
    uint32_t cell, nyp;
  };
  auto piece_of = [&](uint32_t slot) {
    const PRec &rp = recs[slot];
    return Piece{rp.x0, rp.y0, rp.sx, rp.sy, rp.q, rp.cell, rp.nyp};
  };
  auto piece_item = [&](uint32_t u) {       // the last listed i with s_ppre[i] <= u
    int lo = 0, hi = static_cast<int>(s_n) - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_ppre[mid] <= u) lo = mid;
      else hi = mid - 1;
    }
    return lo;
  };
  fetch(static_cast<unsigned long long>(vb) + threadIdx.x);
  fetch_rec();
  for (unsigned long long v0 = vb; v0 < ve; v0 += kStripeScan) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    bool hit = false;
    uint32_t slot = c_slot, npc = 0;
    if (accepted()) {
      const PRec &rp = c_rec;
      const int ixe = static_cast<int>(rp.cell_e & 0xffffu), iye = static_cast<int>(rp.cell_e >> 16);
      if (iye >= r0 && iye < r1) {      // the flight ends in this stripe's rows
        if (rp.bface >= 0) {
          if (!lds_walls) atom_add(&gB[rp.bface], rp.q);
          else lds_add(&Bl[rp.bface], rp.q);
        } else {
          atom_add(&gD[ixe + nx * iye], rp.q);
        }
        ++n_fl;
        n_cross += rp.ncross;
      }
      int f_lo = 0;
      const int c = owned_faces(rp.cell, rp.sy, rp.nyp, f_lo);
      npc = static_cast<uint32_t>((c + kStripePiece - 1) / kStripePiece);
      hit = npc > 0u;
    }
    // listed with their piece counts (one LDS atomic per wavefront)
    const unsigned long long mask = __ballot(hit);
    if (mask) {
      uint32_t off = 0;
      if (lane == 0) off = atomicAdd(&s_n, static_cast<uint32_t>(__popcll(mask)));
      off = __shfl(off, 0, 64);
      if (hit) {
        const uint32_t pos = off + static_cast<uint32_t>(__popcll(mask & ((1ull << lane) - 1ull)));
        s_list[pos] = slot;
        s_ppre[pos] = npc;
      }
    }
    __syncthreads();
    const int nl = static_cast<int>(s_n);
    {
      // exclusive prefix of the piece counts, in place (one entry per thread)
      const int i = static_cast<int>(threadIdx.x);
      const uint32_t c = (i < nl) ? s_ppre[i] : 0u;
      uint32_t incl = c;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), d, 64));
        if (lane >= d) incl += o;
      }
      if (lane == 63) s_wsum[wv] = incl;
      __syncthreads();
      uint32_t off = 0;
      for (int w = 0; w < wv; ++w) off += s_wsum[w];
      if (i < nl) s_ppre[i] = off + incl - c;
      if (i == nl - 1) s_ppre[nl] = off + incl;
      if (nl == 0 && i == 0) s_ppre[0] = 0u;
    }
    __syncthreads();
    fetch(v0 + kStripeScan + threadIdx.x);          // (in flight during the pieces)
    const uint32_t n_piece = s_ppre[nl];
    // the lane's pieces u, u + BS, ...: the next one's record loaded while the
    // current one's crossings run
    uint32_t u = threadIdx.x;
    int ia = 0;
    Piece cur{};
    if (u < n_piece) {
      ia = piece_item(u);
      cur = piece_of(s_list[ia]);
    }
    while (u < n_piece) {
      const uint32_t un = u + BS;
      int ib = 0;
      Piece nxt{};
      if (un < n_piece) {
        ib = piece_item(un);
        nxt = piece_of(s_list[ib]);
      }
      int f_lo = 0;
      const int c = owned_faces(cur.cell, cur.sy, cur.nyp, f_lo);
      const int f0 = f_lo + static_cast<int>(u - s_ppre[ia]) * kStripePiece;
      const int f1 = min(f_lo + c, f0 + kStripePiece);
      const int ix0 = static_cast<int>(cur.cell & 0xffffu);
      const int stx = (cur.sx > 0.0) ? 1 : ((cur.sx < 0.0) ? -1 : 0);
      const double inv_sx = (cur.sx != 0.0) ? 1.0 / cur.sx : 0.0;
      const double inv_sy = 1.0 / cur.sy;                    // (a y face crossed: s_y != 0)
      const long long qy = (cur.sy > 0.0) ? cur.q : -cur.q;
      const int kx0 = (stx > 0) ? ix0 + 1 : ix0;
      const int jwx = (stx > 0) ? nx - kx0 : kx0;
      for (int kyk = f0; kyk < f1; ++kyk) {
        const double ty = (static_cast<double>(kyk) * m.dy - cur.y0) * inv_sy;
        const int cnt = stx ? faces_upto_near(0, kx0, stx, jwx, m.dx, inv_dx, cur.x0, inv_sx, cur.sx, ty) : 0;
        lds_add(&By[(kyk - r0) * nx + ix0 + stx * cnt], qy);
      }
      u = un;
      ia = ib;
      cur = nxt;
    }
    fetch_rec();                                    // (its range has arrived by now)
    __syncthreads();
  }
  if (n_fl) {
    atomicAdd(&s_cnt[0], n_fl);
    atomicAdd(&s_cnt[1], n_fl);        // (one segment per flight)
    atomicAdd(&s_cnt[2], n_cross);
  }
  __syncthreads();
  // row-contiguous flush
  for (int i = threadIdx.x; i < nface * nx; i += BS)
    if (By[i]) atom_add(&gPhiy[r0 * nx + i], By[i]);
  if (lds_walls)
    for (int b = threadIdx.x; b < m.n_b; b += BS)
      if (Bl[b]) atom_add(&gB[b], Bl[b]);
  if (threadIdx.x == 0 && s_cnt[0]) {
    atomicAdd(&in.sc->flights, s_cnt[0]);
    atomicAdd(&in.sc->segments, s_cnt[1]);
    atomicAdd(&in.sc->crossings, s_cnt[2]);
  }
}

// ---------------------------------------------------------------------------
// The expected-value particle step by row stripes (2D single solves).
// Workgroup (chunk c, stripe s) keeps in LDS the deposits D (and W with null
// collisions) of rows [r0, r1), the y-face tallies of faces [r0, r1f) and the
// wall tallies, and follows every ray of its chunk from its start with the
// full arithmetic of fly_expected (optical depth, own exp, rounded surviving
// weight), tallying only the events in its rows: the deposits of a chord in
// an owned row, the owned y faces crossed, a wall face next to an owned row,
// and the crossings made from an owned row; flights are counted by the stripe
// of the start row.  A ray that has left the stripe in its direction of
// travel (or cannot reach it) is dropped.  Integer sums, so the result equals
// the tile kernel's bit for bit, with no global atomic before the final
// row-contiguous flush.
// ---------------------------------------------------------------------------
template <int BS>
__global__ __launch_bounds__(BS) void march_stripes_ev_kernel(const Inst *__restrict__ insts, int R,
                                                              int chunks, int faces)
{
  extern __shared__ long long lds_words[];
  __shared__ unsigned long long s_cnt[3];
  const Inst &in = insts[0];
  const Mesh &m = in.m;
  const int nx = m.nx;
  const int r0 = static_cast<int>(blockIdx.y) * R, r1 = min(r0 + R, m.ny);
  const int r1f = (r1 == m.ny) ? m.ny + 1 : r1;
  const int nrow = r1 - r0, nface = r1f - r0;
  long long *By = lds_words;                                  // [nface][nx]
  long long *Dl = By + nface * nx;                            // [nrow][nx]
  long long *Wl = in.has_null ? Dl + nrow * nx : nullptr;     // [nrow][nx]
  long long *Bl = (in.has_null ? Wl : Dl) + nrow * nx;        // [n_b] when lds_walls
  const int nwords = nface * nx + nrow * nx * (in.has_null ? 2 : 1) + (in.lds_walls ? m.n_b : 0);
  for (int i = threadIdx.x; i < nwords; i += BS) lds_words[i] = 0;
  if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  auto lds_add = [](long long *p, long long v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
  };
  const FlyIn fa = {m, in.lam_min, in.crn ? in.epoch : in.sc->iter, in.key0, in.key1, faces,
                    in.has_null, in.ratio, in.e_off};
  const uint32_t N = in.N;
  const unsigned long long total = static_cast<unsigned long long>(m.n_emit) * N;
  const unsigned long long pb = total * blockIdx.x / chunks;
  const unsigned long long pe = total * (blockIdx.x + 1) / chunks;
  unsigned long long n_fl = 0, n_seg = 0, n_cross = 0;
  int bad = 0;
  auto owned = [&](int row) { return row >= r0 && row < r1; };
  const unsigned long long ne = static_cast<unsigned long long>(m.n_emit);
  const double inv_lam = 1.0 / fa.lam_min;   // = ratio / lambda_min where ratio is 1
  for (unsigned long long pc = pb + threadIdx.x; pc < pe; pc += BS) {
    // emitters fastest: neighbouring lanes start in different cells
    const uint32_t kk = static_cast<uint32_t>(pc / ne);
    const uint32_t e = static_cast<uint32_t>(pc - static_cast<unsigned long long>(kk) * ne);
    const long long q = in.base[e] + ((kk < in.rem[e]) ? 1 : 0);
    if (q == 0) continue;
    int ix, iy;
    double x0, y0, sx, sy;
    sample_particle(fa, e, kk, ix, iy, x0, y0, sx, sy);
    if (owned(iy)) {
      ++n_fl;
      ++n_seg;
    }
    const int stx = (sx > 0.0) ? 1 : ((sx < 0.0) ? -1 : 0);
    const int sty = (sy > 0.0) ? 1 : ((sy < 0.0) ? -1 : 0);
    if ((sty == 0 && !owned(iy)) || (sty > 0 && iy >= r1) || (sty < 0 && iy < r0)) continue;
    const double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
    const double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
    int kx = (stx > 0) ? ix + 1 : ix;
    int ky = (sty > 0) ? iy + 1 : iy;
    const double qd = static_cast<double>(q);
    double T = 0.0, surv = 1.0, tprev = 0.0;
    long long S = q;
    auto cand = [&](int cx, int cy, double v, double ratio) {
      const double x = v / ratio;
      if (!(fabs(x) <= 4611686018427387904.0)) {
        bad = 1;
        return;
      }
      const long long w = static_cast<long long>(rint(x));
      if (w) lds_add(&Wl[(cy - r0) * nx + cx], w);
    };
    for (;;) {
      const bool own = owned(iy);
      const int c = ix + nx * iy;
      const double tx = stx ? (static_cast<double>(kx) * m.dx - x0) * inv_sx : INFINITY;
      const double ty = sty ? (static_cast<double>(ky) * m.dy - y0) * inv_sy : INFINITY;
      const bool along_x = tx <= ty;
      const double tt = along_x ? tx : ty;
      if (!(tt < INFINITY)) {
        if (own) {
          if (S) lds_add(&Dl[(iy - r0) * nx + ix], S);
          if (fa.has_null) cand(ix, iy, qd * surv, fa.ratio[c]);
        }
        break;
      }
      const double ratio = fa.has_null ? fa.ratio[c] : 1.0;
      const double Tn = T + (tt - tprev) * (fa.has_null ? ratio / fa.lam_min : inv_lam);
      const double sn = expm_own(Tn);
      const long long Sn = static_cast<long long>(rint(qd * sn));
      if (own) {
        if (S != Sn) lds_add(&Dl[(iy - r0) * nx + ix], S - Sn);
        if (fa.has_null) cand(ix, iy, qd * (surv - sn), ratio);
      }
      T = Tn;
      surv = sn;
      S = Sn;
      tprev = tt;
      if (S == 0) break;
      if (own) ++n_cross;
      if (along_x) {
        if (kx == 0 || kx == nx) {
          if (own) {
            const int b = (kx == 0) ? iy : m.ny + iy;
            if (in.lds_walls) lds_add(&Bl[b], S);
            else atom_add(&in.B[b], S);
          }
          break;
        }
        ix += stx;
        kx += stx;
      } else {
        if (faces && ky >= r0 && ky < r1f) lds_add(&By[(ky - r0) * nx + ix], sty > 0 ? S : -S);
        if (ky == 0 || ky == m.ny) {
          if (own) {
            const int b = (ky == 0) ? 2 * m.ny + ix : 2 * m.ny + nx + ix;
            if (in.lds_walls) lds_add(&Bl[b], S);
            else atom_add(&in.B[b], S);
          }
          break;
        }
        iy += sty;
        ky += sty;
        if ((sty > 0 && iy >= r1) || (sty < 0 && iy < r0)) break;
      }
    }
  }
  if (bad) atomicOr(&in.sc->flags, 2);
  if (n_fl || n_cross) {
    atomicAdd(&s_cnt[0], n_fl);
    atomicAdd(&s_cnt[1], n_seg);
    atomicAdd(&s_cnt[2], n_cross);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nface * nx; i += BS)
    if (By[i]) atom_add(&in.Phiy[r0 * nx + i], By[i]);
  for (int i = threadIdx.x; i < nrow * nx; i += BS) {
    if (Dl[i]) atom_add(&in.D[r0 * nx + i], Dl[i]);
    if (Wl && Wl[i]) atom_add(&in.W[r0 * nx + i], Wl[i]);
  }
  if (in.lds_walls)
    for (int b = threadIdx.x; b < m.n_b; b += BS)
      if (Bl[b]) atom_add(&in.B[b], Bl[b]);
  if (threadIdx.x == 0 && (s_cnt[0] || s_cnt[2])) {
    atomicAdd(&in.sc->flights, s_cnt[0]);
    atomicAdd(&in.sc->segments, s_cnt[1]);
    atomicAdd(&in.sc->crossings, s_cnt[2]);
  }
}

// ---------------------------------------------------------------------------
// Face fluxes from the tallies (faces on).  Column prefix of the run
// differences completes the y-face tallies; the x-face tallies follow row by
// row from the per-cell balance (net inflow = D - G):
//   Phix[j][0]   = G_left[j] - B_left[j]
//   Phix[j][i+1] = Phix[j][i] + Phiy[j][i] - Phiy[j+1][i] - D[c] + G[c]
// Integer arithmetic modulo 2^64: exact, since every true value fits in int64.
// ---------------------------------------------------------------------------
// One wave's running sums: put(k, carry + get(0) + ... + get(k)) for k < n, in
// wrapping 64-bit integer arithmetic (exact and associative, so the prefix
// sums have the bits of the sequential recurrence).  Four consecutive terms
// per lane, 256 per round; a round's loads all issue before its stores.
template <class Get, class Put>
__device__ __forceinline__ void wave_prefix(int n, unsigned long long carry, Get get, Put put)
{
  const int lane = threadIdx.x & 63;
  for (int k0 = 0; k0 < n; k0 += 256) {
    unsigned long long v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * lane + q;
      s += (k < n) ? get(k) : 0ull;
      v[q] = s;
    }
    unsigned long long t = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const unsigned long long y = __shfl_up(t, d, 64);
      if (lane >= d) t += y;
    }
    const unsigned long long base = carry + (t - s);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + 4 * lane + q;
      if (k < n) put(k, base + v[q]);
    }
    carry += __shfl(t, 63, 64);
  }
}

// y faces from the column differences dB: one wave per column,
// Phiy[k][i] += dB[0][i] + ... + dB[k][i]
__global__ __launch_bounds__(256) void reconstruct_y_kernel(const Inst *__restrict__ insts,
                                                            int faces_mode, int batch)
{
  const Inst &in = insts[blockIdx.y];
  if (inst_idle(in, batch) || !inst_faces(in, faces_mode) || in.m.dim != 2) return;
  const Mesh &m = in.m;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= m.nx) return;
  long long *const Py = in.Phiy;
  const long long *const dB = in.dB;
  wave_prefix(
      m.ny + 1, 0ull,
      [&](int k) { return static_cast<unsigned long long>(dB[k * m.nx + i]); },
      [&](int k, unsigned long long acc) {
        Py[k * m.nx + i] =
            static_cast<long long>(static_cast<unsigned long long>(Py[k * m.nx + i]) + acc);
      });
}

// x faces from the per-cell balance along each row (one wave per row):
// Phix[j][0] = inflow of the left wall face, then
// Phix[j][i+1] = Phix[j][i] + (Phiy[j][i] - Phiy[j+1][i]) + (G - D)[j][i]
__global__ __launch_bounds__(256) void reconstruct_x_kernel(const Inst *__restrict__ insts,
                                                            int faces_mode, int batch)
{
  const Inst &in = insts[blockIdx.y];
  if (inst_idle(in, batch) || !inst_faces(in, faces_mode)) return;
  const Mesh &m = in.m;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= m.ny) return;
  const unsigned long long a0 = static_cast<unsigned long long>(in.G[m.n_cells + j]) -
                                static_cast<unsigned long long>(in.B[j]);
  long long *const px = in.Phix + static_cast<size_t>(j) * (m.nx + 1);
  if ((threadIdx.x & 63) == 0) px[0] = static_cast<long long>(a0);
  const bool two = (m.dim == 2);
  wave_prefix(
      m.nx, a0,
      [&](int i) {
        const int c = j * m.nx + i;
        const unsigned long long dy =
            two ? static_cast<unsigned long long>(in.Phiy[j * m.nx + i]) -
                      static_cast<unsigned long long>(in.Phiy[(j + 1) * m.nx + i])
                : 0ull;
        return dy + (static_cast<unsigned long long>(in.G[c]) -
                     static_cast<unsigned long long>(in.D[c]));
      },
      [&](int i, unsigned long long v) { px[i + 1] = static_cast<long long>(v); });
}

// ---------------------------------------------------------------------------
// macroscopic update (256-wide blocks; block x owns cells [256 x, 256 x + 256))
// Plain path: E^{n+1} = E^{n+1/2} = W / V, next emission = D (Sec. 3.2 step (2)).
// Newton path: E^{n+1/2} and the right-hand side E^{n+1/2} - E^n only.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void update_kernel(const Inst *__restrict__ insts, int batch)
{
  __shared__ double lds[kTree];
  const Inst &in = insts[blockIdx.y];
  if (inst_idle(in, batch)) return;
  const int nbc = (in.m.n_cells + kTree - 1) / kTree;
  if (static_cast<int>(blockIdx.x) >= nbc) return;
  const int c = blockIdx.x * kTree + threadIdx.x;
  double sq = 0.0;
  int bad = 0, over = 0;
  unsigned long long ag = 0;
  if (c < in.m.n_cells) {
    const long long w = in.has_null ? in.W[c] : in.D[c];
    const double eh = ldexp(static_cast<double>(w), -in.F) / in.V;
    in.E_half[c] = eh;
    if (in.newton) {
      in.rhs[c] = eh - in.E[c];
    } else {
      const double d = eh - in.E[c];
      sq = d * d;
      bad = !isfinite(eh);
      in.E[c] = eh;
      // re-emission of the real-collision energy, plus the source
      const long long g = in.Gs ? add_budget(in.D[c], in.Gs[c], &over) : in.D[c];
      in.G[c] = g;
      ag = static_cast<unsigned long long>(g < 0 ? -g : g);
    }
  }
  if (in.newton) return;
  if (bad || over) atomicOr(&in.sc->flags, (bad ? 1 : 0) | (over ? 2 : 0));
  const double s = block_tree256(sq, lds);
  if (threadIdx.x == 0) in.part[blockIdx.x] = s;
  if (in.Gs) {
    // |G| budget partials of the cells (the walls' sum is constant)
    __shared__ unsigned long long lg[kTree];
    lg[threadIdx.x] = ag > kBudgetCap ? kBudgetCap : ag;
    __syncthreads();
    for (int st = kTree / 2; st >= 1; st >>= 1) {
      if (threadIdx.x < st) {
        const unsigned long long u = lg[threadIdx.x] + lg[threadIdx.x + st];
        lg[threadIdx.x] = u > kBudgetCap ? kBudgetCap : u;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) in.gpart[blockIdx.x] = lg[0];
  }
}

// E^{n+1} = E^{n+1/2} + dE, next emission rint(2^F (E^{n+1} V) tau_min / tau_c),
// squared update partials and the saturating |G| budget partials.
__global__ __launch_bounds__(256) void newton_finish_kernel(const Inst *__restrict__ insts,
                                                            int batch)
{
  __shared__ double lds[kTree];
  __shared__ unsigned long long lg[kTree];
  const Inst &in = insts[blockIdx.y];
  if (inst_idle(in, batch) || !in.newton) return;
  const int nbe = (in.m.n_emit + kTree - 1) / kTree;
  if (static_cast<int>(blockIdx.x) >= nbe) return;
  const int c = blockIdx.x * kTree + threadIdx.x;
  double sq = 0.0;
  unsigned long long ag = 0;
  int flags = 0;
  if (c < in.m.n_cells) {
    const double en = in.E_half[c] + in.cg_x[c];
    const double d = en - in.E[c];
    sq = d * d;
    if (!isfinite(en)) flags |= 1;
    in.E[c] = en;
    const double v = ldexp((en * in.V) * in.ratio[c], in.F);
    if (!(fabs(v) <= 4611686018427387904.0)) {
      flags |= 2;
      in.G[c] = 0;
    } else {
      int over = 0;
      long long g = static_cast<long long>(rint(v));
      if (in.Gs) g = add_budget(g, in.Gs[c], &over);
      if (over) flags |= 2;
      in.G[c] = g;
      ag = static_cast<unsigned long long>(g < 0 ? -g : g);
    }
  }
  if (c >= in.m.n_cells && c < in.m.n_emit) {   // wall emitters count toward the budget
    const long long g = in.G[c];
    ag = static_cast<unsigned long long>(g < 0 ? -g : g);
  }
  if (flags) atomicOr(&in.sc->flags, flags);
  const double s = block_tree256(sq, lds);
  lg[threadIdx.x] = ag > kBudgetCap ? kBudgetCap : ag;
  __syncthreads();
  for (int st = kTree / 2; st >= 1; st >>= 1) {
    if (threadIdx.x < st) {
      const unsigned long long u = lg[threadIdx.x] + lg[threadIdx.x + st];
      lg[threadIdx.x] = u > kBudgetCap ? kBudgetCap : u;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    in.part[blockIdx.x] = s;
    in.gpart[blockIdx.x] = lg[0];
  }
}

// Error codes stored in DevScalars::err (same values as the C ABI).
constexpr int kErrDevice = -3, kErrOverflow = -4, kErrNonfinite = -5, kErrBreakdown = -6,
              kErrCgNotConverged = -7, kErrDiverged = -8;

// One workgroup per instance: totals of the partials (fixed order), relative
// residual, counters, status; with `batch` set also the iteration control:
//   state 0: iterate with faces_each until res < res_tol or max_iters,
//   then state 1: avg_iters averaged iterations, or one face-tally iteration
//   in FACES_FINAL mode, or nothing; state 2: done (outputs ready).
__global__ __launch_bounds__(256) void finish_kernel(const Inst *__restrict__ insts, int batch)
{
  __shared__ double lds[kTree];
  __shared__ double lds2[kTree];
  const Inst &in = insts[blockIdx.x];
  if (inst_idle(in, batch)) {
    // finished in an earlier replay: nothing more to accumulate
    if (threadIdx.x == 0) in.sc->acc_mode = 0;
    return;
  }
  DevScalars *sc = in.sc;
  const int nbc = (in.m.n_cells + kTree - 1) / kTree;
  const int nbe = (in.m.n_emit + kTree - 1) / kTree;
  const double dsq = tree_all(in.part, nbc, lds, lds2);
  if (threadIdx.x != 0) return;
  unsigned long long g = 0;
  if (in.newton) {
    for (int i = 0; i < nbe; ++i) {
      g += in.gpart[i];
      if (g > kBudgetCap) g = kBudgetCap;
    }
  } else if (in.persist) {
    for (int i = 0; i < in.n_gpart; ++i) {
      g += in.gpart[i];
      if (g > kBudgetCap) g = kBudgetCap;
    }
  } else if (in.Gs || in.n_bands > 1) {
    g = in.wall_budget;
    for (int i = 0; i < nbc; ++i) {
      g += in.gpart[i];
      if (g > kBudgetCap) g = kBudgetCap;
    }
  }
  sc->gsum = g;
  const double dn = sqrt(dsq);
  sc->dn = dn;
  const int first = (sc->iter == 0);
  if (first) sc->d0 = dn;
  const double d0 = sc->d0;
  const double res = (d0 > 0.0) ? dn / d0 : 0.0;
  sc->res = res;
  // Growth rule of the Newton iteration: the update has grown beyond the
  // first one (res > 1) and either the next emission left the fixed-point
  // range or, with common random numbers (one fixed map, so a rise is the
  // map's and not sampling noise), the residual rose in two consecutive
  // iterations.
  const bool over = (sc->flags & 2) ||
                    ((in.newton || in.Gs || in.n_bands > 1 || in.persist) && g > (1ull << 62));
  sc->grew = (in.newton && res > 1.0 &&
              (over || (in.crn && res > sc->res_p1 && sc->res_p1 > sc->res_p2)))
                 ? 1 : 0;
  sc->res_p2 = sc->res_p1;
  sc->res_p1 = res;
  sc->iter += 1;
  sc->tot_flights += sc->flights;
  sc->tot_segments += sc->segments;
  sc->tot_crossings += sc->crossings;
  if (in.newton) sc->cg_iters_total += sc->cg_iters;
  if (!batch) return;
  // error precedence as in the single-solve driver
  int err = 0;
  if (in.newton && sc->cg_status == -3) err = kErrDevice;
  else if (in.newton && sc->cg_status == -6) err = kErrBreakdown;
  else if (in.newton && sc->cg_status == -7) err = kErrCgNotConverged;
  else if (sc->flags & 1) err = kErrNonfinite;
  else if (sc->grew) err = kErrDiverged;
  else if (over) err = kErrOverflow;
  else if (sc->iter > 1 && res > 1e3) err = kErrDiverged;
  sc->acc_mode = 0;
  if (err) {
    sc->err = err;
    sc->state = 2;
    return;
  }
  if (sc->state == 1) {                  // an output iteration just ended
    sc->acc_mode = (in.avg_iters > 0 && sc->out_left < in.avg_iters) ? 1 : 2;
    if (--sc->out_left == 0) sc->state = 2;
    return;
  }
  const bool conv = res < in.res_tol;
  if (!conv && static_cast<int>(sc->iter) < in.max_iters) return;
  sc->converged = conv ? 1 : 0;
  if (in.avg_iters > 0) {
    sc->state = 1;
    sc->out_left = in.avg_iters;
    sc->faces_now = in.faces_out;
  } else if (in.final_iter) {
    sc->state = 1;
    sc->out_left = 1;
    sc->faces_now = 1;
  } else {
    sc->state = 2;
    sc->acc_mode = 2;
  }
}

__global__ void accumulate_kernel(const Inst *__restrict__ insts, int batch, int force_mode)
{
  const Inst &in = insts[blockIdx.y];
  const int mode = force_mode >= 0 ? force_mode : in.sc->acc_mode;
  if (mode == 0) return;
  const Mesh &m = in.m;
  const int reset = (mode == 2);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m.n_cells) in.acc_E[i] = reset ? in.E[i] : in.acc_E[i] + in.E[i];
  if (i < m.n_fx) {
    const double v = ldexp(static_cast<double>(in.Phix[i]), -in.F);
    in.acc_x[i] = reset ? v : in.acc_x[i] + v;
  }
  if (i < m.n_fy) {
    const double v = ldexp(static_cast<double>(in.Phiy[i]), -in.F);
    in.acc_y[i] = reset ? v : in.acc_y[i] + v;
  }
  (void)batch;
}

// Initial cell emission from E (creation / restored state): G = rint(2^F (E V) r).
__global__ void emission_from_E_kernel(int n_cells, int F, double V, const double *E,
                                       const double *ratio, const long long *Gs, long long *G,
                                       int *flag)
{
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  const double v = ldexp((E[c] * V) * ratio[c], F);
  if (!(fabs(v) <= 4611686018427387904.0)) {
    atomicOr(flag, 2);
    G[c] = 0;
    return;
  }
  long long g = static_cast<long long>(rint(v));
  if (Gs) {
    int over = 0;
    g = add_budget(g, Gs[c], &over);
    if (over) atomicOr(flag, 2);
  }
  G[c] = g;
}

// E0 = cv (T0 - t_ref), ratio = tau_min / tau.
__global__ void init_cells_kernel(int n_cells, double cv, double t_ref, double tau_min,
                                  const double *T0, const double *tau, double *E, double *ratio)
{
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  const double T = T0 ? T0[c] : t_ref;
  E[c] = cv * (T - t_ref);
  ratio[c] = tau_min / tau[c];
}

// ---------------------------------------------------------------------------
// Newton operator (Sec. 3.3): conservative -div(D grad) on the mesh, interior
// face conductance H(D_a, D_b) / d^2 (harmonic mean), wall faces
// D_c / (d (d/2 + 2 lambda_c / 3)) (extrapolation length 2 lambda / 3).
// ---------------------------------------------------------------------------
__global__ void newton_operator_kernel(Mesh m, double vg, const double *tau, const double *Dx,
                                       const double *Dy, double *gx, double *gy, double *diag)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m.n_fx) {
    const int iy = i / (m.nx + 1), kx = i - iy * (m.nx + 1);
    double g;
    if (kx == 0 || kx == m.nx) {
      const int c = iy * m.nx + (kx == 0 ? 0 : m.nx - 1);
      const double lam = vg * tau[c];
      const double den = m.dx * (m.dx / 2.0 + (2.0 * lam) / 3.0);
      g = Dx[c] / den;
    } else {
      const double da = Dx[iy * m.nx + kx - 1], db = Dx[iy * m.nx + kx];
      const double h = ((2.0 * da) * db) / (da + db);
      g = h / (m.dx * m.dx);
    }
    gx[i] = g;
  }
  if (m.dim == 2 && i < m.n_fy) {
    const int ky = i / m.nx, ix = i - ky * m.nx;
    double g;
    if (ky == 0 || ky == m.ny) {
      const int c = (ky == 0 ? 0 : m.ny - 1) * m.nx + ix;
      const double lam = vg * tau[c];
      const double den = m.dy * (m.dy / 2.0 + (2.0 * lam) / 3.0);
      g = Dy[c] / den;
    } else {
      const double da = Dy[(ky - 1) * m.nx + ix], db = Dy[ky * m.nx + ix];
      const double h = ((2.0 * da) * db) / (da + db);
      g = h / (m.dy * m.dy);
    }
    gy[i] = g;
  }
}

__global__ void newton_diag_kernel(Mesh m, const double *gx, const double *gy, double *diag)
{
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m.n_cells) return;
  const int iy = c / m.nx, ix = c - iy * m.nx;
  double d = gx[iy * (m.nx + 1) + ix] + gx[iy * (m.nx + 1) + ix + 1];
  if (m.dim == 2) {
    d = d + gy[iy * m.nx + ix];
    d = d + gy[(iy + 1) * m.nx + ix];
  }
  diag[c] = d;
}

// ---------------------------------------------------------------------------
// Data shared between the workgroups of a persistent group (published rows,
// block sums) is only ever accessed with agent-scope atomic loads and stores
// (xst / xld), which are coherent across the XCDs' L2 caches on their own.
// The group barrier therefore needs no L2 writeback or invalidate: every wave
// waits until its own stores have completed, the workgroup synchronises, and
// one thread bumps a monotone arrival counter (agent-scope RMW); barrier
// number k completes when the counter reaches k * group.  Readers poll the
// counter and only then issue their (coherent) loads.  Ordinary accesses
// stay private to one workgroup or cross kernel boundaries only.
// counter[0] = arrivals, counter[1] = abort flag.  A wait longer than ~1 s sets
// the abort flag; every workgroup then leaves its next barrier at once and the
// kernel reports the failure, so a broken barrier can never hang the device.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void xst(double *p, double v)
{
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double xld(const double *p)
{
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr long kBarrierSpinLimit = 1l << 24;

__device__ __forceinline__ bool grid_barrier(unsigned int *counter, unsigned int &epoch,
                                             unsigned int group)
{
  __shared__ int s_abort;
  __builtin_amdgcn_s_waitcnt(0);          // this wave's coherent stores have completed
  __syncthreads();
  epoch += 1;
  if (threadIdx.x == 0) {
    const unsigned int target = epoch * group;
    const unsigned int old =
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    int abort = 0;
    if (old + 1u < target) {
      while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kBarrierSpinLimit) {
          __hip_atomic_store(counter + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          abort = 1;
          break;
        }
        if ((spins & 1023) == 0 &&
            __hip_atomic_load(counter + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          abort = 1;
          break;
        }
      }
    }
    s_abort = abort;
  }
  __syncthreads();
  return s_abort == 0;
}

// ---------------------------------------------------------------------------
// Conjugate gradients, single-reduction form (Chronopoulos & Gear 1989):
//   x = 0, r = b, w = A r, gamma = (r, r), delta = (w, r), alpha = gamma / delta
//   repeat: p = r + beta p, s = w + beta s (p = r, s = w the first time)
//           x += alpha p, r -= alpha s, w = A r
//           gamma' = (r, r), delta = (w, r); stop if gamma' <= tol^2 (b, b)
//           beta = gamma' / gamma, alpha = gamma' / (delta - beta gamma' / alpha)
// One persistent group of G workgroups, one group barrier per iteration (none
// when G = 1).  Rank g owns the contiguous tree blocks [g TB, (g+1) TB), cells
// [c0, c1).  Register form (TB <= waves per workgroup): wave w owns block
// g TB + w and lane l keeps x, r, w, p, s and the operator row of cells
// l, l + 64, l + 128, l + 192 of it, so the block's pairwise tree
// ((v_l + v_{l+128}) + (v_{l+64} + v_{l+192}), then halving strides across the
// lanes) runs inside the wave.  Global form: the waves take the blocks round
// robin and the state lives in global arrays.  Block sums are published as
// (g, d) pairs; after the barrier every wave reduces all of them itself, in
// the same fixed order, so no workgroup-wide step is needed for the scalars.
// The operator needs r one mesh row (one cell in 1D) beyond the own range:
// before each barrier every workgroup publishes (r, w, s) of the cells its
// neighbours read (double-buffered by iteration parity); after it, each
// workgroup recomputes the neighbours' new r on that halo with the owner's
// exact operations, s = w + beta s_old, r = r - alpha s, so the halo values
// are bit-identical to the owner's.
// ---------------------------------------------------------------------------
constexpr int kCgWavesMax = 12;        // 768 threads: about 170 VGPRs per lane for the register form
constexpr int kCgThreadsMax = 64 * kCgWavesMax;

struct CGArgs {
  Mesh m;
  const double *gx, *gy, *diag, *b;
  double *x;                 // solution
  double *gr, *gw, *gp, *gs; // own-state arrays (global form only)
  double *pub;               // [2][3][n] published (r, w, s)
  double *part;              // [2][nb][2] block sums of (r, r) and (w, r)
  int TB;                    // tree blocks per workgroup
  double tol2;
  int max_iters;
  unsigned int *barrier;     // [2], zero at the start of the solve
  DevScalars *sc;
};

struct CellCoef {
  double d, l, r, dn, up;    // diagonal and the four face conductances (0 if absent)
};

__device__ __forceinline__ CellCoef load_coef(const Mesh &m, const double *gx, const double *gy,
                                              const double *diag, int c)
{
  const int iy = c / m.nx, ix = c - iy * m.nx;
  CellCoef k;
  k.d = diag[c];
  k.l = (ix > 0) ? gx[iy * (m.nx + 1) + ix] : 0.0;
  k.r = (ix < m.nx - 1) ? gx[iy * (m.nx + 1) + ix + 1] : 0.0;
  k.dn = (m.dim == 2 && iy > 0) ? gy[iy * m.nx + ix] : 0.0;
  k.up = (m.dim == 2 && iy < m.ny - 1) ? gy[(iy + 1) * m.nx + ix] : 0.0;
  return k;
}

// (A v)_c with the reference operation order: diag v_c - g_l v_{c-1} - g_r v_{c+1}
// - g_dn v_{c-nx} - g_up v_{c+nx}, absent neighbours skipped.
template <class Get>
__device__ __forceinline__ double apply_cell(const Mesh &m, const CellCoef &k, int c, Get v)
{
  const int iy = c / m.nx, ix = c - iy * m.nx;
  double acc = k.d * v(c);
  if (ix > 0) acc = acc - k.l * v(c - 1);
  if (ix < m.nx - 1) acc = acc - k.r * v(c + 1);
  if (m.dim == 2) {
    if (iy > 0) acc = acc - k.dn * v(c - m.nx);
    if (iy < m.ny - 1) acc = acc - k.up * v(c + m.nx);
  }
  return acc;
}

// The same with the neighbour tests precomputed: bits 0..3 of nbm = left,
// right, down, up neighbour present.
template <class Get>
__device__ __forceinline__ double apply_masked(const CellCoef &k, int c, int nx, unsigned nbm, Get v)
{
  double acc = k.d * v(c);
  if (nbm & 1u) acc = acc - k.l * v(c - 1);
  if (nbm & 2u) acc = acc - k.r * v(c + 1);
  if (nbm & 4u) acc = acc - k.dn * v(c - nx);
  if (nbm & 8u) acc = acc - k.up * v(c + nx);
  return acc;
}

__device__ __forceinline__ unsigned neighbour_mask(const Mesh &m, int c)
{
  const int iy = c / m.nx, ix = c - iy * m.nx;
  unsigned b = 0u;
  if (ix > 0) b |= 1u;
  if (ix < m.nx - 1) b |= 2u;
  if (m.dim == 2 && iy > 0) b |= 4u;
  if (m.dim == 2 && iy < m.ny - 1) b |= 8u;
  return b;
}

// Lane l gets the value of lane l + s (s = 8, 4, 2, 1: DPP row shift within
// the 16-lane row; 16 and 32: the gfx950 permlane swaps).  Only the lanes the
// tree below reads are meaningful.
template <int S>
__device__ __forceinline__ double from_lane_plus(double v)
{
  const unsigned lo = static_cast<unsigned>(__double2loint(v));
  const unsigned hi = static_cast<unsigned>(__double2hiint(v));
  unsigned l2, h2;
  if constexpr (S == 32) {
    l2 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false)[1];
    h2 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false)[1];
  } else if constexpr (S == 16) {
    l2 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false)[1];
    h2 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false)[1];
  } else {
    static_assert(S == 8 || S == 4 || S == 2 || S == 1, "row shift");
    l2 = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(lo), 0x100 + S, 0xf, 0xf, false));
    h2 = static_cast<unsigned>(__builtin_amdgcn_update_dpp(0, static_cast<int>(hi), 0x100 + S, 0xf, 0xf, false));
  }
  return __hiloint2double(static_cast<int>(h2), static_cast<int>(l2));
}

// Pairwise tree of one 256-element block whose element l + 64 q sits in lane l
// as v_q: (v_l + v_{l+128}) + (v_{l+64} + v_{l+192}), then r_l + r_{l+s} for
// s = 32, 16, ..., 1.  The sum is valid in lane 0.
__device__ __forceinline__ double wave_tree256(double v0, double v1, double v2, double v3)
{
  double r = (v0 + v2) + (v1 + v3);
  r = r + from_lane_plus<32>(r);
  r = r + from_lane_plus<16>(r);
  r = r + from_lane_plus<8>(r);
  r = r + from_lane_plus<4>(r);
  r = r + from_lane_plus<2>(r);
  r = r + from_lane_plus<1>(r);
  return r;
}

// lane 0's value in every lane
__device__ __forceinline__ double lane0(double v)
{
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 0);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 0);
  return __hiloint2double(hi, lo);
}

// Sums of the nb published (g, d) pairs in the fixed order of the host-side
// definition: the 256-element tree over each chunk of pairs, then the same
// tree over the chunk sums (nb <= 65536).  Every thread of the workgroup gets
// both results.  One chunk: each wave reduces it itself.  More: wave w
// reduces chunks w, w + nw, ... into LDS (red, 2 * 256 doubles), then every
// wave reduces the chunk sums.
__device__ __forceinline__ void group_tree_pairs(const double *part, int nb, double *red,
                                                 double &sg, double &sd)
{
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nch = (nb + kTree - 1) / kTree;
  auto chunk = [&](int k, double &rg, double &rd) {
    double g[4], d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = k * kTree + lane + 64 * q;
      const bool in = i < nb;
      g[q] = in ? xld(&part[2 * i]) : 0.0;
      d[q] = in ? xld(&part[2 * i + 1]) : 0.0;
    }
    rg = wave_tree256(g[0], g[1], g[2], g[3]);
    rd = wave_tree256(d[0], d[1], d[2], d[3]);
  };
  if (nch == 1) {
    double rg, rd;
    chunk(0, rg, rd);
    sg = lane0(rg);
    sd = lane0(rd);
    return;
  }
  for (int k = wave; k < nch; k += nw) {
    double rg, rd;
    chunk(k, rg, rd);
    if (lane == 0) {
      red[k] = rg;
      red[kTree + k] = rd;
    }
  }
  __syncthreads();
  double g[4], d[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = lane + 64 * q;
    g[q] = k < nch ? red[k] : 0.0;
    d[q] = k < nch ? red[kTree + k] : 0.0;
  }
  sg = lane0(wave_tree256(g[0], g[1], g[2], g[3]));
  sd = lane0(wave_tree256(d[0], d[1], d[2], d[3]));
  __syncthreads();
}

// The solve as seen by one workgroup of rank `rank` in a group of G resident
// workgroups sharing the barrier counter a.barrier.  REG selects the register
// form (requires a.TB <= blockDim.x / 64).
template <bool REG>
__device__ void cg_run(const CGArgs &a, int rank, int G)
{
  extern __shared__ double stage[];       // r on [h0, h1) (register form) or on the halo
  __shared__ double red[2 * kTree];        // chunk sums when nb > 256
  unsigned int epoch = 0;
  const Mesh &m = a.m;
  const int n = m.n_cells;
  const int nb = (n + kTree - 1) / kTree;
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tb0 = rank * a.TB;
  const int tb1 = min(tb0 + a.TB, nb);
  const int c0 = min(tb0 * kTree, n), c1 = min(tb1 * kTree, n);
  const int hw = (m.dim == 2) ? m.nx : 1;
  const int h0 = max(0, c0 - hw), h1 = min(n, c1 + hw);
  const int nlo = c0 - h0;                          // halo cells below the own range
  const int nhalo = (h1 - h0) - (c1 - c0);
  const bool nb_lo = c0 > 0, nb_hi = c1 < n;       // a neighbour below / above exists
  double *const pub[2] = {a.pub, a.pub + 3 * static_cast<size_t>(n)};
  double *const part[2] = {a.part, a.part + 2 * static_cast<size_t>(nb)};
  const int tbr = tb0 + wave;                       // the register form's block
  const bool own = REG && wave < a.TB && tbr < tb1;

  auto halo_cell = [&](int i) { return i < nlo ? h0 + i : c1 + (i - nlo); };
  auto published = [&](int c) { return (nb_lo && c < c0 + hw) || (nb_hi && c >= c1 - hw); };
  auto rget = [&](int c) -> double {
    if constexpr (REG) {
      return stage[c - h0];
    } else {
      if (c < c0) return stage[c - h0];
      if (c >= c1) return stage[nlo + (c - c1)];
      return a.gr[c];
    }
  };

  double xr[4], rr[4], wr[4], pr[4], sr[4];
  CellCoef kr[4];
  // the first kHaloRegs halo slots of this thread: published (r, w, s), loaded
  // right after the barrier together with the block sums
  constexpr int kHaloRegs = 1;
  double hr[kHaloRegs], hwv[kHaloRegs], hs[kHaloRegs];
  auto preload_halo = [&](const double *pp) {
#pragma unroll
    for (int k = 0; k < kHaloRegs; ++k) {
      const int i = threadIdx.x + k * blockDim.x;
      hr[k] = 0.0;
      hwv[k] = 0.0;
      hs[k] = 0.0;
      if (i < nhalo) {
        const int c = halo_cell(i);
        hr[k] = xld(&pp[c]);
        hwv[k] = xld(&pp[n + c]);
        hs[k] = xld(&pp[2 * static_cast<size_t>(n) + c]);
      }
    }
  };
  unsigned cm = 0u;        // register form: per cell q, bits 5q..5q+3 neighbours, 5q+4 published

  // w = A r on the own cells, block sums of (r, r) and (w, r) into pt, (r, w, s)
  // of the published cells into pn
  auto apply_pass = [&](double *pn, double *pt, bool start) {
    if constexpr (REG) {
      if (!own) return;
      double g[4], d[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tbr * kTree + lane + 64 * q;
        g[q] = 0.0;
        d[q] = 0.0;
        if (c < n) {
          const unsigned bits = cm >> (5 * q);
          const double wv = apply_masked(kr[q], c, m.nx, bits, rget);
          wr[q] = wv;
          g[q] = rr[q] * rr[q];
          d[q] = wv * rr[q];
          if (bits & 16u) {
            xst(&pn[c], rr[q]);
            xst(&pn[n + c], wv);
            xst(&pn[2 * static_cast<size_t>(n) + c], sr[q]);
          }
        }
      }
      const double sg = wave_tree256(g[0], g[1], g[2], g[3]);
      const double sd = wave_tree256(d[0], d[1], d[2], d[3]);
      if (lane == 0) {
        xst(&pt[2 * tbr], sg);
        xst(&pt[2 * tbr + 1], sd);
      }
    } else {
      for (int tb = tb0 + wave; tb < tb1; tb += nw) {
        double g[4], d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = tb * kTree + lane + 64 * q;
          g[q] = 0.0;
          d[q] = 0.0;
          if (c < n) {
            const CellCoef k = load_coef(m, a.gx, a.gy, a.diag, c);
            const double wv = apply_cell(m, k, c, rget);
            a.gw[c] = wv;
            const double rv = a.gr[c];
            g[q] = rv * rv;
            d[q] = wv * rv;
            if (published(c)) {
              xst(&pn[c], rv);
              xst(&pn[n + c], wv);
              xst(&pn[2 * static_cast<size_t>(n) + c], start ? 0.0 : a.gs[c]);
            }
          }
        }
        const double sg = wave_tree256(g[0], g[1], g[2], g[3]);
        const double sd = wave_tree256(d[0], d[1], d[2], d[3]);
        if (lane == 0) {
          xst(&pt[2 * tb], sg);
          xst(&pt[2 * tb + 1], sd);
        }
      }
    }
  };
  auto group_barrier = [&]() -> bool {
    if (G == 1) {
      __builtin_amdgcn_s_waitcnt(0);      // coherent stores complete before other waves read
      __syncthreads();
      return true;
    }
    return grid_barrier(a.barrier, epoch, G);
  };

  // ---- start: x = 0, r = b, w = A r
  if constexpr (REG) {
    for (int i = threadIdx.x; i < h1 - h0; i += blockDim.x) stage[i] = a.b[h0 + i];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = tbr * kTree + lane + 64 * q;
      xr[q] = 0.0;
      pr[q] = 0.0;
      sr[q] = 0.0;
      wr[q] = 0.0;
      rr[q] = 0.0;
      kr[q] = CellCoef{0.0, 0.0, 0.0, 0.0, 0.0};
      if (own && c < n) {
        kr[q] = load_coef(m, a.gx, a.gy, a.diag, c);
        rr[q] = a.b[c];
        cm |= (neighbour_mask(m, c) | (published(c) ? 16u : 0u)) << (5 * q);
      }
    }
  } else {
    for (int i = threadIdx.x; i < nhalo; i += blockDim.x) stage[i] = a.b[halo_cell(i)];
    for (int c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
      a.x[c] = 0.0;
      a.gr[c] = a.b[c];
    }
  }
  __syncthreads();
  apply_pass(pub[0], part[0], true);
  int status = -7;
  if (!group_barrier()) status = -3;
  preload_halo(pub[0]);
  double gamma = 0.0, delta = 0.0;
  group_tree_pairs(part[0], nb, red, gamma, delta);
  const double thr = a.tol2 * gamma;
  int it = 0, par = 0;
  double alpha = 0.0, beta = 0.0;
  if (status == -3) {
  } else if (gamma == 0.0) {
    status = 0;
  } else if (!(delta > 0.0)) {
    status = -6;
  } else {
    alpha = gamma / delta;
  }
  while (status == -7 && it < a.max_iters) {
    const bool first = (it == 0);
    const double *pp = pub[par];
    // own cells: direction, x and r updates (register form: stage the new r)
    if constexpr (REG) {
      if (own) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int c = tbr * kTree + lane + 64 * q;
          if (c < n) {
            pr[q] = first ? rr[q] : rr[q] + beta * pr[q];
            sr[q] = first ? wr[q] : wr[q] + beta * sr[q];
            xr[q] = xr[q] + alpha * pr[q];
            rr[q] = rr[q] - alpha * sr[q];
            stage[c - h0] = rr[q];
          }
        }
      }
    } else {
      for (int c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
        const double pv = first ? a.gr[c] : a.gr[c] + beta * a.gp[c];
        const double sv = first ? a.gw[c] : a.gw[c] + beta * a.gs[c];
        a.gp[c] = pv;
        a.gs[c] = sv;
        a.x[c] = a.x[c] + alpha * pv;
        a.gr[c] = a.gr[c] - alpha * sv;
      }
    }
    // halo: the neighbours' new r from their published (r, w, s)
#pragma unroll
    for (int k = 0; k < kHaloRegs; ++k) {
      const int i = threadIdx.x + k * blockDim.x;
      if (i < nhalo) {
        const int c = halo_cell(i);
        const double sv = first ? hwv[k] : hwv[k] + beta * hs[k];
        const double rv = hr[k] - alpha * sv;
        if constexpr (REG) stage[c - h0] = rv;
        else stage[i] = rv;
      }
    }
    for (int i = threadIdx.x + kHaloRegs * blockDim.x; i < nhalo; i += blockDim.x) {
      const int c = halo_cell(i);
      const double sw = xld(&pp[n + c]);
      const double sv = first ? sw : sw + beta * xld(&pp[2 * static_cast<size_t>(n) + c]);
      const double rv = xld(&pp[c]) - alpha * sv;
      if constexpr (REG) stage[c - h0] = rv;
      else stage[i] = rv;
    }
    __syncthreads();
    apply_pass(pub[par ^ 1], part[par ^ 1], false);
    if (!group_barrier()) {
      status = -3;
      break;
    }
    par ^= 1;
    ++it;
    preload_halo(pub[par]);
    double gamma_new = 0.0;
    group_tree_pairs(part[par], nb, red, gamma_new, delta);
    if (gamma_new <= thr) {
      status = 0;
      break;
    }
    beta = gamma_new / gamma;
    double tq = beta * gamma_new;
    tq = tq / alpha;
    const double den = delta - tq;
    if (!(den > 0.0)) {
      status = -6;
      break;
    }
    alpha = gamma_new / den;
    gamma = gamma_new;
  }
  if constexpr (REG) {
    if (own) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tbr * kTree + lane + 64 * q;
        if (c < n) a.x[c] = xr[q];
      }
    }
  }
  if (rank == 0 && threadIdx.x == 0) {
    a.sc->cg_iters = it;
    a.sc->cg_status = status;
  }
}

template <bool REG>
__global__ __launch_bounds__(kCgThreadsMax) void cg_kernel(CGArgs a)
{
  cg_run<REG>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Adjoint of the steady state (uniform relaxation time, common random numbers).
// For fixed counters the paths do not depend on the weights, so one
// iteration is linear in the emission energies, D = T_cc G_cells + T_cw G_walls
// with T_xe the fraction of emitter e's N particles ending in cell x, and the
// steady state with re-emission G_cells = D + G_src is
// D* = (I - T_cc)^-1 (T_cc G_src + T_cw G_walls).  For a loss L(T), with
// u = dL/dD* and psi = (I - T_cc^T)^-1 u,
//   dL/dG_src = T_cc^T psi,   dL/dG_walls = T_cw^T psi,
// and (T^T psi)_e is the mean of psi over the cells where e's particles end:
// the forward paths used in reverse.  psi is the fixed point of
// psi <- T^T psi + u, each pass followed by the forward solve's diffusion
// correction when Newton is on.
// ---------------------------------------------------------------------------
// where particle (e, k) ends: end[e N + k] = its deposit cell, or -1 when a
// wall absorbs it (one thread per particle)
__global__ void adjoint_paths_kernel(FlyIn fa, int n_emit, uint32_t N, int *end)
{
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<long long>(n_emit) * N) return;
  const uint32_t e = static_cast<uint32_t>(i / N);
  const uint32_t k = static_cast<uint32_t>(i - static_cast<long long>(e) * N);
  int out = -1;
  unsigned long long n_seg = 0, n_cross = 0;
  auto none = [](int, int, long long) {};
  fly(fa, e, k, 1ll, none, none, [&](int, long long) { out = -1; }, none,
      [&](int cx, int cy, long long) { out = cx + fa.m.nx * cy; }, n_seg, n_cross);
  end[i] = out;
}

// g_e = (sum over k of psi at end(e, k), 0 for walls) / N; the sum in the
// fixed order of the host definition (256-element pairwise trees, then the
// same tree over the chunk sums; N <= 65536).  One wave per emitter.
__global__ void adjoint_gather_kernel(const int *__restrict__ end, const double *__restrict__ psi,
                                      int n_emit, uint32_t N, double *__restrict__ g)
{
  const int e = static_cast<int>((static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= n_emit) return;                    // whole waves only
  const int *en = end + static_cast<size_t>(e) * N;
  auto val = [&](uint32_t k) -> double {
    if (k >= N) return 0.0;
    const int a = en[k];
    return a >= 0 ? psi[a] : 0.0;
  };
  const uint32_t nch = (N + kTree - 1) / kTree;
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  double total = 0.0;
  for (uint32_t ch = 0; ch < nch; ++ch) {
    const uint32_t b = ch * kTree + lane;
    const double r = lane0(wave_tree256(val(b), val(b + 64), val(b + 128), val(b + 192)));
    if (nch == 1) {
      total = r;
      break;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (static_cast<int>(ch >> 6) == q && static_cast<int>(ch & 63) == lane) c[q] = r;
  }
  if (nch > 1) total = lane0(wave_tree256(c[0], c[1], c[2], c[3]));
  if (lane == 0) g[e] = total / static_cast<double>(N);
}

// u = dL/dD* = ldexp((dL/dT / C) / V, -F) (T = t_ref + ldexp(D, -F) / V / C); psi = u
__global__ void adjoint_init_kernel(int n, double cv, double V, int F, const double *dLdT,
                                    double *u, double *psi)
{
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const double v = ldexp((dLdT[c] / cv) / V, -F);
  u[c] = v;
  psi[c] = v;
}

// half = T^T psi + u.  Without Newton psi <- half directly (squared change
// partials per 256-cell block); with Newton rhs = half - psi for the CG.
__global__ __launch_bounds__(256) void adjoint_half_kernel(int n, const double *g, const double *u,
                                                           double *half, double *psi, double *rhs,
                                                           int newton, double *part)
{
  __shared__ double lds[kTree];
  const int c = blockIdx.x * kTree + threadIdx.x;
  double sq = 0.0;
  if (c < n) {
    const double h = g[c] + u[c];
    if (newton) {
      half[c] = h;
      rhs[c] = h - psi[c];
    } else {
      const double d = h - psi[c];
      sq = d * d;
      psi[c] = h;
    }
  }
  if (newton) return;
  const double s = block_tree256(sq, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// with Newton: psi <- half + x (the CG correction), squared change partials
__global__ __launch_bounds__(256) void adjoint_newton_kernel(int n, const double *half,
                                                             const double *x, double *psi,
                                                             double *part)
{
  __shared__ double lds[kTree];
  const int c = blockIdx.x * kTree + threadIdx.x;
  double sq = 0.0;
  if (c < n) {
    const double nv = half[c] + x[c];
    const double d = nv - psi[c];
    sq = d * d;
    psi[c] = nv;
  }
  const double s = block_tree256(sq, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// one workgroup: out = sqrt(fixed-order sum of the partials)
__global__ __launch_bounds__(256) void adjoint_norm_kernel(const double *part, int nb, double *out)
{
  __shared__ double lds[kTree];
  __shared__ double lds2[kTree];
  const double s = tree_all(part, nb, lds, lds2);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

// chain rule to the inputs: dL/dS_c = g_c ldexp(V tau_min, F), dL/dT_f = g_f
// ldexp(C lambda_min A_f / 4, F) (A_f = dy on the left/right walls, dx else)
__global__ void adjoint_grad_kernel(int n_cells, int n_b, int ny, const double *g, double fs,
                                    double fw_lr, double fw_bt, double *grad_source,
                                    double *grad_wall)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_cells && grad_source) grad_source[i] = g[i] * fs;
  if (i < n_b && grad_wall) grad_wall[i] = g[n_cells + i] * ((i < 2 * ny) ? fw_lr : fw_bt);
}

// ---------------------------------------------------------------------------
// Frequency bands: the coupling step.  Per cell, the absorbed rate
// R = sum_k ldexp(D_k, -F) / tau*_k (+ S V, passed as one product per cell) is
// re-emitted over the bands with the equilibrium spectrum,
// G_k = rint(ldexp(share_k R, F)), share_k = tau*_k ((C_k / tau_k) / den),
// den = sum_k C_k / tau_k (share precomputed per band and cell); the energy
// density is E = sum_k ldexp(W_k, -F) / V (W_k = D_k for a band without null
// collisions).  Bands summed in index order.  Squared-change and |G| budget
// partials per 256-cell block.
// ---------------------------------------------------------------------------
struct BandDev {
  double ts;                    // tau*_k
  const double *share;          // [nc] tau*_k (C_k / tau_k) / sum_j (C_j / tau_j)
  const long long *D, *W;       // [nc]
  long long *G;                 // [nc + nb] (cells first)
  int has_null;
};

__global__ __launch_bounds__(256) void bands_update_kernel(const Inst *__restrict__ main_in,
                                                           const BandDev *__restrict__ bands,
                                                           int K, const double *__restrict__ srcV)
{
  __shared__ double lds[kTree];
  __shared__ unsigned long long lg[kTree];
  const Inst &in = *main_in;
  const int n = in.m.n_cells;
  const int c = blockIdx.x * kTree + threadIdx.x;
  double sq = 0.0;
  unsigned long long ag = 0;
  int flags = 0;
  if (c < n) {
    double R = 0.0, Wsum = 0.0;
    for (int k = 0; k < K; ++k) {
      const BandDev &b = bands[k];
      const long long d = b.D[c];
      R = R + ldexp(static_cast<double>(d), -in.F) / b.ts;
      Wsum = Wsum + ldexp(static_cast<double>(b.has_null ? b.W[c] : d), -in.F);
    }
    if (srcV) R = R + srcV[c];
    const double En = Wsum / in.V;
    const double dd = En - in.E[c];
    sq = dd * dd;
    if (!isfinite(En)) flags |= 1;
    in.E[c] = En;
    for (int k = 0; k < K; ++k) {
      const BandDev &b = bands[k];
      const double v = ldexp(b.share[c] * R, in.F);
      long long g = 0;
      if (!(fabs(v) <= 4611686018427387904.0)) flags |= 2;
      else g = static_cast<long long>(rint(v));
      b.G[c] = g;
      const unsigned long long a = static_cast<unsigned long long>(g < 0 ? -g : g);
      ag = (ag + a > kBudgetCap) ? kBudgetCap : ag + a;
    }
  }
  if (flags) atomicOr(&in.sc->flags, flags);
  const double s = block_tree256(sq, lds);
  lg[threadIdx.x] = ag;
  __syncthreads();
  for (int st = kTree / 2; st >= 1; st >>= 1) {
    if (threadIdx.x < st) {
      const unsigned long long u = lg[threadIdx.x] + lg[threadIdx.x + st];
      lg[threadIdx.x] = u > kBudgetCap ? kBudgetCap : u;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    in.part[blockIdx.x] = s;
    in.gpart[blockIdx.x] = lg[0];
  }
}

// Frequency bands: the outputs.  T = t_ref + E / sum_k C_k; the face fluxes
// q = (sum_k ldexp(Phi_k, -F) / tau*_k) / A over the bands in index order.
__global__ void bands_output_kernel(int n_cells, int n_fx, int n_fy, int F, double t_ref,
                                    double Ctot, double ax, double ay, int faces,
                                    const double *E, const BandDev *bands, const long long *const *phix,
                                    const long long *const *phiy, int K, double *T, double *qx,
                                    double *qy)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_cells) T[i] = t_ref + E[i] / Ctot;
  if (qx && i < n_fx) {
    double v = 0.0;
    for (int k = 0; k < K; ++k) v = v + ldexp(static_cast<double>(phix[k][i]), -F) / bands[k].ts;
    qx[i] = faces ? v / ax : 0.0;
  }
  if (qy && i < n_fy) {
    double v = 0.0;
    for (int k = 0; k < K; ++k) v = v + ldexp(static_cast<double>(phiy[k][i]), -F) / bands[k].ts;
    qy[i] = faces ? v / ay : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Persistent particles: the variable-tau iteration of Sec. 3.2, steps (1)-(6),
// with a fixed population.  Every iteration each particle flies one
// candidate path on the common time scale: real-collision particles are first
// resampled from their cell's equilibrium (uniform point, isotropic
// direction, the cell's share w_c), particles absorbed by a wall face are
// re-emitted from it (uniform point of the face, cosine law, the face's share
// w_b), null particles move on unchanged.  Counter of particle p's draw d:
// (d, p, kPersistStream, slot); creation uses slot kPersistCreate.
// ---------------------------------------------------------------------------
constexpr uint32_t kPersistStream = 0xFFFFFFFFu;
constexpr uint32_t kPersistCreate = 0xFFFFFFFFu;
constexpr uint32_t kLocMask = 0x3FFFFFFFu;

__device__ __forceinline__ void iso_direction(int dim, double2 ucd, double &sx, double &sy)
{
  const double mu = 2.0 * ucd.x - 1.0;
  sx = mu;
  sy = (dim == 2) ? sqrt((1.0 - mu) * (1.0 + mu)) * cos2pi_own(ucd.y) : 0.0;
}

// a = w n + r, 0 <= r < n (n > 0)
__device__ __forceinline__ void share_of(long long a, uint32_t n, long long &w, long long &r)
{
  const long long nn = static_cast<long long>(n);
  long long b = a / nn;
  if (a % nn != 0 && a < 0) b -= 1;
  w = b;
  r = a - b * nn;
}

__device__ __forceinline__ unsigned long long abs_u64(long long v)
{
  return v < 0 ? 0ull - static_cast<unsigned long long>(v) : static_cast<unsigned long long>(v);
}

// Runs of equal consecutive keys in a 64-lane wavefront: head = first lane of
// its run, run = run number (heads at or below the lane).  All lanes call.
__device__ __forceinline__ void wave_runs(int key, int &head, int &run)
{
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  head = (lane == 0 || prev != key) ? 1 : 0;
  const unsigned long long heads = __ballot(head);
  run = __popcll(heads & ((2ull << lane) - 1ull));
}

// Sum of v over the lanes of the same run from this lane on (the head gets the
// run's total); integer, so exact.  All lanes call.
__device__ __forceinline__ long long run_sum(long long v, int run)
{
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int st = 1; st < 64; st <<= 1) {
    const long long u = __shfl_down(v, st, 64);
    const int r = __shfl_down(run, st, 64);
    if (lane + st < 64 && r == run)
      v = static_cast<long long>(static_cast<unsigned long long>(v) + static_cast<unsigned long long>(u));
  }
  return v;
}

// Creation: particle c N + k of cell c (uniform point, isotropic direction,
// the k-th part of the cell's energy G0[c] split over N), then N per wall face
// waiting for re-emission.
__global__ void persist_init_kernel(const Inst *__restrict__ insts, const long long *__restrict__ G0)
{
  const Inst &in = insts[0];
  const Mesh &m = in.m;
  const unsigned int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= in.n_part) return;
  const unsigned int N = in.N;
  const unsigned int cells = static_cast<unsigned int>(m.n_cells) * N;
  if (p < cells) {
    const unsigned int c = p / N, k = p - c * N;
    const int iy = static_cast<int>(c) / m.nx, ix = static_cast<int>(c) - iy * m.nx;
    const double2 uab = draw2(0u, p, kPersistStream, kPersistCreate, in.key0, in.key1);
    const double2 ucd = draw2(1u, p, kPersistStream, kPersistCreate, in.key0, in.key1);
    in.px[p] = (static_cast<double>(ix) + uab.x) * m.dx;
    in.py[p] = (static_cast<double>(iy) + uab.y) * m.dy;
    double sx, sy;
    iso_direction(m.dim, ucd, sx, sy);
    in.psx[p] = sx;
    in.psy[p] = sy;
    long long w, r;
    share_of(G0[c], N, w, r);
    in.pq[p] = w + ((static_cast<long long>(k) < r) ? 1 : 0);
    in.plk[p] = c;
  } else {
    const unsigned int b = (p - cells) / N;
    in.px[p] = 0.0;
    in.py[p] = 0.0;
    in.psx[p] = 0.0;
    in.psy[p] = 0.0;
    in.pq[p] = 0;
    in.plk[p] = b | (2u << 30);
  }
}

__global__ void persist_prepare_kernel(const Inst *__restrict__ insts)
{
  const Inst &in = insts[0];
  const Mesh &m = in.m;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    in.sc->flights = 0;
    in.sc->segments = 0;
    in.sc->crossings = 0;
    in.sc->gsum = 0;
    in.sc->flags = 0;
  }
  if (i < m.n_cells) {
    in.W[i] = 0;
    in.D[i] = 0;
    in.Nrc[i] = 0;
  }
  if (i < m.n_b) {
    in.B[i] = 0;
    in.Nb[i] = 0;
  }
  if (i < m.n_fx) in.Phix[i] = 0;
  if (i < m.n_fy) in.Phiy[i] = 0;
  if (i < (m.ny + 2) * m.nx) in.dB[i] = 0;
}

// One straight path of length ell from (x0, y0) in cell (ix, iy): the walk's
// face rules (strict crossing, x first on ties, the first wall face absorbs),
// the y-face crossings tallied when faces are on (the x faces follow from the
// per-cell balance afterwards); without face tallies a path expected to
// cross more than kJumpMinFaces faces is resolved in closed form.  The y faces
// a path crosses inside one column form a run; a run of three or more faces
// is recorded as +q at its first and -q past its last face of the column
// difference array dB (completed by a column prefix sum), a shorter one face
// by face, so a path costs at most two atomics per column it crosses faces in.
// Returns true when absorbed by wall face bface.
__device__ __forceinline__ bool persist_walk(const Mesh &m, double x0, double y0, int &ix, int &iy,
                                             double sx, double sy, double ell, int faces,
                                             long long q, long long *Phiy, long long *dB,
                                             int &bface, unsigned long long &n_cross)
{
  const double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
  const double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
  const int stx = (sx > 0.0) ? 1 : ((sx < 0.0) ? -1 : 0);
  const int sty = (sy > 0.0) ? 1 : ((sy < 0.0) ? -1 : 0);
  int kx = (stx > 0) ? ix + 1 : ix;
  int ky = (sty > 0) ? iy + 1 : iy;
  bface = -1;
  if (!faces && ell * (fabs(sx) / m.dx + fabs(sy) / m.dy) > kJumpMinFaces) {
    segment_jump(m, x0, y0, ix, iy, stx, sty, inv_sx, inv_sy, kx, ky, ell, bface, n_cross);
    return bface >= 0;
  }
  const long long qy = sty > 0 ? q : -q;
  int run_a = 0, run_n = 0;   // first y face and length of the open run in column ix
  auto close_run = [&]() {
    if (run_n >= 3) {
      const int lo = sty > 0 ? run_a : run_a - (run_n - 1);
      atom_add(&dB[lo * m.nx + ix], qy);
      atom_add(&dB[(lo + run_n) * m.nx + ix], -qy);
    } else {
      for (int r = 0; r < run_n; ++r) atom_add(&Phiy[(run_a + r * sty) * m.nx + ix], qy);
    }
    run_n = 0;
  };
  bool absorbed = false;
  for (;;) {
    const double tx = stx ? (static_cast<double>(kx) * m.dx - x0) * inv_sx : INFINITY;
    const double ty = sty ? (static_cast<double>(ky) * m.dy - y0) * inv_sy : INFINITY;
    const bool along_x = tx <= ty;
    const double tt = along_x ? tx : ty;
    if (!(tt < ell)) break;
    ++n_cross;
    if (along_x) {
      if (run_n) close_run();
      if (kx == 0 || kx == m.nx) {
        bface = (kx == 0) ? iy : m.ny + iy;
        absorbed = true;
        break;
      }
      ix += stx;
      kx += stx;
    } else {
      if (faces) {
        if (run_n == 0) run_a = ky;
        ++run_n;
      }
      if (ky == 0 || ky == m.ny) {
        bface = (ky == 0) ? 2 * m.ny + ix : 2 * m.ny + m.nx + ix;
        absorbed = true;
        break;
      }
      iy += sty;
      ky += sty;
    }
  }
  if (run_n) close_run();
  return absorbed;
}

// The move: kPersistPer particles per thread, consecutive wavefront-wide
// blocks of the population; tallies by global atomics (W, W^h, N_rc, and
// the crossed faces unless the row-stripe pass takes them), the wall faces'
// B and N_b in LDS when lds_walls (a workgroup's 2048 particles then cost one
// global atomic per wall face they reach, not per particle); counters and
// the null particles' |q| sum per workgroup.
// (no y face crossed: an empty range, first > last for every row count up to
// 65534)
constexpr uint32_t kNoFaces = 0x0000FFFFu;
constexpr int kPersistPer = 8;

template <int BS>
__global__ __launch_bounds__(BS) void persist_move_kernel(const Inst *__restrict__ insts, int faces,
                                                          int stripes, int lds_walls)
{
  extern __shared__ long long s_walls[];   // lds_walls: B [n_b], then N_b [n_b] (32-bit)
  __shared__ unsigned long long s_red[3][BS / 64];
  const Inst &in = insts[0];
  const Mesh &m = in.m;
  const uint32_t slot = in.crn ? in.epoch : in.sc->iter;
  long long *const sB = s_walls;
  uint32_t *const sNb = reinterpret_cast<uint32_t *>(s_walls + m.n_b);
  if (lds_walls) {
    for (int b = threadIdx.x; b < m.n_b; b += BS) {
      sB[b] = 0;
      sNb[b] = 0u;
    }
    __syncthreads();
  }
  unsigned long long fl = 0, cr = 0, nul = 0;
  const unsigned long long p_first = static_cast<unsigned long long>(blockIdx.x) * (BS * kPersistPer);
  for (int it = 0; it < kPersistPer; ++it) {
    const unsigned long long pp = p_first + static_cast<unsigned long long>(it) * BS + threadIdx.x;
    const unsigned int p = static_cast<unsigned int>(pp);
    int ckey = -1, wkey = -1, real = 0;   // end cell or wall face of this lane's path
    long long qv = 0;
    if (pp < in.n_part) {
      const uint32_t lk = in.plk[p];
      const uint32_t kind = lk >> 30, loc = lk & kLocMask;
      double x, y, sx, sy;
      long long q;
      int ix, iy;
      if (kind == 1) {
        const double2 uab = draw2(0u, p, kPersistStream, slot, in.key0, in.key1);
        const double2 ucd = draw2(1u, p, kPersistStream, slot, in.key0, in.key1);
        iy = static_cast<int>(loc) / m.nx;
        ix = static_cast<int>(loc) - iy * m.nx;
        x = (static_cast<double>(ix) + uab.x) * m.dx;
        y = (static_cast<double>(iy) + uab.y) * m.dy;
        iso_direction(m.dim, ucd, sx, sy);
        q = in.wc[loc];
      } else if (kind == 2) {
        const int b = static_cast<int>(loc);
        const double2 uab = draw2(0u, p, kPersistStream, slot, in.key0, in.key1);
        const double2 ucd = draw2(1u, p, kPersistStream, slot, in.key0, in.key1);
        const double cn = sqrt(ucd.x);
        const double tg = (m.dim == 2) ? sqrt((1.0 - cn) * (1.0 + cn)) * cos2pi_own(ucd.y) : 0.0;
        q = in.wb[b];
        if (b < m.ny) {
          ix = 0; iy = b;
          x = 0.0; y = (static_cast<double>(iy) + uab.x) * m.dy;
          sx = cn; sy = tg;
        } else if (b < 2 * m.ny) {
          ix = m.nx - 1; iy = b - m.ny;
          x = static_cast<double>(m.nx) * m.dx; y = (static_cast<double>(iy) + uab.x) * m.dy;
          sx = -cn; sy = tg;
        } else if (b < 2 * m.ny + m.nx) {
          ix = b - 2 * m.ny; iy = 0;
          x = (static_cast<double>(ix) + uab.x) * m.dx; y = 0.0;
          sx = tg; sy = cn;
          if (faces) atom_add(&in.Phiy[ix], q);
        } else {
          ix = b - 2 * m.ny - m.nx; iy = m.ny - 1;
          x = (static_cast<double>(ix) + uab.x) * m.dx; y = static_cast<double>(m.ny) * m.dy;
          sx = tg; sy = -cn;
          if (faces) atom_add(&in.Phiy[m.ny * m.nx + ix], -q);
        }
      } else {
        iy = static_cast<int>(loc) / m.nx;
        ix = static_cast<int>(loc) - iy * m.nx;
        x = in.px[p];
        y = in.py[p];
        sx = in.psx[p];
        sy = in.psy[p];
        q = in.pq[p];
      }
      if (q != 0) ++fl;
      const double2 us = draw2(2u, p, kPersistStream, slot, in.key0, in.key1);
      const double ell = -(in.lam_min * log_own(1.0 - us.x));
      int bface;
      uint32_t nlk;
      bool absorbed;
      if (faces && stripes) {
        // the walk in closed form; its y faces are tallied by persist_faces_kernel
        const double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
        const double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
        const int stx = (sx > 0.0) ? 1 : ((sx < 0.0) ? -1 : 0);
        const int sty = (sy > 0.0) ? 1 : ((sy < 0.0) ? -1 : 0);
        const int kx = (stx > 0) ? ix + 1 : ix, ky = (sty > 0) ? iy + 1 : iy;
        const uint32_t cell = static_cast<uint32_t>(ix) | (static_cast<uint32_t>(iy) << 16);
        int nxp = 0, nyp = 0;
        bface = -1;
        segment_end(m, x, y, ix, iy, stx, sty, inv_sx, inv_sy, kx, ky, ell, bface, nxp, nyp);
        cr += static_cast<unsigned long long>(nxp + nyp);
        absorbed = bface >= 0;
        uint32_t key = kNoFaces;
        if (nyp > 0) {
          const int kl = ky + (nyp - 1) * sty;
          key = static_cast<uint32_t>(min(ky, kl)) | (static_cast<uint32_t>(max(ky, kl)) << 16);
          PFace r;
          r.x0 = x;
          r.y0 = y;
          r.sx = sx;
          r.inv_sx = inv_sx;
          r.inv_sy = inv_sy;
          r.q = q;
          r.cell = cell;
          r.nyp = static_cast<uint32_t>(nyp);
          in.pf[p] = r;
        }
        in.pkey[p] = key;
      } else {
        absorbed = persist_walk(m, x, y, ix, iy, sx, sy, ell, faces, q, in.Phiy, in.dB, bface, cr);
      }
      if (absorbed) {
        wkey = bface;
        nlk = static_cast<uint32_t>(bface) | (2u << 30);
      } else {
        const int c = ix + m.nx * iy;
        ckey = c;
        x = clamp_to(x + ell * sx, static_cast<double>(ix) * m.dx, static_cast<double>(ix + 1) * m.dx);
        if (m.dim == 2)
          y = clamp_to(y + ell * sy, static_cast<double>(iy) * m.dy, static_cast<double>(iy + 1) * m.dy);
        if (us.y < in.ratio[c]) {
          real = 1;
          nlk = static_cast<uint32_t>(c) | (1u << 30);
        } else {
          nul += abs_u64(q);                    // (each term <= 2^62: capped below)
          if (nul > kBudgetCap) nul = kBudgetCap;
          nlk = static_cast<uint32_t>(c);
        }
      }
      qv = q;
      in.px[p] = x;
      in.py[p] = y;
      in.psx[p] = sx;
      in.psy[p] = sy;
      in.pq[p] = q;
      in.plk[p] = nlk;
    }
    // end tallies, summed over runs of equal consecutive keys in the wavefront
    // first (particles of neighbouring indices tend to end in the same cell)
    {
      int head, run;
      // (W takes the null particles' weights only here; persist_update_kernel
      // adds W^h, so a real collision costs two atomics, not three)
      wave_runs(ckey, head, run);
      const long long sw = run_sum(real ? 0ll : qv, run);
      const long long sh = run_sum(real ? qv : 0ll, run);
      const long long sn = run_sum(static_cast<long long>(real), run);
      if (head && ckey >= 0) {
        if (sw) atom_add(&in.W[ckey], sw);   // (adding 0 changes nothing)
        if (sn) {
          atom_add(&in.D[ckey], sh);
          atomicAdd(&in.Nrc[ckey], static_cast<uint32_t>(sn));
        }
      }
      wave_runs(wkey, head, run);
      const long long sb = run_sum(wkey >= 0 ? qv : 0ll, run);
      const long long sc = run_sum(wkey >= 0 ? 1ll : 0ll, run);
      if (head && wkey >= 0) {
        if (lds_walls) {
          atomicAdd(reinterpret_cast<unsigned long long *>(&sB[wkey]), static_cast<unsigned long long>(sb));
          atomicAdd(&sNb[wkey], static_cast<uint32_t>(sc));
        } else {
          atom_add(&in.B[wkey], sb);
          atomicAdd(&in.Nb[wkey], static_cast<uint32_t>(sc));
        }
      }
    }
  }
  if (lds_walls) {
    __syncthreads();
    for (int b = threadIdx.x; b < m.n_b; b += BS) {
      if (sB[b]) atom_add(&in.B[b], sB[b]);
      if (sNb[b]) atomicAdd(&in.Nb[b], sNb[b]);
    }
  }
  // per-wave sums (each |q| <= 2^62 and 64 of them fit in 2^68: cap first)
  if (nul > kBudgetCap) nul = kBudgetCap;
#pragma unroll
  for (int st = 32; st >= 1; st >>= 1) {
    fl += __shfl_down(fl, st, 64);
    cr += __shfl_down(cr, st, 64);
    const unsigned long long o = __shfl_down(nul, st, 64);
    nul = (nul + o > kBudgetCap) ? kBudgetCap : nul + o;
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_red[0][wv] = fl;
    s_red[1][wv] = cr;
    s_red[2][wv] = nul;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long f = 0, c = 0, n = 0;
    for (int i = 0; i < BS / 64; ++i) {
      f += s_red[0][i];
      c += s_red[1][i];
      n = (n + s_red[2][i] > kBudgetCap) ? kBudgetCap : n + s_red[2][i];
    }
    if (f) atomicAdd(&in.sc->flights, f);
    atomicAdd(&in.sc->segments, min(static_cast<unsigned long long>(BS * kPersistPer),
                                    static_cast<unsigned long long>(in.n_part) - p_first));
    if (c) atomicAdd(&in.sc->crossings, c);
    in.npart[blockIdx.x] = n;
  }
}

// The y-face tallies of a face-tallied persistent move, by row stripes:
// workgroup (chunk c, stripe s) keeps in LDS the tallies of faces [r0, r1f)
// (the last stripe also owns face ny) and tallies the crossings of its
// chunk's paths with those faces, each in the column reached by the x faces
// crossed before it (x first on ties, as in the walk); then the stripe is
// added to the global tallies row by row.  The chunk is scanned kPersistScan
// ranges at a time: the paths that meet the stripe are listed in LDS, and
// their owned crossings are cut into pieces of at most kPersistPiece
// consecutive faces (a workgroup prefix sum over the list numbers them), one
// piece per lane, so the lanes of a wavefront do nearly equal work whatever
// the spread of path lengths.  A crossing's column needs no earlier crossing
// of its path (faces_upto_near from its own time).  Integer sums: the tallies
// of the face-by-face walk, bit for bit.
constexpr int kPersistScan = 2048;
constexpr int kPersistPiece = 16;

template <int BS>
__global__ __launch_bounds__(BS) void persist_faces_kernel(const Inst *__restrict__ insts, int R,
                                                           int chunks)
{
  static_assert(2 * BS >= kPersistScan, "two listed paths per thread in the piece count scan");
  extern __shared__ long long lds_words[];
  __shared__ uint32_t s_list[kPersistScan];      // listed paths (population index)
  __shared__ uint32_t s_pre[kPersistScan + 1];   // first piece of each listed path
  __shared__ uint32_t s_wsum[BS / 64];
  __shared__ uint32_t s_n;
  const Inst &in = insts[0];
  const Mesh m = in.m;
  const int nx = m.nx;
  const int r0 = static_cast<int>(blockIdx.y) * R, r1 = min(r0 + R, m.ny);
  const int r1f = (r1 == m.ny) ? m.ny + 1 : r1;
  const int nface = r1f - r0;
  long long *By = lds_words;                                  // [nface][nx]
  for (int i = threadIdx.x; i < nface * nx; i += BS) By[i] = 0;
  const PFace *__restrict__ pf = in.pf;
  const uint32_t *__restrict__ pkey = in.pkey;
  const unsigned long long n = in.n_part;
  const unsigned long long pb = n * blockIdx.x / chunks, pe = n * (blockIdx.x + 1) / chunks;
  const double inv_dx = 1.0 / m.dx;       // (only to estimate a face count)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // owned crossed faces [max(lo, r0), min(hi, r1f - 1)] of a range lo | hi << 16
  auto owned_lo = [&](uint32_t key) { return max(static_cast<int>(key & 0xffffu), r0); };
  auto owned_n = [&](uint32_t key) {
    return min(static_cast<int>(key >> 16), r1f - 1) - owned_lo(key) + 1;
  };
  for (unsigned long long base = pb; base < pe; base += kPersistScan) {
    const unsigned long long end = min(pe, base + kPersistScan);
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    // the ranges that meet the stripe, listed (one LDS atomic per wavefront)
    for (unsigned long long p0 = base; p0 < end; p0 += BS) {
      const unsigned long long p = p0 + threadIdx.x;
      bool hit = false;
      if (p < end) {
        const uint32_t key = pkey[p];
        hit = static_cast<int>(key >> 16) >= r0 && static_cast<int>(key & 0xffffu) < r1f;
      }
      const unsigned long long mask = __ballot(hit);
      if (mask) {
        uint32_t off = 0;
        if (lane == 0) off = atomicAdd(&s_n, static_cast<uint32_t>(__popcll(mask)));
        off = __shfl(off, 0, 64);
        if (hit) s_list[off + __popcll(mask & ((1ull << lane) - 1ull))] = static_cast<uint32_t>(p);
      }
    }
    __syncthreads();
    const int nl = static_cast<int>(s_n);
    // pieces per listed path, numbered by an exclusive prefix sum
    {
      const int i0 = 2 * static_cast<int>(threadIdx.x), i1 = i0 + 1;
      const uint32_t c0 = (i0 < nl) ? (owned_n(pkey[s_list[i0]]) + kPersistPiece - 1) / kPersistPiece : 0u;
      const uint32_t c1 = (i1 < nl) ? (owned_n(pkey[s_list[i1]]) + kPersistPiece - 1) / kPersistPiece : 0u;
      uint32_t incl = c0 + c1;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), d, 64));
        if (lane >= d) incl += o;
      }
      if (lane == 63) s_wsum[wv] = incl;
      __syncthreads();
      uint32_t off = 0;
      for (int v = 0; v < wv; ++v) off += s_wsum[v];
      const uint32_t ex = off + incl - c0 - c1;
      if (i0 < nl) s_pre[i0] = ex;
      if (i1 < nl) s_pre[i1] = ex + c0;
      if (i0 < nl && i1 >= nl - 1) s_pre[nl] = ex + c0 + c1;
      if (nl == 0 && threadIdx.x == 0) s_pre[0] = 0;
    }
    __syncthreads();
    const uint32_t n_piece = s_pre[nl];
    for (uint32_t u = threadIdx.x; u < n_piece; u += BS) {
      // the listed path of piece u: the last i with s_pre[i] <= u
      int a = 0, b = nl - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (s_pre[mid] <= u) a = mid;
        else b = mid - 1;
      }
      const uint32_t pi = s_list[a];
      const uint32_t key = pkey[pi];
      const PFace r = pf[pi];
      const int ix0 = static_cast<int>(r.cell & 0xffffu);
      const int stx = (r.sx > 0.0) ? 1 : ((r.sx < 0.0) ? -1 : 0);
      const long long qy = (r.inv_sy > 0.0) ? r.q : -r.q;     // (a y face crossed: s_y != 0)
      const int kx0 = (stx > 0) ? ix0 + 1 : ix0;
      const int jwx = (stx > 0) ? nx - kx0 : kx0;
      const int f0 = owned_lo(key) + static_cast<int>(u - s_pre[a]) * kPersistPiece;
      const int f1 = min(owned_lo(key) + owned_n(key), f0 + kPersistPiece);
      for (int kyk = f0; kyk < f1; ++kyk) {
        const double ty = (static_cast<double>(kyk) * m.dy - r.y0) * r.inv_sy;
        const int cnt = stx ? faces_upto_near(0, kx0, stx, jwx, m.dx, inv_dx, r.x0, r.inv_sx, r.sx, ty) : 0;
        atomicAdd(reinterpret_cast<unsigned long long *>(&By[(kyk - r0) * nx + ix0 + stx * cnt]),
                  static_cast<unsigned long long>(qy));
      }
    }
    __syncthreads();
  }
  __syncthreads();   // (an empty chunk: the zeroed tallies)
  long long *const gPhiy = in.Phiy;
  for (int i = threadIdx.x; i < nface * nx; i += BS)
    if (By[i]) atom_add(&gPhiy[r0 * nx + i], By[i]);
}

// E = W / V, the residual partials, and the shares of the next iteration:
// blocks [0, nbc) cells, then the wall faces, then one block that folds the
// move's null partials; |q| budget partials into gpart.
__global__ __launch_bounds__(256) void persist_update_kernel(const Inst *__restrict__ insts)
{
  __shared__ double lds[kTree];
  __shared__ unsigned long long lg[kTree];
  const Inst &in = insts[0];
  const int nc = in.m.n_cells, nb = in.m.n_b;
  const int nbc = (nc + kTree - 1) / kTree, nbw = (nb + kTree - 1) / kTree;
  const int t = threadIdx.x;
  double sq = 0.0;
  unsigned long long ag = 0;
  int flags = 0;
  if (static_cast<int>(blockIdx.x) < nbc) {
    const int c = blockIdx.x * kTree + t;
    if (c < nc) {
      // W: the move tallied the null particles' weights, W^h the real ones'
      const long long Wc = static_cast<long long>(static_cast<unsigned long long>(in.W[c]) +
                                                  static_cast<unsigned long long>(in.D[c]));
      in.W[c] = Wc;
      const double En = ldexp(static_cast<double>(Wc), -in.F) / in.V;
      const double d = En - in.E[c];
      sq = d * d;
      if (!isfinite(En)) flags |= 1;
      in.E[c] = En;
      int over = 0;
      const long long avail =
          add_budget(add_budget(in.D[c], in.Gs ? in.Gs[c] : 0ll, &over), in.rc[c], &over);
      if (over) flags |= 2;
      const uint32_t n = in.Nrc[c];
      long long w = 0, r = avail;
      if (n) share_of(avail, n, w, r);
      in.wc[c] = w;
      in.rc[c] = r;
      ag = abs_u64(w) * n + abs_u64(r);
      // the next iteration's paths start from this cell with the null
      // particles' weights and the real ones' new share
      in.pstart[c] = static_cast<long long>(static_cast<unsigned long long>(Wc) -
                                            static_cast<unsigned long long>(in.D[c]) +
                                            static_cast<unsigned long long>(w) * n);
    }
  } else if (static_cast<int>(blockIdx.x) < nbc + nbw) {
    const int b = (blockIdx.x - nbc) * kTree + t;
    if (b < nb) {
      int over = 0;
      const long long avail = add_budget(in.Gw[b], in.rb[b], &over);
      if (over) flags |= 2;
      const uint32_t n = in.Nb[b];
      long long w = 0, r = avail;
      if (n) share_of(avail, n, w, r);
      in.wb[b] = w;
      in.rb[b] = r;
      ag = abs_u64(w) * n + abs_u64(r);
      in.pein[b] = static_cast<long long>(static_cast<unsigned long long>(w) * n);
    }
  } else {
    for (int i = t; i < in.n_npart; i += kTree) ag = (ag + in.npart[i] > kBudgetCap) ? kBudgetCap : ag + in.npart[i];
  }
  if (flags) atomicOr(&in.sc->flags, flags);
  const double s = block_tree256(sq, lds);
  lg[t] = ag > kBudgetCap ? kBudgetCap : ag;
  __syncthreads();
  for (int st = kTree / 2; st >= 1; st >>= 1) {
    if (t < st) {
      const unsigned long long u = lg[t] + lg[t + st];
      lg[t] = u > kBudgetCap ? kBudgetCap : u;
    }
    __syncthreads();
  }
  if (t == 0) {
    if (static_cast<int>(blockIdx.x) < nbc) in.part[blockIdx.x] = s;
    in.gpart[blockIdx.x] = lg[0];
  }
}

// x-face fluxes of a persistent iteration from the integer balance of every
// cell, row by row: net inflow = (energy ending its path in the cell) -
// (energy starting from it):
//   Phix[j][0]   = (re-emitted by the left wall face j) - B_left[j]
//   Phix[j][i+1] = Phix[j][i] + Phiy[j][i] - Phiy[j+1][i] - W[c] + start[c]
// (arithmetic modulo 2^64, exact since every true value fits in int64).
__global__ __launch_bounds__(256) void persist_reconstruct_x_kernel(const Inst *__restrict__ insts)
{
  const Inst &in = insts[0];
  const Mesh &m = in.m;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= m.ny) return;
  const unsigned long long a0 = static_cast<unsigned long long>(in.pein[j]) -
                                static_cast<unsigned long long>(in.B[j]);
  long long *const px = in.Phix + static_cast<size_t>(j) * (m.nx + 1);
  if ((threadIdx.x & 63) == 0) px[0] = static_cast<long long>(a0);
  const bool two = (m.dim == 2);
  wave_prefix(
      m.nx, a0,
      [&](int i) {
        const int c = j * m.nx + i;
        const unsigned long long dy =
            two ? static_cast<unsigned long long>(in.Phiy[j * m.nx + i]) -
                      static_cast<unsigned long long>(in.Phiy[(j + 1) * m.nx + i])
                : 0ull;
        // (W is still the null part here: the cell's end weight is W + W^h)
        return dy + (static_cast<unsigned long long>(in.pstart[c]) -
                     static_cast<unsigned long long>(in.W[c]) - static_cast<unsigned long long>(in.D[c]));
      },
      [&](int i, unsigned long long v) { px[i + 1] = static_cast<long long>(v); });
}

// Unpack location | kind << 30.
__global__ void persist_unpack_kernel(const uint32_t *lk, unsigned int n, int32_t *kind, int32_t *loc)
{
  const unsigned int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (kind) kind[i] = static_cast<int32_t>(lk[i] >> 30);
  if (loc) loc[i] = static_cast<int32_t>(lk[i] & kLocMask);
}

// zero a small integer array (used instead of a memset node so the sequence can
// be captured in a graph)
__global__ void zero_u32_kernel(unsigned int *p, int n)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// building-block probes
// ---------------------------------------------------------------------------

// Tally-throughput ceilings: every thread adds 1 to `per_thread` pseudo-random
// words (a multiplicative hash of thread and step) of an int64 array of
// n_words, either in global memory (lds == 0: `words`, n_words of them) or in
// a workgroup's LDS array (lds == 1: 4096 words, flushed to `words` at the end
// so the work is not optimised away).
__global__ __launch_bounds__(256) void atomics_probe_kernel(int lds, long long *words, int n_words,
                                                            int per_thread)
{
  __shared__ long long tab[4096];
  const unsigned int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (lds) {
    for (int i = threadIdx.x; i < 4096; i += blockDim.x) tab[i] = 0;
    __syncthreads();
  }
  uint32_t h = t * 2654435761u + 12345u;
  for (int i = 0; i < per_thread; ++i) {
    h = h * 1664525u + 1013904223u;
    if (lds)
      atomicAdd(reinterpret_cast<unsigned long long *>(&tab[(h >> 8) & 4095u]), 1ull);
    else
      atomicAdd(reinterpret_cast<unsigned long long *>(&words[(h >> 4) % static_cast<uint32_t>(n_words)]),
                1ull);
  }
  if (lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < 4096; i += blockDim.x)
      if (tab[i]) atomicAdd(reinterpret_cast<unsigned long long *>(&words[i % n_words]),
                            static_cast<unsigned long long>(tab[i]));
  }
}
__global__ void philox_probe_kernel(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out,
                                    long long n)
{
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 o = philox4x32_10(make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2],
                                           ctr[4 * i + 3]), k0, k1);
  out[4 * i] = o.x;
  out[4 * i + 1] = o.y;
  out[4 * i + 2] = o.z;
  out[4 * i + 3] = o.w;
}

// segment_jump on given segments: rays[7 i ..] = x0, y0, ix, iy, sx, sy, ell;
// out[3 i ..] = absorbed (0/1), final cell or wall face, crossings
__global__ void segment_probe_kernel(Mesh m, const double *rays, long long n, long long *out)
{
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *r = rays + 7 * i;
  const double x0 = r[0], y0 = r[1], sx = r[4], sy = r[5], ell = r[6];
  int ix = static_cast<int>(r[2]), iy = static_cast<int>(r[3]);
  const double inv_sx = (sx != 0.0) ? 1.0 / sx : 0.0;
  const double inv_sy = (sy != 0.0) ? 1.0 / sy : 0.0;
  const int stx = (sx > 0.0) ? 1 : ((sx < 0.0) ? -1 : 0);
  const int sty = (sy > 0.0) ? 1 : ((sy < 0.0) ? -1 : 0);
  const int kx = (stx > 0) ? ix + 1 : ix, ky = (sty > 0) ? iy + 1 : iy;
  int bface = -1;
  unsigned long long nc = 0;
  segment_jump(m, x0, y0, ix, iy, stx, sty, inv_sx, inv_sy, kx, ky, ell, bface, nc);
  out[3 * i] = bface >= 0 ? 1 : 0;
  out[3 * i + 1] = bface >= 0 ? bface : ix + m.nx * iy;
  out[3 * i + 2] = static_cast<long long>(nc);
}

__global__ void math_probe_kernel(int op, const double *x, const double *y, double *out,
                                  long long n)
{
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[i];
  double r = 0.0;
  switch (op) {
    case 0: r = log_own(a); break;
    case 1: r = cos2pi_own(a); break;
    case 2: r = sqrt(a); break;
    case 3: r = a / y[i]; break;
    case 4: r = static_cast<double>(__double_as_longlong(a)); break;
    case 5: {
      const long long v = static_cast<long long>(rint(ldexp(a, static_cast<int>(y[i]))));
      r = __longlong_as_double(v);
      break;
    }
    case 6: r = expm_own(a); break;
    default: break;
  }
  out[i] = r;
}

}  // namespace iugkp
