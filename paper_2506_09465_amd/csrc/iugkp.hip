// iugkp.hip -- C ABI of the gfx950 IUGKP solver (declarations in include/iugkp.h).
//
// One translation unit: device kernels (kernels.hpp), set-up arithmetic
// (host_math.hpp), the single-problem driver and the batched driver.  Built
// with -ffp-contract=off and no fast-math so that every floating-point result
// is fixed by IEEE binary64 semantics.
//
// Every per-iteration kernel reads its problem from a device-side descriptor
// (iugkp::Inst).  A single solve is a batch of one driven from the host; a
// batch advances all its instances with one launch per phase, the sequence
// captured once in a HIP graph and replayed until every instance is done (the
// per-instance iteration control lives on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/iugkp.h"
#include "host_math.hpp"
#include "kernels.hpp"
#include "mgcg.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg)
{
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(IUGKP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

constexpr int kCgGridMax = 64;               // workgroups of one CG group (barrier arrivals)
constexpr int kCgWavesDefault = 8;           // tree blocks per CG workgroup of a single solve
constexpr int kBarStride = 64;               // batched CG barriers 256 bytes apart (no shared lines)
constexpr double kStripeMinCells = 7.0;      // row stripes for face tallies when lambda_min >= 7 cells
constexpr int kStripeBlock = 1024;           // threads of a stripe workgroup
constexpr int kStripeMinRows = 4;
constexpr size_t kCgLdsMax = 48 * 1024;      // dynamic LDS of a CG workgroup
constexpr int kPersistBlock = 256;           // particles per move workgroup
constexpr int kPersistFacesBlock = 1024;     // threads per workgroup of the row-stripe face pass
constexpr int kTileX = 8;                    // emitter tile of one workgroup (cells per side;
                                             // wall faces per workgroup); batches also 16
constexpr int kWindowHalo = 12;              // window margin around a tile (cells)
constexpr int kWindowHaloNull = 20;          // a single solve's with null collisions (long chains;
                                             // one launch of bands or of a batch takes the
                                             // largest window's LDS for every workgroup)
constexpr size_t kLdsWordsMax = 6144;        // 48 KB of 64-bit tallies per workgroup
constexpr int kLdsWallsMax = 1024;

inline int cdiv(long long a, long long b) { return static_cast<int>((a + b - 1) / b); }

void *cg_kernel_for(int reg)
{
  return reg ? reinterpret_cast<void *>(iugkp::cg_kernel<true>)
             : reinterpret_cast<void *>(iugkp::cg_kernel<false>);
}

// Launch shape of the single-solve CG on a mesh: a group of at most
// kCgGridMax resident workgroups (the barrier cost grows with the arrivals) of
// cg_waves tree blocks each (0: the default); the register form when every
// block has its own wave and the rows fit in LDS (cg_waves < 0 forces the
// global-memory form).
struct CgPlan {
  int grid = 1, tb = 1, reg = 1, threads = 64, per_cu = 1;
  size_t lds = 0;
};

int plan_cg(const iugkp::Mesh &m, int cg_waves, CgPlan &out)
{
  int dev = 0, n_cu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  const int nbt = cdiv(m.n_cells, iugkp::kTree);
  const int hw = (m.dim == 2) ? m.nx : 1;
  const int want = cg_waves != 0 ? std::abs(cg_waves) : kCgWavesDefault;
  int G = std::max(1, std::min(std::min(cdiv(nbt, want), kCgGridMax), n_cu));
  // more workgroups rather than the global form, while one per CU suffices
  if (cdiv(nbt, G) > iugkp::kCgWavesMax && cdiv(nbt, iugkp::kCgWavesMax) <= n_cu)
    G = cdiv(nbt, iugkp::kCgWavesMax);
  const int TB = cdiv(nbt, G);
  G = cdiv(nbt, TB);
  size_t lds = (static_cast<size_t>(TB) * iugkp::kTree + 2 * static_cast<size_t>(hw)) *
               sizeof(double);
  int reg = (cg_waves >= 0 && TB <= iugkp::kCgWavesMax && lds <= kCgLdsMax) ? 1 : 0;
  if (!reg) lds = 2 * static_cast<size_t>(hw) * sizeof(double);
  if (lds > kCgLdsMax) return fail(IUGKP_E_INVALID_ARG, "mesh rows too long for the Newton CG");
  const int threads = 64 * (reg ? TB : std::min(TB, iugkp::kCgWavesMax));
  int per_cu = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cg_kernel_for(reg), threads, lds));
  if (per_cu < 1 || G > per_cu * n_cu)
    return fail(IUGKP_E_DEVICE, "CG workgroups cannot all be resident");
  out.grid = G;
  out.tb = TB;
  out.reg = reg;
  out.threads = threads;
  out.lds = lds;
  out.per_cu = per_cu;
  return IUGKP_OK;
}

}  // namespace

using iugkp::DevScalars;
using iugkp::Inst;
using iugkp::Mesh;
using iugkp::TileDesc;

namespace {

// Host-side record of one problem instance and the device memory it owns.
struct InstHost {
  Inst d{};                          // descriptor (device pointers) as uploaded
  iugkp_options opt{};
  int mem_kind = IUGKP_MEM_HOST;
  std::vector<TileDesc> tiles;       // inst field filled by the owner
  size_t lds_bytes = 0;              // march window
  std::vector<void *> allocs;
  double *tau = nullptr, *Dx = nullptr, *Dy = nullptr, *gx = nullptr, *gy = nullptr,
         *diag = nullptr;
  double *out_T = nullptr, *out_qx = nullptr, *out_qy = nullptr;
  // multi-workgroup CG (single solves)
  double *cg_pub = nullptr, *cg_mpart = nullptr;
  unsigned int *cg_barrier = nullptr;
  int cg_grid = 1, cg_tb = 1, cg_reg = 1, cg_threads = 64;
  size_t cg_lds = 0;
  // the CG group's footprint in compute units (workgroups / resident ones per
  // CU): grouped stepping keeps the CGs in flight within the device
  double cg_cus = 0.0;
  // multigrid-preconditioned CG (cg_precond == IUGKP_PRECOND_MG): level table
  int mg_L = 0, mg_Lg = 0, mg_grid = 1, mg_threads = 64;
  size_t mg_lds = 0;
  iugkp::MGLevel *mg_lv = nullptr;
  // its banded form: the second buffers of r and s, the LDS layout
  int mg_band = 0, mg_stage0 = 0, mg_stage_n = 0;
  double *mg_r2 = nullptr, *mg_s2 = nullptr;
  // row-stripe particle step for face-tallied iterations (single solves)
  int stripe_R = 0, stripe_S = 0, stripe_C = 0;
  size_t stripe_lds = 0;
  int stripe_pref = 0;               // the planner's choice (stripes set up for a search too)
  // the persistent scheme's row-stripe face pass (rows per stripe, stripes,
  // chunks, LDS bytes; 0 rows: y faces as global atomics in the move)
  int pst_R = 0, pst_S = 0, pst_C = 0;
  size_t pst_lds = 0;
  iugkp::StripeRec rec{};            // first segments, sampled once for all stripes

  template <class T>
  hipError_t alloc(T **p, size_t n)
  {
    *p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
    if (e == hipSuccess) allocs.push_back(*p);
    return e;
  }
  void release()
  {
    for (void *p : allocs) (void)hipFree(p);
    allocs.clear();
  }
};

int check_problem(const iugkp_problem *p)
{
  if (!p) return fail(IUGKP_E_INVALID_ARG, "problem is NULL");
  if (p->dim != 1 && p->dim != 2) return fail(IUGKP_E_INVALID_ARG, "dim must be 1 or 2");
  if (p->nx < 1 || p->ny < 1 || (p->dim == 1 && p->ny != 1))
    return fail(IUGKP_E_INVALID_ARG, "bad mesh size");
  // the two-level fixed-order reductions cover 256 * 256 tree blocks
  if ((long long)p->nx * p->ny > (1ll << 24)) return fail(IUGKP_E_INVALID_ARG, "mesh too large");
  if (!(p->dx > 0) || !(p->dy > 0) || !std::isfinite(p->dx) || !std::isfinite(p->dy))
    return fail(IUGKP_E_INVALID_ARG, "cell sizes must be positive and finite");
  if (p->n_bands < 0) return fail(IUGKP_E_INVALID_ARG, "n_bands must be >= 0");
  if (!std::isfinite(p->t_ref)) return fail(IUGKP_E_INVALID_ARG, "t_ref must be finite");
  if (p->n_bands < 2 &&
      (!(p->cv > 0) || !(p->vg > 0) || !std::isfinite(p->cv) || !std::isfinite(p->vg)))
    return fail(IUGKP_E_INVALID_ARG, "cv, vg must be positive and finite");
  if (p->n_bands >= 2 && (!p->band_C || !p->band_vg))
    return fail(IUGKP_E_INVALID_ARG, "band_C and band_vg are required for frequency bands");
  if (!p->tau || !p->wall_T) return fail(IUGKP_E_INVALID_ARG, "tau and wall_T are required");
  if (p->mem_kind != IUGKP_MEM_HOST && p->mem_kind != IUGKP_MEM_DEVICE)
    return fail(IUGKP_E_INVALID_ARG, "bad mem_kind");
  return IUGKP_OK;
}

int check_options(const iugkp_options *o)
{
  if (!o) return fail(IUGKP_E_INVALID_ARG, "options is NULL");
  if (o->particles_per_iter < 1) return fail(IUGKP_E_INVALID_ARG, "particles_per_iter < 1");
  if (o->rng_mode != IUGKP_RNG_FRESH && o->rng_mode != IUGKP_RNG_CRN)
    return fail(IUGKP_E_INVALID_ARG, "bad rng_mode");
  if (o->max_iters < 0 || o->avg_iters < 0) return fail(IUGKP_E_INVALID_ARG, "negative count");
  if (o->tally_faces < 0 || o->tally_faces > 2) return fail(IUGKP_E_INVALID_ARG, "bad tally_faces");
  if (o->newton && (!(o->cg_tol > 0) || o->cg_max_iters < 1))
    return fail(IUGKP_E_INVALID_ARG, "Newton needs cg_tol > 0 and cg_max_iters >= 1");
  const int bs = o->block_size;
  if (bs != 0 && bs != 64 && bs != 128 && bs != 256 && bs != 512 && bs != 1024)
    return fail(IUGKP_E_INVALID_ARG, "block_size must be 0, 64, 128, 256, 512 or 1024");
  if (o->march < 0 || o->march > 3) return fail(IUGKP_E_INVALID_ARG, "march must be 0, 1, 2 or 3");
  if (o->cg_waves < -iugkp::kCgWavesMax || o->cg_waves > iugkp::kCgWavesMax)
    return fail(IUGKP_E_INVALID_ARG, "cg_waves must be -12..12");
  if (o->scheme != IUGKP_SCHEME_EMITTERS && o->scheme != IUGKP_SCHEME_PERSISTENT)
    return fail(IUGKP_E_INVALID_ARG, "bad scheme");
  if (o->scheme == IUGKP_SCHEME_PERSISTENT && o->newton)
    return fail(IUGKP_E_INVALID_ARG, "the persistent scheme has no Newton step");
  if (o->estimator != IUGKP_EST_ANALOG && o->estimator != IUGKP_EST_EXPECTED)
    return fail(IUGKP_E_INVALID_ARG, "bad estimator");
  if (o->estimator == IUGKP_EST_EXPECTED && o->scheme != IUGKP_SCHEME_EMITTERS)
    return fail(IUGKP_E_INVALID_ARG, "the expected-value estimator is for the emitter scheme");
  if (o->cg_precond != IUGKP_PRECOND_NONE && o->cg_precond != IUGKP_PRECOND_MG)
    return fail(IUGKP_E_INVALID_ARG, "bad cg_precond");
  return IUGKP_OK;
}

int fetch_host(const double *src, size_t n, int kind, std::vector<double> &dst)
{
  dst.resize(n);
  if (kind == IUGKP_MEM_HOST) {
    std::memcpy(dst.data(), src, n * sizeof(double));
    return IUGKP_OK;
  }
  HIP_TRY(hipMemcpy(dst.data(), src, n * sizeof(double), hipMemcpyDeviceToHost));
  return IUGKP_OK;
}

// Scale exponent F = 62 - ceil(log2 B), B = 4 max(|E_wall|, |E_0|) total, with
// total = sum of cell volumes + lambda_min (sum of wall-face areas) / 4.
int scale_exponent(const iugkp_problem *p, double tau_min, const std::vector<double> &wall_T,
                   const std::vector<double> &T0, const std::vector<double> &src)
{
  double maxabs = 0.0;
  for (double tw : wall_T) maxabs = std::max(maxabs, std::fabs(p->cv * (tw - p->t_ref)));
  for (double t : T0) maxabs = std::max(maxabs, std::fabs(p->cv * (t - p->t_ref)));
  const double lam_min = p->vg * tau_min;
  const double vol = static_cast<double>(p->nx * p->ny) * (p->dx * p->dy);
  const double area = (p->dim == 2) ? ((2.0 * p->ny) * p->dy + (2.0 * p->nx) * p->dx) : 2.0;
  const double total = vol + (lam_min * area) / 4.0;
  double B = (4.0 * maxabs) * total;
  // a source raises the energy level by at most about S_max tau_min times the
  // iterations energy stays inside, bounded by 1 + 3 (L / lambda_min)^2
  double smax = 0.0;
  for (double sv : src) smax = std::max(smax, std::fabs(sv));
  if (smax > 0.0) {
    double L = static_cast<double>(p->nx) * p->dx;
    if (p->dim == 2 && static_cast<double>(p->ny) * p->dy > L) L = static_cast<double>(p->ny) * p->dy;
    const double rl = L / lam_min;
    const double esrc = (smax * tau_min) * (1.0 + 3.0 * (rl * rl));
    B = (4.0 * (maxabs + esrc)) * total;
  }
  if (!(B > 0.0)) return 62;
  int e = 0;
  const double mant = std::frexp(B, &e);
  return 62 - ((mant == 0.5) ? e - 1 : e);
}

// Tile table and LDS window: the whole domain when its tallies fit in LDS,
// otherwise a window of the tile plus a margin, placed inside the domain.
// Emitter tiles of edge x edge cells (and wall segments of edge faces), each
// with its LDS window: the whole domain when it fits, else the tile and
// halo cells around it.
void plan_tiles(InstHost &ih, int edge = kTileX, int halo = kWindowHalo)
{
  Inst &d = ih.d;
  const Mesh &m = d.m;
  d.lds_walls = (m.n_b <= kLdsWallsMax) ? 1 : 0;
  const size_t whole = iugkp::window_words(m.nx, m.ny, d.has_null, d.lds_walls, m.n_b);
  const bool whole_domain = whole <= kLdsWordsMax;
  if (whole_domain) {
    d.WX = m.nx;
    d.WY = m.ny;
  } else {
    d.WX = std::min(m.nx, edge + 2 * halo);
    d.WY = std::min(m.ny, edge + 2 * halo);
  }
  auto place = [](int lo, int extent, int W, int n) {
    int w0 = lo - (W - extent) / 2;
    if (w0 > n - W) w0 = n - W;
    if (w0 < 0) w0 = 0;
    return w0;
  };
  ih.tiles.clear();
  for (int ty = 0; ty < m.ny; ty += edge)
    for (int tx = 0; tx < m.nx; tx += edge) {
      TileDesc t{};
      t.kind = 0;
      t.x0 = tx;
      t.y0 = ty;
      t.ex = std::min(edge, m.nx - tx);
      t.ey = std::min(edge, m.ny - ty);
      t.wx0 = whole_domain ? 0 : place(tx, t.ex, d.WX, m.nx);
      t.wy0 = whole_domain ? 0 : place(ty, t.ey, d.WY, m.ny);
      ih.tiles.push_back(t);
    }
  // wall segments: left rows, right rows, bottom columns, top columns
  auto wall = [&](int b_first, int count, int along_x, int side_hi) {
    for (int s0 = 0; s0 < count; s0 += edge) {
      TileDesc t{};
      t.kind = 1;
      t.x0 = b_first + s0;
      t.ex = std::min(edge, count - s0);
      t.ey = 1;
      if (whole_domain) {
        t.wx0 = 0;
        t.wy0 = 0;
      } else if (along_x) {
        t.wx0 = place(s0, t.ex, d.WX, m.nx);
        t.wy0 = side_hi ? m.ny - d.WY : 0;
      } else {
        t.wy0 = place(s0, t.ex, d.WY, m.ny);
        t.wx0 = side_hi ? m.nx - d.WX : 0;
      }
      ih.tiles.push_back(t);
    }
  };
  wall(0, m.ny, 0, 0);
  wall(m.ny, m.ny, 0, 1);
  if (m.dim == 2) {
    wall(2 * m.ny, m.nx, 1, 0);
    wall(2 * m.ny + m.nx, m.nx, 1, 1);
  }
  ih.lds_bytes = iugkp::window_words(d.WX, d.WY, d.has_null, d.lds_walls, m.n_b) * sizeof(long long);
}

// Persistent population: N particles per cell in equilibrium (the cell's
// energy E V split over them) and N per wall face waiting to carry the
// face's first emission; shares, remainders, counts and tallies.
int setup_persistent(InstHost &ih, const std::vector<double> &T0, const std::vector<long long> &gw,
                     hipStream_t s)
{
  Inst &d = ih.d;
  const Mesh &m = d.m;
  const int nc = m.n_cells, nb = m.n_b;
  const uint64_t n = static_cast<uint64_t>(d.N) * static_cast<uint64_t>(nc + nb);
  if (n > 0xFFFFFFFEull) return fail(IUGKP_E_INVALID_ARG, "persistent population above 2^32 - 2");
  d.persist = 1;
  d.n_part = static_cast<unsigned int>(n);
  d.n_npart = cdiv(static_cast<long long>(n), kPersistBlock * iugkp::kPersistPer);
  d.n_gpart = cdiv(nc, iugkp::kTree) + cdiv(nb, iugkp::kTree) + 1;
#define PALLOC(ptr, k) \
  if (ih.alloc(&(ptr), (k)) != hipSuccess) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
  PALLOC(d.px, n);
  PALLOC(d.py, n);
  PALLOC(d.psx, n);
  PALLOC(d.psy, n);
  PALLOC(d.pq, n);
  PALLOC(d.plk, n);
  PALLOC(d.Nrc, nc);
  PALLOC(d.Nb, nb);
  PALLOC(d.wc, nc);
  PALLOC(d.rc, nc);
  PALLOC(d.wb, nb);
  PALLOC(d.rb, nb);
  PALLOC(d.npart, d.n_npart);
  PALLOC(d.pstart, nc);
  PALLOC(d.pein, nb);
  long long *dgw = nullptr, *dg0 = nullptr;
  PALLOC(dgw, nb);
  PALLOC(dg0, nc);
#undef PALLOC
  // the y faces of face-tallied moves by row stripes (2D, free paths of at
  // least kStripeMinCells cells or march 2; march 1 keeps them as global
  // atomics in the move): as many rows per workgroup as its LDS holds, about
  // two workgroups per CU
  const bool lam_stripes = d.lam_min >= kStripeMinCells * std::min(m.dx, m.dy);
  if (m.dim == 2 && (ih.opt.march >= 2 || (ih.opt.march == 0 && lam_stripes)) &&
      m.ny <= 0xfffe && m.nx <= 0xffff) {
    int dev = 0, n_cu = 0, lds_max = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // (less the static LDS: the list of paths and their pieces, 16 KB)
    int R = static_cast<int>((lds_max / 8 - 64 - iugkp::kPersistScan) / m.nx) - 1;   // nface <= R + 1
    if (R >= 1) {
      R = std::min(R, m.ny);
      const int S = cdiv(m.ny, R);
      R = cdiv(m.ny, S);
      const size_t lds = static_cast<size_t>(R + 1) * m.nx * sizeof(long long);
      int per_cu = 0;
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void *>(iugkp::persist_faces_kernel<kPersistFacesBlock>),
          kPersistFacesBlock, lds));
      if (per_cu >= 1 && ih.alloc(&d.pf, n) == hipSuccess && ih.alloc(&d.pkey, n) == hipSuccess) {
        ih.pst_R = R;
        ih.pst_S = S;
        ih.pst_C = std::max(1, (2 * per_cu * n_cu) / S);
        ih.pst_lds = lds;
      } else {
        (void)hipGetLastError();   // (without the memory: global atomics)
      }
    }
  }
  d.Gw = dgw;
  // the cells' energies E V in fixed point, the walls' first shares
  std::vector<long long> g0(nc), wb(nb), rb(nb);
  unsigned long long acc = 0;
  bool over = false;
  for (int c = 0; c < nc; ++c) {
    const double e0 = T0.empty() ? d.cv * (d.t_ref - d.t_ref) : d.cv * (T0[c] - d.t_ref);
    const double v = std::ldexp(e0 * d.V, d.F);
    if (!(std::fabs(v) <= 4611686018427387904.0)) return fail(IUGKP_E_FIXED_OVERFLOW, "initial energy exceeds the fixed-point range");
    g0[c] = static_cast<long long>(std::rint(v));
    acc += static_cast<unsigned long long>(g0[c] < 0 ? -g0[c] : g0[c]);
    if (acc > (1ull << 62)) over = true;
  }
  for (int b = 0; b < nb; ++b) {
    const long long nn = static_cast<long long>(d.N);
    long long w = gw[b] / nn;
    if (gw[b] % nn != 0 && gw[b] < 0) w -= 1;
    wb[b] = w;
    rb[b] = gw[b] - w * nn;
    acc += static_cast<unsigned long long>(w < 0 ? -w : w) * d.N + static_cast<unsigned long long>(rb[b]);
    if (acc > (1ull << 62)) over = true;
  }
  if (over) return fail(IUGKP_E_FIXED_OVERFLOW, "initial population exceeds the fixed-point budget");
  HIP_TRY(hipMemcpyAsync(dgw, gw.data(), nb * sizeof(long long), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dg0, g0.data(), nc * sizeof(long long), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.wb, wb.data(), nb * sizeof(long long), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.rb, rb.data(), nb * sizeof(long long), hipMemcpyHostToDevice, s));
  // the first iteration starts every cell's particles and all N per wall face
  std::vector<long long> ein(nb);
  for (int b = 0; b < nb; ++b)
    ein[b] = static_cast<long long>(static_cast<unsigned long long>(wb[b]) * d.N);
  HIP_TRY(hipMemcpyAsync(d.pein, ein.data(), nb * sizeof(long long), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d.pstart, g0.data(), nc * sizeof(long long), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(d.wc, 0, nc * sizeof(long long), s));
  HIP_TRY(hipMemsetAsync(d.rc, 0, nc * sizeof(long long), s));
  HIP_TRY(hipMemsetAsync(d.Nrc, 0, nc * sizeof(uint32_t), s));
  HIP_TRY(hipMemsetAsync(d.Nb, 0, nb * sizeof(uint32_t), s));
  HIP_TRY(hipMemsetAsync(d.D, 0, nc * sizeof(long long), s));
  HIP_TRY(hipMemsetAsync(d.W, 0, nc * sizeof(long long), s));
  HIP_TRY(hipMemsetAsync(d.Phix, 0, m.n_fx * sizeof(long long), s));
  if (m.n_fy) HIP_TRY(hipMemsetAsync(d.Phiy, 0, m.n_fy * sizeof(long long), s));
  HIP_TRY(hipMemsetAsync(d.B, 0, nb * sizeof(long long), s));
  // the descriptor the creation kernel reads (uploaded again by the caller)
  Inst *dinst = nullptr;
  if (ih.alloc(&dinst, 1) != hipSuccess) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
  HIP_TRY(hipMemcpyAsync(dinst, &d, sizeof(Inst), hipMemcpyHostToDevice, s));
  iugkp::persist_init_kernel<<<cdiv(static_cast<long long>(n), 256), 256, 0, s>>>(dinst, dg0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

// The multigrid hierarchy of the Newton operator: level sizes (halved, rounded
// up, down to one cell), the coarse operators built on the device, the
// vectors of the levels spread over the group, the LDS layout of the small
// levels, and the group's launch shape.
int setup_mg(InstHost &ih, const iugkp_options *o, hipStream_t s, bool single)
{
  const Mesh &m = ih.d.m;
  const int has_y = (m.dim == 2) ? 1 : 0;
  std::vector<iugkp::MGLevel> lv;
  for (int nx = m.nx, ny = m.ny;;) {
    iugkp::MGLevel l{};
    l.nx = nx;
    l.ny = ny;
    l.n = nx * ny;
    l.has_y = has_y;
    lv.push_back(l);
    if (nx == 1 && ny == 1) break;
    nx = (nx + 1) / 2;
    ny = (ny + 1) / 2;
  }
  const int L = static_cast<int>(lv.size());
  if (L > iugkp::kMgLevelsMax) return fail(IUGKP_E_INVALID_ARG, "mesh too large for the multigrid");
  // the levels from Lg on live in every workgroup's LDS (three vectors and
  // the five row coefficients per cell): from the first of at most
  // kMgLocalMax cells, or a later one when LDS is short
  int dev = 0, n_cu = 0, lds_max = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const size_t lds_budget = static_cast<size_t>(lds_max) - 12 * 1024;  // static: reductions, level table
  auto local_bytes = [&](int from) {
    size_t w = 0;
    for (int k = from; k < L; ++k) w += 6 * static_cast<size_t>(lv[k].n);
    return w * sizeof(double);
  };
  int Lg = 0;
  while (Lg < L && lv[Lg].n > iugkp::kMgLocalMax) ++Lg;
  while (Lg < L - 1 && local_bytes(Lg) > lds_budget) ++Lg;
  if (local_bytes(Lg) > lds_budget) return fail(IUGKP_E_DEVICE, "no LDS for the multigrid");
  const int waves = o->cg_waves != 0 ? std::abs(o->cg_waves) : kCgWavesDefault;
  const int nb0 = cdiv(lv[0].n, iugkp::kTree);
  const int G = std::max(1, std::min(std::min(cdiv(nb0, waves), kCgGridMax), n_cu));
  // The banded form (2D meshes, or no grid level): LDS for the level Lg
  // result kept through a band phase, then the LDS levels or the staging of
  // a band window, whichever is larger.  Its windows for a group of Gp
  // members (one window per phase when the budget allows; a batch instance's
  // group changes from replay to replay, so it takes the largest stage), and
  // the smallest stage with one row (one block) per window.
  // (the LDS levels' rows, 3 doubles per cell, stay for the whole solve; their
  // vectors, 3 per cell, share the stage with the band windows)
  const long long levels_words = static_cast<long long>(local_bytes(Lg) / sizeof(double)) / 2;
  const long long rows_words = levels_words;
  auto band_need = [&](int Gp) {
    long long w = levels_words;
    for (int k = 0; k < Lg; ++k) {
      const long long nxk = lv[k].nx;
      w = std::max(w, (6ll * cdiv(lv[k + 1].ny, Gp) + 10) * nxk);
      if (k >= 1) w = std::max(w, (3ll * cdiv(lv[k].ny, Gp) + 8) * nxk);
    }
    if (Lg >= 1) {
      const long long nx0 = lv[0].nx;
      const long long rmax = 2 + (static_cast<long long>(iugkp::kTree) * cdiv(nb0, Gp) - 1 + nx0 - 1) / nx0;
      w = std::max(w, (3 * rmax + 14) * nx0);
    }
    return w;
  };
  const long long e_words = (Lg >= 1) ? lv[Lg].n : 0;
  const long long band_budget =
      static_cast<long long>(lds_budget / sizeof(double)) - e_words - rows_words;
  const bool band = (Lg == 0 || has_y) && 64 * waves <= iugkp::kMgBandThreads &&
                    band_need(1 << 20) <= band_budget;
  const int stage0 = band ? static_cast<int>(e_words + rows_words) : 0;
  const long long stage_n =
      band ? std::min(band_budget, band_need(single ? G : 1)) : 0;
#define ALLOC(ptr, cnt) \
  do { if (ih.alloc(&(ptr), (cnt)) != hipSuccess) return fail(IUGKP_E_NOMEM, "hipMalloc failed"); } while (0)
  lv[0].gx = ih.gx;
  lv[0].gy = ih.gy;
  lv[0].diag = ih.diag;
  for (int k = 1; k < L; ++k) {
    double *gx = nullptr, *gy = nullptr, *dg = nullptr;
    ALLOC(gx, static_cast<size_t>(lv[k].ny) * (lv[k].nx + 1));
    if (has_y) ALLOC(gy, static_cast<size_t>(lv[k].ny + 1) * lv[k].nx);
    ALLOC(dg, lv[k].n);
    lv[k].gx = gx;
    lv[k].gy = has_y ? gy : ih.gy;      // 1D: a valid array that is never read from
    lv[k].diag = dg;
  }
  ALLOC(lv[0].b, lv[0].n);                 // r, read by the whole group
  if (band) {
    ALLOC(ih.mg_r2, lv[0].n);
    ALLOC(ih.mg_s2, lv[0].n);
    if (Lg == 0) ALLOC(lv[0].e, lv[0].n);  // u, read by its owner in the next update
  }
  for (int k = 0; k < Lg; ++k) {
    if (k > 0) ALLOC(lv[k].b, lv[k].n);
    ALLOC(lv[k].xa, lv[k].n);
    ALLOC(lv[k].xb, lv[k].n);
    ALLOC(lv[k].xd, lv[k].n);
    ALLOC(lv[k].e, lv[k].n);
  }
  if (Lg > 0) ALLOC(lv[Lg].b, lv[Lg].n);
  // LDS offsets: banded, [E][rows of every LDS level][vectors | staging];
  // otherwise each level's vectors and rows together
  int off = stage0, roff = static_cast<int>(e_words);
  for (int k = Lg; k < L; ++k) {
    lv[k].lb = off;
    lv[k].lx = off + lv[k].n;
    lv[k].lt = off + 2 * lv[k].n;
    off += 3 * lv[k].n;
    if (band) {
      lv[k].lc = roff;
      roff += 3 * lv[k].n;
    } else {
      lv[k].lc = off;
      off += 3 * lv[k].n;
    }
  }
  for (int k = 0; k + 1 < L; ++k) {
    const int nf = std::max(lv[k + 1].ny * (lv[k + 1].nx + 1), (lv[k + 1].ny + 1) * lv[k + 1].nx);
    iugkp::mg_coarsen_faces_kernel<<<cdiv(nf, 256), 256, 0, s>>>(
        lv[k], lv[k + 1], has_y, const_cast<double *>(lv[k + 1].gx),
        const_cast<double *>(lv[k + 1].gy));
    iugkp::mg_coarsen_diag_kernel<<<cdiv(lv[k + 1].n, 256), 256, 0, s>>>(
        lv[k + 1], has_y, const_cast<double *>(lv[k + 1].diag));
  }
  HIP_TRY(hipGetLastError());
  ALLOC(ih.mg_lv, L);
#undef ALLOC
  HIP_TRY(hipMemcpyAsync(ih.mg_lv, lv.data(), L * sizeof(iugkp::MGLevel), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  const size_t lds = band ? static_cast<size_t>(stage0 + stage_n) * sizeof(double)
                          : static_cast<size_t>(off) * sizeof(double);
  int per_cu = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu,
      band ? reinterpret_cast<const void *>(iugkp::mgcg_band_kernel)
           : reinterpret_cast<const void *>(iugkp::mgcg_kernel),
      64 * waves, lds));
  if (per_cu < 1 || G > per_cu * n_cu)
    return fail(IUGKP_E_DEVICE, "multigrid CG workgroups cannot all be resident");
  ih.mg_L = L;
  ih.mg_Lg = Lg;
  ih.mg_band = band ? 1 : 0;
  ih.mg_stage0 = stage0;
  ih.mg_stage_n = static_cast<int>(stage_n);
  ih.cg_cus = static_cast<double>(G) / per_cu;
  ih.mg_grid = G;
  ih.mg_threads = 64 * waves;
  ih.mg_lds = lds;
  return IUGKP_OK;
}

// Validate, allocate and initialise one instance on `s`.  multi_cg: also lay
// out the multi-workgroup CG used by single solves.
// Row stripes for the face-tallied iterations of one instance (a single solve,
// or one frequency band): rows per workgroup, stripes and chunks, and for the
// analog particle step the records and their bins (ih.stripe_*, ih.rec);
// stripe_R stays 0 where they do not fit (tiles are used).  pref: the
// planner's choice for the form search.
int plan_stripes(InstHost &ih, hipStream_t s, bool ev, bool pref)
{
  Inst &d = ih.d;
  const Mesh &m = d.m;
  // row stripes: as many rows per workgroup as its LDS holds (y faces and
  // the walls; the expected-value kernel also D, and W with null
  // collisions), about two workgroups per CU
  int dev = 0, n_cu = 0, lds_max = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  // (less the static LDS: the march's segment table, 8.3 KB, and for flights
  // without null collisions the pieces' lists, 8.2 KB more)
  const bool pieces = !ev && !d.has_null;
  const long long words = lds_max / 8 - (pieces ? 2200 : 1100);
  const long long per_row = static_cast<long long>(m.nx) * (ev ? (d.has_null ? 3 : 2) : 1);
  const long long fixed = m.nx + (d.lds_walls ? m.n_b : 0);
  int R = static_cast<int>((words - fixed) / per_row);
  if (R >= kStripeMinRows || (R >= 1 && R >= m.ny)) {
    R = std::min(R, m.ny);
    const int S = cdiv(m.ny, R);
    R = cdiv(m.ny, S);
    const size_t lds = static_cast<size_t>(fixed + per_row * R) * sizeof(long long);
    int per_cu = 0;
    const void *kern =
        ev ? reinterpret_cast<const void *>(iugkp::march_stripes_ev_kernel<kStripeBlock>)
        : pieces ? reinterpret_cast<const void *>(iugkp::march_stripes_pieces_kernel<kStripeBlock>)
                 : reinterpret_cast<const void *>(iugkp::march_stripes_kernel<kStripeBlock>);
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kStripeBlock, lds));
    // (the analog kernel reads every particle's first segment from a
    // 64-byte record (80 with null collisions) and a 4-byte row range per
    // particle; without the memory, or beyond 65534 rows or 65535
    // columns, tiles are used)
    // The records are binned by start stripe and pre-pass block (sub-bin k
    // of stripe t: the particles that start in t among those of pre-pass
    // blocks k, k + K, ...; counted here exactly): beyond kStripeBinMax / 2
    // stripes or 2^32 particles, tiles are used.
    bool recs = true;
    const size_t np = static_cast<size_t>(m.n_emit) * static_cast<size_t>(d.N);
    if (!ev && (m.ny > 0xfffe || m.nx > 0xffff || 2 * S > iugkp::kStripeBinMax ||
                np > 0xffffffffull))
      recs = false;   // (16-bit rows and columns, 32-bit slots)
    else if (!ev) {
      const size_t rb = d.has_null ? sizeof(iugkp::PRecN) : sizeof(iugkp::PRec);
      const int K = std::max(1, std::min(32, iugkp::kStripeSegMax / (S + 1)));
      const long long per_block = static_cast<long long>(iugkp::kPresampleBlock) * iugkp::kPresamplePer;
      const long long nblk = (static_cast<long long>(np) + per_block - 1) / per_block;
      const long long ne = m.n_emit, nc = m.n_cells;
      // emitters of stripe t in [e0, e1): its rows' cells and left and right
      // wall faces, the bottom wall (first stripe), the top wall (last)
      auto in_stripe = [&](int t, long long e0, long long e1) {
        const long long y0 = static_cast<long long>(t) * R, y1 = std::min<long long>(m.ny, y0 + R);
        auto ov = [&](long long a, long long b) {
          return std::max(0ll, std::min(b, e1) - std::max(a, e0));
        };
        long long c = ov(y0 * m.nx, y1 * m.nx) + ov(nc + y0, nc + y1) + ov(nc + m.ny + y0, nc + m.ny + y1);
        if (t == 0) c += ov(nc + 2ll * m.ny, nc + 2ll * m.ny + m.nx);
        if (t == S - 1) c += ov(nc + 2ll * m.ny + m.nx, nc + 2ll * m.ny + 2ll * m.nx);
        return c;
      };
      std::vector<unsigned long long> cap(static_cast<size_t>(S) * K, 0);
      for (long long b = 0; b < nblk; ++b) {
        const long long p0 = b * per_block, p1 = std::min<long long>(p0 + per_block, np);
        for (long long p = p0; p < p1;) {
          const long long kk = p / ne, e0 = p - kk * ne;
          const long long e1 = std::min(ne, e0 + (p1 - p));
          for (int t = 0; t < S; ++t) cap[static_cast<size_t>(t) * K + (b % K)] += in_stripe(t, e0, e1);
          p += e1 - e0;
        }
      }
      std::vector<uint32_t> base(static_cast<size_t>(S) * K + 1, 0);
      for (size_t i = 0; i < cap.size(); ++i) base[i + 1] = base[i] + static_cast<uint32_t>(cap[i]);
      unsigned char *r = nullptr;
      uint32_t *db = nullptr;
      recs = ih.alloc(&r, np * rb) == hipSuccess && ih.alloc(&ih.rec.key, np) == hipSuccess &&
             ih.alloc(&ih.rec.cnt, 2 * cap.size()) == hipSuccess &&
             ih.alloc(&db, base.size()) == hipSuccess;
      if (recs && base.back() != np) return fail(IUGKP_E_DEVICE, "stripe bins do not cover the particles");
      if (recs) HIP_TRY(hipMemcpyAsync(db, base.data(), base.size() * sizeof(uint32_t),
                                       hipMemcpyHostToDevice, s));
      ih.rec.r = r;
      ih.rec.base = db;
      ih.rec.R = R;
      ih.rec.S = S;
      ih.rec.K = K;
      if (!recs) (void)hipGetLastError();
    }
    if (per_cu >= 1 && recs) {
      ih.stripe_R = R;
      ih.stripe_S = S;
      ih.stripe_C = std::max(1, (2 * per_cu * n_cu) / S);   // whole rounds of resident groups
      ih.stripe_lds = lds;
      ih.stripe_pref = pref ? 1 : 0;
    }
  }
  return IUGKP_OK;
}

int setup_instance(const iugkp_problem *p, const iugkp_options *o, hipStream_t s, bool multi_cg,
                   InstHost &ih)
{
  int rc = check_problem(p);
  if (rc) return rc;
  rc = check_options(o);
  if (rc) return rc;
  if (p->n_bands > 1)
    return fail(IUGKP_E_INVALID_ARG, "frequency-band problems are single solves (iugkp_create)");
  const int nc = p->nx * p->ny;
  const int nb = 2 * p->ny + (p->dim == 2 ? 2 * p->nx : 0);
  std::vector<double> tau, wall, T0, src;
  if ((rc = fetch_host(p->tau, nc, p->mem_kind, tau))) return rc;
  if (p->source && (rc = fetch_host(p->source, nc, p->mem_kind, src))) return rc;
  if ((rc = fetch_host(p->wall_T, nb, p->mem_kind, wall))) return rc;
  if (p->T_init && (rc = fetch_host(p->T_init, nc, p->mem_kind, T0))) return rc;
  double tmin = INFINITY, tmax = 0.0;
  for (double t : tau) {
    if (!(t > 0.0) || !std::isfinite(t)) return fail(IUGKP_E_INVALID_ARG, "tau must be > 0 and finite");
    tmin = std::min(tmin, t);
    tmax = std::max(tmax, t);
  }
  if (tmax > 1e6 * tmin) return fail(IUGKP_E_INVALID_ARG, "tau_max / tau_min exceeds 1e6");
  for (double t : wall)
    if (!std::isfinite(t)) return fail(IUGKP_E_INVALID_ARG, "wall_T must be finite");
  for (double t : T0)
    if (!std::isfinite(t)) return fail(IUGKP_E_INVALID_ARG, "T_init must be finite");
  for (double v : src)
    if (!std::isfinite(v)) return fail(IUGKP_E_INVALID_ARG, "source must be finite");
  const int ne = nc + nb;
  uint64_t N = o->particles_per_iter / static_cast<uint64_t>(ne);
  if (N < 1) N = 1;
  if (N * static_cast<uint64_t>(ne) > 0xFFFFFFFFull)
    return fail(IUGKP_E_INVALID_ARG, "particles per iteration must stay below 2^32");

  ih.opt = *o;
  ih.mem_kind = p->mem_kind;
  Inst &d = ih.d;
  Mesh &m = d.m;
  m.dim = p->dim;
  m.nx = p->nx;
  m.ny = p->ny;
  m.n_cells = nc;
  m.n_b = nb;
  m.n_emit = ne;
  m.n_fx = p->ny * (p->nx + 1);
  m.n_fy = (p->dim == 2) ? (p->ny + 1) * p->nx : 0;
  m.dx = p->dx;
  m.dy = p->dy;
  d.t_ref = p->t_ref;
  d.cv = p->cv;
  d.tau_min = tmin;
  d.lam_min = p->vg * tmin;
  d.V = p->dx * p->dy;
  d.N = static_cast<uint32_t>(N);
  d.key0 = static_cast<uint32_t>(o->seed);
  d.key1 = static_cast<uint32_t>(o->seed >> 32);
  d.crn = (o->rng_mode == IUGKP_RNG_CRN);
  d.epoch = o->rng_epoch;
  d.has_null = (tmax != tmin);
  d.newton = o->newton ? 1 : 0;
  d.estimator = o->estimator;
  d.faces_each = (o->tally_faces == IUGKP_FACES_EVERY);
  d.faces_out = (o->tally_faces != IUGKP_FACES_OFF);
  d.final_iter = (o->tally_faces == IUGKP_FACES_FINAL);
  d.avg_iters = o->avg_iters;
  d.max_iters = o->max_iters;
  d.res_tol = o->res_tol;
  d.tol2 = o->cg_tol * o->cg_tol;
  d.cg_max = o->cg_max_iters;
  d.F = scale_exponent(p, tmin, wall, T0, src);
  plan_tiles(ih, kTileX, (multi_cg && d.has_null) ? kWindowHaloNull : kWindowHalo);

#define ALLOC(ptr, n) \
  if (ih.alloc(&(ptr), (n)) != hipSuccess) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
  const int nbe = cdiv(ne, iugkp::kTree);
  double *ratio = nullptr;
  ALLOC(ih.tau, nc);
  ALLOC(ratio, nc);
  d.ratio = ratio;
  ALLOC(d.E, nc);
  ALLOC(d.E_half, nc);
  ALLOC(d.part, nbe);
  ALLOC(d.G, ne);
  ALLOC(d.base, ne);
  ALLOC(d.rem, ne);
  ALLOC(d.D, nc);
  ALLOC(d.W, nc);
  ALLOC(d.Phix, m.n_fx);
  ALLOC(d.Phiy, m.n_fy);
  ALLOC(d.dB, (p->ny + 2) * p->nx);
  ALLOC(d.B, nb);
  ALLOC(d.acc_E, nc);
  ALLOC(d.acc_x, m.n_fx);
  ALLOC(d.acc_y, m.n_fy);
  ALLOC(ih.out_T, nc);
  ALLOC(ih.out_qx, m.n_fx);
  ALLOC(ih.out_qy, m.n_fy);
  ALLOC(d.sc, 1);
  ALLOC(d.gpart, std::max(nbe, cdiv(nc, iugkp::kTree) + cdiv(nb, iugkp::kTree) + 1));
  if (o->newton) {
    const int nbt = cdiv(nc, iugkp::kTree);
    ALLOC(d.rhs, nc);
    ALLOC(ih.Dx, nc);
    ALLOC(ih.Dy, nc);
    ALLOC(ih.gx, m.n_fx);
    ALLOC(ih.gy, m.n_fy);
    ALLOC(ih.diag, nc);
    d.gx = ih.gx;
    d.gy = ih.gy;
    d.diag = ih.diag;
    ALLOC(d.cg_x, nc);
    ALLOC(d.cg_r, nc);
    ALLOC(d.cg_w, nc);
    ALLOC(d.cg_p, nc);
    ALLOC(d.cg_s, nc);
    ALLOC(ih.cg_pub, 6 * static_cast<size_t>(nc));
    ALLOC(ih.cg_mpart, 4 * static_cast<size_t>(nbt));
    ALLOC(ih.cg_barrier, 2);
    d.cg_pub = ih.cg_pub;
    d.cg_mpart = ih.cg_mpart;
    d.cg_barrier = ih.cg_barrier;
  }
#undef ALLOC
  HIP_TRY(hipMemcpyAsync(ih.tau, tau.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
  double *dT0 = nullptr;
  if (!T0.empty()) {
    if (ih.alloc(&dT0, nc) != hipSuccess) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
    HIP_TRY(hipMemcpyAsync(dT0, T0.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
  }
  iugkp::init_cells_kernel<<<cdiv(nc, 256), 256, 0, s>>>(nc, d.cv, d.t_ref, d.tau_min, dT0,
                                                          ih.tau, d.E, ratio);
  // wall emission E_w lambda_min A / 4 (cosine-law black walls), computed once
  std::vector<long long> gw(nb);
  d.wall_budget = 0;
  for (int b = 0; b < nb; ++b) {
    const double A = (b < 2 * p->ny) ? p->dy : p->dx;
    const double ew = p->cv * (wall[b] - p->t_ref);
    const double v = std::ldexp((ew * (d.lam_min * A)) / 4.0, d.F);
    if (!(std::fabs(v) <= 4611686018427387904.0))
      return fail(IUGKP_E_FIXED_OVERFLOW, "wall emission exceeds the fixed-point range");
    gw[b] = static_cast<long long>(std::rint(v));
    const unsigned long long a = static_cast<unsigned long long>(gw[b] < 0 ? -gw[b] : gw[b]);
    d.wall_budget = std::min(d.wall_budget + a, iugkp::kBudgetCap);
  }
  HIP_TRY(hipMemcpyAsync(d.G + nc, gw.data(), nb * sizeof(long long), hipMemcpyHostToDevice, s));
  // source emission S V tau_min per iteration
  d.Gs = nullptr;
  if (!src.empty()) {
    std::vector<long long> gs(nc);
    for (int c = 0; c < nc; ++c) {
      const double v = std::ldexp((src[c] * d.V) * d.tau_min, d.F);
      if (!(std::fabs(v) <= 4611686018427387904.0))
        return fail(IUGKP_E_FIXED_OVERFLOW, "source emission exceeds the fixed-point range");
      gs[c] = static_cast<long long>(std::rint(v));
    }
    long long *dgs = nullptr;
    if (ih.alloc(&dgs, nc) != hipSuccess) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
    HIP_TRY(hipMemcpyAsync(dgs, gs.data(), nc * sizeof(long long), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    d.Gs = dgs;
  }
  int *dflag = nullptr;
  if (ih.alloc(&dflag, 1) != hipSuccess) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
  HIP_TRY(hipMemsetAsync(dflag, 0, sizeof(int), s));
  iugkp::emission_from_E_kernel<<<cdiv(nc, 256), 256, 0, s>>>(nc, d.F, d.V, d.E, ratio, d.Gs, d.G,
                                                              dflag);
  if (o->newton) {
    std::vector<double> dxv(nc), dyv(nc);
    auto fill = [&](const double *given, double delta, std::vector<double> &out) -> int {
      if (given) return fetch_host(given, nc, p->mem_kind, out);
      std::map<double, double> cache;
      for (int c = 0; c < nc; ++c) {
        auto it = cache.find(tau[c]);
        if (it == cache.end()) it = cache.emplace(tau[c], iugkp::d_eff(p->vg * tau[c], delta)).first;
        out[c] = it->second;
      }
      return IUGKP_OK;
    };
    if ((rc = fill(p->diff_x, p->dx, dxv))) return rc;
    if (p->dim == 2) {
      if ((rc = fill(p->diff_y, p->dy, dyv))) return rc;
    } else {
      dyv = dxv;
    }
    for (int c = 0; c < nc; ++c)
      if (!(dxv[c] > 0.0) || !std::isfinite(dxv[c]) || !(dyv[c] > 0.0) || !std::isfinite(dyv[c]))
        return fail(IUGKP_E_INVALID_ARG, "Newton diffusion coefficients must be > 0");
    HIP_TRY(hipMemcpyAsync(ih.Dx, dxv.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ih.Dy, dyv.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int nf = std::max(m.n_fx, m.n_fy);
    iugkp::newton_operator_kernel<<<cdiv(nf, 256), 256, 0, s>>>(m, p->vg, ih.tau, ih.Dx, ih.Dy,
                                                                 ih.gx, ih.gy, ih.diag);
    iugkp::newton_diag_kernel<<<cdiv(nc, 256), 256, 0, s>>>(m, ih.gx, ih.gy, ih.diag);
    if (multi_cg) {
      CgPlan cp;
      if ((rc = plan_cg(m, o->cg_waves, cp))) return rc;
      ih.cg_grid = cp.grid;
      ih.cg_tb = cp.tb;
      ih.cg_reg = cp.reg;
      ih.cg_threads = cp.threads;
      ih.cg_lds = cp.lds;
      ih.cg_cus = static_cast<double>(cp.grid) / cp.per_cu;
      if (o->cg_precond == IUGKP_PRECOND_MG && (rc = setup_mg(ih, o, s, true))) return rc;
    } else if (o->cg_precond == IUGKP_PRECOND_MG) {
      // batched: the hierarchy only; one workgroup runs the instance's solve
      if ((rc = setup_mg(ih, o, s, false))) return rc;
    }
  }
  // (expected-value rays: only on request, march == 2; every stripe follows a
  // ray from its start, and that re-walk costs more than the tile kernel's
  // global atomics on the 256^2 cavity)
  // (an automatic march with the default block size also sets stripes up for
  // the particle-step form search of the handle)
  const bool ev = (o->estimator == IUGKP_EST_EXPECTED);
  const bool lam_stripes = d.lam_min >= kStripeMinCells * std::min(p->dx, p->dy);
  if (multi_cg && p->dim == 2 && o->scheme == IUGKP_SCHEME_EMITTERS &&
      ((ev && o->march >= 2) ||
       (!ev && o->tally_faces != IUGKP_FACES_OFF &&
        (o->march >= 2 || (o->march == 0 && (lam_stripes || o->block_size == 0)))))) {
    if ((rc = plan_stripes(ih, s, ev, o->march >= 2 || lam_stripes))) return rc;
    if (o->march >= 2 && ih.stripe_R == 0)
      return fail(IUGKP_E_INVALID_ARG, "row stripes do not fit this mesh");
  }
  if (o->scheme == IUGKP_SCHEME_PERSISTENT) {
    if (!multi_cg) return fail(IUGKP_E_INVALID_ARG, "the persistent scheme is for single solves");
    if ((rc = setup_persistent(ih, T0, gw, s))) return rc;
  }
  std::vector<long long> g(ne);
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(g.data(), d.G, ne * sizeof(long long), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  DevScalars sc0{};
  sc0.res_p1 = sc0.res_p2 = HUGE_VAL;
  // iteration control: nothing to iterate -> straight to the output iterations
  if (o->max_iters <= 0) {
    if (o->avg_iters > 0) {
      sc0.state = 1;
      sc0.out_left = o->avg_iters;
      sc0.faces_now = d.faces_out;
    } else if (d.final_iter) {
      sc0.state = 1;
      sc0.out_left = 1;
      sc0.faces_now = 1;
    } else {
      sc0.state = 2;
    }
  } else {
    sc0.faces_now = d.faces_each;
  }
  HIP_TRY(hipMemcpyAsync(d.sc, &sc0, sizeof(DevScalars), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  unsigned long long acc = 0;
  for (long long v : g) {
    const unsigned long long a = static_cast<unsigned long long>(v < 0 ? -v : v);
    acc += a;
    if (a > (1ull << 62) || acc > (1ull << 62)) hflag |= 2;
  }
  if (hflag & 2) return fail(IUGKP_E_FIXED_OVERFLOW, "initial emission exceeds the fixed-point budget");
  return IUGKP_OK;
}

// ---------------------------------------------------------------------------
// Frequency bands.  Band k is an instance of its own (tallies, emission, free
// path v_k tau*_k, acceptance tau*_k / tau_k(c), Philox emitter offset
// k (n_cells + n_b)) that shares the mesh, N, the scale F and the iteration
// scalars with band 0; band 0 also owns the energy density, the residual
// partials and the band table of the coupling kernel.
// ---------------------------------------------------------------------------
struct BandsHost {
  int K = 1;
  double Ctot = 0.0;
  iugkp::BandDev *d_bands = nullptr;
  long long **d_phix = nullptr, **d_phiy = nullptr;
  double *srcV = nullptr;        // S V per cell, or null
};

double to_fixed_host(double v, int F, int *ok)
{
  const double x = std::ldexp(v, F);
  if (!(std::fabs(x) <= 4611686018427387904.0)) {
    *ok = 0;
    return 0.0;
  }
  return std::rint(x);
}

// band 0 into ih0, bands 1.. into rest
int setup_bands(const iugkp_problem *p, const iugkp_options *o, hipStream_t s, InstHost &ih0,
                std::vector<InstHost> &rest, BandsHost &bh)
{
  int rc = check_problem(p);
  if (rc) return rc;
  rc = check_options(o);
  if (rc) return rc;
  if (o->newton || o->avg_iters != 0 || o->estimator != IUGKP_EST_ANALOG ||
      o->scheme != IUGKP_SCHEME_EMITTERS)
    return fail(IUGKP_E_INVALID_ARG,
                "frequency bands: emitter scheme, analog estimator, no Newton, no averaging");
  const int K = p->n_bands;
  const int nc = p->nx * p->ny;
  const int nb = 2 * p->ny + (p->dim == 2 ? 2 * p->nx : 0);
  const int ne = nc + nb;
  std::vector<double> tau, wall, T0, src, bC, bv;
  if ((rc = fetch_host(p->tau, static_cast<size_t>(K) * nc, p->mem_kind, tau))) return rc;
  if ((rc = fetch_host(p->band_C, K, p->mem_kind, bC))) return rc;
  if ((rc = fetch_host(p->band_vg, K, p->mem_kind, bv))) return rc;
  if (p->source && (rc = fetch_host(p->source, nc, p->mem_kind, src))) return rc;
  if ((rc = fetch_host(p->wall_T, nb, p->mem_kind, wall))) return rc;
  if (p->T_init && (rc = fetch_host(p->T_init, nc, p->mem_kind, T0))) return rc;
  for (int k = 0; k < K; ++k)
    if (!(bC[k] > 0.0) || !std::isfinite(bC[k]) || !(bv[k] > 0.0) || !std::isfinite(bv[k]))
      return fail(IUGKP_E_INVALID_ARG, "band_C and band_vg must be > 0 and finite");
  std::vector<double> ts(K), lam(K);
  std::vector<int> has_null(K);
  for (int k = 0; k < K; ++k) {
    double tmin = INFINITY, tmax = 0.0;
    for (int c = 0; c < nc; ++c) {
      const double t = tau[static_cast<size_t>(k) * nc + c];
      if (!(t > 0.0) || !std::isfinite(t)) return fail(IUGKP_E_INVALID_ARG, "tau must be > 0 and finite");
      tmin = std::min(tmin, t);
      tmax = std::max(tmax, t);
    }
    if (tmax > 1e6 * tmin) return fail(IUGKP_E_INVALID_ARG, "tau_max / tau_min exceeds 1e6 in a band");
    ts[k] = tmin;
    lam[k] = bv[k] * tmin;
    has_null[k] = (tmax != tmin);
  }
  for (double t : wall)
    if (!std::isfinite(t)) return fail(IUGKP_E_INVALID_ARG, "wall_T must be finite");
  for (double t : T0)
    if (!std::isfinite(t)) return fail(IUGKP_E_INVALID_ARG, "T_init must be finite");
  for (double v : src)
    if (!std::isfinite(v)) return fail(IUGKP_E_INVALID_ARG, "source must be finite");
  uint64_t N = o->particles_per_iter / (static_cast<uint64_t>(ne) * static_cast<uint64_t>(K));
  if (N < 1) N = 1;
  if (N * static_cast<uint64_t>(ne) > 0xFFFFFFFFull ||
      static_cast<uint64_t>(K) * static_cast<uint64_t>(ne) > 0xFFFFFFFFull)
    return fail(IUGKP_E_INVALID_ARG, "particles per band iteration and emitters must stay below 2^32");
  const double V = p->dx * p->dy;
  double Ctot = 0.0;
  for (int k = 0; k < K; ++k) Ctot = Ctot + bC[k];
  std::vector<double> den(nc, 0.0);
  for (int c = 0; c < nc; ++c)
    for (int k = 0; k < K; ++k) den[c] = den[c] + bC[k] / tau[static_cast<size_t>(k) * nc + c];
  // fixed-point scale: the gray budget with band sums (cells emit at most
  // C dT V per iteration, walls dT sum_k C_k lambda*_k A / 4), plus the
  // source's energy density S_max times the longest residence time of a band,
  // max_k tau*_k (1 + 3 (L / lambda*_k)^2) (the gray bound per band)
  double dT = 0.0;
  for (double t : wall) dT = std::max(dT, std::fabs(t - p->t_ref));
  for (double t : T0) dT = std::max(dT, std::fabs(t - p->t_ref));
  double lam_sum = 0.0;
  for (int k = 0; k < K; ++k) lam_sum = lam_sum + bC[k] * lam[k];
  const double vol = static_cast<double>(nc) * V;
  const double area = (p->dim == 2) ? ((2.0 * static_cast<double>(p->ny)) * p->dy +
                                       (2.0 * static_cast<double>(p->nx)) * p->dx)
                                    : 2.0;
  double esrc = 0.0;
  if (!src.empty()) {
    double smax = 0.0;
    for (double v : src) smax = std::max(smax, std::fabs(v));
    double L = static_cast<double>(p->nx) * p->dx;
    if (p->dim == 2 && static_cast<double>(p->ny) * p->dy > L) L = static_cast<double>(p->ny) * p->dy;
    double res_hi = 0.0;
    for (int k = 0; k < K; ++k) {
      const double rl = L / lam[k];
      res_hi = std::max(res_hi, ts[k] * (1.0 + 3.0 * (rl * rl)));
    }
    esrc = smax * res_hi;
  }
  const double Bb = 4.0 * ((dT * Ctot + esrc) * vol + (dT * lam_sum * area) / 4.0);
  int F = 62;
  if (Bb > 0.0) {
    int ex = 0;
    const double mant = std::frexp(Bb, &ex);
    F = 62 - ((mant == 0.5) ? ex - 1 : ex);
  }
  // initial state: equilibrium at T_init, absorbed rate (T0 - t_ref) V den (+ S V)
  std::vector<double> E0(nc), R0(nc);
  for (int c = 0; c < nc; ++c) {
    const double t0 = T0.empty() ? p->t_ref : T0[c];
    E0[c] = Ctot * (t0 - p->t_ref);
    double R = ((t0 - p->t_ref) * V) * den[c];
    if (!src.empty()) R = R + src[c] * V;
    R0[c] = R;
  }

  rest.assign(K - 1, InstHost{});
  auto band = [&](int k) -> InstHost & { return k == 0 ? ih0 : rest[k - 1]; };
  int ok = 1;
  unsigned long long acc = 0, wall_acc = 0;
  bool over = false;
  std::vector<iugkp::BandDev> table(K);
  std::vector<long long *> phx(K), phy(K);
  std::vector<double> ratio(nc), share(nc);
  std::vector<long long> g(ne);
#define ALLOC(ih, ptr, n) \
  if ((ih).alloc(&(ptr), (n)) != hipSuccess) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
  for (int k = 0; k < K; ++k) {
    InstHost &ih = band(k);
    ih.opt = *o;
    ih.mem_kind = p->mem_kind;
    Inst &d = ih.d;
    Mesh &m = d.m;
    m.dim = p->dim;
    m.nx = p->nx;
    m.ny = p->ny;
    m.n_cells = nc;
    m.n_b = nb;
    m.n_emit = ne;
    m.n_fx = p->ny * (p->nx + 1);
    m.n_fy = (p->dim == 2) ? (p->ny + 1) * p->nx : 0;
    m.dx = p->dx;
    m.dy = p->dy;
    d.t_ref = p->t_ref;
    d.cv = Ctot;
    d.tau_min = ts[k];
    d.lam_min = lam[k];
    d.V = V;
    d.N = static_cast<uint32_t>(N);
    d.key0 = static_cast<uint32_t>(o->seed);
    d.key1 = static_cast<uint32_t>(o->seed >> 32);
    d.crn = (o->rng_mode == IUGKP_RNG_CRN);
    d.epoch = o->rng_epoch;
    d.has_null = has_null[k];
    d.newton = 0;
    d.faces_each = (o->tally_faces == IUGKP_FACES_EVERY);
    d.faces_out = (o->tally_faces != IUGKP_FACES_OFF);
    d.final_iter = (o->tally_faces == IUGKP_FACES_FINAL);
    d.avg_iters = 0;
    d.max_iters = o->max_iters;
    d.res_tol = o->res_tol;
    d.F = F;
    d.e_off = static_cast<uint32_t>(k) * static_cast<uint32_t>(ne);
    d.n_bands = K;
    d.Gs = nullptr;
    plan_tiles(ih);
    // row stripes for a band's face-tallied iterations when its free paths
    // reach half the domain's height (and 7 cells): a band with shorter ones
    // has long chains of null collisions wherever its relaxation time is
    // above the minimum, which the tile march handles better (march 1 keeps
    // every band on tiles)
    if (p->dim == 2 && o->tally_faces != IUGKP_FACES_OFF && o->march != 1 &&
        o->estimator == IUGKP_EST_ANALOG && lam[k] >= kStripeMinCells * std::min(p->dx, p->dy) &&
        lam[k] >= 0.5 * p->ny * p->dy) {
      const int rc = plan_stripes(ih, s, false, true);
      if (rc) return rc;
    }
    double *dratio = nullptr, *dshare = nullptr;
    ALLOC(ih, dratio, nc);
    ALLOC(ih, dshare, nc);
    d.ratio = dratio;
    ALLOC(ih, d.G, ne);
    ALLOC(ih, d.base, ne);
    ALLOC(ih, d.rem, ne);
    ALLOC(ih, d.D, nc);
    ALLOC(ih, d.W, nc);
    ALLOC(ih, d.Phix, m.n_fx);
    ALLOC(ih, d.Phiy, m.n_fy);
    ALLOC(ih, d.dB, (p->ny + 2) * p->nx);
    ALLOC(ih, d.B, nb);
    if (k == 0) {
      const int nbe = cdiv(ne, iugkp::kTree);
      ALLOC(ih, d.E, nc);
      ALLOC(ih, d.part, nbe);
      ALLOC(ih, d.gpart, nbe);
      ALLOC(ih, d.sc, 1);
      ALLOC(ih, ih.out_T, nc);
      ALLOC(ih, ih.out_qx, m.n_fx);
      ALLOC(ih, ih.out_qy, m.n_fy);
      ALLOC(ih, bh.d_bands, K);
      ALLOC(ih, bh.d_phix, K);
      ALLOC(ih, bh.d_phiy, K);
      if (!src.empty()) ALLOC(ih, bh.srcV, nc);
    } else {
      d.E = ih0.d.E;
      d.part = ih0.d.part;
      d.gpart = ih0.d.gpart;
      d.sc = ih0.d.sc;
    }
    const double *tk = tau.data() + static_cast<size_t>(k) * nc;
    for (int c = 0; c < nc; ++c) {
      ratio[c] = ts[k] / tk[c];
      share[c] = ts[k] * ((bC[k] / tk[c]) / den[c]);
      g[c] = static_cast<long long>(to_fixed_host(share[c] * R0[c], F, &ok));
    }
    for (int b = 0; b < nb; ++b) {
      const double A = (b < 2 * p->ny) ? p->dy : p->dx;
      g[nc + b] = static_cast<long long>(
          to_fixed_host(((bC[k] * (wall[b] - p->t_ref)) * (lam[k] * A)) / 4.0, F, &ok));
      const unsigned long long a = static_cast<unsigned long long>(g[nc + b] < 0 ? -g[nc + b] : g[nc + b]);
      wall_acc = std::min(wall_acc + a, iugkp::kBudgetCap);
    }
    for (long long v : g) {
      const unsigned long long a = static_cast<unsigned long long>(v < 0 ? -v : v);
      acc += a;
      if (a > (1ull << 62) || acc > (1ull << 62)) over = true;
      if (over) acc = 1ull << 62;
    }
    HIP_TRY(hipMemcpyAsync(dratio, ratio.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(dshare, share.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d.G, g.data(), ne * sizeof(long long), hipMemcpyHostToDevice, s));
    // tallies read as zero until the first iteration
    HIP_TRY(hipMemsetAsync(d.D, 0, nc * sizeof(long long), s));
    HIP_TRY(hipMemsetAsync(d.W, 0, nc * sizeof(long long), s));
    HIP_TRY(hipMemsetAsync(d.Phix, 0, m.n_fx * sizeof(long long), s));
    if (m.n_fy) HIP_TRY(hipMemsetAsync(d.Phiy, 0, m.n_fy * sizeof(long long), s));
    HIP_TRY(hipMemsetAsync(d.B, 0, nb * sizeof(long long), s));
    HIP_TRY(hipStreamSynchronize(s));   // the staging vectors are reused by the next band
    table[k] = iugkp::BandDev{ts[k], dshare, d.D, d.W, d.G, d.has_null};
    phx[k] = d.Phix;
    phy[k] = d.Phiy;
  }
#undef ALLOC
  if (!ok || over)
    return fail(IUGKP_E_FIXED_OVERFLOW, "initial emission exceeds the fixed-point budget");
  ih0.d.wall_budget = wall_acc;
  bh.K = K;
  bh.Ctot = Ctot;
  HIP_TRY(hipMemcpyAsync(ih0.d.E, E0.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(bh.d_bands, table.data(), K * sizeof(iugkp::BandDev), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(bh.d_phix, phx.data(), K * sizeof(long long *), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(bh.d_phiy, phy.data(), K * sizeof(long long *), hipMemcpyHostToDevice, s));
  std::vector<double> sv;
  if (!src.empty()) {
    sv.resize(nc);
    for (int c = 0; c < nc; ++c) sv[c] = src[c] * V;
    HIP_TRY(hipMemcpyAsync(bh.srcV, sv.data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
  }
  DevScalars sc0{};
  sc0.res_p1 = sc0.res_p2 = HUGE_VAL;
  if (o->max_iters <= 0) {
    if (ih0.d.final_iter) {
      sc0.state = 1;
      sc0.out_left = 1;
      sc0.faces_now = 1;
    } else {
      sc0.state = 2;
    }
  } else {
    sc0.faces_now = ih0.d.faces_each;
  }
  HIP_TRY(hipMemcpyAsync(ih0.d.sc, &sc0, sizeof(DevScalars), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 1; k < K; ++k) rest[k - 1].d.wall_budget = wall_acc;
  return IUGKP_OK;
}

template <bool EV>
void launch_march_as(const Inst *d_insts, const TileDesc *d_tiles, int n_tiles, size_t lds,
                     int block, int faces_mode, int batch, unsigned long long *clk, hipStream_t s)
{
  switch (block) {
    case 64: iugkp::march_kernel<64, EV><<<n_tiles, 64, lds, s>>>(d_insts, d_tiles, faces_mode, batch, clk); break;
    case 128: iugkp::march_kernel<128, EV><<<n_tiles, 128, lds, s>>>(d_insts, d_tiles, faces_mode, batch, clk); break;
    case 512: iugkp::march_kernel<512, EV><<<n_tiles, 512, lds, s>>>(d_insts, d_tiles, faces_mode, batch, clk); break;
    case 1024: iugkp::march_kernel<1024, EV><<<n_tiles, 1024, lds, s>>>(d_insts, d_tiles, faces_mode, batch, clk); break;
    default: iugkp::march_kernel<256, EV><<<n_tiles, 256, lds, s>>>(d_insts, d_tiles, faces_mode, batch, clk); break;
  }
}

// ev: some instance takes the expected-value estimator
int launch_march(const Inst *d_insts, const TileDesc *d_tiles, int n_tiles, size_t lds, int block,
                 int faces_mode, int batch, bool ev, hipStream_t s, unsigned long long *clk = nullptr)
{
  if (ev) launch_march_as<true>(d_insts, d_tiles, n_tiles, lds, block, faces_mode, batch, clk, s);
  else launch_march_as<false>(d_insts, d_tiles, n_tiles, lds, block, faces_mode, batch, clk, s);
  HIP_TRY(hipGetLastError());
  return IUGKP_OK;
}

__global__ void output_kernel(int n_cells, int n_fx, int n_fy, double n_avg, int faces,
                              double t_ref, double cv, double den_x, double den_y,
                              const double *aE, const double *ax, const double *ay, double *T,
                              double *qx, double *qy)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_cells) {
    const double e = (n_avg > 0.0) ? aE[i] / n_avg : aE[i];
    T[i] = t_ref + e / cv;
  }
  if (qx && i < n_fx) {
    const double f = (n_avg > 0.0) ? ax[i] / n_avg : ax[i];
    qx[i] = faces ? f / den_x : 0.0;
  }
  if (qy && i < n_fy) {
    const double f = (n_avg > 0.0) ? ay[i] / n_avg : ay[i];
    qy[i] = faces ? f / den_y : 0.0;
  }
}

// T = t_ref + E / cv and q = flux / (A tau_min) from the output accumulators.
int write_outputs(const InstHost &ih, double n_avg, double *T_out, double *qx_out, double *qy_out,
                  hipStream_t s)
{
  const Inst &d = ih.d;
  const Mesh &m = d.m;
  const int nmax = std::max(std::max(m.n_cells, m.n_fx), m.n_fy);
  const bool dev = (ih.mem_kind == IUGKP_MEM_DEVICE);
  double *T = dev ? T_out : ih.out_T;
  double *qx = qx_out ? (dev ? qx_out : ih.out_qx) : nullptr;
  double *qy = (qy_out && m.n_fy) ? (dev ? qy_out : ih.out_qy) : nullptr;
  output_kernel<<<cdiv(nmax, 256), 256, 0, s>>>(m.n_cells, m.n_fx, m.n_fy, n_avg, d.faces_out,
                                               d.t_ref, d.cv, m.dy * d.tau_min, m.dx * d.tau_min,
                                               d.acc_E, d.acc_x, d.acc_y, T, qx, qy);
  HIP_TRY(hipGetLastError());
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(T_out, ih.out_T, m.n_cells * sizeof(double), hipMemcpyDeviceToHost, s));
    if (qx_out)
      HIP_TRY(hipMemcpyAsync(qx_out, ih.out_qx, m.n_fx * sizeof(double), hipMemcpyDeviceToHost, s));
    if (qy_out && m.n_fy)
      HIP_TRY(hipMemcpyAsync(qy_out, ih.out_qy, m.n_fy * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  return IUGKP_OK;
}

int copy_out(void *dst, const void *src, size_t bytes, int kind, hipStream_t s)
{
  if (!dst) return IUGKP_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, bytes,
                         kind == IUGKP_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                         s));
  return IUGKP_OK;
}

int copy_in(void *dst, const void *src, size_t bytes, int kind, hipStream_t s)
{
  HIP_TRY(hipMemcpyAsync(dst, src, bytes,
                         kind == IUGKP_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                         s));
  return IUGKP_OK;
}

int upload_inst(const InstHost &ih, int inst_index, Inst *d_inst, TileDesc *d_tiles, int tile0,
                hipStream_t s)
{
  std::vector<TileDesc> t = ih.tiles;
  for (auto &x : t) x.inst = inst_index;
  HIP_TRY(hipMemcpyAsync(d_inst + inst_index, &ih.d, sizeof(Inst), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_tiles + tile0, t.data(), t.size() * sizeof(TileDesc),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// single solves
// ---------------------------------------------------------------------------
struct iugkp_handle {
  hipStream_t stream = nullptr;
  bool own_stream = false;        // created (and destroyed) by the library
  InstHost ih;                    // the problem (gray), or band 0 (frequency bands)
  std::vector<InstHost> xb;       // bands 1 .. K-1
  BandsHost bh;
  Inst *d_inst = nullptr;         // [K]
  TileDesc *d_tiles = nullptr;    // the tiles of the bands without row stripes first
  int n_tiles = 0;
  int n_tiles_f = 0;              // face-tallied iterations: tiles of those bands only
  std::vector<int> stripe_bands;  // bands whose face-tallied iterations run row stripes
  size_t lds = 0;                 // march window (largest over the bands)
  int block = 256;
  // the particle-step form of face-tallied iterations (pick_form)
  bool form_search = false;
  int form = -1;                  // chosen (kForm*), -1 while searching
  int form_default = 0;
  bool form_warm = false;         // the first face-tallied iteration has run
  int form_next = 0;              // candidates measured so far
  int form_last = -1;             // candidate of the iteration in flight
  float form_ms[4] = {-1.f, -1.f, -1.f, -1.f};
  DevScalars *hsc = nullptr;   // pinned host mirror
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  uint32_t iter = 0;
  double d0 = 0.0, res = 0.0;
  std::vector<double> res_hist;
  iugkp_stats st{};
};

namespace {

void free_handle(iugkp_handle *h)
{
  if (!h) return;
  if (h->own_stream && h->stream) (void)hipStreamSynchronize(h->stream);
  h->ih.release();
  for (auto &b : h->xb) b.release();
  if (h->d_inst) (void)hipFree(h->d_inst);
  if (h->d_tiles) (void)hipFree(h->d_tiles);
  if (h->hsc) (void)hipHostFree(h->hsc);
  for (auto &e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

// Device allocations of one call, freed (after the stream drains) when it goes
// out of scope.
struct DevScratch {
  hipStream_t s;
  std::vector<void *> p;
  explicit DevScratch(hipStream_t st) : s(st) {}
  ~DevScratch()
  {
    (void)hipStreamSynchronize(s);
    for (void *q : p) (void)hipFree(q);
  }
  template <class T>
  T *get(size_t n)
  {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
    p.push_back(q);
    return static_cast<T *>(q);
  }
};

// The single solve's CG on A x = b (persistent cooperative launch, status and
// iteration count into *sc); bracketed by ev_a / ev_b when given.
int enqueue_cg(const InstHost &ih, const double *b, double *x, DevScalars *sc, hipStream_t s,
               hipEvent_t ev_a, hipEvent_t ev_b)
{
  if (ih.mg_L > 0) {
    iugkp::MGArgs ma;
    ma.lv = ih.mg_lv;
    ma.L = ih.mg_L;
    ma.Lg = ih.mg_Lg;
    ma.b = b;
    ma.x = x;
    ma.p = ih.d.cg_p;
    ma.s = ih.d.cg_s;
    ma.w = ih.d.cg_w;
    ma.part = ih.cg_mpart;
    ma.tol2 = ih.d.tol2;
    ma.max_iters = ih.d.cg_max;
    ma.barrier = ih.cg_barrier;
    ma.sc = sc;
    ma.r2 = ih.mg_r2;
    ma.s2 = ih.mg_s2;
    ma.band = ih.mg_band;
    ma.stage0 = ih.mg_stage0;
    ma.stage_n = ih.mg_stage_n;
    iugkp::zero_u32_kernel<<<1, 64, 0, s>>>(ih.cg_barrier, 2);
    if (ev_a) HIP_TRY(hipEventRecord(ev_a, s));
    void *args[] = {&ma};
    HIP_TRY(hipLaunchKernel(ih.mg_band ? reinterpret_cast<const void *>(iugkp::mgcg_band_kernel)
                                       : reinterpret_cast<const void *>(iugkp::mgcg_kernel),
                            dim3(ih.mg_grid), dim3(ih.mg_threads), args, ih.mg_lds, s));
    if (ev_b) HIP_TRY(hipEventRecord(ev_b, s));
    return IUGKP_OK;
  }
  iugkp::CGArgs ca;
  ca.m = ih.d.m;
  ca.gx = ih.gx;
  ca.gy = ih.gy;
  ca.diag = ih.diag;
  ca.b = b;
  ca.x = x;
  ca.gr = ih.d.cg_r;
  ca.gw = ih.d.cg_w;
  ca.gp = ih.d.cg_p;
  ca.gs = ih.d.cg_s;
  ca.pub = ih.cg_pub;
  ca.part = ih.cg_mpart;
  ca.TB = ih.cg_tb;
  ca.tol2 = ih.d.tol2;
  ca.max_iters = ih.d.cg_max;
  ca.barrier = ih.cg_barrier;
  ca.sc = sc;
  iugkp::zero_u32_kernel<<<1, 64, 0, s>>>(ih.cg_barrier, 2);
  if (ev_a) HIP_TRY(hipEventRecord(ev_a, s));
  // Every workgroup must become resident for the group barrier.  Set-up
  // checked that the group fits the device; a plain launch (not a
  // cooperative one, which HIP serialises on one device-wide queue) lets the
  // CG of one handle run beside the CGs and particle steps of others: a
  // workgroup that is resident early waits in the barrier until the rest are
  // dispatched as other kernels' workgroups retire (none of them waits for the
  // CG), and a wait beyond the barrier's spin limit ends the solve with an
  // error instead of hanging.
  void *args[] = {&ca};
  HIP_TRY(hipLaunchKernel(cg_kernel_for(ih.cg_reg), dim3(ih.cg_grid),
                                     dim3(ih.cg_threads), args, ih.cg_lds, s));
  if (ev_b) HIP_TRY(hipEventRecord(ev_b, s));
  return IUGKP_OK;
}

// The particle step's form for the face-tallied iterations of a 2D gray
// single solve with the automatic march and the default block size: emitter
// tiles with 256 or 512 threads per workgroup, or row stripes.  Measured,
// not guessed: the first face-tallied iteration runs the planner's choice
// (not timed: first launches), the next three one candidate each (timed by
// the step's events), then the fastest, which every later handle of the
// same class (mesh, particles per emitter, null collisions, free path in
// cells to half an octave) takes from its first iteration.  The forms give
// the same tallies bit for bit, so the search changes only the time.
enum : int { kFormTiles256 = 0, kFormTiles512 = 1, kFormStripes = 2, kFormPieces = 3, kForms = 4 };
// (row stripes in pieces only without null collisions)
int n_forms(const InstHost &ih) { return ih.d.has_null ? kFormPieces : kForms; }
struct FormKey {
  int nx, ny, N, has_null, lam2;
  bool operator<(const FormKey &o) const
  {
    if (nx != o.nx) return nx < o.nx;
    if (ny != o.ny) return ny < o.ny;
    if (N != o.N) return N < o.N;
    if (has_null != o.has_null) return has_null < o.has_null;
    return lam2 < o.lam2;
  }
};
std::mutex g_form_mu;
std::map<FormKey, int> g_form_choice;

FormKey form_key(const InstHost &ih)
{
  const Mesh &m = ih.d.m;
  const double cells = ih.d.lam_min / std::min(m.dx, m.dy);
  return FormKey{m.nx, m.ny, static_cast<int>(ih.d.N), ih.d.has_null,
                 static_cast<int>(std::lround(2.0 * std::log2(cells)))};
}

// the form of the next face-tallied iteration (h->form_last: the candidate
// it measures, or -1)
int pick_form(iugkp_handle *h)
{
  h->form_last = -1;
  if (h->form >= 0) return h->form;
  if (!h->form_search) return h->form_default;
  if (!h->form_warm) {
    h->form_warm = true;
    return h->form_default;
  }
  h->form_last = h->form_next;
  return h->form_next;
}

// after the iteration: its particle-step time for the candidate it measured
void record_form(iugkp_handle *h, float ms)
{
  if (h->form_last < 0) return;
  h->form_ms[h->form_last] = ms;
  h->form_last = -1;
  if (++h->form_next < n_forms(h->ih)) return;
  int best = 0;
  for (int f = 1; f < n_forms(h->ih); ++f)
    if (h->form_ms[f] < h->form_ms[best]) best = f;
  h->form = best;
  std::lock_guard<std::mutex> lock(g_form_mu);
  g_form_choice[form_key(h->ih)] = best;
}

// The row-stripe particle step of one instance (ih, its descriptor at
// d_inst): the records' bin counters cleared, the pre-pass, then the march
// (in pieces when asked and the flights have no null collisions).
int launch_stripes(const InstHost &ih, const Inst *d_inst, bool pieces, hipStream_t s)
{
  const Mesh &m = ih.d.m;
  const unsigned long long np =
      static_cast<unsigned long long>(m.n_emit) * static_cast<unsigned long long>(ih.d.N);
  constexpr unsigned int per_block = iugkp::kPresampleBlock * iugkp::kPresamplePer;
  const unsigned int pg = static_cast<unsigned int>((np + per_block - 1) / per_block);
  const dim3 sg(ih.stripe_C, ih.stripe_S);
  const int ncnt = 2 * ih.rec.S * ih.rec.K;
  iugkp::zero_u32_kernel<<<cdiv(ncnt, 256), 256, 0, s>>>(ih.rec.cnt, ncnt);
  constexpr size_t ps_lds = static_cast<size_t>(iugkp::kPresampleBlock) * sizeof(uint32_t);
  if (ih.d.has_null)
    iugkp::stripe_presample_kernel<iugkp::kPresampleBlock, true>
        <<<pg, iugkp::kPresampleBlock, iugkp::kPresampleBlock * sizeof(iugkp::PRecN) + ps_lds, s>>>(
            d_inst, ih.rec);
  else
    iugkp::stripe_presample_kernel<iugkp::kPresampleBlock, false>
        <<<pg, iugkp::kPresampleBlock, iugkp::kPresampleBlock * sizeof(iugkp::PRec) + ps_lds, s>>>(
            d_inst, ih.rec);
  if (!ih.d.has_null && pieces)
    iugkp::march_stripes_pieces_kernel<kStripeBlock>
        <<<sg, kStripeBlock, ih.stripe_lds, s>>>(d_inst, ih.stripe_R, ih.stripe_C, ih.rec);
  else
    iugkp::march_stripes_kernel<kStripeBlock>
        <<<sg, kStripeBlock, ih.stripe_lds, s>>>(d_inst, ih.stripe_R, ih.stripe_C, ih.rec);
  HIP_TRY(hipGetLastError());
  return IUGKP_OK;
}

// Enqueue one iteration on the handle's stream: its kernels and the copy of
// the new scalars into h->hsc (complete_iteration waits for them).
int enqueue_iteration(iugkp_handle *h, int faces)
{
  const InstHost &ih = h->ih;
  const Mesh &m = ih.d.m;
  hipStream_t s = h->stream;
  const int nprep = std::max(std::max(std::max(m.n_emit, m.n_fx), std::max(m.n_fy, m.n_cells)),
                             (m.ny + 2) * m.nx);
  const int K = h->bh.K;
  int rc = IUGKP_OK;
  int form = -1;
  h->form_last = -1;
  if (ih.d.persist) {
    const int nmax = std::max(std::max(std::max(m.n_cells, m.n_b), std::max(m.n_fx, m.n_fy)),
                              (m.ny + 2) * m.nx);
    iugkp::persist_prepare_kernel<<<cdiv(nmax, 256), 256, 0, s>>>(h->d_inst);
    HIP_TRY(hipEventRecord(h->ev[0], s));
    const int stripes = (faces && ih.pst_R > 0) ? 1 : 0;
    // (the wall tallies in LDS up to 16 KB: 1365 wall faces)
    const size_t wall_lds = static_cast<size_t>(m.n_b) * (sizeof(long long) + sizeof(uint32_t));
    const int lds_walls = wall_lds <= 16384 ? 1 : 0;
    iugkp::persist_move_kernel<kPersistBlock>
        <<<ih.d.n_npart, kPersistBlock, lds_walls ? wall_lds : 0, s>>>(h->d_inst, faces, stripes,
                                                                         lds_walls);
    HIP_TRY(hipGetLastError());
    if (stripes) {
      iugkp::persist_faces_kernel<kPersistFacesBlock>
          <<<dim3(ih.pst_C, ih.pst_S), kPersistFacesBlock, ih.pst_lds, s>>>(h->d_inst, ih.pst_R,
                                                                          ih.pst_C);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipEventRecord(h->ev[1], s));
    if (faces) {
      if (m.dim == 2 && !stripes)
        iugkp::reconstruct_y_kernel<<<dim3(cdiv(m.nx, 4), 1), 256, 0, s>>>(h->d_inst, 1, 0);
      iugkp::persist_reconstruct_x_kernel<<<cdiv(m.ny, 4), 256, 0, s>>>(h->d_inst);
    }
    iugkp::persist_update_kernel<<<ih.d.n_gpart, 256, 0, s>>>(h->d_inst);
  } else {
  iugkp::prepare_kernel<<<dim3(cdiv(nprep, 256), K), 256, 0, s>>>(h->d_inst, faces, 0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(h->ev[0], s));
  if (ih.d.estimator && ih.stripe_R > 0) {
    iugkp::march_stripes_ev_kernel<kStripeBlock>
        <<<dim3(ih.stripe_C, ih.stripe_S), kStripeBlock, ih.stripe_lds, s>>>(h->d_inst, ih.stripe_R,
                                                                              ih.stripe_C, faces);
    HIP_TRY(hipGetLastError());
  } else if (K > 1 && faces && !h->stripe_bands.empty()) {
    // frequency bands: the long-path bands by row stripes, the others' tiles
    if (h->n_tiles_f > 0) {
      rc = launch_march(h->d_inst, h->d_tiles, h->n_tiles_f, h->lds, h->block, faces, 0, false, s);
      if (rc) return rc;
    }
    for (int k : h->stripe_bands) {
      const InstHost &bk = (k == 0) ? h->ih : h->xb[k - 1];
      if ((rc = launch_stripes(bk, h->d_inst + k, !bk.d.has_null, s))) return rc;
    }
  } else if (faces && ih.stripe_R > 0 &&
             ((form = pick_form(h)) == kFormStripes || form == kFormPieces)) {
    if ((rc = launch_stripes(ih, h->d_inst, form == kFormPieces, s))) return rc;
  } else {
    const int block = (form == kFormTiles512) ? 512 : h->block;
    rc = launch_march(h->d_inst, h->d_tiles, h->n_tiles, h->lds, block, faces, 0,
                      ih.d.estimator != 0, s);
    if (rc) return rc;
  }
  HIP_TRY(hipEventRecord(h->ev[1], s));
  if (faces) {
    iugkp::reconstruct_y_kernel<<<dim3(cdiv(m.nx, 4), K), 256, 0, s>>>(h->d_inst, faces, 0);
    iugkp::reconstruct_x_kernel<<<dim3(cdiv(m.ny, 4), K), 256, 0, s>>>(h->d_inst, faces, 0);
  }
  const int nbc = cdiv(m.n_cells, iugkp::kTree);
  if (K > 1)
    iugkp::bands_update_kernel<<<nbc, 256, 0, s>>>(h->d_inst, h->bh.d_bands, K, h->bh.srcV);
  else
    iugkp::update_kernel<<<dim3(nbc, 1), 256, 0, s>>>(h->d_inst, 0);
  HIP_TRY(hipGetLastError());
  if (ih.d.newton) {
    rc = enqueue_cg(ih, ih.d.rhs, ih.d.cg_x, ih.d.sc, s, h->ev[2], h->ev[3]);
    if (rc) return rc;
    const int nbe = cdiv(m.n_emit, iugkp::kTree);
    iugkp::newton_finish_kernel<<<dim3(nbe, 1), 256, 0, s>>>(h->d_inst, 0);
  }
  }
  iugkp::finish_kernel<<<1, 256, 0, s>>>(h->d_inst, 0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h->hsc, ih.d.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  return IUGKP_OK;
}

// Wait for the iteration enqueued on the handle's stream; counters, timings,
// residual history and the error checks.
int complete_iteration(iugkp_handle *h)
{
  const InstHost &ih = h->ih;
  hipStream_t s = h->stream;
  const int K = h->bh.K;
  HIP_TRY(hipStreamSynchronize(s));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
  h->st.ms_march += ms;
  record_form(h, ms);
  if (ih.d.newton) {
    HIP_TRY(hipEventElapsedTime(&ms, h->ev[2], h->ev[3]));
    h->st.ms_cg += ms;
  }
  const DevScalars &sc = *h->hsc;
  h->st.flights = sc.flights;
  h->st.segments = sc.segments;
  h->st.crossings = sc.crossings;
  h->st.tot_flights = sc.tot_flights;
  h->st.tot_segments = sc.tot_segments;
  h->st.tot_crossings = sc.tot_crossings;
  if (ih.d.newton) {
    h->st.cg_iters_last = sc.cg_iters;
    h->st.cg_iters_total = sc.cg_iters_total;
  }
  h->iter = sc.iter;
  h->d0 = sc.d0;
  h->res = sc.res;
  h->res_hist.push_back(sc.res);
  h->st.iters = static_cast<int>(h->iter);
  h->st.res = h->res;
  if (ih.d.newton && sc.cg_status == -3) return fail(IUGKP_E_DEVICE, "CG grid barrier timed out");
  if (ih.d.newton && sc.cg_status == -6) return fail(IUGKP_E_CG_BREAKDOWN, "CG breakdown");
  if (ih.d.newton && sc.cg_status == -7)
    return fail(IUGKP_E_CG_NOT_CONVERGED, "CG did not converge within cg_max_iters");
  if (sc.flags & 1) return fail(IUGKP_E_NONFINITE, "non-finite energy");
  if (sc.grew)
    return fail(IUGKP_E_DIVERGED, "Newton iteration diverged: the update grew beyond the first one");
  if ((sc.flags & 2) ||
      ((ih.d.newton || ih.d.Gs || K > 1 || ih.d.persist) && sc.gsum > (1ull << 62)))
    return fail(IUGKP_E_FIXED_OVERFLOW, "emission energy exceeds the fixed-point budget");
  if (h->iter > 1 && h->res > 1e3) return fail(IUGKP_E_DIVERGED, "residual grew above 1e3");
  return IUGKP_OK;
}

// One iteration on the handle's stream; leaves the new scalars in h->hsc.
int iterate(iugkp_handle *h, int faces)
{
  const int rc = enqueue_iteration(h, faces);
  return rc ? rc : complete_iteration(h);
}

// Outputs of a frequency-band problem: T = t_ref + E / sum_k C_k, q = sum over
// the bands of the face tallies / tau*_k, per face area.
int write_band_outputs(iugkp_handle *h, double *T_out, double *qx_out, double *qy_out)
{
  const InstHost &ih = h->ih;
  const Inst &d = ih.d;
  const Mesh &m = d.m;
  hipStream_t s = h->stream;
  const int nmax = std::max(std::max(m.n_cells, m.n_fx), m.n_fy);
  const bool dev = (ih.mem_kind == IUGKP_MEM_DEVICE);
  double *T = dev ? T_out : ih.out_T;
  double *qx = qx_out ? (dev ? qx_out : ih.out_qx) : nullptr;
  double *qy = (qy_out && m.n_fy) ? (dev ? qy_out : ih.out_qy) : nullptr;
  iugkp::bands_output_kernel<<<cdiv(nmax, 256), 256, 0, s>>>(
      m.n_cells, m.n_fx, m.n_fy, d.F, d.t_ref, h->bh.Ctot, m.dy, m.dx, d.faces_out, d.E,
      h->bh.d_bands, h->bh.d_phix, h->bh.d_phiy, h->bh.K, T, qx, qy);
  HIP_TRY(hipGetLastError());
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(T_out, ih.out_T, m.n_cells * sizeof(double), hipMemcpyDeviceToHost, s));
    if (qx_out)
      HIP_TRY(hipMemcpyAsync(qx_out, ih.out_qx, m.n_fx * sizeof(double), hipMemcpyDeviceToHost, s));
    if (qy_out && m.n_fy)
      HIP_TRY(hipMemcpyAsync(qy_out, ih.out_qy, m.n_fy * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  return IUGKP_OK;
}

const InstHost &band_of(const iugkp_handle *h, int k) { return k == 0 ? h->ih : h->xb[k - 1]; }

}  // namespace

extern "C" {

int iugkp_create(const iugkp_problem *problem, const iugkp_options *options, void *stream,
                 iugkp_handle **out)
{
  if (!out) return fail(IUGKP_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  iugkp_handle *h = new iugkp_handle();
  h->stream = static_cast<hipStream_t>(stream);
  if (options && options->own_stream) {
    // a stream of the handle's own (default priority, ordered with the null stream)
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) {
      delete h;
      return fail(IUGKP_E_DEVICE, "hipStreamCreate failed");
    }
    h->stream = st;
    h->own_stream = true;
  }
  const bool bands = problem && problem->n_bands > 1;
  int rc = bands ? setup_bands(problem, options, h->stream, h->ih, h->xb, h->bh)
                 : setup_instance(problem, options, h->stream, true, h->ih);
  if (rc) {
    free_handle(h);
    return rc;
  }
  const int K = h->bh.K;
  h->block = options->block_size ? options->block_size : 256;
  if (!bands && h->ih.stripe_R > 0 && !h->ih.d.estimator) {
    h->form_default = !h->ih.stripe_pref ? kFormTiles256
                      : (options->march == 3 && !h->ih.d.has_null) ? kFormPieces : kFormStripes;
    h->form_search = (options->march == 0 && options->block_size == 0);
    if (h->form_search) {
      std::lock_guard<std::mutex> lock(g_form_mu);
      const auto it = g_form_choice.find(form_key(h->ih));
      if (it != g_form_choice.end()) h->form = it->second;
    }
  }
  h->n_tiles = 0;
  for (int k = 0; k < K; ++k) {
    h->n_tiles += static_cast<int>(band_of(h, k).tiles.size());
    h->lds = std::max(h->lds, band_of(h, k).lds_bytes);
    if (bands && band_of(h, k).stripe_R > 0) h->stripe_bands.push_back(k);
  }
  if (hipMalloc(reinterpret_cast<void **>(&h->d_inst), K * sizeof(Inst)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&h->d_tiles), h->n_tiles * sizeof(TileDesc)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&h->hsc), sizeof(DevScalars)) != hipSuccess) {
    free_handle(h);
    return fail(IUGKP_E_NOMEM, "allocation failed");
  }
  for (auto &e : h->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      free_handle(h);
      return fail(IUGKP_E_DEVICE, "hipEventCreate failed");
    }
  // (the bands without row stripes first: a face-tallied iteration marches
  // the first n_tiles_f tiles, the others run their stripes)
  std::vector<int> order;
  for (int k = 0; k < K; ++k)
    if (!(bands && band_of(h, k).stripe_R > 0)) order.push_back(k);
  for (int k : h->stripe_bands) order.push_back(k);
  for (int i = 0, tile0 = 0; i < K; ++i) {
    const int k = order[i];
    if ((rc = upload_inst(band_of(h, k), k, h->d_inst, h->d_tiles, tile0, h->stream))) {
      free_handle(h);
      return rc;
    }
    tile0 += static_cast<int>(band_of(h, k).tiles.size());
    if (i + 1 == K - static_cast<int>(h->stripe_bands.size())) h->n_tiles_f = tile0;
  }
  if (h->stripe_bands.empty()) h->n_tiles_f = h->n_tiles;
  h->st.fixed_point_F = h->ih.d.F;
  h->st.n_per_emitter = h->ih.d.N;
  h->st.n_emitters = h->ih.d.m.n_emit * K;
  *out = h;
  return IUGKP_OK;
}

void iugkp_destroy(iugkp_handle *h)
{
  if (h && h->stream) (void)hipStreamSynchronize(h->stream);
  free_handle(h);
}

int iugkp_step_faces(iugkp_handle *h, int n_iters, int faces)
{
  if (!h || n_iters < 0) return fail(IUGKP_E_INVALID_ARG, "bad handle or count");
  for (int i = 0; i < n_iters; ++i) {
    const int rc = iterate(h, faces ? 1 : 0);
    if (rc) return rc;
  }
  return IUGKP_OK;
}

int iugkp_step_group(iugkp_handle *const *hs, int n, int n_iters)
{
  if (!hs || n < 1 || n_iters < 0) return fail(IUGKP_E_INVALID_ARG, "bad handle list or count");
  for (int i = 0; i < n; ++i) {
    if (!hs[i]) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(IUGKP_E_INVALID_ARG, "a handle appears twice");
  }
  // each handle runs its iterations back to back; a finished iteration is
  // completed and the handle's next one enqueued as soon as its stream is idle.
  // Every CG group waits at its barriers for all its workgroups, so the CGs
  // that can be in flight together must fit on the device at once: an
  // iteration is enqueued only while the CG footprints (in compute units) of
  // the iterations in flight leave room for its own.  (Particle-step
  // workgroups never wait for a CG, so they only delay residency.)
  int dev = 0, n_cu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  const double room = static_cast<double>(n_cu);
  std::vector<int> left(n, n_iters);
  std::vector<char> busy(n, 0);
  int first = IUGKP_OK, n_busy = 0;
  double in_flight = 0.0;
  auto cus = [&](int i) { return hs[i]->ih.d.newton ? hs[i]->ih.cg_cus : 0.0; };
  auto start = [&](int i) -> bool {
    if (first || left[i] == 0 || busy[i]) return false;
    if (n_busy > 0 && in_flight + cus(i) > room) return false;     // wait for room
    const int rc = enqueue_iteration(hs[i], hs[i]->ih.d.faces_each);
    if (rc) {
      first = rc;
      return false;
    }
    busy[i] = 1;
    ++n_busy;
    in_flight += cus(i);
    return true;
  };
  for (int i = 0; i < n; ++i) start(i);
  int next = 0;                        // round-robin start of the waiting handles
  while (n_busy > 0) {
    bool freed = false;
    for (int i = 0; i < n; ++i) {
      if (!busy[i]) continue;
      const hipError_t q = hipStreamQuery(hs[i]->stream);
      if (q == hipErrorNotReady) continue;
      busy[i] = 0;
      --n_busy;
      in_flight -= cus(i);
      freed = true;
      const int rc = complete_iteration(hs[i]);   // also reports a failed stream
      --left[i];
      if (rc && !first) first = rc;
    }
    if (freed) {
      for (int j = 0; j < n; ++j) start((next + j) % n);
      next = (next + 1) % n;
    }
  }
  return first;
}

int iugkp_step(iugkp_handle *h, int n_iters)
{
  if (!h) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
  return iugkp_step_faces(h, n_iters, h->ih.d.faces_each);
}

int iugkp_solve(iugkp_handle *h, double *T_out, double *qx_out, double *qy_out,
                iugkp_stats *stats)
{
  if (!h || !T_out) return fail(IUGKP_E_INVALID_ARG, "bad handle or T_out");
  const Inst &d = h->ih.d;
  const Mesh &m = d.m;
  hipStream_t s = h->stream;
  bool converged = false;
  int rc;
  while (static_cast<int>(h->iter) < d.max_iters) {
    if ((rc = iterate(h, d.faces_each))) return rc;
    if (h->res < d.res_tol) {
      converged = true;
      break;
    }
  }
  if (h->bh.K > 1) {
    if (d.final_iter && (rc = iterate(h, 1))) return rc;
    if ((rc = write_band_outputs(h, T_out, qx_out, qy_out))) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    h->st.status = converged ? IUGKP_OK : IUGKP_W_NOT_CONVERGED;
    if (stats) *stats = h->st;
    return h->st.status;
  }
  const int nmax = std::max(std::max(m.n_cells, m.n_fx), m.n_fy);
  const dim3 grid(cdiv(nmax, 256), 1);
  double n_avg = 0.0;
  if (d.avg_iters > 0) {
    for (int a = 0; a < d.avg_iters; ++a) {
      if ((rc = iterate(h, d.faces_out))) return rc;
      iugkp::accumulate_kernel<<<grid, 256, 0, s>>>(h->d_inst, 0, a == 0 ? 2 : 1);
    }
    n_avg = static_cast<double>(d.avg_iters);
  } else {
    if (d.final_iter && (rc = iterate(h, 1))) return rc;
    iugkp::accumulate_kernel<<<grid, 256, 0, s>>>(h->d_inst, 0, 2);
  }
  HIP_TRY(hipGetLastError());
  if ((rc = write_outputs(h->ih, n_avg, T_out, qx_out, qy_out, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  h->st.status = converged ? IUGKP_OK : IUGKP_W_NOT_CONVERGED;
  if (stats) *stats = h->st;
  return h->st.status;
}

int iugkp_get_tallies(iugkp_handle *h, int64_t *D, int64_t *W, int64_t *Phi_x, int64_t *Phi_y,
                      int64_t *B)
{
  if (!h) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
  const int k = h->ih.mem_kind;
  hipStream_t s = h->stream;
  int rc;
  for (int b = 0; b < h->bh.K; ++b) {
    const Inst &d = band_of(h, b).d;
    const Mesh &m = d.m;
    const size_t o = static_cast<size_t>(b);
    if ((rc = copy_out(D ? D + o * m.n_cells : nullptr, d.D, m.n_cells * 8, k, s))) return rc;
    if ((rc = copy_out(W ? W + o * m.n_cells : nullptr, (d.has_null || d.persist) ? d.W : d.D,
                       m.n_cells * 8, k, s)))
      return rc;
    if ((rc = copy_out(Phi_x ? Phi_x + o * m.n_fx : nullptr, d.Phix, m.n_fx * 8, k, s))) return rc;
    if (m.n_fy && (rc = copy_out(Phi_y ? Phi_y + o * m.n_fy : nullptr, d.Phiy, m.n_fy * 8, k, s)))
      return rc;
    if ((rc = copy_out(B ? B + o * m.n_b : nullptr, d.B, m.n_b * 8, k, s))) return rc;
  }
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

int iugkp_get_state(iugkp_handle *h, uint32_t *iter, double *d0, double *E, int64_t *G)
{
  if (!h) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
  if (iter) *iter = h->iter;
  if (d0) *d0 = h->d0;
  const Inst &d = h->ih.d;
  int rc;
  if ((rc = copy_out(E, d.E, d.m.n_cells * 8, h->ih.mem_kind, h->stream))) return rc;
  if (d.persist) {
    if ((rc = copy_out(G, d.wc, d.m.n_cells * 8, h->ih.mem_kind, h->stream))) return rc;
    if ((rc = copy_out(G ? G + d.m.n_cells : nullptr, d.wb, d.m.n_b * 8, h->ih.mem_kind, h->stream)))
      return rc;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return IUGKP_OK;
  }
  for (int b = 0; b < h->bh.K; ++b)
    if ((rc = copy_out(G ? G + static_cast<size_t>(b) * d.m.n_emit : nullptr, band_of(h, b).d.G,
                       d.m.n_emit * 8, h->ih.mem_kind, h->stream)))
      return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  return IUGKP_OK;
}

int iugkp_set_state(iugkp_handle *h, uint32_t iter, double d0, const double *E, const int64_t *G)
{
  if (!h || !E || !G) return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  if (h->ih.d.persist)
    return fail(IUGKP_E_INVALID_ARG, "the state of the persistent scheme is its population");
  const Inst &d = h->ih.d;
  const Mesh &m = d.m;
  const size_t ng = static_cast<size_t>(m.n_emit) * h->bh.K;
  std::vector<long long> g(ng);
  if (h->ih.mem_kind == IUGKP_MEM_HOST) {
    std::memcpy(g.data(), G, ng * 8);
  } else {
    HIP_TRY(hipMemcpy(g.data(), G, ng * 8, hipMemcpyDeviceToHost));
  }
  unsigned long long acc = 0;
  for (long long v : g) {
    const unsigned long long a = static_cast<unsigned long long>(v < 0 ? -v : v);
    acc += a;
    if (a > (1ull << 62) || acc > (1ull << 62))
      return fail(IUGKP_E_FIXED_OVERFLOW, "restored emission exceeds the fixed-point budget");
  }
  int rc;
  if ((rc = copy_in(d.E, E, m.n_cells * 8, h->ih.mem_kind, h->stream))) return rc;
  for (int b = 0; b < h->bh.K; ++b)
    HIP_TRY(hipMemcpyAsync(band_of(h, b).d.G, g.data() + static_cast<size_t>(b) * m.n_emit,
                           m.n_emit * 8, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(h->hsc, d.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->hsc->iter = iter;
  h->hsc->d0 = d0;
  h->hsc->res_p1 = h->hsc->res_p2 = HUGE_VAL;
  HIP_TRY(hipMemcpyAsync(d.sc, h->hsc, sizeof(DevScalars), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->iter = iter;
  h->d0 = d0;
  h->st.iters = static_cast<int>(iter);
  return IUGKP_OK;
}

int iugkp_get_residuals(iugkp_handle *h, double *res, int max_n)
{
  if (!h || !res) return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  const int n = std::min<int>(max_n, static_cast<int>(h->res_hist.size()));
  for (int i = 0; i < n; ++i) res[i] = h->res_hist[i];
  return n;
}

int iugkp_get_stats(iugkp_handle *h, iugkp_stats *stats)
{
  if (!h || !stats) return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  *stats = h->st;
  return IUGKP_OK;
}

int iugkp_march_tuning(iugkp_handle *h, int *form, float *ms)
{
  if (!h) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
  if (form) *form = h->form >= 0 ? h->form : (h->form_search ? -1 : h->form_default);
  if (ms)
    for (int f = 0; f < kForms; ++f) ms[f] = h->form_ms[f];
  return IUGKP_OK;
}

int iugkp_get_particles(iugkp_handle *h, double *x, double *y, double *sx, double *sy, int64_t *q,
                        int32_t *kind, int32_t *loc)
{
  if (!h) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
  const Inst &d = h->ih.d;
  if (!d.persist) return fail(IUGKP_E_INVALID_ARG, "no persistent population (emitter scheme)");
  const int k = h->ih.mem_kind;
  hipStream_t s = h->stream;
  const size_t n = d.n_part;
  int rc;
  if ((rc = copy_out(x, d.px, n * 8, k, s))) return rc;
  if ((rc = copy_out(y, d.py, n * 8, k, s))) return rc;
  if ((rc = copy_out(sx, d.psx, n * 8, k, s))) return rc;
  if ((rc = copy_out(sy, d.psy, n * 8, k, s))) return rc;
  if ((rc = copy_out(q, d.pq, n * 8, k, s))) return rc;
  if (kind || loc) {
    DevScratch tmp(s);
    int32_t *dk = nullptr, *dl = nullptr;
    if (kind) dk = (k == IUGKP_MEM_DEVICE) ? kind : tmp.get<int32_t>(n);
    if (loc) dl = (k == IUGKP_MEM_DEVICE) ? loc : tmp.get<int32_t>(n);
    if ((kind && !dk) || (loc && !dl)) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
    iugkp::persist_unpack_kernel<<<cdiv(static_cast<long long>(n), 256), 256, 0, s>>>(
        d.plk, static_cast<unsigned int>(n), dk, dl);
    HIP_TRY(hipGetLastError());
    if (k == IUGKP_MEM_HOST) {
      if (kind) HIP_TRY(hipMemcpyAsync(kind, dk, n * 4, hipMemcpyDeviceToHost, s));
      if (loc) HIP_TRY(hipMemcpyAsync(loc, dl, n * 4, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

int iugkp_get_shares(iugkp_handle *h, uint32_t *n_rc, uint32_t *n_b, int64_t *w_c, int64_t *r_c,
                     int64_t *w_b, int64_t *r_b)
{
  if (!h) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
  const Inst &d = h->ih.d;
  if (!d.persist) return fail(IUGKP_E_INVALID_ARG, "no persistent population (emitter scheme)");
  const int k = h->ih.mem_kind;
  hipStream_t s = h->stream;
  const size_t nc = d.m.n_cells, nb = d.m.n_b;
  int rc;
  if ((rc = copy_out(n_rc, d.Nrc, nc * 4, k, s))) return rc;
  if ((rc = copy_out(n_b, d.Nb, nb * 4, k, s))) return rc;
  if ((rc = copy_out(w_c, d.wc, nc * 8, k, s))) return rc;
  if ((rc = copy_out(r_c, d.rc, nc * 8, k, s))) return rc;
  if ((rc = copy_out(w_b, d.wb, nb * 8, k, s))) return rc;
  if ((rc = copy_out(r_b, d.rb, nb * 8, k, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

int iugkp_adjoint(iugkp_handle *h, const double *dLdT, double *grad_wall, double *grad_source,
                  int max_iters, double tol, int *iters_out)
{
  if (iters_out) *iters_out = 0;
  if (!h || !dLdT || max_iters < 1 || !(tol >= 0.0))
    return fail(IUGKP_E_INVALID_ARG, "bad adjoint arguments");
  if (h->bh.K > 1) return fail(IUGKP_E_INVALID_ARG, "the adjoint covers gray problems only");
  if (h->ih.d.persist || h->ih.d.estimator)
    return fail(IUGKP_E_INVALID_ARG, "the adjoint covers the emitter scheme's analog paths only");
  InstHost &ih = h->ih;
  const Inst &d = ih.d;
  const Mesh &m = d.m;
  if (!d.crn) return fail(IUGKP_E_INVALID_ARG, "the adjoint needs common random numbers (rng_mode CRN)");
  if (d.has_null) return fail(IUGKP_E_INVALID_ARG, "the adjoint needs a uniform relaxation time");
  if (d.N > 65536u) return fail(IUGKP_E_INVALID_ARG, "the adjoint allows at most 65536 particles per emitter");
  hipStream_t s = h->stream;
  const int nc = m.n_cells, ne = m.n_emit, nbc = cdiv(nc, iugkp::kTree);
  const long long np = static_cast<long long>(ne) * d.N;
  DevScratch sc(s);   // freed when the call returns
  int *end = sc.get<int>(static_cast<size_t>(np));
  double *u = sc.get<double>(nc), *psi = sc.get<double>(nc), *half = sc.get<double>(nc);
  double *g = sc.get<double>(ne), *part = sc.get<double>(nbc), *dn = sc.get<double>(1);
  double *dl = sc.get<double>(nc);
  double *gw = sc.get<double>(m.n_b), *gs = sc.get<double>(nc);
  DevScalars *asc = sc.get<DevScalars>(1);
  if (!end || !u || !psi || !half || !g || !part || !dn || !dl || !gw || !gs || !asc)
    return fail(IUGKP_E_NOMEM, "hipMalloc failed");
  HIP_TRY(hipMemcpyAsync(dl, dLdT, nc * sizeof(double),
                         ih.mem_kind == IUGKP_MEM_DEVICE ? hipMemcpyDeviceToDevice
                                                         : hipMemcpyHostToDevice, s));
  const iugkp::FlyIn fa = {m, d.lam_min, d.epoch, d.key0, d.key1, 0, 0, d.ratio};
  iugkp::adjoint_paths_kernel<<<cdiv(np, 256), 256, 0, s>>>(fa, ne, d.N, end);
  iugkp::adjoint_init_kernel<<<cdiv(nc, 256), 256, 0, s>>>(nc, d.cv, d.V, d.F, dl, u, psi);
  HIP_TRY(hipGetLastError());
  const int gather_blocks = cdiv(static_cast<long long>(ne) * 64, 256);
  int passes = 0, rc = IUGKP_W_NOT_CONVERGED;
  double d0 = 0.0;
  for (int it = 0; it < max_iters; ++it) {
    iugkp::adjoint_gather_kernel<<<gather_blocks, 256, 0, s>>>(end, psi, ne, d.N, g);
    iugkp::adjoint_half_kernel<<<nbc, 256, 0, s>>>(nc, g, u, half, psi, d.rhs, d.newton, part);
    if (d.newton) {
      if ((rc = enqueue_cg(ih, d.rhs, d.cg_x, asc, s, nullptr, nullptr))) return rc;
      iugkp::adjoint_newton_kernel<<<nbc, 256, 0, s>>>(nc, half, d.cg_x, psi, part);
    }
    iugkp::adjoint_norm_kernel<<<1, 256, 0, s>>>(part, nbc, dn);
    HIP_TRY(hipGetLastError());
    double hdn = 0.0;
    DevScalars hs{};
    HIP_TRY(hipMemcpyAsync(&hdn, dn, sizeof(double), hipMemcpyDeviceToHost, s));
    if (d.newton) HIP_TRY(hipMemcpyAsync(&hs, asc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    passes = it + 1;
    if (d.newton && hs.cg_status == -3) return fail(IUGKP_E_DEVICE, "CG grid barrier timed out");
    if (d.newton && hs.cg_status == -6) return fail(IUGKP_E_CG_BREAKDOWN, "adjoint CG breakdown");
    if (d.newton && hs.cg_status == -7)
      return fail(IUGKP_E_CG_NOT_CONVERGED, "adjoint CG did not converge within cg_max_iters");
    if (it == 0) d0 = hdn;
    const double res = (d0 > 0.0) ? hdn / d0 : 0.0;
    if (!std::isfinite(res)) return fail(IUGKP_E_NONFINITE, "non-finite adjoint");
    if (res < tol) {
      rc = IUGKP_OK;
      break;
    }
  }
  // gradients from the converged psi: one more reverse pass
  iugkp::adjoint_gather_kernel<<<gather_blocks, 256, 0, s>>>(end, psi, ne, d.N, g);
  const double fs = std::ldexp(d.V * d.tau_min, d.F);
  const double fw_lr = std::ldexp((d.cv * (d.lam_min * m.dy)) / 4.0, d.F);
  const double fw_bt = std::ldexp((d.cv * (d.lam_min * m.dx)) / 4.0, d.F);
  iugkp::adjoint_grad_kernel<<<cdiv(std::max(nc, m.n_b), 256), 256, 0, s>>>(
      nc, m.n_b, m.ny, g, fs, fw_lr, fw_bt, gs, gw);
  HIP_TRY(hipGetLastError());
  const hipMemcpyKind out_kind =
      ih.mem_kind == IUGKP_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (grad_wall) HIP_TRY(hipMemcpyAsync(grad_wall, gw, m.n_b * sizeof(double), out_kind, s));
  if (grad_source) HIP_TRY(hipMemcpyAsync(grad_source, gs, nc * sizeof(double), out_kind, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (iters_out) *iters_out = passes;
  return rc;
}

double iugkp_d_eff(double lam, double delta) { return iugkp::d_eff(lam, delta); }

}  // extern "C"

namespace {

// Device buffers of one stateless diffusion solve, carved from one region.
struct DiffusionBufs {
  double *gx, *gy, *diag, *gr, *gw, *gp, *gs, *pub, *part;
  unsigned int *barrier;
  DevScalars *sc;
};

// Bytes of DiffusionBufs for a mesh (every piece 256-byte aligned).
size_t diffusion_bytes(const Mesh &m)
{
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t nc = m.n_cells, nbt = cdiv(m.n_cells, iugkp::kTree);
  return up(8 * static_cast<size_t>(m.n_fx)) + up(8 * std::max<size_t>(m.n_fy, 1)) +
         5 * up(8 * nc) + up(8 * 6 * nc) + up(8 * 4 * nbt) + up(8) + up(sizeof(DevScalars));
}

DiffusionBufs carve_diffusion(const Mesh &m, unsigned char *base)
{
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t nc = m.n_cells, nbt = cdiv(m.n_cells, iugkp::kTree);
  DiffusionBufs b;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    unsigned char *q = base + o;
    o += up(bytes);
    return q;
  };
  b.gx = reinterpret_cast<double *>(take(8 * static_cast<size_t>(m.n_fx)));
  b.gy = reinterpret_cast<double *>(take(8 * std::max<size_t>(m.n_fy, 1)));
  b.diag = reinterpret_cast<double *>(take(8 * nc));
  b.gr = reinterpret_cast<double *>(take(8 * nc));
  b.gw = reinterpret_cast<double *>(take(8 * nc));
  b.gp = reinterpret_cast<double *>(take(8 * nc));
  b.gs = reinterpret_cast<double *>(take(8 * nc));
  b.pub = reinterpret_cast<double *>(take(8 * 6 * nc));
  b.part = reinterpret_cast<double *>(take(8 * 4 * nbt));
  b.barrier = reinterpret_cast<unsigned int *>(take(8));
  b.sc = reinterpret_cast<DevScalars *>(take(sizeof(DevScalars)));
  return b;
}

int diffusion_mesh(int dim, int nx, int ny, double dx, double dy, double vg, const double *tau,
                   const double *D_x, const double *D_y, const double *b, double *x, double tol,
                   int max_iters, Mesh &m)
{
  if ((dim != 1 && dim != 2) || nx < 1 || ny < 1 || (dim == 1 && ny != 1) || !(dx > 0.0) ||
      !(dy > 0.0) || !(vg > 0.0) || !tau || !D_x || (dim == 2 && !D_y) || !b || !x ||
      !(tol > 0.0) || max_iters < 1 || static_cast<long long>(nx) * ny > (1ll << 28))
    return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  m = Mesh{};
  m.dim = dim;
  m.nx = nx;
  m.ny = ny;
  m.n_cells = nx * ny;
  m.n_b = 2 * ny + (dim == 2 ? 2 * nx : 0);
  m.n_emit = m.n_cells + m.n_b;
  m.n_fx = ny * (nx + 1);
  m.n_fy = (dim == 2) ? (ny + 1) * nx : 0;
  m.dx = dx;
  m.dy = dy;
  return IUGKP_OK;
}

// Assemble the Newton operator into the buffers and run the plain CG from
// x = 0; status and iteration count read back before returning.
int diffusion_run(const Mesh &m, const CgPlan &cp, const DiffusionBufs &q, double vg,
                  const double *tau, const double *D_x, const double *D_y, const double *b,
                  double *x, double tol, int max_iters, int *iters_out, hipStream_t s)
{
  const int nf = std::max(m.n_fx, m.n_fy);
  const int sc_words = static_cast<int>(sizeof(DevScalars) / 4);
  iugkp::zero_u32_kernel<<<cdiv(sc_words, 64), 64, 0, s>>>(reinterpret_cast<unsigned int *>(q.sc),
                                                           sc_words);
  iugkp::newton_operator_kernel<<<cdiv(nf, 256), 256, 0, s>>>(m, vg, tau, D_x,
                                                               m.dim == 2 ? D_y : D_x, q.gx,
                                                               q.gy, q.diag);
  iugkp::newton_diag_kernel<<<cdiv(m.n_cells, 256), 256, 0, s>>>(m, q.gx, q.gy, q.diag);
  iugkp::CGArgs ca;
  ca.m = m;
  ca.gx = q.gx;
  ca.gy = q.gy;
  ca.diag = q.diag;
  ca.b = b;
  ca.x = x;
  ca.gr = q.gr;
  ca.gw = q.gw;
  ca.gp = q.gp;
  ca.gs = q.gs;
  ca.pub = q.pub;
  ca.part = q.part;
  ca.TB = cp.tb;
  ca.tol2 = tol * tol;
  ca.max_iters = max_iters;
  ca.barrier = q.barrier;
  ca.sc = q.sc;
  iugkp::zero_u32_kernel<<<1, 64, 0, s>>>(q.barrier, 2);
  void *args[] = {&ca};
  HIP_TRY(hipLaunchKernel(cg_kernel_for(cp.reg), dim3(cp.grid), dim3(cp.threads), args, cp.lds, s));
  HIP_TRY(hipGetLastError());
  int head[2] = {0, 0};      // cg_iters, cg_status
  HIP_TRY(hipMemcpyAsync(head, &q.sc->cg_iters, sizeof(head), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (iters_out) *iters_out = head[0];
  if (head[1] == -3) return fail(IUGKP_E_DEVICE, "CG grid barrier timed out");
  if (head[1] == -6) return fail(IUGKP_E_CG_BREAKDOWN, "CG breakdown");
  if (head[1] == -7) return fail(IUGKP_E_CG_NOT_CONVERGED, "CG did not converge within max_iters");
  return IUGKP_OK;
}

}  // namespace

namespace {

// Scratch of the no-allocation diffusion solve: one array per device, held
// until the process ends.  Host code never uses the symbol's host-side name as
// an address: each device's copy is looked up once (with that device
// current) and its address kept in g_scratch_dev.
constexpr size_t kNoAllocBytes = 8u << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

int scratch_of_current_device(unsigned char **out)
{
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(IUGKP_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(IUGKP_E_DEVICE, "no device address for the scratch array");
    g_scratch_dev[dev] = ptr;
  }
  *out = static_cast<unsigned char *>(g_scratch_dev[dev]);
  return IUGKP_OK;
}

}  // namespace

extern "C" {

int iugkp_diffusion_solve_noalloc(int dim, int nx, int ny, double dx, double dy, double vg,
                                  const double *tau, const double *D_x, const double *D_y,
                                  const double *b, double *x, double tol, int max_iters,
                                  int *iters_out, void *stream)
{
  Mesh m;
  int rc = diffusion_mesh(dim, nx, ny, dx, dy, vg, tau, D_x, D_y, b, x, tol, max_iters, m);
  if (rc) return rc;
  const size_t need = diffusion_bytes(m);
  if (need > kNoAllocBytes)
    return fail(IUGKP_E_INVALID_ARG, "mesh too large for the no-allocation scratch (" +
                                         std::to_string(need) + " bytes needed, " +
                                         std::to_string(kNoAllocBytes) + " available)");
  CgPlan cp;
  if ((rc = plan_cg(m, 0, cp))) return rc;
  unsigned char *base = nullptr;
  if ((rc = scratch_of_current_device(&base))) return rc;
  return diffusion_run(m, cp, carve_diffusion(m, base), vg, tau, D_x, D_y, b, x, tol, max_iters,
                       iters_out, static_cast<hipStream_t>(stream));
}

int iugkp_diffusion_solve(int dim, int nx, int ny, double dx, double dy, double vg,
                          const double *tau, const double *D_x, const double *D_y,
                          const double *b, double *x, double tol, int max_iters, int *iters_out,
                          void *stream)
{
  Mesh m;
  int rc = diffusion_mesh(dim, nx, ny, dx, dy, vg, tau, D_x, D_y, b, x, tol, max_iters, m);
  if (rc) return rc;
  CgPlan cp;
  if ((rc = plan_cg(m, 0, cp))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevScratch tmp(s);
  unsigned char *base = tmp.get<unsigned char>(diffusion_bytes(m));
  if (!base) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
  return diffusion_run(m, cp, carve_diffusion(m, base), vg, tau, D_x, D_y, b, x, tol, max_iters,
                       iters_out, s);
}

const char *iugkp_strerror(int code)
{
  switch (code) {
    case IUGKP_OK: return "ok";
    case IUGKP_W_NOT_CONVERGED: return "not converged within max_iters";
    case IUGKP_E_INVALID_ARG: return "invalid argument";
    case IUGKP_E_NOMEM: return "out of device memory";
    case IUGKP_E_DEVICE: return "HIP runtime error";
    case IUGKP_E_FIXED_OVERFLOW: return "fixed-point overflow";
    case IUGKP_E_NONFINITE: return "non-finite value";
    case IUGKP_E_CG_BREAKDOWN: return "CG breakdown";
    case IUGKP_E_CG_NOT_CONVERGED: return "CG not converged";
    case IUGKP_E_DIVERGED: return "iteration diverged";
    default: return "unknown error";
  }
}

const char *iugkp_last_error(void) { return g_last_error.c_str(); }

int iugkp_dev_philox(const uint32_t *ctr, uint32_t key0, uint32_t key1, uint32_t *out, int64_t n,
                     void *stream)
{
  if (!ctr || !out || n < 0) return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n > 0) iugkp::philox_probe_kernel<<<cdiv(n, 256), 256, 0, s>>>(ctr, key0, key1, out, n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

int iugkp_dev_math(int op, const double *x, const double *y, double *out, int64_t n, void *stream)
{
  if (!x || !out || n < 0 || op < 0 || op > 6 || ((op == 3 || op == 5) && !y))
    return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n > 0) iugkp::math_probe_kernel<<<cdiv(n, 256), 256, 0, s>>>(op, x, y, out, n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

int iugkp_dev_atomics(int lds, int64_t n_words, int64_t per_thread, int64_t n_threads,
                      double *ms_out, void *stream)
{
  if (!ms_out || (lds != 0 && lds != 1) || n_words < 4096 || n_words > (1ll << 28) ||
      per_thread < 1 || per_thread > 4096 || n_threads < 256 || n_threads > (1ll << 26) ||
      n_threads % 256 != 0)
    return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DevScratch tmp(s);
  long long *words = tmp.get<long long>(n_words);
  if (!words) return fail(IUGKP_E_NOMEM, "hipMalloc failed");
  HIP_TRY(hipMemsetAsync(words, 0, n_words * sizeof(long long), s));
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  const int grid = static_cast<int>(n_threads / 256);
  // one untimed launch, then the timed one
  iugkp::atomics_probe_kernel<<<grid, 256, 0, s>>>(lds, words, static_cast<int>(n_words),
                                                   static_cast<int>(per_thread));
  HIP_TRY(hipEventRecord(a, s));
  iugkp::atomics_probe_kernel<<<grid, 256, 0, s>>>(lds, words, static_cast<int>(n_words),
                                                   static_cast<int>(per_thread));
  HIP_TRY(hipEventRecord(b, s));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventSynchronize(b));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, a, b));
  *ms_out = ms;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return IUGKP_OK;
}

int iugkp_dev_segments(int dim, int nx, int ny, double dx, double dy, const double *rays,
                       int64_t n, int64_t *out, void *stream)
{
  if (!rays || !out || n < 0 || (dim != 1 && dim != 2) || nx < 1 || ny < 1 ||
      (dim == 1 && ny != 1) || !(dx > 0.0) || !(dy > 0.0))
    return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  Mesh m{};
  m.dim = dim;
  m.nx = nx;
  m.ny = ny;
  m.n_cells = nx * ny;
  m.n_b = 2 * ny + (dim == 2 ? 2 * nx : 0);
  m.n_emit = m.n_cells + m.n_b;
  m.n_fx = ny * (nx + 1);
  m.n_fy = (dim == 2) ? (ny + 1) * nx : 0;
  m.dx = dx;
  m.dy = dy;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n > 0)
    iugkp::segment_probe_kernel<<<cdiv(n, 256), 256, 0, s>>>(m, rays, n,
                                                             reinterpret_cast<long long *>(out));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched solves
// ---------------------------------------------------------------------------
struct iugkp_batch {
  hipStream_t stream = nullptr;      // the caller's stream
  hipStream_t own = nullptr;         // capture/replay stream (the legacy default stream cannot be captured)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  std::vector<InstHost> insts;
  Inst *d_insts = nullptr;
  TileDesc *d_tiles = nullptr;
  int n_tiles = 0;
  size_t lds_max = 0;
  int any_newton = 0;
  bool any_ev = false;                // some instance takes the expected-value estimator
  int max_prep = 1, max_nx = 1, max_ny = 1, max_nbc = 1, max_nbe = 1, max_out = 1;
  // batched CG: a pool of resident workgroups and, per replay, the host's
  // schedule of (instance, rank) jobs on it
  struct Pool {
    int size = 0;                    // resident workgroups
    size_t lds = 0;
    int *d_off = nullptr, *h_off = nullptr;
    iugkp::CgJob *d_jobs = nullptr, *h_jobs = nullptr;
    int max_jobs = 0;
    bool used = false;
  };
  Pool pool, mg_pool;                // plain CG; multigrid-preconditioned CG
  std::vector<int> cg_G, cg_tb;      // per instance: group size, blocks per workgroup | form bit
  // the multigrid pool's autotuned group sizes: per instance the largest
  // group, the group of the last replay (0: not run), and the clock rate
  std::vector<int> mg_gmax, mg_last;
  double clock_khz = 0.0;
  // the autotuned tile sizes: per instance the tile edge (8 or 16 cells), its
  // range of the tile table, the measured device time per flight with each
  // edge (-1: not measured); the search phase (0: first replay, 1: edge 8
  // timed, 2: edge 16 timed, 3: chosen); the workgroups' clock stamps
  std::vector<int> edge, tile_first, tile_count;
  std::vector<double> cost8, cost16;
  std::vector<char> edge_known;      // the class's edge came from an earlier batch
  int tile_phase = 3;
  unsigned long long *d_clk = nullptr;
  std::vector<unsigned long long> h_clk;
  iugkp::MGArgs *d_mg_args = nullptr;   // the multigrid jobs' arguments, per instance
  DevScalars *d_scs = nullptr;       // every instance's scalars, contiguous
  unsigned int *d_bars = nullptr;    // every instance's CG barrier [2], kBarStride apart
  DevScalars *hsc = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool solved = false;
};

namespace {

void free_batch(iugkp_batch *b)
{
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto &ih : b->insts) ih.release();
  if (b->d_insts) (void)hipFree(b->d_insts);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->hsc) (void)hipHostFree(b->hsc);
  for (auto *q : {&b->pool, &b->mg_pool}) {
    if (q->h_off) (void)hipHostFree(q->h_off);
    if (q->h_jobs) (void)hipHostFree(q->h_jobs);
    if (q->d_off) (void)hipFree(q->d_off);
    if (q->d_jobs) (void)hipFree(q->d_jobs);
  }
  if (b->d_scs) (void)hipFree(b->d_scs);
  if (b->d_bars) (void)hipFree(b->d_bars);
  if (b->d_mg_args) (void)hipFree(b->d_mg_args);
  if (b->d_clk) (void)hipFree(b->d_clk);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->own) (void)hipStreamDestroy(b->own);
  delete b;
}

// Tile sizes of a batch (A9's autotuner for the tile march).  One launch runs
// every instance's tiles; an instance's tiles are edge x edge emitter cells
// with 8 or 16 cells.  The device stamps each workgroup's start and end and
// its flights; for every instance of a class not yet measured the second
// replay runs edge 8 and the third edge 16, and the instance keeps the edge
// with the smaller device time per flight (the sum of its workgroups'
// durations over its flights: the compute-unit time it takes while the batch
// fills the GPU), which the process keeps for the class (the same key as the
// particle-step form).  The tallies do not depend on the tiles.
std::mutex g_tile_mu;
std::map<FormKey, int> g_tile_choice;

// every instance's tiles with its edge, the instances and the tile table
// uploaded, the largest instances first (their workgroups start early)
int batch_layout(iugkp_batch *b)
{
  const int n = static_cast<int>(b->insts.size());
  for (int i = 0; i < n; ++i) plan_tiles(b->insts[i], b->edge[i]);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return b->insts[a].tiles.size() * b->insts[a].d.N > b->insts[c].tiles.size() * b->insts[c].d.N;
  });
  int tile0 = 0;
  for (int i : order) {
    const int rc = upload_inst(b->insts[i], i, b->d_insts, b->d_tiles, tile0, b->stream);
    if (rc) return rc;
    b->tile_first[i] = tile0;
    b->tile_count[i] = static_cast<int>(b->insts[i].tiles.size());
    tile0 += b->tile_count[i];
  }
  b->n_tiles = tile0;
  return IUGKP_OK;
}

// device time per flight of each instance that ran in the last replay (its
// workgroups' stamps), into cost (-1 where no flight)
int read_tile_costs(iugkp_batch *b, const std::vector<char> &ran, std::vector<double> &cost)
{
  const int n = static_cast<int>(b->insts.size());
  HIP_TRY(hipMemcpy(b->h_clk.data(), b->d_clk, 3 * static_cast<size_t>(b->n_tiles) *
                                                  sizeof(unsigned long long),
                    hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) {
    if (!ran[i]) continue;
    double t = 0.0, f = 0.0;
    for (int k = b->tile_first[i]; k < b->tile_first[i] + b->tile_count[i]; ++k) {
      const unsigned long long *c = &b->h_clk[3 * static_cast<size_t>(k)];
      if (c[1] > c[0]) t += static_cast<double>(c[1] - c[0]);
      f += static_cast<double>(c[2]);
    }
    cost[i] = (f > 0.0) ? t / f : -1.0;
  }
  return IUGKP_OK;
}

int enqueue_batch_iteration(iugkp_batch *b);

// capture one iteration of the whole batch into b->exec (again after a
// change of tiles)
int capture_batch(iugkp_batch *b)
{
  hipStream_t s = b->own;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_batch_iteration(b);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(s, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  HIP_TRY(ce);
  b->graph = g;
  HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return IUGKP_OK;
}

// The per-iteration sequence of a batch; every kernel skips finished instances.
int enqueue_batch_iteration(iugkp_batch *b)
{
  hipStream_t s = b->own;
  const int n = static_cast<int>(b->insts.size());
  iugkp::prepare_kernel<<<dim3(cdiv(b->max_prep, 256), n), 256, 0, s>>>(b->d_insts, -1, 1);
  int rc = launch_march(b->d_insts, b->d_tiles, b->n_tiles, b->lds_max, 256, -1, 1, b->any_ev, s,
                        b->d_clk);
  if (rc) return rc;
  iugkp::reconstruct_y_kernel<<<dim3(cdiv(b->max_nx, 4), n), 256, 0, s>>>(b->d_insts, -1, 1);
  iugkp::reconstruct_x_kernel<<<dim3(cdiv(b->max_ny, 4), n), 256, 0, s>>>(b->d_insts, -1, 1);
  iugkp::update_kernel<<<dim3(b->max_nbc, n), 256, 0, s>>>(b->d_insts, 1);
  if (b->any_newton) {
    iugkp::zero_u32_kernel<<<cdiv(kBarStride * n, 256), 256, 0, s>>>(b->d_bars, kBarStride * n);
    if (b->pool.used)
      iugkp::cg_batch_kernel<<<b->pool.size, iugkp::kCgThreadsMax, b->pool.lds, s>>>(
          b->d_insts, b->pool.d_off, b->pool.d_jobs);
    if (b->mg_pool.used)
      iugkp::mgcg_batch_kernel<<<b->mg_pool.size, 64 * iugkp::kMgPoolWaves, b->mg_pool.lds, s>>>(
          b->mg_pool.d_off, b->mg_pool.d_jobs, b->d_mg_args);
    iugkp::newton_finish_kernel<<<dim3(b->max_nbe, n), 256, 0, s>>>(b->d_insts, 1);
  }
  iugkp::finish_kernel<<<n, 256, 0, s>>>(b->d_insts, 1);
  iugkp::accumulate_kernel<<<dim3(cdiv(b->max_out, 256), n), 256, 0, s>>>(b->d_insts, 1, -1);
  HIP_TRY(hipGetLastError());
  return IUGKP_OK;
}

// Autotuned group sizes of the multigrid pool.  One iteration of an instance
// of n cells on a group of G workgroups is modelled as a + c n / G
// microseconds (a: the group barriers and the levels every workgroup keeps,
// c: one finest-level cell on one workgroup); a and c are fitted by least
// squares to the measured duration of every multigrid job of every replay
// (the device clock at the job's start and end) and kept for the process,
// so a later batch starts from them.  Before a replay the groups are chosen
// for the shortest makespan M the pool can reach: an instance takes the
// smallest group that finishes its iterations within M, and M grows until
// the total work fits the pool (at 75% packing); the result of an instance
// does not depend on its group.
struct MgModel {
  double sx = 0, sy = 0, sxx = 0, sxy = 0, n = 0;   // fit sums, x = cells / G, y = us per iteration
  double a = 40.0, c = 0.02;                       // defaults before any measurement
  void add(double x, double y)
  {
    sx += x;
    sy += y;
    sxx += x * x;
    sxy += x * y;
    n += 1.0;
    const double det = n * sxx - sx * sx;
    if (n >= 3.0 && det > 1e-12 * n * sxx) {
      const double cf = (n * sxy - sx * sy) / det;
      const double af = (sy - cf * sx) / n;
      if (cf > 0.0 && af > 0.0) {
        a = af;
        c = cf;
      }
    }
  }
};
std::mutex g_mg_model_mu;
MgModel g_mg_model;                  // the process's fit, shared by every batch

void choose_mg_groups(iugkp_batch *b, const MgModel &mdl)
{
  const int n = static_cast<int>(b->insts.size());
  const double P = static_cast<double>(b->mg_pool.size);
  struct J {
    int i;
    double its, cells;
    int gmax;
  };
  std::vector<J> js;
  for (int i = 0; i < n; ++i) {
    const InstHost &ih = b->insts[i];
    const DevScalars &sc = b->hsc[i];
    if (!ih.d.newton || ih.mg_L == 0 || sc.state == 2) continue;
    const double its = sc.iter > 0 ? std::max(sc.cg_iters, 1) : std::min(20, ih.d.cg_max);
    js.push_back({i, its, static_cast<double>(ih.d.m.n_cells), b->mg_gmax[i]});
  }
  if (js.empty()) return;
  auto t = [&](const J &j, int G) { return mdl.a + mdl.c * j.cells / G; };
  auto group_for = [&](const J &j, double M) {
    const double per = M / j.its - mdl.a;
    if (!(per > 0.0)) return j.gmax;
    const int g = static_cast<int>(std::ceil(mdl.c * j.cells / per));
    return std::max(1, std::min(j.gmax, g));
  };
  auto work = [&](double M) {
    double w = 0.0;
    for (const J &j : js) {
      const int g = group_for(j, M);
      w += j.its * g * t(j, g);
    }
    return w;
  };
  double lo = 0.0;
  for (const J &j : js) lo = std::max(lo, j.its * t(j, j.gmax));
  double hi = lo;
  while (work(hi) > 0.75 * P * hi) hi *= 2.0;
  if (hi > lo)
    for (int k = 0; k < 40; ++k) {
      const double mid = 0.5 * (lo + hi);
      if (work(mid) > 0.75 * P * mid) lo = mid;
      else hi = mid;
    }
  for (const J &j : js) b->cg_G[j.i] = group_for(j, hi);
}

// List scheduling of the CG jobs of the instances still iterating onto the
// pool, longest first: each job takes the G contiguous workgroups that free up
// earliest (estimated from the previous CG iteration count of the instance, or
// four CG iterations per mesh row before the first one), and is appended to
// their job lists in that global order.  Returns the number of entries.
int schedule_cg(iugkp_batch *b, bool mg_jobs)
{
  const int n = static_cast<int>(b->insts.size());
  iugkp_batch::Pool &pool = mg_jobs ? b->mg_pool : b->pool;
  const int P = pool.size;
  struct Job {
    double cost;
    int inst;
  };
  std::vector<Job> jobs;
  for (int i = 0; i < n; ++i) {
    const InstHost &ih = b->insts[i];
    const DevScalars &sc = b->hsc[i];
    if (!ih.d.newton || sc.state == 2 || (ih.mg_L > 0) != mg_jobs) continue;
    // a multigrid iteration passes 4 Lg + 2 group barriers (Lg grid levels),
    // a plain one one; before the first solve: 20 multigrid iterations, or
    // four plain ones per mesh row
    const bool mg = ih.mg_L > 0;
    const int prior = mg ? 20 : 4 * std::max(ih.d.m.nx, ih.d.m.ny);
    const double its = sc.iter > 0 ? std::max(sc.cg_iters, 1) : std::min(prior, ih.d.cg_max);
    double cost;
    if (mg) {
      std::lock_guard<std::mutex> lock(g_mg_model_mu);
      cost = its * (g_mg_model.a + g_mg_model.c * ih.d.m.n_cells / b->cg_G[i]);
    } else {
      cost = its * (b->cg_G[i] > 1 ? 3.0 : 1.0) * 4.5;     // (a plain iteration: about 4.5 us)
    }
    jobs.push_back({cost, i});
  }
  std::stable_sort(jobs.begin(), jobs.end(), [](const Job &x, const Job &y) { return x.cost > y.cost; });
  std::vector<double> load(P, 0.0);
  std::vector<std::vector<iugkp::CgJob>> lists(P);
  std::deque<int> dq;
  for (const Job &jb : jobs) {
    const int G = b->cg_G[jb.inst];
    // window of G workgroups whose latest free time is smallest (sliding maximum)
    int best = 0;
    double best_t = 0.0;
    dq.clear();
    for (int k = 0; k < P; ++k) {
      while (!dq.empty() && load[dq.back()] <= load[k]) dq.pop_back();
      dq.push_back(k);
      if (dq.front() <= k - G) dq.pop_front();
      if (k >= G - 1) {
        const double t = load[dq.front()];
        if (k == G - 1 || t < best_t) {
          best_t = t;
          best = k - G + 1;
        }
      }
    }
    const double fin = best_t + jb.cost;
    for (int r = 0; r < G; ++r) {
      load[best + r] = fin;
      lists[best + r].push_back({jb.inst, r, G, b->cg_tb[jb.inst]});
    }
  }
  int e = 0;
  for (int k = 0; k < P; ++k) {
    pool.h_off[k] = e;
    for (const auto &x : lists[k]) pool.h_jobs[e++] = x;
  }
  pool.h_off[P] = e;
  return e;
}

}  // namespace

extern "C" {

int iugkp_batch_create(const iugkp_problem *const *problems, const iugkp_options *const *options,
                       int n, void *stream, iugkp_batch **out)
{
  if (!out || !problems || !options || n < 1) return fail(IUGKP_E_INVALID_ARG, "bad batch arguments");
  *out = nullptr;
  iugkp_batch *b = new iugkp_batch();
  b->stream = static_cast<hipStream_t>(stream);
  b->insts.resize(n);
  int mem_kind = -1;
  for (int i = 0; i < n; ++i) {
    if (!problems[i] || !options[i]) {
      free_batch(b);
      return fail(IUGKP_E_INVALID_ARG, "NULL problem or options in the batch");
    }
    if (mem_kind < 0) mem_kind = problems[i]->mem_kind;
    if (problems[i]->mem_kind != mem_kind) {
      free_batch(b);
      return fail(IUGKP_E_INVALID_ARG, "all problems of a batch must use the same mem_kind");
    }
    const int rc = setup_instance(problems[i], options[i], b->stream, false, b->insts[i]);
    if (rc) {
      free_batch(b);
      return rc;
    }
    InstHost &ih = b->insts[i];
    const Mesh &m = ih.d.m;
    // (the table holds the edge-8 tiles, the most; the LDS window of either edge)
    plan_tiles(ih, 16);
    b->lds_max = std::max(b->lds_max, ih.lds_bytes);
    plan_tiles(ih, kTileX);
    b->n_tiles += static_cast<int>(ih.tiles.size());
    b->lds_max = std::max(b->lds_max, ih.lds_bytes);
    b->any_newton |= ih.d.newton;
    b->any_ev = b->any_ev || (ih.d.estimator != 0);
    b->max_prep = std::max({b->max_prep, m.n_emit, m.n_fx, m.n_fy, m.n_cells, (m.ny + 2) * m.nx});
    b->max_nx = std::max(b->max_nx, m.nx);
    b->max_ny = std::max(b->max_ny, m.ny);
    b->max_nbc = std::max(b->max_nbc, cdiv(m.n_cells, iugkp::kTree));
    b->max_nbe = std::max(b->max_nbe, cdiv(m.n_emit, iugkp::kTree));
    b->max_out = std::max({b->max_out, m.n_cells, m.n_fx, m.n_fy});
  }
  b->cg_G.assign(n, 0);
  b->cg_tb.assign(n, 0);
  b->mg_gmax.assign(n, 0);
  b->mg_last.assign(n, 0);
  if (b->any_newton) {
    // the pools: every workgroup resident at once (occupancy times CUs), so the
    // instance groups' barriers always make progress.  An instance's group:
    // one wave per tree block and at most kCgWavesMax blocks per workgroup
    // (register form), or, for rows too long for the LDS staging or groups
    // beyond one workgroup per CU, the global form on kCgGridMax workgroups;
    // with the multigrid preconditioner at most kCgGridMax workgroups of one
    // wave per 256-cell block of the finest level.
    int dev = 0, n_cu = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    b->clock_khz = static_cast<double>(khz);
    for (int i = 0; i < n; ++i) {
      const InstHost &ih = b->insts[i];
      if (!ih.d.newton) continue;
      const Mesh &m = ih.d.m;
      const int nbt = cdiv(m.n_cells, iugkp::kTree);
      if (ih.mg_L > 0) {
        const int G = std::max(1, std::min(std::min(cdiv(nbt, iugkp::kMgPoolWaves), kCgGridMax),
                                           n_cu));
        b->cg_G[i] = G;
        b->mg_gmax[i] = G;
        b->cg_tb[i] = 0;
        b->mg_pool.lds = std::max(b->mg_pool.lds, ih.mg_lds);
        b->mg_pool.max_jobs += G;
        b->mg_pool.used = true;
        continue;
      }
      const size_t hw = (m.dim == 2) ? m.nx : 1;
      int G = cdiv(nbt, iugkp::kCgWavesMax);
      int TB = cdiv(nbt, G);
      size_t lds = (static_cast<size_t>(TB) * iugkp::kTree + 2 * hw) * sizeof(double);
      int reg = 1;
      if (G > n_cu || lds > kCgLdsMax) {
        reg = 0;
        G = std::min(nbt, kCgGridMax);
        TB = cdiv(nbt, G);
        lds = 2 * hw * sizeof(double);
      }
      G = cdiv(nbt, TB);
      if (lds > kCgLdsMax) {
        free_batch(b);
        return fail(IUGKP_E_INVALID_ARG, "mesh rows too long for the Newton CG");
      }
      b->cg_G[i] = G;
      b->cg_tb[i] = TB | (reg ? iugkp::kCgJobReg : 0);
      b->pool.lds = std::max(b->pool.lds, lds);
      b->pool.max_jobs += G;
      b->pool.used = true;
    }
    for (auto *q : {&b->pool, &b->mg_pool}) {
      if (!q->used) continue;
      const void *kern = (q == &b->pool)
                             ? reinterpret_cast<const void *>(iugkp::cg_batch_kernel)
                             : reinterpret_cast<const void *>(iugkp::mgcg_batch_kernel);
      const int threads = (q == &b->pool) ? iugkp::kCgThreadsMax : 64 * iugkp::kMgPoolWaves;
      int per_cu = 0;
      HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, q->lds));
      if (per_cu < 1) {
        free_batch(b);
        return fail(IUGKP_E_DEVICE, "the batched CG kernel does not fit on a CU");
      }
      q->size = per_cu * n_cu;
      if (hipMalloc(reinterpret_cast<void **>(&q->d_off), (q->size + 1) * sizeof(int)) != hipSuccess ||
          hipMalloc(reinterpret_cast<void **>(&q->d_jobs),
                    std::max(q->max_jobs, 1) * sizeof(iugkp::CgJob)) != hipSuccess ||
          hipHostMalloc(reinterpret_cast<void **>(&q->h_off), (q->size + 1) * sizeof(int)) !=
              hipSuccess ||
          hipHostMalloc(reinterpret_cast<void **>(&q->h_jobs),
                        std::max(q->max_jobs, 1) * sizeof(iugkp::CgJob)) != hipSuccess) {
        free_batch(b);
        return fail(IUGKP_E_NOMEM, "allocation failed");
      }
    }
    for (int i = 0; i < n; ++i) {
      const InstHost &ih = b->insts[i];
      if (ih.d.newton && b->cg_G[i] > (ih.mg_L > 0 ? b->mg_pool.size : b->pool.size)) {
        free_batch(b);
        return fail(IUGKP_E_DEVICE, "a CG group exceeds the resident workgroups");
      }
    }
  }
  if (hipMalloc(reinterpret_cast<void **>(&b->d_insts), n * sizeof(Inst)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&b->d_tiles), b->n_tiles * sizeof(TileDesc)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&b->d_scs), n * sizeof(DevScalars)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&b->d_bars), kBarStride * n * sizeof(unsigned int)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&b->hsc), n * sizeof(DevScalars)) != hipSuccess) {
    free_batch(b);
    return fail(IUGKP_E_NOMEM, "allocation failed");
  }
  // gather the instances' scalars into one array (one copy per replay) and
  // give every instance its slot of the barrier array
  for (int i = 0; i < n; ++i) {
    InstHost &ih = b->insts[i];
    HIP_TRY(hipMemcpyAsync(b->d_scs + i, ih.d.sc, sizeof(DevScalars), hipMemcpyDeviceToDevice,
                           b->stream));
    ih.d.sc = b->d_scs + i;
    ih.d.cg_barrier = b->d_bars + kBarStride * i;
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  {
    // the multigrid jobs' arguments, one entry per instance (used by the
    // multigrid instances only)
    std::vector<iugkp::MGArgs> args(n);
    bool any_mg = false;
    for (int i = 0; i < n; ++i) {
      const InstHost &ih = b->insts[i];
      if (!ih.d.newton || ih.mg_L == 0) continue;
      any_mg = true;
      iugkp::MGArgs &ma = args[i];
      ma.lv = ih.mg_lv;
      ma.L = ih.mg_L;
      ma.Lg = ih.mg_Lg;
      ma.b = ih.d.rhs;
      ma.x = ih.d.cg_x;
      ma.p = ih.d.cg_p;
      ma.s = ih.d.cg_s;
      ma.w = ih.d.cg_w;
      ma.part = ih.cg_mpart;
      ma.tol2 = ih.d.tol2;
      ma.max_iters = ih.d.cg_max;
      ma.barrier = ih.d.cg_barrier;
      ma.sc = ih.d.sc;
      ma.r2 = ih.mg_r2;
      ma.s2 = ih.mg_s2;
      ma.band = ih.mg_band;
      ma.stage0 = ih.mg_stage0;
      ma.stage_n = ih.mg_stage_n;
    }
    if (any_mg) {
      if (hipMalloc(reinterpret_cast<void **>(&b->d_mg_args), n * sizeof(iugkp::MGArgs)) !=
          hipSuccess) {
        free_batch(b);
        return fail(IUGKP_E_NOMEM, "allocation failed");
      }
      HIP_TRY(hipMemcpyAsync(b->d_mg_args, args.data(), n * sizeof(iugkp::MGArgs),
                             hipMemcpyHostToDevice, b->stream));
      HIP_TRY(hipStreamSynchronize(b->stream));
    }
  }
  if (hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
    free_batch(b);
    return fail(IUGKP_E_DEVICE, "stream or event creation failed");
  }
  // tile edges: a class already measured in this process takes its edge; the
  // others are measured on the second and third replays
  const int max_tiles = b->n_tiles;
  b->edge.assign(n, kTileX);
  b->tile_first.assign(n, 0);
  b->tile_count.assign(n, 0);
  b->cost8.assign(n, -1.0);
  b->cost16.assign(n, -1.0);
  b->edge_known.assign(n, 0);
  b->tile_phase = 3;
  {
    std::lock_guard<std::mutex> lock(g_tile_mu);
    for (int i = 0; i < n; ++i) {
      const auto it = g_tile_choice.find(form_key(b->insts[i]));
      if (it != g_tile_choice.end()) {
        b->edge[i] = it->second;
        b->edge_known[i] = 1;
      } else {
        b->tile_phase = 0;
      }
    }
  }
  if (hipMalloc(reinterpret_cast<void **>(&b->d_clk), 3 * static_cast<size_t>(max_tiles) *
                                                          sizeof(unsigned long long)) != hipSuccess) {
    free_batch(b);
    return fail(IUGKP_E_NOMEM, "allocation failed");
  }
  b->h_clk.assign(3 * static_cast<size_t>(max_tiles), 0);
  const int rc = batch_layout(b);
  if (rc) {
    free_batch(b);
    return rc;
  }
  *out = b;
  return IUGKP_OK;
}

int iugkp_batch_tiles(iugkp_batch *b, int *edges)
{
  if (!b || !edges) return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  for (size_t i = 0; i < b->edge.size(); ++i) edges[i] = b->edge[i];
  return IUGKP_OK;
}

int iugkp_batch_tuning(iugkp_batch *b, double *per_iter_us, double *per_cell_us, int *groups)
{
  if (!b) return fail(IUGKP_E_INVALID_ARG, "batch is NULL");
  {
    std::lock_guard<std::mutex> lock(g_mg_model_mu);
    if (per_iter_us) *per_iter_us = g_mg_model.a;
    if (per_cell_us) *per_cell_us = g_mg_model.c;
  }
  if (groups)
    for (size_t i = 0; i < b->insts.size(); ++i)
      groups[i] = b->insts[i].d.newton ? b->cg_G[i] : 0;
  return IUGKP_OK;
}

int iugkp_batch_solve(iugkp_batch *b, double *const *T_out, double *const *qx_out,
                      double *const *qy_out, iugkp_stats *stats)
{
  if (!b || !T_out) return fail(IUGKP_E_INVALID_ARG, "bad batch arguments");
  if (b->solved) return fail(IUGKP_E_INVALID_ARG, "a batch is solved once");
  const int n = static_cast<int>(b->insts.size());
  hipStream_t s = b->own;
  for (int i = 0; i < n; ++i)
    if (!T_out[i]) return fail(IUGKP_E_INVALID_ARG, "T_out entries must not be NULL");
  // the batch stream starts after everything already queued on the caller's stream
  HIP_TRY(hipEventRecord(b->ev_in, b->stream));
  HIP_TRY(hipStreamWaitEvent(s, b->ev_in, 0));
  // capture one iteration of the whole batch, replay until every instance is done
  int rc = capture_batch(b);
  if (rc) return rc;
  int cap = 0;
  for (const auto &ih : b->insts) cap = std::max(cap, ih.d.max_iters + ih.d.avg_iters + 2);
  std::vector<char> ran(n, 0);          // instances that ran in the last replay
  for (int it = 0; it <= cap; ++it) {
    HIP_TRY(hipMemcpyAsync(b->hsc, b->d_scs, n * sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool all_done = true;
    for (int i = 0; i < n; ++i) all_done = all_done && (b->hsc[i].state == 2);
    // tile sizes: the costs of the replay just run, then the next phase
    if (it > 0 && b->tile_phase < 3 && !all_done) {
      if (b->tile_phase == 0) {
        b->tile_phase = 1;                   // (the first replay: first launches, not used)
      } else if (b->tile_phase == 1) {
        if ((rc = read_tile_costs(b, ran, b->cost8))) return rc;
        for (int i = 0; i < n; ++i)
          if (!b->edge_known[i]) b->edge[i] = 16;
        if ((rc = batch_layout(b)) || (rc = capture_batch(b))) return rc;
        b->tile_phase = 2;
      } else {
        if ((rc = read_tile_costs(b, ran, b->cost16))) return rc;
        std::lock_guard<std::mutex> lock(g_tile_mu);
        for (int i = 0; i < n; ++i) {
          if (b->edge_known[i]) continue;
          if (b->cost8[i] >= 0.0 && b->cost16[i] >= 0.0) {
            b->edge[i] = (b->cost16[i] < b->cost8[i]) ? 16 : kTileX;
            g_tile_choice[form_key(b->insts[i])] = b->edge[i];
          } else {
            b->edge[i] = kTileX;
          }
        }
        if ((rc = batch_layout(b)) || (rc = capture_batch(b))) return rc;
        b->tile_phase = 3;
      }
    }
    for (int i = 0; i < n; ++i) ran[i] = (b->hsc[i].state != 2) ? 1 : 0;
    if (b->mg_pool.used) {
      std::lock_guard<std::mutex> lock(g_mg_model_mu);
      for (int i = 0; i < n; ++i) {
        const DevScalars &sc = b->hsc[i];
        if (b->mg_last[i] > 0 && sc.cg_t1 > sc.cg_t0 && sc.cg_iters > 0 && b->clock_khz > 0.0) {
          const double us = static_cast<double>(sc.cg_t1 - sc.cg_t0) * 1e3 / b->clock_khz;
          g_mg_model.add(static_cast<double>(b->insts[i].d.m.n_cells) / b->mg_last[i],
                         us / sc.cg_iters);
        }
        b->mg_last[i] = 0;
      }
      if (!all_done) {
        choose_mg_groups(b, g_mg_model);
        for (int i = 0; i < n; ++i)
          if (b->insts[i].mg_L > 0 && b->insts[i].d.newton && b->hsc[i].state != 2)
            b->mg_last[i] = b->cg_G[i];
      }
    }
    if (all_done) break;
    for (auto *q : {&b->pool, &b->mg_pool}) {
      if (!q->used) continue;
      const int ne = schedule_cg(b, q == &b->mg_pool);
      HIP_TRY(hipMemcpyAsync(q->d_off, q->h_off, (q->size + 1) * sizeof(int),
                             hipMemcpyHostToDevice, s));
      if (ne > 0)
        HIP_TRY(hipMemcpyAsync(q->d_jobs, q->h_jobs, ne * sizeof(iugkp::CgJob),
                               hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipGraphLaunch(b->exec, s));
  }
  int worst = IUGKP_OK;
  for (int i = 0; i < n; ++i) {
    const InstHost &ih = b->insts[i];
    const DevScalars &sc = b->hsc[i];
    int status = IUGKP_OK;
    if (sc.state != 2) status = IUGKP_E_DEVICE;       // iteration cap of the replay loop
    else if (sc.err < 0) status = sc.err;
    else if (!sc.converged) status = IUGKP_W_NOT_CONVERGED;
    if (status < 0) {
      if (worst >= 0 || status < worst) worst = status;
    } else if (status > 0 && worst == IUGKP_OK) {
      worst = status;
    }
    if (status >= 0) {
      const double n_avg = ih.d.avg_iters > 0 ? static_cast<double>(ih.d.avg_iters) : 0.0;
      if ((rc = write_outputs(ih, n_avg, T_out[i], qx_out ? qx_out[i] : nullptr,
                              qy_out ? qy_out[i] : nullptr, s)))
        return rc;
    }
    if (stats) {
      iugkp_stats &st = stats[i];
      st = iugkp_stats{};
      st.status = status;
      st.iters = static_cast<int>(sc.iter);
      st.res = sc.res;
      st.flights = sc.flights;
      st.segments = sc.segments;
      st.crossings = sc.crossings;
      st.tot_flights = sc.tot_flights;
      st.tot_segments = sc.tot_segments;
      st.tot_crossings = sc.tot_crossings;
      st.cg_iters_last = sc.cg_iters;
      st.cg_iters_total = sc.cg_iters_total;
      st.fixed_point_F = ih.d.F;
      st.n_per_emitter = ih.d.N;
      st.n_emitters = ih.d.m.n_emit;
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipEventRecord(b->ev_out, s));
  HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_out, 0));
  b->solved = true;
  if (worst < 0) fail(worst, "at least one instance of the batch failed (see stats[i].status)");
  return worst;
}

void iugkp_batch_destroy(iugkp_batch *b)
{
  if (b && b->stream) (void)hipStreamSynchronize(b->stream);
  free_batch(b);
}

}  // extern "C"
