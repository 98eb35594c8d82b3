// iugkp.hip -- C ABI of the gfx950 IUGKP solver (declarations in include/iugkp.h).
//
// One translation unit: device kernels (kernels.hpp), set-up arithmetic
// (host_math.hpp), the single-problem driver and the batched driver
// (batch.hpp).  Built with -ffp-contract=off and no fast-math so that every
// floating-point result is fixed by IEEE binary64 semantics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/iugkp.h"
#include "host_math.hpp"
#include "kernels.hpp"

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

constexpr int kCgGridMax = 64;
constexpr size_t kCgLdsMax = 48 * 1024;      // dynamic LDS of the CG kernel

void *cg_kernel_for(int J)
{
  switch (J) {
    case 1: return reinterpret_cast<void *>(iugkp::cg_kernel<1>);
    case 2: return reinterpret_cast<void *>(iugkp::cg_kernel<2>);
    case 4: return reinterpret_cast<void *>(iugkp::cg_kernel<4>);
    default: return reinterpret_cast<void *>(iugkp::cg_kernel<0>);
  }
}
constexpr int kTileX = 8, kTileY = 8;        // emitter tile of one workgroup (cells)
constexpr int kWallSeg = 8;                  // wall faces per workgroup
constexpr int kWindowHalo = 12;              // window margin around a tile (cells)
constexpr size_t kLdsWordsMax = 6144;        // 48 KB of 64-bit tallies per workgroup
constexpr int kLdsWallsMax = 1024;

inline int cdiv(long long a, long long b) { return static_cast<int>((a + b - 1) / b); }

template <class T>
hipError_t dalloc(T **p, size_t n)
{
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
}

}  // namespace

using iugkp::DevScalars;
using iugkp::Mesh;

struct iugkp_handle {
  hipStream_t stream = nullptr;
  Mesh m{};
  double t_ref = 0, cv = 0, vg = 0, tau_min = 0, lam_min = 0, V = 0;
  int F = 0;
  uint32_t N = 1;
  uint32_t n_particles = 0;
  int has_null = 0;
  int mem_kind = IUGKP_MEM_HOST;
  iugkp_options opt{};
  int block = 256;
  // device memory
  double *tau = nullptr, *ratio = nullptr, *E = nullptr, *E_half = nullptr, *rhs = nullptr;
  double *Dx = nullptr, *Dy = nullptr, *gx = nullptr, *gy = nullptr, *diag = nullptr;
  double *cg_x = nullptr, *cg_r = nullptr, *cg_w = nullptr, *cg_p = nullptr, *cg_s = nullptr;
  double *cg_pub = nullptr;
  double *part = nullptr, *part_a = nullptr, *part_b = nullptr;
  unsigned long long *gpart = nullptr;
  unsigned int *cg_barrier = nullptr;
  long long *G = nullptr, *base = nullptr;
  uint32_t *rem = nullptr;
  long long *D = nullptr, *W = nullptr, *Phix = nullptr, *Phiy = nullptr, *B = nullptr;
  long long *dB = nullptr;
  iugkp::TileDesc *tiles = nullptr;
  int n_tiles = 0, WX = 1, WY = 1, lds_walls = 0;
  size_t lds_bytes = 0;
  double *acc_E = nullptr, *acc_x = nullptr, *acc_y = nullptr;
  double *out_T = nullptr, *out_qx = nullptr, *out_qy = nullptr;
  DevScalars *dsc = nullptr;
  DevScalars *hsc = nullptr;   // pinned host mirror
  int cg_grid = 1, cg_tb = 1, cg_j = 1;
  size_t cg_lds = 0;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // host state
  uint32_t iter = 0;
  double d0 = 0.0, res = 0.0;
  std::vector<double> res_hist;
  iugkp_stats st{};
  bool last_faces = false;
};

namespace {

int check_problem(const iugkp_problem *p)
{
  if (!p) return fail(IUGKP_E_INVALID_ARG, "problem is NULL");
  if (p->dim != 1 && p->dim != 2) return fail(IUGKP_E_INVALID_ARG, "dim must be 1 or 2");
  if (p->nx < 1 || p->ny < 1 || (p->dim == 1 && p->ny != 1))
    return fail(IUGKP_E_INVALID_ARG, "bad mesh size");
  if ((long long)p->nx * p->ny > (1ll << 30)) return fail(IUGKP_E_INVALID_ARG, "mesh too large");
  if (!(p->dx > 0) || !(p->dy > 0) || !std::isfinite(p->dx) || !std::isfinite(p->dy))
    return fail(IUGKP_E_INVALID_ARG, "cell sizes must be positive and finite");
  if (!(p->cv > 0) || !(p->vg > 0) || !std::isfinite(p->cv) || !std::isfinite(p->vg) ||
      !std::isfinite(p->t_ref))
    return fail(IUGKP_E_INVALID_ARG, "cv, vg must be positive, t_ref finite");
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
                   const std::vector<double> &T0)
{
  double maxabs = 0.0;
  for (double tw : wall_T) maxabs = std::max(maxabs, std::fabs(p->cv * (tw - p->t_ref)));
  for (double t : T0) maxabs = std::max(maxabs, std::fabs(p->cv * (t - p->t_ref)));
  const double lam_min = p->vg * tau_min;
  const double vol = static_cast<double>(p->nx * p->ny) * (p->dx * p->dy);
  const double area = (p->dim == 2) ? ((2.0 * p->ny) * p->dy + (2.0 * p->nx) * p->dx) : 2.0;
  const double total = vol + (lam_min * area) / 4.0;
  const double B = (4.0 * maxabs) * total;
  if (!(B > 0.0)) return 62;
  int e = 0;
  const double mant = std::frexp(B, &e);
  return 62 - ((mant == 0.5) ? e - 1 : e);
}

void free_handle(iugkp_handle *h)
{
  if (!h) return;
  void *bufs[] = {h->tau, h->ratio, h->E, h->E_half, h->rhs, h->Dx, h->Dy, h->gx, h->gy,
                  h->diag, h->cg_x, h->cg_r, h->cg_w, h->cg_p, h->cg_s, h->cg_pub, h->part,
                  h->part_a, h->gpart, h->cg_barrier, h->G, h->base, h->rem, h->D, h->W, h->Phix, h->Phiy,
                  h->B, h->dB, h->tiles, h->acc_E, h->acc_x, h->acc_y, h->out_T, h->out_qx, h->out_qy, h->dsc};
  for (void *b : bufs)
    if (b) (void)hipFree(b);
  if (h->hsc) (void)hipHostFree(h->hsc);
  for (auto &e : h->ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
}

int launch_march(iugkp_handle *h, uint32_t slot, int faces)
{
  iugkp::MarchArgs a;
  a.m = h->m;
  a.lam_min = h->lam_min;
  a.N = h->N;
  a.slot = slot;
  a.key0 = static_cast<uint32_t>(h->opt.seed);
  a.key1 = static_cast<uint32_t>(h->opt.seed >> 32);
  a.faces = faces;
  a.has_null = h->has_null;
  a.WX = h->WX;
  a.WY = h->WY;
  a.lds_walls = h->lds_walls;
  a.tiles = h->tiles;
  a.base = h->base;
  a.rem = h->rem;
  a.ratio = h->ratio;
  a.D = h->D;
  a.W = h->W;
  a.Phiy = h->Phiy;
  a.dB = h->dB;
  a.B = h->B;
  a.sc = h->dsc;
  const int grid = h->n_tiles;
  const size_t sh = h->lds_bytes;
  HIP_TRY(hipEventRecord(h->ev[0], h->stream));
  switch (h->block) {
    case 64: iugkp::march_kernel<64><<<grid, 64, sh, h->stream>>>(a); break;
    case 128: iugkp::march_kernel<128><<<grid, 128, sh, h->stream>>>(a); break;
    case 512: iugkp::march_kernel<512><<<grid, 512, sh, h->stream>>>(a); break;
    case 1024: iugkp::march_kernel<1024><<<grid, 1024, sh, h->stream>>>(a); break;
    default: iugkp::march_kernel<256><<<grid, 256, sh, h->stream>>>(a); break;
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(h->ev[1], h->stream));
  if (faces) {
    if (h->m.dim == 2)
      iugkp::reconstruct_y_kernel<<<cdiv(h->m.nx, 256), 256, 0, h->stream>>>(h->m, h->dB, h->Phiy);
    iugkp::reconstruct_x_kernel<<<cdiv(h->m.ny, 256), 256, 0, h->stream>>>(h->m, h->G, h->D, h->Phiy,
                                                                         h->B, h->Phix);
    HIP_TRY(hipGetLastError());
  }
  return IUGKP_OK;
}

// Tile table and LDS window: the whole domain when its tallies fit in LDS,
// otherwise a window of the tile plus a margin, placed inside the domain.
void plan_tiles(iugkp_handle *h, std::vector<iugkp::TileDesc> &tiles)
{
  const Mesh &m = h->m;
  h->lds_walls = (m.n_b <= kLdsWallsMax) ? 1 : 0;
  const size_t whole = iugkp::window_words(m.nx, m.ny, h->has_null, h->lds_walls, m.n_b);
  bool whole_domain = whole <= kLdsWordsMax;
  if (whole_domain) {
    h->WX = m.nx;
    h->WY = m.ny;
  } else {
    h->WX = std::min(m.nx, kTileX + 2 * kWindowHalo);
    h->WY = std::min(m.ny, kTileY + 2 * kWindowHalo);
  }
  auto place = [](int lo, int extent, int W, int n) {
    // window of size W covering [lo, lo + extent) as centrally as the domain allows
    int w0 = lo - (W - extent) / 2;
    if (w0 > n - W) w0 = n - W;
    if (w0 < 0) w0 = 0;
    return w0;
  };
  for (int ty = 0; ty < m.ny; ty += kTileY)
    for (int tx = 0; tx < m.nx; tx += kTileX) {
      iugkp::TileDesc t{};
      t.kind = 0;
      t.x0 = tx;
      t.y0 = ty;
      t.ex = std::min(kTileX, m.nx - tx);
      t.ey = std::min(kTileY, m.ny - ty);
      t.wx0 = whole_domain ? 0 : place(tx, t.ex, h->WX, m.nx);
      t.wy0 = whole_domain ? 0 : place(ty, t.ey, h->WY, m.ny);
      tiles.push_back(t);
    }
  // wall segments: left rows, right rows, bottom columns, top columns
  auto wall = [&](int b_first, int count, int along_x, int side_hi) {
    for (int s0 = 0; s0 < count; s0 += kWallSeg) {
      iugkp::TileDesc t{};
      t.kind = 1;
      t.x0 = b_first + s0;
      t.ex = std::min(kWallSeg, count - s0);
      t.ey = 1;
      if (whole_domain) {
        t.wx0 = 0;
        t.wy0 = 0;
      } else if (along_x) {   // bottom / top wall: segment along x
        t.wx0 = place(s0, t.ex, h->WX, m.nx);
        t.wy0 = side_hi ? m.ny - h->WY : 0;
      } else {                // left / right wall: segment along y
        t.wy0 = place(s0, t.ex, h->WY, m.ny);
        t.wx0 = side_hi ? m.nx - h->WX : 0;
      }
      tiles.push_back(t);
    }
  };
  wall(0, m.ny, 0, 0);
  wall(m.ny, m.ny, 0, 1);
  if (m.dim == 2) {
    wall(2 * m.ny, m.nx, 1, 0);
    wall(2 * m.ny + m.nx, m.nx, 1, 1);
  }
  h->n_tiles = static_cast<int>(tiles.size());
  h->lds_bytes = iugkp::window_words(h->WX, h->WY, h->has_null, h->lds_walls, m.n_b) * sizeof(long long);
}

// One iteration on the handle's stream; leaves the new scalars in h->hsc.
int iterate(iugkp_handle *h, int faces)
{
  const Mesh &m = h->m;
  const uint32_t slot = (h->opt.rng_mode == IUGKP_RNG_CRN) ? h->opt.rng_epoch : h->iter;
  const int nprep = std::max(std::max(std::max(m.n_emit, m.n_fx), std::max(m.n_fy, m.n_cells)),
                             (m.ny + 2) * m.nx);
  iugkp::Tallies t{h->D, h->W, h->Phix, h->Phiy, h->B};
  iugkp::prepare_kernel<<<cdiv(nprep, 256), 256, 0, h->stream>>>(m, h->G, h->N, h->base, h->rem,
                                                                  t, h->dB, faces, h->dsc);
  HIP_TRY(hipGetLastError());
  int rc = launch_march(h, slot, faces);   // records ev[0] / ev[1] around the march kernel
  if (rc) return rc;
  const int nbc = cdiv(m.n_cells, iugkp::kTree);
  iugkp::UpdateArgs ua{m.n_cells, h->F, h->has_null, h->opt.newton, h->V, h->D, h->W,
                       h->E, h->E_half, h->rhs, h->G, h->part, h->dsc};
  iugkp::update_kernel<<<nbc, 256, 0, h->stream>>>(ua);
  HIP_TRY(hipGetLastError());
  const int first = (h->iter == 0);
  if (h->opt.newton) {
    iugkp::CGArgs ca;
    ca.m = m;
    ca.gx = h->gx;
    ca.gy = h->gy;
    ca.diag = h->diag;
    ca.b = h->rhs;
    ca.x = h->cg_x;
    ca.gr = h->cg_r;
    ca.gw = h->cg_w;
    ca.gp = h->cg_p;
    ca.gs = h->cg_s;
    ca.pub = h->cg_pub;
    ca.part = h->part_a;
    ca.TB = h->cg_tb;
    ca.tol2 = h->opt.cg_tol * h->opt.cg_tol;
    ca.max_iters = h->opt.cg_max_iters;
    ca.barrier = h->cg_barrier;
    ca.sc = h->dsc;
    iugkp::zero_u32_kernel<<<1, 64, 0, h->stream>>>(h->cg_barrier, 2);
    HIP_TRY(hipEventRecord(h->ev[2], h->stream));
    // every workgroup must be resident for the grid barrier: the cooperative
    // launch refuses a grid that does not fit instead of letting it hang
    void *args[] = {&ca};
    HIP_TRY(hipLaunchCooperativeKernel(cg_kernel_for(h->cg_j), dim3(h->cg_grid),
                                       dim3(iugkp::kCgThreads), args, h->cg_lds, h->stream));
    HIP_TRY(hipEventRecord(h->ev[3], h->stream));
    const int nbe = cdiv(m.n_emit, iugkp::kTree);
    iugkp::NewtonFinishArgs na{m.n_cells, m.n_emit, h->F, h->V, h->E_half, h->cg_x,
                               h->ratio, h->E, h->G, h->part, h->gpart, h->dsc};
    iugkp::newton_finish_kernel<<<nbe, 256, 0, h->stream>>>(na);
    HIP_TRY(hipGetLastError());
    iugkp::finish_kernel<<<1, 256, 0, h->stream>>>(h->part, nbc, h->gpart, nbe, first, h->dsc);
  } else {
    iugkp::finish_kernel<<<1, 256, 0, h->stream>>>(h->part, nbc, nullptr, 0, first, h->dsc);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(h->hsc, h->dsc, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
  h->st.ms_march += ms;
  if (h->opt.newton) {
    HIP_TRY(hipEventElapsedTime(&ms, h->ev[2], h->ev[3]));
    h->st.ms_cg += ms;
  }
  const DevScalars &s = *h->hsc;
  h->st.flights = s.flights;
  h->st.segments = s.segments;
  h->st.crossings = s.crossings;
  h->st.tot_flights += s.flights;
  h->st.tot_segments += s.segments;
  h->st.tot_crossings += s.crossings;
  if (h->opt.newton) {
    h->st.cg_iters_last = s.cg_iters;
    h->st.cg_iters_total += s.cg_iters;
  }
  if (first) h->d0 = s.d0;
  h->res = s.res;
  h->res_hist.push_back(s.res);
  h->iter++;
  h->last_faces = faces != 0;
  h->st.iters = static_cast<int>(h->iter);
  h->st.res = h->res;
  if (h->opt.newton && s.cg_status == -3)
    return fail(IUGKP_E_DEVICE, "CG grid barrier timed out");
  if (h->opt.newton && s.cg_status == -6) return fail(IUGKP_E_CG_BREAKDOWN, "CG breakdown");
  if (h->opt.newton && s.cg_status == -7)
    return fail(IUGKP_E_CG_NOT_CONVERGED, "CG did not converge within cg_max_iters");
  if (s.flags & 1) return fail(IUGKP_E_NONFINITE, "non-finite energy");
  if ((s.flags & 2) || (h->opt.newton && s.gsum > (1ull << 62)))
    return fail(IUGKP_E_FIXED_OVERFLOW, "emission energy exceeds the fixed-point budget");
  if (h->iter > 1 && h->res > 1e3) return fail(IUGKP_E_DIVERGED, "residual grew above 1e3");
  return IUGKP_OK;
}

__global__ void accumulate_kernel(int n_cells, int n_fx, int n_fy, int F, int reset,
                                  const double *E, const long long *Phix, const long long *Phiy,
                                  double *aE, double *ax, double *ay)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_cells) aE[i] = reset ? E[i] : aE[i] + E[i];
  if (i < n_fx) {
    const double v = ldexp(static_cast<double>(Phix[i]), -F);
    ax[i] = reset ? v : ax[i] + v;
  }
  if (i < n_fy) {
    const double v = ldexp(static_cast<double>(Phiy[i]), -F);
    ay[i] = reset ? v : ay[i] + v;
  }
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

int create_impl(const iugkp_problem *p, const iugkp_options *o, void *stream, iugkp_handle **out)
{
  int rc = check_problem(p);
  if (rc) return rc;
  rc = check_options(o);
  if (rc) return rc;
  const int nc = p->nx * p->ny;
  const int nb = 2 * p->ny + (p->dim == 2 ? 2 * p->nx : 0);
  std::vector<double> tau, wall, T0;
  if ((rc = fetch_host(p->tau, nc, p->mem_kind, tau))) return rc;
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
  const int ne = nc + nb;
  uint64_t N = o->particles_per_iter / static_cast<uint64_t>(ne);
  if (N < 1) N = 1;
  if (N * static_cast<uint64_t>(ne) > 0xFFFFFFFFull)
    return fail(IUGKP_E_INVALID_ARG, "particles per iteration must stay below 2^32");

  iugkp_handle *h = new iugkp_handle();
  h->stream = static_cast<hipStream_t>(stream);
  h->opt = *o;
  h->block = o->block_size ? o->block_size : 256;
  h->mem_kind = p->mem_kind;
  Mesh &m = h->m;
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
  h->t_ref = p->t_ref;
  h->cv = p->cv;
  h->vg = p->vg;
  h->tau_min = tmin;
  h->lam_min = p->vg * tmin;
  h->V = p->dx * p->dy;
  h->N = static_cast<uint32_t>(N);
  h->n_particles = static_cast<uint32_t>(N * ne);
  h->has_null = (tmax != tmin);
  h->F = scale_exponent(p, tmin, wall, T0);

  auto bail = [&](int code) {
    free_handle(h);
    return code;
  };
#define ALLOC(ptr, n)                                                          \
  if (dalloc(&(ptr), (n)) != hipSuccess) return bail(fail(IUGKP_E_NOMEM, "hipMalloc failed"));
  const int nbe = cdiv(ne, iugkp::kTree);
  ALLOC(h->tau, nc);
  ALLOC(h->ratio, nc);
  ALLOC(h->E, nc);
  ALLOC(h->E_half, nc);
  ALLOC(h->part, nbe);
  ALLOC(h->G, ne);
  ALLOC(h->base, ne);
  ALLOC(h->rem, ne);
  ALLOC(h->D, nc);
  ALLOC(h->W, nc);
  ALLOC(h->Phix, m.n_fx);
  ALLOC(h->Phiy, m.n_fy);
  ALLOC(h->B, nb);
  ALLOC(h->dB, (p->ny + 2) * p->nx);
  ALLOC(h->acc_E, nc);
  ALLOC(h->acc_x, m.n_fx);
  ALLOC(h->acc_y, m.n_fy);
  ALLOC(h->out_T, nc);
  ALLOC(h->out_qx, m.n_fx);
  ALLOC(h->out_qy, m.n_fy);
  ALLOC(h->dsc, 1);
  if (hipHostMalloc(reinterpret_cast<void **>(&h->hsc), sizeof(DevScalars)) != hipSuccess)
    return bail(fail(IUGKP_E_NOMEM, "hipHostMalloc failed"));
  for (auto &e : h->ev)
    if (hipEventCreate(&e) != hipSuccess) return bail(fail(IUGKP_E_DEVICE, "hipEventCreate failed"));
  if (o->newton) {
    ALLOC(h->rhs, nc);
    ALLOC(h->Dx, nc);
    ALLOC(h->Dy, nc);
    ALLOC(h->gx, m.n_fx);
    ALLOC(h->gy, m.n_fy);
    ALLOC(h->diag, nc);
    ALLOC(h->cg_x, nc);
    ALLOC(h->cg_r, nc);
    ALLOC(h->cg_w, nc);
    ALLOC(h->cg_p, nc);
    ALLOC(h->cg_s, nc);
    ALLOC(h->cg_pub, 6 * static_cast<size_t>(nc));
    ALLOC(h->part_a, 4 * static_cast<size_t>(cdiv(nc, iugkp::kTree)));
    ALLOC(h->gpart, nbe);
    ALLOC(h->cg_barrier, 2);
  }
#undef ALLOC
  hipStream_t s = h->stream;
  if (copy_in(h->tau, tau.data(), nc * sizeof(double), IUGKP_MEM_HOST, s)) return bail(IUGKP_E_DEVICE);
  {
    std::vector<iugkp::TileDesc> tiles;
    plan_tiles(h, tiles);
    if (dalloc(&h->tiles, tiles.size()) != hipSuccess) return bail(fail(IUGKP_E_NOMEM, "hipMalloc failed"));
    if (copy_in(h->tiles, tiles.data(), tiles.size() * sizeof(iugkp::TileDesc), IUGKP_MEM_HOST, s))
      return bail(IUGKP_E_DEVICE);
    HIP_TRY(hipStreamSynchronize(s));
  }
  double *dT0 = nullptr;
  if (!T0.empty()) {
    if (dalloc(&dT0, nc) != hipSuccess) return bail(fail(IUGKP_E_NOMEM, "hipMalloc failed"));
    if (copy_in(dT0, T0.data(), nc * sizeof(double), IUGKP_MEM_HOST, s)) return bail(IUGKP_E_DEVICE);
  }
  iugkp::init_cells_kernel<<<cdiv(nc, 256), 256, 0, s>>>(nc, h->cv, h->t_ref, h->tau_min, dT0,
                                                          h->tau, h->E, h->ratio);
  // wall emission E_w lambda_min A / 4 (cosine-law black walls), computed once
  std::vector<long long> gw(nb);
  bool ok = true;
  for (int b = 0; b < nb; ++b) {
    const double A = (b < 2 * p->ny) ? p->dy : p->dx;
    const double ew = p->cv * (wall[b] - p->t_ref);
    const double v = std::ldexp((ew * (h->lam_min * A)) / 4.0, h->F);
    if (!(std::fabs(v) <= 4611686018427387904.0)) {
      ok = false;
      break;
    }
    gw[b] = static_cast<long long>(std::rint(v));
  }
  if (!ok) {
    if (dT0) (void)hipFree(dT0);
    return bail(fail(IUGKP_E_FIXED_OVERFLOW, "wall emission exceeds the fixed-point range"));
  }
  if (copy_in(h->G + nc, gw.data(), nb * sizeof(long long), IUGKP_MEM_HOST, s)) return bail(IUGKP_E_DEVICE);
  int *dflag = nullptr;
  if (dalloc(&dflag, 1) != hipSuccess) return bail(fail(IUGKP_E_NOMEM, "hipMalloc failed"));
  (void)hipMemsetAsync(dflag, 0, sizeof(int), s);
  iugkp::emission_from_E_kernel<<<cdiv(nc, 256), 256, 0, s>>>(nc, h->F, h->V, h->E, h->ratio,
                                                              h->G, dflag);
  if (o->newton) {
    std::vector<double> dxv(nc), dyv(nc);
    if (p->diff_x) {
      if ((rc = fetch_host(p->diff_x, nc, p->mem_kind, dxv))) return bail(rc);
    } else {
      std::map<double, double> cache;
      for (int c = 0; c < nc; ++c) {
        auto it = cache.find(tau[c]);
        if (it == cache.end()) it = cache.emplace(tau[c], iugkp::d_eff(p->vg * tau[c], p->dx)).first;
        dxv[c] = it->second;
      }
    }
    if (p->dim == 2) {
      if (p->diff_y) {
        if ((rc = fetch_host(p->diff_y, nc, p->mem_kind, dyv))) return bail(rc);
      } else {
        std::map<double, double> cache;
        for (int c = 0; c < nc; ++c) {
          auto it = cache.find(tau[c]);
          if (it == cache.end()) it = cache.emplace(tau[c], iugkp::d_eff(p->vg * tau[c], p->dy)).first;
          dyv[c] = it->second;
        }
      }
    } else {
      dyv = dxv;
    }
    for (int c = 0; c < nc; ++c)
      if (!(dxv[c] > 0.0) || !std::isfinite(dxv[c]) || !(dyv[c] > 0.0) || !std::isfinite(dyv[c]))
        return bail(fail(IUGKP_E_INVALID_ARG, "Newton diffusion coefficients must be > 0"));
    if (copy_in(h->Dx, dxv.data(), nc * sizeof(double), IUGKP_MEM_HOST, s)) return bail(IUGKP_E_DEVICE);
    if (copy_in(h->Dy, dyv.data(), nc * sizeof(double), IUGKP_MEM_HOST, s)) return bail(IUGKP_E_DEVICE);
    HIP_TRY(hipStreamSynchronize(s));
    const int nf = std::max(m.n_fx, m.n_fy);
    iugkp::newton_operator_kernel<<<cdiv(nf, 256), 256, 0, s>>>(m, h->vg, h->tau, h->Dx, h->Dy,
                                                                 h->gx, h->gy, h->diag);
    iugkp::newton_diag_kernel<<<cdiv(nc, 256), 256, 0, s>>>(m, h->gx, h->gy, h->diag);
    // CG layout: at most kCgGridMax resident workgroups (the barrier cost grows
    // with the number of arrivals), whole 256-cell tree blocks per workgroup,
    // cell state in registers when four-block passes and LDS staging allow
    int dev = 0, n_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const int nbt = cdiv(nc, iugkp::kTree);
    int G = std::max(1, std::min(std::min(nbt, kCgGridMax), n_cu));
    const int TB = cdiv(nbt, G);
    G = cdiv(nbt, TB);
    const int passes = cdiv(TB, iugkp::kCgSlices);
    int J = passes <= 1 ? 1 : passes <= 2 ? 2 : passes <= 4 ? 4 : 0;
    size_t lds = (static_cast<size_t>(TB) * iugkp::kTree + 2 * static_cast<size_t>(p->nx)) * sizeof(double);
    if (J > 0 && lds > kCgLdsMax) J = 0;
    if (J == 0) lds = 2 * static_cast<size_t>(p->nx) * sizeof(double);
    if (lds > kCgLdsMax) return bail(fail(IUGKP_E_INVALID_ARG, "mesh rows too long for the Newton CG"));
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cg_kernel_for(J), iugkp::kCgThreads, lds));
    if (per_cu < 1 || G > per_cu * n_cu)
      return bail(fail(IUGKP_E_DEVICE, "CG workgroups cannot all be resident"));
    h->cg_grid = G;
    h->cg_tb = TB;
    h->cg_j = J;
    h->cg_lds = lds;
  }
  std::vector<long long> g(ne);
  int hflag = 0;
  HIP_TRY(hipMemcpyAsync(g.data(), h->G, ne * sizeof(long long), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (dT0) (void)hipFree(dT0);
  (void)hipFree(dflag);
  unsigned long long acc = 0;
  for (long long v : g) {
    const unsigned long long a = static_cast<unsigned long long>(v < 0 ? -v : v);
    acc += a;
    if (a > (1ull << 62) || acc > (1ull << 62)) hflag |= 2;
  }
  if (hflag & 2) return bail(fail(IUGKP_E_FIXED_OVERFLOW, "initial emission exceeds the fixed-point budget"));
  std::memset(h->hsc, 0, sizeof(DevScalars));
  HIP_TRY(hipMemcpyAsync(h->dsc, h->hsc, sizeof(DevScalars), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  h->st.fixed_point_F = h->F;
  h->st.n_per_emitter = h->N;
  h->st.n_emitters = ne;
  *out = h;
  return IUGKP_OK;
}

}  // namespace

extern "C" {

int iugkp_create(const iugkp_problem *problem, const iugkp_options *options, void *stream,
                 iugkp_handle **out)
{
  if (!out) return fail(IUGKP_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  return create_impl(problem, options, stream, out);
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

int iugkp_step(iugkp_handle *h, int n_iters)
{
  if (!h) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
  return iugkp_step_faces(h, n_iters, h->opt.tally_faces == IUGKP_FACES_EVERY);
}

int iugkp_solve(iugkp_handle *h, double *T_out, double *qx_out, double *qy_out,
                iugkp_stats *stats)
{
  if (!h || !T_out) return fail(IUGKP_E_INVALID_ARG, "bad handle or T_out");
  const Mesh &m = h->m;
  const int faces_each = (h->opt.tally_faces == IUGKP_FACES_EVERY);
  bool converged = false;
  int rc;
  while (static_cast<int>(h->iter) < h->opt.max_iters) {
    if ((rc = iterate(h, faces_each))) return rc;
    if (h->res < h->opt.res_tol) {
      converged = true;
      break;
    }
  }
  const int faces_out = (h->opt.tally_faces != IUGKP_FACES_OFF);
  const int nmax = std::max(std::max(m.n_cells, m.n_fx), m.n_fy);
  const int grid = cdiv(nmax, 256);
  double n_avg = 0.0;
  if (h->opt.avg_iters > 0) {
    for (int a = 0; a < h->opt.avg_iters; ++a) {
      if ((rc = iterate(h, faces_out))) return rc;
      accumulate_kernel<<<grid, 256, 0, h->stream>>>(m.n_cells, m.n_fx, m.n_fy, h->F, a == 0,
                                                    h->E, h->Phix, h->Phiy, h->acc_E, h->acc_x,
                                                    h->acc_y);
    }
    n_avg = static_cast<double>(h->opt.avg_iters);
  } else {
    if (h->opt.tally_faces == IUGKP_FACES_FINAL && (rc = iterate(h, 1))) return rc;
    accumulate_kernel<<<grid, 256, 0, h->stream>>>(m.n_cells, m.n_fx, m.n_fy, h->F, 1, h->E,
                                                  h->Phix, h->Phiy, h->acc_E, h->acc_x, h->acc_y);
  }
  const bool dev = (h->mem_kind == IUGKP_MEM_DEVICE);
  double *T = dev ? T_out : h->out_T;
  double *qx = qx_out ? (dev ? qx_out : h->out_qx) : nullptr;
  double *qy = (qy_out && m.n_fy) ? (dev ? qy_out : h->out_qy) : nullptr;
  output_kernel<<<grid, 256, 0, h->stream>>>(m.n_cells, m.n_fx, m.n_fy, n_avg, faces_out, h->t_ref,
                                            h->cv, m.dy * h->tau_min, m.dx * h->tau_min, h->acc_E,
                                            h->acc_x, h->acc_y, T, qx, qy);
  HIP_TRY(hipGetLastError());
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(T_out, h->out_T, m.n_cells * sizeof(double), hipMemcpyDeviceToHost,
                           h->stream));
    if (qx_out)
      HIP_TRY(hipMemcpyAsync(qx_out, h->out_qx, m.n_fx * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
    if (qy_out && m.n_fy)
      HIP_TRY(hipMemcpyAsync(qy_out, h->out_qy, m.n_fy * sizeof(double), hipMemcpyDeviceToHost,
                             h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (stats) *stats = h->st;
  return converged ? IUGKP_OK : IUGKP_W_NOT_CONVERGED;
}

int iugkp_get_tallies(iugkp_handle *h, int64_t *D, int64_t *W, int64_t *Phi_x, int64_t *Phi_y,
                      int64_t *B)
{
  if (!h) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
  const Mesh &m = h->m;
  int rc;
  if ((rc = copy_out(D, h->D, m.n_cells * 8, h->mem_kind, h->stream))) return rc;
  if ((rc = copy_out(W, h->has_null ? h->W : h->D, m.n_cells * 8, h->mem_kind, h->stream))) return rc;
  if ((rc = copy_out(Phi_x, h->Phix, m.n_fx * 8, h->mem_kind, h->stream))) return rc;
  if (m.n_fy && (rc = copy_out(Phi_y, h->Phiy, m.n_fy * 8, h->mem_kind, h->stream))) return rc;
  if ((rc = copy_out(B, h->B, m.n_b * 8, h->mem_kind, h->stream))) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  return IUGKP_OK;
}

int iugkp_get_state(iugkp_handle *h, uint32_t *iter, double *d0, double *E, int64_t *G)
{
  if (!h) return fail(IUGKP_E_INVALID_ARG, "handle is NULL");
  if (iter) *iter = h->iter;
  if (d0) *d0 = h->d0;
  int rc;
  if ((rc = copy_out(E, h->E, h->m.n_cells * 8, h->mem_kind, h->stream))) return rc;
  if ((rc = copy_out(G, h->G, h->m.n_emit * 8, h->mem_kind, h->stream))) return rc;
  HIP_TRY(hipStreamSynchronize(h->stream));
  return IUGKP_OK;
}

int iugkp_set_state(iugkp_handle *h, uint32_t iter, double d0, const double *E, const int64_t *G)
{
  if (!h || !E || !G) return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  const Mesh &m = h->m;
  std::vector<long long> g(m.n_emit);
  if (h->mem_kind == IUGKP_MEM_HOST) {
    std::memcpy(g.data(), G, m.n_emit * 8);
  } else {
    HIP_TRY(hipMemcpy(g.data(), G, m.n_emit * 8, hipMemcpyDeviceToHost));
  }
  unsigned long long acc = 0;
  for (long long v : g) {
    const unsigned long long a = static_cast<unsigned long long>(v < 0 ? -v : v);
    acc += a;
    if (a > (1ull << 62) || acc > (1ull << 62))
      return fail(IUGKP_E_FIXED_OVERFLOW, "restored emission exceeds the fixed-point budget");
  }
  int rc;
  if ((rc = copy_in(h->E, E, m.n_cells * 8, h->mem_kind, h->stream))) return rc;
  HIP_TRY(hipMemcpyAsync(h->G, g.data(), m.n_emit * 8, hipMemcpyHostToDevice, h->stream));
  h->hsc->d0 = d0;
  HIP_TRY(hipMemcpyAsync(&h->dsc->d0, &h->hsc->d0, sizeof(double), hipMemcpyHostToDevice,
                         h->stream));
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

double iugkp_d_eff(double lam, double delta) { return iugkp::d_eff(lam, delta); }

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
  if (n > 0)
    iugkp::philox_probe_kernel<<<cdiv(n, 256), 256, 0, s>>>(ctr, key0, key1, out, n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

int iugkp_dev_math(int op, const double *x, const double *y, double *out, int64_t n, void *stream)
{
  if (!x || !out || n < 0 || op < 0 || op > 5 || ((op == 3 || op == 5) && !y))
    return fail(IUGKP_E_INVALID_ARG, "bad arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n > 0) iugkp::math_probe_kernel<<<cdiv(n, 256), 256, 0, s>>>(op, x, y, out, n);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return IUGKP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched solves
// ---------------------------------------------------------------------------
struct iugkp_batch {
  std::vector<iugkp_handle *> h;
  hipStream_t stream = nullptr;
};

extern "C" {

int iugkp_batch_create(const iugkp_problem *const *problems, const iugkp_options *const *options,
                       int n, void *stream, iugkp_batch **out)
{
  if (!out || !problems || !options || n < 1) return fail(IUGKP_E_INVALID_ARG, "bad batch arguments");
  *out = nullptr;
  iugkp_batch *b = new iugkp_batch();
  b->stream = static_cast<hipStream_t>(stream);
  for (int i = 0; i < n; ++i) {
    iugkp_handle *h = nullptr;
    const int rc = create_impl(problems[i], options[i], stream, &h);
    if (rc) {
      for (auto *x : b->h) free_handle(x);
      delete b;
      return rc;
    }
    b->h.push_back(h);
  }
  *out = b;
  return IUGKP_OK;
}

int iugkp_batch_solve(iugkp_batch *b, double *const *T_out, double *const *qx_out,
                      double *const *qy_out, iugkp_stats *stats)
{
  if (!b || !T_out) return fail(IUGKP_E_INVALID_ARG, "bad batch arguments");
  int worst = IUGKP_OK;
  for (size_t i = 0; i < b->h.size(); ++i) {
    const int rc = iugkp_solve(b->h[i], T_out[i], qx_out ? qx_out[i] : nullptr,
                               qy_out ? qy_out[i] : nullptr, stats ? &stats[i] : nullptr);
    if (rc < 0) return rc;
    if (rc > 0) worst = rc;
  }
  return worst;
}

void iugkp_batch_destroy(iugkp_batch *b)
{
  if (!b) return;
  for (auto *h : b->h) iugkp_destroy(h);
  delete b;
}

}  // extern "C"
