// mgcg.hpp -- the Newton system A x = b (Sec. 3.3) solved by conjugate
// gradients preconditioned with one multigrid V-cycle, as one persistent
// cooperative launch.
//
// The hierarchy: level k+1 aggregates 2x2 cells of level k (NX = ceil(nx/2),
// NY = ceil(ny/2)) down to one cell; the coarse operator is the Galerkin
// product P^T A P for the piecewise-constant prolongation P, again a 3/5-point
// operator whose faces sum the fine faces they cover.  The V-cycle: two damped
// Jacobi sweeps (omega 0.8) from zero, the residual summed over each
// aggregate, the coarser V-cycle, the correction scaled by 1.8, two sweeps
// again; the one-cell level is solved exactly.  The CG is the single-reduction
// form of Chronopoulos and Gear with u = M r:
//   x = 0, r = b, u = M r, w = A u, gamma = (r, u), delta = (w, u)
//   repeat: p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s,
//           u = M r, w = A u, gamma' = (r, u), delta = (w, u), rho = (r, r);
//           stop if rho <= tol^2 (b, b); beta = gamma' / gamma,
//           alpha = gamma' / (delta - beta gamma' / alpha)
// Every operation is written in the order the host-side definition fixes, so
// the result does not depend on the launch shape.
//
// Work split.  Levels with more than kMgLocalMax cells ("grid levels") are
// spread over all G workgroups: wave v of the group takes the 256-cell blocks
// v, v + G waves, ... of the level, lane l the cells l + 64 q of a block.  A
// phase reads what other workgroups wrote in the phase before it, behind a
// group barrier, with coherent loads and stores.  Per grid level the descent
// takes two phases (second pre-sweep; residual and restriction, which also
// does the first sweep of the next level) and the ascent two (correction with
// the first post-sweep; second post-sweep, which for a level whose finer
// level has at most one cell per thread is recomputed where that level reads
// it instead).  The remaining small levels run
// redundantly in every workgroup's LDS, so the coarse solve needs no barrier
// of its own and its result is at hand wherever the next grid level needs it.
#pragma once

#include <type_traits>

namespace iugkp {

constexpr double kMgOmega = 0.8;        // damped Jacobi weight
constexpr double kMgScale = 1.8;        // coarse-correction scale
constexpr int kMgLevelsMax = 40;
constexpr int kMgLocalMax = 1024;       // levels up to this size live in LDS

struct MGLevel {
  int nx, ny, n, has_y;
  const double *gx, *gy, *diag;         // operator of the level
  double *b, *xa, *xb, *xd, *e;         // grid levels (level 0: b = r, e = u)
  int lb, lx, lt, lc;                   // LDS levels: offsets (doubles) of b, x, t and
                                        // of the rows (3 doubles per cell)
};

struct MGArgs {
  const MGLevel *lv;                    // [L] level table
  int L, Lg;                            // levels; levels 0..Lg-1 are grid levels
  const double *b;                      // right-hand side
  double *x, *p, *s, *w;                // solution and the own-cell CG state
  double *part;                         // [nb][3] block sums of (r, u), (w, u), (r, r)
  double tol2;
  int max_iters;
  unsigned int *barrier;                // [2], zero at the start of the solve
  DevScalars *sc;
  // the banded form (mgband.hpp): second buffers of r and s, and the dynamic
  // LDS layout, [stage0) the coarse result kept across a band phase, then
  // stage_n doubles holding the LDS levels or a band window's staging
  double *r2, *s2;
  int band, stage0, stage_n;
};

// Row c of A_k: the diagonal, the four face conductances and the neighbour
// indices, an absent neighbour's index clamped to c itself.  Every load is
// unconditional, so a cell's loads issue together instead of one latency per
// neighbour.
struct MGRow {
  double dg, gl, gr, gd, gu;
  int jl, jr, jd, ju;
  int ix, iy;
  unsigned m;                           // left, right, down, up neighbour present
};

__device__ __forceinline__ void mg_row_index(MGRow &r, int nx, int ny, int ix, int iy)
{
  const int c = iy * nx + ix;
  r.ix = ix;
  r.iy = iy;
  r.m = (ix > 0 ? 1u : 0u) | (ix < nx - 1 ? 2u : 0u) | (iy > 0 ? 4u : 0u) |
        (iy < ny - 1 ? 8u : 0u);
  r.jl = (r.m & 1u) ? c - 1 : c;
  r.jr = (r.m & 2u) ? c + 1 : c;
  r.jd = (r.m & 4u) ? c - nx : c;
  r.ju = (r.m & 8u) ? c + nx : c;
}

__device__ __forceinline__ MGRow mg_row_at(const MGLevel &l, int ix, int iy)
{
  const int nx = l.nx, c = iy * nx + ix;
  MGRow r;
  mg_row_index(r, nx, l.ny, ix, iy);
  const int fx = iy * (nx + 1) + ix;
  r.dg = l.diag[c];
  r.gl = l.gx[fx];
  r.gr = l.gx[fx + 1];
  r.gd = l.gy[l.has_y ? iy * nx + ix : 0];       // (1D: a valid dummy, never used)
  r.gu = l.gy[l.has_y ? (iy + 1) * nx + ix : 0];
  return r;
}

__device__ __forceinline__ MGRow mg_row(const MGLevel &l, int c)
{
  const int iy = c / l.nx;
  return mg_row_at(l, c - iy * l.nx, iy);
}

// the same row of an LDS level, whose coefficients sit in LDS as three per
// cell: the diagonal and the right and upper faces (a cell's left face is
// its left neighbour's right face, its lower face the one below's upper face;
// an absent neighbour's face is read at the cell itself and never used)
__device__ __forceinline__ MGRow mg_row_lds_at(const MGLevel &l, const double *lds, int ix, int iy)
{
  MGRow r;
  mg_row_index(r, l.nx, l.ny, ix, iy);
  const double *k = lds + l.lc;
  const int c = iy * l.nx + ix;
  r.dg = k[3 * c];
  r.gr = k[3 * c + 1];
  r.gu = k[3 * c + 2];
  r.gl = k[3 * r.jl + 1];
  r.gd = k[3 * r.jd + 2];
  return r;
}

__device__ __forceinline__ MGRow mg_row_lds(const MGLevel &l, const double *lds, int c)
{
  const int iy = c / l.nx;
  return mg_row_lds_at(l, lds, c - iy * l.nx, iy);
}

// aggregates (on a level of nxc columns) of the cell of row r and of its
// four neighbours (an absent one: the cell's own)
__device__ __forceinline__ void mg_parents(const MGRow &r, int nxc, int (&pc)[5])
{
  const int px = r.ix >> 1, py = r.iy >> 1;
  pc[0] = py * nxc + px;
  pc[1] = (r.m & 1u) ? py * nxc + ((r.ix - 1) >> 1) : pc[0];
  pc[2] = (r.m & 2u) ? py * nxc + ((r.ix + 1) >> 1) : pc[0];
  pc[3] = (r.m & 4u) ? ((r.iy - 1) >> 1) * nxc + px : pc[0];
  pc[4] = (r.m & 8u) ? ((r.iy + 1) >> 1) * nxc + px : pc[0];
}

// (A_k v)_c: diag v_c - g_l v_{c-1} - g_r v_{c+1} - g_dn v_{c-nx} - g_up v_{c+nx},
// absent neighbours skipped (their term computed on a clamped value and
// discarded)
template <class Get>
__device__ __forceinline__ double mg_apply_row(const MGRow &r, int c, Get v)
{
  const double vc = v(c), vl = v(r.jl), vr = v(r.jr), vd = v(r.jd), vu = v(r.ju);
  double acc = r.dg * vc;
  const double a1 = acc - r.gl * vl;
  acc = (r.m & 1u) ? a1 : acc;
  const double a2 = acc - r.gr * vr;
  acc = (r.m & 2u) ? a2 : acc;
  const double a3 = acc - r.gd * vd;
  acc = (r.m & 4u) ? a3 : acc;
  const double a4 = acc - r.gu * vu;
  acc = (r.m & 8u) ? a4 : acc;
  return acc;
}

// the same on values already loaded: v = {v_c, v_l, v_r, v_dn, v_up}
__device__ __forceinline__ double mg_apply_vals(const MGRow &r, const double (&v)[5])
{
  double acc = r.dg * v[0];
  const double a1 = acc - r.gl * v[1];
  acc = (r.m & 1u) ? a1 : acc;
  const double a2 = acc - r.gr * v[2];
  acc = (r.m & 2u) ? a2 : acc;
  const double a3 = acc - r.gd * v[3];
  acc = (r.m & 4u) ? a3 : acc;
  const double a4 = acc - r.gu * v[4];
  acc = (r.m & 8u) ? a4 : acc;
  return acc;
}

template <class Get>
__device__ __forceinline__ double mg_apply(const MGLevel &l, int c, Get v)
{
  return mg_apply_row(mg_row(l, c), c, v);
}

// Loads and stores of values other workgroups (SC = agent scope) or only the
// waves of this workgroup (SC = workgroup scope, a solve run by a single
// workgroup) write between barriers.
template <int SC>
__device__ __forceinline__ double mld(const double *p)
{
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, SC);
}
template <int SC>
__device__ __forceinline__ void mst(double *p, double v)
{
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, SC);
}

// Sums of the nb published NV-tuples (layout [nb][NV]) in the fixed order of
// the host-side definition: the 256-element tree over each chunk, then over
// the chunk sums (nb <= 65536).  Every thread gets every result.
template <int NV, int SC>
__device__ __forceinline__ void group_tree_n(const double *part, int nb, double *red,
                                             double (&out)[NV])
{
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int nch = (nb + kTree - 1) / kTree;
  auto chunk = [&](int k, double (&r)[NV]) {
    // (every load issued before the first tree)
    double v[NV][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = k * kTree + lane + 64 * q;
#pragma unroll
      for (int j = 0; j < NV; ++j) v[j][q] = i < nb ? mld<SC>(&part[NV * i + j]) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) r[j] = wave_tree256(v[j][0], v[j][1], v[j][2], v[j][3]);
  };
  if (nch == 1) {
    double r[NV];
    chunk(0, r);
#pragma unroll
    for (int j = 0; j < NV; ++j) out[j] = lane0(r[j]);
    return;
  }
  for (int k = wave; k < nch; k += nw) {
    double r[NV];
    chunk(k, r);
    if (lane == 0)
#pragma unroll
      for (int j = 0; j < NV; ++j) red[j * kTree + k] = r[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = lane + 64 * q;
      v[q] = k < nch ? red[j * kTree + k] : 0.0;
    }
    out[j] = lane0(wave_tree256(v[0], v[1], v[2], v[3]));
  }
  __syncthreads();
}

// the first damped Jacobi sweep, from zero: 0 + (omega b) / diag
__device__ __forceinline__ double mg_sweep_first(double bv, double dg)
{
  return 0.0 + (kMgOmega * bv) / dg;
}
struct MgV2 {
  double a, b;
};

// The level table copied into LDS (read from global memory at every pass, a
// descriptor cost a memory round trip before the pass could load its data).
// Ends with a workgroup barrier; the one before it waits for a previous solve
// of this workgroup to be done with the table.
__device__ __forceinline__ void mg_stage_levels(const MGLevel *src, int L, MGLevel *dst)
{
  constexpr int kW = static_cast<int>(sizeof(MGLevel) / sizeof(int));
  static_assert(sizeof(MGLevel) % sizeof(int) == 0, "level descriptors are whole words");
  __syncthreads();
  const int *from = reinterpret_cast<const int *>(src);
  int *to = reinterpret_cast<int *>(dst);
  for (int i = threadIdx.x; i < L * kW; i += blockDim.x) to[i] = from[i];
  __syncthreads();
}

// The cells i = tid, tid + nt, ... of [0, N), Q per thread at a time: the Q
// loads first (an index past the end replaced by the first), then the Q
// finishes, so that a thread's loads are in flight together.
template <int Q, class Ld, class Fin>
__device__ __forceinline__ void mg_cells(int N, Ld load, Fin finish)
{
  const int nt = static_cast<int>(blockDim.x);
  for (int i0 = static_cast<int>(threadIdx.x); i0 < N; i0 += Q * nt) {
    using V = decltype(load(0));
    V v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = i0 + q * nt;
      v[q] = load(i < N ? i : i0);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = i0 + q * nt;
      if (i < N) finish(i, v[q]);
    }
  }
}

// the five row coefficients of every cell of the LDS levels (no barrier)
__device__ __forceinline__ void mg_lds_rows(const MGLevel *lv, int Lg, int L, double *lds)
{
  for (int k = Lg; k < L; ++k) {
    const MGLevel F = lv[k];
    mg_cells<4>(
        F.n, [&](int i) { return mg_row(F, i); },
        [&](int i, const MGRow &r) {
          double *dst = lds + F.lc + 3 * i;
          dst[0] = r.dg;
          dst[1] = r.gr;
          dst[2] = r.gu;
        });
  }
}

// The V-cycle of the LDS levels Lg..L-1, run by every workgroup on its own
// copy: b of level Lg from global memory (b_global) or already in LDS; its
// result ends in level Lg's t vector.  Descent: b loaded with the first
// sweep; per level the second sweep, then the restriction with the next
// level's first sweep (the one-cell level: its exact solve).  Ascent: the
// correction fused into the first post-sweep (the neighbours' corrected
// values recomputed), the second post-sweep.  Each level's result ends in its
// t vector.
template <int SC>
__device__ __forceinline__ void mg_lds_cycle(const MGLevel *lv, int Lg, int L, double *lds,
                                             bool b_global)
{
  // an LDS level, two cells per thread at a time (computed, then stored),
  // then a workgroup barrier
  auto for_local = [&](int nl, auto compute, auto store) {
    const int bd = blockDim.x;
    for (int i0 = threadIdx.x; i0 < nl; i0 += 2 * bd) {
      const int i1 = i0 + bd;
      const auto v0 = compute(i0);
      const auto v1 = compute(i1 < nl ? i1 : i0);
      store(i0, v0);
      if (i1 < nl) store(i1, v1);
    }
    __syncthreads();
  };
  // a level of at most one cell per lane, run by wavefront 0 alone: its LDS
  // operations execute in order, so a pass needs no workgroup barrier
  auto for_wave = [&](int nl, auto compute, auto store) {
    const int i = static_cast<int>(threadIdx.x);
    const auto v = compute(i < nl ? i : 0);
    if (i < nl) store(i, v);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  const MGLevel T = lv[Lg];
  for_local(
      T.n,
      [&](int i) {
        const double bv = b_global ? mld<SC>(&T.b[i]) : lds[T.lb + i];
        return MgV2{bv, mg_sweep_first(bv, lds[T.lc + 3 * i])};
      },
      [&](int i, MgV2 v) {
        lds[T.lb + i] = v.a;
        if (L - 1 > Lg) lds[T.lx + i] = v.b;
        else lds[T.lt + i] = v.a / lds[T.lc + 3 * i];
      });
  // descent step at level k (second sweep, restriction with the next
  // level's first sweep) and ascent step (corrected first post-sweep,
  // second post-sweep), with `run` one of the two pass forms
  auto down = [&](int k, auto run) {
    const MGLevel F = lv[k], Cl = lv[k + 1];
    const double *B = lds + F.lb, *X = lds + F.lx;
    double *Tm = lds + F.lt;
    run(
        F.n,
        [&](int i) {
          const MGRow r = mg_row_lds(F, lds, i);
          const double t = B[i] - mg_apply_row(r, i, [&](int j) { return X[j]; });
          return X[i] + (kMgOmega * t) / r.dg;
        },
        [&](int i, double v) { Tm[i] = v; });
    const bool last = (k + 1 == L - 1);
    run(
        Cl.n,
        [&](int C) {
          const int J = C / Cl.nx, I = C - J * Cl.nx;
          double q[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int ix = 2 * I + (k & 1), iy = 2 * J + (k >> 1);
            const bool in = (ix < F.nx && iy < F.ny);
            const int cx = in ? ix : 2 * I, cy = in ? iy : 2 * J;
            const int f = cy * F.nx + cx;
            const MGRow r = mg_row_lds_at(F, lds, cx, cy);
            const double res = B[f] - mg_apply_row(r, f, [&](int j) { return Tm[j]; });
            q[k] = in ? res : 0.0;
          }
          return (q[0] + q[1]) + (q[2] + q[3]);
        },
        [&](int C, double v) {
          lds[Cl.lb + C] = v;
          const double dg = lds[Cl.lc + 3 * C];
          if (last) lds[Cl.lt + C] = v / dg;
          else lds[Cl.lx + C] = mg_sweep_first(v, dg);
        });
  };
  auto up = [&](int k, auto run) {
    const MGLevel F = lv[k], Cl = lv[k + 1];
    const double *B = lds + F.lb, *E = lds + Cl.lt;
    double *X = lds + F.lx, *Tm = lds + F.lt;
    run(
        F.n,
        [&](int i) {
          const MGRow r = mg_row_lds(F, lds, i);
          int pc[5];
          mg_parents(r, Cl.nx, pc);
          const int js[5] = {i, r.jl, r.jr, r.jd, r.ju};
          double xc5[5];
#pragma unroll
          for (int q = 0; q < 5; ++q) xc5[q] = Tm[js[q]] + kMgScale * E[pc[q]];
          const double t = B[i] - mg_apply_vals(r, xc5);
          return xc5[0] + (kMgOmega * t) / r.dg;
        },
        [&](int i, double v) { X[i] = v; });
    run(
        F.n,
        [&](int i) {
          const MGRow r = mg_row_lds(F, lds, i);
          const double t = B[i] - mg_apply_row(r, i, [&](int j) { return X[j]; });
          return X[i] + (kMgOmega * t) / r.dg;
        },
        [&](int i, double v) { Tm[i] = v; });
  };
  // the levels of at most 64 cells (from ks on) by wavefront 0 alone
  int ks = Lg;
  while (ks < L - 1 && lv[ks].n > 64) ++ks;
  for (int k = Lg; k < ks; ++k) down(k, for_local);
  if (ks < L - 1) {
    if (threadIdx.x < 64) {
      for (int k = ks; k < L - 1; ++k) down(k, for_wave);
      for (int k = L - 2; k >= ks; --k) up(k, for_wave);
    }
    __syncthreads();
  }
  for (int k = ks - 1; k >= Lg; --k) up(k, for_local);
}

// The preconditioned CG of one system, run by the G workgroups of a group of
// which this one is number bid (G = 1: one workgroup alone, its exchanges
// through workgroup-scope memory operations and workgroup barriers).
template <int SC>
__device__ __forceinline__ void mgcg_solve(const MGArgs &a, int G, int bid, double *lds,
                                           double *red, MGLevel *s_lv)
{
  const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int gwv = bid * nw + wave, gstride = G * nw;
  if (bid == 0 && threadIdx.x == 0) a.sc->cg_t0 = static_cast<unsigned long long>(wall_clock64());
  const int L = a.L, Lg = a.Lg;
  mg_stage_levels(a.lv, L, s_lv);
  const MGLevel *lv = s_lv;
  const MGLevel L0 = lv[0];
  const int n = L0.n, nb = (n + kTree - 1) / kTree;
  unsigned int epoch = 0;

  auto bar = [&]() -> bool {
    if (G == 1) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      return true;
    }
    return grid_barrier(a.barrier, epoch, G);
  };
  // The cells of a grid level this thread owns, Q of a block at a time: the Q
  // are computed first (an index past the end replaced by the block's first
  // cell), then the valid ones stored, so a batch's loads issue before its
  // first store.  Q trades loads in flight against registers.
  auto for_cells = [&](auto Qc, int nl, auto compute, auto store) {
    constexpr int Q = decltype(Qc)::value;
    const int nbl = (nl + kTree - 1) / kTree;
    for (int blk = gwv; blk < nbl; blk += gstride)
#pragma unroll 1
      for (int q0 = 0; q0 < 4; q0 += Q) {
        using R = decltype(compute(0));
        R v[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int c = blk * kTree + lane + 64 * (q0 + q);
          v[q] = compute(c < nl ? c : blk * kTree);
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int c = blk * kTree + lane + 64 * (q0 + q);
          if (c < nl) store(c, v[q]);
        }
      }
  };
  using Q1 = std::integral_constant<int, 1>;
  using Q2 = std::integral_constant<int, 2>;
  using Q4 = std::integral_constant<int, 4>;
  // A phase that touches no own-cell state: the cells of the level spread
  // over every thread of the group (consecutive threads, consecutive cells),
  // two at a time when the level has more cells than the group has threads.
  const int nthr = G * static_cast<int>(blockDim.x);
  const int tid = bid * static_cast<int>(blockDim.x) + static_cast<int>(threadIdx.x);
  auto for_flat = [&](auto Qmax, int nl, auto compute, auto store) {
    auto run = [&](auto Qc) {
      constexpr int Q = decltype(Qc)::value;
      for (int c0 = tid; c0 < nl; c0 += Q * nthr) {
        using R = decltype(compute(0));
        R v[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int c = c0 + q * nthr;
          v[q] = compute(c < nl ? c : c0);
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int c = c0 + q * nthr;
          if (c < nl) store(c, v[q]);
        }
      }
    };
    if (decltype(Qmax)::value > 1 && nl > nthr) run(std::integral_constant<int, 2>{});
    else run(std::integral_constant<int, 1>{});
  };
  auto sweep_first = [&](double bv, double dg) { return mg_sweep_first(bv, dg); };
  using V2 = MgV2;

  // rows of the LDS levels, once per solve
  mg_lds_rows(lv, Lg, L, lds);
  __syncthreads();

  // the V-cycle on r (published as lv[0].b, and lv[0].xa = the first sweep
  // when level 0 is a grid level); u ends in lv[0].e, or in LDS when Lg = 0
  auto vcycle = [&]() -> bool {
    for (int k = 0; k < Lg; ++k) {
      const MGLevel F = lv[k];
      for_flat(
          Q2{}, F.n,
          [&](int c) {
            auto xa = [&](int j) { return mld<SC>(&F.xa[j]); };
            const MGRow r = mg_row(F, c);
            const double t = mld<SC>(&F.b[c]) - mg_apply_row(r, c, xa);
            return xa(c) + (kMgOmega * t) / r.dg;
          },
          [&](int c, double v) { mst<SC>(&F.xb[c], v); });
      if (!bar()) return false;
      const MGLevel Cl = lv[k + 1];
      const bool grid_next = (k + 1 < Lg);
      for_flat(
          Q1{}, Cl.n,
          [&](int C) {
            // the four children (absent ones clamped to the first and
            // discarded): every row and value loaded before any arithmetic
            const int J = C / Cl.nx, I = C - J * Cl.nx;
            MGRow rw[4];
            double bv[4], xv[4][5];
            bool in[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int ix = 2 * I + (k & 1), iy = 2 * J + (k >> 1);
              in[k] = (ix < F.nx && iy < F.ny);
              const int cx = in[k] ? ix : 2 * I, cy = in[k] ? iy : 2 * J;
              const int f = cy * F.nx + cx;
              rw[k] = mg_row_at(F, cx, cy);
              bv[k] = mld<SC>(&F.b[f]);
              xv[k][0] = mld<SC>(&F.xb[f]);
              xv[k][1] = mld<SC>(&F.xb[rw[k].jl]);
              xv[k][2] = mld<SC>(&F.xb[rw[k].jr]);
              xv[k][3] = mld<SC>(&F.xb[rw[k].jd]);
              xv[k][4] = mld<SC>(&F.xb[rw[k].ju]);
            }
            double q[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const double res = bv[k] - mg_apply_vals(rw[k], xv[k]);
              q[k] = in[k] ? res : 0.0;
            }
            const double B = (q[0] + q[1]) + (q[2] + q[3]);
            return V2{B, sweep_first(B, Cl.diag[C])};
          },
          [&](int C, V2 v) {
            mst<SC>(&Cl.b[C], v.a);
            if (grid_next) mst<SC>(&Cl.xa[C], v.b);
          });
      if (!bar()) return false;
    }
    // the LDS levels, in every workgroup
    mg_lds_cycle<SC>(lv, Lg, L, lds, true);
    // Ascent.  The last sweep of a grid level whose finer level has at most
    // one cell per thread is not stored: that finer level's first post-sweep
    // recomputes it at the (at most three) aggregates its cell and neighbours
    // use, with the same operations, so it needs no phase and no barrier of
    // its own.
    auto fused = [&](int k) { return k >= 1 && lv[k - 1].n <= nthr; };
    for (int k = Lg - 1; k >= 0; --k) {
      const MGLevel F = lv[k], Cl = lv[k + 1];
      const bool recompute = (k + 1 < Lg) && fused(k + 1);
      // the coarse level's final value at aggregate P: from LDS, or the
      // second post-sweep of a grid level evaluated here
      auto e_grid = [&](int P) {
        const MGRow rc = mg_row(Cl, P);
        const double b = mld<SC>(&Cl.b[P]);
        double v5[5];
        v5[0] = mld<SC>(&Cl.xd[P]);
        v5[1] = mld<SC>(&Cl.xd[rc.jl]);
        v5[2] = mld<SC>(&Cl.xd[rc.jr]);
        v5[3] = mld<SC>(&Cl.xd[rc.jd]);
        v5[4] = mld<SC>(&Cl.xd[rc.ju]);
        const double t = b - mg_apply_vals(rc, v5);
        return v5[0] + (kMgOmega * t) / rc.dg;
      };
      auto post1 = [&](auto FromLds) {
        // (one cell at a time when the coarse values are recomputed: three
        // rows and stencils of loads per cell)
        using QP = std::conditional_t<decltype(FromLds)::value == 2, Q1, Q2>;
        for_flat(
            QP{}, F.n,
            [&](int c) {
              // x after the coarse correction, x_b + s e(parent), on the cell
              // and its neighbours: loads first, then the arithmetic
              const MGRow r = mg_row(F, c);
              const int js[5] = {c, r.jl, r.jr, r.jd, r.ju};
              int pc[5];
              mg_parents(r, Cl.nx, pc);
              double xb5[5], e5[5];
#pragma unroll
              for (int q = 0; q < 5; ++q) xb5[q] = mld<SC>(&F.xb[js[q]]);
              if constexpr (decltype(FromLds)::value == 1) {
#pragma unroll
                for (int q = 0; q < 5; ++q) e5[q] = lds[Cl.lt + pc[q]];
              } else if constexpr (decltype(FromLds)::value == 0) {
#pragma unroll
                for (int q = 0; q < 5; ++q) e5[q] = mld<SC>(&Cl.e[pc[q]]);
              } else {
                // distinct aggregates: the cell's own, the one across an x
                // face (left or right) and the one across a y face
                const int px = (pc[1] != pc[0]) ? pc[1] : pc[2];
                const int py = (pc[3] != pc[0]) ? pc[3] : pc[4];
                const double e0 = e_grid(pc[0]), ex = e_grid(px), ey = e_grid(py);
                e5[0] = e0;
                e5[1] = (pc[1] == pc[0]) ? e0 : ex;
                e5[2] = (pc[2] == pc[0]) ? e0 : ex;
                e5[3] = (pc[3] == pc[0]) ? e0 : ey;
                e5[4] = (pc[4] == pc[0]) ? e0 : ey;
              }
              const double bc = mld<SC>(&F.b[c]);
              double xc5[5];
#pragma unroll
              for (int q = 0; q < 5; ++q) xc5[q] = xb5[q] + kMgScale * e5[q];
              const double t = bc - mg_apply_vals(r, xc5);
              return xc5[0] + (kMgOmega * t) / r.dg;
            },
            [&](int c, double v) { mst<SC>(&F.xd[c], v); });
      };
      // e of the coarse level: 1 from LDS, 0 stored by its last sweep, 2 recomputed
      if (k + 1 == Lg) post1(std::integral_constant<int, 1>{});
      else if (recompute) post1(std::integral_constant<int, 2>{});
      else post1(std::integral_constant<int, 0>{});
      if (!bar()) return false;
      if (fused(k)) continue;               // (recomputed by the next level)
      for_flat(
          Q2{}, F.n,
          [&](int c) {
            auto xd = [&](int j) { return mld<SC>(&F.xd[j]); };
            const MGRow r = mg_row(F, c);
            const double t = mld<SC>(&F.b[c]) - mg_apply_row(r, c, xd);
            return xd(c) + (kMgOmega * t) / r.dg;
          },
          [&](int c, double v) { mst<SC>(&F.e[c], v); });
      if (!bar()) return false;
    }
    return true;
  };
  auto uget = [&](int j) { return Lg == 0 ? lds[L0.lt + j] : mld<SC>(&L0.e[j]); };
  // w = A u on the own cells and the block sums of (r, u), (w, u), (r, r)
  auto matvec = [&]() -> bool {
    for (int blk = gwv; blk < nb; blk += gstride) {
      double g[4], d[4], rr[4], wq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c0 = blk * kTree + lane + 64 * q;
        const int c = c0 < n ? c0 : blk * kTree;
        const double uc = uget(c);
        const double wv = mg_apply(L0, c, uget);
        const double rv = mld<SC>(&L0.b[c]);
        const bool in = c0 < n;
        wq[q] = wv;
        g[q] = in ? rv * uc : 0.0;
        d[q] = in ? wv * uc : 0.0;
        rr[q] = in ? rv * rv : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = blk * kTree + lane + 64 * q;
        if (c < n) a.w[c] = wq[q];
      }
      const double sg = wave_tree256(g[0], g[1], g[2], g[3]);
      const double sd = wave_tree256(d[0], d[1], d[2], d[3]);
      const double sr = wave_tree256(rr[0], rr[1], rr[2], rr[3]);
      if (lane == 0) {
        mst<SC>(&a.part[3 * blk], sg);
        mst<SC>(&a.part[3 * blk + 1], sd);
        mst<SC>(&a.part[3 * blk + 2], sr);
      }
    }
    return bar();
  };

  int status = -7, it = 0;
  double alpha = 0.0, beta = 0.0, gamma = 0.0, delta = 0.0, thr = 0.0;
  // start: x = 0, r = b
  for_cells(
      Q4{}, n, [&](int c) { return V2{a.b[c], sweep_first(a.b[c], L0.diag[c])}; },
      [&](int c, V2 v) {
        a.x[c] = 0.0;
        mst<SC>(&L0.b[c], v.a);
        if (Lg > 0) mst<SC>(&L0.xa[c], v.b);
      });
  if (!bar() || !vcycle() || !matvec()) {
    status = -3;
  } else {
    double s3[3];
    group_tree_n<3, SC>(a.part, nb, red, s3);
    gamma = s3[0];
    delta = s3[1];
    thr = a.tol2 * s3[2];
    if (s3[2] == 0.0) status = 0;
    else if (!(delta > 0.0)) status = -6;
    else alpha = gamma / delta;
  }
  while (status == -7 && it < a.max_iters) {
    const bool first = (it == 0);
    struct U5 {
      double p, s, x, r, xa;
    };
    for_cells(
        Q4{}, n,
        [&](int c) {
          const double uc = uget(c);
          const double wv = a.w[c];
          const double pv = first ? uc : uc + beta * a.p[c];
          const double sv = first ? wv : wv + beta * a.s[c];
          const double xv = a.x[c] + alpha * pv;
          const double rv = mld<SC>(&L0.b[c]) - alpha * sv;
          return U5{pv, sv, xv, rv, sweep_first(rv, L0.diag[c])};
        },
        [&](int c, U5 v) {
          a.p[c] = v.p;
          a.s[c] = v.s;
          a.x[c] = v.x;
          mst<SC>(&L0.b[c], v.r);
          if (Lg > 0) mst<SC>(&L0.xa[c], v.xa);
        });
    if (!bar() || !vcycle() || !matvec()) {
      status = -3;
      break;
    }
    ++it;
    double s3[3];
    group_tree_n<3, SC>(a.part, nb, red, s3);
    const double gamma_new = s3[0];
    delta = s3[1];
    if (s3[2] <= thr) {
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
  if (bid == 0 && threadIdx.x == 0) {
    a.sc->cg_iters = it;
    a.sc->cg_status = status;
    a.sc->cg_t1 = static_cast<unsigned long long>(wall_clock64());
  }
}

}  // namespace iugkp

#include "mgband.hpp"

namespace iugkp {

__global__ __launch_bounds__(kCgThreadsMax) void mgcg_kernel(MGArgs a)
{
  extern __shared__ double lds[];
  __shared__ double red[3 * kTree];
  __shared__ MGLevel s_lv[kMgLevelsMax];
  mgcg_solve<__HIP_MEMORY_SCOPE_AGENT>(a, static_cast<int>(gridDim.x),
                                       static_cast<int>(blockIdx.x), lds, red, s_lv);
}

// the banded form (mgband.hpp), for the meshes whose rows fit its windows;
// workgroups of at most kMgBandThreads threads, whose lanes then have the
// registers its batched loads take
constexpr int kMgBandThreads = 512;
__global__ __launch_bounds__(kMgBandThreads) void mgcg_band_kernel(MGArgs a)
{
  extern __shared__ double lds[];
  __shared__ double red[3 * kTree];
  __shared__ MGLevel s_lv[kMgLevelsMax];
  mgcg_band_solve<__HIP_MEMORY_SCOPE_AGENT>(a, static_cast<int>(gridDim.x),
                                            static_cast<int>(blockIdx.x), lds, red, s_lv);
}

// ---------------------------------------------------------------------------
// Batched CG over a pool of resident workgroups.  The host hands every active
// Newton instance a group of workgroups and writes, per workgroup, the list of
// (instance, rank) jobs it takes part in; all lists follow one global job
// order, so the earliest unfinished job always has every member at hand and
// the pool cannot deadlock.  The solve of an instance does not depend on how
// many workgroups serve it or where.  Instances with the plain CG and those
// with the multigrid-preconditioned one have pools of their own, launched one
// after the other (one body with both would need more registers than a lane
// has).
// ---------------------------------------------------------------------------
struct CgJob {
  int inst, rank, G, tb;     // tb: blocks per workgroup, bit 30 = register form
};
constexpr int kCgJobReg = 1 << 30;

__global__ __launch_bounds__(kCgThreadsMax) void cg_batch_kernel(const Inst *__restrict__ insts,
                                                                 const int *__restrict__ off,
                                                                 const CgJob *__restrict__ jobs)
{
  const int e0 = off[blockIdx.x], e1 = off[blockIdx.x + 1];
  for (int e = e0; e < e1; ++e) {
    const CgJob jb = jobs[e];
    const Inst &in = insts[jb.inst];
    CGArgs a;
    a.m = in.m;
    a.gx = in.gx;
    a.gy = in.gy;
    a.diag = in.diag;
    a.b = in.rhs;
    a.x = in.cg_x;
    a.gr = in.cg_r;
    a.gw = in.cg_w;
    a.gp = in.cg_p;
    a.gs = in.cg_s;
    a.pub = in.cg_pub;
    a.part = in.cg_mpart;
    a.TB = jb.tb & (kCgJobReg - 1);
    a.tol2 = in.tol2;
    a.max_iters = in.cg_max;
    a.barrier = in.cg_barrier;
    a.sc = in.sc;
    if (jb.tb & kCgJobReg) cg_run<true>(a, jb.rank, jb.G);
    else cg_run<false>(a, jb.rank, jb.G);
    __syncthreads();
  }
}

// the multigrid instances' pool: job (instance, rank) runs member `rank` of
// the instance's group of G workgroups (mg: the instances' arguments); 8-wave
// workgroups, whose lanes have the registers the solve takes when its
// arguments come from memory
constexpr int kMgPoolWaves = 8;
__global__ __launch_bounds__(64 * kMgPoolWaves) void mgcg_batch_kernel(const int *__restrict__ off,
                                                                   const CgJob *__restrict__ jobs,
                                                                   const MGArgs *__restrict__ mg)
{
  extern __shared__ double lds[];
  __shared__ double red[3 * kTree];
  __shared__ MGLevel s_lv[kMgLevelsMax];
  const int e0 = off[blockIdx.x], e1 = off[blockIdx.x + 1];
  for (int e = e0; e < e1; ++e) {
    const CgJob jb = jobs[e];
    const MGArgs &a = mg[jb.inst];
    if (a.band) mgcg_band_solve<__HIP_MEMORY_SCOPE_AGENT>(a, jb.G, jb.rank, lds, red, s_lv);
    else mgcg_solve<__HIP_MEMORY_SCOPE_AGENT>(a, jb.G, jb.rank, lds, red, s_lv);
    __syncthreads();
  }
}

// Level k+1's faces from level k's: a coarse x face sums the fine x faces of
// its two rows at the fine face under it, a coarse y face the fine y faces of
// its two columns (an absent row or column adds 0).
__global__ void mg_coarsen_faces_kernel(MGLevel f, MGLevel c, int has_y, double *gx, double *gy)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nfx = c.ny * (c.nx + 1);
  if (i < nfx) {
    const int J = i / (c.nx + 1), K = i - J * (c.nx + 1);
    const int k = (2 * K < f.nx) ? 2 * K : f.nx;
    const double a = f.gx[(2 * J) * (f.nx + 1) + k];
    const double b = (2 * J + 1 < f.ny) ? f.gx[(2 * J + 1) * (f.nx + 1) + k] : 0.0;
    gx[i] = a + b;
  }
  if (has_y && i < (c.ny + 1) * c.nx) {
    const int K = i / c.nx, I = i - K * c.nx;
    const int k = (2 * K < f.ny) ? 2 * K : f.ny;
    const double a = f.gy[k * f.nx + 2 * I];
    const double b = (2 * I + 1 < f.nx) ? f.gy[k * f.nx + 2 * I + 1] : 0.0;
    gy[i] = a + b;
  }
}

// diagonal = the sum of the cell's faces: (left + right) + down + up
__global__ void mg_coarsen_diag_kernel(MGLevel c, int has_y, double *diag)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  const int J = i / c.nx, I = i - J * c.nx;
  double d = c.gx[J * (c.nx + 1) + I] + c.gx[J * (c.nx + 1) + I + 1];
  if (has_y) {
    d = d + c.gy[J * c.nx + I];
    d = d + c.gy[(J + 1) * c.nx + I];
  }
  diag[i] = d;
}

}  // namespace iugkp
