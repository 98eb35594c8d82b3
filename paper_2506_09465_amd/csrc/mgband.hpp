// mgband.hpp -- the multigrid-preconditioned CG of mgcg.hpp in row bands:
// the same hierarchy, V-cycle and CG recurrences (Sec. 3.3's Newton system),
// every value computed by the same operations in the same order, with about
// half the group barriers.
//
// A grid level's work is split by rows: member g of the group takes a band of
// rows and computes, in LDS, everything its band's outputs need, the few rows
// around the band included (recomputed there by both neighbours, with the same
// operations, so the values agree bit for bit).  One phase per level on the
// way down and one on the way up:
//   descent of level k: (level 0: the CG update of r, s, p, x), the two
//     pre-sweeps and the residual on the band's rows and two rows around
//     them, the restriction to the band's coarse rows;
//   coarse phase: the LDS levels' V-cycle in every workgroup, then the ascent
//     of the finest grid level above it;
//   ascent of level k: the coarse correction and the two post-sweeps (level
//     0: also w = A u and the block sums of (r, u), (w, u), (r, r), its band
//     then whole 256-cell blocks).
// A band phase reads only what earlier phases wrote (behind a group barrier);
// r and s, read around the band by the neighbours while the owner writes the
// next iterate, alternate between two buffers.  Per iteration: 2 Lg group
// barriers for Lg grid levels (1 when every level is an LDS level).  A band
// too long for the LDS is run in windows of rows, one after the other.
#pragma once

namespace iugkp {

// the part [lo, hi) of [0, N) that member g of G takes
__device__ __forceinline__ void band_split(int N, int g, int G, int &lo, int &hi)
{
  lo = static_cast<int>(static_cast<long long>(N) * g / G);
  hi = static_cast<int>(static_cast<long long>(N) * (g + 1) / G);
}

// (A_k v) at the cell of row r, v staged in LDS with the cell at index i and
// rows of nx cells (an absent neighbour read at i itself and discarded)
__device__ __forceinline__ double mg_apply_staged(const MGRow &r, const double *S, int i, int nx)
{
  double v[5];
  v[0] = S[i];
  v[1] = S[(r.m & 1u) ? i - 1 : i];
  v[2] = S[(r.m & 2u) ? i + 1 : i];
  v[3] = S[(r.m & 4u) ? i - nx : i];
  v[4] = S[(r.m & 8u) ? i + nx : i];
  return mg_apply_vals(r, v);
}

// CG update modes of the residual: the start (r = b, x = 0), the first
// iteration (p = u, s = w) and the later ones
constexpr int kMgStart = 0, kMgFirst = 1, kMgNext = 2;

// Window sizes, in the rows of the level, that a stage of `words` doubles
// holds (also used by the host to check that one row fits).
__host__ __device__ inline int band_down_rows(int words, int nx)   // coarse rows
{
  return (words / nx - 10) / 6;
}
__host__ __device__ inline int band_up_rows(int words, int nx)
{
  return (words / nx - 8) / 3;
}
__host__ __device__ inline int band_up0_blocks(int words, int nx, int block)
{
  const int rmax = (words / nx - 14) / 3;     // rows the blocks may span
  return ((rmax - 2) * nx + 1) / block;
}

template <int SC>
__device__ __forceinline__ void mgcg_band_solve(const MGArgs &a, int G, int bid, double *lds,
                                                double *red, MGLevel *s_lv)
{
  const int nt = static_cast<int>(blockDim.x), tid = static_cast<int>(threadIdx.x);
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  if (bid == 0 && tid == 0) a.sc->cg_t0 = static_cast<unsigned long long>(wall_clock64());
  const int L = a.L, Lg = a.Lg;
  mg_stage_levels(a.lv, L, s_lv);
  const MGLevel *lv = s_lv;
  const MGLevel L0 = lv[0];
  const int n = L0.n, nb = (n + kTree - 1) / kTree;
  // LDS: level Lg's result (kept through a band phase), the LDS levels' rows
  // (for the whole solve), then their vectors or a band window's staging
  double *const E = lds;
  double *const S = lds + a.stage0;
  const int SN = a.stage_n;
  unsigned int epoch = 0;
  mg_lds_rows(lv, Lg, L, lds);
  __syncthreads();

  auto bar = [&]() -> bool {
    if (G == 1) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      return true;
    }
    return grid_barrier(a.barrier, epoch, G);
  };

  // Descent of grid level k for the coarse rows of this member: b and the
  // first sweep on the fine rows and two around them, the second sweep on
  // those and one around them (stored for the own rows), the residual and its
  // restriction on the own coarse rows.  Level 0's b is the updated residual:
  //   start: r = b, x = 0
  //   then:  s = w (+ beta s), r = r - alpha s, p = u (+ beta p), x = x + alpha p
  // computed on every staged cell and stored, with s, p and x, for the own ones.
  struct Upd {
    double w, s, r, u, p, x, d;
  };
  auto descend = [&](int k, int mode, double alpha, double beta, const double *r_old,
                     double *r_new, const double *s_old, double *s_new) {
    const MGLevel F = lv[k], Cl = lv[k + 1];
    const int nx = F.nx, ny = F.ny;
    int Y0, Y1;
    band_split(Cl.ny, bid, G, Y0, Y1);
    const int wmax = max(1, band_down_rows(SN, nx));
    const int nwin = (Y1 - Y0 + wmax - 1) / wmax;
    for (int w = 0; w < nwin; ++w) {
      int wY0, wY1;
      band_split(Y1 - Y0, w, nwin, wY0, wY1);
      wY0 += Y0;
      wY1 += Y0;
      const int fy0 = 2 * wY0, fy1 = min(2 * wY1, ny);
      const int by0 = max(0, fy0 - 2), by1 = min(ny, fy1 + 2);
      const int xy0 = max(0, fy0 - 1), xy1 = min(ny, fy1 + 1);
      const int nB = (by1 - by0) * nx, nX = (xy1 - xy0) * nx;
      double *const B = S, *const X1 = S + nB, *const X2 = S + 2 * nB;
      if (k == 0) {
        mg_cells<8>(
            nB,
            [&](int i) {
              const int c = by0 * nx + i, iy = by0 + i / nx;
              const bool own = iy >= fy0 && iy < fy1;
              Upd v{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, F.diag[c]};
              if (mode == kMgStart) {
                v.r = a.b[c];
              } else {
                v.w = mld<SC>(&a.w[c]);
                if (mode != kMgFirst) v.s = mld<SC>(&s_old[c]);
                v.r = mld<SC>(&r_old[c]);
                if (own) {
                  v.u = mld<SC>(&L0.e[c]);
                  v.p = a.p[c];
                  v.x = a.x[c];
                }
              }
              return v;
            },
            [&](int i, const Upd &v) {
              const int c = by0 * nx + i, iy = by0 + i / nx;
              const bool own = iy >= fy0 && iy < fy1;
              double bv = v.r;
              if (mode == kMgStart) {
                if (own) {
                  a.x[c] = 0.0;
                  mst<SC>(&r_new[c], bv);
                }
              } else {
                const double sv = (mode == kMgFirst) ? v.w : v.w + beta * v.s;
                bv = v.r - alpha * sv;
                if (own) {
                  const double pv = (mode == kMgFirst) ? v.u : v.u + beta * v.p;
                  a.p[c] = pv;
                  a.x[c] = v.x + alpha * pv;
                  mst<SC>(&s_new[c], sv);
                  mst<SC>(&r_new[c], bv);
                }
              }
              B[i] = bv;
              X1[i] = mg_sweep_first(bv, v.d);
            });
      } else {
        mg_cells<4>(
            nB,
            [&](int i) {
              const int c = by0 * nx + i;
              return MgV2{mld<SC>(&F.b[c]), F.diag[c]};
            },
            [&](int i, const MgV2 &v) {
              B[i] = v.a;
              X1[i] = mg_sweep_first(v.a, v.b);
            });
      }
      __syncthreads();
      mg_cells<4>(
          nX, [&](int i) { const int r = i / nx; return mg_row_at(F, i - r * nx, xy0 + r); },
          [&](int i, const MGRow &rw) {
            const int iy = rw.iy, ix = rw.ix;
            const int j = (iy - by0) * nx + ix;
            const double t = B[j] - mg_apply_staged(rw, X1, j, nx);
            const double v = X1[j] + (kMgOmega * t) / rw.dg;
            X2[i] = v;
            if (iy >= fy0 && iy < fy1) mst<SC>(&F.xb[iy * nx + ix], v);
          });
      __syncthreads();
      const int NC = (wY1 - wY0) * Cl.nx;
      struct Four {
        MGRow r[4];
      };
      mg_cells<1>(
          NC,
          [&](int i) {
            const int R = i / Cl.nx, I = i - R * Cl.nx, J = wY0 + R;
            Four f;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              const int ix = 2 * I + (h & 1), iy = 2 * J + (h >> 1);
              const bool in = (ix < nx && iy < ny);
              f.r[h] = mg_row_at(F, in ? ix : 2 * I, in ? iy : 2 * J);
            }
            return f;
          },
          [&](int i, const Four &f) {
            const int R = i / Cl.nx, I = i - R * Cl.nx, J = wY0 + R;
            double q[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              const int ix = 2 * I + (h & 1), iy = 2 * J + (h >> 1);
              const bool in = (ix < nx && iy < ny);
              const MGRow &rw = f.r[h];
              const int jb = (rw.iy - by0) * nx + rw.ix, jx = (rw.iy - xy0) * nx + rw.ix;
              const double res = B[jb] - mg_apply_staged(rw, X2, jx, nx);
              q[h] = in ? res : 0.0;
            }
            mst<SC>(&Cl.b[J * Cl.nx + I], (q[0] + q[1]) + (q[2] + q[3]));
          });
      __syncthreads();
    }
  };

  // Ascent of grid level k >= 1 for this member's rows: x after the coarse
  // correction on the rows and two around them, the first post-sweep on the
  // rows and one around them, the second on the rows (stored as e of level k).
  // The coarse result from LDS (e_lds) or from level k+1's e.
  struct Xcb {
    double xb, e, b;
  };
  auto ascend = [&](int k, bool e_lds) {
    const MGLevel F = lv[k], Cl = lv[k + 1];
    const int nx = F.nx, ny = F.ny;
    int y0, y1;
    band_split(ny, bid, G, y0, y1);
    const int wmax = max(1, band_up_rows(SN, nx));
    const int nwin = (y1 - y0 + wmax - 1) / wmax;
    for (int w = 0; w < nwin; ++w) {
      int wy0, wy1;
      band_split(y1 - y0, w, nwin, wy0, wy1);
      wy0 += y0;
      wy1 += y0;
      const int cy0 = max(0, wy0 - 2), cy1 = min(ny, wy1 + 2);
      const int py0 = max(0, wy0 - 1), py1 = min(ny, wy1 + 1);
      const int nC = (cy1 - cy0) * nx, nP = (py1 - py0) * nx;
      double *const XC = S, *const B = S + nC, *const P1 = B + nP;
      mg_cells<8>(
          nC,
          [&](int i) {
            const int c = cy0 * nx + i, iy = cy0 + i / nx, ix = c - iy * nx;
            const int P = (iy >> 1) * Cl.nx + (ix >> 1);
            Xcb v;
            v.xb = mld<SC>(&F.xb[c]);
            v.e = e_lds ? E[P] : mld<SC>(&Cl.e[P]);
            v.b = (iy >= py0 && iy < py1) ? mld<SC>(&F.b[c]) : 0.0;
            return v;
          },
          [&](int i, const Xcb &v) {
            const int c = cy0 * nx + i, iy = cy0 + i / nx;
            XC[i] = v.xb + kMgScale * v.e;
            if (iy >= py0 && iy < py1) B[c - py0 * nx] = v.b;
          });
      __syncthreads();
      mg_cells<4>(
          nP, [&](int i) { const int r = i / nx; return mg_row_at(F, i - r * nx, py0 + r); },
          [&](int i, const MGRow &rw) {
            const int j = (rw.iy - cy0) * nx + rw.ix;
            const double t = B[i] - mg_apply_staged(rw, XC, j, nx);
            P1[i] = XC[j] + (kMgOmega * t) / rw.dg;
          });
      __syncthreads();
      mg_cells<4>(
          (wy1 - wy0) * nx,
          [&](int i) { const int r = i / nx; return mg_row_at(F, i - r * nx, wy0 + r); },
          [&](int i, const MGRow &rw) {
            const int j = (rw.iy - py0) * nx + rw.ix;
            const double t = B[j] - mg_apply_staged(rw, P1, j, nx);
            mst<SC>(&F.e[rw.iy * nx + rw.ix], P1[j] + (kMgOmega * t) / rw.dg);
          });
      __syncthreads();
    }
  };

  // the products of one 256-cell block and its published sums; u and w
  // stored (rows: the block's four rows of A per lane, loaded together)
  auto block_sums = [&](int blk, auto row, auto vals) {
    MGRow rw[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c0 = blk * kTree + lane + 64 * q;
      rw[q] = row(c0 < n ? c0 : blk * kTree);
    }
    double g[4], d[4], rr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c0 = blk * kTree + lane + 64 * q;
      const bool in = c0 < n;
      const int c = in ? c0 : blk * kTree;
      double uc, wv, rv;
      vals(c, rw[q], uc, wv, rv);
      g[q] = in ? rv * uc : 0.0;
      d[q] = in ? wv * uc : 0.0;
      rr[q] = in ? rv * rv : 0.0;
      if (in) {
        mst<SC>(&L0.e[c], uc);
        mst<SC>(&a.w[c], wv);
      }
    }
    const double sg = wave_tree256(g[0], g[1], g[2], g[3]);
    const double sd = wave_tree256(d[0], d[1], d[2], d[3]);
    const double sr = wave_tree256(rr[0], rr[1], rr[2], rr[3]);
    if (lane == 0) {
      mst<SC>(&a.part[3 * blk], sg);
      mst<SC>(&a.part[3 * blk + 1], sd);
      mst<SC>(&a.part[3 * blk + 2], sr);
    }
  };

  // Ascent of level 0 with w = A u and the block sums, for this member's
  // 256-cell blocks, a window of whole blocks at a time: corrected x on the
  // blocks' rows and three around them, the first post-sweep on two around,
  // u on one around, w on the blocks.  r: the current residual.
  auto ascend0 = [&](bool e_lds, const double *r) {
    const MGLevel F = L0, Cl = lv[1];
    const int nx = F.nx, ny = F.ny;
    int b0, b1;
    band_split(nb, bid, G, b0, b1);
    const int per = max(1, band_up0_blocks(SN, nx, kTree));
    const int nwin = (b1 - b0 + per - 1) / per;
    for (int w = 0; w < nwin; ++w) {
      int wb0, wb1;
      band_split(b1 - b0, w, nwin, wb0, wb1);
      wb0 += b0;
      wb1 += b0;
      const int c0 = wb0 * kTree, c1 = min(wb1 * kTree, n);
      const int ya = c0 / nx, yb = (c1 - 1) / nx + 1;
      const int cy0 = max(0, ya - 3), cy1 = min(ny, yb + 3);
      const int py0 = max(0, ya - 2), py1 = min(ny, yb + 2);
      const int uy0 = max(0, ya - 1), uy1 = min(ny, yb + 1);
      const int nC = (cy1 - cy0) * nx, nP = (py1 - py0) * nx, nU = (uy1 - uy0) * nx;
      // (u overwrites the corrected x, read only by the first post-sweep)
      double *const XC = S, *const B = S + nC, *const P1 = B + nP, *const U = S;
      mg_cells<8>(
          nC,
          [&](int i) {
            const int c = cy0 * nx + i, iy = cy0 + i / nx, ix = c - iy * nx;
            const int P = (iy >> 1) * Cl.nx + (ix >> 1);
            Xcb v;
            v.xb = mld<SC>(&F.xb[c]);
            v.e = e_lds ? E[P] : mld<SC>(&Cl.e[P]);
            v.b = (iy >= py0 && iy < py1) ? mld<SC>(&r[c]) : 0.0;
            return v;
          },
          [&](int i, const Xcb &v) {
            const int c = cy0 * nx + i, iy = cy0 + i / nx;
            XC[i] = v.xb + kMgScale * v.e;
            if (iy >= py0 && iy < py1) B[c - py0 * nx] = v.b;
          });
      __syncthreads();
      mg_cells<4>(
          nP, [&](int i) { const int q = i / nx; return mg_row_at(F, i - q * nx, py0 + q); },
          [&](int i, const MGRow &rw) {
            const int j = (rw.iy - cy0) * nx + rw.ix;
            const double t = B[i] - mg_apply_staged(rw, XC, j, nx);
            P1[i] = XC[j] + (kMgOmega * t) / rw.dg;
          });
      __syncthreads();
      mg_cells<4>(
          nU, [&](int i) { const int q = i / nx; return mg_row_at(F, i - q * nx, uy0 + q); },
          [&](int i, const MGRow &rw) {
            const int j = (rw.iy - py0) * nx + rw.ix;
            const double t = B[j] - mg_apply_staged(rw, P1, j, nx);
            U[i] = P1[j] + (kMgOmega * t) / rw.dg;
          });
      __syncthreads();
      for (int blk = wb0 + wave; blk < wb1; blk += nw)
        block_sums(
            blk, [&](int c) { const int iy = c / nx; return mg_row_at(F, c - iy * nx, iy); },
            [&](int c, const MGRow &rw, double &uc, double &wv, double &rv) {
              const int ju = (rw.iy - uy0) * nx + rw.ix;
              uc = U[ju];
              wv = mg_apply_staged(rw, U, ju, nx);
              rv = B[c - py0 * nx];
            });
      __syncthreads();
    }
  };

  // The coarse phase: the LDS levels' V-cycle in every workgroup, then the ascent
  // of grid level Lg - 1 from its result; with no grid level, the CG update
  // of every cell first (its own cells stored) and w = A u with the block
  // sums of the own blocks after.
  auto coarse = [&](int mode, double alpha, double beta, const double *r_old, double *r_new,
                    const double *s_old, double *s_new) {
    const MGLevel T = lv[Lg];
    int o0 = 0, o1 = 0;
    if (Lg == 0) {
      band_split(nb, bid, G, o0, o1);
      const int c0 = o0 * kTree, c1 = min(o1 * kTree, n);
      mg_cells<4>(
          n,
          [&](int c) {
            const bool own = c >= c0 && c < c1;
            Upd v{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if (mode == kMgStart) {
              v.r = a.b[c];
            } else {
              v.w = mld<SC>(&a.w[c]);
              if (mode != kMgFirst) v.s = mld<SC>(&s_old[c]);
              v.r = mld<SC>(&r_old[c]);
              if (own) {
                v.u = mld<SC>(&L0.e[c]);
                v.p = a.p[c];
                v.x = a.x[c];
              }
            }
            return v;
          },
          [&](int c, const Upd &v) {
            const bool own = c >= c0 && c < c1;
            double bv = v.r;
            if (mode == kMgStart) {
              if (own) {
                a.x[c] = 0.0;
                mst<SC>(&r_new[c], bv);
              }
            } else {
              const double sv = (mode == kMgFirst) ? v.w : v.w + beta * v.s;
              bv = v.r - alpha * sv;
              if (own) {
                const double pv = (mode == kMgFirst) ? v.u : v.u + beta * v.p;
                a.p[c] = pv;
                a.x[c] = v.x + alpha * pv;
                mst<SC>(&s_new[c], sv);
                mst<SC>(&r_new[c], bv);
              }
            }
            lds[T.lb + c] = bv;
          });
    }
    __syncthreads();
    mg_lds_cycle<SC>(lv, Lg, L, lds, Lg > 0);
    if (Lg >= 1) {
      for (int i = tid; i < T.n; i += nt) E[i] = lds[T.lt + i];
      __syncthreads();
      if (Lg == 1) ascend0(true, r_new);
      else ascend(Lg - 1, true);
    } else {
      for (int blk = o0 + wave; blk < o1; blk += nw)
        block_sums(
            blk, [&](int c) { return mg_row_lds(T, lds, c); },
            [&](int c, const MGRow &rw, double &uc, double &wv, double &rv) {
              uc = lds[T.lt + c];
              wv = mg_apply_row(rw, c, [&](int j) { return lds[T.lt + j]; });
              rv = lds[T.lb + c];
            });
    }
  };

  // one application of the preconditioner and the operator to the updated
  // residual, with its block sums
  auto iterate = [&](int mode, double alpha, double beta, int cur) -> bool {
    const double *r_old = cur ? a.r2 : L0.b;
    double *r_new = (mode == kMgStart) ? L0.b : (cur ? L0.b : a.r2);
    const double *s_old = cur ? a.s2 : a.s;
    double *s_new = cur ? a.s : a.s2;
    for (int k = 0; k < Lg; ++k) {
      descend(k, mode, alpha, beta, r_old, r_new, s_old, s_new);
      if (!bar()) return false;
    }
    coarse(mode, alpha, beta, r_old, r_new, s_old, s_new);
    if (!bar()) return false;
    for (int k = Lg - 2; k >= 1; --k) {
      ascend(k, false);
      if (!bar()) return false;
    }
    if (Lg >= 2) {
      ascend0(false, r_new);
      if (!bar()) return false;
    }
    return true;
  };

  int status = -7, it = 0, cur = 0;
  double alpha = 0.0, beta = 0.0, gamma = 0.0, delta = 0.0, thr = 0.0;
  if (!iterate(kMgStart, 0.0, 0.0, 0)) {
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
    if (!iterate(it == 0 ? kMgFirst : kMgNext, alpha, beta, cur)) {
      status = -3;
      break;
    }
    cur ^= 1;
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
  if (bid == 0 && tid == 0) {
    a.sc->cg_iters = it;
    a.sc->cg_status = status;
    a.sc->cg_t1 = static_cast<unsigned long long>(wall_clock64());
  }
}

}  // namespace iugkp
