// vp_calib.hip -- peel calibration (Sec. 5.1): per-tile complex gains for
// every (time, channel) cell, fitted so that g_i g_j^* I_ij matches the data
// V_ij by Gauss-Newton iterations of the linearised least-squares problem,
// then the gain-corrupted model is subtracted.
//
// One workgroup per cell; thread k owns tile k.  The step e solves the normal
// equations of the linearised problem, which for this model take the form
//   D_k e_k + g_k sum_o W_ko g_o e_o^* = r_k,
//   W_ko = |I_ko|^2,  D_k = sum_o W_ko |g_o|^2,
//   r_k = sum_{b: ant1 = k} g_j I_b^* R_b + sum_{b: ant2 = k} g_i I_b R_b^*,
// (R = V - g_i g_j^* I the current residual) -- a real-linear, self-adjoint,
// positive semi-definite operator.  Its null space is spanned by i g
// restricted to each connected component of the baseline graph (the data
// leave each component's global phase free).  The step taken is the
// minimum-norm least-squares one, x = (A^T A)^+ A^T b: the right-hand side
// and the solution are projected off that null space, and conjugate
// gradients solve in between.  Without the projections, a right-hand side
// at rounding level (a converged solve) has null-space components of its
// own size that the iteration amplifies into a drift of the global phase.
// The solve also stops once the residual is at the rounding level of r.
// With X_ko = I^* V seen from tile k (a per-cell table built once), the
// right-hand side is r_k = sum_o g_o X_ko - g_k D_k; X streams from HBM once
// per Gauss-Newton iteration as a full n x n table, coalesced over k.  The
// conjugate gradients take one operator application and one workgroup
// reduction per step (Chronopoulos-Gear form).  On the FP64 path the tables
// are FP64, D_k is summed from the FP64 W table, and the operator's W sits
// in LDS, packed, FP64 while it fits (up to 183 tiles) and FP32 beyond: that
// changes the step's operator at the 1e-7 level, not the right-hand side, so
// not the fixed point.  On the mixed path the tables hold X and W rounded to
// FP32 (sums and steps stay FP64, so the solution moves by the tables'
// rounding, ~1e-7 relative), each thread holds its block of W in registers,
// the operator's products are FP32 (its W is FP32 already) and each step's
// solve stops at a relative residual of 1e-6 instead of 1e-12.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "vp_internal.h"

namespace vp {

// Rounding level of the right-hand side, relative to the sum of the
// magnitudes of its terms (64 units of FP64 rounding).
constexpr double kGainFloor = 64.0 * 2.220446049250313e-16;

__device__ __forceinline__ int pair_index(int n, int i, int j) {  // i < j
  return i * n - i * (i + 1) / 2 + (j - i - 1);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

__device__ __forceinline__ double2 load_vis(const void *p, int c64, int64_t i) {
  if (c64) {
    const float2 v = ((const float2 *)p)[i];
    return make_double2(v.x, v.y);
  }
  return ((const double2 *)p)[i];
}

// Table element types: TT (FP64 or FP32) and its complex pair.
template <typename TT>
struct TabPair;
template <>
struct TabPair<float> {
  typedef float2 type;
};
template <>
struct TabPair<double> {
  typedef double2 type;
};

// Cells per workgroup of the table kernel (at most 48 KB of LDS either way).
template <typename TT>
constexpr int tab_cells() {
  return sizeof(TT) == sizeof(float) ? 16 : 8;
}

// Per-cell tables for the solve, from the [T][B][K] model and data:
//   xt [cell][o][k] = X_ko: I_b^* V_b for k = ant1, o = ant2 of baseline b,
//                     its conjugate for k = ant2, o = ant1;
//   wf [cell][o][k] = |I_b|^2 for both orders of the baseline's tiles;
// zero on the diagonal and for tile pairs without a baseline.  Workgroup
// (x, o) writes row o of the tables of C = tab_cells consecutive cells: the
// row's baselines are read C adjacent channels at a time (contiguous in the
// [T][B][K] layout), staged in LDS, and written one row after another
// (contiguous), every entry once, so no clearing pass is needed.  Each
// baseline is read twice, once for the row of either tile.
template <typename TT>
__global__ __launch_bounds__(256) void k_gain_tables(GainArgs a) {
  typedef typename TabPair<TT>::type TT2;
  constexpr int C = tab_cells<TT>();
  // [C][n] pairs, then [C][n] magnitudes (sized for this n, so that small
  // arrays fit more workgroups per CU)
  extern __shared__ __align__(16) unsigned char tsm[];
  const int n = a.n_ant, o = blockIdx.y;
  TT2 *sx = (TT2 *)tsm;
  TT *sw = (TT *)(sx + C * n);
  const int c0 = blockIdx.x * C;
  const int nc = min(C, a.ncell - c0);
  for (int e = threadIdx.x; e < nc * n; e += 256) {
    const int j = e % nc, k = e / nc;
    TT2 x;
    x.x = 0;
    x.y = 0;
    TT w = 0;
    const int b = k == o ? -1 : a.pair_bl[pair_index(n, min(o, k), max(o, k))];
    if (b >= 0) {
      const int cell = a.cell0 + c0 + j, t = cell / a.K, kc = cell % a.K;
      const int64_t i = ((int64_t)t * a.B + b) * a.K + kc;
      const double2 m = load_vis(a.model, a.c64, i);
      const double2 v = load_vis(a.data, a.c64, i);
      // I^* V with k = ant1, o = ant2; its conjugate for the other order
      double2 xv = cmul(cconj(m), v);
      if (a.ant1[b] == o) xv = cconj(xv);
      x.x = (TT)xv.x;
      x.y = (TT)xv.y;
      w = (TT)(m.x * m.x + m.y * m.y);
    }
    sx[j * n + k] = x;
    sw[j * n + k] = w;
  }
  __syncthreads();
  TT2 *X = (TT2 *)a.xt;
  TT *W = (TT *)a.wf;
  for (int e = threadIdx.x; e < nc * n; e += 256) {
    const int j = e / n, k = e - j * n;
    const int64_t off = ((int64_t)(c0 + j) * n + o) * n + k;
    X[off] = sx[j * n + k];
    W[off] = sw[j * n + k];
  }
}

// Sums of two values over the workgroup (NT threads) in one pass, through
// the scratch red[NT / 64].  One barrier: the caller alternates between two
// scratch buffers, and a workgroup barrier separates the last reads of a
// buffer from its next writes.
template <int NT>
__device__ __forceinline__ double2 block_sum2(double u, double v, double2 *red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    u += __shfl_xor(u, o);
    v += __shfl_xor(v, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = make_double2(u, v);
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    s.x += red[w].x;
    s.y += red[w].y;
  }
  return s;
}

// Sums of three values over the workgroup, as block_sum2; red holds 2 NT / 64
// pairs.
template <int NT>
__device__ __forceinline__ double3 block_sum3(double u, double v, double w, double2 *red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    u += __shfl_xor(u, o);
    v += __shfl_xor(v, o);
    w += __shfl_xor(w, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[2 * wave] = make_double2(u, v);
    red[2 * wave + 1] = make_double2(w, 0.0);
  }
  __syncthreads();
  double3 s = make_double3(0.0, 0.0, 0.0);
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) {
    s.x += red[2 * q].x;
    s.y += red[2 * q].y;
    s.z += red[2 * q + 1].x;
  }
  return s;
}

// Removes from v (tile k's entry of a vector over tiles) its part along the
// gauge direction i g of k's connected component:
//   v <- v - i g_k (sum_{o in C} Im(g_o^* v_o)) / (sum_{o in C} |g_o|^2).
// With every used tile in one component (single) the two sums are workgroup
// reductions through redp (NT / 64 pairs); otherwise each tile's sums run
// over the tiles of its component in index order, pv being LDS scratch.
// Deterministic either way.
template <int NT>
__device__ __forceinline__ double2 gauge_project(double2 v, double2 gk, int k, int ck, bool own, int n,
                                                 const int *comp, const double2 *g, double *pv, bool single,
                                                 double2 *redp) {
  if (single) {
    const bool in = own && ck >= 0;
    const double2 s = block_sum2<NT>(in ? gk.x * v.y - gk.y * v.x : 0.0, in ? gk.x * gk.x + gk.y * gk.y : 0.0, redp);
    if (in && s.y > 0.0) {
      const double c = s.x / s.y;
      v.x += c * gk.y;
      v.y -= c * gk.x;
    }
    __syncthreads();  // redp's reads end before its next writes
    return v;
  }
  if (own) pv[k] = ck >= 0 ? gk.x * v.y - gk.y * v.x : 0.0;
  __syncthreads();
  if (own && ck >= 0) {
    double num = 0.0, den = 0.0;
    for (int o = 0; o < n; ++o) {
      if (comp[o] != ck) continue;
      const double2 go = g[o];
      num += pv[o];
      den += go.x * go.x + go.y * go.y;
    }
    if (den > 0.0) {
      const double c = num / den;
      v.x += c * gk.y;
      v.y -= c * gk.x;
    }
  }
  __syncthreads();
  return v;
}

// Index of (i, j) in W packed with its (zero) diagonal: rows i of the upper
// triangle j >= i, one after another.
__device__ __forceinline__ int packed_index(int n, int i, int j) {  // i <= j
  return i * n - i * (i - 1) / 2 + (j - i);
}

// The FP64 path's solve.  One workgroup of NT threads per cell.  Thread
// (k, part) with k = tid mod nk (nk = n rounded up to 64) and part = tid / nk
// sums over a wave-uniform share of the other tiles (the part-th slice
// o0 <= o < o1 for the right-hand side, the part-th share of every 64-tile
// block for the W products); the part-0 thread of tile k holds the tile's
// gain and its conjugate-gradient state; threads with part >= NT / nk (when
// nk does not divide NT) take no share.  W sits in LDS packed with its zero
// diagonal, as WT (FP64 while it fits).  The operator of the step uses these
// W values for its diagonal too, so that i g stays its exact null vector; the
// right-hand side uses the FP64 tables.  The solve is conjugate gradients
// preconditioned by that diagonal (Jacobi).
template <typename WT, int NT>
__global__ __launch_bounds__(NT) void k_gain_solve(GainArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2 *g = (double2 *)smem;                   // [kPeelMaxAnt] gains
  double2 *y = g + kPeelMaxAnt;                   // [kPeelMaxAnt] g_o u_o^* of the current direction
  double2 *pa = y + kPeelMaxAnt;                  // [NT] partial sums
  double *pv = (double *)(pa + NT);               // [kPeelMaxAnt] projection scratch
  int *comp = (int *)(pv + kPeelMaxAnt);          // [kPeelMaxAnt] connected component of each tile
  double2 *red = (double2 *)(comp + kPeelMaxAnt); // [2 NT / 64] reduction scratch
  double2 *redp = red + 2 * (NT / 64);            // [NT / 64] reduction scratch of the projections
  WT *W = (WT *)(redp + NT / 64);                 // [n (n + 1) / 2] |I|^2, packed with the diagonal

  const int cl = blockIdx.x, cell = a.cell0 + cl;
  const int t = cell / a.K, kc = cell % a.K;
  const int n = a.n_ant, tid = threadIdx.x;
  const int nk = (n + 63) & ~63, parts = NT / nk;
  const int k = tid % nk;
  const int pt = __builtin_amdgcn_readfirstlane(tid / nk);  // nk is a multiple of 64: one part per wave
  const int span = (n + parts - 1) / parts;
  const int o0 = min(n, pt * span), o1 = min(n, o0 + span);
  const bool row = k < n;                         // sums for tile k
  const bool own = row && pt == 0;                // holds tile k's state
  const int kr = row ? k : n - 1;                 // a valid row for the others (their sums are unused)
  // packed position of W_{kr,o}: L(o) + kr in the lower part (o < kr), with
  // the wave-uniform L(o) = o n - o (o + 1) / 2, and U + o in the upper part
  const int U = kr * n - kr * (kr + 1) / 2;
  // the W products split every 64-tile block of o among the parts: part pt
  // takes offsets [sa, sb) of each block, so that every wave has the same
  // share of its own diagonal block (the only o where its lanes differ
  // between the lower and the upper part) and the rest needs no test
  const int wb = __builtin_amdgcn_readfirstlane(k >> 6);  // this wave's tiles: 64 wb .. 64 wb + 63
  const int sa = pt < parts ? 64 * pt / parts : 0, sb = pt < parts ? 64 * (pt + 1) / parts : 0;

  const double2 *X = (const double2 *)a.xt + (int64_t)cl * n * n;  // X[o n + k], zero for o == k
  const double *Wf = (const double *)a.wf + (int64_t)cl * n * n;    // |I|^2 [o n + k], zero for o == k
  for (int idx = tid; idx < n * n; idx += NT) {
    const int i = idx / n, j = idx - i * n;
    if (i <= j) W[packed_index(n, i, j)] = (WT)Wf[idx];
  }
  double2 gk = make_double2(1.0, 0.0);
  const int ck = own ? a.comp[k] : -1;
  if (own) {
    g[k] = gk;
    comp[k] = ck;
  }
  __syncthreads();

  // sum over this part's o of W_ko v_o (v in LDS), or of W_ko |v_o|^2 (sq);
  // the diagonal term is zero
  auto wdot = [&](const double2 *v, bool sq) {
    double2 acc = make_double2(0.0, 0.0);
    auto add = [&](int p, int o) {
      const double wv = (double)W[p];
      const double2 vo = v[o];
      if (sq) {
        acc.x += wv * (vo.x * vo.x + vo.y * vo.y);
      } else {
        acc.x += wv * vo.x;
        acc.y += wv * vo.y;
      }
    };
    for (int c = 0; 64 * c < n; ++c) {
      const int oa = min(n, 64 * c + sa), ob = min(n, 64 * c + sb);
      int L = oa * n - oa * (oa + 1) / 2;
      if (c < wb) {  // o < 64 wb <= k: lower part for every lane
#pragma unroll 4
        for (int o = oa; o < ob; ++o) {
          add(L + kr, o);
          L += n - o - 1;
        }
      } else if (c > wb) {  // o >= 64 (wb + 1) > k: upper part for every lane
#pragma unroll 4
        for (int o = oa; o < ob; ++o) add(U + o, o);
      } else {
#pragma unroll 4
        for (int o = oa; o < ob; ++o) {
          add(o < kr ? L + kr : U + o, o);
          L += n - o - 1;
        }
      }
    }
    return acc;
  };

  for (int it = 0; it < a.n_iter; ++it) {
    // r_k = sum_o g_o X_ko - g_k D_k,  D_k = sum_o W_ko |g_o|^2 from the FP64
    // table; Dt_k, the same sum over the LDS copy of W, is the operator's diagonal
    double2 sx = make_double2(0.0, 0.0);
    double sd = 0.0, sa = 0.0;  // sa: sum of |g_o X_ko|, for the rounding level of r_k
    if (row) {
#pragma unroll 8
      for (int o = o0; o < o1; ++o) {
        const double2 go = g[o];
        const double2 x = X[(int64_t)o * n + k];
        const double g2 = go.x * go.x + go.y * go.y;
        sx.x += go.x * x.x - go.y * x.y;
        sx.y += go.x * x.y + go.y * x.x;
        // |g_o X_ko| sets the rounding level only: an FP32 square root will do
        sa += (double)__builtin_amdgcn_sqrtf((float)(g2 * (x.x * x.x + x.y * x.y)));
        sd += g2 * Wf[(int64_t)o * n + k];
      }
    }
    const double sdt = wdot(g, true).x;
    double2 r = make_double2(0.0, 0.0);
    double D = 0.0, Dt = 0.0, scale = 0.0;
    // three rounds through the partial-sum buffer: (sx), (sd, sa), (sdt)
    pa[tid] = sx;
    __syncthreads();
    if (own)
      for (int q = 0; q < parts; ++q) {
        r.x += pa[q * nk + k].x;
        r.y += pa[q * nk + k].y;
      }
    __syncthreads();
    pa[tid] = make_double2(sd, sa);
    __syncthreads();
    if (own)
      for (int q = 0; q < parts; ++q) {
        D += pa[q * nk + k].x;
        scale += pa[q * nk + k].y;
      }
    __syncthreads();
    pa[tid] = make_double2(sdt, 0.0);
    __syncthreads();
    if (own) {
      for (int q = 0; q < parts; ++q) Dt += pa[q * nk + k].x;
      r.x -= gk.x * D;
      r.y -= gk.y * D;
      scale += sqrt(gk.x * gk.x + gk.y * gk.y) * D;
    }
    const double minv = Dt > 0.0 ? 1.0 / Dt : 0.0;
    r = gauge_project<NT>(r, gk, k, ck, own, n, comp, g, pv, a.single_comp, redp);
    // Preconditioned conjugate gradients in the Chronopoulos-Gear form: per
    // step one operator application w = A u to the preconditioned residual u
    // and one workgroup reduction of gamma = (res, u), delta = (u, w) and
    // |res|^2 together (two barriers a step); the direction's image s = A p
    // follows from s = w + beta s, and (p, A p) = delta - beta gamma / alpha.
    // The inner product is the real one, sum_k Re(a_k^* b_k), for which the
    // operator is self-adjoint.  delta's W part, sum_k Re(u_k^* g_k S_k) with
    // S_k = sum_o W_ko y_o and y_o = g_o u_o^*, equals sum_k Re(y_k S_k): each
    // (tile, part) thread adds the share of its part of the sum.
    double2 x = make_double2(0.0, 0.0), res = r;
    const double2 s0 = block_sum2<NT>(res.x * res.x + res.y * res.y, scale * scale, red);
    // below this |r|^2 the right-hand side is rounding noise: no step
    const double floor2 = kGainFloor * kGainFloor * s0.y;
    const double rr0 = s0.x;
    double2 u = make_double2(minv * res.x, minv * res.y);
    double2 pdir = make_double2(0.0, 0.0), sdir = make_double2(0.0, 0.0);
    double gam_old = 1.0, alpha_old = 1.0;
    int steps = 0;  // workgroup-uniform: every stopping test uses block sums
    for (int cg = 0; cg < a.max_cg; ++cg) {
      if (own) y[k] = cmul(gk, cconj(u));
      __syncthreads();
      const double2 sp = wdot(y, false), yr = y[kr];
      double dterm = row ? yr.x * sp.x - yr.y * sp.y : 0.0, gterm = 0.0, rterm = 0.0;
      if (own) {
        dterm += Dt * (u.x * u.x + u.y * u.y);
        gterm = res.x * u.x + res.y * u.y;
        rterm = res.x * res.x + res.y * res.y;
      }
      pa[tid] = sp;
      const double3 sums = block_sum3<NT>(gterm, dterm, rterm, red);  // its barrier also publishes pa
      const double gam = sums.x, delta = sums.y, rr = sums.z;
      if (!(rr > a.cg_tol2 * rr0) || !(rr > floor2) || !(gam > 0.0)) break;
      const double beta = cg > 0 ? gam / gam_old : 0.0;
      const double eta = delta - beta * gam / alpha_old;
      if (!(eta > 0.0)) break;
      const double alpha = gam / eta;
      if (own) {
        double2 sw = make_double2(0.0, 0.0);
        for (int j = 0; j < parts; ++j) {
          const double2 v = pa[j * nk + k];
          sw.x += v.x;
          sw.y += v.y;
        }
        const double2 gs = cmul(gk, sw);
        const double2 w = make_double2(Dt * u.x + gs.x, Dt * u.y + gs.y);
        pdir = make_double2(u.x + beta * pdir.x, u.y + beta * pdir.y);
        sdir = make_double2(w.x + beta * sdir.x, w.y + beta * sdir.y);
        x.x += alpha * pdir.x;
        x.y += alpha * pdir.y;
        res.x -= alpha * sdir.x;
        res.y -= alpha * sdir.y;
        u = make_double2(minv * res.x, minv * res.y);
      }
      gam_old = gam;
      alpha_old = alpha;
      ++steps;
    }
    x = gauge_project<NT>(x, gk, k, ck, own, n, comp, g, pv, a.single_comp, redp);
    gk.x += x.x;
    gk.y += x.y;
    if (own) g[k] = gk;
    __syncthreads();
    // no step taken: the gains did not change, so every further iteration
    // would repeat this one exactly
    if (steps == 0) break;
  }

  if (own) {
    if (a.gains) a.gains[(int64_t)cell * n + k] = gk;
    a.gw[((int64_t)t * n + k) * a.K + kc] = gk;
  }
}

// The mixed path's solve for large arrays (up to kPeelMaxAnt tiles), with W
// held in registers instead of LDS.  One workgroup of 64 NW threads per cell.
// Wave w takes the columns o of [w OPW, (w + 1) OPW) and lane l the rows
// k = l + 64 j (j < RPL), so that each thread holds the RPL x OPW block of W
// (FP32) it multiplies: each broadcast read of the direction's y_o from LDS
// serves RPL rows, and W is never read from LDS.  The partial sums of the
// NW column blocks meet in LDS; thread k (k < n, the first n threads) owns
// tile k's gain and conjugate-gradient state.  Same iteration, stopping rules
// and arithmetic as k_gain_solve's mixed path (FP32 operator, FP64 sums and
// state), with D_k summed from the same FP32 W.
template <int NW, int RPL>
__global__ __launch_bounds__(64 * NW) void k_gain_solve_rw(GainArgs a) {
  // up to 64 RPL tiles: RPL rows per lane, NW column blocks of OPW
  constexpr int NT = 64 * NW, OPW = 64 * RPL / NW;
  extern __shared__ __align__(16) unsigned char smem[];
  double2 *g = (double2 *)smem;                   // [kPeelMaxAnt] gains
  float2 *y32 = (float2 *)(g + kPeelMaxAnt);      // [kPeelMaxAnt] g_o u_o^* of the current direction
  double2 *pa = (double2 *)(y32 + kPeelMaxAnt);   // [NW][kPeelMaxAnt] column-block partial sums
  float2 *pa32 = (float2 *)pa;                    // the same buffer for the FP32 operator's partials
  double *pv = (double *)(pa + NW * kPeelMaxAnt); // [kPeelMaxAnt] projection scratch
  int *comp = (int *)(pv + kPeelMaxAnt);          // [kPeelMaxAnt] connected component of each tile
  double2 *red = (double2 *)(comp + kPeelMaxAnt); // [2 NT / 64] reduction scratch
  double2 *redp = red + 2 * (NT / 64);            // [NT / 64] reduction scratch of the projections

  const int cl = blockIdx.x, cell = a.cell0 + cl;
  const int t = cell / a.K, kc = cell % a.K;
  const int n = a.n_ant, tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ob = wv * OPW, on = max(0, min(OPW, n - ob));  // this wave's columns (wave-uniform)
  const bool own = tid < n;
  const int k = own ? tid : 0;

  const float2 *X = (const float2 *)a.xt + (int64_t)cl * n * n;  // X[o n + k], zero for o == k
  const float *Wf = (const float *)a.wf + (int64_t)cl * n * n;    // |I|^2 [o n + k], zero for o == k
  float Wr[RPL][OPW];
#pragma unroll
  for (int j = 0; j < RPL; ++j) {
    const int kj = lane + 64 * j;
#pragma unroll
    for (int i = 0; i < OPW; ++i) Wr[j][i] = (kj < n && i < on) ? Wf[(int64_t)(ob + i) * n + kj] : 0.f;
  }
  double2 gk = make_double2(1.0, 0.0);
  const int ck = own ? a.comp[k] : -1;
  if (own) {
    g[k] = gk;
    comp[k] = ck;
  }
  // the gains' and the direction's entries past n stay zero, so that the
  // products with the register copy of W (zero there too) need no bounds
  for (int i = tid; i < kPeelMaxAnt; i += NT) {
    y32[i] = make_float2(0.f, 0.f);
    if (i >= n) g[i] = make_double2(0.0, 0.0);
  }
  __syncthreads();

  for (int it = 0; it < a.n_iter; ++it) {
    // r_k = sum_o g_o X_ko - g_k D_k, D_k = sum_o W_ko |g_o|^2 (W from the
    // table: the same FP32 values as the registers); sa: sum of |g_o X_ko|,
    // for the rounding level of r_k.  One row of this lane at a time, so that
    // the register copy of W stays the only large live state.
    double2 sx[RPL];
    double sd[RPL], sa[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const int kj = lane + 64 * j;
      double2 ax = make_double2(0.0, 0.0);
      double ad = 0.0, aa = 0.0;
      if (kj < n) {
#pragma unroll 4
        for (int i = 0; i < on; ++i) {
          const int o = ob + i;
          const double2 go = g[o];
          const double g2 = go.x * go.x + go.y * go.y;
          const float2 xt = X[(int64_t)o * n + kj];
          const double2 xv = make_double2(xt.x, xt.y);
          ax.x += go.x * xv.x - go.y * xv.y;
          ax.y += go.x * xv.y + go.y * xv.x;
          aa += (double)__builtin_amdgcn_sqrtf((float)(g2 * (xv.x * xv.x + xv.y * xv.y)));
          ad += g2 * (double)Wf[(int64_t)o * n + kj];
        }
      }
      sx[j] = ax;
      sd[j] = ad;
      sa[j] = aa;
    }
    // two rounds through the partial-sum buffer: (sx), (sd, sa)
    double2 r = make_double2(0.0, 0.0);
    double Dt = 0.0, scale = 0.0;
#pragma unroll
    for (int j = 0; j < RPL; ++j)
      if (lane + 64 * j < n) pa[wv * kPeelMaxAnt + lane + 64 * j] = sx[j];
    __syncthreads();
    if (own)
      for (int w = 0; w < NW; ++w) {
        r.x += pa[w * kPeelMaxAnt + k].x;
        r.y += pa[w * kPeelMaxAnt + k].y;
      }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RPL; ++j)
      if (lane + 64 * j < n) pa[wv * kPeelMaxAnt + lane + 64 * j] = make_double2(sd[j], sa[j]);
    __syncthreads();
    if (own) {
      for (int w = 0; w < NW; ++w) {
        Dt += pa[w * kPeelMaxAnt + k].x;
        scale += pa[w * kPeelMaxAnt + k].y;
      }
      r.x -= gk.x * Dt;
      r.y -= gk.y * Dt;
      scale += sqrt(gk.x * gk.x + gk.y * gk.y) * Dt;
    }
    const double minv = Dt > 0.0 ? 1.0 / Dt : 0.0;
    r = gauge_project<NT>(r, gk, k, ck, own, n, comp, g, pv, a.single_comp, redp);
    // conjugate gradients in the Chronopoulos-Gear form, as in k_gain_solve
    double2 x = make_double2(0.0, 0.0), res = r;
    const double2 s0 = block_sum2<NT>(res.x * res.x + res.y * res.y, scale * scale, red);
    const double floor2 = kGainFloor * kGainFloor * s0.y;
    const double rr0 = s0.x;
    double2 u = make_double2(minv * res.x, minv * res.y);
    double2 pdir = make_double2(0.0, 0.0), sdir = make_double2(0.0, 0.0);
    double gam_old = 1.0, alpha_old = 1.0;
    int steps = 0;
    for (int cg = 0; cg < a.max_cg; ++cg) {
      if (own) {
        const double2 yk = cmul(gk, cconj(u));
        y32[k] = make_float2((float)yk.x, (float)yk.y);
      }
      __syncthreads();
      float2 acc[RPL];
#pragma unroll
      for (int j = 0; j < RPL; ++j) acc[j] = make_float2(0.f, 0.f);
#pragma unroll
      for (int i = 0; i < OPW; ++i) {
        const float2 yo = y32[ob + i];
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          acc[j].x = fmaf(Wr[j][i], yo.x, acc[j].x);
          acc[j].y = fmaf(Wr[j][i], yo.y, acc[j].y);
        }
      }
      double dterm = 0.0, gterm = 0.0, rterm = 0.0;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {  // rows past n: zero products and a zero direction entry
        const float2 yj = y32[lane + 64 * j];
        dterm += (double)yj.x * acc[j].x - (double)yj.y * acc[j].y;
        pa32[wv * kPeelMaxAnt + lane + 64 * j] = acc[j];
      }
      if (own) {
        dterm += Dt * (u.x * u.x + u.y * u.y);
        gterm = res.x * u.x + res.y * u.y;
        rterm = res.x * res.x + res.y * res.y;
      }
      const double3 sums = block_sum3<NT>(gterm, dterm, rterm, red);  // its barrier also publishes pa32
      const double gam = sums.x, delta = sums.y, rr = sums.z;
      if (!(rr > a.cg_tol2 * rr0) || !(rr > floor2) || !(gam > 0.0)) break;
      const double beta = cg > 0 ? gam / gam_old : 0.0;
      const double eta = delta - beta * gam / alpha_old;
      if (!(eta > 0.0)) break;
      const double alpha = gam / eta;
      if (own) {
        double2 sw = make_double2(0.0, 0.0);
        for (int w = 0; w < NW; ++w) {
          const float2 v = pa32[w * kPeelMaxAnt + k];
          sw.x += v.x;
          sw.y += v.y;
        }
        const double2 gs = cmul(gk, sw);
        const double2 wk = make_double2(Dt * u.x + gs.x, Dt * u.y + gs.y);
        pdir = make_double2(u.x + beta * pdir.x, u.y + beta * pdir.y);
        sdir = make_double2(wk.x + beta * sdir.x, wk.y + beta * sdir.y);
        x.x += alpha * pdir.x;
        x.y += alpha * pdir.y;
        res.x -= alpha * sdir.x;
        res.y -= alpha * sdir.y;
        u = make_double2(minv * res.x, minv * res.y);
      }
      gam_old = gam;
      alpha_old = alpha;
      ++steps;
    }
    x = gauge_project<NT>(x, gk, k, ck, own, n, comp, g, pv, a.single_comp, redp);
    gk.x += x.x;
    gk.y += x.y;
    if (own) g[k] = gk;
    __syncthreads();
    if (steps == 0) break;
  }

  if (own) {
    if (a.gains) a.gains[(int64_t)cell * n + k] = gk;
    a.gw[((int64_t)t * n + k) * a.K + kc] = gk;
  }
}

// data <- data - g_ant1 g_ant2^* I over the whole [T][B][K] array, one
// visibility per thread (adjacent threads on adjacent channels: coalesced),
// with the gains of cell (t, kc) from the [T][n][K] table the solve wrote
// (adjacent channels adjacent there too).
__global__ __launch_bounds__(256) void k_gain_subtract(GainArgs a) {
  const int64_t total = (int64_t)a.T * a.B * a.K;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kc = (int)(i % a.K);
    const int64_t tb = i / a.K;
    const int b = (int)(tb % a.B), t = (int)(tb / a.B);
    const double2 g1 = a.gw[((int64_t)t * a.n_ant + a.ant1[b]) * a.K + kc];
    const double2 g2 = a.gw[((int64_t)t * a.n_ant + a.ant2[b]) * a.K + kc];
    const double2 m = load_vis(a.model, a.c64, i);
    const double2 v = load_vis(a.data, a.c64, i);
    const double2 mdl = cmul(cmul(g1, cconj(g2)), m);
    if (a.c64)
      ((float2 *)a.data)[i] = make_float2((float)(v.x - mdl.x), (float)(v.y - mdl.y));
    else
      ((double2 *)a.data)[i] = make_double2(v.x - mdl.x, v.y - mdl.y);
  }
}

size_t gain_smem_bytes(int n_ant, bool w64, int threads) {
  const size_t packed = (size_t)n_ant * (n_ant + 1) / 2;
  return kPeelMaxAnt * (2 * sizeof(double2) + sizeof(double) + sizeof(int)) + threads * sizeof(double2) +
         3 * (threads / 64) * sizeof(double2) + packed * (w64 ? sizeof(double) : sizeof(float));  // red, redp
}

template <typename WT, int NT>
static hipError_t launch_solve(const GainArgs &a, hipStream_t s) {
  const size_t sm = gain_smem_bytes(a.n_ant, sizeof(WT) == sizeof(double), NT);
  hipError_t e = hipFuncSetAttribute((const void *)k_gain_solve<WT, NT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gain_solve<WT, NT>), dim3((unsigned)a.ncell), dim3(NT), sm, s, a);
  return hipGetLastError();
}

template <typename TT>
static hipError_t launch_tables(const GainArgs &a, hipStream_t s) {
  constexpr int C = tab_cells<TT>();
  const size_t sm = (size_t)C * a.n_ant * (sizeof(typename TabPair<TT>::type) + sizeof(TT));
  hipLaunchKernelGGL(k_gain_tables<TT>, dim3((unsigned)((a.ncell + C - 1) / C), (unsigned)a.n_ant), dim3(256), sm, s,
                     a);
  return hipGetLastError();
}

bool gain_supported(int n_ant) {
  return n_ant >= 2 && n_ant <= kPeelMaxAnt && gain_smem_bytes(n_ant, false, 1024) <= kPeelSmemMax;
}

hipError_t launch_gain_subtract(const GainArgs &a, hipStream_t s) {
  const int64_t total = (int64_t)a.T * a.B * a.K;
  if (total <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_gain_subtract, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

size_t gain_rw_smem_bytes(int nw) {
  return kPeelMaxAnt * (sizeof(double2) + sizeof(float2) + nw * sizeof(double2) + sizeof(double) + sizeof(int)) +
         3 * nw * sizeof(double2);
}

template <int NW, int RPL>
static hipError_t launch_solve_rw(const GainArgs &a, hipStream_t s) {
  const size_t sm = gain_rw_smem_bytes(NW);
  hipError_t e =
      hipFuncSetAttribute((const void *)k_gain_solve_rw<NW, RPL>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gain_solve_rw<NW, RPL>), dim3((unsigned)a.ncell), dim3(64 * NW), sm, s, a);
  return hipGetLastError();
}

size_t gain_cell_bytes(int n_ant, bool w32) {
  return (size_t)n_ant * n_ant * (w32 ? sizeof(float2) + sizeof(float) : sizeof(double2) + sizeof(double));
}

hipError_t launch_gain(const GainArgs &a, hipStream_t s) {
  if (a.ncell <= 0) return hipSuccess;
  if (!gain_supported(a.n_ant) || a.cell0 < 0 || (int64_t)a.cell0 + a.ncell > (int64_t)a.T * a.K)
    return hipErrorInvalidValue;
  hipError_t e = a.w32 ? launch_tables<float>(a, s) : launch_tables<double>(a, s);
  if (e != hipSuccess) return e;
  // the mixed path (FP32 tables): W in registers, 128 tiles per 4 waves or
  // 256 per 8 waves; the FP64 path: W in LDS, FP64 while it fits
  if (a.w32) return a.n_ant <= 128 ? launch_solve_rw<4, 2>(a, s) : launch_solve_rw<8, 4>(a, s);
  if (gain_smem_bytes(a.n_ant, true, 1024) <= kPeelSmemMax) return launch_solve<double, 1024>(a, s);
  return launch_solve<float, 1024>(a, s);
}

}  // namespace vp
