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
// W (one value per tile pair, packed i < j) sits in LDS for the whole cell;
// residuals are formed in FP64 from the data and model in global memory.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

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

// Sum of v over the workgroup (kTileRows threads); every thread gets the sum.
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kTileRows / 64; ++w) s += red[w];
  return s;
}

// Removes from v (tile k's entry of a vector over tiles) its part along the
// gauge direction i g of k's connected component:
//   v <- v - i g_k (sum_{o in C} Im(g_o^* v_o)) / (sum_{o in C} |g_o|^2).
// Sums run over the tiles in index order (deterministic); pv is LDS scratch.
__device__ __forceinline__ double2 gauge_project(double2 v, double2 gk, int ck, bool own, int n,
                                                 const int *comp, const double2 *g, double *pv) {
  const int tid = threadIdx.x;
  if (own) pv[tid] = ck >= 0 ? gk.x * v.y - gk.y * v.x : 0.0;
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

template <typename WT>
__global__ __launch_bounds__(kTileRows) void k_gain_solve(GainArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double2 *g = (double2 *)smem;                   // [kPeelMaxAnt] gains
  double2 *y = g + kPeelMaxAnt;                   // [kPeelMaxAnt] g_o p_o^* of the current direction
  double *pv = (double *)(y + kPeelMaxAnt);       // [kPeelMaxAnt] projection scratch
  int *comp = (int *)(pv + kPeelMaxAnt);          // [kPeelMaxAnt] connected component of each tile
  double *red = (double *)(comp + kPeelMaxAnt);   // [kTileRows / 64] reduction scratch
  WT *W = (WT *)(red + 8);                        // [n_pairs] |I|^2 per tile pair

  const int cell = blockIdx.x;                    // t * K + k
  const int t = cell / a.K, kc = cell % a.K;
  const int n = a.n_ant, tid = threadIdx.x;
  const int npairs = n * (n - 1) / 2;
  const int64_t base = (int64_t)t * a.B * a.K + kc;  // element (t, b, kc) at base + b K

  for (int p = tid; p < npairs; p += kTileRows) {
    const int b = a.pair_bl[p];
    double w2 = 0.0;
    if (b >= 0) {
      const double2 m = load_vis(a.model, a.c64, base + (int64_t)b * a.K);
      w2 = m.x * m.x + m.y * m.y;
    }
    W[p] = (WT)w2;
  }
  const bool own = tid < n;
  double2 gk = make_double2(1.0, 0.0);
  const int ck = own ? a.comp[tid] : -1;
  if (own) {
    g[tid] = gk;
    comp[tid] = ck;
  }
  __syncthreads();

  for (int it = 0; it < a.n_iter; ++it) {
    // right-hand side and diagonal for tile k
    double2 r = make_double2(0.0, 0.0);
    double D = 0.0, scale = 0.0;  // scale: sum of |terms| of r_k, for its rounding level
    if (own) {
      for (int o = 0; o < n; ++o) {
        if (o == tid) continue;
        const int p = tid < o ? pair_index(n, tid, o) : pair_index(n, o, tid);
        const int b = a.pair_bl[p];
        if (b < 0) continue;
        const double2 go = g[o];
        D += (go.x * go.x + go.y * go.y) * (double)W[p];
        const double2 m = load_vis(a.model, a.c64, base + (int64_t)b * a.K);
        const double2 v = load_vis(a.data, a.c64, base + (int64_t)b * a.K);
        const bool first = a.ant1[b] == tid;  // this tile is ant1 of the baseline
        const double2 gi = first ? gk : go, gj = first ? go : gk;
        const double2 mdl = cmul(cmul(gi, cconj(gj)), m);
        const double2 res = make_double2(v.x - mdl.x, v.y - mdl.y);
        const double2 term = first ? cmul(go, cmul(cconj(m), res)) : cmul(go, cmul(m, cconj(res)));
        r.x += term.x;
        r.y += term.y;
        scale += sqrt((go.x * go.x + go.y * go.y) * (m.x * m.x + m.y * m.y)) *
                 (sqrt(v.x * v.x + v.y * v.y) + sqrt(mdl.x * mdl.x + mdl.y * mdl.y));
      }
    }
    r = gauge_project(r, gk, ck, own, n, comp, g, pv);
    // below this |r|^2 the right-hand side is rounding noise: no step
    const double floor2 = kGainFloor * kGainFloor * block_sum(scale * scale, red);
    // conjugate gradients on the normal equations, from e = 0
    double2 x = make_double2(0.0, 0.0), res = r, pdir = r;
    double rr = block_sum(res.x * res.x + res.y * res.y, red);
    const double rr0 = rr;
    for (int cg = 0; cg < a.max_cg; ++cg) {
      if (!(rr > a.cg_tol2 * rr0) || !(rr > floor2)) break;
      if (own) y[tid] = cmul(gk, cconj(pdir));
      __syncthreads();
      double2 q = make_double2(0.0, 0.0);
      if (own) {
        double2 s = make_double2(0.0, 0.0);
        for (int o = 0; o < n; ++o) {
          if (o == tid) continue;
          const int p = tid < o ? pair_index(n, tid, o) : pair_index(n, o, tid);
          const double wv = (double)W[p];
          const double2 yo = y[o];
          s.x += wv * yo.x;
          s.y += wv * yo.y;
        }
        const double2 gs = cmul(gk, s);
        q = make_double2(D * pdir.x + gs.x, D * pdir.y + gs.y);
      }
      const double pq = block_sum(pdir.x * q.x + pdir.y * q.y, red);
      if (!(pq > 0.0)) break;
      const double alpha = rr / pq;
      x.x += alpha * pdir.x;
      x.y += alpha * pdir.y;
      res.x -= alpha * q.x;
      res.y -= alpha * q.y;
      const double rn = block_sum(res.x * res.x + res.y * res.y, red);
      const double beta = rn / rr;
      pdir = make_double2(res.x + beta * pdir.x, res.y + beta * pdir.y);
      rr = rn;
    }
    x = gauge_project(x, gk, ck, own, n, comp, g, pv);
    gk.x += x.x;
    gk.y += x.y;
    __syncthreads();
    if (own) g[tid] = gk;
    __syncthreads();
  }

  if (a.gains && own) a.gains[(int64_t)cell * n + tid] = gk;
  if (a.subtract) {
    for (int b = tid; b < a.B; b += kTileRows) {
      const int64_t i = base + (int64_t)b * a.K;
      const double2 m = load_vis(a.model, a.c64, i);
      const double2 v = load_vis(a.data, a.c64, i);
      const double2 mdl = cmul(cmul(g[a.ant1[b]], cconj(g[a.ant2[b]])), m);
      if (a.c64)
        ((float2 *)a.data)[i] = make_float2((float)(v.x - mdl.x), (float)(v.y - mdl.y));
      else
        ((double2 *)a.data)[i] = make_double2(v.x - mdl.x, v.y - mdl.y);
    }
  }
}

size_t gain_smem_bytes(int n_ant, bool w64) {
  const size_t npairs = (size_t)n_ant * (n_ant - 1) / 2;
  return kPeelMaxAnt * (2 * sizeof(double2) + sizeof(double) + sizeof(int)) + 8 * sizeof(double) +
         npairs * (w64 ? sizeof(double) : sizeof(float));
}

hipError_t launch_gain(const GainArgs &a, hipStream_t s) {
  const int64_t cells = (int64_t)a.T * a.K;
  if (cells <= 0) return hipSuccess;
  if (cells > 0x7fffffff || a.n_ant < 2 || a.n_ant > kPeelMaxAnt) return hipErrorInvalidValue;
  const bool w64 = gain_smem_bytes(a.n_ant, true) <= kPeelSmemMax;
  const size_t sm = gain_smem_bytes(a.n_ant, w64);
  if (sm > kPeelSmemMax) return hipErrorInvalidValue;
  if (w64) {
    hipError_t e = hipFuncSetAttribute((const void *)k_gain_solve<double>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gain_solve<double>, dim3((unsigned)cells), dim3(kTileRows), sm, s, a);
  } else {
    hipError_t e = hipFuncSetAttribute((const void *)k_gain_solve<float>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gain_solve<float>, dim3((unsigned)cells), dim3(kTileRows), sm, s, a);
  }
  return hipGetLastError();
}

}  // namespace vp
