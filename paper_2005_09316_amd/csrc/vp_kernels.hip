// vp_kernels.hip -- gfx950 kernels of libvp.
//
// Direct-Fourier visibility prediction (Line et al., Sec. 3): for every
// (time, baseline, channel) visibility, sum over point, Gaussian and shapelet
// components of flux x uv-envelope x phase term (Eqs. measure_eq_discrete,
// env_visi_def, gauss-env, shape-env).  The work is split in two kernels per
// call, each over tiles of 256 (time, baseline) rows x a block of channels:
//
//   k_pg_tile   points then Gaussians.  One thread owns one row and
//               kPgChan channels; component lists are staged through LDS in
//               chunks and read as wave-uniform broadcasts.  Phase per
//               (row, component) is t0 = u l + v m + w (n-1) in metres (FP64);
//               per channel t = t0 nu/c, reduced to a fraction of a turn in
//               FP64, then sin/cos of 2 pi t in FP32 on the transcendental
//               unit (input in turns); with uniformly spaced channels the
//               mixed path evaluates 3 of every 8 channels and the channel
//               step and rotates the other phasors.  Sums are plain FP32
//               over kFlush components; the mixed path adds two such
//               partials in FP32 and then into FP64 sums (the FP32-only
//               path: Kahan-compensated FP32 sums).
//   k_shp_mfma  shapelets.  Per (visibility, shapelet): rotate uvw into the
//               shapelet's frame, walk the rescaled Hermite recurrence for
//               both axes (FP64 on the mixed path: it costs the same issue
//               slots as FP32 on this chip and removes the argument-rounding
//               and underflow error of an FP32 recurrence), contract against
//               the signed coefficient matrix on MFMA (n1 on M, n2 on K split
//               by parity into real/imaginary accumulators, 32 visibilities on
//               N; 32 x 32 blocks that meet the n1 + n2 <= N triangle only;
//               v_mfma_f32_32x32x16_bf16 on 3-way BF16 splits of the FP64
//               values on the mixed path, v_mfma_f32_32x32x2_f32 on the
//               FP32-only path), fold each block's n1 sum against the first
//               axis (FP64 on the mixed path), and add flux x envelope x
//               phase into an FP64 accumulator held in LDS.
//   k_shp_fp64  the FP64 path of the shapelet term on the vector ALU (and
//               the lookup-table variant of the basis).
//
// All arithmetic is done with the exponent sign +1; a sign of -1 is applied
// by conjugating at the output, which is exact.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "vp_internal.h"

namespace vp {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__constant__ double c_sqn[128];   // sqrt(n)
__constant__ double c_isqn1[128]; // 1 / sqrt(n + 1)
__constant__ double c_half[128];   // n / 2
// scales of the rescaled Hermite values (see shp_tile): [0] = s_16 / s_0,
// [k] = s_{32k+16} / s_{32k-16} for k = 1, 2, 3, with s_n = sqrt(2^n / n!)
__constant__ double c_sc[4];

static constexpr double kPiM14 = 0.75112554446494248285870300477622; // pi^(-1/4)
static constexpr double kHalfLog2e = 0.72134752044448170367996234050095; // log2(e) / 2

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// The hardware dispatches consecutive workgroups round-robin over the 8 XCDs;
// give each XCD a contiguous range of logical tiles so that tiles sharing a
// channel block (and its flux-table rows) share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nt) {
  const int q = nt >> 3, r = nt & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// cos/sin of 2 pi t for an FP64 phase in turns: exact FP64 reduction to
// [0, 1), then the FP32 transcendental unit (which takes turns).
__device__ __forceinline__ void turns_sincos_mixed(double t, float &c, float &s) {
  const float r = (float)__builtin_amdgcn_fract(t);
  s = __builtin_amdgcn_sinf(r);
  c = __builtin_amdgcn_cosf(r);
}

__device__ __forceinline__ void turns_sincos_f32(float t, float &c, float &s) {
  const float r = __builtin_amdgcn_fractf(t);
  s = __builtin_amdgcn_sinf(r);
  c = __builtin_amdgcn_cosf(r);
}

__device__ __forceinline__ void turns_sincos_f64(double t, double &c, double &s) {
  const double r = t - rint(t);  // exact, |r| <= 1/2
  sincospi(2.0 * r, &s, &c);
}

template <typename T>
__device__ __forceinline__ void kahan_add(T &sum, T &cmp, T x) {
  const T y = x - cmp;
  const T t = sum + y;
  cmp = (t - sum) - y;
  sum = t;
}

// ---------------------------------------------------------------------------
// per-(sky, observation) tables
// ---------------------------------------------------------------------------

// Direction cosines of every component relative to the phase centre, the
// Gaussian envelope's quadratic form, and each shapelet's frame vectors.
__device__ __forceinline__ void derive_one(const DeriveArgs &a, int j) {
  const double ra = a.ra[j], dec = a.dec[j];
  const double da = ra - a.ra0;
  const double sd = sin(dec), cd = cos(dec), sd0 = sin(a.dec0), cd0 = cos(a.dec0);
  const double sda = sin(da), cda = cos(da);
  const double l = cd * sda;
  const double m = sd * cd0 - cd * sd0 * cda;
  const double n = sd * sd0 + cd * cd0 * cda;
  const double nm1 = -(l * l + m * m) / (1.0 + n);
  a.d.pos[j] = make_double4(l, m, nm1, 0.0);
  if (j >= a.P && j < a.P + a.G) {
    // exponent of Eq. gauss-env in base 2:
    //   q = pi^2 / (4 ln2 ln2) * (kx^2 maj^2 + ky^2 min^2),
    //   kx = cos(pa) v + sin(pa) u, ky = -sin(pa) v + cos(pa) u
    // expanded in u^2, v^2, u v (metres; the channel scales it by (nu/c)^2).
    const int g = j - a.P;
    const double pa = a.g_pa[g], sp = sin(pa), cp = cos(pa);
    const double M2 = a.g_maj[g] * a.g_maj[g], N2 = a.g_min[g] * a.g_min[g];
    const double k = 3.14159265358979323846 * 3.14159265358979323846 /
                     (4.0 * 0.69314718055994530942 * 0.69314718055994530942);
    a.d.gq[g] = make_double4(k * (sp * sp * M2 + cp * cp * N2),   // u^2
                             k * (cp * cp * M2 + sp * sp * N2),   // v^2
                             k * 2.0 * sp * cp * (M2 - N2),       // u v
                             0.0);
  } else if (j >= a.P + a.G) {
    // Shapelet frame: (u', v', w') = T(ra_j, dec_j) T(ra0, dec0)^T (u, v, w),
    // T's rows being the east, north and pointing unit vectors.  Then
    // a = kappa beta1 (cos(pa) v' + sin(pa) u'), b = kappa beta2 (cos(pa) u' - sin(pa) v').
    const int s = j - a.P - a.G;
    const double sa0 = sin(a.ra0), ca0 = cos(a.ra0), sa = sin(ra), ca = cos(ra);
    const double T0[3][3] = {{-sa0, ca0, 0.0}, {-sd0 * ca0, -sd0 * sa0, cd0}, {cd0 * ca0, cd0 * sa0, sd0}};
    const double Tj[2][3] = {{-sa, ca, 0.0}, {-sd * ca, -sd * sa, cd}};
    double R[2][3];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) R[r][c] = Tj[r][0] * T0[c][0] + Tj[r][1] * T0[c][1] + Tj[r][2] * T0[c][2];
    const double kappa = 3.14159265358979323846 / sqrt(2.0 * 0.69314718055994530942);
    const double pa = a.s_pa[s], sp = sin(pa), cp = cos(pa);
    const double ka = kappa * a.s_beta1[s], kb = kappa * a.s_beta2[s];
    double *f = a.d.sframe + 12 * s;
    for (int c = 0; c < 3; ++c) {
      f[c] = ka * (sp * R[0][c] + cp * R[1][c]);
      f[3 + c] = kb * (cp * R[0][c] - sp * R[1][c]);
    }
    f[6] = l; f[7] = m; f[8] = nm1; f[9] = 0.0; f[10] = 0.0; f[11] = 0.0;
  }
}

// Out of line, so that the table kernels below and the serving kernel's
// table items run the same machine code and build bitwise identical tables.
__device__ __noinline__ void derive_ool(const DeriveArgs &a, int j) { derive_one(a, j); }

__global__ void k_derive(DeriveArgs a) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < a.P + a.G + a.S) derive_ool(a, j);
}

// S_j(nu_k) = S_ref (nu_k / nu_ref)^alpha * B_j(nu_k) for flat index
// idx = j * Kpad + k (zero in the channel padding).
__device__ __forceinline__ void flux_one(const FluxArgs &a, int64_t idx) {
  const int j = (int)(idx / a.Kpad), k = (int)(idx % a.Kpad);
  double S = 0.0;
  if (k < a.K) {
    const double nu = a.freq[k];
    S = a.sref[j] * pow(nu / a.nu_ref, a.alpha[j]);
    if (a.lpow && j >= a.j0) {
      // spectral term q of a shapelet's coefficients: ln(nu / nu_ref)^q
      const double x = log(nu / a.nu_ref);
      for (int q = a.lpow[j - a.j0]; q > 0; --q) S *= x;
    }
    if (a.beam_fwhm > 0.0) {
      // distance from the phase centre: sin(rho) = sqrt(l^2 + m^2)
      const double dec = a.dec[j], da = a.ra[j] - a.ra0;
      const double l = cos(dec) * sin(da);
      const double m = sin(dec) * cos(a.dec0) - cos(dec) * sin(a.dec0) * cos(da);
      const double rho = asin(sqrt(l * l + m * m));
      const double th = a.beam_fwhm * a.beam_nu_ref / nu;
      S *= exp(-4.0 * 0.69314718055994530942 * rho * rho / (th * th));
    }
  }
  a.d.flux32[idx] = (float)S;
  a.d.flux64[idx] = S;
}

__device__ __noinline__ void flux_ool(const FluxArgs &a, int64_t idx) { flux_one(a, idx); }

__global__ void k_flux(FluxArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)a.J * a.Kpad) flux_ool(a, idx);
}

// Coefficient tiles.  Signed coefficients C''[n1][n2] = C[n1][n2] (-1)^floor((n1+n2)/2),
// so that xi = sum_{n1+n2 even} C'' phi phi + i sum_{n1+n2 odd} C'' phi phi
// equals sum C i^(n1+n2) phi phi.  The MFMA tiles hold the 32 x 32 blocks that
// meet the triangle, in pair order (chunk ch of 32 n2-orders outer, row block
// mb inner, 32 (ch + mb) <= N):
//   a32: [pair][parity][s][lane]: lane l supplies A[row = l % 32][k = l / 32] of
//        the 32x32x2 FP32 MFMA for n1 = 32 mb + l % 32,
//        n2 = 32 ch + 4 s + 2 (l / 32) + parity;
//   abf: [part][pair][parity][lane][8]: BF16 hi/mid/lo splits for the
//        32x32x16 MFMA, element e of lane l: n1 = 32 mb + l % 32,
//        n2 = 32 ch + 16 (l / 32) + 2 e + parity;
//   c64: [n1][ld], zero outside the triangle.
// The MFMA tiles hold C'' (s_n1 / s_{32 mb + 16}) (s_n2 / s_{32 ch + 16}): the
// kernels walk the rescaled Hermite values of psi_next (FP64 bases at the
// middle of each block), and these factors undo the rescaling.

// s_n / s_b with s_n = sqrt(2^n / n!), as a product of sqrt(2 / (k + 1)).
__host__ __device__ inline double herm_scale(int b, int n) {
  double r = 1.0;
  for (int k = b; k < n; ++k) r *= sqrt(2.0 / (k + 1));
  for (int k = n; k < b; ++k) r /= sqrt(2.0 / (k + 1));
  return r;
}

__device__ __forceinline__ double signed_coeff(const double *c, int N, int n1, int n2) {
  if (n1 < 0 || n2 < 0 || n1 > N || n2 > N - n1) return 0.0;
  const int64_t off = (int64_t)n1 * (N + 1) - (int64_t)n1 * (n1 - 1) / 2;
  const double v = c[off + n2];
  return (((n1 + n2) >> 1) & 1) ? -v : v;
}

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// (chunk, row block) of pair p; q = N / 32
__device__ __forceinline__ void pair_coords(int q, int p, int &ch, int &mb) {
  ch = 0;
  while (p > q - ch) {
    p -= q - ch + 1;
    ++ch;
  }
  mb = p;
}

__global__ void k_tiles(TileBuildArgs a) {
  const int s = blockIdx.y;
  if (s >= a.S) return;
  const int N = a.nmax[s];
  const double *C = a.coeffs + a.coeff_off[s];
  const int q = N / 32, npairs = shp_pairs(N);
  // FP32 MFMA tiles
  const int n32 = npairs * kA32PerPair;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n32; i += gridDim.x * blockDim.x) {
    const int lane = i & 63, st = (i >> 6) & 7, par = (i >> 9) & 1, p = i >> 10;
    int ch, mb;
    pair_coords(q, p, ch, mb);
    const int n1 = 32 * mb + (lane & 31), n2 = 32 * ch + 4 * st + 2 * (lane >> 5) + par;
    const double v = signed_coeff(C, N, n1, n2);
    a.a32[a.a32_off[s] + i] =
        v == 0.0 ? 0.f : (float)(v * herm_scale(32 * mb + 16, n1) * herm_scale(32 * ch + 16, n2));
  }
  // FP64 dense
  const int ld = a.c64_ld[s];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (N + 1) * ld; i += gridDim.x * blockDim.x) {
    const int n1 = i / ld, n2 = i % ld;
    a.c64[a.c64_off[s] + i] = signed_coeff(C, N, n1, n2);
  }
  // BF16 three-way split tiles
  const int nbf = npairs * kAbfPerPair;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nbf; i += gridDim.x * blockDim.x) {
    const int e = i & 7, lane = (i >> 3) & 63, par = (i >> 9) & 1, p = i >> 10;
    int ch, mb;
    pair_coords(q, p, ch, mb);
    const int n1 = 32 * mb + (lane & 31), n2 = 32 * ch + 16 * (lane >> 5) + 2 * e + par;
    const double v = signed_coeff(C, N, n1, n2);
    // split the FP64 value itself: each residual is formed in FP64 (exactly),
    // so the three parts carry ~27 bits instead of an FP32 rounding's 24
    const double x = v == 0.0 ? 0.0 : v * herm_scale(32 * mb + 16, n1) * herm_scale(32 * ch + 16, n2);
    const uint16_t hi = bf16_rne((float)x);
    const double r1 = x - (double)bf16_to_f(hi);
    const uint16_t mid = bf16_rne((float)r1);
    const double r2 = r1 - (double)bf16_to_f(mid);
    const uint16_t lo = bf16_rne((float)r2);
    uint16_t *dst = a.abf + a.abf_off[s];
    dst[i] = hi;
    dst[nbf + i] = mid;
    dst[2 * nbf + i] = lo;
  }
}

// ---------------------------------------------------------------------------
// point + Gaussian tile kernel
// ---------------------------------------------------------------------------

template <int PREC>
struct PgTypes {
  typedef float acc_t;
};
template <>
struct PgTypes<kFP64> {
  typedef double acc_t;
};

template <typename T>
struct PgSmem {
  double4 pos[kChunk];
  double4 gq[kChunk];
  T flux[kChunk][kPgChan];
};

// One tile: kTileRows rows x kPgChan channels starting at channel block cb.
// UNI (uniformly spaced channels): on the mixed path the phasors of channels
// 0, 3 and 6 of the tile are evaluated (FP64 phase, FP32 sincos) and the
// others are those rotated by one channel step, e^{+-2 pi i t0 dnu/c}: 4
// sincos and 5 complex rotations per (row, component) instead of 8 sincos,
// with at most one rotation between a channel and an evaluated phasor.  On
// the FP64 path channel 0 and the step are evaluated and channels 1-7 are
// reached by successive rotations.
template <int PREC, bool UNI = false>
__device__ __forceinline__ void pg_tile(const TileArgs &a, int rb, int cb,
                                        PgSmem<typename PgTypes<PREC>::acc_t> &sm) {
  static_assert(!UNI || ((PREC == kMixed || PREC == kFP64) && kPgChan == 8),
                "channel rotation: mixed and FP64 paths, 8-channel tiles");
  typedef typename PgTypes<PREC>::acc_t acc_t;
  constexpr int KB = kPgChan;
  double4 *s_pos = sm.pos;
  double4 *s_gq = sm.gq;
  auto &s_flux = sm.flux;
  const int k0 = cb * KB;
  const int tid = threadIdx.x;
  const int64_t row = (int64_t)rb * kTileRows + tid;
  const bool valid = row < a.nrows;
  const int64_t rowc = valid ? row : a.nrows - 1;
  const double u = a.uvw[3 * rowc], v = a.uvw[3 * rowc + 1], w = a.uvw[3 * rowc + 2];

  double f[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) f[k] = a.fk[k0 + k];

  // Partial sums over kFlush components in acc_t; across them, the mixed
  // path adds each pair of partials in FP32 (hld + prt; the pair's rounding
  // error stays within kFlush units of roundoff of its terms' magnitude) and
  // that into FP64 sums (FP64 adds issue at the FP32 rate here, and three
  // operations per value and pair replace Kahan's eight), the FP32-only path
  // keeps Kahan-compensated FP32 sums and the FP64 path Kahan-compensated
  // FP64 sums of its FP64 partials.
  acc_t sum_re[KB], sum_im[KB], cmp_re[KB], cmp_im[KB], prt_re[KB], prt_im[KB], hld_re[KB], hld_im[KB];
  double dsum_re[KB], dsum_im[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    sum_re[k] = sum_im[k] = cmp_re[k] = cmp_im[k] = prt_re[k] = prt_im[k] = hld_re[k] = hld_im[k] = 0;
    dsum_re[k] = dsum_im[k] = 0.0;
  }

  // FP32-path copies of the row's coordinates
  const float uf = (float)u, vf = (float)v, wf = (float)w;
  float ff[KB], f2[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    ff[k] = (float)f[k];
    f2[k] = (float)(f[k] * f[k]);
  }
  const acc_t uu = (acc_t)(u * u), vv = (acc_t)(v * v), uv = (acc_t)(u * v);
  // anchors of the rotation scheme: nu/c of tile channels 3 and 6 on the
  // uniform grid (also when they lie past the last channel)
  const double fa3 = fma(3.0, a.dfk, f[0]), fa6 = fma(6.0, a.dfk, f[0]);

  const int J0[2] = {0, a.P};
  const int JN[2] = {a.P, a.P + a.G};
#pragma unroll
  for (int kind = 0; kind < 2; ++kind) {  // 0: points, 1: Gaussians
    for (int j0 = J0[kind]; j0 < JN[kind]; j0 += kChunk) {
      const int n = min(kChunk, JN[kind] - j0);
      __syncthreads();
      if (tid < n) {
        s_pos[tid] = a.d.pos[j0 + tid];
        if (kind == 1) s_gq[tid] = a.d.gq[j0 - a.P + tid];
      }
      for (int i = tid; i < n * KB; i += kTileRows) {
        const int jj = i / KB, k = i % KB;
        const int64_t fi = (int64_t)(j0 + jj) * a.Kpad + k0 + k;
        if (PREC == kFP64)
          s_flux[jj][k] = (acc_t)a.d.flux64[fi];
        else
          s_flux[jj][k] = (acc_t)a.d.flux32[fi];
      }
      __syncthreads();
      // one component's terms into the plain partial sums
      auto term = [&](int jj) {
        const double4 p = s_pos[jj];
        acc_t Q = 0;
        if (kind == 1) {
          const double4 g = s_gq[jj];
          if (PREC == kFP64)
            Q = fma(g.x, u * u, fma(g.y, v * v, g.z * (u * v)));
          else
            Q = fmaf((float)g.x, (float)uu, fmaf((float)g.y, (float)vv, (float)g.z * (float)uv));
        }
        if (PREC == kFP64 && UNI) {
          // FP64: channel 0's phasor and the channel step are evaluated,
          // channels 1-7 follow by successive rotations (each adds ~2e-16 of
          // the term: FP64 keeps a chain of seven far below its error bar)
          const double t0 = fma(u, p.x, fma(v, p.y, w * p.z));
          double c[KB], s[KB], cd, sd;
          turns_sincos_f64(t0 * f[0], c[0], s[0]);
          turns_sincos_f64(t0 * a.dfk, cd, sd);
#pragma unroll
          for (int k = 1; k < KB; ++k) {
            c[k] = fma(c[k - 1], cd, -s[k - 1] * sd);
            s[k] = fma(s[k - 1], cd, c[k - 1] * sd);
          }
          // Gaussian envelope 2^(-Q f_k^2) on the same grid f_k = f_0 + k df:
          // e_{k+1} = e_k r_k and r_{k+1} = r_k q, with r_0 = 2^(-Q df (2 f_0 + df))
          // and q = 2^(-2 Q df^2) (three exponentials instead of eight)
          double e = 1.0, r = 1.0, q = 1.0;
          if (kind == 1) {
            e = exp2(-(double)Q * (f[0] * f[0]));
            r = exp2(-(double)Q * a.dfk * (2.0 * f[0] + a.dfk));
            q = exp2(-2.0 * (double)Q * a.dfk * a.dfk);
          }
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            double S = (double)s_flux[jj][k];
            if (kind == 1) {
              S *= e;
              e *= r;
              r *= q;
            }
            prt_re[k] = fma(S, c[k], (double)prt_re[k]);
            prt_im[k] = fma(S, s[k], (double)prt_im[k]);
          }
        } else if (PREC == kFP64) {
          const double t0 = fma(u, p.x, fma(v, p.y, w * p.z));
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            double c, s;
            turns_sincos_f64(t0 * f[k], c, s);
            double S = (double)s_flux[jj][k];
            if (kind == 1) S *= exp2(-(double)Q * (f[k] * f[k]));
            prt_re[k] = fma(S, c, (double)prt_re[k]);
            prt_im[k] = fma(S, s, (double)prt_im[k]);
          }
        } else if (PREC == kFP32) {
          const float t0 = fmaf(uf, (float)p.x, fmaf(vf, (float)p.y, wf * (float)p.z));
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            float c, s;
            turns_sincos_f32(t0 * ff[k], c, s);
            float S = (float)s_flux[jj][k];
            if (kind == 1) S *= __builtin_amdgcn_exp2f(-(float)Q * f2[k]);
            prt_re[k] = fmaf(S, c, (float)prt_re[k]);
            prt_im[k] = fmaf(S, s, (float)prt_im[k]);
          }
        } else if (UNI) {
          const double t0 = fma(u, p.x, fma(v, p.y, w * p.z));
          float c[KB], s[KB], cd, sd;
          turns_sincos_mixed(t0 * f[0], c[0], s[0]);
          turns_sincos_mixed(t0 * fa3, c[3], s[3]);
          turns_sincos_mixed(t0 * fa6, c[6], s[6]);
          turns_sincos_mixed(t0 * a.dfk, cd, sd);
          // one step up from channels 0, 3, 6; one step down from 3, 6
          c[1] = fmaf(c[0], cd, -s[0] * sd);
          s[1] = fmaf(s[0], cd, c[0] * sd);
          c[4] = fmaf(c[3], cd, -s[3] * sd);
          s[4] = fmaf(s[3], cd, c[3] * sd);
          c[7] = fmaf(c[6], cd, -s[6] * sd);
          s[7] = fmaf(s[6], cd, c[6] * sd);
          c[2] = fmaf(c[3], cd, s[3] * sd);
          s[2] = fmaf(s[3], cd, -c[3] * sd);
          c[5] = fmaf(c[6], cd, s[6] * sd);
          s[5] = fmaf(s[6], cd, -c[6] * sd);
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            float S = (float)s_flux[jj][k];
            if (kind == 1) S *= __builtin_amdgcn_exp2f(-(float)Q * f2[k]);
            prt_re[k] = fmaf(S, c[k], (float)prt_re[k]);
            prt_im[k] = fmaf(S, s[k], (float)prt_im[k]);
          }
        } else {
          const double t0 = fma(u, p.x, fma(v, p.y, w * p.z));
#pragma unroll
          for (int k = 0; k < KB; ++k) {
            float c, s;
            turns_sincos_mixed(t0 * f[k], c, s);
            float S = (float)s_flux[jj][k];
            if (kind == 1) S *= __builtin_amdgcn_exp2f(-(float)Q * f2[k]);
            prt_re[k] = fmaf(S, c, (float)prt_re[k]);
            prt_im[k] = fmaf(S, s, (float)prt_im[k]);
          }
        }
      };
      // mixed path: a group's first kFlush terms are held aside and added to
      // the second kFlush terms' partial in FP32 before the FP64 add
      auto hold_partials = [&]() {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          hld_re[k] = prt_re[k];
          hld_im[k] = prt_im[k];
          prt_re[k] = prt_im[k] = 0;
        }
      };
      auto flush_partials = [&]() {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          if constexpr (PREC == kMixed) {
            dsum_re[k] += (double)(prt_re[k] + hld_re[k]);
            dsum_im[k] += (double)(prt_im[k] + hld_im[k]);
            hld_re[k] = hld_im[k] = 0;
          } else {
            kahan_add(sum_re[k], cmp_re[k], prt_re[k]);
            kahan_add(sum_im[k], cmp_im[k], prt_im[k]);
          }
          prt_re[k] = prt_im[k] = 0;
        }
      };
      // groups of kGroup components, unrolled, then the remainder
      constexpr int kGroup = PREC == kMixed ? kFlushMixed : kFlush;
      int jg = 0;
      // FP64 terms hold twice the registers: two at a time keep two waves per SIMD
      constexpr int kUnroll = PREC == kFP64 ? 2 : kGroup;
      for (; jg + kGroup <= n; jg += kGroup) {
#pragma unroll kUnroll
        for (int jo = 0; jo < kGroup; ++jo) {
          if (kGroup > kFlush && jo == kFlush) hold_partials();
          term(jg + jo);
        }
        flush_partials();
      }
      if (jg < n) {
        for (int jj = jg; jj < n; ++jj) {
          if (kGroup > kFlush && jj - jg == kFlush) hold_partials();
          term(jj);
        }
        flush_partials();
      }
    }
  }

  if (!valid) return;
  const int64_t base = row * a.K;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    if (k0 + k >= a.K) break;
    const int64_t idx = base + k0 + k;
    const double tre = PREC == kMixed ? dsum_re[k] : (double)sum_re[k] - (double)cmp_re[k];
    const double tim = PREC == kMixed ? dsum_im[k] : (double)sum_im[k] - (double)cmp_im[k];
    if (a.c64) {
      float re = (float)tre, im = (float)tim;
      if (a.conj) im = -im;
      float2 *o = (float2 *)a.vis + idx;
      if (a.subtract) {
        const float2 d = *o;
        *o = make_float2(d.x - re, d.y - im);
      } else {
        *o = make_float2(re, im);
      }
    } else {
      double re = tre, im = tim;
      if (a.conj) im = -im;
      double2 *o = (double2 *)a.vis + idx;
      if (a.subtract) {
        const double2 d = *o;
        *o = make_double2(d.x - re, d.y - im);
      } else {
        *o = make_double2(re, im);
      }
    }
  }
}

template <int PREC, bool UNI = false>
__global__ __launch_bounds__(kTileRows) void k_pg_tile(TileArgs a) {
  __shared__ PgSmem<typename PgTypes<PREC>::acc_t> sm;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  pg_tile<PREC, UNI>(a, tile % a.n_rb, tile / a.n_rb, sm);
}

// ---------------------------------------------------------------------------
// shapelet tile on MFMA (mixed and FP32-only paths)
// ---------------------------------------------------------------------------

// Hermite recurrence step, phi_{n+1} = (sqrt2 x phi_n - sqrt(n) phi_{n-1}) / sqrt(n+1).
template <typename R>
__device__ __forceinline__ R herm_step(R sx, R pn, R pm1, int n) {
  return (R)c_isqn1[n] * fma(sx, pn, -(R)c_sqn[n] * pm1);
}

// Rescaled Hermite functions.  With s_n = sqrt(2^n / n!) and a base order b,
// u_n = phi_n s_b / s_n obeys u_{n+1} = x u_n - (n / 2) u_{n-1}: two
// operations per order and a constant that is a short immediate (n / 2 is a
// half-integer).  The MFMA path walks u with b at the middle of each 32-order
// block (|log10 (s_b / s_n)| <= 14 there) and multiplies the coefficient tiles
// by (s_n1 / s_b1)(s_n2 / s_b2), so that the products are unchanged.
template <typename R>
__device__ __forceinline__ R psi_next(R x, R un, R um1, R half_n) {
  return fma(x, un, -half_n * um1);
}

// Contraction modes: FP32 MFMA, or the coefficients and the second axis's
// Hermite values split into BF16 parts (x = hi + mid + lo) with the partial
// products summed on v_mfma_f32_32x32x16_bf16: 3 parts / 6 products, or
// 2 parts / 3 products.
enum Contraction : int { kCmF32 = 0, kCmBf16x2 = 2, kCmBf16x3 = 3 };

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// LDS of the shapelet tile: the coefficient blocks of one shapelet and the
// tile's visibility sums (one slot per thread and channel, FP64 on the mixed
// paths; kept here rather than in registers, which the MFMA loop needs).
template <int CM>
struct ShpA {
  float A[kPairsMax * kA32PerPair];
};
template <>
struct ShpA<kCmBf16x2> {
  uint4 A[2 * kPairsMax * kAbfPerPair / 8];
};
template <>
struct ShpA<kCmBf16x3> {
  uint4 A[3 * kPairsMax * kAbfPerPair / 8];
};
template <int CM>
struct ShpSmem : ShpA<CM> {
  double acc_re[kShpChan][kTileRows], acc_im[kShpChan][kTileRows];
};

// Per (visibility, shapelet) start value and phasor.  The synthetic envelopes
// reach ~15x their value at the uv origin, so on the mixed path these O(1)
// steps run in FP64 (exp, sincospi, product and sum) to keep their relative
// error from being magnified against the component's total flux.
template <typename R>
__device__ __forceinline__ R shp_phi0(R x);
template <>
__device__ __forceinline__ double shp_phi0<double>(double x) {
  return kPiM14 * exp(-0.5 * x * x);
}
template <>
__device__ __forceinline__ float shp_phi0<float>(float x) {
  return (float)kPiM14 * __builtin_amdgcn_exp2f(-x * x * (float)kHalfLog2e);
}

// Exchange between the two halves of a wave (v_permlane32_swap).  Every lane
// passes (p, q); afterwards lanes 0-31 hold (their own p, the p of lane + 32)
// and lanes 32-63 hold (the q of lane - 32, their own q).  When p is the value
// the lower half needs from a lane's visibility and q the one the upper half
// needs, p ends up as the value for the lower half's visibility and q as the
// value for the upper half's visibility, in every lane.
__device__ __forceinline__ void half_swap(float &p, float &q) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(p), __float_as_uint(q), false, false);
  p = __uint_as_float(r[0]);
  q = __uint_as_float(r[1]);
}
__device__ __forceinline__ void half_swap(uint32_t &p, uint32_t &q) {
  const auto r = __builtin_amdgcn_permlane32_swap(p, q, false, false);
  p = r[0];
  q = r[1];
}
// Fold one 32 x 32 block's FP32 accumulators into the DOT-precision sums:
// walk the first-axis recurrence (rescaled, psi_next) over the block's rows
// n0 + 8 g + r (this lane's visibility), 8 rows at a time, bring each row value to the lanes
// whose accumulator holds that row (half_swap) and add value x accumulator.
// Accumulator register i of a lane in half h holds block row
// 8 (i / 4) + 4 h + i % 4, of parity i % 2; even-n2 accumulators (E) pair
// with even rows for the real part.  Only the first ng 8-row groups are
// walked and folded (the rest of the block lies outside the triangle); with
// ng = 4, (prev, cur) leave as the next block's start values.
template <typename REC, typename DOT>
__device__ __forceinline__ void shp_fold(REC x, REC &prev, REC &cur, int n0, int ng, const floatx16 &E0,
                                         const floatx16 &O0, const floatx16 &E1, const floatx16 &O1, DOT &xr0,
                                         DOT &xi0, DOT &xr1, DOT &xi1) {
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    if (g < ng) {
    REC ra[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      ra[r] = cur;
      const REC nx = psi_next<REC>(x, cur, prev, (REC)(0.5 * (n0 + 8 * g + r)));
      prev = cur;
      cur = nx;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * g + r;
      DOT p0 = (DOT)ra[r], p1 = (DOT)ra[4 + r];
      half_swap(p0, p1);
      const DOT e0 = (DOT)E0[i], o0 = (DOT)O0[i], e1 = (DOT)E1[i], o1 = (DOT)O1[i];
      if ((i & 1) == 0) {
        xr0 = fma(p0, e0, xr0);
        xi0 = fma(p0, o0, xi0);
        xr1 = fma(p1, e1, xr1);
        xi1 = fma(p1, o1, xi1);
      } else {
        xr0 = fma(p0, o0, xr0);
        xi0 = fma(p0, e0, xi0);
        xr1 = fma(p1, o1, xr1);
        xi1 = fma(p1, e1, xi1);
      }
    }
    }
    // keep the 8-row groups in order: hoisting the recurrence ahead of the
    // folds would hold all 32 of the block's values
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One tile of the FP32-only path's shapelet pass: kTileRows rows x kShpChan
// channels starting at channel block cb.  Lane l of wave w owns row 64 w + l
// and runs both Hermite recurrences of its visibility in FP32.  The MFMA's N
// dimension is 32 visibilities: group 0 is the lower half-wave's, group 1 the
// upper's, and each operand value reaches the lane that supplies it through
// one half_swap per pair of values.  M is a 32-row block of the first axis, K
// runs over the second axis's orders (v_mfma_f32_32x32x2f32, K steps of 4
// orders inside the triangle) with even orders in one accumulator and odd
// orders in the other, folded into FP32 sums every 4 steps.
__device__ __forceinline__ void shp_tile_f32(const TileArgs &a, int rb, int cb, ShpSmem<kCmF32> &sm) {
  using REC = float;
  using DOT = float;
  constexpr int KB = kShpChan;
  const int k0 = cb * KB;
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t row = (int64_t)rb * kTileRows + tid;
  const bool valid = row < a.nrows;
  const int64_t rowc = valid ? row : a.nrows - 1;
  const int K = a.K;

  // sums start from what the point/Gaussian pass left (from zero without one)
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    double sr = 0, si = 0;
    if (valid && k0 + c < K && !a.fresh) {
      const int64_t idx = row * K + k0 + c;
      if (a.c64) {
        const float2 x = ((const float2 *)a.vis)[idx];
        sr = x.x;
        si = a.conj ? -x.y : x.y;
      } else {
        const double2 x = ((const double2 *)a.vis)[idx];
        sr = x.x;
        si = a.conj ? -x.y : x.y;
      }
    }
    sm.acc_re[c][tid] = sr;
    sm.acc_im[c][tid] = si;
  }

  const DOT sgn = a.subtract ? -1 : 1;
  const floatx16 zero16 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int j = 0; j < a.S; ++j) {
    const int N = a.t.nmax[j];
    const int q = N / 32;
    const int npairs = (q + 1) * (q + 2) / 2;
    __syncthreads();  // the previous shapelet's blocks are no longer read
    {
      const uint4 *src = (const uint4 *)(a.t.a32 + a.t.a32_off[j]);
      uint4 *dst = (uint4 *)&sm.A[0];
      for (int i = tid; i < npairs * kA32PerPair / 4; i += kTileRows) dst[i] = src[i];
    }
    const double *fr = a.d.sframe + 12 * j;
    const double u = a.uvw[3 * rowc], v = a.uvw[3 * rowc + 1], w = a.uvw[3 * rowc + 2];
    const double am = fma(fr[0], u, fma(fr[1], v, fr[2] * w));
    const double bm = fma(fr[3], u, fma(fr[4], v, fr[5] * w));
    const double t0 = fma(fr[6], u, fma(fr[7], v, fr[8] * w));
    __syncthreads();
    const int jg = a.P + a.G + j;
    for (int c = 0; c < KB; ++c) {
      if (k0 + c >= K) break;
      const double f = a.fk[k0 + c];
      const DOT S = (DOT)a.d.flux32[(int64_t)jg * a.Kpad + k0 + c];
      const REC xa = (REC)am * (REC)f;
      const REC xb = (REC)bm * (REC)f;
      // rescaled walks (psi_next): block or chunk k of 32 orders uses base
      // order 32 k + 16; carried values are rescaled when the base moves
      REC pb_m1 = 0, pb_n = shp_phi0<REC>(xb) * (REC)c_sc[0];
      // start values (u_{32 mb - 1}, u_{32 mb}) of the first axis's blocks,
      // filled in while chunk 0 walks every block
      REC sam[kMBMax], san[kMBMax];
      sam[0] = 0;
      san[0] = shp_phi0<REC>(xa) * (REC)c_sc[0];
#pragma unroll
      for (int k = 1; k < kMBMax; ++k) {
        sam[k] = 0;
        san[k] = 0;
      }
      DOT xr0 = 0, xi0 = 0, xr1 = 0, xi1 = 0;  // partial sums for groups 0 and 1
      int pbase = 0;
      for (int ch = 0; ch <= q; ++ch) {
        // second axis, this lane's visibility: orders 32 ch + t, in groups of
        // 8; groups past N (last chunk only) are zero
        float ob[32];
        {
          const int nb8 = min(4, (N - 32 * ch) / 8 + 1);
          REC prev = pb_m1, cur = pb_n;
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            if (g < nb8) {
#pragma unroll
              for (int t = 8 * g; t < 8 * g + 8; ++t) {
                ob[t] = (float)cur;
                const REC nx = psi_next<REC>(xb, cur, prev, (REC)c_half[32 * ch + t]);
                prev = cur;
                cur = nx;
              }
            } else {
#pragma unroll
              for (int t = 8 * g; t < 8 * g + 8; ++t) ob[t] = 0.f;
            }
          }
          // next chunk's base
          const REC rs = ch < 3 ? (REC)c_sc[ch + 1] : (REC)1;
          pb_m1 = prev * rs;
          pb_n = cur * rs;
        }
        // B operands of both groups (K = 2): lanes of half h supply orders
        // 4 s + 2 h + parity of K step s, stored at [2 s + parity]
        float bg0[16], bg1[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int lo = 4 * (t >> 1) + (t & 1);
          float p = ob[lo], qv = ob[lo + 2];
          half_swap(p, qv);
          bg0[t] = p;
          bg1[t] = qv;
        }
        const int nmb = q - ch + 1;
#pragma unroll
        for (int mb = 0; mb < kMBMax; ++mb) {
          if (mb >= nmb) break;
          const int p = pbase + mb;
          REC prev = sam[mb], cur = san[mb];
          // 8-row groups of this block that meet the triangle; all four while
          // chunk 0 walks towards a further block's start values
          const int ng = (ch == 0 && mb < q) ? 4 : min(4, (N - 32 * (ch + mb)) / 8 + 1);
          // K steps of this block inside the triangle: 32 (ch + mb) + 4 s <= N,
          // in two halves of 4 steps, each folded as soon as it is summed; the
          // second fold walks the rows again
          const int smax = min(8, (N - 32 * (ch + mb)) / 4 + 1);
          const float *Ap = &sm.A[p * kA32PerPair];
          const REC prev0 = prev, cur0 = cur;
          const int nh = smax > 4 ? 2 : 1;
#pragma nounroll
          for (int hf = 0; hf < nh; ++hf) {
            floatx16 E0 = zero16, O0 = zero16, E1 = zero16, O1 = zero16;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int st = 4 * hf + k;
              if (st < smax) {
                const float ae = Ap[st * 64 + lane], ao = Ap[(8 + st) * 64 + lane];
                const float b0e = hf ? bg0[8 + 2 * k] : bg0[2 * k], b0o = hf ? bg0[9 + 2 * k] : bg0[2 * k + 1];
                const float b1e = hf ? bg1[8 + 2 * k] : bg1[2 * k], b1o = hf ? bg1[9 + 2 * k] : bg1[2 * k + 1];
                E0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ae, b0e, E0, 0, 0, 0);
                O0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ao, b0o, O0, 0, 0, 0);
                E1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ae, b1e, E1, 0, 0, 0);
                O1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ao, b1o, O1, 0, 0, 0);
              }
            }
            prev = prev0;
            cur = cur0;
            shp_fold<REC, DOT>(xa, prev, cur, 32 * mb, ng, E0, O0, E1, O1, xr0, xi0, xr1, xi1);
          }
          if (mb + 1 < kMBMax && ch == 0 && mb < q) {
            sam[mb + 1] = prev * (REC)c_sc[mb + 1];
            san[mb + 1] = cur * (REC)c_sc[mb + 1];
          }
        }
        pbase += nmb;
      }
      // each group's two half-wave partial sums, brought to the owning lane
      half_swap(xr0, xr1);
      half_swap(xi0, xi1);
      const DOT xr = xr0 + xr1, xi = xi0 + xi1;
      float cs, sn;
      turns_sincos_f32((float)t0 * (float)f, cs, sn);
      const DOT tr = sgn * S * (xr * cs - xi * sn);
      const DOT ti = sgn * S * (xr * sn + xi * cs);
      sm.acc_re[c][tid] = (double)((DOT)sm.acc_re[c][tid] + tr);
      sm.acc_im[c][tid] = (double)((DOT)sm.acc_im[c][tid] + ti);
    }
  }
  if (!valid) return;
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    if (k0 + c >= K) break;
    const int64_t idx = row * K + k0 + c;
    const double re = sm.acc_re[c][tid], im = sm.acc_im[c][tid];
    if (a.c64)
      ((float2 *)a.vis)[idx] = make_float2((float)re, (float)(a.conj ? -im : im));
    else
      ((double2 *)a.vis)[idx] = make_double2(re, a.conj ? -im : im);
  }
}

// ---------------------------------------------------------------------------
// shapelet tile, BF16-split contraction (mixed path)
// ---------------------------------------------------------------------------

// The products of one MFMA group: even-n2 (E) and odd-n2 (O) accumulators of
// one 32 x 32 block, the two chains interleaved; smallest products first:
// (mid, mid), (lo, hi), (hi, lo), (mid, hi), (hi, mid), (hi, hi), or for the
// 2-way split (mid, hi), (hi, mid), (hi, hi).
template <int CM>
__device__ __forceinline__ void shp_group_mfma(const bf16x8 (&A)[3][2], const bf16x8 (&Bg)[3][2], floatx16 &E,
                                               floatx16 &O) {
  const floatx16 z = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (CM == kCmBf16x3) {
    E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[1][0], Bg[1][0], z, 0, 0, 0);
    O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[1][1], Bg[1][1], z, 0, 0, 0);
    E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[2][0], Bg[0][0], E, 0, 0, 0);
    O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[2][1], Bg[0][1], O, 0, 0, 0);
    E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][0], Bg[2][0], E, 0, 0, 0);
    O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][1], Bg[2][1], O, 0, 0, 0);
    E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[1][0], Bg[0][0], E, 0, 0, 0);
    O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[1][1], Bg[0][1], O, 0, 0, 0);
  } else {
    E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[1][0], Bg[0][0], z, 0, 0, 0);
    O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[1][1], Bg[0][1], z, 0, 0, 0);
  }
  E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][0], Bg[1][0], E, 0, 0, 0);
  O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][1], Bg[1][1], O, 0, 0, 0);
  E = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][0], Bg[0][0], E, 0, 0, 0);
  O = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[0][1], Bg[0][1], O, 0, 0, 0);
}

// One tile of the mixed path's shapelet pass: kTileRows rows x kShpChan
// channels starting at channel block cb.  Lane l of wave w owns row 64 w + l
// and runs both Hermite recurrences of its visibility in FP64 (rescaled,
// psi_next).  The MFMA's N dimension is 32 visibilities: group 0 is the lower
// half-wave's, group 1 the upper's.  M is a 32-row block of the first axis, K
// the second axis's orders, even orders in one accumulator (E) and odd orders
// in the other (O).
//   * Second axis, per chunk of 32 orders: each lane walks its own
//     visibility, splits every value into BF16 parts from its FP64 value
//     (the residual after the high part is formed in FP64, exactly, so the
//     parts carry ~27 bits instead of an FP32 rounding's 24; that rounding
//     measured as the largest single error term of the contraction), packs
//     them two per register and exchanges half of them with the other half
//     of the wave, one v_permlane32_swap per register.
//   * First axis, per block: both groups' MFMAs; then each accumulator
//     register of group 0 is exchanged with the same register of group 1, so
//     that every lane holds all 8 rows of each 8-row group for its own
//     visibility (accumulator register i then holds row 8 (i / 4) + i % 4 in
//     group 0's set and row 8 (i / 4) + 4 + i % 4 in group 1's); the lane
//     walks its own first-axis recurrence over the block and folds the rows
//     into FP64 sums.  No row value crosses lanes.
// The first axis is walked from order 0 in each chunk, carried from one
// block into the next (only a chunk's last block is partial).  Sums start
// from what the point/Gaussian pass left (from zero without one).
template <int CM>
__device__ __forceinline__ void shp_tile_bf(const TileArgs &a, int rb, int cb, ShpSmem<CM> &sm) {
  static_assert(CM == kCmBf16x3 || CM == kCmBf16x2, "BF16-split contraction modes only");
  constexpr int KB = kShpChan;
  constexpr int parts = CM == kCmBf16x3 ? 3 : 2;
  const int k0 = cb * KB;
  const int tid = threadIdx.x;
  const int64_t row = (int64_t)rb * kTileRows + tid;
  const bool valid = row < a.nrows;
  const int64_t rowc = valid ? row : a.nrows - 1;
  const int K = a.K;

#pragma unroll
  for (int c = 0; c < KB; ++c) {
    double sr = 0, si = 0;
    if (valid && k0 + c < K && !a.fresh) {
      const int64_t idx = row * K + k0 + c;
      if (a.c64) {
        const float2 x = ((const float2 *)a.vis)[idx];
        sr = x.x;
        si = a.conj ? -x.y : x.y;
      } else {
        const double2 x = ((const double2 *)a.vis)[idx];
        sr = x.x;
        si = a.conj ? -x.y : x.y;
      }
    }
    sm.acc_re[c][tid] = sr;
    sm.acc_im[c][tid] = si;
  }

  const double sgn = a.subtract ? -1 : 1;
  for (int j = 0; j < a.S; ++j) {
    const int N = a.t.nmax[j];
    const int q = N / 32;
    const int npairs = (q + 1) * (q + 2) / 2;
    __syncthreads();  // the previous shapelet's blocks are no longer read
    {
      const uint4 *src = (const uint4 *)(a.t.abf + a.t.abf_off[j]);
      uint4 *dst = &sm.A[0];
      for (int i = tid; i < parts * npairs * kAbfPerPair / 8; i += kTileRows) dst[i] = src[i];
    }
    const double *fr = a.d.sframe + 12 * j;
    const double u = a.uvw[3 * rowc], v = a.uvw[3 * rowc + 1], w = a.uvw[3 * rowc + 2];
    const double am = fma(fr[0], u, fma(fr[1], v, fr[2] * w));
    const double bm = fma(fr[3], u, fma(fr[4], v, fr[5] * w));
    const double t0 = fma(fr[6], u, fma(fr[7], v, fr[8] * w));
    __syncthreads();
    const int jg = a.P + a.G + j;
    const __bf16 *Ab = (const __bf16 *)&sm.A[0];
    const int part_stride = npairs * kAbfPerPair;
    for (int c = 0; c < KB; ++c) {
      if (k0 + c >= K) break;
      const double f = a.fk[k0 + c];
      const double S = a.d.flux64[(int64_t)jg * a.Kpad + k0 + c];
      const double xa = am * f, xb = bm * f;
      double pb_m1 = 0, pb_n = shp_phi0<double>(xb) * c_sc[0];
      const double ua0 = shp_phi0<double>(xa) * c_sc[0];
      double sr[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
      int pbase = 0;
      for (int ch = 0; ch <= q; ++ch) {
        const int nb8 = min(4, (N - 32 * ch) / 8 + 1);
        // second-axis operands of both groups: Bv[group][part][parity]
        bf16x8 Bv[2][3][2];
        {
          // pkb[part][parity][hc] element jj holds orders 16 hc + 4 jj +
          // parity (low half) and 16 hc + 4 jj + 2 + parity (high half)
          u32x4 pkb[3][2][2];
          double prev = pb_m1, cur = pb_n;
#pragma unroll
          for (int s4 = 0; s4 < 8; ++s4) {
            const int hc = s4 >> 2, jj = s4 & 3;
            if (s4 < 2 * nb8) {
              double v4[4];
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                v4[t] = cur;
                const double nx = psi_next<double>(xb, cur, prev, c_half[32 * ch + 4 * s4 + t]);
                prev = cur;
                cur = nx;
              }
#pragma unroll
              for (int par = 0; par < 2; ++par) {
                const double x0 = v4[par], x1 = v4[par + 2];
                const float2v xf = {(float)x0, (float)x1};
                const bf16x2v h = __builtin_convertvector(xf, bf16x2v);
                const float2v hf = __builtin_convertvector(h, float2v);
                const float2v rf = {(float)(x0 - (double)hf[0]), (float)(x1 - (double)hf[1])};
                const bf16x2v m = __builtin_convertvector(rf, bf16x2v);
                pkb[0][par][hc][jj] = __builtin_bit_cast(uint32_t, h);
                pkb[1][par][hc][jj] = __builtin_bit_cast(uint32_t, m);
                if (CM == kCmBf16x3) {
                  const bf16x2v l = __builtin_convertvector(rf - __builtin_convertvector(m, float2v), bf16x2v);
                  pkb[2][par][hc][jj] = __builtin_bit_cast(uint32_t, l);
                }
              }
            } else {
#pragma unroll
              for (int part = 0; part < 3; ++part)
#pragma unroll
                for (int par = 0; par < 2; ++par) pkb[part][par][hc][jj] = 0u;
            }
          }
          const double rs = ch < 3 ? c_sc[ch + 1] : 1.0;
          pb_m1 = prev * rs;
          pb_n = cur * rs;
          // group 0's operand: orders 0-15 of the lower half's visibility in
          // lanes 0-31, its orders 16-31 in lanes 32-63; group 1's likewise
          // for the upper half's visibility
#pragma unroll
          for (int part = 0; part < 3; ++part)
#pragma unroll
            for (int par = 0; par < 2; ++par) {
              u32x4 g0 = pkb[part][par][0], g1 = pkb[part][par][1];
              if (part < parts) {
#pragma unroll
                for (int jj = 0; jj < 4; ++jj)
                  if (jj < 2 * nb8) {  // else both registers are zero in every lane
                    uint32_t a0 = g0[jj], a1 = g1[jj];
                    half_swap(a0, a1);
                    g0[jj] = a0;
                    g1[jj] = a1;
                  }
              }
              Bv[0][part][par] = __builtin_bit_cast(bf16x8, g0);
              Bv[1][part][par] = __builtin_bit_cast(bf16x8, g1);
            }
        }
        const int nmb = q - ch + 1;
        double prev = 0, cur = ua0;
#pragma unroll
        for (int mb = 0; mb < kMBMax; ++mb) {
          if (mb >= nmb) break;
          if (mb > 0) {  // the next block's base order
            prev *= c_sc[mb];
            cur *= c_sc[mb];
          }
          const int p = pbase + mb;
          bf16x8 Av[3][2];  // [part][parity]
          {
            const int oe = p * kAbfPerPair + (tid & 63) * 8, oo = oe + 64 * 8;
#pragma unroll
            for (int part = 0; part < 3; ++part) {
              const int pp = part < parts ? part : parts - 1;
              Av[part][0] = *(const bf16x8 *)(Ab + pp * part_stride + oe);
              Av[part][1] = *(const bf16x8 *)(Ab + pp * part_stride + oo);
            }
          }
          floatx16 E0, O0, E1, O1;
          shp_group_mfma<CM>(Av, Bv[0], E0, O0);
          shp_group_mfma<CM>(Av, Bv[1], E1, O1);
          // 8-row groups of this block inside the triangle
          const int ng = min(4, (N - 32 * (ch + mb)) / 8 + 1);
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            if (g < ng) {
              double ra[8];
#pragma unroll
              for (int r = 0; r < 8; ++r) {
                ra[r] = cur;
                const double nx = psi_next<double>(xa, cur, prev, 0.5 * (32 * mb + 8 * g + r));
                prev = cur;
                cur = nx;
              }
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = 4 * g + r;
                float e0 = E0[i], e1 = E1[i], o0 = O0[i], o1 = O1[i];
                half_swap(e0, e1);
                half_swap(o0, o1);
                // rows 8 g + r (set 0) and 8 g + 4 + r (set 1), both of parity r % 2;
                // four independent FP64 sums per part (set x row parity)
                const int k = 2 * (r & 1);
                if ((r & 1) == 0) {
                  sr[k] = fma(ra[r], (double)e0, sr[k]);
                  si[k] = fma(ra[r], (double)o0, si[k]);
                  sr[k + 1] = fma(ra[4 + r], (double)e1, sr[k + 1]);
                  si[k + 1] = fma(ra[4 + r], (double)o1, si[k + 1]);
                } else {
                  sr[k] = fma(ra[r], (double)o0, sr[k]);
                  si[k] = fma(ra[r], (double)e0, si[k]);
                  sr[k + 1] = fma(ra[4 + r], (double)o1, sr[k + 1]);
                  si[k + 1] = fma(ra[4 + r], (double)e1, si[k + 1]);
                }
              }
            }
          }
        }
        pbase += nmb;
      }
      const double xr = (sr[0] + sr[1]) + (sr[2] + sr[3]), xi = (si[0] + si[1]) + (si[2] + si[3]);
      double cs, sn;
      turns_sincos_f64(t0 * f, cs, sn);
      sm.acc_re[c][tid] += sgn * S * (xr * cs - xi * sn);
      sm.acc_im[c][tid] += sgn * S * (xr * sn + xi * cs);
    }
  }
  if (!valid) return;
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    if (k0 + c >= K) break;
    const int64_t idx = row * K + k0 + c;
    const double re = sm.acc_re[c][tid], im = sm.acc_im[c][tid];
    if (a.c64)
      ((float2 *)a.vis)[idx] = make_float2((float)re, (float)(a.conj ? -im : im));
    else
      ((double2 *)a.vis)[idx] = make_double2(re, a.conj ? -im : im);
  }
}

template <int CM>
__global__ __launch_bounds__(kTileRows) __attribute__((amdgpu_waves_per_eu(2))) void k_shp_mfma(TileArgs a) {
  __shared__ ShpSmem<CM> sm;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if constexpr (CM == kCmF32)
    shp_tile_f32(a, tile % a.n_rb, tile / a.n_rb, sm);
  else
    shp_tile_bf<CM>(a, tile % a.n_rb, tile / a.n_rb, sm);
}

// ---------------------------------------------------------------------------
// shapelet kernel, FP64 path (vector ALU)
// ---------------------------------------------------------------------------

// One thread per row of the tile, for the tile's kShpChan channels.  The
// second axis is taken in chunks of orders whose Hermite values sit in
// registers; per chunk the matching columns of the signed coefficient matrix
// are staged in LDS and each row n1 of them is dotted with those values while
// the first axis's recurrence advances with n1.  The recurrence path takes
// the four channels together (16-order chunks), the lookup-table variant one
// channel at a time (32-order chunks).
// Lookup-table variant of the basis (the paper's simulator interpolates a
// 1-D table of the basis, Sec. 3.2): phi_n at x_i = i dx, 0 <= i <= kLutSamples,
// dx = kLutXMax / kLutSamples, FP32, rows of kLutStride orders; phi_n(-x) =
// (-1)^n phi_n(x) covers x < 0 and the table reads zero beyond kLutXMax
// (phi_96(32) ~ 1e-78).  Built once per context from the FP64 recurrence.
__global__ __launch_bounds__(256) void k_lut_build(float *T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kLutSamples + 1) return;
  const double x = i * (kLutXMax / kLutSamples);
  const double sx = 1.41421356237309504880 * x;
  double p = kPiM14 * exp(-0.5 * x * x), pm1 = 0.0;
  float *row = T + (int64_t)i * kLutStride;
  for (int n = 0; n < kLutStride; ++n) {
    row[n] = n <= kNmaxLimit ? (float)p : 0.0f;
    if (n < kNmaxLimit) {
      const double nx = herm_step<double>(sx, p, pm1, n);
      pm1 = p;
      p = nx;
    }
  }
}

// Interpolation position in the table: row pointer, fraction and the sign
// of odd orders.
struct LutPos {
  const float *r0;
  float fr, odd;
  bool in;
};

__device__ __forceinline__ LutPos lut_pos(const float *T, double x) {
  LutPos q;
  const double t = fabs(x) * (kLutSamples / kLutXMax);
  q.in = t < (double)kLutSamples;
  const int i = q.in ? (int)t : 0;
  q.fr = q.in ? (float)(t - i) : 0.0f;
  q.r0 = T + (int64_t)i * kLutStride;
  q.odd = x < 0.0 ? -1.0f : 1.0f;
  return q;
}

// Orders n0 .. n0 + 31 of the basis at q: linear interpolation between the
// two bracketing rows, the sign (-1)^n for x < 0, zero past kNmaxLimit and
// beyond the table.  The rows are read with 16-byte loads: a lane's orders
// are contiguous in its rows, and one 4-byte load per order made every load
// instruction touch a cache line per lane.  n0 is a multiple of 32 and rows
// are 16-byte aligned (kLutStride x 4 B); orders past kLutStride read the
// following row (inside the table, which has a spare row) before they are
// masked.
__device__ __forceinline__ void lut_chunk(const LutPos &q, int n0, float (&v)[32]) {
  const float4 *p0 = (const float4 *)(q.r0 + n0), *p1 = (const float4 *)(q.r0 + kLutStride + n0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 a = p0[k], b = p1[k];
    v[4 * k] = fmaf(q.fr, b.x - a.x, a.x);
    v[4 * k + 1] = fmaf(q.fr, b.y - a.y, a.y);
    v[4 * k + 2] = fmaf(q.fr, b.z - a.z, a.z);
    v[4 * k + 3] = fmaf(q.fr, b.w - a.w, a.w);
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const int n = n0 + i;
    const float x = (n & 1) ? q.odd * v[i] : v[i];
    v[i] = q.in && n <= kNmaxLimit ? x : 0.0f;
  }
}

// Second-axis orders per chunk of the FP64 recurrence path: the values of a
// chunk for the tile's four channels (4 x 16 FP64) stay in registers.
constexpr int kF64Chunk = 16;

template <bool LUT>
__global__ __launch_bounds__(kTileRows) __attribute__((amdgpu_waves_per_eu(2))) void k_shp_fp64(TileArgs a) {
  constexpr int KB = kShpChan;
  // one 32-column chunk of the signed coefficient matrix (rows 0 .. N - m0),
  // staged in LDS for the whole workgroup and read as broadcasts: from
  // global memory every row dot waited on its wave-uniform loads
  __shared__ double sC[(kNmaxLimit + 1) * 32];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int cb = tile / a.n_rb, rb = tile % a.n_rb;
  const int k0 = cb * KB;
  const int nc = min(KB, a.K - k0);  // channels of this tile
  const int tid = threadIdx.x;
  const int64_t row = (int64_t)rb * kTileRows + tid;
  const bool valid = row < a.nrows;
  const int64_t rowc = valid ? row : a.nrows - 1;
  const double u = a.uvw[3 * rowc], v = a.uvw[3 * rowc + 1], w = a.uvw[3 * rowc + 2];

  double acc_re[KB], acc_im[KB];
#pragma unroll
  for (int c = 0; c < KB; ++c) acc_re[c] = acc_im[c] = 0.0;
  for (int j = 0; j < a.S; ++j) {
    const int N = a.t.nmax[j];
    const double *fr = a.d.sframe + 12 * j;
    const double am = fma(fr[0], u, fma(fr[1], v, fr[2] * w));
    const double bm = fma(fr[3], u, fma(fr[4], v, fr[5] * w));
    const double t0 = fma(fr[6], u, fma(fr[7], v, fr[8] * w));
    if constexpr (!LUT) {
      // The second axis in chunks of kF64Chunk orders (its recurrence carried
      // across chunks, per channel); per chunk the first axis is walked from
      // order 0 for all of the tile's channels at once, and each row n1 is
      // dotted with the chunk's part of row n1 of the signed coefficient
      // matrix.  Every coefficient read from LDS (a broadcast to all lanes)
      // feeds the tile's four channels: with one channel per read the LDS
      // return path, not the FP64 units, set the pace.  Channels past the
      // last (a ragged tile) are computed on the padded frequency table and
      // not written.
      const double *C = a.t.c64 + a.t.c64_off[j];
      const int ld = a.t.c64_ld[j];
      double bn[KB], bm1[KB], xr[KB], xi[KB], pa0[KB];  // per channel
#pragma unroll
      for (int c = 0; c < KB; ++c) {
        const double f = a.fk[k0 + c];
        const double xb = f * bm, xa = f * am;
        bn[c] = kPiM14 * exp(-0.5 * xb * xb);
        pa0[c] = kPiM14 * exp(-0.5 * xa * xa);
        bm1[c] = xr[c] = xi[c] = 0.0;
      }
      for (int ch = 0; kF64Chunk * ch <= N; ++ch) {
        const int m0 = kF64Chunk * ch;
        __syncthreads();  // the previous chunk is no longer read
        for (int i = tid; i < (N - m0 + 1) * kF64Chunk; i += kTileRows) {
          const int col = m0 + (i % kF64Chunk);
          sC[i] = col < ld ? C[(int64_t)(i / kF64Chunk) * ld + col] : 0.0;
        }
        __syncthreads();
        double pb[KB][kF64Chunk];
#pragma unroll
        for (int c = 0; c < KB; ++c) {
          const double sxb = 1.41421356237309504880 * (a.fk[k0 + c] * bm);
#pragma unroll
          for (int i = 0; i < kF64Chunk; ++i) {
            pb[c][i] = bn[c];
            const double nx = herm_step<double>(sxb, bn[c], bm1[c], m0 + i);  // orders <= 127: table size
            bm1[c] = bn[c];
            bn[c] = nx;
          }
        }
        double pa[KB], pam1[KB], sxa[KB];
#pragma unroll
        for (int c = 0; c < KB; ++c) {
          pa[c] = pa0[c];
          pam1[c] = 0.0;
          sxa[c] = 1.41421356237309504880 * (a.fk[k0 + c] * am);
        }
        // one row n1: its dots with the chunk's second-axis values, folded
        // with the first axis into the real or imaginary sums by the parity
        // of n1 (rows are taken in pairs, so the parity is a constant)
        auto row = [&](int n1, auto ODD) {
          const double *Cr = sC + n1 * kF64Chunk;
          double te[KB], to[KB];
#pragma unroll
          for (int b8 = 0; b8 < kF64Chunk / 8; ++b8) {
            if (b8 == 0 || 8 * b8 <= N - m0 - n1) {
#pragma unroll
              for (int e = 0; e < 8; e += 2) {
                const double ce = Cr[8 * b8 + e], co = Cr[8 * b8 + e + 1];
#pragma unroll
                for (int c = 0; c < KB; ++c) {
                  if (b8 == 0 && e == 0) {
                    te[c] = ce * pb[c][0];
                    to[c] = co * pb[c][1];
                  } else {
                    te[c] = fma(ce, pb[c][8 * b8 + e], te[c]);
                    to[c] = fma(co, pb[c][8 * b8 + e + 1], to[c]);
                  }
                }
              }
            }
          }
#pragma unroll
          for (int c = 0; c < KB; ++c) {
            if constexpr (decltype(ODD)::value) {
              xr[c] = fma(pa[c], to[c], xr[c]);
              xi[c] = fma(pa[c], te[c], xi[c]);
            } else {
              xr[c] = fma(pa[c], te[c], xr[c]);
              xi[c] = fma(pa[c], to[c], xi[c]);
            }
            const double nx = herm_step<double>(sxa[c], pa[c], pam1[c], n1);
            pam1[c] = pa[c];
            pa[c] = nx;
          }
        };
        for (int n1 = 0; n1 <= N - m0; n1 += 2) {
          row(n1, std::integral_constant<bool, false>());
          if (n1 + 1 <= N - m0) row(n1 + 1, std::integral_constant<bool, true>());
        }
      }
#pragma unroll
      for (int c = 0; c < KB; ++c) {
        if (c >= nc) break;
        const double f = a.fk[k0 + c];
        double cs, sn;
        turns_sincos_f64(t0 * f, cs, sn);
        const double S = a.d.flux64[(int64_t)(a.P + a.G + j) * a.Kpad + k0 + c];
        acc_re[c] += S * (xr[c] * cs - xi[c] * sn);
        acc_im[c] += S * (xr[c] * sn + xi[c] * cs);
      }
    } else {
      // Lookup-table basis: the second axis in chunks of 32 orders, one
      // channel at a time; per chunk and channel each row n1 is dotted with
      // the chunk's part of row n1 of the signed coefficient matrix (staged in
      // LDS), and the first axis's table values are read 32 rows at a time,
      // all in flight before the rows that use them: a table read per row,
      // waited on by that row, left the kernel waiting on memory.
      const double *C = a.t.c64 + a.t.c64_off[j];
      const int ld = a.t.c64_ld[j];
      double xr[KB], xi[KB];
#pragma unroll
      for (int c = 0; c < KB; ++c) xr[c] = xi[c] = 0.0;
      for (int ch = 0; 32 * ch <= N; ++ch) {
        const int m0 = 32 * ch;
        __syncthreads();  // the previous chunk is no longer read
        for (int i = tid; i < (N - m0 + 1) * 32; i += kTileRows) {
          const int col = m0 + (i & 31);
          sC[i] = col < ld ? C[(int64_t)(i >> 5) * ld + col] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < KB; ++c) {
          if (c >= nc) break;
          const double f = a.fk[k0 + c];
          const LutPos qa = lut_pos(a.lut, f * am), qb = lut_pos(a.lut, f * bm);
          double pb[32];
          {
            float pbf[32];
            lut_chunk(qb, m0, pbf);
#pragma unroll
            for (int i = 0; i < 32; ++i) pb[i] = (double)pbf[i];
          }
          for (int r0 = 0; r0 <= N - m0; r0 += 32) {
            float pa[32];  // rows past N - m0 are read but not used
            lut_chunk(qa, r0, pa);
#pragma unroll
            for (int r = 0; r < 32; ++r) {
              const int n1 = r0 + r;  // r0 is a multiple of 32: n1 has the parity of r
              if (n1 > N - m0) break;
              const double *Cr = sC + n1 * 32;
              double te = 0.0, to = 0.0;
#pragma unroll
              for (int b8 = 0; b8 < 4; ++b8) {
                if (8 * b8 <= N - m0 - n1) {
#pragma unroll
                  for (int e = 0; e < 8; e += 2) {
                    te = fma(Cr[8 * b8 + e], pb[8 * b8 + e], te);
                    to = fma(Cr[8 * b8 + e + 1], pb[8 * b8 + e + 1], to);
                  }
                }
              }
              const double pv = (double)pa[r];
              if (r & 1) {
                xr[c] = fma(pv, to, xr[c]);
                xi[c] = fma(pv, te, xi[c]);
              } else {
                xr[c] = fma(pv, te, xr[c]);
                xi[c] = fma(pv, to, xi[c]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < KB; ++c) {
        if (c >= nc) break;
        const double f = a.fk[k0 + c];
        double cs, sn;
        turns_sincos_f64(t0 * f, cs, sn);
        const double S = a.d.flux64[(int64_t)(a.P + a.G + j) * a.Kpad + k0 + c];
        acc_re[c] += S * (xr[c] * cs - xi[c] * sn);
        acc_im[c] += S * (xr[c] * sn + xi[c] * cs);
      }
    }
  }
  if (!valid) return;
#pragma unroll
  for (int c = 0; c < KB; ++c) {
    if (c >= nc) break;
    const int64_t idx = row * a.K + k0 + c;
    double2 *o = (double2 *)a.vis;
    float2 *o32 = (float2 *)a.vis;
    double xr = 0.0, xi = 0.0;
    if (a.fresh) {
      // no point/Gaussian pass wrote this visibility
    } else if (a.c64) {
      const float2 x = o32[idx];
      xr = x.x;
      xi = a.conj ? -x.y : x.y;
    } else {
      const double2 x = o[idx];
      xr = x.x;
      xi = a.conj ? -x.y : x.y;
    }
    if (a.subtract) {
      xr -= acc_re[c];
      xi -= acc_im[c];
    } else {
      xr += acc_re[c];
      xi += acc_im[c];
    }
    if (a.conj) xi = -xi;
    if (a.c64)
      o32[idx] = make_float2((float)xr, (float)xi);
    else
      o[idx] = make_double2(xr, xi);
  }
}

// ---------------------------------------------------------------------------
// serving: persistent kernels (continuous batching, mixed path)
// ---------------------------------------------------------------------------
// One kernel per ring.  Every workgroup loops: claim the next published entry
// of its ring (compare-and-swap on a device counter), copy that job's
// arguments from host-mapped memory into LDS, and run the entry's work with
// the same device functions as the standalone kernels, so that a job's result
// is the same alone and in a mix.  An entry stands for a run of consecutive
// units of one job (the host sizes runs so that a job still spreads over every
// workgroup): on ring 0, slices of the job's per-(sky, observation) tables or
// point/Gaussian tiles; on ring 1, the shapelet pass of tiles (each tile's two
// kShpChan-wide halves), which reads what the point/Gaussian tiles wrote.
// Runs keep the claims (one device-wide atomic and two host-memory reads
// each) far below the rate at which small tiles complete.  The passes live in separate kernels
// because each runs at the occupancy of its own register budget (the
// shapelet contraction needs twice the point/Gaussian pass's registers).
// Entries are counted done per job slot; the last one of a phase publishes
// the phase's sequence number to the host, which then publishes the next
// phase.
// A workgroup exits when any workgroup of the launch has found nothing to
// claim for idle_ticks (all exit together, after their current item), or when
// the host sets stop; no workgroup ever waits on another, and neither kernel
// waits on the other.

// Kept out of line so that its FP64 library calls do not add to the register
// allocation of the tile path that shares the kernel.
__device__ __noinline__ void serve_table_item(const ServeJobDesc &job, int64_t item, int tid) {
  const int J = job.da.P + job.da.G + job.da.S;
  const int64_t nder = (J + kTileRows - 1) / kTileRows;
  if (item < nder) {
    const int64_t j = item * kTileRows + tid;
    if (j < J) derive_ool(job.da, (int)j);
  } else {
    const int64_t idx = (item - nder) * kTileRows + tid;
    if (idx < (int64_t)J * job.fa.Kpad) flux_ool(job.fa, idx);
  }
}

template <int RING>
struct ServeSmem;
template <>
struct ServeSmem<0> {
  PgSmem<float> pg;
};
template <>
struct ServeSmem<1> {
  ShpSmem<kCmBf16x3> shp;
};

// A copy of a structure that every lane of the wave holds alike, read from
// lane 0 word by word: the compiler then keeps it in scalar registers (a
// structure loaded from LDS would otherwise occupy vector registers).
template <typename T>
__device__ __forceinline__ T wave_uniform(const T &x) {
  static_assert(sizeof(T) % 4 == 0, "word-sized structure");
  T r;
  const uint32_t *src = (const uint32_t *)&x;
  uint32_t *dst = (uint32_t *)&r;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return r;
}

template <int RING>
__device__ __forceinline__ void serve_kernel(ServeHost *H, ServeDev *D, uint64_t idle_ticks, uint64_t epoch) {
  __shared__ ServeSmem<RING> sm;
  __shared__ ServeJobDesc job;
  __shared__ uint64_t s_claim, s_entry, s_seen, s_cached_seq;
  __shared__ int s_cached_slot, s_cached_table, s_reload;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_seen = 0;
    s_cached_slot = -1;
  }
  for (;;) {
    if (tid == 0) {
      uint64_t claimed = kNoClaim;
      const uint64_t t_idle = wall_clock64();
      unsigned backoff = 1;
      for (;;) {
        if (__hip_atomic_load(&D->quit_epoch[RING], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) break;
        // Relaxed, system-scope accesses: host-mapped memory is read uncached,
        // and the ring entry and job arguments are read through addresses that
        // depend on the claimed index, which orders them after the tail.  An
        // acquire here would invalidate the XCD's L2 on every claim and throw
        // away the component tables the other workgroups are streaming.
        // The host's tail is read over PCIe only when the device-side copy says
        // the ring is empty; claims themselves touch device memory only.
        uint64_t h = __hip_atomic_load(&D->head[RING], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t t = __hip_atomic_load(&D->tail_cache[RING], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h >= t) {
          t = __hip_atomic_load(&H->tail[RING], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          if (t > h) __hip_atomic_fetch_max(&D->tail_cache[RING], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (h < t) {
          // a failed compare-and-swap returns the current head: try the next
          // entry at once while entries remain
          bool ok;
          do {
            ok = __hip_atomic_compare_exchange_strong(&D->head[RING], &h, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
          } while (!ok && h < t);
          if (ok) {
            claimed = h;
            break;
          }
          continue;
        }
        if (__hip_atomic_load(&H->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
        if (__hip_atomic_load(&D->quit_epoch[RING], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) break;
        if (wall_clock64() - t_idle > idle_ticks) {
          // the ring has been empty for idle_ticks: the whole launch exits
          // (workers finish their current item first) so that the other
          // ring's kernel, queued behind this one, can run
          __hip_atomic_store(&D->quit_epoch[RING], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        for (unsigned i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(8);
        backoff = backoff < 64 ? 2 * backoff : 64;
      }
      s_claim = claimed;
      if (claimed != kNoClaim) {
        const uint64_t e = __hip_atomic_load(&H->ring[RING][claimed & (kRingSize - 1)], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_SYSTEM);
        s_entry = e;
        // The job arguments in LDS are reused when the entry belongs to the
        // same slot and phase and the slot still carries the same sequence
        // number (the host rewrites a slot only between jobs or phases,
        // changing it).  On ring 0, the first entry of a phase newer than any
        // this workgroup has run drops cached lines that may predate its
        // inputs: the tables its tiles read are built by table entries of this
        // same launch, and buffers can be reallocated and rewritten while the
        // kernel runs.  A phase's inputs are complete before it is published
        // and sequence numbers grow with publication, so one invalidation per
        // newer sequence number suffices.  Ring 1 needs none: a shapelet phase
        // is published once its point/Gaussian tiles are done, which happens
        // in a launch of ring 0's kernel that ended before this launch began
        // (the two run one after the other on one stream), and the kernel
        // boundary makes their writes and tables visible; its arguments are
        // read from host memory, uncached.  Invalidating here would throw away
        // the coefficient tiles that every workgroup of the XCD streams.
        const int slot = (int)(e >> 48), table = (int)((e >> 47) & 1);
        const uint64_t *seqp =
            table ? &H->jobs[slot].seq_table : (RING == 0 ? &H->jobs[slot].seq : &H->jobs[slot].seq_shp);
        const uint64_t seq = __hip_atomic_load(seqp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        s_reload = !(slot == s_cached_slot && table == s_cached_table && seq == s_cached_seq);
        s_cached_slot = slot;
        s_cached_table = table;
        s_cached_seq = seq;
        if (RING == 0 && seq > s_seen) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          s_seen = seq;
        }
      }
    }
    __syncthreads();
    if (s_claim == kNoClaim) return;
    const int slot = (int)(s_entry >> 48);
    const bool table_item = RING == 0 && ((s_entry >> 47) & 1);
    const int64_t entry = (int64_t)(s_entry & ((1ull << 47) - 1));
    const uint64_t item_seq = s_cached_seq;
    if (s_reload) {
      const uint64_t *src = (const uint64_t *)&H->jobs[slot];
      uint64_t *dst = (uint64_t *)&job;
      constexpr int words = (int)(sizeof(ServeJobDesc) / sizeof(uint64_t));
      for (int i = tid; i < words; i += kTileRows)
        dst[i] = __hip_atomic_load(&src[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();  // the copy is spread over the waves: complete before any field is read
    if (table_item) {
      // per-(sky, observation) tables: units [0, nder) derive kTileRows
      // components each, the rest compute kTileRows flux-table entries each
      const int64_t u1 = min(job.ntable, (entry + 1) * job.per_table);
      for (int64_t u = entry * job.per_table; u < u1; ++u) serve_table_item(job, u, tid);
      __syncthreads();
      if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        const uint64_t old = __hip_atomic_fetch_add(&D->tdone[slot], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == job.table_target)
          __hip_atomic_store(&H->tabled[slot], job.seq_table, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      __syncthreads();
      continue;
    }
    const TileArgs a = wave_uniform(job.a);
    const int64_t per = RING == 0 ? job.per_pg : job.per_shp;
    const int64_t t1 = min(job.ntiles, (entry + 1) * per);
    if (RING == 0 && tid == 0 && entry == 0) {
      // the job's first entry (entries are claimed in order): its start time, then the flag
      __hip_atomic_store(&H->started_clk[slot], wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&H->started[slot], job.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // tile t covers row block t mod n_rb and channel block t / n_rb; the
    // run's blocks are stepped, not divided out per tile
    const int64_t t0 = entry * per;
    int rb = (int)(t0 % a.n_rb), cb = (int)(t0 / a.n_rb);
    for (int64_t tile = t0; tile < t1; ++tile) {
      if constexpr (RING == 0) {
        if (a.uniform)
          pg_tile<kMixed, true>(a, rb, cb, sm.pg);
        else
          pg_tile<kMixed>(a, rb, cb, sm.pg);
      } else {
#pragma unroll 1
        for (int h = 0; h < 2; ++h) shp_tile_bf<kCmBf16x3>(a, rb, 2 * cb + h, sm.shp);
      }
      __syncthreads();  // the tile's LDS is reused by the next one
      if (++rb == a.n_rb) {
        rb = 0;
        ++cb;
      }
    }
    if (tid == 0) {
      // the entry's visibilities are written back to memory before the entry
      // is counted; the phase's last count therefore follows every tile's
      // data, and the host flag follows the last count
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // system-scope release: write back, no invalidate
      const uint64_t target = RING == 0 ? job.done_target : job.shp_target;
      const uint64_t old = __hip_atomic_fetch_add(&D->done[slot], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (old + 1 == target) {
        __hip_atomic_store(&H->finished_clk[slot], wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&H->finished[slot], item_seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
    __syncthreads();  // LDS (job, tiles) is reused by the next claim
  }
}

__global__ __launch_bounds__(kTileRows) void k_serve_pg(
    ServeHost *H, ServeDev *D, uint64_t idle_ticks, uint64_t epoch) {
  serve_kernel<0>(H, D, idle_ticks, epoch);
}

__global__ __launch_bounds__(kTileRows) __attribute__((amdgpu_waves_per_eu(2))) void k_serve_shp(
    ServeHost *H, ServeDev *D, uint64_t idle_ticks, uint64_t epoch) {
  serve_kernel<1>(H, D, idle_ticks, epoch);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// Per-device set-up, once per device and process: the recurrence constants
// into __constant__ memory.
static std::once_flag g_init_once[kMaxDevices];
static hipError_t g_init_err[kMaxDevices];

static hipError_t init_constants() {
  double sq[128], isq[128], half[128], sc[4];
  for (int n = 0; n < 128; ++n) {
    sq[n] = sqrt((double)n);
    isq[n] = 1.0 / sqrt((double)n + 1.0);
    half[n] = 0.5 * n;
  }
  sc[0] = herm_scale(0, 16);
  for (int k = 1; k < 4; ++k) sc[k] = herm_scale(32 * k - 16, 32 * k + 16);
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_sqn), sq, sizeof(sq));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_isqn1), isq, sizeof(isq));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_half), half, sizeof(half));
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_sc), sc, sizeof(sc));
  return e;
}

// Scratch of vp_predict_noalloc (the per-(sky, observation) tables of one
// call), one array per device for the life of the process.  In host code the
// name is only a stand-in: its device address, which differs per device, is
// looked up once per device below and used everywhere instead.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static void *g_scratch[kMaxDevices];

hipError_t device_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::call_once(g_init_once[dev], [dev]() {
    // the caller has made `dev` current
    hipError_t e = init_constants();
    if (e == hipSuccess) {
      void *p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e == hipSuccess) g_scratch[dev] = p;
    }
    g_init_err[dev] = e;
  });
  return g_init_err[dev];
}

void *noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices || device_init(dev) != hipSuccess) return nullptr;
  return g_scratch[dev];
}

static hipError_t upload_tables() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  return device_init(dev);
}

hipError_t launch_derive(const DeriveArgs &a, hipStream_t s) {
  const int J = a.P + a.G + a.S;
  if (J == 0) return hipSuccess;
  hipLaunchKernelGGL(k_derive, dim3((J + 127) / 128), dim3(128), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_flux(const FluxArgs &a, hipStream_t s) {
  const int64_t n = (int64_t)a.J * a.Kpad;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_flux, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tiles_build(const TileBuildArgs &a, int max_nmax, hipStream_t s) {
  (void)max_nmax;
  if (a.S == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tiles, dim3(16, a.S), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pg(const TileArgs &a, int prec, hipStream_t s) {
  hipError_t e = upload_tables();
  if (e != hipSuccess) return e;
  const int64_t nt = (int64_t)a.n_rb * a.n_cb;
  if (nt <= 0) return hipSuccess;
  if (nt > 0x7fffffff) return hipErrorInvalidValue;
  switch (prec) {
    case kFP64:
    case kLut:  // the lookup-table variant differs from the FP64 path in the shapelet basis only
      if (a.uniform)
        hipLaunchKernelGGL((k_pg_tile<kFP64, true>), dim3((unsigned)nt), dim3(kTileRows), 0, s, a);
      else
        hipLaunchKernelGGL((k_pg_tile<kFP64, false>), dim3((unsigned)nt), dim3(kTileRows), 0, s, a);
      break;
    case kFP32:
      hipLaunchKernelGGL(k_pg_tile<kFP32>, dim3((unsigned)nt), dim3(kTileRows), 0, s, a);
      break;
    default:
      if (a.uniform)
        hipLaunchKernelGGL((k_pg_tile<kMixed, true>), dim3((unsigned)nt), dim3(kTileRows), 0, s, a);
      else
        hipLaunchKernelGGL((k_pg_tile<kMixed, false>), dim3((unsigned)nt), dim3(kTileRows), 0, s, a);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_shp(const TileArgs &a, int prec, int max_nmax, hipStream_t s) {
  hipError_t e = upload_tables();
  if (e != hipSuccess) return e;
  const int64_t nt = (int64_t)a.n_rb * a.n_cb;
  if (nt <= 0 || a.S == 0) return hipSuccess;
  if (nt > 0x7fffffff) return hipErrorInvalidValue;
  if (max_nmax < 0 || max_nmax > kNmaxLimit) return hipErrorInvalidValue;
  const dim3 g((unsigned)nt), b(kTileRows);
  switch (prec) {
    case kFP64:
      hipLaunchKernelGGL(k_shp_fp64<false>, g, b, 0, s, a);
      break;
    case kLut:
      if (!a.lut) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_shp_fp64<true>, g, b, 0, s, a);
      break;
    case kFP32:
      hipLaunchKernelGGL(k_shp_mfma<kCmF32>, g, b, 0, s, a);
      break;
    case kMixed:
    case kMixedBf16:
      hipLaunchKernelGGL(k_shp_mfma<kCmBf16x3>, g, b, 0, s, a);
      break;
    case kMixedBf16x2:
      hipLaunchKernelGGL(k_shp_mfma<kCmBf16x2>, g, b, 0, s, a);
      break;
    default:
      return hipErrorNotSupported;
  }
  return hipGetLastError();
}

hipError_t launch_lut_build(float *T, hipStream_t s) {
  hipError_t e = upload_tables();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lut_build, dim3((kLutSamples + 2 + 255) / 256), dim3(256), 0, s, T);
  return hipGetLastError();
}

hipError_t serve_grid(int ring, int *grid) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = ring == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_serve_pg, kTileRows, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_serve_shp, kTileRows, 0);
  if (e != hipSuccess) return e;
  *grid = cus * (per > 0 ? per : 1);
  return hipSuccess;
}

hipError_t launch_serve(int ring, ServeHost *host_dev, ServeDev *dev, uint64_t idle_ticks, uint64_t epoch, int grid,
                        hipStream_t s) {
  hipError_t e = upload_tables();
  if (e != hipSuccess) return e;
  if (ring == 0)
    hipLaunchKernelGGL(k_serve_pg, dim3(grid), dim3(kTileRows), 0, s, host_dev, dev, idle_ticks, epoch);
  else
    hipLaunchKernelGGL(k_serve_shp, dim3(grid), dim3(kTileRows), 0, s, host_dev, dev, idle_ticks, epoch);
  return hipGetLastError();
}

}  // namespace vp
