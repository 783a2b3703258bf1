// vp_internal.h -- structures shared between the libvp host code and its
// gfx950 kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vp {

constexpr double kLightSpeed = 299792458.0;  // m/s

// Tile geometry.  A tile is kTileRows consecutive (time, baseline) rows times
// a block of channels; one workgroup of kTileRows threads processes a tile.
constexpr int kTileRows = 256;
constexpr int kPgChan = 8;     // channels per point/Gaussian tile (per thread)
constexpr int kShpChan = 4;    // channels per shapelet tile
constexpr int kChunk = 64;     // components staged in LDS at a time
constexpr int kFlush = 8;      // components summed plainly before a Kahan step
constexpr int kNmaxLimit = 96; // largest n1 + n2
constexpr int kMBMax = 4;      // 32-row M blocks of the n1 axis: ceil(97 / 32)
constexpr int kS4Max = 25;     // K steps of 4 orders: ceil(97 / 4)
constexpr int kA32PerShp = kMBMax * 2 * kS4Max * 64;  // floats, upper bound
constexpr int kBf16Chunks = 4;  // 16-wide K steps of one parity: ceil(49 / 16)

enum Prec : int { kFP64 = 0, kMixed = 1, kMixedBf16 = 2, kFP32 = 3, kMixedBf16x2 = 4 };

// Per-(sky, observation) tables, built on the device.
struct Derived {
  double4 *pos = nullptr;   // [J] (l, m, n-1, 0), components in order points, Gaussians, shapelets
  double4 *gq = nullptr;    // [G] quadratic form of the Gaussian envelope exponent (base 2), metres^2
  double *sframe = nullptr; // [S][12] a-vector(3), b-vector(3), (l, m, n-1)(3), pad(3)
  float *flux32 = nullptr;  // [J][Kpad]
  double *flux64 = nullptr; // [J][Kpad]
};

// Shapelet coefficient tiles (depend on the sky only).
struct ShpTiles {
  const float *a32 = nullptr;        // MFMA A-operand tiles, FP32
  const int64_t *a32_off = nullptr;  // [S]
  const double *c64 = nullptr;       // dense signed coefficients [n1][ld], FP64
  const int64_t *c64_off = nullptr;  // [S]
  const int32_t *c64_ld = nullptr;   // [S] leading dimension (multiple of 8)
  const uint16_t *abf = nullptr;     // BF16 split A tiles: [part][mb][par][chunk][64][8]
  const int64_t *abf_off = nullptr;  // [S]
  const int32_t *nmax = nullptr;     // [S]
};

struct DeriveArgs {
  int P, G, S;
  const double *ra, *dec;          // [J]
  const double *g_maj, *g_min, *g_pa;  // [G]
  const double *s_beta1, *s_beta2, *s_pa;  // [S]
  double ra0, dec0;
  Derived d;
};

struct FluxArgs {
  int J, K, Kpad;
  const double *sref, *alpha;  // [J]
  const double *freq;          // [K]
  double nu_ref;
  double beam_fwhm, beam_nu_ref;
  Derived d;
};

struct TileBuildArgs {
  int S;
  const int32_t *nmax;
  const int64_t *coeff_off;
  const double *coeffs;
  float *a32;
  const int64_t *a32_off;
  double *c64;
  const int64_t *c64_off;
  const int32_t *c64_ld;
  uint16_t *abf;
  const int64_t *abf_off;
};

// Arguments common to the visibility tile kernels.
struct TileArgs {
  int64_t nrows;       // n_time * n_bl
  int K, Kpad;         // channels, padded to a multiple of kPgChan
  int n_rb, n_cb;      // row blocks, channel blocks (of the kernel's own channel width)
  const double *uvw;   // [nrows][3] metres
  const double *fk;    // [Kpad] nu_k / c (padded with the last channel)
  int P, G, S;
  Derived d;
  ShpTiles t;
  void *vis;           // output (predict) or data (subtract), [nrows][K] complex
  int subtract;        // 0: vis = V; 1: vis = vis - V
  int c64;             // 1: complex64, 0: complex128
  int conj;            // 1 when the exponent sign is -1
  int nb;              // FP64 shapelet kernel: order bucket
};

// Host-side launchers (vp_kernels.hip).
hipError_t launch_derive(const DeriveArgs &a, hipStream_t s);
hipError_t launch_flux(const FluxArgs &a, hipStream_t s);
hipError_t launch_tiles_build(const TileBuildArgs &a, int max_nmax, hipStream_t s);
hipError_t launch_pg(const TileArgs &a, int prec, hipStream_t s);
hipError_t launch_shp(const TileArgs &a, int prec, int max_nmax, hipStream_t s);

// sizes of per-shapelet tile storage
inline int64_t a32_floats(int nmax) {
  int mb = (nmax + 32) / 32, s4 = (nmax + 4) / 4;
  return (int64_t)mb * 2 * s4 * 64;
}
inline int c64_ld(int nmax) { return ((nmax + 1) + 7) / 8 * 8; }
inline int64_t c64_doubles(int nmax) { return (int64_t)(nmax + 1) * c64_ld(nmax); }
inline int bf16_chunks(int nmax) {
  // even orders 0, 2, ... <= nmax: nmax/2 + 1 values; 16 per K step
  return (nmax / 2 + 1 + 15) / 16;
}
inline int64_t abf_elems(int nmax) {
  int mb = (nmax + 32) / 32;
  return (int64_t)3 * mb * 2 * bf16_chunks(nmax) * 64 * 8;
}

}  // namespace vp
