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
constexpr int kFlushMixed = 16; // mixed path: components per FP64 add (two kFlush partials, summed in FP32)
constexpr int kNmaxLimit = 96; // largest n1 + n2
constexpr int kMBMax = 4;      // 32-row blocks of the n1 axis: ceil(97 / 32)

// The MFMA shapelet kernels keep only the 32 x 32 blocks of the signed
// coefficient matrix (32 rows of n1 by 32 orders of n2) that meet the
// triangle n1 + n2 <= N: block (chunk ch, row block mb) with
// 32 (ch + mb) <= N, chunk-major.  With q = N / 32 there are
// (q + 1)(q + 2) / 2 of them.
__host__ __device__ inline int shp_pairs(int nmax) {
  const int q = nmax / 32;
  return (q + 1) * (q + 2) / 2;
}
constexpr int kPairsMax = (kNmaxLimit / 32 + 1) * (kNmaxLimit / 32 + 2) / 2;
constexpr int kA32PerPair = 2 * 8 * 64;  // floats: [parity][K step of 2 orders][lane]
constexpr int kAbfPerPair = 2 * 64 * 8;  // BF16 values of one split part: [parity][lane][8]

// Precision paths, numbered as VP_PREC_*; 5 (the FP32-MFMA contraction of the
// mixed path) is retired and refused at the boundary.
enum Prec : int { kFP64 = 0, kMixed = 1, kMixedBf16 = 2, kFP32 = 3, kMixedBf16x2 = 4, kLut = 6 };

// Lookup table of the basis (the lookup-table variant): kLutSamples + 2 rows
// of kLutStride FP32 values.
constexpr int kLutSamples = 8192;
constexpr double kLutXMax = 32.0;
constexpr int kLutStride = 100;
constexpr size_t kLutBytes = (size_t)(kLutSamples + 2) * kLutStride * sizeof(float);

// Per-(sky, observation) tables, built on the device.  Plain aggregates (no
// member initialisers) so that they can live in LDS inside the serving kernel.
struct Derived {
  double4 *pos;   // [J] (l, m, n-1, 0), components in order points, Gaussians, shapelets
  double4 *gq;    // [G] quadratic form of the Gaussian envelope exponent (base 2), metres^2
  double *sframe; // [S][12] a-vector(3), b-vector(3), (l, m, n-1)(3), pad(3)
  float *flux32;  // [J][Kpad]
  double *flux64; // [J][Kpad]
};

// Shapelet coefficient tiles (depend on the sky only).
struct ShpTiles {
  const float *a32;        // MFMA A-operand tiles, FP32
  const int64_t *a32_off;  // [S]
  const double *c64;       // dense signed coefficients [n1][ld], FP64
  const int64_t *c64_off;  // [S]
  const int32_t *c64_ld;   // [S] leading dimension (multiple of 8)
  const uint16_t *abf;     // BF16 split A tiles: [part][pair][parity][64][8]
  const int64_t *abf_off;  // [S]
  const int32_t *nmax;     // [S]
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
  const double *ra, *dec;      // [J], for the beam
  const double *freq;          // [K]
  double nu_ref;
  double ra0, dec0;
  double beam_fwhm, beam_nu_ref;
  int j0;                      // first shapelet component
  const int32_t *lpow;         // [J - j0] power q of ln(nu / nu_ref) multiplying a shapelet's flux, or null
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
  const float *lut;    // basis table of the lookup-table variant, or null
  double dfk;          // (nu_{k+1} - nu_k) / c when the channels are uniformly spaced
  int uniform;         // 1: channels uniformly spaced (the mixed path rotates phasors by dfk)
  int fresh;           // 1: the shapelet pass starts from zero instead of reading vis (a
                       //    predict with no point/Gaussian pass before it)
};

// ---------------------------------------------------------------------------
// serving: persistent kernels pull (job slot, tile) items from rings that the
// host publishes in host-mapped memory.  Ring 0 holds table items and the
// point/Gaussian pass's tiles; ring 1 the shapelet pass's tiles, published
// once the job's point/Gaussian tiles are done.  One kernel per ring, each at
// the occupancy of its own pass.
// ---------------------------------------------------------------------------
constexpr int kServeSlots = 1024;
constexpr uint64_t kRingSize = 1ull << 20;
constexpr uint64_t kNoClaim = ~0ull;
constexpr int kServeRings = 2;

struct ServeJobDesc {
  TileArgs a;            // tiling of the point/Gaussian pass (kPgChan-wide blocks)
  DeriveArgs da;         // table items (when the job builds its tables)
  FluxArgs fa;
  int64_t ntiles;        // a.n_rb * a.n_cb (tiles of each pass)
  int64_t ntable;        // table work units (kTileRows components or flux entries each)
  int64_t per_pg, per_shp, per_table;  // consecutive tiles / table units behind one ring entry
  uint64_t seq;          // sequence number of the point/Gaussian phase (> 0, grows with publication)
  uint64_t seq_shp;      // sequence number of the shapelet phase
  uint64_t seq_table;    // sequence number of the table phase
  uint64_t done_target;  // slot's entry counter value once the point/Gaussian phase is done
  uint64_t shp_target;   // slot's entry counter value once the shapelet phase is done
  uint64_t table_target; // slot's table counter value once the last table entry is done
};

struct ServeHost {       // host-mapped, coherent
  uint64_t tail[kServeRings];  // items published per ring (written by the host with release order)
  uint64_t stop;         // non-zero: workers exit once idle
  uint64_t started[kServeSlots];   // seq of the job whose first tile has started
  uint64_t finished[kServeSlots];  // seq (or seq_shp) of the job phase whose last tile has finished
  uint64_t started_clk[kServeSlots];   // device wall clock when that first tile started
  uint64_t finished_clk[kServeSlots];  // device wall clock when that last tile finished
  uint64_t tabled[kServeSlots];    // seq_table of the job whose tables are built
  uint64_t ring[kServeRings][kRingSize];  // (slot << 48) | (table entry << 47) | entry index
  ServeJobDesc jobs[kServeSlots];
};

struct ServeDev {        // device memory
  uint64_t head[kServeRings];        // items claimed per ring
  uint64_t tail_cache[kServeRings];  // largest published-item count any worker has read from the host
  uint64_t quit_epoch[kServeRings];  // launch epoch whose workers are to exit
  uint64_t done[kServeSlots];
  uint64_t tdone[kServeSlots];
};

// Kernel classes timed by vp_profile: tables, point/Gaussian, shapelet, calibration.
constexpr int kProfClasses = 4;

// Peel calibration (vp_calib.hip).
constexpr int kPeelMaxAnt = 256;          // tiles per observation (one thread each)
constexpr size_t kPeelSmemMax = 163840;  // LDS per workgroup on gfx950
constexpr size_t kPeelWsMax = size_t(1) << 30;  // per-cell tables of one launch, bytes (at least one cell)

struct GainArgs {
  int T, B, K;            // cells are (time, channel); B baselines per time step
  int n_ant, n_iter, max_cg;
  double cg_tol2;         // squared relative residual that ends a CG solve
  const void *model;      // [T][B][K] complex ideal model I (same type as data)
  void *data;             // [T][B][K] complex data V; the residual on return when subtract
  int c64;                // 1: complex64, 0: complex128
  const int32_t *ant1, *ant2;  // [B] tiles of each baseline
  const int32_t *pair_bl;      // [n_ant (n_ant - 1) / 2] baseline of tile pair (i < j), -1 if none
  const int32_t *comp;         // [n_ant] connected component of each tile in the baseline graph, -1 if idle
  double2 *gains;         // [T][K][n_ant] output, or null
  double2 *gw;            // [T][n_ant][K] gains of every cell (workspace, read by the subtract pass)
  int cell0, ncell;       // the launch covers cells cell0 .. cell0 + ncell - 1 (cell = t K + k)
  void *xt;               // workspace [ncell][n_ant][n_ant] complex X (float2 when w32, else double2)
  void *wf;               // workspace [ncell][n_ant][n_ant] |I|^2 (float when w32, else double)
  int w32;                // 1 (mixed path): FP32 tables and FP32 W in the step's operator, FP64 sums
  int single_comp;        // 1: every tile with a baseline is in one connected component
};

// Device set-up (vp_kernels.hip): the recurrence constants, once per device
// and process (the device must be current).
constexpr int kMaxDevices = 64;
hipError_t device_init(int dev);
// Device address of this device's no-allocation scratch array (valid after
// device_init(dev) succeeded), or null.
void *noalloc_scratch(int dev);
// Size of that array: per-(sky, observation) tables of vp_predict_noalloc.
constexpr uint64_t kNoAllocScratchBytes = 64ull << 20;

// Host-side launchers (vp_kernels.hip).
hipError_t launch_derive(const DeriveArgs &a, hipStream_t s);
hipError_t launch_flux(const FluxArgs &a, hipStream_t s);
hipError_t launch_tiles_build(const TileBuildArgs &a, int max_nmax, hipStream_t s);
hipError_t launch_pg(const TileArgs &a, int prec, hipStream_t s);
hipError_t launch_shp(const TileArgs &a, int prec, int max_nmax, hipStream_t s);
hipError_t launch_lut_build(float *T, hipStream_t s);
hipError_t launch_serve(int ring, ServeHost *host_dev, ServeDev *dev, uint64_t idle_ticks, uint64_t epoch, int grid,
                        hipStream_t s);
hipError_t serve_grid(int ring, int *grid);
hipError_t launch_gain(const GainArgs &a, hipStream_t s);
hipError_t launch_gain_subtract(const GainArgs &a, hipStream_t s);
bool gain_supported(int n_ant);
size_t gain_smem_bytes(int n_ant, bool w64, int threads);
size_t gain_cell_bytes(int n_ant, bool w32);  // workspace bytes per cell

// sizes of per-shapelet tile storage
inline int64_t a32_floats(int nmax) { return (int64_t)shp_pairs(nmax) * kA32PerPair; }
inline int c64_ld(int nmax) { return ((nmax + 1) + 7) / 8 * 8; }
inline int64_t c64_doubles(int nmax) { return (int64_t)(nmax + 1) * c64_ld(nmax); }
inline int64_t abf_elems(int nmax) { return (int64_t)3 * shp_pairs(nmax) * kAbfPerPair; }

}  // namespace vp
