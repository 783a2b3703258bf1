/*
 * vp.h -- C ABI of libvp, direct-Fourier visibility prediction on AMD
 * Instinct MI355X (gfx950).
 *
 * What is computed (Line et al., "Modelling and peeling extended sources with
 * shapelets: a Fornax A case study"):
 *
 *   V(t,b,k) = sum_j S_j(nu_k) xi_j(u,v) exp(sign 2 pi i (u l_j + v m_j + w (n_j - 1)))
 *
 * with (u,v,w) the baseline of (time t, baseline b) in wavelengths at channel
 * k -- uvw are given once per time step in metres and scaled by nu_k / c
 * (Sec. 3.2, last paragraph) -- and
 *   - points:     xi = 1                              (Sec. 3.1, Eq. measure_eq_discrete)
 *   - Gaussians:  xi = exp(-pi^2/(4 ln2) (kx^2 maj^2 + ky^2 min^2)),
 *                 kx = cos(pa) v + sin(pa) u, ky = -sin(pa) v + cos(pa) u
 *                                                     (Sec. 3.2, Eqs. gauss-env, scale-gauss-x/y)
 *   - shapelets:  xi = sum_{n1+n2<=N} C_{n1,n2} (sign i)^(n1+n2) phi_n1(a) phi_n2(b),
 *                 a = kappa beta1 (cos(pa) v' + sin(pa) u'),
 *                 b = kappa beta2 (-sin(pa) v' + cos(pa) u'), kappa = pi / sqrt(2 ln 2),
 *                 (u',v') the baseline re-phased to the shapelet's own centre,
 *                 phi_n the orthonormal Hermite functions
 *                                                     (Sec. 2 Eqs. basis_1D, basis_2D, basis_FT;
 *                                                      Sec. 3.2 Eqs. shape-env, scale-shape-x/y)
 *   - flux:       S_j(nu) = S_ref (nu / nu_ref)^alpha * B_j(nu), one spectral
 *                 index per component (Sec. 4.1); B_j is 1 (flat beam, Sec. 3.1)
 *                 or an optional Gaussian power pattern about the phase centre,
 *                 exp(-4 ln2 rho_j^2 / Theta(nu)^2), Theta(nu) = Theta_ref nu_ref_beam / nu.
 *   - peel:       R = D - V, the residual of Sec. 5.1 with unit gains
 *                 (vp_subtract), or R = D - g_ant1 g_ant2^* V with per-tile gains
 *                 fitted per (time, channel) as in Sec. 5.1 (vp_peel).
 *
 * Conventions: angles in radians, FWHMs and beta as FWHM in radians, PA east of
 * north, fluxes in Jy, frequencies in Hz.  n - 1 is formed as
 * -(l^2 + m^2) / (1 + n).  The exponent sign is -1 in the paper; +1 yields the
 * exact complex conjugate.  Coefficients are used as given (the paper's
 * C <- C / I convention, Sec. 3.2): no extra prefactor is applied.
 *
 * Visibility layout: row-major [n_time][n_bl][n_chan] of interleaved complex
 * numbers, complex128 (VP_C128: double re, double im) or complex64 (VP_C64).
 *
 * Threading: every call is thread-safe; predict/subtract calls that share a
 * stream are ordered by that stream.  Errors: every call returns a VP_* code;
 * vp_last_error() returns a thread-local message for the calling thread's
 * last failure.  Out-parameters are written only on success.
 */
#ifndef VP_H
#define VP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define VP_OK 0
#define VP_EINVAL (-1)     /* invalid argument (NULL, size <= 0, non-finite, out of range) */
#define VP_ENOMEM (-2)     /* device or host allocation failed */
#define VP_EDEVICE (-3)    /* HIP runtime error (including faults of earlier async work) */
#define VP_EAGAIN (-4)     /* job still pending (vp_poll) */
#define VP_ECAPACITY (-5)  /* job footprint exceeds the context's HBM budget: never admissible */
#define VP_ENOTFOUND (-6)  /* unknown ticket */
#define VP_EBUSY (-7)      /* object still in use by pending jobs */

/* precision paths */
#define VP_PREC_FP64 0        /* FP64 everywhere (phase, sincos, envelopes, recurrence, contraction, sums) */
#define VP_PREC_MIXED 1       /* FP64 phase + range reduction; FP32 sincos/envelopes, FP32 partial
                                 sums of 8 terms added into FP64;
                                 FP64 Hermite recurrence; shapelet contraction on MFMA with the
                                 coefficients and Hermite values split into 3 BF16 parts from their
                                 FP64 values (6 products, FP32 accumulation, folded into FP64 per
                                 32 orders) */
#define VP_PREC_MIXED_BF16 2  /* the same path as VP_PREC_MIXED (explicit name of its contraction) */
#define VP_PREC_FP32 3        /* FP32 everywhere, phase included (reported, not accurate) */
#define VP_PREC_MIXED_BF16X2 4 /* as MIXED, contraction as 2-way BF16 split (3 products; reported) */
#define VP_PREC_MIXED_F32MMA 5 /* retired (refused with VP_EINVAL): a contraction on FP32 MFMA was
                                  both slower than the 3-way BF16 split and, at ~1e-6 of the total
                                  flux on heavily cancelling coefficients, not inside the mixed
                                  path's bar; the value stays reserved */
#define VP_PREC_LUT 6         /* as FP64, but the shapelet basis read from a 1-D FP32 table of the
                                 Hermite functions (8192 samples over 0 <= x < 32, linear
                                 interpolation), as the paper's simulator does (Sec. 3.2);
                                 for comparison (reported, not accurate); built per context at
                                 first use (400 x 8194 floats) */

/* output element types */
#define VP_C128 0
#define VP_C64 1

/* serving job kinds */
#define VP_JOB_PREDICT 0
#define VP_JOB_SUBTRACT 1

/* maximum shapelet order n1 + n2 */
#define VP_NMAX_LIMIT 96
#define VP_NTERM_LIMIT 8      /* spectral terms per shapelet */
#define VP_PEEL_MAX_ANT 256   /* tiles a peel can calibrate (one thread per tile) */
#define VP_PEEL_MAX_ITER 1000 /* Gauss-Newton iterations accepted by vp_peel */
#define VP_PEEL_MAX_CG 200    /* conjugate-gradient steps per Gauss-Newton step (bound) */

typedef struct vp_ctx vp_ctx;
typedef struct vp_obs vp_obs;
typedef struct vp_sky vp_sky;

/* Observation (Sec. 3.2: uvw once per time step; channels scale it by nu/c). */
typedef struct {
  int32_t n_time, n_bl, n_chan;
  const double *uvw_m;   /* host, [n_time][n_bl][3] baseline (u,v,w) in metres */
  const double *freq_hz; /* host, [n_chan] channel frequencies */
  double ra0, dec0;      /* phase centre, rad */
  int32_t sign;          /* exponent sign: -1 (paper) or +1 */
  double beam_fwhm_rad;  /* Gaussian power-beam FWHM at beam_nu_ref_hz; 0 => flat beam */
  double beam_nu_ref_hz;
} vp_obs_desc;

/* Sky model (Sec. 3.1 points; Sec. 3.2 Gaussians and shapelets; Sec. 4.1 spectra).
 * Shapelet coefficients are packed per shapelet, n1-major: n1 = 0..N, then
 * n2 = 0..N-n1, (N+1)(N+2)/2 values starting at coeffs[s_coeff_off[s]].
 * Frequency-dependent coefficients (the fit of the coefficients as a function
 * of frequency that Sec. 7 proposes, letting the spectral index vary across a
 * source): with s_nterm non-NULL, shapelet s has Q = s_nterm[s] blocks
 * C_0 .. C_{Q-1} of (N+1)(N+2)/2 values one after another from
 * coeffs[s_coeff_off[s]], and its coefficients at frequency nu are
 * C(nu) = sum_q C_q ln(nu / nu_ref_hz)^q (still multiplied by the power-law
 * flux).  Each term costs one shapelet's work. */
typedef struct {
  double nu_ref_hz; /* reference frequency of S_ref */
  int32_t n_point;
  const double *p_ra, *p_dec, *p_sref, *p_alpha;
  int32_t n_gauss;
  const double *g_ra, *g_dec, *g_sref, *g_alpha;
  const double *g_maj, *g_min, *g_pa; /* FWHM major/minor (rad), PA (rad) */
  int32_t n_shp;
  const double *s_ra, *s_dec, *s_sref, *s_alpha;
  const double *s_beta1, *s_beta2, *s_pa; /* beta as FWHM of the (0,0) basis (rad), PA (rad) */
  const int32_t *s_nmax;                  /* N = max(n1 + n2) per shapelet, 0..VP_NMAX_LIMIT */
  const int64_t *s_coeff_off;             /* offset of each shapelet's coefficients */
  const double *coeffs;
  const int32_t *s_nterm;                 /* NULL (one term each) or [n_shp] 1..VP_NTERM_LIMIT */
} vp_sky_desc;

/* Create a context on HIP device `hip_device`.  hbm_budget_bytes bounds the
 * device memory that admitted serving jobs may hold at once (library tables
 * plus each job's visibility buffer); 0 selects 90% of the device's free
 * memory.  Errors: VP_EINVAL (bad device / NULL out), VP_EDEVICE. */
int vp_create_ctx(int hip_device, uint64_t hbm_budget_bytes, vp_ctx **out);

/* Destroy a context.  Fails with VP_EBUSY while serving jobs are pending;
 * observations and skies still alive are destroyed with it. */
int vp_destroy_ctx(vp_ctx *ctx);

/* Copy an observation to the device.  Host arrays are read during the call
 * and may be freed on return.  Errors: VP_EINVAL for n <= 0, NULL arrays,
 * non-finite uvw/frequencies, frequencies <= 0, |sign| != 1, beam FWHM < 0 or
 * a positive FWHM with beam_nu_ref_hz <= 0; VP_ENOMEM; VP_EDEVICE. */
int vp_create_obs(vp_ctx *ctx, const vp_obs_desc *desc, vp_obs **out);
int vp_destroy_obs(vp_obs *obs); /* VP_EBUSY while a pending job uses it */

/* Copy a sky model to the device.  Host arrays are read during the call and
 * may be freed on return.  Per-(sky, observation) tables (direction cosines,
 * frames, flux per channel, coefficient tiles) are built on the device by the
 * first predict/subtract that pairs them, and cached.  A shapelet is kept to
 * its effective order, the highest n1 + n2 with a non-zero coefficient
 * (zero coefficients above it contribute nothing; the shapelet kernels' work
 * follows the order, so truncating high orders saves time while truncating
 * scattered coefficients does not).  Errors: VP_EINVAL for
 * negative counts, NULL arrays with a positive count, non-finite values,
 * nu_ref <= 0, Gaussian FWHM < 0, beta <= 0, nmax outside 0..VP_NMAX_LIMIT,
 * coefficient offsets < 0, spectral terms outside 1..VP_NTERM_LIMIT; VP_ENOMEM;
 * VP_EDEVICE. */
int vp_create_sky(vp_ctx *ctx, const vp_sky_desc *desc, vp_sky **out);
int vp_destroy_sky(vp_sky *sky); /* VP_EBUSY while a pending job uses it */

/* Predict: write V[n_time][n_bl][n_chan] (interleaved complex, `dtype`) into
 * caller-owned device memory `vis_dev`, asynchronously on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  `precision` is a VP_PREC_* path.
 * Returns once the work is enqueued; faults of the asynchronous work surface
 * as VP_EDEVICE from a later call.  Errors: VP_EINVAL, VP_EDEVICE, VP_ENOMEM. */
int vp_predict(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, int precision, int dtype,
               void *vis_dev, void *hip_stream);

/* vp_predict without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same operation, arguments and results as vp_predict (bitwise
 * the same output), but the per-(sky, observation) tables (direction
 * cosines, Gaussian quadratic forms, shapelet frames, flux per component and
 * channel) are rebuilt on every call into a fixed scratch array of
 * 64 MiB that the library holds on each device until the process ends,
 * instead of being allocated and cached.  Limit: 32 B per component, 32 B
 * per Gaussian, 96 B per shapelet and 12 B per (component, channel padded to
 * a multiple of 8), each part rounded up to 256 B, at most 64 MiB in all
 * (e.g. 20,000 components x 32 channels fit; 5,000 components x 1,024
 * channels fit; 100,000 components x 384 channels do not); a larger pair is
 * refused with VP_EINVAL.  VP_PREC_LUT is refused (its table is per context).
 * No hipMalloc, hipFree, event or other allocating call is made.  Every call
 * on one device uses that device's single array, which keeps the last call's
 * tables: calls that overlap on one device (on different streams, or from
 * different threads without ordering) race and give wrong results; calls
 * ordered on one stream do not.  The sky, observation and context must have
 * been created beforehand (those calls allocate).  Errors as vp_predict. */
int vp_predict_noalloc(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, int precision, int dtype,
                       void *vis_dev, void *hip_stream);

/* Subtract (peel with unit gains): data <- data - V, in place on caller-owned
 * device memory laid out as for vp_predict.  Same errors. */
int vp_subtract(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, int precision, int dtype,
                void *data_dev, void *hip_stream);

/* Serving (continuous batching). */
typedef struct {
  int32_t kind; /* VP_JOB_PREDICT or VP_JOB_SUBTRACT */
  const vp_sky *sky;
  const vp_obs *obs;
  int32_t precision, dtype;
  void *vis_dev;          /* caller-owned device buffer, alive until the job is done */
  uint64_t t_arrival_ns;  /* caller's arrival timestamp (CLOCK_MONOTONIC ns); 0 => now */
} vp_job;

typedef struct {
  int32_t status;   /* VP_OK or the job's error code */
  uint64_t t_submit, t_admit, t_start, t_done; /* CLOCK_MONOTONIC ns, as the scheduler thread saw them */
  /* device wall clock (ticks of hipDeviceAttributeWallClockRate, one clock per
   * device) when the job's first tile started and when its last tile ended;
   * comparable between jobs of one context; 0 for a job that ran no tile */
  uint64_t dev_first_tile, dev_last_tile;
} vp_job_result;

/* Enqueue a job; returns a ticket.  The caller's writes to job->vis_dev (the
 * data of a subtract job) must be complete, i.e. the writing stream
 * synchronised, before the call.  Only VP_PREC_MIXED is served: the
 * persistent kernels that run every admitted job's tiles are compiled
 * instances of the mixed path, and their register use sets the occupancy
 * that all jobs share (FP64 instances beside them would run at lower
 * occupancy and serialise against them); FP64 work goes through vp_predict /
 * vp_subtract on a caller stream, which may run beside serving.  The job is
 * admitted when its HBM footprint fits the budget minus what admitted jobs
 * hold, in FIFO order, and a job slot and ring space are free; an admitted
 * job's tiles (its tables first, when its sky and observation have none yet)
 * are run by two persistent device kernels, one for the point/Gaussian pass
 * and one for the shapelet pass, together with the tiles of other admitted
 * jobs.  A failure of the job's own admission (e.g. its table allocation)
 * ends that job alone; a device failure ends every running job.  Errors:
 * VP_EINVAL, VP_ECAPACITY if the footprint exceeds the whole budget or the job
 * has more tiles than a serving ring holds.  Thread-safe. */
int vp_submit(vp_ctx *ctx, const vp_job *job, uint64_t *ticket);

/* Non-blocking: VP_OK with *res filled when the job is done (res->status holds
 * the job's own result), VP_EAGAIN while pending, VP_ENOTFOUND for an unknown
 * or already-collected ticket.  A completed ticket is released by the VP_OK
 * poll.  Thread-safe. */
int vp_poll(vp_ctx *ctx, uint64_t ticket, vp_job_result *res);

/* Serving measurement: the number of completed launches of the persistent
 * serving kernels since the context's first vp_submit and the total duration
 * in ms of their launch groups (HIP events around each group on the kernels'
 * stream; a group still running is not counted).  Zeros before the first
 * vp_submit.  Errors: VP_EINVAL. */
int vp_serve_stats(vp_ctx *ctx, uint64_t *launches, double *resident_ms);

/* HBM footprint (bytes) that admission charges for `job`.  Errors: VP_EINVAL. */
int vp_job_footprint(vp_ctx *ctx, const vp_job *job, uint64_t *bytes);

/* Peel with calibration (Sec. 5.1): predict the model I of `sky` (the source
 * to peel) on `obs` into a library workspace, fit per-tile complex gains g
 * for every (time, channel) cell so that g_ant1 g_ant2^* I matches the data
 * -- n_iter Gauss-Newton iterations of the linearised least-squares problem
 * of Sec. 5.1, starting from unit gains, each step the minimum-norm
 * least-squares solution (the data leave one global phase free per
 * connected group of tiles; a step stops early once the right-hand side is
 * at FP64 rounding level, and a cell whose step is then zero has converged
 * and takes no further iterations) -- and subtract: data <- data - g_ant1
 * g_ant2^* I.
 * ant1, ant2: host arrays [n_bl] (n_bl of obs), the tiles (0..n_ant-1,
 * distinct, each pair at most once) of each baseline, the same for every
 * time step; read during the call only.
 * precision selects the path of the model prediction and of the solve.
 * VP_PREC_FP64: the per-cell tables (X = I^* V seen from each tile, and
 * |I|^2) in FP64, the step's normal-equation weights |I|^2 in FP64 while
 * they fit in LDS (up to 183 tiles) and FP32 beyond; the right-hand side,
 * and so the solution the iterations converge to, is FP64.  Any other
 * precision: the tables and the weights in FP32, sums and steps in FP64;
 * the solution moves by the tables' FP32 rounding (about 1e-7 relative).
 * gains_dev: caller-owned device memory [n_time][n_chan][n_ant] complex128
 * receiving the gains, or NULL.  data_dev as for vp_subtract.  Asynchronous
 * on hip_stream; calls on one context share a workspace (n_time x n_bl x
 * n_chan complex values, n_time x n_ant x n_chan complex128 gains and up to
 * 1 GiB of per-cell tables) and wait for the previous call to finish with it.
 * Errors: VP_EINVAL (tiles out of range or repeated pairs, n_ant outside
 * 2..VP_PEEL_MAX_ANT, n_iter outside 0..VP_PEEL_MAX_ITER, as vp_subtract),
 * VP_ENOMEM, VP_EDEVICE. */
int vp_peel(vp_ctx *ctx, const vp_sky *sky, const vp_obs *obs, const int32_t *ant1, const int32_t *ant2,
            int32_t n_ant, int32_t n_iter, int precision, int dtype, void *data_dev, void *gains_dev,
            void *hip_stream);

/* Per-kernel timing, for measurement.  When enabled, the library records HIP
 * events around each kernel it launches for vp_predict/vp_subtract on the
 * caller's stream and accumulates their durations by kernel class:
 * 0 = per-(sky,obs) table build, 1 = point/Gaussian tile kernel,
 * 2 = shapelet tile kernel, 3 = peel calibration.  vp_profile_read
 * synchronises the recorded events, fills counts[4] and total_ms[4], and
 * resets the accumulators. */
int vp_profile(vp_ctx *ctx, int enable);
int vp_profile_read(vp_ctx *ctx, int64_t *counts, double *total_ms);

/* Thread-local message describing the calling thread's last error ("" if none). */
const char *vp_last_error(void);

/* Library version string. */
const char *vp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VP_H */
