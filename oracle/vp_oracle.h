/*
 * vp_oracle.h -- declarations of the FP64 CPU oracle (test infrastructure).
 * Not part of the GPU library and not shared with it.
 */
#ifndef VP_ORACLE_H
#define VP_ORACLE_H
#include <stdint.h>

#define ORACLE_NMAX_CAP 255
#define ORACLE_NTERM_CAP 16

typedef struct {
  int32_t n_time, n_bl, n_chan;
  const double *uvw_m;   /* [n_time][n_bl][3], metres */
  const double *freq_hz; /* [n_chan] */
  double ra0, dec0;      /* phase centre, rad */
  int32_t sign;          /* exponent sign, -1 (paper) or +1 */
  double beam_fwhm_rad, beam_nu_ref_hz; /* 0 => flat beam */
} oracle_obs;

typedef struct {
  double nu_ref_hz;
  int32_t n_point;
  const double *p_ra, *p_dec, *p_sref, *p_alpha;
  int32_t n_gauss;
  const double *g_ra, *g_dec, *g_sref, *g_alpha, *g_maj, *g_min, *g_pa;
  int32_t n_shp;
  const double *s_ra, *s_dec, *s_sref, *s_alpha, *s_beta1, *s_beta2, *s_pa;
  const int32_t *s_nmax;
  const int64_t *s_coeff_off;
  const double *coeffs;
  /* NULL, or [n_shp] numbers of spectral terms: shapelet s's coefficients at
   * frequency nu are C(nu) = sum_{q < s_nterm[s]} C_q ln(nu / nu_ref)^q, the
   * blocks C_q of (N+1)(N+2)/2 values following each other from
   * coeffs[s_coeff_off[s]] */
  const int32_t *s_nterm;
} oracle_sky;

void oracle_hermite(int32_t nmax, double x, double *phi);
void oracle_lmn(double ra0, double dec0, double ra, double dec, double *lmn);
void oracle_rotation(double ra0, double dec0, double ra, double dec, double *R);
double oracle_gauss_envelope(double u, double v, double maj, double min, double pa);
int oracle_shapelet_envelope_ab(int32_t nmax, const double *coeffs, double a, double b,
                                int32_t sign, double *out_re, double *out_im);
void oracle_shapelet_args(double up, double vp, double beta1, double beta2, double pa,
                          double *a, double *b);
double oracle_flux(const oracle_obs *obs, double nu_ref, double sref, double alpha,
                   double ra, double dec, double nu);
int oracle_predict(const oracle_obs *obs, const oracle_sky *sky, const int64_t *rows,
                   int64_t nrows, double *out, int32_t nthreads);
int oracle_flux_table(const oracle_obs *obs, const oracle_sky *sky, double *out);
int32_t oracle_max_threads(void);

#endif
