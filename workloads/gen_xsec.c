/*
 * gen_xsec.c — seeded synthetic inputs: line-list cross-section tables.
 *
 * Input generation only.  It stands in for the tabulated molecular
 * cross-sections the paper computes from ExoMol/HITEMP line lists with
 * Voigt profiles (Sect. 2.3); nothing of the forward model's arithmetic
 * lives here.  The line parameters (positions, strengths, lower-state
 * energies, broadening coefficients) are drawn in Python from a seeded
 * generator and passed in, so this file only evaluates
 *
 *   sigma(nu; T, p) = floor + sum_k S_k(T) * V(nu - nu_k; aD_k(T), gL_k(p, T))
 *
 * with S(T) = S_296 (296/T)^1.5 exp(-c2 E (1/T - 1/296)), Doppler HWHM
 * aD = nu_k / c * sqrt(2 ln2 k_B T / (m u)), Lorentz HWHM
 * gL = g_ref (p / 1 bar) (296 / T)^0.5, and V the pseudo-Voigt profile of
 * Thompson, Cox & Hastings (1987, J. Appl. Cryst. 20, 79) normalised to
 * unit area, cut at |nu - nu_k| > wing_cut.  Output is log10(sigma) per row.
 *
 * Rows (T, p) are independent and run in parallel with OpenMP; the result
 * does not depend on the thread count (each row is summed in line order).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const double kC2 = 1.4387768775039337;      /* h c / k_B, cm K        */
static const double kKB = 1.380649e-16;            /* erg / K                */
static const double kAMU = 1.66053906660e-24;      /* g                      */
static const double kCLIGHT = 2.99792458e10;       /* cm / s                 */

/* pseudo-Voigt mixing of a Gaussian and a Lorentzian of common FWHM f */
static void pv_params(double fwhm_g, double fwhm_l, double *f, double *eta) {
  const double g = fwhm_g, l = fwhm_l;
  const double g2 = g * g, g3 = g2 * g, g4 = g3 * g, g5 = g4 * g;
  const double l2 = l * l, l3 = l2 * l, l4 = l3 * l, l5 = l4 * l;
  const double s = g5 + 2.69269 * g4 * l + 2.42843 * g3 * l2 + 4.47163 * g2 * l3 +
                   0.07842 * g * l4 + l5;
  *f = pow(s, 0.2);
  const double r = l / *f;
  *eta = 1.36603 * r - 0.47719 * r * r + 0.11116 * r * r * r;
}

void gen_xsec_table(int n_lines, const double *nu_line, const double *s296,
                    const double *e_low, const double *g_ref, double mass_amu,
                    int n_t, const double *t_axis, int n_p, const double *log10p_axis,
                    double nu0, double dnu, int64_t n_nu, double wing_cut,
                    double floor_sigma, double *out) {
  const int64_t n_rows = (int64_t)n_t * n_p;
#pragma omp parallel
  {
    double *row = (double *)malloc(sizeof(double) * (size_t)n_nu);
#pragma omp for schedule(dynamic, 1)
    for (int64_t r = 0; r < n_rows; ++r) {
      const int it = (int)(r / n_p), ip = (int)(r % n_p);
      const double T = t_axis[it];
      const double p = pow(10.0, log10p_axis[ip]);
      memset(row, 0, sizeof(double) * (size_t)n_nu);
      const double dop = sqrt(2.0 * log(2.0) * kKB * T / (mass_amu * kAMU)) / kCLIGHT;
      for (int k = 0; k < n_lines; ++k) {
        const double S = s296[k] * pow(296.0 / T, 1.5) *
                         exp(-kC2 * e_low[k] * (1.0 / T - 1.0 / 296.0));
        const double aD = nu_line[k] * dop;                  /* HWHM */
        const double gL = g_ref[k] * p * sqrt(296.0 / T);    /* HWHM */
        double f, eta;
        pv_params(2.0 * aD, 2.0 * gL, &f, &eta);
        const double hw = 0.5 * f;
        const double gnorm = sqrt(log(2.0) / M_PI) / hw;
        const double lnorm = 1.0 / (M_PI * hw);
        const double ga = log(2.0) / (hw * hw);
        int64_t lo = (int64_t)ceil((nu_line[k] - wing_cut - nu0) / dnu);
        int64_t hi = (int64_t)floor((nu_line[k] + wing_cut - nu0) / dnu);
        if (lo < 0) lo = 0;
        if (hi > n_nu - 1) hi = n_nu - 1;
        for (int64_t j = lo; j <= hi; ++j) {
          const double x = nu0 + (double)j * dnu - nu_line[k];
          const double gv = gnorm * exp(-ga * x * x);
          const double lv = lnorm / (1.0 + x * x / (hw * hw));
          row[j] += S * (eta * lv + (1.0 - eta) * gv);
        }
      }
      double *dst = out + r * n_nu;
      for (int64_t j = 0; j < n_nu; ++j) dst[j] = log10(floor_sigma + row[j]);
    }
    free(row);
  }
}
