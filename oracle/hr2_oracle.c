/*
 * hr2_oracle.c — plain FP64 CPU oracle of the Helios-r2 emission forward model
 * (Kitzmann et al. 2020, arXiv:1910.01070).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg may load this code; the product path never
 * does.  It shares no source, header, table or helper with the HIP library.
 *
 * Everything is written as the definition reads, in FP64 with libm, one
 * column and one wavenumber at a time, with no blocking, fusion or
 * reordering.  The OpenMP pragmas only distribute independent wavenumbers.
 * Readings of points the paper leaves open are stated where they are used.
 *
 * Units: cgs; wavenumber in cm^-1; pressure in bar at the interface
 * (converted to dyn cm^-2 inside); temperature in K.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

/* CODATA 2018 exact SI-defined constants in cgs, atomic mass constant. */
#define OR_H 6.62607015e-27        /* erg s */
#define OR_C 2.99792458e10         /* cm s^-1 */
#define OR_KB 1.380649e-16         /* erg K^-1 */
#define OR_AMU 1.66053906660e-24   /* g */
#define OR_BAR 1.0e6               /* dyn cm^-2 per bar */
#define OR_M_H2 2.016              /* g mol^-1 */
#define OR_M_HE 4.0026             /* g mol^-1 */
#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------
 * Angular quadrature for Eq. 8: F+ = 2 pi int_0^1 I(mu) mu dmu with an
 * n-point Gauss-Legendre rule on [0, 1] (reading: the paper's "Gauss
 * quadrature" over the outgoing hemisphere).  Nodes are the roots of the
 * Legendre polynomial P_n on [-1, 1] found by Newton's method from the
 * Chebyshev guess, mapped by mu = (1 + t)/2; weights w = 1 / ((1 - t^2)
 * P_n'(t)^2) on [-1, 1], halved for [0, 1].  Returns 0, or -1 if n < 1.
 * ---------------------------------------------------------------------- */
/* P_n(t) and P_{n-1}(t) by the three-term recurrence (k P_k = (2k-1) t P_{k-1} - (k-1) P_{k-2}). */
static void or_legendre_pair(int n, double t, double *pn, double *pnm1) {
  double p0 = 1.0, p1 = t;
  for (int k = 2; k <= n; ++k) {
    const double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *pn = p1;
  *pnm1 = p0;
}

int or_gauss_legendre01(int n, double *mu, double *w) {
  if (n < 1) return -1;
  for (int i = 0; i < n; ++i) {
    double t = cos(OR_PI * (i + 0.75) / (n + 0.5));
    double pn, pnm1, dp;
    for (int it = 0; it < 100; ++it) {
      or_legendre_pair(n, t, &pn, &pnm1);
      dp = n * (t * pn - pnm1) / (t * t - 1.0);   /* P_n'(t) */
      const double dt = pn / dp;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    or_legendre_pair(n, t, &pn, &pnm1);
    dp = n * (t * pn - pnm1) / (t * t - 1.0);
    /* roots come out in decreasing t; store mu increasing */
    mu[n - 1 - i] = 0.5 * (1.0 + t);
    w[n - 1 - i] = 0.5 * 2.0 / ((1.0 - t * t) * dp * dp);
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Eq. 2 source: S = B_nu(T), Planck's law per unit wavenumber,
 * B = 2 h c^2 nu^3 / (exp(h c nu / (k_B T)) - 1), erg s^-1 cm^-2 sr^-1 (cm^-1)^-1.
 * ---------------------------------------------------------------------- */
double or_planck(double nu_cm, double T_K) {
  const double x = OR_H * OR_C * nu_cm / (OR_KB * T_K);
  return 2.0 * OR_H * OR_C * OR_C * nu_cm * nu_cm * nu_cm / expm1(x);
}

void or_planck_n(int64_t n, const double *nu_cm, const double *T_K, double *out) {
  for (int64_t i = 0; i < n; ++i) out[i] = or_planck(nu_cm[i], T_K[i]);
}

/* ------------------------------------------------------------------------
 * Table lookup (reading: bilinear in (T, log10 p) on log10 sigma, clamped).
 * i = largest index with axis[i] <= v, capped at n-2; w = (v - a_i)/(a_{i+1} - a_i).
 * ---------------------------------------------------------------------- */
static void or_locate(const double *axis, int n, double v, int *i_out, double *w_out) {
  if (v < axis[0]) v = axis[0];
  if (v > axis[n - 1]) v = axis[n - 1];
  int i = 0;
  for (int k = 0; k < n; ++k)
    if (axis[k] <= v) i = k;
  if (i > n - 2) i = n - 2;
  *i_out = i;
  *w_out = (v - axis[i]) / (axis[i + 1] - axis[i]);
}

/* ------------------------------------------------------------------------
 * Level state of one column (Sect. 2, 2.4, 5.2; readings on dz and filler).
 *   n_tot_l = p_l / (k_B T_l)                      number density, cm^-3
 *   x_H2 = (1 - sum_s x_s) / (1 + r),  x_He = r x_H2   (isoprofiles)
 *   mubar = sum_s x_s m_s + x_H2 m_H2 + x_He m_He
 *   dz_l  = k_B (T_l + T_{l+1})/2 / (mubar m_u g) * ln(p_l / p_{l+1})
 * Outputs n_tot[L], x_h2, x_he, mubar (scalars), dz[L-1].
 * ---------------------------------------------------------------------- */
void or_column_state(int L, const double *p_bar, const double *T_K, int S, const double *x,
                     const double *molar_mass, double he_h2_ratio, double log_g,
                     double *n_tot, double *x_h2, double *x_he, double *mubar, double *dz) {
  double xs = 0.0, mm = 0.0;
  for (int s = 0; s < S; ++s) {
    xs += x[s];
    mm += x[s] * molar_mass[s];
  }
  const double h2 = (1.0 - xs) / (1.0 + he_h2_ratio);
  const double he = he_h2_ratio * h2;
  mm += h2 * OR_M_H2 + he * OR_M_HE;
  *x_h2 = h2;
  *x_he = he;
  *mubar = mm;
  const double g = pow(10.0, log_g);
  for (int l = 0; l < L; ++l) n_tot[l] = p_bar[l] * OR_BAR / (OR_KB * T_K[l]);
  for (int l = 0; l + 1 < L; ++l) {
    const double tbar = 0.5 * (T_K[l] + T_K[l + 1]);
    dz[l] = OR_KB * tbar / (mm * OR_AMU * g) * log(p_bar[l] / p_bar[l + 1]);
  }
}

/* ------------------------------------------------------------------------
 * Stage 1 (Sect. 2.3, 2.8): absorption coefficient of one column,
 *   chi_l(nu) = sum_s n_s,l sigma_s(nu; T_l, p_l)
 *             + n_H2,l^2 k_H2H2(T_l, nu) + n_H2,l n_He,l k_H2He(T_l, nu)
 * sigma from log10 sigma bilinear in (T, log10 p); CIA linear in T on log10 k.
 * Evaluated at table wavenumber indices nu_idx[n] (any subset).
 * Tables: log10_sigma[S][nT][nP][n_nu], log10_k_cia[n_cia][nT][n_nu] (n_cia 0 or 2).
 * Output chi[L][n].
 * ---------------------------------------------------------------------- */
void or_opacity(int S, int nT, int nP, const double *T_axis, const double *lp_axis, int64_t n_nu,
                const double *log10_sigma, int n_cia, const double *log10_k_cia,
                const double *molar_mass, double he_h2_ratio, int L, const double *p_bar,
                const double *T_K, const double *x, double log_g, int64_t n,
                const int64_t *nu_idx, double *chi) {
  double *n_tot = (double *)malloc(sizeof(double) * L);
  double *dz = (double *)malloc(sizeof(double) * (L > 1 ? L - 1 : 1));
  double x_h2, x_he, mubar;
  or_column_state(L, p_bar, T_K, S, x, molar_mass, he_h2_ratio, log_g, n_tot, &x_h2, &x_he,
                  &mubar, dz);
  for (int l = 0; l < L; ++l) {
    int iT, ip;
    double wT, wp;
    or_locate(T_axis, nT, T_K[l], &iT, &wT);
    or_locate(lp_axis, nP, log10(p_bar[l]), &ip, &wp);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
      const int64_t k = nu_idx[j];
      double c = 0.0;
      for (int s = 0; s < S; ++s) {
        const double *tab = log10_sigma + (size_t)s * nT * nP * n_nu;
        const double l00 = tab[((size_t)iT * nP + ip) * n_nu + k];
        const double l01 = tab[((size_t)iT * nP + ip + 1) * n_nu + k];
        const double l10 = tab[((size_t)(iT + 1) * nP + ip) * n_nu + k];
        const double l11 = tab[((size_t)(iT + 1) * nP + ip + 1) * n_nu + k];
        const double lg = (1.0 - wT) * ((1.0 - wp) * l00 + wp * l01) +
                          wT * ((1.0 - wp) * l10 + wp * l11);
        c += x[s] * n_tot[l] * pow(10.0, lg);
      }
      if (n_cia == 2) {
        const double nh2 = x_h2 * n_tot[l], nhe = x_he * n_tot[l];
        for (int q = 0; q < 2; ++q) {
          const double *tab = log10_k_cia + (size_t)q * nT * n_nu;
          const double lk = (1.0 - wT) * tab[(size_t)iT * n_nu + k] +
                            wT * tab[(size_t)(iT + 1) * n_nu + k];
          c += (q == 0 ? nh2 * nh2 : nh2 * nhe) * pow(10.0, lk);
        }
      }
      chi[(size_t)l * n + j] = c;
    }
  }
  free(n_tot);
  free(dz);
}

/* ------------------------------------------------------------------------
 * Eq. 4-7, short characteristics with a linear source and alpha = 0, for one
 * ray of direction mu from the bottom level (0) to the top (L-1).
 * Readings: the deeper level is upwind; Delta = dtau_l / mu >= 0; the
 * attenuation of Eq. 4 is exp(-Delta); gamma carries the sign that makes
 * beta + gamma = 1 - exp(-Delta); the lower boundary is I = S_0.
 *   u = (1 - e^-Delta)/Delta (u = 1 at Delta = 0)
 *   beta = 1 - u,  gamma = u - e^-Delta
 *   I_{l+1} = e^-Delta I_l + beta S_{l+1} + gamma S_l
 * dtau[L-1] per layer, S[L] at levels.  Returns I at the top.
 * ---------------------------------------------------------------------- */
double or_sc_intensity(int L, const double *dtau, const double *S, double mu) {
  double I = S[0];
  for (int l = 0; l + 1 < L; ++l) {
    const double d = dtau[l] / mu;
    const double e = exp(-d);
    const double u = (d > 0.0) ? -expm1(-d) / d : 1.0;
    const double beta = 1.0 - u;
    const double gamma = u - e;
    I = e * I + beta * S[l + 1] + gamma * S[l];
  }
  return I;
}

/* ------------------------------------------------------------------------
 * Parabolic short characteristics (the higher-order interpolant the paper
 * mentions with Eq. 4-7, coefficients after Olson & Kunasz 1987): on the
 * step from level i-1 (upwind) to level i the source is the quadratic
 * through S_{i-1}, S_i and S_{i+1} (the downwind level).  With optical
 * path lengths du (layer i-1 -> i) and dd (layer i -> i+1) along the ray and
 * x the optical distance back from level i, S(0) = S_i, S(du) = S_{i-1},
 * S(-dd) = S_{i+1}, and
 *   Delta I_i = int_0^du S(x) e^{-x} dx = alpha S_{i+1} + beta S_i + gamma S_{i-1}
 * with the moments w_n = int_0^du x^n e^{-x} dx:
 *   w0 = 1 - e^{-du},  w1 = w0 - du e^{-du},  w2 = 2 w1 - du^2 e^{-du},
 *   gamma = (w2 + dd w1) / (du (du + dd)),
 *   beta  = (du dd w0 - w2 - (dd - du) w1) / (du dd),
 *   alpha = (w2 - du w1) / (dd (du + dd)).
 * Readings (the paper gives no formulas): the top step, which has no
 * downwind level, and a step whose downwind layer has zero optical depth
 * use the linear coefficients (alpha = 0); a step with du = 0 adds nothing.
 * ---------------------------------------------------------------------- */
/* w_n = int_0^x t^n e^{-t} dt is the lower incomplete gamma function
 * gamma(n+1, x).  Up to x = 30 it is summed from its series of positive
 * terms, x^{n+1} e^{-x} sum_k x^k / ((n+1)(n+2)...(n+1+k)), which keeps full
 * relative accuracy for optically thin layers (the closed forms
 * w1 = w0 - x e^{-x} and w2 = 2 w1 - x^2 e^{-x} cancel there); beyond, the
 * closed form n! (1 - e^{-x} sum_{k<=n} x^k/k!) has nothing to cancel. */
static double or_moment(int n, double x) {
  if (x > 30.0) {
    double sum = 0.0, t = 1.0, fact = 1.0;
    for (int k = 0; k <= n; ++k) {
      if (k > 0) t *= x / k;
      sum += t;
    }
    for (int k = 2; k <= n; ++k) fact *= k;
    return fact * (1.0 - exp(-x) * sum);
  }
  const double s = n + 1.0;
  double term = 1.0 / s, sum = term;
  for (int k = 1; k < 400; ++k) {
    term *= x / (s + k);
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return pow(x, s) * exp(-x) * sum;
}

void or_sc_para_coeffs(double du, double dd, double *alpha, double *beta, double *gamma) {
  const double w0 = -expm1(-du);
  const double w1 = or_moment(1, du);
  const double w2 = or_moment(2, du);
  *gamma = (w2 + dd * w1) / (du * (du + dd));
  *beta = (du * dd * w0 - w2 - (dd - du) * w1) / (du * dd);
  *alpha = (w2 - du * w1) / (dd * (du + dd));
}

double or_sc_intensity_para(int L, const double *dtau, const double *S, double mu) {
  double I = S[0];
  for (int l = 0; l + 1 < L; ++l) {
    const double du = dtau[l] / mu;
    if (du == 0.0) continue;
    const double e = exp(-du);
    if (l + 2 < L && dtau[l + 1] > 0.0) {
      double a, b, g;
      or_sc_para_coeffs(du, dtau[l + 1] / mu, &a, &b, &g);
      I = e * I + a * S[l + 2] + b * S[l + 1] + g * S[l];
    } else {
      const double u = -expm1(-du) / du;
      I = e * I + (1.0 - u) * S[l + 1] + (u - e) * S[l];
    }
  }
  return I;
}

/* Eq. 8 with the n_mu-point rule: F+ = 2 pi sum_k w_k mu_k I(mu_k); order 1
 * is the linear source of Eq. 5-6, order 2 the parabolic one. */
double or_sc_flux_o(int L, const double *dtau, const double *S, int n_mu, int order) {
  double mu[64], w[64];
  if (n_mu < 1 || n_mu > 64) return NAN;
  or_gauss_legendre01(n_mu, mu, w);
  double f = 0.0;
  for (int k = 0; k < n_mu; ++k)
    f += w[k] * mu[k] *
         (order == 2 ? or_sc_intensity_para(L, dtau, S, mu[k]) : or_sc_intensity(L, dtau, S, mu[k]));
  return 2.0 * OR_PI * f;
}

double or_sc_flux(int L, const double *dtau, const double *S, int n_mu) {
  return or_sc_flux_o(L, dtau, S, n_mu, 1);
}

/* ------------------------------------------------------------------------
 * Gray cloud layer (App. B): total optical depth tau_c, wavenumber
 * independent, between the cloud top p_top and the cloud bottom
 * p_top * bottom_frac (bottom_frac > 1).  The appendix does not say how the
 * optical depth is spread; reading: uniformly in ln p, so layer l (levels l
 * and l+1, p_l > p_{l+1}) receives tau_c times the share of
 * [ln p_top, ln(p_top bottom_frac)] that [ln p_{l+1}, ln p_l] covers.
 * ---------------------------------------------------------------------- */
void or_cloud_dtau(int L, const double *p_bar, double tau_c, double p_top_bar,
                   double bottom_frac, double *dtau_c) {
  const double a = log(p_top_bar), b = log(p_top_bar * bottom_frac);
  for (int l = 0; l + 1 < L; ++l) {
    const double lo = log(p_bar[l + 1]), hi = log(p_bar[l]);
    double ov = (hi < b ? hi : b) - (lo > a ? lo : a);
    if (ov < 0.0) ov = 0.0;
    dtau_c[l] = tau_c * ov / (b - a);
  }
}

/* ------------------------------------------------------------------------
 * Stage 2 (Eq. 2-8) for one column: dtau_l = (chi_l + chi_{l+1})/2 dz_l
 * (+ dtau_extra[l], a gray cloud's share, when dtau_extra is not NULL),
 * S_l = B(nu, T_l), F+ per wavenumber.  chi[L][n], dz[L-1], T[L], nu[n].
 * ---------------------------------------------------------------------- */
void or_rt_emission_o(int L, int64_t n, const double *chi, const double *dz, const double *T_K,
                      const double *nu, int n_mu, const double *dtau_extra, int order,
                      double *fplus) {
#pragma omp parallel
  {
    double *dtau = (double *)malloc(sizeof(double) * (L > 1 ? L - 1 : 1));
    double *S = (double *)malloc(sizeof(double) * L);
#pragma omp for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
      for (int l = 0; l + 1 < L; ++l) {
        dtau[l] = 0.5 * (chi[(size_t)l * n + j] + chi[(size_t)(l + 1) * n + j]) * dz[l];
        if (dtau_extra) dtau[l] += dtau_extra[l];
      }
      for (int l = 0; l < L; ++l) S[l] = or_planck(nu[j], T_K[l]);
      fplus[j] = or_sc_flux_o(L, dtau, S, n_mu, order);
    }
    free(dtau);
    free(S);
  }
}

void or_rt_emission_x(int L, int64_t n, const double *chi, const double *dz, const double *T_K,
                      const double *nu, int n_mu, const double *dtau_extra, double *fplus) {
  or_rt_emission_o(L, n, chi, dz, T_K, nu, n_mu, dtau_extra, 1, fplus);
}

void or_rt_emission(int L, int64_t n, const double *chi, const double *dz, const double *T_K,
                    const double *nu, int n_mu, double *fplus) {
  or_rt_emission_o(L, n, chi, dz, T_K, nu, n_mu, NULL, 1, fplus);
}

/* ------------------------------------------------------------------------
 * Eq. 17, Gaussian instrument profile truncated at 5 sigma (Sect. 2.7).
 * Window of N points, spacing dnu_eff, first point nu_first.  For output
 * point i: sigma_i = nu_i / (R 2 sqrt(2 ln 2)) (FWHM = nu/R, read from the
 * resolving power), keep window points m with |m - i| dnu_eff <= 5 sigma_i,
 * g = exp(-((m - i) dnu_eff)^2 / (2 sigma_i^2)), Fd_i = sum g F_m / sum g.
 * Output at indices out_idx[n_out].
 * ---------------------------------------------------------------------- */
void or_convolve(int64_t N, double nu_first, double dnu_eff, const double *F, double R,
                 int64_t n_out, const int64_t *out_idx, double *Fd) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < n_out; ++q) {
    const int64_t i = out_idx[q];
    const double nu_i = nu_first + (double)i * dnu_eff;
    const double sig = nu_i / (R * 2.0 * sqrt(2.0 * log(2.0)));
    double num = 0.0, den = 0.0;
    for (int64_t m = 0; m < N; ++m) {
      const double dx = (double)(m > i ? m - i : i - m) * dnu_eff;
      if (dx <= 5.0 * sig) {
        const double g = exp(-dx * dx / (2.0 * sig * sig));
        num += g * F[m];
        den += g;
      }
    }
    Fd[q] = num / den;
  }
}

/* Same, restricted to m within +-(max half width) of i: identical result
 * (the skipped points fail the 5 sigma test), used for large windows. */
void or_convolve_banded(int64_t N, double nu_first, double dnu_eff, const double *F, double R,
                        int64_t n_out, const int64_t *out_idx, double *Fd) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < n_out; ++q) {
    const int64_t i = out_idx[q];
    const double nu_i = nu_first + (double)i * dnu_eff;
    const double sig = nu_i / (R * 2.0 * sqrt(2.0 * log(2.0)));
    const int64_t h = (int64_t)(5.0 * sig / dnu_eff) + 2;
    const int64_t lo = i - h < 0 ? 0 : i - h;
    const int64_t hi = i + h > N - 1 ? N - 1 : i + h;
    double num = 0.0, den = 0.0;
    for (int64_t m = lo; m <= hi; ++m) {
      const double dx = (double)(m > i ? m - i : i - m) * dnu_eff;
      if (dx <= 5.0 * sig) {
        const double g = exp(-dx * dx / (2.0 * sig * sig));
        num += g * F[m];
        den += g;
      }
    }
    Fd[q] = num / den;
  }
}

/* ------------------------------------------------------------------------
 * Edge snapping (reading of the binning): nearest window point,
 * idx = floor((e - nu_first)/dnu_eff + 1/2).  Returns 0, or -1 if an index
 * leaves [0, N-1] or the indices are not strictly increasing.
 * ---------------------------------------------------------------------- */
int or_snap_edges(int n_edges, const double *edges_cm, double nu_first, double dnu_eff,
                  int64_t N, int64_t *idx) {
  for (int e = 0; e < n_edges; ++e) {
    idx[e] = (int64_t)floor((edges_cm[e] - nu_first) / dnu_eff + 0.5);
    if (idx[e] < 0 || idx[e] > N - 1) return -1;
    if (e > 0 && idx[e] <= idx[e - 1]) return -1;
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Binning (Sect. 2.8) with the Eq. 9 scale: bin j spans window points
 * a = edge_idx[j] .. b = edge_idx[j+1];
 *   bin_j = scale * sum_{m=a}^{b-1} (Fd_m + Fd_{m+1})/2 dnu / (nu_b - nu_a)
 * Fd must hold the convolved spectrum on every window point a..b used.
 * ---------------------------------------------------------------------- */
void or_bin(double nu_first, double dnu_eff, const double *Fd, int n_bins,
            const int64_t *edge_idx, double scale, double *bins) {
  for (int j = 0; j < n_bins; ++j) {
    const int64_t a = edge_idx[j], b = edge_idx[j + 1];
    const double nu_a = nu_first + (double)a * dnu_eff;
    const double nu_b = nu_first + (double)b * dnu_eff;
    double s = 0.0;
    for (int64_t m = a; m < b; ++m) s += 0.5 * (Fd[m] + Fd[m + 1]) * dnu_eff;
    bins[j] = scale * s / (nu_b - nu_a);
  }
}

/* ------------------------------------------------------------------------
 * Gaussian log-likelihood of binned data (Sect. 3.1, Eq. 19):
 *   ln L = sum_j ( -(D_j - m_j)^2 / (2 s_j^2) - 1/2 ln(2 pi s_j^2) ),
 * with s_j^2 = sigma_j^2, or with error inflation (Sect. 3.3, Eq. 22-23)
 * s_j^2 = sigma_j^2 + 10^eps when with_eps != 0.  Reading of Eq. 23: its
 * second term belongs inside the sum, as in Eq. 19.
 * ---------------------------------------------------------------------- */
double or_lnl(int n_bins, const double *model, const double *D, const double *sigma,
              int with_eps, double log10_eps) {
  double lnl = 0.0;
  for (int j = 0; j < n_bins; ++j) {
    double s2 = sigma[j] * sigma[j];
    if (with_eps) s2 += pow(10.0, log10_eps);
    const double r = D[j] - model[j];
    lnl += -r * r / (2.0 * s2) - 0.5 * log(2.0 * OR_PI * s2);
  }
  return lnl;
}

/* Threads of the OpenMP loops (timing runs of the oracle; the results do not
 * depend on it: every loop writes independent outputs). */
void or_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

int or_max_threads(void) { return omp_get_max_threads(); }
