/*
 * oracle.c -- plain FP64 CPU oracle for non-linear digital tracking.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU path against a slow,
 * obviously correct statement of what the method computes.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * Method (Golovich et al. 2025, "Survey-Wide Asteroid Discovery with a
 * High-Performance Computing Enabled Non-Linear Digital Tracking Framework"):
 *   - Sec. 3: candidate orbits are Keplerian element sets moving on
 *     elliptical two-body orbits about the Sun; each (image, orbit) pair is
 *     checked by brute force: the orbit is carried to the image epoch and
 *     mapped to pixels through the image's WCS (Calabretta & Greisen TAN).
 *   - Sec. 3: intersections outside an image are discarded; for each kept
 *     one, a Gaussian-PSF matched filter (width from the header) is applied
 *     to the pixels around it, with a per-pixel noise variance.
 *   - Sec. 3: per-image signals are combined under the assumption of a
 *     constant flux across images; Algorithm 1 ends with a significance
 *     decision per orbit.
 * Readings where the paper is silent (frames, constants, light time,
 * pixel origin, stamp size, masking) are fixed below at each function.
 *
 * Everything is evaluated one sample at a time, in FP64, with no blocking,
 * fusion or reordering beyond the definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- constants (reading: Gaussian constant, SI light speed, IAU 2006 obliquity) ---- */
static const double OR_PI = 3.14159265358979323846;
static const double OR_K = 0.01720209895;          /* AU^1.5 / day */
#define OR_MU (OR_K * OR_K)                         /* GM_sun, AU^3/day^2 */
static double or_c_au_per_day(void) { return 299792458.0 * 86400.0 / 149597870700.0; }
static double or_obliquity_rad(void) { return 84381.448 / 3600.0 * OR_PI / 180.0; }

/* Exposure record used by this oracle only (doubles, fixed stride). */
enum {
  X_T = 0, X_OX, X_OY, X_OZ,   /* epoch (days) and heliocentric ecliptic observer (AU) */
  X_RA0, X_DEC0,               /* TAN tangent point, degrees */
  X_CRPIX1, X_CRPIX2,          /* FITS 1-based reference pixel */
  X_CD11, X_CD12, X_CD21, X_CD22, /* deg/px */
  X_W, X_H,                    /* image size in pixels */
  X_FWHM,                      /* Gaussian PSF FWHM in pixels */
  X_STRIDE = 16
};

/* ------------------------------------------------------------------------- */
/* Kepler's equation E - e sin E = M (two-body motion, Sec. 3).               */
/* Newton's method from the starter E0 = M + 0.85 e sign(sin M), kept inside  */
/* the bracket [M - e, M + e] (the root satisfies |E - M| <= e) by bisection. */
/* Returns the iteration count, or -1 if 50 iterations did not converge.      */
/* ------------------------------------------------------------------------- */
double or_reduce_angle(double M) {
  double r = fmod(M + OR_PI, 2.0 * OR_PI);
  if (r < 0) r += 2.0 * OR_PI;
  return r - OR_PI;
}

int or_kepler(double M, double e, double *E_out) {
  M = or_reduce_angle(M);
  double lo = M - e, hi = M + e;
  double s = sin(M);
  double E = M + 0.85 * e * (s > 0 ? 1.0 : (s < 0 ? -1.0 : 0.0));
  if (E < lo) E = lo;
  if (E > hi) E = hi;
  for (int it = 1; it <= 50; ++it) {
    double f = E - e * sin(E) - M;
    double fp = 1.0 - e * cos(E);
    if (f == 0.0) { *E_out = E; return it; }
    if (f > 0) hi = E; else lo = E;
    double dE = -f / fp;
    if (fabs(dE) <= 1e-15 * fmax(1.0, fabs(E))) { *E_out = E + dE; return it; }
    double En = E + dE;
    if (!(En > lo && En < hi)) En = 0.5 * (lo + hi);   /* safeguard */
    E = En;
  }
  *E_out = E;
  return -1;
}

/* Orbital basis: P points to perihelion, Q is 90 deg ahead in the orbit plane,
 * both in heliocentric ecliptic J2000 (textbook two-body geometry). */
void or_orbit_basis(double inc, double node, double peri, double P[3], double Q[3]) {
  double cO = cos(node), sO = sin(node), cw = cos(peri), sw = sin(peri);
  double ci = cos(inc), si = sin(inc);
  P[0] = cO * cw - sO * sw * ci;
  P[1] = sO * cw + cO * sw * ci;
  P[2] = sw * si;
  Q[0] = -cO * sw - sO * cw * ci;
  Q[1] = -sO * sw + cO * cw * ci;
  Q[2] = cw * si;
}

/* Heliocentric ecliptic position (and velocity) at time t of the element set
 * el = (a [AU], e, i, node, peri, M0 [rad]) osculating at epoch t0.
 * Returns the Kepler iteration count (<0 on non-convergence). */
int or_helio_state(const double el[6], double t0, double t, double r[3], double v[3]) {
  double a = el[0], e = el[1];
  double n = OR_K / (a * sqrt(a));
  double P[3], Q[3];
  or_orbit_basis(el[2], el[3], el[4], P, Q);
  double E;
  int it = or_kepler(el[5] + n * (t - t0), e, &E);
  double cE = cos(E), sE = sin(E);
  double sq = sqrt(1.0 - e * e);
  double X = a * (cE - e), Y = a * sq * sE;
  double rn = a * (1.0 - e * cE);
  double vs = sqrt(OR_MU * a) / rn;
  for (int k = 0; k < 3; ++k) {
    r[k] = X * P[k] + Y * Q[k];
    if (v) v[k] = vs * (-sE * P[k] + sq * cE * Q[k]);
  }
  return it;
}

/* Light time (reading: astrometric position, no aberration or deflection).
 * Fixed point tau = |r(t_e - tau) - r_obs| / c from tau = 0, stopped when the
 * change is <= 1e-14 day or after 10 updates; rho = r(t_e - tau) - r_obs.
 * Returns the number of updates, -1 if it did not settle, -2 on Kepler failure. */
int or_light_time(const double el[6], double t0, double t_e, const double robs[3],
                  double rho[3], double *tau_out, double helio[3]) {
  const double c = or_c_au_per_day();
  double tau = 0.0, r[3];
  int status = -1;
  for (int j = 1; j <= 10; ++j) {
    if (or_helio_state(el, t0, t_e - tau, r, NULL) < 0) return -2;
    double d0 = r[0] - robs[0], d1 = r[1] - robs[1], d2 = r[2] - robs[2];
    double tn = sqrt(d0 * d0 + d1 * d1 + d2 * d2) / c;
    double dt = fabs(tn - tau);
    tau = tn;
    if (dt <= 1e-14) { status = j; break; }
  }
  if (or_helio_state(el, t0, t_e - tau, r, NULL) < 0) return -2;
  for (int k = 0; k < 3; ++k) {
    rho[k] = r[k] - robs[k];
    if (helio) helio[k] = r[k];
  }
  *tau_out = tau;
  return status;
}

/* Ecliptic J2000 -> equatorial (rotation about +x by the obliquity). */
void or_ecl_to_eq(const double v[3], double out[3]) {
  double eps = or_obliquity_rad();
  double ce = cos(eps), se = sin(eps);
  out[0] = v[0];
  out[1] = ce * v[1] - se * v[2];
  out[2] = se * v[1] + ce * v[2];
}

/* Equatorial -> ecliptic J2000 (the inverse rotation). */
void or_eq_to_ecl(const double v[3], double out[3]) {
  double eps = or_obliquity_rad();
  double ce = cos(eps), se = sin(eps);
  out[0] = v[0];
  out[1] = ce * v[1] + se * v[2];
  out[2] = -se * v[1] + ce * v[2];
}

/* Gnomonic (FITS TAN, native pole at LONPOLE = 180 deg) projection of the
 * equatorial unit vector u onto 0-based pixel coordinates, centres at
 * integers (reading: FITS 1-based CRPIX minus one).  Returns 0 if u is on or
 * behind the tangent plane's hemisphere (w <= 0), else 1. */
int or_tan_project(const double u[3], double ra0_deg, double dec0_deg,
                   double crpix1, double crpix2, const double cd[4],
                   double *px, double *py) {
  double d2r = OR_PI / 180.0;
  double a0 = ra0_deg * d2r, d0 = dec0_deg * d2r;
  double c_hat[3] = {cos(d0) * cos(a0), cos(d0) * sin(a0), sin(d0)};
  double e_hat[3] = {-sin(a0), cos(a0), 0.0};
  double n_hat[3] = {-sin(d0) * cos(a0), -sin(d0) * sin(a0), cos(d0)};
  double w = u[0] * c_hat[0] + u[1] * c_hat[1] + u[2] * c_hat[2];
  if (!(w > 0.0)) return 0;
  double xi = (180.0 / OR_PI) * (u[0] * e_hat[0] + u[1] * e_hat[1] + u[2] * e_hat[2]) / w;
  double eta = (180.0 / OR_PI) * (u[0] * n_hat[0] + u[1] * n_hat[1] + u[2] * n_hat[2]) / w;
  double det = cd[0] * cd[3] - cd[1] * cd[2];
  double ix = (cd[3] * xi - cd[1] * eta) / det;
  double iy = (-cd[2] * xi + cd[0] * eta) / det;
  *px = (crpix1 - 1.0) + ix;
  *py = (crpix2 - 1.0) + iy;
  return 1;
}

/* One (orbit, exposure) intersection: propagate with light time, rotate to
 * equatorial, project, take the nearest pixel floor(p + 0.5).
 * Output flags: bit0 = in front of the tangent plane, bit1 = inside image.
 * Returns <0 on a Kepler / light-time failure. */
int or_intersect(const double el[6], double t0, const double *x,
                 double *px, double *py, int32_t *ix, int32_t *iy,
                 double helio[3], double *tau, int32_t *flags) {
  double robs[3] = {x[X_OX], x[X_OY], x[X_OZ]};
  double rho[3];
  int lt = or_light_time(el, t0, x[X_T], robs, rho, tau, helio);
  *flags = 0;
  *px = *py = NAN;
  *ix = *iy = INT32_MIN;
  if (lt == -2) return -2;
  double rn = sqrt(rho[0] * rho[0] + rho[1] * rho[1] + rho[2] * rho[2]);
  if (!(rn >= 1e-9)) return lt;
  double ue[3] = {rho[0] / rn, rho[1] / rn, rho[2] / rn}, uq[3];
  or_ecl_to_eq(ue, uq);
  double cd[4] = {x[X_CD11], x[X_CD12], x[X_CD21], x[X_CD22]};
  if (!or_tan_project(uq, x[X_RA0], x[X_DEC0], x[X_CRPIX1], x[X_CRPIX2], cd, px, py))
    return lt;
  *flags |= 1;
  double fx = floor(*px + 0.5), fy = floor(*py + 0.5);
  if (fx > -1e9 && fx < 1e9 && fy > -1e9 && fy < 1e9) {
    *ix = (int32_t)fx;
    *iy = (int32_t)fy;
    if (*ix >= 0 && *ix < (int32_t)x[X_W] && *iy >= 0 && *iy < (int32_t)x[X_H]) *flags |= 2;
  }
  return lt;
}

/* ---- pixels ------------------------------------------------------------- */
/* IEEE binary16 -> double, exact. */
double or_half_to_double(uint16_t h) {
  int s = h >> 15, ex = (h >> 10) & 0x1f, m = h & 0x3ff;
  double v;
  if (ex == 0) v = ldexp((double)m, -24);
  else if (ex == 31) v = m ? NAN : INFINITY;
  else v = ldexp(1024.0 + m, ex - 25);
  return s ? -v : v;
}

static double or_pix(const void *img, int dtype, int64_t k) {
  if (dtype == 0) return (double)((const float *)img)[k];
  return or_half_to_double(((const uint16_t *)img)[k]);
}

/* Gaussian matched filter at the nearest pixel (Sec. 3: Gaussian PSF of
 * header width, per-pixel noise variance).  Reading: point-sampled Gaussian,
 * sigma = FWHM / (2 sqrt(2 ln 2)), square stamp of half-width R = ceil(3 sigma)
 * centred on (ix, iy), normalised to unit sum over the stamp; pixels off the
 * image, with non-finite D or V, or V <= 0 carry zero weight.
 *   psi = sum P D / V,   phi = sum P^2 / V   (summed in (dy, dx) order). */
void or_stamp(const void *D, const void *V, int dtype, int W, int H, int ix, int iy,
              double fwhm, double *psi_out, double *phi_out) {
  double sig = fwhm / (2.0 * sqrt(2.0 * log(2.0)));
  int R = (int)ceil(3.0 * sig);
  double Z = 0.0;
  for (int dy = -R; dy <= R; ++dy)
    for (int dx = -R; dx <= R; ++dx) Z += exp(-(dx * dx + dy * dy) / (2.0 * sig * sig));
  double psi = 0.0, phi = 0.0;
  for (int dy = -R; dy <= R; ++dy) {
    for (int dx = -R; dx <= R; ++dx) {
      int x = ix + dx, y = iy + dy;
      if (x < 0 || x >= W || y < 0 || y >= H) continue;
      int64_t k = (int64_t)y * W + x;
      double d = or_pix(D, dtype, k), v = or_pix(V, dtype, k);
      if (!isfinite(d) || !isfinite(v) || !(v > 0.0)) continue;
      double P = exp(-(dx * dx + dy * dy) / (2.0 * sig * sig)) / Z;
      psi += P * d / v;
      phi += P * P / v;
    }
  }
  *psi_out = psi;
  *phi_out = phi;
}

/* The same filter evaluated at every pixel of one image (the plane form). */
void or_planes(const void *D, const void *V, int dtype, int W, int H, double fwhm,
               double *psi, double *phi) {
#pragma omp parallel for schedule(static)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      or_stamp(D, V, dtype, W, H, x, y, fwhm, &psi[(int64_t)y * W + x], &phi[(int64_t)y * W + x]);
}

/* ---- per-sample debug table --------------------------------------------- */
/* For m orbits (rows of el) and n_exp exposures: pixel coordinates, nearest
 * pixel, flags (bit0 front, bit1 inside, bit2 filter weight > 0 => valid),
 * the filter values, light time and heliocentric position. */
int or_samples(int64_t m, const double *el, double t0, int n_exp, const double *xp,
               const void *const *D, const void *const *V, int dtype,
               double *px, double *py, int32_t *ix, int32_t *iy, int32_t *flags,
               double *psi, double *phi, double *tau, double *helio) {
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
  for (int64_t o = 0; o < m; ++o) {
    for (int e = 0; e < n_exp; ++e) {
      int64_t k = o * n_exp + e;
      const double *x = xp + (int64_t)e * X_STRIDE;
      double h[3];
      int st = or_intersect(el + 6 * o, t0, x, &px[k], &py[k], &ix[k], &iy[k], h, &tau[k], &flags[k]);
      if (st < 0) bad++;
      if (helio) { helio[3 * k] = h[0]; helio[3 * k + 1] = h[1]; helio[3 * k + 2] = h[2]; }
      psi[k] = phi[k] = 0.0;
      if ((flags[k] & 3) == 3 && D) {
        or_stamp(D[e], V[e], dtype, (int)x[X_W], (int)x[X_H], ix[k], iy[k], x[X_FWHM], &psi[k], &phi[k]);
        if (phi[k] > 0.0) flags[k] |= 4; else psi[k] = phi[k] = 0.0;
      }
    }
  }
  return bad;
}

/* ---- constant-flux stack (Sec. 3) --------------------------------------- */
/* Psi = sum_e psi_e, Phi = sum_e phi_e over valid samples (epoch order);
 * S/N = Psi / sqrt(Phi), flux = Psi / Phi; both 0 when Phi = 0. */
static void or_stack_one(const double *el, double t0, int n_exp, const double *xp,
                         const void *const *D, const void *const *V, int dtype,
                         double *snr, double *flux, int32_t *nvalid, int *bad) {
  double Psi = 0.0, Phi = 0.0;
  int nv = 0;
  for (int e = 0; e < n_exp; ++e) {
    const double *x = xp + (int64_t)e * X_STRIDE;
    double px, py, h[3], tau, psi, phi;
    int32_t ix, iy, fl;
    if (or_intersect(el, t0, x, &px, &py, &ix, &iy, h, &tau, &fl) < 0) (*bad)++;
    if ((fl & 3) != 3) continue;
    or_stamp(D[e], V[e], dtype, (int)x[X_W], (int)x[X_H], ix, iy, x[X_FWHM], &psi, &phi);
    if (!(phi > 0.0)) continue;
    Psi += psi;
    Phi += phi;
    nv++;
  }
  *snr = Phi > 0.0 ? Psi / sqrt(Phi) : 0.0;
  *flux = Phi > 0.0 ? Psi / Phi : 0.0;
  *nvalid = nv;
}

int or_stack(int64_t n_orb, const double *el, double t0, int n_exp, const double *xp,
             const void *const *D, const void *const *V, int dtype,
             double *snr, double *flux, int32_t *nvalid, int nthreads) {
  int bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
  for (int64_t o = 0; o < n_orb; ++o)
    or_stack_one(el + 6 * o, t0, n_exp, xp, D, V, dtype, &snr[o], &flux[o], &nvalid[o], &bad);
  return bad;
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---- linear shift-and-stack (classic digital tracking, Sec. 1) ----------- */
/* Track x_e = x0 + vx (t_e - tref), y_e = y0 + vy (t_e - tref) in pixels of
 * every exposure; nearest pixel, validity and filter as above. */
void or_linear_stack(int n_tracks, const double *trk /* n x 4: x0,y0,vx,vy */, double tref,
                     int n_exp, const double *xp, const void *const *D, const void *const *V,
                     int dtype, double *snr, double *flux, int32_t *nvalid) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n_tracks; ++k) {
    double Psi = 0.0, Phi = 0.0;
    int nv = 0;
    for (int e = 0; e < n_exp; ++e) {
      const double *x = xp + (int64_t)e * X_STRIDE;
      double dt = x[X_T] - tref;
      double fx = floor(trk[4 * k] + trk[4 * k + 2] * dt + 0.5);
      double fy = floor(trk[4 * k + 1] + trk[4 * k + 3] * dt + 0.5);
      if (fx < 0 || fy < 0 || fx >= x[X_W] || fy >= x[X_H]) continue;
      double psi, phi;
      or_stamp(D[e], V[e], dtype, (int)x[X_W], (int)x[X_H], (int)fx, (int)fy, x[X_FWHM], &psi, &phi);
      if (!(phi > 0.0)) continue;
      Psi += psi;
      Phi += phi;
      nv++;
    }
    snr[k] = Phi > 0.0 ? Psi / sqrt(Phi) : 0.0;
    flux[k] = Phi > 0.0 ? Psi / Phi : 0.0;
    nvalid[k] = nv;
  }
}

/* ---- detection: threshold + top-k (Algorithm 1, final step) -------------- */
/* Order: S/N descending, ties to the lower orbit index; only S/N >= thr. */
static const double *or_sort_key;
static int or_cmp(const void *pa, const void *pb) {
  int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
  double x = or_sort_key[a], y = or_sort_key[b];
  if (x > y) return -1;
  if (x < y) return 1;
  return (a < b) ? -1 : (a > b);
}

int64_t or_topk(int64_t n, const double *snr, int64_t k, double thr, int64_t *idx_out) {
  int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i)
    if (snr[i] >= thr) ids[m++] = i;
  or_sort_key = snr;
  qsort(ids, (size_t)m, sizeof(int64_t), or_cmp);
  int64_t cnt = m < k ? m : k;
  memcpy(idx_out, ids, sizeof(int64_t) * (size_t)cnt);
  free(ids);
  return cnt;
}

/* ---- per-intersection outlier trimming (Sec. 5.2.3) ------------------------ */
/* Under the constant-flux model every valid intersection e (phi_e > 0) gives
 * an independent flux estimate f_e = psi_e / phi_e of variance 1 / phi_e.
 * The paper removes intersections whose S/N is anomalously far from the
 * expectation by sigma clipping.  Reading: the expectation starts at the
 * median of the f_e (so that one dominant artifact cannot set it) and is
 * then the weighted mean F = sum psi / sum phi of the kept samples; a sample
 * is dropped when its residual chi_e = (psi_e - F phi_e) / sqrt(phi_e) has
 * |chi_e| > kappa (both sides: a one-sided clip lets a deep negative
 * artifact drag F down until the ordinary samples look high).  Iteration 1
 * clips about the median; every later round about the fit of the set the
 * previous round kept, until a round keeps exactly that set or after
 * max_iter rounds.  The median of an even count is the mean of the two
 * middle values.  Returns the S/N, flux and count of the kept set. */
static int or_cmp_dbl(const void *pa, const void *pb) {
  double a = *(const double *)pa, b = *(const double *)pb;
  return (a > b) - (a < b);
}

void or_sigma_clip(int n, const double *psi, const double *phi, double kappa, int max_iter,
                   double *snr, double *flux, int32_t *n_kept, uint8_t *kept) {
  double *f = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  int m = 0;
  for (int i = 0; i < n; ++i) {
    kept[i] = phi[i] > 0.0;
    if (kept[i]) f[m++] = psi[i] / phi[i];
  }
  double F = 0.0;
  if (m > 0) {
    qsort(f, (size_t)m, sizeof(double), or_cmp_dbl);
    F = 0.5 * (f[(m - 1) / 2] + f[m / 2]);
  }
  free(f);
  /* the first round clips about the median; later rounds about the fit of
   * the kept set, until a round keeps exactly the set it started from */
  for (int it = 0; it < max_iter && m > 0; ++it) {
    if (it > 0) {
      double P = 0.0, Q = 0.0;
      for (int i = 0; i < n; ++i)
        if (kept[i]) {
          P += psi[i];
          Q += phi[i];
        }
      F = P / Q;
    }
    int changed = 0;
    for (int i = 0; i < n; ++i) {
      if (!(phi[i] > 0.0)) continue;
      uint8_t k = fabs(psi[i] - F * phi[i]) / sqrt(phi[i]) <= kappa;
      if (k != kept[i]) {
        kept[i] = k;
        changed = 1;
      }
    }
    if (it > 0 && !changed) break;
  }
  double P = 0.0, Q = 0.0;
  int c = 0;
  for (int i = 0; i < n; ++i)
    if (kept[i]) {
      P += psi[i];
      Q += phi[i];
      c++;
    }
  *snr = Q > 0.0 ? P / sqrt(Q) : 0.0;
  *flux = Q > 0.0 ? P / Q : 0.0;
  *n_kept = c;
}

/* ------------------------------------------------------------------------
 * Per-image noise by an iterated median absolute deviation (Sec. 3: the
 * pixel noise variance of each image comes from an iterative MAD).  Reading:
 * S = the finite pixels; repeat at most max_iter times:
 *   m = median(S), MAD = median{|x - m| : x in S}, sigma = 1.4826 MAD,
 *   S' = {finite x : |x - m| <= kappa sigma}; stop when S' == S, else S = S'.
 * The median of an even count is the mean of the two middle values.  The
 * result is the sigma of the last computed step, the size of the set it came
 * from, and the number of steps.  An image with no finite pixel gives NaN.
 * ------------------------------------------------------------------------ */
static double or_median(double *v, int64_t n) {
  qsort(v, (size_t)n, sizeof(double), or_cmp_dbl);
  return 0.5 * (v[(n - 1) / 2] + v[n / 2]);
}

void or_mad_noise(int64_t n, const float *x, double kappa, int max_iter, double *sigma_out, int64_t *n_used,
                  int32_t *iters) {
  uint8_t *kept = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  double *buf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    kept[i] = isfinite(x[i]) ? 1 : 0;
    cnt += kept[i];
  }
  double sigma = NAN;
  int64_t used = 0;
  int it = 0;
  while (it < max_iter && cnt > 0) {
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
      if (kept[i]) buf[m++] = (double)x[i];
    double med = or_median(buf, m);
    m = 0;
    for (int64_t i = 0; i < n; ++i)
      if (kept[i]) buf[m++] = fabs((double)x[i] - med);
    double mad = or_median(buf, m);
    sigma = 1.4826 * mad;
    used = m;
    it++;
    double thr = kappa * sigma;
    int changed = 0;
    int64_t c2 = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (!isfinite(x[i])) continue;
      uint8_t k = fabs((double)x[i] - med) <= thr;
      if (k != kept[i]) {
        kept[i] = k;
        changed = 1;
      }
      c2 += k;
    }
    cnt = c2;
    if (!changed) break;
  }
  *sigma_out = sigma;
  *n_used = used;
  *iters = it;
  free(kept);
  free(buf);
}
