// dt_orbit.hpp -- per-sample device arithmetic of the stack: two-body
// propagation with light time, TAN projection, nearest pixel.
//
// Sec. 3: each candidate orbit is a Keplerian element set on an elliptical
// two-body orbit about the Sun; every (image, orbit) pair is tested by
// carrying the orbit to the image epoch and projecting it through the image's
// WCS.  Everything up to and including the nearest-pixel rounding is FP64, so
// the integer pixel agrees with an exact evaluation except within ~1e-9 px of
// a rounding boundary.
//
// Work per sample is kept low by carrying state from one exposure to the next
// (exposures are visited in epoch order):
//   * Kepler's equation is solved from the previous exposure's eccentric
//     anomaly: a second-order Taylor start in the mean-anomaly step, then
//     Newton steps; sin E and cos E are advanced by exact small-angle
//     rotations (series to O(d^11)) and re-anchored with a full sincos every
//     ANCHOR exposures, so no transcendental is evaluated per sample.
//   * Light time is solved by Newton's method on c (tau_g + D) = |rho(D)|,
//     starting from the previous exposure's light time tau_g, with
//     rho(D) = r(t - tau_g - D) - r_obs expanded to third order in D about the
//     Kepler solution at t - tau_g (velocity, acceleration -mu r/|r|^3 and its
//     time derivative).  When |D| exceeds LT_TAYLOR_MAX the orbit is re-solved
//     at the corrected epoch instead.
#pragma once
#include "dt_common.hpp"

namespace dtk {

constexpr int ANCHOR = 16;                 // exposures between full sincos re-anchors
constexpr double LT_TAYLOR_MAX = 2.0e-3;   // days; larger light-time steps re-solve Kepler
constexpr double ROT_MAX = 0.05;           // rad; larger steps take the full-sincos path

struct Orbit {
  double a, e, n, b, sq, m0;     // a, e, mean motion, b = a sqrt(1-e^2), sqrt(1-e^2), M0
  double P0, P1, P2, Q0, Q1, Q2; // perihelion and semi-latus directions (ecliptic)
};

struct KepState {
  double E, sE, cE, M;  // E solves E - e sin E = M; (sE, cE) ~ (sin E, cos E)
  int since_anchor;
  bool have;
};

__device__ __forceinline__ bool orbit_ok(double a, double e, double inc, double node, double peri, double m0) {
  bool fin = __builtin_isfinite(a) && __builtin_isfinite(e) && __builtin_isfinite(inc) &&
             __builtin_isfinite(node) && __builtin_isfinite(peri) && __builtin_isfinite(m0);
  return fin && a > 0.0 && e >= 0.0 && e < 1.0;
}

// Orbit preparation: mean motion n = k a^-3/2 and the in-plane basis
// P (to perihelion), Q (90 deg ahead) from (i, node, peri).
__device__ __forceinline__ void orbit_prep(double a, double e, double inc, double node, double peri, double m0,
                                           Orbit& o) {
  double si, ci, sO, cO, sw, cw;
  sincos(inc, &si, &ci);
  sincos(node, &sO, &cO);
  sincos(peri, &sw, &cw);
  o.a = a;
  o.e = e;
  o.n = K_GAUSS / (a * sqrt(a));
  o.sq = sqrt((1.0 - e) * (1.0 + e));
  o.b = a * o.sq;
  o.m0 = m0;
  o.P0 = cO * cw - sO * sw * ci;
  o.P1 = sO * cw + cO * sw * ci;
  o.P2 = sw * si;
  o.Q0 = -cO * sw - sO * cw * ci;
  o.Q1 = -sO * sw + cO * cw * ci;
  o.Q2 = cw * si;
}

// Rotate (sE, cE) by a small angle d (|d| <= ROT_MAX): sin d and cos d - 1
// from their Taylor series (truncation < 1e-22 at |d| = 0.05).
__device__ __forceinline__ void kep_rotate(KepState& k, double d) {
  double d2 = d * d;
  double s = d * (1.0 - d2 * (1.0 / 6.0) * (1.0 - d2 * (1.0 / 20.0) * (1.0 - d2 * (1.0 / 42.0) * (1.0 - d2 * (1.0 / 72.0)))));
  double cm1 = -0.5 * d2 * (1.0 - d2 * (1.0 / 12.0) * (1.0 - d2 * (1.0 / 30.0) * (1.0 - d2 * (1.0 / 56.0) * (1.0 - d2 * (1.0 / 90.0)))));
  double sE = fma(k.cE, s, fma(k.sE, cm1, k.sE));
  double cE = fma(-k.sE, s, fma(k.cE, cm1, k.cE));
  k.sE = sE;
  k.cE = cE;
  k.E += d;
}

// Cold solve: Newton with full sincos from E0 = M + 0.85 e sign(sin M), kept
// inside the root bracket [M - e, M + e] by bisection.
__device__ inline void kepler_cold(double M, double e, KepState& k) {
  const double twopi = 2.0 * PI;
  double Mr = M - twopi * rint(M / twopi);  // [-pi, pi]
  double off = M - Mr;
  double lo = Mr - e, hi = Mr + e;
  double E = Mr + 0.85 * e * (Mr > 0.0 ? 1.0 : (Mr < 0.0 ? -1.0 : 0.0));
  E = fmin(fmax(E, lo), hi);
  double s, c;
  for (int it = 0; it < 60; ++it) {
    sincos(E, &s, &c);
    double f = E - e * s - Mr;
    if (f == 0.0) break;
    if (f > 0.0) hi = E; else lo = E;
    double dE = -f / (1.0 - e * c);
    if (fabs(dE) <= 1e-15 * fmax(1.0, fabs(E))) {
      E += dE;
      sincos(E, &s, &c);
      break;
    }
    double En = E + dE;
    if (!(En > lo && En < hi)) En = 0.5 * (lo + hi);
    E = En;
  }
  k.E = E + off;
  k.sE = s;
  k.cE = c;
  k.M = M;
  k.since_anchor = 0;
  k.have = true;
}

// Warm solve from the previous solution (see the file comment).
__device__ inline void kepler_solve(double M, double e, KepState& k) {
  if (!k.have) {
    kepler_cold(M, e, k);
    return;
  }
  double dM = M - k.M;
  double g = 1.0 / (1.0 - e * k.cE);
  double d = dM * g;
  d = fma(-0.5 * e * k.sE * g, d * d, d);  // E''(M) = -e sin E g^3
  if (!(fabs(d) <= ROT_MAX)) {
    kepler_cold(M, e, k);
    return;
  }
  if (k.since_anchor >= ANCHOR) {
    k.E += d;
    sincos(k.E, &k.sE, &k.cE);
    k.since_anchor = 0;
  } else {
    kep_rotate(k, d);
  }
  for (int it = 0; it < 8; ++it) {
    double f = k.E - e * k.sE - M;
    double dd = -f / (1.0 - e * k.cE);
    kep_rotate(k, dd);
    // quadratic convergence: the next step would be < e dd^2 / (1 - e) < 1e-16
    if (fabs(dd) < 1e-8) break;
  }
  k.M = M;
  k.since_anchor++;
}

struct SampleOut {
  double px, py, tau;
  int ix, iy;
  bool front, inside;
};

// One (orbit, exposure) sample.  tau carries the previous light time (0 with
// have_tau == false) and returns this one.
__device__ inline void sample(const Orbit& o, KepState& k, double& tau, bool& have_tau, const ExpMeta& x,
                              double epoch, SampleOut& out) {
  const double dt = x.t - epoch;
  double tg = have_tau ? tau : 0.0;
  double rho0, rho1, rho2, D = 0.0;
  double v0, v1, v2, h0, h1, h2, j0, j1, j2, dist = 0.0;
  for (int pass = 0; pass < 3; ++pass) {
    kepler_solve(fma(o.n, dt - tg, o.m0), o.e, k);
    // state at t - tg
    const double X = o.a * (k.cE - o.e), Y = o.b * k.sE;
    const double r0 = X * o.P0 + Y * o.Q0, r1 = X * o.P1 + Y * o.Q1, r2 = X * o.P2 + Y * o.Q2;
    const double ir = 1.0 / (o.a * (1.0 - o.e * k.cE));       // 1/|r|
    const double vf = o.n * o.a * o.a * ir;                    // sqrt(mu a)/|r|
    const double vs = -vf * k.sE, vc = vf * o.sq * k.cE;
    v0 = vs * o.P0 + vc * o.Q0;
    v1 = vs * o.P1 + vc * o.Q1;
    v2 = vs * o.P2 + vc * o.Q2;
    const double g3 = MU_SUN * ir * ir * ir;                  // mu/|r|^3
    const double rv3 = 3.0 * (r0 * v0 + r1 * v1 + r2 * v2) * ir * ir;
    // half acceleration and one sixth of its time derivative
    h0 = -0.5 * g3 * r0;
    h1 = -0.5 * g3 * r1;
    h2 = -0.5 * g3 * r2;
    j0 = -(g3 / 6.0) * (v0 - rv3 * r0);
    j1 = -(g3 / 6.0) * (v1 - rv3 * r1);
    j2 = -(g3 / 6.0) * (v2 - rv3 * r2);
    rho0 = r0 - x.ox;
    rho1 = r1 - x.oy;
    rho2 = r2 - x.oz;
    // Newton on F(D) = c (tg + D) - |rho(D)|, rho(D) = rho - D v + D^2 h - D^3 j
    const double d0 = sqrt(rho0 * rho0 + rho1 * rho1 + rho2 * rho2);
    const double iFp = 1.0 / (C_AU_DAY + (rho0 * v0 + rho1 * v1 + rho2 * v2) / d0);
    D = 0.0;
    dist = d0;
    for (int it = 0; it < 6; ++it) {
      double F = C_AU_DAY * (tg + D) - dist;
      double dD = -F * iFp;
      D += dD;
      double q0 = fma(D, fma(D, fma(-D, j0, h0), -v0), rho0);
      double q1 = fma(D, fma(D, fma(-D, j1, h1), -v1), rho1);
      double q2 = fma(D, fma(D, fma(-D, j2, h2), -v2), rho2);
      dist = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
      // chord-Newton: the next step is ~ (|v|^2/|rho|)/(2c) dD^2, < 1e-14 day
      // for |dD| < 1e-5 day down to 0.01 AU range
      if (fabs(dD) < 1e-5) break;
    }
    if (fabs(D) <= LT_TAYLOR_MAX || pass == 2) break;
    tg += D;  // large correction: re-solve Kepler at the corrected epoch
  }
  const double q0 = fma(D, fma(D, fma(-D, j0, h0), -v0), rho0);
  const double q1 = fma(D, fma(D, fma(-D, j1, h1), -v1), rho1);
  const double q2 = fma(D, fma(D, fma(-D, j2, h2), -v2), rho2);
  tau = tg + D;
  have_tau = true;
  out.tau = tau;
  // TAN projection: p = CRPIX - 1 + (A . rho) / (c . rho)
  const double w = x.cx * q0 + x.cy * q1 + x.cz * q2;
  out.front = (w > 0.0) && (dist >= 1e-9);
  out.inside = false;
  out.ix = out.iy = (int)0x80000000;
  out.px = out.py = __builtin_nan("");
  if (!out.front) return;
  const double iw = 1.0 / w;
  out.px = fma(x.a0x * q0 + x.a0y * q1 + x.a0z * q2, iw, x.px0);
  out.py = fma(x.a1x * q0 + x.a1y * q1 + x.a1z * q2, iw, x.py0);
  const double fx = floor(out.px + 0.5), fy = floor(out.py + 0.5);
  if (fx >= 0.0 && fx < (double)x.W && fy >= 0.0 && fy < (double)x.H) {
    out.ix = (int)fx;
    out.iy = (int)fy;
    out.inside = true;
  } else if (fabs(fx) < 2.0e9 && fabs(fy) < 2.0e9) {
    out.ix = (int)fx;
    out.iy = (int)fy;
  }
}

// FP32 Kahan summation (the benchmark spec precision scheme): sum ~ s - c.
struct Kahan {
  float s, c;
  __device__ __forceinline__ void init() { s = c = 0.f; }
  __device__ __forceinline__ void add(float x) {
    float y = x - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  // combine with another partial sum (fixed order: this + other)
  __device__ __forceinline__ void merge(float os, float oc) {
    c += oc;
    add(os);
  }
};

}  // namespace dtk
