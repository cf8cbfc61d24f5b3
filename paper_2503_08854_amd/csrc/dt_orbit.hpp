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
//     rotations (Taylor series whose truncation is below 1e-20) and
//     re-anchored with a full sincos every ANCHOR exposures, so no
//     transcendental function is evaluated per sample.
//   * The light time tau solves c tau = |r(t - tau) - r_obs|.  It is predicted
//     by linear extrapolation of the previous exposures' light times; the
//     orbit is solved at t - tau_pred and one Newton step on
//     F(D) = c (tau_pred + D) - |rho - D v| gives the remaining correction D,
//     applied to the position as rho - D v.  The neglected terms are
//     O(D^2 |acc|) in position and O(D^2 |v|^2 / (c |rho|)) in tau; D is kept
//     below LT_LINEAR_MAX = 1e-6 day (else the orbit is re-solved at the
//     corrected epoch), which bounds them below 1e-15 AU.
// The common case (small steps) runs straight-line code; the general paths
// (cold start, long rotations, light-time re-solves) are taken per lane only
// when a bound above is not met, and their loops stay rolled so the loop over
// exposures stays small.
#pragma once
#include "dt_common.hpp"

namespace dtk {

constexpr int ANCHOR = 32;                 // exposures between full sincos re-anchors
constexpr double LT_LINEAR_MAX = 1.0e-6;   // days; larger light-time corrections re-solve Kepler
constexpr double ROT_SHORT = 0.005;        // rad; |d| <= this uses the short series
constexpr double ROT_MAX = 0.05;           // rad; larger steps take the full-sincos path

// Reciprocal from the hardware estimate refined once by Newton-Raphson
// (relative error ~ the square of the estimate's, < 1e-13).
__device__ __forceinline__ double rcp1(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
// Two refinements: within ~1 ulp for normal, well-scaled arguments.
__device__ __forceinline__ double rcp2(double x) {
  double r = rcp1(x);
  double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
// sqrt(x) and 1/sqrt(x) for normal positive x (within ~1 ulp): one
// Goldschmidt iteration from the hardware estimate and a final residual
// correction.
__device__ __forceinline__ void sqrt_rsq(double x, double& s, double& rs) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * y;
  double g = x * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, g, x);
  s = fma(r, h, g);
  rs = 2.0 * h;
}

// Per-orbit constants ("orbit preparation"): with P the unit vector to
// perihelion and Q the one 90 deg ahead in the orbit plane (ecliptic),
// r(E) = (cos E - e) aP + sin E bQ and v(E) = n g (-sin E aP + cos E bQ),
// g = 1 / (1 - e cos E).
struct Orbit {
  double e, n, m0, he;          // eccentricity, mean motion k a^-3/2, M0, -e/2
  double aP0, aP1, aP2;         // a P
  double bQ0, bQ1, bQ2;         // b Q, b = a sqrt(1 - e^2)
  double mq;                    // bound on (1 + 0.1) |D v| for any |D0| <= LT_LINEAR_MAX (AU)
};

struct KepState {
  double E, sE, cE, M;  // E solves E - e sin E = M; (sE, cE) ~ (sin E, cos E)
  double g;             // 1 / (1 - e cE) at the solution
};

__device__ __forceinline__ bool orbit_ok(double a, double e, double inc, double node, double peri, double m0) {
  bool fin = __builtin_isfinite(a) && __builtin_isfinite(e) && __builtin_isfinite(inc) &&
             __builtin_isfinite(node) && __builtin_isfinite(peri) && __builtin_isfinite(m0);
  return fin && a > 0.0 && e >= 0.0 && e < 1.0;
}

__device__ __forceinline__ void orbit_prep(double a, double e, double inc, double node, double peri, double m0,
                                           Orbit& o) {
  double si, ci, sO, cO, sw, cw;
  sincos(inc, &si, &ci);
  sincos(node, &sO, &cO);
  sincos(peri, &sw, &cw);
  const double P0 = cO * cw - sO * sw * ci, P1 = sO * cw + cO * sw * ci, P2 = sw * si;
  const double Q0 = -cO * sw - sO * cw * ci, Q1 = -sO * sw + cO * cw * ci, Q2 = cw * si;
  const double b = a * sqrt((1.0 - e) * (1.0 + e));
  o.e = e;
  o.n = K_GAUSS / (a * sqrt(a));
  o.m0 = m0;
  o.he = -0.5 * e;
  o.aP0 = a * P0;
  o.aP1 = a * P1;
  o.aP2 = a * P2;
  o.bQ0 = b * Q0;
  o.bQ1 = b * Q1;
  o.bQ2 = b * Q2;
  // |v| <= n a sqrt((1 + e) / (1 - e)) (the perihelion speed); the applied
  // correction D = D0 (1 - rv / c) obeys |D| <= |D0| (1 + vmax / c)
  const double vmax = o.n * a * sqrt((1.0 + e) / (1.0 - e));
  o.mq = 1.1002 * LT_LINEAR_MAX * vmax * (1.0 + vmax * (1.0 / C_AU_DAY));
}

// Rotate (sE, cE) by d: sin d and cos d - 1 from their Taylor series.
// Short form for |d| <= ROT_SHORT (truncation < 2e-20), long form for
// |d| <= ROT_MAX (< 1e-22).
__device__ __forceinline__ void rot_apply(KepState& k, double s, double cm1, double d) {
  const double sE = fma(k.cE, s, fma(k.sE, cm1, k.sE));
  const double cE = fma(-k.sE, s, fma(k.cE, cm1, k.cE));
  k.sE = sE;
  k.cE = cE;
  k.E += d;
}
__device__ __forceinline__ void rot_short(KepState& k, double d) {
  const double d2 = d * d;
  const double s = fma(d * d2, fma(d2, 1.0 / 120.0, -1.0 / 6.0), d);
  const double cm1 = d2 * fma(d2, fma(d2, -1.0 / 720.0, 1.0 / 24.0), -0.5);
  rot_apply(k, s, cm1, d);
}
__device__ __forceinline__ void rot_long(KepState& k, double d) {
  const double d2 = d * d;
  const double s =
      fma(d * d2,
          fma(d2, fma(d2, fma(d2, fma(d2, -1.0 / 39916800.0, 1.0 / 362880.0), -1.0 / 5040.0), 1.0 / 120.0),
              -1.0 / 6.0),
          d);
  const double cm1 =
      d2 * fma(d2, fma(d2, fma(d2, fma(d2, -1.0 / 3628800.0, 1.0 / 40320.0), -1.0 / 720.0), 1.0 / 24.0), -0.5);
  rot_apply(k, s, cm1, d);
}
// Tiny step (|d| < 1e-8): sin d = d to < 2e-25; cos d - 1 = -d^2/2 < 5e-17 is
// dropped (below 1/4 ulp of 1; re-anchoring bounds its accumulation).
__device__ __forceinline__ void rot_tiny(KepState& k, double d) {
  const double sE = fma(k.cE, d, k.sE);
  const double cE = fma(-k.sE, d, k.cE);
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
#pragma unroll 1
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
  k.g = rcp2(fma(-e, c, 1.0));
}

// General solve: cold start when `cold`, else warm from the previous solution
// for a start step up to `reach` (larger steps restart cold); the step is
// taken by a full sincos with `anchor`, else by the rotation series (in equal
// parts of at most ROT_MAX).
__device__ inline void kepler_general(double M, double e, KepState& k, bool anchor, bool cold,
                                      double reach = ROT_MAX) {
  double d = 0.0;
  if (!cold) {
    d = (M - k.M) * k.g;
    d = fma(-0.5 * e * k.sE * k.g, d * d, d);  // E''(M) = -e sin E g^3
  }
  if (cold || !(fabs(d) <= reach)) {
    kepler_cold(M, e, k);
    return;
  }
  if (anchor) {
    k.E += d;
    sincos(k.E, &k.sE, &k.cE);
  } else if (fabs(d) <= ROT_MAX) {
    rot_long(k, d);
  } else {
    const int parts = (int)ceil(fabs(d) * (1.0 / ROT_MAX));
    const double dp = d / parts;
#pragma unroll 1
    for (int i = 0; i < parts; ++i) rot_long(k, dp);
  }
#pragma unroll 1
  for (int it = 0; it < 8; ++it) {
    k.g = rcp1(fma(-e, k.cE, 1.0));
    double dd = -fma(-e, k.sE, k.E - M) * k.g;
    if (fabs(dd) < 1e-8) {
      // quadratic convergence: the next step would be < e dd^2 / (1 - e) < 1e-16
      rot_tiny(k, dd);
      break;
    }
    rot_long(k, dd);
  }
  k.M = M;
}

// Warm solve, common case: returns false with the state untouched when a
// re-anchor is due or the step exceeds the short series; otherwise solves
// (one Newton step normally suffices, more are taken if not).
__device__ __forceinline__ bool kepler_warm(double M, double he, double e, KepState& k, bool anchor) {
  double d = (M - k.M) * k.g;
  d = fma(he * k.sE * k.g, d * d, d);
  if (anchor || !(fabs(d) <= ROT_SHORT)) return false;
  rot_short(k, d);
  // the raw reciprocal estimate (relative error ~1e-7) suffices here: it
  // scales a Newton step that is itself below 1e-8 rad, and the next start
  double g = __builtin_amdgcn_rcp(fma(-e, k.cE, 1.0));
  double dd = -fma(-e, k.sE, k.E - M) * g;
  k.g = g;
  if (!(fabs(dd) < 1e-8)) {  // rare: the start was poor, take more Newton steps
#pragma unroll 1
    for (int it = 1; it < 8; ++it) {
      rot_long(k, dd);
      g = rcp1(fma(-e, k.cE, 1.0));
      dd = -fma(-e, k.sE, k.E - M) * g;
      k.g = g;
      if (fabs(dd) < 1e-8) break;
    }
    if (!(fabs(dd) < 1e-8)) {
      rot_long(k, dd);
      dd = 0.0;
    }
  }
  rot_tiny(k, dd);
  k.M = M;
  return true;
}

struct SampleOut {
  double px, py, tau;
  int ix, iy;
  bool front, inside;
  bool solved;  // the full path ran (light-time correction and projection)
};

// Light-time history carried across exposures: last light time and its rate.
struct LtState {
  double tau, rate;
};

// Heliocentric state at t - tg and the one-step light-time correction D.
struct LtSolve {
  double rho0, rho1, rho2, d2, rdist, dist0, dist, v0, v1, v2, D;
};

constexpr double IC = 1.0 / C_AU_DAY;  // days per AU of light travel

// Relative error bound used for the raw hardware estimates of 1/sqrt(x) and
// sqrt(x) = x rsq(x): twice the documented 2^29 ulp (~1.2e-7).
constexpr double RSQ_REL = 2.5e-7;

// rho = r(t - tg) - r_obs given -r_obs = (b0, b1, b2), and |rho| from the raw
// estimate (dist0, relative error below RSQ_REL).
__device__ __forceinline__ void lt_pos(const Orbit& o, const KepState& k, double b0, double b1, double b2,
                                       LtSolve& s) {
  const double cme = k.cE - o.e;
  s.rho0 = fma(cme, o.aP0, fma(k.sE, o.bQ0, b0));
  s.rho1 = fma(cme, o.aP1, fma(k.sE, o.bQ1, b1));
  s.rho2 = fma(cme, o.aP2, fma(k.sE, o.bQ2, b2));
  s.d2 = fma(s.rho0, s.rho0, fma(s.rho1, s.rho1, s.rho2 * s.rho2));
  s.rdist = __builtin_amdgcn_rsq(s.d2);
  s.dist0 = s.d2 * s.rdist;
}
// dist to full precision by one Newton correction of x rsq(x); the raw rdist
// only scales rv, where a relative error of 1e-5 changes D by less than 1e-7
// relative.
__device__ __forceinline__ void lt_refine(LtSolve& s) {
  s.dist = fma(fma(-s.dist0, s.dist0, s.d2), 0.5 * s.rdist, s.dist0);
}

// v = dr/dt and the Newton step on F(D) = c (tg + D) - |rho - D v| from D = 0,
// with 1 / (c + rv) = (1 / c) (1 - rv / c) to a relative (rv / c)^2 < 1e-7.
__device__ __forceinline__ void lt_vel(const Orbit& o, const KepState& k, double tg, LtSolve& s) {
  const double ng = o.n * k.g;
  const double vs = -ng * k.sE, vc = ng * k.cE;
  s.v0 = fma(vc, o.bQ0, vs * o.aP0);
  s.v1 = fma(vc, o.bQ1, vs * o.aP1);
  s.v2 = fma(vc, o.bQ2, vs * o.aP2);
  const double rv = fma(s.rho0, s.v0, fma(s.rho1, s.v1, s.rho2 * s.v2)) * s.rdist;
  s.D = fma(s.dist, IC, -tg) * fma(-rv, IC, 1.0);
}

__device__ __forceinline__ void lt_state(const Orbit& o, const KepState& k, double b0, double b1, double b2,
                                         double tg, LtSolve& s) {
  lt_pos(o, k, b0, b1, b2, s);
  lt_refine(s);
  lt_vel(o, k, tg, s);
}

// Corrected position q = rho - D v projected through the exposure's TAN WCS:
// p = CRPIX - 1 + (A . q) / (c . q), then the nearest pixel and the image test.
__device__ __forceinline__ void project(const ExpMeta& x, const LtSolve& s, SampleOut& out) {
  const double D = s.D;
  const double q0 = fma(-D, s.v0, s.rho0), q1 = fma(-D, s.v1, s.rho1), q2 = fma(-D, s.v2, s.rho2);
  const double w = fma(x.cx, q0, fma(x.cy, q1, x.cz * q2));
  const double iw = rcp1(w);
  out.px = fma(fma(x.a0x, q0, fma(x.a0y, q1, x.a0z * q2)), iw, x.px0);
  out.py = fma(fma(x.a1x, q0, fma(x.a1y, q1, x.a1z * q2)), iw, x.py0);
  out.front = (w > 0.0) && (s.dist >= 1e-9);
  // nearest pixel floor(p + 0.5), clamped into int range before conversion
  const double fx = floor(out.px + 0.5), fy = floor(out.py + 0.5);
  out.ix = (int)fmin(fmax(fx, -2147483648.0), 2147483647.0);
  out.iy = (int)fmin(fmax(fy, -2147483648.0), 2147483647.0);
  out.inside = out.front && (unsigned)out.ix < (unsigned)x.W && (unsigned)out.iy < (unsigned)x.H;
}

// One (orbit, exposure) sample.  FIRST: the orbit's first exposure (cold
// Kepler start, no light-time history).  Otherwise `gap` is t_e minus the
// previous exposure's epoch and inv_gap its reciprocal (0 when gap == 0);
// `anchor` re-anchors sin E, cos E with a full sincos.
//
// EXACT = false (walks that only use `inside`) first tests the uncorrected
// position rho against the exposure's sky cone.  The exact position is
// rho - D v with |D| <= |D0| (1 + vmax / c), D0 = |rho| / c - tg, so when
// |D0| <= LT_LINEAR_MAX (tested on the raw distance with the slack of its
// error bound) it lies within |D v| of rho; moving a point by d
// changes its distance from the cone axis by at most d and its projection on
// the axis by at most d.  A point that can land in the image therefore obeys
// perp(rho) <= tan(theta) (u . rho) + (1 + tan theta) |D v| <= tan(theta) (u . rho) + mq.
// Samples that fail this test keep the Kepler and light-time history (the
// light time is taken as tg + D0) and report inside = front = false; their
// px, py, ix, iy are not computed.  All others, and every sample of an
// EXACT walk, take the full path below.
template <bool FIRST, bool EXACT>
__device__ __forceinline__ void sample(const Orbit& o, KepState& k, LtState& lt, const ExpMeta& x, double epoch,
                                       double gap, double inv_gap, bool anchor, SampleOut& out) {
  const double dt = x.t - epoch;
  double tg = FIRST ? 0.0 : fma(lt.rate, gap, lt.tau);
  const double b0 = -x.ox, b1 = -x.oy, b2 = -x.oz;
  LtSolve s;
  // common path straight-line: warm Kepler step, position, light-time estimate
  double M = fma(o.n, dt - tg, o.m0);
  if (FIRST || !kepler_warm(M, o.he, o.e, k, anchor)) kepler_general(M, o.e, k, !FIRST && anchor, FIRST);
  lt_pos(o, k, b0, b1, b2, s);
  const double D0 = fma(s.dist0, IC, -tg);
  bool full = EXACT || FIRST;
  if (!full) {
    // evaluated without branches (bitwise, not short-circuit, logic)
    const double sc = fma(x.ux, s.rho0, fma(x.uy, s.rho1, x.uz * s.rho2));
    const double R = fma(x.cone_tan, sc, o.mq);
    full = !(fma(s.dist0, RSQ_REL * IC, fabs(D0)) <= LT_LINEAR_MAX) |
           ((R >= 0.0) & (fma(-R, R, fma(-sc, sc, s.d2)) <= x.cone_lim));
  }
  double tau;
  if (full) {
    lt_refine(s);
    lt_vel(o, k, tg, s);
    if (!(fabs(s.D) <= LT_LINEAR_MAX)) {
      // poor prediction: solve the orbit again at the corrected epoch (at most 3 times)
#pragma unroll 1
      for (int pass = 1; pass <= 3; ++pass) {
        tg += s.D;
        M = fma(o.n, dt - tg, o.m0);
        kepler_general(M, o.e, k, false, false);
        lt_state(o, k, b0, b1, b2, tg, s);
        if (fabs(s.D) <= LT_LINEAR_MAX) break;
      }
    }
    tau = tg + s.D;
    project(x, s, out);
  } else {
    tau = tg + D0;
    out.front = out.inside = false;
  }
  out.solved = full;
  lt.rate = FIRST ? 0.0 : (tau - lt.tau) * inv_gap;
  lt.tau = tau;
  out.tau = tau;
}

// The walk over one orbit's exposures in epoch order: calls f(ex, out) for
// every exposure after its sample (EXACT: see sample()).
template <bool EXACT, typename F>
__device__ __forceinline__ void walk_orbit(const Orbit& o, const ExpMeta* __restrict__ meta, int n_exp, double epoch,
                                           F&& f) {
  KepState k;
  LtState lt;
  lt.tau = lt.rate = 0.0;
  for (int ex = 0; ex < n_exp; ++ex) {
    const ExpMeta& x = meta[ex];
    SampleOut so;
    if (ex == 0)
      sample<true, EXACT>(o, k, lt, x, epoch, 0.0, 0.0, false, so);
    else
      sample<false, EXACT>(o, k, lt, x, epoch, x.gap, x.inv_gap, (ex % ANCHOR) == 0, so);
    f(ex, so);
  }
}

// FP32 Kahan summation (precision scheme: FP32 gathers, compensated FP32
// accumulation): the sum is s - c.
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
