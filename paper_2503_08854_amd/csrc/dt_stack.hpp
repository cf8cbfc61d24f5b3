// dt_stack.hpp -- one orbit of the fused plain stack, shared by the
// per-patch kernel, the debug kernel and the batched persistent kernel.
//
// Sec. 3 / Algorithm 1: SearchImages tests every (image, orbit) pair,
// FilterGPUIntersections keeps those inside an image, FindLocalSignal applies
// the matched filter there, and the per-image signals are combined assuming a
// constant flux: Psi = sum psi, Phi = sum phi, S/N = Psi / sqrt(Phi),
// flux = Psi / Phi.
#pragma once
#include "dt_orbit.hpp"

namespace dtk {

template <bool DEBUG>
__device__ __forceinline__ void stack_orbit(const StackArgs& A, int64_t o, const DebugArgs* dbg, int64_t row,
                                            float& snr_out, float& flux_out, int& nv_out) {
  const double a = A.a[o], e = A.e[o], inc = A.inc[o], node = A.node[o], peri = A.peri[o], m0 = A.m0[o];
  if (!orbit_ok(a, e, inc, node, peri, m0)) {
    snr_out = flux_out = __builtin_nanf("");
    nv_out = -1;
    if (DEBUG) {
      for (int ex = 0; ex < A.n_exp; ++ex) {
        int64_t q = row * A.n_exp + A.meta[ex].src;
        if (dbg->flags) dbg->flags[q] = 0;
      }
    }
    return;
  }
  Orbit ob;
  orbit_prep(a, e, inc, node, peri, m0, ob);
  KepState k;
  k.have = false;
  k.since_anchor = 0;
  LtState lt;
  lt.tau = lt.rate = 0.0;
  lt.n = 0;
  Kahan ps, ph;
  ps.init();
  ph.init();
  int nv = 0;
  // The gather of exposure ex is issued when its pixel is known and consumed
  // after the next exposure's propagation, so its latency hides behind FP64
  // work; the accumulation order stays the epoch order.
  float2 pend = make_float2(0.f, 0.f);
  bool have_pend = false;
  for (int ex = 0; ex < A.n_exp; ++ex) {
    const ExpMeta& x = A.meta[ex];
    SampleOut so;
    sample(ob, k, lt, x, A.epoch, x.gap, x.inv_gap, so);
    if (!DEBUG && have_pend && pend.y > 0.f) {
      ps.add(pend.x);
      ph.add(pend.y);
      nv++;
    }
    float2 v = make_float2(0.f, 0.f);
    bool valid = false;
    have_pend = so.inside;
    if (so.inside) {
      v = A.planes[x.plane_off + (int64_t)so.iy * x.W + so.ix];
      valid = v.y > 0.f;
      if (DEBUG && valid) {
        ps.add(v.x);
        ph.add(v.y);
        nv++;
      }
    }
    pend = v;
    if (DEBUG) {
      int64_t q = row * A.n_exp + x.src;
      if (dbg->px) dbg->px[q] = so.px;
      if (dbg->py) dbg->py[q] = so.py;
      if (dbg->ix) dbg->ix[q] = so.ix;
      if (dbg->iy) dbg->iy[q] = so.iy;
      if (dbg->tau) dbg->tau[q] = so.tau;
      if (dbg->flags) dbg->flags[q] = (so.front ? 1 : 0) | (so.inside ? 2 : 0) | (valid ? 4 : 0);
      if (dbg->psi) dbg->psi[q] = valid ? v.x : 0.f;
      if (dbg->phi) dbg->phi[q] = valid ? v.y : 0.f;
    }
  }
  if (!DEBUG && have_pend && pend.y > 0.f) {
    ps.add(pend.x);
    ph.add(pend.y);
    nv++;
  }
  const float Psi = ps.s - ps.c, Phi = ph.s - ph.c;
  snr_out = Phi > 0.f ? Psi / sqrtf(Phi) : 0.f;
  flux_out = Phi > 0.f ? Psi / Phi : 0.f;
  nv_out = nv;
}

}  // namespace dtk
