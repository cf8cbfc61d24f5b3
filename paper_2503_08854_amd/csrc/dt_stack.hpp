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

#ifndef STACK_DEFER
#define STACK_DEFER 1
#endif

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
        if (dbg->off) dbg->off[(int64_t)ex * dbg->m + row] = ~0u;
      }
    }
    return;
  }
  Orbit ob;
  orbit_prep(a, e, inc, node, peri, m0, ob);
  Kahan ps, ph;
  ps.init();
  ph.init();
  int nv = 0;
  // Without the debug table a gather is accumulated STACK_DEFER exposures
  // later (still in epoch order), so its load latency overlaps the arithmetic
  // of the following samples.
  float2 pend[STACK_DEFER];
#pragma unroll
  for (int i = 0; i < STACK_DEFER; ++i) pend[i] = make_float2(0.f, 0.f);
  auto take = [&](float2 v) {
    if (v.y > 0.f) {
      ps.add(v.x);
      ph.add(v.y);
      nv++;
    }
  };
  walk_orbit<DEBUG>(ob, A.meta, A.n_exp, A.epoch, [&](int ex, const SampleOut& so) {
    const ExpMeta& x = A.meta[ex];
    if (!DEBUG) {
      take(pend[0]);
#pragma unroll
      for (int i = 0; i + 1 < STACK_DEFER; ++i) pend[i] = pend[i + 1];
      pend[STACK_DEFER - 1] =
          so.inside ? A.planes[x.plane_off + (int64_t)so.iy * x.W + so.ix] : make_float2(0.f, 0.f);
      return;
    }
    float2 v = make_float2(0.f, 0.f);
    bool valid = false;
    if (so.inside) {
      v = A.planes[x.plane_off + (int64_t)so.iy * x.W + so.ix];
      valid = v.y > 0.f;
      if (valid) {
        ps.add(v.x);
        ph.add(v.y);
        nv++;
      }
    }
    if (DEBUG) {
      const int64_t q = row * A.n_exp + x.src;
      const bool f = so.front;
      if (dbg->px) dbg->px[q] = f ? so.px : __builtin_nan("");
      if (dbg->py) dbg->py[q] = f ? so.py : __builtin_nan("");
      if (dbg->ix) dbg->ix[q] = f ? so.ix : (int)0x80000000;
      if (dbg->iy) dbg->iy[q] = f ? so.iy : (int)0x80000000;
      if (dbg->tau) dbg->tau[q] = so.tau;
      if (dbg->flags) dbg->flags[q] = (f ? 1 : 0) | (so.inside ? 2 : 0) | (valid ? 4 : 0);
      if (dbg->psi) dbg->psi[q] = valid ? v.x : 0.f;
      if (dbg->phi) dbg->phi[q] = valid ? v.y : 0.f;
      if (dbg->off)
        dbg->off[(int64_t)ex * dbg->m + row] = valid ? (uint32_t)(x.plane_off + (int64_t)so.iy * x.W + so.ix) : ~0u;
    }
  });
  if (!DEBUG) {
#pragma unroll
    for (int i = 0; i < STACK_DEFER; ++i) take(pend[i]);
  }
  const float Psi = ps.s - ps.c, Phi = ph.s - ph.c;
  snr_out = Phi > 0.f ? Psi / sqrtf(Phi) : 0.f;
  flux_out = Phi > 0.f ? Psi / Phi : 0.f;
  nv_out = nv;
}

}  // namespace dtk
