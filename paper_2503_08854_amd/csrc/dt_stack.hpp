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

// Debug table of the walk that ran (dt_debug_samples and its stack-walk
// variant): row `row`, column = the exposure's caller index.  flags: bit0 in
// front of the tangent plane, bit1 inside the image, bit2 valid (phi > 0),
// bit3 solved exactly by the walk; a sample the walk excluded by a bound
// keeps the row's initial values (rec_init_row).
__device__ __forceinline__ void rec_init_row(const DebugArgs& d, const ExpMeta* meta, int n_exp, int64_t row) {
  for (int ex = 0; ex < n_exp; ++ex) {
    const int64_t q = row * n_exp + meta[ex].src;
    if (d.px) d.px[q] = __builtin_nan("");
    if (d.py) d.py[q] = __builtin_nan("");
    if (d.ix) d.ix[q] = (int)0x80000000;
    if (d.iy) d.iy[q] = (int)0x80000000;
    if (d.tau) d.tau[q] = __builtin_nan("");
    if (d.flags) d.flags[q] = 0;
    if (d.psi) d.psi[q] = 0.f;
    if (d.phi) d.phi[q] = 0.f;
  }
}
__device__ __forceinline__ void rec_sample(const DebugArgs& d, int n_exp, int64_t row, const ExpMeta& x,
                                           const SampleOut& so, float2 v) {
  const int64_t q = row * n_exp + x.src;
  const bool f = so.front;
  const bool valid = so.inside && v.y > 0.f;
  if (d.px) d.px[q] = f ? so.px : __builtin_nan("");
  if (d.py) d.py[q] = f ? so.py : __builtin_nan("");
  if (d.ix) d.ix[q] = f ? so.ix : (int)0x80000000;
  if (d.iy) d.iy[q] = f ? so.iy : (int)0x80000000;
  if (d.tau) d.tau[q] = so.tau;
  if (d.flags) d.flags[q] = (f ? 1 : 0) | (so.inside ? 2 : 0) | (valid ? 4 : 0) | 8;
  if (d.psi) d.psi[q] = valid ? v.x : 0.f;
  if (d.phi) d.phi[q] = valid ? v.y : 0.f;
}

// {psi, phi} of one pixel, loaded with the non-temporal hint: the gathers of
// the per-sample walk are scattered over the planes and almost never reused,
// and a 16 GB random-gather probe ran 10 % faster with the hint.
__device__ __forceinline__ float2 gather_nt(const float2* __restrict__ planes, int64_t i) {
  const uint64_t v = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(planes) + i);
  return make_float2(__uint_as_float((uint32_t)v), __uint_as_float((uint32_t)(v >> 32)));
}

// Compensated sums of one prepared orbit over exposures [ex0, ex0 + cnt)
// (epoch order; REC: the debug table of the samples solved; n_full counts
// the samples that took the full path, in a register).  Each gather is accumulated one exposure
// later, still in epoch order, so its load latency overlaps the next sample's
// arithmetic (deeper deferral measured slower: the loads are conditional, so
// the wait before a use covers all of them).
struct StackPart {
  Kahan ps, ph;
  int nv;
};
template <bool REC = false>
__device__ __forceinline__ void stack_range(const StackArgs& A, const Orbit& ob, int ex0, int cnt, StackPart& P,
                                            const DebugArgs* dbg, int64_t row, int& n_full) {
  P.ps.init();
  P.ph.init();
  P.nv = 0;
  float2 pend = make_float2(0.f, 0.f);
  auto take = [&](float2 v) {
    if (v.y > 0.f) {
      P.ps.add(v.x);
      P.ph.add(v.y);
      P.nv++;
    }
  };
  walk_orbit<false>(ob, A.meta + ex0, cnt, A.epoch, [&](int i, const SampleOut& so) {
    const ExpMeta& x = A.meta[ex0 + i];
    take(pend);
    pend = so.inside ? gather_nt(A.planes, x.plane_off + (int64_t)so.iy * x.W + so.ix) : make_float2(0.f, 0.f);
    if (REC && so.solved) rec_sample(*dbg, A.n_exp, row, x, so, pend);
    n_full += so.solved ? 1 : 0;
  });
  take(pend);
}
template <bool REC = false>
__device__ __forceinline__ void stack_range(const StackArgs& A, const Orbit& ob, int ex0, int cnt, StackPart& P,
                                            const DebugArgs* dbg = nullptr, int64_t row = 0) {
  int n_full = 0;
  stack_range<REC>(A, ob, ex0, cnt, P, dbg, row, n_full);
}

// S/N = Psi / sqrt(Phi), flux = Psi / Phi (0 when Phi = 0).
__device__ __forceinline__ void stack_finish(const StackPart& P, float& snr_out, float& flux_out, int& nv_out) {
  const float Psi = P.ps.s - P.ps.c, Phi = P.ph.s - P.ph.c;
  snr_out = Phi > 0.f ? Psi / sqrtf(Phi) : 0.f;
  flux_out = Phi > 0.f ? Psi / Phi : 0.f;
  nv_out = P.nv;
}

__device__ __forceinline__ void stack_walk(const StackArgs& A, const Orbit& ob, float& snr_out, float& flux_out,
                                           int& nv_out) {
  StackPart P;
  stack_range(A, ob, 0, A.n_exp, P);
  stack_finish(P, snr_out, flux_out, nv_out);
}

// One orbit of the stack; DEBUG also fills the per-sample table of `dbg`
// (row `row`), walking every sample exactly.
template <bool DEBUG>
__device__ __forceinline__ void stack_orbit(const StackArgs& A, int64_t o, const DebugArgs* dbg, int64_t row,
                                            float& snr_out, float& flux_out, int& nv_out) {
  const double a = A.a[o], e = A.e[o], inc = A.inc[o], node = A.node[o], peri = A.peri[o], m0 = A.m0[o];
  if (!orbit_ok(a, e, inc, node, peri, m0)) {
    snr_out = flux_out = __builtin_nanf("");
    nv_out = -1;
    if (DEBUG) rec_init_row(*dbg, A.meta, A.n_exp, row);
    return;
  }
  Orbit ob;
  orbit_prep(a, e, inc, node, peri, m0, ob);
  if (!DEBUG) {
    stack_walk(A, ob, snr_out, flux_out, nv_out);
    return;
  }
  Kahan ps, ph;
  ps.init();
  ph.init();
  int nv = 0;
  walk_orbit<true>(ob, A.meta, A.n_exp, A.epoch, [&](int ex, const SampleOut& so) {
    const ExpMeta& x = A.meta[ex];
    float2 v = make_float2(0.f, 0.f);
    if (so.inside) {
      v = A.planes[x.plane_off + (int64_t)so.iy * x.W + so.ix];
      if (v.y > 0.f) {
        ps.add(v.x);
        ph.add(v.y);
        nv++;
      }
    }
    rec_sample(*dbg, A.n_exp, row, x, so, v);
  });
  const float Psi = ps.s - ps.c, Phi = ph.s - ph.c;
  snr_out = Phi > 0.f ? Psi / sqrtf(Phi) : 0.f;
  flux_out = Phi > 0.f ? Psi / Phi : 0.f;
  nv_out = nv;
}

}  // namespace dtk
