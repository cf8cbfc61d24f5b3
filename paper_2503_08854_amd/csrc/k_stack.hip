// k_stack.hip -- the fused plain stack: per orbit, per exposure in epoch
// order, propagate (FP64) -> project (FP64) -> nearest pixel -> validity ->
// gather the matched-filter planes (FP32) -> Kahan-accumulate (FP32).
//
// Sec. 3 / Algorithm 1: SearchImages tests every (image, orbit) pair,
// FilterGPUIntersections keeps those inside an image, FindLocalSignal applies
// the matched filter there, and the per-image signals are combined assuming a
// constant flux: Psi = sum psi, Phi = sum phi, S/N = Psi / sqrt(Phi),
// flux = Psi / Phi.  Here the intersection list is never materialised: the
// validity predicate and the gather run in registers of the lane that owns
// the orbit, and only 12 bytes per orbit leave the kernel.
//
// Layout: one lane per orbit (orbit-major, coalesced SoA element loads),
// exposure metadata read with wave-uniform (scalar) loads, planes as
// interleaved float2 {psi, phi} so a valid sample costs one 8-byte gather.
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
  double tau = 0.0;
  bool have_tau = false;
  Kahan ps, ph;
  ps.init();
  ph.init();
  int nv = 0;
  for (int ex = 0; ex < A.n_exp; ++ex) {
    const ExpMeta& x = A.meta[ex];
    SampleOut so;
    sample(ob, k, tau, have_tau, x, A.epoch, so);
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
  const float Psi = ps.s - ps.c, Phi = ph.s - ph.c;
  snr_out = Phi > 0.f ? Psi / sqrtf(Phi) : 0.f;
  flux_out = Phi > 0.f ? Psi / Phi : 0.f;
  nv_out = nv;
}

__global__ __launch_bounds__(256) void k_stack(StackArgs A) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= A.n) return;
  float snr, flux;
  int nv;
  stack_orbit<false>(A, o, nullptr, 0, snr, flux, nv);
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

__global__ __launch_bounds__(64) void k_stack_debug(StackArgs A, DebugArgs D) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.m) return;
  const int64_t o = D.ids[r];
  if (o < 0 || o >= A.n) {
    for (int ex = 0; ex < A.n_exp; ++ex)
      if (D.flags) D.flags[r * A.n_exp + ex] = 0;
    return;
  }
  float snr, flux;
  int nv;
  stack_orbit<true>(A, o, &D, r, snr, flux, nv);
}

__global__ __launch_bounds__(256) void k_validate(StackArgs A, unsigned long long* bad) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= A.n) return;
  if (!orbit_ok(A.a[o], A.e[o], A.inc[o], A.node[o], A.peri[o], A.m0[o])) atomicAdd(bad, 1ull);
}

static inline unsigned int grid_for(int64_t n, int bs) { return (unsigned int)((n + bs - 1) / bs); }

hipError_t launch_stack(const StackArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stack, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_debug(const StackArgs& a, const DebugArgs& d, hipStream_t s) {
  if (d.m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stack_debug, dim3(grid_for(d.m, 64)), dim3(64), 0, s, a, d);
  return hipGetLastError();
}

hipError_t launch_validate(const StackArgs& a, unsigned long long* d_bad, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a, d_bad);
  return hipGetLastError();
}

}  // namespace dtk
