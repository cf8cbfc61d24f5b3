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
#include "dt_track.hpp"

namespace dtk {

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

// The same stack by checkpoint prediction (one wavefront = 64 orbits walking
// together; used when the patch has a finite observer speed bound).
__global__ __launch_bounds__(256, 4) void k_stack_track(StackArgs A) {
  __shared__ TrackQueue tq[4];
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o - (int64_t)__lane_id() >= A.n) return;  // the whole wavefront is past the end
  const bool in = o < A.n;
  double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (in) {
    el[0] = A.a[o]; el[1] = A.e[o]; el[2] = A.inc[o]; el[3] = A.node[o]; el[4] = A.peri[o]; el[5] = A.m0[o];
  }
  float snr, flux;
  int nv;
  track_stack_lane(A, el, in && orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]), tq[threadIdx.x >> 6], snr,
                   flux, nv);
  if (!in) return;
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

__global__ __launch_bounds__(64) void k_stack_debug(StackArgs A, DebugArgs D) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.m) return;
  const int64_t o = D.ids[r];
  if (o < 0 || o >= A.n) {
    for (int ex = 0; ex < A.n_exp; ++ex) {
      if (D.flags) D.flags[r * A.n_exp + ex] = 0;
      if (D.off) D.off[(int64_t)ex * D.m + r] = ~0u;
    }
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

// The stack's gather stream without its arithmetic: lane i visits the
// recorded plane offsets of orbit i in epoch order and sums what it loads
// exactly as k_stack does.  A yardstick for the achievable gather rate.
__global__ __launch_bounds__(256) void k_gather_replay(const float2* __restrict__ planes,
                                                       const uint32_t* __restrict__ off, int64_t m, int n_exp,
                                                       float* __restrict__ snr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  Kahan ps, ph;
  ps.init();
  ph.init();
  for (int ex = 0; ex < n_exp; ++ex) {
    const uint32_t o = off[(int64_t)ex * m + i];
    if (o != ~0u) {
      const float2 v = planes[o];
      if (v.y > 0.f) {
        ps.add(v.x);
        ph.add(v.y);
      }
    }
  }
  const float Psi = ps.s - ps.c, Phi = ph.s - ph.c;
  snr[i] = Phi > 0.f ? Psi / sqrtf(Phi) : 0.f;
}

static inline unsigned int grid_for(int64_t n, int bs) { return (unsigned int)((n + bs - 1) / bs); }

hipError_t launch_gather_replay(const float2* planes, const uint32_t* off, int64_t m, int n_exp, float* snr,
                                hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_replay, dim3(grid_for(m, 256)), dim3(256), 0, s, planes, off, m, n_exp, snr);
  return hipGetLastError();
}

hipError_t launch_stack(const StackArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.vobs < __builtin_inf())
    hipLaunchKernelGGL(k_stack_track, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a);
  else
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
