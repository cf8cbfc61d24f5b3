// k_clip.hip -- per-intersection outlier trimming of candidate orbits
// (Sec. 5.2.3): an artifact in one image can carry a chance alignment above
// threshold; under the constant-flux model each valid intersection e is an
// independent flux estimate psi_e / phi_e of variance 1 / phi_e, so the
// residuals chi_e = (psi_e - F phi_e) / sqrt(phi_e) about the kept samples'
// fit F = sum psi / sum phi are standard normal.  Samples with |chi_e| >
// kappa are dropped and the fit repeated until the kept set is stable.
//
// Pass 1 (one lane per candidate) walks the candidate's exposures with the
// stack's device code and writes its (psi, phi) per exposure; pass 2 (one
// wavefront per candidate, each lane owning up to 8 exposures) iterates the
// clipping with FP64 wave reductions.
#include "dt_stack.hpp"

namespace dtk {

constexpr int CLIP_PER_LANE = 8;  // exposures per lane: n_exp <= 512

__global__ __launch_bounds__(256) void k_clip_samples(StackArgs A, const int64_t* __restrict__ ids, int64_t m,
                                                      float2* __restrict__ buf) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  float2* out = buf + r * A.n_exp;
  const int64_t o = ids[r];
  bool ok = o >= 0 && o < A.n;
  double a = 0, e = 0, inc = 0, node = 0, peri = 0, m0 = 0;
  if (ok) {
    a = A.a[o]; e = A.e[o]; inc = A.inc[o]; node = A.node[o]; peri = A.peri[o]; m0 = A.m0[o];
    ok = orbit_ok(a, e, inc, node, peri, m0);
  }
  if (!ok) {
    for (int ex = 0; ex < A.n_exp; ++ex) out[ex] = make_float2(0.f, 0.f);
    return;
  }
  Orbit ob;
  orbit_prep(a, e, inc, node, peri, m0, ob);
  walk_orbit(ob, A.meta, A.n_exp, A.epoch, [&](int ex, const SampleOut& so) {
    const ExpMeta& x = A.meta[ex];
    float2 v = make_float2(0.f, 0.f);
    if (so.inside) {
      v = A.planes[x.plane_off + (int64_t)so.iy * x.W + so.ix];
      if (!(v.y > 0.f)) v = make_float2(0.f, 0.f);
    }
    out[ex] = v;
  });
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(64) void k_clip_fit(const float2* __restrict__ buf, int n_exp, int64_t m,
                                                 double kappa, int max_iter, float* __restrict__ snr,
                                                 float* __restrict__ flux, int32_t* __restrict__ nkept) {
  const int64_t r = blockIdx.x;
  if (r >= m) return;
  const int lane = threadIdx.x;
  double ps[CLIP_PER_LANE], ph[CLIP_PER_LANE];
  bool kept[CLIP_PER_LANE];
#pragma unroll
  for (int q = 0; q < CLIP_PER_LANE; ++q) {
    const int ex = lane + 64 * q;
    float2 v = ex < n_exp ? buf[r * n_exp + ex] : make_float2(0.f, 0.f);
    ps[q] = v.x;
    ph[q] = v.y;
    kept[q] = v.y > 0.f;
  }
  for (int it = 0; it < max_iter; ++it) {
    double P = 0.0, F = 0.0;
#pragma unroll
    for (int q = 0; q < CLIP_PER_LANE; ++q)
      if (kept[q]) {
        P += ps[q];
        F += ph[q];
      }
    P = wave_sum_d(P);
    F = wave_sum_d(F);
    if (!(F > 0.0)) break;
    const double mu = P / F;
    bool changed = false;
#pragma unroll
    for (int q = 0; q < CLIP_PER_LANE; ++q) {
      if (!(ph[q] > 0.0)) continue;
      const bool k = fabs(ps[q] - mu * ph[q]) / sqrt(ph[q]) <= kappa;
      changed |= k != kept[q];
      kept[q] = k;
    }
    if (__ballot(changed) == 0ull) break;
  }
  double P = 0.0, F = 0.0;
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < CLIP_PER_LANE; ++q)
    if (kept[q]) {
      P += ps[q];
      F += ph[q];
      cnt++;
    }
  P = wave_sum_d(P);
  F = wave_sum_d(F);
  cnt = (int)wave_sum_d((double)cnt);
  if (lane == 0) {
    if (snr) snr[r] = F > 0.0 ? (float)(P / sqrt(F)) : 0.f;
    if (flux) flux[r] = F > 0.0 ? (float)(P / F) : 0.f;
    if (nkept) nkept[r] = cnt;
  }
}

hipError_t launch_clip(const StackArgs& a, const int64_t* d_ids, int64_t m, double kappa, int max_iter,
                       float2* d_buf, float* snr, float* flux, int32_t* nkept, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (a.n_exp > 64 * CLIP_PER_LANE) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_clip_samples, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, d_ids, m, d_buf);
  hipLaunchKernelGGL(k_clip_fit, dim3((unsigned)m), dim3(64), 0, s, d_buf, a.n_exp, m, kappa, max_iter, snr, flux,
                     nkept);
  return hipGetLastError();
}

}  // namespace dtk
