// k_clip.hip -- per-intersection outlier trimming of candidate orbits
// (Sec. 5.2.3): an artifact in one image can carry a chance alignment above
// threshold; under the constant-flux model each valid intersection e is an
// independent flux estimate f_e = psi_e / phi_e of variance 1 / phi_e, so the
// residuals chi_e = (psi_e - F phi_e) / sqrt(phi_e) about the expectation F
// are standard normal.  Iteration 1 takes F = median(f_e), so that one dominant
// artifact cannot set it; every later round takes the weighted mean
// F = sum psi / sum phi of the samples the previous round kept.  A round
// keeps the samples with |chi_e| <= kappa; it stops when a round keeps
// exactly the set it started from, or after max_iter rounds.
//
// Pass 1 (one lane per candidate) walks the candidate's exposures with the
// stack's device code and writes its (psi, phi) per exposure; pass 2 (one
// wavefront per candidate, each lane owning up to 8 exposures) finds the
// median by ranking in LDS and iterates the clipping with FP64 wave
// reductions.  The per-sample arithmetic is FP64 without contraction, as in
// the definition.
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
  walk_orbit<false>(ob, A.meta, A.n_exp, A.epoch, [&](int ex, const SampleOut& so) {
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
#pragma clang fp contract(off)
  const int64_t r = blockIdx.x;
  if (r >= m) return;
  const int lane = threadIdx.x;
  __shared__ double fl[64 * CLIP_PER_LANE];  // per-sample flux psi / phi
  __shared__ int vf[64 * CLIP_PER_LANE];     // sample valid (phi > 0)
  double ps[CLIP_PER_LANE], ph[CLIP_PER_LANE];
  bool valid[CLIP_PER_LANE], kept[CLIP_PER_LANE];
  int nv = 0;
#pragma unroll
  for (int q = 0; q < CLIP_PER_LANE; ++q) {
    const int ex = lane + 64 * q;
    float2 v = ex < n_exp ? buf[r * n_exp + ex] : make_float2(0.f, 0.f);
    ps[q] = v.x;
    ph[q] = v.y;
    valid[q] = v.y > 0.f;
    kept[q] = valid[q];
    nv += valid[q] ? 1 : 0;
    fl[ex] = valid[q] ? ps[q] / ph[q] : 0.0;
    vf[ex] = valid[q] ? 1 : 0;
  }
  __syncthreads();
  const int nvalid = (int)wave_sum_d((double)nv);
  // iteration 1 expectation: the median of the per-sample fluxes (ranks with
  // ties broken by exposure index; mean of the two middle values)
  const int lo = (nvalid - 1) / 2, hi = nvalid / 2;
  double vlo = 0.0, vhi = 0.0;
#pragma unroll
  for (int q = 0; q < CLIP_PER_LANE; ++q) {
    if (!valid[q]) continue;
    const int me = lane + 64 * q;
    const double f = fl[me];
    int rank = 0;
    for (int j = 0; j < n_exp; ++j) rank += (vf[j] && (fl[j] < f || (fl[j] == f && j < me))) ? 1 : 0;
    if (rank == lo) vlo = f;
    if (rank == hi) vhi = f;
  }
  // exactly one lane holds each middle value; the others add zeros
  double F = 0.5 * (wave_sum_d(vlo) + wave_sum_d(vhi));
  for (int it = 0; it < max_iter && nvalid > 0; ++it) {
    if (it > 0) {
      double P = 0.0, Q = 0.0;
#pragma unroll
      for (int q = 0; q < CLIP_PER_LANE; ++q)
        if (kept[q]) {
          P += ps[q];
          Q += ph[q];
        }
      F = wave_sum_d(P) / wave_sum_d(Q);
    }
    bool changed = false;
#pragma unroll
    for (int q = 0; q < CLIP_PER_LANE; ++q) {
      if (!valid[q]) continue;
      const bool k = fabs(ps[q] - F * ph[q]) / sqrt(ph[q]) <= kappa;
      changed |= k != kept[q];
      kept[q] = k;
    }
    if (it > 0 && __ballot(changed) == 0ull) break;
  }
  double P = 0.0, Q = 0.0;
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < CLIP_PER_LANE; ++q)
    if (kept[q]) {
      P += ps[q];
      Q += ph[q];
      cnt++;
    }
  P = wave_sum_d(P);
  Q = wave_sum_d(Q);
  cnt = (int)wave_sum_d((double)cnt);
  if (lane == 0) {
    if (snr) snr[r] = Q > 0.0 ? (float)(P / sqrt(Q)) : 0.f;
    if (flux) flux[r] = Q > 0.0 ? (float)(P / Q) : 0.f;
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
