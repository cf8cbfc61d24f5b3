// k_generate.hip -- GenerateOrbits of Algorithm 1 on the device: candidate
// orbits sampled from given distributions, as a pure function of (seed,
// orbit index), so every orbit of a dense grid is defined without a host
// upload and can be generated inside the stack itself.
//
// Sampling (this library's reading of "sample orbital parameters from
// specified distributions", Sec. 3): (a, e, i) uniform in their ranges; a
// line of sight uniform over a tangent-plane rectangle around a field
// centre; the orbit is placed so that its geometric heliocentric position at
// the epoch lies on that line of sight: with a true anomaly nu drawn uniform,
// the distance r = a (1 - e^2) / (1 + e cos nu) fixes the point where the
// line of sight meets the sphere |X| = r; the orbit plane through X with the
// drawn inclination (raised to |latitude| when needed, on a random nodal
// branch) gives the node and the argument of perihelion, and nu gives M0.
// Up to 16 attempts per index (counter-based draws); an index whose attempts
// all miss gets a = NaN, which the stack reports as outside the domain.
#include "dt_track.hpp"

namespace dtk {

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
// uniform in [0, 1) with 53 random bits, from (seed, index, attempt, draw)
__device__ __forceinline__ double u01(uint64_t seed, uint64_t idx, int att, int k) {
  const uint64_t h = mix64(seed ^ mix64(idx * 0x100000001B3ull + (uint64_t)(att * 16 + k)));
  return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

// Writes el[] only for an index that yields an orbit (returns true); the
// caller fills el[] for the other case (storing it on both exits kept el[] in
// scratch memory).
__device__ inline bool gen_orbit(const dt_orbit_sampler& S, uint64_t idx, double el[6]) {
  for (int att = 0; att < 16; ++att) {
    const double xi = (2.0 * u01(S.seed, idx, att, 0) - 1.0) * S.half_w;
    const double eta = (2.0 * u01(S.seed, idx, att, 1) - 1.0) * S.half_h;
    double d0 = S.center[0] + xi * S.east[0] + eta * S.north[0];
    double d1 = S.center[1] + xi * S.east[1] + eta * S.north[1];
    double d2 = S.center[2] + xi * S.east[2] + eta * S.north[2];
    const double dn = 1.0 / sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    d0 *= dn;
    d1 *= dn;
    d2 *= dn;
    const double a = S.a_range[0] + (S.a_range[1] - S.a_range[0]) * u01(S.seed, idx, att, 2);
    const double e = S.e_range[0] + (S.e_range[1] - S.e_range[0]) * u01(S.seed, idx, att, 3);
    double inc = S.inc_range[0] + (S.inc_range[1] - S.inc_range[0]) * u01(S.seed, idx, att, 4);
    const double nu = PI * (2.0 * u01(S.seed, idx, att, 5) - 1.0);
    const bool branch = u01(S.seed, idx, att, 6) < 0.5;
    const double r = a * (1.0 - e * e) / (1.0 + e * cos(nu));
    // the observer by value (a pointer into the argument struct would put a
    // copy of it in scratch memory)
    const double O0 = S.obs_xyz_au[0], O1 = S.obs_xyz_au[1], O2 = S.obs_xyz_au[2];
    const double ou = d0 * O0 + d1 * O1 + d2 * O2;
    const double disc = ou * ou - (O0 * O0 + O1 * O1 + O2 * O2) + r * r;
    if (!(disc > 0.0)) continue;
    const double s = -ou + sqrt(disc);
    if (!(s > 0.0)) continue;
    const double X0 = O0 + s * d0, X1 = O1 + s * d1, X2 = O2 + s * d2;
    const double xn = sqrt(X0 * X0 + X1 * X1 + X2 * X2);
    const double beta = asin(fmin(fmax(X2 / xn, -1.0), 1.0));
    const double lam = atan2(X1, X0);
    inc = fmax(inc, fabs(beta) * (1.0 + 1e-9) + 1e-12);
    double u = asin(fmin(fmax(sin(beta) / sin(inc), -1.0), 1.0));
    if (branch) u = PI - u;
    const double node = lam - atan2(cos(inc) * sin(u), cos(u));
    const double peri = u - nu;
    const double E = 2.0 * atan2(sqrt(1.0 - e) * sin(0.5 * nu), sqrt(1.0 + e) * cos(0.5 * nu));
    const double M0 = E - e * sin(E);
    const double tp = 2.0 * PI;
    el[0] = a;
    el[1] = e;
    el[2] = inc;
    el[3] = node - tp * floor(node / tp);
    el[4] = peri - tp * floor(peri / tp);
    el[5] = (M0 + PI) - tp * floor((M0 + PI) / tp) - PI;
    return true;
  }
  return false;
}

__global__ __launch_bounds__(256) void k_generate(dt_orbit_sampler S, int64_t first, int64_t n, double* __restrict__ a,
                                                  double* __restrict__ e, double* __restrict__ inc,
                                                  double* __restrict__ node, double* __restrict__ peri,
                                                  double* __restrict__ m0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double el[6] = {__builtin_nan(""), 0.0, 0.0, 0.0, 0.0, 0.0};  // a = NaN: no orbit at this index
  gen_orbit(S, (uint64_t)(first + i), el);
  a[i] = el[0];
  e[i] = el[1];
  inc[i] = el[2];
  node[i] = el[3];
  peri[i] = el[4];
  m0[i] = el[5];
}

// Generate-and-stack: orbit first + i is generated in registers and stacked;
// no element arrays exist.
__global__ __launch_bounds__(256) void k_stack_generated(StackArgs A, dt_orbit_sampler S, int64_t first) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  float snr = __builtin_nanf(""), flux = __builtin_nanf("");
  int nv = -1;
  if (gen_orbit(S, (uint64_t)(first + i), el) && orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5])) {
    Orbit ob;
    orbit_prep(el[0], el[1], el[2], el[3], el[4], el[5], ob);
    stack_walk(A, ob, snr, flux, nv);
  }
  if (A.snr) A.snr[i] = snr;
  if (A.flux) A.flux[i] = flux;
  if (A.nvalid) A.nvalid[i] = nv;
}

// The same by checkpoint prediction (one wavefront per 64 generated orbits).
__global__ __launch_bounds__(64, 4) void k_stack_generated_track(StackArgs A, dt_orbit_sampler S, int64_t first) {
  __shared__ TrackQueue tq[1];
  if (wave_base() >= A.n) return;  // the whole wavefront is past the end
  bool in;
  float snr, flux;
  int nv;
  {
    const int64_t i = wave_base() + __lane_id();
    in = i < A.n;
    double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const bool live = in && gen_orbit(S, (uint64_t)(first + i), el) &&
                      orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]);
    if (track_stack_lane<false, true, true>(A, el, live, tq[threadIdx.x >> 6], snr, flux, nv)) {
      defer_wave(A, wave_base());
      return;
    }
  }
  if (!in) return;
  const int64_t i = thread_index_after_walk();
  if (A.snr) A.snr[i] = snr;
  if (A.flux) A.flux[i] = flux;
  if (A.nvalid) A.nvalid[i] = nv;
}

// The deferred wavefronts of k_stack_generated_track, walked per sample: one
// wavefront per list entry (the first orbit index of 64); wavefronts past the
// number of entries return at once.  (A persistent loop over the entries kept
// loop-invariant sampler and metadata values live across the walk and
// spilled.)
__global__ __launch_bounds__(256, 4) void k_stack_generated_deferred(StackArgs A, dt_orbit_sampler S, int64_t first) {
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= (int64_t)*A.defer_count) return;
  const int64_t i = A.defer_list[j] + (int64_t)__lane_id();
  const bool in = i < A.n;
  double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const bool live = in && gen_orbit(S, (uint64_t)(first + i), el) &&
                    orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]);
  float snr, flux;
  int nv;
  deferred_lane(A, el, live, snr, flux, nv);
  if (!in) return;
  if (A.snr) A.snr[i] = snr;
  if (A.flux) A.flux[i] = flux;
  if (A.nvalid) A.nvalid[i] = nv;
}

hipError_t launch_generate(const dt_orbit_sampler& S, int64_t first, int64_t n, double* a, double* e, double* inc,
                           double* node, double* peri, double* m0, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_generate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, first, n, a, e, inc, node,
                     peri, m0);
  return hipGetLastError();
}

// The per-sample walk of orbits first + i with the work counters (all
// wavefronts walk; used for the orbits after a probe whose wavefronts almost
// all deferred).
__global__ __launch_bounds__(256, 4) void k_stack_generated_walk(StackArgs A, dt_orbit_sampler S, int64_t first) {
  if (wave_base() >= A.n) return;  // the whole wavefront is past the end
  const int64_t i = wave_base() + __lane_id();
  const bool in = i < A.n;
  double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const bool live = in && gen_orbit(S, (uint64_t)(first + i), el) &&
                    orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]);
  float snr, flux;
  int nv;
  deferred_lane(A, el, live, snr, flux, nv);
  if (!in) return;
  if (A.snr) A.snr[i] = snr;
  if (A.flux) A.flux[i] = flux;
  if (A.nvalid) A.nvalid[i] = nv;
}

hipError_t launch_stack_generated_walk(const StackArgs& a, const dt_orbit_sampler& S, int64_t first, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stack_generated_walk, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, S, first);
  return hipGetLastError();
}

hipError_t launch_stack_generated(const StackArgs& a, const dt_orbit_sampler& S, int64_t first, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.vobs < __builtin_inf()) {
    if (a.defer_list) {
      hipError_t e = launch_zero_u32(a.defer_count, s);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_stack_generated_track, dim3((unsigned)((a.n + 63) / 64)), dim3(64), 0, s, a, S, first);
    if (a.defer_list)
      hipLaunchKernelGGL(k_stack_generated_deferred, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, S,
                         first);
  } else {
    hipLaunchKernelGGL(k_stack_generated, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, S, first);
  }
  return hipGetLastError();
}

}  // namespace dtk
