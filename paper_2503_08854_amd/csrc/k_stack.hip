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
// together; used when the patch has a finite observer speed bound).  One
// wavefront per workgroup: the wavefronts are independent, and single-wave
// workgroups measured 3 % faster than four-wave ones on the survey set.
__global__ __launch_bounds__(64, 4) void k_stack_track(StackArgs A) {
  __shared__ TrackQueue tq[1];
  if (wave_base() >= A.n) return;  // the whole wavefront is past the end
  bool in;
  float snr, flux;
  int nv;
  {
    const int64_t o = wave_base() + __lane_id();
    in = o < A.n;
    double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (in) {
      el[0] = A.a[o]; el[1] = A.e[o]; el[2] = A.inc[o]; el[3] = A.node[o]; el[4] = A.peri[o]; el[5] = A.m0[o];
    }
    if (track_stack_lane<false, true, true>(A, el, in && orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]),
                                           tq[threadIdx.x >> 6], snr, flux, nv)) {
      defer_wave(A, wave_base());
      return;
    }
  }
  if (!in) return;
  const int64_t o = thread_index_after_walk();
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

// The wavefronts k_stack_track deferred, walked per sample: one wavefront
// per list entry (the first orbit of 64); wavefronts past the number of
// entries return at once.
__global__ __launch_bounds__(256, 4) void k_stack_deferred(StackArgs A) {
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= (int64_t)*A.defer_count) return;
  const int64_t o = A.defer_list[j] + (int64_t)__lane_id();
  const bool in = o < A.n;
  double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (in) {
    el[0] = A.a[o]; el[1] = A.e[o]; el[2] = A.inc[o]; el[3] = A.node[o]; el[4] = A.peri[o]; el[5] = A.m0[o];
  }
  float snr, flux;
  int nv;
  deferred_lane(A, el, in && orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]), snr, flux, nv);
  if (!in) return;
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

__global__ __launch_bounds__(64) void k_stack_debug(StackArgs A, DebugArgs D) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.m) return;
  const int64_t o = D.ids[r];
  if (o < 0 || o >= A.n) {
    rec_init_row(D, A.meta, A.n_exp, r);
    return;
  }
  float snr, flux;
  int nv;
  stack_orbit<true>(A, o, &D, r, snr, flux, nv);
}

// The debug table from the walks dt_stack runs: the checkpoint walk (row r =
// the wavefront's rows, queued samples written to their owner's row) and,
// for patches without an observer speed bound, the per-sample walk with its
// sky-cone test.  Only samples the walk solves exactly are written.
__global__ __launch_bounds__(256, 4) void k_stack_track_debug(StackArgs A, DebugArgs D) {
  __shared__ TrackQueue tq[4];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)__lane_id();
  if (r - lane >= D.m) return;  // the whole wavefront is past the end
  const bool in = r < D.m;
  const int64_t o = in ? D.ids[r] : -1;
  const bool has = o >= 0 && o < A.n;
  double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (has) {
    el[0] = A.a[o]; el[1] = A.e[o]; el[2] = A.inc[o]; el[3] = A.node[o]; el[4] = A.peri[o]; el[5] = A.m0[o];
  }
  if (in) rec_init_row(D, A.meta, A.n_exp, r);
  __syncthreads();  // the rows' initial values land before any lane's solves overwrite them
  float snr, flux;
  int nv;
  const bool live = has && orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]);
  if (track_stack_lane<true>(A, el, live, tq[threadIdx.x >> 6], snr, flux, nv, &D, r - lane)) {
    // deferred: as the deferred-walk kernel, the per-sample walk from the start
    __threadfence_block();
    if (in) rec_init_row(D, A.meta, A.n_exp, r);
    if (live) {
      Orbit ob;
      orbit_prep(el[0], el[1], el[2], el[3], el[4], el[5], ob);
      StackPart P;
      stack_range<true>(A, ob, 0, A.n_exp, P, &D, r);
    }
  }
}

__global__ __launch_bounds__(64) void k_stack_walk_debug(StackArgs A, DebugArgs D) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= D.m) return;
  const int64_t o = D.ids[r];
  rec_init_row(D, A.meta, A.n_exp, r);
  if (o < 0 || o >= A.n) return;
  const double a = A.a[o], e = A.e[o], inc = A.inc[o], node = A.node[o], peri = A.peri[o], m0 = A.m0[o];
  if (!orbit_ok(a, e, inc, node, peri, m0)) return;
  Orbit ob;
  orbit_prep(a, e, inc, node, peri, m0, ob);
  StackPart P;
  stack_range<true>(A, ob, 0, A.n_exp, P, &D, r);
}

__global__ __launch_bounds__(256) void k_validate(StackArgs A, unsigned long long* bad) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= A.n) return;
  if (!orbit_ok(A.a[o], A.e[o], A.inc[o], A.node[o], A.peri[o], A.m0[o])) atomicAdd(bad, 1ull);
}

// Measurement yardstick: the stack's gathers without its arithmetic.
// k_record_gathers walks orbit o exactly and either counts the samples that
// land inside an image (the gathers the stack makes) into cnt[o], or writes
// their global plane offsets, in epoch order, into the slot-major list of
// its group of 64 orbits: entry (k, lane) at gstart[g] + 64 k + lane, -1 past
// the lane's count up to the group's width (gstart[g + 1] - gstart[g]) / 64.
__global__ __launch_bounds__(256) void k_record_gathers(StackArgs A, int64_t* __restrict__ cnt,
                                                        const int64_t* __restrict__ gstart, int64_t* __restrict__ list) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= A.n) return;
  const int lane = (int)(o & 63);
  const int64_t g = o >> 6;
  int64_t* L = list ? list + gstart[g] + lane : nullptr;
  int64_t k = 0;
  const double a = A.a[o], e = A.e[o], inc = A.inc[o], node = A.node[o], peri = A.peri[o], m0 = A.m0[o];
  if (orbit_ok(a, e, inc, node, peri, m0)) {
    Orbit ob;
    orbit_prep(a, e, inc, node, peri, m0, ob);
    walk_orbit<true>(ob, A.meta, A.n_exp, A.epoch, [&](int ex, const SampleOut& so) {
      if (so.inside) {
        const ExpMeta& x = A.meta[ex];
        if (L) L[64 * k] = x.plane_off + (int64_t)so.iy * x.W + so.ix;
        k++;
      }
    });
  }
  if (cnt) cnt[o] = k;
  if (L) {
    const int64_t w = (gstart[g + 1] - gstart[g]) >> 6;
    for (; k < w; ++k) L[64 * k] = -1;
  }
}

// Lane o loads its recorded offsets (eight gathers in flight; a slot past
// the lane's list reads the first plane element and drops it) and sums them
// exactly as the stack does, in epoch order: its S/N equals the stack's.  A
// lane's list is compacted, so it stops after the batch that reaches its
// first -1: at most REPLAY_DEPTH - 1 padding entries are read per lane.
constexpr int REPLAY_DEPTH = 8;
__global__ __launch_bounds__(256) void k_gather_replay(const float2* __restrict__ planes,
                                                       const int64_t* __restrict__ gstart,
                                                       const int64_t* __restrict__ list, int64_t n,
                                                       float* __restrict__ snr) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const int lane = (int)(o & 63);
  const int64_t g = o >> 6;
  const int64_t base = gstart[g];
  const int64_t w = (gstart[g + 1] - base) >> 6;
  const int64_t* L = list + base + lane;
  Kahan ps, ph;
  ps.init();
  ph.init();
  bool done = false;
#pragma unroll 1
  for (int64_t k = 0; k < w && !done; k += REPLAY_DEPTH) {
    int64_t off[REPLAY_DEPTH];
    float2 v[REPLAY_DEPTH];
#pragma unroll
    for (int j = 0; j < REPLAY_DEPTH; ++j) off[j] = k + j < w ? L[64 * (k + j)] : -1;
#pragma unroll
    for (int j = 0; j < REPLAY_DEPTH; ++j) v[j] = planes[off[j] >= 0 ? off[j] : 0];
#pragma unroll
    for (int j = 0; j < REPLAY_DEPTH; ++j) {
      if (off[j] >= 0 && v[j].y > 0.f) {
        ps.add(v[j].x);
        ph.add(v[j].y);
      }
    }
    done = off[REPLAY_DEPTH - 1] < 0;
  }
  const float Psi = ps.s - ps.c, Phi = ph.s - ph.c;
  snr[o] = Phi > 0.f ? Psi / sqrtf(Phi) : 0.f;
}

static inline unsigned int grid_for(int64_t n, int bs) { return (unsigned int)((n + bs - 1) / bs); }

hipError_t launch_record_gathers(const StackArgs& a, int64_t* cnt, const int64_t* gstart, int64_t* list,
                                 hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_record_gathers, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a, cnt, gstart, list);
  return hipGetLastError();
}

hipError_t launch_gather_replay(const float2* planes, const int64_t* gstart, const int64_t* list, int64_t n,
                                float* snr, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_replay, dim3(grid_for(n, 256)), dim3(256), 0, s, planes, gstart, list, n, snr);
  return hipGetLastError();
}

hipError_t launch_stack(const StackArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.vobs < __builtin_inf()) {
    if (a.defer_list) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, a.defer_count);
    hipLaunchKernelGGL(k_stack_track, dim3(grid_for(a.n, 64)), dim3(64), 0, s, a);
    if (a.defer_list) hipLaunchKernelGGL(k_stack_deferred, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_stack, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_debug(const StackArgs& a, const DebugArgs& d, hipStream_t s) {
  if (d.m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stack_debug, dim3(grid_for(d.m, 64)), dim3(64), 0, s, a, d);
  return hipGetLastError();
}

hipError_t launch_debug_stack(const StackArgs& a, const DebugArgs& d, hipStream_t s) {
  if (d.m <= 0) return hipSuccess;
  if (a.vobs < __builtin_inf())
    hipLaunchKernelGGL(k_stack_track_debug, dim3(grid_for(d.m, 256)), dim3(256), 0, s, a, d);
  else
    hipLaunchKernelGGL(k_stack_walk_debug, dim3(grid_for(d.m, 64)), dim3(64), 0, s, a, d);
  return hipGetLastError();
}

hipError_t launch_validate(const StackArgs& a, unsigned long long* d_bad, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a, d_bad);
  return hipGetLastError();
}

}  // namespace dtk
