// k_batched.hip -- many patches with uneven exposure counts, image sizes and
// orbit-set sizes in one persistent launch.
//
// The host splits every patch's orbit set into work items of up to `chunk`
// orbits, orders them by cost (exposures x orbits, largest first) and cuts
// them into wavefront items of at most 64 orbits in that order.  A grid
// sized to the machine, not to the work, then pulls items from one device
// counter: each wavefront takes the next item, runs the same per-orbit stack
// as the single-patch kernel over that patch's exposures (the checkpoint
// walk without deferral), and asks for another until the counter passes the
// end.  Large and small patches share the CUs, and the tail is made of the
// cheapest items.  The counter is zeroed by a one-thread kernel so the whole
// sequence can be captured in a graph.
#include "dt_track.hpp"

namespace dtk {

__global__ void k_reset_counter(unsigned int* counter) { *counter = 0u; }

__global__ __launch_bounds__(64, 4) void k_stack_persistent(const StackArgs* __restrict__ descs,
                                                             const WorkItem* __restrict__ items, int n_items,
                                                             unsigned int* __restrict__ counter) {
  __shared__ TrackQueue tq[1];
  // every wavefront pulls items of at most 64 orbits on its own (no
  // workgroup barrier); item, descriptor and first orbit are wave-uniform
  // scalar loads
  while (true) {
    unsigned int t = 0;
    if (__lane_id() == 0) t = atomicAdd(counter, 1u);
    const int it = __builtin_amdgcn_readfirstlane((int)t);
    if (it >= n_items) break;
    const WorkItem w = items[it];
    const StackArgs& A = descs[w.patch];
    const int64_t b = w.begin;
    if (A.vobs < __builtin_inf()) {
      // checkpoint prediction, one wavefront per 64 orbits (as k_stack_track)
      bool in;
      float snr, flux;
      int nv;
      {
        const int64_t o = b + __lane_id();
        in = (int)__lane_id() < w.count;
        double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (in) {
          // the descriptor's pointers are generic to the compiler: read as global
          el[0] = global_load(A.a, o);
          el[1] = global_load(A.e, o);
          el[2] = global_load(A.inc, o);
          el[3] = global_load(A.node, o);
          el[4] = global_load(A.peri, o);
          el[5] = global_load(A.m0, o);
        }
        track_stack_lane<false, false, true>(A, el, in && orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]),
                                       tq[threadIdx.x >> 6], snr, flux, nv);
      }
      if (in) {
        // the lane id again, opaque to the compiler (see thread_index_after_walk)
        int lane = (int)__lane_id();
        asm volatile("" : "+v"(lane));
        const int64_t o = b + lane;
        if (A.snr) A.snr[o] = snr;
        if (A.flux) A.flux[o] = flux;
        if (A.nvalid) A.nvalid[o] = nv;
      }
      continue;
    }
    if ((int)__lane_id() < w.count) {
      float snr, flux;
      int nv;
      stack_orbit<false>(A, b + __lane_id(), nullptr, 0, snr, flux, nv);
      int lane = (int)__lane_id();  // opaque again, as above
      asm volatile("" : "+v"(lane));
      const int64_t o = b + lane;
      if (A.snr) A.snr[o] = snr;
      if (A.flux) A.flux[o] = flux;
      if (A.nvalid) A.nvalid[o] = nv;
    }
  }
}

hipError_t launch_batched(const StackArgs* d_descs, const WorkItem* d_items, int n_items, unsigned int* d_counter,
                          int n_wg, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, d_counter);
  // n_wg groups of four wavefronts, launched as single-wavefront workgroups
  // (each with its own LDS queue; the wavefronts share nothing)
  hipLaunchKernelGGL(k_stack_persistent, dim3(4 * n_wg), dim3(64), 0, s, d_descs, d_items, n_items, d_counter);
  return hipGetLastError();
}

}  // namespace dtk
