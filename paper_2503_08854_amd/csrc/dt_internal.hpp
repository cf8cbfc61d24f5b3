// dt_internal.hpp -- host-side objects of libdtrack shared by the API files.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "dt_common.hpp"

namespace dtk {
struct BatchGraph;
dt_status fail(dt_status st, const char* fmt, ...);
dt_status hip_fail(hipError_t e, const char* what);
}  // namespace dtk

struct dt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t mem_limit = 0;
  size_t mem_used = 0;
  int n_patches = 0;
  void* topk_scratch = nullptr;
  size_t topk_bytes = 0;
  unsigned long long* d_counter = nullptr;
  void* noise_ws = nullptr;  // staging + selection state of dt_image_noise
  size_t noise_bytes = 0;
  dtk::BatchGraph* graph = nullptr;  // last captured batched launch
  hipStream_t capture_stream = nullptr;
  unsigned long long* d_work = nullptr;  // work counters (dt_ctx_count_work), WORK_SLOTS x WORK_N
  bool count_work = false;
  int64_t* d_defer = nullptr;            // deferral list of the checkpoint walk (first orbit of 64)
  int64_t defer_cap = 0;                 // its entries
  unsigned int* d_defer_count = nullptr;
  bool alive = true;
};

struct dt_patch {
  dt_ctx* ctx = nullptr;
  int32_t n_exp = 0;
  dt_dtype dtype = DT_F32;
  std::vector<int32_t> order;      // sorted position -> caller index
  std::vector<int32_t> where;      // caller index -> sorted position
  std::vector<int64_t> plane_off;  // caller index -> plane offset
  std::vector<int32_t> W, H;       // caller order
  int rmax = 0;
  double vobs = 0.0;               // observer speed bound (AU/day), see StackArgs
  int64_t n_tiles = 0;
  std::vector<int64_t> group_off;  // pre-pass tiles grouped by stamp half-width
  std::vector<int32_t> group_R;
  size_t plane_elems = 0;
  dtk::ExpMeta* d_meta = nullptr;
  float2* d_planes = nullptr;
  dtk::PrepTile* d_tiles = nullptr;
  const void** d_flux = nullptr;
  const void** d_var = nullptr;
  bool images_released = false;
  // no variance planes: per-exposure noise by iterated MAD at every pre-pass
  bool est_noise = false;
  int64_t max_pix = 0;
  int64_t* d_npix = nullptr;   // caller order
  double* d_sigma = nullptr;   // caller order
  void* noise_ws = nullptr;
};

namespace dtk {
dt_status ctx_alloc(dt_ctx* c, void** p, size_t bytes, const char* what);
void ctx_free(dt_ctx* c, void* p, size_t bytes);
dt_status check_orbits(const dt_orbits* o);
// Deferral list for a checkpoint-walk launch of n orbits (grown on demand);
// sets a.defer_list / a.defer_count.
dt_status defer_setup(dt_ctx* c, int64_t n, StackArgs& a);
StackArgs stack_args(const dt_patch* p, const dt_orbits* o);
dt_status run_prepass(dt_patch* p, hipStream_t s);
void batch_graph_drop(dt_ctx* c);
bool batch_graph_uses(const dt_ctx* c, const dt_patch* p);

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};
}  // namespace dtk
