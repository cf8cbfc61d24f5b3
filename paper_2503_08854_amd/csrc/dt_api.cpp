// dt_api.cpp -- the C ABI of libdtrack: contexts, patches, argument
// validation, memory accounting and stream plumbing.  All numerical work is
// in the kernels; this file only checks arguments, sizes buffers and enqueues.
#include <cmath>

#include "dt_internal.hpp"

namespace dtk {
namespace {
thread_local char g_err[512] = "";
}

dt_status fail(dt_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

dt_status hip_fail(hipError_t e, const char* what) {
  return fail(DT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err; }

dt_status ctx_alloc(dt_ctx* c, void** p, size_t bytes, const char* what) {
  *p = nullptr;
  if (bytes == 0) return DT_OK;
  if (c->mem_limit && c->mem_used + bytes > c->mem_limit)
    return fail(DT_E_OOM, "%s: %zu bytes would exceed the context limit (%zu of %zu used)", what, bytes,
                c->mem_used, c->mem_limit);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(DT_E_OOM, "%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
  }
  c->mem_used += bytes;
  return DT_OK;
}

void ctx_free(dt_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  c->mem_used -= bytes;
}

namespace {
bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

dt_status check_exposure(const dt_exposure& x, int i) {
  if (x.width <= 0 || x.height <= 0) return fail(DT_E_ARG, "exposure %d: width/height must be positive", i);
  if ((int64_t)x.width * x.height > (int64_t)1 << 31)
    return fail(DT_E_ARG, "exposure %d: more than 2^31 pixels", i);
  if (!std::isfinite(x.t) || !finite_all(x.obs_xyz_au, 3) || !finite_all(x.crval_deg, 2) ||
      !finite_all(x.crpix, 2) || !finite_all(x.cd_deg, 4))
    return fail(DT_E_DOMAIN, "exposure %d: non-finite epoch, observer or WCS value", i);
  if (std::fabs(x.crval_deg[1]) > 90.0) return fail(DT_E_DOMAIN, "exposure %d: |CRVAL2| > 90", i);
  double det = x.cd_deg[0] * x.cd_deg[3] - x.cd_deg[1] * x.cd_deg[2];
  double scale = std::fabs(x.cd_deg[0]) + std::fabs(x.cd_deg[1]) + std::fabs(x.cd_deg[2]) + std::fabs(x.cd_deg[3]);
  if (!(std::fabs(det) > 1e-12 * scale * scale) || !std::isfinite(det))
    return fail(DT_E_DOMAIN, "exposure %d: CD matrix is singular", i);
  if (!(x.psf_fwhm_px >= 0.5f && x.psf_fwhm_px <= 8.0f))
    return fail(DT_E_DOMAIN, "exposure %d: PSF FWHM %g outside [0.5, 8] px", i, (double)x.psf_fwhm_px);
  return DT_OK;
}

void patch_free(dt_patch* p) {
  dt_ctx* c = p->ctx;
  ctx_free(c, p->d_meta, sizeof(ExpMeta) * (p->n_exp + 1));
  ctx_free(c, p->d_planes, sizeof(float2) * p->plane_elems);
  ctx_free(c, p->d_tiles, sizeof(PrepTile) * p->n_tiles);
  ctx_free(c, p->d_flux, sizeof(void*) * p->n_exp);
  ctx_free(c, p->d_var, sizeof(void*) * p->n_exp);
  ctx_free(c, p->d_npix, sizeof(int64_t) * p->n_exp);
  ctx_free(c, p->d_sigma, sizeof(double) * p->n_exp);
  ctx_free(c, p->noise_ws, noise_scratch_bytes(p->n_exp));
  p->d_npix = nullptr;
  p->d_sigma = nullptr;
  p->noise_ws = nullptr;
  p->d_meta = nullptr;
  p->d_planes = nullptr;
  p->d_tiles = nullptr;
  p->d_flux = p->d_var = nullptr;
}
}  // namespace

dt_status check_orbits(const dt_orbits* o) {
  if (!o) return fail(DT_E_ARG, "orbits is NULL");
  if (o->n < 0) return fail(DT_E_ARG, "orbits->n < 0");
  if (o->n > 0 && (!o->a || !o->e || !o->inc || !o->node || !o->peri || !o->m0))
    return fail(DT_E_ARG, "orbit element pointer is NULL");
  if (!std::isfinite(o->epoch)) return fail(DT_E_DOMAIN, "orbit epoch is not finite");
  if (o->n >= ((int64_t)1 << 32)) return fail(DT_E_ARG, "at most 2^32 - 1 orbits per call");
  return DT_OK;
}

StackArgs stack_args(const dt_patch* p, const dt_orbits* o) {
  StackArgs a;
  a.meta = p->d_meta;
  a.n_exp = p->n_exp;
  a.planes = p->d_planes;
  a.n = o->n;
  a.epoch = o->epoch;
  a.a = o->a;
  a.e = o->e;
  a.inc = o->inc;
  a.node = o->node;
  a.peri = o->peri;
  a.m0 = o->m0;
  a.snr = nullptr;
  a.flux = nullptr;
  a.nvalid = nullptr;
  a.vobs = p->vobs;
  a.work = p->ctx->count_work ? p->ctx->d_work : nullptr;
  return a;
}

dt_status defer_setup(dt_ctx* c, int64_t n, StackArgs& a) {
  const int64_t need = (n + 63) / 64;
  if (!c->d_defer_count) {
    dt_status st = ctx_alloc(c, reinterpret_cast<void**>(&c->d_defer_count), sizeof(unsigned int), "deferral count");
    if (st != DT_OK) return st;
  }
  if (need > c->defer_cap) {
    // the old list may still be read by enqueued work: wait before freeing it
    if (c->d_defer) {
      hipError_t e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return hip_fail(e, "deferral list resize");
      ctx_free(c, c->d_defer, sizeof(int64_t) * c->defer_cap);
      c->d_defer = nullptr;
      c->defer_cap = 0;
    }
    dt_status st = ctx_alloc(c, reinterpret_cast<void**>(&c->d_defer), sizeof(int64_t) * need, "deferral list");
    if (st != DT_OK) return st;
    c->defer_cap = need;
  }
  a.defer_list = c->d_defer;
  a.defer_count = c->d_defer_count;
  return DT_OK;
}

dt_status run_prepass(dt_patch* p, hipStream_t s) {
  if (p->images_released) return fail(DT_E_STATE, "the patch's images were released; the pre-pass cannot run");
  if (p->est_noise) {
    hipError_t e = launch_noise(p->d_flux, p->d_npix, p->max_pix, p->n_exp, p->dtype, NOISE_KAPPA, NOISE_MAX_ITER,
                                p->noise_ws, p->d_sigma, nullptr, nullptr, p->d_meta, s);
    if (e != hipSuccess) return hip_fail(e, "noise estimate launch");
  }
  hipError_t e = launch_prepass(p->d_meta, p->d_tiles, p->group_off.data(), p->group_R.data(),
                                (int)p->group_R.size(), p->d_flux, p->d_var, p->dtype, p->d_planes, s);
  if (e != hipSuccess) return hip_fail(e, "matched-filter pre-pass launch");
  return DT_OK;
}

}  // namespace dtk

using namespace dtk;

extern "C" {

const char* dt_last_error(void) { return dtk::last_error(); }
const char* dt_version(void) { return "dtrack 0.1 (gfx950)"; }

dt_status dt_ctx_create(int device, void* hip_stream, dt_ctx** out) {
  if (!out) return fail(DT_E_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(DT_E_ARG, "device %d out of range (%d devices)", device, n);
  DeviceGuard g(device);
  e = topk_noalloc_setup(device);
  if (e != hipSuccess) return hip_fail(e, "allocation-free top-k scratch address");
  dt_ctx* c = new dt_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  dt_status st = ctx_alloc(c, reinterpret_cast<void**>(&c->d_counter), sizeof(unsigned long long), "counter");
  if (st != DT_OK) {
    delete c;
    return st;
  }
  *out = c;
  return DT_OK;
}

dt_status dt_ctx_set_stream(dt_ctx* c, void* hip_stream) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  c->stream = static_cast<hipStream_t>(hip_stream);
  return DT_OK;
}

dt_status dt_ctx_set_mem_limit(dt_ctx* c, size_t bytes) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  c->mem_limit = bytes;
  return DT_OK;
}

dt_status dt_ctx_mem_used(dt_ctx* c, size_t* out) {
  if (!c || !c->alive || !out) return fail(DT_E_ARG, "invalid context or NULL out");
  *out = c->mem_used;
  return DT_OK;
}

dt_status dt_ctx_destroy(dt_ctx* c) {
  if (!c) return fail(DT_E_ARG, "context is NULL");
  if (c->n_patches) return fail(DT_E_STATE, "context still owns %d patch(es)", c->n_patches);
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  batch_graph_drop(c);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  ctx_free(c, c->topk_scratch, c->topk_bytes);
  ctx_free(c, c->noise_ws, c->noise_bytes);
  ctx_free(c, c->d_counter, sizeof(unsigned long long));
  ctx_free(c, c->d_work, sizeof(unsigned long long) * WORK_SLOTS * WORK_N);
  ctx_free(c, c->d_defer, sizeof(int64_t) * c->defer_cap);
  ctx_free(c, c->d_defer_count, sizeof(unsigned int));
  c->alive = false;
  delete c;
  return DT_OK;
}

dt_status dt_ctx_count_work(dt_ctx* c, int32_t on) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  DeviceGuard g(c->device);
  const size_t bytes = sizeof(unsigned long long) * WORK_SLOTS * WORK_N;
  if (on && !c->d_work) {
    dt_status st = ctx_alloc(c, reinterpret_cast<void**>(&c->d_work), bytes, "work counters");
    if (st != DT_OK) return st;
  }
  if (on) {
    hipError_t e = hipMemsetAsync(c->d_work, 0, bytes, c->stream);
    if (e != hipSuccess) return hip_fail(e, "work counter reset");
  }
  c->count_work = on != 0;
  return DT_OK;
}

dt_status dt_ctx_work(dt_ctx* c, uint64_t* out) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  if (!out) return fail(DT_E_ARG, "out is NULL");
  for (int k = 0; k < DT_WORK_COUNTERS; ++k) out[k] = 0;
  if (!c->d_work) return DT_OK;
  DeviceGuard g(c->device);
  std::vector<unsigned long long> h(WORK_SLOTS * WORK_N);
  hipError_t e = hipMemcpyAsync(h.data(), c->d_work, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_work, 0, sizeof(unsigned long long) * h.size(), c->stream);
  if (e != hipSuccess) return hip_fail(e, "work counter read");
  for (int sl = 0; sl < WORK_SLOTS; ++sl)
    for (int k = 0; k < DT_WORK_COUNTERS && k < WORK_N; ++k) out[k] += h[sl * WORK_N + k];
  return DT_OK;
}

dt_status dt_patch_create(dt_ctx* c, const dt_exposure* exps, int32_t n_exp, const void* const* d_flux,
                          const void* const* d_var, dt_dtype dtype, dt_patch** out) {
  if (!out) return fail(DT_E_ARG, "out is NULL");
  *out = nullptr;
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  if (n_exp <= 0 || !exps || !d_flux) return fail(DT_E_ARG, "need n_exp > 0 and non-NULL arrays");
  if (dtype != DT_F32 && dtype != DT_F16) return fail(DT_E_ARG, "unknown dtype %d", (int)dtype);
  for (int i = 0; i < n_exp; ++i) {
    dt_status st = check_exposure(exps[i], i);
    if (st != DT_OK) return st;
    if (!d_flux[i] || (d_var && !d_var[i])) return fail(DT_E_ARG, "exposure %d: image pointer is NULL", i);
  }
  DeviceGuard g(c->device);
  dt_patch* p = new dt_patch();
  p->ctx = c;
  p->n_exp = n_exp;
  p->dtype = dtype;
  p->est_noise = d_var == nullptr;
  p->order.resize(n_exp);
  std::iota(p->order.begin(), p->order.end(), 0);
  std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int b) { return exps[a].t < exps[b].t; });
  p->where.resize(n_exp);
  for (int s = 0; s < n_exp; ++s) p->where[p->order[s]] = s;
  std::vector<dt_exposure> sorted(n_exp);
  std::vector<int64_t> off_sorted(n_exp);
  std::vector<int32_t> rad(n_exp);
  p->plane_off.resize(n_exp);
  p->W.resize(n_exp);
  p->H.resize(n_exp);
  int64_t off = 0;
  std::vector<PrepTile> tiles;
  for (int s = 0; s < n_exp; ++s) {
    const dt_exposure& x = exps[p->order[s]];
    sorted[s] = x;
    off_sorted[s] = off;
    p->plane_off[p->order[s]] = off;
    p->W[p->order[s]] = x.width;
    p->H[p->order[s]] = x.height;
    rad[s] = stamp_radius((double)x.psf_fwhm_px);
    p->rmax = std::max(p->rmax, rad[s]);
    off += (int64_t)x.width * x.height;
  }
  p->plane_elems = (size_t)off;
  // observer speed bound over epoch neighbours (the stack's prediction bound
  // chains it over any span by the triangle inequality)
  for (int s = 1; s < n_exp; ++s) {
    const dt_exposure &x = sorted[s], &y = sorted[s - 1];
    const double d0 = x.obs_xyz_au[0] - y.obs_xyz_au[0], d1 = x.obs_xyz_au[1] - y.obs_xyz_au[1];
    const double d2 = x.obs_xyz_au[2] - y.obs_xyz_au[2];
    const double dist = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2), dt = x.t - y.t;
    if (dist > 0.0) p->vobs = std::max(p->vobs, dt > 0.0 ? dist / dt : HUGE_VAL);
  }
  // the checkpoint walk packs an exposure index into 25 bits; beyond that (and
  // without a finite bound) the per-sample walk runs
  if (!std::isfinite(p->vobs) || n_exp >= (1 << 25)) p->vobs = HUGE_VAL;
  if (p->rmax > PREP_RMAX) {
    delete p;
    return fail(DT_E_DOMAIN, "stamp half-width %d exceeds %d", p->rmax, PREP_RMAX);
  }
  // pre-pass tiles, grouped by stamp half-width (one kernel instance per R)
  for (int R = 1; R <= PREP_RMAX; ++R) {
    size_t before = tiles.size();
    for (int s = 0; s < n_exp; ++s) {
      if (rad[s] != R) continue;
      const dt_exposure& x = sorted[s];
      for (int y0 = 0; y0 < x.height; y0 += PREP_TY)
        for (int x0 = 0; x0 < x.width; x0 += PREP_TX) tiles.push_back(PrepTile{s, x0, y0, 0});
    }
    if (tiles.size() > before) {
      p->group_off.push_back((int64_t)before);
      p->group_R.push_back(R);
    }
  }
  p->group_off.push_back((int64_t)tiles.size());
  p->n_tiles = (int64_t)tiles.size();
  dt_exposure* d_exps = nullptr;
  int64_t* d_off = nullptr;
  int32_t* d_src = nullptr;
  int32_t* d_rad = nullptr;
  dt_status st = DT_OK;
  auto A = [&](void** ptr, size_t bytes, const char* what) {
    if (st == DT_OK) st = ctx_alloc(c, ptr, bytes, what);
  };
  A((void**)&p->d_meta, sizeof(ExpMeta) * (n_exp + 1), "exposure metadata");  // + the repeated last record
  A((void**)&p->d_planes, sizeof(float2) * p->plane_elems, "matched-filter planes");
  A((void**)&p->d_tiles, sizeof(PrepTile) * p->n_tiles, "pre-pass tiles");
  A((void**)&p->d_flux, sizeof(void*) * n_exp, "flux pointers");
  A((void**)&p->d_var, sizeof(void*) * n_exp, "variance pointers");
  std::vector<int64_t> npix(n_exp);
  for (int i = 0; i < n_exp; ++i) {
    npix[i] = (int64_t)exps[i].width * exps[i].height;
    p->max_pix = std::max(p->max_pix, npix[i]);
  }
  std::vector<const void*> no_var(n_exp, nullptr);
  if (p->est_noise) {
    A((void**)&p->d_npix, sizeof(int64_t) * n_exp, "noise pixel counts");
    A((void**)&p->d_sigma, sizeof(double) * n_exp, "noise estimates");
    A(&p->noise_ws, noise_scratch_bytes(n_exp), "noise selection state");
  }
  A((void**)&d_exps, sizeof(dt_exposure) * n_exp, "staging");
  A((void**)&d_off, sizeof(int64_t) * n_exp, "staging");
  A((void**)&d_src, sizeof(int32_t) * n_exp, "staging");
  A((void**)&d_rad, sizeof(int32_t) * n_exp, "staging");
  auto cleanup = [&]() {
    ctx_free(c, d_exps, sizeof(dt_exposure) * n_exp);
    ctx_free(c, d_off, sizeof(int64_t) * n_exp);
    ctx_free(c, d_src, sizeof(int32_t) * n_exp);
    ctx_free(c, d_rad, sizeof(int32_t) * n_exp);
  };
  if (st != DT_OK) {
    cleanup();
    patch_free(p);
    delete p;
    return st;
  }
  hipStream_t s = c->stream;
  hipError_t e = hipSuccess;
  auto H2D = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  H2D(d_exps, sorted.data(), sizeof(dt_exposure) * n_exp);
  H2D(d_off, off_sorted.data(), sizeof(int64_t) * n_exp);
  H2D(d_src, p->order.data(), sizeof(int32_t) * n_exp);
  H2D(d_rad, rad.data(), sizeof(int32_t) * n_exp);
  H2D(p->d_tiles, tiles.data(), sizeof(PrepTile) * p->n_tiles);
  H2D(p->d_flux, d_flux, sizeof(void*) * n_exp);
  H2D(p->d_var, d_var ? (const void*)d_var : (const void*)no_var.data(), sizeof(void*) * n_exp);
  if (p->est_noise) H2D(p->d_npix, npix.data(), sizeof(int64_t) * n_exp);
  if (e == hipSuccess) e = launch_exposure_prep(d_exps, d_off, d_src, d_rad, n_exp, p->d_meta, s);
  // staging buffers must outlive the async copies
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) {
    patch_free(p);
    delete p;
    return hip_fail(e, "patch upload");
  }
  st = run_prepass(p, c->stream);
  if (st != DT_OK) {
    patch_free(p);
    delete p;
    return st;
  }
  c->n_patches++;
  *out = p;
  return DT_OK;
}

dt_status dt_patch_refresh(dt_patch* p) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  DeviceGuard g(p->ctx->device);
  return run_prepass(p, p->ctx->stream);
}

dt_status dt_patch_noise(dt_patch* p, double* d_sigma) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  if (!p->est_noise) return fail(DT_E_STATE, "the patch was created with variance planes");
  if (!d_sigma) return fail(DT_E_ARG, "d_sigma is NULL");
  DeviceGuard g(p->ctx->device);
  hipError_t e = hipMemcpyAsync(d_sigma, p->d_sigma, sizeof(double) * p->n_exp, hipMemcpyDeviceToDevice,
                                p->ctx->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "noise copy");
}

dt_status dt_image_noise(dt_ctx* c, int32_t n_img, const void* const* d_images, const int64_t* n_pixels,
                         dt_dtype dtype, double kappa, int32_t max_iter, double* d_sigma, int64_t* d_n_used,
                         int32_t* d_iters) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  if (n_img < 0 || n_img > 65535) return fail(DT_E_ARG, "n_img must be in [0, 65535]");
  if (n_img == 0) return DT_OK;
  if (!d_images || !n_pixels) return fail(DT_E_ARG, "NULL image or size array");
  if (dtype != DT_F32 && dtype != DT_F16) return fail(DT_E_ARG, "unknown dtype %d", (int)dtype);
  if (!(kappa > 0.0) || !std::isfinite(kappa)) return fail(DT_E_DOMAIN, "kappa must be finite and > 0");
  if (max_iter < 1 || max_iter > 100) return fail(DT_E_ARG, "max_iter must be in [1, 100]");
  int64_t max_pix = 0;
  for (int i = 0; i < n_img; ++i) {
    if (n_pixels[i] < 0) return fail(DT_E_ARG, "image %d: negative pixel count", i);
    if (n_pixels[i] > 0 && !d_images[i]) return fail(DT_E_ARG, "image %d: NULL pointer", i);
    max_pix = std::max(max_pix, n_pixels[i]);
  }
  DeviceGuard g(c->device);
  const size_t stage = ((sizeof(void*) + sizeof(int64_t)) * (size_t)n_img + 255) / 256 * 256;
  const size_t need = stage + noise_scratch_bytes(n_img);
  if (need > c->noise_bytes) {
    (void)hipStreamSynchronize(c->stream);
    ctx_free(c, c->noise_ws, c->noise_bytes);
    c->noise_ws = nullptr;
    c->noise_bytes = 0;
    dt_status st = ctx_alloc(c, &c->noise_ws, need, "noise scratch");
    if (st != DT_OK) return st;
    c->noise_bytes = need;
  }
  char* ws = static_cast<char*>(c->noise_ws);
  const void** d_ptrs = reinterpret_cast<const void**>(ws);
  int64_t* d_npix = reinterpret_cast<int64_t*>(ws + sizeof(void*) * (size_t)n_img);
  hipError_t e = hipMemcpyAsync(d_ptrs, d_images, sizeof(void*) * n_img, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_npix, n_pixels, sizeof(int64_t) * n_img, hipMemcpyHostToDevice, c->stream);
  // the caller's host arrays must not be read after return
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess)
    e = launch_noise(d_ptrs, d_npix, max_pix, n_img, dtype, kappa, max_iter, ws + stage, d_sigma, d_n_used, d_iters,
                     nullptr, c->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "noise estimate");
}

dt_status dt_patch_release_images(dt_patch* p) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  if (batch_graph_uses(p->ctx, p)) batch_graph_drop(p->ctx);
  p->images_released = true;
  return DT_OK;
}

dt_status dt_patch_destroy(dt_patch* p) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  DeviceGuard g(p->ctx->device);
  (void)hipStreamSynchronize(p->ctx->stream);
  if (batch_graph_uses(p->ctx, p)) batch_graph_drop(p->ctx);
  p->ctx->n_patches--;
  patch_free(p);
  p->ctx = nullptr;
  delete p;
  return DT_OK;
}

dt_status dt_patch_plane(dt_patch* p, int32_t e, float* d_out) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  if (e < 0 || e >= p->n_exp || !d_out) return fail(DT_E_ARG, "bad exposure index or NULL output");
  DeviceGuard g(p->ctx->device);
  size_t bytes = sizeof(float2) * (size_t)p->W[e] * p->H[e];
  hipError_t err = hipMemcpyAsync(d_out, p->d_planes + p->plane_off[e], bytes, hipMemcpyDeviceToDevice,
                                  p->ctx->stream);
  if (err != hipSuccess) return hip_fail(err, "plane copy");
  return DT_OK;
}

dt_status dt_stack(dt_patch* p, const dt_orbits* o, float* d_snr, float* d_flux, int32_t* d_nvalid) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  dt_status st = check_orbits(o);
  if (st != DT_OK) return st;
  DeviceGuard g(p->ctx->device);
  StackArgs a = stack_args(p, o);
  a.snr = d_snr;
  a.flux = d_flux;
  a.nvalid = d_nvalid;
  if (o->n > 0 && p->vobs < __builtin_inf()) {
    st = defer_setup(p->ctx, o->n, a);
    if (st != DT_OK) return st;
  }
  hipError_t e = launch_stack(a, p->ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "stack launch");
  return DT_OK;
}

dt_status dt_orbits_validate(dt_ctx* c, const dt_orbits* o, int64_t* n_bad) {
  if (!c || !c->alive || !n_bad) return fail(DT_E_ARG, "invalid context or NULL n_bad");
  dt_status st = check_orbits(o);
  if (st != DT_OK) return st;
  DeviceGuard g(c->device);
  StackArgs a{};
  a.n = o->n;
  a.a = o->a;
  a.e = o->e;
  a.inc = o->inc;
  a.node = o->node;
  a.peri = o->peri;
  a.m0 = o->m0;
  unsigned long long h = 0;
  hipError_t e = hipMemcpyAsync(c->d_counter, &h, sizeof(h), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_validate(a, c->d_counter, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, c->d_counter, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "orbit validation");
  *n_bad = (int64_t)h;
  if (h) return fail(DT_E_DOMAIN, "%llu orbit(s) outside the domain (non-finite, a <= 0 or e not in [0, 1))", h);
  return DT_OK;
}

static dt_status topk_call(dt_ctx* c, const float* d_snr, int64_t n, int32_t k, float threshold, int64_t* d_idx,
                           float* d_val, int32_t* d_count, bool ordered) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  if (n < 0 || (n > 0 && !d_snr)) return fail(DT_E_ARG, "bad S/N array");
  if (n >= ((int64_t)1 << 32)) return fail(DT_E_ARG, "n must be < 2^32");
  if (k < 1 || k > 4096) return fail(DT_E_ARG, "k must be in [1, 4096]");
  if (!d_idx || !d_val || !d_count) return fail(DT_E_ARG, "NULL output");
  if (std::isnan(threshold)) return fail(DT_E_ARG, "threshold is NaN");
  DeviceGuard g(c->device);
  size_t need = topk_scratch_bytes(n, k);
  if (need > c->topk_bytes) {
    (void)hipStreamSynchronize(c->stream);
    ctx_free(c, c->topk_scratch, c->topk_bytes);
    c->topk_scratch = nullptr;
    c->topk_bytes = 0;
    dt_status st = ctx_alloc(c, &c->topk_scratch, need, "top-k scratch");
    if (st != DT_OK) return st;
    c->topk_bytes = need;
  }
  hipError_t e = launch_topk(d_snr, n, k, threshold, d_idx, d_val, d_count, c->topk_scratch, c->stream, ordered);
  if (e != hipSuccess) return hip_fail(e, "top-k launch");
  return DT_OK;
}

dt_status dt_topk(dt_ctx* c, const float* d_snr, int64_t n, int32_t k, float threshold, int64_t* d_idx,
                  float* d_val, int32_t* d_count) {
  return topk_call(c, d_snr, n, k, threshold, d_idx, d_val, d_count, true);
}

dt_status dt_topk_unordered(dt_ctx* c, const float* d_snr, int64_t n, int32_t k, float threshold, int64_t* d_idx,
                            float* d_val, int32_t* d_count) {
  return topk_call(c, d_snr, n, k, threshold, d_idx, d_val, d_count, false);
}

dt_status dt_debug_samples(dt_patch* p, const dt_orbits* o, const int64_t* d_ids, int64_t m, double* d_px,
                           double* d_py, int32_t* d_ix, int32_t* d_iy, int32_t* d_flags, float* d_psi,
                           float* d_phi, double* d_tau) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  dt_status st = check_orbits(o);
  if (st != DT_OK) return st;
  if (m < 0 || (m > 0 && !d_ids)) return fail(DT_E_ARG, "bad id array");
  DeviceGuard g(p->ctx->device);
  StackArgs a = stack_args(p, o);
  DebugArgs d{d_ids, m, d_px, d_py, d_tau, d_ix, d_iy, d_flags, d_psi, d_phi};
  hipError_t e = launch_debug(a, d, p->ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "debug launch");
  return DT_OK;
}

dt_status dt_debug_stack_samples(dt_patch* p, const dt_orbits* o, const int64_t* d_ids, int64_t m, double* d_px,
                                 double* d_py, int32_t* d_ix, int32_t* d_iy, int32_t* d_flags, float* d_psi,
                                 float* d_phi, double* d_tau) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  dt_status st = check_orbits(o);
  if (st != DT_OK) return st;
  if (m < 0 || (m > 0 && !d_ids)) return fail(DT_E_ARG, "bad id array");
  DeviceGuard g(p->ctx->device);
  StackArgs a = stack_args(p, o);
  DebugArgs d{d_ids, m, d_px, d_py, d_tau, d_ix, d_iy, d_flags, d_psi, d_phi};
  hipError_t e = launch_debug_stack(a, d, p->ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "stack-walk debug launch");
  return DT_OK;
}

dt_status dt_record_gathers(dt_patch* p, const dt_orbits* o, int64_t* d_start, int64_t* d_list, int64_t* h_entries,
                            int64_t* h_gathers) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  dt_status st = check_orbits(o);
  if (st != DT_OK) return st;
  const int64_t n = o->n;
  if (n > 0 && !d_start) return fail(DT_E_ARG, "d_start is NULL");
  DeviceGuard g(p->ctx->device);
  StackArgs a = stack_args(p, o);
  hipStream_t s = p->ctx->stream;
  if (d_list) {
    hipError_t e = launch_record_gathers(a, nullptr, d_start, d_list, s);
    return e == hipSuccess ? DT_OK : hip_fail(e, "gather recording launch");
  }
  if (!h_entries) return fail(DT_E_ARG, "h_entries is NULL");
  const int64_t groups = (n + 63) / 64;
  std::vector<int64_t> cnt(n), start(groups + 1, 0);
  int64_t* d_cnt = nullptr;
  if (n > 0) {
    st = ctx_alloc(p->ctx, (void**)&d_cnt, sizeof(int64_t) * n, "gather counts");
    if (st != DT_OK) return st;
    hipError_t e = launch_record_gathers(a, d_cnt, nullptr, nullptr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt.data(), d_cnt, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ctx_free(p->ctx, d_cnt, sizeof(int64_t) * n);
    if (e != hipSuccess) return hip_fail(e, "gather counting");
  }
  int64_t total = 0;
  for (int64_t gi = 0; gi < groups; ++gi) {
    int64_t w = 0;
    for (int64_t i = gi * 64; i < std::min(n, gi * 64 + 64); ++i) {
      w = std::max(w, cnt[i]);
      total += cnt[i];
    }
    start[gi + 1] = start[gi] + 64 * w;
  }
  if (n > 0) {
    hipError_t e = hipMemcpyAsync(d_start, start.data(), sizeof(int64_t) * (groups + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "gather group starts");
  }
  *h_entries = start[groups];
  if (h_gathers) *h_gathers = total;
  return DT_OK;
}

dt_status dt_gather_replay(dt_patch* p, const int64_t* d_start, const int64_t* d_list, int64_t n, float* d_snr) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  if (n < 0 || (n > 0 && (!d_start || !d_list || !d_snr))) return fail(DT_E_ARG, "bad start, list or output array");
  DeviceGuard g(p->ctx->device);
  hipError_t e = launch_gather_replay(p->d_planes, d_start, d_list, n, d_snr, p->ctx->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "gather replay launch");
}

}  // extern "C"
