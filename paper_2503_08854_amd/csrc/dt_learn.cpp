// dt_learn.cpp -- C ABI of the learned-proposal path: coarse stamps of
// orbit-grid cells and the stack restricted to selected cells.
#include "dt_internal.hpp"

using namespace dtk;

extern "C" {

dt_status dt_cell_stamps(dt_patch* p, const dt_orbits* reps, double da, double dm, uint16_t* d_stamps_bf16,
                         float* d_stamps_f32, uint16_t* d_feats_bf16, float* d_feats_f32) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  dt_status st = check_orbits(reps);
  if (st != DT_OK) return st;
  if (!d_stamps_bf16 && !d_stamps_f32 && !d_feats_bf16 && !d_feats_f32) return fail(DT_E_ARG, "no output");
  if (!(da > 0.0) || !(dm > 0.0) || !std::isfinite(da) || !std::isfinite(dm))
    return fail(DT_E_DOMAIN, "cell half-widths da and dm must be finite and > 0");
  DeviceGuard guard(p->ctx->device);
  dt_ctx* c = p->ctx;
  if (p->n_exp > STAMP_MAX_EXP) return fail(DT_E_ARG, "cell stamps support at most %d exposures", STAMP_MAX_EXP);
  StackArgs a = stack_args(p, reps);
  hipError_t e = launch_cell_stamps(a, da, dm, d_stamps_bf16, d_stamps_f32, d_feats_bf16, d_feats_f32, c->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "cell stamps");
}

dt_status dt_gemm_bf16(dt_ctx* c, const uint16_t* d_A, int32_t lda, int32_t transA, const uint16_t* d_B,
                       int32_t ldb, int32_t transB, int32_t M, int32_t N, int32_t K, const float* d_bias,
                       int32_t relu, float* d_C, int32_t ldc) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  if (M < 0 || N < 0 || K < 1 || !d_A || !d_B || !d_C) return fail(DT_E_ARG, "bad GEMM shape or NULL pointer");
  if (ldc < N || lda < (transA ? M : K) || ldb < (transB ? K : N)) return fail(DT_E_ARG, "leading dimension too small");
  DeviceGuard guard(c->device);
  const size_t part_elems = (size_t)1 << 22;
  float* part = nullptr;
  dt_status st = ctx_alloc(c, (void**)&part, sizeof(float) * part_elems, "GEMM split-K scratch");
  if (st != DT_OK) return st;
  GemmArgs g{d_A, lda, transA ? 1 : 0, d_B, ldb, transB ? 1 : 0, M, N, K, d_bias, relu ? 1 : 0, d_C, ldc, nullptr, 0};
  hipError_t e = launch_gemm_bf16(g, part, part_elems, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  ctx_free(c, part, sizeof(float) * part_elems);
  return e == hipSuccess ? DT_OK : hip_fail(e, "GEMM");
}

dt_status dt_clip_candidates(dt_patch* p, const dt_orbits* orbits, const int64_t* d_ids, int64_t m, double kappa,
                             int32_t max_iter, float* d_snr, float* d_flux, int32_t* d_nkept) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  dt_status st = check_orbits(orbits);
  if (st != DT_OK) return st;
  if (m < 0 || (m > 0 && !d_ids)) return fail(DT_E_ARG, "bad id array");
  if (!(kappa > 0.0) || max_iter < 1) return fail(DT_E_ARG, "kappa must be > 0 and max_iter >= 1");
  if (p->n_exp > 512) return fail(DT_E_ARG, "outlier trimming supports at most 512 exposures per patch");
  if (m == 0) return DT_OK;
  DeviceGuard guard(p->ctx->device);
  dt_ctx* c = p->ctx;
  const size_t need = sizeof(float2) * (size_t)m * p->n_exp;
  float2* buf = nullptr;
  st = ctx_alloc(c, (void**)&buf, need, "outlier-trimming scratch");
  if (st != DT_OK) return st;
  StackArgs a = stack_args(p, orbits);
  hipError_t e = launch_clip(a, d_ids, m, kappa, max_iter, buf, d_snr, d_flux, d_nkept, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // the scratch is freed below
  ctx_free(c, buf, need);
  return e == hipSuccess ? DT_OK : hip_fail(e, "outlier trimming");
}

namespace {
dt_status check_sampler(const dt_orbit_sampler* S) {
  if (!S) return fail(DT_E_ARG, "sampler is NULL");
  const double* v[] = {&S->epoch, S->obs_xyz_au, S->center, S->east, S->north, &S->half_w, &S->half_h,
                       S->a_range, S->e_range, S->inc_range};
  const int nv[] = {1, 3, 3, 3, 3, 1, 1, 2, 2, 2};
  for (int k = 0; k < 10; ++k)
    for (int j = 0; j < nv[k]; ++j)
      if (!std::isfinite(v[k][j])) return fail(DT_E_DOMAIN, "sampler has a non-finite value");
  if (!(S->a_range[0] > 0.0 && S->a_range[1] >= S->a_range[0])) return fail(DT_E_DOMAIN, "bad a range");
  if (!(S->e_range[0] >= 0.0 && S->e_range[1] >= S->e_range[0] && S->e_range[1] < 1.0))
    return fail(DT_E_DOMAIN, "bad e range");
  if (!(S->inc_range[0] >= 0.0 && S->inc_range[1] >= S->inc_range[0])) return fail(DT_E_DOMAIN, "bad i range");
  if (!(S->half_w > 0.0 && S->half_h > 0.0)) return fail(DT_E_DOMAIN, "field half-widths must be > 0");
  return DT_OK;
}
}  // namespace

dt_status dt_generate_orbits(dt_ctx* c, const dt_orbit_sampler* S, int64_t first, int64_t n, double* d_a,
                             double* d_e, double* d_inc, double* d_node, double* d_peri, double* d_m0) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  dt_status st = check_sampler(S);
  if (st != DT_OK) return st;
  if (first < 0 || n < 0 || n >= ((int64_t)1 << 32)) return fail(DT_E_ARG, "need first >= 0 and 0 <= n < 2^32");
  if (n > 0 && (!d_a || !d_e || !d_inc || !d_node || !d_peri || !d_m0)) return fail(DT_E_ARG, "NULL output");
  DeviceGuard guard(c->device);
  hipError_t e = launch_generate(*S, first, n, d_a, d_e, d_inc, d_node, d_peri, d_m0, c->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "orbit generation");
}

// Generated-orbit calls of more than GEN_PROBE_MIN orbits run the first
// GEN_PROBE with the checkpoint walk; when at least GEN_PROBE_DEFER of its
// wavefronts defer, the rest go straight to the per-sample walk.  (The
// probe's read-back costs a stream synchronisation, under 1 % of a call
// this large.)
constexpr int64_t GEN_PROBE = (int64_t)1 << 22;
constexpr int64_t GEN_PROBE_MIN = (int64_t)1 << 26;
constexpr double GEN_PROBE_DEFER = 0.9;

dt_status dt_stack_generated(dt_patch* p, const dt_orbit_sampler* S, int64_t first, int64_t n, float* d_snr,
                             float* d_flux, int32_t* d_nvalid) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  dt_status st = check_sampler(S);
  if (st != DT_OK) return st;
  if (first < 0 || n < 0 || n >= ((int64_t)1 << 32)) return fail(DT_E_ARG, "bad first / n");
  DeviceGuard guard(p->ctx->device);
  StackArgs a{};
  a.meta = p->d_meta;
  a.n_exp = p->n_exp;
  a.planes = p->d_planes;
  a.n = n;
  a.epoch = S->epoch;
  a.vobs = p->vobs;
  a.work = p->ctx->count_work ? p->ctx->d_work : nullptr;
  a.snr = d_snr;
  a.flux = d_flux;
  a.nvalid = d_nvalid;
  if (n > 0 && p->vobs < __builtin_inf()) {
    st = defer_setup(p->ctx, n, a);
    if (st != DT_OK) return st;
  }
  if (n <= GEN_PROBE_MIN || !a.defer_list) {
    hipError_t e = launch_stack_generated(a, *S, first, p->ctx->stream);
    return e == hipSuccess ? DT_OK : hip_fail(e, "generate-and-stack launch");
  }
  // Probe: the first GEN_PROBE orbits with the checkpoint walk.  The orbits
  // of one sampler are alike, so the share of its wavefronts that defer
  // (read back once; a pure function of those orbits and the exposures)
  // picks the walk for the rest.
  StackArgs a1 = a;
  a1.n = GEN_PROBE;
  hipError_t e = launch_stack_generated(a1, *S, first, p->ctx->stream);
  unsigned int deferred = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&deferred, a.defer_count, sizeof(deferred), hipMemcpyDeviceToHost, p->ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "generate-and-stack probe");
  StackArgs a2 = a;
  a2.n = n - GEN_PROBE;
  if (a2.snr) a2.snr += GEN_PROBE;
  if (a2.flux) a2.flux += GEN_PROBE;
  if (a2.nvalid) a2.nvalid += GEN_PROBE;
  const bool walk = (double)deferred >= GEN_PROBE_DEFER * (double)(GEN_PROBE / 64);
  e = walk ? launch_stack_generated_walk(a2, *S, first + GEN_PROBE, p->ctx->stream)
           : launch_stack_generated(a2, *S, first + GEN_PROBE, p->ctx->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "generate-and-stack launch");
}

dt_status dt_segment_max(dt_ctx* c, const float* d_x, int64_t n_seg, int32_t seg, float* d_out) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  if (n_seg < 0 || seg < 1 || (n_seg > 0 && (!d_x || !d_out))) return fail(DT_E_ARG, "bad segments or arrays");
  DeviceGuard guard(c->device);
  hipError_t e = launch_segment_max(d_x, n_seg, seg, d_out, c->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "segment maximum");
}

dt_status dt_cell_members_near(dt_ctx* c, const dt_orbits* grid, const int64_t* d_cells, int64_t n_cells,
                               int32_t cell_size, const float* d_uv, int32_t uv_stride, double da, double dm,
                               double radius, int64_t* d_ids, int64_t* d_count) {
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  dt_status st = check_orbits(grid);
  if (st != DT_OK) return st;
  if (n_cells < 0 || (n_cells > 0 && (!d_cells || !d_uv || !d_ids))) return fail(DT_E_ARG, "bad cell or output array");
  if (!d_count) return fail(DT_E_ARG, "d_count is NULL");
  if (cell_size < 1 || uv_stride < 2) return fail(DT_E_ARG, "need cell_size >= 1 and uv_stride >= 2");
  if (n_cells * (int64_t)cell_size >= ((int64_t)1 << 40)) return fail(DT_E_ARG, "too many orbits");
  if (!(da > 0.0 && dm > 0.0 && radius >= 0.0)) return fail(DT_E_DOMAIN, "need da > 0, dm > 0, radius >= 0");
  DeviceGuard guard(c->device);
  StackArgs a{};
  a.n = grid->n;
  a.a = grid->a;
  a.m0 = grid->m0;
  hipError_t e = launch_cell_members_near(a, d_cells, n_cells, cell_size, d_uv, uv_stride, da, dm, radius, d_ids,
                                          d_count, c->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "cell member selection");
}

dt_status dt_stack_ids(dt_patch* p, const dt_orbits* orbits, const int64_t* d_ids, const int64_t* d_count,
                       int64_t m_max, float* d_snr, float* d_flux, int32_t* d_nvalid) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  dt_status st = check_orbits(orbits);
  if (st != DT_OK) return st;
  if (m_max < 0 || (m_max > 0 && (!d_ids || !d_count))) return fail(DT_E_ARG, "bad id list or count");
  DeviceGuard guard(p->ctx->device);
  StackArgs a = stack_args(p, orbits);
  a.snr = d_snr;
  a.flux = d_flux;
  a.nvalid = d_nvalid;
  if (m_max > STACK_IDS_SHORT && p->vobs < __builtin_inf()) {
    st = defer_setup(p->ctx, m_max, a);
    if (st != DT_OK) return st;
  }
  hipError_t e = launch_stack_ids(a, d_ids, d_count, m_max, p->ctx->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "id-list stack launch");
}

dt_status dt_stack_cells(dt_patch* p, const dt_orbits* grid, const int64_t* d_cells, int64_t n_cells,
                         int32_t cell_size, float* d_snr, float* d_flux, int32_t* d_nvalid) {
  if (!p || !p->ctx) return fail(DT_E_ARG, "invalid patch");
  dt_status st = check_orbits(grid);
  if (st != DT_OK) return st;
  if (n_cells < 0 || (n_cells > 0 && !d_cells)) return fail(DT_E_ARG, "bad cell list");
  if (cell_size < 1) return fail(DT_E_ARG, "cell_size must be >= 1");
  if (n_cells * (int64_t)cell_size >= ((int64_t)1 << 40)) return fail(DT_E_ARG, "too many orbits");
  DeviceGuard guard(p->ctx->device);
  StackArgs a = stack_args(p, grid);
  a.snr = d_snr;
  a.flux = d_flux;
  a.nvalid = d_nvalid;
  hipError_t e = launch_stack_cells(a, d_cells, n_cells, cell_size, p->ctx->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "cell stack launch");
}

}  // extern "C"
