// dt_nn.cpp -- the learned cell scorer: a small CNN over 21x21 coarse-stacked
// stamps plus an MLP over per-cell features, trained and evaluated entirely by
// this library's HIP kernels (BF16 MFMA GEMMs, FP32 master weights, Adam).
//
// Architecture (activations channels-last, weights [K, N] row-major with
// K = (ky * 3 + kx) * C_in + c_in for 3x3 convolutions, zero padding 1):
//   stamp 21x21x1 -> conv s1 (16) -> ReLU -> conv s2 (32) -> ReLU (11x11)
//                 -> conv s2 (32) -> ReLU (6x6) -> FC 1152->64 -> ReLU = h_img
//   features 16   -> FC 16->64 -> ReLU = h_feat
//   [h_img, h_feat] -> FC 128->64 -> ReLU -> FC 64->1 = logit
// Loss: mean binary cross-entropy of the logit.
#include "dt_internal.hpp"

namespace dtk {
namespace {

struct Layer {
  int64_t w, b;  // offsets in the parameter vector
  int K, N;      // weight shape [K, N]
};
// w1 b1 w2 b2 w3 b3 w4 b4 w5 b5 w6 b6 w7 b7
constexpr int NL = 7;
constexpr int LK[NL] = {9, 144, 288, 1152, 16, 128, 64};
constexpr int LN[NL] = {16, 32, 32, 64, 64, 64, 1};

int64_t layer_table(Layer* L) {
  int64_t off = 0;
  for (int i = 0; i < NL; ++i) {
    L[i].K = LK[i];
    L[i].N = LN[i];
    L[i].w = off;
    off += (int64_t)LK[i] * LN[i];
    L[i].b = off;
    off += LN[i];
  }
  return off;
}

}  // namespace
}  // namespace dtk

using namespace dtk;

struct dt_scorer {
  dt_ctx* ctx = nullptr;
  int max_b = 0;
  Layer L[NL];
  int64_t np = 0;
  int64_t step = 0;
  std::vector<std::pair<void*, size_t>> allocs;
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t* wb = nullptr;
  // activations (BF16) and backward buffers
  uint16_t *col1, *h1, *col2, *h2, *col3, *h3, *cat, *h6;
  uint16_t* wt = nullptr;  // transposed BF16 weights for the fused inference kernel
  int64_t wver = 0;        // bumped whenever wb is rewritten
  int64_t wt_ver = -1;     // the wb version wt was transposed from
  float* z;
  float *dz, *df, *dbig, *dmid;
  uint16_t *dz_b, *d_b, *d_mid_b;
  float* part;
  size_t part_elems = 0;
  float* loss_tmp = nullptr;
};

namespace {

template <typename T>
dt_status salloc(dt_scorer* s, T** p, size_t count, const char* what) {
  dt_status st = ctx_alloc(s->ctx, (void**)p, sizeof(T) * count, what);
  if (st == DT_OK) s->allocs.push_back({(void*)*p, sizeof(T) * count});
  return st;
}

void sfree(dt_scorer* s) {
  for (auto& a : s->allocs) ctx_free(s->ctx, a.first, a.second);
  s->allocs.clear();
}

hipError_t gemm(dt_scorer* s, const uint16_t* A, int lda, int tA, const uint16_t* B, int ldb, int tB, int M, int N,
                int K, const float* bias, int relu, float* Cf, int ldcf, uint16_t* Cb, int ldcb) {
  GemmArgs g{A, lda, tA, B, ldb, tB, M, N, K, bias, relu, Cf, ldcf, Cb, ldcb};
  return launch_gemm_bf16(g, s->part, s->part_elems, s->ctx->stream);
}

// Forward pass for B samples; logits (FP32) to z (or out if given).
hipError_t forward(dt_scorer* s, const uint16_t* stamps, const uint16_t* feats, int B, float* out) {
  hipStream_t st = s->ctx->stream;
  const Layer* L = s->L;
  hipError_t e = launch_im2col(stamps, B, 21, 21, 1, 1, 21, 21, s->col1, st);
  if (e == hipSuccess)
    e = gemm(s, s->col1, 9, 0, s->wb + L[0].w, 16, 0, B * 441, 16, 9, s->w + L[0].b, 1, nullptr, 0, s->h1, 16);
  if (e == hipSuccess) e = launch_im2col(s->h1, B, 21, 21, 16, 2, 11, 11, s->col2, st);
  if (e == hipSuccess)
    e = gemm(s, s->col2, 144, 0, s->wb + L[1].w, 32, 0, B * 121, 32, 144, s->w + L[1].b, 1, nullptr, 0, s->h2, 32);
  if (e == hipSuccess) e = launch_im2col(s->h2, B, 11, 11, 32, 2, 6, 6, s->col3, st);
  if (e == hipSuccess)
    e = gemm(s, s->col3, 288, 0, s->wb + L[2].w, 32, 0, B * 36, 32, 288, s->w + L[2].b, 1, nullptr, 0, s->h3, 32);
  if (e == hipSuccess)
    e = gemm(s, s->h3, 1152, 0, s->wb + L[3].w, 64, 0, B, 64, 1152, s->w + L[3].b, 1, nullptr, 0, s->cat, 128);
  if (e == hipSuccess)
    e = gemm(s, feats, 16, 0, s->wb + L[4].w, 64, 0, B, 64, 16, s->w + L[4].b, 1, nullptr, 0, s->cat + 64, 128);
  if (e == hipSuccess)
    e = gemm(s, s->cat, 128, 0, s->wb + L[5].w, 64, 0, B, 64, 128, s->w + L[5].b, 1, nullptr, 0, s->h6, 64);
  if (e == hipSuccess)
    e = gemm(s, s->h6, 64, 0, s->wb + L[6].w, 1, 0, B, 1, 64, s->w + L[6].b, 0, out ? out : s->z, 1, nullptr, 0);
  return e;
}

// Backward pass (after forward with the same inputs): gradients into grad.
hipError_t backward(dt_scorer* s, const uint16_t* feats, const float* labels, int B, float* loss, float* grad) {
  hipStream_t st = s->ctx->stream;
  const Layer* L = s->L;
  hipError_t e = launch_bce(s->z, labels, B, loss ? loss : s->loss_tmp, s->dz, s->dz_b, st);
  // FC7: dW7 = h6^T dz, db7 = sum dz, dh6 = dz W7^T
  if (e == hipSuccess) e = gemm(s, s->h6, 64, 1, s->dz_b, 1, 0, 64, 1, B, nullptr, 0, grad + L[6].w, 1, nullptr, 0);
  if (e == hipSuccess) e = launch_colsum(s->dz, B, 1, grad + L[6].b, st);
  if (e == hipSuccess) e = gemm(s, s->dz_b, 1, 0, s->wb + L[6].w, 1, 1, B, 64, 1, nullptr, 0, s->dbig, 64, nullptr, 0);
  if (e == hipSuccess) e = launch_relu_mask(s->dbig, 64, s->h6, 64, B, 64, s->d_b, s->df, st);
  // FC6: dW6 = cat^T d6, db6, dcat = d6 W6^T
  if (e == hipSuccess) e = gemm(s, s->cat, 128, 1, s->d_b, 64, 0, 128, 64, B, nullptr, 0, grad + L[5].w, 64, nullptr, 0);
  if (e == hipSuccess) e = launch_colsum(s->df, B, 64, grad + L[5].b, st);
  if (e == hipSuccess) e = gemm(s, s->d_b, 64, 0, s->wb + L[5].w, 64, 1, B, 128, 64, nullptr, 0, s->dbig, 128, nullptr, 0);
  // split into the image branch (columns 0..63) and the feature branch (64..127)
  if (e == hipSuccess) e = launch_relu_mask(s->dbig, 128, s->cat, 128, B, 64, s->d_b, s->df, st);
  if (e == hipSuccess) e = launch_relu_mask(s->dbig + 64, 128, s->cat + 64, 128, B, 64, s->d_mid_b, s->dmid, st);
  // FC5: dW5 = feats^T d5, db5
  if (e == hipSuccess) e = gemm(s, feats, 16, 1, s->d_mid_b, 64, 0, 16, 64, B, nullptr, 0, grad + L[4].w, 64, nullptr, 0);
  if (e == hipSuccess) e = launch_colsum(s->dmid, B, 64, grad + L[4].b, st);
  // FC4: dW4 = h3^T d4, db4, dh3 = d4 W4^T
  if (e == hipSuccess) e = gemm(s, s->h3, 1152, 1, s->d_b, 64, 0, 1152, 64, B, nullptr, 0, grad + L[3].w, 64, nullptr, 0);
  if (e == hipSuccess) e = launch_colsum(s->df, B, 64, grad + L[3].b, st);
  if (e == hipSuccess) e = gemm(s, s->d_b, 64, 0, s->wb + L[3].w, 64, 1, B, 1152, 64, nullptr, 0, s->dbig, 1152, nullptr, 0);
  if (e == hipSuccess) e = launch_relu_mask(s->dbig, 1152, s->h3, 1152, B, 1152, s->d_b, s->df, st);
  // conv3: dW3 = col3^T d3, db3, dcol3 = d3 W3^T, col2im -> dh2 (masked)
  if (e == hipSuccess) e = gemm(s, s->col3, 288, 1, s->d_b, 32, 0, 288, 32, B * 36, nullptr, 0, grad + L[2].w, 32, nullptr, 0);
  if (e == hipSuccess) e = launch_colsum(s->df, B * 36, 32, grad + L[2].b, st);
  if (e == hipSuccess) e = gemm(s, s->d_b, 32, 0, s->wb + L[2].w, 32, 1, B * 36, 288, 32, nullptr, 0, s->dbig, 288, nullptr, 0);
  if (e == hipSuccess) e = launch_col2im_mask(s->dbig, B, 11, 11, 32, 2, 6, 6, s->h2, s->d_mid_b, s->dmid, st);
  // conv2: dW2 = col2^T d2, db2, dcol2 = d2 W2^T, col2im -> dh1 (masked)
  if (e == hipSuccess) e = gemm(s, s->col2, 144, 1, s->d_mid_b, 32, 0, 144, 32, B * 121, nullptr, 0, grad + L[1].w, 32, nullptr, 0);
  if (e == hipSuccess) e = launch_colsum(s->dmid, B * 121, 32, grad + L[1].b, st);
  if (e == hipSuccess) e = gemm(s, s->d_mid_b, 32, 0, s->wb + L[1].w, 32, 1, B * 121, 144, 32, nullptr, 0, s->dbig, 144, nullptr, 0);
  if (e == hipSuccess) e = launch_col2im_mask(s->dbig, B, 21, 21, 16, 2, 11, 11, s->h1, s->d_b, s->df, st);
  // conv1: dW1 = col1^T d1, db1
  if (e == hipSuccess) e = gemm(s, s->col1, 9, 1, s->d_b, 16, 0, 9, 16, B * 441, nullptr, 0, grad + L[0].w, 16, nullptr, 0);
  if (e == hipSuccess) e = launch_colsum(s->df, B * 441, 16, grad + L[0].b, st);
  return e;
}

dt_status check_io(dt_scorer* s, const uint16_t* stamps, const uint16_t* feats, int B) {
  if (!s || !s->ctx) return fail(DT_E_ARG, "invalid scorer");
  if (B < 1 || B > s->max_b) return fail(DT_E_ARG, "batch %d outside [1, %d]", B, s->max_b);
  if (!stamps || !feats) return fail(DT_E_ARG, "NULL input");
  return DT_OK;
}

}  // namespace

extern "C" {

int64_t dt_scorer_num_params(void) {
  Layer L[NL];
  return layer_table(L);
}

dt_status dt_scorer_create(dt_ctx* c, int32_t max_batch, uint64_t seed, dt_scorer** out) {
  if (!out) return fail(DT_E_ARG, "out is NULL");
  *out = nullptr;
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  if (max_batch < 1 || max_batch > 32768) return fail(DT_E_ARG, "max_batch must be in [1, 32768]");
  DeviceGuard guard(c->device);
  dt_scorer* s = new dt_scorer();
  s->ctx = c;
  s->max_b = max_batch;
  s->np = layer_table(s->L);
  const size_t B = (size_t)max_batch;
  s->part_elems = (size_t)1 << 22;
  dt_status st = DT_OK;
  auto A = [&](auto** p, size_t n, const char* what) {
    if (st == DT_OK) st = salloc(s, p, n, what);
  };
  A(&s->w, s->np, "scorer weights");
  A(&s->m, s->np, "scorer Adam m");
  A(&s->v, s->np, "scorer Adam v");
  A(&s->g, s->np, "scorer gradients");
  A(&s->wb, s->np, "scorer BF16 weights");
  A(&s->wt, s->np, "scorer transposed BF16 weights");
  A(&s->col1, B * 441 * 9, "scorer col1");
  A(&s->h1, B * 441 * 16, "scorer h1");
  A(&s->col2, B * 121 * 144, "scorer col2");
  A(&s->h2, B * 121 * 32, "scorer h2");
  A(&s->col3, B * 36 * 288, "scorer col3");
  A(&s->h3, B * 1152, "scorer h3");
  A(&s->cat, B * 128, "scorer cat");
  A(&s->h6, B * 64, "scorer h6");
  A(&s->z, B, "scorer logits");
  A(&s->dz, B, "scorer dz");
  A(&s->dz_b, B, "scorer dz bf16");
  A(&s->df, B * 441 * 16, "scorer grad f32");
  A(&s->d_b, B * 441 * 16, "scorer grad bf16");
  A(&s->dmid, B * 121 * 32, "scorer grad mid f32");
  A(&s->d_mid_b, B * 121 * 32, "scorer grad mid bf16");
  A(&s->dbig, B * 121 * 144, "scorer dcols");
  A(&s->part, s->part_elems, "scorer split-K");
  A(&s->loss_tmp, 1, "scorer loss");
  if (st != DT_OK) {
    sfree(s);
    delete s;
    return st;
  }
  hipError_t e = hipSuccess;
  for (int i = 0; i < NL && e == hipSuccess; ++i) {
    e = launch_init_params(s->w, s->L[i].w, (int64_t)s->L[i].K * s->L[i].N, s->L[i].K, seed, 0, c->stream);
    if (e == hipSuccess) e = launch_init_params(s->w, s->L[i].b, s->L[i].N, 1, seed, 1, c->stream);
  }
  if (e == hipSuccess) e = hipMemsetAsync(s->m, 0, sizeof(float) * s->np, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->v, 0, sizeof(float) * s->np, c->stream);
  if (e == hipSuccess) e = launch_cast_bf16(s->w, s->np, s->wb, c->stream);
  s->wver++;
  if (e != hipSuccess) {
    sfree(s);
    delete s;
    return hip_fail(e, "scorer init");
  }
  *out = s;
  return DT_OK;
}

dt_status dt_scorer_destroy(dt_scorer* s) {
  if (!s || !s->ctx) return fail(DT_E_ARG, "invalid scorer");
  DeviceGuard guard(s->ctx->device);
  (void)hipStreamSynchronize(s->ctx->stream);
  sfree(s);
  s->ctx = nullptr;
  delete s;
  return DT_OK;
}

dt_status dt_scorer_get_params(dt_scorer* s, float* d_out) {
  if (!s || !s->ctx || !d_out) return fail(DT_E_ARG, "invalid scorer or NULL output");
  DeviceGuard guard(s->ctx->device);
  hipError_t e = hipMemcpyAsync(d_out, s->w, sizeof(float) * s->np, hipMemcpyDeviceToDevice, s->ctx->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "scorer params copy");
}

dt_status dt_scorer_set_params(dt_scorer* s, const float* d_in) {
  if (!s || !s->ctx || !d_in) return fail(DT_E_ARG, "invalid scorer or NULL input");
  DeviceGuard guard(s->ctx->device);
  hipStream_t st = s->ctx->stream;
  hipError_t e = hipMemcpyAsync(s->w, d_in, sizeof(float) * s->np, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(s->m, 0, sizeof(float) * s->np, st);
  if (e == hipSuccess) e = hipMemsetAsync(s->v, 0, sizeof(float) * s->np, st);
  if (e == hipSuccess) e = launch_cast_bf16(s->w, s->np, s->wb, st);
  s->wver++;
  s->step = 0;
  return e == hipSuccess ? DT_OK : hip_fail(e, "scorer set params");
}

dt_status dt_scorer_forward(dt_scorer* s, const uint16_t* d_stamps, const uint16_t* d_feats, int32_t B,
                            float* d_logits) {
  dt_status st = check_io(s, d_stamps, d_feats, B);
  if (st != DT_OK) return st;
  if (!d_logits) return fail(DT_E_ARG, "NULL logits");
  DeviceGuard guard(s->ctx->device);
  hipError_t e = forward(s, d_stamps, d_feats, B, nullptr);
  if (e == hipSuccess) e = hipMemcpyAsync(d_logits, s->z, sizeof(float) * B, hipMemcpyDeviceToDevice, s->ctx->stream);
  return e == hipSuccess ? DT_OK : hip_fail(e, "scorer forward");
}

dt_status dt_scorer_infer(dt_scorer* s, const uint16_t* d_stamps, const uint16_t* d_feats, int32_t B,
                          float* d_logits) {
  return dt_scorer_infer_rows(s, d_stamps, d_feats, nullptr, B, d_logits);
}

dt_status dt_scorer_infer_rows(dt_scorer* s, const uint16_t* d_stamps, const uint16_t* d_feats,
                               const int64_t* d_rows, int32_t B, float* d_logits) {
  if (!s || !s->ctx) return fail(DT_E_ARG, "invalid scorer");
  if (B < 0) return fail(DT_E_ARG, "B < 0");
  if (B == 0) return DT_OK;
  if (!d_stamps || !d_feats || !d_logits) return fail(DT_E_ARG, "NULL input or output");
  DeviceGuard guard(s->ctx->device);
  ScorerFusedArgs a{};
  a.stamps = d_stamps;
  a.feats = d_feats;
  a.B = B;
  a.wb = s->wb;
  a.w = s->w;
  int64_t t = 0;
  for (int i = 0; i < NL; ++i) {
    a.w_off[i] = s->L[i].w;
    a.b_off[i] = s->L[i].b;
    a.K[i] = s->L[i].K;
    a.N[i] = s->L[i].N;
    a.t_off[i] = t;
    t += (int64_t)s->L[i].K * s->L[i].N;
  }
  a.t_off[NL] = t;
  a.wt = s->wt;
  a.z = d_logits;
  a.rows = d_rows;
  // the transposed weights are rebuilt only after the weights changed
  hipError_t e = launch_scorer_fused(a, s->wt_ver != s->wver, s->ctx->stream);
  if (e != hipSuccess) return hip_fail(e, "scorer inference");
  s->wt_ver = s->wver;
  return DT_OK;
}

dt_status dt_scorer_grad(dt_scorer* s, const uint16_t* d_stamps, const uint16_t* d_feats, const float* d_labels,
                         int32_t B, float* d_loss, float* d_grad) {
  dt_status st = check_io(s, d_stamps, d_feats, B);
  if (st != DT_OK) return st;
  if (!d_labels) return fail(DT_E_ARG, "NULL labels");
  DeviceGuard guard(s->ctx->device);
  hipError_t e = forward(s, d_stamps, d_feats, B, nullptr);
  if (e == hipSuccess) e = backward(s, d_feats, d_labels, B, d_loss, d_grad ? d_grad : s->g);
  return e == hipSuccess ? DT_OK : hip_fail(e, "scorer gradient");
}

dt_status dt_scorer_train_step(dt_scorer* s, const uint16_t* d_stamps, const uint16_t* d_feats,
                               const float* d_labels, int32_t B, float lr, float* d_loss) {
  dt_status st = check_io(s, d_stamps, d_feats, B);
  if (st != DT_OK) return st;
  if (!d_labels || !(lr > 0.f)) return fail(DT_E_ARG, "NULL labels or non-positive learning rate");
  DeviceGuard guard(s->ctx->device);
  hipError_t e = forward(s, d_stamps, d_feats, B, nullptr);
  if (e == hipSuccess) e = backward(s, d_feats, d_labels, B, d_loss, s->g);
  if (e == hipSuccess) e = launch_adam(s->w, s->m, s->v, s->g, s->np, lr, ++s->step, s->wb, s->ctx->stream);
  s->wver++;
  return e == hipSuccess ? DT_OK : hip_fail(e, "scorer train step");
}

}  // extern "C"
