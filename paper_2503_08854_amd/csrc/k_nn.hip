// k_nn.hip -- kernels of the learned cell scorer: a BF16 MFMA GEMM (used for
// every convolution via im2col and every fully connected layer, forward and
// backward), im2col / col2im, ReLU masks, bias gradients, the binary
// cross-entropy loss, Adam and parameter initialisation.
//
// GEMM: C[M x N] = op(A)[M x K] op(B)[K x N], A and B bfloat16, FP32
// accumulation on gfx950's v_mfma_f32_16x16x32_bf16.  A workgroup of four
// waves owns a 64 x 64 tile of C (each wave 32 x 32 = 2 x 2 MFMA tiles); K
// advances in steps of 32 (one MFMA per tile) through LDS tiles stored
// K-contiguous so that every lane's MFMA operand (eight consecutive K values)
// is one 16-byte LDS read.  A lane's A and B operands cover the same eight K
// indices, so the products the instruction pairs are those of one K.  Split-K writes
// FP32 partial tiles that a second kernel sums in a fixed order, so results
// are deterministic.
#include "dt_common.hpp"

namespace dtk {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even (NaN kept quiet)
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

constexpr int GT_M = 64, GT_N = 64, GT_K = 32;

// Partial GEMM over k in [k0, k1).  Output: if part != null, raw FP32 tile to
// part (ldc = N); otherwise the epilogue (bias, ReLU, FP32 and/or BF16 out).
__global__ __launch_bounds__(256) void k_gemm_bf16(const uint16_t* __restrict__ A, int lda, int transA,
                                                   const uint16_t* __restrict__ B, int ldb, int transB, int M,
                                                   int N, int K, int k_per_split, float* __restrict__ part,
                                                   const float* __restrict__ bias, int relu, float* __restrict__ Cf,
                                                   int ldcf, uint16_t* __restrict__ Cb, int ldcb) {
  // [m][k] and [n][k]; rows of 80 bytes keep every 8-element operand 16-byte aligned
  __shared__ __attribute__((aligned(16))) uint16_t sA[GT_M][GT_K + 8];
  __shared__ __attribute__((aligned(16))) uint16_t sB[GT_N][GT_K + 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * GT_M, n0 = blockIdx.y * GT_N;
  const int kb = blockIdx.z * k_per_split;
  const int ke = min(K, kb + k_per_split);
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  float4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += GT_K) {
    // stage A (64 x 32) and B (32 x 64): 2048 elements each, 8 per thread
    // consecutive threads walk the dimension that is contiguous in memory
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = tid + q * 256;
      int r, c;  // r: m (or n), c: k
      if (!transA) { r = idx >> 5; c = idx & 31; } else { c = idx >> 6; r = idx & 63; }
      const int gm = m0 + r, gk = k0 + c;
      uint16_t va = 0;
      if (gm < M && gk < ke) va = transA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      sA[r][c] = va;
      if (transB) { r = idx >> 5; c = idx & 31; } else { c = idx >> 6; r = idx & 63; }
      const int gn = n0 + r, gk2 = k0 + c;
      uint16_t vb = 0;
      if (gn < N && gk2 < ke) vb = transB ? B[(int64_t)gn * ldb + gk2] : B[(int64_t)gk2 * ldb + gn];
      sB[r][c] = vb;
    }
    __syncthreads();
    {
      const int kk = 8 * (lane >> 4);
      bf16x8_t a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = *(const bf16x8_t*)&sA[wm + 16 * i + (lane & 15)][kk];
        b[i] = *(const bf16x8_t*)&sB[wn + 16 * i + (lane & 15)][kk];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout: lane holds column (lane & 15), rows 4 * (lane >> 4) + r
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int gn = n0 + wn + 16 * j + (lane & 15);
        if (gm >= M || gn >= N) continue;
        float v = acc[i][j][r];
        if (part) {
          part[((int64_t)blockIdx.z * M + gm) * N + gn] = v;
          continue;
        }
        if (bias) v += bias[gn];
        if (relu) v = fmaxf(v, 0.f);
        if (Cf) Cf[(int64_t)gm * ldcf + gn] = v;
        if (Cb) Cb[(int64_t)gm * ldcb + gn] = f2bf(v);
      }
}

__global__ void k_splitk_reduce(const float* __restrict__ part, int splits, int M, int N,
                                const float* __restrict__ bias, int relu, float* __restrict__ Cf, int ldcf,
                                uint16_t* __restrict__ Cb, int ldcb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const int gm = (int)(i / N), gn = (int)(i % N);
  float v = 0.f;
  for (int s = 0; s < splits; ++s) v += part[(int64_t)s * M * N + i];
  if (bias) v += bias[gn];
  if (relu) v = fmaxf(v, 0.f);
  if (Cf) Cf[(int64_t)gm * ldcf + gn] = v;
  if (Cb) Cb[(int64_t)gm * ldcb + gn] = f2bf(v);
}

hipError_t launch_gemm_bf16(const GemmArgs& g, float* d_part, size_t part_elems, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int gm = (g.M + GT_M - 1) / GT_M, gn = (g.N + GT_N - 1) / GT_N;
  int splits = 1;
  // split long K so that small outputs still fill the machine
  while (splits < 256 && (int64_t)gm * gn * splits < 512 && g.K / (splits * 2) >= 256) splits *= 2;
  if (splits > 1 && (size_t)splits * g.M * g.N > part_elems) splits = 1;
  int kps = ((g.K + splits - 1) / splits + GT_K - 1) / GT_K * GT_K;
  splits = kps > 0 ? (g.K + kps - 1) / kps : 1;
  if (splits < 1) splits = 1;
  if (splits == 1) {
    hipLaunchKernelGGL(k_gemm_bf16, dim3(gm, gn, 1), dim3(256), 0, s, g.A, g.lda, g.transA, g.B, g.ldb, g.transB,
                       g.M, g.N, g.K, g.K > 0 ? ((g.K + GT_K - 1) / GT_K) * GT_K : GT_K, nullptr, g.bias, g.relu,
                       g.Cf, g.ldcf, g.Cb, g.ldcb);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_gemm_bf16, dim3(gm, gn, splits), dim3(256), 0, s, g.A, g.lda, g.transA, g.B, g.ldb,
                     g.transB, g.M, g.N, g.K, kps, d_part, nullptr, 0, nullptr, 0, nullptr, 0);
  const int64_t mn = (int64_t)g.M * g.N;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, d_part, splits, g.M, g.N,
                     g.bias, g.relu, g.Cf, g.ldcf, g.Cb, g.ldcb);
  return hipGetLastError();
}

// im2col of a channels-last BF16 tensor for a 3x3, pad-1 convolution:
// cols[(b, oy, ox)][(ky * 3 + kx) * C + c].
__global__ void k_im2col(const uint16_t* __restrict__ x, int Bn, int H, int W, int C, int stride, int Ho, int Wo,
                         uint16_t* __restrict__ cols) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)Bn * Ho * Wo * 9 * C;
  if (i >= total) return;
  const int kc = (int)(i % (9 * C));
  const int64_t p = i / (9 * C);
  const int ox = (int)(p % Wo), oy = (int)((p / Wo) % Ho), b = (int)(p / ((int64_t)Wo * Ho));
  const int tap = kc / C, c = kc % C;
  const int iy = oy * stride + tap / 3 - 1, ix = ox * stride + tap % 3 - 1;
  uint16_t v = 0;
  if (iy >= 0 && iy < H && ix >= 0 && ix < W) v = x[(((int64_t)b * H + iy) * W + ix) * C + c];
  cols[i] = v;
}

// col2im (adjoint of im2col) with the ReLU mask of the layer input applied
// and a BF16 copy for the next GEMM: each input element gathers the (at most
// nine) column entries that read it, in a fixed order.
__global__ void k_col2im_mask(const float* __restrict__ dcols, int Bn, int H, int W, int C, int stride, int Ho,
                              int Wo, const uint16_t* __restrict__ act, uint16_t* __restrict__ dx_bf,
                              float* __restrict__ dx_f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)Bn * H * W * C;
  if (i >= total) return;
  const int c = (int)(i % C);
  const int64_t p = i / C;
  const int ix = (int)(p % W), iy = (int)((p / W) % H), b = (int)(p / ((int64_t)W * H));
  float v = 0.f;
  for (int ky = 0; ky < 3; ++ky) {
    const int ty = iy + 1 - ky;
    if (ty < 0 || ty % stride) continue;
    const int oy = ty / stride;
    if (oy >= Ho) continue;
    for (int kx = 0; kx < 3; ++kx) {
      const int tx = ix + 1 - kx;
      if (tx < 0 || tx % stride) continue;
      const int ox = tx / stride;
      if (ox >= Wo) continue;
      v += dcols[(((int64_t)b * Ho + oy) * Wo + ox) * 9 * C + (ky * 3 + kx) * C + c];
    }
  }
  if (!(bf2f(act[i]) > 0.f)) v = 0.f;
  dx_bf[i] = f2bf(v);
  if (dx_f) dx_f[i] = v;
}

// d_pre = d_out * (act > 0), as BF16 (act is the post-ReLU BF16 activation);
// src has leading dimension lds, act and dst are dense [M x N].
__global__ void k_relu_mask(const float* __restrict__ src, int lds, const uint16_t* __restrict__ act, int lda,
                            int M, int N, uint16_t* __restrict__ dst, float* __restrict__ dst_f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const int m = (int)(i / N), n = (int)(i % N);
  float v = src[(int64_t)m * lds + n];
  if (!(bf2f(act[(int64_t)m * lda + n]) > 0.f)) v = 0.f;
  dst[i] = f2bf(v);
  if (dst_f) dst_f[i] = v;
}

// Column sums (bias gradients) of a dense FP32 [M x N] matrix, fixed order.
__global__ void k_colsum(const float* __restrict__ d, int M, int N, float* __restrict__ out) {
  const int n = blockIdx.x;
  __shared__ float red[256];
  float v = 0.f;
  for (int m = threadIdx.x; m < M; m += 256) v += d[(int64_t)m * N + n];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = red[0];
}

// Mean binary cross-entropy of logits z against labels y, and dL/dz.
__global__ void k_bce(const float* __restrict__ z, const float* __restrict__ y, int Bn, float* __restrict__ loss,
                      float* __restrict__ dz, uint16_t* __restrict__ dz_bf) {
  __shared__ float red[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < Bn; i += 256) {
    const float zi = z[i], yi = y[i];
    acc += fmaxf(zi, 0.f) - zi * yi + log1pf(expf(-fabsf(zi)));
    const float g = (1.f / (1.f + expf(-zi)) - yi) / (float)Bn;
    dz[i] = g;
    dz_bf[i] = f2bf(g);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / (float)Bn;
}

// Adam (Kingma & Ba) on FP32 master weights, refreshing the BF16 copy.
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2, uint16_t* __restrict__ w_bf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  w_bf[i] = f2bf(wi);
}

__global__ void k_cast_bf16(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// He-normal weights (std sqrt(2 / fan_in)) and zero biases from a counter-based
// generator: splitmix64 of (seed, index) -> two uniforms -> Box-Muller.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__global__ void k_init_params(float* __restrict__ w, int64_t off, int64_t n, int fan_in, uint64_t seed,
                              int is_bias) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (is_bias) {
    w[off + i] = 0.f;
    return;
  }
  const uint64_t r = splitmix64(seed ^ splitmix64((uint64_t)(off + i)));
  const double u1 = ((double)(r >> 11) + 1.0) * (1.0 / 9007199254740993.0);
  const double u2 = (double)(splitmix64(r) >> 11) * (1.0 / 9007199254740992.0);
  const double z = sqrt(-2.0 * log(u1)) * cos(2.0 * PI * u2);
  w[off + i] = (float)(z * sqrt(2.0 / fan_in));
}

static unsigned g1d(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_im2col(const uint16_t* x, int Bn, int H, int W, int C, int stride, int Ho, int Wo, uint16_t* cols,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_im2col, dim3(g1d((int64_t)Bn * Ho * Wo * 9 * C)), dim3(256), 0, s, x, Bn, H, W, C, stride, Ho,
                     Wo, cols);
  return hipGetLastError();
}
hipError_t launch_col2im_mask(const float* dcols, int Bn, int H, int W, int C, int stride, int Ho, int Wo,
                              const uint16_t* act, uint16_t* dx, float* dx_f, hipStream_t s) {
  hipLaunchKernelGGL(k_col2im_mask, dim3(g1d((int64_t)Bn * H * W * C)), dim3(256), 0, s, dcols, Bn, H, W, C, stride,
                     Ho, Wo, act, dx, dx_f);
  return hipGetLastError();
}
hipError_t launch_relu_mask(const float* src, int lds, const uint16_t* act, int lda, int M, int N, uint16_t* dst,
                            float* dst_f, hipStream_t s) {
  hipLaunchKernelGGL(k_relu_mask, dim3(g1d((int64_t)M * N)), dim3(256), 0, s, src, lds, act, lda, M, N, dst, dst_f);
  return hipGetLastError();
}
hipError_t launch_colsum(const float* d, int M, int N, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3(N), dim3(256), 0, s, d, M, N, out);
  return hipGetLastError();
}
hipError_t launch_bce(const float* z, const float* y, int Bn, float* loss, float* dz, uint16_t* dz_bf, hipStream_t s) {
  hipLaunchKernelGGL(k_bce, dim3(1), dim3(256), 0, s, z, y, Bn, loss, dz, dz_bf);
  return hipGetLastError();
}
hipError_t launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, int64_t t, uint16_t* w_bf,
                       hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - pow(0.9, (double)t)), c2 = (float)(1.0 - pow(0.999, (double)t));
  hipLaunchKernelGGL(k_adam, dim3(g1d(n)), dim3(256), 0, s, w, m, v, g, n, lr, b1, b2, 1e-8f, c1, c2, w_bf);
  return hipGetLastError();
}
hipError_t launch_cast_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_bf16, dim3(g1d(n)), dim3(256), 0, s, x, n, y);
  return hipGetLastError();
}
hipError_t launch_init_params(float* w, int64_t off, int64_t n, int fan_in, uint64_t seed, int is_bias,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_init_params, dim3(g1d(n)), dim3(256), 0, s, w, off, n, fan_in, seed, is_bias);
  return hipGetLastError();
}

}  // namespace dtk
