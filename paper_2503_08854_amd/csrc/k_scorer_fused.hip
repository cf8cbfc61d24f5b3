// k_scorer_fused.hip -- inference forward of the cell scorer in one kernel.
//
// The same network and rounding points as the layer-by-layer path (every
// activation rounded to BF16 after bias and ReLU, FP32 accumulation on
// v_mfma_f32_16x16x16_bf16 in the same K order except that the 1152-deep
// layer sums two K halves, FP32 biases), with every intermediate kept in LDS.
// A workgroup of eight waves (two per SIMD, so one wave's MFMA and LDS
// latency overlaps the other's; the LDS holds one workgroup per CU) takes 16
// cells at a time and makes them the M dimension of every MFMA tile: a convolution
// output pixel is one 16 (cells) x 16 (channels) tile whose A operand reads
// the input pixel's 16-channel group of every cell (one 8-byte LDS read per
// lane), so all pixel and tap arithmetic is uniform across the wave.  The
// convolutions stream row by row through three-row ring buffers; the fully
// connected layers then run on the group's 16 rows.  Per cell only the
// 441 + 16 BF16 inputs are read and one FP32 logit is written.  Weights
// arrive transposed ([N][K], one block per layer) so that every B operand
// (four consecutive K of one output column) is one 8-byte load.
#include "dt_common.hpp"

namespace dtk {

namespace {
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// round to nearest even with the hardware conversion (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint16_t relu_bf(float v, float b) { return f2bf(fmaxf(v + b, 0.f)); }
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
// two values to BF16 in one hardware conversion (round to nearest even)
__device__ __forceinline__ uint32_t cvt2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(float2_t{a, b}, bf16x2_t));
}
__device__ __forceinline__ short4_t as4(uint2 v) {
  return short4_t{(short)(v.x & 0xffffu), (short)(v.x >> 16), (short)(v.y & 0xffffu), (short)(v.y >> 16)};
}
__device__ __forceinline__ short4_t ld4(const uint16_t* p) {  // 8-byte aligned read
  return as4(*reinterpret_cast<const uint2*>(p));
}
__device__ __forceinline__ float4_t mfma(short4_t a, short4_t b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// D tile rows 4 kq + r (cells), column r16: relu(d + bias) as BF16 into o[row * stride + r16]
__device__ __forceinline__ void store4(uint16_t* o, int kq, int r16, int stride, float4_t d, float bias) {
  const uint32_t p01 = cvt2(fmaxf(d[0] + bias, 0.f), fmaxf(d[1] + bias, 0.f));
  const uint32_t p23 = cvt2(fmaxf(d[2] + bias, 0.f), fmaxf(d[3] + bias, 0.f));
  o[(4 * kq + 0) * stride + r16] = (uint16_t)p01;
  o[(4 * kq + 1) * stride + r16] = (uint16_t)(p01 >> 16);
  o[(4 * kq + 2) * stride + r16] = (uint16_t)p23;
  o[(4 * kq + 3) * stride + r16] = (uint16_t)(p23 >> 16);
}

constexpr int G = 16;                        // cells per workgroup
constexpr int NW = 8;                        // waves per workgroup
constexpr int NTH = 64 * NW;                 // threads per workgroup
constexpr int W1K = 16, W2K = 148, W3K = 292;  // padded K strides of the conv weights in LDS
constexpr int FTS = 20, CTS = 132, H6S = 68;
constexpr int SPAD = 23 * 23;                // the stamp with a one-pixel zero border
}  // namespace

// wt[toff[i] + n * K_i + k] = wb[w_off[i] + k * N_i + n]
__global__ void k_scorer_transpose(const uint16_t* __restrict__ wb, uint16_t* __restrict__ wt, ScorerFusedArgs A,
                                   int total) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int l = 0;
  while (l < 6 && i >= A.t_off[l + 1]) ++l;
  const int r = i - (int)A.t_off[l];
  const int K = A.K[l], N = A.N[l];
  const int n = r / K, k = r % K;
  wt[i] = wb[A.w_off[l] + (int64_t)k * N + n];
}

template <bool ROWS>
__global__ __launch_bounds__(NTH) void k_scorer_fused(ScorerFusedArgs A) {
  // A workgroup owns 16 cells at a time; the cells are the M (row) dimension
  // of every MFMA tile, so all pixel / tap index arithmetic is uniform.
  // Activations are [pixel][cell][channel]; the convolutions stream by rows
  // with three-row ring buffers (a stride-2 3x3 layer needs three input rows
  // per output row), and only conv3's output is kept whole for FC4.
  __shared__ __align__(16) uint16_t w1s[16 * W1K];           // [n][k], k < 9 used
  __shared__ __align__(16) uint16_t w2s[32 * W2K];           // [n][k]
  __shared__ __align__(16) uint16_t w3s[32 * W3K];           // [n][k]
  __shared__ __align__(16) uint16_t stg[SPAD * G];           // stamps [pixel of the 23 x 23 zero-bordered stamp][cell]
  __shared__ __align__(16) uint16_t h1r[3 * 21 * G * 16];    // conv1 rows (ring of 3) [row][x][cell][16]
  __shared__ __align__(16) uint16_t h2r[3 * 11 * G * 32];    // conv2 rows (ring of 3) [row][x][cell][32]
  __shared__ __align__(16) uint16_t h3s[36 * G * 32];        // conv3 output [pixel][cell][32]
  __shared__ __align__(16) uint16_t ftg[G * FTS];
  __shared__ __align__(16) uint16_t cat[G * CTS];
  __shared__ __align__(16) uint16_t h6[G * H6S];
  __shared__ int srow[G];  // the group's rows of the inputs and logits
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const uint16_t* wt = A.wt;
  // conv weights into LDS, 8 bytes per load, all loads of a thread issued together
  {
    const uint2* g2 = reinterpret_cast<const uint2*>(wt + A.t_off[1]);  // 32 rows x 36 quads
    const uint2* g3 = reinterpret_cast<const uint2*>(wt + A.t_off[2]);  // 32 rows x 72 quads
    constexpr int Q2 = (32 * 36 + NTH - 1) / NTH, Q3 = (32 * 72 + NTH - 1) / NTH;
    uint2 v2[Q2], v3[Q3];
#pragma unroll
    for (int q = 0; q < Q2; ++q) {
      const int i = tid + NTH * q;
      v2[q] = i < 32 * 36 ? g2[i] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int q = 0; q < Q3; ++q) {
      const int i = tid + NTH * q;
      v3[q] = i < 32 * 72 ? g3[i] : make_uint2(0u, 0u);
    }
    uint16_t w1v = 0;
    if (tid < 16 * W1K) {
      const int n = tid / W1K, k = tid % W1K;
      w1v = k < 9 ? wt[A.t_off[0] + n * 9 + k] : (uint16_t)0;
    }
#pragma unroll
    for (int q = 0; q < Q2; ++q) {
      const int i = tid + NTH * q;
      if (i < 32 * 36) *reinterpret_cast<uint2*>(&w2s[(i / 36) * W2K + 4 * (i % 36)]) = v2[q];
    }
#pragma unroll
    for (int q = 0; q < Q3; ++q) {
      const int i = tid + NTH * q;
      if (i < 32 * 72) *reinterpret_cast<uint2*>(&w3s[(i / 72) * W3K + 4 * (i % 72)]) = v3[q];
    }
    if (tid < 16 * W1K) w1s[tid] = w1v;
  }
  const float* b1 = A.w + A.b_off[0];
  const float* b2 = A.w + A.b_off[1];
  const float* b3 = A.w + A.b_off[2];
  const float bias1 = b1[r16], bias2a = b2[r16], bias2b = b2[16 + r16], bias3a = b3[r16], bias3b = b3[16 + r16];
  float* red = reinterpret_cast<float*>(h1r);  // FC4 partial sums (h1r is free by then)
  // this lane's conv1 taps k = 4 kq + i as LDS offsets into the bordered
  // stamp (taps 9..15 are padding: zero)
  int toff[4];
  bool tapv[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = 4 * kq + i;
    tapv[i] = k < 9;
    toff[i] = (k < 9 ? ((k / 3) * 23 + k % 3) * G : 0) + r16;
  }
  // the zero border (never written below)
  for (int i = tid; i < SPAD * G; i += NTH) stg[i] = 0;
  const int n_groups = (A.B + G - 1) / G;
  for (int grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    __syncthreads();  // the previous group's readers of stg / h3s / cat / h6 / srow are done; weights loaded
    const int cell0 = grp * G;
    if (ROWS) {
      if (tid < G) srow[tid] = cell0 + tid < A.B ? (int)A.rows[cell0 + tid] : 0;
      __syncthreads();
    }
    {
      // the group's stamps: all loads of a thread issued together, then stored [pixel][cell]
      constexpr int NQ = (441 * G + NTH - 1) / NTH;
      uint16_t v[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = tid + NTH * q;
        const int c = i / 441;
        const bool in = i < 441 * G && cell0 + c < A.B;
        v[q] = in ? A.stamps[ROWS ? (int64_t)srow[c] * 441 + (i - 441 * c) : (int64_t)cell0 * 441 + i] : (uint16_t)0;
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int i = tid + NTH * q;
        const int px = i % 441;
        if (i < 441 * G) stg[((px / 21 + 1) * 23 + px % 21 + 1) * G + i / 441] = v[q];
      }
    }
    for (int i = tid; i < G * 16; i += NTH) {
      const int r = i / 16, c = i % 16;
      ftg[r * FTS + c] = cell0 + r < A.B ? A.feats[(ROWS ? (int64_t)srow[r] : (int64_t)(cell0 + r)) * 16 + c]
                                         : (uint16_t)0;
    }
    __syncthreads();
    const short4_t bw1 = ld4(&w1s[r16 * W1K + 4 * kq]);
    int h1_done = 0;  // conv1 rows computed so far
    for (int oy2 = 0; oy2 < 11; ++oy2) {
      // conv1 rows up to 2 oy2 + 1: pixel (y, x) of the row is one 16 x 16 tile, wave w takes x = w, w + NW, ...
      const int need = min(21, 2 * oy2 + 2);
      for (int y = h1_done; y < need; ++y) {
        for (int x = wave; x < 21; x += NW) {
          // output pixel (y, x) reads bordered pixels (y + dy, x + dx), dy, dx in 0..2
          const uint16_t* b = stg + (y * 23 + x) * G;
          short v[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = tapv[i] ? (short)b[toff[i]] : (short)0;
          const short4_t a = short4_t{v[0], v[1], v[2], v[3]};
          const float4_t d = mfma(a, bw1, float4_t{0.f, 0.f, 0.f, 0.f});
          uint16_t* o = h1r + ((y % 3) * 21 + x) * (G * 16);
          store4(o, kq, r16, 16, d, bias1);
        }
      }
      h1_done = need;
      __syncthreads();
      // conv2 row oy2: 11 pixels x 2 column tiles, wave w takes units w, w + NW, ...; K step s = tap s
      for (int u = wave; u < 22; u += NW) {
        const int ox = u >> 1, nt = u & 1;
        float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 9; ++s) {
          const int iy = 2 * oy2 + s / 3 - 1, ix = 2 * ox + s % 3 - 1;
          short4_t a = short4_t{0, 0, 0, 0};
          if ((unsigned)iy < 21u && (unsigned)ix < 21u) a = ld4(&h1r[((iy % 3) * 21 + ix) * (G * 16) + r16 * 16 + 4 * kq]);
          acc = mfma(a, ld4(&w2s[(16 * nt + r16) * W2K + s * 16 + 4 * kq]), acc);
        }
        uint16_t* o = h2r + ((oy2 % 3) * 11 + ox) * (G * 32);
        store4(o + 16 * nt, kq, r16, 32, acc, nt ? bias2b : bias2a);
      }
      __syncthreads();
      // conv3 row oy3 once conv2 rows up to 2 oy3 + 1 exist: 6 pixels x 2 column tiles
      if ((oy2 & 1) || oy2 == 10) {
        const int oy3 = oy2 == 10 ? 5 : (oy2 - 1) / 2;
        for (int u = wave; u < 12; u += NW) {
          const int ox = u >> 1, nt = u & 1;
          float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < 9; ++s) {
            const int iy = 2 * oy3 + s / 3 - 1, ix = 2 * ox + s % 3 - 1;
            const bool in = (unsigned)iy < 11u && (unsigned)ix < 11u;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              short4_t a = short4_t{0, 0, 0, 0};
              if (in) a = ld4(&h2r[((iy % 3) * 11 + ix) * (G * 32) + r16 * 32 + 16 * h + 4 * kq]);
              acc = mfma(a, ld4(&w3s[(16 * nt + r16) * W3K + s * 32 + 16 * h + 4 * kq]), acc);
            }
          }
          const float bias3 = nt ? bias3b : bias3a;
          store4(h3s + (oy3 * 6 + ox) * (G * 32) + 16 * nt, kq, r16, 32, acc, bias3);
        }
        __syncthreads();
      }
    }
    // FC4 (1152 -> 64; K = pixel * 32 + channel) and FC5 (16 -> 64): waves w and w + 4 own columns
    // 16w .. 16w + 15 and K steps 0..35 and 36..71; the second half's partial sums go through LDS
    {
      const int ct = wave & 3, kh = wave >> 2;
      const int n = 16 * ct + r16;
      const uint16_t* w4 = wt + A.t_off[3] + (int64_t)n * 1152;
      float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
      for (int s0 = 36 * kh; s0 < 36 * kh + 36; s0 += 18) {
        short4_t b[18];
#pragma unroll
        for (int u = 0; u < 18; ++u) b[u] = ld4(&w4[(s0 + u) * 16 + 4 * kq]);
#pragma unroll
        for (int u = 0; u < 18; ++u) {
          const int s = s0 + u;
          acc = mfma(ld4(&h3s[((s >> 1) * G + r16) * 32 + (s & 1) * 16 + 4 * kq]), b[u], acc);
        }
      }
      if (kh) {
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(ct * 4 + r) * 64 + lane] = acc[r];
      }
      __syncthreads();
      if (kh == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] += red[(ct * 4 + r) * 64 + lane];
        const float bias4 = A.w[A.b_off[3] + n];
#pragma unroll
        for (int r = 0; r < 4; ++r) cat[(4 * kq + r) * CTS + n] = f2bf(fmaxf(acc[r] + bias4, 0.f));
        const short4_t b5 = ld4(wt + A.t_off[4] + (int64_t)n * 16 + 4 * kq);
        const float4_t d5 = mfma(ld4(&ftg[r16 * FTS + 4 * kq]), b5, float4_t{0.f, 0.f, 0.f, 0.f});
        const float bias5 = A.w[A.b_off[4] + n];
#pragma unroll
        for (int r = 0; r < 4; ++r) cat[(4 * kq + r) * CTS + 64 + n] = f2bf(fmaxf(d5[r] + bias5, 0.f));
      }
    }
    __syncthreads();
    // FC6 (128 -> 64): waves 0..3
    if (wave < 4) {
      const int n = 16 * wave + r16;
      const uint16_t* w6 = wt + A.t_off[5] + (int64_t)n * 128;
      short4_t b[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) b[s] = ld4(&w6[s * 16 + 4 * kq]);
      float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 8; ++s) acc = mfma(ld4(&cat[r16 * CTS + s * 16 + 4 * kq]), b[s], acc);
      const float bias6 = A.w[A.b_off[5] + n];
#pragma unroll
      for (int r = 0; r < 4; ++r) h6[(4 * kq + r) * H6S + n] = f2bf(fmaxf(acc[r] + bias6, 0.f));
    }
    __syncthreads();
    // FC7 (64 -> 1), no ReLU: one wave, column 0 of a 16-wide tile
    if (wave == 0) {
      const uint16_t* w7 = wt + A.t_off[6];
      float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = s * 16 + 4 * kq;
        const short4_t b = r16 == 0 ? ld4(&w7[k]) : short4_t{0, 0, 0, 0};
        acc = mfma(ld4(&h6[r16 * H6S + k]), b, acc);
      }
      if (r16 == 0) {
        const float bias7 = A.w[A.b_off[6]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int cell = cell0 + 4 * kq + r;
          if (cell < A.B) A.z[ROWS ? (int64_t)srow[4 * kq + r] : (int64_t)cell] = acc[r] + bias7;
        }
      }
    }
  }
}

hipError_t launch_scorer_fused(const ScorerFusedArgs& a, bool transpose, hipStream_t s) {
  if (a.B <= 0) return hipSuccess;
  const int total = (int)a.t_off[7];
  if (transpose)
    hipLaunchKernelGGL(k_scorer_transpose, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a.wb, a.wt, a,
                       total);
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const int groups = (a.B + G - 1) / G;
  const int grid = groups < n_cu ? groups : n_cu;
  if (a.rows)
    hipLaunchKernelGGL(k_scorer_fused<true>, dim3((unsigned)grid), dim3(NTH), 0, s, a);
  else
    hipLaunchKernelGGL(k_scorer_fused<false>, dim3((unsigned)grid), dim3(NTH), 0, s, a);
  return hipGetLastError();
}

}  // namespace dtk
