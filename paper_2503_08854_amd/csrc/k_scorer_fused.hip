// k_scorer_fused.hip -- inference forward of the cell scorer in one kernel.
//
// The same network and rounding points as the layer-by-layer path (every
// activation rounded to BF16 after bias and ReLU, FP32 accumulation on
// v_mfma_f32_16x16x16_bf16, FP32 biases), but with every intermediate kept in
// LDS: a workgroup of four waves owns a group of 16 cells; each wave runs the
// three convolutions of four cells as small GEMMs whose A operands are read
// straight out of the channels-last activation in LDS (a 3x3 tap with 16
// input channels is one 16-deep K step, four channels per lane = one 8-byte
// read), and the fully connected layers then run with the 16 cells as the M
// dimension of the MFMA tiles.  Per cell only the 441 + 16 BF16 inputs are
// read and one FP32 logit is written.
//
// Weights arrive transposed ([N][K], one block per layer) so that every B
// operand (four consecutive K of one output column) is one 8-byte load.  The
// four-channel groups of a pixel are stored XOR-swizzled by pixel so that the
// stride-2 convolutions, whose lanes read every other pixel, spread over the
// LDS banks.
#include "dt_common.hpp"

namespace dtk {

namespace {
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// round to nearest even with the hardware conversion (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint16_t relu_bf(float v, float b) { return f2bf(fmaxf(v + b, 0.f)); }
__device__ __forceinline__ short4_t as4(uint2 v) {
  return short4_t{(short)(v.x & 0xffffu), (short)(v.x >> 16), (short)(v.y & 0xffffu), (short)(v.y >> 16)};
}
__device__ __forceinline__ short4_t ld4(const uint16_t* p) {  // 8-byte aligned read
  return as4(*reinterpret_cast<const uint2*>(p));
}
__device__ __forceinline__ float4_t mfma(short4_t a, short4_t b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// LDS writes of a wave visible to all its lanes
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// swizzled channels-last addresses (elements): 16 and 32 channels per pixel
__device__ __forceinline__ int h1a(int p, int c) { return p * 16 + (((c >> 2) ^ ((p >> 1) & 3)) << 2) + (c & 3); }
__device__ __forceinline__ int h2a(int p, int c) { return p * 32 + (((c >> 2) ^ ((p >> 1) & 7)) << 2) + (c & 3); }

constexpr int G = 16;                        // cells per workgroup
constexpr int W1K = 16, W2K = 148, W3K = 292;  // padded K strides of the conv weights in LDS
constexpr int H3S = 1156, FTS = 20, CTS = 132, H6S = 68;
constexpr int SPW = 7;                       // stamp values per lane (441 = 64 * 7 - 7)
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

__global__ __launch_bounds__(256) void k_scorer_fused(ScorerFusedArgs A) {
  __shared__ __align__(16) uint16_t w1s[16 * W1K];       // [n][k], k < 9 used
  __shared__ __align__(16) uint16_t w2s[32 * W2K];       // [n][k]
  __shared__ __align__(16) uint16_t w3s[32 * W3K];       // [n][k]
  __shared__ __align__(16) uint16_t h1s[4][441 * 16];    // per wave, channels-last, swizzled
  __shared__ __align__(16) uint16_t h2s[4][121 * 32];    // per wave; holds the stamp during conv1
  __shared__ __align__(16) uint16_t h3g[G * H3S];        // the group's flattened conv3 outputs
  __shared__ __align__(16) uint16_t ftg[G * FTS];
  __shared__ __align__(16) uint16_t cat[G * CTS];
  __shared__ __align__(16) uint16_t h6[G * H6S];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const uint16_t* wt = A.wt;
  for (int i = tid; i < 16 * W1K; i += 256) {
    const int n = i / W1K, k = i % W1K;
    w1s[i] = k < 9 ? wt[A.t_off[0] + n * 9 + k] : (uint16_t)0;
  }
  for (int i = tid; i < 32 * W2K; i += 256) {
    const int n = i / W2K, k = i % W2K;
    w2s[i] = k < 144 ? wt[A.t_off[1] + n * 144 + k] : (uint16_t)0;
  }
  for (int i = tid; i < 32 * W3K; i += 256) {
    const int n = i / W3K, k = i % W3K;
    w3s[i] = k < 288 ? wt[A.t_off[2] + n * 288 + k] : (uint16_t)0;
  }
  const float* b1 = A.w + A.b_off[0];
  const float* b2 = A.w + A.b_off[1];
  const float* b3 = A.w + A.b_off[2];
  const float bias1 = b1[r16], bias2a = b2[r16], bias2b = b2[16 + r16], bias3a = b3[r16], bias3b = b3[16 + r16];
  const int n_groups = (A.B + G - 1) / G;
  uint16_t* h1 = h1s[wave];
  uint16_t* h2 = h2s[wave];
  uint16_t* st = h2s[wave];  // the stamp lives where h2 will be written
  // stamp of the next cell this wave handles, prefetched into registers
  uint16_t nxt[SPW];
  auto fetch = [&](int cell) {
#pragma unroll
    for (int q = 0; q < SPW; ++q) {
      const int i = lane + 64 * q;
      nxt[q] = (cell < A.B && i < 441) ? A.stamps[(int64_t)cell * 441 + i] : (uint16_t)0;
    }
  };
  fetch(blockIdx.x * G + wave * (G / 4));
  for (int grp = blockIdx.x; grp < n_groups; grp += gridDim.x) {
    __syncthreads();  // previous group's FC reads of h3g / cat / h6 are done; weights are loaded
    const int cell0 = grp * G;
    for (int i = tid; i < G * 16; i += 256) {
      const int r = i / 16, c = i % 16;
      ftg[r * FTS + c] = cell0 + r < A.B ? A.feats[(int64_t)(cell0 + r) * 16 + c] : (uint16_t)0;
    }
    for (int cc = 0; cc < G / 4; ++cc) {
      const int slot = wave * (G / 4) + cc;
      const int cell = cell0 + slot;
      uint16_t* h3 = h3g + slot * H3S;
#pragma unroll
      for (int q = 0; q < SPW; ++q)
        if (lane + 64 * q < 441) st[lane + 64 * q] = nxt[q];
      // prefetch the following cell (next slot of this group, or this wave's first slot of its next group)
      fetch(cc + 1 < G / 4 ? cell + 1 : (grp + gridDim.x) * G + wave * (G / 4));
      if (cell >= A.B) {  // a missing cell of the last group: zero inputs to the FC layers
        for (int i = lane; i < 1152; i += 64) h3[i] = 0;
        continue;
      }
      wave_sync();
      // conv1: [441 x 9] x [9 x 16], one K step (taps 9..15 zero); this lane's
      // taps k = 4 kq + i are fixed, its output pixel advances by 16 per tile
      const short4_t bw1 = ld4(&w1s[r16 * W1K + 4 * kq]);
      int dy[4], dx[4];
      bool tap[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 4 * kq + i;
        tap[i] = k < 9;
        dy[i] = k / 3 - 1;
        dx[i] = k % 3 - 1;
      }
      int oy = 0, ox = r16;
      for (int mt = 0; mt < 28; ++mt) {
        const bool live = mt * 16 + r16 < 441;
        short v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int iy = oy + dy[i], ix = ox + dx[i];
          v[i] = (live && tap[i] && (unsigned)iy < 21u && (unsigned)ix < 21u) ? (short)st[iy * 21 + ix] : (short)0;
        }
        const float4_t d = mfma(short4_t{v[0], v[1], v[2], v[3]}, bw1, float4_t{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int mo = mt * 16 + 4 * kq + r;
          if (mo < 441) h1[h1a(mo, r16)] = relu_bf(d[r], bias1);
        }
        ox += 16;
        if (ox >= 21) {
          ox -= 21;
          ++oy;
        }
      }
      wave_sync();
      // conv2: stride 2 -> 11 x 11, [121 x 144] x [144 x 32]; K step s = tap s, 16 channels
      for (int mt = 0; mt < 8; ++mt) {
        const int m = mt * 16 + r16;
        const int oy = m / 11, ox = m % 11;
        float4_t acc0 = float4_t{0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
        short4_t a[9];
#pragma unroll
        for (int s = 0; s < 9; ++s) {
          const int iy = 2 * oy + s / 3 - 1, ix = 2 * ox + s % 3 - 1;
          const int p = iy * 21 + ix;
          a[s] = (m < 121 && iy >= 0 && iy < 21 && ix >= 0 && ix < 21) ? ld4(&h1[h1a(p, 4 * kq)])
                                                                       : short4_t{0, 0, 0, 0};
        }
#pragma unroll
        for (int s = 0; s < 9; ++s) {
          acc0 = mfma(a[s], ld4(&w2s[r16 * W2K + s * 16 + 4 * kq]), acc0);
          acc1 = mfma(a[s], ld4(&w2s[(16 + r16) * W2K + s * 16 + 4 * kq]), acc1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int mo = mt * 16 + 4 * kq + r;
          if (mo < 121) {
            h2[h2a(mo, r16)] = relu_bf(acc0[r], bias2a);
            h2[h2a(mo, 16 + r16)] = relu_bf(acc1[r], bias2b);
          }
        }
      }
      wave_sync();
      // conv3: stride 2 -> 6 x 6, [36 x 288] x [288 x 32]; K steps: tap s, channel half h
      for (int mt = 0; mt < 3; ++mt) {
        const int m = mt * 16 + r16;
        const int oy = m / 6, ox = m % 6;
        float4_t acc0 = float4_t{0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
        for (int s = 0; s < 9; ++s) {
          const int iy = 2 * oy + s / 3 - 1, ix = 2 * ox + s % 3 - 1;
          const bool in = m < 36 && iy >= 0 && iy < 11 && ix >= 0 && ix < 11;
          const int p = iy * 11 + ix;
          short4_t a[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) a[h] = in ? ld4(&h2[h2a(p, 16 * h + 4 * kq)]) : short4_t{0, 0, 0, 0};
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int k = s * 32 + 16 * h + 4 * kq;
            acc0 = mfma(a[h], ld4(&w3s[r16 * W3K + k]), acc0);
            acc1 = mfma(a[h], ld4(&w3s[(16 + r16) * W3K + k]), acc1);
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int mo = mt * 16 + 4 * kq + r;
          if (mo < 36) {
            h3[mo * 32 + r16] = relu_bf(acc0[r], bias3a);
            h3[mo * 32 + 16 + r16] = relu_bf(acc1[r], bias3b);
          }
        }
      }
      wave_sync();
    }
    __syncthreads();
    // FC4 (1152 -> 64) and FC5 (16 -> 64): wave w owns output columns 16w .. 16w + 15
    {
      const int n = 16 * wave + r16;
      const uint16_t* w4 = wt + A.t_off[3] + (int64_t)n * 1152;
      float4_t acc = float4_t{0.f, 0.f, 0.f, 0.f};
      for (int s0 = 0; s0 < 72; s0 += 8) {
        short4_t b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = ld4(&w4[(s0 + u) * 16 + 4 * kq]);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = mfma(ld4(&h3g[r16 * H3S + (s0 + u) * 16 + 4 * kq]), b[u], acc);
      }
      const float bias4 = A.w[A.b_off[3] + n];
#pragma unroll
      for (int r = 0; r < 4; ++r) cat[(4 * kq + r) * CTS + n] = f2bf(fmaxf(acc[r] + bias4, 0.f));
      const short4_t b5 = ld4(wt + A.t_off[4] + (int64_t)n * 16 + 4 * kq);
      const float4_t d5 = mfma(ld4(&ftg[r16 * FTS + 4 * kq]), b5, float4_t{0.f, 0.f, 0.f, 0.f});
      const float bias5 = A.w[A.b_off[4] + n];
#pragma unroll
      for (int r = 0; r < 4; ++r) cat[(4 * kq + r) * CTS + 64 + n] = f2bf(fmaxf(d5[r] + bias5, 0.f));
    }
    __syncthreads();
    // FC6 (128 -> 64)
    {
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
          if (cell < A.B) A.z[cell] = acc[r] + bias7;
        }
      }
    }
  }
}

hipError_t launch_scorer_fused(const ScorerFusedArgs& a, hipStream_t s) {
  if (a.B <= 0) return hipSuccess;
  const int total = (int)a.t_off[7];
  hipLaunchKernelGGL(k_scorer_transpose, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a.wb, a.wt, a,
                     total);
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const int groups = (a.B + G - 1) / G;
  const int grid = groups < n_cu ? groups : n_cu;
  hipLaunchKernelGGL(k_scorer_fused, dim3((unsigned)grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace dtk
