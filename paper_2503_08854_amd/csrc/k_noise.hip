// k_noise.hip -- per-image noise sigma by an iterated median absolute
// deviation (Sec. 3): S = finite pixels; m = median(S),
// sigma = 1.4826 median{|x - m| : x in S}; S' = {finite x : |x - m| <=
// kappa sigma}; repeat until S' == S or max_iter steps.  The median of an
// even count is the mean of the two middle values.
//
// Exact selection by radix select: the two middle ranks are found digit by
// digit (11-bit digits) over an order-preserving integer key -- the float
// bits for x, the double bits of |x - m| (non-negative, so the raw bits
// order) for the deviations.  Every pass re-reads the image and builds an
// LDS histogram of the digit among the pixels that match the prefix chosen so
// far; a one-block pick kernel per image scans it.  The set S is never
// stored: membership is the predicate |x - m_cur| <= thr_cur evaluated in
// FP64, the same arithmetic for every pass, so selection, clipping and the
// change test are exact and the result equals the FP64 definition.
//
// Passes per step: the median's second and third digits (its first is
// histogrammed by the previous step's clip pass, which already knows the
// next set), the deviation key's first two digits, then one pass that both
// histograms its third digit and compacts the few keys that share the
// chosen 22-bit prefix into a per-image list; its last three digits come
// from that list (or from the image again if the list overflows), and one
// clip pass: six image reads per step instead of ten.
#include <algorithm>

#include "dt_common.hpp"

namespace dtk {

constexpr int NZ_BITS = 11;
constexpr int NZ_BINS = 1 << NZ_BITS;
constexpr int NZ_TX = 256;

template <typename T>
__device__ __forceinline__ float nz_load(const void* p, int64_t k);
template <>
__device__ __forceinline__ float nz_load<float>(const void* p, int64_t k) {
  return static_cast<const float*>(p)[k];
}
template <>
__device__ __forceinline__ float nz_load<_Float16>(const void* p, int64_t k) {
  return (float)static_cast<const _Float16*>(p)[k];
}

__device__ __forceinline__ uint64_t fkey(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint64_t)((u & 0x80000000u) ? ~u : (u | 0x80000000u));
}
__device__ __forceinline__ double fkey_value(uint64_t k) {
  const uint32_t u = (uint32_t)k;
  return (double)__uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ bool in_set(float x, const NoiseState& S) {
  return __builtin_isfinite(x) && fabs((double)x - S.m_cur) <= S.thr_cur;
}

__global__ void k_noise_init(NoiseState* st, uint32_t* hist, int n_img) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nh = (int64_t)n_img * 2 * NZ_BINS;
  if (i < nh) hist[i] = 0u;
  if (i < n_img) {
    NoiseState z{};
    z.m_cur = 0.0;
    z.thr_cur = __builtin_inf();
    z.sigma = __builtin_nan("");
    st[i] = z;
  }
}

template <typename T>
__global__ __launch_bounds__(NZ_TX) void k_noise_count(const void* const* imgs, const int64_t* npix, NoiseState* st) {
  const int img = blockIdx.y;
  const void* X = imgs[img];
  const int64_t n = npix[img];
  uint64_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * NZ_TX + threadIdx.x; i < n; i += (int64_t)gridDim.x * NZ_TX)
    c += __builtin_isfinite(nz_load<T>(X, i)) ? 1u : 0u;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd((unsigned long long*)&st[img].n, (unsigned long long)c);
}

// Start of a step: ranks of the two middle elements of the current set.
__device__ __forceinline__ void begin_select(NoiseState& S) {
  S.rank[0] = (S.n - 1) / 2;
  S.rank[1] = S.n / 2;
  S.prefix[0] = S.prefix[1] = 0;
}

__global__ void k_noise_begin(NoiseState* st, int n_img) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_img) return;
  NoiseState& S = st[i];
  if (S.n <= 0) {
    S.done = 1;
    return;
  }
  begin_select(S);
}

// One digit pass.  KIND 0: key of x; KIND 1: bits of |x - m_new|.
// SRC 0: the image; SRC 1: the image, and keys sharing the prefix above
// this digit are also appended to the image's list; SRC 2: the list (or the
// image when the list overflowed).
template <typename T, int KIND, int SRC>
__global__ __launch_bounds__(NZ_TX) void k_noise_hist(const void* const* imgs, const int64_t* npix, NoiseState* st,
                                                     uint32_t* hist, uint64_t* lists, int lo, int nb) {
  const int img = blockIdx.y;
  const NoiseState S = st[img];
  if (S.done) return;
  __shared__ uint32_t h[2][NZ_BINS];
  const bool two = S.prefix[0] != S.prefix[1];
  for (int b = threadIdx.x; b < 2 * NZ_BINS; b += NZ_TX) (&h[0][0])[b] = 0u;
  __syncthreads();
  const int hi = lo + nb;  // <= 63 for both key kinds
  const uint64_t p0 = S.prefix[0] >> hi, p1 = S.prefix[1] >> hi;
  const uint32_t mask = (1u << nb) - 1u;
  uint64_t* list = lists + (int64_t)img * NOISE_LIST_CAP;
  auto take = [&](uint64_t key) {
    const uint32_t d = (uint32_t)(key >> lo) & mask;
    const uint64_t top = key >> hi;
    if (top == p0) atomicAdd(&h[0][d], 1u);
    if (two && top == p1) atomicAdd(&h[1][d], 1u);
    return top == p0 || (two && top == p1);
  };
  if (SRC == 2 && S.n_list <= NOISE_LIST_CAP) {
    for (int64_t i = (int64_t)blockIdx.x * NZ_TX + threadIdx.x; i < S.n_list; i += (int64_t)gridDim.x * NZ_TX)
      (void)take(list[i]);
  } else {
    const void* X = imgs[img];
    const int64_t n = npix[img];
    for (int64_t i0 = (int64_t)blockIdx.x * NZ_TX; i0 < n; i0 += (int64_t)gridDim.x * NZ_TX) {
      const int64_t i = i0 + threadIdx.x;
      bool keep = false;
      uint64_t key = 0;
      if (i < n) {
        const float x = nz_load<T>(X, i);
        if (in_set(x, S)) {
          key = KIND == 0 ? fkey(x) : (uint64_t)__double_as_longlong(fabs((double)x - S.m_new));
          keep = take(key);
        }
      }
      if (SRC == 1) {
        // one atomic per wave for the list position of its kept keys
        const uint64_t ball = __ballot(keep);
        if (ball) {
          const int lane = threadIdx.x & 63;
          int64_t base = 0;
          if (lane == 0)
            base = (int64_t)atomicAdd((unsigned long long*)&st[img].n_list, (unsigned long long)__popcll(ball));
          base = __shfl(base, 0);
          if (keep) {
            const int64_t pos = base + __popcll(ball & ((1ull << lane) - 1ull));
            if (pos < NOISE_LIST_CAP) list[pos] = key;
          }
        }
      }
    }
  }
  __syncthreads();
  uint32_t* g = hist + (int64_t)img * 2 * NZ_BINS;
  for (int b = threadIdx.x; b < NZ_BINS; b += NZ_TX) {
    if (h[0][b]) atomicAdd(&g[b], h[0][b]);
    if (two && h[1][b]) atomicAdd(&g[NZ_BINS + b], h[1][b]);
  }
}

// Choose the digit holding each target rank; one block per image.
__global__ __launch_bounds__(NZ_TX) void k_noise_pick(NoiseState* st, uint32_t* hist, int lo, int kind) {
  constexpr int PER = NZ_BINS / NZ_TX;
  const int img = blockIdx.x;
  NoiseState& S = st[img];
  if (S.done) return;
  __shared__ uint64_t part[NZ_TX];
  __shared__ int dig[2];
  __shared__ uint64_t below[2];
  const bool two = S.prefix[0] != S.prefix[1];
  uint32_t* g = hist + (int64_t)img * 2 * NZ_BINS;
  const int tid = threadIdx.x;
  for (int t = 0; t < 2; ++t) {
    const uint32_t* H = g + (two ? t : 0) * NZ_BINS;
    uint64_t loc[PER];
    uint64_t s = 0;
    for (int j = 0; j < PER; ++j) {
      loc[j] = H[tid * PER + j];
      s += loc[j];
    }
    part[tid] = s;
    __syncthreads();
    // inclusive scan (Hillis-Steele over 256 entries)
    for (int o = 1; o < NZ_TX; o <<= 1) {
      const uint64_t v = tid >= o ? part[tid - o] : 0;
      __syncthreads();
      part[tid] += v;
      __syncthreads();
    }
    const uint64_t r = (uint64_t)S.rank[t];
    const uint64_t start = part[tid] - s;
    if (r >= start && r < part[tid]) {
      uint64_t c = start;
      for (int j = 0; j < PER; ++j) {
        if (r < c + loc[j]) {
          dig[t] = tid * PER + j;
          below[t] = c;
          break;
        }
        c += loc[j];
      }
    }
    __syncthreads();
  }
  for (int b = tid; b < 2 * NZ_BINS; b += NZ_TX) g[b] = 0u;
  if (tid == 0) {
    for (int t = 0; t < 2; ++t) {
      S.prefix[t] |= (uint64_t)dig[t] << lo;
      S.rank[t] -= (int64_t)below[t];
    }
    if (lo == 0) {
      for (int t = 0; t < 2; ++t)
        S.val[t] = kind == 0 ? fkey_value(S.prefix[t]) : __longlong_as_double((long long)S.prefix[t]);
    }
  }
}

// Median found: m_new, then select the deviations over the same set.
__global__ void k_noise_mid(NoiseState* st, int n_img) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_img) return;
  NoiseState& S = st[i];
  if (S.done) return;
  S.m_new = 0.5 * (S.val[0] + S.val[1]);
  S.n_list = 0;
  begin_select(S);
}

__global__ void k_noise_sigma(NoiseState* st, int n_img, double kappa) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_img) return;
  NoiseState& S = st[i];
  if (S.done) return;
  const double mad = 0.5 * (S.val[0] + S.val[1]);
  S.sigma = 1.4826 * mad;
  S.thr_new = kappa * S.sigma;
  S.n_used = S.n;
  S.iter += 1;
  S.n_new = 0;
  S.changed = 0;
}

// Size of the clipped set and whether any pixel changed membership; also the
// histogram of the first median digit (top 11 bits of the float key) over
// the clipped set, which is the next step's set if the step is repeated.
template <typename T>
__global__ __launch_bounds__(NZ_TX) void k_noise_clip(const void* const* imgs, const int64_t* npix, NoiseState* st,
                                                     uint32_t* hist) {
  const int img = blockIdx.y;
  const NoiseState S = st[img];
  if (S.done) return;
  __shared__ uint32_t h[NZ_BINS];
  for (int b = threadIdx.x; b < NZ_BINS; b += NZ_TX) h[b] = 0u;
  __syncthreads();
  const void* X = imgs[img];
  const int64_t n = npix[img];
  uint64_t c = 0;
  int ch = 0;
  for (int64_t i = (int64_t)blockIdx.x * NZ_TX + threadIdx.x; i < n; i += (int64_t)gridDim.x * NZ_TX) {
    const float x = nz_load<T>(X, i);
    if (!__builtin_isfinite(x)) continue;
    const double xd = (double)x;
    const bool k_old = fabs(xd - S.m_cur) <= S.thr_cur;
    const bool k_new = fabs(xd - S.m_new) <= S.thr_new;
    c += k_new ? 1u : 0u;
    ch |= (k_old != k_new) ? 1 : 0;
    if (k_new) atomicAdd(&h[(uint32_t)(fkey(x) >> 21) & (NZ_BINS - 1)], 1u);
  }
  for (int o = 32; o > 0; o >>= 1) {
    c += __shfl_xor(c, o);
    ch |= __shfl_xor(ch, o);
  }
  if ((threadIdx.x & 63) == 0) {
    if (c) atomicAdd((unsigned long long*)&st[img].n_new, (unsigned long long)c);
    if (ch) atomicOr(&st[img].changed, 1);
  }
  __syncthreads();
  uint32_t* g = hist + (int64_t)img * 2 * NZ_BINS;
  for (int b = threadIdx.x; b < NZ_BINS; b += NZ_TX)
    if (h[b]) atomicAdd(&g[b], h[b]);
}

__global__ void k_noise_update(NoiseState* st, int n_img, int max_iter) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_img) return;
  NoiseState& S = st[i];
  if (S.done) return;
  if (!S.changed || S.iter >= max_iter || S.n_new <= 0) {
    S.done = 1;
    return;
  }
  S.m_cur = S.m_new;
  S.thr_cur = S.thr_new;
  S.n = S.n_new;
  begin_select(S);
}

__global__ void k_noise_out(const NoiseState* st, int n_img, double* sigma, int64_t* n_used, int32_t* iters,
                            ExpMeta* meta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_img) return;
  if (sigma) sigma[i] = st[i].sigma;
  if (n_used) n_used[i] = st[i].n_used;
  if (iters) iters[i] = st[i].iter;
  if (meta) {
    // meta is in epoch order; meta[i].src names the image
    const double s = st[meta[i].src].sigma;
    meta[i].vs = (float)(s * s);
  }
}

size_t noise_scratch_bytes(int n_img) {
  return (sizeof(NoiseState) + 2 * NZ_BINS * sizeof(uint32_t) + NOISE_LIST_CAP * sizeof(uint64_t)) * (size_t)n_img;
}

template <typename T>
static hipError_t noise_t(const void* const* d_imgs, const int64_t* d_npix, int64_t max_pix, int n_img, double kappa,
                          int max_iter, void* scratch, double* d_sigma, int64_t* d_used, int32_t* d_iters,
                          ExpMeta* d_meta, hipStream_t s) {
  NoiseState* st = static_cast<NoiseState*>(scratch);
  uint32_t* hist = reinterpret_cast<uint32_t*>(static_cast<char*>(scratch) + sizeof(NoiseState) * (size_t)n_img);
  uint64_t* lists = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(hist) +
                                                2 * NZ_BINS * sizeof(uint32_t) * (size_t)n_img);
  const int64_t nh = (int64_t)n_img * 2 * NZ_BINS;
  const unsigned g1 = (unsigned)((std::max<int64_t>(nh, n_img) + 255) / 256);
  const unsigned gi = (unsigned)((n_img + 63) / 64);
  // 64 pixels per thread per pass, at most 1024 blocks per image
  const unsigned bx = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (max_pix + NZ_TX * 64 - 1) / (NZ_TX * 64)));
  const dim3 grid(bx, (unsigned)n_img);
  hipLaunchKernelGGL(k_noise_init, dim3(g1), dim3(256), 0, s, st, hist, n_img);
  hipLaunchKernelGGL(k_noise_count<T>, grid, dim3(NZ_TX), 0, s, d_imgs, d_npix, st);
  hipLaunchKernelGGL(k_noise_begin, dim3(gi), dim3(64), 0, s, st, n_img);
  static const int lo_x[3] = {21, 10, 0}, nb_x[3] = {11, 11, 10};
  static const int lo_d[6] = {52, 41, 30, 19, 8, 0}, nb_d[6] = {11, 11, 11, 11, 11, 8};
  // the first step's first median digit; later steps get it from the clip pass
  hipLaunchKernelGGL((k_noise_hist<T, 0, 0>), grid, dim3(NZ_TX), 0, s, d_imgs, d_npix, st, hist, lists, lo_x[0],
                     nb_x[0]);
  for (int it = 0; it < max_iter; ++it) {
    hipLaunchKernelGGL(k_noise_pick, dim3(n_img), dim3(NZ_TX), 0, s, st, hist, lo_x[0], 0);
    for (int p = 1; p < 3; ++p) {
      hipLaunchKernelGGL((k_noise_hist<T, 0, 0>), grid, dim3(NZ_TX), 0, s, d_imgs, d_npix, st, hist, lists, lo_x[p],
                         nb_x[p]);
      hipLaunchKernelGGL(k_noise_pick, dim3(n_img), dim3(NZ_TX), 0, s, st, hist, lo_x[p], 0);
    }
    hipLaunchKernelGGL(k_noise_mid, dim3(gi), dim3(64), 0, s, st, n_img);
    for (int p = 0; p < 6; ++p) {
      if (p < 2)
        hipLaunchKernelGGL((k_noise_hist<T, 1, 0>), grid, dim3(NZ_TX), 0, s, d_imgs, d_npix, st, hist, lists, lo_d[p],
                           nb_d[p]);
      else if (p == 2)
        hipLaunchKernelGGL((k_noise_hist<T, 1, 1>), grid, dim3(NZ_TX), 0, s, d_imgs, d_npix, st, hist, lists, lo_d[p],
                           nb_d[p]);
      else
        hipLaunchKernelGGL((k_noise_hist<T, 1, 2>), grid, dim3(NZ_TX), 0, s, d_imgs, d_npix, st, hist, lists, lo_d[p],
                           nb_d[p]);
      hipLaunchKernelGGL(k_noise_pick, dim3(n_img), dim3(NZ_TX), 0, s, st, hist, lo_d[p], 1);
    }
    hipLaunchKernelGGL(k_noise_sigma, dim3(gi), dim3(64), 0, s, st, n_img, kappa);
    hipLaunchKernelGGL(k_noise_clip<T>, grid, dim3(NZ_TX), 0, s, d_imgs, d_npix, st, hist);
    hipLaunchKernelGGL(k_noise_update, dim3(gi), dim3(64), 0, s, st, n_img, max_iter);
  }
  hipLaunchKernelGGL(k_noise_out, dim3(gi), dim3(64), 0, s, st, n_img, d_sigma, d_used, d_iters, d_meta);
  return hipGetLastError();
}

hipError_t launch_noise(const void* const* d_imgs, const int64_t* d_npix, int64_t max_pix, int n_img, dt_dtype dtype,
                        double kappa, int max_iter, void* scratch, double* d_sigma, int64_t* d_used, int32_t* d_iters,
                        ExpMeta* d_meta, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  return dtype == DT_F16 ? noise_t<_Float16>(d_imgs, d_npix, max_pix, n_img, kappa, max_iter, scratch, d_sigma, d_used,
                                             d_iters, d_meta, s)
                         : noise_t<float>(d_imgs, d_npix, max_pix, n_img, kappa, max_iter, scratch, d_sigma, d_used,
                                          d_iters, d_meta, s);
}

}  // namespace dtk
