// k_topk.hip -- detection: threshold + top-k of the per-orbit S/N
// (Algorithm 1, FindSignificantResults).
//
// Each orbit becomes one 64-bit key: the order-preserving bits of its S/N in
// the high word and (2^32 - 1 - index) in the low word, so sorting keys in
// descending order sorts by S/N descending with ties to the lower index, and
// every key is distinct.  Orbits below the threshold (or NaN) get key 0.
// A tournament of LDS bitonic sorts keeps the best k of every TOPK_T-key tile
// until a single tile remains.
#include <mutex>

#include "dt_internal.hpp"

namespace dtk {

constexpr int TOPK_T = 8192;       // keys per tile
constexpr int TOPK_THREADS = 512;  // 16 keys per thread

__device__ __forceinline__ uint64_t make_key(float f, uint64_t i) {
  uint32_t u = __float_as_uint(f);
  uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)ord << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
}

__device__ __forceinline__ float key_val(uint64_t k) {
  uint32_t ord = (uint32_t)(k >> 32);
  uint32_t u = (ord & 0x80000000u) ? (ord & 0x7FFFFFFFu) : ~ord;
  return __uint_as_float(u);
}

__device__ __forceinline__ int64_t key_idx(uint64_t k) { return (int64_t)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFu)); }

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort of the first S keys of s (S a power of two, 64 <= S <=
// TOPK_T), descending.  Thread t < NT = S / PER holds keys [PER t, PER t + PER)
// in r[]; a compare-exchange at distance j runs in registers when j < PER,
// between lanes of one wavefront (shuffles) when PER <= j < 64 PER, and
// through LDS with a barrier only when j >= 64 PER (6 of the 91 stages for
// 8192 keys).  In LDS stages key e = PER t + q sits at q NT + t, so the
// lanes of a wavefront touch consecutive words.  Every thread of the block
// calls it; on return s[0, S) holds the sorted keys in natural order.
template <int PER>
__device__ __forceinline__ void bitonic_desc(uint64_t* s, int S) {
  const int t = threadIdx.x;
  const int NT = S / PER;
  const bool act = t < NT;
  uint64_t r[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) r[q] = act ? s[PER * t + q] : 0;
  __syncthreads();
  for (int k = 2; k <= S; k <<= 1) {
    for (int j = k >> 1; j >= PER; j >>= 1) {
      if (j >= 64 * PER) {
        if (act) {
#pragma unroll
          for (int q = 0; q < PER; ++q) s[q * NT + t] = r[q];
        }
        __syncthreads();
        if (act) {
          const int tp = t ^ (j / PER);
          uint64_t o[PER];
#pragma unroll
          for (int q = 0; q < PER; ++q) o[q] = s[q * NT + tp];
          const int e0 = PER * t;
          const bool keep_max = ((e0 & j) == 0) == ((e0 & k) == 0);
#pragma unroll
          for (int q = 0; q < PER; ++q) r[q] = ((o[q] > r[q]) == keep_max) ? o[q] : r[q];  // keys distinct or both empty
        }
        __syncthreads();
      } else if (act) {
        // all shuffles of the stage first, so that they are in flight together
        const int m = j / PER;
        uint64_t o[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) o[q] = shfl_xor64(r[q], m);
        // the direction bits are the same for all q of a thread at these strides
        const int e0 = PER * t;
        const bool keep_max = ((e0 & j) == 0) == ((e0 & k) == 0);
#pragma unroll
        for (int q = 0; q < PER; ++q) r[q] = ((o[q] > r[q]) == keep_max) ? o[q] : r[q];
      }
    }
    if (act) {
#pragma unroll
      for (int jj = PER / 2; jj > 0; jj >>= 1) {
        if (jj <= (k >> 1)) {
#pragma unroll
          for (int q = 0; q < PER; ++q) {
            if (q & jj) continue;
            const int e = PER * t + q;
            const uint64_t a = r[q], b = r[q | jj];
            const bool desc = (e & k) == 0;
            if (desc ? (a < b) : (a > b)) {
              r[q] = b;
              r[q | jj] = a;
            }
          }
        }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int q = 0; q < PER; ++q) s[PER * t + q] = r[q];
  }
  __syncthreads();
}

// One tournament round.  Input either S/N values (snr != null, key built from
// value and index) or keys from the previous round.  A tile with at most kk
// non-empty keys is not sorted unless it is the last round: its keys are
// only compacted (in index order) since a later round sorts them.
// The tile of keys base .. base + T - 1 (of n_in) keeps its best kk in out.
template <int T>
__device__ __forceinline__ void topk_tile(const float* __restrict__ snr, const uint64_t* __restrict__ keys_in,
                                          int64_t base, int64_t n_in, float thr, int kk, int final_round,
                                          uint64_t* __restrict__ out) {
  constexpr int PER = T / TOPK_THREADS;  // keys owned by a thread
  __shared__ uint64_t s[T];
  __shared__ int scan[TOPK_THREADS];
  for (int j = threadIdx.x; j < T; j += TOPK_THREADS) {
    int64_t i = base + j;
    uint64_t key = 0;
    if (i < n_in) {
      if (snr) {
        float f = snr[i];
        if (f >= thr) key = make_key(f, (uint64_t)i);  // false for NaN
      } else {
        key = keys_in[i];
      }
    }
    s[j] = key;
  }
  __syncthreads();
  // count the non-empty keys of this thread's PER contiguous keys, block prefix sum
  uint64_t mine[PER];
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    mine[q] = s[threadIdx.x * PER + q];
    cnt += mine[q] != 0;
  }
  scan[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 1; off < TOPK_THREADS; off <<= 1) {
    int v = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
    __syncthreads();
    scan[threadIdx.x] += v;
    __syncthreads();
  }
  const int total = scan[TOPK_THREADS - 1];
  if (!final_round && total <= kk) {
    int pos = scan[threadIdx.x] - cnt;
#pragma unroll
    for (int q = 0; q < PER; ++q)
      if (mine[q] != 0) out[pos++] = mine[q];
    for (int j = total + threadIdx.x; j < kk; j += TOPK_THREADS) out[j] = 0;
    return;
  }
  // sort only the non-empty keys (compacted to the front, zero-padded to a
  // power of two): the later rounds and sparse tiles hold few of them
  {
    int pos = scan[threadIdx.x] - cnt;
#pragma unroll
    for (int q = 0; q < PER; ++q)
      if (mine[q] != 0) s[pos++] = mine[q];
  }
  int S = 64;
  while (S < total) S <<= 1;
  for (int j = total + threadIdx.x; j < S; j += TOPK_THREADS) s[j] = 0;
  __syncthreads();
  switch (S / TOPK_THREADS) {
    case 16: if constexpr (T >= 8192) bitonic_desc<16>(s, S); break;
    case 8: if constexpr (T >= 4096) bitonic_desc<8>(s, S); break;
    case 4: if constexpr (T >= 2048) bitonic_desc<4>(s, S); break;
    case 2: bitonic_desc<2>(s, S); break;
    default: bitonic_desc<1>(s, S); break;
  }
  for (int j = threadIdx.x; j < kk; j += TOPK_THREADS) out[j] = j < total ? s[j] : 0;
}

template <int T>
__global__ __launch_bounds__(TOPK_THREADS) void k_topk_round(const float* __restrict__ snr,
                                                             const uint64_t* __restrict__ keys_in, int64_t n_in,
                                                             float thr, int kk, int final_round,
                                                             uint64_t* __restrict__ keys_out) {
  topk_tile<T>(snr, keys_in, (int64_t)blockIdx.x * T, n_in, thr, kk, final_round,
               keys_out + (int64_t)blockIdx.x * kk);
}

__global__ void k_topk_emit(const uint64_t* __restrict__ keys, int k, int64_t* __restrict__ idx,
                            float* __restrict__ val, int32_t* __restrict__ count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int local = 0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    uint64_t key = keys[j];
    if (key != 0) {
      idx[j] = key_idx(key);
      val[j] = key_val(key);
      local++;
    } else {
      idx[j] = -1;
      val[j] = __builtin_nanf("");
    }
  }
  atomicAdd(&cnt, local);
  __syncthreads();
  if (threadIdx.x == 0) *count = cnt;
}

// Inputs of at most TOPK_SMALL_MAX keys in one workgroup and one launch: the
// keys stay in registers, an exact radix select (eight 8-bit digits from the
// top) finds the k-th largest key K*, the keys >= K* (exactly
// min(k, non-empty) of them, keys being distinct) are compacted into LDS,
// sorted, and emitted.  The leading digits of nearby S/N values coincide, so
// a thread counts runs of equal digits in registers and each wavefront adds
// them into its own LDS histogram.
constexpr int TOPK_SMALL_MAX = 16384;
constexpr int SMALL_THREADS = 1024;
constexpr int SMALL_PER = TOPK_SMALL_MAX / SMALL_THREADS;

// The best k (<= TOPK_T / 2) of the n <= TOPK_SMALL_MAX keys load(i) (0 =
// empty), emitted as indices, values and their count; one workgroup of
// SMALL_THREADS threads.  SORTED false skips the sort: the selected keys are
// written in thread order (thread t's keys t, t + 1024, ... after those of
// threads below t), which depends on the input alone.
template <bool SORTED = true, typename Load>
__device__ __forceinline__ void select_small(int n, int k, Load load, int64_t* __restrict__ idx,
                                             float* __restrict__ val, int32_t* __restrict__ count) {
  __shared__ uint64_t s[TOPK_T / 2];
  __shared__ int hist[SMALL_THREADS / 64][256];
  __shared__ int sh_total, sh_sel, sh_want, sh_done;
  __shared__ uint64_t sh_prefix;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  uint64_t key[SMALL_PER];
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < SMALL_PER; ++q) {
    const int i = q * SMALL_THREADS + t;
    const uint64_t kq = i < n ? load(i) : 0ull;
    key[q] = kq;
    cnt += kq != 0;
  }
  if (t == 0) {
    sh_total = 0;
    sh_sel = 0;
  }
  __syncthreads();
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (lane == 0) atomicAdd(&sh_total, cnt);
  __syncthreads();
  const int total = sh_total;
  const int m = total < k ? total : k;
  uint64_t kth = 1;  // every non-empty key is >= 2^32
  if (total > k) {
    uint64_t prefix = 0;
    int want = k;  // rank from the top still to find below `prefix`
    // a pass whose chosen digit holds exactly `want` keys ends the search:
    // all keys >= prefix (lower digits zero) are then the k largest
    for (int shift = 56; shift >= 0; shift -= 8) {
      for (int i = t; i < (SMALL_THREADS / 64) * 256; i += SMALL_THREADS) (&hist[0][0])[i] = 0;
      __syncthreads();
      const uint64_t hmask = shift == 56 ? 0ull : (~0ull << (shift + 8));
      // runs of equal digits among a thread's keys are counted in registers
      // first (in the leading passes nearly all keys share one digit)
      int run_d = -1, run_c = 0;
#pragma unroll
      for (int q = 0; q < SMALL_PER; ++q) {
        if (key[q] != 0 && (key[q] & hmask) == prefix) {
          const int d = (int)((key[q] >> shift) & 255u);
          if (d != run_d) {
            if (run_c) atomicAdd(&hist[wv][run_d], run_c);
            run_d = d;
            run_c = 0;
          }
          run_c++;
        }
      }
      if (run_c) atomicAdd(&hist[wv][run_d], run_c);
      __syncthreads();
      if (t < 256) {
        int sum = 0;
#pragma unroll
        for (int w = 1; w < SMALL_THREADS / 64; ++w) sum += hist[w][t];
        hist[0][t] += sum;
      }
      __syncthreads();
      if (t < 64) {
        // lane l holds digits 255 - 4 l - r, r = 0..3 (descending)
        int c[4], sum = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          c[r] = hist[0][255 - 4 * t - r];
          sum += c[r];
        }
        int inc = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int v = __shfl_up(inc, o, 64);
          if (t >= o) inc += v;
        }
        const int exc = inc - sum;
        if (exc < want && want <= inc) {
          int acc = exc;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (acc + c[r] >= want) {
              sh_prefix = prefix | ((uint64_t)(255 - 4 * t - r) << shift);
              sh_want = want - acc;
              sh_done = acc + c[r] == want;
              break;
            }
            acc += c[r];
          }
        }
      }
      __syncthreads();
      prefix = sh_prefix;
      want = sh_want;
      // uniform: every thread read the same flag; the next pass rewrites
      // sh_* only after two more barriers
      if (sh_done) break;
    }
    kth = prefix;
  }
  if (!SORTED) {
    // exclusive prefix of the per-thread counts of selected keys: within
    // each wavefront by shuffles, across wavefronts through LDS
    int mine = 0;
#pragma unroll
    for (int q = 0; q < SMALL_PER; ++q) mine += (key[q] != 0 && key[q] >= kth) ? 1 : 0;
    int inc = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(inc, o, 64);
      if (lane >= o) inc += v;
    }
    if (lane == 63) hist[0][wv] = inc;
    __syncthreads();
    int pos = inc - mine;
    for (int w = 0; w < wv; ++w) pos += hist[0][w];
#pragma unroll
    for (int q = 0; q < SMALL_PER; ++q) {
      if (key[q] != 0 && key[q] >= kth) {
        idx[pos] = key_idx(key[q]);
        val[pos] = key_val(key[q]);
        pos++;
      }
    }
    for (int j = m + t; j < k; j += SMALL_THREADS) {
      idx[j] = -1;
      val[j] = __builtin_nanf("");
    }
    if (t == 0) *count = m;
    return;
  }
#pragma unroll
  for (int q = 0; q < SMALL_PER; ++q)
    if (key[q] != 0 && key[q] >= kth) s[atomicAdd(&sh_sel, 1)] = key[q];
  __syncthreads();
  int S = 64;
  while (S < m) S <<= 1;
  for (int j = m + t; j < S; j += SMALL_THREADS) s[j] = 0;
  __syncthreads();
  switch (S / TOPK_THREADS) {
    case 8: bitonic_desc<8>(s, S); break;
    case 4: bitonic_desc<4>(s, S); break;
    case 2: bitonic_desc<2>(s, S); break;
    default: bitonic_desc<1>(s, S); break;
  }
  for (int j = t; j < k; j += SMALL_THREADS) {
    if (j < m) {
      idx[j] = key_idx(s[j]);
      val[j] = key_val(s[j]);
    } else {
      idx[j] = -1;
      val[j] = __builtin_nanf("");
    }
  }
  if (t == 0) *count = m;
}

template <bool SORTED>
__global__ __launch_bounds__(SMALL_THREADS) void k_topk_small(const float* __restrict__ snr, int n, float thr, int k,
                                                              int64_t* __restrict__ idx, float* __restrict__ val,
                                                              int32_t* __restrict__ count) {
  select_small<SORTED>(n, k, [&](int i) -> uint64_t {
    const float f = snr[i];
    return f >= thr ? make_key(f, (uint64_t)i) : 0ull;  // false for NaN
  }, idx, val, count);
}

// Top-k of many S/N arrays (the patches of a batch) in two launches: every
// TOPK_T tile of every array keeps its best k (one workgroup per tile), then
// one workgroup per array selects from its tiles' survivors.  Needs
// k * tiles <= TOPK_SMALL_MAX for every array (checked by the host).
__global__ __launch_bounds__(TOPK_THREADS) void k_topk_seg_tiles(SegTopkArgs a) {
  const int t = blockIdx.x;
  const int p = a.tile_patch[t];
  const int64_t lt = t - a.tile_first[p];
  topk_tile<TOPK_T>(a.snr[p], nullptr, lt * TOPK_T, a.n[p], a.thr, a.k, 0, a.keys + (int64_t)t * a.k);
}

__global__ __launch_bounds__(SMALL_THREADS) void k_topk_seg_final(SegTopkArgs a) {
  const int p = blockIdx.x;
  const int64_t t0 = a.tile_first[p];
  const int n = (int)((a.tile_first[p + 1] - t0) * a.k);
  const uint64_t* keys = a.keys + t0 * a.k;
  select_small(n, a.k, [&](int i) -> uint64_t { return keys[i]; }, a.idx + (int64_t)p * a.k,
               a.val + (int64_t)p * a.k, a.cnt + p);
}

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tile of the first round: small inputs use tiles just large enough to cut
// the keys fourfold (cheaper sorts, more workgroups); large inputs 8192.
static int first_tile(int64_t n, int32_t k) {
  if (n > 65536) return TOPK_T;
  int t = 1024;
  while (t < 4 * k && t < TOPK_T) t <<= 1;
  return t;
}
static int round_tile(int64_t n_in) {
  if (n_in > TOPK_T) return TOPK_T;
  int t = 1024;
  while (t < n_in) t <<= 1;
  return t;
}

int64_t topk_seg_tile() { return TOPK_T; }
int64_t topk_seg_max_keys() { return TOPK_SMALL_MAX; }

hipError_t launch_topk_segmented(const SegTopkArgs& a, int n_tiles, int n_arrays, hipStream_t s) {
  if (a.k < 1 || a.k > TOPK_T / 2 || n_arrays <= 0) return hipErrorInvalidValue;
  if (n_tiles > 0) hipLaunchKernelGGL(k_topk_seg_tiles, dim3((unsigned)n_tiles), dim3(TOPK_THREADS), 0, s, a);
  hipLaunchKernelGGL(k_topk_seg_final, dim3((unsigned)n_arrays), dim3(SMALL_THREADS), 0, s, a);
  return hipGetLastError();
}

size_t topk_scratch_bytes(int64_t n, int32_t k) {
  int64_t tiles = ceil_div(n > 0 ? n : 1, first_tile(n, k));
  int64_t kk = k < TOPK_T ? k : TOPK_T;
  return (size_t)(2 * tiles * kk + TOPK_T) * sizeof(uint64_t);
}

static void launch_round(int T, unsigned tiles, const float* snr, const uint64_t* in, int64_t n_in, float thr, int k,
                         int final_round, uint64_t* out, hipStream_t s) {
  switch (T) {
    case 1024:
      hipLaunchKernelGGL(k_topk_round<1024>, dim3(tiles), dim3(TOPK_THREADS), 0, s, snr, in, n_in, thr, k,
                         final_round, out);
      break;
    case 2048:
      hipLaunchKernelGGL(k_topk_round<2048>, dim3(tiles), dim3(TOPK_THREADS), 0, s, snr, in, n_in, thr, k,
                         final_round, out);
      break;
    case 4096:
      hipLaunchKernelGGL(k_topk_round<4096>, dim3(tiles), dim3(TOPK_THREADS), 0, s, snr, in, n_in, thr, k,
                         final_round, out);
      break;
    default:
      hipLaunchKernelGGL(k_topk_round<TOPK_T>, dim3(tiles), dim3(TOPK_THREADS), 0, s, snr, in, n_in, thr, k,
                         final_round, out);
      break;
  }
}

hipError_t launch_topk(const float* d_snr, int64_t n, int32_t k, float thr, int64_t* d_idx, float* d_val,
                       int32_t* d_count, void* d_scratch, hipStream_t s, bool ordered) {
  if (k < 1 || k > TOPK_T / 2) return hipErrorInvalidValue;
  if (n <= TOPK_SMALL_MAX) {
    if (ordered)
      hipLaunchKernelGGL(k_topk_small<true>, dim3(1), dim3(SMALL_THREADS), 0, s, d_snr, (int)(n > 0 ? n : 0), thr, k,
                         d_idx, d_val, d_count);
    else
      hipLaunchKernelGGL(k_topk_small<false>, dim3(1), dim3(SMALL_THREADS), 0, s, d_snr, (int)(n > 0 ? n : 0), thr,
                         k, d_idx, d_val, d_count);
    return hipGetLastError();
  }
  const int T1 = first_tile(n, k);
  int64_t tiles = ceil_div(n > 0 ? n : 1, T1);
  uint64_t* buf[2] = {static_cast<uint64_t*>(d_scratch), static_cast<uint64_t*>(d_scratch) + tiles * k};
  int cur = 0;
  int64_t n_in = n > 0 ? n : 0;
  launch_round(T1, (unsigned)tiles, d_snr, nullptr, n_in, thr, k, tiles == 1 ? 1 : 0, buf[cur], s);
  n_in = tiles * k;
  while (tiles > 1) {
    const int T = round_tile(n_in);
    tiles = ceil_div(n_in, T);
    launch_round(T, (unsigned)tiles, nullptr, buf[cur], n_in, thr, k, tiles == 1 ? 1 : 0, buf[cur ^ 1], s);
    cur ^= 1;
    n_in = tiles * k;
  }
  hipLaunchKernelGGL(k_topk_emit, dim3(1), dim3(256), 0, s, buf[cur], k, d_idx, d_val, d_count);
  return hipGetLastError();
}

// ---- allocation-free variant (dt_topk_noalloc) ----
// The tournament's key buffers live in a fixed device array instead of
// context scratch.  Host code never passes the array's name to a kernel: the
// name is a host-side stand-in, so the device address of each GPU's copy is
// resolved once per device (hipGetSymbolAddress, with that device current)
// and kept in noalloc_ptr[].
constexpr size_t NOALLOC_BYTES = (size_t)DT_TOPK_NOALLOC_BYTES;
static __device__ __align__(256) uint64_t scratch[NOALLOC_BYTES / sizeof(uint64_t)];

constexpr int NOALLOC_MAX_DEV = 64;
static std::mutex noalloc_mu;
static void* noalloc_ptr[NOALLOC_MAX_DEV];

// Called by dt_ctx_create with `device` current.
hipError_t topk_noalloc_setup(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (noalloc_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  noalloc_ptr[device] = ptr;
  return hipSuccess;
}

static void* topk_noalloc_ptr(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEV) return nullptr;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  return noalloc_ptr[device];
}

}  // namespace dtk

extern "C" dt_status dt_topk_noalloc(dt_ctx* c, const float* d_snr, int64_t n, int32_t k, float threshold,
                                     int64_t* d_idx, float* d_val, int32_t* d_count) {
  using namespace dtk;
  if (!c || !c->alive) return fail(DT_E_ARG, "invalid context");
  if (n < 0 || (n > 0 && !d_snr)) return fail(DT_E_ARG, "bad S/N array");
  if (n >= ((int64_t)1 << 32)) return fail(DT_E_ARG, "n must be < 2^32");
  if (k < 1 || k > 4096) return fail(DT_E_ARG, "k must be in [1, 4096]");
  if (!d_idx || !d_val || !d_count) return fail(DT_E_ARG, "NULL output");
  if (std::isnan(threshold)) return fail(DT_E_ARG, "threshold is NaN");
  const size_t need = topk_scratch_bytes(n, k);
  if (need > NOALLOC_BYTES)
    return fail(DT_E_ARG, "n = %lld, k = %d needs %zu bytes of top-k scratch; the allocation-free top-k holds %zu",
                (long long)n, (int)k, need, NOALLOC_BYTES);
  void* ptr = topk_noalloc_ptr(c->device);
  if (!ptr) return fail(DT_E_STATE, "the scratch address of device %d was not resolved", c->device);
  DeviceGuard g(c->device);
  hipError_t e = launch_topk(d_snr, n, k, threshold, d_idx, d_val, d_count, ptr, c->stream);
  if (e != hipSuccess) return hip_fail(e, "top-k launch");
  return DT_OK;
}
