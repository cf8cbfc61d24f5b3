// k_stamps.hip -- coarse-stacked stamps of orbit-grid cells and the stack
// restricted to selected cells (the learned-proposal path).
//
// A cell is a block of `cell_size` consecutive orbits of a grid whose first
// member is the cell's representative; the other members differ from it in
// semi-major axis by at most da and in mean anomaly by at most dm.  Over a
// cell, a member's pixel track is linear in (delta a / da, delta M0 / dm) to
// a small fraction of a pixel, so the stamp is a 21 x 21 lattice in that
// parameter box: node (u, v), u, v in {-1, -0.9, ..., 1}, follows the track
//   p_e(u, v) = p_e + u (p_e[a + da] - p_e) + v (p_e[M0 + dm] - p_e)
// built from three walks (representative, a + da, M0 + dm) with the stack's
// device code, rounded to the nearest pixel; the stamp value is the
// constant-flux S/N of the matched-filter planes stacked along it (Sec. 3).
// A source on any member therefore shows as a peak near its (u, v).  One
// wavefront per cell; each lane owns 7 of the 441 nodes.  Per-cell features
// summarise the stamp and the cell's elements.
#include "dt_track.hpp"

namespace dtk {

constexpr int SH = 10;               // stamp half-width
constexpr int SW = 2 * SH + 1;       // 21
constexpr int SP = SW * SW;          // 441
constexpr int NFEAT = 16;

__device__ __forceinline__ uint16_t f2bf_s(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// One wavefront per cell.  The three walks (k = 0 the representative, k = 1
// with a + da, k = 2 with M0 + dm) are split over 63 lanes, lane = 21 k + c
// walking chunk c of the exposures from a cold start; their pixel
// coordinates (NaN behind the tangent plane, or for an orbit outside the
// domain) go to this wave's LDS, 3 x n_exp x 16 bytes.
constexpr int STAMP_CHUNKS = 21;

// GB: usable exposures whose gathers are issued together (more loads in
// flight per lane where a cell has many usable exposures).
template <int GB>
__global__ __launch_bounds__(64) void k_cell_stamps(StackArgs R, double da, double dm, uint16_t* __restrict__ st_bf,
                                                    float* __restrict__ st_f, uint16_t* __restrict__ ft_bf,
                                                    float* __restrict__ ft_f) {
  extern __shared__ double2 trk[];  // [3][n_exp]
  const int64_t cell = blockIdx.x;
  if (cell >= R.n) return;
  const int lane = threadIdx.x;
  const ExpMeta* __restrict__ meta = R.meta;
  const int n_exp = R.n_exp;
  const float2* __restrict__ planes = R.planes;
  const double nan = __builtin_nan("");
  if (lane < 3 * STAMP_CHUNKS) {
    const int k = lane / STAMP_CHUNKS, c = lane % STAMP_CHUNKS;
    const int ch = (n_exp + STAMP_CHUNKS - 1) / STAMP_CHUNKS;
    const int ex0 = c * ch;
    const int cnt = min(ch, n_exp - ex0);
    if (cnt > 0) {
      double2* tr = trk + k * n_exp + ex0;
      const double a = R.a[cell] + (k == 1 ? da : 0.0), e = R.e[cell], inc = R.inc[cell], node = R.node[cell];
      const double peri = R.peri[cell], m0 = R.m0[cell] + (k == 2 ? dm : 0.0);
      if (!orbit_ok(a, e, inc, node, peri, m0)) {
        for (int i = 0; i < cnt; ++i) tr[i] = make_double2(nan, nan);
      } else {
        Orbit ob;
        orbit_prep(a, e, inc, node, peri, m0, ob);
        walk_orbit<true>(ob, meta + ex0, cnt, R.epoch, [&](int i, const SampleOut& so) {
          tr[i] = so.front ? make_double2(so.px, so.py) : make_double2(nan, nan);
        });
      }
    }
  }
  __syncthreads();
  constexpr int PER = (SP + 63) / 64;  // 7
  float ps[PER], ph[PER];
  double u[PER], v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    ps[q] = ph[q] = 0.f;
    const int j = lane + 64 * q;
    u[q] = (double)(j % SW - SH) / (double)SH;
    v[q] = (double)(j / SW - SH) / (double)SH;
  }
  const double* ea = R.a;
  const double* ee = R.e;
  const double* ei = R.inc;
  int near = 0;
  const double2* t0 = trk;
  const double2* ta = trk + n_exp;
  const double2* tm = trk + 2 * n_exp;
  // exposures where the three walks are in front and the lattice can touch
  // the image, found 64 at a time (one per lane), then visited in order
  auto usable = [&](int ex, double2& p0, double& Ax, double& Ay, double& Bx, double& By) {
    p0 = t0[ex];
    const double2 pa = ta[ex], pm = tm[ex];
    const ExpMeta& x = meta[ex];
    Ax = pa.x - p0.x;
    Ay = pa.y - p0.y;
    Bx = pm.x - p0.x;
    By = pm.y - p0.y;
    const double rx = fabs(Ax) + fabs(Bx) + 1.0, ry = fabs(Ay) + fabs(By) + 1.0;
    return __builtin_isfinite(pa.x) && __builtin_isfinite(pm.x) && p0.x + rx >= -0.5 && p0.x - rx < x.W - 0.5 &&
           p0.y + ry >= -0.5 && p0.y - ry < x.H - 0.5;
  };
  // The gathers of up to GB usable exposures are issued together, then
  // accumulated in exposure order.  Every lane issues all its loads (a node
  // off the image reads the plane's first pixel and is dropped), so the wait
  // before each accumulation covers only the older loads.
  for (int c0 = 0; c0 < n_exp; c0 += 64) {
    bool use = false;
    if (c0 + lane < n_exp) {
      double2 p0;
      double Ax, Ay, Bx, By;
      use = usable(c0 + lane, p0, Ax, Ay, Bx, By);
    }
    uint64_t mask = __ballot(use);
    while (mask) {
      float2 cur[GB][PER];
      bool cur_ok[GB][PER];
#pragma unroll
      for (int b = 0; b < GB; ++b) {
        // no branch: a stage past the last usable exposure reloads exposure
        // c0's first pixel and drops it, so all GB x PER loads are in flight
        const bool has = mask != 0;  // wave-uniform
        const int ex = c0 + (has ? __builtin_ctzll(mask) : 0);
        mask &= mask - 1;
        double2 p0;
        double Ax, Ay, Bx, By;
        (void)usable(ex, p0, Ax, Ay, Bx, By);
        const ExpMeta& x = meta[ex];
        near += (has && p0.x >= -0.5 && p0.x < x.W - 0.5 && p0.y >= -0.5 && p0.y < x.H - 0.5) ? 1 : 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int j = lane + 64 * q;
          // the node's track point p0 + u A + v B (two fused multiply-adds)
          const double px = fma(v[q], Bx, fma(u[q], Ax, p0.x));
          const double py = fma(v[q], By, fma(u[q], Ay, p0.y));
          const double fx = floor(px + 0.5), fy = floor(py + 0.5);
          cur_ok[b][q] = has && j < SP && fx >= 0.0 && fx < (double)x.W && fy >= 0.0 && fy < (double)x.H;
          const int64_t off = cur_ok[b][q] ? (int64_t)fy * x.W + (int64_t)fx : 0;
          cur[b][q] = planes[x.plane_off + off];
        }
      }
#pragma unroll
      for (int b = 0; b < GB; ++b) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          if (cur_ok[b][q] && cur[b][q].y > 0.f) {
            ps[q] += cur[b][q].x;
            ph[q] += cur[b][q].y;
          }
        }
      }
    }
  }
  float smax = -1e30f, ssum = 0.f, ssq = 0.f, cov = 0.f, smax_c = -1e30f, center = 0.f;
  int amax = 0;
  for (int q = 0; q < PER; ++q) {
    const int j = lane + 64 * q;
    if (j >= SP) continue;
    const float snr = ph[q] > 0.f ? ps[q] / sqrtf(ph[q]) : 0.f;
    if (st_bf) st_bf[cell * SP + j] = f2bf_s(snr);
    if (st_f) st_f[cell * SP + j] = snr;
    ssum += snr;
    ssq += snr * snr;
    cov += ph[q] > 0.f ? 1.f : 0.f;
    if (snr > smax) {
      smax = snr;
      amax = j;
    }
    const int dx = j % SW - SH, dy = j / SW - SH;
    if (abs(dx) <= 3 && abs(dy) <= 3) smax_c = fmaxf(smax_c, snr);
    if (j == SP / 2) center = snr;
  }
  const float gmax = wave_max(smax);
  // node of the maximum: the lowest node index holding it (a lane's amax is
  // its own first maximum; lanes hold nodes lane, lane + 64, ...)
  int jmax = smax == gmax ? amax : SP;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) jmax = min(jmax, __shfl_xor(jmax, m, 64));
  ssum = wave_sum(ssum);
  ssq = wave_sum(ssq);
  cov = wave_sum(cov);
  center = wave_sum(center);
  smax_c = wave_max(smax_c);
  if (lane < NFEAT) {
    const float mean = ssum / SP;
    const float var = fmaxf(ssq / SP - mean * mean, 0.f);
    const float dxm = (float)(jmax % SW - SH), dym = (float)(jmax / SW - SH);
    float f = 0.f;
    switch (lane) {
      case 0: f = gmax; break;
      case 1: f = center; break;
      case 2: f = mean; break;
      case 3: f = sqrtf(var); break;
      case 4: f = cov / SP; break;
      case 5: f = sqrtf(dxm * dxm + dym * dym) / SH; break;
      case 6: f = (float)near / (float)max(n_exp, 1); break;
      case 7: f = (float)((ea[cell] - 2.75) / 0.75); break;
      case 8: f = (float)(ee[cell] / 0.3); break;
      case 9: f = (float)(ei[cell] / 0.2618); break;
      case 10: f = smax_c; break;
      case 11: f = dxm / SH; break;  // lattice coordinates (u, v) of the maximum
      case 12: f = dym / SH; break;
      default: f = 0.f; break;
    }
    if (ft_bf) ft_bf[cell * NFEAT + lane] = f2bf_s(f);
    if (ft_f) ft_f[cell * NFEAT + lane] = f;
  }
}

// The plain stack restricted to the orbits of selected cells: orbit
// cells[c] * cell_size + m for m < cell_size; outputs at the orbit's index.
// A few hundred thousand orbits give a few wavefronts per SIMD, whose
// 200-exposure walks are latency-bound, so `split` wavefronts of a workgroup
// share 64 orbits: wavefront j walks the j-th contiguous range of exposures
// (starting cold; the range is uniform over the wavefront, so exposure
// records stay scalar loads) and the first merges the ranges' compensated
// sums in range order through LDS.
__global__ __launch_bounds__(256) void k_stack_cells(StackArgs A, const int64_t* __restrict__ cells, int64_t n_sel,
                                                     int cell_size, int split) {
  __shared__ float part[4][4][64];  // [wavefront][ps.s, ps.c, ph.s, ph.c][lane]
  __shared__ int part_nv[4][64];
  const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int j = w % split;
  const int64_t r = (int64_t)blockIdx.x * (256 / split) + (w / split) * 64 + lane;
  int64_t o = -1;
  if (r < n_sel * cell_size) {
    const int64_t c = cells[r / cell_size];
    if (c >= 0) o = c * cell_size + r % cell_size;
  }
  const bool ok = o >= 0 && o < A.n;
  double a = 0, e = 0, inc = 0, node = 0, peri = 0, m0 = 0;
  if (ok) {
    a = A.a[o]; e = A.e[o]; inc = A.inc[o]; node = A.node[o]; peri = A.peri[o]; m0 = A.m0[o];
  }
  const bool good = ok && orbit_ok(a, e, inc, node, peri, m0);
  StackPart P;
  P.ps.init();
  P.ph.init();
  P.nv = 0;
  if (good) {
    const int ch = (A.n_exp + split - 1) / split;
    const int ex0 = j * ch;
    const int cnt = min(ch, A.n_exp - ex0);
    if (cnt > 0) {
      Orbit ob;
      orbit_prep(a, e, inc, node, peri, m0, ob);
      stack_range(A, ob, ex0, cnt, P);
    }
  }
  if (split > 1) {
    part[w][0][lane] = P.ps.s;
    part[w][1][lane] = P.ps.c;
    part[w][2][lane] = P.ph.s;
    part[w][3][lane] = P.ph.c;
    part_nv[w][lane] = P.nv;
    __syncthreads();
    if (j == 0) {
      for (int q = 1; q < split; ++q) {
        P.ps.merge(part[w + q][0][lane], part[w + q][1][lane]);
        P.ph.merge(part[w + q][2][lane], part[w + q][3][lane]);
        P.nv += part_nv[w + q][lane];
      }
    }
  }
  if (!ok || j != 0) return;
  float snr, flux;
  int nv;
  if (good) {
    stack_finish(P, snr, flux, nv);
  } else {
    snr = flux = __builtin_nanf("");
    nv = -1;
  }
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

// The cell stack by checkpoint prediction: one lane per member, a wavefront
// walks 64 members together (as the full stack's k_stack_track).  Splitting
// the exposures over several wavefronts, as k_stack_cells does, measured
// slower here: every range starts from a cold checkpoint.
__global__ __launch_bounds__(256, 4) void k_stack_cells_track(StackArgs A, const int64_t* __restrict__ cells,
                                                              int64_t n_sel, int cell_size) {
  __shared__ TrackQueue tq[4];
  if (wave_base() >= n_sel * cell_size) return;  // the whole wavefront is past the end
  // member orbit of a row (-1: none), taken again after the walk rather than
  // kept live through it
  auto member = [&](int64_t r) -> int64_t {
    if (r >= n_sel * cell_size) return -1;
    const int64_t c = cells[r / cell_size];
    const int64_t o = c >= 0 ? c * cell_size + r % cell_size : -1;
    return o < A.n ? o : -1;
  };
  float snr, flux;
  int nv;
  {
    const int64_t o = member(wave_base() + __lane_id());
    double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (o >= 0) {
      el[0] = A.a[o]; el[1] = A.e[o]; el[2] = A.inc[o]; el[3] = A.node[o]; el[4] = A.peri[o]; el[5] = A.m0[o];
    }
    track_stack_lane(A, el, o >= 0 && orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]), tq[threadIdx.x >> 6], snr,
                     flux, nv);
  }
  const int64_t o = member(thread_index_after_walk());
  if (o < 0) return;
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

// Members of selected cells near their stamp peak: member m of cell c sits at
// lattice coordinates u = (a_m - a_rep) / da, v = (M0_m - M0_rep) / dm (the
// representative is the cell's first member); it is listed when |u - u*| and
// |v - v*| are both at most `radius`, (u*, v*) = uv[c * uv_stride + 0, 1].
// One lane per member; a workgroup appends its listed members with one atomic.
constexpr int NEAR_WG = 1024;  // members per workgroup (one atomic per workgroup)
__global__ __launch_bounds__(NEAR_WG) void k_cell_members_near(StackArgs A, const int64_t* __restrict__ cells,
                                                           int64_t n_sel, int cell_size, const float* __restrict__ uv,
                                                           int uv_stride, double ida, double idm, double radius,
                                                           int64_t* __restrict__ ids, int64_t* __restrict__ count) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool take = false;
  int64_t o = -1;
  if (r < n_sel * cell_size) {
    const int64_t c = cells[r / cell_size];
    if (c >= 0) {
      const int64_t rep = c * cell_size;
      o = rep + r % cell_size;
      if (o < A.n && rep < A.n) {
        const double u = (A.a[o] - A.a[rep]) * ida, v = (A.m0[o] - A.m0[rep]) * idm;
        const double us = (double)uv[c * uv_stride], vs = (double)uv[c * uv_stride + 1];
        take = fabs(u - us) <= radius && fabs(v - vs) <= radius;
      }
    }
  }
  // the workgroup's listed members get consecutive slots from one atomic
  // (one per wavefront made the atomics on the single counter the cost)
  __shared__ int wcnt[NEAR_WG / 64];
  __shared__ int64_t wbase[NEAR_WG / 64];
  const uint64_t mask = __builtin_amdgcn_ballot_w64(take);
  const int lane = (int)__lane_id(), wave = (int)(threadIdx.x >> 6);
  if (lane == 0) wcnt[wave] = __builtin_popcountll(mask);
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t tot = 0;
    for (int w = 0; w < NEAR_WG / 64; ++w) {
      wbase[w] = tot;
      tot += wcnt[w];
    }
    const int64_t b = tot > 0 ? (int64_t)atomicAdd((unsigned long long*)count, (unsigned long long)tot) : 0;
    for (int w = 0; w < NEAR_WG / 64; ++w) wbase[w] += b;
  }
  __syncthreads();
  if (take) {
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    ids[wbase[wave] + rank] = o;
  }
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

// The plain stack on a device list of orbit ids (the first *count of them;
// outputs at the orbits' own indices), by checkpoint prediction with deferral
// of wavefronts whose samples land often (list index of their first lane).
__global__ __launch_bounds__(256, 4) void k_stack_ids_track(StackArgs A, const int64_t* __restrict__ ids,
                                                            const int64_t* __restrict__ count) {
  __shared__ TrackQueue tq[4];
  const int64_t m = *count;
  if (m <= STACK_IDS_SHORT) return;  // a short list: k_stack_ids_split walks it
  if (wave_base() >= m) return;      // the whole wavefront is past the end
  bool ok;
  float snr, flux;
  int nv;
  {
    const int64_t r = wave_base() + __lane_id();
    const int64_t o = r < m ? ids[r] : -1;
    ok = o >= 0 && o < A.n;
    double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (ok) {
      el[0] = A.a[o]; el[1] = A.e[o]; el[2] = A.inc[o]; el[3] = A.node[o]; el[4] = A.peri[o]; el[5] = A.m0[o];
    }
    if (track_stack_lane(A, el, ok && orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]), tq[threadIdx.x >> 6], snr,
                         flux, nv)) {
      defer_wave(A, wave_base());
      return;
    }
  }
  if (!ok) return;
  const int64_t o = ids[thread_index_after_walk()];  // read again rather than kept through the walk
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

__global__ __launch_bounds__(256, 4) void k_stack_ids_deferred(StackArgs A, const int64_t* __restrict__ ids,
                                                               const int64_t* __restrict__ count) {
  const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= (int64_t)*A.defer_count) return;
  const int64_t r = A.defer_list[j] + (int64_t)__lane_id();
  const int64_t o = r < *count ? ids[r] : -1;
  const bool ok = o >= 0 && o < A.n;
  double el[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (ok) {
    el[0] = A.a[o]; el[1] = A.e[o]; el[2] = A.inc[o]; el[3] = A.node[o]; el[4] = A.peri[o]; el[5] = A.m0[o];
  }
  float snr, flux;
  int nv;
  deferred_lane(A, el, ok && orbit_ok(el[0], el[1], el[2], el[3], el[4], el[5]), snr, flux, nv);
  if (!ok) return;
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

// Per-sample walk of a listed orbit (patches without an observer speed bound).
__global__ __launch_bounds__(256) void k_stack_ids(StackArgs A, const int64_t* __restrict__ ids,
                                                   const int64_t* __restrict__ count) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = *count;
  if (m <= STACK_IDS_SHORT || r >= m) return;  // a short list: k_stack_ids_split walks it
  const int64_t o = ids[r];
  if (o < 0 || o >= A.n) return;
  float snr, flux;
  int nv;
  stack_orbit<false>(A, o, nullptr, 0, snr, flux, nv);
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

// The id-list stack for short lists: a few thousand orbits walk 200
// exposures in about the time one wavefront takes, so IDS_SPLIT wavefronts of
// a workgroup share 64 listed orbits, wavefront j walking the j-th contiguous
// range of exposures per sample (cold start, range uniform over the
// wavefront), and the first merges the ranges' compensated sums in range
// order through LDS (S/N agrees with the full walk's to rounding).
constexpr int IDS_SPLIT = 8;
__global__ __launch_bounds__(64 * IDS_SPLIT) void k_stack_ids_split(StackArgs A, const int64_t* __restrict__ ids,
                                                                    const int64_t* __restrict__ count) {
  __shared__ float part[IDS_SPLIT][4][64];  // [wavefront][ps.s, ps.c, ph.s, ph.c][lane]
  __shared__ int part_nv[IDS_SPLIT][64];
  // the long-list kernels run after this one: it zeroes their deferral counter
  if (A.defer_count && blockIdx.x == 0 && threadIdx.x == 0) *A.defer_count = 0u;
  const int64_t m = *count;
  const int j = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  if (m > STACK_IDS_SHORT) return;            // a long list: k_stack_ids_track walks it
  if ((int64_t)blockIdx.x * 64 >= m) return;  // the whole workgroup is past the end
  const int64_t o = r < m ? ids[r] : -1;
  const bool ok = o >= 0 && o < A.n;
  double a = 0, e = 0, inc = 0, node = 0, peri = 0, m0 = 0;
  if (ok) {
    a = A.a[o]; e = A.e[o]; inc = A.inc[o]; node = A.node[o]; peri = A.peri[o]; m0 = A.m0[o];
  }
  const bool good = ok && orbit_ok(a, e, inc, node, peri, m0);
  StackPart P;
  P.ps.init();
  P.ph.init();
  P.nv = 0;
  const int ch = (A.n_exp + IDS_SPLIT - 1) / IDS_SPLIT;
  const int ex0 = j * ch;
  const int cnt = min(ch, A.n_exp - ex0);
  if (good && cnt > 0) {
    Orbit ob;
    orbit_prep(a, e, inc, node, peri, m0, ob);
    stack_range(A, ob, ex0, cnt, P);
  }
  part[j][0][lane] = P.ps.s;
  part[j][1][lane] = P.ps.c;
  part[j][2][lane] = P.ph.s;
  part[j][3][lane] = P.ph.c;
  part_nv[j][lane] = P.nv;
  __syncthreads();
  if (j != 0 || !ok) return;
  for (int q = 1; q < IDS_SPLIT; ++q) {
    P.ps.merge(part[q][0][lane], part[q][1][lane]);
    P.ph.merge(part[q][2][lane], part[q][3][lane]);
    P.nv += part_nv[q][lane];
  }
  float snr = __builtin_nanf(""), flux = __builtin_nanf("");
  int nv = -1;
  if (good) stack_finish(P, snr, flux, nv);
  if (A.snr) A.snr[o] = snr;
  if (A.flux) A.flux[o] = flux;
  if (A.nvalid) A.nvalid[o] = nv;
}

// out[i] = max(x[i * seg], ..., x[i * seg + seg - 1]) (NaN entries ignored;
// -inf when all are NaN): one lane per segment.
__global__ __launch_bounds__(256) void k_segment_max(const float* __restrict__ x, int64_t n_seg, int seg,
                                                     float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_seg) return;
  float m = -__builtin_inff();
  for (int k = 0; k < seg; ++k) {
    const float v = x[i * seg + k];
    if (v > m) m = v;
  }
  out[i] = m;
}

hipError_t launch_segment_max(const float* x, int64_t n_seg, int seg, float* out, hipStream_t s) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_segment_max, dim3((unsigned)((n_seg + 255) / 256)), dim3(256), 0, s, x, n_seg, seg, out);
  return hipGetLastError();
}

hipError_t launch_cell_members_near(const StackArgs& a, const int64_t* d_cells, int64_t n_sel, int cell_size,
                                    const float* d_uv, int uv_stride, double da, double dm, double radius,
                                    int64_t* d_ids, int64_t* d_count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, s, d_count);
  const int64_t n = n_sel * cell_size;
  if (n > 0)
    hipLaunchKernelGGL(k_cell_members_near, dim3((unsigned)((n + NEAR_WG - 1) / NEAR_WG)), dim3(NEAR_WG), 0, s, a,
                       d_cells, n_sel, cell_size, d_uv, uv_stride, 1.0 / da, 1.0 / dm, radius, d_ids, d_count);
  return hipGetLastError();
}

hipError_t launch_stack_ids(const StackArgs& a, const int64_t* d_ids, const int64_t* d_count, int64_t m_max,
                            hipStream_t s) {
  if (m_max <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((m_max + 255) / 256);
  const int64_t m_short = m_max < STACK_IDS_SHORT ? m_max : STACK_IDS_SHORT;
  hipLaunchKernelGGL(k_stack_ids_split, dim3((unsigned)((m_short + 63) / 64)), dim3(64 * IDS_SPLIT), 0, s, a, d_ids,
                     d_count);
  if (m_max > STACK_IDS_SHORT) {  // the count may be long: the kernels for long lists too
    if (a.vobs < __builtin_inf()) {
      // (the deferral counter was zeroed by k_stack_ids_split)
      hipLaunchKernelGGL(k_stack_ids_track, dim3(grid), dim3(256), 0, s, a, d_ids, d_count);
      if (a.defer_list) hipLaunchKernelGGL(k_stack_ids_deferred, dim3(grid), dim3(256), 0, s, a, d_ids, d_count);
    } else {
      hipLaunchKernelGGL(k_stack_ids, dim3(grid), dim3(256), 0, s, a, d_ids, d_count);
    }
  }
  return hipGetLastError();
}

hipError_t launch_cell_stamps(const StackArgs& reps, double da, double dm, uint16_t* st_bf, float* st_f,
                              uint16_t* ft_bf, float* ft_f, hipStream_t s) {
  if (reps.n <= 0) return hipSuccess;
  if (reps.n_exp > STAMP_MAX_EXP) return hipErrorInvalidValue;
  const size_t lds = sizeof(double2) * 3 * (size_t)reps.n_exp;
  if (reps.n_exp > 256)
    hipLaunchKernelGGL(k_cell_stamps<4>, dim3((unsigned)reps.n), dim3(64), lds, s, reps, da, dm, st_bf, st_f, ft_bf,
                       ft_f);
  else
    hipLaunchKernelGGL(k_cell_stamps<2>, dim3((unsigned)reps.n), dim3(64), lds, s, reps, da, dm, st_bf, st_f, ft_bf,
                       ft_f);
  return hipGetLastError();
}

hipError_t launch_stack_cells(const StackArgs& a, const int64_t* d_cells, int64_t n_sel, int cell_size,
                              hipStream_t s) {
  const int64_t n = n_sel * cell_size;
  if (n <= 0) return hipSuccess;
  // lanes per orbit: up to four, while that keeps the launch near a million
  // lanes and the ranges at six exposures or more
  int split = 1;
  while (split < 4 && n * split * 2 <= (int64_t)1 << 20 && a.n_exp >= 12 * split) split *= 2;
  const int64_t per_block = 256 / split;  // orbits per workgroup
  if (a.vobs < __builtin_inf()) {
    hipLaunchKernelGGL(k_stack_cells_track, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, d_cells, n_sel,
                       cell_size);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_stack_cells, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(256), 0, s, a, d_cells,
                     n_sel, cell_size, split);
  return hipGetLastError();
}

}  // namespace dtk
