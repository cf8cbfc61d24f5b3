// k_prepass.hip -- exposure metadata and the matched-filter pre-pass.
//
// Sec. 3 (FindLocalSignal): detection significance comes from a matched
// filter with a Gaussian PSF whose width is in the image header, weighted by
// the pixel noise variance.  For a stamp P centred on the nearest pixel of an
// intersection, the filter output is psi = sum P D / V and its variance is
// phi = sum P^2 / V.  Both are linear in the pixels, so evaluating them once
// per pixel of every exposure ("planes") and gathering at the intersection
// gives exactly the per-intersection filter.  The Gaussian stamp is
// separable, so each plane is a row pass followed by a column pass of a 1-D
// kernel over LDS-staged tiles.
#include <algorithm>

#include "dt_common.hpp"

namespace dtk {

// ----------------------------------------------------------------------------
// Exposure metadata (one thread per exposure).  TAN (gnomonic) projection
// with the native pole at LONPOLE = 180 deg: intermediate coordinates are
// xi = u.east / u.centre and eta = u.north / u.centre (radians) for a
// direction u; pixels are CRPIX - 1 + CD^-1 (xi, eta) in degrees.  The basis
// is rotated from equatorial to ecliptic J2000 so that samples need no frame
// rotation.
// ----------------------------------------------------------------------------
__global__ void k_exposure_prep(const dt_exposure* __restrict__ in, const int64_t* __restrict__ plane_off,
                                const int32_t* __restrict__ src, const int32_t* __restrict__ rad, int n,
                                ExpMeta* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const dt_exposure x = in[i];
  const double d2r = PI / 180.0;
  double sa, ca, sd, cd;
  sincos(x.crval_deg[0] * d2r, &sa, &ca);
  sincos(x.crval_deg[1] * d2r, &sd, &cd);
  double eps = OBLIQUITY_ARCSEC / 3600.0 * d2r;
  double se, ce;
  sincos(eps, &se, &ce);
  // equatorial basis
  double c[3] = {cd * ca, cd * sa, sd};
  double ea[3] = {-sa, ca, 0.0};
  double no[3] = {-sd * ca, -sd * sa, cd};
  // equatorial -> ecliptic: (x, ce*y + se*z, -se*y + ce*z)
  auto to_ecl = [&](const double v[3], double w[3]) {
    w[0] = v[0];
    w[1] = ce * v[1] + se * v[2];
    w[2] = -se * v[1] + ce * v[2];
  };
  double cE[3], eE[3], nE[3];
  to_ecl(c, cE);
  to_ecl(ea, eE);
  to_ecl(no, nE);
  double det = x.cd_deg[0] * x.cd_deg[3] - x.cd_deg[1] * x.cd_deg[2];
  double i00 = x.cd_deg[3] / det, i01 = -x.cd_deg[1] / det;
  double i10 = -x.cd_deg[2] / det, i11 = x.cd_deg[0] / det;
  double r2d = 180.0 / PI;
  ExpMeta m;
  m.t = x.t;
  m.ox = x.obs_xyz_au[0];
  m.oy = x.obs_xyz_au[1];
  m.oz = x.obs_xyz_au[2];
  m.cx = cE[0];
  m.cy = cE[1];
  m.cz = cE[2];
  m.a0x = r2d * (i00 * eE[0] + i01 * nE[0]);
  m.a0y = r2d * (i00 * eE[1] + i01 * nE[1]);
  m.a0z = r2d * (i00 * eE[2] + i01 * nE[2]);
  m.a1x = r2d * (i10 * eE[0] + i11 * nE[0]);
  m.a1y = r2d * (i10 * eE[1] + i11 * nE[1]);
  m.a1z = r2d * (i10 * eE[2] + i11 * nE[2]);
  m.px0 = x.crpix[0] - 1.0;
  m.py0 = x.crpix[1] - 1.0;
  m.gap = i > 0 ? x.t - in[i - 1].t : 0.0;  // input is in epoch order
  m.inv_gap = m.gap > 0.0 ? 1.0 / m.gap : 0.0;
  m.plane_off = plane_off[i];
  m.W = x.width;
  m.H = x.height;
  m.src = src[i];
  m.fwhm = x.psf_fwhm_px;
  m.R = rad[i];
  m.vs = 0.f;
  // first later exposure whose epoch exceeds this one by more than CK_SPAN
  // (the input is in epoch order and t_j - t is non-decreasing in j); n + 1
  // when there is none
  int lo = i + 1, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (in[mid].t - x.t > CK_SPAN) hi = mid;
    else lo = mid + 1;
  }
  m.ck_next = lo < n ? lo : n + 1;
  // Sky cone of the image.  The pixel (x, y) is the direction
  // c + xi e + eta n with (xi, eta) = CD (x - px0, y - py0) in radians; the
  // axis is the centre pixel's direction and the half-angle is the largest
  // angle to a corner of the rectangle widened by one pixel.  The cone's
  // trace on the tangent plane is an ellipse (convex) when the axis is within
  // ~78 deg of c and the half-angle below ~6 deg, so holding the four corners
  // it holds the whole rectangle.  Otherwise no cone is used.
  auto dir = [&](double px, double py, double d[3]) {
    const double dx = px - m.px0, dy = py - m.py0;
    const double xi = d2r * (x.cd_deg[0] * dx + x.cd_deg[1] * dy);
    const double eta = d2r * (x.cd_deg[2] * dx + x.cd_deg[3] * dy);
    for (int k = 0; k < 3; ++k) d[k] = cE[k] + xi * eE[k] + eta * nE[k];
  };
  double u[3];
  dir(0.5 * (x.width - 1), 0.5 * (x.height - 1), u);
  const double un = 1.0 / sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  for (int k = 0; k < 3; ++k) u[k] *= un;
  bool cone = (u[0] * cE[0] + u[1] * cE[1] + u[2] * cE[2]) > 0.2;
  double tmax = 0.0;
  for (int q = 0; q < 4; ++q) {
    double d[3];
    dir((q & 1) ? x.width + 0.5 : -1.5, (q & 2) ? x.height + 0.5 : -1.5, d);
    const double cs = u[0] * d[0] + u[1] * d[1] + u[2] * d[2];
    const double c0 = u[1] * d[2] - u[2] * d[1], c1 = u[2] * d[0] - u[0] * d[2], c2 = u[0] * d[1] - u[1] * d[0];
    const double sn = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    if (!(cs > 0.0)) cone = false;
    else tmax = fmax(tmax, sn / cs);
  }
  cone = cone && tmax <= 0.1;
  m.ux = cone ? u[0] : 0.0;
  m.uy = cone ? u[1] : 0.0;
  m.uz = cone ? u[2] : 0.0;
  m.cone_tan = cone ? tmax * 1.0001 + 1e-12 : 0.0;
  m.cone_lim = cone ? 0.0 : __builtin_inf();
  out[i] = m;
  if (i == n - 1) out[n] = m;  // the repeated last record
}

hipError_t launch_exposure_prep(const dt_exposure* d_in, const int64_t* d_plane_off, const int32_t* d_src,
                                const int32_t* d_R, int n, ExpMeta* d_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exposure_prep, dim3((n + 63) / 64), dim3(64), 0, s, d_in, d_plane_off, d_src, d_R, n,
                     d_out);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Matched-filter planes.  One workgroup of PREP_TX threads per PREP_TX-wide
// column strip and PREP_TY output rows.  The workgroup streams the input rows
// y0 - R .. y0 + TY + R - 1: each row is loaded once (coalesced, the next row
// prefetched into registers), turned into {D w, w} with w = 1/V (0 where the
// pixel is masked or off the image) in a double-buffered LDS row, filtered
// along x with the 1-D Gaussian, and pushed into a (2R+1)-row register window
// per column that is filtered along y to give one output row.  R is a
// template parameter so the window lives in registers.
// ----------------------------------------------------------------------------
// The image pointers come from a device array, so they are generic to the
// compiler; reading through global pointers keeps these loads off the LDS
// counter (a generic load is counted with the LDS operations, so the waits
// for a row's LDS reads would also wait for rows still in flight).
template <typename T>
__device__ __forceinline__ float load_px(const void* p, int64_t k);
template <>
__device__ __forceinline__ float load_px<float>(const void* p, int64_t k) {
  return __builtin_nontemporal_load(global_ptr(static_cast<const float*>(p)) + k);
}
template <>
__device__ __forceinline__ float load_px<_Float16>(const void* p, int64_t k) {
  return (float)__builtin_nontemporal_load(global_ptr(static_cast<const _Float16*>(p)) + k);
}

__device__ __forceinline__ float2 weight_pair(float d, float v) {
  if (__builtin_isfinite(d) && __builtin_isfinite(v) && v > 0.f) {
    float w = 1.0f / v;
    return make_float2(d * w, w);
  }
  return make_float2(0.f, 0.f);
}

__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb) {
  constexpr unsigned NX = 8;
  const unsigned q = nb / NX, r = nb % NX;
  const unsigned x = b % NX, l = b / NX;
  return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

template <typename T, int R>
__global__ __launch_bounds__(PREP_TX) void k_prepass(const ExpMeta* __restrict__ meta,
                                                     const PrepTile* __restrict__ tiles,
                                                     const void* const* __restrict__ flux,
                                                     const void* const* __restrict__ var,
                                                     float2* __restrict__ planes) {
  constexpr int K = 2 * R + 1;
  constexpr int RW = PREP_TX + 2 * R;
  constexpr int DEPTH = PREP_DEPTH;  // input rows in flight per thread
  __shared__ float2 row[2][RW];
  // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs,
  // so give each XCD a contiguous run of tiles; neighbouring tiles (which
  // share halo rows and halo cache lines) then meet in the same L2
  const PrepTile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const ExpMeta& m = meta[tl.e];
  const int W = m.W, H = m.H;
  const int tid = threadIdx.x;
  // 1-D weights g and g^2; the 2-D stamp is g(dx) g(dy) / Z with Z = (sum g)^2
  const double sig = (double)m.fwhm / (2.0 * sqrt(2.0 * log(2.0)));
  float g1[K], g2[K];
  double zs = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double d = (double)(j - R);
    double g = exp(-d * d / (2.0 * sig * sig));
    zs += g;
    g1[j] = (float)g;
    g2[j] = (float)(g * g);
  }
  const double z = zs * zs;
  const float n1 = (float)(1.0 / z), n2 = (float)(1.0 / (z * z));
  const void* Dp = flux[m.src];
  const void* Vp = var[m.src];
  // this thread's input columns: x0 - R + tid, and (halo) x0 + TX - R + tid
  const int cx = tl.x0 - R + tid;
  const int hx = tl.x0 + PREP_TX - R + tid;
  const bool has_h = tid < 2 * R;
  const bool in_c = cx >= 0 && cx < W;
  const bool in_h = has_h && hx >= 0 && hx < W;
  const int gx = tl.x0 + tid;  // output column
  const int rows = PREP_TY + 2 * R;
  // ring of DEPTH prefetched rows: (D, V) at the centre column and the halo column
  float rd[DEPTH], rv[DEPTH], hd[DEPTH], hv[DEPTH];
  auto fetch = [&](int r, float& d, float& v, float& dh, float& vh) {
    d = v = dh = vh = __builtin_nanf("");
    const int gy = tl.y0 - R + r;
    if (r < rows && gy >= 0 && gy < H) {
      const int64_t base = (int64_t)gy * W;
      if (in_c) {
        d = load_px<T>(Dp, base + cx);
        v = Vp ? load_px<T>(Vp, base + cx) : m.vs;
      }
      if (in_h) {
        dh = load_px<T>(Dp, base + hx);
        vh = Vp ? load_px<T>(Vp, base + hx) : m.vs;
      }
    }
  };
#pragma unroll
  for (int q = 0; q < DEPTH; ++q) fetch(q, rd[q], rv[q], hd[q], hv[q]);
  float2 win[K];
#pragma unroll
  for (int j = 0; j < K; ++j) win[j] = make_float2(0.f, 0.f);
  for (int r = 0; r < rows; ++r) {
    float2* buf = row[r & 1];
    buf[tid] = weight_pair(rd[0], rv[0]);
    if (has_h) buf[PREP_TX + tid] = weight_pair(hd[0], hv[0]);
#pragma unroll
    for (int q = 0; q < DEPTH - 1; ++q) {
      rd[q] = rd[q + 1];
      rv[q] = rv[q + 1];
      hd[q] = hd[q + 1];
      hv[q] = hv[q + 1];
    }
    fetch(r + DEPTH, rd[DEPTH - 1], rv[DEPTH - 1], hd[DEPTH - 1], hv[DEPTH - 1]);
    __syncthreads();
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      float2 v = buf[tid + j];
      a = fmaf(g1[j], v.x, a);
      b = fmaf(g2[j], v.y, b);
    }
#pragma unroll
    for (int j = 0; j < K - 1; ++j) win[j] = win[j + 1];
    win[K - 1] = make_float2(a, b);
    const int gy = tl.y0 + r - 2 * R;  // output row centred in the window
    if (r >= 2 * R && gy < H && gx < W) {
      float pa = 0.f, pb = 0.f;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        pa = fmaf(g1[j], win[j].x, pa);
        pb = fmaf(g2[j], win[j].y, pb);
      }
      const uint64_t bits = (uint64_t)__float_as_uint(pa * n1) | ((uint64_t)__float_as_uint(pb * n2) << 32);
      __builtin_nontemporal_store(bits, reinterpret_cast<uint64_t*>(planes + m.plane_off + (int64_t)gy * W + gx));
    }
  }
}

template <typename T>
static hipError_t launch_prepass_t(int R, const ExpMeta* d_meta, const PrepTile* d_tiles, unsigned g,
                                   const void* const* d_flux, const void* const* d_var, float2* d_planes,
                                   hipStream_t s) {
  switch (R) {
#define DT_CASE(RR)                                                                                          \
  case RR:                                                                                                   \
    hipLaunchKernelGGL((k_prepass<T, RR>), dim3(g), dim3(PREP_TX), 0, s, d_meta, d_tiles, d_flux, d_var,  \
                       d_planes);                                                                            \
    break;
    DT_CASE(1) DT_CASE(2) DT_CASE(3) DT_CASE(4) DT_CASE(5) DT_CASE(6)
    DT_CASE(7) DT_CASE(8) DT_CASE(9) DT_CASE(10) DT_CASE(11) DT_CASE(12)
#undef DT_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_prepass(const ExpMeta* d_meta, const PrepTile* d_tiles, const int64_t* group_off,
                          const int32_t* group_R, int n_groups, const void* const* d_flux,
                          const void* const* d_var, dt_dtype dtype, float2* d_planes, hipStream_t s) {
  for (int gi = 0; gi < n_groups; ++gi) {
    const int64_t beg = group_off[gi], end = group_off[gi + 1];
    for (int64_t off = beg; off < end; off += 0x7fffffff) {
      unsigned g = (unsigned)std::min<int64_t>(end - off, 0x7fffffff);
      hipError_t e = dtype == DT_F32
                         ? launch_prepass_t<float>(group_R[gi], d_meta, d_tiles + off, g, d_flux, d_var, d_planes, s)
                         : launch_prepass_t<_Float16>(group_R[gi], d_meta, d_tiles + off, g, d_flux, d_var,
                                                      d_planes, s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace dtk
