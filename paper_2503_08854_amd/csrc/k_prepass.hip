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
  m.plane_off = plane_off[i];
  m.W = x.width;
  m.H = x.height;
  m.src = src[i];
  m.fwhm = x.psf_fwhm_px;
  m.R = rad[i];
  m.pad = 0;
  out[i] = m;
}

hipError_t launch_exposure_prep(const dt_exposure* d_in, const int64_t* d_plane_off, const int32_t* d_src,
                                const int32_t* d_R, int n, ExpMeta* d_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exposure_prep, dim3((n + 63) / 64), dim3(64), 0, s, d_in, d_plane_off, d_src, d_R, n,
                     d_out);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Matched-filter planes.  One workgroup per PREP_TX x PREP_TY output tile.
// LDS holds the haloed input as {D*w, w} with w = 1/V (0 where masked), then
// the row-filtered intermediate.  Stamp half-width R = ceil(3 sigma).
// ----------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ float load_px(const void* p, int64_t k);
template <>
__device__ __forceinline__ float load_px<float>(const void* p, int64_t k) {
  return __builtin_nontemporal_load(static_cast<const float*>(p) + k);
}
template <>
__device__ __forceinline__ float load_px<_Float16>(const void* p, int64_t k) {
  return (float)__builtin_nontemporal_load(static_cast<const _Float16*>(p) + k);
}

template <typename T>
__global__ __launch_bounds__(256) void k_prepass(const ExpMeta* __restrict__ meta, const PrepTile* __restrict__ tiles,
                                                 const void* const* __restrict__ flux,
                                                 const void* const* __restrict__ var, float2* __restrict__ planes,
                                                 int rmax) {
  extern __shared__ float2 lds[];
  __shared__ float g1[2 * PREP_RMAX + 1], g2[2 * PREP_RMAX + 1];
  __shared__ float s_norm1, s_norm2;
  const PrepTile tl = tiles[blockIdx.x];
  const ExpMeta& m = meta[tl.e];
  const int W = m.W, H = m.H;
  const double sig = (double)m.fwhm / (2.0 * sqrt(2.0 * log(2.0)));
  const int R = m.R;  // <= rmax, checked on the host
  const int IW = PREP_TX + 2 * rmax;        // LDS row pitch (input)
  const int IH = PREP_TY + 2 * R;
  float2* in = lds;                          // [IH][IW]
  float2* hr = lds + (PREP_TY + 2 * rmax) * IW;  // [IH][PREP_TX]
  const int tid = threadIdx.x;
  if (tid <= 2 * R) {
    double d = tid - R;
    double g = exp(-d * d / (2.0 * sig * sig));
    g1[tid] = (float)g;
    g2[tid] = (float)(g * g);
  }
  if (tid == 0) {
    double z = 0.0;
    for (int j = -R; j <= R; ++j) z += exp(-(double)(j * j) / (2.0 * sig * sig));
    z = z * z;  // the 2-D stamp sum is the square of the 1-D sum
    s_norm1 = (float)(1.0 / z);
    s_norm2 = (float)(1.0 / (z * z));
  }
  const void* Dp = flux[m.src];
  const void* Vp = var[m.src];
  const int gx0 = tl.x0 - R, gy0 = tl.y0 - R;
  const int inw = PREP_TX + 2 * R;
  for (int k = tid; k < IH * inw; k += 256) {
    int r = k / inw, c = k - r * inw;
    int gx = gx0 + c, gy = gy0 + r;
    float2 v2 = make_float2(0.f, 0.f);
    if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
      int64_t q = (int64_t)gy * W + gx;
      float d = load_px<T>(Dp, q);
      float v = load_px<T>(Vp, q);
      if (__builtin_isfinite(d) && __builtin_isfinite(v) && v > 0.f) {
        float w = 1.0f / v;
        v2 = make_float2(d * w, w);
      }
    }
    in[r * IW + c] = v2;
  }
  __syncthreads();
  // row pass: hr[r][x] = sum_j g[j] in[r][x + j]
  for (int k = tid; k < IH * PREP_TX; k += 256) {
    int r = k / PREP_TX, x = k - r * PREP_TX;
    const float2* row = in + r * IW + x;
    float a = 0.f, b = 0.f;
    for (int j = 0; j <= 2 * R; ++j) {
      float2 v = row[j];
      a = fmaf(g1[j], v.x, a);
      b = fmaf(g2[j], v.y, b);
    }
    hr[r * PREP_TX + x] = make_float2(a, b);
  }
  __syncthreads();
  const float n1 = s_norm1, n2 = s_norm2;
  for (int k = tid; k < PREP_TY * PREP_TX; k += 256) {
    int y = k / PREP_TX, x = k - y * PREP_TX;
    int gx = tl.x0 + x, gy = tl.y0 + y;
    if (gx >= W || gy >= H) continue;
    float a = 0.f, b = 0.f;
    for (int j = 0; j <= 2 * R; ++j) {
      float2 v = hr[(y + j) * PREP_TX + x];
      a = fmaf(g1[j], v.x, a);
      b = fmaf(g2[j], v.y, b);
    }
    planes[m.plane_off + (int64_t)gy * W + gx] = make_float2(a * n1, b * n2);
  }
}

hipError_t launch_prepass(const ExpMeta* d_meta, const PrepTile* d_tiles, int64_t n_tiles,
                          const void* const* d_flux, const void* const* d_var, dt_dtype dtype,
                          float2* d_planes, int rmax, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (rmax < 0 || rmax > PREP_RMAX) return hipErrorInvalidValue;
  size_t lds = sizeof(float2) * ((size_t)(PREP_TY + 2 * rmax) * (PREP_TX + 2 * rmax) +
                                 (size_t)(PREP_TY + 2 * rmax) * PREP_TX);
  if (lds > 64 * 1024) {
    hipError_t e = dtype == DT_F32
                       ? hipFuncSetAttribute((const void*)k_prepass<float>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                       : hipFuncSetAttribute((const void*)k_prepass<_Float16>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t max_grid = 0x7fffffff;
  for (int64_t off = 0; off < n_tiles; off += max_grid) {
    unsigned int g = (unsigned int)((n_tiles - off) < max_grid ? (n_tiles - off) : max_grid);
    if (dtype == DT_F32)
      hipLaunchKernelGGL(k_prepass<float>, dim3(g), dim3(256), lds, s, d_meta, d_tiles + off, d_flux, d_var,
                         d_planes, rmax);
    else
      hipLaunchKernelGGL(k_prepass<_Float16>, dim3(g), dim3(256), lds, s, d_meta, d_tiles + off, d_flux, d_var,
                         d_planes, rmax);
  }
  return hipGetLastError();
}

}  // namespace dtk
