// dt_common.hpp -- structures and helpers shared by the host API and the HIP
// kernels of libdtrack (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtrack.h"

namespace dtk {

// Gaussian gravitational constant k (AU^1.5/day); GM_sun = k^2 (Sec. 3:
// two-body motion about the Sun, the asteroid's mass neglected).
constexpr double K_GAUSS = 0.01720209895;
constexpr double MU_SUN = K_GAUSS * K_GAUSS;
// Speed of light in AU/day from the SI metre, second and the IAU astronomical unit.
constexpr double C_AU_DAY = 299792458.0 * 86400.0 / 149597870700.0;
// Mean obliquity of the ecliptic at J2000 (IAU 2006), arcseconds.
constexpr double OBLIQUITY_ARCSEC = 84381.448;
constexpr double PI = 3.14159265358979323846;

// Days of epochs between checkpoints of the checkpoint walk (at least this often).
constexpr double CK_SPAN = 12.0;

// Per-exposure constants, prepared on the device from a dt_exposure.
// Everything is expressed in the heliocentric ecliptic frame so no rotation
// is needed per sample: the TAN basis is rotated once per exposure instead.
struct alignas(16) ExpMeta {
  // The fields every step of the checkpoint walk reads come first (72 bytes,
  // two scalar loads issued together).
  double t;                 // epoch (days)
  double ox, oy, oz;        // observer (AU, ecliptic)
  // Sky cone holding every direction that projects into the pixel rectangle
  // widened by one pixel: unit axis u, tangent of the half-angle, and the
  // limit of the cone test (0; +inf with u = 0 when no cone is used).
  double ux, uy, uz, cone_tan, cone_lim;
  double cx, cy, cz;        // tangent-point direction (ecliptic)
  double a0x, a0y, a0z;     // row 0 of (180/pi) CD^-1 [east; north] (px per unit, ecliptic)
  double a1x, a1y, a1z;     // row 1
  double px0, py0;          // CRPIX - 1
  double gap, inv_gap;      // epoch step from the previous exposure (epoch order) and its reciprocal
  int64_t plane_off;        // offset of this exposure's plane (in float2 units)
  int32_t W, H;             // image size
  int32_t src;              // caller's index of this exposure
  float fwhm;               // PSF FWHM (px)
  int32_t R;                // stamp half-width ceil(3 sigma)
  float vs;                 // scalar pixel variance when the patch has no variance planes
  int32_t ck_next;          // first exposure (epoch order) more than CK_SPAN days after this one (n + 1 when none)
};
// A patch holds n + 1 records: the last exposure's record is repeated once
// (the checkpoint walk's final queue-serving step reads it, uses nothing of it).
static_assert(sizeof(ExpMeta) == 224, "ExpMeta layout");

// Exposure records, planes and elements seen through a named address space.
// A pointer read from device memory (a batched launch's per-patch
// descriptor) is generic to the compiler, and generic (flat) loads count as
// possibly per-lane: a wave-uniform record read through one would make the
// whole exposure walk per-lane (vector registers, masked branches).  The
// records are read through the constant address space (device memory no
// kernel writes while it runs), so a uniform record is read with scalar
// loads even where the kernel also stores to global memory; planes and
// elements through the global one.  Functions that take a generic
// reference get an explicit cast, which the compiler sees through.
typedef const __attribute__((address_space(4))) ExpMeta GExpMeta;
__device__ __forceinline__ GExpMeta* global_meta(const ExpMeta* p) { return (GExpMeta*)p; }
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* global_ptr(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ T global_load(const T* p, int64_t i) {
  return *(const T*)&global_ptr(p)[i];
}

// One tile of the matched-filter pre-pass.
struct PrepTile {
  int32_t e;       // exposure (sorted index)
  int32_t x0, y0;  // tile origin
  int32_t pad;
};

constexpr int PREP_TX = 256;  // tile width (output pixels) = threads per workgroup
constexpr int PREP_TY = 128;  // tile height (output rows streamed per workgroup)
constexpr int PREP_DEPTH = 4; // input rows each thread keeps in flight
constexpr int PREP_RMAX = 12; // largest stamp half-width supported (FWHM <= 8 px gives R = 11)

// Launchers (defined in the .hip files; all enqueue on `s`).
hipError_t launch_exposure_prep(const dt_exposure* d_in, const int64_t* d_plane_off, const int32_t* d_src,
                                const int32_t* d_R, int n, ExpMeta* d_out, hipStream_t s);
// Tiles are grouped by stamp half-width: group gi covers tiles
// [group_off[gi], group_off[gi+1]) whose exposures all have R = group_R[gi].
hipError_t launch_prepass(const ExpMeta* d_meta, const PrepTile* d_tiles, const int64_t* group_off,
                          const int32_t* group_R, int n_groups, const void* const* d_flux,
                          const void* const* d_var, dt_dtype dtype, float2* d_planes, hipStream_t s);

// Stamp half-width for a PSF FWHM: R = ceil(3 sigma), sigma = FWHM / (2 sqrt(2 ln 2)).
inline int stamp_radius(double fwhm) {
  double sig = fwhm / (2.0 * __builtin_sqrt(2.0 * __builtin_log(2.0)));
  return (int)__builtin_ceil(3.0 * sig);
}

struct StackArgs {
  const ExpMeta* meta;
  int32_t n_exp;
  const float2* planes;
  int64_t n;
  double epoch;
  const double *a, *e, *inc, *node, *peri, *m0;
  float* snr;
  float* flux;
  int32_t* nvalid;
  // Bound on the observer's speed (AU/day) between any two exposures of the
  // patch: the largest |obs_i - obs_j| / (t_i - t_j) over epoch neighbours
  // (infinite when two exposures share an epoch but not an observer).
  double vobs = __builtin_inf();
  // Work counters of the checkpoint walk (measurement only; NULL = off):
  // WORK_SLOTS slots of WORK_N counters, slot = workgroup index mod WORK_SLOTS.
  unsigned long long* work = nullptr;
  // Deferral (NULL = not allowed): a wavefront of the checkpoint walk whose
  // samples land often appends its first orbit index to defer_list (slot from
  // *defer_count, zeroed before the launch) and writes no outputs; the
  // deferred-walk kernel then stacks those orbits per sample.
  int64_t* defer_list = nullptr;
  unsigned int* defer_count = nullptr;
};

// Work counters (one slot; see dt_ctx_count_work): samples tested by
// prediction, queued exact solves, checkpoint solves, samples walked by the
// per-sample tail, tail samples that took the full path, wavefronts that
// switched to the tail.
enum { WORK_PRED = 0, WORK_QUEUED, WORK_CKPT, WORK_TAIL, WORK_TAIL_FULL, WORK_SWITCHED, WORK_N = 8 };
constexpr int WORK_SLOTS = 64;

struct DebugArgs {
  const int64_t* ids;
  int64_t m;
  double *px, *py, *tau;
  int32_t *ix, *iy, *flags;
  float *psi, *phi;
};

// Work item of the batched persistent launch: orbits [begin, begin + count)
// of patch `patch`.
struct WorkItem {
  int32_t patch;
  int32_t count;
  int64_t begin;
};

// The stack: the checkpoint walk (then, when a.defer_list is set, the
// per-sample walk of the wavefronts it deferred), or the per-sample walk for
// an unbounded observer speed.
hipError_t launch_stack(const StackArgs& a, hipStream_t s);
hipError_t launch_zero_u32(unsigned int* p, hipStream_t s);
hipError_t launch_batched(const StackArgs* d_descs, const WorkItem* d_items, int n_items, unsigned int* d_counter,
                          int n_wg, hipStream_t s);
hipError_t launch_debug(const StackArgs& a, const DebugArgs& d, hipStream_t s);
// The same table from the walk launch_stack runs on this patch (solved samples only).
hipError_t launch_debug_stack(const StackArgs& a, const DebugArgs& d, hipStream_t s);
hipError_t launch_validate(const StackArgs& a, unsigned long long* d_bad, hipStream_t s);

// BF16 GEMM C = op(A) op(B) (+ bias, ReLU) with FP32 accumulation; op(A) is
// M x K (A stored [K x M] when transA), op(B) is K x N (B stored [N x K] when
// transB).  Outputs FP32 (Cf) and/or BF16 (Cb), each with its own leading
// dimension; d_part is split-K scratch of part_elems floats.
struct GemmArgs {
  const uint16_t* A;
  int lda, transA;
  const uint16_t* B;
  int ldb, transB;
  int M, N, K;
  const float* bias;
  int relu;
  float* Cf;
  int ldcf;
  uint16_t* Cb;
  int ldcb;
};
hipError_t launch_gemm_bf16(const GemmArgs& g, float* d_part, size_t part_elems, hipStream_t s);
hipError_t launch_im2col(const uint16_t* x, int Bn, int H, int W, int C, int stride, int Ho, int Wo, uint16_t* cols,
                         hipStream_t s);
hipError_t launch_col2im_mask(const float* dcols, int Bn, int H, int W, int C, int stride, int Ho, int Wo,
                              const uint16_t* act, uint16_t* dx, float* dx_f, hipStream_t s);
hipError_t launch_relu_mask(const float* src, int lds, const uint16_t* act, int lda, int M, int N, uint16_t* dst,
                            float* dst_f, hipStream_t s);
hipError_t launch_colsum(const float* d, int M, int N, float* out, hipStream_t s);
hipError_t launch_bce(const float* z, const float* y, int Bn, float* loss, float* dz, uint16_t* dz_bf, hipStream_t s);
hipError_t launch_adam(float* w, float* m, float* v, const float* g, int64_t n, float lr, int64_t t, uint16_t* w_bf,
                       hipStream_t s);
hipError_t launch_cast_bf16(const float* x, int64_t n, uint16_t* y, hipStream_t s);
hipError_t launch_init_params(float* w, int64_t off, int64_t n, int fan_in, uint64_t seed, int is_bias,
                              hipStream_t s);

// Coarse stamps (21 x 21) and 16 features per representative orbit; d_track
// is n x n_exp int2 scratch.  Any output may be null.
constexpr int STAMP_MAX_EXP = 1024;  // the stamps keep three walks of every exposure in LDS
hipError_t launch_cell_stamps(const StackArgs& reps, double da, double dm, uint16_t* st_bf, float* st_f,
                              uint16_t* ft_bf, float* ft_f, hipStream_t s);
hipError_t launch_segment_max(const float* x, int64_t n_seg, int seg, float* out, hipStream_t s);
hipError_t launch_cell_members_near(const StackArgs& a, const int64_t* d_cells, int64_t n_sel, int cell_size,
                                    const float* d_uv, int uv_stride, double da, double dm, double radius,
                                    int64_t* d_ids, int64_t* d_count, hipStream_t s);
// Id lists whose count (read on the device) is at most STACK_IDS_SHORT are
// walked per sample with the exposures split over eight wavefronts per 64
// orbits (latency-bound sizes); longer ones by the checkpoint walk with
// deferral.  Both kernels are launched when m_max exceeds STACK_IDS_SHORT;
// the one not meant for the count returns at once.
constexpr int64_t STACK_IDS_SHORT = (int64_t)1 << 17;
hipError_t launch_stack_ids(const StackArgs& a, const int64_t* d_ids, const int64_t* d_count, int64_t m_max,
                            hipStream_t s);
hipError_t launch_stack_cells(const StackArgs& a, const int64_t* d_cells, int64_t n_sel, int cell_size,
                              hipStream_t s);

// Outlier trimming of m candidate orbits (n_exp <= 512); d_buf is m x n_exp float2 scratch.
hipError_t launch_clip(const StackArgs& a, const int64_t* d_ids, int64_t m, double kappa, int max_iter,
                       float2* d_buf, float* snr, float* flux, int32_t* nkept, hipStream_t s);

// Fused inference forward of the cell scorer.
struct ScorerFusedArgs {
  const uint16_t* stamps;  // B x 441 BF16
  const uint16_t* feats;   // B x 16 BF16
  int B;
  const uint16_t* wb;      // BF16 weights, layer-wise [K][N]
  uint16_t* wt;            // scratch: the BF16 weights transposed, layer i at t_off[i] as [N][K]
  const float* w;          // FP32 master parameters (the biases are read here)
  int64_t w_off[7], b_off[7], t_off[8];
  int K[7], N[7];
  float* z;                // B logits
  const int64_t* rows;     // NULL, or cell i of the batch is row rows[i] of stamps / feats and of z
};
// Top-k of many S/N arrays at once (device tables, one entry per array or
// per TOPK tile; see launch_topk_segmented).
struct SegTopkArgs {
  const float* const* snr;    // [arrays]
  const int64_t* n;           // [arrays]
  const int64_t* tile_first;  // [arrays + 1] first tile of each array
  const int32_t* tile_patch;  // [tiles] array of each tile
  uint64_t* keys;             // [tiles * k] scratch
  float thr;
  int32_t k;
  int64_t* idx;               // [arrays * k]
  float* val;                 // [arrays * k]
  int32_t* cnt;               // [arrays]
};
int64_t topk_seg_tile();      // keys per tile
int64_t topk_seg_max_keys();  // largest k * tiles of one array
hipError_t launch_topk_segmented(const SegTopkArgs& a, int n_tiles, int n_arrays, hipStream_t s);

// transpose: rebuild A.wt from A.wb first (needed after the weights changed).
hipError_t launch_scorer_fused(const ScorerFusedArgs& a, bool transpose, hipStream_t s);

// Replay of a recorded gather stream (measurement yardstick).
hipError_t launch_record_gathers(const StackArgs& a, int64_t* cnt, const int64_t* gstart, int64_t* list,
                                 hipStream_t s);
hipError_t launch_gather_replay(const float2* planes, const int64_t* gstart, const int64_t* list, int64_t n,
                                float* snr, hipStream_t s);

// Per-image iterated-MAD noise: per-image selection state.
struct NoiseState {
  double m_cur, thr_cur;  // current set: finite x with |x - m_cur| <= thr_cur
  double m_new, thr_new;  // median of the set and the next clip half-width
  double sigma;
  double val[2];          // the two selected middle values
  uint64_t prefix[2];     // key bits chosen so far
  int64_t rank[2];        // target ranks among keys sharing the prefix
  int64_t n, n_new, n_used;
  int64_t n_list;         // deviation keys compacted for the last digits (> NOISE_LIST_CAP: not used)
  int32_t iter, done, changed, pad;
};
constexpr int64_t NOISE_LIST_CAP = 65536;  // compacted deviation keys per image
constexpr double NOISE_KAPPA = 3.0;   // clip half-width in sigma (patches without variance planes)
constexpr int NOISE_MAX_ITER = 10;
size_t noise_scratch_bytes(int n_img);
hipError_t launch_noise(const void* const* d_imgs, const int64_t* d_npix, int64_t max_pix, int n_img, dt_dtype dtype,
                        double kappa, int max_iter, void* scratch, double* d_sigma, int64_t* d_used, int32_t* d_iters,
                        ExpMeta* d_meta, hipStream_t s);

// Device-side orbit sampling (GenerateOrbits) and generate-and-stack.
hipError_t launch_generate(const dt_orbit_sampler& S, int64_t first, int64_t n, double* a, double* e, double* inc,
                           double* node, double* peri, double* m0, hipStream_t s);
hipError_t launch_stack_generated(const StackArgs& a, const dt_orbit_sampler& S, int64_t first, hipStream_t s);
// Per-sample walk of every generated orbit (no checkpoint kernel, no list).
hipError_t launch_stack_generated_walk(const StackArgs& a, const dt_orbit_sampler& S, int64_t first, hipStream_t s);


// Resolves, with `device` current, the device address of the allocation-free
// top-k's fixed scratch array (once per device).
hipError_t topk_noalloc_setup(int device);
// Top-k scratch requirement (bytes) for n inputs and k outputs.
size_t topk_scratch_bytes(int64_t n, int32_t k);
// ordered false: inputs of at most 16384 keys skip the final sort (the
// selection is the same; larger inputs come out sorted either way).
hipError_t launch_topk(const float* d_snr, int64_t n, int32_t k, float thr, int64_t* d_idx, float* d_val,
                       int32_t* d_count, void* d_scratch, hipStream_t s, bool ordered = true);

}  // namespace dtk
