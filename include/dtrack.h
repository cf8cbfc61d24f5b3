/*
 * dtrack.h -- C ABI of libdtrack, the MI355X (gfx950) implementation of the
 * hot path of non-linear digital tracking (Golovich et al. 2025, "Survey-Wide
 * Asteroid Discovery with a High-Performance Computing Enabled Non-Linear
 * Digital Tracking Framework").
 *
 * The library answers the problem stated by Algorithm 1 and Sec. 3 of the
 * paper: given images with per-pixel noise variance, their epochs, observer
 * positions and WCS, and a set of candidate Keplerian orbits, it carries every
 * orbit to every exposure, maps it to pixels, applies a Gaussian matched filter
 * where it lands, combines the per-image signals under a constant-flux model
 * into one S/N per orbit, and selects the significant orbits.
 *
 * Conventions shared by every entry point
 *   - Every function returns dt_status; DT_OK == 0.  No C++ exception crosses
 *     the ABI.  On failure dt_last_error() returns a thread-local message.
 *   - All arguments are validated before any work is enqueued; on DT_E_ARG or
 *     DT_E_DOMAIN nothing is written.
 *   - "device" pointers are HIP device allocations on the context's device;
 *     "host" pointers are ordinary host memory read during the call only.
 *   - The caller owns every buffer it passes.  Image buffers are borrowed by a
 *     patch for its lifetime; the library owns (and frees in *_destroy) the
 *     matched-filter planes, metadata and scratch it allocates.
 *   - All GPU work is enqueued on the context's HIP stream; outputs are valid
 *     after that stream is synchronised.  A context is used by one host thread.
 *   - Units: days, AU, radians for orbital elements, degrees for WCS.
 *
 * Entry points by step of the method
 *   image set, exposure metadata, matched-filter planes: dt_patch_create
 *   propagate, project, gather, stack (orbits in HBM): dt_stack
 *   the same with orbits drawn on the device:           dt_stack_generated
 *   many patches in one persistent launch:               dt_stack_batched
 *   threshold + top-k selection:                         dt_topk (dt_topk_noalloc,
 *                                                        dt_topk_unordered)
 *   learned cell proposer: dt_cell_stamps, dt_scorer_*, dt_cell_members_near,
 *                          dt_stack_ids, dt_stack_cells
 *   checking only: dt_debug_samples, dt_debug_stack_samples, dt_record_gathers,
 *                  dt_gather_replay, dt_ctx_count_work
 */
#ifndef DTRACK_H
#define DTRACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DT_OK = 0,
  DT_E_ARG = -1,     /* null pointer, bad size or shape */
  DT_E_DOMAIN = -2,  /* value outside the method's domain (e.g. e >= 1, a <= 0, singular CD) */
  DT_E_OOM = -3,     /* device allocation failed or the context memory limit would be exceeded */
  DT_E_HIP = -4,     /* a HIP runtime call failed; message has hipGetErrorString */
  DT_E_STATE = -5    /* object used in the wrong state (e.g. destroyed context) */
} dt_status;

typedef enum { DT_F32 = 0, DT_F16 = 1 } dt_dtype;

typedef struct dt_ctx dt_ctx;
typedef struct dt_patch dt_patch;

/* One exposure (host record, copied at patch creation).  Sec. 3: each image
 * header supplies the epoch, the WCS and the PSF width; the observer position
 * at the epoch is supplied by the caller (the paper takes it from an
 * ephemeris).  The WCS is FITS TAN with a CD matrix: pixel (x, y) with
 * 0-based centres at integers maps to intermediate coordinates
 * CD * (x + 1 - CRPIX1, y + 1 - CRPIX2) in degrees. */
typedef struct {
  double t;               /* mid-exposure epoch (days), same scale as the orbit epoch */
  double obs_xyz_au[3];   /* heliocentric observer position, ecliptic J2000, AU */
  double crval_deg[2];    /* TAN tangent point (RA, Dec), equatorial J2000, degrees */
  double crpix[2];        /* FITS 1-based reference pixel (x, y) */
  double cd_deg[4];       /* CD1_1, CD1_2, CD2_1, CD2_2 (deg/px); must be invertible */
  int32_t width, height;  /* pixels; images are row-major [height][width] */
  float psf_fwhm_px;      /* Gaussian PSF FWHM in pixels, 0.5 <= fwhm <= 8 */
  float reserved;         /* set to 0 */
} dt_exposure;

/* A set of candidate orbits in SoA form (device pointers, n doubles each):
 * osculating heliocentric ecliptic-J2000 elements at the common epoch
 * `epoch`: semi-major axis a (AU), eccentricity e in [0, 1), inclination,
 * longitude of the ascending node, argument of perihelion and mean anomaly
 * (radians).  Sec. 3: two-body elliptical motion about a fixed Sun. */
typedef struct {
  int64_t n;
  double epoch;
  const double *a, *e, *inc, *node, *peri, *m0;
} dt_orbits;

/* Thread-local message describing the last failure of this thread ("" if none). */
const char *dt_last_error(void);
/* Library version string. */
const char *dt_version(void);

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
dt_status dt_ctx_create(int device, void *hip_stream, dt_ctx **out);
/* Change the stream later calls enqueue on. */
dt_status dt_ctx_set_stream(dt_ctx *ctx, void *hip_stream);
/* Cap the bytes of device memory the context may hold (planes, metadata,
 * scratch); 0 = no cap.  Later allocations beyond it fail with DT_E_OOM. */
dt_status dt_ctx_set_mem_limit(dt_ctx *ctx, size_t bytes);
/* Bytes of device memory currently held by the context. */
dt_status dt_ctx_mem_used(dt_ctx *ctx, size_t *out);
/* Destroy the context; its patches must be destroyed first (DT_E_STATE otherwise). */
dt_status dt_ctx_destroy(dt_ctx *ctx);

/* Work counters (measurement, no paper counterpart).  While counting is on
 * (on != 0; turning it on zeroes the counters), every stack launch of the
 * context that runs the checkpoint walk (dt_stack, dt_stack_generated,
 * dt_stack_batched, dt_stack_cells) adds what it did.  dt_ctx_work
 * synchronises the context stream, writes the totals since the last read
 * (out, host, DT_WORK_COUNTERS values) and zeroes them:
 *   out[0] samples tested by the checkpoint prediction (live orbit x exposure)
 *   out[1] queued samples solved exactly   out[2] checkpoint solves
 *   out[3] samples walked by the per-sample tail after a wavefront switched
 *   out[4] tail samples that took the full path (light time and projection)
 *   out[5] wavefronts that switched        out[6..7] 0
 * Launches captured into a graph count on every replay while counting was
 * on at capture time.  Counting costs atomics per wavefront; leave it off
 * when timing. */
#define DT_WORK_COUNTERS 8
dt_status dt_ctx_count_work(dt_ctx *ctx, int32_t on);
dt_status dt_ctx_work(dt_ctx *ctx, uint64_t *out);

/* Build a patch: n_exp exposures (host array `exps`) with their flux and
 * variance images (host arrays of n_exp device pointers, each a row-major
 * height x width image of `dtype`).  Enqueues the exposure-metadata kernel
 * and the matched-filter pre-pass (Sec. 3, FindLocalSignal): for every pixel
 * the planes psi = sum P D / V and phi = sum P^2 / V over a (2R+1)^2 stamp of
 * the unit-sum Gaussian P (sigma = FWHM / 2.3548, R = ceil(3 sigma)), pixels
 * off the image, non-finite or with V <= 0 carrying no weight.  By linearity
 * this equals the filter applied at the nearest pixel of any intersection.
 * Image buffers are borrowed until dt_patch_destroy; the planes are owned.
 * d_var == NULL: no variance planes; every pre-pass (here and in
 * dt_patch_refresh) first estimates each image's noise sigma by the iterated
 * MAD of dt_image_noise (kappa = 3, at most 10 steps) and uses V = sigma^2
 * (rounded to FP32) at every pixel. */
dt_status dt_patch_create(dt_ctx *ctx, const dt_exposure *exps, int32_t n_exp,
                          const void *const *d_flux, const void *const *d_var, dt_dtype dtype,
                          dt_patch **out);
/* Per-image noise by an iterated median absolute deviation (Sec. 3: the
 * pixel noise of each image comes from an iterative MAD).  For each image i
 * (host arrays: d_images[i] a device pointer to n_pixels[i] values of
 * `dtype`): S = its finite pixels; repeat at most max_iter times: m =
 * median(S), sigma = 1.4826 median{|x - m| : x in S}, S' = {finite x :
 * |x - m| <= kappa sigma}; stop when S' == S, else S = S'.  The median of an
 * even count is the mean of the two middle values; m, |x - m|, sigma and the
 * clip test are FP64, so the result is exact.  Outputs (device, n_img each,
 * any may be NULL): sigma of the last step (NaN for an image with no finite
 * pixel), the size of the set it came from, the number of steps.  Enqueued
 * on the context stream; the host arrays are not read after return.
 * 0 <= n_img <= 65535. */
dt_status dt_image_noise(dt_ctx *ctx, int32_t n_img, const void *const *d_images, const int64_t *n_pixels,
                         dt_dtype dtype, double kappa, int32_t max_iter, double *d_sigma, int64_t *d_n_used,
                         int32_t *d_iters);
/* Copy the noise sigma of a patch created without variance planes (device,
 * n_exp doubles, caller order; valid after the pre-pass has run). */
dt_status dt_patch_noise(dt_patch *p, double *d_sigma);

/* Re-run the pre-pass after the caller changed the borrowed images in place. */
dt_status dt_patch_refresh(dt_patch *p);
dt_status dt_patch_destroy(dt_patch *p);
/* Copy the (psi, phi) plane of exposure `e` (caller order) into d_out
 * (device, height*width float2 interleaved {psi, phi}, row-major). */
dt_status dt_patch_plane(dt_patch *p, int32_t e, float *d_out);

/* The plain stack (Algorithm 1 SearchImages + FilterGPUIntersections +
 * FindLocalSignal + constant-flux combination, Sec. 3): for every orbit,
 * over every exposure in epoch order, propagate with light time, project
 * through the TAN WCS, take the nearest pixel floor(p + 0.5); a sample is
 * valid if it is in front of the tangent plane, inside the image and the
 * filter weight phi there is > 0.  Outputs (device, n each):
 *   d_snr    = Psi / sqrt(Phi), Psi = sum psi, Phi = sum phi over valid samples
 *   d_flux   = Psi / Phi       (both 0 when Phi == 0)
 *   d_nvalid = number of valid samples.
 * Any output pointer may be NULL.  The call does not synchronise: an orbit
 * outside the domain (non-finite element, a <= 0, e outside [0, 1)) gets
 * S/N = flux = NaN and nvalid = -1; dt_orbits_validate reports such orbits
 * as an error before any stacking if the caller wants that. */
dt_status dt_stack(dt_patch *p, const dt_orbits *orbits, float *d_snr, float *d_flux,
                   int32_t *d_nvalid);

/* Count the orbits outside the domain (synchronises the context stream).
 * Returns DT_E_DOMAIN if *n_bad > 0, DT_OK otherwise. */
dt_status dt_orbits_validate(dt_ctx *ctx, const dt_orbits *orbits, int64_t *n_bad);

/* Detection (Algorithm 1 FindSignificantResults): the k orbits of largest
 * S/N among those with S/N >= threshold, ordered by S/N descending, ties to
 * the lower index.  d_snr: device, n floats (NaN never selected).
 * Outputs (device): d_idx[k] int64, d_val[k] float, d_count[1] = number
 * written (<= k).  1 <= k <= 4096, n < 2^32. */
dt_status dt_topk(dt_ctx *ctx, const float *d_snr, int64_t n, int32_t k, float threshold,
                  int64_t *d_idx, float *d_val, int32_t *d_count);

/* The same selection as dt_topk (same arguments, rules and errors; the same
 * set of orbits and count), for callers that only need the set, such as the
 * learned proposer's choice of cells: for n <= 16384 the first *d_count
 * entries are in an order fixed by the input but not sorted (the final sort
 * is skipped); larger inputs come out sorted as by dt_topk.  Entries past
 * the count are idx -1, val NaN. */
dt_status dt_topk_unordered(dt_ctx *ctx, const float *d_snr, int64_t n, int32_t k, float threshold,
                            int64_t *d_idx, float *d_val, int32_t *d_count);

/* Allocation-free top-k, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same selection, order, outputs and argument rules as
 * dt_topk, but the tournament's key buffers live in a fixed device array of
 * DT_TOPK_NOALLOC_BYTES bytes that the library holds on every GPU it runs on
 * until the process ends (its address is resolved by dt_ctx_create); the
 * call allocates nothing.  Inputs whose tournament needs more than that --
 * (2 ceil(n / T) k + 8192) * 8 bytes with tiles of T = 8192 keys when
 * n > 65536, so e.g. n = 10^7 with k <= 1700 or n = 10^9 with k <= 17 fit --
 * fail with DT_E_ARG before anything is enqueued; n <= 16384 needs none.
 * Every call on one GPU shares that array: calls that may overlap on a GPU
 * (different streams or contexts on the same device) race and must be
 * serialised by the caller.  No part of the array needs clearing between
 * calls (every key a round reads was written by the previous round of the
 * same call). */
#define DT_TOPK_NOALLOC_BYTES (32u << 20)
dt_status dt_topk_noalloc(dt_ctx *ctx, const float *d_snr, int64_t n, int32_t k, float threshold,
                          int64_t *d_idx, float *d_val, int32_t *d_count);

/* Launch shape of the batched stack: orbits per work item for the
 * largest-first ordering (multiple of 256 in [256, 65536]) and persistent
 * groups of four wavefronts per compute unit ([1, 16]). */
typedef struct {
  int32_t chunk;
  int32_t wg_per_cu;
} dt_batch_config;

enum {
  DT_BATCH_PREPASS = 1, /* run every patch's matched-filter pre-pass first */
  DT_BATCH_EAGER = 2    /* launch directly instead of capturing / replaying a graph */
};

/* Many patches, each with its own exposures and orbit set, stacked by one
 * persistent launch (the same per-orbit computation as dt_stack, Sec. 3):
 * every patch's orbits are cut into work items of cfg->chunk orbits, ordered
 * largest first (exposures x orbits), cut again into items of 64 orbits in
 * that order and pulled from a device counter by 4 cfg->wg_per_cu persistent
 * wavefronts per CU.  Then, if k > 0, the top-k of
 * every patch (as dt_topk) is written to d_topk_idx / d_topk_val
 * [n_patches * k] and d_topk_count [n_patches] (device).  patches, sets and
 * the output arrays are host arrays of n_patches entries; d_snr / d_flux /
 * d_nvalid entries are device pointers (n floats / ints each; NULL allowed
 * unless k > 0 needs the S/N).  cfg NULL = {1024, 4}.
 * Unless DT_BATCH_EAGER, the sequence is captured once into a HIP graph kept
 * by the context and replayed by later calls with identical arguments
 * (patches, orbit pointers and sizes, outputs, k, threshold, cfg, flags);
 * any change re-captures.  The graph is dropped when a patch it uses is
 * destroyed or releases its images, and with the context. */
dt_status dt_stack_batched(dt_ctx *ctx, dt_patch *const *patches, const dt_orbits *sets, int32_t n_patches,
                           float *const *d_snr, float *const *d_flux, int32_t *const *d_nvalid,
                           int32_t k, float threshold, int64_t *d_topk_idx, float *d_topk_val,
                           int32_t *d_topk_count, const dt_batch_config *cfg, uint32_t flags);

/* Pick the batched launch shape by timing candidate shapes on these very
 * inputs (chunk in {256..4096}, wg_per_cu in {2, 4, 8}); writes the outputs
 * as a side effect.  With cache_path (a text file, one "shape-class chunk
 * wg_per_cu ms" line per entry) a cached entry for the inputs' shape class
 * (patch count and log2 of total samples, largest orbit set and largest
 * exposure count) is returned without timing (*best_ms = -1), and a new
 * result is appended.  best_ms may be NULL. */
dt_status dt_autotune_batched(dt_ctx *ctx, dt_patch *const *patches, const dt_orbits *sets, int32_t n_patches,
                              float *const *d_snr, float *const *d_flux, int32_t *const *d_nvalid,
                              const char *cache_path, dt_batch_config *best, double *best_ms);

/* Forget the patch's image buffers (the planes stay): the caller may free
 * the images afterwards; dt_patch_refresh and DT_BATCH_PREPASS then fail
 * with DT_E_STATE. */
dt_status dt_patch_release_images(dt_patch *p);

/* Measurement yardstick for the stack's gathers (no paper counterpart).
 * dt_record_gathers records, for orbits 0 .. n - 1 of `orbits`, the global
 * plane offset (float2 units, int64) of every sample that lands inside an
 * image -- the gathers dt_stack makes -- in epoch order per orbit.  Orbits
 * are taken in groups of 64 (one wavefront's lanes); group g has width w_g =
 * the largest count among its orbits and holds its entries slot-major:
 * entry k of lane l at d_list[d_start[g] + 64 k + l], -1 past that orbit's
 * count; d_start[g] = 64 (w_0 + ... + w_{g-1}), g = 0 .. ceil(n / 64).
 * Two calls: with d_list == NULL it counts, writes d_start (device,
 * ceil(n / 64) + 1 int64) and the host values *h_entries (= d_start's last
 * entry, the list length) and *h_gathers (the number of recorded gathers;
 * may be NULL), and synchronises; then, with the same d_start and a device
 * d_list of *h_entries int64, it records (enqueued, no synchronisation).
 * dt_gather_replay loads those offsets' (psi, phi) -- eight loads in flight
 * per lane, no orbit arithmetic -- and sums them in order exactly as
 * dt_stack does (d_snr, device, n floats: equal to dt_stack's S/N of every
 * orbit with n_valid > 0, 0 otherwise).  Its rate is the achievable gather
 * rate of the stack's own access stream. */
dt_status dt_record_gathers(dt_patch *p, const dt_orbits *orbits, int64_t *d_start, int64_t *d_list,
                            int64_t *h_entries, int64_t *h_gathers);
dt_status dt_gather_replay(dt_patch *p, const int64_t *d_start, const int64_t *d_list, int64_t n, float *d_snr);

/* Candidate-orbit distribution for on-device sampling (Algorithm 1,
 * GenerateOrbits): a, e, i uniform in their ranges (AU, -, radians); a line
 * of sight uniform over the tangent-plane rectangle |xi| <= half_w,
 * |eta| <= half_h (radians) about the unit vector `center` with axes
 * `east`, `north` (ecliptic); the orbit's geometric heliocentric position at
 * `epoch` lies on that line of sight from `obs_xyz_au`, with a uniform true
 * anomaly and nodal branch; the inclination is raised to |latitude| when the
 * line of sight needs it.  Orbit k is a pure function of (seed, k). */
typedef struct {
  double epoch;
  double obs_xyz_au[3];
  double center[3], east[3], north[3];
  double half_w, half_h;
  double a_range[2], e_range[2], inc_range[2];
  uint64_t seed;
} dt_orbit_sampler;

/* Orbits first .. first + n - 1 of the sampler into device SoA arrays
 * (an index whose 16 attempts all miss gets a = NaN); 0 <= n < 2^32. */
dt_status dt_generate_orbits(dt_ctx *ctx, const dt_orbit_sampler *sampler, int64_t first, int64_t n, double *d_a,
                             double *d_e, double *d_inc, double *d_node, double *d_peri, double *d_m0);
/* dt_stack on orbits first .. first + n - 1 of the sampler, generated in
 * registers (no element arrays); outputs (device, n each) as dt_stack.
 * With a finite observer-speed bound and n > 2^26, the first 2^22 orbits
 * run the checkpoint walk first; if at least 90 % of their wavefronts defer
 * to the per-sample walk (orbits that land in most exposures), the other
 * orbits go to the per-sample walk directly.  That decision reads one count
 * back, so such a call synchronises the context stream once (it cannot be
 * captured into a graph); it depends only on those orbits and the
 * exposures, so results stay deterministic. */
dt_status dt_stack_generated(dt_patch *p, const dt_orbit_sampler *sampler, int64_t first, int64_t n, float *d_snr,
                             float *d_flux, int32_t *d_nvalid);

/* Per-intersection outlier trimming of candidate orbits (Sec. 5.2.3): for
 * each of m orbits (device int64 ids into `orbits`), the valid samples'
 * (psi_e, phi_e) from the stack's device code are clipped two-sided at
 * |psi_e - F phi_e| / sqrt(phi_e) > kappa.  Iteration 1 takes F = the median of
 * the per-sample fluxes psi_e / phi_e (mean of the two middle values for an
 * even count); each later round takes F = sum psi / sum phi of the samples
 * the previous round kept; it stops when a round keeps exactly the set it
 * started from, or after max_iter rounds.  Outputs (device, m each, may be
 * NULL): S/N, flux and the kept count after trimming (0, 0, 0 when nothing
 * is kept).  Patches of at most 512 exposures.  Synchronises. */
dt_status dt_clip_candidates(dt_patch *p, const dt_orbits *orbits, const int64_t *d_ids, int64_t m,
                             double kappa, int32_t max_iter, float *d_snr, float *d_flux, int32_t *d_nkept);

/* ---- learned proposal (this library's extension, not part of the paper) ----
 * Orbit-grid cells: a grid stored cell-major, cell c owning orbits
 * [c * cell_size, (c + 1) * cell_size), its first member the representative.
 *
 * Coarse-stacked stamps of n representative orbits (reps, device SoA) of
 * cells whose members differ from the representative by at most da (AU) in
 * semi-major axis and dm (rad) in mean anomaly.  Per exposure, three walks
 * with the stack's device code give the pixel coordinates p (the
 * representative), p_a (a + da) and p_m (M0 + dm); if any is behind the
 * tangent plane the exposure is skipped.  Node (u, v) of a 21 x 21 lattice,
 * u = (col - 10) / 10, v = (row - 10) / 10, follows
 * q = (p + u (p_a - p)) + v (p_m - p) (FP64, in this order), rounded to the
 * nearest pixel floor(q + 0.5); its value is the constant-flux S/N
 * sum psi / sqrt(sum phi) over the nodes' valid pixels (inside, phi > 0),
 * i.e. the paper's stack (Sec. 3) along the linearised tracks of the cell's
 * members.  Plus 16 features per cell: stamp max, centre, mean, std,
 * coverage, lattice distance of the max, fraction of exposures with the
 * representative inside, normalised a, e, i, max over the central 7x7, the
 * lattice coordinates (u, v) of the max (its first node in row-major order),
 * zeros.  Outputs (device, any may be NULL): stamps n x 441 (row-major) as
 * BF16 and/or FP32, features n x 16 as BF16 and/or FP32.  Enqueued on the
 * context stream; patches of at most 1024 exposures (the walks of a cell
 * are held on chip). */
dt_status dt_cell_stamps(dt_patch *p, const dt_orbits *reps, double da, double dm, uint16_t *d_stamps_bf16,
                         float *d_stamps_f32, uint16_t *d_feats_bf16, float *d_feats_f32);

/* The plain stack (as dt_stack) on the orbits of n_cells selected cells
 * (device int64 cell ids; negative ids are skipped); outputs are written at
 * the orbits' indices in the full-grid arrays d_snr / d_flux / d_nvalid
 * (device, grid->n each), other entries are left untouched.  Valid counts
 * equal dt_stack's; when few orbits are selected each orbit's exposures are
 * walked in up to four contiguous ranges whose compensated sums are merged
 * in range order, so S/N and flux agree with dt_stack's to rounding
 * (deterministically for a given selection size). */
dt_status dt_stack_cells(dt_patch *p, const dt_orbits *grid, const int64_t *d_cells, int64_t n_cells,
                         int32_t cell_size, float *d_snr, float *d_flux, int32_t *d_nvalid);

/* Maximum of each of n_seg consecutive segments of seg values (device FP32
 * in, device FP32 out, NaN ignored, -inf for a segment of NaN only): the
 * coarse-to-fine ranking takes each cell's best sub-representative (Sec.
 * 5.2.2).  Enqueued, no synchronisation. */
dt_status dt_segment_max(dt_ctx *ctx, const float *d_x, int64_t n_seg, int32_t seg, float *d_out);

/* Members of selected cells near their stamp peak (fine stacking around a
 * coarse peak, Sec. 5.2.2): for each of the n_cells selected cells c (device
 * int64 ids; negative ids are skipped) of a cell-major grid, member m
 * (orbit c * cell_size + m; the representative is member 0) sits at lattice
 * coordinates u = (a_m - a_rep) / da, v = (M0_m - M0_rep) / dm; it is listed
 * when |u - u*| <= radius and |v - v*| <= radius, where (u*, v*) =
 * (d_uv[c * uv_stride], d_uv[c * uv_stride + 1]) -- features 11 and 12 of
 * dt_cell_stamps (FP32 output, uv_stride 16) give the stamp maximum's.
 * d_ids (device, n_cells * cell_size capacity) receives the listed orbit ids
 * in no particular order and *d_count (device int64) their number; the count
 * is zeroed first by a kernel, so the call can be captured in a graph.
 * Nothing synchronises. */
dt_status dt_cell_members_near(dt_ctx *ctx, const dt_orbits *grid, const int64_t *d_cells, int64_t n_cells,
                               int32_t cell_size, const float *d_uv, int32_t uv_stride, double da, double dm,
                               double radius, int64_t *d_ids, int64_t *d_count);

/* The plain stack (as dt_stack) on the orbits of a device id list: the first
 * *d_count (device int64, at most m_max) entries of d_ids (device int64 ids
 * into `orbits`; ids outside [0, orbits->n) are skipped).  Outputs are written
 * at the orbits' own indices of d_snr / d_flux / d_nvalid (device, orbits->n
 * each); other entries are left untouched.  Valid counts equal dt_stack's
 * for the same orbits (up to samples within ~1e-11 px of a rounding
 * boundary); a list whose count is at most 2^17 is walked with each orbit's
 * exposures split over eight wavefronts whose compensated sums are merged
 * in exposure order, so S/N and flux agree with dt_stack's to rounding.  The
 * count stays on the device (the kernels read it; nothing synchronises). */
dt_status dt_stack_ids(dt_patch *p, const dt_orbits *orbits, const int64_t *d_ids, const int64_t *d_count,
                       int64_t m_max, float *d_snr, float *d_flux, int32_t *d_nvalid);

/* The scorer's GEMM on its own: C = op(A) op(B) (+ bias[n]) (ReLU if relu),
 * BF16 inputs, FP32 accumulation and output (device, row-major with leading
 * dimensions; op(A) is M x K and A is stored K x M when transA; op(B) is
 * K x N and B is stored N x K when transB).  Synchronises. */
dt_status dt_gemm_bf16(dt_ctx *ctx, const uint16_t *d_A, int32_t lda, int32_t transA, const uint16_t *d_B,
                       int32_t ldb, int32_t transB, int32_t M, int32_t N, int32_t K, const float *d_bias,
                       int32_t relu, float *d_C, int32_t ldc);

/* The cell scorer: CNN on the 21x21 stamp + MLP on the 16 features -> one
 * logit per cell, trained with binary cross-entropy and Adam on FP32 master
 * weights; all GEMMs are BF16 MFMA with FP32 accumulation.  Parameters are
 * one FP32 vector of dt_scorer_num_params() values (layer order w1 b1 ... w7
 * b7, weights [K, N] row-major).  Inputs are device BF16 arrays: stamps
 * B x 441, features B x 16; labels FP32 0/1.  1 <= B <= max_batch. */
typedef struct dt_scorer dt_scorer;
int64_t dt_scorer_num_params(void);
/* He-normal weights from a counter-based generator seeded by `seed`, zero biases;
 * 1 <= max_batch <= 32768 (the activations of max_batch cells are held). */
dt_status dt_scorer_create(dt_ctx *ctx, int32_t max_batch, uint64_t seed, dt_scorer **out);
dt_status dt_scorer_destroy(dt_scorer *s);
dt_status dt_scorer_get_params(dt_scorer *s, float *d_params);
/* Replace the weights (device FP32) and reset the optimiser state. */
dt_status dt_scorer_set_params(dt_scorer *s, const float *d_params);
dt_status dt_scorer_forward(dt_scorer *s, const uint16_t *d_stamps, const uint16_t *d_feats, int32_t B,
                            float *d_logits);
/* Inference logits of any number B >= 0 of cells in one fused kernel (no
 * activations leave the chip; no batch limit): the same layers, BF16 rounding
 * points and FP32 biases as dt_scorer_forward; the fully connected 1152 -> 64
 * layer accumulates its K in one sequence, so logits may differ from
 * dt_scorer_forward's (which may split that K) by FP32 rounding and the BF16
 * roundings it moves.  d_logits: device, B floats. */
dt_status dt_scorer_infer(dt_scorer *s, const uint16_t *d_stamps, const uint16_t *d_feats, int32_t B,
                          float *d_logits);
/* dt_scorer_infer on selected rows: cell i of the batch (i < B) is row
 * d_rows[i] (device int64) of d_stamps (rows of 441) and d_feats (rows of
 * 16), and its logit is written to d_logits[d_rows[i]]; other entries of
 * d_logits are left untouched (a caller scoring a pre-selected subset of
 * its cells fills the rest first).  Rows may repeat only with equal logits. */
dt_status dt_scorer_infer_rows(dt_scorer *s, const uint16_t *d_stamps, const uint16_t *d_feats,
                               const int64_t *d_rows, int32_t B, float *d_logits);
/* Loss (device float[1], may be NULL) and gradient (device FP32 vector of
 * num_params values, may be NULL) of the mean BCE at the current weights. */
dt_status dt_scorer_grad(dt_scorer *s, const uint16_t *d_stamps, const uint16_t *d_feats, const float *d_labels,
                         int32_t B, float *d_loss, float *d_grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at learning rate lr. */
dt_status dt_scorer_train_step(dt_scorer *s, const uint16_t *d_stamps, const uint16_t *d_feats,
                               const float *d_labels, int32_t B, float lr, float *d_loss);

/* Per-sample table for m selected orbits (device int64 ids into `orbits`)
 * from the exact per-sample walk: every sample propagated with light time,
 * projected and gathered by the device functions the stack kernels use
 * (Sec. 3 SearchImages + FilterGPUIntersections, Algorithm 1), with no
 * pruning.  Outputs (device, m x n_exp each, exposures in caller order; any
 * may be NULL):
 *   px, py  0-based pixel coordinates (FP64), ix, iy nearest pixel,
 *   flags   bit0 in front, bit1 inside image, bit2 valid (phi > 0), bit3 solved
 *           (always set here),
 *   psi, phi the gathered plane values (0 when not valid), tau light time (days).
 * An id outside [0, orbits->n) or an orbit outside the domain gets the
 * initial row: flags 0, NaN coordinates and light time, ix = iy = INT32_MIN. */
dt_status dt_debug_samples(dt_patch *p, const dt_orbits *orbits, const int64_t *d_ids, int64_t m,
                           double *d_px, double *d_py, int32_t *d_ix, int32_t *d_iy,
                           int32_t *d_flags, float *d_psi, float *d_phi, double *d_tau);
/* The same table from the walk dt_stack itself runs on this patch (the
 * checkpoint walk with its queue, and the per-sample tail it may switch to;
 * or, for patches without an observer speed bound, the per-sample walk with
 * its sky-cone test): only the samples that walk solves exactly carry
 * flags bit3 and their px, py, ix, iy, tau, psi, phi; the samples its bounds
 * exclude keep the initial row values.  Every sample that lands in an image
 * is among the solved ones. */
dt_status dt_debug_stack_samples(dt_patch *p, const dt_orbits *orbits, const int64_t *d_ids, int64_t m,
                                 double *d_px, double *d_py, int32_t *d_ix, int32_t *d_iy,
                                 int32_t *d_flags, float *d_psi, float *d_phi, double *d_tau);

#ifdef __cplusplus
}
#endif
#endif /* DTRACK_H */
