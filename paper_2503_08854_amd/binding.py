"""ctypes binding of libdtrack: argument marshalling only.

Torch tensors provide device memory; their ``data_ptr()`` values cross the
C ABI as plain pointers and the current torch stream is the library's stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdtrack.so")

DT_OK, DT_E_ARG, DT_E_DOMAIN, DT_E_OOM, DT_E_HIP, DT_E_STATE = 0, -1, -2, -3, -4, -5
DT_F32, DT_F16 = 0, 1
_NAMES = {DT_E_ARG: "DT_E_ARG", DT_E_DOMAIN: "DT_E_DOMAIN", DT_E_OOM: "DT_E_OOM", DT_E_HIP: "DT_E_HIP",
          DT_E_STATE: "DT_E_STATE"}


class DtrackError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class DtExposure(C.Structure):
    _fields_ = [("t", C.c_double), ("obs_xyz_au", C.c_double * 3), ("crval_deg", C.c_double * 2),
                ("crpix", C.c_double * 2), ("cd_deg", C.c_double * 4), ("width", C.c_int32),
                ("height", C.c_int32), ("psf_fwhm_px", C.c_float), ("reserved", C.c_float)]


class DtOrbits(C.Structure):
    _fields_ = [("n", C.c_int64), ("epoch", C.c_double), ("a", C.c_void_p), ("e", C.c_void_p),
                ("inc", C.c_void_p), ("node", C.c_void_p), ("peri", C.c_void_p), ("m0", C.c_void_p)]


class DtBatchConfig(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("wg_per_cu", C.c_int32)]


DT_BATCH_PREPASS, DT_BATCH_EAGER = 1, 2


class DtOrbitSampler(C.Structure):
    _fields_ = [("epoch", C.c_double), ("obs_xyz_au", C.c_double * 3), ("center", C.c_double * 3),
                ("east", C.c_double * 3), ("north", C.c_double * 3), ("half_w", C.c_double),
                ("half_h", C.c_double), ("a_range", C.c_double * 2), ("e_range", C.c_double * 2),
                ("inc_range", C.c_double * 2), ("seed", C.c_uint64)]

_lib = None
_P = C.c_void_p


def lib():
    """Load libdtrack.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    sig = {
        "dt_last_error": ([], C.c_char_p),
        "dt_version": ([], C.c_char_p),
        "dt_ctx_create": ([C.c_int, _P, C.POINTER(_P)], C.c_int),
        "dt_ctx_set_stream": ([_P, _P], C.c_int),
        "dt_ctx_set_mem_limit": ([_P, C.c_size_t], C.c_int),
        "dt_ctx_mem_used": ([_P, C.POINTER(C.c_size_t)], C.c_int),
        "dt_ctx_destroy": ([_P], C.c_int),
        "dt_ctx_count_work": ([_P, C.c_int32], C.c_int),
        "dt_ctx_work": ([_P, C.POINTER(C.c_uint64)], C.c_int),
        "dt_patch_create": ([_P, C.POINTER(DtExposure), C.c_int32, C.POINTER(_P), C.POINTER(_P), C.c_int,
                             C.POINTER(_P)], C.c_int),
        "dt_patch_refresh": ([_P], C.c_int),
        "dt_patch_destroy": ([_P], C.c_int),
        "dt_patch_plane": ([_P, C.c_int32, _P], C.c_int),
        "dt_stack": ([_P, C.POINTER(DtOrbits), _P, _P, _P], C.c_int),
        "dt_orbits_validate": ([_P, C.POINTER(DtOrbits), C.POINTER(C.c_int64)], C.c_int),
        "dt_topk": ([_P, _P, C.c_int64, C.c_int32, C.c_float, _P, _P, _P], C.c_int),
        "dt_topk_noalloc": ([_P, _P, C.c_int64, C.c_int32, C.c_float, _P, _P, _P], C.c_int),
        "dt_topk_unordered": ([_P, _P, C.c_int64, C.c_int32, C.c_float, _P, _P, _P], C.c_int),
        "dt_debug_samples": ([_P, C.POINTER(DtOrbits), _P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P], C.c_int),
        "dt_stack_batched": ([_P, C.POINTER(_P), C.POINTER(DtOrbits), C.c_int32, C.POINTER(_P), C.POINTER(_P),
                              C.POINTER(_P), C.c_int32, C.c_float, _P, _P, _P, C.POINTER(DtBatchConfig),
                              C.c_uint32], C.c_int),
        "dt_autotune_batched": ([_P, C.POINTER(_P), C.POINTER(DtOrbits), C.c_int32, C.POINTER(_P),
                                 C.POINTER(_P), C.POINTER(_P), C.c_char_p, C.POINTER(DtBatchConfig),
                                 C.POINTER(C.c_double)], C.c_int),
        "dt_patch_release_images": ([_P], C.c_int),
        "dt_cell_stamps": ([_P, C.POINTER(DtOrbits), C.c_double, C.c_double, _P, _P, _P, _P], C.c_int),
        "dt_image_noise": ([_P, C.c_int32, _P, _P, C.c_int, C.c_double, C.c_int32, _P, _P, _P], C.c_int),
        "dt_patch_noise": ([_P, _P], C.c_int),
        "dt_record_gathers": ([_P, C.POINTER(DtOrbits), _P, _P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
                              C.c_int),
        "dt_gather_replay": ([_P, _P, _P, C.c_int64, _P], C.c_int),
        "dt_debug_stack_samples": ([_P, C.POINTER(DtOrbits), _P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P],
                                   C.c_int),
        "dt_scorer_infer": ([_P, _P, _P, C.c_int32, _P], C.c_int),
        "dt_scorer_infer_rows": ([_P, _P, _P, _P, C.c_int32, _P], C.c_int),
        "dt_generate_orbits": ([_P, C.POINTER(DtOrbitSampler), C.c_int64, C.c_int64, _P, _P, _P, _P, _P, _P],
                               C.c_int),
        "dt_stack_generated": ([_P, C.POINTER(DtOrbitSampler), C.c_int64, C.c_int64, _P, _P, _P], C.c_int),
        "dt_clip_candidates": ([_P, C.POINTER(DtOrbits), _P, C.c_int64, C.c_double, C.c_int32, _P, _P, _P],
                               C.c_int),
        "dt_stack_cells": ([_P, C.POINTER(DtOrbits), _P, C.c_int64, C.c_int32, _P, _P, _P], C.c_int),
        "dt_cell_members_near": ([_P, C.POINTER(DtOrbits), _P, C.c_int64, C.c_int32, _P, C.c_int32, C.c_double,
                                  C.c_double, C.c_double, _P, _P], C.c_int),
        "dt_stack_ids": ([_P, C.POINTER(DtOrbits), _P, _P, C.c_int64, _P, _P, _P], C.c_int),
        "dt_segment_max": ([_P, _P, C.c_int64, C.c_int32, _P], C.c_int),
        "dt_gemm_bf16": ([_P, _P, C.c_int32, C.c_int32, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                          _P, C.c_int32, _P, C.c_int32], C.c_int),
        "dt_scorer_num_params": ([], C.c_int64),
        "dt_scorer_create": ([_P, C.c_int32, C.c_uint64, C.POINTER(_P)], C.c_int),
        "dt_scorer_destroy": ([_P], C.c_int),
        "dt_scorer_get_params": ([_P, _P], C.c_int),
        "dt_scorer_set_params": ([_P, _P], C.c_int),
        "dt_scorer_forward": ([_P, _P, _P, C.c_int32, _P], C.c_int),
        "dt_scorer_grad": ([_P, _P, _P, _P, C.c_int32, _P, _P], C.c_int),
        "dt_scorer_train_step": ([_P, _P, _P, _P, C.c_int32, C.c_float, _P], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(st):
    if st != DT_OK:
        raise DtrackError(st, lib().dt_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def exposure_struct(exps):
    """List of exposure dicts (t, obs, crval, crpix, cd, width, height, fwhm) -> dt_exposure array."""
    arr = (DtExposure * len(exps))()
    for k, x in enumerate(exps):
        r = arr[k]
        r.t = float(x["t"])
        r.obs_xyz_au[:] = [float(v) for v in x["obs"]]
        r.crval_deg[:] = [float(v) for v in x["crval"]]
        r.crpix[:] = [float(v) for v in x["crpix"]]
        r.cd_deg[:] = [float(v) for v in x["cd"]]
        r.width = int(x["width"])
        r.height = int(x["height"])
        r.psf_fwhm_px = float(x["fwhm"])
        r.reserved = 0.0
    return arr


class Context:
    """A dt_ctx bound to a device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        self._h = _P()
        with torch.cuda.device(device):
            s = C.c_void_p(stream.cuda_stream) if stream is not None else _stream_handle()
            _check(lib().dt_ctx_create(device, s, C.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream):
        _check(lib().dt_ctx_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    def set_mem_limit(self, nbytes: int):
        _check(lib().dt_ctx_set_mem_limit(self._h, int(nbytes)))

    def mem_used(self) -> int:
        v = C.c_size_t()
        _check(lib().dt_ctx_mem_used(self._h, C.byref(v)))
        return v.value

    WORK_KEYS = ("predicted", "queued_solves", "checkpoint_solves", "tail_samples", "tail_full", "switched_waves")

    def count_work(self, on: bool = True):
        """Turn the stack kernels' work counters on (zeroed) or off."""
        _check(lib().dt_ctx_count_work(self._h, 1 if on else 0))

    def work(self) -> dict:
        """Work counted since the last read (synchronises; zeroes the counters)."""
        out = (C.c_uint64 * 8)()
        _check(lib().dt_ctx_work(self._h, out))
        return {k: int(out[i]) for i, k in enumerate(self.WORK_KEYS)}

    def close(self):
        if self._h:
            _check(lib().dt_ctx_destroy(self._h))
            self._h = _P()

    def __del__(self):
        try:
            if self._h:
                lib().dt_ctx_destroy(self._h)
        except Exception:
            pass


class Patch:
    """Exposures + borrowed device images; owns the matched-filter planes."""

    def __init__(self, ctx: Context, exps, flux, var=None):
        """var=None: no variance planes; each pre-pass estimates every image's
        noise by the iterated MAD and uses V = sigma^2 (see noise())."""
        import torch
        if len(exps) != len(flux) or (var is not None and len(exps) != len(var)):
            raise ValueError("exposures, flux and variance lists differ in length")
        dt = flux[0].dtype
        if dt not in (torch.float32, torch.float16):
            raise TypeError("images must be float32 or float16")
        for k, (x, d) in enumerate(zip(exps, flux)):
            v = var[k] if var is not None else d
            if d.dtype != dt or v.dtype != dt or not d.is_cuda or not v.is_cuda:
                raise TypeError("all images must be CUDA tensors of one dtype")
            if tuple(d.shape) != (int(x["height"]), int(x["width"])) or d.shape != v.shape:
                raise ValueError("image shape does not match its exposure")
            if not d.is_contiguous() or not v.is_contiguous():
                raise ValueError("images must be contiguous")
        self.ctx = ctx
        self.exps = list(exps)
        self.device = flux[0].device
        self._flux = list(flux)   # borrowed: keep alive
        self._var = list(var) if var is not None else None
        n = len(exps)
        xs = exposure_struct(exps)
        fp = (_P * n)(*[d.data_ptr() for d in flux])
        vp = (_P * n)(*[v.data_ptr() for v in var]) if var is not None else None
        self._h = _P()
        _check(lib().dt_patch_create(ctx.handle, xs, n, fp, vp, DT_F32 if dt == torch.float32 else DT_F16,
                                     C.byref(self._h)))

    @property
    def handle(self):
        return self._h

    @property
    def n_exp(self):
        return len(self.exps)

    def refresh(self):
        _check(lib().dt_patch_refresh(self._h))

    def plane(self, e: int):
        import torch
        x = self.exps[e]
        out = torch.empty((int(x["height"]), int(x["width"]), 2), dtype=torch.float32, device=self.device)
        _check(lib().dt_patch_plane(self._h, int(e), _ptr(out)))
        return out

    def noise(self):
        """Per-exposure noise sigma (FP64, caller order) of a patch without variance planes."""
        import torch
        out = torch.empty(self.n_exp, dtype=torch.float64, device=self.device)
        _check(lib().dt_patch_noise(self._h, _ptr(out)))
        return out

    def release_images(self):
        """Drop the borrowed images (the planes stay); refresh is no longer possible."""
        _check(lib().dt_patch_release_images(self._h))
        self._flux = self._var = None

    def close(self):
        if self._h:
            _check(lib().dt_patch_destroy(self._h))
            self._h = _P()

    def __del__(self):
        try:
            if self._h:
                lib().dt_patch_destroy(self._h)
        except Exception:
            pass


class OrbitSet:
    """SoA FP64 element arrays on the device (a, e, i, node, peri, M0) + epoch."""

    def __init__(self, elements, epoch: float, device="cuda"):
        import torch
        el = elements
        if isinstance(el, np.ndarray):
            el = torch.from_numpy(np.ascontiguousarray(el, dtype=np.float64))
        el = el.to(device=device, dtype=torch.float64)
        if el.dim() != 2 or el.shape[1] != 6:
            raise ValueError("elements must be (n, 6)")
        self.soa = el.t().contiguous()      # (6, n)
        self.n = int(el.shape[0])
        self.epoch = float(epoch)

    def struct(self):
        s = DtOrbits()
        s.n = self.n
        s.epoch = self.epoch
        base = self.soa.data_ptr()
        stride = self.n * 8
        for k, name in enumerate(("a", "e", "inc", "node", "peri", "m0")):
            setattr(s, name, base + k * stride if self.n else None)
        return s


def stack(patch: Patch, orbits: OrbitSet, out=None):
    """S/N, flux, n_valid per orbit (float32, float32, int32 device tensors)."""
    import torch
    dev = orbits.soa.device
    if out is None:
        out = (torch.empty(orbits.n, dtype=torch.float32, device=dev),
               torch.empty(orbits.n, dtype=torch.float32, device=dev),
               torch.empty(orbits.n, dtype=torch.int32, device=dev))
    snr, flux, nv = out
    s = orbits.struct()
    _check(lib().dt_stack(patch.handle, C.byref(s), _ptr(snr), _ptr(flux), _ptr(nv)))
    return snr, flux, nv


def validate_orbits(ctx: Context, orbits: OrbitSet) -> int:
    n_bad = C.c_int64()
    st = lib().dt_orbits_validate(ctx.handle, C.byref(orbits.struct()), C.byref(n_bad))
    if st not in (DT_OK, DT_E_DOMAIN):
        _check(st)
    return n_bad.value


def topk(ctx: Context, snr, k: int, threshold: float = float("-inf"), ordered: bool = True):
    """(idx int64[k], val float32[k], count int32[1]) device tensors;
    ordered=False calls dt_topk_unordered (the same set, not sorted)."""
    import torch
    dev = snr.device
    idx = torch.empty(k, dtype=torch.int64, device=dev)
    val = torch.empty(k, dtype=torch.float32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    fn = lib().dt_topk if ordered else lib().dt_topk_unordered
    _check(fn(ctx.handle, _ptr(snr), int(snr.numel()), int(k), float(threshold), _ptr(idx), _ptr(val), _ptr(cnt)))
    return idx, val, cnt


def topk_noalloc(ctx: Context, snr, idx, val, cnt, k: int, threshold: float = float("-inf")):
    """dt_topk_noalloc into caller-provided outputs (idx int64[k], val
    float32[k], cnt int32[1] device tensors): nothing is allocated."""
    _check(lib().dt_topk_noalloc(ctx.handle, _ptr(snr), int(snr.numel()), int(k), float(threshold), _ptr(idx),
                                 _ptr(val), _ptr(cnt)))
    return idx, val, cnt


def debug_samples(patch: Patch, orbits: OrbitSet, ids, walk: str = "exact"):
    """Per-sample table (m x n_exp, caller exposure order): walk="exact" is the
    exact per-sample walk (dt_debug_samples), walk="stack" the walk dt_stack
    runs, recording only the samples it solves (dt_debug_stack_samples)."""
    import torch
    dev = orbits.soa.device
    ids = torch.as_tensor(ids, dtype=torch.int64).to(dev)
    m, n = int(ids.numel()), patch.n_exp
    o = dict(px=torch.empty((m, n), dtype=torch.float64, device=dev),
             py=torch.empty((m, n), dtype=torch.float64, device=dev),
             ix=torch.empty((m, n), dtype=torch.int32, device=dev),
             iy=torch.empty((m, n), dtype=torch.int32, device=dev),
             flags=torch.empty((m, n), dtype=torch.int32, device=dev),
             psi=torch.empty((m, n), dtype=torch.float32, device=dev),
             phi=torch.empty((m, n), dtype=torch.float32, device=dev),
             tau=torch.empty((m, n), dtype=torch.float64, device=dev))
    s = orbits.struct()
    fn = {"exact": lib().dt_debug_samples, "stack": lib().dt_debug_stack_samples}[walk]
    _check(fn(patch.handle, C.byref(s), _ptr(ids), m, _ptr(o["px"]), _ptr(o["py"]), _ptr(o["ix"]), _ptr(o["iy"]),
              _ptr(o["flags"]), _ptr(o["psi"]), _ptr(o["phi"]), _ptr(o["tau"])))
    return o


def _batch_arrays(patches, orbit_sets, outs):
    n = len(patches)
    ph = (_P * n)(*[p.handle.value for p in patches])
    sets = (DtOrbits * n)(*[o.struct() for o in orbit_sets])
    snr = (_P * n)(*[o[0].data_ptr() if o[0] is not None else None for o in outs])
    flux = (_P * n)(*[o[1].data_ptr() if o[1] is not None else None for o in outs])
    nv = (_P * n)(*[o[2].data_ptr() if o[2] is not None else None for o in outs])
    return ph, sets, snr, flux, nv


def batch_outputs(orbit_sets):
    import torch
    return [(torch.empty(o.n, dtype=torch.float32, device=o.soa.device),
             torch.empty(o.n, dtype=torch.float32, device=o.soa.device),
             torch.empty(o.n, dtype=torch.int32, device=o.soa.device)) for o in orbit_sets]


def stack_batched(ctx: Context, patches, orbit_sets, outs=None, k: int = 0, threshold: float = float("-inf"),
                  cfg=None, prepass: bool = False, eager: bool = False, topk_out=None):
    """One persistent launch over many patches (graph-captured unless eager).
    Returns (outs, (idx[n_patches, k], val[n_patches, k], count[n_patches]) or None)."""
    import torch
    if outs is None:
        outs = batch_outputs(orbit_sets)
    n = len(patches)
    dev = orbit_sets[0].soa.device
    if k > 0 and topk_out is None:
        topk_out = (torch.empty((n, k), dtype=torch.int64, device=dev),
                    torch.empty((n, k), dtype=torch.float32, device=dev),
                    torch.empty(n, dtype=torch.int32, device=dev))
    ph, sets, snr, flux, nv = _batch_arrays(patches, orbit_sets, outs)
    c = None
    if cfg is not None:
        c = DtBatchConfig(int(cfg[0]), int(cfg[1]))
    flags = (DT_BATCH_PREPASS if prepass else 0) | (DT_BATCH_EAGER if eager else 0)
    ti, tv, tc = topk_out if k > 0 else (None, None, None)
    _check(lib().dt_stack_batched(ctx.handle, ph, sets, n, snr, flux, nv, int(k), float(threshold), _ptr(ti),
                                  _ptr(tv), _ptr(tc), C.byref(c) if c is not None else None, flags))
    return outs, (topk_out if k > 0 else None)


def autotune_batched(ctx: Context, patches, orbit_sets, outs=None, cache_path=None):
    """Time candidate launch shapes; returns ((chunk, wg_per_cu), ms or -1 if cached)."""
    if outs is None:
        outs = batch_outputs(orbit_sets)
    ph, sets, snr, flux, nv = _batch_arrays(patches, orbit_sets, outs)
    best = DtBatchConfig()
    ms = C.c_double()
    _check(lib().dt_autotune_batched(ctx.handle, ph, sets, len(patches), snr, flux, nv,
                                     cache_path.encode() if cache_path else None, C.byref(best), C.byref(ms)))
    return (best.chunk, best.wg_per_cu), ms.value


class GatherRecord:
    """The stack's gathers of an orbit set (dt_record_gathers): group starts,
    the slot-major offset list, and the number of recorded gathers."""

    def __init__(self, start, lst, count):
        self.start, self.list, self.count = start, lst, count
        self.n = 0

    @property
    def index_bytes(self):
        return 8 * int(self.list.numel())


def record_valid_gathers(patch: Patch, orbits: OrbitSet):
    """Record the plane offsets of every gather the stack makes for `orbits`."""
    import torch
    n = orbits.n
    start = torch.empty((n + 63) // 64 + 1, dtype=torch.int64, device=patch.device)
    entries, gathers = C.c_int64(), C.c_int64()
    s = orbits.struct()
    _check(lib().dt_record_gathers(patch.handle, C.byref(s), _ptr(start), None, C.byref(entries), C.byref(gathers)))
    lst = torch.empty(max(entries.value, 1), dtype=torch.int64, device=patch.device)
    _check(lib().dt_record_gathers(patch.handle, C.byref(s), _ptr(start), _ptr(lst), C.byref(entries), None))
    rec = GatherRecord(start, lst, gathers.value)
    rec.n = n
    return rec


def replay_valid_gathers(patch: Patch, rec: GatherRecord, snr=None):
    """Replay a recorded gather stream; returns the S/N (the stack's where n_valid > 0, else 0)."""
    import torch
    if snr is None:
        snr = torch.empty(rec.n, dtype=torch.float32, device=patch.device)
    _check(lib().dt_gather_replay(patch.handle, _ptr(rec.start), _ptr(rec.list), rec.n, _ptr(snr)))
    return snr


def image_noise(ctx: Context, images, kappa: float = 3.0, max_iter: int = 10):
    """Iterated-MAD noise of device images: (sigma f64, n_used i64, steps i32) device tensors."""
    import torch
    n = len(images)
    if n == 0:
        e = torch.empty(0, device="cuda")
        return e.double(), e.long(), e.int()
    dt = images[0].dtype
    if dt not in (torch.float32, torch.float16) or any(x.dtype != dt or not x.is_contiguous() for x in images):
        raise TypeError("images must be contiguous float32 or float16 tensors of one dtype")
    dev = images[0].device
    sig = torch.empty(n, dtype=torch.float64, device=dev)
    used = torch.empty(n, dtype=torch.int64, device=dev)
    it = torch.empty(n, dtype=torch.int32, device=dev)
    ptrs = (_P * n)(*[x.data_ptr() if x.numel() else None for x in images])
    npx = (C.c_int64 * n)(*[x.numel() for x in images])
    _check(lib().dt_image_noise(ctx.handle, n, ptrs, npx, DT_F32 if dt == torch.float32 else DT_F16, float(kappa),
                                int(max_iter), _ptr(sig), _ptr(used), _ptr(it)))
    return sig, used, it


def orbit_sampler(field: dict, epoch: float, a_range, e_range, inc_deg_range, seed: int):
    """A dt_orbit_sampler from a grid-field description (center/east/north/obs/half_w/half_h)."""
    import math
    s = DtOrbitSampler()
    s.epoch = float(epoch)
    s.obs_xyz_au[:] = [float(v) for v in field["obs"]]
    s.center[:] = [float(v) for v in field["center"]]
    s.east[:] = [float(v) for v in field["east"]]
    s.north[:] = [float(v) for v in field["north"]]
    s.half_w, s.half_h = float(field["half_w"]), float(field["half_h"])
    s.a_range[:] = [float(v) for v in a_range]
    s.e_range[:] = [float(v) for v in e_range]
    s.inc_range[:] = [math.radians(float(v)) for v in inc_deg_range]
    s.seed = int(seed)
    return s


def generate_orbits(ctx: Context, sampler, first: int, n: int):
    """(n, 6) device tensor of sampled elements (also usable as OrbitSet)."""
    import torch
    soa = torch.empty((6, n), dtype=torch.float64, device="cuda")
    ptrs = [soa[k].data_ptr() if n else None for k in range(6)]
    _check(lib().dt_generate_orbits(ctx.handle, C.byref(sampler), int(first), int(n), *ptrs))
    return soa.t()


def stack_generated(patch: Patch, sampler, first: int, n: int, out=None):
    """dt_stack_generated: (S/N, flux, n_valid) of orbits first .. first + n - 1
    of the sampler; out = caller-provided (float32, float32, int32) tensors."""
    import torch
    if out is None:
        out = (torch.empty(n, dtype=torch.float32, device=patch.device),
               torch.empty(n, dtype=torch.float32, device=patch.device),
               torch.empty(n, dtype=torch.int32, device=patch.device))
    snr, flux, nv = out
    _check(lib().dt_stack_generated(patch.handle, C.byref(sampler), int(first), int(n), _ptr(snr), _ptr(flux),
                                    _ptr(nv)))
    return snr, flux, nv


def clip_candidates(patch: Patch, orbits: OrbitSet, ids, kappa: float = 3.0, max_iter: int = 10):
    """Outlier trimming of candidate orbits: (S/N, flux, kept count) after sigma clipping."""
    import torch
    dev = orbits.soa.device
    ids = torch.as_tensor(ids, dtype=torch.int64).to(dev)
    m = int(ids.numel())
    snr = torch.empty(m, dtype=torch.float32, device=dev)
    flux = torch.empty(m, dtype=torch.float32, device=dev)
    nk = torch.empty(m, dtype=torch.int32, device=dev)
    _check(lib().dt_clip_candidates(patch.handle, C.byref(orbits.struct()), _ptr(ids), m, float(kappa),
                                    int(max_iter), _ptr(snr), _ptr(flux), _ptr(nk)))
    return snr, flux, nk


# ------------------------------------------------------------ learned proposal
def cell_stamps(patch: Patch, reps: OrbitSet, da: float, dm: float, bf16=True, f32=True, feats_f32=None):
    """Coarse stamps (n x 21 x 21 over the cell's (a, M0) box) and features (n x 16) of representative
    orbits: BF16 stamps and features when bf16, FP32 stamps when f32, FP32 features when feats_f32
    (default: f32)."""
    import torch
    dev = reps.soa.device
    n = reps.n
    feats_f32 = f32 if feats_f32 is None else feats_f32
    sb = torch.empty((n, 21, 21), dtype=torch.bfloat16, device=dev) if bf16 else None
    sf = torch.empty((n, 21, 21), dtype=torch.float32, device=dev) if f32 else None
    fb = torch.empty((n, 16), dtype=torch.bfloat16, device=dev) if bf16 else None
    ff = torch.empty((n, 16), dtype=torch.float32, device=dev) if feats_f32 else None
    _check(lib().dt_cell_stamps(patch.handle, C.byref(reps.struct()), float(da), float(dm), _ptr(sb), _ptr(sf),
                                _ptr(fb), _ptr(ff)))
    return dict(stamps_bf16=sb, stamps=sf, feats_bf16=fb, feats=ff)


def stack_cells(patch: Patch, grid: OrbitSet, cells, cell_size: int, out=None):
    """The plain stack on the orbits of the selected cells; outputs at the orbits' indices."""
    import torch
    dev = grid.soa.device
    if out is None:
        out = (torch.full((grid.n,), float("nan"), dtype=torch.float32, device=dev),
               torch.full((grid.n,), float("nan"), dtype=torch.float32, device=dev),
               torch.full((grid.n,), -2, dtype=torch.int32, device=dev))
    cells = torch.as_tensor(cells, dtype=torch.int64).to(dev)
    _check(lib().dt_stack_cells(patch.handle, C.byref(grid.struct()), _ptr(cells), int(cells.numel()),
                                int(cell_size), _ptr(out[0]), _ptr(out[1]), _ptr(out[2])))
    return out


def cell_members_near(ctx: Context, grid: OrbitSet, cells, cell_size: int, uv, da: float, dm: float,
                      radius: float, ids=None, count=None):
    """Orbit ids of the selected cells' members within `radius` (lattice units)
    of each cell's (u, v) in `uv` (device float rows, u and v first: the FP32
    stamp features, columns 11 and 12, are passed as uv[:, 11:]).  Returns
    (ids int64 [capacity], count int64 [1]) device tensors; only the first
    count ids are meaningful."""
    import torch
    dev = grid.soa.device
    cells = torch.as_tensor(cells, dtype=torch.int64).to(dev)
    cap = max(int(cells.numel()) * int(cell_size), 1)
    if ids is None or ids.numel() < cap:
        ids = torch.empty(cap, dtype=torch.int64, device=dev)
    if count is None:
        count = torch.empty(1, dtype=torch.int64, device=dev)
    _check(lib().dt_cell_members_near(ctx.handle, C.byref(grid.struct()), _ptr(cells), int(cells.numel()),
                                      int(cell_size), _ptr(uv), int(uv.stride(0)), float(da), float(dm),
                                      float(radius), _ptr(ids), _ptr(count)))
    return ids, count


def segment_max(ctx: Context, x, seg: int, out=None):
    """Maximum of each run of `seg` consecutive values of a device float tensor (NaN ignored)."""
    import torch
    n_seg = int(x.numel()) // int(seg)
    if out is None:
        out = torch.empty(n_seg, dtype=torch.float32, device=x.device)
    _check(lib().dt_segment_max(ctx.handle, _ptr(x), n_seg, int(seg), _ptr(out)))
    return out


def stack_ids(patch: Patch, orbits: OrbitSet, ids, count, out=None, m_max: int = None):
    """The plain stack on the first count ids of a device id list; outputs at the orbits' indices."""
    import torch
    dev = orbits.soa.device
    if out is None:
        out = (torch.full((orbits.n,), float("nan"), dtype=torch.float32, device=dev),
               torch.full((orbits.n,), float("nan"), dtype=torch.float32, device=dev),
               torch.full((orbits.n,), -2, dtype=torch.int32, device=dev))
    m = int(ids.numel()) if m_max is None else int(m_max)
    _check(lib().dt_stack_ids(patch.handle, C.byref(orbits.struct()), _ptr(ids), _ptr(count), m, _ptr(out[0]),
                              _ptr(out[1]), _ptr(out[2])))
    return out


def gemm_bf16(ctx: Context, A, B, transA=False, transB=False, bias=None, relu=False):
    """C = op(A) op(B) (+ bias) (ReLU) with the library's BF16 MFMA GEMM (FP32 out)."""
    import torch
    A = A.to(torch.bfloat16).contiguous()
    B = B.to(torch.bfloat16).contiguous()
    M, K = (A.shape[1], A.shape[0]) if transA else (A.shape[0], A.shape[1])
    N = B.shape[0] if transB else B.shape[1]
    Cm = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(lib().dt_gemm_bf16(ctx.handle, _ptr(A), A.shape[1], int(transA), _ptr(B), B.shape[1], int(transB),
                              M, N, K, _ptr(bias), int(relu), _ptr(Cm), N))
    return Cm


class Scorer:
    """The learned cell scorer (BF16 MFMA training and inference kernels)."""

    def __init__(self, ctx: Context, max_batch: int = 512, seed: int = 0):
        self.ctx = ctx
        self.max_batch = max_batch
        self._h = _P()
        _check(lib().dt_scorer_create(ctx.handle, int(max_batch), C.c_uint64(seed), C.byref(self._h)))

    @staticmethod
    def num_params() -> int:
        return int(lib().dt_scorer_num_params())

    def params(self):
        import torch
        p = torch.empty(self.num_params(), dtype=torch.float32, device="cuda")
        _check(lib().dt_scorer_get_params(self._h, _ptr(p)))
        return p

    def set_params(self, p):
        import torch
        p = torch.as_tensor(p, dtype=torch.float32).to("cuda").contiguous()
        _check(lib().dt_scorer_set_params(self._h, _ptr(p)))

    def forward(self, stamps_bf16, feats_bf16):
        import torch
        B = stamps_bf16.shape[0]
        z = torch.empty(B, dtype=torch.float32, device=stamps_bf16.device)
        for s in range(0, B, self.max_batch):
            e = min(B, s + self.max_batch)
            _check(lib().dt_scorer_forward(self._h, _ptr(stamps_bf16[s:e].contiguous()),
                                           _ptr(feats_bf16[s:e].contiguous()), e - s, _ptr(z[s:])))
        return z

    def infer(self, stamps_bf16, feats_bf16, out=None):
        """Logits of any number of cells with the fused inference kernel."""
        import torch
        B = stamps_bf16.shape[0]
        z = out if out is not None else torch.empty(B, dtype=torch.float32, device=stamps_bf16.device)
        _check(lib().dt_scorer_infer(self._h, _ptr(stamps_bf16.contiguous()), _ptr(feats_bf16.contiguous()), B,
                                     _ptr(z)))
        return z

    def infer_rows(self, stamps_bf16, feats_bf16, rows, out):
        """Logits of the cells at `rows` (device int64) written to out[rows]; other entries untouched."""
        _check(lib().dt_scorer_infer_rows(self._h, _ptr(stamps_bf16.contiguous()), _ptr(feats_bf16.contiguous()),
                                          _ptr(rows), int(rows.numel()), _ptr(out)))
        return out

    def grad(self, stamps_bf16, feats_bf16, labels):
        import torch
        g = torch.empty(self.num_params(), dtype=torch.float32, device=stamps_bf16.device)
        loss = torch.empty(1, dtype=torch.float32, device=stamps_bf16.device)
        labels = labels.to(torch.float32).contiguous()
        _check(lib().dt_scorer_grad(self._h, _ptr(stamps_bf16.contiguous()), _ptr(feats_bf16.contiguous()),
                                    _ptr(labels), int(stamps_bf16.shape[0]), _ptr(loss), _ptr(g)))
        return loss, g

    def train_step(self, stamps_bf16, feats_bf16, labels, lr: float, loss_out=None):
        import torch
        loss = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float32, device=stamps_bf16.device)
        labels = labels.to(torch.float32).contiguous()
        _check(lib().dt_scorer_train_step(self._h, _ptr(stamps_bf16.contiguous()), _ptr(feats_bf16.contiguous()),
                                          _ptr(labels), int(stamps_bf16.shape[0]), float(lr), _ptr(loss)))
        return loss

    def close(self):
        if self._h:
            _check(lib().dt_scorer_destroy(self._h))
            self._h = _P()

    def __del__(self):
        try:
            if self._h:
                lib().dt_scorer_destroy(self._h)
        except Exception:
            pass
