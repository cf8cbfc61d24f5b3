"""Plain FP64 CPU oracle for non-linear digital tracking (test infrastructure).

Only tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path never does: it runs on the HIP
library alone.  The numerical work lives in ``oracle.c`` (plain C, FP64,
one sample at a time); this module only marshals numpy arrays through
ctypes and builds the shared object with gcc when asked.

Functions and the passages they follow (Golovich et al. 2025):
  kepler, helio_state   -- Sec. 3, elliptical two-body motion about the Sun
  light_time            -- reading: astrometric light-time fixed point
  ecl_to_eq, tan_project-- Sec. 3, WCS (TAN) projection to pixels
  intersect, samples    -- Sec. 3 / Algorithm 1 SearchImages + filtering
  stamp, planes         -- Sec. 3 FindLocalSignal, Gaussian matched filter
  stack                 -- Sec. 3 constant-flux combination of signals
  topk                  -- Algorithm 1 FindSignificantResults
  sigma_clip            -- Sec. 5.2.3 outlier trimming of intersections
  linear_stack          -- Sec. 1 classic (linear) digital tracking
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
X_STRIDE = 16

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.or_kepler.argtypes = [C.c_double, C.c_double, dp]
        L.or_kepler.restype = C.c_int
        L.or_reduce_angle.argtypes = [C.c_double]
        L.or_reduce_angle.restype = C.c_double
        L.or_helio_state.argtypes = [dp, C.c_double, C.c_double, dp, dp]
        L.or_helio_state.restype = C.c_int
        L.or_light_time.argtypes = [dp, C.c_double, C.c_double, dp, dp, dp, dp]
        L.or_light_time.restype = C.c_int
        L.or_ecl_to_eq.argtypes = [dp, dp]
        L.or_eq_to_ecl.argtypes = [dp, dp]
        L.or_tan_project.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double, dp, dp, dp]
        L.or_tan_project.restype = C.c_int
        L.or_intersect.argtypes = [dp, C.c_double, dp, dp, dp, ip, ip, dp, dp, ip]
        L.or_intersect.restype = C.c_int
        L.or_half_to_double.argtypes = [C.c_uint16]
        L.or_half_to_double.restype = C.c_double
        L.or_stamp.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                               C.c_double, dp, dp]
        L.or_planes.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, dp, dp]
        L.or_samples.argtypes = [C.c_int64, dp, C.c_double, C.c_int, dp, C.c_void_p, C.c_void_p,
                                 C.c_int, dp, dp, ip, ip, ip, dp, dp, dp, dp]
        L.or_samples.restype = C.c_int
        L.or_stack.argtypes = [C.c_int64, dp, C.c_double, C.c_int, dp, C.c_void_p, C.c_void_p,
                               C.c_int, dp, dp, ip, C.c_int]
        L.or_stack.restype = C.c_int
        L.or_max_threads.restype = C.c_int
        L.or_linear_stack.argtypes = [C.c_int, dp, C.c_double, C.c_int, dp, C.c_void_p, C.c_void_p,
                                      C.c_int, dp, dp, ip]
        L.or_sigma_clip.argtypes = [C.c_int, dp, dp, C.c_double, C.c_int, dp, dp, ip, C.POINTER(C.c_uint8)]
        L.or_mad_noise.argtypes = [C.c_int64, C.POINTER(C.c_float), C.c_double, C.c_int, dp,
                                   C.POINTER(C.c_int64), ip]
        L.or_topk.argtypes = [C.c_int64, dp, C.c_int64, C.c_double, C.POINTER(C.c_int64)]
        L.or_topk.restype = C.c_int64
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


# ---------------------------------------------------------------- exposures
def pack_exposures(exps) -> np.ndarray:
    """Exposure list (dicts with t, obs, crval, crpix, cd, width, height, fwhm)
    -> the oracle's own (n, 16) float64 record array."""
    out = np.zeros((len(exps), X_STRIDE), dtype=np.float64)
    for k, x in enumerate(exps):
        out[k, 0] = x["t"]
        out[k, 1:4] = x["obs"]
        out[k, 4:6] = x["crval"]
        out[k, 6:8] = x["crpix"]
        out[k, 8:12] = x["cd"]
        out[k, 12] = x["width"]
        out[k, 13] = x["height"]
        out[k, 14] = x["fwhm"]
    return out


def _img_ptrs(images):
    """List of 2-D float32 / float16 arrays -> (keepalive, void** array, dtype code)."""
    if images is None:
        return None, None, 0
    imgs = [np.ascontiguousarray(im) for im in images]
    dt = imgs[0].dtype
    code = 0 if dt == np.float32 else 1
    if dt not in (np.float32, np.float16):
        raise TypeError("images must be float32 or float16")
    arr = (C.c_void_p * len(imgs))(*[im.ctypes.data for im in imgs])
    return imgs, arr, code


# ---------------------------------------------------------------- wrappers
def kepler(M: float, e: float):
    E = C.c_double()
    it = lib().or_kepler(float(M), float(e), C.byref(E))
    return E.value, it


def reduce_angle(M: float) -> float:
    return lib().or_reduce_angle(float(M))


def helio_state(el, t0, t):
    el, pe = _d(el)
    r = np.zeros(3)
    v = np.zeros(3)
    it = lib().or_helio_state(pe, float(t0), float(t), r.ctypes.data_as(C.POINTER(C.c_double)),
                              v.ctypes.data_as(C.POINTER(C.c_double)))
    return r, v, it


def light_time(el, t0, t_e, robs):
    el, pe = _d(el)
    robs, po = _d(robs)
    rho = np.zeros(3)
    helio = np.zeros(3)
    tau = C.c_double()
    st = lib().or_light_time(pe, float(t0), float(t_e), po, rho.ctypes.data_as(C.POINTER(C.c_double)),
                             C.byref(tau), helio.ctypes.data_as(C.POINTER(C.c_double)))
    return rho, tau.value, helio, st


def ecl_to_eq(v):
    v, pv = _d(v)
    out = np.zeros(3)
    lib().or_ecl_to_eq(pv, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def eq_to_ecl(v):
    v, pv = _d(v)
    out = np.zeros(3)
    lib().or_eq_to_ecl(pv, out.ctypes.data_as(C.POINTER(C.c_double)))
    return out


def tan_project(u_eq, crval, crpix, cd):
    u, pu = _d(u_eq)
    cd, pc = _d(cd)
    px, py = C.c_double(), C.c_double()
    ok = lib().or_tan_project(pu, float(crval[0]), float(crval[1]), float(crpix[0]), float(crpix[1]),
                              pc, C.byref(px), C.byref(py))
    return px.value, py.value, bool(ok)


def half_to_double(h: int) -> float:
    return lib().or_half_to_double(int(h))


def stamp(D, V, ix, iy, fwhm):
    D = np.ascontiguousarray(D)
    V = np.ascontiguousarray(V)
    code = 0 if D.dtype == np.float32 else 1
    psi, phi = C.c_double(), C.c_double()
    lib().or_stamp(D.ctypes.data, V.ctypes.data, code, D.shape[1], D.shape[0], int(ix), int(iy),
                   float(fwhm), C.byref(psi), C.byref(phi))
    return psi.value, phi.value


def planes(D, V, fwhm):
    D = np.ascontiguousarray(D)
    V = np.ascontiguousarray(V)
    code = 0 if D.dtype == np.float32 else 1
    H, W = D.shape
    psi = np.zeros((H, W))
    phi = np.zeros((H, W))
    lib().or_planes(D.ctypes.data, V.ctypes.data, code, W, H, float(fwhm),
                    psi.ctypes.data_as(C.POINTER(C.c_double)), phi.ctypes.data_as(C.POINTER(C.c_double)))
    return psi, phi


def samples(elements, t0, exps, D=None, V=None):
    """Per-(orbit, exposure) table for the given orbits (m x 6 elements)."""
    el, pe = _d(np.atleast_2d(elements))
    m = el.shape[0]
    xp, px_ = _d(exps if isinstance(exps, np.ndarray) else pack_exposures(exps))
    n = xp.shape[0]
    keepD, pD, code = _img_ptrs(D)
    keepV, pV, _ = _img_ptrs(V)
    out = {k: np.zeros((m, n)) for k in ("px", "py", "psi", "phi", "tau")}
    out["ix"] = np.zeros((m, n), np.int32)
    out["iy"] = np.zeros((m, n), np.int32)
    out["flags"] = np.zeros((m, n), np.int32)
    out["helio"] = np.zeros((m, n, 3))
    f = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    bad = lib().or_samples(m, pe, float(t0), n, px_, pD, pV, code, f(out["px"]), f(out["py"]),
                           _i(out["ix"]), _i(out["iy"]), _i(out["flags"]), f(out["psi"]),
                           f(out["phi"]), f(out["tau"]), f(out["helio"]))
    out["bad"] = bad
    out["valid"] = (out["flags"] & 4) != 0 if D is not None else (out["flags"] & 3) == 3
    return out


def stack(elements, t0, exps, D, V, nthreads: int = 0):
    el, pe = _d(np.atleast_2d(elements))
    m = el.shape[0]
    xp, px_ = _d(exps if isinstance(exps, np.ndarray) else pack_exposures(exps))
    keepD, pD, code = _img_ptrs(D)
    keepV, pV, _ = _img_ptrs(V)
    snr = np.zeros(m)
    flux = np.zeros(m)
    nv = np.zeros(m, np.int32)
    f = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    bad = lib().or_stack(m, pe, float(t0), xp.shape[0], px_, pD, pV, code, f(snr), f(flux), _i(nv),
                         int(nthreads))
    if bad:
        raise RuntimeError(f"oracle: {bad} samples failed to converge")
    return snr, flux, nv


def max_threads() -> int:
    return lib().or_max_threads()


def linear_stack(tracks, tref, exps, D, V):
    tr, pt = _d(np.atleast_2d(tracks))
    xp, px_ = _d(exps if isinstance(exps, np.ndarray) else pack_exposures(exps))
    keepD, pD, code = _img_ptrs(D)
    keepV, pV, _ = _img_ptrs(V)
    k = tr.shape[0]
    snr = np.zeros(k)
    flux = np.zeros(k)
    nv = np.zeros(k, np.int32)
    f = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    lib().or_linear_stack(k, pt, float(tref), xp.shape[0], px_, pD, pV, code, f(snr), f(flux), _i(nv))
    return snr, flux, nv


def topk(snr, k, thr=-np.inf):
    s, ps = _d(snr)
    out = np.zeros(max(int(k), 1), np.int64)
    cnt = lib().or_topk(s.shape[0], ps, int(k), float(thr), out.ctypes.data_as(C.POINTER(C.c_int64)))
    return out[:cnt]


def sigma_clip(psi, phi, kappa=3.0, max_iter=10):
    """Outlier trimming of one orbit's intersections: (S/N, flux, n_kept, kept mask)."""
    ps, pp = _d(psi)
    ph, pph = _d(phi)
    n = ps.shape[0]
    kept = np.zeros(max(n, 1), np.uint8)
    snr, flux = C.c_double(), C.c_double()
    nk = C.c_int32()
    lib().or_sigma_clip(n, pp, pph, float(kappa), int(max_iter), C.byref(snr), C.byref(flux), C.byref(nk),
                        kept.ctypes.data_as(C.POINTER(C.c_uint8)))
    return snr.value, flux.value, nk.value, kept[:n].astype(bool)


def mad_noise(image, kappa=3.0, max_iter=10):
    """Iterated-MAD noise of one image (float32 values): (sigma, n_used, iterations)."""
    x = np.ascontiguousarray(np.asarray(image, dtype=np.float32).ravel())
    sig, nu, it = C.c_double(), C.c_int64(), C.c_int32()
    lib().or_mad_noise(x.size, x.ctypes.data_as(C.POINTER(C.c_float)), float(kappa), int(max_iter), C.byref(sig),
                       C.byref(nu), C.byref(it))
    return sig.value, nu.value, it.value
