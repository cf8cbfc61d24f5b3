"""Shared test helpers: run a workload through the GPU library and the oracle."""
from __future__ import annotations

import numpy as np

BAND = 1e-6       # pixels: boundary band excluded from the bit-exact index assertion
SNR_TOL = 1e-5    # |dS/N| <= SNR_TOL * max(1, |S/N_oracle|) for FP32 images


def band_mask(px, py, W, H):
    """Samples whose coordinate is within BAND of a rounding boundary
    (x + 0.5 integer) or of the image edge, where two correct FP64
    evaluations may round differently."""
    def near(p):
        f = p + 0.5
        return np.abs(f - np.round(f)) < BAND
    return near(px) | near(py)


def to_torch_images(D, V, device="cuda"):
    import torch
    return ([torch.from_numpy(np.ascontiguousarray(d)).to(device) for d in D],
            [torch.from_numpy(np.ascontiguousarray(v)).to(device) for v in V])


def gpu_run(w, device="cuda", ids=None, k=64, thr=float("-inf")):
    """Stack a synth Workload on the GPU; optionally the debug table for ids."""
    import torch
    import paper_2503_08854_amd as dt
    ctx = dt.Context(0)
    if isinstance(w.D[0], np.ndarray):
        Dt, Vt = to_torch_images(w.D, w.V, device)
    else:
        Dt, Vt = w.D, w.V
    patch = dt.Patch(ctx, w.exps, Dt, Vt)
    orb = dt.OrbitSet(w.elements, w.t0, device)
    snr, flux, nv = dt.stack(patch, orb)
    out = dict(snr=snr, flux=flux, nv=nv)
    if ids is not None:
        out["dbg"] = dt.debug_samples(patch, orb, ids)
    idx, val, cnt = dt.topk(ctx, snr, k, thr)
    torch.cuda.synchronize()
    out.update(topk_idx=idx.cpu().numpy(), topk_val=val.cpu().numpy(), topk_cnt=int(cnt.cpu()[0]))
    out = {k2: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k2, v in out.items()}
    if "dbg" in out:
        out["dbg"] = {k2: v.cpu().numpy() for k2, v in out["dbg"].items()}
    out["_keep"] = (ctx, patch, orb, Dt, Vt)
    return out


def compare_samples(g, o, exps):
    """GPU debug table g vs oracle table o (same orbits, caller exposure order).
    Returns (n_band, n_checked); asserts index parity outside the band."""
    W = np.array([x["width"] for x in exps])[None, :]
    H = np.array([x["height"] for x in exps])[None, :]
    front = (o["flags"] & 1) != 0
    gfront = (g["flags"] & 1) != 0
    band = np.zeros_like(front)
    band[front] = band_mask(o["px"][front], o["py"][front], W.repeat(front.shape[0], 0)[front],
                            H.repeat(front.shape[0], 0)[front])
    assert np.array_equal(front, gfront), "front-of-tangent-plane flags differ"
    f = front
    assert np.max(np.abs(g["px"][f] - o["px"][f]), initial=0) < 1e-6, "pixel x differs by >= 1e-6 px"
    assert np.max(np.abs(g["py"][f] - o["py"][f]), initial=0) < 1e-6, "pixel y differs by >= 1e-6 px"
    ok = f & ~band
    assert np.array_equal(g["ix"][ok], o["ix"][ok]) and np.array_equal(g["iy"][ok], o["iy"][ok])
    assert np.array_equal(g["flags"][ok] & 7, o["flags"][ok] & 7)
    return int(band.sum()), int(ok.sum())


def snr_close(gpu, ora, tol=SNR_TOL):
    return np.abs(gpu - ora) <= tol * np.maximum(1.0, np.abs(ora))
