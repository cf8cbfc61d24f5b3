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


def oracle_sampler(gs):
    """synth.grid_sampler(...) description -> the dict oracle.generate takes."""
    import math
    f = gs["field"]
    return dict(center=f["center"], east=f["east"], north=f["north"], obs=f["obs"], half_w=f["half_w"],
                half_h=f["half_h"], a=tuple(gs["a"]), e=tuple(gs["e"]),
                inc=tuple(math.radians(v) for v in gs["inc_deg"]), seed=int(gs["seed"]), epoch=gs["epoch"])


def gpu_sampler(gs):
    """synth.grid_sampler(...) description -> the library's dt_orbit_sampler."""
    import paper_2503_08854_amd as dt
    return dt.orbit_sampler(gs["field"], gs["epoch"], gs["a"], gs["e"], gs["inc_deg"], gs["seed"])


def band_orbits(elements, t0, exps):
    """Per orbit: does any in-front sample lie within BAND of a rounding
    boundary (where the GPU and the oracle may pick different pixels)?"""
    import oracle
    o = oracle.samples(elements, t0, exps)
    W = np.array([x["width"] for x in exps])[None, :].repeat(o["px"].shape[0], 0)
    H = np.array([x["height"] for x in exps])[None, :].repeat(o["px"].shape[0], 0)
    return (band_mask(o["px"], o["py"], W, H) & ((o["flags"] & 1) != 0)).any(axis=1)


def decode_gathers(rec):
    """dt_record_gathers' slot-major group list -> (n, width) int64 array of
    each orbit's recorded plane offsets in order, -1 padded."""
    start = rec.start.cpu().numpy()
    lst = rec.list.cpu().numpy()
    n = rec.n
    groups = (n + 63) // 64
    widths = np.diff(start) // 64
    out = np.full((groups * 64, max(int(widths.max(initial=0)), 1)), -1, np.int64)
    for g in range(groups):
        w = int(widths[g])
        if w:
            out[g * 64:(g + 1) * 64, :w] = lst[start[g]:start[g + 1]].reshape(w, 64).T
    return out[:n]


def plane_offsets(dbg, exps):
    """Global plane offsets (float2 units) of a debug table's samples, in the
    library's plane layout (exposures in epoch order, row-major planes), and
    the epoch order itself."""
    order = np.argsort([x["t"] for x in exps], kind="stable")
    sizes = np.array([x["width"] * x["height"] for x in exps])[order]
    base = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    W = np.array([x["width"] for x in exps])[order]
    off = base[None, :] + dbg["iy"][:, order].astype(np.int64) * W[None, :] + dbg["ix"][:, order]
    return off, order


def compare_stack_walk(g, o, exps):
    """The stack walk's debug table g (solved samples only) vs the oracle's
    table o: every sample that lands (oracle inside) was solved; solved
    samples match the oracle's coordinates, light time and flags.  Returns
    (n_band, n_solved, n_checked)."""
    W = np.array([x["width"] for x in exps])[None, :].repeat(o["px"].shape[0], 0)
    H = np.array([x["height"] for x in exps])[None, :].repeat(o["px"].shape[0], 0)
    front = (o["flags"] & 1) != 0
    band = front & band_mask(o["px"], o["py"], W, H)
    solved = (g["flags"] & 8) != 0
    inside = (o["flags"] & 2) != 0
    assert np.all(solved[inside & ~band]), "a sample that lands was not solved by the stack walk"
    # pruned samples keep the initial row
    assert np.all(g["flags"][~solved] == 0) and np.all(np.isnan(g["px"][~solved]))
    s = solved & front
    assert np.array_equal((g["flags"][solved] & 1) != 0, front[solved]), "front flags differ"
    assert np.max(np.abs(g["px"][s] - o["px"][s]), initial=0) < 1e-6, "pixel x differs by >= 1e-6 px"
    assert np.max(np.abs(g["py"][s] - o["py"][s]), initial=0) < 1e-6, "pixel y differs by >= 1e-6 px"
    assert np.max(np.abs(g["tau"][solved] - o["tau"][solved]), initial=0) < 1e-12, "light time differs"
    ok = s & ~band
    assert np.array_equal(g["ix"][ok], o["ix"][ok]) and np.array_equal(g["iy"][ok], o["iy"][ok])
    assert np.array_equal(g["flags"][ok] & 7, o["flags"][ok] & 7)
    return int(band.sum()), int(solved.sum()), int(ok.sum())
