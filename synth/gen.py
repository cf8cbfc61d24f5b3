"""Seeded input generators (no tracking arithmetic; see the package docstring).

Recipe (the paper's ZTF data are not available; these stand in for them):
  * epochs uniform over the span, sorted; the observer moves on a circular
    1 AU orbit in the ecliptic (stand-in for the Earth ephemeris);
  * every image is Gaussian noise with a per-exposure sigma, its variance
    plane is sigma^2, and a fraction of pixels is masked as NaN in both;
  * injected sources are point-sampled Gaussians of unit integral rendered at
    the pixel positions stored in the workload file;
  * candidate orbits are drawn uniformly in (a, e, i) and placed, by an
    inverse construction (line of sight -> position -> elements), so that
    their geometric position at the grid epoch lies on a random line of
    sight through the grid field.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "K_OBS", "GOLDEN_DIR", "make_rng", "sorted_epochs", "observer_circular", "unit",
    "tangent_basis", "orbits_through", "Workload", "load_geometry", "exposures_of",
    "candidate_orbits", "perturbed_cloud", "noise_images", "render_sources", "build_workload",
    "radec_to_vec", "vec_to_radec", "hw_pixscale_deg", "cell_grid", "render_sources_fast", "grid_sampler",
    "artifacts",
]

# Mean motion (rad/day) of the synthetic observer on a circular 1 AU orbit.
K_OBS = 0.01720209895
GOLDEN_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")


def make_rng(seed: int, *stream: int) -> np.random.Generator:
    """Independent PCG64 stream for (seed, stream...)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), *map(int, stream)])))


def sorted_epochs(rng, n: int, span: float, start: float = 0.0) -> np.ndarray:
    return np.sort(rng.uniform(start, start + span, n))


def observer_circular(t, t_mid: float, lam_mid: float) -> np.ndarray:
    """Heliocentric ecliptic observer position (AU) on a circular 1 AU orbit."""
    t = np.asarray(t, dtype=np.float64)
    lam = lam_mid + K_OBS * (t - t_mid)
    return np.stack([np.cos(lam), np.sin(lam), np.zeros_like(lam)], axis=-1)


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def radec_to_vec(ra_deg, dec_deg):
    a = np.radians(ra_deg)
    d = np.radians(dec_deg)
    return np.stack([np.cos(d) * np.cos(a), np.cos(d) * np.sin(a), np.sin(d)], axis=-1)


def vec_to_radec(v):
    v = unit(v)
    ra = np.degrees(np.arctan2(v[..., 1], v[..., 0])) % 360.0
    dec = np.degrees(np.arcsin(np.clip(v[..., 2], -1.0, 1.0)))
    return ra, dec


def tangent_basis(center):
    """Orthonormal (east-like, north-like) axes perpendicular to ``center``."""
    c = unit(center)
    z = np.array([0.0, 0.0, 1.0])
    e1 = unit(np.cross(z, c))
    e2 = np.cross(c, e1)
    return e1, e2


def hw_pixscale_deg(arcsec_per_px: float) -> float:
    return arcsec_per_px / 3600.0


def orbits_through(rng, dirs, r_obs, a, e, inc, t0=None):
    """Element sets (a, e, i, node, peri, M0) whose geometric heliocentric
    position at the element epoch lies on the line of sight ``dirs`` (unit,
    ecliptic) from ``r_obs``.  The true anomaly and the nodal branch are
    drawn at random; i is raised to |latitude| where the line of sight needs
    it.  Returns (elements (n, 6), ok mask) -- ok is False where no
    intersection with the orbit's distance exists."""
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    n = dirs.shape[0]
    a = np.broadcast_to(np.asarray(a, np.float64), (n,)).copy()
    e = np.broadcast_to(np.asarray(e, np.float64), (n,)).copy()
    inc = np.broadcast_to(np.asarray(inc, np.float64), (n,)).copy()
    nu = rng.uniform(-math.pi, math.pi, n)
    branch = rng.integers(0, 2, n)
    r = a * (1.0 - e * e) / (1.0 + e * np.cos(nu))
    O = np.asarray(r_obs, dtype=np.float64)
    ou = dirs @ O
    disc = ou * ou - O @ O + r * r
    ok = disc > 0
    s = -ou + np.sqrt(np.where(ok, disc, 0.0))
    ok &= s > 0
    X = O[None, :] + s[:, None] * dirs
    Xh = unit(X)
    beta = np.arcsin(np.clip(Xh[:, 2], -1.0, 1.0))
    lam = np.arctan2(Xh[:, 1], Xh[:, 0])
    inc = np.maximum(inc, np.abs(beta) * (1.0 + 1e-9) + 1e-12)
    su = np.clip(np.sin(beta) / np.sin(inc), -1.0, 1.0)
    u = np.arcsin(su)
    u = np.where(branch == 1, math.pi - u, u)
    node = lam - np.arctan2(np.cos(inc) * np.sin(u), np.cos(u))
    peri = u - nu
    E = 2.0 * np.arctan2(np.sqrt(1.0 - e) * np.sin(nu / 2.0), np.sqrt(1.0 + e) * np.cos(nu / 2.0))
    M0 = E - e * np.sin(E)
    wrap = lambda x: np.mod(x, 2.0 * math.pi)
    el = np.stack([a, e, inc, wrap(node), wrap(peri), np.mod(M0 + math.pi, 2 * math.pi) - math.pi], axis=1)
    return el, ok


# ------------------------------------------------------------------ workloads
@dataclass
class Workload:
    name: str
    exps: list
    t0: float
    elements: np.ndarray           # (n, 6) float64: a, e, i, node, peri, M0
    D: list = field(default_factory=list)
    V: list = field(default_factory=list)
    injections: list = field(default_factory=list)
    inj_index: np.ndarray = None   # orbit index of every injected (true) orbit
    dtype: str = "f32"
    geom: dict = None


def load_geometry(name_or_path: str) -> dict:
    path = name_or_path
    if not os.path.exists(path):
        path = os.path.join(GOLDEN_DIR, f"geom_{name_or_path}.json")
    with open(path) as f:
        return json.load(f)


def exposures_of(geom: dict) -> list:
    return [dict(x) for x in geom["exposures"]]


def candidate_orbits(gf: dict, n: int, seed: int, a_rng, e_rng, inc_deg_rng, stream: int = 0):
    """n candidate orbits through random lines of sight in the grid field."""
    rng = make_rng(seed, 101, stream)
    out = np.empty((n, 6))
    c = np.asarray(gf["center"])
    ex, ny = np.asarray(gf["east"]), np.asarray(gf["north"])
    filled = 0
    while filled < n:
        m = int((n - filled) * 1.15) + 16
        xi = rng.uniform(-gf["half_w"], gf["half_w"], m)
        eta = rng.uniform(-gf["half_h"], gf["half_h"], m)
        dirs = unit(c[None, :] + xi[:, None] * ex[None, :] + eta[:, None] * ny[None, :])
        a = rng.uniform(*a_rng, m)
        e = rng.uniform(*e_rng, m)
        inc = np.radians(rng.uniform(*inc_deg_rng, m))
        el, ok = orbits_through(rng, dirs, gf["obs"], a, e, inc)
        el = el[ok]
        take = min(el.shape[0], n - filled)
        out[filled:filled + take] = el[:take]
        filled += take
    return out


def perturbed_cloud(el, n: int, da_max: float, seed: int, stream: int = 0):
    """n copies of ``el`` with the semi-major axis perturbed uniformly by
    +-da_max (AU), the other elements unchanged."""
    rng = make_rng(seed, 202, stream)
    out = np.repeat(np.asarray(el, np.float64)[None, :], n, axis=0)
    out[:, 0] += rng.uniform(-da_max, da_max, n)
    return out


def noise_images(exps, seed: int, nan_frac: float = 0.0, dtype: str = "f32", device=None):
    """Per exposure: D ~ N(0, sigma^2) and V = sigma^2, NaN-masked jointly.
    On a torch CUDA ``device`` the draws come from torch's device generator
    (same recipe, different stream); otherwise from numpy PCG64."""
    D, V = [], []
    if device is not None:
        import torch
        g = torch.Generator(device=device)
        tdt = torch.float32 if dtype == "f32" else torch.float16
        for k, x in enumerate(exps):
            g.manual_seed(int(seed) * 1000003 + k)
            H, W = int(x["height"]), int(x["width"])
            s = float(x.get("sigma", 1.0))
            d = torch.randn((H, W), generator=g, device=device, dtype=torch.float32) * s
            v = torch.full((H, W), s * s, device=device, dtype=torch.float32)
            if nan_frac > 0:
                m = torch.rand((H, W), generator=g, device=device) < nan_frac
                d[m] = float("nan")
                v[m] = float("nan")
            D.append(d.to(tdt))
            V.append(v.to(tdt))
        return D, V
    npdt = np.float32 if dtype == "f32" else np.float16
    for k, x in enumerate(exps):
        rng = make_rng(seed, 303, k)
        H, W = int(x["height"]), int(x["width"])
        s = float(x.get("sigma", 1.0))
        d = (rng.standard_normal((H, W)) * s).astype(np.float32)
        v = np.full((H, W), s * s, dtype=np.float32)
        if nan_frac > 0:
            m = rng.random((H, W)) < nan_frac
            d[m] = np.nan
            v[m] = np.nan
        D.append(d.astype(npdt))
        V.append(v.astype(npdt))
    return D, V


def render_sources(D, exps, injections, device=None):
    """Add every injection's flux F, as a unit-integral point-sampled Gaussian
    (sigma = FWHM / 2.3548...), at its stored pixel position in each exposure."""
    for inj in injections:
        F = float(inj["flux"])
        for e, px, py in inj["hits"]:
            e = int(e)
            x = exps[e]
            sig = float(x["fwhm"]) / (2.0 * math.sqrt(2.0 * math.log(2.0)))
            R = int(math.ceil(5.0 * sig))
            H, W = int(x["height"]), int(x["width"])
            cx, cy = int(math.floor(px + 0.5)), int(math.floor(py + 0.5))
            x0, x1 = max(cx - R, 0), min(cx + R + 1, W)
            y0, y1 = max(cy - R, 0), min(cy + R + 1, H)
            if x0 >= x1 or y0 >= y1:
                continue
            xs = np.arange(x0, x1, dtype=np.float64)
            ys = np.arange(y0, y1, dtype=np.float64)
            g = np.exp(-((xs[None, :] - px) ** 2 + (ys[:, None] - py) ** 2) / (2 * sig * sig))
            g *= F / (2.0 * math.pi * sig * sig)
            if device is not None:
                import torch
                t = D[e]
                t[y0:y1, x0:x1] += torch.from_numpy(g).to(device=t.device, dtype=torch.float32).to(t.dtype)
            else:
                sub = D[e][y0:y1, x0:x1].astype(np.float64) + g
                D[e][y0:y1, x0:x1] = sub.astype(D[e].dtype)
    return D


def build_workload(geom: dict, n_orbits: int = None, seed: int = None, device=None,
                   images: bool = True, cloud: int = None) -> Workload:
    """Assemble a workload from a stored geometry: exposures, candidate orbits
    (true injected orbits at recorded indices, optional perturbed clouds)
    and images."""
    seed = geom["seed"] if seed is None else seed
    exps = exposures_of(geom)
    g = geom["grid"]
    n = g["n"] if n_orbits is None else int(n_orbits)
    injs = geom.get("injections", [])
    if g.get("generated"):
        # the grid is a counter-based sampler (grid_sampler); injections sit
        # on grid orbits at their stored indices
        W = Workload(name=geom["name"], exps=exps, t0=float(geom["t0"]), elements=None, injections=injs,
                     inj_index=np.array([int(i["index"]) for i in injs], dtype=np.int64),
                     dtype=geom.get("dtype", "f32"), geom=geom)
        if images:
            D, V = noise_images(exps, seed, geom.get("nan_frac", 0.0), W.dtype, device)
            hits = [(h[0], h[1], h[2], i["flux"]) for i in injs for h in i["hits"]]
            render_sources_fast(D, exps, hits, device)
            W.D, W.V = D, V
        return W
    cloud = g.get("cloud", 0) if cloud is None else cloud
    extra = len(injs) * (1 + cloud)
    n_rand = max(n - extra, 0)
    el = candidate_orbits(geom["grid_field"], n_rand, seed, g["a"], g["e"], g["inc_deg"])
    parts = [el]
    inj_idx = []
    pos = n_rand
    for k, inj in enumerate(injs):
        parts.append(np.asarray(inj["el"], np.float64)[None, :])
        inj_idx.append(pos)
        pos += 1
        if cloud:
            parts.append(perturbed_cloud(inj["el"], cloud, g.get("cloud_da", 1.5e-4), seed, k))
            pos += cloud
    el = np.concatenate(parts, axis=0)
    # interleave deterministically so injections are not all at the tail
    perm = make_rng(seed, 404).permutation(el.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    el = el[perm]
    inj_idx = inv[np.asarray(inj_idx, dtype=np.int64)] if inj_idx else np.zeros(0, np.int64)
    W = Workload(name=geom["name"], exps=exps, t0=float(geom["t0"]), elements=el,
                 injections=injs, inj_index=inj_idx, dtype=geom.get("dtype", "f32"), geom=geom)
    if images:
        D, V = noise_images(exps, seed, geom.get("nan_frac", 0.0), W.dtype, device)
        render_sources(D, exps, injs, device)
        W.D, W.V = D, V
    return W


def grid_sampler(geom: dict) -> dict:
    """Parameters of a generated grid: the field (center/east/north/obs/half
    widths), the epoch, the (a, e, inclination in degrees) ranges and the
    sampler seed.  Orbit k of the grid is a pure function of these and k."""
    g = geom["grid"]
    return dict(field=geom["grid_field"], epoch=float(geom["grid_field"]["t"]), a=tuple(g["a"]), e=tuple(g["e"]),
                inc_deg=tuple(g["inc_deg"]), seed=int(g["sampler_seed"]), n=int(g["n"]))


def cell_grid(gf: dict, n_cells: int, cell_size: int, seed: int, a_rng, e_rng, inc_deg_rng,
              da: float, dm: float):
    """Cell-structured orbit grid, cell-major: cell c owns orbits
    [c * cell_size, (c + 1) * cell_size).  Member 0 is the cell's
    representative (drawn like the random candidates); the other members
    perturb its semi-major axis by U(-da, da) AU and its mean anomaly by
    U(-dm, dm) rad, so their tracks stay near the representative's."""
    reps = candidate_orbits(gf, n_cells, seed, a_rng, e_rng, inc_deg_rng, stream=77)
    rng = make_rng(seed, 505)
    el = np.repeat(reps, cell_size, axis=0)
    pert = rng.uniform(-1.0, 1.0, (n_cells * cell_size, 2))
    pert[::cell_size] = 0.0
    el[:, 0] += da * pert[:, 0]
    el[:, 5] += dm * pert[:, 1]
    return el


def artifacts(exps, per_image: int, snr_rng, seed: int):
    """Single-exposure point artifacts (transients that appear in one image
    only): per_image positions uniform over every image, each with a
    per-image S/N drawn from U(snr_rng).  Returns an (n, 4) array of
    (exposure, px, py, s); the caller turns s into a flux."""
    rng = make_rng(seed, 606)
    out = []
    for e, x in enumerate(exps):
        px = rng.uniform(-0.5, x["width"] - 0.5, per_image)
        py = rng.uniform(-0.5, x["height"] - 0.5, per_image)
        s = rng.uniform(*snr_rng, per_image)
        out.append(np.stack([np.full(per_image, float(e)), px, py, s], axis=1))
    return np.concatenate(out, axis=0) if out else np.zeros((0, 4))


def render_sources_fast(D, exps, hits, device=None):
    """Vectorised render of many sources: hits is an (n, 4) array of
    (exposure, px, py, flux); unit-integral point-sampled Gaussians as in
    render_sources, added per exposure with one scatter-add."""
    hits = np.asarray(hits, dtype=np.float64).reshape(-1, 4)
    if hits.size == 0:
        return D
    by_e = {}
    for e in np.unique(hits[:, 0].astype(int)):
        by_e[e] = hits[hits[:, 0].astype(int) == e]
    for e, h in by_e.items():
        x = exps[e]
        sig = float(x["fwhm"]) / (2.0 * math.sqrt(2.0 * math.log(2.0)))
        R = int(math.ceil(5.0 * sig))
        H, W = int(x["height"]), int(x["width"])
        off = np.arange(-R, R + 1)
        cx = np.floor(h[:, 1] + 0.5).astype(np.int64)
        cy = np.floor(h[:, 2] + 0.5).astype(np.int64)
        X = cx[:, None, None] + off[None, None, :]
        Y = cy[:, None, None] + off[None, :, None]
        g = np.exp(-((X - h[:, 1, None, None]) ** 2 + (Y - h[:, 2, None, None]) ** 2) / (2 * sig * sig))
        g *= (h[:, 3] / (2.0 * math.pi * sig * sig))[:, None, None]
        X, Y = np.broadcast_to(X, g.shape), np.broadcast_to(Y, g.shape)
        ok = (X >= 0) & (X < W) & (Y >= 0) & (Y < H)
        idx = (Y[ok] * W + X[ok]).ravel()
        val = g[ok].ravel()
        if device is not None:
            import torch
            t = D[e].view(-1)
            t.index_put_((torch.from_numpy(idx).to(t.device),),
                         torch.from_numpy(val).to(device=t.device, dtype=torch.float32).to(t.dtype), accumulate=True)
        else:
            flat = D[e].reshape(-1)
            acc = flat.astype(np.float64)
            np.add.at(acc, idx, val)
            flat[:] = acc.astype(flat.dtype)
    return D
