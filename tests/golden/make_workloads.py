"""Write the stored workload geometries ``geom_<name>.json``.

Run from the repository root:  python tests/golden/make_workloads.py [names...]

Everything here that needs the tracking method (where a reference orbit
appears at each epoch, where an injected source lands in each image, the
matched filter's sum of squared weights) is computed by ``oracle/`` only;
random draws come from ``synth``.  No value is taken from the GPU library.

Geometry recipe (a co-moving, "focused" survey, Sec. 4.2): every exposure's
tangent point follows a reference orbit's apparent direction at its epoch,
plus a seeded jitter of up to 10% of the field width and, for mosaics, one of
several fixed field offsets.  The grid field is the tangent plane of the
middle exposure; candidate orbits are drawn through it by ``synth``.
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import generate as ogen  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def apparent_eq(el, t0, t, robs):
    rho, tau, helio, st = oracle.light_time(el, t0, t, robs)
    u = rho / np.linalg.norm(rho)
    return oracle.ecl_to_eq(u)


def sum_p2(fwhm):
    """Sum of squared filter weights: the oracle's phi on a unit-variance image."""
    R = 16
    z = np.zeros((2 * R + 1, 2 * R + 1), np.float32)
    one = np.ones_like(z)
    return oracle.stamp(z, one, R, R, fwhm)[1]


def make_epochs(rng, n, span, t_start=0.0):
    """Sorted epochs; the orbit epoch t0 is the middle exposure's epoch."""
    t = synth.sorted_epochs(rng, n, span, t_start)
    return t, float(t[n // 2])


def make_exposures(rng, t, W, H, arcsec, el_ref, t0, lam_mid, offsets, sigma_rng, fwhm,
                   jitter=0.1):
    n = len(t)
    obs = synth.observer_circular(t, t0, lam_mid)
    scale = arcsec / 3600.0
    fw = math.radians(W * scale)
    fh = math.radians(H * scale)
    exps = []
    for k in range(n):
        u = apparent_eq(el_ref, t0, t[k], obs[k])
        e1, e2 = synth.tangent_basis(u)
        ox, oy = offsets[k % len(offsets)]
        jx, jy = rng.uniform(-jitter, jitter, 2)
        d = synth.unit(u + (ox + jx) * fw * e1 + (oy + jy) * fh * e2)
        ra, dec = synth.vec_to_radec(d)
        s = float(rng.uniform(*sigma_rng)) if sigma_rng[0] != sigma_rng[1] else float(sigma_rng[0])
        exps.append(dict(t=float(t[k]), obs=[float(v) for v in obs[k]], crval=[float(ra), float(dec)],
                         crpix=[W / 2.0 + 0.5, H / 2.0 + 0.5], cd=[-scale, 0.0, 0.0, scale],
                         width=int(W), height=int(H), fwhm=float(fwhm), sigma=s, field=k % len(offsets)))
    return exps


def grid_field(exps, t0, lam_mid, W, H, arcsec):
    mid = int(np.argmin([abs(x["t"] - t0) for x in exps]))
    x = exps[mid]
    c = oracle.eq_to_ecl(synth.radec_to_vec(x["crval"][0], x["crval"][1]))
    e1, e2 = synth.tangent_basis(c)
    hw = math.radians(0.5 * W * arcsec / 3600.0)
    hh = math.radians(0.5 * H * arcsec / 3600.0)
    obs = synth.observer_circular([t0], t0, lam_mid)[0]
    return dict(t=t0, obs=[float(v) for v in obs], center=[float(v) for v in c],
                east=[float(v) for v in e1], north=[float(v) for v in e2], half_w=hw, half_h=hh)


def hits_of(el, t0, exps):
    s = oracle.samples(np.asarray(el)[None, :], t0, exps)
    ok = (s["flags"][0] & 3) == 3
    return [[int(e), float(s["px"][0, e]), float(s["py"][0, e])] for e in np.nonzero(ok)[0]]


def reference_orbit(seed, t0, lam_mid, a, e, inc_deg, beta_deg):
    """An orbit at opposition at t0: on the anti-Sun line of sight, latitude beta."""
    rng = synth.make_rng(seed, 7)
    b = math.radians(beta_deg)
    d = np.array([math.cos(b) * math.cos(lam_mid), math.cos(b) * math.sin(lam_mid), math.sin(b)])
    obs = synth.observer_circular([t0], t0, lam_mid)[0]
    for _ in range(100):
        el, ok = synth.orbits_through(rng, d[None, :], obs, a, e, math.radians(inc_deg))
        if ok[0]:
            return el[0]
    raise RuntimeError("no reference orbit")


def draw_injections(seed, gf, t0, exps, n, s_rng, a_rng, e_rng, inc_rng, fwhm, min_snr=3.0,
                    stream=0):
    rng = synth.make_rng(seed, 55, stream)
    p2 = sum_p2(fwhm)
    out = []
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > 200000:
            raise RuntimeError("injection rejection sampling did not finish")
        el = synth.candidate_orbits(gf, 1, seed, a_rng, e_rng, inc_rng, stream=100000 * stream + tries)[0]
        s = float(rng.uniform(*s_rng))
        hits = hits_of(el, t0, exps)
        if s * math.sqrt(len(hits)) < min_snr:
            continue
        out.append(dict(el=[float(v) for v in el], s=s, flux=s / math.sqrt(p2), hits=hits))
    return out


def tiny(seed=1):
    """20 x 256^2 FP32, sigma 1, 0.2"/px, 30 days, one source s=1.5 on the
    reference orbit (a 2.7, e 0.1, i 5 deg), 10^4 candidate orbits."""
    lam = 0.4
    rng = synth.make_rng(seed, 1)
    t, t0 = make_epochs(rng, 20, 30.0)
    el_ref = reference_orbit(seed, t0, lam, 2.7, 0.1, 5.0, 1.0)
    exps = make_exposures(rng, t, 256, 256, 0.2, el_ref, t0, lam, [(0.0, 0.0)], (1.0, 1.0), 3.0)
    gf = grid_field(exps, t0, lam, 256, 256, 0.2)
    p2 = sum_p2(3.0)
    inj = [dict(el=[float(v) for v in el_ref], s=1.5, flux=1.5 / math.sqrt(p2), hits=hits_of(el_ref, t0, exps))]
    return dict(name="tiny", seed=seed, t0=t0, dtype="f32", nan_frac=0.0, exposures=exps, grid_field=gf,
                grid=dict(n=10000, a=[2.0, 3.5], e=[0.0, 0.3], inc_deg=[0.0, 15.0], cloud=0),
                injections=inj)


MOSAIC10 = [((k % 5) - 2) * 0.9 for k in range(10)]
MOSAIC10 = [(MOSAIC10[k], ((k // 5) - 0.5) * 0.9) for k in range(10)]


def survey(seed=2, n_exp=200, side=2048, n_orb=10_000_000, n_inj=20, cloud=1000, name="survey",
           span=60.0, nan_frac=0.005, offsets=MOSAIC10, width=None, ref=(2.7, 0.1, 5.0, 0.8),
           a_rng=(2.0, 3.5), e_rng=(0.0, 0.3), inc_rng=(0.0, 15.0), s_rng=(0.5, 2.0), dtype="f32",
           sigma_rng=(0.8, 1.25)):
    """Survey-scale mosaic: FP32 images plus variance, sigma U(0.8, 1.25),
    NaN-masked pixels, 0.2"/px, 10 field offsets; injections at per-image
    S/N U(0.5, 2) conditioned on s sqrt(n_hit) >= 3, each with a cloud of
    perturbed-a orbits."""
    lam = 1.1
    W = side if width is None else width
    H = side
    rng = synth.make_rng(seed, 1)
    t, t0 = make_epochs(rng, n_exp, span)
    el_ref = reference_orbit(seed, t0, lam, *ref)
    exps = make_exposures(rng, t, W, H, 0.2, el_ref, t0, lam, offsets, sigma_rng, 3.0)
    gf = grid_field(exps, t0, lam, W, H, 0.2)
    injs = draw_injections(seed, gf, t0, exps, n_inj, s_rng, a_rng, e_rng, inc_rng, 3.0)
    return dict(name=name, seed=seed, t0=t0, dtype=dtype, nan_frac=nan_frac, exposures=exps, grid_field=gf,
                grid=dict(n=n_orb, a=list(a_rng), e=list(e_rng), inc_deg=list(inc_rng), cloud=cloud,
                          cloud_da=1.5e-4), injections=injs)


def survey_small(seed=3):
    """Scaled-down survey for full oracle parity: 24 ragged 600x440 images,
    4 field offsets, 2x10^4 orbits, 3 injections with clouds of 50."""
    offs = [(-0.45, -0.45), (0.45, -0.45), (-0.45, 0.45), (0.45, 0.45)]
    return survey(seed=seed, n_exp=24, side=440, width=600, n_orb=20000, n_inj=3, cloud=50,
                  name="survey_small", span=8.0, offsets=offs)


def distant_small(seed=6):
    """Scaled-down distant-object case: 40 FP16 512x512 images over a year,
    reference orbit at 45 AU, candidates a 30-60 AU, e 0-0.3, i 0-40 deg,
    3 injections at per-image S/N U(0.2, 1) (rejection: s sqrt(n_hit) >= 3)."""
    return survey(seed=seed, n_exp=40, side=512, n_orb=20000, n_inj=3, cloud=50, name="distant_small",
                  span=365.0, nan_frac=0.0, offsets=[(0.0, 0.0)], ref=(45.0, 0.1, 10.0, 1.0),
                  a_rng=(30.0, 60.0), e_rng=(0.0, 0.3), inc_rng=(0.0, 40.0), s_rng=(0.2, 1.0), dtype="f16",
                  sigma_rng=(0.9, 1.1))


def oracle_sampler(gf, grid):
    """The generated grid's sampler in the form oracle.generate takes."""
    return dict(center=gf["center"], east=gf["east"], north=gf["north"], obs=gf["obs"], half_w=gf["half_w"],
                half_h=gf["half_h"], a=tuple(grid["a"]), e=tuple(grid["e"]),
                inc=tuple(math.radians(v) for v in grid["inc_deg"]), seed=int(grid["sampler_seed"]), epoch=gf["t"])


def draw_generated_injections(seed, gf, grid, t0, exps, n, s_rng, fwhm, min_snr=3.0, batch=64):
    """Injections on orbits of a device-generated grid: orbit indices drawn
    uniformly from [0, grid n), elements from the oracle's generator (so the
    true orbit is a member of the grid the stack searches), per-image S/N
    s ~ U(s_rng) kept when s sqrt(n_hit) >= min_snr."""
    rng = synth.make_rng(seed, 57)
    So = oracle_sampler(gf, grid)
    p2 = sum_p2(fwhm)
    out, used = [], set()
    for _ in range(1000):
        idx = rng.integers(0, int(grid["n"]), batch)
        s = rng.uniform(*s_rng, batch)
        el = np.array([ogen.sample_orbit(So, int(j)) or (np.nan,) * 6 for j in idx])
        ok = ~np.isnan(el[:, 0])
        smp = oracle.samples(el[ok], t0, exps)
        hit = (smp["flags"] & 3) == 3
        for r, k in enumerate(np.nonzero(ok)[0]):
            j = int(idx[k])
            nh = int(hit[r].sum())
            if j in used or s[k] * math.sqrt(nh) < min_snr:
                continue
            used.add(j)
            hits = [[int(e), float(smp["px"][r, e]), float(smp["py"][r, e])] for e in np.nonzero(hit[r])[0]]
            out.append(dict(index=j, el=[float(v) for v in el[k]], s=float(s[k]), flux=float(s[k] / math.sqrt(p2)),
                            hits=hits))
            if len(out) == n:
                return out
    raise RuntimeError("injection rejection sampling did not finish")


def distant(seed=8, n_exp=400, side=4096, n_orb=1_000_000_000, n_inj=100, name="distant"):
    """Distant objects at full size: 400 FP16 4096^2 images plus variance over
    365 days, 0.2"/px, the field following a reference orbit at 45 AU (e 0.1,
    i 10 deg); 10^9 candidate orbits a 30-60 AU, e 0-0.3, i 0-40 deg generated
    on the device from a counter-based sampler (the grid is the sampler, no
    element arrays); 100 injections on grid orbits at per-image S/N
    U(0.2, 1), kept when s sqrt(n_hit) >= 3."""
    lam = 1.1
    rng = synth.make_rng(seed, 1)
    t, t0 = make_epochs(rng, n_exp, 365.0)
    el_ref = reference_orbit(seed, t0, lam, 45.0, 0.1, 10.0, 1.0)
    exps = make_exposures(rng, t, side, side, 0.2, el_ref, t0, lam, [(0.0, 0.0)], (0.9, 1.1), 3.0)
    gf = grid_field(exps, t0, lam, side, side, 0.2)
    grid = dict(n=n_orb, a=[30.0, 60.0], e=[0.0, 0.3], inc_deg=[0.0, 40.0], cloud=0, generated=True,
                sampler_seed=seed * 1000 + 17)
    injs = draw_generated_injections(seed, gf, grid, t0, exps, n_inj, (0.2, 1.0), 3.0)
    return dict(name=name, seed=seed, t0=t0, dtype="f16", nan_frac=0.0, exposures=exps, grid_field=gf, grid=grid,
                injections=injs)


def reference_orbit_general(rng, obs, a_rng, e_rng, inc_rng, near_earth=False):
    """A reference orbit whose geometric position at the epoch is on a line of
    sight from the observer at elongation 60-180 deg (opposition excluded for
    a < 1 AU by the construction itself); near_earth puts it at r ~ 1.001 AU,
    elongation 90 deg, i.e. ~0.05 AU from the observer."""
    for _ in range(10000):
        a = float(rng.uniform(*a_rng))
        e = float(rng.uniform(*e_rng))
        inc = math.radians(float(rng.uniform(*inc_rng)))
        if near_earth:
            elong = math.radians(90.0)
        else:
            elong = math.radians(float(rng.uniform(60.0, 180.0)))
        lam_obs = math.atan2(obs[1], obs[0])
        side = 1.0 if rng.random() < 0.5 else -1.0
        lam = lam_obs + side * elong
        beta = math.radians(float(rng.uniform(-0.5, 0.5))) * min(1.0, math.degrees(inc) / 5.0)
        d = np.array([math.cos(beta) * math.cos(lam), math.cos(beta) * math.sin(lam), math.sin(beta)])
        el, ok = synth.orbits_through(rng, d[None, :], obs, a, e, inc)
        if not ok[0]:
            continue
        if near_earth:
            r, _, _ = oracle.helio_state(el[0], 0.0, 0.0)
            if not (0.02 < np.linalg.norm(r - obs) < 0.05):
                continue
        return el[0]
    raise RuntimeError("no reference orbit")


def batched(seed=4, n_patches=64, ne_rng=(30, 400), side_rng=(512, 2048), no_rng=(1e4, 1e6), span=30.0,
            name="batched", n_near=4, width_step=64, extra=()):
    """Uneven patches: N_e log-uniform, square sides uniform on a 64-px grid,
    N_o log-uniform, FP16 images, NEO-to-MBA elements (a 0.8-3.5 AU,
    e 0-0.6, i 0-30 deg), one injection on each patch's reference orbit at
    per-image S/N 1; the first n_near patches are near-Earth geometries.
    `extra` appends patches of given (exposures, span in days, side, orbits)."""
    rng = synth.make_rng(seed, 9)
    patches = []
    p2 = sum_p2(3.0)
    for p in range(n_patches + len(extra)):
        ne = int(round(math.exp(rng.uniform(math.log(ne_rng[0]), math.log(ne_rng[1])))))
        side = int(rng.integers(side_rng[0] // width_step, side_rng[1] // width_step + 1)) * width_step
        no = int(round(math.exp(rng.uniform(math.log(no_rng[0]), math.log(no_rng[1])))))
        p_span = span
        if p >= n_patches:
            ne, p_span, side, no = extra[p - n_patches]
        prng = synth.make_rng(seed, 10, p)
        t, t0 = make_epochs(prng, ne, p_span)
        lam = float(prng.uniform(0, 2 * math.pi))
        obs0 = synth.observer_circular([t0], t0, lam)[0]
        el_ref = reference_orbit_general(prng, obs0, (0.8, 3.5), (0.0, 0.6), (0.0, 30.0), near_earth=p < n_near)
        exps = make_exposures(prng, t, side, side, 0.2, el_ref, t0, lam, [(0.0, 0.0)], (0.9, 1.1), 3.0)
        gf = grid_field(exps, t0, lam, side, side, 0.2)
        inj = [dict(el=[float(v) for v in el_ref], s=1.0, flux=1.0 / math.sqrt(p2), hits=hits_of(el_ref, t0, exps))]
        patches.append(dict(name=f"{name}_{p}", seed=seed * 1000 + p, t0=t0, dtype="f16", nan_frac=0.0,
                            exposures=exps, grid_field=gf,
                            grid=dict(n=no, a=[0.8, 3.5], e=[0.0, 0.6], inc_deg=[0.0, 30.0], cloud=0),
                            injections=inj))
    return dict(name=name, seed=seed, patches=patches)


def batched_small(seed=5):
    """Scaled-down batch for full oracle parity: 6 patches, N_e 5-40,
    sides 128-320, N_o 300-3000, one near-Earth patch, plus one patch of 90
    exposures over 200 days (a dozen checkpoints and their re-anchors per orbit)."""
    return batched(seed=seed, n_patches=6, ne_rng=(5, 40), side_rng=(128, 320), no_rng=(300, 3000), span=6.0,
                   name="batched_small", n_near=1, width_step=64, extra=[(90, 200.0, 256, 2000)])


def learned(seed=2, n_cells=10000, cell_size=1000, n_real=50, n_inj=20, name="learned", base=None,
            snr_rng=(4.0, 12.0), da=2e-3, dm=5e-6, a_rng=(2.0, 3.5), e_rng=(0.0, 0.3), inc_rng=(0.0, 15.0)):
    """Cell-structured grid on the survey exposures (or those of `base`) for
    the learned proposer: n_cells representatives x cell_size members
    (perturbed a and M0); n_real realizations of n_inj injections, each on a
    random member of a random cell, flux set for a stacked S/N target
    U(snr_rng) over its hits."""
    g = base if base is not None else survey(seed=seed)
    gf = g["grid_field"]
    grid = dict(cells=n_cells, cell_size=cell_size, a=list(a_rng), e=list(e_rng), inc_deg=list(inc_rng), da=da, dm=dm,
                seed=seed + 100)
    el = synth.cell_grid(gf, n_cells, cell_size, grid["seed"], grid["a"], grid["e"], grid["inc_deg"], da, dm)
    rng = synth.make_rng(seed, 66)
    p2 = sum_p2(3.0)
    reals = []
    for r in range(n_real):
        injs = []
        while len(injs) < n_inj:
            c = int(rng.integers(0, n_cells))
            m = int(rng.integers(1, cell_size))
            o = c * cell_size + m
            hits = hits_of(el[o], g["t0"], g["exposures"])
            if len(hits) < 2:
                continue
            target = float(rng.uniform(*snr_rng))
            s = target / math.sqrt(len(hits))
            injs.append(dict(orbit=o, cell=c, el=[float(v) for v in el[o]], s=s, flux=s / math.sqrt(p2),
                             target=target, hits=hits))
        reals.append(injs)
    return dict(name=name, seed=seed, t0=g["t0"], dtype=g.get("dtype", "f32"), nan_frac=g["nan_frac"],
                exposures=g["exposures"], grid_field=gf, cell_grid=grid, realizations=reals)


def learned_small(seed=3):
    """Scaled-down learned-proposer geometry on the small survey."""
    return learned(seed=seed, n_cells=200, cell_size=50, n_real=4, n_inj=10, name="learned_small",
                   base=survey_small(seed=seed))


def distant_cells(seed=9):
    """The learned proposer on the distant-object exposures (400 FP16 4096^2
    images over 365 days, 0.2"/px): 10^4 cells x 10^3 members drawn like the
    distant candidates (a 30-60 AU, e 0-0.3, i 0-40 deg), the box +-0.02 AU in
    a and +-1.5e-5 rad in M0 (member tracks within about +-15 px of the
    representative's); 20 realizations of 20 injections at stacked S/N
    U(5, 12)."""
    return learned(seed=seed, n_cells=10000, cell_size=1000, n_real=20, n_inj=20, name="distant_cells",
                   base=distant(), snr_rng=(5.0, 12.0), da=0.02, dm=1.5e-5, a_rng=(30.0, 60.0), e_rng=(0.0, 0.3),
                   inc_rng=(0.0, 40.0))


WORKLOADS = {"tiny": tiny, "survey": survey, "survey_small": survey_small, "batched": batched,
             "batched_small": batched_small, "learned": learned, "learned_small": learned_small,
             "distant_small": distant_small, "distant": distant, "distant_cells": distant_cells}


def main(names):
    for nm in names or list(WORKLOADS):
        g = WORKLOADS[nm]()
        path = os.path.join(OUT, f"geom_{nm}.json")
        with open(path, "w") as f:
            json.dump(g, f, indent=None, separators=(",", ":"))
        if "realizations" in g:
            nh = [len(i["hits"]) for r in g["realizations"] for i in r]
            print(f"{nm}: {g['cell_grid']['cells']} cells x {g['cell_grid']['cell_size']}, "
                  f"{len(g['realizations'])} realizations, mean hits {np.mean(nh):.1f} -> {path}")
        elif "patches" in g:
            ne = [len(p["exposures"]) for p in g["patches"]]
            nh = [len(p["injections"][0]["hits"]) for p in g["patches"]]
            print(f"{nm}: {len(ne)} patches, exposures {sum(ne)}, orbits {sum(p['grid']['n'] for p in g['patches'])}, "
                  f"injection hits {nh} -> {path}")
        else:
            nh = [len(i["hits"]) for i in g["injections"]]
            print(f"{nm}: {len(g['exposures'])} exposures, {len(g['injections'])} injections, hits {nh} -> {path}")


if __name__ == "__main__":
    main(sys.argv[1:])
