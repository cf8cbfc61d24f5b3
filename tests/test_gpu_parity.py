"""GPU (HIP) path vs the CPU oracle, element by element (MI355X only)."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import (compare_samples, compare_stack_walk, decode_gathers, gpu_run, plane_offsets, snr_close,
                     to_torch_images)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    return synth.build_workload(synth.load_geometry("tiny"))


@pytest.fixture(scope="module")
def small():
    return synth.build_workload(synth.load_geometry("survey_small"))


def _planes_vs_oracle(w, exps_idx):
    import torch
    import paper_2503_08854_amd as dt
    ctx = dt.Context(0)
    Dt, Vt = to_torch_images(w.D, w.V)
    patch = dt.Patch(ctx, w.exps, Dt, Vt)
    for e in exps_idx:
        got = patch.plane(e).cpu().numpy().astype(np.float64)
        psi, phi = oracle.planes(w.D[e], w.V[e], w.exps[e]["fwhm"])
        # FP32 separable correlation vs FP64 stamps: relative to the plane scale
        sc_psi = np.sqrt(np.maximum(phi, 1e-30))
        assert np.max(np.abs(got[..., 0] - psi) / np.maximum(sc_psi, 1e-3)) < 2e-6
        assert np.max(np.abs(got[..., 1] - phi) / np.maximum(phi, 1e-30)) < 2e-6
        np.testing.assert_array_equal(got[..., 1] > 0, phi > 0)


def test_planes_tiny(tiny):
    _planes_vs_oracle(tiny, [0, 7, 19])


def test_planes_ragged_masked(small):
    _planes_vs_oracle(small, [0, 5, 23])


def test_samples_tiny_all(tiny):
    w = tiny
    ids = np.arange(w.elements.shape[0])
    g = gpu_run(w, ids=ids)
    o = oracle.samples(w.elements, w.t0, w.exps, w.D, w.V)
    nb, nc = compare_samples(g["dbg"], o, w.exps)
    assert nc > 10000 and nb < 5
    # gathered plane values at valid samples: psi/phi agree with the stamps
    v = (o["flags"] & 4) != 0
    assert np.max(np.abs(g["dbg"]["phi"][v] - o["phi"][v]) / o["phi"][v]) < 2e-6
    # light time agrees to 1e-13 day
    f = (o["flags"] & 1) != 0
    assert np.max(np.abs(g["dbg"]["tau"][f] - o["tau"][f])) < 1e-12


def test_stack_tiny(tiny):
    w = tiny
    g = gpu_run(w, k=16)
    snr, flux, nv = oracle.stack(w.elements, w.t0, w.exps, w.D, w.V)
    np.testing.assert_array_equal(g["nv"], nv)
    assert snr_close(g["snr"], snr).all()
    m = (nv > 0) & (np.abs(snr) > 1.0)
    assert np.all(np.abs(g["flux"][m] - flux[m]) <= 1e-4 * np.abs(flux[m]))
    # the injected orbit is the detection
    i = w.inj_index[0]
    assert g["topk_idx"][0] == i and g["snr"][i] > 5.0
    # top-k order: the oracle's ordering of the GPU's own S/N values
    want = oracle.topk(g["snr"].astype(np.float64), 16)
    np.testing.assert_array_equal(g["topk_idx"][:g["topk_cnt"]], want)


@pytest.mark.parametrize("name", ["tiny", "survey_small", "distant_small"])
def test_stack_walk_samples_match_oracle(name):
    """The per-sample table of the walk dt_stack runs (checkpoint prediction,
    its queue and its per-sample tail): every sample that lands was solved,
    and solved samples carry the oracle's pixel (bit-exact outside the 1e-6 px
    band), coordinates within 1e-6 px and light time within 1e-12 day."""
    import torch
    import paper_2503_08854_amd as dt
    w = synth.build_workload(synth.load_geometry(name))
    n = w.elements.shape[0]
    ids = np.unique(np.r_[np.arange(min(n, 4000)), w.inj_index])
    g = gpu_run(w)
    ctx, patch, orb, _, _ = g["_keep"]
    st = {k: v.cpu().numpy() for k, v in dt.debug_samples(patch, orb, ids, walk="stack").items()}
    torch.cuda.synchronize()
    o = oracle.samples(w.elements[ids], w.t0, w.exps, w.D, w.V)
    nb, ns, nc = compare_stack_walk(st, o, w.exps)
    assert o["bad"] == 0 and nb <= 2 and nc > 1000
    # pruning did its job: far fewer samples solved than walked
    assert ns < 0.5 * st["flags"].size
    # the table's valid samples are the stack's own: same counts as dt_stack
    np.testing.assert_array_equal(((st["flags"] & 4) != 0).sum(axis=1), np.maximum(g["nv"][ids], 0))


@pytest.mark.parametrize("name", ["tiny", "survey_small", "distant_small"])
def test_work_counters(name):
    """The stack's work counters: a wavefront either walks every exposure by
    prediction or gives up (deferred) and its live orbits are then walked per
    sample over every exposure; checkpoints follow the 12-day rule when no
    wavefront defers; every valid sample was solved (queued or on the per-sample
    walk's full path); counting changes no result."""
    import torch
    import paper_2503_08854_amd as dt
    import bench
    w = synth.build_workload(synth.load_geometry(name))
    g = gpu_run(w)
    ctx, patch, orb, _, _ = g["_keep"]
    ctx.count_work(True)
    snr, flux, nv = dt.stack(patch, orb)
    wk = ctx.work()
    ctx.count_work(False)
    np.testing.assert_array_equal(nv.cpu().numpy(), g["nv"])
    np.testing.assert_array_equal(snr.cpu().numpy(), g["snr"])
    n, ne = orb.n, patch.n_exp
    assert wk["tail_samples"] % ne == 0 and wk["tail_samples"] <= 64 * ne * wk["switched_waves"]
    assert wk["predicted"] + wk["tail_samples"] >= n * ne
    assert wk["predicted"] <= n * ne
    assert wk["checkpoint_solves"] <= n * bench.checkpoints(w.exps)
    if wk["switched_waves"] == 0:
        assert wk["predicted"] == n * ne and wk["tail_samples"] == 0
        assert wk["checkpoint_solves"] == n * bench.checkpoints(w.exps)
    assert wk["queued_solves"] + wk["tail_full"] >= int(np.maximum(g["nv"], 0).sum())
    assert wk["tail_full"] <= wk["tail_samples"]
    assert ctx.work()["predicted"] == 0     # reading zeroes the counters
    print(name, wk)


def test_stack_survey_small(small):
    w = small
    ids = np.arange(w.elements.shape[0])
    g = gpu_run(w, ids=ids, k=100)
    o = oracle.samples(w.elements, w.t0, w.exps, w.D, w.V)
    nb, nc = compare_samples(g["dbg"], o, w.exps)
    snr, flux, nv = oracle.stack(w.elements, w.t0, w.exps, w.D, w.V)
    np.testing.assert_array_equal(g["nv"], nv)
    ok = snr_close(g["snr"], snr)
    assert ok.all(), f"{(~ok).sum()} orbits outside tolerance, max err {np.max(np.abs(g['snr'] - snr))}"
    want = oracle.topk(g["snr"].astype(np.float64), 100)
    np.testing.assert_array_equal(g["topk_idx"][:g["topk_cnt"]], want)


def test_fp16_images_match_oracle_on_the_same_values(small):
    w = small
    w16 = synth.Workload(name="f16", exps=w.exps, t0=w.t0, elements=w.elements,
                         D=[d.astype(np.float16) for d in w.D], V=[v.astype(np.float16) for v in w.V],
                         injections=w.injections, inj_index=w.inj_index, dtype="f16")
    g = gpu_run(w16, k=10)
    snr, flux, nv = oracle.stack(w16.elements, w16.t0, w16.exps, w16.D, w16.V)
    np.testing.assert_array_equal(g["nv"], nv)
    assert snr_close(g["snr"], snr).all()
    # storage error of FP16 images against the FP32 images, reported
    snr32, _, _ = oracle.stack(w.elements, w.t0, w.exps, w.D, w.V)
    err = np.abs(g["snr"] - snr32) / np.maximum(1.0, np.abs(snr32))
    print(f"FP16-image S/N error vs FP32 images: max {err.max():.3g}, p99 {np.percentile(err, 99):.3g}")


def test_exposure_order_does_not_matter(small):
    w = small
    perm = synth.make_rng(5, 5).permutation(len(w.exps))
    wp = synth.Workload(name="perm", exps=[w.exps[i] for i in perm], t0=w.t0, elements=w.elements,
                        D=[w.D[i] for i in perm], V=[w.V[i] for i in perm])
    ids = np.arange(0, w.elements.shape[0], 97)
    a = gpu_run(w, ids=ids)
    b = gpu_run(wp, ids=ids)
    np.testing.assert_array_equal(a["snr"], b["snr"])
    np.testing.assert_array_equal(a["nv"], b["nv"])
    for key in ("ix", "iy", "flags", "px", "py"):
        np.testing.assert_array_equal(a["dbg"][key][:, perm], b["dbg"][key])


def test_deterministic(small):
    a = gpu_run(small)
    b = gpu_run(small)
    np.testing.assert_array_equal(a["snr"], b["snr"])
    np.testing.assert_array_equal(a["flux"], b["flux"])


def test_invalid_orbits_and_empty_sets(tiny):
    import torch
    import paper_2503_08854_amd as dt
    w = tiny
    el = w.elements[:8].copy()
    el[1, 0] = np.nan
    el[3, 1] = 1.2
    el[5, 0] = -1.0
    el[6, 1] = 1.0
    g = gpu_run(synth.Workload(name="bad", exps=w.exps, t0=w.t0, elements=el, D=w.D, V=w.V), k=4)
    bad = np.array([1, 3, 5, 6])
    assert np.all(np.isnan(g["snr"][bad])) and np.all(g["nv"][bad] == -1)
    good = np.setdiff1d(np.arange(8), bad)
    snr, _, nv = oracle.stack(el[good], w.t0, w.exps, w.D, w.V)
    assert snr_close(g["snr"][good], snr).all() and np.array_equal(g["nv"][good], nv)
    assert not np.isin(g["topk_idx"][:g["topk_cnt"]], bad).any()
    ctx, patch, orb, _, _ = g["_keep"]
    assert dt.validate_orbits(ctx, orb) == 4
    # empty orbit set
    e = dt.OrbitSet(np.zeros((0, 6)), w.t0)
    snr0, flux0, nv0 = dt.stack(patch, e)
    idx, val, cnt = dt.topk(ctx, snr0, 5)
    torch.cuda.synchronize()
    assert snr0.numel() == 0 and int(cnt.cpu()[0]) == 0 and np.all(idx.cpu().numpy() == -1)


def test_tiny_images_and_behind_the_plane():
    import torch
    import paper_2503_08854_amd as dt
    el = np.array([[2.7, 0.1, math.radians(5), 0.4, 1.0, 0.3]])
    t0 = 0.0
    robs = synth.observer_circular([0.0], 0.0, 0.2)[0]
    rho, _, _, _ = oracle.light_time(el[0], t0, 0.0, robs)
    ra, dec = synth.vec_to_radec(oracle.ecl_to_eq(rho / np.linalg.norm(rho)))
    s = 0.2 / 3600
    base = dict(t=0.0, obs=list(robs), crval=[float(ra), float(dec)], cd=[-s, 0, 0, s], fwhm=3.0)
    exps = [dict(base, crpix=[3.0, 2.0], width=5, height=3),                       # 5x3 image, hit at (2, 1)
            dict(base, crpix=[1.0, 1.0], width=1, height=1),                       # 1x1 image
            dict(base, crval=[(float(ra) + 180) % 360, -float(dec)], crpix=[3, 3], width=5, height=5)]  # behind
    rng = np.random.default_rng(0)
    D = [rng.standard_normal((x["height"], x["width"])).astype(np.float32) for x in exps]
    V = [np.full((x["height"], x["width"]), 2.0, np.float32) for x in exps]
    w = synth.Workload(name="edge", exps=exps, t0=t0, elements=el, D=D, V=V)
    g = gpu_run(w, ids=[0], k=1)
    o = oracle.samples(el, t0, exps, D, V)
    assert list(g["dbg"]["flags"][0] & 7) == list(o["flags"][0] & 7) == [7, 7, 0]
    assert np.all((g["dbg"]["flags"][0] & 8) != 0)   # the exact walk solves every sample
    snr, flux, nv = oracle.stack(el, t0, exps, D, V)
    assert snr_close(g["snr"], snr).all() and g["nv"][0] == nv[0] == 2


def test_topk_edge_cases():
    import torch
    import paper_2503_08854_amd as dt
    ctx = dt.Context(0)
    rng = np.random.default_rng(1)
    # inputs of at most 16384 keys take the one-workgroup radix-select path,
    # larger ones the tournament; the last two cases are all ties
    for n, k, thr in [(1, 1, -np.inf), (10, 50, -np.inf), (100000, 4096, -np.inf), (100000, 100, 2.5),
                      (8192 * 3 + 17, 1000, 0.0), (5000, 10, 100.0), (10000, 200, -np.inf),
                      (16384, 4096, -np.inf), (16384, 3000, 0.5), (16385, 200, -np.inf), (12000, 777, None),
                      (7, 3, None)]:
        if thr is None:
            v = np.zeros(n, np.float32)
            thr = -np.inf
        else:
            v = np.round(rng.standard_normal(n), 2).astype(np.float32)
            v[rng.integers(0, n, max(1, n // 100))] = np.nan
        t = torch.from_numpy(v).cuda()
        idx, val, cnt = dt.topk(ctx, t, k, thr)
        torch.cuda.synchronize()
        c = int(cnt.cpu()[0])
        vv = np.where(np.isnan(v), -np.inf, v).astype(np.float64)
        want = oracle.topk(vv, k, thr if np.isfinite(thr) else -1e300)
        want = want[~np.isnan(v[want])]
        np.testing.assert_array_equal(idx.cpu().numpy()[:c], want)
        np.testing.assert_array_equal(val.cpu().numpy()[:c], v[want])
        assert np.all(idx.cpu().numpy()[c:] == -1)
        # the unordered call: the same count and set, each index with its value
        iu, vu, cu = dt.topk(ctx, t, k, thr, ordered=False)
        torch.cuda.synchronize()
        assert int(cu.cpu()[0]) == c
        iu, vu = iu.cpu().numpy(), vu.cpu().numpy()
        np.testing.assert_array_equal(np.sort(iu[:c]), np.sort(want))
        np.testing.assert_array_equal(vu[:c], v[iu[:c]])
        assert np.all(iu[c:] == -1) and np.all(np.isnan(vu[c:]))
        if n > 16384:
            np.testing.assert_array_equal(iu[:c], want)  # larger inputs come out sorted


def test_argument_errors():
    import torch
    import paper_2503_08854_amd as dt
    ctx = dt.Context(0)
    t = torch.zeros(10, device="cuda")
    with pytest.raises(dt.DtrackError, match="DT_E_ARG"):
        dt.topk(ctx, t, 0)
    with pytest.raises(dt.DtrackError, match="DT_E_ARG"):
        dt.topk(ctx, t, 5000)
    x = dict(t=0.0, obs=[1, 0, 0], crval=[0, 0], crpix=[1, 1], cd=[1e-4, 0, 0, 1e-4], width=4, height=4, fwhm=9.0)
    im = torch.zeros((4, 4), device="cuda")
    with pytest.raises(dt.DtrackError, match="DT_E_DOMAIN"):
        dt.Patch(ctx, [x], [im], [im])
    with pytest.raises(dt.DtrackError, match="DT_E_DOMAIN"):
        dt.Patch(ctx, [dict(x, fwhm=3.0, cd=[1e-4, 1e-4, 1e-4, 1e-4])], [im], [im])
    used = ctx.mem_used()
    ctx.set_mem_limit(used + 200)
    with pytest.raises(dt.DtrackError, match="DT_E_OOM"):
        dt.Patch(ctx, [dict(x, fwhm=3.0)], [im], [im])
    assert ctx.mem_used() == used
    ctx.set_mem_limit(0)
    p = dt.Patch(ctx, [dict(x, fwhm=3.0)], [im], [im])
    # follow-on rows: argument and domain errors are reported, nothing is launched
    with pytest.raises(dt.DtrackError, match="DT_E_DOMAIN"):
        dt.image_noise(ctx, [im], kappa=0.0)
    with pytest.raises(dt.DtrackError, match="DT_E_ARG"):
        dt.image_noise(ctx, [im], max_iter=0)
    f = synth.load_geometry("tiny")["grid_field"]
    with pytest.raises(dt.DtrackError, match="DT_E_DOMAIN"):
        dt.generate_orbits(ctx, dt.orbit_sampler(f, f["t"], (2.0, 1.0), (0.0, 0.3), (0.0, 15.0), 1), 0, 10)
    with pytest.raises(dt.DtrackError, match="DT_E_DOMAIN"):
        dt.generate_orbits(ctx, dt.orbit_sampler(f, f["t"], (2.0, 3.0), (0.0, 1.0), (0.0, 15.0), 1), 0, 10)
    orb = dt.OrbitSet(np.array([[2.5, 0.1, 0.1, 0.0, 0.0, 0.0]]), 0.0)
    with pytest.raises(dt.DtrackError, match="DT_E_ARG"):
        dt.clip_candidates(p, orb, np.array([0]), kappa=0.0)
    with pytest.raises(dt.DtrackError, match="DT_E_DOMAIN"):
        dt.cell_stamps(p, orb, 0.0, 1e-5)
    with pytest.raises(dt.DtrackError, match="DT_E_STATE"):
        p.noise()                       # the patch has variance planes
    p.close()
    assert ctx.mem_used() == used


def test_survey_full_size_sampled():
    """Bench-size survey (200 x 2048^2, 10^7 orbits) in the launch the bench
    times; the oracle recomputes a sample of orbits one by one."""
    import torch
    geom = synth.load_geometry("survey")
    w = synth.build_workload(geom, device="cuda")
    rng = np.random.default_rng(7)
    n = w.elements.shape[0]
    dbg_ids = np.sort(rng.choice(n, 200, replace=False))
    g = gpu_run(w, k=100, thr=5.0, ids=dbg_ids)
    ids = np.unique(np.r_[rng.choice(n, 3000, replace=False), w.inj_index, g["topk_idx"][:g["topk_cnt"]]])
    D = [d.cpu().numpy() for d in w.D]
    V = [v.cpu().numpy() for v in w.V]
    snr, flux, nv = oracle.stack(w.elements[ids], w.t0, w.exps, D, V)
    np.testing.assert_array_equal(g["nv"][ids], nv)
    ok = snr_close(g["snr"][ids], snr)
    assert ok.all(), f"{(~ok).sum()} sampled orbits outside tolerance"
    o = oracle.samples(w.elements[dbg_ids], w.t0, w.exps, D, V)
    nb, nc = compare_samples(g["dbg"], o, w.exps)
    assert o["bad"] == 0 and nb <= 2
    # top-k: every reported orbit really has S/N >= 5 and the order is the oracle's on GPU values
    want = oracle.topk(g["snr"].astype(np.float64), 100, 5.0)
    np.testing.assert_array_equal(g["topk_idx"][:g["topk_cnt"]], want)


def test_outlier_trimming_matches_oracle(small):
    """Sigma clipping of candidate intersections (Sec. 5.2.3) on the GPU vs the
    oracle's clipping of its own FP64 stamp values; an artifact planted in one
    image under an orbit is removed."""
    import torch
    import paper_2503_08854_amd as dt
    w = small
    o = oracle.samples(w.elements, w.t0, w.exps)
    nv = ((o["flags"] & 3) == 3).sum(1)
    rng = np.random.default_rng(3)
    pool = np.nonzero(nv >= 3)[0]
    ids = np.sort(rng.choice(pool, min(400, pool.size), replace=False))
    target = int(ids[0])
    e_art = int(np.nonzero((o["flags"][target] & 3) == 3)[0][0])
    D = [d.copy() for d in w.D]
    ix, iy = o["ix"][target, e_art], o["iy"][target, e_art]
    yy, xx = np.mgrid[-4:5, -4:5]
    blob = 40.0 * np.exp(-(xx ** 2 + yy ** 2) / 3.2)
    y0, x0 = iy - 4, ix - 4
    ys = slice(max(y0, 0), min(y0 + 9, D[e_art].shape[0]))
    xs = slice(max(x0, 0), min(x0 + 9, D[e_art].shape[1]))
    D[e_art][ys, xs] += blob[ys.start - y0:ys.stop - y0, xs.start - x0:xs.stop - x0].astype(np.float32)
    wa = synth.Workload(name="art", exps=w.exps, t0=w.t0, elements=w.elements, D=D, V=w.V)
    g = gpu_run(wa)
    ctx, patch, orb, _, _ = g["_keep"]
    snr_c, flux_c, nk_c = dt.clip_candidates(patch, orb, ids, 3.0, 10)
    torch.cuda.synchronize()
    snr_c, nk_c = snr_c.cpu().numpy(), nk_c.cpu().numpy()
    so = oracle.samples(w.elements[ids], w.t0, w.exps, D, w.V)
    n_band = 0
    for r in range(ids.size):
        v = so["valid"][r]
        psi, phi = so["psi"][r][v], so["phi"][r][v]
        s_or, f_or, k_or, kept = oracle.sigma_clip(psi, phi, 3.0, 10)
        mu = psi[kept].sum() / phi[kept].sum() if kept.any() else 0.0
        chi = np.abs(psi - mu * phi) / np.sqrt(phi)
        if np.any(np.abs(chi - 3.0) < 1e-4):
            n_band += 1
            continue
        assert nk_c[r] == k_or, (r, nk_c[r], k_or)
        assert abs(snr_c[r] - s_or) <= 1e-5 * max(1.0, abs(s_or)), (r, snr_c[r], s_or)
    assert n_band <= 2
    assert g["snr"][target] > 5.0 and snr_c[0] < 3.0 and nk_c[0] == nv[target] - 1


def _sampler_pair(seed, a=(2.0, 3.5), e=(0.0, 0.3), inc_deg=(0.0, 15.0), name="survey_small"):
    import paper_2503_08854_amd as dt
    f = synth.load_geometry(name)["grid_field"]
    ora = dict(center=f["center"], east=f["east"], north=f["north"], obs=f["obs"], half_w=f["half_w"],
               half_h=f["half_h"], a=a, e=e, inc=tuple(math.radians(v) for v in inc_deg), seed=seed, epoch=f["t"])
    return dt.orbit_sampler(f, f["t"], a, e, inc_deg, seed), ora


def _angle_diff(x, y):
    d = np.mod(x - y + math.pi, 2 * math.pi) - math.pi
    return np.abs(d)


def test_generated_orbits_match_oracle():
    import torch
    import paper_2503_08854_amd as dt
    from oracle import generate as G
    ctx = dt.Context(0)
    for seed, first, n in [(7, 0, 3000), (8, 123456789, 777), (9, 5, 0)]:
        S, So = _sampler_pair(seed)
        got = dt.generate_orbits(ctx, S, first, n)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        want = G.generate(So, first, n)
        np.testing.assert_array_equal(np.isnan(got[:, 0]), np.isnan(want[:, 0]))
        ok = ~np.isnan(want[:, 0])
        np.testing.assert_allclose(got[ok, :3], want[ok, :3], rtol=1e-12, atol=1e-12)
        assert np.max(_angle_diff(got[ok, 3:], want[ok, 3:]), initial=0) < 1e-9


def test_generate_and_stack_matches_stack_and_oracle(small):
    import torch
    import paper_2503_08854_amd as dt
    from oracle import generate as G
    w = small
    ctx = dt.Context(0)
    Dt, Vt = to_torch_images(w.D, w.V)
    patch = dt.Patch(ctx, w.exps, Dt, Vt)
    S, So = _sampler_pair(21)
    n, first = 20000, 1000
    snr_g, flux_g, nv_g = dt.stack_generated(patch, S, first, n)
    el = dt.generate_orbits(ctx, S, first, n)
    orb = dt.OrbitSet(el.cpu().numpy(), So["epoch"], "cuda")
    snr_s, flux_s, nv_s = dt.stack(patch, orb)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(nv_g.cpu().numpy(), nv_s.cpu().numpy())
    a, b = snr_g.cpu().numpy(), snr_s.cpu().numpy()
    assert np.array_equal(np.isnan(a), np.isnan(b))
    assert snr_close(a[~np.isnan(a)], b[~np.isnan(b)], 1e-6).all()
    # the oracle on its own generated orbits (a sample the C oracle stacks in seconds)
    m = 2000
    elo = G.generate(So, first, m)
    snr_o, _, nv_o = oracle.stack(elo, So["epoch"], w.exps, w.D, w.V)
    ok = snr_close(a[:m], snr_o)
    same_nv = nv_g.cpu().numpy()[:m] == nv_o
    assert ok[same_nv].all()
    # an orbit may differ only through a sample within 1e-6 px of a rounding boundary
    bad = np.nonzero(~same_nv | ~ok)[0]
    if bad.size:
        o = oracle.samples(elo[bad], So["epoch"], w.exps)
        W = np.array([x["width"] for x in w.exps])[None, :].repeat(bad.size, 0)
        H = np.array([x["height"] for x in w.exps])[None, :].repeat(bad.size, 0)
        from helpers import band_mask
        inb = band_mask(o["px"], o["py"], W, H) & ((o["flags"] & 1) != 0)
        assert inb.any(axis=1).all()
    assert (nv_o > 0).sum() > 100


def test_generated_probe_then_rest_matches_stack(small):
    """More than 2^26 generated orbits: the first 2^22 run the checkpoint walk
    as a probe, whose deferral rate picks the walk for the rest.  Whichever
    it picks, valid counts equal those of dt_stack on the same generated
    elements and S/N agrees to rounding."""
    import torch
    import paper_2503_08854_amd as dt
    w = small
    ctx = dt.Context(0)
    Dt, Vt = to_torch_images(w.D, w.V)
    patch = dt.Patch(ctx, w.exps, Dt, Vt)
    S, So = _sampler_pair(21)
    n, first = (1 << 26) + 3 * (1 << 16) + 37, 5
    ctx.count_work(True)
    snr_g, flux_g, nv_g = dt.stack_generated(patch, S, first, n)
    wk = ctx.work()
    ctx.count_work(False)
    el = dt.generate_orbits(ctx, S, first, n)
    orb = dt.OrbitSet(el, So["epoch"], "cuda")   # device to device
    del el
    snr_s, flux_s, nv_s = dt.stack(patch, orb)
    torch.cuda.synchronize()
    print("probe path:", wk)
    np.testing.assert_array_equal(nv_g.cpu().numpy(), nv_s.cpu().numpy())
    a, b = snr_g.cpu().numpy(), snr_s.cpu().numpy()
    assert np.array_equal(np.isnan(a), np.isnan(b))
    assert snr_close(a[~np.isnan(a)], b[~np.isnan(b)], 1e-6).all()
    assert (nv_g.cpu().numpy() > 0).sum() > 1000


def _noise_images(rng):
    ims = []
    x = rng.normal(0.0, 2.0, (256, 256)).astype(np.float32)
    x[rng.random(x.shape) < 0.01] = np.nan
    x[rng.random(x.shape) < 0.005] = 400.0          # bright outliers
    ims.append(x)
    ims.append(rng.normal(5.0, 0.3, (37, 1001)).astype(np.float32))   # ragged, offset
    ims.append(np.full((3, 5), 7.0, np.float32))                     # constant: sigma 0
    ims.append(np.full((4, 4), np.nan, np.float32))                  # no finite pixel
    ims.append(np.array([[1.5]], np.float32))                        # one pixel
    ims.append(np.zeros((0, 8), np.float32))                         # empty
    ims.append(np.round(rng.normal(0, 3, (64, 80))).astype(np.float32))   # many ties
    y = rng.standard_cauchy((128, 96)).astype(np.float32)            # heavy tails, +-0
    y[0, :4] = [0.0, -0.0, 0.0, -0.0]
    ims.append(y)
    return ims


def test_image_noise_matches_oracle_exactly():
    import torch
    import paper_2503_08854_amd as dt
    rng = np.random.default_rng(17)
    ims = _noise_images(rng)
    ctx = dt.Context(0)
    for kappa, max_iter in [(3.0, 10), (2.5, 10), (3.0, 1), (4.0, 3)]:
        dev = [torch.from_numpy(x).cuda() for x in ims]
        sig, used, it = dt.image_noise(ctx, dev, kappa, max_iter)
        torch.cuda.synchronize()
        sig, used, it = sig.cpu().numpy(), used.cpu().numpy(), it.cpu().numpy()
        for i, x in enumerate(ims):
            ws, wu, wi = oracle.mad_noise(x, kappa, max_iter)
            assert (it[i], used[i]) == (wi, wu), (i, kappa, max_iter)
            if math.isnan(ws):
                assert math.isnan(sig[i])
            else:
                assert sig[i] == ws, (i, kappa, max_iter, sig[i], ws)


def test_image_noise_fp16_and_many_images():
    import torch
    import paper_2503_08854_amd as dt
    rng = np.random.default_rng(23)
    ctx = dt.Context(0)
    ims = [rng.normal(0, rng.uniform(0.5, 3), (int(rng.integers(1, 300)), int(rng.integers(1, 300))))
           .astype(np.float16) for _ in range(40)]
    sig, used, it = dt.image_noise(ctx, [torch.from_numpy(x).cuda() for x in ims])
    torch.cuda.synchronize()
    sig, used, it = sig.cpu().numpy(), used.cpu().numpy(), it.cpu().numpy()
    for i, x in enumerate(ims):
        ws, wu, wi = oracle.mad_noise(x.astype(np.float32))
        assert sig[i] == ws and used[i] == wu and it[i] == wi


def test_patch_without_variance_uses_mad_noise(small):
    import torch
    import paper_2503_08854_amd as dt
    w = small
    ctx = dt.Context(0)
    Dt, _ = to_torch_images(w.D, w.V)
    patch = dt.Patch(ctx, w.exps, Dt)
    sig = patch.noise().cpu().numpy()
    Vo = []
    for e, d in enumerate(w.D):
        ws, _, _ = oracle.mad_noise(d)
        assert sig[e] == ws
        v = np.full(d.shape, np.float32(ws * ws), np.float32)
        Vo.append(v)
    for e in (0, len(w.exps) // 2, len(w.exps) - 1):
        got = patch.plane(e).cpu().numpy().astype(np.float64)
        psi, phi = oracle.planes(w.D[e], Vo[e], w.exps[e]["fwhm"])
        sc = np.sqrt(np.maximum(phi, 1e-30))
        assert np.max(np.abs(got[..., 0] - psi) / np.maximum(sc, 1e-3)) < 2e-6
        assert np.max(np.abs(got[..., 1] - phi) / np.maximum(phi, 1e-30)) < 2e-6
    orb = dt.OrbitSet(w.elements, w.t0, "cuda")
    snr, _, nv = dt.stack(patch, orb)
    torch.cuda.synchronize()
    snr_o, _, nv_o = oracle.stack(w.elements, w.t0, w.exps, w.D, Vo)
    np.testing.assert_array_equal(nv.cpu().numpy(), nv_o)
    assert snr_close(snr.cpu().numpy(), snr_o).all()
    # refresh after an in-place change re-estimates the noise
    for d in Dt:
        d.mul_(2.0)
    patch.refresh()
    sig2 = patch.noise().cpu().numpy()
    np.testing.assert_array_equal(sig2, 2.0 * sig)


def test_gather_replay_equals_stack(small):
    import torch
    import paper_2503_08854_amd as dt
    w = small
    g = gpu_run(w, ids=np.arange(w.elements.shape[0]))
    ctx, patch, orb, _, _ = g["_keep"]
    rec = dt.record_valid_gathers(patch, orb)
    snr = dt.replay_valid_gathers(patch, rec)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(snr.cpu().numpy(), np.where(g["nv"] > 0, g["snr"], 0.0).astype(np.float32))
    # the recorded offsets are the exact walk's inside samples, in epoch order
    lists = decode_gathers(rec)
    dbg = g["dbg"]
    want, order = plane_offsets(dbg, w.exps)
    inside = ((dbg["flags"] & 2) != 0)[:, order]
    assert rec.count == int(inside.sum())
    for i in range(orb.n):
        k = int(inside[i].sum())
        np.testing.assert_array_equal(lists[i, :k], want[i][inside[i]])
        assert np.all(lists[i, k:] == -1)


def _pruned_vs_exact(w):
    import torch
    import paper_2503_08854_amd as dt
    ids = np.arange(w.elements.shape[0])
    g = gpu_run(w, ids=ids)
    ctx, patch, orb, _, _ = g["_keep"]
    rec = dt.record_valid_gathers(patch, orb)
    snr = dt.replay_valid_gathers(patch, rec)
    torch.cuda.synchronize()
    nv_exact = ((g["dbg"]["flags"] & 4) != 0).sum(axis=1)
    np.testing.assert_array_equal(np.maximum(g["nv"], 0), nv_exact)
    np.testing.assert_array_equal(snr.cpu().numpy(), np.where(g["nv"] > 0, g["snr"], 0.0).astype(np.float32))
    # the walk the stack runs solves every sample the exact walk finds inside, identically
    st = {k: v.cpu().numpy() for k, v in dt.debug_samples(patch, orb, ids, walk="stack").items()}
    ex = g["dbg"]
    inside = (ex["flags"] & 2) != 0
    assert np.all((st["flags"][inside] & 8) != 0)
    np.testing.assert_array_equal(st["ix"][inside], ex["ix"][inside])
    np.testing.assert_array_equal(st["iy"][inside], ex["iy"][inside])
    np.testing.assert_array_equal(st["flags"][inside] & 7, ex["flags"][inside] & 7)
    return int(nv_exact.sum())


@pytest.mark.parametrize("name", ["tiny", "survey_small", "distant_small"])
def test_pruned_stack_equals_exact_walk(name):
    """The stack skips the light-time correction and projection of samples
    whose uncorrected position is outside the exposure's sky cone by more than
    the bound on the light-time shift; the debug walk projects every sample.
    Valid counts and S/N agree exactly on every orbit."""
    w = synth.build_workload(synth.load_geometry(name))
    assert _pruned_vs_exact(w) > 100


def _far_tangent(x, deg):
    """The exposure re-expressed with its TAN tangent point `deg` degrees from
    its field centre and CRPIX moved so that the centre pixel still looks at
    the field (a strongly distorted projection of the same sky)."""
    d2r = np.pi / 180.0
    ra, dec = x["crval"][0] * d2r, x["crval"][1] * d2r
    f = np.array([np.cos(dec) * np.cos(ra), np.cos(dec) * np.sin(ra), np.sin(dec)])
    north = np.array([-np.sin(dec) * np.cos(ra), -np.sin(dec) * np.sin(ra), np.cos(dec)])
    c = np.cos(deg * d2r) * f + np.sin(deg * d2r) * north
    rc, dc = np.arctan2(c[1], c[0]), np.arcsin(c[2])
    e_c = np.array([-np.sin(rc), np.cos(rc), 0.0])
    n_c = np.array([-np.sin(dc) * np.cos(rc), -np.sin(dc) * np.sin(rc), np.cos(dc)])
    xi, eta = (e_c @ f) / (c @ f) / d2r, (n_c @ f) / (c @ f) / d2r
    cd = np.array(x["cd"]).reshape(2, 2)
    off = np.linalg.solve(cd, [xi, eta])
    y = dict(x)
    y["crval"] = [float(rc / d2r % 360.0), float(dc / d2r)]
    y["crpix"] = [float(x["crpix"][0] - off[0]), float(x["crpix"][1] - off[1])]
    return y


@pytest.mark.parametrize("case", ["wide", "far60", "far80"])
def test_sky_cone_edge_geometries(tiny, case):
    """Exposures whose sky cone is too wide to be used (200"/px), whose image
    is 60 deg from the tangent point (a heavily distorted cone) or 80 deg from
    it (no cone): the stack equals the exact walk and the oracle."""
    w = tiny
    if case == "wide":
        exps = [dict(x, cd=[v * 1000.0 for v in x["cd"]]) for x in w.exps]
    else:
        exps = [_far_tangent(x, 60.0 if case == "far60" else 80.0) for x in w.exps]
    el = w.elements[:4000] if case == "wide" else w.elements
    w2 = synth.Workload(name=case, exps=exps, t0=w.t0, elements=el, D=w.D, V=w.V)
    n_valid = _pruned_vs_exact(w2)
    assert n_valid > 20  # the 80-deg image covers a much smaller piece of sky
    g = gpu_run(w2)
    snr, flux, nv = oracle.stack(w2.elements, w2.t0, exps, w.D, w.V)
    np.testing.assert_array_equal(g["nv"], nv)
    ok = snr_close(g["snr"], snr)
    assert ok.all(), f"{(~ok).sum()} orbits outside tolerance"


def _tracked_long_gaps(w):
    """Epochs of the small field spread over a year; even exposures point at
    a main-belt orbit, odd ones at a short-period eccentric orbit (a = 1 AU,
    e = 0.7), with 2 arcsec pixels; orbits: a cloud around each."""
    import math
    t0 = w.t0
    ref_mb = w.elements[w.inj_index[0]]
    ref_fast = np.array([1.0, 0.7, math.radians(12.0), 1.0, 2.0, 0.5])

    def point(x, el):
        rho, _, _, _ = oracle.light_time(el, t0, x["t"], np.array(x["obs"], float))
        u = oracle.ecl_to_eq(rho / np.linalg.norm(rho))
        ra, dec = math.degrees(math.atan2(u[1], u[0])) % 360.0, math.degrees(math.asin(u[2]))
        return dict(x, crval=[ra, dec], crpix=[x["width"] / 2 + 0.5, x["height"] / 2 + 0.5])

    exps = [dict(x, t=t0 + 12.0 * (x["t"] - t0), cd=[v * 10.0 for v in x["cd"]]) for x in w.exps]
    exps = [point(x, ref_mb if i % 2 == 0 else ref_fast) for i, x in enumerate(exps)]
    rng = np.random.default_rng(3)

    def cloud(ref, n, da, dm):
        c = np.repeat(ref[None], n, 0)
        c[:, 0] += rng.uniform(-da, da, n)
        c[:, 5] += rng.uniform(-dm, dm, n)
        return c

    return exps, np.concatenate([cloud(ref_mb, 3000, 2e-3, 2e-3), cloud(ref_fast, 3000, 2e-4, 2e-3)])


@pytest.mark.parametrize("case", ["shared_epoch", "long_gaps", "one_exposure", "repeated_exposure"])
def test_checkpoint_walk_edge_cases(tiny, case):
    """The stack's checkpoint prediction (a bound on the observer's speed, a
    checkpoint every few weeks of epochs) against the exact walk and the
    oracle.  shared_epoch: two exposures at one epoch seen from different
    observers leave the observer speed unbounded, and the per-sample walk
    runs instead.  long_gaps: gaps of weeks between exposures and orbits
    whose Kepler steps between checkpoints exceed the warm start's reach
    (a = 1 AU, e = 0.7), landing in up to ten exposures each.  one_exposure:
    a patch of the exposure nearest the grid epoch alone.  repeated_exposure:
    that exposure twice (same epoch and observer, so the observer speed stays
    bounded), each copy with its own images."""
    w = tiny
    D, V = w.D, w.V
    if case == "shared_epoch":
        exps = [dict(x) for x in w.exps]
        exps[1] = dict(exps[1], t=exps[0]["t"], obs=[v + 1e-4 for v in exps[0]["obs"]])
        el = w.elements
    elif case == "long_gaps":
        exps, el = _tracked_long_gaps(w)
    else:
        k = int(np.argmin([abs(x["t"] - w.t0) for x in w.exps]))
        j = (k + 1) % len(w.exps)
        exps = [dict(w.exps[k])] if case == "one_exposure" else [dict(w.exps[k]), dict(w.exps[k])]
        D, V = ([w.D[k]], [w.V[k]]) if case == "one_exposure" else ([w.D[k], w.D[j]], [w.V[k], w.V[j]])
        el = w.elements
    w2 = synth.Workload(name=case, exps=exps, t0=w.t0, elements=el, D=D, V=V)
    n_valid = _pruned_vs_exact(w2)
    assert n_valid > (5000 if case in ("shared_epoch", "long_gaps") else 500)
    g = gpu_run(w2)
    snr, flux, nv = oracle.stack(w2.elements, w2.t0, exps, D, V)
    np.testing.assert_array_equal(g["nv"], nv)
    ok = snr_close(g["snr"], snr)
    assert ok.all(), f"{(~ok).sum()} orbits outside tolerance"


def test_stack_distant_objects_fp16():
    """Distant-object regime (a 30-60 AU over a year, light time 0.1-0.45 day,
    FP16 images): every sample and S/N against the oracle on the same FP16
    values."""
    w = synth.build_workload(synth.load_geometry("distant_small"))
    assert w.D[0].dtype == np.float16
    ids = np.arange(w.elements.shape[0])
    g = gpu_run(w, ids=ids, k=50)
    o = oracle.samples(w.elements, w.t0, w.exps, w.D, w.V)
    nb, nc = compare_samples(g["dbg"], o, w.exps)
    assert nc > 10000
    np.testing.assert_allclose(g["dbg"]["tau"][(o["flags"] & 1) != 0], o["tau"][(o["flags"] & 1) != 0],
                               rtol=0, atol=1e-12)
    snr, flux, nv = oracle.stack(w.elements, w.t0, w.exps, w.D, w.V)
    np.testing.assert_array_equal(g["nv"], nv)
    ok = snr_close(g["snr"], snr)
    assert ok.all(), f"{(~ok).sum()} orbits outside tolerance"
    want = oracle.topk(g["snr"].astype(np.float64), 50)
    np.testing.assert_array_equal(g["topk_idx"][:g["topk_cnt"]], want)


def test_checkpoint_epochs_at_the_span_boundary(tiny):
    """The checkpoint schedule taken per exposure in the exposure preparation
    follows the walk's rule exactly at the boundary: epochs on a 1/64-day
    grid (exact differences), one exposure exactly 12 days after the first
    checkpoint and one exactly 12 days after the second (neither is a
    checkpoint: the span must be exceeded), and the stack against the oracle
    on these exposures."""
    import paper_2503_08854_amd as dt
    import bench
    w = tiny
    order = np.argsort([x["t"] for x in w.exps])
    t_rel = np.array([w.exps[i]["t"] for i in order]) - w.exps[order[0]]["t"]
    new = np.round(t_rel * 64.0) / 64.0
    new[9] = 12.0                    # was 12.96: exactly the span after the first checkpoint (0)
    new[16] = new[10] + 12.0         # was 24.27: exactly the span after the checkpoint at new[10]
    assert np.all(np.diff(new) > 0) and new[10] > 12.0 and new[17] > new[16]
    base = float(np.floor(w.exps[order[0]]["t"]))
    exps = [dict(x) for x in w.exps]
    for rank, i in enumerate(order):
        exps[i]["t"] = base + float(new[rank])
    assert bench.checkpoints(exps) == 3      # at new[0], new[10] and new[17]
    w2 = synth.Workload(name="span_boundary", exps=exps, t0=w.t0, elements=w.elements, D=w.D, V=w.V)
    g = gpu_run(w2)
    ctx, patch, orb, _, _ = g["_keep"]
    ctx.count_work(True)
    snr, flux, nv = dt.stack(patch, orb)
    wk = ctx.work()
    ctx.count_work(False)
    np.testing.assert_array_equal(nv.cpu().numpy(), g["nv"])
    # every wavefront that walks to the end takes exactly the three checkpoints
    # (live lanes only are counted; a deferring wavefront stops early)
    sw = wk["switched_waves"]
    assert 3 * (orb.n - 64 * sw) <= wk["checkpoint_solves"] <= 3 * orb.n
    if sw == 0:
        assert wk["checkpoint_solves"] == 3 * orb.n
    snr_o, _, nv_o = oracle.stack(w2.elements, w2.t0, exps, w2.D, w2.V)
    np.testing.assert_array_equal(g["nv"], nv_o)
    ok = snr_close(g["snr"], snr_o)
    assert ok.all(), f"{(~ok).sum()} orbits outside tolerance"
