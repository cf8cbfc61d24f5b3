"""Benchmark of the plain stack on one MI355X.

A step is one pass of the whole hot path over a workload resident in HBM:
the matched-filter pre-pass over every exposure, the fused stack (propagate
-> project -> gather -> accumulate) of every orbit over every exposure, and
the top-k detection.  The metric is dense orbit x exposure samples per
second.  The headline workload is the distant-object set (400 FP16 4096^2
images plus variance over 365 days, 10^9 candidate orbits at 30-60 AU
generated on the device inside the stack); the survey set (200 FP32 2048^2
images, 10^7 stored orbits), the batched patches and the learned proposer
are measured in blocks of the same line.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload distant|survey|tiny]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 operations of the stack kernel's path as written (an FMA counts 2;
# add / mul / hardware reciprocal or rsqrt estimate 1).  Every dense sample:
# the prediction p = r + D (v + D h) - obs 15 and the sky-cone test of it 22
# (axis projection 5, squared distance 5, bound 6, widened radius 2, test 4).
# Every exact solve (each orbit at each checkpoint, and each sample that lands
# in an image; samples that are solved but miss are not counted): mean anomaly
# 5, warm Kepler step 39 (2nd-order start 7, short rotation 20, Newton step
# with a tiny rotation 12), position and distance 25, velocity and light-time
# correction 23, corrected position 6, light time 1, projection with one-
# refinement reciprocal 24, rounding 2.
FLOPS_PER_SAMPLE = 37
FLOPS_PER_SOLVE = 125
# A wavefront whose samples land often leaves the prediction for the
# per-sample walk: per sample 82 (mean anomaly with the predicted light time
# 5, warm Kepler step 39, position and raw distance 20, light-time estimate 2,
# sky-cone test 13, light-time history 3), plus 60 for each sample that takes
# the full path (light-time correction 23, corrected position 6, projection
# 24, rounding 2, light time 5).
FLOPS_PER_TAIL_SAMPLE = 82
FLOPS_PER_TAIL_FULL = 60
CK_SPAN_DAYS = 12.0  # the kernel's checkpoint span (epoch days, CK_SPAN in the library)
# HBM bytes of one full-size stack launch per workload from the committed
# FETCH_SIZE / WRITE_SIZE passes; reported only while the kernel's sources
# are the ones those counters were taken on.
TRAFFIC_RECORDS = {"survey": os.path.join(ROOT, "profiles", "k_stack_track_survey_traffic.json"),
                   "distant": os.path.join(ROOT, "profiles", "k_stack_generated_track_distant_traffic.json")}
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def checkpoints(exps):
    """Checkpoints of one orbit's walk: the first exposure in epoch order and
    every exposure more than CK_SPAN_DAYS after the last checkpoint."""
    n, tc = 0, None
    for t in sorted(x["t"] for x in exps):
        if tc is None or t - tc > CK_SPAN_DAYS:
            n, tc = n + 1, t
    return n


def stack_traffic(workload_name):
    import hashlib
    import json as _json
    path = TRAFFIC_RECORDS.get(workload_name)
    if path is None or not os.path.exists(path):
        return None
    rec = _json.load(open(path))
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update((hashlib.sha256(open(os.path.join(ROOT, f), "rb").read()).hexdigest() + "  " + f + "\n").encode())
    return float(rec["traffic_bytes"]) if h.hexdigest() == rec["sources_sha256"] else None


def workload(name, device):
    import synth
    g = synth.load_geometry(name)
    t = time.time()
    w = synth.build_workload(g, device=device)
    log(f"workload {name}: {len(w.exps)} exposures, {w.elements.shape[0]} orbits ({time.time() - t:.1f} s)")
    return w


def cpu_baseline(w, gpu_snr, seconds=12.0):
    """The oracle on a bounded random sample of the same workload's orbits."""
    import oracle
    D = [d.cpu().numpy() if hasattr(d, "cpu") else d for d in w.D]
    V = [v.cpu().numpy() if hasattr(v, "cpu") else v for v in w.V]
    nth = oracle.max_threads()
    rng = np.random.default_rng(123)
    n_tot = w.elements.shape[0]
    m = 500
    ids = rng.choice(n_tot, m, replace=False)
    t = time.time()
    oracle.stack(w.elements[ids], w.t0, w.exps, D, V)
    dt = max(time.time() - t, 1e-3)
    m2 = int(min(n_tot, max(m, m * seconds / dt)))
    ids = np.sort(rng.choice(n_tot, m2, replace=False))
    t = time.time()
    snr, _, _ = oracle.stack(w.elements[ids], w.t0, w.exps, D, V)
    dt = time.time() - t
    samples = m2 * len(w.exps)
    err = np.abs(gpu_snr[ids] - snr) / np.maximum(1.0, np.abs(snr))
    return dict(value=samples / dt, unit="samples/s", cores=nth, kind="oracle",
                sample=f"{m2} random orbits x {len(w.exps)} exposures ({samples:.3g} samples, {dt:.1f} s)",
                snr_max_err=float(err.max()), snr_p99_err=float(np.percentile(err, 99)))


def bench_next_rows(ctx, patch, orb, w, snr, dev, reps=3):
    """The follow-on rows on the survey workload: per-image iterated-MAD noise,
    on-device orbit generation and generate-and-stack, outlier trimming of
    the top candidates."""
    import torch
    import paper_2503_08854_amd as dt

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    res = {}
    # f-2: iterated MAD over the 200 flux images (one full read per digit pass)
    out = {}
    t_noise = timed(lambda: out.update(r=dt.image_noise(ctx, w.D)))
    sig, used, it = (x.cpu().numpy() for x in out["r"])
    npix = np.array([x.numel() for x in w.D], dtype=np.float64)
    # count pass + first median digit, then per step two median digits, three
    # deviation digits (the third also compacts the last digits' keys) and the clip
    passes = 2 + 6 * it.astype(np.float64)
    nbytes = float((passes * npix * 4).sum())
    res["noise"] = dict(images=len(w.D), ms=t_noise, steps_mean=float(it.mean()), steps_max=int(it.max()),
                        sigma_mean=float(sig.mean()), bytes_read=nbytes,
                        achieved_GBs=nbytes / (t_noise * 1e-3) / 1e9, peak_GBs=HBM_PEAK_GBS)
    # f-4: candidate orbits sampled on the device, then stacked without element arrays
    gf = w.geom["grid_field"]
    gr = w.geom["grid"]
    S = dt.orbit_sampler(gf, gf["t"], gr["a"], gr["e"], gr["inc_deg"], seed=99)
    n = orb.n
    holder = {}
    t_gen = timed(lambda: holder.update(el=dt.generate_orbits(ctx, S, 0, n)))
    gen_set = dt.OrbitSet(holder["el"], gf["t"], dev)
    o2 = dt.batch_outputs([gen_set])[0]
    t_stack = timed(lambda: dt.stack(patch, gen_set, o2))
    t_fused = timed(lambda: holder.update(g=dt.stack_generated(patch, S, 0, n)))
    same = bool(torch.equal(holder["g"][2], o2[2]))
    res["generation"] = dict(orbits=n, generate_ms=t_gen, orbits_per_s=n / (t_gen * 1e-3), stack_ms=t_stack,
                             generate_and_stack_ms=t_fused,
                             generate_and_stack_samples_per_s=n * patch.n_exp / (t_fused * 1e-3),
                             element_bytes_not_moved=48.0 * n, nvalid_equal=same)
    del holder, gen_set, o2
    # f-1: outlier trimming of the 100 best candidates
    ids = torch.as_tensor(np.argsort(-np.nan_to_num(snr, nan=-np.inf))[:100].copy(), device=dev)
    t_clip = timed(lambda: dt.clip_candidates(patch, orb, ids))
    res["outlier_trimming"] = dict(candidates=100, ms=t_clip)
    return res


def bench_batched(dev, steps=5, check=True, per_patch=200):
    """The batched-patches workload: 64 uneven FP16 patches, one graph-captured
    persistent launch (stack + per-patch top-k) after autotuning.  With
    check, the oracle recomputes per_patch random orbits of every patch and
    its injection on the same FP16 values (while the images are still
    resident), and the S/N error of the batched launch is reported."""
    import tempfile
    import torch
    import oracle
    import paper_2503_08854_amd as dt
    import synth
    geom = synth.load_geometry("batched")
    ctx = dt.Context(0)
    patches, sets, checks = [], [], []
    t = time.time()
    n_px = 0
    t_or = 0.0
    for pi, pg in enumerate(geom["patches"]):
        w = synth.build_workload(pg, device=dev)
        p = dt.Patch(ctx, w.exps, w.D, w.V)
        torch.cuda.synchronize()
        if check:
            rng = np.random.default_rng(1000 + pi)
            n_o = w.elements.shape[0]
            ids = np.unique(np.r_[rng.choice(n_o, min(per_patch, n_o), replace=False), w.inj_index])
            D = [d.cpu().numpy() for d in w.D]
            V = [v.cpu().numpy() for v in w.V]
            t1 = time.time()
            so, _, nvo = oracle.stack(w.elements[ids], w.t0, w.exps, D, V)
            t_or += time.time() - t1
            checks.append((ids, so, nvo))
            del D, V
        p.release_images()           # planes stay; the FP16 images are freed
        n_px += sum(x["width"] * x["height"] for x in w.exps)
        patches.append(p)
        sets.append(dt.OrbitSet(w.elements, w.t0, dev))
        del w
    torch.cuda.synchronize()
    log(f"batched: {len(patches)} patches built ({time.time() - t:.1f} s, oracle {t_or:.1f} s)")
    outs = dt.batch_outputs(sets)
    with tempfile.TemporaryDirectory() as td:
        cfg, ms = dt.autotune_batched(ctx, patches, sets, outs, cache_path=os.path.join(td, "tune.txt"))
    log(f"batched: autotuned chunk={cfg[0]} wg_per_cu={cfg[1]} ({ms:.2f} ms)")
    outs, tk = dt.stack_batched(ctx, patches, sets, outs=outs, k=10, threshold=5.0, cfg=cfg)  # capture
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        dt.stack_batched(ctx, patches, sets, outs=outs, k=10, threshold=5.0, cfg=cfg, topk_out=tk)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    samples = sum(o.n * p.n_exp for o, p in zip(sets, patches))
    # the same orbits as 64 single-patch stacks (one dt_stack per patch), to
    # separate the cost of this patch mix from that of the persistent launch
    single = []
    for _ in range(3):
        e0.record()
        for p, o, out in zip(patches, sets, outs):
            dt.stack(p, o, out)
        e1.record()
        torch.cuda.synchronize()
        single.append(e0.elapsed_time(e1))
    # one more (eager) launch with the walk's work counters, per dense sample
    work, flops = counted_work(ctx, lambda: dt.stack_batched(ctx, patches, sets, outs=outs, k=10, threshold=5.0,
                                                             cfg=cfg, eager=True, topk_out=tk))
    res = dict(workload=f"batched: {len(patches)} patches, {sum(p.n_exp for p in patches)} FP16 exposures, "
                        f"{sum(o.n for o in sets)} orbits", samples=samples, ms_per_step=ms_step,
               samples_per_s=samples / (ms_step * 1e-3), cfg={"chunk": cfg[0], "wg_per_cu": cfg[1]}, pixels=n_px,
               work=work, work_per_sample={k: v / samples for k, v in work.items()}, fp64_flops=flops,
               orbits=sum(o.n for o in sets), single_patch_stacks_ms=float(np.median(single)))
    if check:
        g_all, o_all, nv_diff = [], [], 0
        for (ids, so, nvo), o in zip(checks, outs):
            sel = torch.as_tensor(ids, device=dev)
            g_all.append(o[0][sel].cpu().numpy())
            o_all.append(so)
            nv_diff += int((o[2][sel].cpu().numpy() != nvo).sum())
        res["snr_error_vs_oracle"] = dict(snr_errors(np.concatenate(g_all), np.concatenate(o_all)),
                                          nvalid_differences=nv_diff, images="the same FP16 values",
                                          sample=f"{per_patch} random orbits and the injection of every patch")
        log(f"batched: S/N error vs oracle max {res['snr_error_vs_oracle']['max']:.3g}, "
            f"p99 {res['snr_error_vs_oracle']['p99']:.3g}, n_valid differences {nv_diff}")
    for p in patches:
        p.close()
    ctx.close()
    return res


LEARNED_RADIUS = 0.35     # member window around the stamp peak (lattice units)
LEARNED_PREFILTER = 0.2   # fraction of cells (largest stamp maximum) the scorer sees
TIME_CURVE = (0.005, 0.01, 0.02, 0.03, 0.05, 0.08, 0.12, 0.2, 0.3)  # budgets timed for the equal-time comparison (top-k takes at most 4096 cells)


def bench_learned(dev, n_train=100, n_eval=50, budgets=(0.01, 0.02, 0.05), n_eval_side=20, radius=LEARNED_RADIUS,
                  prefilter=LEARNED_PREFILTER, setup="learned", coarse_to_fine=True):
    """Learned vs plain recall at S/N >= 5 and speedup on a cell-structured
    grid (the survey exposures, or with setup="distant_cells" the distant-
    object exposures), on two populations: the injections alone ("clean")
    and with single-exposure point artifacts in every image ("artifacts",
    where the stamp maximum alone no longer ranks cells).  One scorer,
    trained on method-generated stacks with artifacts.  Coarse-max is
    evaluated at the same budget and at equal time: at the budget whose pass
    takes as long as the learned pass (interpolated in a timed budget
    curve); coarse-to-fine when its widened-PSF patch is built."""
    import torch
    import learned_eval as le
    import paper_2503_08854_amd as dt
    t = time.time()
    s = le.load_setup(setup)
    ctx = dt.Context(0)
    b = le.Bench(s, ctx, dev, coarse_to_fine=coarse_to_fine)
    X, F, Y = le.training_set(b, n_train, seed=1, artifacts=le.ARTIFACTS)
    torch.cuda.synchronize()
    log(f"learned: {X.shape[0]} method-generated stacks with artifacts ({time.time() - t:.1f} s)")
    t = time.time()
    sc, hist = le.train_scorer(ctx, X, F, Y, epochs=2, batch=512, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.time() - t
    log(f"learned: trained in {t_train:.1f} s, loss {hist[0][1]:.3f} -> {hist[-1][1]:.3f}")
    del X, F, Y
    keys = ("budget_frac", "injections", "plain_found", "recall_ratio_learned", "recall_ratio_coarse",
            "recall_ratio_coarse_to_fine", "t_plain_ms", "t_learned_ms", "t_coarse_ms", "speedup", "speedup_coarse",
            "coarse_equal_time_budget_frac", "recall_ratio_coarse_equal_time", "t_coarse_equal_time_ms")
    res = dict(setup=f"{setup}: {s.n_cells} cells x {s.cell_size} orbits on {len(s.exps)} exposures "
                     f"({s.geom.get('dtype', 'f32')})", train_stacks=n_train * s.n_cells, train_s=t_train,
               loss_first=hist[0][1], loss_last=hist[-1][1],
               artifacts={"per_image": le.ARTIFACTS[0], "snr": list(le.ARTIFACTS[1])}, radius=radius,
               prefilter=prefilter, coarse_to_fine_subs=b.sub_k * b.sub_k if coarse_to_fine else None)
    for pop, art in (("clean", None), ("artifacts", le.ARTIFACTS)):
        curve = le.pass_times(b, sc, TIME_CURVE, radius=radius, prefilter=prefilter, artifacts=art)
        res[f"time_curve_{pop}"] = dict(budget_frac=list(TIME_CURVE), learned_ms=curve["learned"],
                                        coarse_ms=curve["coarse"])
        rows = []
        for bud in budgets:
            t_l = float(np.interp(bud, TIME_CURVE, curve["learned"]))
            b_eq = le.equal_time_budget(t_l, TIME_CURVE, curve["coarse"])
            r = le.evaluate(b, sc, budget_frac=bud, n_real=n_eval if bud == 0.02 else n_eval_side, artifacts=art,
                            radius=radius, prefilter=prefilter, coarse_equal_time_frac=b_eq)
            rows.append({k: r[k] for k in keys})
            c2f = r['recall_ratio_coarse_to_fine']
            log(f"{setup} {pop} {bud:.0%}: recall ratio learned {r['recall_ratio_learned']:.3f} coarse "
                f"{r['recall_ratio_coarse']:.3f} (equal time, {b_eq:.1%}: {r['recall_ratio_coarse_equal_time']:.3f}) "
                f"c2f {'-' if c2f is None else f'{c2f:.3f}'}; speedup {r['speedup']:.1f}x "
                f"(coarse {r['speedup_coarse']:.1f}x)")
        res[pop] = rows
    # headline fields: both populations at a 2 % budget
    h = next(r for r in res["artifacts"] if r["budget_frac"] == 0.02)
    c = next(r for r in res["clean"] if r["budget_frac"] == 0.02)
    res.update(budget_frac=0.02, recall_ratio_learned=h["recall_ratio_learned"],
               recall_ratio_coarse=h["recall_ratio_coarse"],
               recall_ratio_coarse_equal_time=h["recall_ratio_coarse_equal_time"], speedup=h["speedup"],
               population="artifacts", clean_recall_ratio_learned=c["recall_ratio_learned"],
               clean_speedup=c["speedup"])
    sc.close()
    b.close()
    ctx.close()
    return res


def bench_learned_distant(dev):
    """The learned proposer against the plain stack on the distant-object
    exposures (400 FP16 4096^2 images, 365 days): 10^4 cells x 10^3 orbits,
    scorer trained on 30 realizations, 20 (2 %) or 10 evaluation
    realizations; member window 0.5 (0.35 lost 2 % of the recall here, 0.5
    about 0.5 %); no coarse-to-fine (its widened-PSF patch would add 54 GB of
    planes)."""
    return bench_learned(dev, n_train=30, n_eval=20, n_eval_side=10, setup="distant_cells", coarse_to_fine=False,
                         radius=0.5)


def timed_steps(step, steps, warmup, n_ev):
    """warmup untimed steps, then `steps` timed ones bracketed by synchronisations;
    every step records n_ev events (phase boundaries) on the current stream."""
    import torch
    for i in range(warmup):
        step(None)
        log(f"warmup {i + 1}/{warmup}")
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(n_ev)] for _ in range(steps)]
    t0 = time.perf_counter()
    res = None
    for i in range(steps):
        res = step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = [float(np.mean([e[j].elapsed_time(e[j + 1]) for e in evs])) for j in range(n_ev - 1)]
    return wall, phases, res


def counted_work(ctx, launch):
    """Run one more launch with the kernel's work counters on; returns the
    counts and the FP64 flops they imply."""
    import torch
    ctx.count_work(True)
    launch()
    w = ctx.work()
    ctx.count_work(False)
    torch.cuda.synchronize()
    flops = (FLOPS_PER_SAMPLE * w["predicted"] + FLOPS_PER_SOLVE * (w["queued_solves"] + w["checkpoint_solves"])
             + FLOPS_PER_TAIL_SAMPLE * w["tail_samples"] + FLOPS_PER_TAIL_FULL * w["tail_full"])
    return w, flops


def roofline_block(kernel, ms, n_orbits, n_exp, valid, flops, stored, traffic):
    """Both rooflines of the dominant launch.  HBM: algorithmic bytes = 8 B per
    valid sample (the psi, phi gather) + 12 B of outputs per orbit + 48 B of
    elements per stored orbit + 224 B per exposure record.  FP64: the
    kernel's own flop count (its work counters).  The binding one is HBM when
    the measured traffic (committed counters, same sources) keeps HBM busier
    than the FP64 units are, else the one whose algorithmic fraction is
    nearer its peak."""
    nbytes = 8.0 * valid + (12.0 + (48.0 if stored else 0.0)) * n_orbits + 224.0 * n_exp
    hbm = dict(bound="hbm", achieved=nbytes / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
               algorithmic_bytes=nbytes, traffic=traffic)
    hbm["frac"] = hbm["achieved"] / HBM_PEAK_GBS
    if traffic is not None:
        hbm["traffic_GBs"] = traffic / (ms * 1e-3) / 1e9
        hbm["traffic_frac"] = hbm["traffic_GBs"] / HBM_PEAK_GBS
    alu = dict(bound="alu", achieved=flops / (ms * 1e-3) / 1e12, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
               algorithmic_flops=flops)
    alu["frac"] = alu["achieved"] / FP64_PEAK_TFLOPS
    hbm_busy = hbm.get("traffic_frac", hbm["frac"])
    top, other = (hbm, alu) if hbm_busy >= alu["frac"] else (alu, hbm)
    out = dict(top)
    out.setdefault("traffic", traffic)
    out.update(kernel=kernel, kernel_ms=ms, other=other)
    return out


def snr_errors(gpu, ora):
    err = np.abs(np.asarray(gpu, np.float64) - ora) / np.maximum(1.0, np.abs(ora))
    return dict(max=float(err.max()), p99=float(np.percentile(err, 99)), n=int(err.size))


def oracle_generated(gs, ids):
    """Elements of grid orbits `ids` from the oracle's own generator."""
    import math
    from oracle import generate as G
    f = gs["field"]
    So = dict(center=f["center"], east=f["east"], north=f["north"], obs=f["obs"], half_w=f["half_w"],
              half_h=f["half_h"], a=tuple(gs["a"]), e=tuple(gs["e"]),
              inc=tuple(math.radians(v) for v in gs["inc_deg"]), seed=int(gs["seed"]), epoch=gs["epoch"])
    return np.array([G.sample_orbit(So, int(j)) for j in ids], dtype=np.float64)


def bench_distant(args, dev):
    """Headline: the distant-object workload, orbits generated inside the stack."""
    import torch
    import synth
    import oracle
    import paper_2503_08854_amd as dt
    geom = synth.load_geometry("distant")
    gs = synth.grid_sampler(geom)
    t = time.time()
    w = synth.build_workload(geom, device=dev)
    torch.cuda.synchronize()
    log(f"workload distant: {len(w.exps)} exposures 4096^2 FP16, {gs['n']} generated orbits ({time.time() - t:.1f} s)")
    ctx = dt.Context(0)
    patch = dt.Patch(ctx, w.exps, w.D, w.V)
    S = dt.orbit_sampler(gs["field"], gs["epoch"], gs["a"], gs["e"], gs["inc_deg"], gs["seed"])
    n, ne = gs["n"], patch.n_exp
    out = (torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
           torch.empty(n, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()

    def step(ev):
        if ev is not None:
            ev[0].record()
        patch.refresh()
        if ev is not None:
            ev[1].record()
        dt.stack_generated(patch, S, 0, n, out)
        if ev is not None:
            ev[2].record()
        r = dt.topk(ctx, out[0], args.k, 5.0)
        if ev is not None:
            ev[3].record()
        return r

    steps = args.steps if args.steps is not None else 5
    warmup = args.warmup if args.warmup is not None else 1
    wall, (pre, stk, tk), res = timed_steps(step, steps, warmup, 4)
    log(f"timed {steps} steps: {wall:.3f} s; prepass {pre:.3f} ms, stack {stk:.3f} ms, topk {tk:.3f} ms")
    samples = n * ne
    nv = out[2]
    valid = int(nv.clamp(min=0).sum(dtype=torch.int64))
    work, flops = counted_work(ctx, lambda: dt.stack_generated(patch, S, 0, n, out))
    idx, val, cnt = (x.cpu().numpy() for x in res)
    inj = w.inj_index
    inj_snr = out[0][torch.as_tensor(inj, device=dev)].cpu().numpy()
    rec = {
        "metric": "orbit x exposure samples/s",
        "value": samples * steps / wall,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"distant: {ne} exposures 4096x4096 f16 + variance over 365 days, "
                               f"{n} candidate orbits (a 30-60 AU) generated in the stack, top-{args.k} at S/N>=5",
                   "orbits": n, "exposures": ne, "valid_samples": valid, "valid_frac": valid / samples,
                   "phase_ms": {"prepass": pre, "stack": stk, "topk": tk}},
        "roofline": roofline_block("k_stack_generated_track + k_stack_generated_deferred + k_stack_generated_walk",
                                   stk, n, ne, valid,
                                   flops, False, stack_traffic("distant")),
        "work": work,
        "detections": int(cnt[0]),
        "injections": {"n": int(len(inj)), "recovered_snr5": int((inj_snr >= 5).sum())},
    }
    r = rec["roofline"]
    log(f"roofline: {r['bound']} {r['frac']:.3f} ({r['achieved']:.3g} {r['unit']}); "
        f"{r['other']['bound']} {r['other']['frac']:.3f}")
    if not args.no_cpu:
        D = [d.cpu().numpy() for d in w.D]
        V = [v.cpu().numpy() for v in w.V]
        rng = np.random.default_rng(123)
        # the oracle on a bounded random sample: first a probe to size it to ~12 s
        ids = np.sort(rng.choice(n, 300, replace=False))
        el = oracle_generated(gs, ids)
        t = time.time()
        oracle.stack(el, w.t0, w.exps, D, V)
        dt_probe = max(time.time() - t, 1e-3)
        m = int(min(200000, max(300, 300 * 12.0 / dt_probe)))
        ids = np.unique(np.r_[np.sort(rng.choice(n, m, replace=False)), inj, idx[:int(cnt[0])]])
        el = oracle_generated(gs, ids)
        t = time.time()
        so, fo, nvo = oracle.stack(el, w.t0, w.exps, D, V)
        dt_o = time.time() - t
        sel = torch.as_tensor(ids, device=dev)
        g_snr, g_nv = out[0][sel].cpu().numpy(), nv[sel].cpu().numpy()
        rec["cpu_baseline"] = dict(value=ids.size * ne / dt_o, unit="samples/s", cores=oracle.max_threads(),
                                   kind="oracle",
                                   sample=f"{ids.size} orbits (random, the injections and the top-{args.k}) x {ne} "
                                          f"exposures ({ids.size * ne:.3g} samples, {dt_o:.1f} s)")
        rec["snr_error_vs_oracle"] = dict(snr_errors(g_snr, so), nvalid_differences=int((g_nv != nvo).sum()),
                                          images="the same FP16 values")
        log(f"cpu baseline: {rec['cpu_baseline']['value']:.3g} samples/s on {rec['cpu_baseline']['cores']} threads; "
            f"S/N error max {rec['snr_error_vs_oracle']['max']:.3g}")
        rec["fp16_storage_error"] = fp16_storage_error(geom, w, gs, D, V, ids[:2000], so[:2000], dev)
        del D, V
    if not args.skip_gather:
        rec["gather"] = dict(distant=gather_yardstick_generated(patch, S, gs, dev))
    patch.close()
    ctx.close()
    del w, out, patch
    torch.cuda.empty_cache()
    return rec


def fp16_storage_error(geom, w, gs, D16, V16, ids, snr16, dev):
    """S/N of the oracle on the FP16-stored images vs on the FP32 values they
    were rounded from (same seeds), for a sample of orbits."""
    import torch
    import synth
    import oracle
    g32 = dict(geom)
    g32["dtype"] = "f32"
    w32 = synth.build_workload(g32, device=dev)
    D32 = [d.cpu().numpy() for d in w32.D]
    V32 = [v.cpu().numpy() for v in w32.V]
    del w32
    torch.cuda.empty_cache()
    el = oracle_generated(gs, ids)
    s32, _, _ = oracle.stack(el, w.t0, w.exps, D32, V32)
    del D32, V32
    e = snr_errors(snr16, s32)
    log(f"FP16 storage: S/N error vs the FP32 values max {e['max']:.3g}, p99 {e['p99']:.3g}")
    return e


def gather_yardstick_generated(patch, S, gs, dev, m=10_000_000):
    """Achievable gather rate of the generated stack's own valid gathers
    (first m orbits): the stack of those orbits vs a replay of exactly their
    gathers without the orbit arithmetic."""
    import torch
    import paper_2503_08854_amd as dt
    ctx = patch.ctx
    el = dt.generate_orbits(ctx, S, 0, m)
    sub = dt.OrbitSet(el, gs["epoch"], dev)
    del el
    return _yardstick(patch, sub, lambda o: dt.stack_generated(patch, S, 0, m, o), dev)


def _yardstick(patch, sub, stack_fn, dev, reps=3):
    import torch
    import paper_2503_08854_amd as dt
    m = sub.n
    rec = dt.record_valid_gathers(patch, sub)
    out = dt.batch_outputs([sub])[0]
    snr_r = torch.empty(m, dtype=torch.float32, device=dev)
    stack_fn(out)
    dt.replay_valid_gathers(patch, rec, snr_r)
    torch.cuda.synchronize()
    same = bool(torch.equal(torch.where(out[2] > 0, out[0], torch.zeros_like(out[0])), snr_r))

    def timed(fn):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    t_stack = timed(lambda: stack_fn(out))
    t_rep = timed(lambda: dt.replay_valid_gathers(patch, rec, snr_r))
    valid = int(rec.count)
    useful = 8.0 * valid
    res = dict(orbits=m, valid_samples=valid, dense_samples=m * patch.n_exp, stack_ms=t_stack, replay_ms=t_rep,
               stack_useful_GBs=useful / (t_stack * 1e-3) / 1e9, replay_useful_GBs=useful / (t_rep * 1e-3) / 1e9,
               replay_index_bytes_read_max=8.0 * (valid + 7 * m), frac_of_achievable_gather=t_rep / t_stack,
               replay_equals_stack=same)
    log(f"gather yardstick: stack {t_stack:.3f} ms vs replay {t_rep:.3f} ms on {m} orbits, {valid} valid gathers "
        f"({t_rep / t_stack:.2f} of the achievable gather rate)")
    del rec, out, snr_r
    return res


def bench_survey(args, dev, name="survey", steps=10, warmup=2, with_next=True, with_gather=True):
    """The survey workload (stored orbits): pre-pass + stack + top-k per step."""
    import torch
    import paper_2503_08854_amd as dt
    w = workload(name, dev)
    ctx = dt.Context(0)
    patch = dt.Patch(ctx, w.exps, w.D, w.V)
    orb = dt.OrbitSet(w.elements, w.t0, dev)
    n, ne = orb.n, patch.n_exp
    out = (torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
           torch.empty(n, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()

    def step(ev):
        if ev is not None:
            ev[0].record()
        patch.refresh()
        if ev is not None:
            ev[1].record()
        dt.stack(patch, orb, out)
        if ev is not None:
            ev[2].record()
        r = dt.topk(ctx, out[0], args.k, 5.0)
        if ev is not None:
            ev[3].record()
        return r

    wall, (pre, stk, tk), res = timed_steps(step, steps, warmup, 4)
    log(f"{name}: {steps} steps {wall:.3f} s; prepass {pre:.3f} ms, stack {stk:.3f} ms, topk {tk:.3f} ms")
    samples = n * ne
    snr = out[0].cpu().numpy()
    nv = out[2].cpu().numpy()
    idx, val, cnt = (x.cpu().numpy() for x in res)
    valid = int(nv[nv > 0].sum())
    work, flops = counted_work(ctx, lambda: dt.stack(patch, orb, out))
    rec = dict(workload=f"{name}: {ne} exposures {w.exps[0]['width']}x{w.exps[0]['height']} {w.dtype} + variance, "
                        f"{n} stored orbits, top-{args.k} at S/N>=5",
               value=samples * steps / wall, unit="samples/s", steps=steps, warmup=warmup,
               ms_per_step=wall / steps * 1e3, orbits=n, exposures=ne, valid_samples=valid,
               phase_ms={"prepass": pre, "stack": stk, "topk": tk},
               roofline=roofline_block("k_stack_track + k_stack_deferred", stk, n, ne, valid, flops, True,
                                       stack_traffic(name)),
               work=work, detections=int(cnt[0]))
    inj = w.inj_index
    if len(inj):
        rec["injections"] = {"n": int(len(inj)), "recovered_snr5": int((snr[inj] >= 5).sum())}
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(w, snr)
        rec["snr_error_vs_oracle"] = dict(max=cb.pop("snr_max_err"), p99=cb.pop("snr_p99_err"))
        rec["cpu_baseline"] = cb
    if with_next and not args.skip_next:
        rec["next_rows"] = bench_next_rows(ctx, patch, orb, w, snr, dev)
        N = rec["next_rows"]
        log(f"next rows: noise {N['noise']['ms']:.2f} ms ({N['noise']['achieved_GBs']:.0f} GB/s), generation "
            f"{N['generation']['orbits_per_s']:.3g} orbits/s, generate+stack {N['generation']['generate_and_stack_ms']:.2f} "
            f"ms vs stack {N['generation']['stack_ms']:.2f} ms, trimming {N['outlier_trimming']['ms']:.3f} ms")
    if with_gather and not args.skip_gather:
        rec["gather"] = _yardstick(patch, orb, lambda o: dt.stack(patch, orb, o), dev)
    patch.close()
    ctx.close()
    del w, orb, out, patch
    torch.cuda.empty_cache()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="distant", choices=["distant", "survey", "tiny"])
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--probe-copy", action="store_true",
                    help="run one 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--headline-only", action="store_true", help="only the headline workload's block")
    ap.add_argument("--only", choices=["survey", "batched", "learned", "learned_distant"], default=None,
                    help="run only this block (for profiling; prints its JSON)")
    ap.add_argument("--skip-survey", action="store_true")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-learned", action="store_true")
    ap.add_argument("--skip-gather", action="store_true")
    ap.add_argument("--skip-next", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the stack would shard by orbit, "
              f"but no multi-GPU path is implemented", file=sys.stderr)
        sys.exit(2)
    import torch

    dev = torch.device("cuda:0")
    if args.probe_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.only:
        fn = {"survey": lambda: bench_survey(args, dev, steps=args.steps or 10,
                                             warmup=args.warmup if args.warmup is not None else 2),
              "batched": lambda: bench_batched(dev, steps=args.steps or 5, check=not args.no_cpu),
              "learned": lambda: bench_learned(dev),
              "learned_distant": lambda: bench_learned_distant(dev)}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    if args.workload == "distant":
        rec = bench_distant(args, dev)
    else:
        s = bench_survey(args, dev, args.workload, steps=args.steps or 10,
                         warmup=args.warmup if args.warmup is not None else 2)
        rec = {"metric": "orbit x exposure samples/s", "value": s.pop("value"), "unit": "samples/s", "n_gpus": 1,
               "steps": s.pop("steps"), "warmup": s.pop("warmup"), "ms_per_step": s.pop("ms_per_step"),
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic", "config": {"workload": s.pop("workload"), "orbits": s.pop("orbits"),
                                               "exposures": s.pop("exposures"),
                                               "valid_samples": s.pop("valid_samples"),
                                               "phase_ms": s.pop("phase_ms")}}
        rec.update(s)
    if args.headline_only:
        print(json.dumps(rec), flush=True)
        return
    if args.workload == "distant" and not args.skip_survey:
        rec["survey"] = bench_survey(args, dev)
        log(f"survey: {rec['survey']['value']:.3g} samples/s")
    if not args.skip_batched:
        rec["batched"] = bench_batched(dev, check=not args.no_cpu)
        log(f"batched: {rec['batched']['samples_per_s']:.3g} samples/s")
        torch.cuda.empty_cache()
    if not args.skip_learned:
        rec["learned"] = bench_learned(dev)
        L = rec["learned"]
        log(f"learned (artifacts, 2 %): recall ratio {L['recall_ratio_learned']:.3f} (coarse "
            f"{L['recall_ratio_coarse']:.3f}), speedup {L['speedup']:.1f}x")
        torch.cuda.empty_cache()
        rec["learned_distant"] = bench_learned_distant(dev)
        L = rec["learned_distant"]
        log(f"learned on the distant exposures (artifacts, 2 %): recall ratio {L['recall_ratio_learned']:.3f} "
            f"(coarse {L['recall_ratio_coarse']:.3f}), speedup {L['speedup']:.1f}x")
        torch.cuda.empty_cache()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
