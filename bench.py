"""Benchmark of the plain stack on one MI355X.

A step is one pass of the whole hot path over the survey workload resident
in HBM: the matched-filter pre-pass over every exposure, the fused stack
(propagate -> project -> gather -> accumulate) of every orbit over every
exposure, and the top-k detection.  The metric is dense orbit x exposure
samples per second.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload survey|tiny]
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
CK_SPAN_DAYS = 16.0  # the kernel's checkpoint span (epoch days)
# HBM bytes of one full-size stack launch on the survey workload from the
# committed FETCH_SIZE / WRITE_SIZE passes; reported only while the kernel's
# sources are the ones those counters were taken on.
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_stack_track_survey_traffic.json")
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
    if workload_name != "survey" or not os.path.exists(TRAFFIC_RECORD):
        return None
    rec = _json.load(open(TRAFFIC_RECORD))
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
                snr_max_err=float(err.max()))


def gather_yardstick(patch, w, dev, m=None, reps=3):
    """The stack's own gather stream replayed without the orbit arithmetic, on
    the first m orbits (default: all of them, the launch the benchmark times):
    the achievable gather rate of that access pattern."""
    import torch
    import paper_2503_08854_amd as dt
    m = w.elements.shape[0] if m is None else min(m, w.elements.shape[0])
    sub = dt.OrbitSet(w.elements[:m], w.t0, dev)
    off = dt.record_gathers(patch, sub, torch.arange(m, device=dev))
    out = dt.batch_outputs([sub])[0]
    snr_r = torch.empty(m, dtype=torch.float32, device=dev)
    dt.stack(patch, sub, out)
    dt.gather_replay(patch, off, snr_r)
    torch.cuda.synchronize()
    same = bool(torch.equal(torch.where(out[2] >= 0, out[0], torch.zeros_like(out[0])), snr_r))

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

    t_stack = timed(lambda: dt.stack(patch, sub, out))
    t_rep = timed(lambda: dt.gather_replay(patch, off, snr_r))
    valid = int((off != -1).sum())
    useful = 8.0 * valid
    res = dict(orbits=m, valid_samples=valid, dense_samples=m * patch.n_exp, stack_ms=t_stack, replay_ms=t_rep,
               stack_useful_GBs=useful / (t_stack * 1e-3) / 1e9, replay_useful_GBs=useful / (t_rep * 1e-3) / 1e9,
               replay_index_stream_GB=4.0 * m * patch.n_exp / 1e9, frac_of_achievable_gather=t_rep / t_stack,
               replay_equals_stack=same)
    del off, sub, out, snr_r
    return res


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


def bench_batched(dev, steps=5):
    """The batched-patches workload: 64 uneven FP16 patches, one graph-captured
    persistent launch (stack + per-patch top-k) after autotuning."""
    import tempfile
    import torch
    import paper_2503_08854_amd as dt
    import synth
    geom = synth.load_geometry("batched")
    ctx = dt.Context(0)
    patches, sets = [], []
    t = time.time()
    n_px = 0
    for pg in geom["patches"]:
        w = synth.build_workload(pg, device=dev)
        p = dt.Patch(ctx, w.exps, w.D, w.V)
        torch.cuda.synchronize()
        p.release_images()           # planes stay; the FP16 images are freed
        n_px += sum(x["width"] * x["height"] for x in w.exps)
        patches.append(p)
        sets.append(dt.OrbitSet(w.elements, w.t0, dev))
        del w
    torch.cuda.synchronize()
    log(f"batched: {len(patches)} patches built ({time.time() - t:.1f} s)")
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
    res = dict(workload=f"batched: {len(patches)} patches, {sum(p.n_exp for p in patches)} FP16 exposures, "
                        f"{sum(o.n for o in sets)} orbits", samples=samples, ms_per_step=ms_step,
               samples_per_s=samples / (ms_step * 1e-3), cfg={"chunk": cfg[0], "wg_per_cu": cfg[1]}, pixels=n_px)
    for p in patches:
        p.close()
    ctx.close()
    return res


def bench_learned(dev, n_train=100, n_eval=50, budget=0.02, budget_wide=0.05, n_eval_wide=20, budget_tight=0.01):
    """Learned vs plain recall at S/N >= 5 and speedup on the cell-structured survey grid."""
    import torch
    import learned_eval as le
    import paper_2503_08854_amd as dt
    t = time.time()
    s = le.load_setup("learned")
    ctx = dt.Context(0)
    b = le.Bench(s, ctx, dev)
    X, F, Y = le.training_set(b, n_train, seed=1)
    torch.cuda.synchronize()
    log(f"learned: {X.shape[0]} method-generated stacks ({time.time() - t:.1f} s)")
    t = time.time()
    sc, hist = le.train_scorer(ctx, X, F, Y, epochs=2, batch=512, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.time() - t
    log(f"learned: trained in {t_train:.1f} s, loss {hist[0][1]:.3f} -> {hist[-1][1]:.3f}")
    del X, F, Y
    res = le.evaluate(b, sc, budget_frac=budget, n_real=n_eval)
    res.update(train_stacks=n_train * s.n_cells, train_s=t_train, loss_first=hist[0][1], loss_last=hist[-1][1])
    wide = le.evaluate(b, sc, budget_frac=budget_wide, n_real=n_eval_wide)
    keys = ("budget_frac", "injections", "recall_ratio_learned", "recall_ratio_coarse",
            "recall_ratio_coarse_to_fine", "speedup")
    res["wider_budget"] = {k: wide[k] for k in keys}
    tight = le.evaluate(b, sc, budget_frac=budget_tight, n_real=n_eval_wide)
    res["tighter_budget"] = {k: tight[k] for k in keys}
    sc.close()
    b.patch.close()
    b.coarse.close()
    ctx.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="survey")
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--probe-copy", action="store_true",
                    help="run one 1 GiB device copy first (reference for HBM byte counters)")
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
    import paper_2503_08854_amd as dt

    dev = torch.device("cuda:0")
    if args.probe_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    w = workload(args.workload, dev)
    ctx = dt.Context(0)
    patch = dt.Patch(ctx, w.exps, w.D, w.V)
    orb = dt.OrbitSet(w.elements, w.t0, dev)
    n, ne = orb.n, patch.n_exp
    out = (torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float32, device=dev),
           torch.empty(n, dtype=torch.int32, device=dev))
    torch.cuda.synchronize()

    def step(ev=None):
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

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pre = np.mean([e[0].elapsed_time(e[1]) for e in evs])
    stk = np.mean([e[1].elapsed_time(e[2]) for e in evs])
    tk = np.mean([e[2].elapsed_time(e[3]) for e in evs])
    log(f"timed {args.steps} steps: {wall:.3f} s; prepass {pre:.3f} ms, stack {stk:.3f} ms, topk {tk:.3f} ms")
    samples = n * ne
    value = samples * args.steps / wall
    snr = out[0].cpu().numpy()
    nv = out[2].cpu().numpy()
    idx, val, cnt = (x.cpu().numpy() for x in res)
    valid = int(nv[nv > 0].sum())
    n_ck = checkpoints(w.exps)
    achieved = (FLOPS_PER_SAMPLE * samples + FLOPS_PER_SOLVE * (valid + n * n_ck)) / (stk * 1e-3) / 1e12
    rec = {
        "metric": "orbit x exposure samples/s",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {ne} exposures "
                               f"{w.exps[0]['width']}x{w.exps[0]['height']} {w.dtype} + variance, "
                               f"{n} orbits, top-{args.k} at S/N>=5",
                   "orbits": n, "exposures": ne, "valid_samples": valid,
                   "phase_ms": {"prepass": pre, "stack": stk, "topk": tk}},
        "roofline": {"bound": "alu", "kernel": "k_stack_track", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": stack_traffic(args.workload),
                     "flops_per_sample": FLOPS_PER_SAMPLE, "flops_per_solve": FLOPS_PER_SOLVE,
                     "solves": valid + n * n_ck},
        "detections": int(cnt[0]),
    }
    inj = w.inj_index
    if len(inj):
        rec["injections"] = {"n": int(len(inj)), "recovered_snr5": int((snr[inj] >= 5).sum())}
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        rec["cpu_baseline"] = cpu_baseline(w, snr)
        log(f"cpu baseline: {rec['cpu_baseline']['value']:.3g} samples/s on {rec['cpu_baseline']['cores']} threads")
    if not args.skip_next:
        rec["next_rows"] = bench_next_rows(ctx, patch, orb, w, snr, dev)
        N = rec["next_rows"]
        log(f"next rows: noise {N['noise']['ms']:.2f} ms ({N['noise']['achieved_GBs']:.0f} GB/s), generation "
            f"{N['generation']['orbits_per_s']:.3g} orbits/s, generate+stack {N['generation']['generate_and_stack_ms']:.2f} "
            f"ms vs stack {N['generation']['stack_ms']:.2f} ms, trimming {N['outlier_trimming']['ms']:.3f} ms")
    if not args.skip_gather:
        rec["gather"] = gather_yardstick(patch, w, dev)
        G = rec["gather"]
        log(f"gather yardstick: stack {G['stack_ms']:.3f} ms vs replay {G['replay_ms']:.3f} ms on {G['orbits']} "
            f"orbits ({G['frac_of_achievable_gather']:.2f} of the achievable gather rate)")
    patch.close()
    ctx.close()
    del w, orb, out, patch
    torch.cuda.empty_cache()
    if not args.skip_batched:
        rec["batched"] = bench_batched(dev)
        log(f"batched: {rec['batched']['samples_per_s']:.3g} samples/s")
        torch.cuda.empty_cache()
    if not args.skip_learned:
        rec["learned"] = bench_learned(dev)
        L = rec["learned"]
        log(f"learned: recall ratio {L['recall_ratio_learned']:.3f} (coarse {L['recall_ratio_coarse']:.3f}), "
            f"speedup {L['speedup']:.1f}x at a {L['budget_frac']:.0%} budget")
        for key in ("tighter_budget", "wider_budget"):
            T = L[key]
            log(f"learned: recall ratio {T['recall_ratio_learned']:.3f}, speedup {T['speedup']:.1f}x "
                f"at a {T['budget_frac']:.0%} budget")
        torch.cuda.empty_cache()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
