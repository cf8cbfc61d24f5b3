"""Training data, training and evaluation of the learned cell proposer.

Used by bench.py (the learned-vs-plain recall and speedup fields) and by the
GPU tests.  Images and injected sources come from `synth`; every tracking
step (tracks, planes, stamps, scoring, stacking) runs in the HIP library.

Evaluation protocol: a cell-structured grid (representative + perturbed
members per cell) on the survey exposures; per realization, fresh noise and
sources injected on member orbits at the pixel positions the oracle stored.
The exhaustive stack over every orbit is the reference: an injection counts as
found by a method if its own orbit's stacked S/N is >= 5 in that method's
output.  Recall ratio = learned-found / plain-found.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

import synth


C2F_SUB = 3  # coarse-to-fine: sub-representatives per cell side
ARTIFACTS = (100, (20.0, 60.0))  # single-exposure point artifacts per image, per-image S/N range


@dataclass
class Setup:
    geom: dict
    exps: list
    t0: float
    el: np.ndarray
    cell_size: int
    n_cells: int
    da: float
    dm: float


def load_setup(name: str = "learned") -> Setup:
    g = synth.load_geometry(name)
    cg = g["cell_grid"]
    el = synth.cell_grid(g["grid_field"], cg["cells"], cg["cell_size"], cg["seed"], cg["a"], cg["e"], cg["inc_deg"],
                         cg["da"], cg["dm"])
    return Setup(g, synth.exposures_of(g), float(g["t0"]), el, int(cg["cell_size"]), int(cg["cells"]),
                 float(cg["da"]), float(cg["dm"]))


def _sum_p2(fwhm: float) -> float:
    sig = fwhm / (2 * math.sqrt(2 * math.log(2)))
    R = math.ceil(3 * sig)
    y, x = np.mgrid[-R:R + 1, -R:R + 1]
    P = np.exp(-(x * x + y * y) / (2 * sig * sig))
    P /= P.sum()
    return float((P ** 2).sum())


class Bench:
    """Device state for one setup: images (refilled per realization), patch, grids."""

    def __init__(self, s: Setup, ctx, device="cuda", coarse_to_fine=True):
        import paper_2503_08854_amd as dt
        self.s = s
        self.ctx = ctx
        self.dev = device
        self.dtype = s.geom.get("dtype", "f32")
        self.D, self.V = synth.noise_images(s.exps, 1, s.geom.get("nan_frac", 0.0), self.dtype, device)
        self.patch = dt.Patch(ctx, s.exps, self.D, self.V)
        from paper_2503_08854_amd import proposer
        # coarse-to-fine needs a second patch (widened-PSF planes); optional for large image sets
        self.coarse = proposer.coarse_patch(ctx, s.exps, self.D, self.V) if coarse_to_fine else None
        self.grid = dt.OrbitSet(s.el, s.t0, device)
        self.reps = dt.OrbitSet(s.el[::s.cell_size], s.t0, device)
        self.sub_k = C2F_SUB
        self.subs = dt.OrbitSet(proposer.sub_representatives(s.el[::s.cell_size], s.da, s.dm, self.sub_k), s.t0,
                                device)

    def realize(self, seed: int, hits, artifacts=None):
        """Fresh noise (seeded) in place, then sources at hits (e, px, py, flux),
        then, with artifacts = (per_image, (s_lo, s_hi)), single-exposure point
        artifacts of per-image S/N U(s_lo, s_hi) (seeded by the same seed), then
        the pre-pass."""
        D, V = synth.noise_images(self.s.exps, seed, self.s.geom.get("nan_frac", 0.0), self.dtype, self.dev)
        for a, b in zip(self.D, D):
            a.copy_(b)
        for a, b in zip(self.V, V):
            a.copy_(b)
        del D, V
        synth.render_sources_fast(self.D, self.s.exps, hits, self.dev)
        if artifacts:
            art = synth.artifacts(self.s.exps, artifacts[0], artifacts[1], seed)
            sig = np.array([x.get("sigma", 1.0) for x in self.s.exps])[art[:, 0].astype(int)]
            art[:, 3] = art[:, 3] * sig / math.sqrt(_sum_p2(self.s.exps[0]["fwhm"]))
            synth.render_sources_fast(self.D, self.s.exps, art, self.dev)
        self.patch.refresh()
        if self.coarse is not None:
            self.coarse.refresh()

    def close(self):
        self.patch.close()
        if self.coarse is not None:
            self.coarse.close()


def training_set(bench: Bench, n_real: int, seed: int, pos_frac: float = 0.5, snr_rng=(3.0, 10.0), log=None,
                 artifacts=None):
    """Method-generated stacks: per realization, sources on random members of
    pos_frac of the cells (stacked S/N target U(snr_rng) over their hits, the
    tracks from the stack's own debug table), optional single-exposure
    artifacts (see Bench.realize); stamps of every cell; labels 1 for injected
    cells.  Returns device tensors (stamps, feats, labels)."""
    import torch
    import paper_2503_08854_amd as dt
    from paper_2503_08854_amd import proposer
    s = bench.s
    p2 = _sum_p2(s.exps[0]["fwhm"])
    rng = np.random.default_rng(seed)
    S, F, Y = [], [], []
    for r in range(n_real):
        n_pos = int(s.n_cells * pos_frac)
        cells = rng.choice(s.n_cells, n_pos, replace=False)
        members = cells * s.cell_size + rng.integers(1, s.cell_size, n_pos)
        px, py, fl = proposer.member_tracks(bench.patch, bench.grid, members)
        inside = (fl & 2) != 0
        nh = inside.sum(1)
        target = rng.uniform(*snr_rng, n_pos)
        flux = np.where(nh > 0, target / np.sqrt(np.maximum(nh, 1)) / math.sqrt(p2), 0.0)
        ii, ee = np.nonzero(inside)
        hits = np.stack([ee, px[ii, ee], py[ii, ee], flux[ii]], axis=1)
        bench.realize(seed * 7919 + r, hits, artifacts)
        st = dt.cell_stamps(bench.patch, bench.reps, s.da, s.dm, bf16=True, f32=False)
        lab = np.zeros(s.n_cells, np.float32)
        lab[cells[nh > 0]] = 1.0
        S.append(st["stamps_bf16"])
        F.append(st["feats_bf16"])
        Y.append(torch.from_numpy(lab).to(bench.dev))
        if log and (r % 10 == 0 or r == n_real - 1):
            log(f"training realization {r + 1}/{n_real}: {int(lab.sum())} positive cells")
    return torch.cat(S), torch.cat(F), torch.cat(Y)


def train_scorer(ctx, stamps, feats, labels, epochs: int = 2, batch: int = 512, lr: float = 1e-3, seed: int = 0,
                 log=None):
    import paper_2503_08854_amd as dt
    from paper_2503_08854_amd import proposer
    sc = dt.Scorer(ctx, max_batch=max(batch, 16384), seed=seed)
    hist = proposer.train(sc, proposer.minibatches(stamps, feats, labels, batch, epochs, seed), lr=lr, log=log)
    return sc, hist


def _clear(outs):
    """Mark every output as not computed (NaN S/N and flux, -2 valid count)."""
    import torch
    for t in outs:
        t.fill_(float("nan")) if t.dtype == torch.float32 else t.fill_(-2)


def pass_times(bench: Bench, scorer, budgets, radius=None, prefilter=None, artifacts=None, reps: int = 5,
               seed: int = 10_000):
    """Wall time (ms, median of reps after one warm-up) of one learned pass and
    one coarse-max pass at each budget fraction, on one realization."""
    import torch
    import paper_2503_08854_amd as dt
    from paper_2503_08854_amd import proposer
    s = bench.s
    bench.realize(seed, np.zeros((0, 4)), artifacts)
    out = dt.batch_outputs([bench.grid])[0]
    res = {"learned": [], "coarse": []}
    for frac in budgets:
        budget = max(1, int(round(frac * s.n_cells)))
        pre = None if prefilter is None else max(budget, int(prefilter * s.n_cells))
        runs = {
            "learned": lambda: proposer.run_learned(bench.ctx, bench.patch, bench.grid, bench.reps, s.cell_size, s.da,
                                                    s.dm, scorer, budget, out=out, radius=radius, prefilter=pre),
            "coarse": lambda: proposer.run_coarse(bench.ctx, bench.patch, bench.grid, bench.reps, s.cell_size, s.da,
                                                  s.dm, budget, out=out, radius=radius),
        }
        for name, run in runs.items():
            ts = []
            for i in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                run()
                torch.cuda.synchronize()
                if i:
                    ts.append(time.perf_counter() - t0)
            res[name].append(float(np.median(ts)) * 1e3)
    return res


def equal_time_budget(t_ms: float, budgets, coarse_ms) -> float:
    """The coarse-max budget whose pass time equals t_ms, by linear
    interpolation in the measured (budget, time) points (clamped to their
    range)."""
    b = np.asarray(budgets, float)
    t = np.maximum.accumulate(np.asarray(coarse_ms, float))  # time grows with the budget
    if t_ms <= t[0]:
        return float(b[0])
    if t_ms >= t[-1]:
        return float(b[-1])
    return float(np.interp(t_ms, t, b))


def evaluate(bench: Bench, scorer, budget_frac: float = 0.05, n_real: int = None, log=None, artifacts=None,
             radius=None, prefilter=None, coarse_equal_time_frac=None):
    """Recall of plain / learned / coarse-max / coarse-to-fine selection over
    stored realizations (optionally with single-exposure artifacts), and
    timings.  radius: the learned and coarse-max paths stack only the
    selected cells' members within it of the stamp peak; prefilter: the
    fraction of cells (largest stamp maximum) the scorer sees;
    coarse_equal_time_frac: a second coarse-max budget (the one whose pass
    takes as long as the learned pass, see equal_time_budget) evaluated on
    the same realizations."""
    import torch
    import paper_2503_08854_amd as dt
    from paper_2503_08854_amd import proposer
    s = bench.s
    reals = s.geom["realizations"][:n_real] if n_real else s.geom["realizations"]
    budget = max(1, int(round(budget_frac * s.n_cells)))
    n = bench.grid.n
    out_full = dt.batch_outputs([bench.grid])[0]
    out_sel = tuple(torch.empty_like(t) for t in out_full)
    found = dict(plain=0, learned=0, coarse=0, c2f=0, coarse_eq=0)
    tot = 0
    t_plain, t_learn, t_coarse, t_coarse_eq = [], [], [], []
    for r, injs in enumerate(reals):
        hits = np.array([[h[0], h[1], h[2], inj["flux"]] for inj in injs for h in inj["hits"]])
        bench.realize(10_000 + r, hits, artifacts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dt.stack(bench.patch, bench.grid, out_full)
        torch.cuda.synchronize()
        t_plain.append(time.perf_counter() - t0)
        for t in out_sel:
            t.fill_(float("nan")) if t.dtype == torch.float32 else t.fill_(-2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, cells = proposer.run_learned(bench.ctx, bench.patch, bench.grid, bench.reps, s.cell_size, s.da, s.dm,
                                        scorer, budget, out=out_sel, radius=radius,
                                        prefilter=None if prefilter is None else max(budget, int(prefilter * s.n_cells)))
        torch.cuda.synchronize()
        t_learn.append(time.perf_counter() - t0)
        learned_snr = out_sel[0].cpu().numpy()
        for t in out_sel:
            t.fill_(float("nan")) if t.dtype == torch.float32 else t.fill_(-2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        proposer.run_coarse(bench.ctx, bench.patch, bench.grid, bench.reps, s.cell_size, s.da, s.dm, budget,
                            out=out_sel, radius=radius)
        torch.cuda.synchronize()
        t_coarse.append(time.perf_counter() - t0)
        coarse_snr = out_sel[0].cpu().numpy()
        if coarse_equal_time_frac is not None:
            _clear(out_sel)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            proposer.run_coarse(bench.ctx, bench.patch, bench.grid, bench.reps, s.cell_size, s.da, s.dm,
                                max(1, int(round(coarse_equal_time_frac * s.n_cells))), out=out_sel, radius=radius)
            torch.cuda.synchronize()
            t_coarse_eq.append(time.perf_counter() - t0)
            coarse_eq_snr = out_sel[0].cpu().numpy()
        for t in out_sel:
            t.fill_(float("nan")) if t.dtype == torch.float32 else t.fill_(-2)
        if bench.coarse is not None:
            proposer.run_coarse_to_fine(bench.ctx, bench.patch, bench.coarse, bench.grid, bench.subs,
                                        bench.sub_k * bench.sub_k, s.cell_size, budget, out=out_sel)
        c2f_snr = out_sel[0].cpu().numpy()
        plain_snr = out_full[0].cpu().numpy()
        orbits = np.array([inj["orbit"] for inj in injs])
        pf = plain_snr[orbits] >= 5.0
        lf = np.nan_to_num(learned_snr[orbits], nan=-np.inf) >= 5.0
        cf = np.nan_to_num(coarse_snr[orbits], nan=-np.inf) >= 5.0
        c2 = np.nan_to_num(c2f_snr[orbits], nan=-np.inf) >= 5.0
        found["c2f"] += int((c2 & pf).sum())
        found["plain"] += int(pf.sum())
        found["learned"] += int((lf & pf).sum())
        found["coarse"] += int((cf & pf).sum())
        if coarse_equal_time_frac is not None:
            ce = np.nan_to_num(coarse_eq_snr[orbits], nan=-np.inf) >= 5.0
            found["coarse_eq"] += int((ce & pf).sum())
        tot += len(orbits)
    # steady-state timings: drop the first realization (warm-up)
    tp = float(np.median(t_plain[1:] if len(t_plain) > 1 else t_plain))
    tl = float(np.median(t_learn[1:] if len(t_learn) > 1 else t_learn))
    tc = float(np.median(t_coarse[1:] if len(t_coarse) > 1 else t_coarse))
    res = dict(injections=tot, plain_found=found["plain"], learned_found=found["learned"],
               coarse_found=found["coarse"], budget_cells=budget, cells=s.n_cells, budget_frac=budget / s.n_cells,
               recall_plain=found["plain"] / max(tot, 1),
               recall_ratio_learned=found["learned"] / max(found["plain"], 1),
               recall_ratio_coarse=found["coarse"] / max(found["plain"], 1),
               recall_ratio_coarse_to_fine=(found["c2f"] / max(found["plain"], 1)) if bench.coarse is not None
               else None,
               t_plain_ms=tp * 1e3, t_learned_ms=tl * 1e3, t_coarse_ms=tc * 1e3, speedup=tp / tl,
               speedup_coarse=tp / tc, radius=radius, prefilter=prefilter, orbits=n)
    if coarse_equal_time_frac is not None:
        tce = float(np.median(t_coarse_eq[1:] if len(t_coarse_eq) > 1 else t_coarse_eq))
        res.update(coarse_equal_time_budget_frac=coarse_equal_time_frac, t_coarse_equal_time_ms=tce * 1e3,
                   recall_ratio_coarse_equal_time=found["coarse_eq"] / max(found["plain"], 1))
    if log:
        log(f"learned eval: {res}")
    return res


def stage_times(bench: Bench, scorer, budget_frac: float = 0.02, reps: int = 4, radius=None, prefilter=None):
    """Per-stage device times (ms, median over reps after one warm-up) of one
    learned pass on the current images (stamps, scores, selection, stack), its
    wall time, and the exhaustive stack's time."""
    import torch
    import paper_2503_08854_amd as dt
    from paper_2503_08854_amd import proposer
    s = bench.s
    budget = max(1, int(round(budget_frac * s.n_cells)))
    pre = None if prefilter is None else max(budget, int(prefilter * s.n_cells))
    out = dt.batch_outputs([bench.grid])[0]
    rows = []
    for it in range(reps + 1):
        evs = [torch.cuda.Event(enable_timing=True)]

        def mark(stage):
            evs.append(torch.cuda.Event(enable_timing=True))
            evs[-1].record()

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record()
        proposer.run_learned(bench.ctx, bench.patch, bench.grid, bench.reps, s.cell_size, s.da, s.dm, scorer, budget,
                             out=out, radius=radius, prefilter=pre, mark=mark)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dt.stack(bench.patch, bench.grid, out)
        e1.record()
        torch.cuda.synchronize()
        if it:
            rows.append([evs[i].elapsed_time(evs[i + 1]) for i in range(4)] + [wall, e0.elapsed_time(e1)])
    m = np.median(np.array(rows), axis=0)
    return dict(stamps_ms=m[0], scores_ms=m[1], select_ms=m[2], stack_ms=m[3], learned_wall_ms=m[4],
                full_stack_ms=m[5], budget_cells=budget, radius=radius, prefilter=prefilter)


def main():
    """Stage timing of the learned path on the learned workload (a short
    training run first; realization 0's injections in fresh noise)."""
    import argparse
    import paper_2503_08854_amd as dt
    ap = argparse.ArgumentParser()
    ap.add_argument("--setup", default="learned")
    ap.add_argument("--train-realizations", type=int, default=4)
    ap.add_argument("--budget", type=float, default=0.02)
    ap.add_argument("--radius", type=float, default=0.35)
    ap.add_argument("--prefilter", type=float, default=0.2)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    s = load_setup(args.setup)
    ctx = dt.Context(0)
    b = Bench(s, ctx)
    X, F, Y = training_set(b, args.train_realizations, seed=1, artifacts=ARTIFACTS)
    sc, _ = train_scorer(ctx, X, F, Y, epochs=1)
    del X, F, Y
    injs = s.geom["realizations"][0]
    hits = np.array([[h[0], h[1], h[2], inj["flux"]] for inj in injs for h in inj["hits"]])
    b.realize(10_000, hits, ARTIFACTS)
    print(stage_times(b, sc, args.budget, args.reps, args.radius, args.prefilter), flush=True)
    sc.close()
    b.close()
    ctx.close()


if __name__ == "__main__":
    main()
