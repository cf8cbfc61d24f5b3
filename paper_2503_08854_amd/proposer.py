"""Learned proposal over orbit-grid cells (this library's extension).

Pipeline, every numerical step in the library's kernels:
  1. coarse stamps + features of every cell's representative (dt_cell_stamps);
  2. the scorer's logit per cell (fused BF16 MFMA inference kernel), on every
     cell or on the cells of largest stamp maximum only (a pre-filter: a cell
     the maximum ranks low holds no detectable source);
  3. the `budget` best cells by logit (dt_topk on the logits);
  4. the plain stack on the orbits of those cells only (dt_stack_cells), or,
     with a radius, only on the members whose lattice coordinates lie within
     it of the cell's stamp peak (dt_cell_members_near + dt_stack_ids): the
     peak node follows the member whose track carries the source, so the
     fine stack runs around the coarse peak (Sec. 5.2.2).
The exhaustive stack over every orbit stays the fallback and the reference.
Two non-learned counterparts rank cells the same way: by the coarse stamp's
maximum (run_coarse) and by the representatives' S/N on planes smoothed with
a Gaussian wider than the PSF (run_coarse_to_fine).

Training uses stacks the method itself produces: synthetic exposures with
sources injected on member orbits of chosen cells (their pixel tracks from the
stack's own debug table), planes from the pre-pass, and stamps from (1); cells
with an injection are positives, the others negatives.
"""
from __future__ import annotations

import numpy as np

from . import binding as B


def cell_inputs(patch, reps, da: float, dm: float):
    """(stamps BF16 n x 21 x 21, features BF16 n x 16) over each cell's (a, M0) box."""
    out = B.cell_stamps(patch, reps, da, dm, bf16=True, f32=False)
    return out["stamps_bf16"], out["feats_bf16"]


def score_cells(scorer, stamps_bf16, feats_bf16):
    return scorer.infer(stamps_bf16, feats_bf16)


def select_cells(ctx, scores, budget: int):
    """Indices of the `budget` highest scores (ties to the lower index), as a
    set: the stacks that follow do not depend on their order."""
    idx, val, cnt = B.topk(ctx, scores, int(budget), ordered=False)
    return idx


def stack_selected(ctx, patch, grid, cells, cell_size: int, da: float, dm: float, feats_f32, radius, out=None):
    """The plain stack on the selected cells: every member (radius None) or the
    members within `radius` (lattice units) of each cell's stamp peak."""
    if radius is None:
        return B.stack_cells(patch, grid, cells, cell_size, out=out)
    ids, cnt = B.cell_members_near(ctx, grid, cells, cell_size, feats_f32[:, 11:], da, dm, radius)
    return B.stack_ids(patch, grid, ids, cnt, out=out)


def run_learned(ctx, patch, grid, reps, cell_size: int, da: float, dm: float, scorer, budget: int, out=None,
                radius=None, prefilter=None, mark=None):
    """Stamps -> scores -> top cells -> stack on their orbits (all members, or
    those near the stamp peak). With prefilter = m, only the m cells of
    largest stamp maximum are scored (the rest rank last).  mark(stage), if
    given, is called after each stage (for timing).  Returns (outputs,
    selected cell ids)."""
    mark = mark or (lambda stage: None)
    o = B.cell_stamps(patch, reps, da, dm, bf16=True, f32=False,
                      feats_f32=radius is not None or prefilter is not None)
    mark("stamps")
    if prefilter is None:
        z = score_cells(scorer, o["stamps_bf16"], o["feats_bf16"])
    else:
        import torch
        rows = select_cells(ctx, o["feats"][:, 0].contiguous(), prefilter)
        z = torch.full((reps.n,), float("-inf"), dtype=torch.float32, device=rows.device)
        scorer.infer_rows(o["stamps_bf16"], o["feats_bf16"], rows, z)
    mark("scores")
    cells = select_cells(ctx, z, budget)
    mark("select")
    out = stack_selected(ctx, patch, grid, cells, cell_size, da, dm, o["feats"], radius, out=out)
    mark("stack")
    return out, cells


def run_coarse(ctx, patch, grid, reps, cell_size: int, da: float, dm: float, budget: int, out=None, radius=None):
    """The non-learned counterpart: rank cells by the stamp maximum (feature 0)."""
    o = B.cell_stamps(patch, reps, da, dm, bf16=False, f32=False, feats_f32=True)
    cells = select_cells(ctx, o["feats"][:, 0].contiguous(), budget)
    out = stack_selected(ctx, patch, grid, cells, cell_size, da, dm, o["feats"], radius, out=out)
    return out, cells


def coarse_exposures(exps, factor: float, fwhm_max: float = 8.0):
    """Exposure records whose PSF FWHM is widened by `factor` (capped at fwhm_max px)."""
    return [dict(x, fwhm=min(float(x["fwhm"]) * factor, fwhm_max)) for x in exps]


def coarse_patch(ctx, exps, flux, var, factor: float = 2.5):
    """A patch over the same images whose planes use the widened Gaussian (Sec. 5.2.2 smoothing)."""
    return B.Patch(ctx, coarse_exposures(exps, factor), flux, var)


def sub_representatives(rep_elements, da: float, dm: float, k: int = 3):
    """A k x k lattice of orbits per cell around its representative (the
    cell's (a, M0) box cut into k x k squares, one orbit at each centre):
    rows are (cell, v, u) in that order, the elements of the representatives
    with a + u da and M0 + v dm, u, v in {-1 + 1/k, ..., 1 - 1/k}.  A grid
    construction on the host, like the cell grid itself."""
    el = np.asarray(rep_elements, dtype=np.float64)
    off = -1.0 + (2.0 * np.arange(k) + 1.0) / k
    uu, vv = np.meshgrid(off, off)  # [v][u]
    out = np.repeat(el, k * k, axis=0)
    out[:, 0] += np.tile(uu.ravel(), el.shape[0]) * da
    out[:, 5] += np.tile(vv.ravel(), el.shape[0]) * dm
    return out


def run_coarse_to_fine(ctx, patch, coarse, grid, subs, per_cell: int, cell_size: int, budget: int, out=None):
    """Coarse-to-fine (Sec. 5.2.2): a sparse grid -- per_cell sub-representatives
    per cell (sub_representatives) -- stacked on the widened-PSF planes, each
    cell ranked by its best sub-representative, the `budget` best cells, then
    the plain stack on every orbit of those cells.  Returns (outputs, cells,
    coarse cell scores)."""
    snr_c, _, _ = B.stack(coarse, subs)
    score = B.segment_max(ctx, snr_c, per_cell)
    cells = select_cells(ctx, score, budget)
    out = B.stack_cells(patch, grid, cells, cell_size, out=out)
    return out, cells, score


def member_tracks(patch, grid, orbit_ids):
    """Pixel tracks (exposure, px, py) of chosen orbits from the stack's own device code."""
    d = B.debug_samples(patch, grid, orbit_ids)
    px = d["px"].cpu().numpy()
    py = d["py"].cpu().numpy()
    fl = d["flags"].cpu().numpy()
    return px, py, fl


def train(scorer, batches, lr: float = 1e-3, log=None):
    """Run scorer.train_step over an iterable of (stamps, feats, labels); returns the loss history."""
    import torch
    hist = []
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for k, (s, f, y) in enumerate(batches):
        scorer.train_step(s, f, y, lr, loss_out=loss)
        if k % 50 == 0:
            hist.append((k, float(loss.cpu()[0])))
            if log:
                log(f"step {k}: loss {hist[-1][1]:.4f}")
    return hist


def minibatches(stamps, feats, labels, batch: int, epochs: int, seed: int = 0):
    """Shuffled minibatches over device tensors."""
    import torch
    n = stamps.shape[0]
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    for _ in range(epochs):
        perm = torch.randperm(n, generator=g).to(stamps.device)
        for s in range(0, n - batch + 1, batch):
            i = perm[s:s + batch]
            yield stamps[i], feats[i], labels[i]


def recall(snr, inj_orbits, thr: float = 5.0):
    """Fraction of injected orbits whose stacked S/N reaches thr (NaN = not stacked)."""
    v = np.asarray(snr)[np.asarray(inj_orbits, dtype=np.int64)]
    return float(np.mean(np.nan_to_num(v, nan=-np.inf) >= thr)), v
