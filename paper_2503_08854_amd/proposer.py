"""Learned proposal over orbit-grid cells (this library's extension).

Pipeline, every numerical step in the library's kernels:
  1. coarse stamps + features of every cell's representative (dt_cell_stamps);
  2. the scorer's logit per cell (fused BF16 MFMA inference kernel);
  3. the `budget` best cells by logit (dt_topk on the logits);
  4. the plain stack on the orbits of those cells only (dt_stack_cells).
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
    """Indices of the `budget` highest scores (ties to the lower index)."""
    idx, val, cnt = B.topk(ctx, scores, int(budget))
    return idx


def run_learned(ctx, patch, grid, reps, cell_size: int, da: float, dm: float, scorer, budget: int, out=None):
    """Stamps -> scores -> top cells -> stack on their orbits. Returns (outputs, selected cell ids)."""
    st, ft = cell_inputs(patch, reps, da, dm)
    z = score_cells(scorer, st, ft)
    cells = select_cells(ctx, z, budget)
    out = B.stack_cells(patch, grid, cells, cell_size, out=out)
    return out, cells


def run_coarse(ctx, patch, grid, reps, cell_size: int, da: float, dm: float, budget: int, out=None):
    """The non-learned counterpart: rank cells by the stamp maximum (feature 0)."""
    o = B.cell_stamps(patch, reps, da, dm, bf16=False, f32=True)
    cells = select_cells(ctx, o["feats"][:, 0].contiguous(), budget)
    out = B.stack_cells(patch, grid, cells, cell_size, out=out)
    return out, cells


def coarse_exposures(exps, factor: float, fwhm_max: float = 8.0):
    """Exposure records whose PSF FWHM is widened by `factor` (capped at fwhm_max px)."""
    return [dict(x, fwhm=min(float(x["fwhm"]) * factor, fwhm_max)) for x in exps]


def coarse_patch(ctx, exps, flux, var, factor: float = 2.5):
    """A patch over the same images whose planes use the widened Gaussian (Sec. 5.2.2 smoothing)."""
    return B.Patch(ctx, coarse_exposures(exps, factor), flux, var)


def run_coarse_to_fine(ctx, patch, coarse, grid, reps, cell_size: int, budget: int, out=None):
    """Coarse-to-fine: the sparse grid (one representative per cell) stacked on
    the widened-PSF planes, the `budget` cells of highest coarse S/N, then the
    plain stack on every orbit of those cells.  Returns (outputs, cells, coarse S/N)."""
    snr_c, _, _ = B.stack(coarse, reps)
    cells = select_cells(ctx, snr_c, budget)
    out = B.stack_cells(patch, grid, cells, cell_size, out=out)
    return out, cells, snr_c


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
