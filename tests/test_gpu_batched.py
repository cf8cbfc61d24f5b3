"""Batched uneven patches in one persistent launch, graph capture/replay and
the launch-shape autotuner, against per-patch stacks and the oracle (MI355X)."""
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import snr_close, to_torch_images

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    import torch
    import paper_2503_08854_amd as dt
    geom = synth.load_geometry("batched_small")
    ws = [synth.build_workload(g) for g in geom["patches"]]
    ctx = dt.Context(0)
    patches, sets, imgs = [], [], []
    for w in ws:
        D, V = to_torch_images(w.D, w.V)
        imgs.append((D, V))
        patches.append(dt.Patch(ctx, w.exps, D, V))
        sets.append(dt.OrbitSet(w.elements, w.t0))
    torch.cuda.synchronize()
    return dict(ws=ws, ctx=ctx, patches=patches, sets=sets, imgs=imgs)


def _np(outs):
    return [tuple(t.cpu().numpy() for t in o) for o in outs]


def test_batched_equals_per_patch_and_oracle(batch):
    import torch
    import paper_2503_08854_amd as dt
    ws, ctx, patches, sets = batch["ws"], batch["ctx"], batch["patches"], batch["sets"]
    assert all(w.dtype == "f16" for w in ws)
    outs, tk = dt.stack_batched(ctx, patches, sets, k=8, eager=True, cfg=(256, 2))
    torch.cuda.synchronize()
    got = _np(outs)
    for p, (w, patch, orb) in enumerate(zip(ws, patches, sets)):
        snr, flux, nv = dt.stack(patch, orb)
        idx, val, cnt = dt.topk(ctx, snr, 8)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got[p][0], snr.cpu().numpy())
        np.testing.assert_array_equal(got[p][2], nv.cpu().numpy())
        c = int(cnt.cpu()[0])
        assert int(tk[2][p].cpu()) == c
        np.testing.assert_array_equal(tk[0][p].cpu().numpy()[:c], idx.cpu().numpy()[:c])
        so, fo, no = oracle.stack(w.elements, w.t0, w.exps, w.D, w.V)
        np.testing.assert_array_equal(got[p][2], no)
        ok = snr_close(got[p][0], so)
        assert ok.all(), f"patch {p}: {(~ok).sum()} orbits off"


def test_pruned_stack_equals_exact_walk(batch):
    """Sky-cone pruning against the exact walk on every patch, near-Earth
    geometries (light-time shift up to pixels) included."""
    import torch
    import paper_2503_08854_amd as dt
    for p, (patch, orb) in enumerate(zip(batch["patches"], batch["sets"])):
        snr, flux, nv = dt.stack(patch, orb)
        rec = dt.record_valid_gathers(patch, orb)
        rep = dt.replay_valid_gathers(patch, rec)
        ex = {k: v.cpu().numpy() for k, v in dt.debug_samples(patch, orb, np.arange(orb.n)).items()}
        torch.cuda.synchronize()
        nv = nv.cpu().numpy()
        np.testing.assert_array_equal(np.maximum(nv, 0), ((ex["flags"] & 4) != 0).sum(axis=1), err_msg=f"patch {p}")
        np.testing.assert_array_equal(rep.cpu().numpy(), np.where(nv > 0, snr.cpu().numpy(), 0.0).astype(np.float32))


def test_batched_topk_both_paths(batch):
    """Batched top-k against the single-array top-k: small k (all patches in
    two launches) and k = 4096 with a 40000-orbit patch (more survivors than
    one workgroup selects from: the batch takes per-patch tournaments)."""
    import torch
    import paper_2503_08854_amd as dt
    ws, ctx, patches = batch["ws"], batch["ctx"], batch["patches"]
    w0 = ws[0]
    reps = -(-40000 // w0.elements.shape[0])
    big = dt.OrbitSet(np.tile(w0.elements, (reps, 1))[:40000], w0.t0)
    for k, sets, pats in [(3, batch["sets"], patches), (4096, [big, batch["sets"][1]], patches[:2])]:
        outs, tk = dt.stack_batched(ctx, pats, sets, k=k, eager=True, cfg=(512, 2))
        torch.cuda.synchronize()
        for p, (patch, orb) in enumerate(zip(pats, sets)):
            idx, val, cnt = dt.topk(ctx, outs[p][0], k)
            torch.cuda.synchronize()
            c = int(cnt.cpu()[0])
            assert int(tk[2][p].cpu()) == c
            np.testing.assert_array_equal(tk[0][p].cpu().numpy()[:c], idx.cpu().numpy()[:c])
            np.testing.assert_array_equal(tk[1][p].cpu().numpy()[:c], val.cpu().numpy()[:c])


def test_graph_replay_matches_eager(batch):
    import torch
    import paper_2503_08854_amd as dt
    ctx, patches, sets = batch["ctx"], batch["patches"], batch["sets"]
    ref, rtk = dt.stack_batched(ctx, patches, sets, k=8, eager=True)
    torch.cuda.synchronize()
    ref, rtk = _np(ref), [t.cpu().numpy() for t in rtk]
    outs, tk = dt.stack_batched(ctx, patches, sets, k=8)
    for rep in range(4):
        for o in outs:                       # poison the outputs between replays
            o[0].fill_(-7.0)
            o[2].fill_(-7)
        x = torch.randn(1 << 20, device="cuda")
        _ = (x * 2).sum().item()             # unrelated eager work and a sync
        dt.stack(patches[0], sets[0])
        outs, tk = dt.stack_batched(ctx, patches, sets, outs=outs, k=8, topk_out=tk)  # replay
        torch.cuda.synchronize()
        got = _np(outs)
        for p in range(len(patches)):
            np.testing.assert_array_equal(got[p][0], ref[p][0])
            np.testing.assert_array_equal(got[p][2], ref[p][2])
        for a, b in zip(tk, rtk):
            np.testing.assert_array_equal(a.cpu().numpy(), b)


def test_graph_with_prepass_sees_new_images(batch):
    import torch
    import paper_2503_08854_amd as dt
    ctx, patches, sets, imgs, ws = batch["ctx"], batch["patches"], batch["sets"], batch["imgs"], batch["ws"]
    outs, _ = dt.stack_batched(ctx, patches, sets, prepass=True)
    torch.cuda.synchronize()
    before = outs[1][0].cpu().numpy().copy()
    D = imgs[1][0]
    for d in D:
        d.add_(0.5)                          # brighten every image of patch 1 in place
    outs, _ = dt.stack_batched(ctx, patches, sets, outs=outs, prepass=True)  # replay re-runs the pre-pass
    torch.cuda.synchronize()
    after = outs[1][0].cpu().numpy()
    w = ws[1]
    Dh = [d.cpu().numpy() for d in D]
    so, _, _ = oracle.stack(w.elements, w.t0, w.exps, Dh, w.V)
    assert snr_close(after, so).all()
    assert not np.array_equal(before, after)
    for d in D:
        d.sub_(0.5)
    patches[1].refresh()
    torch.cuda.synchronize()


def test_autotune_and_cache(batch, tmp_path):
    import torch
    import paper_2503_08854_amd as dt
    ctx, patches, sets = batch["ctx"], batch["patches"], batch["sets"]
    path = str(tmp_path / "tune.txt")
    cfg, ms = dt.autotune_batched(ctx, patches, sets, cache_path=path)
    assert cfg[0] % 256 == 0 and 1 <= cfg[1] <= 16 and ms > 0
    cfg2, ms2 = dt.autotune_batched(ctx, patches, sets, cache_path=path)
    assert cfg2 == cfg and ms2 == -1.0
    assert open(path).read().count("\n") == 1
    outs, _ = dt.stack_batched(ctx, patches, sets, cfg=cfg)
    ref = [dt.stack(p, o)[0] for p, o in zip(patches, sets)]
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        np.testing.assert_array_equal(o[0].cpu().numpy(), r.cpu().numpy())


def test_release_images_and_destroy(batch):
    import torch
    import paper_2503_08854_amd as dt
    ctx, ws = batch["ctx"], batch["ws"]
    w = ws[0]
    D, V = to_torch_images(w.D, w.V)
    p = dt.Patch(ctx, w.exps, D, V)
    o = dt.OrbitSet(w.elements, w.t0)
    ref = dt.stack(p, o)[0].cpu().numpy()
    outs, _ = dt.stack_batched(ctx, [p], [o])
    p.release_images()
    del D, V
    with pytest.raises(dt.DtrackError, match="DT_E_STATE"):
        p.refresh()
    with pytest.raises(dt.DtrackError, match="DT_E_STATE"):
        dt.stack_batched(ctx, [p], [o], prepass=True)
    outs, _ = dt.stack_batched(ctx, [p], [o])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(outs[0][0].cpu().numpy(), ref)
    p.close()                                # drops the context's graph that used it
    p2 = dt.Patch(ctx, w.exps, *to_torch_images(w.D, w.V))
    outs, _ = dt.stack_batched(ctx, [p2], [o])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(outs[0][0].cpu().numpy(), ref)
    p2.close()


def test_batched_bad_arguments(batch):
    import paper_2503_08854_amd as dt
    ctx, patches, sets = batch["ctx"], batch["patches"], batch["sets"]
    with pytest.raises(dt.DtrackError, match="DT_E_ARG"):
        dt.stack_batched(ctx, patches, sets, cfg=(300, 4))
    with pytest.raises(dt.DtrackError, match="DT_E_ARG"):
        dt.stack_batched(ctx, patches, sets, cfg=(256, 0))
    with pytest.raises(dt.DtrackError, match="DT_E_ARG"):
        dt.stack_batched(ctx, patches, sets, k=5000)
