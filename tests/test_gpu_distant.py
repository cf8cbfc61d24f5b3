"""Distant objects at full size (MI355X only): 400 FP16 4096^2 images plus
variance over 365 days, 10^9 candidate orbits at 30-60 AU generated on the
device, in the launch the benchmark times; the oracle recomputes a sample of
orbits one by one from its own generator and the same FP16 values."""
import numpy as np
import pytest

import oracle
import synth
from oracle import generate as G
from helpers import band_orbits, compare_samples, gpu_sampler, oracle_sampler, snr_close

pytestmark = pytest.mark.gpu


def test_distant_full_size_sampled():
    import torch
    import paper_2503_08854_amd as dt
    geom = synth.load_geometry("distant")
    gs = synth.grid_sampler(geom)
    n = gs["n"]
    print(f"distant: {len(geom['exposures'])} exposures, {n} generated orbits", flush=True)
    w = synth.build_workload(geom, device="cuda")
    assert w.D[0].dtype == torch.float16 and tuple(w.D[0].shape) == (4096, 4096)
    ctx = dt.Context(0)
    patch = dt.Patch(ctx, w.exps, w.D, w.V)
    out = (torch.empty(n, dtype=torch.float32, device="cuda"), torch.empty(n, dtype=torch.float32, device="cuda"),
           torch.empty(n, dtype=torch.int32, device="cuda"))
    ctx.count_work(True)
    dt.stack_generated(patch, gpu_sampler(gs), 0, n, out)
    wk = ctx.work()
    ctx.count_work(False)
    # these orbits land in most exposures: the probe's wavefronts all defer and
    # the rest go straight to the per-sample walk
    assert wk["switched_waves"] == (1 << 22) // 64, wk
    assert wk["tail_samples"] == n * len(w.exps), wk
    k = 100
    idx, val, cnt = dt.topk(ctx, out[0], k, 5.0)
    torch.cuda.synchronize()
    snr, nv = out[0], out[2]
    assert int((nv < 0).sum()) == 0, "a generated orbit fell outside the domain"
    # top-k: sorted, all >= 5, and no unreported orbit above the k-th value
    c = int(cnt.cpu()[0])
    iv, vv = idx.cpu().numpy()[:c], val.cpu().numpy()[:c]
    assert c == k and np.all(vv >= 5.0) and np.all(np.diff(vv) <= 0)
    np.testing.assert_array_equal(snr[idx[:c]].cpu().numpy(), vv)
    assert int((snr > float(vv[-1])).sum()) <= k
    # the oracle on 3000 random orbits, every injection and the top-k members
    rng = np.random.default_rng(11)
    ids = np.unique(np.r_[rng.choice(n, 3000, replace=False), w.inj_index, iv])
    g_snr = snr[torch.as_tensor(ids, device="cuda")].cpu().numpy()
    g_nv = nv[torch.as_tensor(ids, device="cuda")].cpu().numpy()
    el = np.array([G.sample_orbit(oracle_sampler(gs), int(j)) for j in ids], dtype=np.float64)
    D = [d.cpu().numpy() for d in w.D]
    V = [v.cpu().numpy() for v in w.V]
    so, fo, nvo = oracle.stack(el, w.t0, w.exps, D, V)
    same = g_nv == nvo
    ok = snr_close(g_snr, so)
    print(f"distant: {ids.size} orbits checked, {int((~same).sum())} n_valid differences, "
          f"max S/N error {np.max(np.abs(g_snr - so) / np.maximum(1, np.abs(so))):.3g}", flush=True)
    assert ok[same].all(), f"{int((~ok[same]).sum())} orbits outside the S/N tolerance"
    bad = np.nonzero(~same | ~ok)[0]
    if bad.size:
        # only through a sample within 1e-6 px of a rounding boundary
        assert bad.size <= 3 and band_orbits(el[bad], w.t0, w.exps).all()
    assert (nvo > 0).sum() > 2000
    # the injections are grid members with their oracle elements
    inj_el = np.array([i["el"] for i in geom["injections"]])
    np.testing.assert_allclose(el[np.searchsorted(ids, w.inj_index)], inj_el, rtol=0, atol=0)
    # per-sample table of 100 orbits by the library's exact walk vs the oracle
    sub = np.r_[np.arange(80), np.searchsorted(ids, w.inj_index[:20])]
    orb = dt.OrbitSet(el[sub], w.t0)
    dbg = {kk: v.cpu().numpy() for kk, v in dt.debug_samples(patch, orb, np.arange(sub.size)).items()}
    o = oracle.samples(el[sub], w.t0, w.exps, D, V)
    nb, nc = compare_samples(dbg, o, w.exps)
    assert o["bad"] == 0 and nb <= 2 and nc > 5000
    f = (o["flags"] & 1) != 0
    np.testing.assert_allclose(dbg["tau"][f], o["tau"][f], rtol=0, atol=1e-12)
    patch.close()
    ctx.close()
    del w, D, V, out, patch
    torch.cuda.empty_cache()
