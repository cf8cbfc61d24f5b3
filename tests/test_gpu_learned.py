"""Learned proposal path on the GPU: BF16 MFMA GEMM, the scorer's forward and
backward passes and Adam against the FP64 NumPy reference, coarse stamps
against the oracle, and the cell-restricted stack (MI355X)."""
import numpy as np
import pytest

import oracle
import synth
from helpers import snr_close, to_torch_images
from oracle import nn_ref as nn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2503_08854_amd as dt
    return dt.Context(0)


def _bf16(x):
    return nn.bf16_round(x)


@pytest.mark.parametrize("M,N,K", [(16, 16, 16), (64, 64, 32), (100, 37, 53), (9, 16, 20000), (300, 1, 64),
                                   (1, 64, 1), (130, 70, 300)])
def test_gemm_matches_float64(ctx, M, N, K):
    import torch
    import paper_2503_08854_amd as dt
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = _bf16(rng.standard_normal((M, K)))
    B = _bf16(rng.standard_normal((K, N)))
    bias = rng.standard_normal(N).astype(np.float32)
    ref = A @ B
    scale = np.abs(A) @ np.abs(B)
    for tA in (False, True):
        for tB in (False, True):
            a = torch.from_numpy(A.T.copy() if tA else A).cuda()
            b = torch.from_numpy(B.T.copy() if tB else B).cuda()
            for use_bias, relu in ((False, False), (True, True)):
                C = dt.gemm_bf16(ctx, a, b, tA, tB, torch.from_numpy(bias).cuda() if use_bias else None, relu)
                want = ref + (bias if use_bias else 0)
                if relu:
                    want = np.maximum(want, 0)
                err = np.abs(C.cpu().numpy() - want)
                assert np.all(err <= 2e-6 * (scale + np.abs(bias)) + 1e-6), (tA, tB, err.max())


def _scorer_and_batch(ctx, B=32, seed=3):
    import torch
    import paper_2503_08854_amd as dt
    sc = dt.Scorer(ctx, max_batch=64, seed=seed)
    th = sc.params().double().cpu().numpy()
    rng = np.random.default_rng(seed)
    X = _bf16(rng.standard_normal((B, 21, 21)))
    F = _bf16(rng.standard_normal((B, 16)))
    Y = (rng.random(B) < 0.5).astype(np.float64)
    # the GPU multiplies BF16 weights; biases stay FP32 (exact in FP64)
    p = nn.unflatten(th)
    for k in p:
        if k.startswith("w"):
            p[k] = _bf16(p[k])
    thb = nn.flatten(p)
    Xt = torch.from_numpy(X).to(torch.bfloat16).cuda()
    Ft = torch.from_numpy(F).to(torch.bfloat16).cuda()
    Yt = torch.from_numpy(Y).float().cuda()
    return sc, th, thb, X, F, Y, Xt, Ft, Yt


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def _grad_bf16_model(theta, X, F, Y):
    """The FP64 reference with the GPU's BF16 rounding points applied
    (activations after each layer, gradient activations before each GEMM):
    the precision model the GPU result should follow closely."""
    R = nn.bf16_round
    p = nn.unflatten(theta)
    B = X.shape[0]
    c1 = nn.im2col(X.reshape(B, 21, 21, 1), 1)
    h1 = R(nn.relu(c1 @ p["w1"] + p["b1"]))
    c2 = nn.im2col(h1, 2)
    h2 = R(nn.relu(c2 @ p["w2"] + p["b2"]))
    c3 = nn.im2col(h2, 2)
    h3 = R(nn.relu(c3 @ p["w3"] + p["b3"]))
    f3 = h3.reshape(B, -1)
    h4 = R(nn.relu(f3 @ p["w4"] + p["b4"]))
    h5 = R(nn.relu(F @ p["w5"] + p["b5"]))
    cat = np.concatenate([h4, h5], 1)
    h6 = R(nn.relu(cat @ p["w6"] + p["b6"]))
    z = (h6 @ p["w7"] + p["b7"])[:, 0]
    dz = (1 / (1 + np.exp(-z)) - Y) / B
    g = {"w7": h6.T @ R(dz)[:, None], "b7": np.array([dz.sum()])}
    d6 = (R(dz)[:, None] @ p["w7"].T) * (h6 > 0)
    g["w6"], g["b6"] = cat.T @ R(d6), d6.sum(0)
    dcat = R(d6) @ p["w6"].T
    d4, d5 = dcat[:, :64] * (h4 > 0), dcat[:, 64:] * (h5 > 0)
    g["w5"], g["b5"] = F.T @ R(d5), d5.sum(0)
    g["w4"], g["b4"] = f3.T @ R(d4), d4.sum(0)
    d3 = (R(d4) @ p["w4"].T).reshape(h3.shape) * (h3 > 0)
    g["w3"], g["b3"] = c3.reshape(-1, 288).T @ R(d3).reshape(-1, 32), d3.reshape(-1, 32).sum(0)
    d2 = nn.col2im(R(d3) @ p["w3"].T, h2.shape, 2) * (h2 > 0)
    g["w2"], g["b2"] = c2.reshape(-1, 144).T @ R(d2).reshape(-1, 32), d2.reshape(-1, 32).sum(0)
    d1 = nn.col2im(R(d2) @ p["w2"].T, h1.shape, 2) * (h1 > 0)
    g["w1"], g["b1"] = c1.reshape(-1, 9).T @ R(d1).reshape(-1, 16), d1.reshape(-1, 16).sum(0)
    return nn.flatten(g)


def test_scorer_forward_and_gradients_vs_oracle(ctx):
    import torch
    sc, th, thb, X, F, Y, Xt, Ft, Yt = _scorer_and_batch(ctx)
    assert sc.num_params() == nn.n_params()
    z = sc.forward(Xt, Ft).cpu().numpy()
    zo = nn.forward(thb, X, F)
    assert _rel(z, zo) < 1e-2
    loss, g = sc.grad(Xt, Ft, Yt)
    lo, go = nn.loss_and_grad(thb, X, F, Y)
    assert abs(float(loss.cpu()[0]) - lo) <= 1e-2 * abs(lo)
    g = g.double().cpu().numpy()
    gu, gou = nn.unflatten(g), nn.unflatten(go)
    gmu = nn.unflatten(_grad_bf16_model(thb, X, F, Y))
    errs = {k: _rel(gu[k], gou[k]) for k in gu}
    errm = {k: _rel(gu[k], gmu[k]) for k in gu}
    cos = {k: float(np.dot(gu[k].ravel(), gou[k].ravel()) / (np.linalg.norm(gu[k]) * np.linalg.norm(gou[k])))
           for k in gu}
    print("gradient rel. L2 vs exact FP64:", {k: f"{v:.2e}" for k, v in errs.items()})
    print("gradient rel. L2 vs BF16-rounding model:", {k: f"{v:.2e}" for k, v in errm.items()})
    # BF16 activations and gradient activations cost up to ~6% in the first
    # layers (the rounding model shows the same); the GPU must follow the model
    # closely and point the same way as the exact gradient
    assert all(v < 1e-1 for v in errs.values()), errs
    assert all(v < 3e-2 for v in errm.values()), errm
    assert all(v > 0.99 for v in cos.values()), cos
    # closed form: the last bias gradient is mean(sigmoid(z) - y)
    assert gu["b7"][0] == pytest.approx(np.mean(1 / (1 + np.exp(-zo)) - Y), rel=2e-2, abs=1e-4)


def test_scorer_fused_inference_matches_forward_and_oracle(ctx):
    """The fused inference kernel against the layer-by-layer forward (same
    rounding points; only the 1152-deep layer's summation order may differ)
    and the FP64 oracle, on a ragged last group and on more groups than the
    grid has workgroups."""
    import torch
    import paper_2503_08854_amd as dt
    sc, th, thb, X, F, Y, Xt, Ft, Yt = _scorer_and_batch(ctx, B=37)
    z = sc.infer(Xt, Ft).cpu().numpy()
    zf = sc.forward(Xt, Ft).cpu().numpy()
    zo = nn.forward(thb, X, F)
    assert _rel(z, zo) < 1e-2
    assert _rel(z, zf) < 2e-3
    # 5000 cells: 313 groups of 16 over at most one workgroup per CU
    big = dt.Scorer(ctx, max_batch=1024, seed=5)
    rng = np.random.default_rng(11)
    Xb = torch.from_numpy(rng.standard_normal((5000, 21, 21))).to(torch.bfloat16).cuda()
    Fb = torch.from_numpy(rng.standard_normal((5000, 16))).to(torch.bfloat16).cuda()
    zi = big.infer(Xb, Fb).cpu().numpy()
    zl = big.forward(Xb, Fb).cpu().numpy()
    assert np.all(np.isfinite(zi))
    assert _rel(zi, zl) < 2e-3, _rel(zi, zl)
    assert np.max(np.abs(zi - zl)) < 2e-2 * max(1.0, np.max(np.abs(zl)))
    assert big.infer(Xb[:0], Fb[:0]).numel() == 0
    # scoring a subset of rows: the same logits at those rows, nothing written elsewhere
    rows = torch.from_numpy(rng.choice(5000, 1234, replace=False)).cuda()
    zr = torch.full((5000,), -7.0, dtype=torch.float32, device="cuda")
    big.infer_rows(Xb, Fb, rows, zr)
    zr = zr.cpu().numpy()
    r = rows.cpu().numpy()
    np.testing.assert_array_equal(zr[r], zi[r])
    assert np.all(np.delete(zr, r) == -7.0)
    big.close()


def test_adam_step_matches_oracle(ctx):
    import torch
    sc, th, thb, X, F, Y, Xt, Ft, Yt = _scorer_and_batch(ctx, seed=5)
    _, g = sc.grad(Xt, Ft, Yt)
    g = g.double().cpu().numpy()
    sc.train_step(Xt, Ft, Yt, lr=1e-3)
    th1 = sc.params().double().cpu().numpy()
    want, _, _ = nn.adam_step(th, np.zeros_like(th), np.zeros_like(th), g, 1, 1e-3)
    assert np.max(np.abs(th1 - want)) < 1e-6


def test_training_learns_a_separable_task(ctx):
    import torch
    import paper_2503_08854_amd as dt
    sc = dt.Scorer(ctx, max_batch=256, seed=11)
    rng = np.random.default_rng(0)
    yy, xx = np.mgrid[-10:11, -10:11]
    blob = np.exp(-(xx ** 2 + yy ** 2) / 8.0)

    def batch(n):
        y = (rng.random(n) < 0.5).astype(np.float32)
        X = rng.standard_normal((n, 21, 21)) + 3.0 * y[:, None, None] * blob
        F = rng.standard_normal((n, 16)) * 0.1
        return (torch.from_numpy(X).to(torch.bfloat16).cuda(), torch.from_numpy(F).to(torch.bfloat16).cuda(),
                torch.from_numpy(y).cuda())

    Xv, Fv, Yv = batch(256)
    l0 = float(sc.grad(Xv, Fv, Yv)[0].cpu()[0])
    for _ in range(150):
        sc.train_step(*batch(256), lr=2e-3)
    l1 = float(sc.grad(Xv, Fv, Yv)[0].cpu()[0])
    acc = ((sc.forward(Xv, Fv) > 0).float() == Yv).float().mean().item()
    assert l1 < 0.5 * l0 and acc > 0.95, (l0, l1, acc)


@pytest.fixture(scope="module")
def cells():
    import torch
    import paper_2503_08854_amd as dt
    g = synth.load_geometry("learned_small")
    cg = g["cell_grid"]
    el = synth.cell_grid(g["grid_field"], cg["cells"], cg["cell_size"], cg["seed"], cg["a"], cg["e"], cg["inc_deg"],
                         cg["da"], cg["dm"])
    exps = synth.exposures_of(g)
    D, V = synth.noise_images(exps, 21, g["nan_frac"])
    hits = [[h[0], h[1], h[2], inj["flux"]] for inj in g["realizations"][0] for h in inj["hits"]]
    synth.render_sources_fast(D, exps, hits)
    c = dt.Context(0)
    Dt, Vt = to_torch_images(D, V)
    patch = dt.Patch(c, exps, Dt, Vt)
    grid = dt.OrbitSet(el, g["t0"])
    reps = dt.OrbitSet(el[::cg["cell_size"]], g["t0"])
    return dict(g=g, el=el, exps=exps, D=D, V=V, ctx=c, patch=patch, grid=grid, reps=reps, keep=(Dt, Vt))


def _lattice_stamps_oracle(c, reps, da, dm, planes=None):
    """The stamp definition on the oracle's walks and planes: per exposure the
    lattice q = (p + u (p_a - p)) + v (p_m - p), nearest pixel, constant-flux
    S/N over the nodes' valid pixels; exposures with a walk behind the plane
    are skipped.  Also returns, per representative, whether any lattice
    coordinate fell within 1e-6 px of a rounding boundary."""
    t0 = c["g"]["t0"]
    if planes is None:
        planes = [oracle.planes(d, v, x["fwhm"]) for d, v, x in zip(c["D"], c["V"], c["exps"])]
    u = (np.arange(21) - 10) / 10.0
    U = np.broadcast_to(u[None, :], (21, 21))
    Vv = np.broadcast_to(u[:, None], (21, 21))
    out = np.zeros((reps.shape[0], 21, 21))
    band = np.zeros(reps.shape[0], bool)
    for r in range(reps.shape[0]):
        ra, rm = reps[r].copy(), reps[r].copy()
        ra[0] += da
        rm[5] += dm
        sm = oracle.samples(np.stack([reps[r], ra, rm]), t0, c["exps"])
        Ps = np.zeros((21, 21))
        Ph = np.zeros((21, 21))
        for e, x in enumerate(c["exps"]):
            if not np.all(sm["flags"][:, e] & 1):
                continue
            p0x, p0y = sm["px"][0, e], sm["py"][0, e]
            qx = (p0x + U * (sm["px"][1, e] - p0x)) + Vv * (sm["px"][2, e] - p0x)
            qy = (p0y + U * (sm["py"][1, e] - p0y)) + Vv * (sm["py"][2, e] - p0y)
            for q in (qx, qy):
                f = q + 0.5
                band[r] |= bool(np.any(np.abs(f - np.round(f)) < 1e-6))
            X, Y = np.floor(qx + 0.5).astype(np.int64), np.floor(qy + 0.5).astype(np.int64)
            ok = (X >= 0) & (X < x["width"]) & (Y >= 0) & (Y < x["height"])
            psi = np.zeros((21, 21))
            phi = np.zeros((21, 21))
            psi[ok] = planes[e][0][Y[ok], X[ok]]
            phi[ok] = planes[e][1][Y[ok], X[ok]]
            use = phi > 0
            Ps[use] += psi[use]
            Ph[use] += phi[use]
        out[r] = np.where(Ph > 0, Ps / np.sqrt(np.where(Ph > 0, Ph, 1.0)), 0.0)
    return out, band


def test_cell_stamps_match_oracle_planes(cells):
    import torch
    import paper_2503_08854_amd as dt
    c = cells
    cg = c["g"]["cell_grid"]
    out = dt.cell_stamps(c["patch"], c["reps"], cg["da"], cg["dm"])
    torch.cuda.synchronize()
    st = out["stamps"].cpu().numpy()
    ft = out["feats"].cpu().numpy()
    np.testing.assert_array_equal(out["stamps_bf16"].float().cpu().numpy(), nn.bf16_round(st).astype(np.float32))
    reps = c["el"][::cg["cell_size"]]
    want, band = _lattice_stamps_oracle(c, reps, cg["da"], cg["dm"])
    err = np.abs(st - want) / np.maximum(1.0, np.abs(want))
    worst = err.reshape(err.shape[0], -1).max(1)
    assert np.all(worst[~band] < 1e-4), worst[~band].max()
    # a node within 1e-6 px of a rounding boundary may round either way
    assert band.mean() < 0.2
    for r in range(reps.shape[0]):
        assert ft[r, 0] == pytest.approx(st[r].max(), abs=1e-6)
        assert ft[r, 1] == pytest.approx(st[r][10, 10], abs=1e-6)
        row, col = divmod(int(np.argmax(st[r])), 21)   # the first node holding the maximum
        assert ft[r, 11] == np.float32((col - 10) / 10.0) and ft[r, 12] == np.float32((row - 10) / 10.0)


def test_cell_stamps_many_exposures_match_oracle(cells):
    """Stamps over more than 256 exposures (the kernel then keeps the gathers
    of four usable exposures in flight per lane instead of two): the small
    set's exposures repeated eleven times (same images, epochs and observer),
    against the oracle's lattice on the same list, on 40 cells."""
    import torch
    import paper_2503_08854_amd as dt
    c = cells
    cg = c["g"]["cell_grid"]
    rep = 11
    exps = c["exps"] * rep
    assert len(exps) > 256
    Dt, Vt = c["keep"]
    patch = dt.Patch(c["ctx"], exps, list(Dt) * rep, list(Vt) * rep)
    reps_el = c["el"][::cg["cell_size"]][:40]
    reps = dt.OrbitSet(reps_el, c["g"]["t0"])
    out = dt.cell_stamps(patch, reps, cg["da"], cg["dm"])
    torch.cuda.synchronize()
    st = out["stamps"].cpu().numpy()
    planes = [oracle.planes(d, v, x["fwhm"]) for d, v, x in zip(c["D"], c["V"], c["exps"])] * rep
    cd = dict(c, exps=exps)
    want, band = _lattice_stamps_oracle(cd, reps_el, cg["da"], cg["dm"], planes=planes)
    err = np.abs(st - want) / np.maximum(1.0, np.abs(want))
    worst = err.reshape(err.shape[0], -1).max(1)
    assert np.all(worst[~band] < 1e-4), worst[~band].max()
    assert (~band).sum() >= 30 and np.abs(want).max() > 1.0
    # the same cells over the single set: every node's S/N scales by sqrt(11)
    one = dt.cell_stamps(c["patch"], reps, cg["da"], cg["dm"])["stamps"].cpu().numpy()
    np.testing.assert_allclose(st[~band], one[~band] * np.sqrt(rep), rtol=1e-4, atol=1e-4)
    patch.close()


def test_cell_stamps_peak_at_a_member_source(cells):
    """A source on a member shows as a stamp peak near the member's (u, v):
    the lattice follows the members' tracks, so the peak S/N is close to the
    member's own stacked S/N."""
    import torch
    import paper_2503_08854_amd as dt
    c = cells
    cg = c["g"]["cell_grid"]
    cs = cg["cell_size"]
    # the first cell with a non-representative member inside >= 8 exposures
    mem = None
    for cell in range(cg["cells"]):
        ids = cell * cs + np.arange(1, cs)
        d = dt.debug_samples(c["patch"], c["grid"], ids)
        n_in = ((d["flags"].cpu().numpy() & 2) != 0).sum(1)
        if n_in.max() >= 8:
            k = int(np.argmax(n_in))
            mem = int(ids[k])
            px, py, fl = (d[key].cpu().numpy()[k] for key in ("px", "py", "flags"))
            break
    assert mem is not None
    inside = (fl & 2) != 0
    D = [x.copy() for x in c["D"]]
    hits = [[e, px[e], py[e], 20.0] for e in np.nonzero(inside)[0]]
    synth.render_sources_fast(D, c["exps"], hits)
    Dt, Vt = to_torch_images(D, c["V"])
    patch = dt.Patch(c["ctx"], c["exps"], Dt, Vt)
    out = dt.cell_stamps(patch, c["reps"], cg["da"], cg["dm"])
    snr, _, _ = dt.stack(patch, c["grid"])
    torch.cuda.synchronize()
    st = out["stamps"].cpu().numpy()[cell]
    s_mem = float(snr.cpu().numpy()[mem])
    el = c["el"][mem]
    rep = c["el"][cell * cs]
    u0 = (el[0] - rep[0]) / cg["da"]
    v0 = (el[5] - rep[5]) / cg["dm"]
    r, q = np.unravel_index(np.argmax(st), st.shape)
    assert abs((q - 10) / 10.0 - u0) <= 0.25 and abs((r - 10) / 10.0 - v0) <= 0.25, (q, r, u0, v0)
    assert st.max() >= 0.7 * s_mem and s_mem > 8.0
    patch.close()


def test_stack_cells_equals_full_stack(cells):
    """The stack on selected cells walks each orbit's exposures in up to four
    ranges and merges the ranges' compensated sums in range order: valid
    counts equal the full stack's, S/N and flux agree to rounding."""
    import torch
    import paper_2503_08854_amd as dt
    c = cells
    full = dt.stack(c["patch"], c["grid"])
    sel = np.array([3, 17, 0, 150, 199])
    part = dt.stack_cells(c["patch"], c["grid"], sel, c["g"]["cell_grid"]["cell_size"])
    torch.cuda.synchronize()
    cs = c["g"]["cell_grid"]["cell_size"]
    mask = np.zeros(c["grid"].n, bool)
    for s_ in sel:
        mask[s_ * cs:(s_ + 1) * cs] = True
    a = [t.cpu().numpy() for t in full]
    b = [t.cpu().numpy() for t in part]
    np.testing.assert_array_equal(a[2][mask], b[2][mask])
    assert (b[2][mask] > 0).sum() > 100
    for k in (0, 1):
        np.testing.assert_allclose(b[k][mask], a[k][mask], rtol=1e-6, atol=1e-6)
    assert np.all(b[2][~mask] == -2)


def test_members_near_and_id_stack(cells):
    """The member window around given lattice points lists exactly the
    members the rule selects (u = (a_m - a_rep) / da, v = (M0_m - M0_rep) / dm
    within the radius of (u*, v*)), and the stack of the listed ids equals
    the full stack on those orbits; other outputs are untouched."""
    import torch
    import paper_2503_08854_amd as dt
    c = cells
    cg = c["g"]["cell_grid"]
    cs, da, dm = cg["cell_size"], cg["da"], cg["dm"]
    el = c["el"]
    rng = np.random.default_rng(5)
    sel = np.array([3, 17, 0, 150, -1, 199])
    uv = np.zeros((cg["cells"], 16), np.float32)
    uv[:, 11:13] = rng.uniform(-1, 1, (cg["cells"], 2)).astype(np.float32)
    uv_t = torch.from_numpy(uv).cuda()
    for radius in (0.0, 0.3, 2.0):
        ids, cnt = dt.cell_members_near(c["ctx"], c["grid"], sel, cs, uv_t[:, 11:], da, dm, radius)
        torch.cuda.synchronize()
        got = np.sort(ids.cpu().numpy()[:int(cnt.cpu()[0])])
        want = []
        for cc in sel[sel >= 0]:
            o = cc * cs + np.arange(cs)
            u = (el[o, 0] - el[cc * cs, 0]) / da
            v = (el[o, 5] - el[cc * cs, 5]) / dm
            d = np.maximum(np.abs(u - uv[cc, 11]), np.abs(v - uv[cc, 12]))
            assert not np.any(np.abs(d - radius) < 1e-9)     # no member on the window's edge
            want.extend(o[d <= radius])
        np.testing.assert_array_equal(got, np.sort(np.array(want, dtype=np.int64)))
        if radius == 2.0:
            assert got.size == (sel >= 0).sum() * cs       # the whole (u, v) box of every selected cell
    ids, cnt = dt.cell_members_near(c["ctx"], c["grid"], sel, cs, uv_t[:, 11:], da, dm, 0.8)
    full = [t.cpu().numpy() for t in dt.stack(c["patch"], c["grid"])]
    part = [t.cpu().numpy() for t in dt.stack_ids(c["patch"], c["grid"], ids, cnt)]
    torch.cuda.synchronize()
    listed = np.zeros(c["grid"].n, bool)
    listed[ids.cpu().numpy()[:int(cnt.cpu()[0])]] = True
    assert listed.sum() > 30
    np.testing.assert_array_equal(part[2][listed], full[2][listed])
    for k in (0, 1):
        np.testing.assert_allclose(part[k][listed], full[k][listed], rtol=1e-6, atol=1e-6)
    assert np.all(part[2][~listed] == -2) and np.all(np.isnan(part[0][~listed]))


def test_id_stack_short_and_long_lists(cells):
    """The id-list stack picks its walk from the count on the device: a short
    list in a long buffer (the per-sample split walk, with the long-list
    kernels launched and returning at once) and a list longer than 2^17 (the
    checkpoint walk with deferral; every orbit listed several times) both
    give the full stack's valid counts and S/N on the listed orbits."""
    import torch
    import paper_2503_08854_amd as dt
    c = cells
    n = c["grid"].n
    full = [t.cpu().numpy() for t in dt.stack(c["patch"], c["grid"])]
    rng = np.random.default_rng(9)
    reps = (1 << 17) // n + 2
    long_ids = np.tile(np.arange(n, dtype=np.int64), reps)
    rng.shuffle(long_ids)
    ids = torch.from_numpy(long_ids).cuda()
    for count, name in ((min(n, 5000), "short"), (long_ids.size, "long")):
        assert (count > (1 << 17)) == (name == "long")
        cnt = torch.tensor([count], dtype=torch.int64, device="cuda")
        part = [t.cpu().numpy() for t in dt.stack_ids(c["patch"], c["grid"], ids, cnt)]
        torch.cuda.synchronize()
        listed = np.zeros(n, bool)
        listed[long_ids[:count]] = True
        assert listed.sum() > 100, name
        np.testing.assert_array_equal(part[2][listed], full[2][listed], err_msg=name)
        for k in (0, 1):
            np.testing.assert_allclose(part[k][listed], full[k][listed], rtol=1e-6, atol=1e-6, err_msg=name)
        assert np.all(part[2][~listed] == -2), name


def test_coarse_to_fine_matches_oracle(cells):
    """Coarse-to-fine: 3 x 3 sub-representatives per cell stacked on the
    widened-PSF planes (against the oracle on the same widened exposures),
    each cell ranked by its best one, the top cells stacked in full."""
    import torch
    import paper_2503_08854_amd as dt
    from paper_2503_08854_amd import proposer
    c = cells
    cg = c["g"]["cell_grid"]
    cs = cg["cell_size"]
    Dt, Vt = c["keep"]
    coarse = proposer.coarse_patch(c["ctx"], c["exps"], Dt, Vt, factor=2.5)
    budget, k = 20, 3
    reps = c["el"][::cs]
    sub_el = proposer.sub_representatives(reps, cg["da"], cg["dm"], k)
    assert sub_el.shape == (reps.shape[0] * k * k, 6)
    # the centre sub-representative is the representative itself
    np.testing.assert_array_equal(sub_el[k * k // 2::k * k], reps)
    subs = dt.OrbitSet(sub_el, c["g"]["t0"])
    out, sel, score = proposer.run_coarse_to_fine(c["ctx"], c["patch"], coarse, c["grid"], subs, k * k, cs, budget)
    snr_sub = dt.stack(coarse, subs)[0]
    torch.cuda.synchronize()
    score = score.cpu().numpy()
    snr_sub = snr_sub.cpu().numpy()
    sel = sel.cpu().numpy()
    # coarse S/N of the sub-representatives vs the oracle on widened-PSF planes
    wide = proposer.coarse_exposures(c["exps"], 2.5)
    snr_o, _, _ = oracle.stack(sub_el, c["g"]["t0"], wide, c["D"], c["V"])
    assert snr_close(snr_sub, snr_o).all()
    np.testing.assert_array_equal(score, snr_sub.reshape(-1, k * k).max(axis=1))
    # selection: the top `budget` of the GPU's cell scores (same precision on
    # both sides), as a set (the proposer takes it unordered)
    np.testing.assert_array_equal(np.sort(sel), np.sort(oracle.topk(score.astype(np.float64), budget)))
    # fine stack on the selected cells vs the oracle on those orbits
    ids = (sel[:, None] * cs + np.arange(cs)[None, :]).ravel()
    snr_f, _, nv_f = oracle.stack(c["el"][ids], c["g"]["t0"], c["exps"], c["D"], c["V"])
    got = out[0].cpu().numpy()
    np.testing.assert_array_equal(out[2].cpu().numpy()[ids], nv_f)
    assert snr_close(got[ids], snr_f).all()
    assert np.all(np.isnan(np.delete(got, ids)))


def test_learned_beats_coarse_max_on_artifacts(ctx):
    """What the trained network adds to the method.  With single-exposure
    point artifacts in every image the stamp maximum ranks the artifact cells
    first; on held-out realizations (the stored injections) at a 2 % budget
    the scorer, trained on 30 fresh realizations, keeps most of what the
    exhaustive stack finds while coarse-max at the same budget keeps almost
    nothing.  At equal time (coarse-max given the budget its pass can afford
    in the learned pass's time) the figures are printed for the record."""
    import learned_eval as le
    s = le.load_setup("learned")
    b = le.Bench(s, ctx, "cuda")
    X, F, Y = le.training_set(b, 30, seed=3, artifacts=le.ARTIFACTS)
    sc, hist = le.train_scorer(ctx, X, F, Y, epochs=2, batch=512, lr=1e-3)
    del X, F, Y
    assert hist[-1][1] < hist[0][1]
    curve_b = (0.01, 0.02, 0.04, 0.08, 0.16)
    curve = le.pass_times(b, sc, curve_b, radius=0.35, prefilter=0.2, artifacts=le.ARTIFACTS, reps=3)
    b_eq = le.equal_time_budget(float(np.interp(0.02, curve_b, curve["learned"])), curve_b, curve["coarse"])
    r = le.evaluate(b, sc, budget_frac=0.02, n_real=12, artifacts=le.ARTIFACTS, radius=0.35, prefilter=0.2,
                    coarse_equal_time_frac=b_eq)
    print(f"learned {r['recall_ratio_learned']:.3f} coarse-max {r['recall_ratio_coarse']:.3f} at 2 %; coarse-max at "
          f"equal time ({b_eq:.1%}) {r['recall_ratio_coarse_equal_time']:.3f}; coarse-to-fine "
          f"{r['recall_ratio_coarse_to_fine']:.3f}; times (ms) learned {r['t_learned_ms']:.3f} coarse "
          f"{r['t_coarse_ms']:.3f} coarse at equal time {r['t_coarse_equal_time_ms']:.3f}")
    assert r["plain_found"] >= 100
    assert r["recall_ratio_learned"] >= 0.85
    assert r["recall_ratio_learned"] - r["recall_ratio_coarse"] >= 0.5
    assert b_eq >= 0.02
    sc.close()
    b.close()
