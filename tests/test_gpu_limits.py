"""Exposure-count limits on the GPU: outlier trimming at its largest patch
(512 exposures), the coarse cell stamps at theirs (1024), the plain stack on
the same 1024-exposure patch, and the argument error one exposure past each
limit (MI355X)."""
import numpy as np
import pytest

import oracle
import synth
from helpers import snr_close, to_torch_images

pytestmark = pytest.mark.gpu

SIZE = 128          # image side (px)
DT = 1e-5           # epoch step between consecutive exposures (days)


def _many(n_exp):
    """n_exp exposures of the small test field's pointing at the grid epoch,
    DT apart and centred on it, on SIZE x SIZE images; candidate orbits pass
    through the middle of the field at that epoch."""
    g = synth.load_geometry("tiny")
    t0 = g["grid_field"]["t"]
    base = min(g["exposures"], key=lambda x: abs(x["t"] - t0))
    exps = []
    for j in range(n_exp):
        x = dict(base)
        x.update(t=t0 + DT * (j - n_exp // 2), width=SIZE, height=SIZE, crpix=[SIZE / 2 + 0.5, SIZE / 2 + 0.5])
        exps.append(x)
    gf = dict(g["grid_field"], half_w=3e-5, half_h=3e-5)
    return g, exps, gf


def _patch(ctx, exps, seed):
    import paper_2503_08854_amd as dt
    D, V = synth.noise_images(exps, seed)
    Dt, Vt = to_torch_images(D, V)
    return D, V, dt.Patch(ctx, exps, Dt, Vt), (Dt, Vt)


@pytest.fixture(scope="module")
def ctx():
    import paper_2503_08854_amd as dt
    return dt.Context(0)


def test_trimming_at_512_exposures(ctx):
    """Sigma clipping over a full 512-exposure patch (eight exposures per lane
    of the fitting wavefront) against the oracle's clipping of its own FP64
    samples; 513 exposures are refused."""
    import torch
    import paper_2503_08854_amd as dt
    g, exps, gf = _many(512)
    D, V, patch, keep = _patch(ctx, exps, 5)
    el = synth.candidate_orbits(gf, 300, 9, g["grid"]["a"], g["grid"]["e"], g["grid"]["inc_deg"])
    orb = dt.OrbitSet(el, g["t0"])
    ids = np.arange(el.shape[0])
    snr_c, flux_c, nk_c = dt.clip_candidates(patch, orb, ids, 3.0, 10)
    torch.cuda.synchronize()
    snr_c, nk_c = snr_c.cpu().numpy(), nk_c.cpu().numpy()
    so = oracle.samples(el, g["t0"], exps, D, V)
    n_band = n_many = 0
    for r in ids:
        v = so["valid"][r]
        psi, phi = so["psi"][r][v], so["phi"][r][v]
        s_or, _, k_or, kept = oracle.sigma_clip(psi, phi, 3.0, 10)
        mu = psi[kept].sum() / phi[kept].sum() if kept.any() else 0.0
        chi = np.abs(psi - mu * phi) / np.sqrt(phi)
        if np.any(np.abs(chi - 3.0) < 1e-4):
            n_band += 1
            continue
        n_many += v.sum() >= 256
        assert nk_c[r] == k_or, (r, nk_c[r], k_or)
        assert abs(snr_c[r] - s_or) <= 1e-5 * max(1.0, abs(s_or)), (r, snr_c[r], s_or)
    assert n_band <= 3
    assert n_many >= 20, "too few orbits cover most of the 512 exposures"
    g2, exps2, _ = _many(513)
    _, _, p513, keep2 = _patch(ctx, exps2, 6)
    with pytest.raises(dt.DtrackError, match="DT_E_ARG"):
        dt.clip_candidates(p513, orb, ids[:4], 3.0, 10)


def test_stamps_and_stack_at_1024_exposures(ctx):
    """Cell stamps over a full 1024-exposure patch (three walks of every
    exposure held in LDS) against the stamp definition on the oracle's walks
    and planes, and the plain stack on the same patch against the oracle;
    1025 exposures are refused by the stamps."""
    import torch
    import paper_2503_08854_amd as dt
    g, exps, gf = _many(1024)
    D, V, patch, keep = _patch(ctx, exps, 7)
    da, dm = 0.002, 5e-6
    reps_el = synth.candidate_orbits(gf, 6, 13, g["grid"]["a"], g["grid"]["e"], g["grid"]["inc_deg"])
    reps = dt.OrbitSet(reps_el, g["t0"])
    out = dt.cell_stamps(patch, reps, da, dm)
    el = synth.candidate_orbits(gf, 1500, 17, g["grid"]["a"], g["grid"]["e"], g["grid"]["inc_deg"])
    orb = dt.OrbitSet(el, g["t0"])
    snr, _, nv = dt.stack(patch, orb)
    torch.cuda.synchronize()
    st = out["stamps"].cpu().numpy()

    planes = [oracle.planes(d, v, x["fwhm"]) for d, v, x in zip(D, V, exps)]
    u = (np.arange(21) - 10) / 10.0
    U = np.broadcast_to(u[None, :], (21, 21))
    Vv = np.broadcast_to(u[:, None], (21, 21))
    n_used = 0
    for r in range(reps_el.shape[0]):
        ra, rm = reps_el[r].copy(), reps_el[r].copy()
        ra[0] += da
        rm[5] += dm
        sm = oracle.samples(np.stack([reps_el[r], ra, rm]), g["t0"], exps)
        Ps = np.zeros((21, 21))
        Ph = np.zeros((21, 21))
        band = np.zeros((21, 21), bool)  # a node within 1e-6 px of a rounding boundary may round either way
        for e, x in enumerate(exps):
            if not np.all(sm["flags"][:, e] & 1):
                continue
            p0x, p0y = sm["px"][0, e], sm["py"][0, e]
            qx = (p0x + U * (sm["px"][1, e] - p0x)) + Vv * (sm["px"][2, e] - p0x)
            qy = (p0y + U * (sm["py"][1, e] - p0y)) + Vv * (sm["py"][2, e] - p0y)
            for q in (qx, qy):
                f = q + 0.5
                band |= np.abs(f - np.round(f)) < 1e-6
            X, Y = np.floor(qx + 0.5).astype(np.int64), np.floor(qy + 0.5).astype(np.int64)
            ok = (X >= 0) & (X < SIZE) & (Y >= 0) & (Y < SIZE)
            psi = np.zeros((21, 21))
            phi = np.zeros((21, 21))
            psi[ok] = planes[e][0][Y[ok], X[ok]]
            phi[ok] = planes[e][1][Y[ok], X[ok]]
            use = phi > 0
            Ps[use] += psi[use]
            Ph[use] += phi[use]
            n_used += int(use.any())
        want = np.where(Ph > 0, Ps / np.sqrt(np.where(Ph > 0, Ph, 1.0)), 0.0)
        assert band.mean() < 0.05
        err = np.abs(st[r] - want) / np.maximum(1.0, np.abs(want))
        assert err[~band].max() < 1e-4, (r, err[~band].max())
    assert n_used >= 1000, "the lattices touch too few exposures"

    s_or, _, nv_or = oracle.stack(el, g["t0"], exps, D, V)
    nv = nv.cpu().numpy()
    np.testing.assert_array_equal(nv, nv_or)
    assert snr_close(snr.cpu().numpy(), s_or).all()
    assert (nv_or >= 512).sum() >= 100, "too few orbits cover most of the 1024 exposures"

    g2, exps2, _ = _many(1025)
    _, _, p1025, keep2 = _patch(ctx, exps2, 8)
    with pytest.raises(dt.DtrackError, match="DT_E_ARG"):
        dt.cell_stamps(p1025, reps, da, dm)
