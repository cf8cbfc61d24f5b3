"""GPU (HIP) path vs the CPU oracle, element by element (MI355X only)."""
import math

import numpy as np
import pytest

import oracle
import synth
from helpers import compare_samples, gpu_run, snr_close, to_torch_images

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
