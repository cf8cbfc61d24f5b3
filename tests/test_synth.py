"""The seeded input generators: determinism and the inverse orbit construction."""
import math

import numpy as np

import oracle
import synth


def test_orbits_through_land_on_the_line_of_sight():
    rng = synth.make_rng(4, 0)
    obs = np.array([0.6, 0.8, 0.0])
    dirs = synth.unit(rng.standard_normal((300, 3)) * [0.1, 0.1, 0.05] + [0.6, 0.8, 0.02])
    a = rng.uniform(0.8, 40, 300)
    e = rng.uniform(0, 0.6, 300)
    inc = np.radians(rng.uniform(0, 30, 300))
    el, ok = synth.orbits_through(rng, dirs, obs, a, e, inc)
    assert ok.mean() > 0.5
    for k in np.nonzero(ok)[0]:
        r, _, _ = oracle.helio_state(el[k], 7.0, 7.0)
        d = synth.unit(r - obs)
        assert np.linalg.norm(np.cross(d, dirs[k])) < 1e-11 and d @ dirs[k] > 0
        assert el[k, 2] >= inc[k] - 1e-15 and 0 <= el[k, 1] < 1


def test_workload_is_deterministic():
    g = synth.load_geometry("tiny")
    a = synth.build_workload(g)
    b = synth.build_workload(g)
    np.testing.assert_array_equal(a.elements, b.elements)
    for x, y in zip(a.D, b.D):
        np.testing.assert_array_equal(x, y)
    assert a.elements.shape == (10000, 6)
    np.testing.assert_array_equal(a.elements[a.inj_index[0]], np.asarray(g["injections"][0]["el"]))


def test_noise_and_mask_recipe():
    g = synth.load_geometry("survey_small")
    w = synth.build_workload(g)
    nan = np.mean([np.isnan(d).mean() for d in w.D])
    assert 0.003 < nan < 0.007
    for d, v, x in zip(w.D, w.V, w.exps):
        m = np.isnan(d)
        np.testing.assert_array_equal(m, np.isnan(v))
        assert np.allclose(v[~m], np.float32(x["sigma"] ** 2))
        assert abs(np.nanstd(d) - x["sigma"]) < 0.02 * x["sigma"] + 0.05


def test_cell_grid_geometries_match_their_injections():
    """The learned geometries (survey and distant exposures): the cell grid
    rebuilt from the stored recipe holds every injection's elements at its
    orbit index, and the stored hits are the oracle's landing pixels of that
    orbit (checked on three injections per geometry)."""
    for name in ("learned_small", "distant_cells"):
        g = synth.load_geometry(name)
        cg = g["cell_grid"]
        el = synth.cell_grid(g["grid_field"], cg["cells"], cg["cell_size"], cg["seed"], cg["a"], cg["e"],
                             cg["inc_deg"], cg["da"], cg["dm"])
        exps = synth.exposures_of(g)
        injs = [i for r in g["realizations"] for i in r]
        for inj in injs:
            np.testing.assert_array_equal(el[inj["orbit"]], np.asarray(inj["el"]))
            assert inj["orbit"] // cg["cell_size"] == inj["cell"] and inj["orbit"] % cg["cell_size"] != 0
        for inj in injs[:3]:
            s = oracle.samples(np.asarray(inj["el"])[None, :], g["t0"], exps)
            land = np.nonzero((s["flags"][0] & 3) == 3)[0]
            h = np.asarray(inj["hits"], dtype=np.float64)
            np.testing.assert_array_equal(h[:, 0].astype(int), land)
            np.testing.assert_allclose(h[:, 1], s["px"][0, land], atol=1e-9)
            np.testing.assert_allclose(h[:, 2], s["py"][0, land], atol=1e-9)
    assert g["dtype"] == "f16" and len(exps) == 400 and np.mean([len(i["hits"]) for i in injs]) > 100
