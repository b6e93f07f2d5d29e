"""Seeded input generators: determinism, fill bands, value grids."""
import numpy as np

import workloads as W


def test_designs_are_deterministic_and_in_band():
    a = W.design_2d_discs_rects()
    assert np.array_equal(a, W.design_2d_discs_rects())
    assert 0.35 <= a.mean() <= 0.45 and a.dtype == np.uint8
    b = W.design_3d_boxes_cyls(64)
    assert np.array_equal(b, W.design_3d_boxes_cyls(64))
    assert 0.25 <= b.mean() <= 0.35


def test_density_design_is_on_the_q24_grid():
    d = W.design_density(48, seed=99)
    assert d.dtype == np.float32
    q = d.astype(np.float64) * W.Q24
    assert np.array_equal(q, np.rint(q)) and d.min() >= 0 and d.max() <= 1
    assert abs(d.mean() - 0.35) < 0.002
    assert np.array_equal(d, W.design_density(48, seed=99))


def test_direction_sets():
    f = W.fib_hemisphere(130)
    assert f.shape == (130, 3) and (f[:, 2] > 0).all()
    assert np.all(np.abs(np.linalg.norm(f, axis=1) - 1) < 1e-12)
    l26 = W.lattice26()
    assert len({tuple(v) for v in l26}) == 26 and not (l26 == 0).all(axis=1).any()
    assert len(W.circle8()) == 8


def test_fixtures():
    p = W.fixture_plate((10, 12, 14), 6)
    assert p[:6].all() and not p[6:].any()
    c = W.fixture_plate_clamps(96)
    assert c[:6].all() and c[6:12, :, :4].all() and not c[6:12, :, 10:80].any()


def test_serving_stream():
    s = W.serving_stream(16)
    assert len(s) == 16 and all(6 <= len(r["dir_index"]) <= 130 for r in s)
    assert all(s[i]["t"] < s[i + 1]["t"] for i in range(15))
