"""Pins of the CPU oracle against things other than itself: closed forms,
invariants the paper states, and brute force on tiny grids."""
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import (TOOL_BALL, TOOL_FLAT, TOOL_RECT2D, circle8, fixture_plate,
                       lattice26, tool)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gauss_counts():
    out = {}
    for line in open(os.path.join(GOLD, "gauss_circle.txt")):
        if line.startswith("#") or not line.strip():
            continue
        r, c = line.split()
        out[int(r)] = int(c)
    return out


def offsets_set(offs):
    return set(map(tuple, np.asarray(offs).tolist()))


# ---------------------------------------------------------------------------
# rasterizer
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("r", [3, 4, 10, 12, 14])
def test_raster_axis_slices_match_gauss_circle(r):
    """Each slice of an axis-aligned flat cutter is a lattice disc (Gauss circle)."""
    gc = gauss_counts()
    L = 7
    for d, kind in [((0, 0, 1), 1), ((0, 0, 1.0), 0), ((1, 0, 0), 1), ((0, -1, 0), 1)]:
        dd = np.array(d, dtype=np.int32 if kind == 1 else np.float64)
        offs, cut = oracle.raster(tool(TOOL_FLAT, r, L, 0, 0), dd, kind)
        assert cut.all()
        assert len(offs) == gc[r] * L
        ax = int(np.nonzero(np.asarray(d))[0][0])
        sgn = int(np.sign(np.asarray(d)[ax]))
        vals, counts = np.unique(offs[:, ax] * sgn, return_counts=True)
        assert list(vals) == list(range(L)) and (counts == gc[r]).all()


@pytest.mark.parametrize("kind", [0, 1])
def test_raster_totals_of_the_workload_tools(kind):
    """Axis-aligned voxel totals of the three tools of the 3D workloads.

    Flat r3 L40: 29*40 = 1160; holder r10 L40: 317*40 = 12680.  Ball r4 L60:
    cylinder 49*56 = 2744 plus the lower half-ball slices 45+37+21+1 = 104 ->
    2848; holder r14 L60: 613*60 = 36780.  Flat r3 L80: 2320; holder r12 L80:
    441*80 = 35280."""
    d = np.array([0, 0, 1], dtype=np.int32 if kind == 1 else np.float64)
    for tl, nk, nh in [(tool(TOOL_FLAT, 3, 40, 10, 40), 1160, 12680),
                       (tool(TOOL_BALL, 4, 60, 14, 60), 2848, 36780),
                       (tool(TOOL_FLAT, 3, 80, 12, 80), 2320, 35280)]:
        offs, cut = oracle.raster(tl, d, kind)
        assert cut.sum() == nk and len(offs) - cut.sum() == nh


def test_raster_ball_end_lowest_point_is_origin():
    offs, cut = oracle.raster(tool(TOOL_BALL, 4, 60, 14, 60), np.array([0, 0, 1], np.int32))
    assert offs[:, 2].min() == 0
    assert offsets_set(offs[offs[:, 2] == 0]) == {(0, 0, 0)}


def test_raster_2d_rectangles():
    """C1 tool along +y: cutter 3 x 24 and holder 9 x 30 (half-open axial test)."""
    offs, cut = oracle.raster(tool(TOOL_RECT2D, 1.5, 24, 4.5, 30), np.array([0, 1], np.int32))
    assert cut.sum() == 3 * 24 and len(offs) == 3 * 24 + 9 * 30
    k = offs[cut]
    assert set(k[:, 0]) == {-1, 0, 1} and k[:, 1].min() == 0 and k[:, 1].max() == 23
    h = offs[~cut]
    assert h[:, 1].min() == 24 and h[:, 1].max() == 53 and set(h[:, 0]) == set(range(-4, 5))


def test_raster_antipodal_symmetry_lattice():
    """raster(-v) = -raster(v) for every lattice direction (exact integer forms)."""
    for tl in [tool(TOOL_FLAT, 3, 40, 10, 40), tool(TOOL_BALL, 4, 20, 6, 10)]:
        for v in lattice26():
            a, ca = oracle.raster(tl, v)
            b, cb = oracle.raster(tl, -v)
            assert offsets_set(a) == offsets_set(-b)
            assert offsets_set(a[ca]) == offsets_set(-b[cb])


def test_raster_axis_permutation_symmetry_lattice():
    """Permuting the axes of v permutes the raster."""
    tl = tool(TOOL_BALL, 3, 12, 5, 6)
    for v in [(1, 1, 0), (1, 1, 1), (0, 1, -1), (1, 0, 0)]:
        v = np.array(v, np.int32)
        a, _ = oracle.raster(tl, v)
        for perm in [(1, 2, 0), (2, 0, 1), (1, 0, 2)]:
            b, _ = oracle.raster(tl, v[list(perm)])
            assert offsets_set(a[:, list(perm)]) == offsets_set(b)


def test_raster_lattice_matches_exact_rational_brute_force():
    for tl in [tool(TOOL_FLAT, 1.5, 5, 3, 4), tool(TOOL_BALL, 2, 6, 3.5, 3)]:
        for v in lattice26()[::3]:
            T, K = brute.raster(tl, v)
            offs, cut = oracle.raster(tl, v)
            assert offsets_set(offs) == set(T)
            assert offsets_set(offs[cut]) == set(K)
    for v in circle8():
        tl = tool(TOOL_RECT2D, 1.5, 6, 2.5, 4)
        T, K = brute.raster(tl, v)
        offs, cut = oracle.raster(tl, v)
        assert {p[:2] for p in offsets_set(offs)} == {p[:2] for p in T}


def test_raster_float_axis_equals_lattice_axis():
    tl = tool(TOOL_BALL, 4, 60, 14, 60)
    for ax in range(3):
        for s in (1, -1):
            v = np.zeros(3, np.int32)
            v[ax] = s
            a, ca = oracle.raster(tl, v, 1)
            b, cb = oracle.raster(tl, v.astype(np.float64), 0)
            assert offsets_set(a) == offsets_set(b) and ca.sum() == cb.sum()


def test_raster_rejects_bad_input():
    with pytest.raises(ValueError):
        oracle.raster(tool(TOOL_FLAT, 3, 40, 10, 40), np.array([0, 0, 1.1]), 0)
    with pytest.raises(ValueError):
        oracle.raster(tool(TOOL_RECT2D, 1.5, 4, 3, 3), np.array([0, 0, 1], np.int32), 1)
    with pytest.raises(ValueError):   # lattice mode needs half-integer sizes
        oracle.raster(tool(TOOL_FLAT, 3.3, 40, 10, 40), np.array([0, 0, 1], np.int32), 1)


# ---------------------------------------------------------------------------
# overlap (collision measure) closed forms
# ---------------------------------------------------------------------------

def _interval_overlap(a0, a1, b0, b1):
    return max(0, min(a1, b1) - max(a0, b0))


def test_overlap_box_design_rect_tool_closed_form():
    """Box design x rectangle-union tool: g is a sum of products of 1D interval
    overlaps (Eq. ident as vol[O n (t + T)])."""
    n = 40
    d = np.zeros((n, n), np.uint8)
    bx0, bx1, by0, by1 = 7, 19, 11, 30
    d[by0:by1, bx0:bx1] = 1
    tl = tool(TOOL_RECT2D, 1.5, 6, 3.5, 5)   # cutter x in [-1,1], y in [0,6); holder x in [-3,3], y in [6,11)
    req = oracle.Request(d, tools=tl, dirs=np.array([[0, 1]], np.int32), dir_kind=1)
    g, lo = oracle.overlap_full(req, 0)
    rects = [(-1, 2, 0, 6), (-3, 4, 6, 11)]
    for ty in range(g.shape[1]):
        for tx in range(g.shape[2]):
            t = (tx + lo[0], ty + lo[1])
            exp = sum(_interval_overlap(t[0] + x0, t[0] + x1, bx0, bx1) *
                      _interval_overlap(t[1] + y0, t[1] + y1, by0, by1)
                      for (x0, x1, y0, y1) in rects)
            assert g[0, ty, tx] == exp


def test_overlap_sum_rule_and_minkowski_support():
    """sum_t g(t) = (sum rho_O) |T|, and {g > 0} = O (+) (-T) exactly."""
    rng = np.random.default_rng(3)
    d = (rng.random((12, 13, 14)) < 0.2).astype(np.uint8)
    tl = tool(TOOL_BALL, 2, 6, 3, 3)
    for v in [(0, 0, 1), (1, 1, 1), (-1, 0, 1)]:
        req = oracle.Request(d, tools=tl, dirs=np.array([v], np.int32), dir_kind=1)
        g, lo = oracle.overlap_full(req, 0)
        offs, _ = oracle.raster(tl, np.array(v, np.int32))
        assert g.sum() == int(d.sum()) * len(offs)
        occ = np.argwhere(d)[:, ::-1]   # (x, y, z)
        mink = {tuple(p - o) for p in occ for o in offs}
        got = {(x + lo[0], y + lo[1], z + lo[2]) for z, y, x in np.argwhere(g > 0)}
        assert got == mink


def test_single_voxel_tool_gives_rho():
    """A one-voxel tool: g = rho_O and f = rho_O (with fixture union as max)."""
    rng = np.random.default_rng(5)
    d = (rng.integers(0, 1 << 24, size=(9, 10, 11)) / float(1 << 24)).astype(np.float32)
    fx = fixture_plate(d.shape, 2)
    tl = tool(TOOL_FLAT, 0.5, 0.5, 0, 0)
    offs, _ = oracle.raster(tl, np.array([0, 0, 1], np.int32))
    assert offsets_set(offs) == {(0, 0, 0)}
    req = oracle.Request(d, fx, tools=tl, dirs=np.array([[0, 0, 1]], np.int32), dir_kind=1)
    out = oracle.imf(req, masks=False)
    rho_o = np.where(fx > 0, 1.0, d.astype(np.float64))
    assert np.array_equal(out["imf"], rho_o)


def test_pointwise_gamma_matches_brute_force():
    """gamma at single voxels (the sampled checks at full size) against the
    literal brute force: its minimum over orientations is f, and gamma <= 0
    is the accessible mask of each orientation (lambda = 0)."""
    rng = np.random.default_rng(21)
    d = (rng.random((7, 8, 9)) < 0.3).astype(np.uint8)
    fx = fixture_plate(d.shape, 1)
    tl = tool(TOOL_FLAT, 1, 3, 2, 2)
    dirs = lattice26()[::3]
    b = brute.imf(d.astype(np.int64), fx, tl, dirs)
    req = oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1)
    zz, yy, xx = np.meshgrid(np.arange(7), np.arange(8), np.arange(9), indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    gam = oracle.gamma_at_all(req, pts)
    assert np.array_equal(gam.min(0), b["imf"].ravel())
    om = (fx == 0).ravel()
    assert np.array_equal((gam <= 0) & om, b["masks"].reshape(len(dirs), -1))
    assert np.array_equal(oracle.gamma_at(req, 3, pts[::5]), gam[3, ::5])


# ---------------------------------------------------------------------------
# full IMF against brute force
# ---------------------------------------------------------------------------

def _compare_with_brute(d, fx, tl, dirs, lam=0.0, scale=1):
    b = brute.imf((np.asarray(d, np.float64) * scale).astype(np.int64), fx, tl, dirs,
                  lam=lam, scale=scale)
    req = oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1, lam=lam,
                         density=(scale != 1))
    o = oracle.imf(req)
    nx = req.nx
    assert np.array_equal(o["imf"] * scale, b["imf"].astype(np.float64))
    assert o["F_max"] * scale == b["F_max"]
    assert np.array_equal(o["imf_norm"], b["imf_norm"])
    assert np.array_equal(o["secluded"].astype(bool), b["secluded"])
    m = oracle.unpack_masks(o["masks"], nx).reshape(b["masks"].shape)
    md = oracle.unpack_masks(o["masks_dil"], nx).reshape(b["masks"].shape)
    assert np.array_equal(m, b["masks"])
    assert np.array_equal(md, b["masks"])
    return o


def test_oracle_equals_brute_force_3d_binary():
    rng = np.random.default_rng(11)
    d = (rng.random((8, 8, 8)) < 0.25).astype(np.uint8)
    fx = fixture_plate(d.shape, 2)
    _compare_with_brute(d, fx, tool(TOOL_FLAT, 1, 3, 2, 2), lattice26()[::2])


def test_oracle_equals_brute_force_2d_binary():
    rng = np.random.default_rng(12)
    d = (rng.random((12, 12)) < 0.3).astype(np.uint8)
    fx = fixture_plate(d.shape, 2)
    _compare_with_brute(d, fx, tool(TOOL_RECT2D, 1.5, 4, 2.5, 3), circle8())


def test_oracle_equals_brute_force_2d_density_with_allowance():
    rng = np.random.default_rng(13)
    d = (rng.integers(0, (1 << 24) + 1, size=(12, 12)) / float(1 << 24)).astype(np.float32)
    fx = fixture_plate(d.shape, 1)
    _compare_with_brute(d, fx, tool(TOOL_RECT2D, 1.5, 4, 2.5, 3), circle8(), lam=0.05,
                        scale=1 << 24)


def test_oracle_equals_brute_force_ball_tool():
    rng = np.random.default_rng(14)
    d = (rng.random((7, 8, 9)) < 0.2).astype(np.uint8)
    _compare_with_brute(d, None, tool(TOOL_BALL, 1.5, 4, 2, 2), lattice26()[1::3])


# ---------------------------------------------------------------------------
# invariants stated by the paper
# ---------------------------------------------------------------------------

def _req3(d, fx=None, dirs=None, tl=None, **kw):
    tl = tl or tool(TOOL_FLAT, 1.5, 5, 3, 4)
    dirs = lattice26() if dirs is None else dirs
    return oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1, **kw)


def test_empty_design_is_fully_accessible():
    d = np.zeros((10, 11, 12), np.uint8)
    o = oracle.imf(_req3(d))
    assert (o["imf"] == 0).all() and o["F_max"] == 0 and (o["imf_norm"] == 0).all()
    assert not o["secluded"].any()
    m = oracle.unpack_masks(o["masks"], 12)
    assert m.all()


def test_imf_bounds_and_part_is_inaccessible():
    """f >= rho_O (the sharp point itself lies in the tool), so Omega is in B and
    never accessible; fbar in [0, 1] with maximum exactly 1."""
    rng = np.random.default_rng(21)
    d = (rng.random((10, 10, 10)) < 0.3).astype(np.uint8)
    fx = fixture_plate(d.shape, 2)
    o = oracle.imf(_req3(d, fx))
    rho_o = np.maximum(d, fx)
    assert (o["imf"] >= rho_o).all()
    part = (d > 0) & (fx == 0)
    assert (o["imf"][part] > 0).all()
    m = oracle.unpack_masks(o["masks"], 10)
    assert not (m & part[None]).any()
    nb = o["imf_norm"]
    assert nb.min() >= 0 and nb.max() == 1.0
    assert not (o["secluded"].astype(bool) & (d > 0)).any()


def test_masks_union_is_complement_of_B():
    """union_R A_R = Omega_0 minus B (Algorithm 1 classification vs Eq. A)."""
    rng = np.random.default_rng(22)
    d = (rng.random((10, 10, 10)) < 0.3).astype(np.uint8)
    fx = fixture_plate(d.shape, 2)
    o = oracle.imf(_req3(d, fx))
    acc = oracle.unpack_masks(o["masks"], 10).any(axis=0)
    B = (fx == 0) & (o["imf"] > 0)
    assert np.array_equal(acc, (fx == 0) & ~B)
    assert np.array_equal(o["secluded"].astype(bool), B & (d == 0))


def test_more_orientations_never_increase_imf():
    rng = np.random.default_rng(23)
    d = (rng.random((10, 10, 10)) < 0.3).astype(np.uint8)
    dirs = lattice26()
    prev = None
    prev_acc = None
    for k in (3, 9, 18, 26):
        o = oracle.imf(_req3(d, dirs=dirs[:k]))
        acc = oracle.unpack_masks(o["masks"], 10).any(axis=0)
        if prev is not None:
            assert (o["imf"] <= prev).all()
            assert (acc >= prev_acc).all()
        prev, prev_acc = o["imf"], acc


def test_more_sharp_points_never_increase_imf():
    """Sec. 2.1.5: sampling the cutter more densely can only lower the IMF
    (tip subset of boundary subset of all cutter voxels)."""
    rng = np.random.default_rng(24)
    d = (rng.random((10, 10, 10)) < 0.3).astype(np.uint8)
    f = {s: oracle.imf(_req3(d, sharp=s), masks=False)["imf"] for s in (0, 1, 2)}
    assert (f[0] <= f[1]).all() and (f[1] <= f[2]).all()
    assert (f[0] < f[2]).any()


def test_adding_material_never_decreases_imf():
    rng = np.random.default_rng(25)
    d = (rng.random((10, 10, 10)) < 0.2).astype(np.uint8)
    d2 = d | (rng.random(d.shape) < 0.1).astype(np.uint8)
    f1 = oracle.imf(_req3(d), masks=False)["imf"]
    f2 = oracle.imf(_req3(d2), masks=False)["imf"]
    assert (f2 >= f1).all()


def test_translation_equivariance():
    rng = np.random.default_rng(26)
    core = (rng.random((6, 6, 6)) < 0.4).astype(np.uint8)
    a = np.zeros((14, 14, 14), np.uint8)
    b = np.zeros_like(a)
    a[3:9, 4:10, 2:8] = core
    b[5:11, 4:10, 5:11] = core          # shift (dx, dy, dz) = (3, 0, 2)
    fa = oracle.imf(_req3(a), masks=False)["imf"]
    fb = oracle.imf(_req3(b), masks=False)["imf"]
    assert np.array_equal(fa[:-2, :, :-3], fb[2:, :, 3:])


def test_density_imf_is_between_binary_thresholds():
    """Scaling a binary design by a density c in (0, 1] scales f exactly by c."""
    rng = np.random.default_rng(27)
    d = (rng.random((9, 9, 9)) < 0.3).astype(np.uint8)
    c = 0.375   # on the 2^-24 grid
    fb = oracle.imf(_req3(d), masks=False)["imf"]
    fd = oracle.imf(_req3((d * c).astype(np.float32)), masks=False)["imf"]
    assert np.array_equal(fd, fb * c)


# ---------------------------------------------------------------------------
# accessibility closed forms
# ---------------------------------------------------------------------------

def test_slot_depth_closed_form_2d():
    """A 5-wide slot of depth 20 in a solid block, tool from above (d = +y):
    the 3-wide cutter fits, the 9-wide holder stops at the top face, so slot
    voxels are reachable exactly down to L = 8 below the top."""
    nx, ny = 40, 60
    d = np.zeros((ny, nx), np.uint8)
    d[:40, :] = 1
    d[20:40, 18:23] = 0
    tl = tool(TOOL_RECT2D, 1.5, 8, 4.5, 10)
    req = oracle.Request(d, tools=tl, dirs=np.array([[0, 1]], np.int32), dir_kind=1)
    o = oracle.imf(req)
    acc = oracle.unpack_masks(o["masks"], nx)[0, 0]
    yy, xx = np.mgrid[0:ny, 0:nx]
    slot = (yy >= 20) & (yy < 40) & (xx >= 18) & (xx < 23)
    expect = (yy >= 40) | (slot & (yy >= 32))
    assert np.array_equal(acc, expect)
    assert np.array_equal(o["secluded"].astype(bool), slot & (yy < 32))


def test_pocket_corners_closed_form_3d():
    """A 5x5 square pocket entered from above by a radius-1 flat cutter (a plus
    shaped raster): the pocket's 4 corner columns are never touched, and the
    reachable depth is L below the top face."""
    n = 20
    d = np.zeros((n + 12, n, n), np.uint8)
    d[:16] = 1
    c = 10
    d[4:16, c - 2:c + 3, c - 2:c + 3] = 0
    tl = tool(TOOL_FLAT, 1, 5, 4, 6)
    req = oracle.Request(d, tools=tl, dirs=np.array([[0, 0, 1]], np.int32), dir_kind=1)
    o = oracle.imf(req)
    acc = oracle.unpack_masks(o["masks"], n)[0]
    zz, yy, xx = np.mgrid[0:n + 12, 0:n, 0:n]
    pocket = (zz >= 4) & (zz < 16) & (abs(xx - c) <= 2) & (abs(yy - c) <= 2)
    corner = (abs(xx - c) == 2) & (abs(yy - c) == 2)
    expect = (zz >= 16) | (pocket & (zz >= 11) & ~corner)
    assert np.array_equal(acc, expect)


def test_sealed_cavity_is_secluded_and_large_cavity_is_not():
    """A closed shell: a cavity smaller than the tool is secluded in every
    orientation.  A cavity that holds the whole tool is reported accessible:
    the measure has no path-connectedness test (Sec. 4 limitation)."""
    tl = tool(TOOL_FLAT, 1, 3, 1, 2)   # whole tool fits a 3x3x5 box
    small = np.ones((12, 12, 12), np.uint8)
    small[5:8, 5:8, 5:7] = 0
    o = oracle.imf(_req3(small, tl=tl))
    cav = small == 0
    assert o["secluded"].astype(bool)[cav].all()
    big = np.ones((20, 20, 20), np.uint8)
    big[4:16, 4:16, 4:16] = 0
    o = oracle.imf(_req3(big, tl=tl))
    cav = big == 0
    acc = oracle.unpack_masks(o["masks"], 20).any(axis=0)
    zz, yy, xx = np.mgrid[0:20, 0:20, 0:20]
    inner = (zz >= 8) & (zz < 12) & (yy >= 8) & (yy < 12) & (xx >= 8) & (xx < 12)
    assert acc[inner].all() and not o["secluded"].astype(bool)[inner].any()
    assert cav[inner].all()


def test_fixture_blocks_tools_from_below():
    """With a fixture plate at the bottom, a tool coming from below (d = -z)
    collides with it unless the whole tool clears the plate."""
    d = np.zeros((16, 10, 10), np.uint8)
    fx = fixture_plate(d.shape, 3)
    tl = tool(TOOL_FLAT, 1, 3, 2, 3)
    req = oracle.Request(d, fx, tools=tl, dirs=np.array([[0, 0, -1], [0, 0, 1]], np.int32),
                         dir_kind=1)
    o = oracle.imf(req)
    m = oracle.unpack_masks(o["masks"], 10)
    # tip + cutter + holder span 6 slices below the touched voxel's tip: a voxel
    # is reachable from below only if the lowest tool slice clears z = 3
    assert not m[0, 3:6].any() and m[0, 6:].all()
    assert m[1, 3:].all()               # from above everything off the plate
    assert not m[:, :3].any()           # fixture voxels are outside Omega_0


# ---------------------------------------------------------------------------
# voxel-model tools: inverse nearest-neighbour re-sampling under a rotation
# ---------------------------------------------------------------------------

def _label_offsets(t):
    lab = t["labels"]
    z, y, x = np.nonzero(lab)
    o = t["origin"]
    return {(int(a) - o[0], int(b) - o[1], int(c) - o[2]): int(lab[c, b, a])
            for a, b, c in zip(x, y, z)}


def test_voxel_tool_identity_and_cube_rotations_are_exact():
    from workloads import asymmetric_tool, cube_rotations
    t = asymmetric_tool()
    ref = _label_offsets(t)
    for R in [np.eye(3)] + list(cube_rotations()):
        offs, cut = oracle.raster(t, R)
        got = {tuple(p): 2 if c else 1 for p, c in zip(offs.tolist(), cut)}
        # R maps the tool-frame offset p to the grid offset R p exactly
        want = {tuple(int(v) for v in np.rint(R @ np.array(p, float))): lab
                for p, lab in ref.items()}
        assert got == want


def test_voxelized_tool_rotated_onto_axes_equals_the_analytic_raster():
    from workloads import voxel_tool, rotation_to
    tl = tool(TOOL_FLAT, 1.5, 6, 3, 5)
    offs, cut = oracle.raster(tl, np.array([0, 0, 1], np.int32))
    lo = offs.min(0)
    dims = offs.max(0) - lo + 1
    lab = np.zeros(dims[::-1], np.uint8)
    lab[offs[:, 2] - lo[2], offs[:, 1] - lo[1], offs[:, 0] - lo[0]] = np.where(cut, 2, 1)
    vt = voxel_tool(lab, -lo)
    for d in ([1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]):
        R = np.rint(rotation_to(np.array(d, float)))
        a_offs, a_cut = oracle.raster(tl, np.array(d, np.int32))
        v_offs, v_cut = oracle.raster(vt, R)
        assert {tuple(p): c for p, c in zip(a_offs.tolist(), a_cut)} == \
               {tuple(p): c for p, c in zip(v_offs.tolist(), v_cut)}, d


def test_voxel_tool_imf_equals_analytic_on_axis_directions():
    """End to end: the voxelized flat tool under the 6 axis rotations gives the
    same IMF and masks as the analytic tool along the 6 lattice axes."""
    from workloads import voxel_tool, rotation_to
    rng = np.random.default_rng(77)
    d = (rng.random((10, 11, 12)) < 0.3).astype(np.uint8)
    fx = fixture_plate(d.shape, 1)
    tl = tool(TOOL_FLAT, 1, 3, 2, 2)
    offs, cut = oracle.raster(tl, np.array([0, 0, 1], np.int32))
    lo = offs.min(0)
    lab = np.zeros((offs.max(0) - lo + 1)[::-1], np.uint8)
    lab[offs[:, 2] - lo[2], offs[:, 1] - lo[1], offs[:, 0] - lo[0]] = np.where(cut, 2, 1)
    vt = voxel_tool(lab, -lo)
    axes = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.int32)
    rots = np.stack([np.rint(rotation_to(a.astype(float))) for a in axes])
    a = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=axes, dir_kind=1))
    v = oracle.imf(oracle.Request(d, fx, tools=vt, dirs=rots, dir_kind=2))
    for k in ("imf", "imf_norm", "secluded", "masks", "masks_dil"):
        assert np.array_equal(a[k], v[k]), k


def test_voxel_tool_random_rotations_keep_the_volume():
    from workloads import asymmetric_tool, random_rotations
    t = asymmetric_tool()
    n = int(np.count_nonzero(t["labels"]))
    for R in random_rotations(12, 5):
        offs, cut = oracle.raster(t, R)
        assert abs(len(offs) - n) <= 0.2 * n
        assert cut.any() and (~cut).any()
    with pytest.raises(ValueError):
        oracle.raster(t, np.diag([1.0, 1.0, -1.0]))        # a reflection, not a rotation


# ---------------------------------------------------------------------------
# fixtures that change with the setup
# ---------------------------------------------------------------------------

def test_fixture_sets_equal_brute_force():
    rng = np.random.default_rng(91)
    d = (rng.random((7, 8, 9)) < 0.3).astype(np.uint8)
    fx = fixture_plate(d.shape, 1)
    sets = np.zeros((2,) + d.shape, np.uint8)
    sets[0][:, :, :2] = 1          # a clamp on the low-x side
    sets[1][:, :2, :] = 1          # a clamp on the low-y side
    tl = tool(TOOL_FLAT, 1, 3, 2, 2)
    dirs = lattice26()[::4]
    fof = np.array([0, 0, 1, 1, 0, 1, 1][:len(dirs)], np.int32)
    b = brute.imf(d.astype(np.int64), fx, tl, dirs, fixture_sets=sets, fixture_of=fof)
    o = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1, fixture_sets=sets,
                                  fixture_of=fof))
    assert np.array_equal(o["imf"], b["imf"].astype(np.float64))
    assert np.array_equal(o["secluded"].astype(bool), b["secluded"])
    m = oracle.unpack_masks(o["masks"], 9).reshape(b["masks"].shape)
    assert np.array_equal(m, b["masks"])
    assert np.array_equal(oracle.unpack_masks(o["masks_dil"], 9).reshape(b["masks"].shape),
                          b["masks"])
    # the design domain excludes every setup's fixture
    assert not o["imf_norm"][sets.any(0) != 0].any()


def test_identical_fixture_sets_reduce_to_one_fixture():
    rng = np.random.default_rng(92)
    d = (rng.random((8, 9, 10)) < 0.3).astype(np.uint8)
    fx = fixture_plate(d.shape, 2)
    tl = tool(TOOL_FLAT, 1, 3, 2, 2)
    dirs = lattice26()[::3]
    a = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1))
    sets = np.stack([fx, fx, fx])
    fof = np.arange(len(dirs)) % 3
    b = oracle.imf(oracle.Request(d, None, tools=tl, dirs=dirs, dir_kind=1, fixture_sets=sets,
                                  fixture_of=fof))
    for k in ("imf", "imf_norm", "secluded", "masks"):
        assert np.array_equal(a[k], b[k]), k


# ---------------------------------------------------------------------------
# float64 raster at oblique directions (the path of every Fibonacci request)
# ---------------------------------------------------------------------------

def _grid_of(offs, sel, lo, shape):
    g = np.zeros(shape, bool)
    o = offs[sel]
    g[o[:, 2] - lo[2], o[:, 1] - lo[1], o[:, 0] - lo[0]] = True
    return g


@pytest.mark.parametrize("tl", [tool(TOOL_BALL, 4, 60, 14, 60), tool(TOOL_FLAT, 3, 40, 10, 40),
                                tool(TOOL_FLAT, 3, 80, 12, 80)])
def test_raster_f64_oblique_equals_exact_lattice_up_to_ties(tl):
    """The float64 predicate at d = v / |v| against an independent exact integer
    evaluation of the raster definition (Algorithm 1, Rotate; reading of the
    analytic raster) for oblique lattice vectors v: the two agree at every
    offset where no boundary test holds with equality, and the oracle's own
    exact lattice mode agrees with the independent one everywhere."""
    for v in [(1, 1, 1), (1, 2, 2), (2, -1, 1), (1, -2, 3), (0, 1, 2), (-3, 1, 2)]:
        v = np.array(v)
        offs, cut = oracle.raster(tl, v / np.sqrt(float((v * v).sum())), 0)
        lo, hi = offs.min(0) - 2, offs.max(0) + 2
        T, K, tie = brute.raster_exact_box(tl, v, lo, hi)
        F = _grid_of(offs, slice(None), lo, T.shape)
        Fk = _grid_of(offs, cut, lo, T.shape)
        diff = (F != T) | (Fk != K)
        assert not (diff & ~tie).any(), (v, int((diff & ~tie).sum()))
        assert diff.sum() <= max(2, T.sum() // 200)
        lo2, cut2 = oracle.raster(tl, v.astype(np.int32), 1)
        assert np.array_equal(_grid_of(lo2, slice(None), lo, T.shape), T)
        assert np.array_equal(_grid_of(lo2, cut2, lo, T.shape), K)


@pytest.mark.parametrize("tl,n", [(tool(TOOL_BALL, 4, 60, 14, 60), 130),
                                  (tool(TOOL_FLAT, 3, 80, 12, 80), 512)])
def test_raster_f64_fibonacci_equals_extended_precision(tl, n):
    """Fibonacci-hemisphere directions (no lattice form): the float64 raster
    equals the same definition evaluated in extended precision at every offset
    more than 1e-9 from a boundary of the predicate."""
    from workloads import fib_hemisphere
    dirs = fib_hemisphere(n)
    for q in (0, 1, 5, n // 3, n // 2, n - 2, n - 1):
        offs, cut = oracle.raster(tl, dirs[q], 0)
        lo, hi = offs.min(0) - 2, offs.max(0) + 2
        T, K, near = brute.raster_margin_box(tl, dirs[q], lo, hi)
        F = _grid_of(offs, slice(None), lo, T.shape)
        Fk = _grid_of(offs, cut, lo, T.shape)
        diff = (F != T) | (Fk != K)
        assert not (diff & ~near).any(), q
        # the box holds the whole raster (two voxels of margin on each side)
        assert not T[[0, -1]].any() and not T[:, [0, -1]].any() and not T[..., [0, -1]].any()


def test_raster_extended_reference_catches_a_dropped_term():
    """The extended-precision reference is sensitive to the predicate: a radial
    distance that drops the z term of o - a d disagrees with it far from any
    boundary (a mistake the comparison above would flag)."""
    tl = tool(TOOL_FLAT, 3, 40, 10, 40)
    d = np.array([1.0, 2.0, 2.0]) / 3.0
    offs, _ = oracle.raster(tl, d, 0)
    lo, hi = offs.min(0) - 2, offs.max(0) + 2
    T, _, near = brute.raster_margin_box(tl, d, lo, hi)
    z, y, x = np.meshgrid(*(np.arange(lo[a], hi[a] + 1) for a in (2, 1, 0)), indexing="ij")
    a = x * d[0] + y * d[1] + z * d[2]
    q2_wrong = (x - a * d[0]) ** 2 + (y - a * d[1]) ** 2
    wrong = ((a >= 0) & (a < 40) & (q2_wrong <= 9)) | ((a >= 40) & (a < 80) & (q2_wrong <= 100))
    assert ((wrong != T) & ~near).sum() > 1000


# ---------------------------------------------------------------------------
# several tools (Eq. imf_3: the minimum over tools and their orientations)
# ---------------------------------------------------------------------------

def test_two_tools_equal_the_minimum_of_single_tool_brute_force():
    """Binary, lambda = 0: f of tools [t1, t2] is the element-wise minimum of
    the single-tool brute-force IMFs, the masks are theirs concatenated, and
    B, fbar and Gamma follow from that minimum."""
    rng = np.random.default_rng(31)
    d = (rng.random((8, 9, 10)) < 0.3).astype(np.uint8)
    fx = fixture_plate(d.shape, 1)
    t1, t2 = tool(TOOL_FLAT, 1, 3, 2, 2), tool(TOOL_BALL, 1.5, 4, 2, 2)
    D1, D2 = lattice26()[::4], lattice26()[1::5]
    both = oracle.imf(oracle.Request(d, fx, tools=[t1, t2], dirs=[D1, D2], dir_kind=1))
    b1 = brute.imf(d.astype(np.int64), fx, t1, D1)
    b2 = brute.imf(d.astype(np.int64), fx, t2, D2)
    f = np.minimum(b1["imf"], b2["imf"])
    assert np.array_equal(both["imf"], f.astype(np.float64))
    om = fx == 0
    fmax = int(f[om].max())
    assert both["F_max"] == fmax
    B = om & (f > 0)
    assert np.array_equal(both["secluded"].astype(bool), B & (d == 0))
    assert np.array_equal(both["imf_norm"], np.where(B, f / fmax, 0).astype(np.float32))
    m = oracle.unpack_masks(both["masks"], d.shape[2])
    assert np.array_equal(m, np.concatenate([b1["masks"], b2["masks"]]))


def test_two_tools_density_with_allowance_threshold_of_the_joint_maximum():
    """Density, lambda > 0: the masks of a two-tool request use lambda times the
    joint F_max (the maximum of the minimum over both tools), not either
    tool's own; checked against the brute-force gammas of each tool."""
    rng = np.random.default_rng(32)
    Q = 1 << 24
    d = (rng.integers(0, Q + 1, size=(7, 8, 9)) / float(Q)).astype(np.float32)
    fx = fixture_plate(d.shape, 1)
    t1, t2 = tool(TOOL_FLAT, 1, 3, 2, 2), tool(TOOL_BALL, 1.5, 3, 2, 2)
    D1, D2 = lattice26()[2::5], lattice26()[::6]
    lam = 0.3
    both = oracle.imf(oracle.Request(d, fx, tools=[t1, t2], dirs=[D1, D2], dir_kind=1,
                                     lam=lam))
    di = (d.astype(np.float64) * Q).astype(np.int64)
    g = np.concatenate([brute.imf(di, fx, t1, D1, scale=Q)["gammas"],
                        brute.imf(di, fx, t2, D2, scale=Q)["gammas"]])
    f = g.min(0)
    om = fx == 0
    fmax = int(f[om].max())
    assert both["F_max"] * Q == fmax
    theta = lam * float(fmax)
    B = om & (f.astype(np.float64) > theta)
    assert np.array_equal(both["imf"] * Q, f.astype(np.float64))
    assert np.array_equal(both["imf_norm"], np.where(B, f / float(fmax), 0).astype(np.float32))
    m = oracle.unpack_masks(both["masks"], d.shape[2])
    assert np.array_equal(m, om[None] & (g.astype(np.float64) <= theta))
    assert np.array_equal(oracle.unpack_masks(both["masks_dil"], d.shape[2]), m)
    # the second tool's masks use the joint threshold, which differs from its own here
    assert fmax < int(g[len(D1):].min(0)[om].max())
