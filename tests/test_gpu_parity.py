"""GPU parity: the HIP library, called through its C interface, against the
CPU oracle on the same seeded inputs.

Bar: overlap counts, masks, f, fbar and Gamma bit-exact for binary designs;
density f within 1e-4 * max(|f_ref|, lambda * F_max_ref) per voxel (fbar
correspondingly), with F_max, B, Gamma and the masks bit-exact, whether the
masks' threshold is given or is lambda * F_max."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = imf.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def masks_u64(t):
    return host(t).view(np.uint64)


def random_boxes(shape, n, seed, lo=3, hi=12):
    rng = np.random.default_rng(seed)
    d = np.zeros(shape, np.uint8)
    for _ in range(n):
        c = [rng.integers(0, s) for s in shape]
        e = [rng.integers(lo, hi) for _ in shape]
        sl = tuple(slice(max(ci - ei // 2, 0), ci + ei - ei // 2) for ci, ei in zip(c, e))
        d[sl] = 1
    return d


def check_density(out, st, ref, lam, masks=True):
    """Density bar: f and fbar within the relative tolerance, F_max, B (fbar > 0),
    Gamma and the masks exact, and the float32 error model held."""
    fref = ref["imf"]
    f = host(out["imf"]).astype(np.float64).reshape(fref.shape)
    tol = 1e-4 * np.maximum(np.abs(fref), lam * ref["F_max"])
    assert (np.abs(f - fref) <= tol).all(), np.abs(f - fref).max()
    assert st.F_max == ref["F_max"], (st.F_max, ref["F_max"])
    nb = host(out["imf_norm"]).reshape(fref.shape)
    fbar = ref["imf_norm"].reshape(fref.shape)
    assert np.array_equal(nb > 0, fbar > 0), "B differs at %d voxels" % int(((nb > 0) != (fbar > 0)).sum())
    assert np.all(np.abs(nb.astype(np.float64) - fbar) <= 1e-4 * np.maximum(fbar, lam) + 1e-7)
    assert np.array_equal(host(out["secluded"]).reshape(fref.shape),
                          ref["secluded"].reshape(fref.shape))
    if masks:
        m = masks_u64(out["masks"])
        assert np.array_equal(m, ref["masks"].reshape(m.shape)), \
            "masks differ in %d words" % int((m != ref["masks"].reshape(m.shape)).sum())
    assert st.max_abs_err <= st.guard_band / 2


def check_binary(out, ref, n_orient=None):
    f = host(out["imf"]).astype(np.float64)
    assert np.array_equal(f, ref["imf"].reshape(f.shape)), \
        "f differs at %d voxels" % int((f != ref["imf"].reshape(f.shape)).sum())
    assert np.array_equal(host(out["imf_norm"]), ref["imf_norm"].reshape(f.shape))
    assert np.array_equal(host(out["secluded"]), ref["secluded"].reshape(f.shape))
    if "masks" in out:
        m = masks_u64(out["masks"])
        assert np.array_equal(m, ref["masks"].reshape(m.shape)), "masks differ"


# ---------------------------------------------------------------------------
# single steps
# ---------------------------------------------------------------------------

def test_raster_bit_exact(ctx):
    import paper_2002_07627_amd as imf
    cases = [(W.TOOL_C2, W.lattice26()), (W.TOOL_C3, W.fib_hemisphere(40)),
             (W.TOOL_C5, W.fib_hemisphere(512)[::37]), (W.TOOL_C1, W.circle8()),
             (W.tool(W.TOOL_BALL, 2.5, 9, 4, 7), W.lattice26())]
    for tl, dirs in cases:
        for d in dirs:
            kind = 1 if dirs.dtype.kind in "iu" else 0
            go, gf = ctx.raster(tl, d, kind)
            oo, oc = oracle.raster(tl, d, kind)
            a = {tuple(p): int(f) & 3 for p, f in zip(go.tolist(), gf)}
            b = {tuple(p): 1 | (2 if c else 0) for p, c in zip(oo.tolist(), oc)}
            assert a == b, (tl, d)
    # sharp subsets: tip and boundary of the cutter raster
    tl = W.tool(W.TOOL_BALL, 3, 12, 5, 6)
    for d in W.fib_hemisphere(10):
        oo, oc = oracle.raster(tl, d, 0)
        cut = {tuple(p) for p, c in zip(oo.tolist(), oc) if c}
        bnd = {p for p in cut if any((p[0] + e[0], p[1] + e[1], p[2] + e[2]) not in cut
                                     for e in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                                               (0, 0, 1), (0, 0, -1)])}
        go, gf = ctx.raster(tl, d, 0, sharp=imf.SHARP_BOUNDARY)
        assert {tuple(p) for p, f in zip(go.tolist(), gf) if f & 4} == bnd
        go, gf = ctx.raster(tl, d, 0, sharp=imf.SHARP_TIP)
        assert {tuple(p) for p, f in zip(go.tolist(), gf) if f & 4} == {(0, 0, 0)}


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7, 8, 12, 16, 48, 60, 105, 128, 216, 256, 384, 560,
                               576, 1024])
def test_fft_c2c_against_float64_dft(ctx, n):
    rng = np.random.default_rng(n)
    x = (rng.standard_normal((n, 37)) + 1j * rng.standard_normal((n, 37))).astype(np.complex64)
    ref = np.fft.fft(x.astype(np.complex128), axis=0)
    y = host(ctx.fft_c2c(dev(x)))
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err < 3e-7 * max(np.log2(n), 1) * 4, err
    yi = host(ctx.fft_c2c(dev(x), inverse=True))
    refi = np.fft.ifft(x.astype(np.complex128), axis=0) * n
    assert np.abs(yi - refi).max() / np.abs(refi).max() < 3e-7 * max(np.log2(n), 1) * 4


def test_fft_r2c_3d_against_numpy(ctx):
    rng = np.random.default_rng(9)
    x = rng.random((20, 22, 24)).astype(np.float32)
    P = (48, 40, 30)
    y = host(ctx.fft_r2c_3d(dev(x), P))
    xp = np.zeros((P[2], P[1], P[0]))
    xp[:20, :22, :24] = x
    ref = np.fft.rfftn(xp)                      # [pz][py][px/2+1]
    ref = np.transpose(ref, (1, 2, 0))          # [py][px/2+1][pz]
    assert np.abs(y - ref).max() / np.abs(ref).max() < 1e-6


# ---------------------------------------------------------------------------
# whole requests
# ---------------------------------------------------------------------------

def test_c1_direct_2d_bit_exact(ctx):
    import paper_2002_07627_amd as imf
    w = W.c1()
    out, st = ctx.compute(dev(w.design), dev(w.fixture), tools=w.tool, dirs=w.dirs,
                          dir_kind=imf.DIR_LATTICE, method=imf.METHOD_DIRECT)
    ref = oracle.imf(oracle.Request(w.design, w.fixture, tools=w.tool, dirs=w.dirs, dir_kind=1))
    check_binary(out, ref)
    assert st.method == imf.METHOD_DIRECT and st.F_max == ref["F_max"]


@pytest.mark.parametrize("method", ["fft", "direct"])
def test_small_3d_binary_bit_exact(ctx, method):
    import paper_2002_07627_amd as imf
    d = random_boxes((30, 34, 40), 14, 5)
    fx = W.fixture_plate(d.shape, 3)
    tl = W.tool(W.TOOL_FLAT, 1.5, 6, 3, 5)
    dirs = W.lattice26()
    m = imf.METHOD_FFT if method == "fft" else imf.METHOD_DIRECT
    req = oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1)
    ref = oracle.imf(req, debug_orient=7)
    info = oracle.orient_info(req, 7)
    box = [n + info["kmax"][a] - info["kmin"][a] for a, n in enumerate((40, 34, 30))]
    out, st = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE,
                          method=m, debug_orient=7, debug_numel=int(np.prod(box)))
    check_binary(out, ref)
    g = host(out["debug"]).reshape(box[2], box[1], box[0])
    assert np.array_equal(g.astype(np.int64), ref["g_debug"])
    assert tuple(out["debug_box"][:3]) == ref["debug_lo"]
    if method == "fft":
        assert st.max_frac_err < 0.05


def test_binary_deferred_appends_bit_exact(monkeypatch):
    """The inverse x pass with its guard-band appends written after its rows
    (IMF_DEFER_APPENDS=1): rounded overlaps, masks and F_max bit-exact, on a
    grid whose rows take full and partial 64-voxel chunks."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    monkeypatch.setenv("IMF_DEFER_APPENDS", "1")
    d = random_boxes((30, 34, 70), 16, 11)
    fx = W.fixture_plate(d.shape, 3)
    tl = W.tool(W.TOOL_FLAT, 1.5, 6, 3, 5)
    dirs = W.lattice26()
    c = imf.Context(0)
    try:
        out, st = c.compute(dev(d), dev(fx), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE,
                            method=imf.METHOD_FFT)
    finally:
        c.close()
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1))
    check_binary(out, ref)
    assert st.F_max == ref["F_max"] and st.max_frac_err < 0.05


def test_plain_batched_and_cached_are_identical(ctx):
    import paper_2002_07627_amd as imf
    d = random_boxes((32, 32, 32), 12, 6)
    tl = W.tool(W.TOOL_BALL, 2, 7, 3.5, 5)
    dirs = W.fib_hemisphere(20)
    kw = dict(tools=tl, dirs=dirs, dir_kind=imf.DIR_F64, method=imf.METHOD_FFT)
    a, sa = ctx.compute(dev(d), **kw, flags=imf.FLAG_PLAIN)
    b, sb = ctx.compute(dev(d), **kw, batch=8)
    c, sc = ctx.compute(dev(d), **kw, batch=5)
    assert sb.cache_misses == 20 and sc.cache_hits == 20
    for k in ("imf", "imf_norm", "secluded", "masks"):
        assert torch.equal(a[k], b[k]) and torch.equal(a[k], c[k]), k
    ref = oracle.imf(oracle.Request(d, None, tools=tl, dirs=dirs, dir_kind=0))
    check_binary(b, ref)


def test_sweep_route_equals_threshold_route(ctx):
    import paper_2002_07627_amd as imf
    d = random_boxes((28, 30, 33), 10, 7)
    fx = W.fixture_plate(d.shape, 2)
    tl = W.tool(W.TOOL_FLAT, 1.5, 6, 3, 5)
    dirs = W.lattice26()
    kw = dict(tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE, method=imf.METHOD_FFT)
    a, _ = ctx.compute(dev(d), dev(fx), **kw)
    b, _ = ctx.compute(dev(d), dev(fx), **kw, flags=imf.FLAG_MASK_SWEEP)
    assert torch.equal(a["masks"], b["masks"])
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1))
    assert np.array_equal(masks_u64(b["masks"]), ref["masks_dil"])


@pytest.mark.parametrize("sharp", [1, 2])
def test_sharp_point_subsets(ctx, sharp):
    import paper_2002_07627_amd as imf
    d = random_boxes((26, 28, 30), 10, 8)
    tl = W.tool(W.TOOL_FLAT, 1.5, 6, 3, 5)
    dirs = W.lattice26()[::2]
    out, _ = ctx.compute(dev(d), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE, sharp=sharp,
                         method=imf.METHOD_FFT)
    ref = oracle.imf(oracle.Request(d, None, tools=tl, dirs=dirs, dir_kind=1, sharp=sharp))
    check_binary(out, ref)


def test_two_tools_take_the_minimum(ctx):
    import paper_2002_07627_amd as imf
    d = random_boxes((26, 26, 26), 9, 9)
    t1 = W.tool(W.TOOL_FLAT, 1, 5, 3, 4)
    t2 = W.tool(W.TOOL_BALL, 1.5, 4, 2.5, 3)
    dirs1, dirs2 = W.lattice26()[:13], W.lattice26()[13:]
    out, st = ctx.compute(dev(d), tools=[t1, t2], dirs=[dirs1, dirs2],
                          dir_kind=imf.DIR_LATTICE, method=imf.METHOD_FFT)
    ref = oracle.imf(oracle.Request(d, None, tools=[t1, t2], dirs=[dirs1, dirs2], dir_kind=1))
    check_binary(out, ref)
    assert st.n_orient == 26


def test_density_within_tolerance_and_masks_exact(ctx):
    """Masks at a given threshold (decided by the first-pass recheck), B at
    lambda F_max (exact F_max, then the band around it)."""
    import paper_2002_07627_amd as imf
    d = W.design_density(36, seed=11)
    fx = W.fixture_plate(d.shape, 3)
    tl = W.tool(W.TOOL_BALL, 2, 8, 4, 6)
    dirs = W.fib_hemisphere(12)
    lam = 0.01
    ref0 = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam))
    theta = 0.5 * float(np.median(ref0["imf"]))
    out, st = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, dir_kind=imf.DIR_F64, lam=lam,
                          mask_theta_abs=theta, method=imf.METHOD_FFT)
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam,
                                    mask_theta_abs=theta))
    check_density(out, st, ref, lam)
    assert st.guard_flags > 0 and st.passes == 1


def test_density_two_phase_masks(ctx):
    """Masks and B at lambda F_max: F_max from the exact f of its candidates,
    the band around lambda F_max read from the stored overlaps."""
    import paper_2002_07627_amd as imf
    d = W.design_density(32, seed=12)
    fx = W.fixture_plate(d.shape, 3)
    tl = W.tool(W.TOOL_BALL, 2, 8, 4, 6)
    dirs = W.fib_hemisphere(10)
    lam = 0.05
    out, st = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, lam=lam, method=imf.METHOD_FFT)
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam))
    check_density(out, st, ref, lam)
    assert st.band_entries > 0 and st.post_exact > 0 and st.passes == 1
    # union of the masks is the complement of B within Omega_0 (same threshold)
    m = oracle.unpack_masks(masks_u64(out["masks"]), 32)
    B = host(out["imf_norm"]) > 0
    om = fx == 0
    assert not (m.any(axis=0) & B).any() and ((m.any(axis=0) | B) == om).all()


@pytest.mark.parametrize("masks,defer", [(True, "-1"), (False, "-1"), (True, "1")])
def test_density_second_pass_without_stored_overlaps(masks, defer, monkeypatch):
    """Without room for the overlaps of every orientation, the first pass ends
    at the exact F_max and a second pass decides lambda F_max like a known
    threshold; with and without mask outputs, and with the inverse x pass's
    guard-band appends written after its rows (IMF_DEFER_APPENDS=1)."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    monkeypatch.setenv("IMF_OVERLAP_STACK", "0")
    if defer != "-1":
        monkeypatch.setenv("IMF_DEFER_APPENDS", defer)
    d = W.design_density(30, seed=14)
    fx = W.fixture_plate(d.shape, 2)
    tl = W.tool(W.TOOL_BALL, 2, 7, 3, 5)
    dirs = W.fib_hemisphere(9)
    lam = 0.04
    c = imf.Context(0)
    try:
        out, st = c.compute(dev(d), dev(fx), tools=tl, dirs=dirs, lam=lam,
                            method=imf.METHOD_FFT, masks=masks)
    finally:
        c.close()
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam))
    check_density(out, st, ref, lam, masks=masks)
    assert st.passes == 2


@pytest.mark.parametrize("stack,defer", [("1", "-1"), ("0", "-1"), ("1", "1"), ("0", "1")])
def test_density_expected_threshold_bracket(stack, defer, monkeypatch):
    """A request shape seen before lists the overlaps around lambda times its
    last F_max during the inverse transform: the same request again holds the
    band in that bracket (no scan, no second pass); a different design of the
    same shape may miss it and then takes the scan (or the second pass).  Every
    result is exact, with the bracket's appends made where they are found or
    written after the x pass's rows (IMF_DEFER_APPENDS=1)."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    monkeypatch.setenv("IMF_OVERLAP_STACK", stack)
    if defer != "-1":
        monkeypatch.setenv("IMF_DEFER_APPENDS", defer)
    tl = W.tool(W.TOOL_BALL, 2, 7, 3, 5)
    dirs = W.fib_hemisphere(9)
    lam = 0.04
    d1 = W.design_density(30, seed=17)
    d2 = W.quantize_q24(np.clip(d1 * 0.7, 0, 1).astype(np.float32))
    fx = W.fixture_plate(d1.shape, 2)
    c = imf.Context(0)
    try:
        seen = []
        for d in (d1, d1, d2, d2):
            out, st = c.compute(dev(d), dev(fx), tools=tl, dirs=dirs, lam=lam,
                                method=imf.METHOD_FFT, flags=imf.FLAG_NO_GRAPH)
            ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam))
            check_density(out, st, ref, lam)
            seen.append((st.hinted, st.passes))
    finally:
        c.close()
    assert seen[0] == (0, 1 if stack == "1" else 2)
    assert seen[1] == (1, 1)
    assert seen[2][0] in (1, 2) and seen[3] == (1, 1)


def test_density_lambda_zero_and_no_masks(ctx):
    """lambda = 0: B = [f > 0] decided by the first-pass recheck around 0; and
    lambda > 0 without mask outputs: B from masks kept in the workspace."""
    import paper_2002_07627_amd as imf
    d = W.design_density(28, seed=15)
    fx = W.fixture_plate(d.shape, 2)
    tl = W.tool(W.TOOL_FLAT, 1.5, 7, 3, 5)
    dirs = W.fib_hemisphere(8)
    out, st = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, lam=0.0, method=imf.METHOD_FFT)
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=0.0))
    f = host(out["imf"]).astype(np.float64)
    assert (np.abs(f - ref["imf"]) <= 1e-4 * np.maximum(ref["imf"], 1e-2 * ref["F_max"])).all()
    assert np.array_equal(host(out["imf_norm"]) > 0, ref["imf_norm"] > 0)
    assert np.array_equal(host(out["secluded"]), ref["secluded"])
    assert np.array_equal(masks_u64(out["masks"]), ref["masks"])
    lam = 0.03
    out, st = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, lam=lam, method=imf.METHOD_FFT,
                          masks=False)
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam))
    check_density(out, st, ref, lam, masks=False)


def test_density_direct_route_exact(ctx):
    """The direct route on a small grid: exact sums rounded once, the same exact
    F_max, band and masks."""
    import paper_2002_07627_amd as imf
    d = W.design_density(20, seed=16)
    fx = W.fixture_plate(d.shape, 2)
    tl = W.tool(W.TOOL_BALL, 1.5, 5, 3, 4)
    dirs = W.fib_hemisphere(7)
    lam = 0.05
    out, st = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, lam=lam,
                          method=imf.METHOD_DIRECT)
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam))
    check_density(out, st, ref, lam)


def test_rejects_invalid_requests(ctx):
    import paper_2002_07627_amd as imf
    d = dev(np.zeros((8, 8, 8), np.uint8))
    with pytest.raises(imf.IMFError):
        ctx.compute(d, tools=W.TOOL_C2, dirs=np.array([[0, 0, 1.5]]))
    with pytest.raises(imf.IMFError):
        ctx.compute(d, tools=W.TOOL_C1, dirs=np.array([[0, 0, 1]], np.int32),
                    dir_kind=imf.DIR_LATTICE)
    with pytest.raises(imf.IMFError):
        ctx.compute(d, tools=W.tool(W.TOOL_FLAT, 3.3, 4, 1, 1),
                    dirs=np.array([[0, 0, 1]], np.int32), dir_kind=imf.DIR_LATTICE)


def test_empty_design_all_accessible(ctx):
    import paper_2002_07627_amd as imf
    d = dev(np.zeros((20, 21, 22), np.uint8))
    out, st = ctx.compute(d, tools=W.tool(W.TOOL_FLAT, 1.5, 5, 3, 4), dirs=W.lattice26(),
                          dir_kind=imf.DIR_LATTICE, method=imf.METHOD_FFT)
    assert st.F_max == 0 and (host(out["imf"]) == 0).all()
    m = oracle.unpack_masks(masks_u64(out["masks"]), 22)
    assert m.all()


# ---------------------------------------------------------------------------
# branch and bound in the sharp-point minimum: every block shape, every mask
# threshold mode, with and without the bound, against the oracle
# ---------------------------------------------------------------------------
_BND_REF = {}


def _bound_case():
    d = random_boxes((40, 48, 90), 24, 21, lo=6, hi=22)
    fx = W.fixture_plate(d.shape, 3)
    tl = W.tool(W.TOOL_BALL, 2, 8, 4, 6)
    dirs = W.fib_hemisphere(16)
    return d, fx, tl, dirs


@pytest.mark.parametrize("mode", ["zero", "abs", "two_phase"])
@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
def test_bound_every_block_shape(shape, mode, monkeypatch):
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d, fx, tl, dirs = _bound_case()
    kw = {"zero": dict(lam=0.0), "abs": dict(lam=0.02, mask_theta_abs=6.0),
          "two_phase": dict(lam=0.02)}[mode]
    if mode not in _BND_REF:
        _BND_REF[mode] = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, **kw))
    ref = _BND_REF[mode]
    monkeypatch.setenv("IMF_MINFILTER_SHAPE", str(shape))
    monkeypatch.setenv("IMF_BOUND_MIN_VOXELS", "0")   # the bound on this small grid too
    c = imf.Context(0)
    try:
        a, sa = c.compute(dev(d), dev(fx), tools=tl, dirs=dirs, method=imf.METHOD_FFT, **kw)
        b, sb = c.compute(dev(d), dev(fx), tools=tl, dirs=dirs, method=imf.METHOD_FFT, **kw,
                          flags=imf.FLAG_NO_BOUND)
    finally:
        c.close()
    check_binary(a, ref)
    for k in ("imf", "imf_norm", "secluded", "masks"):
        assert torch.equal(a[k], b[k]), k
    assert sa.bound_blocks > 0 and sb.bound_blocks == 0
    assert 0 < sa.bound_skipped < sa.bound_blocks


@pytest.mark.parametrize("shape", [2, 4])
def test_bound_direct_route_cell_minima(shape, monkeypatch):
    """The direct correlation route computes the bound's cell minima in a pass
    of its own (cells of up to 8 rows for the 8 x 4 x 2 blocks)."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d, fx, tl, dirs = _bound_case()
    if "zero" not in _BND_REF:
        _BND_REF["zero"] = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0))
    monkeypatch.setenv("IMF_MINFILTER_SHAPE", str(shape))
    monkeypatch.setenv("IMF_BOUND_MIN_VOXELS", "0")
    c = imf.Context(0)
    try:
        a, sa = c.compute(dev(d), dev(fx), tools=tl, dirs=dirs, method=imf.METHOD_DIRECT)
    finally:
        c.close()
    check_binary(a, _BND_REF["zero"])
    assert sa.mf_shape == shape and 0 < sa.bound_skipped < sa.bound_blocks


def test_long_cutter_uses_more_than_six_levels(ctx):
    """A cutter longer than 128 voxels: runs of S need sparse-table levels
    beyond the register forms (the LDS level pass), on every axis."""
    import paper_2002_07627_amd as imf
    d = random_boxes((20, 22, 24), 8, 31, lo=3, hi=9)
    fx = W.fixture_plate(d.shape, 2)
    tl = W.tool(W.TOOL_FLAT, 1, 140, 2, 4)
    dirs = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1]], np.int32)
    out, st = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE,
                          method=imf.METHOD_FFT)
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1))
    check_binary(out, ref)


# ---------------------------------------------------------------------------
# voxel-model tools under rotation matrices
# ---------------------------------------------------------------------------

def test_voxel_tool_raster_bit_exact(ctx):
    import paper_2002_07627_amd as imf
    t = W.asymmetric_tool()
    rots = np.concatenate([W.random_rotations(24, 61), W.cube_rotations()[:6],
                           np.stack([W.rotation_to([1, 1, 1], r) for r in (0.0, 0.7, 2.1)])])
    for R in rots:
        go, gf = ctx.raster(t, R, imf.DIR_ROTATION)
        oo, oc = oracle.raster(t, R, 2)
        a = {tuple(p): int(f) & 3 for p, f in zip(go.tolist(), gf)}
        b = {tuple(p): 1 | (2 if c else 0) for p, c in zip(oo.tolist(), oc)}
        assert a == b


@pytest.mark.parametrize("sharp", [0, 1])
def test_voxel_tool_imf_bit_exact(ctx, sharp):
    """Non-axisymmetric voxel tool at random rotations and at one axis with three
    rolls (roll matters for it), together with an axisymmetric tool given by
    rotations, against the oracle."""
    import paper_2002_07627_amd as imf
    d = random_boxes((26, 28, 30), 11, 62)
    fx = W.fixture_plate(d.shape, 2)
    vt = W.asymmetric_tool(r=1, length=6, holder_half=3, holder_len=4)
    ft = W.tool(W.TOOL_FLAT, 1, 5, 2, 3)
    rv = np.concatenate([W.random_rotations(7, 63),
                         np.stack([W.rotation_to([0, 1, 2], r) for r in (0.0, 1.0, 2.5)])])
    rf = W.random_rotations(4, 64)
    out, st = ctx.compute(dev(d), dev(fx), tools=[vt, ft], dirs=[rv, rf],
                          dir_kind=imf.DIR_ROTATION, sharp=sharp, method=imf.METHOD_FFT)
    ref = oracle.imf(oracle.Request(d, fx, tools=[vt, ft], dirs=[rv, rf], dir_kind=2,
                                    sharp=sharp))
    check_binary(out, ref)
    assert st.n_orient == 14
    # the three rolls about one axis give three different accessible sets
    m = masks_u64(out["masks"])
    assert len({m[7 + i].tobytes() for i in range(3)}) > 1


def test_voxel_tool_rejects_bad_rotations(ctx):
    import paper_2002_07627_amd as imf
    d = dev(np.zeros((8, 8, 8), np.uint8))
    vt = W.asymmetric_tool()
    with pytest.raises(imf.IMFError):
        ctx.compute(d, tools=vt, dirs=np.diag([1.0, 1.0, -1.0])[None], dir_kind=imf.DIR_ROTATION)
    with pytest.raises(imf.IMFError):
        ctx.compute(d, tools=vt, dirs=np.array([[0.0, 0.0, 1.0]]), dir_kind=imf.DIR_F64)


# ---------------------------------------------------------------------------
# sharp-point runs along lattice vectors against runs along a coordinate axis
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["binary_lattice", "density_two_phase"])
def test_lattice_vector_runs_equal_axis_runs(mode, monkeypatch):
    """The minimum over S is the same whichever exact cover of S by runs is
    used: results with runs along lattice vectors (chosen per orientation)
    equal those with runs along a coordinate axis, bit for bit, with the
    bound on, and equal the oracle."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if mode == "binary_lattice":
        d = random_boxes((36, 40, 44), 16, 51, lo=4, hi=14)
        fx = W.fixture_plate(d.shape, 3)
        tl = W.tool(W.TOOL_BALL, 2, 9, 4, 6)
        dirs = W.lattice26()
        kw = dict(tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE, method=imf.METHOD_FFT)
        req = oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1)
    else:
        d = W.design_density(44, seed=52)
        fx = W.fixture_plate(d.shape, 3)
        tl = W.tool(W.TOOL_BALL, 2, 10, 4, 6)
        dirs = W.fib_hemisphere(24)
        kw = dict(tools=tl, dirs=dirs, lam=0.02, method=imf.METHOD_FFT)
        req = oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=0.02)
    monkeypatch.setenv("IMF_BOUND_MIN_VOXELS", "0")
    outs = {}
    for axis_only in ("0", "1"):
        monkeypatch.setenv("IMF_AXIS_RUNS", axis_only)
        c = imf.Context(0)
        try:
            o, st = c.compute(dev(d), dev(fx), **kw)
            outs[axis_only] = ({k: v.clone() for k, v in o.items()}, st)
        finally:
            c.close()
    (a, sa), (b, sb) = outs["0"], outs["1"]
    assert sa.lattice_runs > 0 and sb.lattice_runs == 0
    assert sa.bound_blocks > 0
    for k in ("imf", "imf_norm", "secluded", "masks"):
        assert torch.equal(a[k], b[k]), k
    ref = oracle.imf(req)
    if mode == "binary_lattice":
        check_binary(a, ref)
    else:
        f = host(a["imf"]).astype(np.float64)
        tol = 1e-4 * np.maximum(np.abs(ref["imf"]), 0.02 * ref["F_max"])
        assert (np.abs(f - ref["imf"]) <= tol).all()


def test_processing_order_changes_no_result(monkeypatch):
    """Orientations are processed in farthest-point order of their tool axes;
    every output (f, fbar, Gamma, per-orientation masks in the caller's order,
    the overlaps of a chosen orientation) equals processing them in the given
    order, bit for bit: two tools, two-phase masks, the bound on."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = W.design_density(40, seed=53)
    fx = W.fixture_plate(d.shape, 3)
    t1, t2 = W.tool(W.TOOL_BALL, 2, 9, 4, 6), W.tool(W.TOOL_FLAT, 1.5, 7, 3, 5)
    d1, d2 = W.fib_hemisphere(14), W.fib_hemisphere(9)
    req = oracle.Request(d, fx, tools=[t1, t2], dirs=[d1, d2], dir_kind=0, lam=0.02)
    q = 17
    info = oracle.orient_info(req, q)
    box = [n + info["kmax"][a] - info["kmin"][a] for a, n in enumerate((40, 40, 40))]
    monkeypatch.setenv("IMF_BOUND_MIN_VOXELS", "0")
    outs = {}
    for given in ("0", "1"):
        monkeypatch.setenv("IMF_GIVEN_ORDER", given)
        c = imf.Context(0)
        try:
            o, st = c.compute(dev(d), dev(fx), tools=[t1, t2], dirs=[d1, d2], lam=0.02,
                              method=imf.METHOD_FFT, batch=3, debug_orient=q,
                              debug_numel=int(np.prod(box)))
            outs[given] = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in o.items()}
            outs[given]["E"] = st.guard_band
        finally:
            c.close()
    a, b = outs["0"], outs["1"]
    for k in ("imf", "imf_norm", "secluded", "masks", "debug"):
        assert torch.equal(a[k], b[k]), k
    assert a["debug_box"] == b["debug_box"]
    assert tuple(a["debug_box"][:3]) == tuple(-np.asarray(info["kmax"]))
    ref = oracle.imf(req, debug_orient=q)
    g = host(a["debug"]).reshape(box[2], box[1], box[0]).astype(np.float64)
    E = a["E"]                 # the float32 transform error model of the guard band
    r = ref["g_debug"] / float(1 << 24)
    assert (np.abs(g - r) <= np.maximum(1e-4 * np.abs(r), E)).all()


def test_minimum_pass_wave_modes_equal(monkeypatch):
    """The list pass of the minimum with independent waves, four waves in step
    and eight waves in step gives identical outputs (two-phase masks, bound on)."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d, fx, tl, dirs = _bound_case()
    monkeypatch.setenv("IMF_BOUND_MIN_VOXELS", "0")
    outs = []
    for mode in ("0", "1", "2"):
        monkeypatch.setenv("IMF_MINFILTER_SYNC", mode)
        c = imf.Context(0)
        try:
            o, st = c.compute(dev(d), dev(fx), tools=tl, dirs=dirs, lam=0.02,
                              method=imf.METHOD_FFT)
            outs.append({k: v.clone() for k, v in o.items()})
            assert st.bound_blocks > 0
        finally:
            c.close()
    for o in outs[1:]:
        for k in ("imf", "imf_norm", "secluded", "masks"):
            assert torch.equal(o[k], outs[0][k]), k


@pytest.mark.parametrize("design", ["density", "binary"])
@pytest.mark.parametrize("frac", ["0", "0.5", "0.01"])
def test_compact_gamma_stack(design, frac, monkeypatch):
    """With the bound, the two-phase gamma stack holds only the blocks the
    bound keeps (the others have no mask bit), in a pool sized from the kept
    fraction of the last request of the shape.  Off (0), at the default first
    capacity (0.5) and at one too small for this request (0.01: the pool
    overflows and a second pass with the threshold known decides the
    request), every result is exact; the repeated request, with the pool sized
    from the first one's kept fraction, takes one pass."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d, fx, tl, dirs = _bound_case()
    lam = 0.02
    if design == "density":  # a crop of a density design, same shape
        d = np.ascontiguousarray(W.design_density(max(d.shape), seed=23)[:d.shape[0], :d.shape[1],
                                                                        :d.shape[2]])
    key = "compact_" + design
    if key not in _BND_REF:
        _BND_REF[key] = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0,
                                                  lam=lam))
    ref = _BND_REF[key]
    monkeypatch.setenv("IMF_BOUND_MIN_VOXELS", "0")
    monkeypatch.setenv("IMF_COMPACT_GAMMA", frac)
    monkeypatch.setenv("IMF_OVERLAP_STACK", "1")
    c = imf.Context(0)
    try:
        passes = []
        for rep in range(2):
            print("compact gamma", design, frac, rep, flush=True)
            out, st = c.compute(dev(d), dev(fx), tools=tl, dirs=dirs, lam=lam,
                                method=imf.METHOD_FFT, flags=imf.FLAG_NO_GRAPH)
            if design == "density":
                check_density(out, st, ref, lam)
            else:
                check_binary(out, ref)
            assert 0 < st.bound_skipped < st.bound_blocks
            passes.append(st.passes)
    finally:
        c.close()
    # the one-pass repeat's bound kept what the first request's first pass
    # kept: the first pool overflowed exactly when that exceeds its capacity
    kept = st.bound_blocks - st.bound_skipped
    over = float(frac) > 0 and kept > int(np.ceil(float(frac) * st.bound_blocks))
    assert passes == [2 if over else 1, 1], (passes, kept, st.bound_blocks)
    if frac == "0.01":
        assert over
