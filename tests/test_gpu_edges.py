"""GPU parity on degenerate grids: one- and two-voxel-thick slabs, a single
voxel, and a row that crosses a 64-voxel mask word, through both correlation
routes, against the CPU oracle (binary: bit-exact; density: the per-voxel
tolerance of the parity suite)."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(1, 9, 70), (3, 1, 5), (2, 2, 2), (1, 1, 1), (6, 1, 1)]


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


def thin_design(shape, seed):
    rng = np.random.default_rng(seed)
    return (rng.random(shape) < 0.3).astype(np.uint8)


@pytest.mark.parametrize("method", ["fft", "direct"])
@pytest.mark.parametrize("shape", SHAPES)
def test_thin_grids_binary_bit_exact(ctx, shape, method):
    import paper_2002_07627_amd as imf
    d = thin_design(shape, 7627100 + sum(shape))
    fx = np.zeros(shape, np.uint8)
    fx[0, 0, 0] = 1  # one fixture voxel (outside the design domain)
    tl = W.tool(W.TOOL_BALL, 1.5, 5, 2.5, 4)
    dirs = W.lattice26()
    m = imf.METHOD_FFT if method == "fft" else imf.METHOD_DIRECT
    print("thin binary", shape, method, flush=True)
    out, _ = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE,
                         method=m)
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1))
    f = host(out["imf"]).astype(np.float64)
    assert np.array_equal(f, ref["imf"].reshape(f.shape))
    assert np.array_equal(host(out["imf_norm"]), ref["imf_norm"].reshape(f.shape))
    assert np.array_equal(host(out["secluded"]), ref["secluded"].reshape(f.shape))
    mk = host(out["masks"]).view(np.uint64)
    assert np.array_equal(mk, ref["masks"].reshape(mk.shape))


@pytest.mark.parametrize("shape", [(1, 9, 70), (3, 1, 5)])
def test_thin_grids_density_with_bound(shape, monkeypatch):
    """The branch-and-bound pass on (its size threshold lifted) over slabs
    thinner than one block."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(7627200 + sum(shape))
    d = W.quantize_q24(rng.random(shape).astype(np.float32))
    tl = W.tool(W.TOOL_BALL, 1.5, 5, 2.5, 4)
    dirs = W.fib_hemisphere(12)
    lam = 0.05
    print("thin density", shape, flush=True)
    monkeypatch.setenv("IMF_BOUND_MIN_VOXELS", "0")
    c = imf.Context(0)
    try:
        out, st = c.compute(dev(d), tools=tl, dirs=dirs, dir_kind=imf.DIR_F64, lam=lam,
                            method=imf.METHOD_FFT)
    finally:
        c.close()
    assert st.bound_blocks > 0
    ref = oracle.imf(oracle.Request(d, None, tools=tl, dirs=dirs, dir_kind=0, lam=lam))
    f = host(out["imf"]).astype(np.float64)
    fr = ref["imf"].reshape(f.shape)
    tol = 1e-4 * np.maximum(np.abs(fr), lam * ref["F_max"])
    assert np.all(np.abs(f - fr) <= tol)
    # two-phase masks, F_max, B and Gamma: exact
    assert st.F_max == ref["F_max"]
    mk = host(out["masks"]).view(np.uint64)
    assert np.array_equal(mk, ref["masks"].reshape(mk.shape))
    assert np.array_equal(host(out["imf_norm"]) > 0, ref["imf_norm"].reshape(f.shape) > 0)
    assert np.array_equal(host(out["secluded"]), ref["secluded"].reshape(f.shape))


@pytest.mark.parametrize("radius", [13, 19])
def test_wide_cutter_run_lists_beyond_the_staging(ctx, radius):
    """A ball cutter so wide that its sharp-point windows (radius 13: about
    1000 runs' windows) or even its runs (radius 19: about 1130) outnumber the
    1024 entries the minimum pass stages in LDS: the run lists stay whole and
    the surplus runs are read from memory one by one."""
    import paper_2002_07627_amd as imf
    rng = np.random.default_rng(7627300 + radius)
    d = (rng.random((8, 12, 18)) < 0.25).astype(np.uint8)
    tl = W.tool(W.TOOL_BALL, radius, radius, 2, 2)  # the ball alone cuts
    dirs = np.array([[0, 0, 1], [1, 0, 0], [0, -1, 0]], np.int32)
    print("wide cutter r", radius, flush=True)
    out, _ = ctx.compute(dev(d), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE,
                         method=imf.METHOD_FFT)
    ref = oracle.imf(oracle.Request(d, None, tools=tl, dirs=dirs, dir_kind=1))
    f = host(out["imf"]).astype(np.float64)
    assert np.array_equal(f, ref["imf"].reshape(f.shape))
    mk = host(out["masks"]).view(np.uint64)
    assert np.array_equal(mk, ref["masks"].reshape(mk.shape))


@pytest.mark.parametrize("case", ["off_grid", "above_one", "negative", "nan", "binary_two",
                                  "under_fixture"])
def test_design_outside_the_value_set_is_rejected(ctx, case):
    """A design value the fixed-point overlaps cannot hold exactly (a density
    off the 2^-24 grid or outside [0, 1], a binary value above 1) fails the
    request with EINVAL, under a fixture voxel too, as the oracle's input check
    does; the context then serves a valid request unchanged."""
    import paper_2002_07627_amd as imf
    shape = (12, 10, 70)
    rng = np.random.default_rng(7627150)
    tl = W.tool(W.TOOL_BALL, 1.5, 5, 2.5, 4)
    dirs = W.lattice26()
    fx = np.zeros(shape, np.uint8)
    if case == "binary_two":
        d = (rng.random(shape) < 0.3).astype(np.uint8)
        d[5, 4, 33] = 2
    else:
        d = (np.floor(rng.random(shape) * 2 ** 24) / 2 ** 24).astype(np.float32)
        bad = {"off_grid": np.float32(0.25 + 2.0 ** -25), "above_one": np.float32(1.5),
               "negative": np.float32(-2.0 ** -24), "nan": np.float32(np.nan),
               "under_fixture": np.float32(2.0 ** -30)}[case]
        d[5, 4, 33] = bad
        if case == "under_fixture":
            fx[5, 4, 33] = 1
    print("invalid design", case, flush=True)
    with pytest.raises(imf.IMFError) as ei:
        ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE)
    assert ei.value.status == 1
    d[5, 4, 33] = 1
    out, _ = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE)
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1))
    mk = host(out["masks"]).view(np.uint64)
    assert np.array_equal(mk, ref["masks"].reshape(mk.shape))
