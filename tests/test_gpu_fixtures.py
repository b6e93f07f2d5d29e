"""GPU parity of fixtures that change with the setup (Sec. 2.1.5): every
orientation sees the common fixture plus its setup's own, and Omega_0 excludes
the fixtures of all setups.  Against the oracle on the same seeded inputs, to
the bars of the other parity tests: bit-exact for binary designs, density f
within 1e-4 relative with masks bit-exact for a given threshold."""
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


def _binary_case(shape=(30, 34, 40), n_sets=3, seed=41):
    rng = np.random.default_rng(seed)
    d = (rng.random(shape) < 0.12).astype(np.uint8)
    d[8:20, 10:24, 12:30] = 1
    fx = W.fixture_plate(shape, 3)
    sets = W.setup_clamps(shape, n_sets, seed=seed)
    return d, fx, sets


def _check_exact(out, ref):
    for k in ("imf", "imf_norm", "secluded"):
        a = host(out[k])
        assert np.array_equal(a.astype(ref[k].dtype), ref[k].reshape(a.shape)), k
    m = host(out["masks"]).view(np.uint64)
    assert np.array_equal(m, ref["masks"].reshape(m.shape)), "masks"


@pytest.mark.parametrize("method", ["fft", "direct"])
def test_binary_sets_bit_exact(ctx, method):
    import paper_2002_07627_amd as imf
    d, fx, sets = _binary_case()
    tl = W.tool(W.TOOL_FLAT, 1.5, 6, 3, 5)
    dirs = W.lattice26()
    fof = (np.arange(len(dirs)) * 7 // 3) % 3        # sets interleaved: batches split
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1, fixture_sets=sets,
                                    fixture_of=fof))
    m = imf.METHOD_FFT if method == "fft" else imf.METHOD_DIRECT
    out, st = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE,
                          method=m, batch=4, fixture_sets=dev(sets), fixture_of=fof)
    _check_exact(out, ref)
    assert st.F_max == ref["F_max"]
    # nothing of any setup's fixture is in the design domain
    assert not host(out["imf_norm"])[sets.any(0) != 0].any()


def test_sets_without_common_fixture_and_with_domain(ctx):
    import paper_2002_07627_amd as imf
    d, _, sets = _binary_case((24, 28, 32), 2, seed=42)
    tl = W.tool(W.TOOL_BALL, 2, 7, 3.5, 5)
    dirs = W.fib_hemisphere(14)
    fof = W.setup_of_dirs(dirs, 2)
    dom = np.ones(d.shape, np.uint8)
    dom[:, :, :5] = 0
    for fxa, doma in ((None, None), (None, dom)):
        ref = oracle.imf(oracle.Request(d, fxa, domain=doma, tools=tl, dirs=dirs, dir_kind=0,
                                        fixture_sets=sets, fixture_of=fof))
        out, _ = ctx.compute(dev(d), None if fxa is None else dev(fxa),
                             None if doma is None else dev(doma), tools=tl, dirs=dirs,
                             method=imf.METHOD_FFT, fixture_sets=dev(sets), fixture_of=fof)
        _check_exact(out, ref)


def test_identical_sets_equal_one_fixture(ctx):
    import paper_2002_07627_amd as imf
    d, fx, _ = _binary_case(seed=43)
    tl = W.tool(W.TOOL_FLAT, 1.5, 6, 3, 5)
    dirs = W.lattice26()
    kw = dict(tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE, method=imf.METHOD_FFT)
    a, _ = ctx.compute(dev(d), dev(fx), **kw)
    sets = np.stack([fx, fx])
    b, _ = ctx.compute(dev(d), None, **kw, fixture_sets=dev(sets),
                       fixture_of=np.arange(len(dirs)) % 2)
    for k in ("imf", "imf_norm", "secluded", "masks"):
        assert torch.equal(a[k], b[k]), k


def test_density_sets_with_bound(monkeypatch):
    """Density design, absolute mask threshold, the branch-and-bound pass on:
    f within 1e-4 relative; masks, F_max, B and Gamma bit-exact."""
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = W.design_density(40, seed=44)
    fx = W.fixture_plate(d.shape, 3)
    sets = W.setup_clamps(d.shape, 4, seed=44)
    tl = W.tool(W.TOOL_BALL, 2, 8, 4, 6)
    dirs = W.fib_hemisphere(20)
    fof = W.setup_of_dirs(dirs, 4)
    order = np.argsort(fof, kind="stable")          # setups grouped
    dirs, fof = dirs[order], fof[order]
    lam = 0.01
    ref0 = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam,
                                     fixture_sets=sets, fixture_of=fof))
    theta = 0.5 * float(np.median(ref0["imf"]))
    ref = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam,
                                    mask_theta_abs=theta, fixture_sets=sets, fixture_of=fof))
    monkeypatch.setenv("IMF_BOUND_MIN_VOXELS", "0")
    c = imf.Context(0)
    try:
        out, st = c.compute(dev(d), dev(fx), tools=tl, dirs=dirs, lam=lam, mask_theta_abs=theta,
                            method=imf.METHOD_FFT, fixture_sets=dev(sets), fixture_of=fof)
    finally:
        c.close()
    assert st.bound_blocks > 0
    f = host(out["imf"]).astype(np.float64)
    fref = ref["imf"]
    tol = 1e-4 * np.maximum(np.abs(fref), lam * ref["F_max"])
    assert (np.abs(f - fref) <= tol).all(), np.abs(f - fref).max()
    assert np.array_equal(host(out["masks"]).view(np.uint64), ref["masks"])
    # F_max, B and Gamma at lambda F_max: exact
    assert st.F_max == ref["F_max"]
    assert np.array_equal(host(out["imf_norm"]) > 0, ref["imf_norm"] > 0)
    assert np.array_equal(host(out["secluded"]), ref["secluded"])


def test_serving_and_graph_replay_follow_the_sets(ctx):
    """A request submitted to the serving loop equals the synchronous one; a
    request replayed from a graph and then one with other set indices each
    equal the oracle."""
    import paper_2002_07627_amd as imf
    d, fx, sets = _binary_case((26, 30, 36), 3, seed=45)
    tl = W.tool(W.TOOL_FLAT, 1.5, 6, 3, 5)
    dirs = W.lattice26()
    kw = dict(tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE, method=imf.METHOD_FFT)
    dd, dfx, ds = dev(d), dev(fx), dev(sets)
    fof_a = np.arange(len(dirs)) % 3
    fof_b = (np.arange(len(dirs)) // 9) % 3
    ref_a = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1, fixture_sets=sets,
                                      fixture_of=fof_a))
    ref_b = oracle.imf(oracle.Request(d, fx, tools=tl, dirs=dirs, dir_kind=1, fixture_sets=sets,
                                      fixture_of=fof_b))
    ctx.compute(dd, dfx, **kw, fixture_sets=ds, fixture_of=fof_a, flags=imf.FLAG_NO_GRAPH)
    out = None
    graphs = []
    for _ in range(3):          # launched, captured, replayed
        out, st = ctx.compute(dd, dfx, **kw, fixture_sets=ds, fixture_of=fof_a, out=out)
        graphs.append(st.graph)
        _check_exact(out, ref_a)
    assert graphs == [0, 1, 2]
    out, st = ctx.compute(dd, dfx, **kw, fixture_sets=ds, fixture_of=fof_b, out=out)
    assert st.graph == 0
    _check_exact(out, ref_b)
    t = ctx.submit(dd, dfx, **kw, fixture_sets=ds, fixture_of=fof_b)
    o2, _ = ctx.wait(t)
    _check_exact(o2, ref_b)


def test_rejects_bad_sets(ctx):
    import paper_2002_07627_amd as imf
    d, fx, sets = _binary_case((16, 16, 16), 2, seed=46)
    dirs = W.lattice26()[:4]
    kw = dict(tools=W.tool(W.TOOL_FLAT, 1.5, 4, 2, 3), dirs=dirs, dir_kind=imf.DIR_LATTICE)
    with pytest.raises(imf.IMFError):
        ctx.compute(dev(d), dev(fx), **kw, fixture_sets=dev(sets),
                    fixture_of=np.array([0, 1, 2, 0]))
    with pytest.raises(imf.IMFError):
        ctx.compute(dev(d), dev(fx), **kw, fixture_sets=dev(sets),
                    fixture_of=np.array([0, -1, 1, 0]))
    with pytest.raises(ValueError):
        ctx.compute(dev(d), dev(fx), **kw, fixture_sets=dev(sets), fixture_of=np.array([0, 1]))
