"""GPU parity of the TO-coupling steps (Sec. 2.2) through the C interface:
Heaviside projection bit-exact against the float64 oracle (outside the
rounding-tie zone, where a last-bit difference of exp could flip the 2^-24
rounding), accessibility filter and filtered sensitivity bit-exact, and a short
projection -> IMF -> filter -> update loop checked step by step."""
import numpy as np
import pytest

import oracle
from oracle import coupling as cp
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


def not_tie(xi, beta):
    x = np.clip(np.asarray(xi, np.float64), 0, 1)
    r = (1.0 - np.exp(-beta * x)) + x * np.exp(-beta)
    fr = r * 2 ** 24 - np.floor(r * 2 ** 24)
    return np.abs(fr - 0.5) > 1e-6


@pytest.mark.parametrize("beta", [2.0, 8.0])
def test_heaviside_matches_oracle(ctx, beta):
    rng = np.random.default_rng(int(beta))
    xi = rng.random(1 << 20).astype(np.float32)
    xi[:6] = [0.0, 1.0, -0.5, 1.5, 1e-7, 0.5]
    got = ctx.heaviside(dev(xi), beta).cpu().numpy()
    ref = cp.heaviside(xi, beta)
    ok = not_tie(xi, beta)
    assert ok.mean() > 0.999
    assert np.array_equal(got[ok], ref[ok])
    assert np.abs(got.astype(np.float64) - ref).max() <= 2 ** -24
    assert np.array_equal(got * 2 ** 24, np.round(got.astype(np.float64) * 2 ** 24))


def test_access_filter_and_sensitivity_bit_exact(ctx):
    import paper_2002_07627_amd as imf
    d = W.design_density(36, seed=41)
    fx = W.fixture_plate(d.shape, 3)
    out, st = ctx.compute(dev(d), dev(fx), tools=W.tool(W.TOOL_BALL, 2, 8, 4, 6),
                          dirs=W.fib_hemisphere(12), lam=0.05, method=imf.METHOD_FFT)
    rng = np.random.default_rng(42)
    sens = rng.normal(size=d.shape).astype(np.float32)
    for w in (0.0, 0.35, 1.0):
        filt, so = ctx.access_filter(dev(d), out["imf_norm"], out["secluded"], dev(fx),
                                     tau=0.5, sens=dev(sens), w=w)
        fref = cp.access_filter(d, out["imf_norm"].cpu().numpy(), out["secluded"].cpu().numpy())
        assert np.array_equal(filt.cpu().numpy(), fref)
        sref = cp.filtered_sensitivity(sens, fref, w, cp.omega0_of(d.shape, fx))
        assert np.array_equal(so.cpu().numpy(), sref), w
    # the filter is 1 exactly on the secluded set and fbar inside the design
    f = filt.cpu().numpy()
    sec = out["secluded"].cpu().numpy() != 0
    assert (f[sec] == 1).all()
    solid = d > 0.5
    assert np.array_equal(f[solid], out["imf_norm"].cpu().numpy()[solid])
    # binary design, filter only
    b = (d > 0.5).astype(np.uint8)
    ob, _ = ctx.compute(dev(b), dev(fx), tools=W.tool(W.TOOL_FLAT, 1.5, 6, 3, 5),
                        dirs=W.lattice26()[::3], dir_kind=imf.DIR_LATTICE, method=imf.METHOD_FFT)
    fb, none = ctx.access_filter(dev(b), ob["imf_norm"], ob["secluded"], dev(fx))
    assert none is None
    assert np.array_equal(fb.cpu().numpy(), cp.access_filter(b, ob["imf_norm"].cpu().numpy(),
                                                             ob["secluded"].cpu().numpy()))


def test_coupled_loop_step_by_step(ctx):
    """xi -> Heaviside -> IMF -> filter -> filtered sensitivity -> xi update, three
    iterations; each GPU step against the oracle on the GPU's previous result."""
    import paper_2002_07627_amd as imf
    n = 28
    fx = W.fixture_plate((n, n, n), 3)
    tl = W.tool(W.TOOL_BALL, 2, 8, 4, 6)
    dirs = W.fib_hemisphere(10)
    lam, beta, w = 0.05, 8.0, 0.4
    rng = np.random.default_rng(7)
    xi = (0.3 + 0.4 * rng.random((n, n, n))).astype(np.float32)
    for it in range(3):
        rho = ctx.heaviside(dev(xi), beta)
        rho_h = rho.cpu().numpy()
        ok = not_tie(xi, beta)
        assert np.array_equal(rho_h[ok], cp.heaviside(xi, beta)[ok])
        out, st = ctx.compute(rho, dev(fx), tools=tl, dirs=dirs, lam=lam, method=imf.METHOD_FFT)
        ref = oracle.imf(oracle.Request(rho_h, fx, tools=tl, dirs=dirs, dir_kind=0, lam=lam),
                         masks=False)
        f = out["imf"].cpu().numpy().astype(np.float64)
        tol = 1e-4 * np.maximum(np.abs(ref["imf"]), lam * ref["F_max"])
        assert (np.abs(f - ref["imf"]) <= tol).all(), it
        sens = -(rho_h.astype(np.float64) ** 3).astype(np.float32)   # a compliance-like field
        filt, s = ctx.access_filter(rho, out["imf_norm"], out["secluded"], dev(fx), sens=dev(sens),
                                    w=w)
        fref = cp.access_filter(rho_h, out["imf_norm"].cpu().numpy(), out["secluded"].cpu().numpy())
        assert np.array_equal(filt.cpu().numpy(), fref)
        sref = cp.filtered_sensitivity(sens, fref, w, fx == 0)
        assert np.array_equal(s.cpu().numpy(), sref)
        xi = np.clip(xi - 0.05 * s.cpu().numpy(), 0, 1).astype(np.float32)


def test_greedy_plan_matches_oracle(ctx):
    """Greedy machining plan on a 64^3 binary part with 26 lattice directions:
    the GPU plan equals the oracle plan on the same masks (which are themselves
    bit-exact against the oracle), and on a small case the oracle's own masks."""
    import paper_2002_07627_amd as imf
    d = W.design_3d_boxes_cyls(64, seed=51)
    fx = W.fixture_plate(d.shape, 3)
    tl = W.tool(W.TOOL_FLAT, 1.5, 12, 4, 12)
    dirs = W.lattice26()
    out, _ = ctx.compute(dev(d), dev(fx), tools=tl, dirs=dirs, dir_kind=imf.DIR_LATTICE,
                         method=imf.METHOD_FFT)
    steps, left = ctx.plan_greedy(out["masks"], dev(d), dev(fx))
    m = oracle.unpack_masks(out["masks"].cpu().numpy().view(np.uint64), 64)
    ref_steps, ref_left = cp.plan_greedy(m, d, omega0=fx == 0)
    assert steps == ref_steps and left == ref_left
    assert len(steps) >= 2
    s1, l1 = ctx.plan_greedy(out["masks"], dev(d), dev(fx), max_steps=1)
    assert s1 == steps[:1] and l1 == left + sum(r for _, r in steps[1:])
    # small case through the oracle's masks
    d2 = W.design_3d_boxes_cyls(24, seed=52)
    fx2 = W.fixture_plate(d2.shape, 2)
    tl2 = W.tool(W.TOOL_FLAT, 1, 5, 2, 4)
    out2, _ = ctx.compute(dev(d2), dev(fx2), tools=tl2, dirs=dirs, dir_kind=imf.DIR_LATTICE,
                          method=imf.METHOD_FFT)
    ref = oracle.imf(oracle.Request(d2, fx2, tools=tl2, dirs=dirs, dir_kind=1))
    s2, l2 = ctx.plan_greedy(out2["masks"], dev(d2), dev(fx2))
    assert (s2, l2) == cp.plan_greedy(oracle.unpack_masks(ref["masks"], 24), d2, omega0=fx2 == 0)
