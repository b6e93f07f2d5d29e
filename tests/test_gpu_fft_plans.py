"""Every transform plan of the inverse passes (composite or base radices,
full- or half-width tiles; chosen per pass by the autotuner) gives the same
results: binary requests bit for bit (the rounded overlaps are exact under
any plan), density requests the same masks, B and Gamma (thresholds decided
exactly) and f within float32 rounding of the overlaps.  The plan is set
through an autotune table, the way a tuned context applies it."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def imf_mod():
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return imf


PLANS = [0b010101, 0b101010, 0b111111, 0b011001]


@pytest.mark.parametrize("density", [False, True])
def test_transform_plans_agree(imf_mod, tmp_path, density):
    imf = imf_mod
    n = 150
    d = W.design_density(n, seed=98) if density else W.design_3d_boxes_cyls(n, seed=98)
    fx = W.fixture_plate(d.shape, 4)
    kw = dict(tools=W.tool(W.TOOL_BALL, 3, 24, 8, 20), dirs=W.fib_hemisphere(12),
              dir_kind=imf.DIR_F64, method=imf.METHOD_FFT, lam=0.01 if density else 0.0)
    ctx = imf.Context(0)
    try:
        print("plans, density" if density else "plans, binary", flush=True)
        o0, s0 = ctx.compute(dev(d), dev(fx), **kw)
        o0 = {k: v.clone() for k, v in o0.items()}
        # the default: per pass the plan whose kernels fit more workgroups
        # per CU (composite radices on a tie), 2 bits per pass
        assert 0 <= s0.fft_plan < 64 and all((s0.fft_plan >> (2 * i)) & 2 == 0 for i in range(3))
        P = tuple(s0.P)
        assert any(p in (192, 216, 256, 288, 320, 384, 448, 512) for p in P), P
        for plan in PLANS:
            path = str(tmp_path / ("plan%d.txt" % plan))
            with open(path, "w") as f:
                f.write("imf-autotune 2\n%d|%d,%d,%d|%d,%d,%d %d %d %d %d\n" % (
                    imf.METHOD_FFT, n, n, n, P[0], P[1], P[2], s0.batch, s0.mf_shape,
                    s0.mf_wg_per_cu, plan))
            assert ctx.autotune_load(path) == 1
            o1, s1 = ctx.compute(dev(d), dev(fx), batch=0, **kw)
            assert s1.fft_plan == plan
            for k in ("masks", "secluded"):
                assert torch.equal(o1[k], o0[k]), (plan, k)
            if density:
                a, b = o1["imf"].double(), o0["imf"].double()
                assert torch.allclose(a, b, rtol=1e-4, atol=1e-3), plan
            else:
                for k in ("imf", "imf_norm"):
                    assert torch.equal(o1[k], o0[k]), (plan, k)
            assert s1.F_max == s0.F_max
    finally:
        ctx.close()
