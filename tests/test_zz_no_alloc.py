"""The allocation-free greedy planner (imf_plan_greedy_noalloc) through the C
interface: the same plan as imf_plan_greedy and the oracle on two calls in a
row, the second on a smaller grid with fewer orientations (the fixed scratch
keeps the first call's contents), and plans beyond its scratch rejected."""
import numpy as np
import pytest

from oracle import coupling as cp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(seed, shape, nq):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    words = (nx + 63) // 64
    design = (rng.random(shape) < 0.35).astype(np.uint8)
    fixture = np.zeros(shape, np.uint8)
    fixture[:2] = 1
    bits = rng.random((nq, nz, ny, nx)) < rng.uniform(0.05, 0.5, size=(nq, 1, 1, 1))
    padded = np.zeros((nq, nz, ny, words * 64), bool)
    padded[..., :nx] = bits
    masks = np.packbits(padded.reshape(nq, nz, ny, words, 64), axis=-1,
                        bitorder="little").view(np.uint64).reshape(nq, nz, ny, words)
    return design, fixture, bits, masks


def test_noalloc_plan_equals_the_allocating_plan_twice_then_smaller():
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = imf.Context(0)
    try:
        for seed, shape, nq in ((71, (40, 50, 130), 23), (72, (9, 17, 33), 6)):
            print("no-alloc plan: seed %d grid %s orientations %d" % (seed, shape, nq), flush=True)
            design, fixture, bits, masks = _case(seed, shape, nq)
            dm = torch.from_numpy(masks.view(np.int64)).cuda()
            dd = torch.from_numpy(design).cuda()
            df = torch.from_numpy(fixture).cuda()
            a = ctx.plan_greedy(dm, dd, df, noalloc=True)
            b = ctx.plan_greedy(dm, dd, df)
            ref = cp.plan_greedy(bits, design, omega0=fixture == 0)
            assert a == b, seed
            assert a[0] == ref[0] and a[1] == ref[1], seed
            assert len(a[0]) > 1
            # a step limit, as the allocating planner takes it
            assert ctx.plan_greedy(dm, dd, df, max_steps=2, noalloc=True) == \
                ctx.plan_greedy(dm, dd, df, max_steps=2)
            torch.cuda.synchronize()
    finally:
        ctx.close()


def test_noalloc_plan_rejects_grids_beyond_its_scratch():
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = imf.Context(0)
    try:
        # 2^20 scratch words: a 1024 x 1024 x 64 grid needs 2^20 mask words plus the counts
        shape = (1024, 1024, 64)
        dm = torch.zeros((1, 1024, 1024, 1), dtype=torch.int64, device="cuda")
        dd = torch.zeros(shape, dtype=torch.uint8, device="cuda")
        with pytest.raises(imf.IMFError) as e:
            ctx.plan_greedy(dm, dd, noalloc=True)
        assert e.value.status == 1 and "scratch" in str(e.value)
    finally:
        ctx.close()
