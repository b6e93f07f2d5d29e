"""Serving loop, admission and autotuning through the C interface.

The serving mix takes requests of different grid sizes, orientation counts,
binary and density designs and both cutters (subsets of one master Fibonacci
set, so tool spectra are shared); every result in the mix must equal the same
request computed alone (bit-identical: the per-orientation arithmetic does not
depend on what else runs; f of density requests up to float rounding where
the two took a different number of passes), and the small binary ones the
oracle."""
import time

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _mix(n_req=8, seed=91):
    descs = W.serving_stream(n_req, seed=seed, sizes=(32, 40, 48, 56, 64), master_dirs=40)
    return [dict(W.serving_request(d, master_dirs=40), desc=d) for d in descs]


@pytest.fixture(scope="module")
def imf_mod():
    import paper_2002_07627_amd as imf
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return imf


def _kw(imf, r):
    return dict(tools=r["tool"], dirs=r["dirs"], dir_kind=imf.DIR_F64, lam=r["lam"],
                method=imf.METHOD_FFT)


def _same(o, a, same_passes, i, F_max=0.0, lam=0.0):
    """A served result against the same request alone: bit for bit, except
    f of a density request decided in two passes on one side and in one on
    the other: the second pass replaces the overlaps it rechecks by their
    exact values (float32 rounded), so f may move by up to the guard band
    there; both sides are within the parity tolerance of the exact f, so
    within twice it of each other.  The masks, B and Gamma are exact either
    way."""
    for k in ("secluded", "masks"):
        assert torch.equal(o[k], a[k]), (i, k)
    if same_passes:
        for k in ("imf", "imf_norm"):
            assert torch.equal(o[k], a[k]), (i, k)
    else:
        assert torch.equal(o["imf_norm"] > 0, a["imf_norm"] > 0), i
        f, g = o["imf"].double(), a["imf"].double()
        tol = 2e-4 * torch.clamp(g.abs(), min=lam * F_max)
        assert bool(((f - g).abs() <= tol).all()), i


def test_mix_equals_alone(imf_mod):
    imf = imf_mod
    reqs = _mix()
    ctx = imf.Context(0)
    try:
        alone, passes = [], []
        for r in reqs:
            o, st = ctx.compute(dev(r["design"]), dev(r["fixture"]), **_kw(imf, r))
            alone.append({k: v.clone() for k, v in o.items()})
            passes.append(st.passes)
        inputs = [(dev(r["design"]), dev(r["fixture"])) for r in reqs]
        tickets = [ctx.submit(d, fx, **_kw(imf, r)) for (d, fx), r in zip(inputs, reqs)]
        lat = []
        for i, t in enumerate(tickets):
            o, st = ctx.wait(t)
            lat.append(st.t_ms[7])
            _same(o, alone[i], st.passes == passes[i], i, st.F_max, reqs[i]["lam"])
        assert all(x > 0 for x in lat)
    finally:
        ctx.close()
    # the binary ones against the oracle
    for r, a in zip(reqs, alone):
        if r["desc"]["density"] or r["desc"]["n"] > 40:
            continue
        ref = oracle.imf(oracle.Request(r["design"], r["fixture"], tools=r["tool"],
                                        dirs=r["dirs"], dir_kind=0))
        f = a["imf"].cpu().numpy().astype(np.float64)
        assert np.array_equal(f, ref["imf"].reshape(f.shape))
        assert np.array_equal(a["masks"].cpu().numpy().view(np.uint64),
                              ref["masks"].reshape(a["masks"].shape))


def test_cancel_and_timeout(imf_mod):
    imf = imf_mod
    reqs = _mix(6, seed=92)
    ctx = imf.Context(0)
    try:
        inputs = [(dev(r["design"]), dev(r["fixture"])) for r in reqs]
        tickets = [ctx.submit(d, fx, **_kw(imf, r)) for (d, fx), r in zip(inputs, reqs)]
        # the last request is cancelled unless it already started
        cancelled = True
        try:
            ctx.cancel(tickets[-1])
        except imf.IMFError as e:
            assert e.status == 4  # IMF_EBUSY: already running
            cancelled = False
        # a zero timeout on the first request either finds it done or times out
        try:
            ctx.wait(tickets[0], timeout_ms=0)
            done0 = True
        except imf.IMFError as e:
            assert e.status == 5  # IMF_ETIMEOUT
            done0 = False
        for t in tickets[:-1] if done0 else tickets[:-1]:
            if t == tickets[0] and done0:
                continue
            ctx.wait(t)
        if cancelled:
            with pytest.raises(imf.IMFError) as ei:
                ctx.wait(tickets[-1])
            assert ei.value.status == 6  # IMF_ECANCELLED
        else:
            ctx.wait(tickets[-1])
    finally:
        ctx.close()


def test_admission_by_footprint(imf_mod):
    imf = imf_mod
    r = _mix(1, seed=93)[0]
    ctx = imf.Context(0)
    try:
        need = ctx.footprint(dev(r["design"]), dev(r["fixture"]), **_kw(imf, r))
        assert need > r["design"].size * 4
    finally:
        ctx.close()
    small = imf.Context(0, budget_bytes=need // 4)
    try:
        with pytest.raises(imf.IMFError) as ei:
            small.compute(dev(r["design"]), dev(r["fixture"]), **_kw(imf, r))
        assert ei.value.status == 2  # IMF_ENOMEM
    finally:
        small.close()


def test_autotune_then_batch_is_used_and_results_unchanged(imf_mod):
    imf = imf_mod
    d = W.design_3d_boxes_cyls(48, seed=94)
    fx = W.fixture_plate(d.shape, 3)
    kw = dict(tools=W.tool(W.TOOL_FLAT, 2, 10, 4, 8), dirs=W.fib_hemisphere(24),
              dir_kind=imf.DIR_F64, method=imf.METHOD_FFT)
    ctx = imf.Context(0)
    try:
        best = ctx.autotune(dev(d), dev(fx), **kw)
        assert 1 <= best <= 24
        o, st = ctx.compute(dev(d), dev(fx), **kw)
        assert st.batch == best
        p, _ = ctx.compute(dev(d), dev(fx), **kw, flags=imf.FLAG_PLAIN)
        for k in ("imf", "imf_norm", "secluded", "masks"):
            assert torch.equal(o[k], p[k]), k
    finally:
        ctx.close()


def test_autotune_table_saved_and_loaded(imf_mod, tmp_path):
    """A tuned table written by one context and read by a fresh one: the
    fresh context uses the tuned batch and block parameters without tuning,
    with the same results; a malformed table is rejected and changes nothing."""
    imf = imf_mod
    d = W.design_3d_boxes_cyls(48, seed=97)
    fx = W.fixture_plate(d.shape, 3)
    kw = dict(tools=W.tool(W.TOOL_FLAT, 2, 10, 4, 8), dirs=W.fib_hemisphere(20),
              dir_kind=imf.DIR_F64, method=imf.METHOD_FFT)
    path = str(tmp_path / "tuned.txt")
    ctx = imf.Context(0)
    try:
        best = ctx.autotune(dev(d), dev(fx), **kw)
        o1, s1 = ctx.compute(dev(d), dev(fx), **kw)
        o1 = {k: v.clone() for k, v in o1.items()}
        ctx.autotune_save(path)
    finally:
        ctx.close()
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        f.write("imf-autotune 1\n1|48,48,48|96,96,96 0 2 6\n")   # batch 0 is invalid
    ctx = imf.Context(0)
    try:
        with pytest.raises(imf.IMFError):
            ctx.autotune_load(bad)
        assert ctx.autotune_load(path) >= 1
        o2, s2 = ctx.compute(dev(d), dev(fx), **kw)
        assert s2.batch == best == s1.batch
        assert (s2.mf_shape, s2.mf_wg_per_cu) == (s1.mf_shape, s1.mf_wg_per_cu)
        for k in ("imf", "imf_norm", "secluded", "masks"):
            assert torch.equal(o2[k], o1[k]), k
    finally:
        ctx.close()


def test_graph_replays_equal_eager(imf_mod):
    """The second identical request is captured into a HIP graph and later
    ones replay it; every replay equals the kernel-by-kernel result, with
    other (eager) requests and synchronizations on the context in between."""
    imf = imf_mod
    d = W.design_density(40, seed=95)
    fx = W.fixture_plate(d.shape, 3)
    kw = dict(tools=W.TOOL_C3, dirs=W.fib_hemisphere(12), dir_kind=imf.DIR_F64, lam=0.01,
              method=imf.METHOD_FFT)
    other = W.design_3d_boxes_cyls(32, seed=96)
    okw = dict(tools=W.TOOL_C2, dirs=W.lattice26()[:9], dir_kind=imf.DIR_LATTICE,
               method=imf.METHOD_FFT)
    ctx = imf.Context(0)
    try:
        dd, dfx, do = dev(d), dev(fx), dev(other)
        # persistent outputs: the signature includes the output pointers
        ref, _ = ctx.compute(dd, dfx, **kw, flags=imf.FLAG_NO_GRAPH)
        ref = {k: v.clone() for k, v in ref.items()}
        modes = []
        keep = {k: torch.empty_like(v) for k, v in ref.items()}
        for i in range(5):
            for v in keep.values():
                v.fill_(7)
            o, st = ctx.compute(dd, dfx, **kw, out=keep)
            modes.append(st.graph)
            for k in ("imf", "imf_norm", "secluded", "masks"):
                assert torch.equal(o[k], ref[k]), (i, k)
            ctx.compute(do, **okw, flags=imf.FLAG_NO_GRAPH)   # eager work in between
            torch.cuda.synchronize()
        # the first sighting launches kernel by kernel, the second is captured,
        # the rest replay
        assert modes == [0, 1, 2, 2, 2], modes
    finally:
        ctx.close()


def test_mix_equals_alone_large_grids(imf_mod):
    """Served requests of 128^3 to 256^3 (binary and density, both cutters,
    overlapping on the device) equal the same requests computed alone, bit
    for bit."""
    imf = imf_mod
    descs = W.serving_stream(6, seed=93, sizes=(128, 160, 192, 224, 256), master_dirs=24)
    reqs = [dict(W.serving_request(d, master_dirs=24), desc=d) for d in descs]
    ctx = imf.Context(0)
    try:
        inputs = [(dev(r["design"]), dev(r["fixture"])) for r in reqs]
        alone, passes = [], []
        for (d, fx), r in zip(inputs, reqs):
            print("alone", r["desc"]["n"], len(r["dirs"]), r["desc"]["density"], flush=True)
            o, st = ctx.compute(d, fx, **_kw(imf, r))
            alone.append({k: v.clone() for k, v in o.items()})
            passes.append(st.passes)
        print("served", flush=True)
        tickets = [ctx.submit(d, fx, **_kw(imf, r)) for (d, fx), r in zip(inputs, reqs)]
        for i, t in enumerate(tickets):
            o, st = ctx.wait(t)
            assert st.t_ms[7] >= st.queue_ms >= 0
            # host time planning and enqueueing under the context lock, and
            # waiting for it: both part of the time after admission
            assert st.hold_ms > 0 and st.lock_ms >= 0
            assert st.queue_ms + st.lock_ms + st.hold_ms <= st.t_ms[7] + 1e-3
            _same(o, alone[i], st.passes == passes[i], i, st.F_max, reqs[i]["lam"])
    finally:
        ctx.close()


def test_admission_passes_a_waiting_large_request(imf_mod):
    """While a long request runs, a large one whose workspace does not fit
    beside it waits; smaller requests behind it that fit are admitted ahead of
    it, at most four times, after which the queue waits for the large one.
    Every result equals the request computed alone."""
    imf = imf_mod
    big_d = W.design_3d_boxes_cyls(256, seed=94)
    long_d = W.design_density(112, seed=94)
    small_d = [W.design_3d_boxes_cyls(48, seed=95 + i) for i in range(6)]
    tl = W.tool(W.TOOL_BALL, 3, 20, 7, 16)
    dirs = W.fib_hemisphere(60)
    # no spectrum cache: the budget below is sized for the workspaces alone
    nc = imf.FLAG_NO_CACHE
    kw_big = dict(tools=tl, dirs=dirs[:24], dir_kind=imf.DIR_F64, method=imf.METHOD_FFT,
                  batch=4, flags=nc)
    kw_long = dict(tools=tl, dirs=dirs, dir_kind=imf.DIR_F64, method=imf.METHOD_FFT, batch=4,
                   lam=0.01, flags=nc)
    kw_small = dict(tools=tl, dirs=dirs[:6], dir_kind=imf.DIR_F64, method=imf.METHOD_FFT,
                    batch=2, flags=nc)
    big = (dev(big_d), dev(W.fixture_plate(big_d.shape, 3)))
    lng = (dev(long_d), dev(W.fixture_plate(long_d.shape, 3)))
    sml = [(dev(d), dev(W.fixture_plate(d.shape, 3))) for d in small_d]
    probe = imf.Context(0)
    try:
        F_big = probe.footprint(*big, **kw_big)
        F_long = probe.footprint(*lng, **kw_long)
        F_small = max(probe.footprint(*s, **kw_small) for s in sml)
        alone_big = {k: v.clone() for k, v in probe.compute(*big, **kw_big)[0].items()}
        alone_long = {k: v.clone() for k, v in probe.compute(*lng, **kw_long)[0].items()}
        alone_small = [{k: v.clone() for k, v in probe.compute(*s, **kw_small)[0].items()}
                       for s in sml]
    finally:
        probe.close()
    # every worker arena that can coexist fits the budget; the running
    # footprints may use half of it: the long request and three small ones
    # fit together, the large one fits only an idle context
    budget = F_long + F_big + 4 * F_small + (256 << 20)
    assert F_long + 3 * F_small <= budget // 2 < F_big + F_small, (F_big, F_long, F_small)
    ctx = imf.Context(0, budget_bytes=budget)
    try:
        assert ctx.footprint(*big, **kw_big) == F_big
        print("admission: long, large, 6 small", flush=True)
        t_long = ctx.submit(*lng, **kw_long)
        time.sleep(0.002)
        t_big = ctx.submit(*big, **kw_big)
        t_small = [ctx.submit(*s, **kw_small) for s in sml]
        o_long, st_long = ctx.wait(t_long)
        o_big, st_big = ctx.wait(t_big)
        res_small = [ctx.wait(t) for t in t_small]
        # the first four small requests ran before the large one was admitted
        for o, st in res_small[:4]:
            assert st.t_ms[7] <= st_big.queue_ms + 1.0, (st.t_ms[7], st_big.queue_ms)
        # the fifth and sixth were not admitted ahead of it
        for o, st in res_small[4:]:
            assert st.queue_ms >= st_big.queue_ms - 1.0, (st.queue_ms, st_big.queue_ms)
        for k in ("imf", "imf_norm", "secluded", "masks"):
            assert torch.equal(o_big[k], alone_big[k]), k
            assert torch.equal(o_long[k], alone_long[k]), k
            for i, (o, _) in enumerate(res_small):
                assert torch.equal(o[k], alone_small[i][k]), (i, k)
    finally:
        ctx.close()
