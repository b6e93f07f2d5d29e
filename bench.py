#!/usr/bin/env python3
"""Throughput of the IMF hot path on one MI355X.

One step is one whole request of Algorithm 1 (Sec. 2.1.5) on the 256^3
density workload: rasters (cached), forward transform of rho_O, tool spectra
(cached after the warm-up), 130 fused product + inverse transforms, rounding /
guard band, sharp-point minimum with the running minimum over orientations,
F_max, fbar, B, Gamma and the 130 accessible masks (threshold lambda F_max).
Inputs are resident in HBM before the timed region.

Prints one JSON line: value = voxel-orientations per second (256^3 * 130 per
step / seconds per step), the roofline of the dominant kernel (its algorithmic
work / its event-timed duration), the HBM roofline of the transform passes, the
plain per-orientation path on the same GPU, a cold-cache request, the serving
mix (p50 / p99 latency under Poisson arrivals) and the CPU oracle timed on a
bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# kernel instances this run launched, per class whose instance depends on the
# launch configuration (set once the block shape in effect is known)
RUN_KERNELS = {}


def minfilter_kernels(shape):
    """Template instances of the sharp-point minimum's list pass and its bound
    for a block shape, with the default eight waves in step (None otherwise)."""
    if os.environ.get("IMF_MINFILTER_SYNC", "2") != "2":
        return {"minfilter": None, "bound": None}
    wx, wy, wz = {1: (32, 2, 1), 2: (16, 2, 2), 3: (16, 4, 1), 4: (8, 4, 2)}.get(shape, (64, 1, 1))
    return {"minfilter": ["void k_minfilter_list<%d, %d, %d, true, 8>" % (wx, wy, wz)],
            "bound": ["void k_bound<%d, %d, %d>" % (wx, wy, wz), "k_scan_masks",
                      "void k_scatter<%d, %d, %d>" % (wx, wy, wz)]}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE
    summary, or None when the kernel's source changed since it was measured or
    the summary covers another instance than the one this run launched."""
    import hashlib
    f = os.path.join(ROOT, "profiles", "traffic_c3_256x130.json")
    if not os.path.exists(f):
        return None
    e = json.load(open(f)).get(kernel)
    if not e:
        return None
    if kernel in RUN_KERNELS and RUN_KERNELS[kernel] != e.get("kernels"):
        return None
    src = os.path.join(ROOT, e["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != e["sha256"]:
        return None
    return e["bytes_per_launch"] or None


# on-chip vector memory rate: 16 lanes (4-byte dwords) per clock per CU,
# 256 CUs at 2.4 GHz -> 9.83e12 lane loads/s = 39.3 TB/s of gathered data.
# Derived from unit counts, not a published peak: reported beside the HBM
# roofline only, as the rate at which the sharp-point minimum gathers.
GATHER_RATE_GBS = 256 * 16 * 4 * 2.4


def minfilter_bytes_per_launch(st, N):
    """Algorithmic HBM bytes of one launch of the sharp-point minimum (one
    orientation): the query box of g read once (4 M^3, M^3 the orientation's box
    volume), the running minimum f read and written (8 N^3), the orientation's
    mask bits (N^3 / 8) and, for masks at lambda F_max, its gamma written (4 N^3)."""
    return 4.0 * st.box_voxels / st.n_orient + N * (8.0 + 1.0 / 8.0 + 4.0)


def roofline_of(cls, kms, kn, kb, ko, st=None, N=None):
    """HBM roofline of one kernel class: algorithmic bytes per launch (the
    minimum pass by the model above, the others by the library's count of
    their compulsory reads and writes) over the event-timed launch duration."""
    avg_ms = kms[cls] / kn[cls]
    if cls == "minfilter":
        work = minfilter_bytes_per_launch(st, N)
    else:
        work = kb[cls] / kn[cls]
    achieved = work / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(cls)
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "traffic_over_algorithmic": round(traffic / work, 3) if traffic else None,
           "kernel": cls, "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": work}
    if cls == "minfilter":
        out["bytes_model"] = "4 M^3 + 8 N^3 + N^3/8 + 4 N^3 per orientation"
        g = 4.0 * ko[cls] / kn[cls] / (avg_ms * 1e-3) / 1e9
        out["gather_rate"] = {"achieved": round(g, 1), "unit": "GB/s",
                              "vector_memory_lane_rate": GATHER_RATE_GBS,
                              "frac": round(g / GATHER_RATE_GBS, 4),
                              "note": "gathered lane bytes of the computed blocks; the lane "
                                      "rate is derived from unit counts and clock"}
    return out


def serving_leg(imf, W, torch, n_req=64, load=0.7, seed=7627004, other_loads=(0.3, 1.0)):
    """The serving mix: n_req requests (grids 64..256^3, binary or density,
    flat or ball cutter, 6-130 orientations of one master Fibonacci set).
    A back-to-back pass calibrates the saturation rate (and fills the spectrum
    cache); the mix is then replayed with Poisson arrivals at `load` times that
    rate, and the submit-to-completion latencies give p50 / p99.  The same
    arrivals, rescaled, are replayed at `other_loads` times the rate as well."""
    import numpy as np
    descs = W.serving_stream(n_req, seed=seed)
    cache = {}
    reqs = []
    for d in descs:
        key = (d["n"], d["density"])
        if key not in cache:
            r = W.serving_request(d)
            cache[key] = (torch.from_numpy(r["design"]).cuda(),
                          torch.from_numpy(r["fixture"]).cuda(), r["lam"])
        des, fx, lam = cache[key]
        reqs.append((des, fx, dict(tools=d["tool"], dirs=W.fib_hemisphere(130)[d["dir_index"]],
                                   dir_kind=imf.DIR_F64, lam=lam, method=imf.METHOD_FFT)))
    ctx = imf.Context(0)
    vo = sum(int(r[0].numel()) * len(r[2]["dirs"]) for r in reqs)

    def replay(ld, t_sat):
        rate = ld * n_req / t_sat
        arrive = np.array([d["t"] for d in descs]) * (1.0 / rate) / (descs[-1]["t"] / n_req)
        tickets = []
        t0 = time.perf_counter()
        for (des, fx, kw), ta in zip(reqs, arrive):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets.append(ctx.submit(des, fx, **kw))
        sts = [ctx.wait(t)[1] for t in tickets]
        return sts, time.perf_counter() - t0, rate

    try:
        alone = []
        t0 = time.perf_counter()
        for des, fx, kw in reqs:
            _, st = ctx.compute(des, fx, **kw)
            alone.append(st.t_ms[7])
        torch.cuda.synchronize()
        t_sat = time.perf_counter() - t0
        sts, t_all, rate = replay(load, t_sat)
        others = {}
        for ld in other_loads:
            s2, t2, r2 = replay(ld, t_sat)
            lat2 = np.array([st.t_ms[7] for st in s2])
            others["%.1f" % ld] = {
                "arrival_rate_per_s": round(r2, 2),
                "p50_ms": round(float(np.percentile(lat2, 50)), 2),
                "p99_ms": round(float(np.percentile(lat2, 99)), 2),
                "throughput_vo_per_s": vo / t2,
                "slowdown_p50": round(float(np.percentile(lat2 / np.array(alone), 50)), 2),
                "slowdown_p99": round(float(np.percentile(lat2 / np.array(alone), 99)), 2)}
    finally:
        ctx.close()
    lat = np.array([st.t_ms[7] for st in sts])
    queued = np.array([st.queue_ms for st in sts])
    lockw = np.array([st.lock_ms for st in sts])
    hold = np.array([st.hold_ms for st in sts])
    alone = np.array(alone)
    slow = lat / alone
    i99 = int(np.argsort(lat)[min(n_req - 1, int(round(0.99 * (n_req - 1))))])
    return {"requests": n_req, "load": load, "arrival_rate_per_s": round(rate, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2),
            "throughput_vo_per_s": vo / t_all,
            "saturation_vo_per_s": vo / t_sat,
            # each request's latency over its own time back to back (the
            # calibration pass): separates waiting from the mix of sizes
            "alone_p50_ms": round(float(np.percentile(alone, 50)), 2),
            "alone_max_ms": round(float(alone.max()), 2),
            "slowdown_p50": round(float(np.percentile(slow, 50)), 2),
            "slowdown_p99": round(float(np.percentile(slow, 99)), 2),
            "queue_p50_ms": round(float(np.percentile(queued, 50)), 2),
            "queue_p99_ms": round(float(np.percentile(queued, 99)), 2),
            # host time waiting for the context lock / holding it (planning
            # and enqueueing), per request
            "lock_wait_p50_ms": round(float(np.percentile(lockw, 50)), 2),
            "lock_wait_p99_ms": round(float(np.percentile(lockw, 99)), 2),
            "lock_hold_p50_ms": round(float(np.percentile(hold, 50)), 2),
            "lock_hold_p99_ms": round(float(np.percentile(hold, 99)), 2),
            "p99_request": {"grid": int(descs[i99]["n"]), "orientations": len(reqs[i99][2]["dirs"]),
                            "density": bool(descs[i99]["density"]),
                            "alone_ms": round(float(alone[i99]), 2),
                            "latency_ms": round(float(lat[i99]), 2)},
            # the same arrivals at other multiples of the saturation rate
            "other_loads": others}


def to_loop_leg(imf, W, torch, iters):
    """The TO-loop workload: a 384^3 density design with fixture plate and two
    clamp blocks, flat cutter r3 L80 + holder r12 L80, 512 Fibonacci-hemisphere
    orientations, lambda 0.01, masks at lambda F_max; every iteration perturbs
    rho by seeded smooth noise (amplitude 0.05, generated on the device) and
    recomputes the IMF on one context, so tool spectra are reused (those that
    fit the cache) and lambda times the last F_max is the expected threshold.
    Reports seconds per iteration and each iteration's cache hits, passes and
    whether the expected threshold's bracket held."""
    w = W.c5()
    dev = torch.device("cuda:0")
    fx = torch.from_numpy(w.fixture).to(dev)
    rho = torch.from_numpy(w.design).to(dev)
    kw = dict(tools=w.tool, dirs=w.dirs, dir_kind=imf.DIR_F64, lam=w.lam, tau=w.tau,
              method=imf.METHOD_FFT)
    ctx = imf.Context(0)
    its = []
    out = None
    try:
        for i in range(iters):
            if i:
                rho = W.perturb_density_device(rho, seed=7627005 + i)
            torch.cuda.synchronize()
            t = time.perf_counter()
            out, st = ctx.compute(rho, fx, **kw, out=out)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            its.append({"s": round(dt, 4), "hits": st.cache_hits, "misses": st.cache_misses,
                        "passes": st.passes, "hinted": st.hinted, "F_max": st.F_max,
                        "listed": st.band_entries})
            log("TO loop iteration %d: %.2f s (spectra cached %d, computed %d, passes %d, "
                "bracket %s, %d listed, F_max %.4f)" % (
                    i, dt, st.cache_hits, st.cache_misses, st.passes,
                    {0: "-", 1: "held", 2: "missed", 3: "overflowed"}[st.hinted],
                    st.band_entries, st.F_max))
    finally:
        ctx.close()
        del out
        torch.cuda.empty_cache()
    N = int(np.prod(w.design.shape))
    steady = [x["s"] for x in its[1:]] or [its[0]["s"]]
    return {"workload": "384^3 density, fixture plate + clamps, flat r3 L80 + holder r12 L80, "
                        "512 Fibonacci-hemisphere orientations, lambda 0.01, masks at "
                        "lambda*F_max, rho perturbed each iteration (amplitude 0.05)",
            "iterations": len(its), "s_per_iteration_median": float(np.median(steady)),
            "s_first_iteration": its[0]["s"], "s_total": float(sum(x["s"] for x in its)),
            "voxel_orientations_per_s": N * len(w.dirs) / float(np.median(steady)),
            "per_iteration": its}


def cpu_baseline(w, target_s=15.0):
    """The CPU oracle as it stands on a crop of the same workload: the full
    pipeline (exact overlaps over the query box, sharp-point minimum, masks off)
    for one orientation of the 130, on an n^3 corner crop of the 256^3 design
    and fixture; n is chosen from a short calibration run to take ~target_s."""
    import numpy as np

    import oracle

    def run(n, k):
        d = np.ascontiguousarray(w.design[:n, :n, :n])
        fx = np.ascontiguousarray(w.fixture[:n, :n, :n])
        req = oracle.Request(d, fx, tools=w.tool, dirs=w.dirs[k:k + 1], dir_kind=0,
                             lam=w.lam)
        t = time.perf_counter()
        oracle.imf(req, masks=False)
        return time.perf_counter() - t

    k = 64
    n0 = 40
    t0 = run(n0, k)
    # cost ~ (n + e)^3 |T| with e ~ 60 for this tool: solve for the crop size
    n = n0
    for cand in range(n0, 257, 8):
        pred = t0 * ((cand + 60.0) / (n0 + 60.0)) ** 3
        if pred > target_s:
            break
        n = cand
    t = run(n, k)
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    # one core: the same pipeline in a child process with one OpenMP thread, on
    # the smallest crop (its cost is the overlaps over the query box, whose
    # sides are the crop plus the cutter's extent); scaled to the all-core
    # sample by the ratio of the two query boxes
    def box(m):
        d = np.ascontiguousarray(w.design[:m, :m, :m])
        info = oracle.orient_info(oracle.Request(d, None, tools=w.tool, dirs=w.dirs[k:k + 1],
                                                 dir_kind=0), 0)
        return float(np.prod([m + info["kmax"][a] - info["kmin"][a] for a in range(3)]))
    n1 = 16
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r); import numpy as np; import oracle; "
            "import workloads as W; w = W.c3(); n = %d; k = %d; "
            "req = oracle.Request(np.ascontiguousarray(w.design[:n, :n, :n]), "
            "np.ascontiguousarray(w.fixture[:n, :n, :n]), tools=w.tool, dirs=w.dirs[k:k + 1], "
            "dir_kind=0, lam=w.lam); t = time.perf_counter(); oracle.imf(req, masks=False); "
            "print(time.perf_counter() - t)" % (ROOT, n1, k))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    one = None
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=600)
        t1c = float(r.stdout.strip().splitlines()[-1])
        t_scaled = t1c * box(n) / box(n1)
        one = {"value": n ** 3 / t_scaled, "cores": 1, "measured_s": round(t1c, 2),
               "sample": "%d^3 corner crop, orientation %d, %.1f s on one core, scaled to the "
                         "%d^3 sample by the query-box volume (%.0f s)"
                         % (n1, k, t1c, n, t_scaled),
               "parallel_speedup": round(t_scaled / t, 1)}
    except Exception as e:  # the all-core figure stands alone
        log("one-core oracle run failed: %s" % e)
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": n ** 3 / t, "unit": "voxel-orientations/s", "cores": cores,
            "kind": "oracle", "cpu_model": model, "one_core": one,
            "sample": "%d^3 corner crop of the 256^3 design + fixture, orientation %d of 130, "
                      "full oracle pipeline (int64 overlaps over the query box, sharp-point "
                      "min), %.1f s" % (n, k, t)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain 1 GiB device copy (stream-copy bandwidth; the reference "
                         "kernel for the FETCH_SIZE / WRITE_SIZE counter scale); on by default "
                         "unless --no-copy-probe")
    ap.add_argument("--no-copy-probe", action="store_true")
    ap.add_argument("--to-loop-iters", type=int, default=50,
                    help="iterations of the 384^3 x 512 TO loop (0: skip the leg)")
    ap.add_argument("--only-to-loop", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the IMF path here runs on a single MI355X "
              "(--gpus %d is not supported; orientation sharding across GPUs is a design "
              "note, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2002_07627_amd as imf
    import workloads as W

    if args.only_to_loop:
        print(json.dumps({"to_loop": to_loop_leg(imf, W, torch, args.to_loop_iters)}), flush=True)
        return

    copy_gbs = None
    if args.copy_probe or not args.no_copy_probe:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(10):
            y.copy_(x)
        torch.cuda.synchronize()
        copy_gbs = 10 * 2 * x.numel() * 4 / (time.perf_counter() - t) / 1e9
        log("stream copy (1 GiB read + 1 GiB write): %.0f GB/s" % copy_gbs)
        del x, y
    log("generating the 256^3 density workload")
    w = W.c3()
    N = int(np.prod(w.design.shape))
    nR = len(w.dirs)
    dev = torch.device("cuda:0")
    design = torch.from_numpy(w.design).to(dev)
    fixture = torch.from_numpy(w.fixture).to(dev)
    ctx = imf.Context(0)
    kw = dict(tools=w.tool, dirs=w.dirs, dir_kind=imf.DIR_F64, lam=w.lam, tau=w.tau,
              method=imf.METHOD_FFT, batch=args.batch)
    tuned = None
    if not args.no_autotune and args.batch == 0:
        t1 = time.perf_counter()
        tuned = ctx.autotune(design, fixture, **kw)
        log("autotune: batch %d (%.1f s)" % (tuned, time.perf_counter() - t1))
    for i in range(args.warmup):
        _, st = ctx.compute(design, fixture, **kw)
        log("warmup %d: %.1f ms (cache hits %d, misses %d)" % (i, st.t_ms[7], st.cache_hits,
                                                                 st.cache_misses))
    torch.cuda.synchronize()
    stats, per_step = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        _, st = ctx.compute(design, fixture, **kw, flags=imf.FLAG_PROFILE)  # returns when done
        per_step.append(time.perf_counter() - t1)
        stats.append(st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = 1000 * el / args.steps
    value = N * nR / (el / args.steps)
    log("timed: %.2f ms/step, %.3e voxel-orientations/s (block shape %d, %d workgroups/CU, "
        "%d orientations with lattice-vector runs)" % (ms, value, stats[-1].mf_shape,
                                                      stats[-1].mf_wg_per_cu,
                                                      stats[-1].lattice_runs))
    if stats[-1].bound_blocks:
        log("bound: %d of %d (block, orientation) pairs skipped (%.1f%%)" % (
            stats[-1].bound_skipped, stats[-1].bound_blocks,
            100.0 * stats[-1].bound_skipped / stats[-1].bound_blocks))

    # per kernel class over the timed steps
    kms, kn, kb, ko = {}, {}, {}, {}
    for st in stats:
        for k, v in st.kernel_ms.items():
            kms[k] = kms.get(k, 0) + v
            kn[k] = kn.get(k, 0) + st.kernel_launches[k]
            kb[k] = kb.get(k, 0) + st.kernel_bytes[k]
            ko[k] = ko.get(k, 0) + st.kernel_ops[k]
    dom = max(kms, key=kms.get)
    kernels = {k: {"ms_per_step": kms[k] / args.steps, "launches_per_step": kn[k] / args.steps,
                   "GBps": (kb[k] / (kms[k] * 1e-3) / 1e9) if kms[k] > 0 else None}
               for k in sorted(kms, key=kms.get, reverse=True)}
    for k, v in kernels.items():
        log("  %-14s %8.2f ms/step  %5.1f launches  %s GB/s" %
            (k, v["ms_per_step"], v["launches_per_step"],
             "%.0f" % v["GBps"] if v["GBps"] else "-"))
    RUN_KERNELS.update(minfilter_kernels(stats[-1].mf_shape))
    # the committed traffic covers the default transform plan of each pass
    for i, k in enumerate(("inv_z_product", "inv_y", "inv_x_c2r")):
        if (stats[-1].fft_plan >> (2 * i)) & 3:
            RUN_KERNELS[k] = "plan %d" % ((stats[-1].fft_plan >> (2 * i)) & 3)
    roofline = roofline_of(dom, kms, kn, kb, ko, stats[-1], N)
    # measured HBM traffic of the whole request: per-launch FETCH + WRITE bytes
    # of the committed counter runs times this run's launches, for the kernel
    # classes those runs cover (null when any of them changed since)
    hbm_req = None
    tr = {k: measured_traffic(k) for k in ("minfilter", "bound", "inv_z_product", "inv_y",
                                           "inv_x_c2r", "levels")}
    if all(v is not None for v in tr.values()) and all(k in kn for k in tr):
        b_req = sum(tr[k] * kn[k] / args.steps for k in tr)
        covered_ms = sum(kms[k] / args.steps for k in tr)
        hbm_req = {"bytes_per_request": b_req, "GBps_over_request": b_req / (ms * 1e-3) / 1e9,
                   "frac_of_peak": b_req / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                   "classes": sorted(tr), "share_of_request_time": covered_ms / ms}
    # the transform passes are HBM-bound: their roofline beside the dominant one
    fft = {k: roofline_of(k, kms, kn, kb, ko) for k in ("inv_z_product", "inv_y", "inv_x_c2r")
           if k in kms}

    # the same request replayed from a captured HIP graph (persistent outputs:
    # the first call launches kernel by kernel, the second is captured)
    keep = None
    for i in range(2):
        keep, sg = ctx.compute(design, fixture, **kw, out=keep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        _, sg = ctx.compute(design, fixture, **kw, out=keep)
    torch.cuda.synchronize()
    graph_ms = 1000 * (time.perf_counter() - t1) / args.steps
    log("graph replay: %.2f ms/step (mode %d)" % (graph_ms, sg.graph))
    del keep

    plain = None
    if not args.no_plain:
        tps = []
        for i in range(3):
            t1 = time.perf_counter()
            _, sp = ctx.compute(design, fixture, **dict(kw, batch=0), flags=imf.FLAG_PLAIN)
            torch.cuda.synchronize()
            tps.append(time.perf_counter() - t1)
        tp = float(np.median(tps))
        plain = {"value": N * nR / tp, "ms_per_step": 1000 * tp, "runs": 3,
                 "ms_each": [round(1000 * t, 2) for t in tps],
                 "speedup": (N * nR / (el / args.steps)) / (N * nR / tp)}
        log("plain path: %.1f ms (median of 3)" % (1000 * tp))
    # TO-coupling steps on the same grid (pointwise, HBM-bound) and the greedy
    # machining plan from the request's masks
    coupling = None
    out_c, _ = ctx.compute(design, fixture, **kw)
    xi = torch.rand(design.shape, device=dev, generator=torch.Generator(device=dev).manual_seed(1))
    sens = -xi.pow(3)
    ctx.heaviside(xi, 8.0)
    ctx.access_filter(design, out_c["imf_norm"], out_c["secluded"], fixture, sens=sens, w=0.3)
    torch.cuda.synchronize()
    reps = 20
    t1 = time.perf_counter()
    for i in range(reps):
        rho_c = ctx.heaviside(xi, 8.0)
    torch.cuda.synchronize()
    t_h = (time.perf_counter() - t1) / reps
    t1 = time.perf_counter()
    for i in range(reps):
        ctx.access_filter(design, out_c["imf_norm"], out_c["secluded"], fixture, sens=sens, w=0.3)
    torch.cuda.synchronize()
    t_f = (time.perf_counter() - t1) / reps
    t1 = time.perf_counter()
    plan, left = ctx.plan_greedy(out_c["masks"], design, fixture)
    t_p = time.perf_counter() - t1
    # bytes: Heaviside reads xi, writes rho; the filter reads the design, fbar,
    # Gamma, S_phi (twice: max, then combine), the filter, and writes both fields
    bh, bf = 8.0 * N, N * (4 + 4 + 1 + 4 + 4 + 4 + 4 + 4 + 1)
    coupling = {"heaviside_ms": 1000 * t_h, "heaviside_GBps": bh / t_h / 1e9,
                "access_filter_ms": 1000 * t_f, "access_filter_GBps": bf / t_f / 1e9,
                "plan_ms": 1000 * t_p, "plan_steps": len(plan), "plan_left": left}
    log("coupling: heaviside %.3f ms (%.0f GB/s), filter + sensitivity %.3f ms (%.0f GB/s), "
        "greedy plan %d steps in %.1f ms" % (1000 * t_h, bh / t_h / 1e9, 1000 * t_f,
                                             bf / t_f / 1e9, len(plan), 1000 * t_p))
    del out_c, xi, sens, rho_c
    # fixtures that change with the setup: four vise setups, the orientations
    # grouped by azimuth sector (one extra design transform and prefix sum per
    # setup, batches split at setup changes)
    n_sets = 4
    fof = W.setup_of_dirs(w.dirs, n_sets)
    order = np.argsort(fof, kind="stable")
    sets = torch.from_numpy(W.setup_clamps(w.design.shape, n_sets)).to(dev)
    skw = dict(kw, dirs=w.dirs[order])
    ctx.compute(design, fixture, **skw, fixture_sets=sets, fixture_of=fof[order])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        _, ss = ctx.compute(design, fixture, **skw, fixture_sets=sets, fixture_of=fof[order],
                            flags=imf.FLAG_NO_GRAPH)
    torch.cuda.synchronize()
    set_ms = 1000 * (time.perf_counter() - t1) / args.steps
    setups = {"n_sets": n_sets, "ms_per_step": set_ms, "value": N * nR / (set_ms * 1e-3),
              "vs_one_fixture": ms / set_ms}
    log("%d setups with their own fixtures: %.2f ms/step" % (n_sets, set_ms))
    del sets
    ctx.close()
    # cold tool-spectrum cache: the same request on a fresh context (every
    # spectrum, raster and workspace made anew), median of 5 after 2 warm-ups.
    # A context made right after another one's ~30 GB were released can stall
    # for seconds; two idle seconds after each destroy avoid that.
    cold_runs = []
    for i in range(7):
        ctx = imf.Context(0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, sc = ctx.compute(design, fixture, **kw)
        torch.cuda.synchronize()
        if i >= 2:
            cold_runs.append(1000 * (time.perf_counter() - t1))
        ctx.close()
        time.sleep(2.0)
    cold_ms = float(np.median(cold_runs))
    log("cold-cache request: %.1f ms median of %d fresh contexts (%d spectra computed)" % (
        cold_ms, len(cold_runs), sc.cache_misses))
    del design, fixture
    torch.cuda.empty_cache()

    serving = None
    if not args.no_serving:
        log("serving mix: 64 requests, Poisson arrivals at 0.7x saturation")
        serving = serving_leg(imf, W, torch)
        log("serving: p50 %.1f ms, p99 %.1f ms, %.3e voxel-orientations/s" % (
            serving["p50_ms"], serving["p99_ms"], serving["throughput_vo_per_s"]))
        log("serving: slowdown (latency / back-to-back time) p50 %.2f, p99 %.2f; queue p50 %.1f "
            "ms, p99 %.1f ms; back-to-back p50 %.1f ms, max %.1f ms" % (
                serving["slowdown_p50"], serving["slowdown_p99"], serving["queue_p50_ms"],
                serving["queue_p99_ms"], serving["alone_p50_ms"], serving["alone_max_ms"]))
        for ld, v in serving["other_loads"].items():
            log("serving at %sx saturation: p50 %.1f ms, p99 %.1f ms, %.3e voxel-orientations/s" % (
                ld, v["p50_ms"], v["p99_ms"], v["throughput_vo_per_s"]))
        torch.cuda.empty_cache()

    to_loop = None
    if args.to_loop_iters > 0:
        log("TO loop: 384^3 x 512 orientations, %d iterations" % args.to_loop_iters)
        to_loop = to_loop_leg(imf, W, torch, args.to_loop_iters)
        log("TO loop: %.2f s per iteration (median), first %.2f s" % (
            to_loop["s_per_iteration_median"], to_loop["s_first_iteration"]))

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(w)
        log("cpu oracle: %.3e voxel-orientations/s (%s)" % (cpu["value"], cpu["sample"]))

    last = stats[-1]
    line = {
        "metric": "IMF voxel-orientations/s at 256^3\u00d7130 orient. vs plain; "
                  "p50/p99 request latency",
        "value": value, "unit": "voxel-orientations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms,
        "ms_per_step_median": 1000 * float(np.median(per_step)), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "256^3 density (sigmoid of sigma-4 smoothed noise, mean 0.35, "
                               "2^-24 grid), fixture plate z<6, ball cutter r4 L60 + holder "
                               "r14 L60, 130 Fibonacci-hemisphere orientations, lambda 0.01, "
                               "masks at lambda*F_max",
                   "grid": list(w.design.shape), "orientations": nR, "P": list(last.P),
                   "batch": last.batch, "autotuned": tuned is not None,
                   "minfilter_block_shape": last.mf_shape, "minfilter_wg_per_cu": last.mf_wg_per_cu,
                   "fft_plan": {"inv_z": last.fft_plan & 3, "inv_y": (last.fft_plan >> 2) & 3,
                                "inv_x": (last.fft_plan >> 4) & 3,
                                "bits": "1: one stage per radix 8,4,2,3,5,7; 2: half-width tiles"},
                   "lattice_run_orientations": last.lattice_runs,
                   "spectra": "cached (warm)"},
        "roofline": roofline,
        "roofline_transform_passes": fft,
        "cpu_baseline": cpu,
        "plain": plain,
        "cold_cache_ms": cold_ms,
        "cold_cache_runs_ms": [round(t, 2) for t in cold_runs],
        "graph_replay_ms_per_step": graph_ms,
        "coupling": coupling,
        "setups": setups,
        "serving": serving,
        "to_loop": to_loop,
        "kernels": kernels,
        "guard": {"F_max": last.F_max, "E": last.guard_band, "max_abs_err": last.max_abs_err,
                  "flags": last.guard_flags, "band_entries": last.band_entries,
                  "post_exact": last.post_exact, "passes": last.passes},
        "bound": {"blocks": last.bound_blocks, "skipped": last.bound_skipped,
                  "frac": (last.bound_skipped / last.bound_blocks) if last.bound_blocks else None},
        "stream_copy_GBps": copy_gbs,
        "request_hbm_traffic": hbm_req,
        "model_bytes_per_step": last.model_bytes,
        "model_GBps": last.model_bytes / (ms * 1e-3) / 1e9,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
