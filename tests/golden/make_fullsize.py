"""Writes the stored expected values of the full-size parity tests, calling
only the CPU oracle (oracle/) on the seeded workloads (workloads/):

* c2_128_binary_26.json: SHA-256 digests of the whole-grid oracle outputs of
  the 128^3 binary design x 26 lattice directions (f as int64, fbar float32,
  Gamma uint8, the masks as uint64 words), F_max, and the digest of the
  design and fixture they were computed from;
* c3_256_density_130_gamma.npz: exact gamma_R(x) (2^-24 units) at 256
  voxels of Omega_0 x all 130 orientations of the 256^3 density workload,
  the voxels drawn from four strata of the design (uniform over Omega_0, the
  layers just above the fixture plate, the material boundary rho in
  [0.3, 0.7], the solid rho > 0.99), seeded.

Run from the repository root: python tests/golden/make_fullsize.py [c2] [c3]
(both by default; the 256^3 samples take about 40 minutes on 8 cores, the
128^3 grid about 20)."""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def c3_strata(w, rng, per=64):
    """Voxels (x, y, z) of Omega_0 from four strata of the design."""
    om = w.fixture == 0
    rho = w.design
    zz = np.arange(rho.shape[0])[:, None, None]
    strata = [om,
              om & (zz >= 6) & (zz < 30),
              om & (rho >= 0.3) & (rho <= 0.7),
              om & (rho > 0.99)]
    pts = []
    for s in strata:
        z, y, x = np.nonzero(s)
        pick = rng.choice(len(x), size=per, replace=False)
        pts.append(np.stack([x[pick], y[pick], z[pick]], axis=1))
    return np.concatenate(pts).astype(np.int32)


def make_c2():
    w = W.c2()
    t = time.time()
    req = oracle.Request(w.design, w.fixture, tools=w.tool, dirs=w.dirs, dir_kind=1)
    o = oracle.imf(req)
    rec = {
        "workload": "128^3 binary, 26 lattice directions (workloads.c2)",
        "design_sha256": sha(w.design), "fixture_sha256": sha(w.fixture),
        "F_max": o["F_max"],
        "imf_int64_sha256": sha(o["imf"].astype(np.int64)),
        "imf_norm_float32_sha256": sha(o["imf_norm"].astype(np.float32)),
        "secluded_uint8_sha256": sha(o["secluded"].astype(np.uint8)),
        "masks_uint64_sha256": sha(o["masks"].astype(np.uint64)),
        "masks_equal_dilation_route": bool(np.array_equal(o["masks"], o["masks_dil"])),
    }
    assert rec["masks_equal_dilation_route"]
    with open(os.path.join(HERE, "c2_128_binary_26.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print("c2 written in %.0f s" % (time.time() - t), flush=True)


def make_c3():
    w = W.c3()
    t = time.time()
    req = oracle.Request(w.design, w.fixture, tools=w.tool, dirs=w.dirs, dir_kind=0, lam=w.lam)
    pts = c3_strata(w, np.random.default_rng(7627256))
    gam = np.zeros((len(w.dirs), len(pts)), np.int64)
    for i in range(0, len(pts), 16):
        gam[:, i:i + 16] = oracle.gamma_at_all(req, pts[i:i + 16])
        print("c3 %d/%d voxels, %.0f s" % (i + 16, len(pts), time.time() - t), flush=True)
    np.savez_compressed(os.path.join(HERE, "c3_256_density_130_gamma.npz"), points=pts, gamma=gam,
                        design_sha256=np.array(sha(w.design)),
                        fixture_sha256=np.array(sha(w.fixture)))
    print("c3 written in %.0f s" % (time.time() - t), flush=True)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c3"]
    if "c2" in which:
        make_c2()
    if "c3" in which:
        make_c3()
