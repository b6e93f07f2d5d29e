"""Seeded generators for designs, fixtures, tools and orientation sets.

Conventions shared by every consumer:

* arrays are indexed ``[z][y][x]`` (``[y][x]`` in 2D), x fastest, voxel centres
  at integer indices;
* the random source is ``numpy.random.Generator(PCG64(seed))``; when a fill band
  is missed the draw is repeated with ``seed + 1000*k`` (k = 1, 2, ...);
* density designs are float32 values on the 2**-24 grid in [0, 1], so every
  overlap sum is an exact multiple of 2**-24;
* a direction is the unit tool axis pointing from the cutter tip toward the
  holder (the tool approaches the part along ``-d``).

The workloads stand in for the paper's parts (cantilever, GE bracket,
quadcopter and support bracket of the Results section), whose geometry is not
available: the grids span the paper's scales up to 384^3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# tool kinds, same numbering as the C interface
TOOL_FLAT = 0
TOOL_BALL = 1
TOOL_RECT2D = 2

Q24 = float(1 << 24)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# tools
# --------------------------------------------------------------------------

def tool(kind: int, cutter_r: float, cutter_len: float, holder_r: float,
         holder_len: float) -> dict:
    """A cutter of radius/half-width ``cutter_r`` occupying axial [0, L) and a
    holder of radius/half-width ``holder_r`` occupying axial [L, L+holder_len)."""
    return {"kind": int(kind), "cutter_r": float(cutter_r),
            "cutter_len": float(cutter_len), "holder_r": float(holder_r),
            "holder_len": float(holder_len)}


TOOL_C1 = tool(TOOL_RECT2D, 1.5, 24.0, 4.5, 30.0)   # 3x24 cutter, 9x30 holder
TOOL_C2 = tool(TOOL_FLAT, 3.0, 40.0, 10.0, 40.0)    # flat end mill
TOOL_C3 = tool(TOOL_BALL, 4.0, 60.0, 14.0, 60.0)    # ball end mill
TOOL_C5 = tool(TOOL_FLAT, 3.0, 80.0, 12.0, 80.0)


# --------------------------------------------------------------------------
# orientation sets (input data, shared byte for byte)
# --------------------------------------------------------------------------

def circle8() -> np.ndarray:
    """The 8 lattice directions of the plane, as int32 [8, 2] (x, y)."""
    return np.array([(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1),
                     (0, -1), (1, -1)], dtype=np.int32)


def lattice26() -> np.ndarray:
    """The 26 face/edge/corner directions of the cube, int32 [26, 3] (x, y, z)."""
    out = []
    for z in (-1, 0, 1):
        for y in (-1, 0, 1):
            for x in (-1, 0, 1):
                if (x, y, z) != (0, 0, 0):
                    out.append((x, y, z))
    return np.array(out, dtype=np.int32)


def fib_hemisphere(n: int) -> np.ndarray:
    """n directions on the upper hemisphere, float64 [n, 3] (x, y, z).

    z_i = 1 - (i + 1/2)/n, phi_i = i*pi*(3 - sqrt 5)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (i + 0.5) / n
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)


def unit_rows(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# --------------------------------------------------------------------------
# designs
# --------------------------------------------------------------------------

def design_2d_discs_rects(n: int = 128, seed: int = 7627001,
                          band=(0.35, 0.45)) -> np.ndarray:
    """Union of 12 discs and 8 axis-aligned rectangles, u8 [n, n]."""
    s = n / 128.0
    yy, xx = np.mgrid[0:n, 0:n]
    for k in range(64):
        r = _rng(seed + 1000 * k)
        img = np.zeros((n, n), dtype=bool)
        for _ in range(12):
            cx, cy = r.uniform(0, n, size=2)
            rad = r.uniform(6, 20) * s
            img |= (xx - cx) ** 2 + (yy - cy) ** 2 <= rad * rad
        for _ in range(8):
            cx, cy = r.uniform(0, n, size=2)
            w, h = (r.integers(8, 41, size=2) * s).round().astype(int)
            w, h = max(w, 1), max(h, 1)
            x0, y0 = int(math.floor(cx - w / 2)), int(math.floor(cy - h / 2))
            img[max(y0, 0):max(y0 + h, 0), max(x0, 0):max(x0 + w, 0)] = True
        fill = img.mean()
        if band[0] <= fill <= band[1]:
            return img.astype(np.uint8)
    raise RuntimeError("fill band not reached")


def design_3d_boxes_cyls(n: int = 128, seed: int = 7627002,
                         band=(0.25, 0.35)) -> np.ndarray:
    """10 boxes and 10 cylinders minus 10 through-holes, u8 [n, n, n]."""
    s = n / 128.0
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                             indexing="ij")
    coords = (xx, yy, zz)
    for k in range(64):
        r = _rng(seed + 1000 * k)
        vol = np.zeros((n, n, n), dtype=bool)
        for _ in range(10):
            c = r.uniform(0, n, size=3)
            sides = np.maximum((r.integers(16, 65, size=3) * s).round(), 1)
            m = np.ones_like(vol)
            for a in range(3):
                lo = int(math.floor(c[a] - sides[a] / 2))
                m &= (coords[a] >= lo) & (coords[a] < lo + int(sides[a]))
            vol |= m
        for _ in range(10):
            ax = int(r.integers(0, 3))
            rad = r.uniform(4, 14) * s
            ln = max(int(round(r.uniform(20, 96) * s)), 1)
            c = r.uniform(0, n, size=3)
            p, q = [a for a in range(3) if a != ax]
            m = (coords[p] - c[p]) ** 2 + (coords[q] - c[q]) ** 2 <= rad * rad
            lo = int(math.floor(c[ax] - ln / 2))
            m &= (coords[ax] >= lo) & (coords[ax] < lo + ln)
            vol |= m
        for _ in range(10):
            ax = int(r.integers(0, 3))
            rad = r.uniform(2, 6) * s
            c = r.uniform(0, n, size=3)
            p, q = [a for a in range(3) if a != ax]
            vol &= ~((coords[p] - c[p]) ** 2 + (coords[q] - c[q]) ** 2
                     <= rad * rad)
        fill = vol.mean()
        if band[0] <= fill <= band[1]:
            return vol.astype(np.uint8)
    raise RuntimeError("fill band not reached")


def _periodic_gauss_filter(a: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian filter (truncated at 4 sigma) with periodic wrap."""
    out = np.fft.rfftn(a)
    half = int(math.ceil(4 * sigma))
    taps = np.exp(-0.5 * (np.arange(-half, half + 1) / sigma) ** 2)
    taps /= taps.sum()
    for ax in range(a.ndim):
        n = a.shape[ax]
        ker = np.zeros(n)
        for j, t in zip(range(-half, half + 1), taps):
            ker[j % n] += t
        kf = np.fft.rfft(ker) if ax == a.ndim - 1 else np.fft.fft(ker)
        shape = [1] * a.ndim
        shape[ax] = kf.shape[0]
        out = out * kf.reshape(shape)
    return np.fft.irfftn(out, s=a.shape, axes=tuple(range(a.ndim)))


def quantize_q24(rho: np.ndarray) -> np.ndarray:
    """Round to the 2**-24 grid and clip to [0, 1]; float32 (exactly)."""
    q = np.rint(np.clip(rho, 0.0, 1.0) * Q24) / Q24
    return q.astype(np.float32)


def smooth_noise(shape, seed: int, sigma: float = 4.0) -> np.ndarray:
    """Standardized Gaussian-filtered white noise (float64)."""
    r = _rng(seed)
    n = _periodic_gauss_filter(r.standard_normal(shape), sigma)
    n -= n.mean()
    n /= n.std()
    return n


def design_density(n: int = 256, seed: int = 7627003, mean: float = 0.35,
                   ndim: int = 3, sigma: float = 4.0) -> np.ndarray:
    """Sigmoid of smooth noise with mean ``mean`` (+-0.001), on the 2**-24 grid."""
    shape = (n,) * ndim
    nz = smooth_noise(shape, seed, sigma).astype(np.float32)
    lo, hi = -6.0, 6.0
    for _ in range(60):
        c = 0.5 * (lo + hi)
        m = float(np.mean(1.0 / (1.0 + np.exp(-6.0 * (nz - np.float32(c)))),
                          dtype=np.float64))
        if abs(m - mean) <= 0.0005:
            break
        if m > mean:
            lo = c
        else:
            hi = c
    rho = 1.0 / (1.0 + np.exp(-6.0 * (nz.astype(np.float64) - c)))
    return quantize_q24(rho)


def perturb_density(rho: np.ndarray, seed: int, amp: float = 0.05) -> np.ndarray:
    """One TO-loop update stand-in: rho + amp * smooth noise, clipped, quantized."""
    n = smooth_noise(rho.shape, seed)
    return quantize_q24(rho.astype(np.float64) + amp * n)


# --------------------------------------------------------------------------
# fixtures
# --------------------------------------------------------------------------

def fixture_plate(shape, thickness: int = 6) -> np.ndarray:
    """A plate on the low end of the last axis (z < t in 3D, y < t in 2D)."""
    f = np.zeros(shape, dtype=np.uint8)
    f[:thickness] = 1
    return f


def fixture_plate_clamps(n: int = 384) -> np.ndarray:
    """Plate z < 6 plus clamp blocks x in [0,16) and [n-16,n), z in [6,48)."""
    f = fixture_plate((n, n, n), 6)
    s = n / 384.0
    w, zt = int(round(16 * s)), int(round(48 * s))
    f[6:zt, :, :w] = 1
    f[6:zt, :, n - w:] = 1
    return f


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    ndim: int
    design: np.ndarray
    fixture: np.ndarray | None
    tool: dict
    dir_kind: int          # 0 = float64 unit vectors, 1 = int32 lattice vectors
    dirs: np.ndarray
    density: bool
    lam: float
    tau: float = 0.5
    extra: dict = field(default_factory=dict)


def c1(n: int = 128) -> Workload:
    """2D n^2 binary design, 8 lattice directions, direct correlation."""
    d = design_2d_discs_rects(n)
    return Workload("c1_2d_%d_x8" % n, 2, d, fixture_plate(d.shape, 4),
                    TOOL_C1, 1, circle8(), False, 0.0)


def c2(n: int = 128, tool_=None) -> Workload:
    """3D n^3 binary design, 26 lattice directions."""
    d = design_3d_boxes_cyls(n)
    return Workload("c2_3d_%d_x26" % n, 3, d, fixture_plate(d.shape, 6),
                    tool_ or TOOL_C2, 1, lattice26(), False, 0.0)


def c3(n: int = 256, n_dirs: int = 130, tool_=None) -> Workload:
    """3D n^3 density design, Fibonacci-hemisphere directions, lambda 0.01."""
    d = design_density(n)
    return Workload("c3_3d_density_%d_x%d" % (n, n_dirs), 3, d,
                    fixture_plate(d.shape, 6), tool_ or TOOL_C3, 0,
                    fib_hemisphere(n_dirs), True, 0.01)


def c5(n: int = 384, n_dirs: int = 512) -> Workload:
    d = design_density(n, seed=7627005)
    return Workload("c5_3d_density_%d_x%d" % (n, n_dirs), 3, d,
                    fixture_plate_clamps(n), TOOL_C5, 0, fib_hemisphere(n_dirs),
                    True, 0.01)


def serving_stream(n_req: int = 64, seed: int = 7627004, rate: float = 1.0,
                   sizes=(64, 96, 128, 192, 256), master_dirs: int = 130):
    """Request descriptors for the serving mix: Poisson arrival times (seconds at
    ``rate`` requests/s), grid size, binary/density, tool and direction subset."""
    r = _rng(seed)
    t = np.cumsum(r.exponential(1.0 / rate, size=n_req))
    out = []
    for i in range(n_req):
        n = int(r.choice(sizes))
        density = bool(r.integers(0, 2))
        ball = bool(r.integers(0, 2))
        k = int(r.integers(6, master_dirs + 1))
        sub = np.sort(r.choice(master_dirs, size=k, replace=False))
        out.append({"t": float(t[i]), "n": n, "density": density,
                    "tool": TOOL_C3 if ball else TOOL_C2, "dir_index": sub,
                    "seed": seed * 100 + i})
    return out


def serving_request(desc: dict, master_dirs: int = 130) -> dict:
    """Materialize one serving-mix descriptor: design (binary boxes/cylinders
    scaled to the grid, or density), fixture plate, tool, its subset of the
    master Fibonacci set, lambda (0 for binary, 0.01 for density)."""
    n = desc["n"]
    if desc["density"]:
        d = design_density(n, seed=desc["seed"])
    else:
        d = design_3d_boxes_cyls(n, seed=desc["seed"])
    return {"design": d, "fixture": fixture_plate(d.shape, 6), "tool": desc["tool"],
            "dirs": fib_hemisphere(master_dirs)[desc["dir_index"]],
            "lam": 0.01 if desc["density"] else 0.0}


# ---------------------------------------------------------------------------
# voxel-model tools and rotations
# ---------------------------------------------------------------------------
TOOL_VOXEL = 3


def voxel_tool(labels, origin) -> dict:
    """A voxel-model tool: labels [z][y][x] (0 empty, 1 holder, 2 cutter) in the
    tool frame; origin = (x, y, z) index of the tip voxel."""
    lab = np.ascontiguousarray(labels, dtype=np.uint8)
    assert lab.ndim == 3 and set(np.unique(lab)) <= {0, 1, 2}
    return {"kind": TOOL_VOXEL, "labels": lab, "origin": tuple(int(v) for v in origin)}


def asymmetric_tool(r: int = 2, length: int = 14, holder_half: int = 5,
                    holder_len: int = 10) -> dict:
    """A non-axisymmetric voxel tool: cylindrical cutter of radius r along +z
    over [0, length) with a side tooth (x in [r, r + 2], |y| <= 1, z < 3), and a
    square holder (|x|, |y| <= holder_half) over [length, length + holder_len)."""
    h = holder_half
    x = np.arange(-h, h + 1)
    zs = np.arange(0, length + holder_len)
    Z, Y, X = np.meshgrid(zs, x, x, indexing="ij")
    lab = np.zeros(Z.shape, np.uint8)
    cutter = ((X ** 2 + Y ** 2 <= r * r) & (Z < length)) | \
             ((X >= r) & (X <= r + 2) & (np.abs(Y) <= 1) & (Z < 3))
    holder = (Z >= length)
    lab[holder] = 1
    lab[cutter] = 2
    return voxel_tool(lab, (h, h, 0))


def quat_to_matrix(q) -> np.ndarray:
    """Rotation matrix (row-major, tool frame to grid) of a quaternion (w, x, y, z)."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def random_rotations(n: int, seed: int) -> np.ndarray:
    """n uniformly distributed rotations (Shoemake's method), [n, 3, 3]."""
    r = _rng(seed)
    u1, u2, u3 = r.random(n), r.random(n), r.random(n)
    q = np.stack([np.sqrt(1 - u1) * np.sin(2 * np.pi * u2), np.sqrt(1 - u1) * np.cos(2 * np.pi * u2),
                  np.sqrt(u1) * np.sin(2 * np.pi * u3), np.sqrt(u1) * np.cos(2 * np.pi * u3)], 1)
    return np.stack([quat_to_matrix(v) for v in q])


def cube_rotations() -> np.ndarray:
    """The 24 proper rotations of the cube (signed permutation matrices, det +1)."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            m = np.zeros((3, 3))
            for i, j in enumerate(perm):
                m[i, j] = signs[i]
            if np.linalg.det(m) > 0:
                out.append(m)
    return np.array(out)


def rotation_to(d, roll: float = 0.0) -> np.ndarray:
    """A rotation taking the tool's +z axis to the unit vector d, then rolled
    by `roll` radians about d."""
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d)
    a = np.array([1.0, 0, 0]) if abs(d[0]) < 0.9 else np.array([0, 1.0, 0])
    e1 = np.cross(a, d)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    c, s = np.cos(roll), np.sin(roll)
    u, v = c * e1 + s * e2, -s * e1 + c * e2
    return np.stack([u, v, d], axis=1)   # columns: images of x, y, z


def setup_clamps(shape, n_sets: int, seed: int = 7627007, depth: int = 3,
                 height: int = 10) -> np.ndarray:
    """One extra fixture per machining setup: a pair of vise jaws gripping the
    part from opposite sides along x or y (alternating), at a seeded position
    along the other axis, above the plate.  Returns uint8 [n_sets, *shape]."""
    rng = _rng(seed)
    nz, ny, nx = shape
    out = np.zeros((n_sets,) + tuple(shape), np.uint8)
    for s in range(n_sets):
        z0 = int(rng.integers(0, max(nz // 4, 1)))
        z1 = min(nz, z0 + height)
        if s % 2 == 0:
            a = int(rng.integers(0, max(ny - ny // 3, 1)))
            b = min(ny, a + max(ny // 3, 1))
            out[s, z0:z1, a:b, :depth] = 1
            out[s, z0:z1, a:b, nx - depth:] = 1
        else:
            a = int(rng.integers(0, max(nx - nx // 3, 1)))
            b = min(nx, a + max(nx // 3, 1))
            out[s, z0:z1, :depth, a:b] = 1
            out[s, z0:z1, ny - depth:, a:b] = 1
    return out


def setup_of_dirs(dirs, n_sets: int) -> np.ndarray:
    """The setup of each orientation: sectors of the azimuth of its direction
    (x, y components), n_sets sectors of equal angle."""
    d = np.asarray(dirs, np.float64).reshape(len(dirs), -1)
    phi = np.arctan2(d[:, 1], d[:, 0]) % (2 * np.pi)
    return np.minimum((phi / (2 * np.pi) * n_sets).astype(np.int32), n_sets - 1)


def perturb_density_device(rho, seed: int, amp: float = 0.05, sigma: float = 4.0):
    """``perturb_density`` on the device (torch): rho + amp * standardized smooth
    noise (the same periodic Gaussian filter, truncated at 4 sigma, applied by
    FFT), clipped to [0, 1] and rounded to the 2**-24 grid.  The white noise is
    torch's seeded normal generator on the device, so the values differ from the
    numpy recipe; the TO-loop benchmark uses it to keep host time out of the
    loop."""
    import torch
    dev = rho.device
    g = torch.Generator(device=dev).manual_seed(int(seed))
    w = torch.randn(rho.shape, generator=g, device=dev, dtype=torch.float64)
    half = int(math.ceil(4 * sigma))
    taps = np.exp(-0.5 * (np.arange(-half, half + 1) / sigma) ** 2)
    taps /= taps.sum()
    spec = torch.fft.rfftn(w)
    for ax in range(rho.dim()):
        n = rho.shape[ax]
        ker = np.zeros(n)
        for j, t in zip(range(-half, half + 1), taps):
            ker[j % n] += t
        kf = np.fft.rfft(ker) if ax == rho.dim() - 1 else np.fft.fft(ker)
        shape = [1] * rho.dim()
        shape[ax] = kf.shape[0]
        spec = spec * torch.from_numpy(kf.reshape(shape)).to(dev)
    noise = torch.fft.irfftn(spec, s=rho.shape)
    noise = (noise - noise.mean()) / noise.std(unbiased=False)
    out = (rho.double() + amp * noise).clamp_(0.0, 1.0)
    return (torch.round(out * Q24) / Q24).float()
