"""TEST INFRASTRUCTURE ONLY: a brute-force IMF for tiny grids, in Python.

Independent of ``imf_oracle.c``: its own rasterizer (exact rational arithmetic,
lattice directions only) and the definitions applied literally:

* collision measure of placing the tool so that sharp point k touches x:
  the number (or density) of occupied voxels among {x - k + o : o in T_R}
  (Eq. access_meas / Eq. imf_1 of Sec. 2.1.3);
* IMF: the minimum over orientations and sharp points (Eq. imf_1);
* accessibility: x is accessible iff some collision-free placement puts a sharp
  point on x (Eq. access_def), enumerated as the union of K placed at every
  free translation (Eq. sweep).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _in_tool(kind, r, L, rh, Lh, o, v):
    """Exact membership of integer offset o for lattice direction v.

    Returns (in_tool, in_cutter).  Let a = o.v/|v| (axial coordinate) and
    q^2 = |o|^2 - a^2 (squared distance from the axis)."""
    r, L, rh, LH = Fraction(r), Fraction(L), Fraction(rh), Fraction(L) + Fraction(Lh)
    dot = sum(int(a) * int(b) for a, b in zip(o, v))
    n = sum(int(b) * int(b) for b in v)
    o2 = sum(int(a) * int(a) for a in o)
    a2 = Fraction(dot * dot, n)            # a^2 (a has the sign of dot)
    q2 = Fraction(o2) - a2

    def a_lt(c):   # a < c for c > 0
        return dot < 0 or a2 < c * c

    def a_ge(c):   # a >= c for c >= 0
        return dot >= 0 and a2 >= c * c

    cyl = a_lt(L) and q2 <= r * r
    if kind == 1:
        # ball of radius r centred at r*d:  |o|^2 - 2 r a <= 0
        ball = dot >= 0 and Fraction(o2) * Fraction(o2) <= 4 * r * r * a2
        cut = ball or (a_ge(r) and cyl)
    else:
        cut = a_ge(0) and cyl
    hold = a_ge(L) and a_lt(LH) and q2 <= rh * rh
    return (cut or hold), cut


def raster(tool, v):
    """Sets T (tool) and K (cutter) of integer offsets, as sorted lists of tuples."""
    v = [int(c) for c in v]
    ndim = len(v)
    r, L, rh, Lh = tool["cutter_r"], tool["cutter_len"], tool["holder_r"], tool["holder_len"]
    ext = int(np.ceil(max(L + Lh, 2 * r) + max(r, rh))) + 2
    rng = range(-ext, ext + 1)
    T, K = [], []
    if ndim == 2:
        pts = ((x, y, 0) for y in rng for x in rng)
    else:
        pts = ((x, y, z) for z in rng for y in rng for x in rng)
    for p in pts:
        t, k = _in_tool(tool["kind"], r, L, rh, Lh, p[:ndim], v)
        if t:
            T.append(p)
        if k:
            K.append(p)
    return T, K


def _shift_sum(field, offsets, lo, dims):
    """S(t) = sum_{o in offsets} field(t + o) for t in the box lo + [0, dims)."""
    nz, ny, nx = field.shape
    out = np.zeros((dims[2], dims[1], dims[0]), dtype=np.int64)
    tz = np.arange(dims[2]) + lo[2]
    ty = np.arange(dims[1]) + lo[1]
    tx = np.arange(dims[0]) + lo[0]
    for (ox, oy, oz) in offsets:
        zz, yy, xx = tz + oz, ty + oy, tx + ox
        mz = (zz >= 0) & (zz < nz)
        my = (yy >= 0) & (yy < ny)
        mx = (xx >= 0) & (xx < nx)
        sub = field[np.ix_(zz.clip(0, nz - 1), yy.clip(0, ny - 1), xx.clip(0, nx - 1))]
        out += sub * (mz[:, None, None] & my[None, :, None] & mx[None, None, :])
    return out


def imf(design, fixture, tool, dirs, lam=0.0, tau=0.5, scale=1, fixture_sets=None,
        fixture_of=None):
    """Brute-force f, F_max, fbar, Gamma and accessible masks (bool [nR, ...]).

    ``design`` holds integers in fixed point (``scale`` = 1 for binary).  With
    ``fixture_sets``, orientation i sees the fixture ``fixture | fixture_sets[
    fixture_of[i]]`` and the design domain excludes every fixture voxel."""
    design = np.asarray(design, dtype=np.int64)
    ndim = design.ndim
    d3 = design.reshape((1,) * (3 - ndim) + design.shape)
    fix = np.zeros_like(d3) if fixture is None else \
        np.asarray(fixture).reshape(d3.shape).astype(np.int64)
    rhoO = np.where(fix > 0, scale, d3)
    omega0 = fix == 0
    rhoO_of = [rhoO] * len(dirs)
    if fixture_sets is not None:
        sets = [np.asarray(f).reshape(d3.shape) != 0 for f in fixture_sets]
        rhoO_of = [np.where(sets[fixture_of[i]], scale, rhoO) for i in range(len(dirs))]
        for f in sets:
            omega0 = omega0 & ~f
    nz, ny, nx = d3.shape
    f = np.full(d3.shape, np.iinfo(np.int64).max, dtype=np.int64)
    gammas, frees = [], []
    for i, v in enumerate(dirs):
        T, K = raster(tool, v)
        # gamma_R(x) = min over k of the overlap of the tool placed with k on x
        gam = np.full(d3.shape, np.iinfo(np.int64).max, dtype=np.int64)
        for k in K:
            placed = [(o[0] - k[0], o[1] - k[1], o[2] - k[2]) for o in T]
            ov = _shift_sum(rhoO_of[i], placed, (0, 0, 0), (nx, ny, nz))
            gam = np.minimum(gam, ov)
        gammas.append(gam)
        f = np.minimum(f, gam)
        frees.append((T, K))
    fmax = int(f[omega0].max()) if omega0.any() else 0
    thB = lam * float(fmax)
    B = omega0 & (f.astype(np.float64) > thB)
    fbar = np.where(B, f / float(fmax) if fmax else 0.0, 0.0).astype(np.float32)
    solid = d3.astype(np.float64) > tau * scale
    gamma_set = B & ~solid
    # accessibility by sweeping free translations (threshold theta = lambda F_max)
    masks = []
    for i, (T, K) in enumerate(frees):
        Tarr = np.array(T)
        lo = tuple(int(-Tarr[:, a].max()) for a in range(3))
        dims = tuple(int((nx, ny, nz)[a] + Tarr[:, a].max() - Tarr[:, a].min())
                     for a in range(3))
        g = _shift_sum(rhoO_of[i], T, lo, dims)
        free = g.astype(np.float64) <= thB
        acc = np.zeros(d3.shape, dtype=bool)
        fz, fy, fx = np.nonzero(free)
        for k in K:
            x = fx + lo[0] + k[0]
            y = fy + lo[1] + k[1]
            z = fz + lo[2] + k[2]
            m = (x >= 0) & (x < nx) & (y >= 0) & (y < ny) & (z >= 0) & (z < nz)
            acc[z[m], y[m], x[m]] = True
        masks.append(acc & omega0)
    shp = design.shape
    return {"imf": f.reshape(shp), "F_max": fmax, "imf_norm": fbar.reshape(shp),
            "secluded": gamma_set.reshape(shp),
            "masks": np.stack([m.reshape(shp) for m in masks]),
            "gammas": np.stack([g.reshape(shp) for g in gammas])}


def raster_exact_box(tool, v, lo, hi):
    """Membership of every integer offset of the box [lo, hi] (inclusive, x, y, z)
    for a lattice direction v, in exact integer arithmetic (numpy int64), with
    the points where some boundary test of the predicate holds with equality.

    Same definition as ``_in_tool``: a = o.v/|v|, q^2 = |o|^2 - a^2, every
    comparison multiplied through by |v|^2 and by 4 so that half-integer sizes
    stay integral.  Returns (T, K, tie) boolean arrays indexed [z][y][x]."""
    v = [int(c) for c in v] + [0] * (3 - len(v))
    zs, ys, xs = (np.arange(lo[a], hi[a] + 1, dtype=np.int64) for a in (2, 1, 0))
    z, y, x = np.meshgrid(zs, ys, xs, indexing="ij")
    dot = x * v[0] + y * v[1] + z * v[2]
    n = v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
    o2 = x * x + y * y + z * z
    r2, L2 = int(round(2 * tool["cutter_r"])), int(round(2 * tool["cutter_len"]))
    rh2 = int(round(2 * tool["holder_r"]))
    LH2 = int(round(2 * (tool["cutter_len"] + tool["holder_len"])))
    assert abs(r2 - 2 * tool["cutter_r"]) < 1e-12 and abs(L2 - 2 * tool["cutter_len"]) < 1e-12
    perp = 4 * (o2 * n - dot * dot)          # 4 q^2 |v|^2
    ax = 4 * dot * dot                       # 4 a^2 |v|^2 (a >= 0 where dot >= 0)
    pos = dot >= 0

    def a_ge(c2):                            # a >= c for c = c2 / 2 >= 0
        return pos & (ax >= c2 * c2 * n)

    def a_lt(c2):                            # a < c for c = c2 / 2 > 0
        return ~pos | (ax < c2 * c2 * n)

    in_r = perp <= r2 * r2 * n
    if tool["kind"] == 1:
        ball = pos & (o2 * o2 * n <= r2 * r2 * dot * dot)
        cut = ball | (a_ge(r2) & a_lt(L2) & in_r)
    else:
        cut = pos & a_lt(L2) & in_r
    hold = a_ge(L2) & a_lt(LH2) & (perp <= rh2 * rh2 * n)
    tie = (perp == r2 * r2 * n) | (perp == rh2 * rh2 * n) | (dot == 0)
    for c2 in (L2, LH2) + ((r2,) if tool["kind"] == 1 else ()):
        tie |= pos & (ax == c2 * c2 * n)
    if tool["kind"] == 1:
        tie |= pos & (o2 * o2 * n == r2 * r2 * dot * dot)
    return cut | hold, cut, tie


def raster_margin_box(tool, d, lo, hi, eps=1e-9):
    """Membership of every integer offset of the box [lo, hi] (inclusive) for a
    float64 unit direction d, evaluated in extended precision (numpy
    longdouble) from the definitions a = o.d, q^2 = |o - a d|^2 and, for the
    ball end, |o - r d|^2 <= r^2; plus the points where some boundary test is
    within eps of equality (there the float64 raster may go either way).
    Returns (T, K, near) boolean arrays indexed [z][y][x]."""
    ld = np.longdouble
    d = [ld(float(c)) for c in d] + [ld(0)] * (3 - len(d))
    zs, ys, xs = (np.arange(lo[a], hi[a] + 1).astype(ld) for a in (2, 1, 0))
    z, y, x = np.meshgrid(zs, ys, xs, indexing="ij")
    a = x * d[0] + y * d[1] + z * d[2]
    q2 = (x - a * d[0]) ** 2 + (y - a * d[1]) ** 2 + (z - a * d[2]) ** 2
    r, L = ld(tool["cutter_r"]), ld(tool["cutter_len"])
    rh, LH = ld(tool["holder_r"]), ld(tool["cutter_len"]) + ld(tool["holder_len"])
    margins = [r * r - q2, rh * rh - q2, a, L - a, LH - a]
    in_cyl = (a < L) & (q2 <= r * r)
    if tool["kind"] == 1:
        b2 = (x - r * d[0]) ** 2 + (y - r * d[1]) ** 2 + (z - r * d[2]) ** 2
        margins += [r * r - b2, a - r]
        cut = (b2 <= r * r) | ((a >= r) & in_cyl)
    else:
        cut = (a >= 0) & in_cyl
    hold = (a >= L) & (a < LH) & (q2 <= rh * rh)
    near = np.zeros(a.shape, bool)
    for m in margins:
        near |= np.abs(m) <= eps
    return cut | hold, cut, near
