"""TEST INFRASTRUCTURE ONLY: ctypes front end of the plain CPU IMF oracle.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  The product library never imports it, and this package never
imports the product.  The C source is ``imf_oracle.c`` (exact int64 / 2^-24
fixed point); ``brute.py`` is an even plainer pure-Python version for tiny grids.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "imf_oracle.c")
_LIB = os.path.join(_HERE, "_imf_oracle.so")

Q24 = float(1 << 24)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Tool(C.Structure):
    _fields_ = [("kind", C.c_int), ("cutter_r", C.c_double), ("cutter_len", C.c_double),
                ("holder_r", C.c_double), ("holder_len", C.c_double),
                ("vox", C.c_void_p), ("vdim", C.c_int * 3), ("vorg", C.c_int * 3)]


VOXEL = 3   # tool kind: voxel model (labels 0 empty, 1 holder, 2 cutter)


def _tool_c(t):
    """ctypes tool; voxel tools keep a contiguous uint8 copy of their labels."""
    if t["kind"] == VOXEL:
        lab = np.ascontiguousarray(t["labels"], dtype=np.uint8)
        nz, ny, nx = lab.shape
        ct = _Tool(VOXEL, 0.0, 0.0, 0.0, 0.0, _ptr(lab), (C.c_int * 3)(nx, ny, nz),
                   (C.c_int * 3)(*[int(v) for v in t["origin"]]))
        return ct, lab
    return _Tool(t["kind"], t["cutter_r"], t["cutter_len"], t["holder_r"], t["holder_len"]), None


class _Req(C.Structure):
    _fields_ = [("ndim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("density", C.c_int), ("design", C.c_void_p), ("fixture", C.c_void_p),
                ("domain", C.c_void_p), ("n_tools", C.c_int), ("tools", C.POINTER(_Tool)),
                ("n_dirs", C.POINTER(C.c_int)), ("dir_kind", C.c_int), ("dirs", C.c_void_p),
                ("sharp", C.c_int), ("lam", C.c_double), ("tau", C.c_double),
                ("mask_theta_abs", C.c_double), ("fixture_sets", C.c_void_p),
                ("n_fixture_sets", C.c_int), ("fixture_of", C.c_void_p)]


class _Out(C.Structure):
    _fields_ = [("imf", C.c_void_p), ("imf_norm", C.c_void_p), ("secluded", C.c_void_p),
                ("masks", C.c_void_p), ("masks_dil", C.c_void_p), ("F_max", C.c_void_p),
                ("g_debug", C.c_void_p), ("debug_orient", C.c_int), ("debug_box", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.or_raster.restype = C.c_longlong
        L.or_raster.argtypes = [C.c_int, C.POINTER(_Tool), C.c_int, C.c_void_p, C.c_int,
                                C.c_void_p, C.c_void_p, C.c_longlong]
        for name in ("or_imf", "or_overlap_at", "or_gamma_at", "or_gamma_at_all",
                     "or_overlap_full", "or_orient_info"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Request:
    """Host-side request.  Arrays are numpy; the geometry conventions are those
    of :mod:`workloads`: ``[z][y][x]`` arrays, direction = tip toward holder."""

    def __init__(self, design, fixture=None, domain=None, tools=(), dirs=(), dir_kind=0,
                 density=None, sharp=0, lam=0.0, tau=0.5, mask_theta_abs=-1.0,
                 fixture_sets=None, fixture_of=None):
        design = np.ascontiguousarray(design)
        self.ndim = design.ndim
        if self.ndim == 2:
            design = design.reshape((1,) + design.shape)
        self.density = (design.dtype == np.float32) if density is None else bool(density)
        self.design = np.ascontiguousarray(design, dtype=np.float32 if self.density else np.uint8)
        self.nz, self.ny, self.nx = self.design.shape
        self.fixture = None if fixture is None else np.ascontiguousarray(
            np.asarray(fixture).reshape(self.design.shape), dtype=np.uint8)
        self.domain = None if domain is None else np.ascontiguousarray(
            np.asarray(domain).reshape(self.design.shape), dtype=np.uint8)
        if isinstance(tools, dict):
            tools = [tools]
            dirs = [dirs]
        self.tools = list(tools)
        dirs = [np.asarray(d) for d in dirs]
        self.n_dirs = np.array([len(d) for d in dirs], dtype=np.int32)
        self.dir_kind = int(dir_kind)
        dt = np.int32 if self.dir_kind == 1 else np.float64
        if self.dir_kind == 2:  # rotation matrices, 9 values each
            dirs = [d.reshape(-1, 9) for d in dirs]
        self.dirs = np.ascontiguousarray(np.concatenate(dirs, axis=0), dtype=dt)
        assert self.dirs.shape[1] == (9 if self.dir_kind == 2 else self.ndim)
        self.sharp, self.lam, self.tau = int(sharp), float(lam), float(tau)
        self.mask_theta_abs = float(mask_theta_abs)
        # fixtures per setup: orientation R sees fixture | fixture_sets[fixture_of[R]]
        self.fixture_sets = None if fixture_sets is None else np.ascontiguousarray(
            np.asarray(fixture_sets).reshape((-1,) + self.design.shape), dtype=np.uint8)
        self.fixture_of = None if fixture_of is None else np.ascontiguousarray(
            fixture_of, dtype=np.int32)
        self._c = self._make()

    @property
    def n_orient(self):
        return int(self.n_dirs.sum())

    @property
    def shape(self):
        return self.design.shape

    def _make(self):
        made = [_tool_c(t) for t in self.tools]
        tl = (_Tool * len(self.tools))(*[m[0] for m in made])
        self._keep = (tl, [m[1] for m in made])
        r = _Req()
        r.ndim, r.nx, r.ny, r.nz = self.ndim, self.nx, self.ny, self.nz
        r.density = int(self.density)
        r.design, r.fixture, r.domain = _ptr(self.design), _ptr(self.fixture), _ptr(self.domain)
        r.n_tools = len(self.tools)
        r.tools = tl
        r.n_dirs = self.n_dirs.ctypes.data_as(C.POINTER(C.c_int))
        r.dir_kind, r.dirs = self.dir_kind, _ptr(self.dirs)
        r.sharp, r.lam, r.tau, r.mask_theta_abs = self.sharp, self.lam, self.tau, \
            self.mask_theta_abs
        if self.fixture_sets is not None:
            r.fixture_sets = _ptr(self.fixture_sets)
            r.n_fixture_sets = len(self.fixture_sets)
            r.fixture_of = _ptr(self.fixture_of)
        return r

    @property
    def scale(self):
        return Q24 if self.density else 1.0


def raster(tool_, d, dir_kind=None, ndim=None):
    """Raster of one oriented tool: (offsets int32 [n, 3] as x,y,z, is_cutter bool [n])."""
    d = np.asarray(d)
    if dir_kind is None:
        dir_kind = 2 if d.size == 9 else (1 if d.dtype.kind in "iu" else 0)
    if dir_kind == 2:
        ndim = 3
        dd = np.ascontiguousarray(d.reshape(1, 9), dtype=np.float64)
    else:
        ndim = ndim or d.shape[-1]
        dd = np.ascontiguousarray(d.reshape(1, ndim),
                                  dtype=np.int32 if dir_kind == 1 else np.float64)
    t, keep = _tool_c(tool_)
    L = lib()
    n = L.or_raster(ndim, C.byref(t), dir_kind, _ptr(dd), 0, None, None, 0)
    if n == -1:
        raise ValueError("invalid tool or direction")
    n = -n - 2
    offs = np.zeros((max(n, 1), 3), dtype=np.int32)
    cut = np.zeros(max(n, 1), dtype=np.uint8)
    m = L.or_raster(ndim, C.byref(t), dir_kind, _ptr(dd), 0, _ptr(offs), _ptr(cut), n)
    assert m == n
    return offs[:n], cut[:n].astype(bool)


def imf(req: Request, masks=True, debug_orient=-1):
    """Run the whole IMF on the CPU.  Returns a dict of numpy arrays."""
    N = req.nx * req.ny * req.nz
    words = (req.nx + 63) // 64
    out = {"imf": np.zeros(N, np.float64), "imf_norm": np.zeros(N, np.float32),
           "secluded": np.zeros(N, np.uint8), "F_max": np.zeros(1, np.float64)}
    if masks:
        shp = (req.n_orient, req.nz, req.ny, words)
        out["masks"] = np.zeros(shp, np.uint64)
        out["masks_dil"] = np.zeros(shp, np.uint64)
    o = _Out()
    o.imf, o.imf_norm, o.secluded = _ptr(out["imf"]), _ptr(out["imf_norm"]), _ptr(out["secluded"])
    o.masks = _ptr(out.get("masks"))
    o.masks_dil = _ptr(out.get("masks_dil"))
    o.F_max = _ptr(out["F_max"])
    box = np.zeros(6, np.int32)
    if debug_orient >= 0:
        info = orient_info(req, debug_orient)
        kmin, kmax = info["kmin"], info["kmax"]
        dims = [n + kmax[a] - kmin[a] for a, n in enumerate((req.nx, req.ny, req.nz))]
        out["g_debug"] = np.zeros(int(np.prod(dims)), np.int64)
        o.g_debug = _ptr(out["g_debug"])
        o.debug_box = _ptr(box)
    o.debug_orient = debug_orient
    st = lib().or_imf(C.byref(req._c), C.byref(o))
    if st:
        raise RuntimeError("oracle or_imf failed with status %d" % st)
    shp = req.design.shape
    res = {"imf": out["imf"].reshape(shp), "imf_norm": out["imf_norm"].reshape(shp),
           "secluded": out["secluded"].reshape(shp), "F_max": float(out["F_max"][0])}
    if masks:
        res["masks"] = out["masks"]
        res["masks_dil"] = out["masks_dil"]
    if debug_orient >= 0:
        d = box[3:]
        res["g_debug"] = out["g_debug"].reshape(d[2], d[1], d[0])
        res["debug_lo"] = tuple(int(v) for v in box[:3])
    if req.ndim == 2:
        for k in ("imf", "imf_norm", "secluded"):
            res[k] = res[k].reshape(shp[1:])
    return res


def orient_info(req: Request, orient: int):
    km = np.zeros(6, np.int32)
    cnt = np.zeros(2, np.int64)
    st = lib().or_orient_info(C.byref(req._c), orient, _ptr(km), _ptr(cnt))
    if st:
        raise RuntimeError("oracle or_orient_info failed with status %d" % st)
    return {"kmin": tuple(int(v) for v in km[:3]), "kmax": tuple(int(v) for v in km[3:]),
            "nT": int(cnt[0]), "nS": int(cnt[1])}


def overlap_at(req: Request, orient: int, t) -> np.ndarray:
    """Exact g_R(t) (fixed-point integer units) at translations t [n, 3] (x,y,z)."""
    t = np.ascontiguousarray(np.asarray(t, dtype=np.int32).reshape(-1, 3))
    out = np.zeros(len(t), np.int64)
    st = lib().or_overlap_at(C.byref(req._c), orient, _ptr(t), C.c_longlong(len(t)), _ptr(out))
    if st:
        raise RuntimeError("oracle or_overlap_at failed with status %d" % st)
    return out


def gamma_at(req: Request, orient: int, x) -> np.ndarray:
    """Exact gamma_R(x) (fixed-point integer units) at voxels x [n, 3] (x,y,z)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1, 3))
    out = np.zeros(len(x), np.int64)
    st = lib().or_gamma_at(C.byref(req._c), orient, _ptr(x), C.c_longlong(len(x)), _ptr(out))
    if st:
        raise RuntimeError("oracle or_gamma_at failed with status %d" % st)
    return out


def gamma_at_all(req: Request, x) -> np.ndarray:
    """Exact gamma_R(x) for every orientation R: [n_orient, n] (fixed-point units)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((req.n_orient, len(x)), np.int64)
    st = lib().or_gamma_at_all(C.byref(req._c), _ptr(x), C.c_longlong(len(x)), _ptr(out))
    if st:
        raise RuntimeError("oracle or_gamma_at_all failed with status %d" % st)
    return out


def overlap_full(req: Request, orient: int):
    """g_R over every translation where it can be nonzero: (array [z][y][x], lo (x,y,z))."""
    box = np.zeros(6, np.int32)
    st = lib().or_overlap_full(C.byref(req._c), orient, None, _ptr(box))
    if st:
        raise RuntimeError("oracle or_overlap_full failed with status %d" % st)
    d = box[3:]
    out = np.zeros(int(np.prod(d)), np.int64)
    lib().or_overlap_full(C.byref(req._c), orient, _ptr(out), _ptr(box))
    return out.reshape(d[2], d[1], d[0]), tuple(int(v) for v in box[:3])


def unpack_masks(words: np.ndarray, nx: int) -> np.ndarray:
    """[..., words] uint64 -> [..., nx] bool (bit x % 64 of word x // 64)."""
    w = np.ascontiguousarray(words).view(np.uint8)
    bits = np.unpackbits(w.reshape(words.shape[:-1] + (-1,)), axis=-1, bitorder="little")
    return bits[..., :nx].astype(bool)
