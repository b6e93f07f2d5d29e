"""ctypes binding of libimf.so: argument marshalling only.

Every step of the computation runs in the HIP kernels of the library.  When the
library has not been built, or cannot be loaded, importing works but any call
raises: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libimf.so")

TOOL_FLAT, TOOL_BALL, TOOL_RECT2D, TOOL_VOXEL = 0, 1, 2, 3
DIR_F64, DIR_LATTICE, DIR_ROTATION = 0, 1, 2
SHARP_ALL, SHARP_BOUNDARY, SHARP_TIP = 0, 1, 2
METHOD_AUTO, METHOD_FFT, METHOD_DIRECT = 0, 1, 2
FLAG_PLAIN, FLAG_MASK_SWEEP, FLAG_NO_CACHE, FLAG_PROFILE, FLAG_NO_BOUND = 1, 2, 4, 8, 16
FLAG_NO_GRAPH = 32
KERNEL_CLASSES = ("raster", "setup", "fwd_design", "tool_x", "tool_y", "tool_z",
                  "inv_z_product", "inv_y", "inv_x_c2r", "recheck", "levels", "minfilter",
                  "sweep", "finalize", "copies", "bound")

_STATUS = {0: "IMF_OK", 1: "IMF_EINVAL", 2: "IMF_ENOMEM", 3: "IMF_EDEVICE", 4: "IMF_EBUSY",
           5: "IMF_ETIMEOUT", 6: "IMF_ECANCELLED", 7: "IMF_EACCURACY", 8: "IMF_ENOTIMPL"}


class IMFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class _Tool(C.Structure):
    _fields_ = [("kind", C.c_int), ("cutter_r", C.c_double), ("cutter_len", C.c_double),
                ("holder_r", C.c_double), ("holder_len", C.c_double)]


class _Request(C.Structure):
    _fields_ = [("ndim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("design_is_density", C.c_int), ("design", C.c_void_p), ("fixture", C.c_void_p),
                ("domain", C.c_void_p), ("n_tools", C.c_int), ("tool_ids", C.c_void_p),
                ("n_dirs", C.c_void_p), ("dir_kind", C.c_int), ("dirs", C.c_void_p),
                ("sharp", C.c_int), ("lam", C.c_double), ("tau", C.c_double),
                ("mask_theta_abs", C.c_double), ("method", C.c_int), ("batch", C.c_int),
                ("flags", C.c_uint), ("n_fixture_sets", C.c_int),
                ("fixture_sets", C.c_void_p), ("fixture_of", C.c_void_p)]


class _Outputs(C.Structure):
    _fields_ = [("imf", C.c_void_p), ("imf_norm", C.c_void_p), ("secluded", C.c_void_p),
                ("acc_masks", C.c_void_p), ("debug_overlap", C.c_void_p),
                ("debug_orient", C.c_int), ("debug_box", C.c_int * 6)]


class _Stats(C.Structure):
    _fields_ = [("F_max", C.c_double), ("guard_flags", C.c_longlong),
                ("max_frac_err", C.c_float), ("guard_band", C.c_double),
                ("t_ms", C.c_double * 8), ("model_bytes", C.c_double), ("P", C.c_int * 3),
                ("n_orient", C.c_int), ("method", C.c_int), ("batch", C.c_int),
                ("cache_hits", C.c_int), ("cache_misses", C.c_int),
                ("k_ms", C.c_double * 16), ("k_n", C.c_int * 16),
                ("k_bytes", C.c_double * 16), ("k_ops", C.c_double * 16),
                ("bound_blocks", C.c_longlong), ("bound_skipped", C.c_longlong),
                ("graph", C.c_int), ("lattice_runs", C.c_int), ("mf_shape", C.c_int),
                ("mf_wg_per_cu", C.c_int), ("max_abs_err", C.c_float),
                ("post_exact", C.c_longlong), ("band_entries", C.c_longlong),
                ("passes", C.c_int), ("box_voxels", C.c_double), ("hinted", C.c_int),
                ("fft_plan", C.c_int), ("queue_ms", C.c_double),
                ("lock_ms", C.c_double), ("hold_ms", C.c_double)]


@dataclass
class Stats:
    F_max: float
    guard_flags: int
    max_frac_err: float
    guard_band: float
    t_ms: list
    model_bytes: float
    P: tuple
    n_orient: int
    method: int
    batch: int
    cache_hits: int
    cache_misses: int
    kernel_ms: dict
    kernel_launches: dict
    kernel_bytes: dict
    kernel_ops: dict
    bound_blocks: int
    bound_skipped: int
    graph: int  # 0 kernel by kernel, 1 captured into a HIP graph, 2 graph replay
    lattice_runs: int  # orientations with sharp-point runs along a lattice vector
    mf_shape: int      # block shape of the sharp-point minimum (imf.h)
    mf_wg_per_cu: int  # resident workgroups per CU of its list pass
    max_abs_err: float  # density: largest |g32 - g| an exact recomputation found
    post_exact: int     # exact overlaps computed after the first pass
    band_entries: int   # overlaps within guard_band of lambda F_max
    passes: int         # 2 when lambda F_max was decided by a second pass
    box_voxels: float   # sum over orientations of the query-box volume
    hinted: int         # 1 expected threshold's bracket held, 2 missed, 0 none
    fft_plan: int       # inverse transform plans, 2 bits per pass (z | y << 2 | x << 4)
    queue_ms: float     # served requests: submission to admission
    lock_ms: float      # host time waiting for the context lock
    hold_ms: float      # host time holding it (planning and enqueueing)

    @classmethod
    def _from(cls, s: _Stats):
        kms = {k: s.k_ms[i] for i, k in enumerate(KERNEL_CLASSES) if s.k_n[i]}
        kn = {k: s.k_n[i] for i, k in enumerate(KERNEL_CLASSES) if s.k_n[i]}
        kb = {k: s.k_bytes[i] for i, k in enumerate(KERNEL_CLASSES) if s.k_n[i]}
        ko = {k: s.k_ops[i] for i, k in enumerate(KERNEL_CLASSES) if s.k_n[i]}
        return cls(s.F_max, s.guard_flags, s.max_frac_err, s.guard_band, list(s.t_ms),
                   s.model_bytes, tuple(s.P), s.n_orient, s.method, s.batch, s.cache_hits,
                   s.cache_misses, kms, kn, kb, ko, s.bound_blocks, s.bound_skipped, s.graph,
                   s.lattice_runs, s.mf_shape, s.mf_wg_per_cu, s.max_abs_err, s.post_exact,
                   s.band_entries, s.passes, s.box_voxels, s.hinted, s.fft_plan, s.queue_ms,
                   s.lock_ms, s.hold_ms)


_lib = None


def library_path() -> str:
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libimf.so is not built (run __graft_entry__.build() or "
                              "python paper_2002_07627_amd/build.py)")
        L = C.CDLL(_LIB_PATH)
        L.imf_last_error.restype = C.c_char_p
        L.imf_fft_size.restype = C.c_int
        for name in ("imf_create", "imf_destroy", "imf_tool_register", "imf_query_footprint",
                     "imf_compute", "imf_submit", "imf_wait", "imf_cancel", "imf_autotune",
                     "imf_autotune_save", "imf_autotune_load",
                     "imf_raster", "imf_fft_c2c", "imf_fft_r2c_3d"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise IMFError(st, _L().imf_last_error().decode())


def fft_size(n: int) -> int:
    return int(_L().imf_fft_size(int(n)))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """A library context on one GPU: workspace, tool-raster and spectrum caches."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        self._ctx = C.c_void_p()
        self.device = device
        _check(_L().imf_create(int(device), C.c_size_t(budget_bytes), C.byref(self._ctx)))
        self._tools = {}
        self._pending = {}

    def close(self):
        if self._ctx:
            _L().imf_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tool(self, t: dict) -> int:
        if t["kind"] == TOOL_VOXEL:
            lab = np.ascontiguousarray(t["labels"], dtype=np.uint8)
            key = ("voxel", lab.shape, lab.tobytes(), tuple(t["origin"]))
            if key not in self._tools:
                tid = C.c_int()
                nz, ny, nx = lab.shape
                org = (C.c_int * 3)(*[int(v) for v in t["origin"]])
                _check(_L().imf_tool_register_voxel(self._ctx, nx, ny, nz,
                                                    lab.ctypes.data_as(C.c_void_p), org,
                                                    C.byref(tid)))
                self._tools[key] = tid.value
            return self._tools[key]
        key = (t["kind"], t["cutter_r"], t["cutter_len"], t["holder_r"], t["holder_len"])
        if key not in self._tools:
            tid = C.c_int()
            ct = _Tool(*key)
            _check(_L().imf_tool_register(self._ctx, C.byref(ct), C.byref(tid)))
            self._tools[key] = tid.value
        return self._tools[key]

    # ------------------------------------------------------------------ request
    def _request(self, design, fixture, domain, tools, dirs, dir_kind, sharp, lam, tau,
                 mask_theta_abs, method, batch, flags, fixture_sets=None, fixture_of=None):
        import torch
        if not design.is_cuda:
            raise ValueError("design must be a device tensor")
        ndim = design.dim()
        if ndim == 2:
            nz, (ny, nx) = 1, design.shape
        else:
            nz, ny, nx = design.shape
        density = design.dtype == torch.float32
        if not density and design.dtype != torch.uint8:
            raise ValueError("design must be uint8 {0,1} or float32 density")
        for t in (fixture, domain):
            if t is not None and (t.dtype != torch.uint8 or t.numel() != design.numel()
                                  or not t.is_cuda or not t.is_contiguous()):
                raise ValueError("fixture/domain must be contiguous uint8 device tensors "
                                 "of the design's shape")
        if not design.is_contiguous():
            raise ValueError("design must be contiguous")
        if isinstance(tools, dict):
            tools, dirs = [tools], [dirs]
        ids = np.array([self.tool(t) for t in tools], dtype=np.int32)
        dirs = [np.asarray(d) for d in dirs]
        nd = np.array([len(d) for d in dirs], dtype=np.int32)
        dt = np.int32 if dir_kind == DIR_LATTICE else np.float64
        if dir_kind == DIR_ROTATION:
            dirs = [d.reshape(-1, 9) for d in dirs]
            nd = np.array([len(d) for d in dirs], dtype=np.int32)
        dd = np.ascontiguousarray(np.concatenate(dirs, axis=0), dtype=dt)
        if dd.shape[1] != (9 if dir_kind == DIR_ROTATION else ndim):
            raise ValueError("directions must have %d components" % ndim)
        r = _Request()
        r.ndim, r.nx, r.ny, r.nz = ndim, nx, ny, nz
        r.design_is_density = int(density)
        r.design, r.fixture, r.domain = _ptr(design), _ptr(fixture), _ptr(domain)
        r.n_tools = len(ids)
        r.tool_ids = ids.ctypes.data_as(C.c_void_p)
        r.n_dirs = nd.ctypes.data_as(C.c_void_p)
        r.dir_kind = dir_kind
        r.dirs = dd.ctypes.data_as(C.c_void_p)
        r.sharp, r.lam, r.tau, r.mask_theta_abs = sharp, lam, tau, mask_theta_abs
        r.method, r.batch, r.flags = method, batch, flags
        fof = None
        if fixture_sets is not None:
            # one fixture per setup: [n_sets, *design.shape] uint8 on the device,
            # fixture_of[q] names the set of orientation q
            if fixture_sets.dtype != torch.uint8 or not fixture_sets.is_cuda or \
                    not fixture_sets.is_contiguous() or \
                    fixture_sets.numel() % max(design.numel(), 1) or fixture_sets.numel() == 0:
                raise ValueError("fixture_sets must be a contiguous uint8 device tensor of "
                                 "shape [n_sets, *design.shape]")
            fof = np.ascontiguousarray(fixture_of, dtype=np.int32).reshape(-1)
            if len(fof) != int(nd.sum()):
                raise ValueError("fixture_of needs one set index per orientation")
            r.n_fixture_sets = fixture_sets.numel() // design.numel()
            r.fixture_sets = _ptr(fixture_sets)
            r.fixture_of = fof.ctypes.data_as(C.c_void_p)
        keep = (ids, nd, dd, design, fixture, domain, fixture_sets, fof)
        return r, keep, (nz, ny, nx), int(nd.sum())

    def _outputs(self, shape, n_orient, masks, debug_orient, device, debug_numel=0, out=None):
        import torch
        nz, ny, nx = shape
        want = {"imf": (shape, torch.float32), "imf_norm": (shape, torch.float32),
                "secluded": (shape, torch.uint8)}
        if masks:
            want["masks"] = ((n_orient, nz, ny, (nx + 63) // 64), torch.int64)
        o = {}
        for k, (shp, dt) in want.items():
            t = None if out is None else out.get(k)
            if t is None:
                t = torch.empty(shp, dtype=dt, device=device)
            elif (tuple(t.shape) != tuple(shp) and t.numel() != int(np.prod(shp))) or \
                    t.dtype != dt or not t.is_contiguous() or t.device != device:
                raise ValueError("output %r must be a contiguous %s tensor of shape %s on %s"
                                 % (k, dt, shp, device))
            o[k] = t
        co = _Outputs()
        co.imf, co.imf_norm, co.secluded = _ptr(o["imf"]), _ptr(o["imf_norm"]), \
            _ptr(o["secluded"])
        co.acc_masks = _ptr(o.get("masks"))
        co.debug_orient = debug_orient
        if debug_orient >= 0:
            o["debug"] = torch.empty(debug_numel, dtype=torch.float32, device=device)
            co.debug_overlap = _ptr(o["debug"])
        return o, co

    def footprint(self, design, fixture=None, domain=None, *, tools, dirs, dir_kind=DIR_F64,
                  sharp=SHARP_ALL, lam=0.0, tau=0.5, mask_theta_abs=-1.0, method=METHOD_AUTO,
                  batch=0, flags=0, fixture_sets=None, fixture_of=None) -> int:
        r, keep, _, _ = self._request(design, fixture, domain, tools, dirs, dir_kind, sharp, lam,
                                      tau, mask_theta_abs, method, batch, flags, fixture_sets,
                                      fixture_of)
        b = C.c_size_t()
        _check(_L().imf_query_footprint(self._ctx, C.byref(r), C.byref(b)))
        return b.value

    def compute(self, design, fixture=None, domain=None, *, tools, dirs, dir_kind=DIR_F64,
                sharp=SHARP_ALL, lam=0.0, tau=0.5, mask_theta_abs=-1.0, method=METHOD_AUTO,
                batch=0, flags=0, masks=True, debug_orient=-1, debug_numel=0, stream=None,
                out=None, fixture_sets=None, fixture_of=None):
        """Run one request; returns a dict of device tensors and a Stats.  `out`
        may hold preallocated outputs ("imf", "imf_norm", "secluded", "masks"),
        which a loop reuses so that its repeated requests replay one HIP graph.
        `fixture_sets` ([n_sets, *shape] uint8, device) with `fixture_of` (one set
        index per orientation) give each setup its own extra fixture."""
        r, keep, shape, n_orient = self._request(design, fixture, domain, tools, dirs,
                                                 dir_kind, sharp, lam, tau, mask_theta_abs,
                                                 method, batch, flags, fixture_sets, fixture_of)
        o, co = self._outputs(shape, n_orient, masks, debug_orient, design.device, debug_numel,
                              out)
        st = _Stats()
        _check(_L().imf_compute(self._ctx, C.byref(r), C.byref(co), C.byref(st),
                                _stream_handle(stream)))
        if debug_orient >= 0:
            o["debug_box"] = tuple(co.debug_box)
        if design.dim() == 2:
            for k in ("imf", "imf_norm", "secluded"):
                o[k] = o[k].reshape(shape[1:])
        return o, Stats._from(st)

    def submit(self, design, fixture=None, domain=None, *, tools, dirs, dir_kind=DIR_F64,
               sharp=SHARP_ALL, lam=0.0, tau=0.5, mask_theta_abs=-1.0, method=METHOD_AUTO,
               batch=0, flags=0, masks=True, fixture_sets=None, fixture_of=None):
        """Enqueue a request in the serving loop; returns a ticket."""
        r, keep, shape, n_orient = self._request(design, fixture, domain, tools, dirs,
                                                 dir_kind, sharp, lam, tau, mask_theta_abs,
                                                 method, batch, flags, fixture_sets, fixture_of)
        o, co = self._outputs(shape, n_orient, masks, -1, design.device)
        t = C.c_uint64()
        _check(_L().imf_submit(self._ctx, C.byref(r), C.byref(co), C.byref(t)))
        self._pending[t.value] = (o, keep, co, design.dim(), shape)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        st = _Stats()
        try:
            _check(_L().imf_wait(self._ctx, C.c_uint64(ticket), int(timeout_ms), C.byref(st)))
        except IMFError as e:
            if e.status != 5:
                self._pending.pop(ticket, None)
            raise
        o, keep, co, ndim, shape = self._pending.pop(ticket)
        if ndim == 2:
            for k in ("imf", "imf_norm", "secluded"):
                o[k] = o[k].reshape(shape[1:])
        return o, Stats._from(st)

    def cancel(self, ticket: int):
        _check(_L().imf_cancel(self._ctx, C.c_uint64(ticket)))

    def autotune(self, design, fixture=None, domain=None, *, tools, dirs, **kw) -> int:
        masks = kw.pop("masks", True)
        r, keep, shape, n_orient = self._request(
            design, fixture, domain, tools, dirs, kw.get("dir_kind", DIR_F64),
            kw.get("sharp", SHARP_ALL), kw.get("lam", 0.0), kw.get("tau", 0.5),
            kw.get("mask_theta_abs", -1.0), kw.get("method", METHOD_AUTO), 0,
            kw.get("flags", 0), kw.get("fixture_sets"), kw.get("fixture_of"))
        o, co = self._outputs(shape, n_orient, masks, -1, design.device)
        b = C.c_int()
        _check(_L().imf_autotune(self._ctx, C.byref(r), C.byref(co), C.byref(b)))
        return b.value

    def autotune_save(self, path: str):
        """Write the context's autotuned table to a text file."""
        _check(_L().imf_autotune_save(self._ctx, os.fsencode(path)))

    def autotune_load(self, path: str) -> int:
        """Merge a saved autotune table; returns the number of entries."""
        n = C.c_int()
        _check(_L().imf_autotune_load(self._ctx, os.fsencode(path), C.byref(n)))
        return n.value

    # -------------------------------------------------- coupling to the TO loop
    def heaviside(self, xi, beta: float, out=None, stream=None):
        """Heaviside projection of design variables (float32 device tensor),
        rounded to the 2^-24 grid: usable as the density design of a request."""
        import torch
        if xi.dtype != torch.float32 or not xi.is_cuda or not xi.is_contiguous():
            raise ValueError("xi must be a contiguous float32 device tensor")
        rho = torch.empty_like(xi) if out is None else out
        _check(_L().imf_heaviside(self._ctx, C.c_longlong(xi.numel()), _ptr(xi),
                                  C.c_double(beta), _ptr(rho), _stream_handle(stream)))
        return rho

    def access_filter(self, design, imf_norm, secluded, fixture=None, domain=None, *, tau=0.5,
                      sens=None, w=0.0, stream=None):
        """Accessibility filter (and, with `sens`, the filtered sensitivity) from a
        request's outputs; returns (filter, filtered sensitivity or None)."""
        import torch
        shape = design.shape if design.dim() == 3 else (1,) + tuple(design.shape)
        nz, ny, nx = shape
        for t in (design, imf_norm, secluded, fixture, domain, sens):
            if t is not None and (not t.is_cuda or not t.is_contiguous()
                                  or t.numel() != design.numel()):
                raise ValueError("all fields must be contiguous device tensors of the design's size")
        filt = torch.empty(design.shape, dtype=torch.float32, device=design.device)
        so = torch.empty_like(filt) if sens is not None else None
        _check(_L().imf_access_filter(
            self._ctx, nx, ny, nz, _ptr(design), int(design.dtype == torch.float32),
            _ptr(fixture), _ptr(domain), _ptr(imf_norm), _ptr(secluded), C.c_double(tau),
            _ptr(sens), C.c_double(w), _ptr(filt), _ptr(so), _stream_handle(stream)))
        return filt, so

    def plan_greedy(self, masks, design, fixture=None, domain=None, *, tau=0.5, max_steps=None,
                    stream=None, noalloc=False):
        """Greedy machining plan from a request's accessible masks: returns
        ([(orientation, voxels removed), ...], voxels left)."""
        shape = design.shape if design.dim() == 3 else (1,) + tuple(design.shape)
        nz, ny, nx = shape
        nq = masks.shape[0]
        if masks.numel() != nq * nz * ny * ((nx + 63) // 64) or not masks.is_contiguous():
            raise ValueError("masks must be the [n_orient][nz][ny][ceil(nx/64)] words of a request")
        ms = nq if max_steps is None else int(max_steps)
        orient = np.zeros(max(ms, 1), np.int32)
        removed = np.zeros(max(ms, 1), np.int64)
        n = C.c_int()
        left = C.c_longlong()
        import torch
        fn = _L().imf_plan_greedy_noalloc if noalloc else _L().imf_plan_greedy
        _check(fn(
            self._ctx, nx, ny, nz, nq, _ptr(masks), _ptr(design),
            int(design.dtype == torch.float32), _ptr(fixture), _ptr(domain), C.c_double(tau), ms,
            orient.ctypes.data_as(C.c_void_p), removed.ctypes.data_as(C.c_void_p), C.byref(n),
            C.byref(left), _stream_handle(stream)))
        return [(int(orient[i]), int(removed[i])) for i in range(n.value)], left.value

    # -------------------------------------------------------------- single steps
    def raster(self, tool: dict, d, dir_kind=None, sharp=SHARP_ALL):
        """(offsets int32 [n, 3] as x, y, z; flags uint8 [n]) of one oriented tool."""
        d = np.asarray(d)
        if dir_kind is None:
            dir_kind = DIR_ROTATION if d.size == 9 else (
                DIR_LATTICE if d.dtype.kind in "iu" else DIR_F64)
        if dir_kind == DIR_ROTATION:
            ndim = 3
            dd = np.ascontiguousarray(d.reshape(1, 9), dtype=np.float64)
        else:
            ndim = d.shape[-1]
            dd = np.ascontiguousarray(d.reshape(1, ndim),
                                      dtype=np.int32 if dir_kind == DIR_LATTICE else np.float64)
        tid = self.tool(tool)
        n = C.c_longlong()
        st = _L().imf_raster_tool(self._ctx, tid, ndim, dir_kind, dd.ctypes.data_as(C.c_void_p),
                                  sharp, None, None, C.c_longlong(0), C.byref(n))
        if st not in (0, 1) or n.value <= 0:
            _check(st)
        offs = np.zeros((n.value, 3), np.int32)
        fl = np.zeros(n.value, np.uint8)
        _check(_L().imf_raster_tool(self._ctx, tid, ndim, dir_kind,
                                    dd.ctypes.data_as(C.c_void_p), sharp,
                                    offs.ctypes.data_as(C.c_void_p),
                                    fl.ctypes.data_as(C.c_void_p), C.c_longlong(n.value),
                                    C.byref(n)))
        return offs, fl

    def fft_c2c(self, x, inverse=False, stream=None):
        """FFT of the columns of a complex64 device tensor [n, batch]."""
        import torch
        if x.dtype != torch.complex64 or x.dim() != 2 or not x.is_contiguous():
            raise ValueError("expected a contiguous complex64 [n, batch] tensor")
        y = torch.empty_like(x)
        _check(_L().imf_fft_c2c(self._ctx, x.shape[0], x.shape[1], _ptr(x), _ptr(y),
                                int(inverse), _stream_handle(stream)))
        return y

    def fft_r2c_3d(self, x, P, stream=None):
        """R2C transform of a float32 [nz, ny, nx] tensor zero-padded to P = (px, py, pz);
        returns complex64 [py, px//2+1, pz]."""
        import torch
        nz, ny, nx = x.shape
        px, py, pz = P
        y = torch.empty((py, px // 2 + 1, pz), dtype=torch.complex64, device=x.device)
        _check(_L().imf_fft_r2c_3d(self._ctx, nx, ny, nz, px, py, pz, _ptr(x), _ptr(y),
                                   _stream_handle(stream)))
        return y
