"""Ball Mapper construction on AMD Instinct MI355X (gfx950).

Thin ctypes binding of ``libbm.so`` (C ABI declared in ``include/bm.h``).  This
module only marshals arguments: every step of the construction — range
queries, the blocked greedy, membership CSR and edges — runs in the library's
HIP kernels.  There is no CPU fallback: if the library is missing or cannot be
loaded, every call raises.

Method: arXiv 2601.01405 (greedy eps-net of Sec. 2.2, nerve 1-skeleton of
Sec. 2.1, range queries of Sec. 3, error models of Sec. 5).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbm.so")

BM_OK, BM_EINVAL, BM_ENOMEM, BM_ENODEVICE, BM_EDEVICE, BM_ENONFINITE, BM_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "BM_OK", -1: "BM_EINVAL", -2: "BM_ENOMEM", -3: "BM_ENODEVICE", -4: "BM_EDEVICE",
                -5: "BM_ENONFINITE", -6: "BM_EINTERNAL"}
PATHS = {"auto": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "f16": 4}
PATH_NAMES = {v: k for k, v in PATHS.items()}
DTYPES = {np.dtype(np.float64): 0, np.dtype(np.float32): 1, np.dtype(np.float16): 2}


class BmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("refine", ctypes.c_int32), ("block", ctypes.c_int32),
                ("device", ctypes.c_int32), ("points_on_device", ctypes.c_int32),
                ("results_on_device", ctypes.c_int32), ("max_device_bytes", ctypes.c_int64),
                ("init_member_capacity", ctypes.c_int64), ("stream", ctypes.c_void_p),
                ("profile", ctypes.c_int32), ("no_graph", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_prepare", ctypes.c_double), ("ms_greedy", ctypes.c_double),
                ("ms_csr", ctypes.c_double), ("ms_edges", ctypes.c_double), ("ms_download", ctypes.c_double),
                ("pairs_useful", ctypes.c_int64), ("pairs_issued", ctypes.c_int64),
                ("band_pairs", ctypes.c_int64), ("blocks", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("path", ctypes.c_int32), ("block", ctypes.c_int32), ("ms_range_kernel", ctypes.c_double),
                ("range_launches", ctypes.c_int64), ("range_pairs", ctypes.c_int64),
                ("ms_range_events", ctypes.c_double), ("ms_resolve_kernel", ctypes.c_double),
                ("ms_serial_steps", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["path"] = PATH_NAMES.get(d["path"], d["path"])
        return d


class _Result(ctypes.Structure):
    _fields_ = [("n_landmarks", ctypes.c_int64), ("landmarks", ctypes.c_void_p),
                ("member_ptr", ctypes.c_void_p), ("member_idx", ctypes.c_void_p),
                ("n_edges", ctypes.c_int64), ("edges", ctypes.c_void_p),
                ("on_device", ctypes.c_int32), ("device", ctypes.c_int32), ("stats", Stats)]


class Problem(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("eps", ctypes.POINTER(ctypes.c_double)), ("n_eps", ctypes.c_int32),
                ("order", ctypes.POINTER(ctypes.c_int64))]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbm.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    # PyTorch ships its own HIP runtime with the same soname as the system one.
    # Loading torch first makes libbm.so bind to that runtime, so device memory
    # and streams are shared with torch and only one runtime touches the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    R = ctypes.POINTER(_Result)
    lib.bm_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.bm_build.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(Options), ctypes.POINTER(R)]
    lib.bm_range_sets.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_double, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64,
                                  ctypes.POINTER(Options), ctypes.POINTER(R)]
    lib.bm_build_many.argtypes = [ctypes.POINTER(Problem), ctypes.c_int32, ctypes.POINTER(Options),
                                  ctypes.POINTER(R)]
    lib.bm_result_free.argtypes = [R]
    lib.bm_result_free.restype = None
    lib.bm_last_error.restype = ctypes.c_char_p
    lib.bm_device_count.restype = ctypes.c_int
    lib.bm_abi_version.restype = ctypes.c_int
    lib.bm_error_bound.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    lib.bm_error_bound.restype = ctypes.c_int
    lib.bm_device_selfcheck.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.bm_device_selfcheck.restype = ctypes.c_int
    lib.bm_trim_cache.argtypes = [ctypes.c_int32]
    lib.bm_trim_cache.restype = ctypes.c_int
    for f in ("bm_default_options", "bm_build", "bm_range_sets", "bm_build_many"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


EXPORTED_SYMBOLS = ("bm_default_options", "bm_build", "bm_build_many", "bm_range_sets", "bm_result_free",
                    "bm_last_error", "bm_device_count", "bm_abi_version", "bm_error_bound",
                    "bm_device_selfcheck", "bm_trim_cache")


class Bound(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("abs_err", ctypes.c_double),
                ("rel_err", ctypes.c_double), ("t_in", ctypes.c_double), ("t_out", ctypes.c_double),
                ("delta", ctypes.c_double), ("exact_range", ctypes.c_int32)]


def error_bound(path, dtype, d: int, eps: float, max_sq_norm: float, max_abs: float) -> dict:
    """Constants of a path's deterministic error bound (bm_error_bound)."""
    b = Bound()
    code = DTYPES[np.dtype(dtype)]
    _check(load_library().bm_error_bound(PATHS[path] if isinstance(path, str) else int(path), code, int(d),
                                         float(eps), float(max_sq_norm), float(max_abs), ctypes.byref(b)))
    return {f: getattr(b, f) for f, _ in Bound._fields_}


def device_selfcheck(device: int = -1) -> int:
    """Matrix-core self-check flags of a device (bm_device_selfcheck)."""
    f = ctypes.c_int32()
    _check(load_library().bm_device_selfcheck(int(device), ctypes.byref(f)))
    return int(f.value)


def _check(rc: int):
    if rc != BM_OK:
        raise BmError(rc, load_library().bm_last_error().decode())


@dataclass
class BallMapper:
    """Host copy of a result: landmarks (original indices, selection order),
    membership CSR (columns ascending), edges (i < j landmark ordinals, lexicographic)."""
    landmarks: np.ndarray
    member_ptr: np.ndarray
    member_idx: np.ndarray
    edges: np.ndarray
    stats: dict

    @property
    def n_landmarks(self) -> int:
        return int(self.landmarks.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    def row(self, i: int) -> np.ndarray:
        return self.member_idx[self.member_ptr[i]:self.member_ptr[i + 1]]


class DeviceBallMapper:
    """A result whose arrays stay in device memory (results_on_device=True).
    Pointers are raw device addresses; call free() (or use as a context manager)."""

    def __init__(self, ptr):
        self._p = ptr
        r = ptr.contents
        self.n_landmarks, self.n_edges = int(r.n_landmarks), int(r.n_edges)
        self.landmarks, self.member_ptr, self.member_idx, self.edges = r.landmarks, r.member_ptr, r.member_idx, r.edges
        self.stats = r.stats.as_dict()

    def free(self):
        if self._p is not None:
            load_library().bm_result_free(self._p)
            self._p = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.free()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _take(ptr) -> BallMapper:
    r = ptr.contents
    L, E = int(r.n_landmarks), int(r.n_edges)

    def arr(p, ct, count):
        if count == 0:
            return np.zeros(0, dtype=np.dtype(ct))
        return np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ct)), shape=(count,)).copy()

    ptrs = arr(r.member_ptr, ctypes.c_int64, L + 1)
    out = BallMapper(arr(r.landmarks, ctypes.c_int32, L), ptrs,
                     arr(r.member_idx, ctypes.c_int32, int(ptrs[-1])),
                     arr(r.edges, ctypes.c_int32, 2 * E).reshape(E, 2), r.stats.as_dict())
    load_library().bm_result_free(ptr)
    return out


def _points(points):
    """numpy array (host) or torch tensor (host or device) -> (ptr, n, d, dtype, on_device, stream, keepalive)."""
    try:
        import torch  # noqa: WPS433 - optional, only for device memory and streams
        if isinstance(points, torch.Tensor):
            t = points.contiguous()
            if t.dim() != 2:
                raise ValueError("points must be (n, d)")
            code = {torch.float64: 0, torch.float32: 1, torch.float16: 2}.get(t.dtype)
            if code is None:
                raise ValueError(f"unsupported dtype {t.dtype}")
            if t.is_cuda:
                stream = torch.cuda.current_stream(t.device).cuda_stream
                return t.data_ptr(), t.shape[0], t.shape[1], code, 1, stream, t, t.device.index
            t = t.numpy()
            points = t
    except ImportError:
        pass
    x = np.ascontiguousarray(points)
    if x.ndim != 2:
        raise ValueError("points must be (n, d)")
    if x.dtype not in DTYPES:
        raise ValueError(f"unsupported dtype {x.dtype}")
    return x.ctypes.data, x.shape[0], x.shape[1], DTYPES[x.dtype], 0, None, x, None


def options(path="auto", refine=True, block=0, device=-1, results_on_device=False, max_device_bytes=0,
            init_member_capacity=0, stream=None, points_on_device=0, profile=False, graph=True) -> Options:
    o = Options()
    _check(load_library().bm_default_options(ctypes.byref(o)))
    o.path = PATHS[path] if isinstance(path, str) else int(path)
    o.refine = 1 if refine else 0
    o.block = int(block)
    o.device = int(device)
    o.points_on_device = int(points_on_device)
    o.results_on_device = 1 if results_on_device else 0
    o.max_device_bytes = int(max_device_bytes)
    o.init_member_capacity = int(init_member_capacity)
    o.stream = stream
    o.profile = 1 if profile else 0
    o.no_graph = 0 if graph else 1
    return o


def build(points, eps: float, order=None, **kw):
    """Greedy Ball Mapper of `points` at radius `eps` (bm_build)."""
    ptr, n, d, code, on_dev, stream, keep, dev = _points(points)
    o = options(points_on_device=on_dev, stream=kw.pop("stream", stream),
                device=kw.pop("device", dev if dev is not None else -1), **kw)
    ordp = None
    if order is not None:
        ordv = np.ascontiguousarray(order, dtype=np.int64)
        if ordv.shape != (n,):
            raise ValueError("order must have n entries")
        ordp = ordv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    out = ctypes.POINTER(_Result)()
    _check(load_library().bm_build(ptr, n, d, code, float(eps), ordp, ctypes.byref(o), ctypes.byref(out)))
    return DeviceBallMapper(out) if o.results_on_device else _take(out)


def range_sets(points, landmarks, eps: float, **kw):
    """Memberships and edges of a fixed landmark list (bm_range_sets)."""
    ptr, n, d, code, on_dev, stream, keep, dev = _points(points)
    o = options(points_on_device=on_dev, stream=kw.pop("stream", stream),
                device=kw.pop("device", dev if dev is not None else -1), **kw)
    lm = np.ascontiguousarray(landmarks, dtype=np.int32)
    out = ctypes.POINTER(_Result)()
    _check(load_library().bm_range_sets(ptr, n, d, code, float(eps),
                                        lm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), lm.shape[0],
                                        ctypes.byref(o), ctypes.byref(out)))
    return DeviceBallMapper(out) if o.results_on_device else _take(out)


def build_many(problems, **kw):
    """Ball Mappers of many point clouds, each over its own eps sweep (bm_build_many).

    `problems` is a list of (points, eps_list) or (points, eps_list, order).
    Returns a list (per problem) of lists (per eps)."""
    keep, probs = [], (Problem * max(1, len(problems)))()
    on_dev_all, stream0, dev0 = None, None, None
    for i, item in enumerate(problems):
        pts, eps_list = item[0], item[1]
        order = item[2] if len(item) > 2 else None
        ptr, n, d, code, on_dev, stream, kp, dev = _points(pts)
        on_dev_all = on_dev if on_dev_all is None else on_dev_all
        if on_dev != on_dev_all:
            raise ValueError("all problems must be on the host or all on the device")
        stream0 = stream0 or stream
        dev0 = dev if dev0 is None else dev0
        ev = np.ascontiguousarray(eps_list, dtype=np.float64)
        keep += [kp, ev]
        probs[i].points, probs[i].n, probs[i].d, probs[i].dtype = ptr, n, d, code
        probs[i].eps = ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        probs[i].n_eps = ev.shape[0]
        if order is not None:
            ov = np.ascontiguousarray(order, dtype=np.int64)
            keep.append(ov)
            probs[i].order = ov.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    o = options(points_on_device=on_dev_all or 0, stream=kw.pop("stream", stream0),
                device=kw.pop("device", dev0 if dev0 is not None else -1), **kw)
    total = sum(int(probs[i].n_eps) for i in range(len(problems)))
    outs = (ctypes.POINTER(_Result) * max(1, total))()
    _check(load_library().bm_build_many(probs, len(problems), ctypes.byref(o), outs))
    res, k = [], 0
    for i in range(len(problems)):
        row = []
        for _ in range(int(probs[i].n_eps)):
            row.append(DeviceBallMapper(outs[k]) if o.results_on_device else _take(outs[k]))
            k += 1
        res.append(row)
    return res


def device_count() -> int:
    return int(load_library().bm_device_count())


def trim_cache(device: int = -1) -> None:
    """Free the device blocks and pinned buffers the library keeps between
    calls (bm_trim_cache); device -1 = every device."""
    _check(load_library().bm_trim_cache(int(device)))
