"""FP64 brute-force Ball Mapper oracle (arXiv 2601.01405).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_2601_01405_amd``) never imports, links or executes anything here, and
this package imports nothing from the product.

The heavy lifting is a plain C library (``bm_oracle.c``, built by ``buildlib.py``)
loaded with ctypes; ``tiny.py`` holds pure-Python versions for small inputs.

Parity pins (what ties the oracle to the paper rather than to itself) live in
``tests/test_oracle_*.py``:
  * the Gaussian worked example of Sec. 6.3 (printed eps, landmark and edge counts),
  * a hand-computed 1-D example with an exact tie at eps,
  * exact rational arithmetic for the distance predicate,
  * the eps-net certificate of Sec. 2.1 (cover and separation) and the
    lexicographically-first characterisation of the greedy of Sec. 2.2,
  * brute-force shared-membership edges on small inputs,
  * closed-form special cases (eps above the diameter, eps below the closest pair).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbm_oracle.so")
_lib = None

DTYPE_CODE = {np.dtype(np.float64): 0, np.dtype(np.float32): 1, np.dtype(np.float16): 2}


class _Result(ctypes.Structure):
    _fields_ = [
        ("n_landmarks", ctypes.c_int64),
        ("landmarks", ctypes.POINTER(ctypes.c_int32)),
        ("member_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("member_idx", ctypes.POINTER(ctypes.c_int32)),
        ("n_edges", ctypes.c_int64),
        ("edges", ctypes.POINTER(ctypes.c_int32)),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import buildlib as _b
        _b.build()
    _lib = configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def configure(lib):
    """Declare the C signatures on a loaded oracle library (also used by the
    mutation test, which loads deliberately broken copies)."""
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    lib.bmo_sqdist.argtypes = [vp, i32, i32, i64, i64]
    lib.bmo_sqdist.restype = f64
    lib.bmo_build.argtypes = [vp, i64, i32, i32, f64, P(i64), i32, i64, P(_Result)]
    lib.bmo_build.restype = ctypes.c_int
    lib.bmo_range_sets.argtypes = [vp, i64, i32, i32, f64, P(i32), i64, P(_Result)]
    lib.bmo_range_sets.restype = ctypes.c_int
    lib.bmo_edges.argtypes = [i64, i64, P(i64), P(i32), P(_Result)]
    lib.bmo_edges.restype = ctypes.c_int
    lib.bmo_knn_eps.argtypes = [vp, i64, i32, i32, i32, P(f64), P(f64)]
    lib.bmo_knn_eps.restype = ctypes.c_int
    lib.bmo_covering_radius.argtypes = [vp, i64, i32, i32, P(i32), i64]
    lib.bmo_covering_radius.restype = f64
    lib.bmo_separation.argtypes = [vp, i64, i32, i32, P(i32), i64]
    lib.bmo_separation.restype = f64
    lib.bmo_free.argtypes = [P(_Result)]
    lib.bmo_free.restype = None
    lib.bmo_threads.restype = ctypes.c_int
    lib.bmo_first_member.argtypes = [vp, i64, i32, i32, f64, P(i32), i64, P(i32), i64, P(i64)]
    lib.bmo_first_member.restype = ctypes.c_int
    return lib


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_load().bmo_threads())


@dataclass
class BallMapper:
    """Landmarks (original indices, selection order), membership CSR and edges."""
    landmarks: np.ndarray   # int32[L]
    member_ptr: np.ndarray  # int64[L+1]
    member_idx: np.ndarray  # int32[M], ascending within each row
    edges: np.ndarray       # int32[E, 2], (i, j) landmark ordinals, i < j, lexicographic

    @property
    def n_landmarks(self) -> int:
        return int(self.landmarks.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    def row(self, i: int) -> np.ndarray:
        return self.member_idx[self.member_ptr[i]:self.member_ptr[i + 1]]


def _points(points):
    x = np.ascontiguousarray(points)
    if x.ndim != 2:
        raise ValueError("points must be a 2-D (n, d) array")
    if x.dtype not in DTYPE_CODE:
        raise ValueError(f"unsupported dtype {x.dtype}")
    return x


def _take(res: _Result) -> BallMapper:
    L, E = res.n_landmarks, res.n_edges
    lm = np.ctypeslib.as_array(res.landmarks, shape=(max(L, 1),))[:L].copy()
    ptr = np.ctypeslib.as_array(res.member_ptr, shape=(L + 1,)).copy()
    M = int(ptr[-1])
    idx = np.ctypeslib.as_array(res.member_idx, shape=(max(M, 1),))[:M].copy()
    if E > 0:
        ed = np.ctypeslib.as_array(res.edges, shape=(2 * E,)).reshape(E, 2).copy()
    else:
        ed = np.zeros((0, 2), np.int32)
    _load().bmo_free(ctypes.byref(res))
    return BallMapper(lm, ptr, idx, ed)


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _i32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def sqdist(points, a: int, b: int) -> float:
    """The oracle's squared distance s(a,b) (sequential k, no FMA)."""
    x = _points(points)
    return _load().bmo_sqdist(x.ctypes.data, x.shape[1], DTYPE_CODE[x.dtype], a, b)


def build(points, eps: float, order=None, early_exit: bool = True,
          max_landmarks: int = 0) -> BallMapper:
    """Greedy Ball Mapper (Sec. 2.2) with full-ball memberships and nerve edges."""
    x = _points(points)
    n, d = x.shape
    ordp = None
    if order is not None:
        o = np.ascontiguousarray(order, dtype=np.int64)
        if o.shape != (n,) or not np.array_equal(np.sort(o), np.arange(n)):
            raise ValueError("order must be a permutation of 0..n-1")
        ordp = _i64p(o)
    res = _Result()
    rc = _load().bmo_build(x.ctypes.data, n, d, DTYPE_CODE[x.dtype], float(eps), ordp,
                           1 if early_exit else 0, int(max_landmarks), ctypes.byref(res))
    if rc != 0:
        raise ValueError(f"bmo_build failed with code {rc}")
    return _take(res)


def range_sets(points, landmarks, eps: float) -> BallMapper:
    """Exact range sets R_eps(l) of a fixed landmark list (fixed-landmark mode, Sec. 6.2)."""
    x = _points(points)
    n, d = x.shape
    lm = np.ascontiguousarray(landmarks, dtype=np.int32)
    res = _Result()
    rc = _load().bmo_range_sets(x.ctypes.data, n, d, DTYPE_CODE[x.dtype], float(eps),
                                _i32p(lm), lm.shape[0], ctypes.byref(res))
    if rc != 0:
        raise ValueError(f"bmo_range_sets failed with code {rc}")
    return _take(res)


def edges_from_csr(n: int, member_ptr, member_idx) -> np.ndarray:
    ptr = np.ascontiguousarray(member_ptr, dtype=np.int64)
    idx = np.ascontiguousarray(member_idx, dtype=np.int32)
    res = _Result()
    rc = _load().bmo_edges(n, ptr.shape[0] - 1, _i64p(ptr), _i32p(idx), ctypes.byref(res))
    if rc != 0:
        raise ValueError(f"bmo_edges failed with code {rc}")
    E = res.n_edges
    ed = (np.ctypeslib.as_array(res.edges, shape=(2 * E,)).reshape(E, 2).copy()
          if E > 0 else np.zeros((0, 2), np.int32))
    res.landmarks = ctypes.POINTER(ctypes.c_int32)()
    res.member_ptr = ctypes.POINTER(ctypes.c_int64)()
    res.member_idx = ctypes.POINTER(ctypes.c_int32)()
    _load().bmo_free(ctypes.byref(res))
    return ed


def knn_eps(points, k: int):
    """Target-occupancy eps of Sec. 6.1: (eps, per-point k-th neighbour distance)."""
    x = _points(points)
    n, d = x.shape
    kd = np.empty(n, np.float64)
    eps = ctypes.c_double()
    rc = _load().bmo_knn_eps(x.ctypes.data, n, d, DTYPE_CODE[x.dtype], int(k),
                             kd.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(eps))
    if rc != 0:
        raise ValueError(f"bmo_knn_eps failed with code {rc}")
    return eps.value, kd


def first_member(points, landmarks, eps: float, queries) -> np.ndarray:
    """Position (selection order) of the first landmark whose ball holds each query, or -1."""
    x = _points(points)
    lm = np.ascontiguousarray(landmarks, dtype=np.int32)
    q = np.ascontiguousarray(queries, dtype=np.int32)
    out = np.empty(q.shape[0], np.int64)
    rc = _load().bmo_first_member(x.ctypes.data, x.shape[0], x.shape[1], DTYPE_CODE[x.dtype], float(eps),
                                  _i32p(lm), lm.shape[0], _i32p(q), q.shape[0], _i64p(out))
    if rc != 0:
        raise ValueError(f"bmo_first_member failed with code {rc}")
    return out


def covering_radius(points, landmarks) -> float:
    x = _points(points)
    lm = np.ascontiguousarray(landmarks, dtype=np.int32)
    return _load().bmo_covering_radius(x.ctypes.data, x.shape[0], x.shape[1],
                                       DTYPE_CODE[x.dtype], _i32p(lm), lm.shape[0])


def separation(points, landmarks) -> float:
    x = _points(points)
    lm = np.ascontiguousarray(landmarks, dtype=np.int32)
    return _load().bmo_separation(x.ctypes.data, x.shape[0], x.shape[1],
                                  DTYPE_CODE[x.dtype], _i32p(lm), lm.shape[0])
