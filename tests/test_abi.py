"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects bad arguments with the documented status codes
before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2601_01405_amd as bm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "bm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*\*?\s*(bm_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = bm.load_library()
    names = header_functions()
    assert len(names) >= 8, names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in bm.h but not exported"
    assert set(names) == set(bm.EXPORTED_SYMBOLS)
    assert lib.bm_abi_version() == 2


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors have the sizes and field offsets the C compiler gives bm.h."""
    mirrors = {"bm_options": bm.Options, "bm_stats": bm.Stats, "bm_result": bm._Result,
               "bm_problem": bm.Problem, "bm_bound": bm.Bound}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bm.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_default_options():
    o = bm.options()
    assert (o.path, o.refine, o.block, o.device, o.points_on_device, o.results_on_device) == (0, 1, 0, -1, 0, 0)
    assert bm.load_library().bm_default_options(None) == bm.BM_EINVAL


def _code(fn):
    with pytest.raises(bm.BmError) as e:
        fn()
    return e.value.code


@pytest.mark.parametrize("eps", [0.0, -1.0, float("nan"), float("inf"), 1e-170])
def test_bad_eps(eps):
    x = np.zeros((4, 2))
    assert _code(lambda: bm.build(x, eps)) == bm.BM_EINVAL


def test_bad_arguments():
    x = np.zeros((4, 2))
    assert _code(lambda: bm.build(x, 1.0, order=[0, 1, 1, 2])) == bm.BM_EINVAL
    assert _code(lambda: bm.build(x, 1.0, order=[0, 1, 2, 4])) == bm.BM_EINVAL
    assert _code(lambda: bm.build(x, 1.0, block=20000)) == bm.BM_EINVAL
    assert _code(lambda: bm.build(x, 1.0, path=9)) == bm.BM_EINVAL
    assert _code(lambda: bm.range_sets(x, [0, 4], 1.0)) == bm.BM_EINVAL
    lib = bm.load_library()
    out = ctypes.POINTER(bm._Result)()
    assert lib.bm_build(None, 3, 2, 0, 1.0, None, None, ctypes.byref(out)) == bm.BM_EINVAL
    assert lib.bm_build(None, 0, 0, 0, 1.0, None, None, ctypes.byref(out)) == bm.BM_EINVAL   # d < 1
    assert lib.bm_build(None, -1, 2, 0, 1.0, None, None, ctypes.byref(out)) == bm.BM_EINVAL
    assert lib.bm_build(None, 0, 2, 7, 1.0, None, None, ctypes.byref(out)) == bm.BM_EINVAL   # dtype
    assert not out
    assert "dtype" in lib.bm_last_error().decode()


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.float16])
def test_non_finite(dtype):
    x = np.zeros((5, 3), dtype=dtype)
    x[3, 1] = np.inf if dtype != np.float64 else np.nan
    assert _code(lambda: bm.build(x, 1.0)) == bm.BM_ENONFINITE


def test_no_device_reported():
    if bm.device_count() > 0:
        pytest.skip("a GPU is visible")
    x = np.random.default_rng(0).standard_normal((10, 3))
    assert _code(lambda: bm.build(x, 1.0)) == bm.BM_ENODEVICE
    assert _code(lambda: bm.build_many([(x, [1.0, 2.0])])) == bm.BM_ENODEVICE


def test_result_free_is_null_safe():
    bm.load_library().bm_result_free(None)


def test_trim_cache_rejects_unknown_device():
    lib = bm.load_library()
    assert lib.bm_trim_cache(-2) == bm.BM_EINVAL
    assert lib.bm_trim_cache(1 << 20) == bm.BM_EINVAL
    assert b"no such device" in lib.bm_last_error()
