"""The library's cache of device blocks, pinned staging and streams between
calls: reused memory never changes a result, the memory cap still holds, and
trimming the cache leaves the library usable."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2601_01405_amd as bm
from paper_2601_01405_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if bm.device_count() == 0:
        pytest.skip("no GPU visible")


def say(*a):
    print("[case]", *a, flush=True)


def assert_same(got, ref, what=""):
    for name in ("landmarks", "member_ptr", "member_idx", "edges"):
        a, b = getattr(got, name), getattr(ref, name)
        assert a.shape == b.shape and np.array_equal(a, b), f"{what}: {name} differs"


def test_reused_blocks_give_the_same_results():
    """Alternating sizes: each build takes blocks a larger or smaller one left
    behind (stale contents), and must still equal the oracle."""
    big = W.clusters(20000, 16, k=12, box=10.0, seed=5, dtype=np.float32)
    small = W.clusters(3000, 8, k=4, box=3.0, seed=6, dtype=np.float32)
    refs = {("big", 1.2): oracle.build(big, 1.2), ("small", 0.7): oracle.build(small, 0.7),
            ("small", 2.5): oracle.build(small, 2.5)}
    for rnd in range(3):
        for name, x, eps in (("big", big, 1.2), ("small", small, 0.7), ("small", small, 2.5)):
            say("cache round", rnd, name, eps)
            assert_same(bm.build(x, eps), refs[(name, eps)], f"{name} eps={eps} round {rnd}")
    bm.trim_cache()
    assert_same(bm.build(small, 0.7), refs[("small", 0.7)], "after trim")


def test_memory_cap_still_enforced():
    x = W.clusters(50000, 16, k=8, box=8.0, seed=8, dtype=np.float32)
    ref = bm.build(x, 1.5)
    say("cap of 1 MiB")
    with pytest.raises(bm.BmError) as ei:
        bm.build(x, 1.5, max_device_bytes=1 << 20)
    assert ei.value.code == bm.BM_ENOMEM
    say("generous cap")
    assert_same(bm.build(x, 1.5, max_device_bytes=1 << 33), ref, "8 GiB cap")
    assert_same(bm.build(x, 1.5), ref, "after the failed call")


def test_device_results_outlive_the_cache():
    """Device-resident results are the caller's: a trim and later builds do not
    touch them."""
    x = W.clusters(8000, 12, k=5, box=5.0, seed=9, dtype=np.float32)
    host = bm.build(x, 1.1)
    dres = bm.build(x, 1.1, results_on_device=True)
    bm.trim_cache(-1)
    for _ in range(2):
        bm.build(W.clusters(9000, 12, k=6, box=5.0, seed=10, dtype=np.float32), 0.9)
    L, E = dres.n_landmarks, dres.n_edges
    assert (L, E) == (host.n_landmarks, host.n_edges)
    assert np.array_equal(d2h(dres.landmarks, L, np.int32), host.landmarks)
    mp = d2h(dres.member_ptr, L + 1, np.int64)
    assert np.array_equal(mp, host.member_ptr)
    assert np.array_equal(d2h(dres.member_idx, int(mp[-1]), np.int32), host.member_idx)
    assert np.array_equal(d2h(dres.edges, 2 * E, np.int32).reshape(E, 2), host.edges)
    dres.free()


def d2h(ptr, count, dtype):
    """Copy a raw device array of a result to the host (hipMemcpy of the HIP
    runtime the library is linked against)."""
    out = np.empty(count, dtype)
    if count:
        lib = bm.load_library()
        lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        assert lib.hipMemcpy(out.ctypes.data, ctypes.c_void_p(ptr), out.nbytes, 2) == 0
    return out
