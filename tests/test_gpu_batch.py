"""bm_build_many on the device: every (problem, radius) chain of a batch runs in
shared launches and is finished on the union of all chains.  Each result must
equal the oracle's (and the single build's) element by element."""
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


def mixed_problems():
    """Uneven n, d and dtypes; one with a visiting order; radii that give
    singleton balls, chains of overlaps and one huge ball."""
    rng = np.random.default_rng(7)
    probs = []
    for i, (n, d, dt) in enumerate([(1, 3, np.float64), (37, 2, np.float32), (700, 8, np.float32),
                                    (2500, 3, np.float64), (1200, 40, np.float32), (900, 16, np.float16),
                                    (3001, 5, np.float32), (64, 100, np.float32)]):
        x = W.clusters(n, d, k=3 + i, box=2.0 + i, seed=10 + i, dtype=dt)
        span = float(np.ptp(x.astype(np.float64), axis=0).max()) if n > 1 else 1.0
        eps = [0.05 * span + 1e-3, 0.2 * span + 1e-3, 0.6, 3.0 * span + 1.0]
        order = rng.permutation(n) if i == 3 else None
        probs.append((x, eps, order))
    return probs


def oracle_of(x, eps, order):
    return oracle.build(x, eps, order=order)


def test_batch_mixed_vs_oracle():
    probs = mixed_problems()
    say("batch: 8 mixed problems x 4 radii, host results")
    many = bm.build_many(probs)
    for (x, eps_list, order), row in zip(probs, many):
        for eps, got in zip(eps_list, row):
            assert_same(got, oracle_of(x, eps, order), f"n={x.shape} {x.dtype} eps={eps}")


def d2h(ptr, count, dtype):
    """Copy a raw device array of a result to the host (hipMemcpy of the HIP
    runtime the library is linked against)."""
    out = np.empty(count, dtype)
    if count:
        lib = bm.load_library()
        lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        assert lib.hipMemcpy(out.ctypes.data, ctypes.c_void_p(ptr), out.nbytes, 2) == 0
    return out


def test_batch_device_results_and_free():
    probs = mixed_problems()[2:6]
    say("batch: device-resident results, freed one by one")
    many = bm.build_many(probs, results_on_device=True)
    host = bm.build_many(probs)
    for row_d, row_h in zip(many, host):
        for d_res, h_res in zip(row_d, row_h):
            L, E = d_res.n_landmarks, d_res.n_edges
            assert (L, E) == (h_res.n_landmarks, h_res.n_edges)
            assert np.array_equal(d2h(d_res.landmarks, L, np.int32), h_res.landmarks)
            mp = d2h(d_res.member_ptr, L + 1, np.int64)
            assert np.array_equal(mp, h_res.member_ptr)
            assert np.array_equal(d2h(d_res.member_idx, int(mp[-1]), np.int32), h_res.member_idx)
            assert np.array_equal(d2h(d_res.edges, 2 * E, np.int32).reshape(E, 2), h_res.edges)
    # free in an interleaved order: the shared arrays go with the last result
    flat = [r for row in many for r in row]
    for r in flat[1::2] + flat[0::2]:
        r.free()


def test_batch_with_unbatchable_problems():
    """FP32-path problems (d past the matrix-core K) and empty clouds run one by
    one next to the batch; every slot is filled in order."""
    rng = np.random.default_rng(3)
    wide = rng.standard_normal((50, 500)).astype(np.float32)
    empty = np.zeros((0, 4), np.float32)
    small = W.clusters(400, 6, k=4, box=3.0, seed=2, dtype=np.float32)
    probs = [(small, [0.5, 1.5]), (wide, [30.0]), (empty, [1.0]), (small, [2.5])]
    say("batch with a d=500 cloud and an empty one")
    many = bm.build_many(probs)
    for (x, eps_list), row in zip(probs, many):
        for eps, got in zip(eps_list, row):
            if x.shape[0] == 0:
                assert got.n_landmarks == 0 and got.n_edges == 0
            else:
                assert_same(got, oracle.build(x, eps), f"n={x.shape} eps={eps}")
    assert many[1][0].stats["path"] == "fp32"


def test_batch_key_overflow_recomputes():
    probs = mixed_problems()[2:5]
    say("batch with a 16-key buffer (forces the recompute)")
    many = bm.build_many(probs, init_member_capacity=16)
    for (x, eps_list, order), row in zip(probs, many):
        for eps, got in zip(eps_list, row):
            assert_same(got, oracle_of(x, eps, order), f"overflow n={x.shape} eps={eps}")


@pytest.mark.parametrize("B", [1, 33, 512])
def test_batch_block_sizes(B):
    probs = mixed_problems()[1:5]
    say("batch block", B)
    many = bm.build_many(probs, block=B)
    for (x, eps_list, order), row in zip(probs, many):
        for eps, got in zip(eps_list, row):
            assert_same(got, oracle_of(x, eps, order), f"B={B} n={x.shape} eps={eps}")


def test_batch_matches_single_builds_unrefined():
    """refine = 0: the batch and the single builds take the same decisions."""
    probs = [(W.clusters(1500, 12, k=5, box=4.0, seed=9, dtype=np.float32), [0.8, 2.0]),
             (W.gaussian(800, 24, seed=4, dtype=np.float32), [3.0, 5.0])]
    say("batch unrefined vs single unrefined")
    many = bm.build_many(probs, refine=False, path="bf16")
    for (x, eps_list), row in zip(probs, many):
        for eps, got in zip(eps_list, row):
            assert_same(got, bm.build(x, eps, refine=False, path="bf16"), f"unrefined eps={eps}")


def test_batch_no_graph_same():
    probs = mixed_problems()[4:8]
    say("batch with direct launches")
    a = bm.build_many(probs, graph=False)
    b = bm.build_many(probs)
    for ra, rb in zip(a, b):
        for x, y in zip(ra, rb):
            assert_same(x, y, "graph vs direct")
