"""Parity at the benchmark workloads' full sizes, in the launch configuration
bench.py times (device-resident points, automatic path and block size).

The 200k-point clustered workload is compared with the oracle in full.  For
the larger ones the oracle computes sampled outputs one by one (rows of
sampled landmarks, the first covering landmark of sampled points), and
properties that hold at any size are checked on the whole result (every
point covered, each landmark in its own row, rows sorted, edges exactly the
pairs of rows that share a point, on sampled pairs).
"""
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


def gpu_build(x, eps, **kw):
    import torch
    xd = torch.from_numpy(x).cuda()
    return bm.build(xd, eps, **kw)


def check_sampled(x, eps, got, rng, n_rows=12, n_points=300, n_pairs=3000):
    n = x.shape[0]
    L = got.n_landmarks
    lm = got.landmarks
    # landmarks: distinct, in index (selection) order
    assert L > 0 and np.all(np.diff(lm) > 0)
    ptr, idx = got.member_ptr, got.member_idx
    # rows: sorted, each landmark in its own row
    sizes = np.diff(ptr)
    assert np.all(sizes > 0)
    for i in rng.choice(L, min(L, 2000), replace=False):
        r = idx[ptr[i]:ptr[i + 1]]
        assert np.all(np.diff(r) > 0) and lm[i] in r
    # every point is in some ball (the greedy covers X)
    covered = np.zeros(n, bool)
    covered[idx] = True
    assert covered.all()
    # sampled rows equal the oracle's range sets
    pick = rng.choice(L, min(L, n_rows), replace=False)
    ref = oracle.range_sets(x, lm[pick], eps)
    for j, i in enumerate(pick):
        assert np.array_equal(got.row(int(i)), ref.row(j)), f"row {i}"
    # sampled points: the first landmark (selection order) holding them is not after them,
    # and a non-landmark's first holder comes before it (greedy in index order)
    q = rng.choice(n, n_points, replace=False).astype(np.int32)
    first = oracle.first_member(x, lm, eps, q)
    is_lm = np.zeros(n, bool)
    is_lm[lm] = True
    for qi, f in zip(q, first):
        assert f >= 0
        if is_lm[qi]:
            assert lm[f] == qi            # nothing earlier covers a landmark (separation)
        else:
            assert lm[f] < qi
    # edges: sampled edges share a point; sampled landmark pairs not listed share none
    E = got.n_edges
    ed = got.edges
    if E:
        assert np.all(ed[:, 0] < ed[:, 1])
        keys = ed[:, 0].astype(np.int64) * L + ed[:, 1]
        assert np.all(np.diff(keys) > 0)
        for i, j in ed[rng.choice(E, min(E, n_pairs), replace=False)]:
            assert np.intersect1d(got.row(int(i)), got.row(int(j)), assume_unique=True).size > 0
        edge_set = set(keys.tolist())
    else:
        edge_set = set()
    if L > 1:
        for _ in range(n_pairs):
            i, j = sorted(rng.choice(L, 2, replace=False))
            share = np.intersect1d(got.row(int(i)), got.row(int(j)), assume_unique=True).size > 0
            assert share == ((int(i) * L + int(j)) in edge_set)


@pytest.mark.parametrize("eps", [1.0, 2.0])
def test_clusters16d_full_vs_oracle(eps):
    x = W.clusters_16d()
    say("clusters16d n=200000 eps", eps, "full oracle")
    got = gpu_build(x, eps)
    ref = oracle.build(x, eps)
    for name in ("landmarks", "member_ptr", "member_idx", "edges"):
        assert np.array_equal(getattr(got, name), getattr(ref, name)), name
    assert got.stats["path"] == "bf16x3"


@pytest.mark.parametrize("eps", [13.0, 14.5])
def test_gaussian128d_full_sampled(eps):
    x = W.gaussian_128d()
    say("gauss128d n=1000000 eps", eps, "sampled")
    got = gpu_build(x, eps, block=256)
    say("   L", got.n_landmarks, "M", int(got.member_ptr[-1]), "E", got.n_edges, "stats", got.stats)
    check_sampled(x, eps, got, np.random.default_rng(int(eps * 10)))


@pytest.mark.parametrize("eps", [0.3, 0.1])
def test_torus64d_full_sampled(eps):
    x = W.torus_64d()
    say("torus64d n=2000000 f16 eps", eps, "sampled")
    got = gpu_build(x, eps)
    say("   L", got.n_landmarks, "M", int(got.member_ptr[-1]), "E", got.n_edges, "stats", got.stats)
    check_sampled(x, eps, got, np.random.default_rng(int(eps * 100)), n_points=100)


def test_batched_workload_subset():
    probs = W.batched()
    order = np.argsort([p.points.shape[0] for p in probs])
    small = [probs[i] for i in order[:6]]
    say("batched: 6 smallest of 256 datasets x 8 eps, full oracle; largest sampled")
    many = bm.build_many([(p.points, p.eps) for p in small])
    for p, row in zip(small, many):
        for eps, got in zip(p.eps, row):
            ref = oracle.build(p.points, eps)
            for name in ("landmarks", "member_ptr", "member_idx", "edges"):
                assert np.array_equal(getattr(got, name), getattr(ref, name)), (p.points.shape, eps, name)
    big = probs[order[-1]]
    for eps in (big.eps[0], big.eps[-1]):
        got = gpu_build(big.points, eps)
        check_sampled(big.points, eps, got, np.random.default_rng(5), n_points=100)
