"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from
the paper's printed worked example, a hand computation, exact rational
arithmetic, a closed form, or an independent brute force.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import tiny
from paper_2601_01405_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pairwise_s(x):
    """All-pairs squared distance, summed over k left to right in float64
    (numpy elementwise ops round to nearest and never fuse)."""
    w = np.asarray(x, dtype=np.float64)
    n, d = w.shape
    acc = np.zeros((n, n))
    for k in range(d):
        t = w[:, k][:, None] - w[:, k][None, :]
        acc = acc + t * t
    return acc


def gamma(m, u=2.0 ** -53):
    return m * u / (1 - m * u)


def check_certificate(x, eps, res, order=None):
    """Eps-net + greedy certificate with an independent all-pairs predicate:
    rows are the exact range sets, landmarks are pairwise non-members
    (separation, Sec. 2.1), every non-landmark is a member of a landmark that
    comes before it in the order (the greedy of Sec. 2.2 takes the first
    uncovered point), and edges are exactly the pairs with a shared member."""
    n = x.shape[0]
    e2 = eps * eps
    mem = pairwise_s(x) < e2
    order = np.arange(n) if order is None else np.asarray(order)
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    lm = res.landmarks
    L = lm.shape[0]
    for i in range(L):
        assert np.array_equal(res.row(i), np.nonzero(mem[lm[i]])[0]), f"row {i}"
    sub = mem[np.ix_(lm, lm)]
    assert not np.any(sub & ~np.eye(L, dtype=bool)), "two landmarks within eps"
    is_lm = np.zeros(n, bool)
    is_lm[lm] = True
    for xi in np.nonzero(~is_lm)[0]:
        cov = lm[mem[lm, xi]]
        assert cov.size and rank[cov].min() < rank[xi], f"point {xi} not covered by an earlier landmark"
    assert np.all(np.diff(rank[lm]) > 0), "landmarks not in selection order"
    M = np.zeros((L, n), np.int64)
    for i in range(L):
        M[i, res.row(i)] = 1
    share = (M @ M.T) > 0
    iu = np.triu_indices(L, 1)
    exp = np.stack([iu[0][share[iu]], iu[1][share[iu]]], axis=1).astype(np.int32)
    assert np.array_equal(res.edges, exp.reshape(-1, 2))


# ---------------------------------------------------------------- worked examples

def test_paper_gaussian_worked_example():
    """Sec. 6.3: Gaussian n=20000, d=50, k=50 -> eps ~ 7.5536, 6361 landmarks, 936690 edges."""
    g = {}
    for line in open(os.path.join(GOLDEN, "gaussian_n20000_d50_k50.txt")):
        if line.strip() and not line.startswith("#"):
            key, val = line.split()
            g[key] = val
    x = W.gaussian(int(g["n"]), int(g["d"]), seed=int(g["seed"]), dtype=np.float64)
    eps, kd = oracle.knn_eps(x, int(g["k"]))
    assert round(eps, int(g["eps_printed_decimals"])) == float(g["eps_printed"])
    res = oracle.build(x, eps)
    assert res.n_landmarks == int(g["landmarks"])
    assert res.n_edges == int(g["edges"])
    # Theorem of Sec. 5.1 with delta = 0: an exact eps-net covers within eps and
    # keeps landmarks at least eps apart.
    lm = res.landmarks
    assert oracle.separation(x, lm) >= eps
    sample = np.random.default_rng(1).choice(x.shape[0], 400, replace=False)
    e2 = eps * eps
    for xi in sample:   # every sampled point has a landmark strictly within eps
        assert any(oracle.sqdist(x, int(xi), int(l)) < e2 for l in lm[:])


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.float16])
def test_hand_computed_line(dtype):
    g = json.load(open(os.path.join(GOLDEN, "line7_eps1.json")))
    x = np.asarray(g["points"], dtype=dtype)[:, None]
    eps = g["eps"]
    for a, b in g["member_pairs"]:
        assert oracle.sqdist(x, a, b) < eps * eps
    for a, b in g["tie_pairs"]:
        assert oracle.sqdist(x, a, b) == eps * eps
    for key, order in (("index_order", None), ("reverse_order", g["reverse_order"]["order"])):
        res = oracle.build(x, eps, order=order)
        exp = g[key]
        assert res.landmarks.tolist() == exp["landmarks"]
        assert res.member_ptr.tolist() == exp["member_ptr"]
        assert res.member_idx.tolist() == exp["member_idx"]
        assert res.edges.tolist() == exp["edges"]


# ---------------------------------------------------------------- the predicate

@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.float16])
def test_sqdist_bitwise_equals_plain_float64(dtype):
    """The C loop must round exactly like Python floats (RN, no FMA, k in order)."""
    rng = np.random.default_rng(7)
    x = (rng.standard_normal((60, 13)) * rng.uniform(0.1, 100, (60, 1))).astype(dtype)
    w = tiny.widen(x)
    for a in range(0, 60, 3):
        for b in range(60):
            assert oracle.sqdist(x, a, b) == tiny.sqdist_f64(w[a], w[b])


def test_sqdist_within_rounding_bound_of_exact():
    """|s - D| <= gamma_{d+2} D against exact rational arithmetic, and the
    decision s < RN(eps^2) matches the exact D < eps^2 except within that bound."""
    rng = np.random.default_rng(11)
    d = 9
    x = rng.standard_normal((40, d))
    eps = 3.3
    e2 = eps * eps
    eps_sq_exact = Fraction(eps) ** 2
    g = gamma(d + 2)
    w = tiny.widen(x)
    for a in range(40):
        for b in range(40):
            s = oracle.sqdist(x, a, b)
            D = tiny.sqdist_exact(w[a], w[b])
            assert abs(Fraction(s) - D) <= Fraction(g) * D
            if (s < e2) != (D < eps_sq_exact):
                assert abs(D - eps_sq_exact) <= Fraction(g) * D + abs(Fraction(e2) - eps_sq_exact)


def test_exact_ties_are_excluded():
    """Open balls (Sec. 2.1): a point at distance exactly eps is not a member."""
    rng = np.random.default_rng(3)
    x = rng.integers(-4, 5, (50, 3)).astype(np.float64) / 2.0   # dyadic grid
    eps = 1.5
    res = oracle.build(x, eps)
    w = tiny.widen(x)
    for i, l in enumerate(res.landmarks):
        row = set(res.row(i).tolist())
        for p in range(50):
            D = tiny.sqdist_exact(w[l], w[p])
            assert (p in row) == (D < Fraction(9, 4))


# ---------------------------------------------------------------- special cases

def test_eps_above_diameter():
    x = W.gaussian(300, 4, seed=5)
    order = np.random.default_rng(0).permutation(300)
    res = oracle.build(x, 100.0, order=order)
    assert res.landmarks.tolist() == [order[0]]
    assert res.row(0).tolist() == list(range(300))
    assert res.n_edges == 0


def test_eps_below_closest_pair():
    x = W.gaussian(200, 3, seed=6)
    smin = np.min(pairwise_s(x) + np.eye(200) * 1e9)
    eps = math.sqrt(smin)
    while eps * eps > smin:            # largest eps with RN(eps^2) <= the closest pair
        eps = math.nextafter(eps, 0.0)
    order = np.random.default_rng(1).permutation(200)
    res = oracle.build(x, eps, order=order)   # every pair is >= eps apart: nobody shares a ball
    assert res.landmarks.tolist() == order.tolist()
    assert res.member_idx.tolist() == res.landmarks.tolist()
    assert res.member_ptr.tolist() == list(range(201))
    assert res.n_edges == 0


def test_unit_spaced_line_is_a_path():
    """Points 0..n-1 on a line, 1 < eps <= 2: even points are landmarks, balls
    {2m-1, 2m, 2m+1}, consecutive landmarks share one point -> a path graph."""
    n = 11
    x = np.arange(n, dtype=np.float32)[:, None]
    res = oracle.build(x, 1.5)
    assert res.landmarks.tolist() == list(range(0, n, 2))
    assert res.edges.tolist() == [[i, i + 1] for i in range(n // 2)]
    for i, l in enumerate(res.landmarks):
        assert res.row(i).tolist() == [p for p in (l - 1, l, l + 1) if 0 <= p < n]


def test_duplicates_n1_and_empty():
    x = np.array([[1.0, 2.0], [1.0, 2.0], [5.0, 5.0], [1.0, 2.0]])
    res = oracle.build(x, 0.1)
    assert res.landmarks.tolist() == [0, 2]
    assert res.row(0).tolist() == [0, 1, 3]
    assert oracle.build(x[:1], 0.5).member_idx.tolist() == [0]
    empty = oracle.build(np.zeros((0, 3)), 1.0)
    assert empty.n_landmarks == 0 and empty.n_edges == 0 and empty.member_ptr.tolist() == [0]


def test_rejects_bad_arguments():
    x = np.zeros((4, 2))
    for eps in (0.0, -1.0, float("nan"), float("inf"), 1e-200):
        with pytest.raises(ValueError):
            oracle.build(x, eps)
    with pytest.raises(ValueError):
        oracle.build(x, 1.0, order=[0, 1, 1, 2])


# ---------------------------------------------------------------- certificates

@pytest.mark.parametrize("seed", range(4))
def test_certificate_random(seed):
    rng = np.random.default_rng(seed)
    n, d = int(rng.integers(50, 700)), int(rng.integers(1, 12))
    x = W.clusters(n, d, k=int(rng.integers(1, 6)), box=3.0, seed=seed, dtype=np.float32)
    s = pairwise_s(x)
    eps = float(np.sqrt(np.quantile(s[s > 0], rng.uniform(0.01, 0.2))))
    order = rng.permutation(n) if seed % 2 else None
    res = oracle.build(x, eps, order=order)
    check_certificate(x, eps, res, order)
    # no early exit gives the same bytes
    res2 = oracle.build(x, eps, order=order, early_exit=False)
    assert np.array_equal(res.member_idx, res2.member_idx)


@pytest.mark.parametrize("seed", range(6))
def test_matches_pure_python_greedy(seed):
    rng = np.random.default_rng(100 + seed)
    n, d = int(rng.integers(1, 60)), int(rng.integers(1, 5))
    x = rng.integers(-3, 4, (n, d)).astype(np.float64) / 2   # many exact ties
    eps = float(rng.choice([0.5, 1.0, 1.5, 2.0]))
    order = rng.permutation(n)
    lm, rows, edges = tiny.greedy(x, eps, order)
    res = oracle.build(x, eps, order=order)
    assert res.landmarks.tolist() == lm
    assert [res.row(i).tolist() for i in range(len(lm))] == rows
    assert [tuple(e) for e in res.edges.tolist()] == edges


def test_fixed_landmark_range_sets_and_edges():
    x = W.clusters(800, 5, k=4, box=4.0, seed=2)
    res = oracle.build(x, 1.2)
    fixed = oracle.range_sets(x, res.landmarks, 1.2)
    assert np.array_equal(fixed.member_ptr, res.member_ptr)
    assert np.array_equal(fixed.member_idx, res.member_idx)
    assert np.array_equal(fixed.edges, res.edges)
    assert np.array_equal(oracle.edges_from_csr(800, res.member_ptr, res.member_idx), res.edges)
    # cover / separation of the eps-net (Sec. 2.1)
    assert oracle.covering_radius(x, res.landmarks) < 1.2
    assert oracle.separation(x, res.landmarks) >= 1.2


def test_knn_eps_closed_form():
    """Points 0..n-1 on a line, k = 3 (self first): interior points have the
    sorted distances 0, 1, 1, ... so the 3rd is 1; the two end points have 0, 1, 2."""
    n = 9
    x = np.arange(n, dtype=np.float64)[:, None]
    eps, kd = oracle.knn_eps(x, 3)
    assert kd.tolist() == [2.0] + [1.0] * (n - 2) + [2.0]
    assert eps == 1.0
    eps2, _ = oracle.knn_eps(x[:4], 3)       # kd = [2, 1, 1, 2], even n -> mean of 1 and 2
    assert eps2 == 1.5


def test_threshold_is_rounded_in_double():
    """e2 = RN(eps^2) in float64: with eps = 1 + 2^-52, e2 = 1 + 2^-51 > 1, so
    two points at distance exactly 1 share a ball (a float32 threshold would
    round e2 down to 1 and split them)."""
    x = np.array([[0.0], [1.0]])
    eps = math.nextafter(1.0, 2.0)
    res = oracle.build(x, eps)
    assert res.landmarks.tolist() == [0]
    assert res.row(0).tolist() == [0, 1]


def test_first_member_matches_all_pairs_predicate():
    x = W.clusters(400, 4, k=3, box=2.0, seed=8, dtype=np.float32)
    res = oracle.build(x, 0.8)
    mem = pairwise_s(x) < 0.8 * 0.8
    got = oracle.first_member(x, res.landmarks, 0.8, np.arange(400))
    for q in range(400):
        hits = np.nonzero(mem[res.landmarks, q])[0]
        assert got[q] == (hits[0] if hits.size else -1)


def test_net_measures_hand_computed():
    """Covering radius (largest distance from a point to its nearest landmark)
    and separation (smallest distance between two landmarks) of the Theorem in
    Sec. 5.1, by hand: on the line 0..9 with landmarks at 0 and 5 the farthest
    point is 9 (4 from 5); with landmarks 0, 4, 9 every point is within 2 and
    the closest landmarks are 0 and 4.  In the plane, (0,0), (3,4), (6,8),
    (3,0) with landmarks (0,0) and (6,8): (3,4) is 5 from both, (3,0) is 3 from
    (0,0), and the landmarks are 10 apart (3-4-5 triangles)."""
    line = np.arange(10, dtype=np.float64)[:, None]
    assert oracle.covering_radius(line, [0, 5]) == 4.0
    assert oracle.separation(line, [0, 5]) == 5.0
    assert oracle.covering_radius(line, [0, 4, 9]) == 2.0
    assert oracle.separation(line, [0, 4, 9]) == 4.0
    plane = np.array([[0.0, 0.0], [3.0, 4.0], [6.0, 8.0], [3.0, 0.0]])
    assert oracle.covering_radius(plane, [0, 2]) == 5.0
    assert oracle.separation(plane, [0, 2]) == 10.0
    assert oracle.separation(plane, [1]) == math.inf       # one landmark: no pair


def test_first_member_hand_computed():
    """First landmark (selection position) whose open ball of radius 2.5 holds
    each query, on the line 0..9 with landmarks 0 then 4: 2 is 2 from both (the
    first, position 0, wins); 3 is 3 from 0 but 1 from 4; 8 is 4 from 4 and in
    no ball; 1 is 1 from 0 only.  With the landmarks listed as 4 then 0, the
    shared query 2 goes to 4 (now position 0)."""
    line = np.arange(10, dtype=np.float64)[:, None]
    assert oracle.first_member(line, [0, 4], 2.5, [2, 3, 8, 1]).tolist() == [0, 1, -1, 0]
    assert oracle.first_member(line, [4, 0], 2.5, [2, 3, 8, 1]).tolist() == [0, 0, -1, 1]
