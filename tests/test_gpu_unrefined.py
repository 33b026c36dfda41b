"""The unrefined low-precision path (refine = 0) against the paper's error models.

With refine = 0 the matrix-core (or FP32) estimate decides every pair alone: a
compressed-distance range oracle (Sec. 5.4) with both false negatives and
false positives.  bm_error_bound gives the additive radius error delta of
Sec. 5.1 for the data's largest norm; the checks are the paper's statements:

* every lost (FN) or spurious (FP) membership has its true distance within
  delta of eps (Def. of the delta-accurate oracle, Sec. 5.1; FN/FP of Sec. 5.3);
* end to end, the landmarks cover X within eps + delta and are at least
  eps - delta apart (Theorem, Sec. 5.1);
* with the exact landmarks held fixed, G_{eps-delta} <= G~_eps <= G_{eps+delta}
  (Prop. nerve_incl, Sec. 5.2).
"""
import numpy as np
import pytest

import oracle
import paper_2601_01405_amd as bm
from paper_2601_01405_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [
    # (name, maker, eps, path)
    ("gauss128d", lambda: W.gaussian(3000, 128, seed=0, dtype=np.float32), 14.5, "bf16"),
    ("clusters16d", lambda: W.clusters(6000, 16, k=10, seed=0, dtype=np.float32), 2.0, "bf16x3"),
    ("clusters16d-bf16", lambda: W.clusters(4000, 16, k=10, seed=1, dtype=np.float32), 9.0, "bf16"),
    ("torus64d", lambda: W.torus(8000, 64, seed=0, dtype=np.float16), 0.3, "f16"),
    ("gauss8d-fp32", lambda: W.gaussian(3000, 8, seed=2, dtype=np.float64), 1.0, "fp32"),
]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if bm.device_count() == 0:
        pytest.skip("no GPU visible")


def sets(res):
    return [set(res.row(i).tolist()) for i in range(res.n_landmarks)]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_unrefined_within_error_model(case):
    name, make, eps, path = case
    x = make()
    w = x.astype(np.float64)
    nu = np.einsum("ij,ij->i", w, w)
    b = bm.error_bound(path, x.dtype, x.shape[1], eps, nu.max(), np.abs(w).max())
    delta = b["delta"]
    print(f"[case] unrefined {name} path={path} eps={eps} delta={delta:.3g}", flush=True)
    assert 0 < delta < eps

    # fixed landmarks: exact vs unrefined rows of the same landmark list
    ref = oracle.build(x, eps)
    lm = ref.landmarks
    approx = bm.range_sets(x, lm, eps, path=path, refine=False)
    exact_rows, approx_rows = sets(ref), sets(approx)
    e2 = eps * eps
    lo2, hi2 = (eps - delta) ** 2 * (1 - 1e-12), (eps + delta) ** 2 * (1 + 1e-12)
    fn = fp = 0
    for i, (e, a) in enumerate(zip(exact_rows, approx_rows)):
        for p in e - a:                 # lost: a true member, so s < e2
            fn += 1
            assert lo2 <= oracle.sqdist(x, int(lm[i]), int(p)) < e2
        for p in a - e:                 # spurious: not a member, so s >= e2
            fp += 1
            assert e2 <= oracle.sqdist(x, int(lm[i]), int(p)) < hi2
    m = int(ref.member_ptr[-1])
    print(f"    fixed landmarks: {m} memberships, FN={fn} FP={fp}", flush=True)

    # graph inclusion: G_{eps-delta}(L) <= G~_eps(L) <= G_{eps+delta}(L)
    lo = {tuple(e) for e in oracle.range_sets(x, lm, eps - delta).edges.tolist()}
    hi = {tuple(e) for e in oracle.range_sets(x, lm, eps + delta).edges.tolist()}
    mid = {tuple(e) for e in approx.edges.tolist()}
    assert lo <= mid <= hi

    # end to end: the unrefined greedy's own landmarks
    e2e = bm.build(x, eps, path=path, refine=False)
    L = e2e.landmarks
    assert oracle.covering_radius(x, L) < eps + delta
    assert oracle.separation(x, L) >= eps - delta
    print(f"    end to end: landmark ratio {e2e.n_landmarks / ref.n_landmarks:.4f}", flush=True)


@pytest.mark.parametrize("eps", [13.0, 14.5])
def test_unrefined_report_gauss128d_full(eps):
    """The unrefined BF16 oracle at full size (10^6 x 128 Gaussian): membership
    errors of 256 sampled landmarks against the exact FP64 rows, every error
    inside the delta band, and the end-to-end net within the Theorem's bounds
    (every one of 20000 sampled points within eps + delta of a landmark; the
    separation when the net has at most 40000 landmarks).  Prints the figures
    of the report."""
    import torch
    say = lambda *a: print("[report]", *a, flush=True)
    x = W.gaussian_128d()
    n, d = x.shape
    w = x.astype(np.float64)
    nu = np.einsum("ij,ij->i", w, w)
    b = bm.error_bound("bf16", x.dtype, d, eps, nu.max(), np.abs(w).max())
    delta = b["delta"]
    say(f"gauss128d eps={eps} delta={delta:.4g}")
    xd = torch.from_numpy(x).cuda()
    rng = np.random.default_rng(11)
    lm = np.sort(rng.choice(n, 256, replace=False)).astype(np.int32)
    exact = oracle.range_sets(x, lm, eps)
    approx = bm.range_sets(xd, lm, eps, path="bf16", refine=False)
    e2 = eps * eps
    lo2, hi2 = (eps - delta) ** 2 * (1 - 1e-12), (eps + delta) ** 2 * (1 + 1e-12)
    fn = fp = 0
    for i in range(lm.shape[0]):
        e, a = set(exact.row(i).tolist()), set(approx.row(i).tolist())
        for p in e - a:
            fn += 1
            assert lo2 <= oracle.sqdist(x, int(lm[i]), int(p)) < e2
        for p in a - e:
            fp += 1
            assert e2 <= oracle.sqdist(x, int(lm[i]), int(p)) < hi2
    m = int(exact.member_ptr[-1])
    say(f"  256 fixed landmarks: {m} exact memberships, FN={fn} FP={fp}, "
        f"recall={(m - fn) / max(m, 1):.6f} precision={(m - fn) / max(m - fn + fp, 1):.6f}")
    ref = bm.build(xd, eps)
    e2e = bm.build(xd, eps, path="bf16", refine=False)
    L = e2e.landmarks
    say(f"  end to end: L~/L={e2e.n_landmarks}/{ref.n_landmarks}={e2e.n_landmarks / ref.n_landmarks:.4f} "
        f"E~/E={e2e.n_edges}/{ref.n_edges}")
    sample = np.sort(rng.choice(n, 20000, replace=False)).astype(np.int32)
    first = oracle.first_member(x, L, eps + delta, sample)
    assert (first >= 0).all()
    say(f"  all {sample.shape[0]} sampled points within eps + delta of a landmark of the unrefined net")
    if L.shape[0] <= 40000:
        s = oracle.separation(x, L)
        assert s >= eps - delta
        say(f"  separation s/eps={s / eps:.4f} (>= 1 - delta/eps = {1 - delta / eps:.4f})")
