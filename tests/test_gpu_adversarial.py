"""Near-eps pairs at scale: 2048 landmarks in a tiny cloud around a far-off
centre and 2^19 points on spheres around it.  "thin": radius eps with radial
jitter 1e-6, so each of the 1.07e9 landmark-point pairs lies within about 1e-5
of eps (relative), inside or at the edge of every path's error band.  "wide":
radius eps (1 + s), s uniform in [-0.05, 0.05], so the pairs straddle the
band edges of the split and F16 paths (their band is a few per cent of eps^2
at these norms) and the filter decides most of them.  Each refined path must
return exactly the FP64 oracle's memberships: a pair the filter decided on
the wrong side (sure-in or sure-out) would show as a difference."""
import numpy as np
import pytest

import oracle
import paper_2601_01405_amd as bm

pytestmark = pytest.mark.gpu

EPS = 2.0


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if bm.device_count() == 0:
        pytest.skip("no GPU visible")


@pytest.fixture(scope="module", params=["thin", "wide"])
def case(request):
    rng = np.random.default_rng(5)
    d, n, L = 16, 1 << 19, 2048
    c = rng.uniform(-20.0, 20.0, d)                       # |c|^2 ~ 2000: large norms
    u = rng.standard_normal((n, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    if request.param == "thin":
        r = EPS * (1.0 + 1e-6 * rng.standard_normal(n))
    else:
        r = EPS * (1.0 + rng.uniform(-0.05, 0.05, n))
    pts = c + u * r[:, None]
    lms = c + 1e-5 * rng.standard_normal((L, d))
    x = np.concatenate([lms, pts]).astype(np.float32)
    lm = np.arange(L, dtype=np.int32)
    print(f"[case] near-eps {request.param}: {L} landmarks x {n + L} points, oracle rows", flush=True)
    ref = oracle.range_sets(x, lm, EPS)
    print(f"[case] oracle: {int(ref.member_ptr[-1])} memberships, {ref.n_edges} edges", flush=True)
    return x, lm, ref


@pytest.mark.parametrize("path", ["bf16x3", "bf16", "f16", "fp32"])
def test_near_eps_pairs_exact(case, path):
    x, lm, ref = case
    print(f"[case] near-eps path={path}", flush=True)
    got = bm.range_sets(x, lm, EPS, path=path)
    for name in ("landmarks", "member_ptr", "member_idx", "edges"):
        a, b = getattr(got, name), getattr(ref, name)
        assert a.shape == b.shape and np.array_equal(a, b), f"{path}: {name} differs"
    print(f"[case] near-eps path={path}: identical, {got.stats['band_pairs']} pairs rechecked in FP64",
          flush=True)
