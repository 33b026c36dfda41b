"""Candidate-block autotuner.

Times the greedy for every candidate block size B on seeded clustered clouds
(centres uniform in [-20, 20]^d, unit spread, the value law of the benchmark
workloads) in a grid of (n, d) buckets, for single builds and for batches
of same-bucket clouds, and writes the fastest B of each bucket to a C++
header that the library reads when the block size is automatic:

    python -m paper_2601_01405_amd.autotune --out paper_2601_01405_amd/csrc/tuned_blocks.h

Results do not depend on B (the blocked greedy reproduces the sequential
one exactly); only the time does.  Needs the built library and a GPU.
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# bucket edges: a cloud with n points and d coordinates falls in the last n
# bucket whose lower edge is <= n and the first d bucket whose upper edge is >= d
N_EDGES = (0, 1 << 11, 1 << 13, 1 << 15, 1 << 17)
D_EDGES = (8, 16, 32, 64, 128, 256)
BLOCKS = (64, 128, 256, 512, 1024, 2048, 4096, 8192)


def clouds(n, d, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(rng.integers(1, 21))
        centres = rng.uniform(-20.0, 20.0, (k, d))
        labels = rng.integers(0, k, n)
        out.append((centres[labels] + rng.standard_normal((n, d))).astype(np.float32))
    return out


def radii(d):
    # a singleton-ball radius and one where balls hold part of a cluster
    return [1.0, 0.6 * math.sqrt(2.0 * d)]


def time_call(fn, reps=2):
    import torch
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def bucket_point(lo_n, hi_n, d_hi):
    """A cloud size inside the bucket: the geometric middle (200000 for the open top bucket)."""
    n = int(math.sqrt(max(lo_n, 1024) * hi_n)) if hi_n else 200000
    return n, d_hi


def tune(verbose=True, quick=False):
    import torch

    import paper_2601_01405_amd as bm
    rows = []
    n_edges = list(N_EDGES) + [None]
    for i in range(len(N_EDGES)):
        lo, hi = n_edges[i], n_edges[i + 1]
        for d in D_EDGES:
            n, _ = bucket_point(lo, hi, d)
            n = min(n, 200000)
            blocks = [b for b in BLOCKS if b <= max(64, 2 * n)]
            # single build
            x = torch.from_numpy(clouds(n, d, 1, seed=n + d)[0]).cuda()
            best_s, t_s = None, float("inf")
            for B in blocks:
                t = time_call(lambda: [bm.build(x, e, block=B, results_on_device=True).free() for e in radii(d)])
                if t < t_s:
                    best_s, t_s = B, t
            # batch of same-bucket clouds
            count = 4 if quick else max(4, min(32, 2_000_000 // n))
            probs = [(torch.from_numpy(c).cuda(), radii(d)) for c in clouds(n, d, count, seed=7 * n + d)]
            best_b, t_b = None, float("inf")
            for B in blocks:
                def run():
                    for row in bm.build_many(probs, block=B, results_on_device=True):
                        for r in row:
                            r.free()
                t = time_call(run)
                if t < t_b:
                    best_b, t_b = B, t
            rows.append((lo, d, best_s, best_b))
            if verbose:
                print(f"n>={lo} d<={d} (n={n}): single B={best_s} ({t_s * 1e3:.2f} ms), "
                      f"batch of {count} B={best_b} ({t_b * 1e3:.2f} ms)", flush=True)
    return rows


def write_header(rows, path, device_name):
    lines = [
        "// tuned_blocks.h — candidate block sizes measured by paper_2601_01405_amd/autotune.py",
        f"// on {device_name}: the fastest B of each (n, d) bucket for single builds and for",
        "// batches of same-bucket clouds (clustered clouds, a singleton-ball radius and a",
        "// radius inside the clusters).  Generated; rerun the tuner to refresh.",
        "#pragma once",
        "#include <stdint.h>",
        "",
        "namespace bm {",
        "",
        "struct TunedBlock {",
        "    int64_t n_min;      // the bucket holds n >= n_min (up to the next row's n_min)",
        "    int32_t d_max;      // and d <= d_max (above the previous row's d_max)",
        "    int32_t single;     // B for one build",
        "    int32_t batch;      // B for each chain of a batch",
        "};",
        "",
        "constexpr TunedBlock kTunedBlocks[] = {",
    ]
    for lo, d, bs, bb in rows:
        lines.append(f"    {{{lo}, {d}, {bs}, {bb}}},")
    lines += ["};", "", "} // namespace bm", ""]
    with open(path, "w") as fh:
        fh.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2601_01405_amd", "csrc", "tuned_blocks.h"))
    ap.add_argument("--quick", action="store_true", help="small batches (a smoke run of the tuner)")
    a = ap.parse_args()
    import torch
    rows = tune(quick=a.quick)
    props = torch.cuda.get_device_properties(0)
    write_header(rows, a.out, f"{props.name} ({getattr(props, 'gcnArchName', 'unknown arch')})")
    print(f"wrote {a.out}")


if __name__ == "__main__":
    main()
