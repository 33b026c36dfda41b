#!/usr/bin/env python3
"""Ball Mapper construction benchmark on one MI355X.

One step = the whole hot path (greedy landmark selection by blocked range
queries, membership CSR, nerve edges) at every eps of the workload, with the
points already resident in HBM and the results left in device memory.  The
headline value is landmark-point pair distances per second of the refined
low-precision path (bit-identical to the FP64 oracle); the plain FP32 path is
timed on the same inputs for comparison.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G pair-dists/s + Ball Mapper graph time, refined-BF16 vs FP32, bit-exact"
PEAK_BF16_TFLOPS = 2500.0       # MI355X dense bf16 matrix peak
PEAK_F16_TFLOPS = 2500.0
PEAK_FP32_VALU_TFLOPS = 157.3
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "range_mfma_clusters16d_n200k_traffic.txt")
TRAFFIC_WORKLOAD = "clusters16d_n200k_f32"     # the workload those counters were taken on
KERNEL_SRC = os.path.join(ROOT, "paper_2601_01405_amd", "csrc", "range_mfma.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="clusters16d_n200k_f32",
                    help="a named single-cloud workload, or 'batched' (256 clouds x 8 radii)")
    ap.add_argument("--path", default="auto", help="refined path (auto, bf16, bf16x3, f16)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, run a plain copy kernel of known size (HBM counter calibration)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("DB", "OUT"),
                    help="write a kernel-trace summary of a rocprofv3 database and exit")
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("FETCH_DB", "WRITE_DB", "OUT"),
                    help="write the range pass's HBM traffic per launch from two rocprofv3 --pmc databases")
    ap.add_argument("--summarize-sq", nargs=2, metavar=("DB", "OUT"),
                    help="write the range pass's matrix-core use from a rocprofv3 --pmc run of the SQ counters")
    ap.add_argument("--command", default="", help="the profiled command, recorded in a summary")
    return ap.parse_args()


def digest(r):
    h = hashlib.sha256()
    for a in (r.landmarks, r.member_ptr, r.member_idx, r.edges):
        h.update(a.tobytes())
    return h.hexdigest()


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(pairs_per_launch_known):
    """HBM bytes per range-pass launch from the committed rocprofv3 counter
    summary, or None if it is missing or was taken on another kernel version."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---- rocprofv3 summaries (run on the host after a profiled bench run) -------------------
PROBE_ELEMS = 1 << 26                    # float32: 256 MiB read + 256 MiB written per launch
PROBE_BYTES = PROBE_ELEMS * 4


def copy_probe():
    """A plain elementwise kernel with known traffic, for scaling the counters."""
    import torch
    src = torch.ones(PROBE_ELEMS, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()


def _template_args(name):
    a = name.find("<")
    b = name.find(">(")
    return [t.strip() for t in name[a + 1:b].split(",")] if a >= 0 and b > a else []


def is_range_pass(name):
    """The membership range pass (not the candidate-block resolve, which
    instantiates the same kernel with CONFLICT = true)."""
    if "k_range_mfma<" not in name:
        return False
    ta = _template_args(name)
    return len(ta) >= 3 and ta[2] == "false"


def _dispatch_values(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 --pmc output: the
    counter_collection CSV (--output-format csv) or the SQLite database."""
    per = {}
    if path.endswith(".csv"):
        import csv
        for row in csv.DictReader(open(path)):
            if row.get("Counter_Name") != counter:
                continue
            key = (row["Kernel_Name"], row["Dispatch_Id"])
            per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
        return per
    import sqlite3
    con = sqlite3.connect(path)
    for name, disp, value in con.execute(
            "select kernel_name, dispatch_id, value from counters_collection where counter_name = ?", (counter,)):
        key = (name, disp)
        per[key] = per.get(key, 0.0) + float(value)
    con.close()
    return per


def _kernel_spans(path):
    """(name, start_ns, end_ns) of every dispatch in a rocprofv3 kernel trace
    (kernel_trace CSV or SQLite database)."""
    if path.endswith(".csv"):
        import csv
        return [(r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                for r in csv.DictReader(open(path))]
    import sqlite3
    con = sqlite3.connect(path)
    rows = list(con.execute("select name, start, \"end\" from kernels"))
    con.close()
    return rows


def summarize_traffic(fetch_db, write_db, out, command):
    lines = ["# HBM traffic of the range pass (k_range_mfma, membership mode), from rocprofv3 counters",
             f"# command (run twice, once per counter): {command}",
             "# FETCH_SIZE and WRITE_SIZE are in KiB per dispatch; each is scaled by the factor that",
             f"# makes it read {PROBE_BYTES} bytes for a plain copy kernel (torch.neg over {PROBE_ELEMS} float32)"]
    res = {}
    for counter, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        per = _dispatch_values(db, counter)
        rng = [v for (name, _), v in per.items() if is_range_pass(name)]
        probe = [v for (name, _), v in per.items() if "neg_kernel" in name]
        if not rng or not probe:
            raise SystemExit(f"{db}: {counter}: {len(rng)} range-pass and {len(probe)} probe dispatches")
        f = PROBE_BYTES / (sum(probe) / len(probe) * 1024.0)
        kib = sum(rng) / len(rng)
        res[counter] = kib * 1024.0 * f
        lines += [f"{counter.lower()}_range_dispatches = {len(rng)}",
                  f"{counter.lower()}_kib_per_launch = {kib:.1f}",
                  f"{counter.lower()}_probe_kib = {sum(probe) / len(probe):.1f}",
                  f"{counter.lower()}_scale = {f:.5f}",
                  f"{counter.lower()}_bytes_per_launch = {res[counter]:.0f}"]
    lines += [f"kernel_source_sha256_16 = {kernel_hash()}",
              f"hbm_bytes_per_launch = {res['FETCH_SIZE'] + res['WRITE_SIZE']:.0f}"]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


SQ_COUNTERS = ("SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_MFMA", "SQ_INSTS_VALU", "SQ_INSTS_LDS",
               "SQ_WAVES", "SQ_BUSY_CYCLES")


def summarize_sq(db, out, command, durations_db=None):
    """Matrix-core use of the range pass from one rocprofv3 --pmc run of the SQ
    counters: per dispatch averages, and MFMA busy cycles over GPU-active cycles
    of all 1024 SIMDs (rocprofv3's MfmaUtil definition)."""
    lines = ["# Matrix-core use of the range pass (k_range_mfma, membership mode), rocprofv3 SQ counters",
             f"# command: {command}",
             "# values are per dispatch, averaged over the range-pass dispatches"]
    avg = {}
    for c in SQ_COUNTERS:
        per = _dispatch_values(db, c)
        v = [x for (name, _), x in per.items() if is_range_pass(name)]
        if v:
            avg[c] = sum(v) / len(v)
            lines.append(f"{c.lower()}_per_dispatch = {avg[c]:.0f}")
    if "SQ_VALU_MFMA_BUSY_CYCLES" in avg and avg.get("GRBM_GUI_ACTIVE"):
        # the CSV sums GRBM_GUI_ACTIVE over the 8 XCDs (it reads about 8x the
        # dispatch's duration in 2.4 GHz cycles); one XCD's count is the GPU's
        # active time
        active = avg["GRBM_GUI_ACTIVE"] / 8.0
        util = avg["SQ_VALU_MFMA_BUSY_CYCLES"] / (active * 1024.0)
        lines.append(f"gpu_active_cycles_per_dispatch = {active:.0f}   # GRBM_GUI_ACTIVE / 8 XCDs")
        lines.append(f"mfma_busy_fraction = {util:.4f}   "
                     "# SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x 1024 SIMDs)")
    if "SQ_INSTS_MFMA" in avg and "SQ_INSTS_VALU" in avg:
        lines.append(f"valu_insts_per_mfma = {avg['SQ_INSTS_VALU'] / max(avg['SQ_INSTS_MFMA'], 1.0):.2f}")
    lines.append(f"kernel_source_sha256_16 = {kernel_hash()}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_trace(db, out, command):
    rows = {}
    for name, start, end in _kernel_spans(db):
        key = name.split("(")[0].replace("void ", "")
        if is_range_pass(name):
            key += "  [range pass]"
        c, t = rows.get(key, (0, 0.0))
        rows[key] = (c + 1, t + (end - start) / 1e3)
    total = sum(t for _, t in rows.values()) or 1.0
    lines = [f"# Kernel trace summary (rocprofv3 --kernel-trace --stats), durations in microseconds",
             f"# command: {command}", "",
             "| kernel | calls | total us | avg us | % |", "|---|---:|---:|---:|---:|"]
    for key, (c, t) in sorted(rows.items(), key=lambda kv: -kv[1][1])[:25]:
        lines.append(f"| {key} | {c} | {t:.0f} | {t / c:.2f} | {100 * t / total:.2f} |")
    rp = [(c, t) for k, (c, t) in rows.items() if k.endswith("[range pass]")]
    if rp:
        c = sum(x for x, _ in rp)
        t = sum(y for _, y in rp)
        lines += ["", f"range pass: {c} launches, average {t / c:.2f} us"]
    lines.append(f"kernel_source_sha256_16 = {kernel_hash()}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def range_roofline(runs, d, used_path, steps, workload):
    """Roofline entry of the range pass from profiled runs (device-clock windows).
    The HBM traffic comes from counters taken on one workload; other workloads
    report none."""
    range_ms = sum(s["ms_range_kernel"] for run in runs for s in run)
    launches = sum(s["range_launches"] for run in runs for s in run)
    range_pairs = sum(s["range_pairs"] for run in runs for s in run)
    flops = 2.0 * d * range_pairs
    achieved = flops / (range_ms * 1e-3) / 1e12 if range_ms > 0 else None
    peak = PEAK_F16_TFLOPS if used_path == "f16" else PEAK_BF16_TFLOPS
    return {"bound": "mfma", "kernel": "k_range_mfma", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": (achieved / peak) if achieved else None,
            "traffic": read_traffic(range_pairs / max(launches, 1)) if workload == TRAFFIC_WORKLOAD else None,
            "per_launch_ms": range_ms / max(launches, 1),
            "launches_per_step": launches / steps,
            "flops_per_pair": 2 * d, "pairs_per_launch": range_pairs / max(launches, 1),
            "timing": "per_launch_ms: execution window of each range-pass launch on the device clock "
                      "(first wave start to last wave end), summed over a profiled repeat of the timed "
                      "steps; achieved = 2 d flops per landmark-point pair of those launches / that time"}


def bench_batched(args):
    """The batched workload: 256 seeded Gaussian mixtures (n log-uniform in
    [1000, 200000], d in {8, 32, 96}) x 8 radii, one bm_build_many per step."""
    import numpy as np
    import torch

    import paper_2601_01405_amd as bm
    from paper_2601_01405_amd import workloads as W

    probs = W.batched()
    ntot = sum(p.points.shape[0] for p in probs)
    log(f"workload batched: {len(probs)} clouds, sum n = {ntot}, 8 radii each")
    dev = [(torch.from_numpy(p.points).cuda(), p.eps) for p in probs]
    torch.cuda.synchronize()

    def step(profile=False):
        res = bm.build_many(dev, results_on_device=True, profile=profile)
        st = [r.stats for row in res for r in row]
        for row in res:
            for r in row:
                r.free()
        return st

    # parity of the same batch (host results), outside the timed region: the three
    # smallest clouds in full against the oracle at three radii each, and sampled
    # rows of the largest cloud at its smallest and largest radius
    import oracle
    exact = True
    host = bm.build_many(dev)
    order = np.argsort([p.points.shape[0] for p in probs])
    for i in order[:3]:
        p, row = probs[i], host[i]
        for eps, got in zip(p.eps[::3], row[::3]):
            ref = oracle.build(p.points, eps)
            for name in ("landmarks", "member_ptr", "member_idx", "edges"):
                exact &= bool(np.array_equal(getattr(got, name), getattr(ref, name)))
    big = int(order[-1])
    rng = np.random.default_rng(0)
    for j in (0, len(probs[big].eps) - 1):
        got = host[big][j]
        pick = rng.choice(got.n_landmarks, min(8, got.n_landmarks), replace=False)
        ref = oracle.range_sets(probs[big].points, got.landmarks[pick], probs[big].eps[j])
        for k, i in enumerate(pick):
            exact &= bool(np.array_equal(got.row(int(i)), ref.row(k)))
    del host
    log(f"bit-exact (3 smallest clouds in full, sampled rows of the largest): {exact}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pairs = sum(s["pairs_useful"] for run in runs for s in run)
    value = pairs / elapsed / 1e9
    paths = {}
    for p, s in zip([p for p in probs for _ in p.eps], runs[0]):
        key = f"d={p.points.shape[1]}:{s['path']}"
        paths[key] = paths.get(key, 0) + 1
    log(f"batched: {value:.1f} G pair-dists/s, {elapsed / args.steps * 1e3:.1f} ms/step, paths {paths}")
    line = {
        "metric": METRIC + " (batched sweep)", "value": value, "unit": "G pair-dists/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16/f16",
        "data": "synthetic",
        "config": {"workload": "batched_256x8", "clouds": len(probs), "sum_n": ntot, "radii": 8,
                   "chains": sum(len(p.eps) for p in probs), "paths": paths},
        "graph_ms": runs[0][0]["ms_total"], "bit_exact": exact,
    }
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.command)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace, args.command)
        return
    if args.summarize_sq:
        summarize_sq(*args.summarize_sq, args.command)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
        return
    import numpy as np
    import torch

    import paper_2601_01405_amd as bm
    from paper_2601_01405_amd import workloads as W

    spec = W.WORKLOADS[args.workload]
    x = spec["make"]()
    eps_list = spec["eps"]
    n, d = x.shape
    log(f"workload {args.workload}: n={n} d={d} dtype={x.dtype} eps={eps_list}")
    xd = torch.from_numpy(x).to("cuda:0")
    torch.cuda.synchronize()

    def step(path, profile=False):
        out = []
        for eps in eps_list:
            r = bm.build(xd, eps, path=path, block=args.block, results_on_device=True, profile=profile)
            out.append(dict(r.stats, n_landmarks=r.n_landmarks, n_edges=r.n_edges))
            r.free()
        return out

    # -- bit-exactness across paths, outside the timed region
    ref_path = "fp32"
    exact = True
    host = {}
    for eps in eps_list:
        a = bm.build(xd, eps, path=args.path, block=args.block)
        b = bm.build(xd, eps, path=ref_path, block=args.block)
        host[eps] = a
        same = digest(a) == digest(b)
        exact &= same
        log(f"eps={eps}: L={a.n_landmarks} M={int(a.member_ptr[-1])} E={a.n_edges} path={a.stats['path']} "
            f"identical to {ref_path}: {same}")
    # sampled check of full-size rows against the FP64 oracle (one by one)
    import oracle
    rng = np.random.default_rng(0)
    for eps in eps_list:
        a = host[eps]
        pick = rng.choice(a.n_landmarks, min(8, a.n_landmarks), replace=False)
        ref = oracle.range_sets(x, a.landmarks[pick], eps)
        for j, i in enumerate(pick):
            exact &= bool(np.array_equal(a.row(int(i)), ref.row(j)))
    log(f"bit-exact (paths identical, sampled rows equal the oracle): {exact}")

    # -- refined path, timed (the product path: no profiling)
    for _ in range(args.warmup):
        step(args.path)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(args.path) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pairs = sum(s["pairs_useful"] for run in runs for s in run)
    value = pairs / elapsed / 1e9
    used_path = runs[0][0]["path"]
    block = runs[0][0]["block"]
    graph_ms = {f"eps={eps}": float(np.median([run[i]["ms_total"] for run in runs]))
                for i, eps in enumerate(eps_list)}
    log(f"refined {used_path}: {value:.1f} G pair-dists/s, {elapsed / args.steps * 1e3:.2f} ms/step")
    # -- the same steps again with the range passes' device-clock windows recorded
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pruns = [step(args.path, profile=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    prof_ms = (time.perf_counter() - t0) / args.steps * 1e3
    roofline = range_roofline(pruns, d, used_path, args.steps, args.workload)
    log(f"profiled repeat: {prof_ms:.2f} ms/step, range passes {roofline['per_launch_ms'] * 1e3:.1f} us/launch, "
        f"{roofline['achieved']:.1f} TFLOP/s algorithmic")

    # -- plain FP32 path on the same inputs
    fp32 = None
    if not args.no_fp32:
        step("fp32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fsteps = max(1, min(args.steps, 3))
        fr = [step("fp32") for _ in range(fsteps)]
        torch.cuda.synchronize()
        fel = time.perf_counter() - t0
        fpairs = sum(s["pairs_useful"] for run in fr for s in run)
        fp32 = {"value": fpairs / fel / 1e9, "ms_per_step": fel / fsteps * 1e3, "steps": fsteps}
        log(f"fp32: {fp32['value']:.1f} G pair-dists/s, {fp32['ms_per_step']:.2f} ms/step")

    # -- the FP64 oracle on the host, a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        eps = eps_list[0]
        t0 = time.perf_counter()
        probe = oracle.build(x, eps, max_landmarks=50)
        tp = time.perf_counter() - t0
        k = int(max(50, min(50 * args.cpu_seconds / max(tp, 1e-3), 200000)))
        t0 = time.perf_counter()
        smp = oracle.build(x, eps, max_landmarks=k)
        tc = time.perf_counter() - t0
        cpu = {"value": smp.n_landmarks * n / tc / 1e9, "unit": "G pair-dists/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"first {smp.n_landmarks} landmarks of the greedy at eps={eps} "
                         f"(each against all {n} points), {tc:.1f} s, incl. their CSR rows and edges"}
        log(f"cpu oracle: {cpu['value']:.3f} G pair-dists/s on {cpu['cores']} threads ({cpu['sample']})")

    line = {
        "metric": METRIC, "value": value, "unit": "G pair-dists/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if used_path != "f16" else "f16",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "storage": str(x.dtype), "eps": eps_list,
                   "path": used_path, "block": block, "order": "index"},
        "graph_ms": graph_ms,
        "ms_per_step_profiled": prof_ms,
        "landmarks": [s["n_landmarks"] for s in runs[0]], "edges": [s["n_edges"] for s in runs[0]],
        "fp32_path": fp32,
        "speedup_vs_fp32": (value / fp32["value"]) if fp32 else None,
        "bit_exact": exact,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if args.copy_probe:
        copy_probe()


if __name__ == "__main__":
    main()
