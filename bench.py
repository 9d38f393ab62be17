"""Benchmark: PI-RRT# Replan on the 6D 1,000,000-vertex random geometric graph.

One step = one full Replan (Alg. 2: Evaluate, then promising set, Improve domain,
Improve and Evaluate to the fixed point) of the 1M-vertex graph from its
insertion-time policy, on one MI355X.  Each step first restores that policy from
the device-side snapshot (a 12 MB device copy, inside the timed region).  The
graph, the heuristic and the outputs stay in device memory throughout.

Prints one JSON line.  `value` is Replan GTEPS = edges examined by Improve / wall
time of the timed steps.  `roofline` is the Improve kernel against HBM bandwidth,
timed with HIP events on the library's stream; `cpu_baseline` is the serial
oracle on this host's cores for one Replan of the same graph.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
IMPROVE_SRC = os.path.join(ROOT, "paper_2003_04920_amd", "csrc", "improve.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_improve_6d_1m_traffic.txt")
CALIB_BYTES = 1 << 30  # the calibration kernel reads 1 GiB and writes 1 GiB


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def improve_bytes(edges: int, sum_d: int, n: int, launches: int) -> int:
    """Algorithmic HBM bytes of the Improve launches: 8 B per examined edge (int32
    neighbour + binary32 cost, streamed) and 24 B per domain vertex (its entry of
    the compacted domain list, two row offsets, its g and the parent / pcost
    update).  The g values the edges gather (4 MB at 1M vertices) are L2 / MALL
    resident and not counted; `traffic` shows what the gathers cost in HBM bytes.
    n and launches are kept for the signature: Improve no longer touches every
    slot in a launch."""
    del n, launches
    return 8 * edges + 24 * sum_d


def source_digest() -> str:
    with open(IMPROVE_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per k_improve launch from the committed counter summary, or None
    when the summary is missing or was taken on another version of the kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("improve_hip_sha256_16") != source_digest():
        return None
    try:
        return int(vals["k_improve_traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _short(name: str) -> str:
    name = name.replace("pirrt::(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0]


def profile_summary(paths):
    """Summarises rocprofv3 CSV output: kernel statistics (--kernel-trace --stats)
    and per-dispatch counters (--pmc FETCH_SIZE, --pmc WRITE_SIZE, in KiB).  The
    counters are scaled by what they read for the calibration kernel (a 1 GiB
    elementwise negation: 1 GiB read, 1 GiB written)."""
    out = []
    for path in paths:
        for f in sorted(glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True)):
            out.append("kernel statistics (%s):" % os.path.basename(f))
            out.append("  %-60s %7s %12s %12s %7s" % ("kernel", "calls", "total_us", "avg_us", "pct"))
            with open(f) as fh:
                for row in list(csv.DictReader(fh))[:16]:
                    out.append("  %-60s %7s %12.1f %12.2f %7.2f" % (
                        _short(row["Name"])[:60], row["Calls"], float(row["TotalDurationNs"]) / 1e3,
                        float(row["AverageNs"]) / 1e3, float(row["Percentage"])))
    per = {}
    for path in paths:
        for f in sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    key = (_short(row["Kernel_Name"]), row["Counter_Name"])
                    per.setdefault(key, []).append(float(row["Counter_Value"]))
    if per:
        out.append("counters, mean KiB per dispatch:")
        for (k, c), v in sorted(per.items()):
            out.append("  %-60s %-11s dispatches %5d mean %14.1f" % (k[:60] or "(unnamed)", c, len(v),
                                                                      sum(v) / len(v)))
        def mean(pred, counter):
            v = [x for (k, c), xs in per.items() if c == counter and pred(k) for x in xs]
            return sum(v) / len(v) if v else None
        calib = lambda k: "native::neg" in k
        imp = lambda k: k.startswith("k_improve")
        cf, cw = mean(calib, "FETCH_SIZE"), mean(calib, "WRITE_SIZE")
        f_imp, w_imp = mean(imp, "FETCH_SIZE"), mean(imp, "WRITE_SIZE")
        if cf and cw and f_imp is not None and w_imp is not None:
            sf, sw = CALIB_BYTES / (cf * 1024), CALIB_BYTES / (cw * 1024)
            traffic = int(round(f_imp * 1024 * sf + w_imp * 1024 * sw))
            out.append("calibration: FETCH_SIZE reads %.1f KiB and WRITE_SIZE %.1f KiB for 1 GiB each: "
                       "scale %.4f (fetch), %.4f (write)" % (cf, cw, sf, sw))
            out.append("k_improve_fetch_bytes_per_launch: %d" % int(round(f_imp * 1024 * sf)))
            out.append("k_improve_write_bytes_per_launch: %d" % int(round(w_imp * 1024 * sw)))
            out.append("k_improve_traffic_bytes_per_launch: %d" % traffic)
            out.append("improve_hip_sha256_16: %s" % source_digest())
    print("\n".join(out))


def bench_multi(args):
    """Batched multi-graph Replan: `args.problems` independent problems (d in
    {2,3,4,6,8}, n log-uniform in [5k, 200k], 10-40 sphere / box obstacles), each
    sampled and connected on the device, replanned together by one pirrt_batch
    call per step, beside the same problems replanned one pirrt_replan call at a
    time."""
    import numpy as np
    import torch

    import paper_2003_04920_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream().cuda_stream
    specs = [W.multi_problem_spec(i) for i in range(args.problems)]
    B = P.Batch(stream=stream)
    rrgs, hs = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for sp in specs:
        R = P.Rrg(sp.d, sp.obstacles, stream=stream, point_capacity=sp.n)
        R.add_points(np.stack([np.full(sp.d, 0.05), np.full(sp.d, 0.95)]))
        R.sample(sp.sample_seed, 0, 0, sp.n - 2)
        R.connect_problem(sp.radius, B)
        hs.append(R.heuristic(1, out=torch.empty(sp.n, dtype=torch.float32, device=dev)))
        rrgs.append(R)
        if len(rrgs) % 64 == 0:
            log("built %d problems (%.1fs)" % (len(rrgs), time.perf_counter() - t0))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    n, nnz = B.n, B.nnz
    log("batch: %d problems, %d vertices, %d directed edges, built on the device in %.2fs" %
        (len(specs), n, nnz, build_s))
    h = torch.cat(hs)
    g_out = torch.empty(n, dtype=torch.float32, device=dev)
    p_out = torch.empty(n, dtype=torch.int32, device=dev)
    B.snapshot_save()
    roots = np.zeros(len(specs), np.int32)
    goals = np.ones(len(specs), np.int32)

    def batch_step():
        B.snapshot_restore()
        return B.replan(roots, goals, h, True, g_out=g_out, parent_out=p_out)[2]

    for _ in range(args.warmup):
        st = batch_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = batch_step()
    torch.cuda.synchronize()
    ms_batch = 1e3 * (time.perf_counter() - t0) / max(1, args.steps)
    edges = sum(x["edges_examined"] for x in st)
    iters = [x["iterations"] for x in st]
    log("batched: %.3f ms per Replan of all problems, %.1f GTEPS, iterations max %d mean %.1f" %
        (ms_batch, edges / ms_batch / 1e6, max(iters), sum(iters) / len(iters)))
    # the same problems, one graph handle and one pirrt_replan call each
    graphs = []
    off = B.offsets
    for i, (R, sp) in enumerate(zip(rrgs, specs)):
        G = P.Graph(stream=stream)
        R.connect(0, sp.radius, G)
        G.snapshot_save()
        graphs.append((G, h[off[i]:off[i + 1]], g_out[off[i]:off[i + 1]], p_out[off[i]:off[i + 1]]))

    def seq_step():
        tot = 0
        for G, hh, gg, pp in graphs:
            G.snapshot_restore()
            tot += G.replan(0, 1, hh, True, g_out=gg, parent_out=pp)[2]["edges_examined"]
        return tot

    for _ in range(max(1, args.warmup // 2)):
        seq_edges = seq_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = max(1, args.steps // 2)
    for _ in range(reps):
        seq_edges = seq_step()
    torch.cuda.synchronize()
    ms_seq = 1e3 * (time.perf_counter() - t0) / reps
    assert seq_edges == edges, (seq_edges, edges)
    log("sequential: %.3f ms for %d pirrt_replan calls" % (ms_seq, len(graphs)))
    out = {
        "metric": "Batched multi-graph Replan GTEPS (%d problems, one pirrt_batch_replan per step)" % len(specs),
        "value": round(edges / ms_batch / 1e6, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_batch, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%d independent RRG problems, d in {2,3,4,6,8}, n log-uniform in [5k, 200k], "
                               "10-40 sphere/box obstacles, r = (ln n/n)^(1/d); sampled and connected on the "
                               "device; pruning on, h = Euclidean distance to goal" % len(specs),
                   "problems": len(specs), "vertices": n, "directed_edges": nnz,
                   "edges_examined_per_step": edges, "iterations_max": max(iters),
                   "parallelism": "single GPU"},
        "sequential_ms": round(ms_seq, 3), "speedup_vs_sequential": round(ms_seq / ms_batch, 2),
        "sequential_gteps": round(edges / ms_seq / 1e6, 3),
        "device_build_s": round(build_s, 3),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--samples", type=int, default=1_000_000)
    ap.add_argument("--extra", type=int, default=10_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB elementwise copy (reference for HBM byte counters)")
    ap.add_argument("--profile-summary", nargs="+", metavar="DIR",
                    help="summarise rocprofv3 CSV output under DIR(s) and exit")
    ap.add_argument("--workload", choices=["plain6d", "multi"], default="plain6d",
                    help="plain6d: the 6D 1M-vertex Replan (default); multi: batched multi-graph Replan")
    ap.add_argument("--problems", type=int, default=512, help="problems of the multi workload")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(args.profile_summary)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the Replan library runs on a single device and "
              "this build has no multi-GPU path (--gpus %d requested)" % args.gpus)
        sys.exit(2)
    if args.workload == "multi":
        bench_multi(args)
        return

    import numpy as np
    import torch

    import paper_2003_04920_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    t0 = time.time()
    wl = W.plain_6d(samples=args.samples, extra=0 if args.no_extra else args.extra, seed=200)
    log("workload %s: n=%d, batches=%d, directed edges=%d (%.1fs)" %
        (wl.name, wl.n, len(wl.batches), 2 * wl.nnz, time.time() - t0))
    b0 = wl.batches[0]
    G = P.Graph(stream=stream.cuda_stream, device=0)
    t0 = time.time()
    G.insert_rows(b0)
    torch.cuda.synchronize()
    insert_s = time.time() - t0
    n = G.n
    log("inserted %d vertices, %d directed entries in %.3fs" % (n, G.nnz, insert_s))
    G.snapshot_save()
    h = torch.from_numpy(wl.heuristic(n)).to(dev)
    g_out = torch.empty(n, dtype=torch.float32, device=dev)
    p_out = torch.empty(n, dtype=torch.int32, device=dev)

    def step(timing=False):
        G.snapshot_restore()
        _, _, st = G.replan(0, 1, h, True, timing=timing, g_out=g_out, parent_out=p_out)
        return st

    for i in range(args.warmup):
        st = step()
        log("warmup %d: %.3f ms, iterations %d, edges %d" % (i, st["ms_total"], st["iterations"],
                                                             st["edges_examined"]))
    # phase breakdown (HIP events around every launch; separate from the timed steps)
    tst = step(timing=True)
    log("timing pass: %s" % json.dumps({k: tst[k] for k in ("ms_total", "ms_evaluate", "ms_mark", "ms_improve",
                                                              "improve_launches", "evaluate_calls")}))

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / max(1, args.steps)
    edges = sum(s["edges_examined"] for s in stats)
    gteps = edges / elapsed / 1e9
    st = stats[-1]
    for s in stats:
        assert s["edges_examined"] == st["edges_examined"] and s["iterations"] == st["iterations"]
    log("timed: %d steps, %.3f ms/step, %.1f GTEPS" % (args.steps, ms_per_step, gteps))

    nbytes = improve_bytes(tst["edges_examined"], tst["sum_D"], n, tst["improve_launches"])
    achieved = nbytes / (tst["ms_improve"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                "kernel": "k_improve", "launches": tst["improve_launches"],
                "avg_launch_us": round(1e3 * tst["ms_improve"] / max(1, tst["improve_launches"]), 2),
                "bytes_per_launch": int(nbytes / max(1, tst["improve_launches"]))}

    extra = None
    if not args.no_extra and len(wl.batches) > 1:
        # a further 10,000-vertex batch on the converged 1M-vertex policy
        G.snapshot_restore()
        G.replan(0, 1, h, True, g_out=g_out, parent_out=p_out)
        b1 = wl.batches[1]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.insert_rows(b1)
        torch.cuda.synchronize()
        t_ins = time.perf_counter() - t0
        h2 = torch.from_numpy(wl.heuristic(G.n)).to(dev)
        g2 = torch.empty(G.n, dtype=torch.float32, device=dev)
        p2 = torch.empty(G.n, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, s2 = G.replan(0, 1, h2, True, g_out=g2, parent_out=p2)
        torch.cuda.synchronize()
        t_rep = time.perf_counter() - t0
        extra = {"batch": b1.n_new, "insert_ms": round(1e3 * t_ins, 3), "replan_ms": round(1e3 * t_rep, 3),
                 "iterations": s2["iterations"], "edges_examined": s2["edges_examined"],
                 "gteps": round(s2["edges_examined"] / t_rep / 1e9, 2)}
        log("+%d batch: %s" % (b1.n_new, json.dumps(extra)))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        R = oracle.Graph()
        assert R.insert_batch(b0) == 0
        hh = wl.heuristic(n)
        t0 = time.perf_counter()
        rc, so = R.replan(0, 1, hh, True)
        t_cpu = time.perf_counter() - t0
        assert rc == 0 and so["edges_examined"] == st["edges_examined"], (so, st)
        cpu = {"value": round(so["edges_examined"] / t_cpu / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": "one full Replan of the same 1M-vertex graph from its insertion-time policy "
                         "(serial C oracle, one thread, %.2f s)" % t_cpu}
        log("cpu baseline: %s" % json.dumps(cpu))

    if args.copy_calibration:
        x = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        torch.neg(x, out=y)  # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")

    out = {
        "metric": "Replan GTEPS + ms/replan (6D 1M-vertex RRG), HBM % peak; plain vs learned",
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "6D unit-cube RRG, 40 sphere obstacles, %d vertices, r=(ln n/n)^(1/6), "
                               "%d directed FP32-cost edges; one full Replan from the insertion-time "
                               "policy, pruning on, h = Euclidean distance to goal" % (n, 2 * b0.nnz),
                   "vertices": n, "directed_edges": 2 * b0.nnz, "iterations": st["iterations"],
                   "edges_examined_per_replan": st["edges_examined"], "sum_D": st["sum_D"],
                   "parallelism": "single GPU"},
        "phases_ms": {k: round(tst[k], 4) for k in ("ms_evaluate", "ms_mark", "ms_improve")},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra_batch": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
