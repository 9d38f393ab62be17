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

Other records (`--workload`): multi (512 problems batched against one call each),
learned (the learned sampling proposal: training, inference, planner comparison),
sweep (Batched-Extension planning time against batch size, 2D), async (exploration
concurrent with exploitation), breakeven (Replan time against graph size, library
and oracle), berrt6d (100 batches of 1,000 in 6D, Replan after each).
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

BF16_PEAK_TFLOPS = 2500.0  # dense bf16 matrix-core peak of the MI355X
FP64_PEAK_TFLOPS = 78.6  # binary64 vector peak of the MI355X (fused multiply-adds counted as two)
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
IMPROVE_SRC = os.path.join(ROOT, "paper_2003_04920_amd", "csrc", "improve.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_improve_6d_1m_traffic.txt")
MULTI_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_improve_multi512_traffic.txt")
BATCH_BLOCKS = (2048, 1024, 4096, 8192)  # batch grid sizes, in the autotuner's order
CALIB_BYTES = 1 << 30  # the calibration kernel reads 1 GiB and writes 1 GiB


CPU_REPS = 3  # oracle Replans timed for cpu_baseline (median)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info() -> dict:
    """The host CPU model string and the number of CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        nproc = os.cpu_count() or 0
    return {"cpu": model, "nproc": nproc}


def host_fields() -> dict:
    h = host_info()
    return {"host_cpu": h["cpu"], "host_nproc": h["nproc"]}


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


def replan_bytes(st: dict, n: int) -> dict:
    """Algorithmic HBM bytes of one whole Replan, by phase, from its counters:
    - Evaluate walk: 28 B per vertex and call (stamp word read 8, parent and cost 8,
      stamp word and g written 12);
    - promising list: 8 B per vertex and iteration (g, h) + 5 B per promising vertex
      (its list entry and stamp);
    - mark: 20 B per promising vertex (list entry, two row offsets) + 5 B per entry of
      a promising row (neighbour read 4, stamp written 1);
    - domain list: 1 B per vertex and iteration (stamps) + 4 B per domain vertex;
    - Improve: 8 B per examined edge + 24 B per domain vertex.
    The g gathers of Improve (L2 / MALL resident) are not counted."""
    it, calls = st["iterations"], st["iterations"]  # one Evaluate before each Improve
    parts = {"evaluate": 28 * n * calls,
             "promising_list": 8 * n * it + 5 * st["sum_P"],
             "mark": 20 * st["sum_P"] + 5 * st["mark_edges"],
             "domain_list": 1 * n * it + 4 * st["sum_D"],
             "improve": 8 * st["edges_examined"] + 24 * st["sum_D"]}
    parts["total"] = sum(parts.values())
    return parts


def source_digest() -> str:
    """Digest of the Improve kernel's sources (its file and the shared row-pass header)."""
    h = hashlib.sha256()
    for path in (IMPROVE_SRC, os.path.join(os.path.dirname(IMPROVE_SRC), "rowpass.h")):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per k_improve launch from the committed counter summary, or None
    when the summary is missing or was taken on another version of the kernel."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("improve_src_sha256_16") != source_digest():
        return None
    try:
        return int(vals["k_improve_traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _short(name: str) -> str:
    name = name.replace("pirrt::", "").replace("(anonymous namespace)::", "").replace("void ", "")
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
        # the Replan loop's kernels and the calibration kernel (the other kernels of the
        # run, graph building and exploration, are left out)
        shown = lambda k: k.split("<")[0] in LOOP_KERNELS or k.startswith("k_mark") or "native::neg" in k
        out.append("counters, mean KiB per dispatch (Replan loop kernels and the calibration kernel):")
        for (k, c), v in sorted(per.items()):
            if shown(k):
                out.append("  %-60s %-11s dispatches %5d mean %14.1f" % (k[:60], c, len(v), sum(v) / len(v)))
        def mean(pred, counter):
            v = [x for (k, c), xs in per.items() if c == counter and pred(k) for x in xs]
            return sum(v) / len(v) if v else None
        calib = lambda k: "native::neg" in k
        # the Improve variant the run used most (the autotuner also runs the others once)
        imp_names = {}
        for (k, c), v in per.items():
            if k.startswith("k_improve") and c == "FETCH_SIZE":
                imp_names[k] = len(v)
        imp_main = max(imp_names, key=imp_names.get) if imp_names else None
        imp = lambda k: k == imp_main
        cf, cw = mean(calib, "FETCH_SIZE"), mean(calib, "WRITE_SIZE")
        f_imp, w_imp = mean(imp, "FETCH_SIZE"), mean(imp, "WRITE_SIZE")
        if cf and cw and f_imp is not None and w_imp is not None:
            sf, sw = CALIB_BYTES / (cf * 1024), CALIB_BYTES / (cw * 1024)
            traffic = int(round(f_imp * 1024 * sf + w_imp * 1024 * sw))
            out.append("calibration: FETCH_SIZE reads %.1f KiB and WRITE_SIZE %.1f KiB for 1 GiB each: "
                       "scale %.4f (fetch), %.4f (write)" % (cf, cw, sf, sw))
            out.append("k_improve_kernel: %s" % imp_main)
            out.append("k_improve_fetch_bytes_per_launch: %d" % int(round(f_imp * 1024 * sf)))
            out.append("k_improve_write_bytes_per_launch: %d" % int(round(w_imp * 1024 * sw)))
            out.append("k_improve_traffic_bytes_per_launch: %d" % traffic)
            out.append("improve_src_sha256_16: %s" % source_digest())
    for path in paths:
        for f in sorted(glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True)):
            out.extend(loop_windows(f))
    print("\n".join(out))


LOOP_KERNELS = ("k_promising_list", "k_mark", "k_domain_list", "k_improve", "k_finish", "k_eval_walk",
                "k_after_eval")


def copy_ceiling(nbytes=1 << 30, reps=5):
    """Measured copy bandwidth of the GPU: a device-to-device copy of 1 GiB (1 GiB read
    and 1 GiB written per copy), timed with events after two warm-ups; the practical
    HBM ceiling next to the 8 TB/s peak."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    for _ in range(2):
        y.copy_(x)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    gbs = 2 * nbytes / (ms * 1e-3) / 1e9
    return {"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "note": "device-to-device copy of 1 GiB (read + write), mean of %d after 2 warm-ups" % reps}


def loop_windows(path, min_kernels=30):
    """Replan loops in a kernel trace: maximal runs of loop kernels (any other
    dispatch, such as a copy, ends a run).  For the last run: its span from the first
    start to the last end, the time some kernel was running (the union of the
    dispatch intervals) and the rest, the gaps a single persistent launch could
    remove, with the time per kernel."""
    with open(path) as fh:
        ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"]))
                    for r in csv.DictReader(fh))
    runs, cur = [], []
    for e in ev:
        if e[2].split("<")[0] in LOOP_KERNELS or e[2].startswith("k_mark"):
            cur.append(e)
            continue
        if len(cur) >= min_kernels:
            runs.append(cur)
        cur = []
    if len(cur) >= min_kernels:
        runs.append(cur)
    if not runs:
        return []
    w = runs[-1]
    span = w[-1][1] - w[0][0]
    busy, last = 0, 0
    for s0, e0, _ in w:
        lo = max(s0, last)
        if e0 > lo:
            busy += e0 - lo
        last = max(last, e0)
    per = {}
    for s0, e0, k in w:
        t = per.setdefault(k, [0, 0])
        t[0] += 1
        t[1] += e0 - s0
    out = ["Replan loop (%s, last of %d runs): %d dispatches, span %.3f ms, kernels running %.3f ms, "
           "gaps %.3f ms (%.2f%%)" % (os.path.basename(path), len(runs), len(w), span / 1e6, busy / 1e6,
                                      (span - busy) / 1e6, 100.0 * (span - busy) / max(1, span))]
    for k, (c, t) in sorted(per.items(), key=lambda x: -x[1][1]):
        out.append("  %-60s %6d dispatches %10.3f ms %9.2f us avg" % (k[:60], c, t / 1e6, t / 1e3 / c))
    return out


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
    if args.config >= 0:  # a fixed kernel configuration instead of the autotuner's choice
        os.environ["PIRRT_ROW_VARIANT"] = str(args.config % 4)
        os.environ["PIRRT_WALK_COHERENT"] = "0" if (args.config // 4) % 2 else "1"
        os.environ["PIRRT_BATCH_BLOCKS"] = str(BATCH_BLOCKS[args.config // 8])
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
    t0 = time.perf_counter()
    tuned = B.tune(roots, goals, h, True) if args.config < 0 else args.config
    log("autotuner: configuration %d (row split %d, %s-scope Evaluate stamps, %d workgroups per launch), %.2f s" %
        (tuned, tuned % 4, "workgroup" if (tuned // 4) % 2 else "device", BATCH_BLOCKS[tuned // 8],
         time.perf_counter() - t0))

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
    # phase timing (HIP events around every launch) for the Improve roofline
    B.snapshot_restore()
    tst = B.replan(roots, goals, h, True, timing=True, g_out=g_out, parent_out=p_out)[2]
    t0s = tst[0]
    sum_d = sum(x["sum_D"] for x in tst)
    nbytes = improve_bytes(edges, sum_d, n, t0s["improve_launches"])
    achieved = nbytes / (t0s["ms_improve"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(MULTI_TRAFFIC_FILE),
                "kernel": "k_improve (batched)",
                "launches": t0s["improve_launches"],
                "avg_launch_us": round(1e3 * t0s["ms_improve"] / max(1, t0s["improve_launches"]), 2),
                "bytes_per_launch": int(nbytes / max(1, t0s["improve_launches"]))}
    log("timing pass: improve %.3f ms over %d launches, %.1f GB/s algorithmic" %
        (t0s["ms_improve"], t0s["improve_launches"], achieved))
    if args.copy_calibration:
        x = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        torch.neg(x, out=y)  # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        del x, y
        log("copy calibration: 1 GiB read + 1 GiB written")
    # the same problems, one graph handle and one pirrt_replan call each
    graphs = []
    off = B.offsets
    ms_seq = None
    for i, (R, sp) in enumerate(zip(rrgs, specs) if not args.no_sequential else []):
        G = P.Graph(stream=stream)
        R.connect(0, sp.radius, G)
        G.snapshot_save()
        if args.tune_each:
            G.tune(0, 1, h[off[i]:off[i + 1]], True)
        graphs.append((G, h[off[i]:off[i + 1]], g_out[off[i]:off[i + 1]], p_out[off[i]:off[i + 1]]))

    def seq_step():
        tot = 0
        for G, hh, gg, pp in graphs:
            G.snapshot_restore()
            tot += G.replan(0, 1, hh, True, g_out=gg, parent_out=pp)[2]["edges_examined"]
        return tot

    if not args.no_sequential:
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
    cpu = None
    if not args.no_cpu_baseline:
        # the serial oracle on the first problems, up to about 15 s of host time
        import oracle
        spent = cpu_edges = 0
        used = 0
        for i, (R, sp) in enumerate(zip(rrgs, specs)):
            rp_, col_, cost_ = R.rows(0, sp.radius)
            O = oracle.Graph()
            assert O.insert(rp_, col_, cost_) == 0
            hh = h[off[i]:off[i + 1]].cpu().numpy()
            t0 = time.perf_counter()
            rc, so = O.replan(0, 1, hh, True)
            spent += time.perf_counter() - t0
            assert rc == 0 and so["edges_examined"] == st[i]["edges_examined"], (i, so, st[i])
            cpu_edges += so["edges_examined"]
            used += 1
            if spent > 15.0:
                break
        cpu = {"value": round(cpu_edges / spent / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": "one full Replan of each of the first %d problems (%d examined edges, serial C oracle, "
                         "one thread, %.2f s)" % (used, cpu_edges, spent)}
        cpu.update(host_fields())
        log("cpu baseline: %s" % json.dumps(cpu))
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
        "roofline": roofline,
        "cpu_baseline": cpu,
        "sequential_ms": round(ms_seq, 3) if ms_seq else None,
        "speedup_vs_sequential": round(ms_seq / ms_batch, 2) if ms_seq else None,
        "sequential_gteps": round(edges / ms_seq / 1e6, 3) if ms_seq else None,
        "device_build_s": round(build_s, 3),
        "autotuned_config": tuned,
    }
    print(json.dumps(out), flush=True)


def bench_learned(args):
    """Learned sampling proposal on the 6D generator (40 spheres): training data from
    converged Replans on `args.layouts` layouts at 200k vertices (label: a path
    through the vertex within 5% of the best, from a root-rooted and a goal-rooted
    Replan without pruning), the network trained on the device, then the planner
    grown to `args.plan_n` vertices in batches of `args.batch` on held-out layouts,
    uniform sampling against half learned / half uniform sampling, with Replan
    after every batch."""
    import numpy as np
    import torch

    import paper_2003_04920_amd as P
    import workloads as W
    from paper_2003_04920_amd import learned as L
    from paper_2003_04920_amd import planner as PL

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream().cuda_stream
    d, n_train = 6, 200_000
    root_goal = PL.root_goal(d)

    # ---- exploration support on its own: one 200k-vertex 6D graph, the radius search
    # (two passes over every pair u < v, binary64 squared distance: 3d - 1 = 17 flops
    # a pair, no fused multiply-add) and the segment tests
    obs0 = W.make_obstacles(d, 40, "sphere", 19_990)
    R0 = P.Rrg(d, obs0, stream=stream, point_capacity=n_train)
    R0.add_points(root_goal)
    R0.sample(19_991, 0, 0, n_train - 2)
    G0 = P.Graph(stream=stream, vertex_capacity=n_train)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R0.connect(0, W.radius(n_train, d), G0)
    torch.cuda.synchronize()
    connect_s = time.perf_counter() - t0
    pair_tests = 2 * n_train * (n_train - 1) // 2
    tf = pair_tests * (3 * d - 1) / connect_s / 1e12
    explore = {"points": n_train, "d": d, "connect_ms": round(1e3 * connect_s, 2), "directed_edges": G0.nnz,
               "pair_tests": pair_tests, "fp64_tflops": round(tf, 2), "fp64_peak_tflops": FP64_PEAK_TFLOPS,
               "frac": round(tf / FP64_PEAK_TFLOPS, 4)}
    log("exploration: %s" % json.dumps(explore))
    del R0, G0

    # ---- training data and training on the device (paper_2003_04920_amd.learned)
    def scene(seed):
        return W.make_obstacles(d, 40, "sphere", seed)

    net, trec = L.build_and_train(d, scene, [20_000 + 10 * i for i in range(args.layouts)], n_train, args.per_layout,
                                  args.epochs, stream=stream, log=log)
    data_s, train_s, steps, bs = trec["data_seconds"], trec["train_seconds"], trec["steps"], trec["batch"]
    log("training data: %d layouts, %d samples (%.1f%% positive), %.1f s" %
        (args.layouts, trec["samples"], 100.0 * trec["positive_share"], data_s))
    # held-out accuracy on fresh layouts (features and labels as in training)
    rng = np.random.default_rng(8)
    xv, yv = zip(*[L.layout_samples(d, scene(25_000 + 10 * i), 25_001 + 10 * i, n_train, args.per_layout, rng,
                                    stream=stream) for i in range(max(1, args.layouts // 10))])
    Xv = torch.from_numpy(np.ascontiguousarray(np.concatenate(xv), np.float32)).to(dev)
    Yv = torch.from_numpy(np.concatenate(yv)).to(dev)
    in_dim = Xv.shape[1]
    nval = len(Yv)
    zv = torch.cat([net.forward(Xv[i:i + 8192].contiguous()) for i in range(0, nval, 8192)])
    pred = zv > 0
    acc = float((pred == (Yv > 0)).float().mean())
    recall = float((pred & (Yv > 0)).float().sum() / (Yv > 0).float().sum().clamp(min=1))
    precision = float((pred & (Yv > 0)).float().sum() / pred.float().sum().clamp(min=1))
    log("training: %d steps of %d in %.2f s (%.0f samples/s); loss %.4f -> %.4f; held-out accuracy %.3f, "
        "recall %.3f, precision %.3f" % (steps, bs, train_s, steps * bs / max(train_s, 1e-9),
                                         trec["loss_first"], trec["loss_last"], acc, recall, precision))
    Xt, Yt = Xv, Yv  # resident batches for the timing probes below
    init = L.init_params(in_dim, 11)
    xb = Xt[:8192].contiguous()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(20):
        net.forward(xb)
    torch.cuda.synchronize()
    infer_us = 1e6 * (time.perf_counter() - t1) / 20

    # the network's training step against the bf16 matrix-core peak (multiply-adds per
    # sample: forward 288x256 + 256x256 + 256, backward the two weight gradients, the
    # hidden-layer input gradient and the output layer)
    macs = (288 * 256 + 256 * 256 + 256) + (288 * 256 + 2 * 256 * 256 + 2 * 256)
    # steps on one resident batch (the training loop above also gathers its batches)
    xr, yr = Xt[:bs].contiguous(), Yt[:bs].contiguous()
    probe = P.Mlp(in_dim, bs, lr=1e-3, stream=stream)
    probe.set_params(init)
    for _ in range(5):
        probe.train_step(xr, yr)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(100):
        probe.train_step(xr, yr)
    torch.cuda.synchronize()
    step_us = 1e6 * (time.perf_counter() - t1) / 100
    tflops = 2.0 * macs * bs / (step_us * 1e-6) / 1e12
    roofline = {"bound": "mfma", "achieved": round(tflops, 3), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tflops / BF16_PEAK_TFLOPS, 6), "traffic": None,
                "kernel": "network training step (bf16 MFMA GEMMs + epilogues, batch %d)" % bs,
                "avg_step_us": round(step_us, 1),
                "note": "one train_step call (features, 2 forward GEMMs, loss, backward GEMMs and column sums, "
                        "Adam, bf16 weight refresh, loss read back) on a resident batch"}
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's training step (numpy, one BLAS thread) on the same batch size
        from threadpoolctl import threadpool_limits
        from oracle import mlp as M
        xh = Xt[:bs].cpu().numpy()
        yh = Yt[:bs].cpu().numpy()
        prm = M.init_params(np.random.default_rng(11), in_dim)
        opt = M.Adam(lr=1e-3)
        reps = 0
        with threadpool_limits(limits=1):
            t2 = time.perf_counter()
            while time.perf_counter() - t2 < 10.0:
                _, grads, _ = M.loss_and_grads(prm, xh, yh)
                prm = opt.step(prm, grads)
                reps += 1
            cpu_s = time.perf_counter() - t2
        cpu = {"value": round(reps * bs / cpu_s, 1), "unit": "training samples/s", "cores": 1, "kind": "oracle",
               "sample": "%d training steps of %d samples with the numpy oracle (forward, backward, Adam; "
                         "one BLAS thread, %.1f s)" % (reps, bs, cpu_s)}
        cpu.update(host_fields())
        log("cpu baseline: %s" % json.dumps(cpu))

    # ---- planner comparison on held-out layouts (paper_2003_04920_amd.planner)
    def plan(seed, learned):
        obs = scene(seed)
        pl = PL.Planner(d, obs, seed + 1, args.plan_n + args.batch + 2, stream=torch.cuda.current_stream(),
                        trigger=False, net=net if learned else None,
                        enc=L.sphere_encoding(obs) if learned else None)
        return [(r["seconds"], r["n"], r["cost"]) for r in pl.run(args.plan_n, args.batch)]

    rows = []
    for j in range(args.heldout):
        seed = 30_000 + 10 * j
        hp = plan(seed, False)
        hl = plan(seed, True)
        cost_p, t_p = hp[-1][2], hp[-1][0]
        reach = [t for t, _, c in hl if c <= 1.01 * cost_p]
        t_reach = reach[0] if reach else None
        rows.append({"layout": seed, "plain_cost": round(cost_p, 5), "plain_s": round(t_p, 3),
                     "learned_cost": round(hl[-1][2], 5), "learned_s": round(hl[-1][0], 3),
                     "learned_s_to_1pct_of_plain": None if t_reach is None else round(t_reach, 3),
                     "time_ratio": None if t_reach is None else round(t_reach / t_p, 3),
                     "plain_cost_at_10pct_time": round(min(c for t, _, c in hp if t <= 0.1 * t_p + 1e-9)
                                                       if any(t <= 0.1 * t_p for t, _, _ in hp) else hp[0][2], 5),
                     "learned_cost_at_10pct_time": round(min(c for t, _, c in hl if t <= 0.1 * t_p + 1e-9)
                                                         if any(t <= 0.1 * t_p for t, _, _ in hl) else hl[0][2], 5)})
        log("layout %d: %s" % (seed, json.dumps(rows[-1])))
    ratios = [r["time_ratio"] for r in rows if r["time_ratio"] is not None]
    out = {
        "metric": "Learned-proposal planner: wall time to within 1%% of the plain planner's %d-vertex path cost, "
                  "as a fraction of the plain planner's time" % args.plan_n,
        "value": round(float(np.median(ratios)), 4) if ratios else None, "unit": "fraction",
        "higher_is_better": False, "n_gpus": 1, "dtype": "bf16 network / f32 Replan", "data": "synthetic",
        "config": {"workload": "6D unit cube, 40 spheres; %d training layouts at %d vertices (%d samples each, "
                               "positive-balanced); planner to %d vertices in batches of %d, Replan after each; "
                               "learned = half of each batch the best of 8192 scored candidates" %
                               (args.layouts, n_train, args.per_layout, args.plan_n, args.batch)},
        "training": {"steps": steps, "batch": bs, "seconds": round(train_s, 3),
                     "samples_per_s": round(steps * bs / max(train_s, 1e-9)), "loss_first": round(trec["loss_first"], 4),
                     "loss_last": round(trec["loss_last"], 4), "heldout_accuracy": round(acc, 4),
                     "heldout_recall": round(recall, 4), "heldout_precision": round(precision, 4),
                     "data_seconds": round(data_s, 2)},
        "inference_us_per_8192": round(infer_us, 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "exploration": explore,
        "layouts": rows,
    }
    print(json.dumps(out), flush=True)


def bench_sweep(args):
    """Batched-Extension batch-size sweep (the paper's planning-time experiment, Sec.
    VI and Alg. 3) on the 2D scene of the small configuration (unit square, 8 boxes):
    for each total sample count N and batch size S, grow the RRG S free samples at a
    time (device sampler and radius search, r at the current n) and replan only when
    the batch added a promising vertex (|B'| > |B|: a new vertex whose insertion-time
    g + h is below g(goal)).  Planning time is the whole loop; exploitation runs on
    the GPU (the library) or, for the CPU columns, in the serial oracle on the host."""
    import numpy as np
    import torch

    import paper_2003_04920_amd as P
    import workloads as W
    from paper_2003_04920_amd import planner as PL

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream().cuda_stream
    d = 2
    root_goal = PL.root_goal(d)
    Ns = [int(x) for x in args.sweep_n.split(",")]
    Ss = [int(x) for x in args.sweep_s.split(",")]

    def plan(N, S, seed, cpu):
        obs = W.make_obstacles(d, 8, "box", seed)
        if not cpu:  # the package's BERRT# planner (replan test on the device)
            pl = PL.Planner(d, obs, seed + 1, N + 2, stream=torch.cuda.current_stream(), trigger=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hist = pl.run(N, S)
            torch.cuda.synchronize()
            return time.perf_counter() - t0, pl.replans, hist[-1]["cost"]
        R = P.Rrg(d, obs, stream=stream, point_capacity=N + 2)
        R.add_points(root_goal)
        import oracle
        O = oracle.Graph()
        rp_, col_, cost_ = R.rows(0, W.radius(2, d))
        assert O.insert(rp_, col_, cost_) == 0
        counter, n_old, replans = 0, 2, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while R.n - 2 < N:
            counter = R.sample(seed + 1, 0, counter, min(S, N - (R.n - 2)))
            n = R.n
            r = W.radius(n, d)
            h = R.heuristic(1, out=torch.empty(n, dtype=torch.float32, device=dev))
            rp_, col_, cost_ = R.rows(n_old, r)
            assert O.insert(rp_, col_, cost_) == 0
            g = O.state().g
            hh = h.cpu().numpy()
            if bool(((g[n_old:] + hh[n_old:]) < g[1]).any()):  # the same replan test on the oracle's state
                rc, _ = O.replan(0, 1, hh, True)
                assert rc == 0
                replans += 1
            n_old = n
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        return t, replans, float(O.state().g[1])

    rows = []
    for N in Ns:
        for S in Ss:
            for cpu in ([False, True] if not args.no_cpu_baseline else [False]):
                if cpu and N * 1.0 / S > args.sweep_cpu_batches:
                    continue  # bounded host time: the oracle leg skips the smallest batches
                ts, rs, cs = [], [], []
                for trial in range(args.sweep_trials):
                    t, rp_n, c = plan(N, S, 500 + 10 * trial, cpu)
                    ts.append(t)
                    rs.append(rp_n)
                    cs.append(c)
                row = {"N": N, "S": S, "exploitation": "cpu oracle" if cpu else "gpu",
                       "planning_s": round(float(np.mean(ts)), 4), "planning_s_std": round(float(np.std(ts)), 4),
                       "replans": round(float(np.mean(rs)), 1), "final_cost": round(float(np.mean(cs)), 5)}
                rows.append(row)
                log("sweep: %s" % json.dumps(row))
    gpu = {(r["N"], r["S"]): r["planning_s"] for r in rows if r["exploitation"] == "gpu"}
    cpu = {(r["N"], r["S"]): r["planning_s"] for r in rows if r["exploitation"] != "gpu"}
    speed = {}
    for N in Ns:
        if (N, 1) in gpu:
            speed["N=%d" % N] = {"S=%d" % S: round(gpu[(N, 1)] / gpu[(N, S)], 2) for S in Ss if (N, S) in gpu}
    out = {
        "metric": "Batched-Extension planning time vs batch size (2D, 8 boxes); speedup over S=1",
        "value": max((v for d_ in speed.values() for v in d_.values()), default=None), "unit": "x",
        "higher_is_better": True, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2D unit square, 8 boxes (sides U(0.05,0.2)), root (0.05,0.05), goal (0.95,0.95); "
                               "N free samples in batches of S, r = (ln n/n)^(1/2) at the current n, Replan when a "
                               "batch adds a promising vertex; %d trial(s) per cell" % args.sweep_trials,
                   "N": Ns, "S": Ss},
        "speedup_over_s1": speed,
        "gpu_over_cpu_exploitation": {"N=%d,S=%d" % k: round(cpu[k] / gpu[k], 2) for k in cpu if k in gpu},
        "cells": rows,
    }
    print(json.dumps(out), flush=True)


def bench_async(args):
    """Exploration concurrent with exploitation (the asynchronous scheme the paper
    proposes as future work, Sec. VII), on the Batched-Extension 6D scene (40 spheres,
    batches of 1,000, r at the current n): an explorer thread samples and builds the
    rows of each batch on its own stream and queues them; the exploiter inserts every
    queued batch and replans on another stream, so the radius searches of later batches
    overlap the Replan of earlier ones.  Against the same loop run in lockstep (sample,
    connect, Replan per batch).  The two build the same graph; the exploiter replans
    less often (once per drained queue)."""
    import torch

    import workloads as W
    from paper_2003_04920_amd import planner as PL

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d, N, S = 6, args.async_n, args.async_s
    obs = W.make_obstacles(d, 40, "sphere", 100)

    def lockstep():
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            pl = PL.Planner(d, obs, 101, N + 2, stream=st, trigger=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hist = pl.run(N, S)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, pl.replans, hist[-1]["cost"], pl.graph.n, pl.graph.nnz

    def concurrent():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G, R, replans, _ = PL.plan_concurrent(d, obs, 101, N, S)
        t = time.perf_counter() - t0
        return t, replans, float(G.get_policy()[0][1]), G.n, G.nnz

    lockstep()  # warm-up (kernel loading, allocations)
    t_l, r_l, c_l, n_l, m_l = lockstep()
    t_c, r_c, c_c, n_c, m_c = concurrent()
    assert (n_l, m_l) == (n_c, m_c), ((n_l, m_l), (n_c, m_c))
    out = {
        "metric": "Exploration concurrent with exploitation: planning time, lockstep / concurrent",
        "value": round(t_l / t_c, 3), "unit": "x", "higher_is_better": True, "n_gpus": 1, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "6D unit cube, 40 spheres; %d free samples in batches of %d, r = (ln n/n)^(1/6) at "
                               "the current n, h = Euclidean distance to goal; explorer and exploiter on two "
                               "streams of one GPU" % (N, S), "vertices": n_l, "directed_edges": m_l},
        "lockstep": {"seconds": round(t_l, 3), "replans": r_l, "final_cost": c_l},
        "concurrent": {"seconds": round(t_c, 3), "replans": r_c, "final_cost": c_c},
    }
    log("lockstep: %s" % json.dumps(out["lockstep"]))
    log("concurrent: %s" % json.dumps(out["concurrent"]))
    print(json.dumps(out), flush=True)


def bench_breakeven(args):
    """Replan time against graph size, GPU library and serial oracle side by side (the
    paper's exploitation-time comparison, Sec. VI): 2D scene of the small configuration
    (unit square, 8 boxes), n free samples in one batch, one full Replan from the
    insertion-time policy with pruning on.  The break-even size is where the library
    overtakes the oracle on one host thread."""
    import numpy as np
    import torch

    import oracle
    import paper_2003_04920_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream().cuda_stream
    def timed(n_host_max, b, hd, prune=True, reps=7, skip=2):
        """Median synchronous Replan time (ms) on a fresh handle created with
        PIRRT_HOST_MAX = n_host_max (0: the device loop; huge: the host Replan)."""
        if n_host_max is None:
            os.environ.pop("PIRRT_HOST_MAX", None)
        else:
            os.environ["PIRRT_HOST_MAX"] = str(n_host_max)
        G = P.Graph(stream=stream)
        os.environ.pop("PIRRT_HOST_MAX", None)
        G.insert_rows(b)
        G.snapshot_save()
        ts = []
        for i in range(reps):
            G.snapshot_restore()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, st = G.replan(0, 1, hd, prune)
            ts.append(time.perf_counter() - t0)
        return 1e3 * float(np.median(ts[skip:])), st

    rows = []
    for n in [int(x) for x in args.breakeven_n.split(",")]:
        wl = W.plain_2d(samples=n, seed=0)
        b = wl.batches[0]
        h = wl.heuristic(wl.n)
        hd = torch.from_numpy(h).to(dev)
        gpu_ms, st = timed(0, b, hd)
        host_ms, sh = timed(1 << 30, b, hd) if wl.n <= 100_000 else (None, None)
        auto_ms, sa = timed(None, b, hd)
        O = oracle.Graph()
        assert O.insert_batch(b) == 0
        t0 = time.perf_counter()
        rc, so = O.replan(0, 1, h, True)
        cpu_ms = 1e3 * (time.perf_counter() - t0)
        assert rc == 0 and so["edges_examined"] == st["edges_examined"] == sa["edges_examined"]
        row = {"n": wl.n, "directed_edges": 2 * b.nnz, "iterations": st["iterations"],
               "edges_examined": st["edges_examined"], "gpu_ms": round(gpu_ms, 3),
               "host_replan_ms": None if host_ms is None else round(host_ms, 3),
               "adaptive_ms": round(auto_ms, 3), "adaptive_on_host": bool(sa["on_host"]),
               "cpu_oracle_ms": round(cpu_ms, 3), "speedup": round(cpu_ms / gpu_ms, 2)}
        rows.append(row)
        log("breakeven: %s" % json.dumps(row))
    n0 = next((r["n"] for r in rows if r["speedup"] > 1.0), None)
    # the small configuration itself (2,000 free samples, 2,002 vertices): time per
    # Replan with pruning on and off, same protocol
    small = []
    wl = W.plain_2d()
    b = wl.batches[0]
    h = wl.heuristic(wl.n)
    hd = torch.from_numpy(h).to(dev)
    for prune in (True, False):
        G = P.Graph(stream=stream)
        G.insert_rows(b)
        G.snapshot_save()
        ts = []
        for i in range(25):
            G.snapshot_restore()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, st = G.replan(0, 1, hd, prune)
            ts.append(time.perf_counter() - t0)
        O = oracle.Graph()
        assert O.insert_batch(b) == 0
        t0 = time.perf_counter()
        rc, so = O.replan(0, 1, h, prune)
        cpu_us = 1e6 * (time.perf_counter() - t0)
        assert rc == 0 and so["edges_examined"] == st["edges_examined"]
        row = {"prune": prune, "n": wl.n, "iterations": st["iterations"], "edges_examined": st["edges_examined"],
               "gpu_us": round(1e6 * float(np.median(ts[5:])), 1), "cpu_oracle_us": round(cpu_us, 1)}
        small.append(row)
        log("small configuration: %s" % json.dumps(row))
    out = {
        "metric": "Replan time vs graph size, GPU library against the serial oracle (2D, 8 boxes); the library's "
                  "host Replan and its adaptive placement beside them",
        "value": n0, "unit": "vertices (break-even)", "higher_is_better": False, "n_gpus": 1, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D unit square, 8 boxes; n free samples in one batch, r = (ln n/n)^(1/2); one full "
                               "Replan from the insertion-time policy, pruning on, h = Euclidean distance to goal; "
                               "GPU: median of 5 after 2 warm-ups, synchronous call; oracle: one serial run"},
        "cpu_baseline": dict({"kind": "oracle", "cores": 1, "unit": "ms", "sample": "one Replan per size"},
                             **host_fields()),
        "sizes": rows,
        "small_config": small,
    }
    print(json.dumps(out), flush=True)


def bench_berrt6d(args):
    """The Batched-Extension 6D configuration: 100,000 vertices inserted in batches of
    1,000 (r at the current n, 40 spheres), a full Replan (pruning on, h = Euclidean
    distance to goal) after every batch.  Reports Replan time per batch and in total,
    iterations and edges examined, and the serial oracle on the first batches."""
    import numpy as np
    import torch

    import paper_2003_04920_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream().cuda_stream
    t0 = time.time()
    wl = W.batched_6d(batches=args.berrt_batches, batch=args.berrt_batch, seed=100)
    log("workload %s: n=%d, %d batches (%.1fs)" % (wl.name, wl.n, len(wl.batches), time.time() - t0))

    host_rows = [(b.row_ptr, b.col, b.cost) for b in wl.batches]
    dev_rows = [tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in r) for r in host_rows]

    def run(rows, capacity=False):
        # capacity: the graph is created with the workload's final vertex and edge counts
        G = (P.Graph(stream=stream, vertex_capacity=wl.n, edge_capacity=2 * sum(b.nnz for b in wl.batches))
             if capacity else P.Graph(stream=stream))
        per, ins = [], []
        edges = iters = 0
        for r in rows:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            G.insert_batch(*r)  # now and then also the renumbering; host rows include their copy
            torch.cuda.synchronize()
            ins.append(time.perf_counter() - t1)
            h = torch.from_numpy(wl.heuristic(G.n)).to(dev)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            g, _, st = G.replan(0, 1, h, True)
            per.append(time.perf_counter() - t1)
            edges += st["edges_examined"]
            iters += st["iterations"]
        return per, ins, edges, iters, float(g[1].item())

    run(host_rows)  # warm-up: kernel loading and allocations
    per, ins, edges, iters, cost = run(host_rows)
    per_d, ins_d, edges_d, _, cost_d = run(dev_rows, capacity=True)
    assert edges_d == edges and cost_d == cost, "device rows gave another Replan sequence"
    log("inserts: host rows %.2f ms (median %.3f, max %.3f); device rows into a graph created with its capacity "
        "%.2f ms (median %.3f, max %.3f); Replans %.2f ms and %.2f ms"
        % (1e3 * sum(ins), 1e3 * float(np.median(ins)), 1e3 * max(ins), 1e3 * sum(ins_d),
           1e3 * float(np.median(ins_d)), 1e3 * max(ins_d), 1e3 * sum(per), 1e3 * sum(per_d)))
    tot = sum(per)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        R = oracle.Graph()
        spent = cpu_edges = 0
        used = 0
        for b in wl.batches:
            assert R.insert_batch(b) == 0
            t1 = time.perf_counter()
            rc, so = R.replan(0, 1, wl.heuristic(R.n), True)
            spent += time.perf_counter() - t1
            assert rc == 0
            cpu_edges += so["edges_examined"]
            used += 1
            if spent > 15.0:
                break
        gpu_same = sum(per[:used])
        cpu = {"value": round(cpu_edges / spent / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": "the Replans after the first %d batches (serial C oracle, one thread, %.2f s; the library "
                         "took %.3f s for the same Replans)" % (used, spent, gpu_same)}
        cpu.update(host_fields())
        log("cpu baseline: %s" % json.dumps(cpu))
    out = {
        "metric": "Batched-Extension 6D: Replan after every batch, GTEPS over all Replans",
        "value": round(edges / tot / 1e9, 3), "unit": "GTEPS", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "6D unit cube, 40 spheres; %d batches of %d free samples, r = (ln n/n)^(1/6) at "
                               "the current n; full Replan after every batch, pruning on, h = Euclidean distance "
                               "to goal" % (len(wl.batches), args.berrt_batch), "vertices": wl.n},
        "replans": len(per), "replan_total_ms": round(1e3 * tot, 2), "replan_mean_ms": round(1e3 * tot / len(per), 3),
        "replan_last_ms": round(1e3 * per[-1], 3), "insert_total_ms": round(1e3 * sum(ins), 2),
        "insert_total_ms_device_rows_with_capacity": round(1e3 * sum(ins_d), 2),
        "replan_total_ms_device_rows_run": round(1e3 * sum(per_d), 2),
        "iterations_total": iters, "edges_examined": edges,
        "final_cost": cost, "cpu_baseline": cpu,
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
    ap.add_argument("--no-sequential", action="store_true",
                    help="multi: skip the one-call-per-problem comparison (for counter runs)")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB elementwise copy (reference for HBM byte counters)")
    ap.add_argument("--profile-summary", nargs="+", metavar="DIR",
                    help="summarise rocprofv3 CSV output under DIR(s) and exit")
    ap.add_argument("--workload", choices=["plain6d", "multi", "learned", "sweep", "async", "breakeven", "berrt6d"], default="plain6d",
                    help="plain6d: the 6D 1M-vertex Replan (default); multi: batched multi-graph Replan; "
                         "learned: learned proposal trained and compared with the uniform planner")
    ap.add_argument("--problems", type=int, default=512, help="problems of the multi workload")
    ap.add_argument("--tune-each", action="store_true", help="multi: autotune every sequential graph too")
    ap.add_argument("--sweep-n", default="10000,30000", help="sweep: total free samples per plan")
    ap.add_argument("--sweep-s", default="1,3,10,30,100,300,1000", help="sweep: batch sizes")
    ap.add_argument("--sweep-trials", type=int, default=2)
    ap.add_argument("--async-n", type=int, default=100_000, help="async: free samples")
    ap.add_argument("--berrt-batches", type=int, default=100, help="berrt6d: batches")
    ap.add_argument("--berrt-batch", type=int, default=1000, help="berrt6d: free samples per batch")
    ap.add_argument("--breakeven-n", default="30,100,200,300,1000,3000,10000,30000,100000,300000",
                    help="breakeven: free samples per graph")
    ap.add_argument("--async-s", type=int, default=1000, help="async: batch size")
    ap.add_argument("--sweep-cpu-batches", type=int, default=3000,
                    help="sweep: oracle exploitation only for cells with at most this many batches")
    ap.add_argument("--config", type=int, default=-1,
                    help="fixed kernel configuration instead of the autotuner: row split + 4 x workgroup-scope "
                         "stamps (0-7); multi adds 8 x the index of the batch grid size in (2048, 1024, 4096, 8192)")
    ap.add_argument("--layouts", type=int, default=100, help="learned: training layouts")
    ap.add_argument("--per-layout", type=int, default=8192, help="learned: samples kept per layout")
    ap.add_argument("--epochs", type=int, default=4, help="learned: training epochs")
    ap.add_argument("--heldout", type=int, default=3, help="learned: held-out layouts for the planner")
    ap.add_argument("--plan-n", type=int, default=1_000_000, help="learned: planner vertex count")
    ap.add_argument("--batch", type=int, default=1000, help="learned: samples per planner batch")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(args.profile_summary)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the Replan library runs on a single device and "
              "the library has no multi-GPU path (--gpus %d requested)" % args.gpus)
        sys.exit(2)
    if args.workload == "multi":
        bench_multi(args)
        return
    if args.workload == "sweep":
        bench_sweep(args)
        return
    if args.workload == "async":
        bench_async(args)
        return
    if args.workload == "breakeven":
        bench_breakeven(args)
        return
    if args.workload == "berrt6d":
        bench_berrt6d(args)
        return
    if args.workload == "learned":
        bench_learned(args)
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
    if args.config >= 0:  # a fixed kernel configuration instead of the autotuner's choice
        os.environ["PIRRT_ROW_VARIANT"] = str(args.config % 4)
        os.environ["PIRRT_WALK_COHERENT"] = "0" if args.config >= 4 else "1"
    # capacity declared up front for the whole workload (the 1M build and the +10k batch),
    # so the extra batch's insert is timed without growing the device arrays
    G = P.Graph(stream=stream.cuda_stream, device=0, vertex_capacity=wl.n,
                edge_capacity=2 * sum(b.nnz for b in wl.batches))
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

    # the library's autotuner picks the kernel configuration (outside the timed region),
    # unless --config fixed it when the graph was created
    tuned = G.tune(0, 1, h, True) if args.config < 0 else args.config
    log("autotuner: configuration %d (row split %d, %s-scope Evaluate stamps)" %
        (tuned, tuned % 4, "workgroup" if tuned >= 4 else "device"))

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
    stats, marks = [], [t0]
    for _ in range(args.steps):  # each call returns once its outputs are valid
        stats.append(step())
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / max(1, args.steps)
    step_ms = [1e3 * (b - a) for a, b in zip(marks, marks[1:])]
    edges = sum(s["edges_examined"] for s in stats)
    gteps = edges / elapsed / 1e9
    st = stats[-1]
    for s in stats:
        assert s["edges_examined"] == st["edges_examined"] and s["iterations"] == st["iterations"]
    log("timed: %d steps, %.3f ms/step, %.1f GTEPS" % (args.steps, ms_per_step, gteps))
    # the policy the last timed step produced (the captured-graph path), kept for the
    # bit-exact comparison with the oracle below
    g_timed = g_out.cpu().numpy().copy()
    p_timed = p_out.cpu().numpy().copy()

    nbytes = improve_bytes(tst["edges_examined"], tst["sum_D"], n, tst["improve_launches"])
    achieved = nbytes / (tst["ms_improve"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                "kernel": "k_improve", "launches": tst["improve_launches"],
                "avg_launch_us": round(1e3 * tst["ms_improve"] / max(1, tst["improve_launches"]), 2),
                "bytes_per_launch": int(nbytes / max(1, tst["improve_launches"]))}
    # the 4-byte g gather of every examined edge, counted separately (it is served mostly
    # by L2 and MALL, and `traffic` shows what it costs in fetched lines)
    gbytes = nbytes + 4 * tst["edges_examined"]
    achieved_g = gbytes / (tst["ms_improve"] * 1e-3) / 1e9
    roofline["with_gather"] = {"achieved": round(achieved_g, 1), "frac": round(achieved_g / HBM_PEAK_GBS, 4),
                               "bytes_per_launch": int(gbytes / max(1, tst["improve_launches"]))}

    goal_exact = float(g_out[1].item())
    g_ref = g_out.clone()  # the timed calls' g (the extras below write g_out)
    # the narrowed Improve domain (PIRRT_LOOKAHEAD) on the same graph and policy
    look = None
    if not args.no_extra:
        G.snapshot_restore()
        G.replan(0, 1, h, True, g_out=g_out, parent_out=p_out, lookahead=True)
        reps = 5
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            G.snapshot_restore()
            _, _, s4 = G.replan(0, 1, h, True, g_out=g_out, parent_out=p_out, lookahead=True)
        torch.cuda.synchronize()
        t_lk = (time.perf_counter() - t0) / reps
        goal_look = float(g_out[1].item())
        look = {"replan_ms": round(1e3 * t_lk, 3), "speedup_vs_full_domain": round(ms_per_step / (1e3 * t_lk), 3),
                "iterations": s4["iterations"], "edges_examined": s4["edges_examined"], "sum_D": s4["sum_D"],
                "goal_cost": goal_look, "goal_cost_full_domain": goal_exact,
                "goal_cost_rel_diff": abs(goal_look - goal_exact) / goal_exact}
        log("narrowed domain: %s" % json.dumps(look))

    # the same Replan with h read from and g / parent written to pinned host memory:
    # the rate a caller sees when its buffers are on the host (PCIe included)
    host_io = None
    if not args.no_extra:
        h_host = h.cpu().pin_memory()
        g_host = torch.empty(n, dtype=torch.float32).pin_memory()
        p_host = torch.empty(n, dtype=torch.int32).pin_memory()
        G.snapshot_restore()
        G.replan(0, 1, h_host, True, g_out=g_host, parent_out=p_host)
        reps = 5
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            G.snapshot_restore()
            _, _, s6 = G.replan(0, 1, h_host, True, g_out=g_host, parent_out=p_host)
        torch.cuda.synchronize()
        t_io = (time.perf_counter() - t0) / reps
        assert np.array_equal(g_host.numpy().view(np.uint32), g_ref.cpu().numpy().view(np.uint32))
        host_io = {"replan_ms": round(1e3 * t_io, 3), "gteps": round(s6["edges_examined"] / t_io / 1e9, 2),
                   "bytes_over_pcie": int(12 * n),
                   "note": "h from and g, parent to pinned host memory; same bits as the device-buffer call"}
        log("host buffers: %s" % json.dumps(host_io))

    # the truncated Evaluate (PIRRT_TRUNCATED) on the same graph and policy
    trunc = None
    if not args.no_extra:
        G.snapshot_restore()
        G.replan(0, 1, h, True, g_out=g_out, parent_out=p_out, truncated=True)
        reps = 5
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            G.snapshot_restore()
            _, _, s5 = G.replan(0, 1, h, True, g_out=g_out, parent_out=p_out, truncated=True)
        torch.cuda.synchronize()
        t_tr = (time.perf_counter() - t0) / reps
        g_tr, p_tr, c_tr = G.get_policy()
        att = p_tr >= 0
        # vertices whose g is not their parent's g plus the parent-edge cost (stale g)
        stale = int(np.count_nonzero(g_tr[att] != (g_tr[p_tr[att]] + c_tr[att])))
        goal_tr = float(g_tr[1])
        trunc = {"replan_ms": round(1e3 * t_tr, 3), "speedup_vs_full_evaluate": round(ms_per_step / (1e3 * t_tr), 3),
                 "iterations": s5["iterations"], "edges_examined": s5["edges_examined"], "sum_P": s5["sum_P"],
                 "sum_D": s5["sum_D"], "stale_vertices": stale, "goal_cost": goal_tr,
                 "goal_cost_full_evaluate": goal_exact,
                 "goal_cost_rel_diff": abs(goal_tr - goal_exact) / goal_exact}
        log("truncated Evaluate: %s" % json.dumps(trunc))

    # the same Replan with pruning off (G = +inf: every reachable vertex is promising)
    noprune = None
    if not args.no_extra:
        G.snapshot_restore()
        G.replan(0, 1, h, False, g_out=g_out, parent_out=p_out)
        reps = 2
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            G.snapshot_restore()
            _, _, s3 = G.replan(0, 1, h, False, g_out=g_out, parent_out=p_out)
        torch.cuda.synchronize()
        t_np = (time.perf_counter() - t0) / reps
        noprune = {"replan_ms": round(1e3 * t_np, 3), "iterations": s3["iterations"],
                   "edges_examined": s3["edges_examined"], "gteps": round(s3["edges_examined"] / t_np / 1e9, 2)}
        # Improve alone with every reachable vertex in the domain: long runs of whole rows
        G.snapshot_restore()
        t3 = G.replan(0, 1, h, False, timing=True, g_out=g_out, parent_out=p_out)[2]
        nb3 = improve_bytes(t3["edges_examined"], t3["sum_D"], n, t3["improve_launches"])
        a3 = nb3 / (t3["ms_improve"] * 1e-3) / 1e9
        noprune["improve"] = {"achieved": round(a3, 1), "frac": round(a3 / HBM_PEAK_GBS, 4), "unit": "GB/s",
                              "launches": t3["improve_launches"],
                              "avg_launch_us": round(1e3 * t3["ms_improve"] / max(1, t3["improve_launches"]), 2),
                              "bytes_per_launch": int(nb3 / max(1, t3["improve_launches"]))}
        log("pruning off: %s" % json.dumps(noprune))

    # Evaluate (walk): every vertex once per call, 28 B each (parent 4, parent-edge cost 4,
    # the 8-byte epoch stamp read and written, g written 4): a latency-bound pointer chase
    ev_bytes = 28 * n * tst["evaluate_calls"]
    ev_gbs = ev_bytes / (tst["ms_evaluate"] * 1e-3) / 1e9
    evaluate = {"calls": tst["evaluate_calls"], "ms": round(tst["ms_evaluate"], 4),
                "bytes_per_call": 28 * n, "achieved_GBs": round(ev_gbs, 1),
                "frac_of_hbm_peak": round(ev_gbs / HBM_PEAK_GBS, 4)}

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
        s0 = R.state()
        times = []
        for rep in range(CPU_REPS):
            if rep:
                assert R.set_state(s0.g, s0.parent, s0.pcost) == 0
            t0 = time.perf_counter()
            rc, so = R.replan(0, 1, hh, True)
            times.append(time.perf_counter() - t0)
            assert rc == 0
        t_cpu = sorted(times)[len(times) // 2]
        # the timed GPU steps against the oracle: g bit for bit, parents and counters exact
        ref = R.state()
        bad_g = int(np.count_nonzero(g_timed.view(np.uint32) != ref.g.view(np.uint32)))
        bad_p = int(np.count_nonzero(p_timed != ref.parent))
        if bad_g or bad_p:
            raise SystemExit("timed Replan differs from the oracle: %d g values, %d parents" % (bad_g, bad_p))
        for k in ("iterations", "edges_examined", "sum_P", "sum_D", "changed_total", "mark_edges"):
            if so[k] != st[k]:
                raise SystemExit("timed Replan differs from the oracle in %s: %d against %d" % (k, st[k], so[k]))
        cpu = {"value": round(so["edges_examined"] / t_cpu / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": "one full Replan of the same 1M-vertex graph from its insertion-time policy, median of %d "
                         "(serial C oracle, one thread, %.2f s each)" % (CPU_REPS, t_cpu),
               "parity": "timed GPU Replan equals the oracle: g bit for bit, parents and counters exact"}
        cpu.update(host_fields())
        log("cpu baseline: %s" % json.dumps(cpu))

    if args.copy_calibration:
        x = torch.empty(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        torch.neg(x, out=y)  # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")

    rb = replan_bytes(st, n)
    replan_hbm = {"bytes_per_replan": rb["total"], "by_phase": {k: v for k, v in rb.items() if k != "total"},
                  "achieved": round(rb["total"] / (ms_per_step * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(rb["total"] / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "note": "the whole Replan's algorithmic bytes (every phase, counters of the timed call) over "
                          "the timed ms per Replan"}
    log("replan HBM: %s" % json.dumps(replan_hbm))
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
                   "autotuned_config": tuned, "parallelism": "single GPU"},
        "step_ms": {"mean": round(ms_per_step, 4), "median": round(float(np.median(step_ms)), 4),
                    "min": round(min(step_ms), 4)},
        "copy_ceiling": copy_ceiling(),
        "phases_ms": {k: round(tst[k], 4) for k in ("ms_evaluate", "ms_mark", "ms_improve")},
        "roofline": roofline,
        "replan_hbm": replan_hbm,
        "evaluate": evaluate,
        "cpu_baseline": cpu,
        "extra_batch": extra,
        "pruning_off": noprune,
        "host_buffers": host_io,
        "lookahead_domain": look,
        "truncated_evaluate": trunc,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
