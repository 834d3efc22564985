"""Throughput of the per-frame tile-and-depth sort on one MI355X.

One step = the whole hot path (count, scan, duplicate, radix sort, ranges)
over one synthetic frame whose records are already resident in HBM.  The
default workload is the large heavy-tailed frame (1920x1080, 8,160 tiles,
N = 6,000,000 Gaussians, about 27.6M pairs); the same run adds the full-HD
and 256x256 frames (p50/p99 latency) and the 64-frame batch against 64 plain
launches as extra keys.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline] [--no-extras]

Profiles (run under rocprofv3, then summarised into profiles/ with
``--summarize-profiles DIR``; the exact commands are written into each summary):

    rocprofv3 --kernel-trace --stats --output-format csv -d DIR/stats -o run -- \
        python3 bench.py --workload large-6m --steps 20 --warmup 5 --no-cpu-baseline --no-extras
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/fetch -o run -- \
        python3 bench.py --workload large-6m --steps 3 --warmup 1 --no-cpu-baseline --no-extras --copy-mib 512
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/write -o run -- \
        python3 bench.py --workload large-6m --steps 3 --warmup 1 --no-cpu-baseline --no-extras --copy-mib 512
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

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, published
DEFAULT_WORKLOAD = "large-6m"
PASS_SOURCE = os.path.join(ROOT, "paper_2511_16298_amd", "csrc", "onesweep.hip")
API_SOURCE = os.path.join(ROOT, "paper_2511_16298_amd", "csrc", "api.hip")
PROFILES = os.path.join(ROOT, "profiles")
PASS_KERNEL = "k_onesweep"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default=DEFAULT_WORKLOAD,
                   choices=sorted(synth.FRAME_WORKLOADS) + sorted(synth.SUPPLEMENTARY_WORKLOADS)
                   + ["batch-64", "serve", "sweep", "render", "preprocess", "shard-large-6m"])
    p.add_argument("--bands", type=int, default=8, help="tile-row bands = GPUs of the sharded frame (shard-*)")
    p.add_argument("--serve-seconds", type=float, default=30.0, help="arrival window per rate (serve)")
    p.add_argument("--serve-rates", default="200,1000,3000,6000,12000", help="requests per second (serve)")
    p.add_argument("--serve-closed-seconds", type=float, default=10.0,
                   help="closed-loop run per mode (serve; 0: skip)")
    p.add_argument("--serve-outstanding", type=int, default=48,
                   help="requests kept in flight by the closed loop (serve)")
    p.add_argument("--arena-gib", type=float, default=64.0, help="HBM budget of the server (serve)")
    p.add_argument("--small-arena-gib", type=float, default=0.5,
                   help="second budget, run at the highest rate to force admission stalls (serve; 0: skip)")
    p.add_argument("--pool-frames", type=int, default=512, help="device-resident request frames (serve)")
    p.add_argument("--sweep-mpairs", default="0.5,1,2,4,8,17,32,64,100",
                   help="sort-only sizes in millions of pairs (sweep)")
    p.add_argument("--radix-bits", type=int, default=0)
    p.add_argument("--items", type=int, default=0)
    p.add_argument("--wg", type=int, default=0, help="sort-pass workgroup size")
    p.add_argument("--algorithm", default="depth-first",
                   choices=["depth-first", "direct", "bitonic", "bitonic-key32", "tile-first"],
                   help="frame sort algorithm (frames, sweep); bitonic-key32 = the paper's normalised "
                        "32-bit float key (lossy within a tile, frames only)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true",
                   help="default workload only: skip the full-HD and 256x256 frames and the batch comparison")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="budget of the oracle baseline (whole frames until exceeded)")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="run one streaming copy of this size first (traffic-counter calibration)")
    p.add_argument("--summarize-profiles", metavar="DIR",
                   help="summarise rocprofv3 output under DIR/{stats,fetch,write} into profiles/ and exit")
    p.add_argument("--profiled-args", default="--steps 20 --warmup 5 --no-cpu-baseline --no-extras",
                   help="with --summarize-profiles: the bench arguments of the profiled kernel-trace run")
    return p.parse_args()


def source_hash(paths=None) -> str:
    """sha256[:16] of the sources that decide a profiled kernel: the sort pass
    kernel together with the host code that picks its launch shapes."""
    if paths is None:
        paths = (PASS_SOURCE, API_SOURCE)
    if isinstance(paths, str):
        paths = (paths,)
    h = hashlib.sha256()
    for path in paths:
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def dominant_kernel(workload: str):
    """(kernel-name prefix, name filter, source file) of the kernel a
    workload's roofline is quoted on: the projection kernel for the
    preprocessing workload, else the 64-bit-key (tile) sort pass."""
    if workload == "preprocess":
        return "k_preprocess", "", os.path.join(ROOT, "paper_2511_16298_amd", "csrc", "preprocess.hip")
    if workload == "render":
        return "k_render", "", os.path.join(ROOT, "paper_2511_16298_amd", "csrc", "render.hip")
    return PASS_KERNEL, "unsigned long", (PASS_SOURCE, API_SOURCE)


def _rows(pattern: str):
    files = sorted(glob.glob(pattern))
    if not files:
        raise SystemExit(f"no rocprofv3 csv matches {pattern}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def summarize_profiles(d: str, workload: str, copy_mib: int = 512,
                       profiled_args: str = "--steps 20 --warmup 5 --no-cpu-baseline --no-extras"):
    """Write the kernel-time and HBM-traffic summaries of the pass kernel."""
    os.makedirs(PROFILES, exist_ok=True)
    stats = _rows(os.path.join(d, "stats", "*kernel_stats.csv"))
    lines = [f"# rocprofv3 kernel statistics, workload {workload}",
             "command: rocprofv3 --kernel-trace --stats --output-format csv -d DIR/stats -o run -- "
             f"python3 bench.py --workload {workload} {profiled_args}",
             f"{dominant_kernel(workload)[0]} sources (kernel, launch shapes) sha256[:16]: {source_hash(dominant_kernel(workload)[2])}", "",
             "| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in stats:
        name = r["Name"]
        short = name.replace("ss::(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        if short.startswith("at::") or "rocclr" in short:
            continue
        lines.append(f"| {short} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['Percentage']):.1f} |")
    with open(os.path.join(PROFILES, f"kernel_stats_{workload}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    if not os.path.isdir(os.path.join(d, "fetch")):
        return   # kernel times only (e.g. the render workload, which is ALU-bound)

    def short_name(name):
        return name.replace("ss::(anonymous namespace)::", "").replace("void ", "").split("(")[0]

    def per_kernel(kind):
        rows = _rows(os.path.join(d, kind, "*counter_collection.csv"))
        by = {}
        for r in rows:
            by.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        copy = [v for k, vs in by.items() if k.startswith("k_copy") for v in vs]
        return copy, by
    fc, fby = per_kernel("fetch")
    wc, wby = per_kernel("write")
    kib = copy_mib * 1024.0
    f_scale, w_scale = kib / (sum(fc) / len(fc)), kib / (sum(wc) / len(wc))
    # the measured kernel
    kname, kfilter, ksrc = dominant_kernel(workload)
    # every instantiation of it (the tile passes: 8-bit, and a narrower last
    # pass), averaged per launch like the benchmark's timing of the group
    tile = sorted(k for k in fby if k.startswith(kname) and kfilter in k)
    assert tile, kname
    fp = [v for k in tile for v in fby[k]]
    wp = [v for k in tile for v in wby[k]]
    fetch = sum(fp) / len(fp) * f_scale * 1024.0
    write = sum(wp) / len(wp) * w_scale * 1024.0
    # the whole frame step: every kernel launched at least once per frame
    # (launches per frame = its calls / the calls of the per-frame count
    # kernel in the timing run), its measured bytes and its time
    calls = {short_name(r["Name"]): (int(r["Calls"]), float(r["AverageNs"])) for r in stats}
    per_frame = calls.get("k_count_keys", (0, 0.0))[0]
    step = None
    if per_frame and workload != "preprocess":
        b = t_ns = 0.0
        for k, (c, avg) in calls.items():
            if c < per_frame or k not in fby or k not in wby or k.startswith("at::") or "rocclr" in k:
                continue
            lpf = c / per_frame
            b += lpf * (sum(fby[k]) / len(fby[k]) * f_scale + sum(wby[k]) / len(wby[k]) * w_scale) * 1024.0
            t_ns += lpf * avg
        step = {"bytes_per_frame": b, "kernel_us_per_frame": t_ns / 1e3,
                "GB/s": b / t_ns, "frac_of_peak": b / t_ns / PEAK_HBM_GBS}
    others = {k: {"dispatches": len(fby[k]),
                  "fetch_bytes_per_launch": round(sum(fby[k]) / len(fby[k]) * f_scale * 1024.0),
                  "write_bytes_per_launch": round(sum(wby[k]) / len(wby[k]) * w_scale * 1024.0)}
              for k in sorted(fby) if k in wby and not k.startswith("at::") and "rocclr" not in k}
    wl = f"--workload {workload} "
    rec = {"kernel": " + ".join(tile), "workload": workload, "source_sha256_16": source_hash(ksrc),
           "copy_calibration_mib": copy_mib, "fetch_scale": f_scale, "write_scale": w_scale,
           "dispatches": len(fp), "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "traffic_bytes_per_launch": fetch + write, "per_kernel": others, "step_measured": step,
           "commands": ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/fetch -o run -- python3 bench.py "
                        f"{wl}--steps 3 --warmup 1 --no-cpu-baseline --no-extras --copy-mib {copy_mib}",
                        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/write -o run -- python3 bench.py "
                        f"{wl}--steps 3 --warmup 1 --no-cpu-baseline --no-extras --copy-mib {copy_mib}"]}
    with open(os.path.join(PROFILES, f"{kname}_{workload}_traffic.txt"), "w") as f:
        f.write(f"# HBM traffic of one {kname} launch (FETCH_SIZE x fetch_scale + WRITE_SIZE x write_scale;\n"
                "# the scales make a plain copy of copy_calibration_mib MiB read and write exactly that),\n"
                "# and the same per launch for every kernel of the step\n")
        f.write(json.dumps(rec, indent=1) + "\n")
    print(json.dumps(rec))


def profiled_record(workload: str):
    """The committed traffic record of the workload's roofline kernel, if it
    was taken on that kernel's current source; else None."""
    kname, _, ksrc = dominant_kernel(workload)
    path = os.path.join(PROFILES, f"{kname}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    rec = json.loads(text[text.index("{"):])
    return rec if rec.get("source_sha256_16") == source_hash(ksrc) else None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def profiled_traffic(workload: str):
    """Traffic per launch of the workload's roofline kernel from the committed
    profile, if it was taken on that kernel's current source; else None."""
    kname, _, ksrc = dominant_kernel(workload)
    path = os.path.join(PROFILES, f"{kname}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    rec = json.loads(text[text.index("{"):])
    if rec.get("source_sha256_16") != source_hash(ksrc):
        return None
    return rec["traffic_bytes_per_launch"]


def calibration_copy(args, dev, stream):
    """One streaming copy of --copy-mib MiB (traffic-counter calibration)."""
    if not args.copy_mib:
        return
    import torch
    import paper_2511_16298_amd as ss
    nb = args.copy_mib << 20
    a = torch.ones(nb // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    ss.copy_bytes(b, a, nb, stream)
    torch.cuda.synchronize()
    del a, b


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def bench_serve(args):
    """Poisson request streams over a pool of device-resident frames drawn as
    in the batch workload: continuous batching against one request at a time,
    at offered rates below and above what one request at a time sustains,
    plus a closed loop that keeps a fixed number of requests outstanding (the
    most each mode can serve).  A sample of served results is kept and
    compared, after each run, with the plain single-frame path's output for
    the same frame."""
    import collections
    import threading
    import torch
    import paper_2511_16298_amd as ss

    # the request pool is drawn on the host before anything touches the GPU
    # (forked workers, one frame each)
    import multiprocessing as mp
    t_gen = time.perf_counter()
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as workers:
        pool = workers.starmap(synth.batch_frame, [(synth.SEED_BASE + 4, f) for f in range(args.pool_frames)])
    print(f"# pool: {len(pool)} frames, N={sum(len(r) for _, _, r in pool)}, drawn in "
          f"{time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    recs = []
    for i in range(len(pool)):
        recs.append(ss.records_to_device(pool[i][2], dev))
        pool[i] = (pool[i][0], pool[i][1], None)   # keep the shape only
    rates = [float(x) for x in args.serve_rates.split(",")]
    arena = int(args.arena_gib * (1 << 30))
    copy_stream = torch.cuda.Stream(device=dev)

    class Sampler:
        """Keeps device copies of every `every`-th served result (at most
        `cap`), to be compared with the plain path afterwards."""

        def __init__(self, srv, every=53, cap=16):
            self.srv, self.every, self.cap, self.kept, self.n = srv, every, cap, [], 0

        def take(self, r, k):
            self.n += 1
            if r.status != 0 or self.n % self.every or len(self.kept) >= self.cap:
                return
            base = self.srv.arena.data_ptr()
            m = int(r.num_pairs)
            w, h, _ = pool[k]
            tx, ty, _ = ss.geometry(w, h)
            with torch.cuda.stream(copy_stream):
                def grab(ptr, nbytes):
                    off = int(ptr) - base
                    return self.srv.arena[off:off + nbytes].clone()
                kk = grab(r.keys, 8 * m).view(torch.int64) - (int(r.tile_base) << 32)
                vv = grab(r.values, 4 * m).view(torch.int32)
                rg = grab(r.tile_ranges, 8 * tx * ty).view(torch.int32) - int(r.pair_base)
            copy_stream.synchronize()
            self.kept.append((k, kk, vv, rg))

        def verify(self):
            """(compared, all equal): each kept result against ss_sort_frame."""
            ok = True
            for k, kk, vv, rg in self.kept:
                w, h, _ = pool[k]
                out = ss.sort_frame(recs[k], w, h)
                st, m = out.result()
                ok &= bool(st == 0 and m == kk.numel() and torch.equal(out.keys[:m], kk)
                           and torch.equal(out.values[:m], vv) and torch.equal(out.tile_ranges.view(-1), rg))
            n = len(self.kept)
            self.kept = []
            return n, bool(ok)

    def summarize(got, span_s, offered_window_s=None):
        g = np.array([x[:5] for x in got], dtype=np.float64)
        ok = g[:, 0] == 0
        lat = (g[:, 4] - g[:, 2]) / 1e3   # ms
        keep = ok & ((g[:, 2] - g[:, 2].min()) > 1e6)   # skip the first second of arrivals
        if not keep.any():
            keep = ok
        res = {"requests": len(got), "ok": int(ok.sum()), "rejected_budget": int((g[:, 0] == 8).sum()),
               "pairs": int(g[ok, 1].sum()), "pairs_per_s": float(g[ok, 1].sum() / span_s),
               "requests_per_s": float(ok.sum() / span_s),
               "p50_ms": pct(lat[keep], 50), "p99_ms": pct(lat[keep], 99),
               "mean_round_frames": float(np.mean([x[5] for x in got]))}
        if offered_window_s:
            res["offered_pairs_per_s"] = float(g[ok, 1].sum() / offered_window_s)
        return res

    def run_trace(srv, rate):
        seed = synth.SEED_BASE + 4 + int(rate)
        arr = synth.poisson_arrivals(rate, args.serve_seconds, seed)
        picks = synth.uniform_int(synth.stream_key(seed, 7), len(arr), len(pool))
        tickets = []
        lock = threading.Condition()
        got = []
        done_submitting = [False]
        sampler = Sampler(srv)

        def collect():
            i = 0
            last = time.perf_counter()
            while True:
                with lock:
                    while i >= len(tickets) and not done_submitting[0]:
                        lock.wait(0.01)
                    if i >= len(tickets):
                        return
                    t, k = tickets[i]
                r = srv.wait(t)
                got.append((r.status, r.num_pairs, r.submit_us, r.start_us, r.done_us, r.round_frames))
                sampler.take(r, k)
                srv.release(t)
                i += 1
                if time.perf_counter() - last > 10.0:  # a backlog can take minutes to drain
                    last = time.perf_counter()
                    print(f"# serve at {int(rate)}/s: {i} of {len(arr)} requests completed", file=sys.stderr, flush=True)
        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for a, k in zip(arr, picks):
            delay = t0 + a - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            w, h, _ = pool[int(k)]
            t = srv.submit(recs[int(k)], w, h)
            with lock:
                tickets.append((t, int(k)))
                lock.notify()
        with lock:
            done_submitting[0] = True
            lock.notify()
        th.join()
        g = np.array([x[:5] for x in got], dtype=np.float64)
        span = (g[:, 4].max() - g[:, 2].min()) / 1e6
        res = summarize(got, span, args.serve_seconds)
        res["offered_requests_per_s"] = rate
        res["verified_results"], res["verified_equal_plain"] = sampler.verify()
        return res

    def run_closed(srv, outstanding, seconds):
        """Closed loop: `outstanding` requests in flight at all times."""
        seed = synth.SEED_BASE + 4 + 99
        picks = synth.uniform_int(synth.stream_key(seed, 7), 1 << 20, len(pool))
        sampler = Sampler(srv)
        q = collections.deque()
        got = []
        j = 0
        t_end = time.perf_counter() + seconds
        for _ in range(outstanding):
            k = int(picks[j]); j += 1
            w, h, _ = pool[k]
            q.append((srv.submit(recs[k], w, h), k))
        while q:
            t, k = q.popleft()
            r = srv.wait(t)
            got.append((r.status, r.num_pairs, r.submit_us, r.start_us, r.done_us, r.round_frames))
            sampler.take(r, k)
            srv.release(t)
            if time.perf_counter() < t_end:
                k2 = int(picks[j % len(picks)]); j += 1
                w, h, _ = pool[k2]
                q.append((srv.submit(recs[k2], w, h), k2))
        g = np.array([x[:5] for x in got], dtype=np.float64)
        span = (g[:, 4].max() - g[:, 2].min()) / 1e6
        res = summarize(got, span)
        res["outstanding"] = outstanding
        res["verified_results"], res["verified_equal_plain"] = sampler.verify()
        return res

    runs = [("batched", 64, 2, arena, rates), ("one_at_a_time", 1, 1, arena, rates)]
    if args.small_arena_gib > 0:
        runs.append(("batched_small_arena", 64, 2, int(args.small_arena_gib * (1 << 30)), rates[-1:]))
    results = {}
    for mode, frames, streams, budget, mode_rates in runs:
        srv = ss.Server(budget, max_batch_frames=frames, n_streams=streams, device=dev)
        for rate in mode_rates:
            key = f"{mode}@{int(rate)}"
            results[key] = run_trace(srv, rate)
            print(f"# {key}: {results[key]}", file=sys.stderr, flush=True)
        if args.serve_closed_seconds > 0 and mode != "batched_small_arena":
            key = f"{mode}@closed"
            results[key] = run_closed(srv, args.serve_outstanding, args.serve_closed_seconds)
            print(f"# {key}: {results[key]}", file=sys.stderr, flush=True)
        srv.close()
        del srv
        torch.cuda.empty_cache()
    top = f"batched@{int(rates[-1])}"
    line = {"metric": "served frame-sort requests: pairs/s and p50/p99 request latency",
            "value": results[top]["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
            "steps": None, "warmup": None, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"serve: Poisson arrivals {args.serve_rates}/s for {args.serve_seconds:g} s "
                                   f"each, frames drawn from a pool of {len(pool)} device-resident frames of "
                                   f"the batch distribution, HBM budget {args.arena_gib:g} GiB (and "
                                   f"{args.small_arena_gib:g} GiB at the highest rate); closed loop with "
                                   f"{args.serve_outstanding} requests outstanding for "
                                   f"{args.serve_closed_seconds:g} s",
                       "parallelism": "single GPU"},
            "runs": results}
    if "batched@closed" in results and "one_at_a_time@closed" in results:
        line["closed_loop_speedup_pairs_per_s"] = (results["batched@closed"]["pairs_per_s"]
                                                   / results["one_at_a_time@closed"]["pairs_per_s"])
    line["all_verified_equal_plain"] = all(r.get("verified_equal_plain", True) for r in results.values())
    print(json.dumps(line), flush=True)


RENDER_FLOPS_PER_EVAL = 18   # dy 1, quadratic form 4, scale 1, exp 1, alpha 1, cap 1, T 2, weight 1, colour 6


def bench_shard(args):
    """One GPU's share of the heavy-tailed frame sharded over --bands GPUs by
    tile-row bands (the design for more than one GPU: every GPU counts all N
    Gaussians, sorts them by depth, and expands and sorts only its band's
    pairs).  Each band runs alone on this GPU, in the launch configuration of
    the whole frame; the slowest band bounds the sharded frame."""
    import torch
    import paper_2511_16298_amd as ss
    from paper_2511_16298_amd import _abi

    spec, seed = synth.workload("large-6m")
    rec = synth.make_frame(spec, seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    K, W = args.steps, args.warmup

    def timed(sorter, d):
        for _ in range(W):
            sorter(d, stream)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
        ev[0].record(stream)
        for i in range(K):
            sorter(d, stream)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        st, m = sorter.out.result()
        assert st == 0
        return [ev[i].elapsed_time(ev[i + 1]) for i in range(K)], m

    def sorter_for(h, d, drop):
        _, _, m_t, s_t = ss.count_pairs(d, spec.width, h)
        assert int(s_t.item()) == 0
        return ss.FrameSorter(spec.width, h, int(d.shape[0]), int(m_t.item()) & 0xFFFFFFFF, device=dev,
                              drop_culled=drop)

    d_full = ss.records_to_device(rec, dev)
    full_ms, m_full = timed(sorter_for(spec.height, d_full, False), d_full)
    del d_full
    rows = []
    slowest = None
    for h, r0, rb in synth.band_frames(rec, spec.width, spec.height, args.bands):
        d = ss.records_to_device(rb, dev)
        # most of the frame's Gaussians miss a band: the depth sort drops them
        srt = sorter_for(h, d, True)
        ms, m = timed(srt, d)
        rows.append({"first_tile_row": r0, "height": h, "num_pairs": m, "p50_ms": pct(ms, 50), "p99_ms": pct(ms, 99)})
        if slowest is None or pct(ms, 50) > slowest[0]:
            timer = ss.Timer(max_launches=K * 12 + 16)
            for _ in range(K):
                srt(d, stream, timer=timer)
            torch.cuda.synchronize()
            pms, pn = timer.read(_abi.SS_KERNEL_SORT_PASS)
            timer.close()
            slowest = (pct(ms, 50), m, h, r0, rb, 1e3 * pms / pn)
        del d, srt
    t_band, m_band, h_band, r0_band, rec_band, pass_us = slowest
    assert sum(r["num_pairs"] for r in rows) == m_full
    achieved = 24.0 * m_band / (pass_us * 1e-6) / 1e9
    line = {"metric": f"sorted key-value pairs/s of one GPU's share (1 of {args.bands} tile-row bands)",
            "value": m_band / (t_band * 1e-3), "unit": "pairs/s", "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": t_band, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
            "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"shard-large-6m: large-6m ({spec.width}x{spec.height}, N={len(rec)}, "
                                   f"M={m_full}) cut into {args.bands} bands of whole tile rows; the slowest "
                                   f"band (tile rows from {r0_band}, {h_band} px) on one GPU",
                       "parallelism": f"one GPU's band of {args.bands}", "flags": "SS_FLAG_DROP_CULLED"},
            "bands": rows,
            "whole_frame_p50_ms": pct(full_ms, 50),
            "sharded_frame_bound_ms": t_band,
            "roofline": {"bound": "hbm", "kernel": "sort_pass", "achieved": achieved, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                         "bytes_per_launch": 24.0 * m_band, "avg_launch_us": pass_us}}
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        o = oracle.sort_frame(spec.width, h_band, rec_band, stages=False)
        spent = time.perf_counter() - t
        line["cpu_baseline"] = {"value": o.num_pairs / spent, "unit": "pairs/s", "cores": 1, "kind": "oracle",
                                "sample": f"the slowest band once ({spent:.1f} s, single-threaded oracle on "
                                          f"{cpu_model()})"}
    print(json.dumps(line), flush=True)


def bench_render(args):
    """Alpha blending of the sorted full-HD frame (the step after the sort):
    frames/s with the records, render inputs and sorted lists resident in HBM."""
    import torch
    import paper_2511_16298_amd as ss

    spec, seed = synth.workload("fullhd-1m")
    rec = synth.make_frame(spec, seed)
    co, cl = synth.make_render_attrs(rec, seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    d = ss.records_to_device(rec, dev)
    srt = ss.sort_frame(d, spec.width, spec.height)
    st, M = srt.result()
    assert st == 0
    cod, cld = ss.render_attrs_to_device(co, cl, dev)
    bg = (0.0, 0.0, 0.0)
    r = ss.Renderer(spec.width, spec.height, device=dev)
    for _ in range(args.warmup):
        r(d, cod, cld, srt.values, srt.tile_ranges, srt.status, bg)
    torch.cuda.synchronize()
    K = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    ev[0].record(stream)
    for i in range(K):
        r(d, cod, cld, srt.values, srt.tile_ranges, srt.status, bg)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(K)]
    ms = ev[0].elapsed_time(ev[K]) / K
    # evaluations (pixel, Gaussian) the method performs, from the counting variant
    rs = ss.Renderer(spec.width, spec.height, device=dev, want_T=True, want_contrib=True, want_tile_evals=True)
    rs(d, cod, cld, srt.values, srt.tile_ranges, srt.status, bg)
    torch.cuda.synchronize()
    evals = int(rs.out.tile_evals.cpu().numpy().view(np.uint32).astype(np.int64).sum())
    tflops = RENDER_FLOPS_PER_EVAL * evals / (ms * 1e-3) / 1e12
    line = {"metric": "rendered frames/s (alpha blending of a sorted frame, FP32)", "value": 1e3 / ms,
            "unit": "frames/s", "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"render fullhd-1m: {spec.width}x{spec.height}, N={len(rec)}, M={M} sorted pairs, "
                                   f"synthetic conic/opacity/colour (seed {seed}), 3DGS thresholds",
                       "parallelism": "single GPU"},
            "latency_ms": {"p50": pct(step_ms, 50), "p99": pct(step_ms, 99)},
            "roofline": {"bound": "alu", "kernel": "k_render", "achieved": tflops, "peak": 157.3, "unit": "TFLOP/s",
                         "frac": tflops / 157.3, "traffic": None, "evaluations": evals,
                         "flops_per_evaluation": RENDER_FLOPS_PER_EVAL}}
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        o = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
        ref = oracle.render(spec.width, spec.height, rec, co, cl, o.values, o.ranges, bg)
        spent = time.perf_counter() - t
        gpu = rs.out.color.cpu().numpy().astype(np.float64)
        ok = ref.margin >= 1e-4
        tol = 2e-6 + 2.4e-7 * ref.n_contrib.astype(np.float64)
        line["cpu_baseline"] = {"value": 1.0 / spent, "unit": "frames/s", "cores": 1, "kind": "oracle",
                                "sample": f"one fullhd-1m frame, oracle sort + FP64 render ({spent:.1f} s, single-threaded)"}
        line["parity_vs_oracle"] = bool(np.all((np.abs(gpu - ref.color).max(axis=0) <= tol)[ok]))
        line["parity_unambiguous_pixels"] = float(ok.mean())
    print(json.dumps(line), flush=True)


# bytes one Gaussian moves through the preprocess kernel at SH degree 3:
# mean + opacity 16, covariance row 32 (24 used, padded to 16-byte loads),
# 48 SH floats 192 in; record 16, conic + opacity 16, colour 16 out
PREPROCESS_BYTES = 16 + 32 + 192 + 48


def bench_preprocess(args):
    """Projection of 10^6 synthetic 3D Gaussians for a full-HD camera (the step
    before the sort): Gaussians/s with the scene resident in HBM, and the same
    frame carried on through the sort (preprocess + sort per frame)."""
    import torch
    import paper_2511_16298_amd as ss
    from paper_2511_16298_amd import _abi

    cam = synth.SCENE_CAMERA
    n = 1_000_000
    scene = synth.make_scene(n, cam, synth.SCENE_SEED)
    params = synth.camera_params(cam)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    m3, cv, sh = (torch.from_numpy(scene[k]).to(dev) for k in ("mean3d_opacity", "cov3d", "sh"))
    c = ss.camera(**params)
    pre = ss.Preprocessor(n, device=dev)
    calibration_copy(args, dev, stream)
    for _ in range(args.warmup):
        pre(c, m3, cv, sh, stream)
    torch.cuda.synchronize()
    K = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    ev[0].record(stream)
    for i in range(K):
        pre(c, m3, cv, sh, stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(K)]
    ms = ev[0].elapsed_time(ev[K]) / K
    # the kernel's own duration: HIP events around each launch, on its stream
    timer = ss.Timer(max_launches=K + 4)
    for _ in range(K):
        pre(c, m3, cv, sh, stream, timer=timer)
    torch.cuda.synchronize()
    kms, kn = timer.read(_abi.SS_KERNEL_PREPROCESS)
    timer.close()
    kern_us = 1e3 * kms / kn
    achieved = PREPROCESS_BYTES * n / (kern_us * 1e-6) / 1e9
    out = pre(c, m3, cv, sh, stream)
    torch.cuda.synchronize()
    # the frame carried through the sort: preprocess + depth-first sort
    recs = out.records
    _, _, m_t, s_t = ss.count_pairs(recs, cam.width, cam.height)
    assert int(s_t.item()) == 0
    M = int(m_t.item()) & 0xFFFFFFFF
    sorter = ss.FrameSorter(cam.width, cam.height, n, M, device=dev)
    for _ in range(args.warmup):
        pre(c, m3, cv, sh, stream)
        sorter(recs, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(K):
        pre(c, m3, cv, sh, stream)
        sorter(recs, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    chain_ms = e0.elapsed_time(e1) / K
    st, m_chk = sorter.out.result()
    assert st == 0 and m_chk == M
    line = {"metric": "preprocessed Gaussians/s (projection of 3D Gaussians, FP32)", "value": n / (ms * 1e-3),
            "unit": "Gaussians/s", "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"preprocess scene-1m: N={n} 3D Gaussians (seed {synth.SCENE_SEED}), "
                                   f"{cam.width}x{cam.height} camera, focal {cam.focal}, SH degree {cam.sh_degree}",
                       "parallelism": "single GPU"},
            "latency_ms": {"p50": pct(step_ms, 50), "p99": pct(step_ms, 99)},
            "roofline": {"bound": "hbm", "kernel": "k_preprocess", "achieved": achieved, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": profiled_traffic("preprocess"),
                         "bytes_per_launch": PREPROCESS_BYTES * n, "avg_launch_us": kern_us},
            "frame_with_sort": {"ms_per_frame": chain_ms, "num_pairs": M,
                                "pairs_per_s": M / (chain_ms * 1e-3)}}
    if not args.no_cpu_baseline:
        import oracle
        oc = oracle.camera(np.asarray(params["view"], np.float64).reshape(3, 4), params["fx"], params["fy"],
                           params["cx"], params["cy"], params["tan_fovx"], params["tan_fovy"], params["cam_pos"],
                           params["near_plane"], params["sh_degree"])
        runs, spent = 0, 0.0
        while spent < args.cpu_seconds or runs == 0:
            t = time.perf_counter()
            o = oracle.preprocess(oc, scene["mean3d_opacity"], scene["cov3d"], scene["sh"])
            spent += time.perf_counter() - t
            runs += 1
        g = out.records.cpu().numpy().view(np.uint32).reshape(-1, 4)
        same = np.all(g == o.records.view(np.uint32).reshape(-1, 4), axis=1)
        # records may differ only where the oracle sits next to a rounding boundary
        near_boundary = np.any(o.margin < 0.01, axis=1) | (np.abs(scene["mean3d_opacity"][:, 2] -
                                                                  params["near_plane"]) < 1e-3)
        line["cpu_baseline"] = {"value": runs * n / spent, "unit": "Gaussians/s", "cores": 1, "kind": "oracle",
                                "sample": f"{runs} whole scene-1m projections ({spent:.1f} s, single-threaded "
                                          f"FP64 oracle)"}
        line["records_bit_equal"] = float(same.mean())
        line["parity_vs_oracle"] = bool(np.all(same | near_boundary))
    print(json.dumps(line), flush=True)

def bench_sweep(args):
    """Sort alone (through ss_sort_pairs) over random 45-bit keys, the
    paper's random key-value sweep extended to 10^8 pairs."""
    import torch
    import paper_2511_16298_amd as ss
    from paper_2511_16298_amd import _abi

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    key_bits = 45
    rows = {}
    for mp_ in [float(x) for x in args.sweep_mpairs.split(",")]:
        m = int(mp_ * 1e6)
        keys, vals = synth.sort_sweep_pairs(m, key_bits, seed=synth.SEED_BASE + 5)
        ki = torch.from_numpy(keys.view(np.int64)).to(dev)
        vi = torch.from_numpy(vals.view(np.int32)).to(dev)
        del keys, vals
        ko, vo = torch.empty_like(ki), torch.empty_like(vi)
        opts = ss.make_options(algorithm=ss.SS_ALGO_BITONIC if args.algorithm == "bitonic" else 0)
        st, ws = _abi.ss_sort_pairs_workspace_bytes(m, key_bits, opts)
        assert st == 0
        work = torch.empty(max(ws, 256), dtype=torch.uint8, device=dev)

        def step():
            st_ = _abi.ss_sort_pairs(ki.data_ptr(), vi.data_ptr(), m, key_bits, ko.data_ptr(), vo.data_ptr(),
                                     work.data_ptr(), ws, stream.cuda_stream, opts)
            assert st_ == 0
        reps = max(3, min(args.steps, int(2e9 / max(m, 1))))
        for _ in range(min(args.warmup, 5)):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        ok = bool(torch.all(ko[1:] >= ko[:-1]).item()) if m > 1 else True
        passes = -(-key_bits // 8)
        rows[f"{mp_:g}M"] = {"pairs": m, "ms": ms, "pairs_per_s": m / (ms * 1e-3),
                             "pass_bytes_GBps": 24.0 * m * passes / (ms * 1e-3) / 1e9, "sorted": ok}
        print(f"# sweep {mp_:g}M: {rows[f'{mp_:g}M']}", file=sys.stderr, flush=True)
        del ki, vi, ko, vo, work
        torch.cuda.empty_cache()
    best = max(rows.values(), key=lambda r: r["pairs_per_s"])
    line = {"metric": "sort-only pairs/s over random 45-bit keys (supplementary sweep)",
            "value": best["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": None, "warmup": None,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u64", "data": "synthetic",
            "config": {"workload": f"sweep: ss_sort_pairs, uniform 45-bit keys, sizes {args.sweep_mpairs} M pairs",
                       "parallelism": "single GPU"},
            "runs": rows}
    print(json.dumps(line), flush=True)


def packed_pairs(n: int, max_frame_n: int, tile_bits: int, tile_passes: int) -> bool:
    """Whether the default tile passes carry each pair as one 64-bit item:
    tile, a depth field of at least 27 bits and the frame-local index fit,
    and so does the depth-order position that replaces the depth field when
    the depths span too many binades (the library's rule, default shapes)."""
    idx_bits = (max_frame_n - 1).bit_length() if max_frame_n > 1 else 0
    field = 64 - tile_bits - idx_bits
    pos_bits = (n - 1).bit_length() if n > 1 else 0
    return tile_passes >= 1 and tile_bits <= 32 and idx_bits < 32 and field >= 27 and pos_bits <= field


def step_bytes_model(n: int, m: int, tiles_x: int, tiles_y: int, key_bits: int, rb: int = 8) -> tuple:
    """(depth-first step bytes, direct-path bytes, tile passes, packed) of one frame.

    Depth-first, frames of at most 256 tiles per axis: count 16N read + 12N
    write (packed rectangle, depth key, index), four depth passes 24N each
    (the rectangle rides with the index), expand 12N read.  Then, with packed 64-bit pairs: expand writes 8M, the
    Pt - 1 first tile passes 16M each, the last one reads 8M and writes the
    12-byte pairs and the ranges (8T) -- 136 N + (12 + 16 Pt) M + 8 T;
    otherwise expand writes 12M, each tile pass moves 24M and the ranges
    kernel reads 8M and writes 8T -- 136 N + (20 + 24 Pt) M + 8 T.  Frames
    wider or taller than 256 tiles: 16N count write, 16N per depth pass,
    expand 8N read + 8N rectangle gather -- 112 N + ....  The direct path would move
    48 N + (28 + 24 P) M + 8 T."""
    tile_bits = key_bits - 32
    tile_passes = -(-tile_bits // rb)
    passes = -(-key_bits // rb)
    per_gaussian = 136.0 if tiles_x <= 256 and tiles_y <= 256 else 112.0
    packed = packed_pairs(n, n, tile_bits, tile_passes)
    per_pair = (12.0 + 16.0 * tile_passes) if packed else (20.0 + 24.0 * tile_passes)
    step = per_gaussian * n + per_pair * m + 8.0 * tiles_x * tiles_y
    direct = 48.0 * n + (28.0 + 24.0 * passes) * m + 8.0 * tiles_x * tiles_y
    return step, direct, tile_passes, packed


def time_frame(args, workload: str, steps: int, warmup: int, dev, stream, kernel_timer: bool = True):
    """K whole steps of one frame workload (records resident in HBM): per-step
    HIP-event times on the launching stream, host wall time, and (optionally)
    per-kernel durations from a second run with events around each launch."""
    import torch
    import paper_2511_16298_amd as ss
    from paper_2511_16298_amd import _abi

    spec, seed = synth.workload(workload)
    rec = synth.make_frame(spec, seed)
    d = ss.records_to_device(rec, dev)
    _, _, m_t, s_t = ss.count_pairs(d, spec.width, spec.height)
    assert int(s_t.item()) == 0
    M = int(m_t.item()) & 0xFFFFFFFF
    algo = {"depth-first": ss.SS_ALGO_DEPTH_FIRST, "direct": ss.SS_ALGO_DIRECT,
            "bitonic": ss.SS_ALGO_BITONIC, "bitonic-key32": ss.SS_ALGO_BITONIC,
            "tile-first": ss.SS_ALGO_TILE_FIRST}[args.algorithm]
    key32 = args.algorithm == "bitonic-key32"
    sorter = ss.FrameSorter(spec.width, spec.height, len(rec), M, args.radix_bits, args.items, device=dev,
                            workgroup_size=args.wg, algorithm=algo, key32=key32)
    print(f"# workload {workload}: {spec.width}x{spec.height}, N={len(rec)}, M={M}, "
          f"T={sorter.tiles_x * sorter.tiles_y}, key bits {sorter.key_bits}", file=sys.stderr, flush=True)
    for _ in range(warmup):
        sorter(d, stream)
    torch.cuda.synchronize()
    st, m_chk = sorter.out.result()
    assert st == 0 and m_chk == M, (st, m_chk)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        sorter(d, stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    ms_per_step = ev[0].elapsed_time(ev[steps]) / steps
    print(f"# {workload}: timed {steps} steps: {ms_per_step * 1e3:.1f} us/step "
          f"(host wall {wall / steps * 1e6:.1f} us/step)", file=sys.stderr, flush=True)
    kern, instr_ms = {}, None
    if kernel_timer:
        timer = ss.Timer(max_launches=steps * 16 + 16)
        torch.cuda.synchronize()
        evk0, evk1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        evk0.record(stream)
        for i in range(steps):
            sorter(d, stream, timer=timer)
        evk1.record(stream)
        torch.cuda.synchronize()
        instr_ms = evk0.elapsed_time(evk1) / steps
        for name, kind in (("clear", _abi.SS_KERNEL_CLEAR), ("count", _abi.SS_KERNEL_COUNT_DUP),
                           ("digit_bases", _abi.SS_KERNEL_DIGIT_BASES), ("depth_pass", _abi.SS_KERNEL_DEPTH_PASS),
                           ("expand", _abi.SS_KERNEL_EXPAND), ("sort_pass", _abi.SS_KERNEL_SORT_PASS),
                           ("ranges", _abi.SS_KERNEL_RANGES), ("tile_sort", _abi.SS_KERNEL_TILE_SORT)):
            ms, n = timer.read(kind)
            if n:
                kern[name] = {"launches": n, "avg_us": 1e3 * ms / n, "us_per_step": 1e3 * ms / steps}
        timer.close()
    return {"spec": spec, "seed": seed, "rec": rec, "d": d, "M": M, "sorter": sorter, "key32": key32,
            "step_ms": step_ms, "ms_per_step": ms_per_step, "wall_s": wall, "kernels": kern,
            "instrumented_ms_per_step": instr_ms}


def frame_parity(t) -> bool:
    """The timed frame's GPU output against the oracle, pair for pair."""
    import oracle
    spec, rec, M, sorter = t["spec"], t["rec"], t["M"], t["sorter"]
    res = (oracle.sort_frame_key32(spec.width, spec.height, rec) if t["key32"]
           else oracle.sort_frame(spec.width, spec.height, rec, stages=False))
    keys_gpu = sorter.out.keys.cpu().numpy().view(np.uint64)[:M]
    vals_gpu = sorter.out.values.cpu().numpy().view(np.uint32)[:M]
    rng_gpu = sorter.out.tile_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    return bool(res.num_pairs == M and np.array_equal(res.keys, keys_gpu)
                and np.array_equal(res.values, vals_gpu) and np.array_equal(res.ranges, rng_gpu))


def batch_vs_plain(args, dev, stream, steps: int, warmup: int) -> dict:
    """The 64-frame batch as one segmented sort (eager, and replayed from an
    autotuned graph) against the same frames as 64 plain per-frame launches,
    with every frame's plain output compared to its batch segment."""
    import torch
    import paper_2511_16298_amd as ss

    frames = synth.make_batch(64)
    recs = [ss.records_to_device(r, dev) for (_, _, r) in frames]
    ms = []
    for (w, h, _), d in zip(frames, recs):
        _, _, m, st = ss.count_pairs(d, w, h)
        assert int(st.item()) == 0
        ms.append(int(m.item()))
    total = sum(ms)
    shapes = [(w, h, len(r)) for (w, h, r) in frames]
    print(f"# batch-64: N={sum(s[2] for s in shapes)}, M={total}", file=sys.stderr, flush=True)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(stream)
        for i in range(steps):
            fn()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
        return ev[0].elapsed_time(ev[steps]) / steps, per

    eager = ss.BatchSorter(shapes, total, device=dev)
    t_eager, _ = timed(lambda: eager(recs, stream))
    assert eager.result() == (0, total)
    del eager
    gsorter = ss.BatchSorter(shapes, total, device=dev, plan_workspace=True)
    plan = ss.Plan(gsorter, recs, autotune=True, stream=stream)
    t_graph, per_graph = timed(lambda: plan.launch(stream))
    assert gsorter.result() == (0, total)
    plain = [ss.FrameSorter(w, h, n, m, device=dev) for (w, h, n), m in zip(shapes, ms)]

    def run_plain():
        for so, d in zip(plain, recs):
            so(d, stream)
    t_plain, per_plain = timed(run_plain)
    base = gsorter.frame_pair_base.cpu().numpy().astype(np.int64)
    gk = gsorter.keys.cpu().numpy().view(np.uint64)
    gv = gsorter.values.cpu().numpy().view(np.uint32)
    same = True
    for f, so in enumerate(plain):
        k = so.out.keys.cpu().numpy().view(np.uint64)[:ms[f]]
        v = so.out.values.cpu().numpy().view(np.uint32)[:ms[f]]
        tb = np.uint64(int(gsorter.tile_base[f])) << np.uint64(32)
        seg = slice(int(base[f]), int(base[f]) + ms[f])
        same &= bool(np.array_equal(gk[seg] - tb, k) and np.array_equal(gv[seg], v))
    cfg = plan.config()
    plan.close()
    return {"frames": 64, "num_pairs": total, "num_gaussians": int(sum(s[2] for s in shapes)),
            "graph_ms": t_graph, "eager_ms": t_eager, "plain_64_launches_ms": t_plain,
            "batch_graph_pairs_per_s": total / (t_graph * 1e-3),
            "batch_eager_pairs_per_s": total / (t_eager * 1e-3),
            "plain_64_launches_pairs_per_s": total / (t_plain * 1e-3),
            "speedup_vs_plain": t_plain / t_graph,
            "latency_ms": {"p50": pct(per_graph, 50), "p99": pct(per_graph, 99)},
            "autotuned": cfg, "outputs_identical": bool(same), "steps": steps}


def bench_batch(args):
    """64 uneven frames: one segmented sort (eager, and captured in an
    autotuned graph) against 64 plain per-frame launches, same outputs."""
    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    b = batch_vs_plain(args, dev, torch.cuda.current_stream(), args.steps, args.warmup)
    line = {"metric": "sorted key-value pairs/s, 64-frame segmented batch vs 64 plain launches",
            "value": b["batch_graph_pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": b["graph_ms"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "batch-64: 64 frames, resolution uniform over 640x360/1280x720/1920x1080, "
                                   "N log-uniform in [5e4, 2e6], seed 1003", "num_pairs": b["num_pairs"],
                       "parallelism": "single GPU"}}
    line.update(b)
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args.workload, profiled_args=args.profiled_args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs on a single GPU (the sort of one frame runs "
              "on one device, and frames or tile-row bands would shard across GPUs without exchanging "
              "keys); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload in ("batch-64", "serve", "sweep", "render", "preprocess", "shard-large-6m"):
        {"batch-64": bench_batch, "serve": bench_serve, "sweep": bench_sweep,
         "render": bench_render, "preprocess": bench_preprocess, "shard-large-6m": bench_shard}[args.workload](args)
        return

    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    calibration_copy(args, dev, stream)
    t = time_frame(args, args.workload, args.steps, args.warmup, dev, stream)
    spec, seed, rec, M, sorter = t["spec"], t["seed"], t["rec"], t["M"], t["sorter"]
    tx, ty, key_bits = sorter.tiles_x, sorter.tiles_y, sorter.key_bits
    rb = args.radix_bits or 8
    K, ms_per_step, step_ms, kern = args.steps, t["ms_per_step"], t["step_ms"], t["kernels"]
    N = len(rec)
    pass_us = kern["sort_pass"]["avg_us"]
    pass_bytes = 24.0 * M                       # read + write of (u64 key, u32 value) per pair
    achieved = pass_bytes / (pass_us * 1e-6) / 1e9
    step_bytes, direct_bytes, tile_passes, packed = step_bytes_model(N, M, tx, ty, key_bits, rb)
    if (packed and args.algorithm == "depth-first" and args.radix_bits in (0, 8) and args.items in (0, 8, 16)
            and args.wg in (0, 512)):
        # packed pairs: the first Pt - 1 passes move 8-byte items (16 B per
        # pair), the last reads 8 and writes 12; per launch on average
        pass_bytes = (16.0 * (tile_passes - 1) + 20.0) / tile_passes * M
        achieved = pass_bytes / (pass_us * 1e-6) / 1e9
    else:
        packed = False
    pairs_per_s = M / (ms_per_step * 1e-3)
    p50 = pct(step_ms, 50)
    line = {
        "metric": "sorted key-value pairs/s (HBM-roofline %) + p50/p99 frame-sort latency",
        "value": pairs_per_s,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {spec.width}x{spec.height} image, 16x16 tiles "
                               f"({tx}x{ty}={tx * ty}), N={N} projected Gaussians, seed {seed}",
                   "num_pairs": M, "key_bits": key_bits, "radix_bits": rb, "path": args.algorithm,
                   "depth_passes": kern.get("depth_pass", {}).get("launches", 0) // K,
                   "tile_passes": tile_passes, "packed_pairs": packed, "parallelism": "single GPU"},
        "latency_ms": {"p50": p50, "p99": pct(step_ms, 99), "max": max(step_ms)},
        # the dominant kernel of the step: the 64-bit-key (tile) sort pass
        "roofline": {"bound": "hbm", "kernel": "sort_pass", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": profiled_traffic(args.workload),
                     "bytes_per_launch": pass_bytes, "avg_launch_us": pass_us},
        # the whole step: the running path's algorithmic bytes over the p50
        # step time (HIP events), and the plain method's bytes at that time
        "step_roofline": {"path": "depth-first", "bytes": step_bytes, "p50_ms": p50,
                          "GB/s": step_bytes / (p50 * 1e-3) / 1e9,
                          "frac": step_bytes / (p50 * 1e-3) / 1e9 / PEAK_HBM_GBS,
                          "direct_path_bytes": direct_bytes,
                          "direct_path_effective_frac": direct_bytes / (p50 * 1e-3) / 1e9 / PEAK_HBM_GBS},
        "kernels": kern,
        "instrumented_ms_per_step": t["instrumented_ms_per_step"],
        "host_wall_us_per_step": t["wall_s"] / K * 1e6,
    }
    prof = profiled_record(args.workload)
    if prof and prof.get("step_measured") and args.algorithm == "depth-first" and not args.radix_bits:
        # whole-step HBM bytes measured by the counters (committed profile of
        # this source) over the summed kernel time of the step
        line["step_measured"] = prof["step_measured"]

    if not args.no_cpu_baseline:
        import oracle
        line["parity_vs_oracle"] = frame_parity(t)
        key32 = t["key32"]
        frames, spent = 0, 0.0
        while spent < args.cpu_seconds or frames == 0:
            t0 = time.perf_counter()
            res = (oracle.sort_frame_key32(spec.width, spec.height, rec) if key32
                   else oracle.sort_frame(spec.width, spec.height, rec, stages=False))
            spent += time.perf_counter() - t0
            frames += 1
        line["cpu_baseline"] = {"value": frames * M / spent, "unit": "pairs/s", "cores": 1, "kind": "oracle",
                                "sample": f"{frames} whole {args.workload} frames ({spent:.1f} s, "
                                          f"single-threaded oracle on {cpu_model()}, "
                                          f"{os.cpu_count()} host CPUs visible)"}
        if not key32:
            # the oracle's steps one at a time on one thread (median of three
            # runs of the frame), and the stage outputs checked against the
            # whole-frame call
            st_ms = {"count": [], "scan": [], "duplicate": [], "sort": [], "ranges": []}
            for _ in range(3):
                t0 = time.perf_counter(); cnt, _r = oracle.count(spec.width, spec.height, rec)
                st_ms["count"].append(time.perf_counter() - t0)
                t0 = time.perf_counter(); off, tot = oracle.scan(cnt)
                st_ms["scan"].append(time.perf_counter() - t0)
                t0 = time.perf_counter(); uk, uv = oracle.duplicate(spec.width, spec.height, rec, off, tot)
                st_ms["duplicate"].append(time.perf_counter() - t0)
                t0 = time.perf_counter(); sk, sv = oracle.sort_pairs(uk, uv)
                st_ms["sort"].append(time.perf_counter() - t0)
                t0 = time.perf_counter(); rg = oracle.ranges(sk, tx * ty)
                st_ms["ranges"].append(time.perf_counter() - t0)
                del uk, uv
            stages_same = (tot == M and np.array_equal(sk, res.keys) and np.array_equal(sv, res.values)
                           and np.array_equal(rg, res.ranges))
            del sk, sv
            line["cpu_baseline_stages_ms"] = {k: round(1e3 * float(np.median(v)), 2) for k, v in st_ms.items()}
            line["cpu_baseline_stages_ms"]["same_result_as_oracle"] = bool(stages_same)
            # the same oracle steps on all the host threads this job may use
            # (OpenMP count/duplicate, parallel-mode stable sort), checked
            # against the plain oracle's result before it is timed
            threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
            mt = oracle.sort_frame_mt(spec.width, spec.height, rec, threads)
            same = (mt.status == res.status and np.array_equal(mt.keys, res.keys)
                    and np.array_equal(mt.values, res.values) and np.array_equal(mt.ranges, res.ranges))
            del mt
            mframes, mspent = 0, 0.0
            while mspent < args.cpu_seconds / 4 or mframes < 3:
                t0 = time.perf_counter()
                oracle.sort_frame_mt(spec.width, spec.height, rec, threads)
                mspent += time.perf_counter() - t0
                mframes += 1
            line["cpu_baseline_parallel"] = {
                "value": mframes * M / mspent, "unit": "pairs/s", "cores": threads, "kind": "oracle-threaded",
                "same_result_as_oracle": bool(same),
                "sample": f"{mframes} whole {args.workload} frames ({mspent:.1f} s, oracle steps with OpenMP "
                          f"count/duplicate and a parallel-mode stable sort on {threads} threads)"}
        else:
            # how lossy the normalised key is on this frame: pairs whose position
            # differs from the exact (tile, depth, index) order
            ex = oracle.sort_frame(spec.width, spec.height, rec, stages=False)
            vals_gpu = sorter.out.values.cpu().numpy().view(np.uint32)[:M]
            line["key32_pairs_out_of_exact_order"] = float(np.mean(ex.values != vals_gpu))
        del res
    del t

    if args.workload == DEFAULT_WORKLOAD and not args.no_extras and args.algorithm == "depth-first":
        # the other single-frame workloads (p50/p99 over at least 200 steps),
        # and the 64-frame batch against 64 plain launches
        others = {}
        for wl in ("fullhd-1m", "small-256x256"):
            steps = max(K, 200)
            o = time_frame(args, wl, steps, max(args.warmup, 20), dev, stream, kernel_timer=False)
            sb, _, _, _ = step_bytes_model(len(o["rec"]), o["M"], o["sorter"].tiles_x, o["sorter"].tiles_y,
                                           o["sorter"].key_bits)
            p50o = pct(o["step_ms"], 50)
            others[wl] = {"num_pairs": o["M"], "num_gaussians": len(o["rec"]), "steps": steps,
                          "pairs_per_s": o["M"] / (o["ms_per_step"] * 1e-3), "ms_per_step": o["ms_per_step"],
                          "latency_ms": {"p50": p50o, "p99": pct(o["step_ms"], 99)},
                          "host_wall_us_per_step": o["wall_s"] / steps * 1e6,
                          "step_frac_of_peak": sb / (p50o * 1e-3) / 1e9 / PEAK_HBM_GBS,
                          "parity_vs_oracle": frame_parity(o)}
            del o
        line["other_frames"] = others
        torch.cuda.empty_cache()
        bsteps = max(3, min(K, 10))
        line["batch_64"] = batch_vs_plain(args, dev, stream, bsteps, min(args.warmup, 3))
        torch.cuda.empty_cache()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
