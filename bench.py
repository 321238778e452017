#!/usr/bin/env python3
"""Benchmark: weighted elements hashed per second at m = 1024.

One step hashes the mixed-size workload (100,000 weighted sets, sizes
log-uniform in [1, 10^4], 20% of ids from a shared pool of 10^6, Pareto(1.5)
weights normalised per set, ~1.09e8 elements) with ProbMinHash1 and with
ProbMinHash3 in the batched persistent launch, inputs resident in HBM.
Also reported: the one-launch-per-set (plain) form on the same inputs; the
plain workload of 1,000 sets x 100 elements at m = 256; p50 / p99 / p99.9
latency of the continuous-batching server under Poisson arrivals at 50k
requests/s (ProbMinHash3, m = 1024, sizes log-uniform in [10, 10^5], 20,000
warm-up and 200,000 measured requests); 10^6 sets x 1,000 Zipf-popular ids at
m = 4096 (ProbMinHash1 vs ProbMinHash3, ten launches of 10^5 sets) with
all-pairs counting over its first 20,000 signatures; the heavy-skew batch for
all four variants with their rooflines; the P-MinHash break-even study;
binary weights; incremental updates; the roofline of the dominant kernel and
the CPU reference on host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    PMH_LIB=stats python bench.py --points-summary   # writes the committed
        points-generated summary with the statistics build (libpmh_stats.so)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M = 1024
SEED = 0x5EED
VARIANTS = (1, 3)
# VALU instructions per algorithmic unit on gfx950, counted on the common path
# of this library's own primitives in their compiled ISA (constants hoisted, the
# rare branches -- Lemire redraw, truncated-exponential rejection, accumulator
# above 2^52 -- left out): an element needs its weight check, 1/w and key hash
# (32) and its first point; a point below the final stop limit needs its word
# hash, value, key, label and one LDS min (ProbMinHash1 62 with the Exp(1)
# logarithm and the fixed-point step, ProbMinHash3 33 with the
# truncated-exponential fast path).
# ProbMinHash2/4 add to ProbMinHash1/3 what probe kernels of one point
# differ by in the compiled ISA: the beta_i multiply and the Fisher-Yates
# step's address arithmetic (its table reads and write are LDS instructions):
# 3 and 1 VALU instructions.
OPS_PER_ELEMENT = {1: 32 + 62, 2: 32 + 65, 3: 32 + 33, 4: 32 + 34}
OPS_PER_POINT = {1: 62, 2: 65, 3: 33, 4: 34}
# P-MinHash: VALU instructions per (element, component) pair in its inner loop
# (word hash, Exp(1) by the stream logarithm, scaling, key, running minimum),
# counted in the compiled gfx950 ISA of k_pmin.
OPS_PER_PMIN_PAIR = 48
BREAK_EVEN_N = (1, 2, 5, 10, 20, 50, 100, 200, 500, 1000)
BREAK_EVEN_SETS = 2000
PEAK_VALU = 256 * 64 * 2.4e9          # lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
PEAK_HBM = 8.0e12                     # bytes/s


def harmonic(n):
    return float(np.sum(1.0 / np.arange(1, n + 1)))


KERNEL_SOURCES = ("paper_1911_00675_amd/csrc/pmh_kernels.hip", "paper_1911_00675_amd/csrc/pmh_internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_hash_persistent_mixed_sizes_m1024_traffic.json")
POINTS_FILE = os.path.join(ROOT, "profiles", "k_hash_persistent_points.json")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(variant, num_sets):
    """HBM bytes per launch of the hash kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, scaled by the counters' reading for a copy
    of known size; None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, "no committed counter summary"
    if t.get("kernel_source_sha256") != kernel_source_sha():
        return None, "kernel changed since the counters were taken"
    if t.get("num_sets") != num_sets:
        return None, "counters were taken on another workload size"
    k = t["kernels"].get(f"pmh{variant}")
    if k is None:
        return None, "no counters for this variant"
    cal = t["calibration"]
    return (k["fetch_kib"] * 1024.0 * cal["fetch_factor"] + k["write_kib"] * 1024.0 * cal["write_factor"],
            f"rocprofv3 FETCH_SIZE x {cal['fetch_factor']:.3f} + WRITE_SIZE x {cal['write_factor']:.3f} "
            f"(copy calibration), {os.path.relpath(TRAFFIC_FILE, ROOT)}")


def committed_points():
    """Points generated per set, from the committed statistics-build summary,
    or None when the kernel sources changed since it was taken."""
    try:
        with open(POINTS_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_sha():
        return None
    return t


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def traffic_summary(fetch_dir, write_dir, out_path):
    """HBM bytes of the hash kernel from two rocprofv3 runs of
    `bench.py --profile --steps 1 --warmup 0 --copy-calibrate` (FETCH_SIZE,
    then WRITE_SIZE, csv output): per-dispatch KiB of the last dispatch of each
    variant's k_hash_persistent, scaled by the counters' reading for the 1 GiB
    device copy; written with the kernel sources' hash."""
    import csv
    import glob

    def per_dispatch(d, counter):
        vals = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for row in csv.DictReader(fh):
                    if row.get("Counter_Name") != counter:
                        continue
                    key = (int(row["Dispatch_Id"]), row["Kernel_Name"], int(row["Grid_Size"]))
                    vals[key] = vals.get(key, 0.0) + float(row["Counter_Value"])
        return vals

    out = {"kernel": "k_hash_persistent", "workload": "mixed_sizes (100,000 sets, 1.089e8 elements), m=1024",
           "num_sets": 100000, "kernel_source_sha256": kernel_source_sha(),
           "commands": ["cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out> "
                        "-o run -- python3 <repo>/bench.py --profile --steps 1 --warmup 0 --copy-calibrate",
                        "cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out> "
                        "-o run -- python3 <repo>/bench.py --profile --steps 1 --warmup 0 --copy-calibrate",
                        "python bench.py --traffic-summary <fetch out> <write out>"],
           "kernels": {}}
    cal = {}
    for counter, d, key in (("FETCH_SIZE", fetch_dir, "fetch"), ("WRITE_SIZE", write_dir, "write")):
        vals = per_dispatch(d, counter)
        # the calibration copies: the copy dispatches of the largest grid (the
        # uploads of the inputs are copies too, of other sizes)
        grid = max(g for (i, k, g) in vals if "copyBuffer" in k)
        copies = [v for (i, k, g), v in sorted(vals.items()) if "copyBuffer" in k and g == grid]
        cal[f"copy_{key}_kib"] = float(np.mean(copies))
        for variant in (1, 3):
            ks = [v for (i, k, g), v in sorted(vals.items()) if f"k_hash_persistent<{variant}," in k]
            out["kernels"].setdefault(f"pmh{variant}", {})[f"{key}_kib"] = ks[-1]
    gib = float(1 << 30)
    out["calibration"] = {"copy_bytes": int(gib), **cal, "fetch_factor": gib / 1024.0 / cal["copy_fetch_kib"],
                          "write_factor": gib / 1024.0 / cal["copy_write_kib"]}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


def points_summary(out_path):
    """Statistics build (PMH_LIB=stats): points generated per set and
    variant on the mixed and skewed batches, written to POINTS_FILE."""
    import ctypes
    import torch
    from paper_1911_00675_amd import pmh, workloads as W
    assert pmh.LIB_PATH.endswith("libpmh_stats.so"), "run with PMH_LIB=stats"
    L = pmh.lib()
    L.pmh_stats_read.restype = ctypes.c_int
    L.pmh_stats_read.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    out = {"kernel_source_sha256": kernel_source_sha(),
           "command": "python -m paper_1911_00675_amd.build --stats && PMH_LIB=stats python bench.py --points-summary",
           "counters": "lane-mode, mini-chain and chain points per set (statistics build of the same kernels)",
           "workloads": {}}
    for name, gen, m in (("mixed_sizes", W.mixed_sizes, 1024), ("skewed", W.skewed, 4096)):
        b = gen()
        ids, w, off = pmh.to_device(b.ids), pmh.to_device(b.weights), pmh.to_device(b.offsets)
        q = m * harmonic(m)
        nz = int((b.sizes() > 0).sum())
        res = {"m": m, "num_sets": b.num_sets, "m_H_m": q}
        for v in (1, 2, 3, 4):
            ctx = pmh.Context(SEED, m, v)
            o = ctx.alloc_outputs(b.num_sets, ("idx", "val"))
            ctx.hash_sets(ids, w, off, out=o)
            buf = np.zeros(24, dtype=np.uint64)
            torch.cuda.synchronize()
            L.pmh_stats_read(ctx._c, buf.ctypes.data, 1)
            ctx.hash_sets(ids, w, off, out=o)
            torch.cuda.synchronize()
            L.pmh_stats_read(ctx._c, buf.ctypes.data, 1)
            pts = int(buf[3]) + int(buf[7]) + int(buf[10])  # lane, mini-chain and chain points
            res[f"pmh{v}"] = {"points_per_set": pts / nz, "over_m_H_m": pts / (nz * q),
                              "rounds_per_item": int(buf[1]) / max(int(buf[0]), 1)}
            ctx.close()
        out["workloads"][name] = res
        log(f"points: {name} {res}")
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    # the first launches of a process run a few percent slower (clocks still
    # ramping): ten untimed steps (about 0.1 s) reach the steady state
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--sets", type=int, default=100_000)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-break-even", action="store_true")
    ap.add_argument("--no-allpairs", action="store_true")
    ap.add_argument("--no-binary", action="store_true")
    ap.add_argument("--no-update", action="store_true")
    ap.add_argument("--no-skewed", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuned timings of the skewed batch (profiled runs)")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=200_000, help="measured requests (after 20,000 warm-up)")
    ap.add_argument("--serving-pool", type=int, default=20_000, help="distinct requests the arrivals draw from")
    ap.add_argument("--large-chunks", type=int, default=10, help="launches of 10^5 sets of the 10^6-set workload")
    ap.add_argument("--cpu-sets", type=int, default=20_000)
    ap.add_argument("--cpu-single-sets", type=int, default=2_000)
    ap.add_argument("--points-summary", nargs="?", const=POINTS_FILE, default=None, metavar="OUT",
                    help="statistics build only: write the points-generated summary (default: profiles/)")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"),
                    help="write the HBM traffic summary from two rocprofv3 counter runs")
    ap.add_argument("--profile", action="store_true", help="short run for profilers: no plain/serving/cpu legs")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="also run a 1 GiB device-to-device copy (3 times) to calibrate HBM byte counters")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.points_summary:
        points_summary(args.points_summary)
        return
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.profile:
        args.no_plain = args.no_serving = args.no_cpu = args.no_break_even = args.no_allpairs = True
        args.no_binary = args.no_update = args.no_skewed = args.no_small = args.no_large = True
    import torch
    from paper_1911_00675_amd import pmh, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.time()
    b = W.mixed_sizes(num_sets=args.sets)
    log(f"workload: {b.num_sets} sets, {b.num_elements} elements ({time.time() - t0:.1f}s to generate)")
    ids, w, off = pmh.to_device(b.ids), pmh.to_device(b.weights), pmh.to_device(b.offsets)
    S, N = b.num_sets, b.num_elements
    ctxs = {v: pmh.Context(SEED, M, v) for v in VARIANTS}
    outs = {v: ctxs[v].alloc_outputs(S, ("idx", "val", "id")) for v in VARIANTS}
    stream = torch.cuda.current_stream()

    def step(events=None):
        for v in VARIANTS:
            if events is not None:
                events[v][0].record(stream)
            ctxs[v].hash_sets(ids, w, off, out=outs[v])
            if events is not None:
                events[v][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for v in VARIANTS:
        assert ctxs[v].status() == pmh.PMH_OK
    ev = [{v: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for v in VARIANTS}
          for _ in range(args.steps)]
    for v in VARIANTS:  # HIP events around the persistent hash kernel itself, on the launch stream
        ctxs[v].timing_begin(args.steps)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    call_ms = {v: float(np.mean([e[v][0].elapsed_time(e[v][1]) for e in ev])) for v in VARIANTS}
    launch_ms = {v: float(np.mean(ctxs[v].timing_read(args.steps))) for v in VARIANTS}
    ms_per_step = elapsed * 1e3 / args.steps
    value = len(VARIANTS) * N / (elapsed / args.steps)
    log(f"batched: {ms_per_step:.3f} ms/step, per call {call_ms}, hash kernel {launch_ms}")
    if args.copy_calibrate:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ------------------------------------------------------------ roofline
    sizes = b.sizes()
    nz = sizes > 0
    q = M * harmonic(M)
    units_e = int(sizes.sum())
    units_p = float(q * nz.sum())
    roof = {}
    for v in VARIANTS:
        ops = units_e * OPS_PER_ELEMENT[v] + units_p * OPS_PER_POINT[v]
        roof[v] = ops / (launch_ms[v] * 1e-3)
    dom = max(VARIANTS, key=lambda v: launch_ms[v])
    hbm_bytes = 16.0 * N + 8.0 * (S + 1) + 20.0 * S * M
    traffic, traffic_note = measured_traffic(dom, S)
    roofline = {
        "bound": "alu", "kernel": f"k_hash_persistent<ProbMinHash{dom}>",
        "achieved": roof[dom] / 1e12, "peak": PEAK_VALU / 1e12, "unit": "TOP/s",
        "frac": roof[dom] / PEAK_VALU, "traffic": traffic, "traffic_note": traffic_note,
        "launch_ms": launch_ms[dom], "timing": "HIP events around the persistent kernel on its stream",
        "ops_model": {"per_element": OPS_PER_ELEMENT[dom], "per_point": OPS_PER_POINT[dom],
                      "elements": units_e, "points": units_p,
                      "points_rule": "m*H_m per non-empty set (points below the final stop limit)"},
        "per_variant_frac": {f"pmh{v}": roof[v] / PEAK_VALU for v in VARIANTS},
        "hbm_algorithmic_GBps": hbm_bytes / (launch_ms[dom] * 1e-3) / 1e9,
        "hbm_frac": hbm_bytes / (launch_ms[dom] * 1e-3) / PEAK_HBM,
    }
    pts = committed_points()
    if pts and pts["workloads"].get("mixed_sizes", {}).get("num_sets") == S:
        wm = pts["workloads"]["mixed_sizes"]
        roofline["points_generated"] = {
            f"pmh{v}": {"per_set": wm[f"pmh{v}"]["points_per_set"], "over_m_H_m": wm[f"pmh{v}"]["over_m_H_m"]}
            for v in (1, 2, 3, 4)}
        roofline["points_generated_note"] = f"statistics build, {os.path.relpath(POINTS_FILE, ROOT)}"
    else:
        roofline["points_generated"] = None
        roofline["points_generated_note"] = "kernel changed since the points summary was taken"

    # ------------------------------------------------------------ plain form
    plain = None
    if not args.no_plain:
        plain = {}
        for v in VARIANTS:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctxs[v].hash_sets(ids, w, off, out=outs[v], mode="plain")
            e1.record(stream)
            torch.cuda.synchronize()
            pms = e0.elapsed_time(e1)
            plain[f"pmh{v}"] = {"ms": pms, "elements_per_s": N / (pms * 1e-3),
                                "batched_over_plain": pms / launch_ms[v]}
        log(f"plain: {plain}")

    # --------------------------------------------- plain workload, m = 256
    # 1,000 sets x 100 elements, ProbMinHash1: one launch per set (the form the
    # workload is quoted in) and one batched launch.
    small = None
    if not args.no_small:
        sb = W.plain_pairs()
        sctx = pmh.Context(SEED, 256, 1)
        sd = [pmh.to_device(a) for a in (sb.ids, sb.weights, sb.offsets)]
        so = sctx.alloc_outputs(sb.num_sets, ("idx", "val"))
        small = {"num_sets": sb.num_sets, "num_elements": sb.num_elements, "m": 256, "variant": "ProbMinHash1"}
        for mode in ("plain", "batched"):
            sctx.hash_sets(*sd, out=so, mode=mode)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                sctx.hash_sets(*sd, out=so, mode=mode)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            small[mode] = {"ms": ms, "elements_per_s": sb.num_elements / (ms * 1e-3),
                           "components_per_s": sb.num_sets * 256 / (ms * 1e-3)}
        if sctx.status() != pmh.PMH_OK:
            raise RuntimeError("plain-workload leg: bad status")
        small["plain_over_batched"] = small["plain"]["ms"] / small["batched"]["ms"]
        sctx.close()
        log(f"small: {small}")

    # ------------------------------------------------------------ serving
    # Poisson arrivals at 50,000 requests/s, 20,000 warm-up then the measured
    # requests; the arrivals draw their sets from a pool of distinct requests
    # staged once in pinned host memory (2.4e9 elements of fresh requests
    # would not fit it), each request copied in, hashed and copied out anew.
    latency = None
    if not args.no_serving:
        warm = 20_000
        num = warm + args.serving_requests
        rq = W.serving_requests(num_requests=args.serving_pool)
        rng = np.random.default_rng(44)
        order = rng.integers(0, rq.num_sets, size=num)
        arrival = np.cumsum(rng.exponential(1.0 / rq.meta["rate"], size=num))
        srv = pmh.Server(ctxs[3], slots=4, slot_elems=1 << 23, slot_sets=4096)
        lat, wall = srv.replay_indexed(rq.ids, rq.weights, rq.offsets, order, arrival)
        st = srv.stats()
        srv.close()
        lm = lat[warm:] * 1e6
        n_el = float(rq.sizes()[order].sum())
        latency = {"p50_us": float(np.percentile(lm, 50)), "p99_us": float(np.percentile(lm, 99)),
                   "p999_us": float(np.percentile(lm, 99.9)), "max_us": float(lm.max()),
                   "requests": int(num - warm), "warmup_requests": warm, "distinct_requests": rq.num_sets,
                   "offered_req_per_s": rq.meta["rate"], "achieved_req_per_s": num / wall,
                   "elements_per_s": n_el / wall, "variant": "ProbMinHash3", "m": M, "server": st}
        log(f"serving: {latency}")

    # ------------------------------------------- P-MinHash break-even study
    # Sec. 4 compares the ProbMinHash variants with P-MinHash over the set
    # size n: batches of BREAK_EVEN_SETS sets of n elements (Exp(1) weights),
    # m = M, one whole call each (ordering, kernels, finishing).
    break_even = None
    if not args.no_break_even:
        bctx = {v: pmh.Context(SEED, M, v) for v in (1, 2, 3, 4)}
        times = {k: [] for k in ("pminhash", "pmh1", "pmh2", "pmh3", "pmh4")}
        pmin_kernel_ms = None
        for n in BREAK_EVEN_N:
            bb = W.random_sets(n, BREAK_EVEN_SETS, n, n, "exp")
            bi, bw, bo = pmh.to_device(bb.ids), pmh.to_device(bb.weights), pmh.to_device(bb.offsets)
            bout = bctx[1].alloc_outputs(BREAK_EVEN_SETS, ("idx", "id"))
            for name, ctx, mode in [("pminhash", bctx[1], "pminhash")] + [(f"pmh{v}", bctx[v], "batched")
                                                                            for v in (1, 2, 3, 4)]:
                ctx.hash_sets(bi, bw, bo, out=bout, mode=mode)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                if name == "pminhash" and n == BREAK_EVEN_N[-1]:
                    ctx.timing_begin(3)
                e0.record(stream)
                for _ in range(3):
                    ctx.hash_sets(bi, bw, bo, out=bout, mode=mode)
                e1.record(stream)
                torch.cuda.synchronize()
                times[name].append(e0.elapsed_time(e1) / 3)
                if name == "pminhash" and n == BREAK_EVEN_N[-1]:
                    pmin_kernel_ms = float(np.mean(ctx.timing_read(3)))
                if ctx.status() != pmh.PMH_OK:
                    raise RuntimeError(f"break-even {name} n={n}: status {ctx.status()}")
        for ctx in bctx.values():
            ctx.close()
        def break_even_n(tp, tv):
            """Smallest n from which the variant is faster at every larger n."""
            for i in range(len(BREAK_EVEN_N)):
                if all(tv[j] < tp[j] for j in range(i, len(BREAK_EVEN_N))):
                    return BREAK_EVEN_N[i]
            return None
        be = {f"pmh{v}": break_even_n(times["pminhash"], times[f"pmh{v}"]) for v in (1, 2, 3, 4)}
        pairs = BREAK_EVEN_SETS * BREAK_EVEN_N[-1] * M
        pmin_ops = pairs * OPS_PER_PMIN_PAIR / (pmin_kernel_ms * 1e-3)
        break_even = {
            "m": M, "sets_per_call": BREAK_EVEN_SETS, "n": list(BREAK_EVEN_N), "weights": "Exp(1)",
            "ms_per_call": times,
            "break_even_n": be,
            "pminhash_roofline": {"bound": "alu", "kernel": "k_pmin", "n": BREAK_EVEN_N[-1],
                                  "achieved": pmin_ops / 1e12, "peak": PEAK_VALU / 1e12, "unit": "TOP/s",
                                  "frac": pmin_ops / PEAK_VALU, "launch_ms": pmin_kernel_ms,
                                  "ops_model": {"per_pair": OPS_PER_PMIN_PAIR, "pairs": pairs}},
        }
        log(f"break-even: {break_even}")

    # ------------------------------- 10^6 sets x 1,000 ids, m = 4096, all pairs
    # The Zipf-popularity workload in ten launches of 10^5 sets (each 10^8
    # elements), ProbMinHash1 and ProbMinHash3; the sets are generated by a
    # process pool in independently seeded blocks while the GPU runs.  Then
    # eq. (3) over every pair of the first 20,000 ProbMinHash1 signatures:
    # 32-bit fingerprints of the element ids, and the b-bit reductions of
    # Sec. 1.3 (b = 1 and 4).
    large = None
    allpairs = None
    if not args.no_large:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        m5, chunk = 4096, 100_000
        per = chunk // W.LARGE_BLOCK
        lctx = {v: pmh.Context(SEED, m5, v) for v in VARIANTS}
        louts = {v: lctx[v].alloc_outputs(chunk, ("idx", "val", "id")) for v in VARIANTS}
        kern = {v: [] for v in VARIANTS}
        calls = {v: [] for v in VARIANTS}
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
        t_gen = time.time()
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            pending = ex.map(W.large_block, [5] * (args.large_chunks * per), range(args.large_chunks * per))
            for c in range(args.large_chunks):
                parts = [next(pending) for _ in range(per)]
                d = [pmh.to_device(np.concatenate([p.ids for p in parts])),
                     pmh.to_device(np.concatenate([p.weights for p in parts])),
                     pmh.to_device(np.arange(chunk + 1, dtype=np.uint64) * np.uint64(1000))]
                del parts
                for v in VARIANTS:
                    if c == 0:  # first call of the context: work buffers
                        lctx[v].hash_sets(*d, out=louts[v])
                    torch.cuda.synchronize()
                    lctx[v].timing_begin(1)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    lctx[v].hash_sets(*d, out=louts[v])
                    e1.record(stream)
                    torch.cuda.synchronize()
                    kern[v].append(float(lctx[v].timing_read(1)[0]))
                    calls[v].append(e0.elapsed_time(e1))
                    if lctx[v].status() != pmh.PMH_OK:
                        raise RuntimeError(f"large leg PMH{v}: bad status")
                if c == 0 and not args.no_allpairs:
                    ka = 20_000
                    sig_id = louts[1].id[:ka].contiguous()
                    idx1 = louts[1].idx[:ka]
                    afp = torch.where(idx1 == -1, torch.zeros_like(idx1), (sig_id & 0xFFFFFFFF).to(torch.int32))
                    afp = afp.contiguous()

                    def timed(fn, reps=3):
                        fn()
                        torch.cuda.synchronize()
                        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        a0.record(stream)
                        for _ in range(reps):
                            fn()
                        a1.record(stream)
                        torch.cuda.synchronize()
                        return a0.elapsed_time(a1) / reps

                    allpairs = {"signatures": ka, "m": m5, "pairs": ka * ka,
                                "source": "first 20,000 ProbMinHash1 signatures of the 10^6-set workload",
                                "fp32_ms": timed(lambda: pmh.allpairs_counts(afp))}
                    for bb in (1, 4):
                        packed = pmh.bbit_pack(sig_id, bb)
                        allpairs[f"b{bb}_pack_ms"] = timed(lambda: pmh.bbit_pack(sig_id, bb))
                        allpairs[f"b{bb}_ms"] = timed(lambda: pmh.bbit_allpairs(packed, m5, bb))
                        del packed
                    # the 1-bit reduction fused into the hash kernel's epilogue
                    # (pmh_hash_sets_bbit) against the same launch without it
                    fused = louts[1]
                    lctx[1].hash_sets(*d, out=fused, bbit=1)
                    torch.cuda.synchronize()
                    lctx[1].timing_begin(1)
                    lctx[1].hash_sets(*d, out=fused, bbit=1)
                    allpairs["b1_fused_hash_kernel_ms"] = float(lctx[1].timing_read(1)[0])
                    allpairs["hash_kernel_ms"] = kern[1][0]
                    fused.bbit = None
                    allpairs["component_compares_per_s"] = {
                        k.replace("_ms", ""): ka * ka * m5 / (v_ * 1e-3) for k, v_ in allpairs.items()
                        if k.endswith("_ms") and "pack" not in k and "kernel" not in k}
                    del afp, sig_id
                    log(f"allpairs: {allpairs}")
                del d
        n5 = args.large_chunks * chunk * 1000
        large = {"num_sets": args.large_chunks * chunk, "num_elements": n5, "m": m5, "launches": args.large_chunks,
                 "wall_s_incl_generation": time.time() - t_gen}
        for v in VARIANTS:
            tk, tc = float(np.sum(kern[v])), float(np.sum(calls[v]))
            large[f"pmh{v}"] = {"kernel_ms_per_launch": tk / args.large_chunks, "call_ms_per_launch": tc / args.large_chunks,
                                "elements_per_s": n5 / (tk * 1e-3),
                                "components_per_s": args.large_chunks * chunk * m5 / (tk * 1e-3),
                                "elements_per_s_whole_calls": n5 / (tc * 1e-3)}
            lctx[v].close()
        del louts
        log(f"large: {large}")

    # ------------------------------------------- binary-weight specialisations
    # Sec. 2.9: the same mixed batch without weights (every weight 1), each
    # variant's persistent kernel timed weighted (unit weights) and binary.
    binary = None
    if not args.no_binary:
        ones = torch.ones_like(w)
        binary = {}
        for v in (1, 2, 3, 4):
            bc = ctxs[v] if v in ctxs else pmh.Context(SEED, M, v)
            bo = outs[v] if v in outs else bc.alloc_outputs(S, ("idx", "val", "id"))
            res = {}
            for name, wts, mode in (("weighted_ms", ones, "batched"), ("binary_ms", None, "binary")):
                bc.hash_sets(ids, wts, off, out=bo, mode=mode)
                bc.timing_begin(3)
                for _ in range(3):
                    bc.hash_sets(ids, wts, off, out=bo, mode=mode)
                res[name] = float(np.mean(bc.timing_read(3)))
                if bc.status() != pmh.PMH_OK:
                    raise RuntimeError(f"binary leg PMH{v} {mode}: status {bc.status()}")
            res["binary_elements_per_s"] = N / (res["binary_ms"] * 1e-3)
            res["weighted_over_binary"] = res["weighted_ms"] / res["binary_ms"]
            binary[f"pmh{v}"] = res
            if v not in ctxs:
                bc.close()
        del ones
        log(f"binary: {binary}")

    # ------------------------------------------------ incremental signatures
    # The mixed batch arriving in two calls (the first half of every set's
    # elements, then the second): pmh_update_sets twice against one
    # pmh_hash_sets call, persistent kernel time and whole calls.
    update = None
    if not args.no_update:
        sizes_u = b.sizes().astype(np.int64)
        local = np.arange(N, dtype=np.int64) - np.repeat(b.offsets[:-1].astype(np.int64), sizes_u)
        first = local < np.repeat(sizes_u // 2, sizes_u)
        halves = []
        for sel, cnt in ((first, sizes_u // 2), (~first, sizes_u - sizes_u // 2)):
            ho = np.concatenate([[0], np.cumsum(cnt)]).astype(np.uint64)
            halves.append((pmh.to_device(b.ids[sel]), pmh.to_device(b.weights[sel]), pmh.to_device(ho)))
        update = {"calls": 2, "split": "first half of every set, then the second"}
        for v in VARIANTS:
            st = ctxs[v].new_state(S, with_id=True)
            ctxs[v].update_sets(*halves[0], st)
            ctxs[v].update_sets(*halves[1], st)  # warm-up pair
            torch.cuda.synchronize()
            reps = 3
            ctxs[v].timing_begin(2 * reps)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                st.keys.fill_(-1)
                st.counts.zero_()
                ctxs[v].update_sets(*halves[0], st)
                ctxs[v].update_sets(*halves[1], st)
            e1.record(stream)
            torch.cuda.synchronize()
            kern = ctxs[v].timing_read(2 * reps).reshape(reps, 2)
            if ctxs[v].status() != pmh.PMH_OK:
                raise RuntimeError(f"update leg PMH{v}: status {ctxs[v].status()}")
            update[f"pmh{v}"] = {"kernel_ms_per_call": [float(kern[:, 0].mean()), float(kern[:, 1].mean())],
                                 "kernel_ms_total": float(kern.sum(axis=1).mean()),
                                 "one_call_kernel_ms": launch_ms[v],
                                 "wall_ms_two_calls": e0.elapsed_time(e1) / reps,
                                 "elements_per_s": N / (float(kern.sum(axis=1).mean()) * 1e-3)}
            del st
        del halves
        log(f"update: {update}")

    # ------------------------------------------------------- skewed batch
    # 10,000 sets, 90% of 10-100 elements and 10% of 10^5-10^6 (split across
    # workgroups), uniform(0,1] weights, m = 4096, all four variants: the
    # persistent kernel timed with HIP events, two calls each after a warm-up.
    # ProbMinHash2/4 are timed again after the autotuner has run on the batch
    # (`autotuned`: its time and the fields it changed).
    skewed = None
    if not args.no_skewed:
        sb = W.skewed()
        sids, sw, soff = pmh.to_device(sb.ids), pmh.to_device(sb.weights), pmh.to_device(sb.offsets)
        skewed = {"num_sets": sb.num_sets, "num_elements": sb.num_elements, "m": 4096}
        for v in (1, 2, 3, 4):
            sc = pmh.Context(SEED, 4096, v)
            so = sc.alloc_outputs(sb.num_sets, ("idx", "val"))
            sc.hash_sets(sids, sw, soff, out=so)
            sc.timing_begin(2)
            for _ in range(2):
                sc.hash_sets(sids, sw, soff, out=so)
            kms = float(np.mean(sc.timing_read(2)))
            if sc.status() != pmh.PMH_OK:
                raise RuntimeError(f"skewed leg PMH{v}: status {sc.status()}")
            q4 = 4096 * harmonic(4096)
            ops = sb.num_elements * OPS_PER_ELEMENT[v] + float((sb.sizes() > 0).sum()) * q4 * OPS_PER_POINT[v]
            skewed[f"pmh{v}"] = {"kernel_ms": kms, "elements_per_s": sb.num_elements / (kms * 1e-3),
                                 "waves": sc.get_tuning().waves,
                                 "roofline": {"bound": "alu", "achieved": ops / (kms * 1e-3) / 1e12,
                                              "peak": PEAK_VALU / 1e12, "unit": "TOP/s",
                                              "frac": ops / (kms * 1e-3) / PEAK_VALU,
                                              "ops_model": {"per_element": OPS_PER_ELEMENT[v],
                                                            "per_point": OPS_PER_POINT[v]},
                                              "hbm_frac": (16.0 * sb.num_elements + 12.0 * sb.num_sets * 4096)
                                              / (kms * 1e-3) / PEAK_HBM}}
            if v in (2, 4) and not args.no_autotune:
                default = sc.get_tuning().as_dict()
                sc.autotune(sids, sw, soff, trials=2)
                tuned = sc.get_tuning().as_dict()
                sc.hash_sets(sids, sw, soff, out=so)
                sc.timing_begin(2)
                for _ in range(2):
                    sc.hash_sets(sids, sw, soff, out=so)
                tms = float(np.mean(sc.timing_read(2)))
                if sc.status() != pmh.PMH_OK:
                    raise RuntimeError(f"skewed leg PMH{v} (autotuned): status {sc.status()}")
                skewed[f"pmh{v}"]["autotuned"] = {
                    "kernel_ms": tms, "elements_per_s": sb.num_elements / (tms * 1e-3),
                    "frac": ops / (tms * 1e-3) / PEAK_VALU,
                    "changed": {k: tuned[k] for k in tuned if tuned[k] != default[k]}}
            sc.close()
            del so
        del sids, sw, soff, sb
        log(f"skewed: {skewed}")

    # ------------------------------------------------------------ CPU oracle
    cpu = None
    if not args.no_cpu:
        import oracle
        oracle.build()
        cores = len(os.sched_getaffinity(0))
        samp = b.subset(np.arange(min(args.cpu_sets, S)))
        tc = {}
        for v in VARIANTS:
            c0 = time.perf_counter()
            oracle.sign_batch(v, SEED, M, samp.ids, samp.weights, samp.offsets, nthreads=cores)
            tc[v] = time.perf_counter() - c0
        cpu_val = len(VARIANTS) * samp.num_elements / sum(tc.values())
        one = b.subset(np.arange(min(args.cpu_single_sets, S)))
        t1 = {}
        for v in VARIANTS:
            c0 = time.perf_counter()
            oracle.sign_batch(v, SEED, M, one.ids, one.weights, one.offsets, nthreads=1)
            t1[v] = time.perf_counter() - c0
        cpu = {"value": cpu_val, "unit": "elements/s", "cores": cores, "kind": "oracle",
               "sample": f"first {samp.num_sets} sets ({samp.num_elements} elements) of the same workload, "
                         f"ProbMinHash1+3 sequential per set, {cores} threads (one set per task)",
               "seconds": {f"pmh{v}": tc[v] for v in VARIANTS},
               "cpu_model": cpu_model(), "compiler": "gcc " + " ".join(oracle.CFLAGS),
               "single_core": {"value": len(VARIANTS) * one.num_elements / sum(t1.values()), "unit": "elements/s",
                               "sample": f"first {one.num_sets} sets ({one.num_elements} elements), one thread",
                               "seconds": {f"pmh{v}": t1[v] for v in VARIANTS}}}
        log(f"cpu: {cpu}")

    out = {
        "metric": "weighted elements hashed/s at m=1024 (batched vs per-set launch); p99 latency",
        "value": value, "unit": "elements/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"mixed_sizes: {S} sets, sizes log-uniform [1,1e4], 20% pooled ids, "
                               f"Pareto(1.5) weights, m={M}, ProbMinHash1+ProbMinHash3, batched persistent",
                   "num_sets": S, "num_elements": N, "m": M, "variants": list(VARIANTS),
                   "per_launch_ms": {f"pmh{v}": launch_ms[v] for v in VARIANTS},
                   "per_call_ms": {f"pmh{v}": call_ms[v] for v in VARIANTS},
                   "elements_per_s": {f"pmh{v}": N / (launch_ms[v] * 1e-3) for v in VARIANTS},
                   "components_per_s": {f"pmh{v}": S * M / (launch_ms[v] * 1e-3) for v in VARIANTS}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain": plain,
        "plain_small": small,
        "latency": latency,
        "large_uniform": large,
        "break_even": break_even,
        "allpairs": allpairs,
        "binary": binary,
        "update": update,
        "skewed": skewed,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
