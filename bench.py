#!/usr/bin/env python3
"""Throughput benchmark of the bulk PRNG-stream library on one MI355X.

One step = the store-mode hot path over the bulk workload: XorShift (the
r = 8 generator of eq. (5) and the xorshift32 of eq. (6)) and KISS, each
producing 2^20 streams x 256 samples as uint32 and as FP32 uniforms, with
per-stream states seeded from SplitMix64(1), read and written back every
call.  That is 6 launches and 6 x 2^28 samples per step, inputs resident in
HBM.  The JSON line reports whole-step GSamples/s, the roofline of the
dominant kernel (HBM bytes over its duration from live HIP events around it
in the timed steps; the other launches carry no events there, since each
event adds a few microseconds to the step), the measured write-only
ceiling, side workloads (MWC32 4096 x 1024, jump-ahead split of 2^30
samples, fused pi over 2^34 KISS samples), and the serial CPU oracle timed
on a bounded sample.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-extra]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0           # MI355X HBM3E, 8 TB/s
# Full-rate 32-bit integer VALU: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz.
# The 157.3 TFLOP/s FP32 figure counts packed FP32 FMAs (2 FLOPs x 2 per lane),
# which integer work cannot use.
VALU_INT32_SPEC = 256 * 4 * 16 * 2.4e9
# Abstract operations per fused sample (eq. (9)): KISS 20 (MWC1616 10, xorshift32
# 6, LCG 2, combine 2) and about 4 for the pair test.
FUSED_OPS_PER_SAMPLE = 24

S_BULK, N_BULK = 1 << 20, 256
TUNE_REPS = 8  # timed launches per shape when the step's launch shapes are autotuned
PER_KERNEL_STEPS = 10  # untimed steps with an event at every launch boundary (per-kernel durations)
STEP_GENS = ["XS256", "XS32", "KISS"]
STEP_DTYPES = ["u32", "f32"]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-extra", action="store_true", help="skip the side workloads")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-tune", action="store_true", help="keep the library's default launch shapes")
    p.add_argument("--only", choices=["batched", "served", "split", "fused", "small", "placement", "fold"],
                   help="run one side workload alone and print its JSON record")
    p.add_argument("--profile", metavar="GEN_DTYPE",
                   help="counter-collection mode: a 1 GiB device copy (calibration) then 3 launches of "
                        "one step kernel, e.g. XS256_u32; 'counter' (the layout ceiling's kernel); or 'fused' (fused pi and "
                        "its VALU calibration); "
                        "prints nothing else")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported "
              "(streams shard by range across GPUs with no exchange)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1101_1846_amd as R

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    R.rng_init()
    stream = torch.cuda.current_stream()
    if args.only:
        print(json.dumps(side_workloads(torch, R, dev, stream, only=args.only)))
        return

    # ---------------------------------------------------------------- inputs
    states = {}
    for name in STEP_GENS:
        g = R.GENERATORS[name]
        st = torch.empty((R.rng_state_words(g), S_BULK), dtype=torch.int32, device=dev)
        R.rng_seed(g, 1, 0, S_BULK, st)
        states[name] = st
    out = torch.empty(S_BULK * N_BULK, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    launches = [(n, d) for n in STEP_GENS for d in STEP_DTYPES]

    if args.profile:
        profile_mode(torch, R, dev, states, out, args.profile)
        return

    tuned = {}
    if not args.no_tune:
        # the library's autotuner picks (workgroup, unroll) per generator and
        # dtype on this problem; untimed set-up, like any tuning cache
        for name, d in launches:
            g = R.GENERATORS[name]
            scratch = states[name].clone()
            wg, un, us = R.rng_autotune(g, R.DTYPES[d], S_BULK, N_BULK, scratch, out, TUNE_REPS)
            tuned["%s_%s" % (name, d)] = {"wg": wg, "unroll": un, "us": round(us, 1)}
            del scratch
        torch.cuda.synchronize()

    def step(events=None, only=None):
        # events at launch boundaries: launch i runs between events[i] and events[i + 1]
        # (with `only`, two events around that launch alone)
        for i, (name, d) in enumerate(launches):
            if events is not None and (only is None or i == only):
                events[0 if only is not None else i].record(stream)
            R.rng_generate(R.GENERATORS[name], states[name], S_BULK, N_BULK, R.DTYPES[d], out)
            if events is not None and (only is None or i == only):
                events[1 if only is not None else i + 1].record(stream)

    def bytes_of(name):
        return S_BULK * N_BULK * 4 + 2 * S_BULK * R.rng_state_words(R.GENERATORS[name]) * 4

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Per-kernel durations, from an untimed pass with an event at every launch
    # boundary (each event costs the step a few microseconds, so the timed
    # steps below carry events around the dominant launch only).
    KP = PER_KERNEL_STEPS
    evp = [[torch.cuda.Event(enable_timing=True) for _ in range(len(launches) + 1)] for _ in range(KP)]
    for k in range(KP):
        step(evp[k])
    torch.cuda.synchronize()
    per = {}
    for i, (name, d) in enumerate(launches):
        durs = [evp[k][i].elapsed_time(evp[k][i + 1]) for k in range(KP)]
        mean_ms = float(np.mean(durs))
        per["%s_%s" % (name, d)] = {
            "ms": round(mean_ms, 4),
            "GSamples_s": round(S_BULK * N_BULK / (mean_ms * 1e-3) / 1e9, 2),
            "GB_s": round(bytes_of(name) / (mean_ms * 1e-3) / 1e9, 1),
            "bytes": bytes_of(name),
        }
    dom_i = max(range(len(launches)), key=lambda i: per["%s_%s" % launches[i]]["ms"])
    dom_key = "%s_%s" % launches[dom_i]

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(K)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for k in range(K):
        step(ev[k], only=dom_i)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    samples_per_step = len(launches) * S_BULK * N_BULK
    value = samples_per_step * K / (ms_total * 1e-3) / 1e9

    # the dominant launch's duration in the timed steps (live events on its stream)
    dom_ms = float(np.mean([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)]))
    dom = {"ms": round(dom_ms, 4), "bytes": bytes_of(launches[dom_i][0])}
    achieved = dom["bytes"] / (dom_ms * 1e-3) / 1e9

    # ------------------------------------------------- measured write ceiling
    ceil = write_ceiling(torch, dev)
    shapes = [R.rng_get_shape(R.GENERATORS[name], R.DTYPES[d]) for name, d in launches]
    layout = layout_ceiling(torch, R, dev, out, shapes)

    extra = {} if args.no_extra else side_workloads(torch, R, dev, stream)

    cpu = None if args.no_cpu else cpu_baseline(args.cpu_seconds)

    line = {
        "metric": "GSamples/s & HBM write GB/s (% peak), bit-exact; batched p50/p99 latency",
        "value": round(value, 2),
        "unit": "GSamples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_total / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32+f32",
        "data": "synthetic: per-stream states from SplitMix64(seed=1), no dataset",
        "config": {
            "workload": "bulk store mode: XS256 (eq. 5), XS32 (eq. 6), KISS; 2^20 streams x 256 samples; "
                        "uint32 and FP32 (u>>8)*2^-24 outputs; state read+write-back per call",
            "streams": S_BULK, "samples_per_stream": N_BULK, "launches_per_step": len(launches),
            "samples_per_step": samples_per_step, "parallelism": "single GPU",
        },
        "hbm_write_GB_s": round(samples_per_step * 4 * K / (ms_total * 1e-3) / 1e9, 1),
        "frac_hbm_peak": round(samples_per_step * 4 * K / (ms_total * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "roofline": {
            "kernel": "k_generate<%s> (store mode)" % dom_key,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": measured_traffic(dom_key),
            "bytes_per_launch": dom["bytes"],
            "avg_launch_ms": dom["ms"],
        },
        "launch_shapes": tuned,
        "write_ceiling": ceil,
        "frac_of_write_ceiling": round(achieved / ceil["best_GB_s"], 4) if ceil else None,
        "layout_write_ceiling": layout,
        "frac_of_layout_ceiling": round(achieved / layout["GB_s"], 4),
        "per_kernel": per,
        "per_kernel_note": "%d untimed steps with an event at every launch boundary, before the timed steps; the "
                           "roofline's avg_launch_ms is the dominant launch's in the timed steps" % KP,
        "side_workloads": extra,
        "served_latency_us": {k: {"p50": v["p50_us"], "p99": v["p99_us"]}
                              for k, v in extra.get("served", {}).items() if isinstance(v, dict)},
        "cpu_baseline": cpu,
        "paper_reported": {
            "hardware": "NVIDIA GTX280 (GT200), CUDA 2.3",
            "GSamples_s_with_writeback": {"%s_%s" % (n, d): PAPER_WITH_WRITEBACK[n][i]
                                          for n in PAPER_WITH_WRITEBACK for i, d in enumerate(("u32", "f32"))},
            "note": "Tables II-III, about 4e7 numbers per call; context only (vs_baseline stays null)",
        },
        "wall_s_timed": round(wall, 3),
    }
    print(json.dumps(line))


def write_ceiling(torch, dev):
    """Write-only bandwidth of plain fills over 4 GiB (torch's fill kernel and
    hipMemsetD32), the paper's own practice of measuring the achievable rate."""
    import ctypes
    n = 1 << 30
    buf = torch.empty(n, dtype=torch.int32, device=dev)
    res = {}
    for _ in range(2):
        buf.fill_(7)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        buf.fill_(7)
    e1.record()
    torch.cuda.synchronize()
    res["torch_fill_GB_s"] = round(4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    try:
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemsetD32Async.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p]
        s = torch.cuda.current_stream().cuda_stream
        for _ in range(2):
            hip.hipMemsetD32Async(buf.data_ptr(), 5, n, s)
        e0.record()
        for _ in range(reps):
            hip.hipMemsetD32Async(buf.data_ptr(), 5, n, s)
        e1.record()
        torch.cuda.synchronize()
        res["hipMemsetD32_GB_s"] = round(4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    except OSError:
        pass
    res["best_GB_s"] = max(v for k, v in res.items() if k.endswith("GB_s"))
    res["bytes"] = 4 * n
    del buf
    torch.cuda.empty_cache()
    return res


def layout_ceiling(torch, R, dev, out, shapes):
    """Write rate of the generation kernel's own store schedule at the step's
    size: rng_calibrate_store runs the same resident schedule, LDS transpose
    and pipelined 16-byte stores with a counter in place of a generator (one
    state word per stream, read and written back).  Best over the step's
    launch shapes; algorithmic bytes as for a one-word generator."""
    st = torch.zeros(S_BULK, dtype=torch.int32, device=dev)
    nbytes = S_BULK * N_BULK * 4 + 2 * S_BULK * 4
    best = None
    for wg, un in sorted(set(shapes)):
        ms = _time(torch, lambda: R.rng_calibrate_store(st, S_BULK, N_BULK, out, wg, un), 20, warm=3)
        gbs = nbytes / (ms * 1e-3) / 1e9
        if best is None or gbs > best["GB_s"]:
            best = {"GB_s": round(gbs, 1), "ms": round(ms, 4), "wg": wg, "unroll": un}
    best["bytes"] = nbytes
    best["kernel"] = "k_generate<counter> (store mode, rng_calibrate_store)"
    del st
    return best


def _time(torch, fn, reps, warm=1):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def side_workloads(torch, R, dev, stream, only=None):
    """Every workload besides the timed step, or only the one named."""
    parts = {"small": small_workloads, "split": split_workload, "placement": placement_workload,
             "fold": fold_workload}
    res = {}
    if only in parts:
        res.update(parts[only](torch, R, dev))
        return res
    if only == "batched":
        res["batched_10k_requests"] = batched_workload(torch, R, dev)
        return res
    if only == "fused":
        res.update(fused_workload(torch, R, dev))
        return res
    if only == "served":
        res["served"] = served_workload(R, batched_workload(torch, R, dev)["single_large_call_GSamples_s"])
        return res
    res.update(small_workloads(torch, R, dev))
    res.update(split_workload(torch, R, dev))
    res["batched_10k_requests"] = batched_workload(torch, R, dev)
    res["served"] = served_workload(R, res["batched_10k_requests"]["single_large_call_GSamples_s"])
    res.update(fused_workload(torch, R, dev))
    res.update(placement_workload(torch, R, dev))
    res.update(fold_workload(torch, R, dev))
    torch.cuda.empty_cache()
    return res


def small_workloads(torch, R, dev):
    """MWC32 4096 streams x 1024 (launch-bound; chunked by jump-ahead) and the
    MWC1616 / MWC32 store mode at the bulk size."""
    res = {}
    g = R.RNG_MWC32
    S, N = 4096, 1024
    st = torch.empty((2, S), dtype=torch.int32, device=dev)
    R.rng_seed(g, 0, 0, S, st)
    o = torch.empty(S * N, dtype=torch.int32, device=dev)
    # the launch shape tuned for this size (rows of 4 KiB: the shape class of
    # 16 KiB runs, restored afterwards for the other workloads)
    prev = R.rng_row_shape(g, R.RNG_U32, S, N)
    scratch = torch.empty_like(st)
    R.rng_seed(g, 0, 0, S, scratch)
    wg, un, _ = R.rng_autotune(g, R.RNG_U32, S, N, scratch, o, 5)
    R.rng_set_row_shape(g, R.RNG_U32, S, N, *prev)
    ms = _time(torch, lambda: R.rng_generate_ex(g, st, S, N, R.RNG_U32, o, wg, un), 200)
    # the same call 100 times in one captured HIP graph: the device time per
    # call without the host's launch overhead
    calls = 100
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.stream(cs):
        R.rng_generate_ex(g, st, S, N, R.RNG_U32, o, wg, un, cs)  # outside the capture: lazy set-up
        torch.cuda.synchronize()
        with torch.cuda.graph(gr, stream=cs):
            for _ in range(calls):
                R.rng_generate_ex(g, st, S, N, R.RNG_U32, o, wg, un, cs)
    torch.cuda.synchronize()
    graph_ms = _time(torch, gr.replay, 10) / calls
    del gr
    res["mwc32_4096x1024"] = {"us_per_call": round(ms * 1e3, 2), "wg": wg, "unroll": un,
                              "GSamples_s": round(S * N / (ms * 1e-3) / 1e9, 1),
                              "us_per_call_in_graph": round(graph_ms * 1e3, 2),
                              "GSamples_s_in_graph": round(S * N / (graph_ms * 1e-3) / 1e9, 1)}
    for name in ("MWC1616", "MWC32"):
        g = R.GENERATORS[name]
        st = torch.empty((R.rng_state_words(g), S_BULK), dtype=torch.int32, device=dev)
        R.rng_seed(g, 1, 0, S_BULK, st)
        o = torch.empty(S_BULK * N_BULK, dtype=torch.int32, device=dev)
        for dname, d in R.DTYPES.items():
            ms = _time(torch, lambda: R.rng_generate(g, st, S_BULK, N_BULK, d, o), 10)
            res["%s_bulk_%s" % (name, dname)] = {"ms": round(ms, 4),
                                                  "GSamples_s": round(S_BULK * N_BULK / (ms * 1e-3) / 1e9, 1)}
        del o
    return res


def split_workload(torch, R, dev):
    """One 2^30-sample sequence over 2^20 threads: jump-ahead splitting, and leapfrogging."""
    res = {}
    total, T = 1 << 30, 1 << 20
    o = torch.empty(total, dtype=torch.int32, device=dev)
    for name in ("MWC32", "XS256"):
        g = R.GENERATORS[name]
        W = R.rng_state_words(g)
        s1 = torch.empty(W, dtype=torch.int32, device=dev)
        R.rng_seed(g, 2, 0, 1, s1)
        fin = torch.empty(W, dtype=torch.int32, device=dev)
        wsb = R.rng_split_workspace_bytes(g, T)
        ws = torch.empty(wsb // 4, dtype=torch.int32, device=dev)
        ms = _time(torch, lambda: R.rng_generate_split(g, s1, total, T, R.RNG_U32, o, fin, ws, wsb), 5)
        # the generation phase alone: the same launch over T states of T x (total / T) samples
        C, rows = total // T, T
        st = torch.empty((W, rows), dtype=torch.int32, device=dev)
        R.rng_seed(g, 2, 0, rows, st)
        gen_ms = _time(torch, lambda: R.rng_generate(g, st, rows, C, R.RNG_U32, o), 5)
        gen_bytes = 4 * rows * C + 2 * 4 * W * rows
        res["split_2^30_%s" % name] = {"ms": round(ms, 3),
                                       "GSamples_s": round(total / (ms * 1e-3) / 1e9, 1),
                                       "GB_s": round(4 * total / (ms * 1e-3) / 1e9, 1),
                                       "samples_per_thread": C,
                                       "generation_shape": list(R.rng_row_shape(g, R.RNG_U32, rows, C)),
                                       "generation_ms": round(gen_ms, 3),
                                       "generation_GB_s": round(gen_bytes / (gen_ms * 1e-3) / 1e9, 1),
                                       "setup_ms": round(max(ms - gen_ms, 0.0), 3)}
        del ws, st
    # jump-ahead alone: every one of 2^20 states skipped by one 64-bit distance
    # (38 set bits: 38 modular or GF(2) products per state)
    K = 0x9E3779B97F4A7C15
    for name in ("MWC32", "MWC1616", "XS32", "KISS", "XS256"):
        g = R.GENERATORS[name]
        W = R.rng_state_words(g)
        st = torch.empty((W, T), dtype=torch.int32, device=dev)
        R.rng_seed(g, 2, 0, T, st)
        ms = _time(torch, lambda: R.rng_skip(g, st, T, K), 5)
        res["skip_2^20_states_%s" % name] = {"us": round(ms * 1e3, 1),
                                             "Gjumps_s": round(T / (ms * 1e-3) / 1e9, 2),
                                             "state_GB_s": round(2 * 4 * W * T / (ms * 1e-3) / 1e9, 1)}
        del st
    # the same sequence by leapfrogging: thread j emits numbers j, j + T, ...
    for name in ("MWC32", "XS32", "KISS", "MWC1616", "XS256"):
        g = R.GENERATORS[name]
        W = R.rng_state_words(g)
        s1 = torch.empty(W, dtype=torch.int32, device=dev)
        R.rng_seed(g, 2, 0, 1, s1)
        fin = torch.empty(W, dtype=torch.int32, device=dev)
        wsb = R.rng_leapfrog_workspace_bytes(g, T)
        ws = torch.empty(wsb // 4, dtype=torch.int32, device=dev)
        ms = _time(torch, lambda: R.rng_generate_leapfrog(g, s1, total, T, R.RNG_U32, o, fin, ws, wsb), 3)
        res["leapfrog_2^30_%s" % name] = {"ms": round(ms, 3),
                                          "GSamples_s": round(total / (ms * 1e-3) / 1e9, 1),
                                          "GB_s": round(4 * total / (ms * 1e-3) / 1e9, 1)}
        del ws
    del o
    return res


# The paper's XorShift placement table on its GTX280 (GSamples/s with and without write-back for the
# implicit, explicit and register forms), quoted for context only: other hardware, its own sizes.
PAPER_TABLE2_RATE = {"lds_indexed": (4.4, 4.8), "lds_unrolled": (8.1, 13.8), "vgpr": (12.5, 14.5)}
XS256_USEFUL_OPS = 18  # useful operations per XorShift number (11 XORs, 7 shifts)


# Useful operations per number (eq. (9)'s n_ops): the paper's counts for its MWC (10), XorShift (18) and
# KISS (18); the counterparts here for the base-2^32 MWC (one 32x32+32 -> 64 multiply-add: 2) and xorshift32 (6).
USEFUL_OPS = {"MWC32": 2, "MWC1616": 10, "XS32": 6, "XS256": 18, "KISS": 18}
# The paper's GTX280 rates without write-back (integer, uniform), GSamples/s: context only.
PAPER_NO_WRITEBACK = {"MWC1616": (37.5, 23.6), "XS256": (14.5, 12.9), "KISS": (19.1, 10.3)}
# The paper's GTX280 rates with write-back (integer, uniform), GSamples/s, for the generators of the step
# (Tables II and III; its XorShift with the state in registers): context only, other hardware and sizes.
PAPER_WITH_WRITEBACK = {"XS256": (12.5, 11.5), "KISS": (9.2, 8.5)}


def fold_workload(torch, R, dev):
    """Every generator without write-back (2^20 streams x 2^12 numbers, per-stream XOR
    only) and with it (the same streams, 2^20 x 256 store mode), uint32 and FP32."""
    S = S_BULK
    res = {}
    fold = torch.zeros(S, dtype=torch.int32, device=dev)
    out = torch.empty(S * N_BULK, dtype=torch.int32, device=dev)
    for name, g in R.GENERATORS.items():
        st = torch.empty((R.rng_state_words(g), S), dtype=torch.int32, device=dev)
        R.rng_seed(g, 7, 0, S, st)
        row = {}
        for dname, d in R.DTYPES.items():
            n = 1 << 12
            ms = _time(torch, lambda: R.rng_generate_fold(g, st, S, n, d, fold), 5)
            rate = S * n / (ms * 1e-3)
            ms_wb = _time(torch, lambda: R.rng_generate(g, st, S, N_BULK, d, out), 5)
            rate_wb = S * N_BULK / (ms_wb * 1e-3)
            row[dname] = {"without_writeback_GSamples_s": round(rate / 1e9, 1),
                          "with_writeback_GSamples_s": round(rate_wb / 1e9, 1),
                          "useful_Gops_without_writeback": round(rate * USEFUL_OPS[name] / 1e9, 1)}
        if name in PAPER_NO_WRITEBACK:
            row["paper_gtx280_without_writeback_GSamples_s"] = dict(zip(("u32", "f32"), PAPER_NO_WRITEBACK[name]))
        res[name] = row
    del out
    torch.cuda.empty_cache()
    return {"without_writeback_2^20x2^12": res}


def placement_workload(torch, R, dev):
    """The XorShift state placements of the paper's Table II at 2^20 streams x 256:
    with write-back (every number stored, sample-major) and without (per-stream XOR)."""
    S, N = S_BULK, N_BULK
    st = torch.empty((8, S), dtype=torch.int32, device=dev)
    R.rng_seed(R.RNG_XS256, 1, 0, S, st)
    out = torch.empty(S * N, dtype=torch.int32, device=dev)
    fold = torch.empty(S, dtype=torch.int32, device=dev)
    res = {}
    for name, pl in R.PLACEMENTS.items():
        row = {}
        for dname, d in R.DTYPES.items():
            ms_wb = _time(torch, lambda: R.rng_xs256_placement(pl, st, S, N, d, d_out=out), 10)
            ms_nw = _time(torch, lambda: R.rng_xs256_placement(pl, st, S, N, d, d_fold=fold), 10)
            rate_wb, rate_nw = S * N / (ms_wb * 1e-3), S * N / (ms_nw * 1e-3)
            row[dname] = {"with_writeback": {"ms": round(ms_wb, 4), "GSamples_s": round(rate_wb / 1e9, 1),
                                             "GB_s": round((4 * S * N + 64 * S) / (ms_wb * 1e-3) / 1e9, 1),
                                             "useful_Gops": round(rate_wb * XS256_USEFUL_OPS / 1e9, 1)},
                          "without_writeback": {"ms": round(ms_nw, 4), "GSamples_s": round(rate_nw / 1e9, 1),
                                                "useful_Gops": round(rate_nw * XS256_USEFUL_OPS / 1e9, 1)}}
        row["paper_gtx280_GSamples_s"] = dict(zip(("with_writeback", "without_writeback"), PAPER_TABLE2_RATE[name]))
        res[name] = row
    del out
    torch.cuda.empty_cache()
    return {"xs256_placement_2^20x256": res}


def fused_workload(torch, R, dev):
    """Fused consumer over 2^34 KISS samples (no stores: integer-VALU bound),
    held against the measured ceiling of its own instruction mix (the same
    loop body on four independent streams per lane, rng_calibrate_valu op 3).
    VALU instructions per sample come from SQ_INSTS_VALU counter runs on the
    current kernel sources (profiles/valu.json), else stay null."""
    res = {}
    g = R.RNG_KISS
    S, N = 1 << 20, 1 << 14
    st = torch.empty((6, S), dtype=torch.int32, device=dev)
    R.rng_seed(g, 6, 0, S, st)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    ms = _time(torch, lambda: R.rng_fused_pi(g, st, S, N, cnt), 5)
    rate = S * N / (ms * 1e-3)
    calib = {name: R.rng_calibrate_valu(op) for op, name in enumerate(("add_xor", "mad_u24", "mul_lo"))}
    mix = max(R.rng_calibrate_valu(3) for _ in range(2))  # lane-samples/s of the fused loop's mix
    vps = measured_valu()
    fv, cv = (vps or {}).get("fused_valu_per_sample"), (vps or {}).get("calib_valu_per_sample")
    roof = {"kernel": "k_fused_pi<KISS>", "bound": "alu", "unit": "GSamples/s",
            "achieved": round(rate / 1e9, 1), "peak": round(mix / 1e9, 1), "frac": round(rate / mix, 4),
            "peak_kind": "measured: the same loop body on 1, 2, 4 or 8 independent streams per lane, the fastest "
                         "(rng_calibrate_valu op 3)",
            "abstract_ops_per_sample": FUSED_OPS_PER_SAMPLE,
            "abstract_Gop_s": round(rate * FUSED_OPS_PER_SAMPLE / 1e9, 1),
            "valu_instructions_per_sample": fv, "calib_valu_instructions_per_sample": cv,
            "int32_spec_lane_ops_per_s": VALU_INT32_SPEC,
            "measured_single_class_lane_ops_per_s": {k: round(v / 1e9, 1) for k, v in calib.items()}}
    if fv and cv:
        peak_instr = mix * cv  # lane-instructions/s the mix sustains
        roof.update({"valu_lane_instructions_per_s": round(rate * fv / 1e9, 1),
                     "peak_valu_lane_instructions_per_s": round(peak_instr / 1e9, 1),
                     "frac_valu_instructions": round(rate * fv / peak_instr, 4),
                     "frac_abstract_ops": round(rate * FUSED_OPS_PER_SAMPLE / peak_instr, 4),
                     "frac_of_int32_spec": round(rate * fv / VALU_INT32_SPEC, 4)})
    res["fused_pi_kiss_2^34"] = {"ms": round(ms, 3), "GSamples_s": round(rate / 1e9, 1), "roofline": roof}
    torch.cuda.empty_cache()
    return res


def batch_pools(torch, R, dev, tab, seed=5):
    """Per-generator state pools [words][n_g] seeded from SplitMix64(seed), and the
    (pointer, stride) of every request's stream inside them."""
    names = tab["generators"]
    pools, where = {}, []
    counts = {g: int((tab["gen"] == i).sum()) for i, g in enumerate(names)}
    for g, c in counts.items():
        if c:
            gid = R.GENERATORS[g]
            st = torch.empty((R.rng_state_words(gid), c), dtype=torch.int32, device=dev)
            R.rng_seed(gid, seed, 0, c, st)
            pools[g] = st
    seen = {g: 0 for g in names}
    for gi in tab["gen"]:
        g = names[gi]
        where.append((pools[g].data_ptr() + 4 * seen[g], counts[g], seen[g]))
        seen[g] += 1
    return pools, where


def batched_workload(torch, R, dev, reps=10):
    """10,000 independent requests (generator uniform over MWC32/XS256/KISS,
    dtype 50/50, length log-uniform in [2^8, 2^22]) in one persistent
    generation launch, its kernels launched directly (and, for comparison,
    replayed from a captured HIP graph); compared with the same samples
    generated by one large rng_generate call per (generator, dtype)."""
    from paper_1101_1846_amd import workloads as W
    tab = W.batch_table(10000, seed=4)
    names = tab["generators"]
    pools, where = batch_pools(torch, R, dev, tab)
    offs, words = W.layout_outputs(tab["length"])
    out = torch.empty(words, dtype=torch.int32, device=dev)
    base = out.data_ptr()
    reqs = [(R.GENERATORS[names[g]], int(d), p, stride, 0, int(n), base + 4 * int(o))
            for g, d, (p, stride, _), n, o in zip(tab["gen"], tab["dtype"], where, tab["length"], offs)]
    total = int(tab["length"].sum())
    h = R.rng_batch_create(len(reqs), total)
    try:
        R.rng_batch_set(h, reqs)
        wg, un, chunk, tune_us = R.rng_batch_autotune(h, reps=1)
        # the generation kernel takes 6-8 launches of a new plan to settle
        # (3.6 -> 3.15 ms in a kernel trace, in either launch mode): both
        # modes are warmed before either is timed
        for use_graph in (False, True):
            R.rng_batch_set_graph(h, use_graph)
            _time(torch, lambda: R.rng_batch_launch(h), 4, warm=4)
        R.rng_batch_set_graph(h, False)
        ms = _time(torch, lambda: R.rng_batch_launch(h), reps)
        R.rng_batch_set_graph(h, True)
        graph_ms = _time(torch, lambda: R.rng_batch_launch(h), reps)
    finally:
        R.rng_batch_destroy(h)
    # single large calls over the same per-(generator, dtype) sample counts
    single_ms = 0.0
    S = 1 << 20
    for gi, g in enumerate(names):
        gid = R.GENERATORS[g]
        st = torch.empty((R.rng_state_words(gid), S), dtype=torch.int32, device=dev)
        R.rng_seed(gid, 9, 0, S, st)
        for d in (0, 1):
            n_g = int(tab["length"][(tab["gen"] == gi) & (tab["dtype"] == d)].sum())
            N = max(64, round(n_g / S / 64) * 64)  # rows a multiple of the 64-sample tile
            single_ms += _time(torch, lambda: R.rng_generate(gid, st, S, N, d, out), 3) * n_g / (S * N)
    del out
    torch.cuda.empty_cache()
    rate = total / (ms * 1e-3) / 1e9
    single = total / (single_ms * 1e-3) / 1e9
    return {"requests": len(reqs), "samples": total, "bytes": 4 * total, "ms_per_batch": round(ms, 3),
            "GSamples_s": round(rate, 1), "GB_s": round(4 * total / (ms * 1e-3) / 1e9, 1),
            "single_large_call_GSamples_s": round(single, 1), "frac_of_single_call": round(rate / single, 4),
            "graph_replay_ms_per_batch": round(graph_ms, 3), "shape": {"wg": wg, "unroll": un, "chunk": chunk}}


# The server's worker keeps polling this long after its last activity before it
# sleeps, so that a request arriving at low load finds it awake.
SERVED_IDLE_SPIN_US = 2000


def served_workload(R, single_rate):
    """Poisson arrivals at 2k, 20k and 200k requests/s over 10^6 resident streams
    (generator = stream id mod 3 over MWC32/XS256/KISS), sizes log-uniform in
    [2^10, 2^24] samples, dtype 50/50, a 16 GiB output pool for admission, three
    batches in flight; then a saturating burst of 20,000 requests."""
    from paper_1101_1846_amd import workloads as W
    gens = [R.GENERATORS[g] for g in ("MWC32", "XS256", "KISS")]
    h = R.rng_server_create(10 ** 6, gens, 8, 16 << 30, 4096, 1 << 31, inflight=3, auto_release=True,
                            idle_spin_us=SERVED_IDLE_SPIN_US)
    out = {"worker_idle_spin_us": SERVED_IDLE_SPIN_US}
    try:
        for lam, dur in ((2000, 1.0), (20000, 0.5), (200000, 0.25)):
            n = int(lam * dur)
            tab = W.served_table(n, seed=7)
            t = W.poisson_arrivals(lam, n, seed=7)
            R.rng_server_reset_stats(h)
            R.rng_server_replay(h, t, tab["stream"], tab["length"], tab["dtype"])
            st = R.rng_server_stats(h)
            out["lambda_%d" % lam] = {
                "requests": n, "p50_us": round(st["p50_us"], 1), "p99_us": round(st["p99_us"], 1),
                "mean_us": round(st["mean_us"], 1), "mean_queue_submit_device_us":
                    [round(st["mean_queue_us"], 1), round(st["mean_submit_us"], 1), round(st["mean_device_us"], 1)],
                "offered_GB_s": round(4 * tab["length"].sum() / t[-1] / 1e9, 1),
                "GSamples_s": round(st["gsamples_per_s"], 1), "batches": st["batches"],
                "mean_batch_requests": round(st["mean_batch_requests"], 1)}
        n = 20000
        tab = W.served_table(n, seed=17)
        R.rng_server_reset_stats(h)
        R.rng_server_replay(h, [0.0] * n, tab["stream"], tab["length"], tab["dtype"])
        st = R.rng_server_stats(h)
        out["saturation_burst_20000"] = {
            "GSamples_s": round(st["gsamples_per_s"], 1), "GB_s": round(4 * st["gsamples_per_s"], 1),
            "frac_of_single_call": round(st["gsamples_per_s"] / single_rate, 4),
            "p50_us": round(st["p50_us"], 1), "p99_us": round(st["p99_us"], 1), "batches": st["batches"],
            "mean_batch_requests": round(st["mean_batch_requests"], 1), "admission_waits": st["admission_waits"]}
    finally:
        R.rng_server_destroy(h)
    return out


def host_cpu():
    """CPU model, logical CPUs, and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "affinity": allowed}


# A one-GPU job may use this many host cores (the host's share per GPU), whatever
# the machine reports: the all-cores legs use min(affinity, this).
HOST_CORES_PER_GPU = 16


def cpu_baseline(seconds):
    """The serial oracle on the host over a bounded sample of the step's
    workload: whole streams of 256 samples for every generator and dtype of
    the step, streams split over host threads.  Four legs, each repeated
    until about seconds / 4 of wall time: the oracle as built for the tests
    (gcc -O2, the paper's CPU optimisation level) and the same source at
    -O3 -march=native (built here, for this CPU), each on one thread (the
    paper's single-thread CPU rows) and on all the cores the job may use.
    ``value`` is the -O2 all-cores leg: the oracle as it stands."""
    import tempfile

    import oracle
    cpu = host_cpu()
    cores = max(1, min(cpu["affinity"], HOST_CORES_PER_GPU))
    oracle.mwc16_table()  # one-time table search, not part of the rate
    variants = {"gcc -O2": oracle.lib()}
    tmpdir = tempfile.mkdtemp(prefix="oracle_o3_")
    try:
        path = oracle.build_variant(os.path.join(tmpdir, "liboracle_o3native.so"), ["-O3", "-march=native"])
        variants["gcc -O3 -march=native"] = oracle.lib(path)
    except Exception as e:  # noqa: BLE001 - the leg is reported as missing
        variants["gcc -O3 -march=native"] = "build failed: %s" % e
    gens = [(n, d) for n in STEP_GENS for d in ("u32", "f32")]
    budget = seconds / 4.0

    def run(L, S, threads):
        per = {}
        for n, d in gens:
            g = oracle.GENERATORS[n]
            st = oracle.seed(g, 1, S)
            t = time.perf_counter()
            oracle.generate(g, st, N_BULK, oracle.F32 if d == "f32" else oracle.U32, threads=threads, library=L)
            per["%s_%s" % (n, d)] = time.perf_counter() - t
        return per

    legs = []
    for flags, L in variants.items():
        for threads in (1, cores):
            if isinstance(L, str):
                legs.append({"flags": flags, "threads": threads, "error": L})
                continue
            S = 1 << 12
            run(L, S, threads)  # warm-up: thread start, page faults
            dt = sum(run(L, S, threads).values())
            # one pass of about a fifth of the leg's budget, repeated until it is spent
            S = int(min(S_BULK, max(S, S * 0.2 * budget / max(dt, 1e-3))))
            S = max(threads, S // threads * threads)
            reps, tot = 0, {}
            while sum(tot.values()) < budget and reps < 1000:
                for k, v in run(L, S, threads).items():
                    tot[k] = tot.get(k, 0.0) + v
                reps += 1
            t_all = sum(tot.values())
            legs.append({"flags": flags, "threads": threads,
                         "GSamples_s": round(reps * len(gens) * S * N_BULK / t_all / 1e9, 4),
                         "per_generator_GSamples_s": {k: round(reps * S * N_BULK / v / 1e9, 4) for k, v in tot.items()},
                         "sample": "%d pass(es) over %d streams x %d samples per (generator, dtype), %.1f s"
                                   % (reps, S, N_BULK, t_all)})
    try:
        for f in os.listdir(tmpdir):
            os.remove(os.path.join(tmpdir, f))
        os.rmdir(tmpdir)
    except OSError:
        pass
    head = next(l for l in legs if l["flags"] == "gcc -O2" and l["threads"] == cores)
    return {"value": head["GSamples_s"], "unit": "GSamples/s", "cores": cores, "kind": "oracle",
            "sample": "%s; the step's 6 (generator, dtype) pairs, gcc -O2, %d threads" % (head["sample"], cores),
            "cpu_model": cpu["model"], "nproc": cpu["nproc"], "affinity_cpus": cpu["affinity"],
            "cores_note": "all-cores legs use min(affinity, %d): the host cores one GPU's job may use"
                          % HOST_CORES_PER_GPU,
            "legs": legs,
            "paper_single_thread_cpu_GSamples_s": {"hardware": "Xeon Q6600, MSVC 2005 -O2",
                                                   "MWC": 0.3, "XorShift": 0.1, "KISS": 0.2}}


# The sources of the step's generation kernels (gate profiles/traffic.json) and
# of the fused kernel and its calibration loop (gate profiles/valu.json).
KERNEL_SOURCES = ["paper_1101_1846_amd/csrc/rng_device.hpp", "paper_1101_1846_amd/csrc/rng_kernels.hpp",
                  "paper_1101_1846_amd/csrc/rng_internal.hpp", "include/rng_inline.hpp"]
VALU_SOURCES = KERNEL_SOURCES + ["paper_1101_1846_amd/csrc/rng_calib.hip"]


def kernel_source_sha(files=None):
    import hashlib
    h = hashlib.sha256()
    for f in files or KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    """HBM bytes per launch from the committed counter runs (profiles/traffic.json),
    or None when they are missing or were taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get("kernels", {}).get(key)
    if not ent or rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return ent.get("hbm_bytes_per_launch")


def measured_valu():
    """VALU instructions per sample of the fused kernel and of its calibration
    loop from the committed counter runs (profiles/valu.json), or None when
    missing or taken on other kernel sources."""
    try:
        with open(os.path.join(ROOT, "profiles", "valu.json")) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    return rec if rec.get("kernel_source_sha") == kernel_source_sha(VALU_SOURCES) else None


def profile_mode(torch, R, dev, states, out, key):
    """Launch sequence for the counter runs: a plain 1 GiB device-to-device copy
    (its FETCH_SIZE and WRITE_SIZE calibrate the counters), then three launches
    of the chosen step kernel; key "fused": one fused pi launch over 2^34 KISS
    samples and one launch of its calibration loop (SQ_INSTS_VALU runs)."""
    if key == "counter":
        # the layout ceiling's kernel in the step's commonest shape: 3 launches
        st = torch.zeros(S_BULK, dtype=torch.int32, device=dev)
        for _ in range(3):
            R.rng_calibrate_store(st, S_BULK, N_BULK, out, 256, 4)
        torch.cuda.synchronize()
        print("profile launches done: 3 x k_generate<counter> 256 x 4", flush=True)
        return
    if key == "fused":
        g, S, N = R.RNG_KISS, 1 << 20, 1 << 14
        st = torch.empty((6, S), dtype=torch.int32, device=dev)
        R.rng_seed(g, 6, 0, S, st)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        R.rng_fused_pi(g, st, S, N, cnt)
        R.rng_calibrate_valu(3)
        torch.cuda.synchronize()
        print("profile launches done: k_fused_pi<KISS> 2^20 x 2^14, k_valu_fused<1, 2, 4, 8> x 4 each", flush=True)
        return
    name, d = key.split("_")
    g = R.GENERATORS[name]
    # the launch shape the timed step uses: the same autotuning first
    scratch = states[name].clone()
    R.rng_autotune(g, R.DTYPES[d], S_BULK, N_BULK, scratch, out, TUNE_REPS)
    del scratch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    for _ in range(3):
        R.rng_generate(g, states[name], S_BULK, N_BULK, R.DTYPES[d], out)
    torch.cuda.synchronize()
    print("profile launches done: copy 1 GiB, 3 x k_generate<%s>" % key, flush=True)


if __name__ == "__main__":
    main()
