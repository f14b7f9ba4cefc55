"""Summaries of rocprofv3 result databases (the rocpd SQLite files written by
``rocprofv3 -d DIR -o run``): kernel-trace statistics and per-dispatch PMC
counters, as short text tables.

    python -m paper_1101_1846_amd.prof trace RUN_results.db
    python -m paper_1101_1846_amd.prof pmc FETCH_results.db WRITE_results.db KEY
    python -m paper_1101_1846_amd.prof valu VALU_results.db KERNEL_SOURCE_SHA
    python -m paper_1101_1846_amd.prof counters KERNEL_NAME_PART PASS1_results.db [PASS2_results.db ...]
    python -m paper_1101_1846_amd.prof steps RUN_results.db BENCH_LINE.json

The ``pmc`` form scales each counter by what it reads for the plain 1 GiB
device-to-device copy that ``bench.py --profile KEY`` launches first (the copy
moves exactly 2^30 bytes each way), and prints the JSON record that
``profiles/traffic.json`` keeps for that kernel.  The ``valu`` form reads the
SQ_INSTS_VALU run of ``bench.py --profile fused`` and prints the record that
``profiles/valu.json`` keeps (VALU instructions per sample of the fused kernel
and of its calibration loop).
"""
import json
import sqlite3
import sys
from collections import defaultdict

COPY_BYTES = 1 << 30


def _rows(db, sql):
    con = sqlite3.connect(db)
    try:
        return list(con.execute(sql))
    finally:
        con.close()


def short(name, width=96):
    name = name.replace("rngx::", "").replace("(GenArgs)", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def trace_table(db):
    """Per kernel: calls, total/avg/min/max duration in microseconds."""
    stats = defaultdict(list)
    for name, dur in _rows(db, "select name, duration from kernels"):
        stats[name].append(dur / 1000.0)
    lines = ["| kernel | calls | total us | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    for name, d in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        lines.append("| %s | %d | %.1f | %.2f | %.2f | %.2f |" % (short(name), len(d), sum(d), sum(d) / len(d),
                                                                  min(d), max(d)))
    return "\n".join(lines), stats


def pmc_per_dispatch(db, counter):
    """[(kernel name, grid size, value in KiB)] in dispatch order."""
    return [(n, g, v) for n, g, v in _rows(
        db, "select kernel_name, grid_size, value from counters_collection where counter_name = '%s' "
            "order by dispatch_id" % counter)]


def copy_value(rows):
    vals = [v for n, g, v in rows if "copy" in n.lower() or "elementwise" in n.lower()]
    return vals[-1] if vals else None


def pmc_record(fetch_db, write_db, key):
    f = pmc_per_dispatch(fetch_db, "FETCH_SIZE")
    w = pmc_per_dispatch(write_db, "WRITE_SIZE")
    fc, wc = copy_value(f), copy_value(w)
    fs = COPY_BYTES / (fc * 1024.0)
    ws = COPY_BYTES / (wc * 1024.0)
    kf = [v for n, g, v in f if "k_generate" in n][-3:]
    kw = [v for n, g, v in w if "k_generate" in n][-3:]
    fetch = sum(kf) / len(kf) * 1024.0 * fs
    write = sum(kw) / len(kw) * 1024.0 * ws
    return {
        "copy_calibration": {"bytes_each_way": COPY_BYTES, "FETCH_SIZE_KiB": fc, "WRITE_SIZE_KiB": wc,
                             "fetch_scale": round(fs, 4), "write_scale": round(ws, 4)},
        "FETCH_SIZE_KiB_per_launch": [round(v, 1) for v in kf],
        "WRITE_SIZE_KiB_per_launch": [round(v, 1) for v in kw],
        "hbm_fetch_bytes_per_launch": int(fetch),
        "hbm_write_bytes_per_launch": int(write),
        "hbm_bytes_per_launch": int(fetch + write),
    }


# Samples per dispatch of the kernels that `bench.py --profile fused` launches:
# fused pi over 2^20 streams x 2^14 samples, and the calibration loop
# k_valu_fused<NS>: its lanes x 64 iterations x 8 samples x NS streams.
FUSED_SAMPLES = 1 << 34
CALIB_SAMPLES_PER_LANE_PER_STREAM = 64 * 8


def valu_record(db, sha):
    """VALU instructions per lane-sample of the fused kernel and of its
    calibration loop, from SQ_INSTS_VALU (wave instructions) x 64 lanes."""
    per = defaultdict(float)
    grid = {}
    for did, name, g, v in _rows(db, "select dispatch_id, kernel_name, grid_size, value from counters_collection "
                                      "where counter_name = 'SQ_INSTS_VALU' order by dispatch_id"):
        per[(did, name)] += v
        grid[(did, name)] = g
    fused = [v for (d, n), v in per.items() if "k_fused_pi" in n]
    calib = defaultdict(list)  # streams per lane -> VALU instructions per lane-sample, per dispatch
    for (d, n), v in per.items():
        if "k_valu_fused<" in n:
            ns = int(n.split("k_valu_fused<")[1].split(">")[0])
            calib[ns].append(v * 64 / (grid[(d, n)] * CALIB_SAMPLES_PER_LANE_PER_STREAM * ns))
    per_ns = {ns: round(sum(v) / len(v), 3) for ns, v in sorted(calib.items())}
    return {"kernel_source_sha": sha,
            "fused_valu_per_sample": round(sum(fused) / len(fused) * 64 / FUSED_SAMPLES, 3),
            "calib_valu_per_sample": round(sum(per_ns.values()) / len(per_ns), 3),
            "calib_valu_per_sample_by_streams_per_lane": per_ns,
            "fused_SQ_INSTS_VALU_per_dispatch": [int(v) for v in fused]}


def counters_table(match, dbs):
    """Per counter: the mean over the last three dispatches whose kernel name
    contains `match` (each dispatch's instances summed), from one or more
    PMC databases."""
    out = {}
    for db in dbs:
        per = defaultdict(lambda: defaultdict(float))
        for did, name, c, v in _rows(db, "select dispatch_id, kernel_name, counter_name, value "
                                         "from counters_collection order by dispatch_id"):
            if match in name:
                per[did][c] += v
        last = sorted(per)[-3:]
        for did in last:
            for c, v in per[did].items():
                out.setdefault(c, []).append(v)
    return {c: sum(v) / len(v) for c, v in out.items()}


def step_table(db, bench_line):
    """The step kernels of a traced `bench.py` run, in the shapes its JSON line
    names (launch_shapes), averaged over the timed launches only: the last
    `steps` dispatches of each before the run's first torch fill kernel (the
    write-ceiling measurement that follows the timed steps).  Beside each, the
    same run's HIP-event average from the JSON line (per_kernel: an untimed
    pass with an event at every launch boundary; for the dominant kernel also
    the timed steps' own events, roofline.avg_launch_ms)."""
    line = json.load(open(bench_line))
    steps = line["steps"]
    rows = [(short(n, 10 ** 6), st, dur) for n, st, dur in _rows(db, "select name, start, duration from kernels "
                                                                       "order by start")]
    fills = [st for n, st, d in rows if "FillFunctor" in n]
    t_fill = fills[0] if fills else float("inf")
    out = ["| kernel | timed launches | trace avg us | trace min us | trace max us | bench event avg us |",
           "|---|---|---|---|---|---|"]
    dom = line["roofline"]["kernel"]
    for key, sh in line["launch_shapes"].items():
        g, d = key.split("_")
        pat = "k_generate<Gen%s, %d, %d, %d, 128, 2>" % (g, 1 if d == "f32" else 0, sh["wg"], sh["unroll"])
        durs = [dur / 1000.0 for n, st, dur in rows if pat in n and st < t_fill][-steps:]
        ev = "%.2f" % (line["per_kernel"][key]["ms"] * 1e3)
        if "<%s>" % key in dom:
            ev += " (timed steps: %.2f)" % (line["roofline"]["avg_launch_ms"] * 1e3)
        out.append("| %s | %d | %.2f | %.2f | %.2f | %s |" % (pat, len(durs), sum(durs) / len(durs), min(durs),
                                                            max(durs), ev))
    return "\n".join(out)


def main(argv):
    if not argv:
        raise SystemExit(__doc__)
    if argv[0] == "trace":
        table, _ = trace_table(argv[1])
        print(table)
    elif argv[0] == "pmc":
        print(json.dumps({argv[3]: pmc_record(argv[1], argv[2], argv[3])}, indent=1))
    elif argv[0] == "steps":
        print(step_table(argv[1], argv[2]))
    elif argv[0] == "counters":
        for c, v in sorted(counters_table(argv[1], argv[2:]).items()):
            print("| %s | %.4g |" % (c, v))
    elif argv[0] == "valu":
        print(json.dumps(valu_record(argv[1], argv[2]), indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
