"""Summaries of rocprofv3 output for the benchmark (kernel times and HBM traffic).

Usage (on the GPU machine, after the profiled runs):

  python -m paper_2207_05612_amd.profiling trace <dir> [<out.txt>]
      Per-kernel calls, total and average time over the whole run and over the
      benchmark's timed region (the launches between its first two spin-kernel
      markers), from rocprofv3 --kernel-trace --output-format csv.

  python -m paper_2207_05612_amd.profiling traffic <kernel-regex> <fetch-dir> <write-dir>
                                           <bench-json> <roofline-key> <out.json>
      HBM bytes per launch of the kernels matching <kernel-regex> in the timed
      region, from one rocprofv3 --pmc FETCH_SIZE run and one --pmc WRITE_SIZE
      run (KiB per dispatch), each scaled by what the same counter reads for a
      known copy in the same process (bench.py --calibrate-copy-mib: a fill
      writes the buffer once, a sum reads it once), and their ratio to the
      algorithmic bytes per launch that the benchmark line of the same run
      reports under <roofline-key>.

  python -m paper_2207_05612_amd.profiling mfma <kernel-regex> <dir> [<out.txt>]
      Executed BF16 matrix-core work of the kernels matching <kernel-regex> in
      the timed region, from one rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_BF16
      run (512 flops per MOP): flops, summed launch time and their ratio,
      against the dense BF16 peak.

The files are found by name below the given directories (rocprofv3 places
them in per-host / per-process subdirectories).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import OrderedDict

HERE = os.path.dirname(os.path.abspath(__file__))
SPIN = re.compile(r"spin", re.I)


def _find(directory: str, suffix: str):
    hits = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError("no *%s below %s" % (suffix, directory))
    return hits


def _col(row_keys, *needles):
    low = {k.lower(): k for k in row_keys}
    for needle in needles:
        for lk, k in low.items():
            if lk == needle:
                return k
    for needle in needles:
        for lk, k in low.items():
            if needle in lk:
                return k
    raise KeyError("none of %s in %s" % (needles, list(row_keys)))


def short_name(name: str) -> str:
    """Kernel name without return type, namespaces and argument list (templates kept)."""
    n = name.replace("(anonymous namespace)::", "")
    depth, cut = 0, len(n)
    for i, ch in enumerate(n):           # the argument list: the first '(' outside template brackets
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    n = re.sub(r"^void ", "", n[:cut].strip())
    n = re.sub(r"^(?:[A-Za-z_0-9]+::)+", "", n)
    return n.strip()


def read_dispatches(directory: str):
    """[(start_ns, end_ns, kernel name)] of every dispatch, in start order."""
    rows = []
    for path in _find(directory, "kernel_trace.csv"):
        with open(path, newline="") as fh:
            rd = csv.DictReader(fh)
            k_name = k_start = k_end = None
            for r in rd:
                if k_name is None:
                    k_name = _col(r.keys(), "kernel_name")
                    k_start = _col(r.keys(), "start_timestamp", "start")
                    k_end = _col(r.keys(), "end_timestamp", "end")
                rows.append((int(r[k_start]), int(r[k_end]), r[k_name]))
    rows.sort()
    return rows


def timed_region(items, name_of):
    """The items between the first two spin-kernel markers (exclusive)."""
    marks = [i for i, it in enumerate(items) if SPIN.search(name_of(it))]
    if len(marks) < 2:
        raise ValueError("fewer than two spin-kernel markers in the trace")
    return items[marks[0] + 1:marks[1]]


def kernel_table(dispatches):
    acc = OrderedDict()
    for s, e, name in dispatches:
        a = acc.setdefault(short_name(name), [0, 0.0])
        a[0] += 1
        a[1] += (e - s) * 1e-6
    total = sum(v[1] for v in acc.values())
    rows = sorted(acc.items(), key=lambda kv: -kv[1][1])
    return total, [(k, c, ms, ms / c, 100.0 * ms / total if total else 0.0) for k, (c, ms) in rows]


def format_table(title: str, dispatches, limit: int = 40) -> str:
    total, rows = kernel_table(dispatches)
    wall = (dispatches[-1][1] - dispatches[0][0]) * 1e-6 if dispatches else 0.0
    out = ["# %s: total kernel time %.1f ms over %d kernel names (wall %.1f ms)" % (title, total, len(rows), wall),
           "%-70s %9s %12s %10s %6s" % ("kernel", "calls", "total_ms", "avg_ms", "pct")]
    for k, c, ms, avg, pct in rows[:limit]:
        out.append("%-70s %9d %12.1f %10.4f %6.2f" % (k[:70], c, ms, avg, pct))
    return "\n".join(out)


def trace_summary(directory: str) -> str:
    disp = read_dispatches(directory)
    parts = [format_table("whole run", disp)]
    try:
        parts.append(format_table("timed region (the headline's timed layers, between the first two "
                                  "spin-kernel markers)", timed_region(disp, lambda d: d[2])))
    except ValueError as err:
        parts.append("# timed region: %s" % err)
    return "\n\n".join(parts) + "\n"


def read_counters(directory: str):
    """[(dispatch id, kernel name, value)] of one counter, in dispatch order."""
    rows = []
    for path in _find(directory, "counter_collection.csv"):
        with open(path, newline="") as fh:
            rd = csv.DictReader(fh)
            keys = None
            for r in rd:
                if keys is None:
                    keys = (_col(r.keys(), "dispatch_id", "dispatch"), _col(r.keys(), "kernel_name"),
                            _col(r.keys(), "counter_value", "value"))
                rows.append((int(r[keys[0]]), r[keys[1]], float(r[keys[2]])))
    rows.sort()
    # several rows per dispatch (one per hardware instance) are summed
    merged = OrderedDict()
    for d, name, v in rows:
        if d in merged:
            merged[d][1] += v
        else:
            merged[d] = [name, v]
    return [(d, nv[0], nv[1]) for d, nv in merged.items()]


def calibration(rows, counter: str):
    """KiB the counter reads for the bench's 1 GiB fill (writes) or sum (reads)."""
    pick = "fill" if counter == "WRITE_SIZE" else "reduce"
    vals = [v for _, name, v in rows if pick in name.lower() and not SPIN.search(name)]
    if not vals:
        raise ValueError("no calibration dispatch (%s) in the %s run" % (pick, counter))
    return max(vals)


def source_hash(names) -> str:
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(HERE, "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


SOURCES = {"cgemm_bf16": ("cgemm_bf16.hip",), "cgemm_kernel": ("cgemm.hip",), "hetrd_kernel": ("hetrd.hip",)}


def traffic(kernel_regex: str, fetch_dir: str, write_dir: str, bench_json: str, roofline_key: str) -> dict:
    pat = re.compile(kernel_regex)
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = read_counters(d)
        kib_1gib = calibration(rows, counter)
        timed = timed_region(rows, lambda r: r[1])
        vals = [v for _, name, v in timed if pat.search(name)]
        if not vals:
            raise ValueError("no %s dispatch matching %r in the timed region" % (counter, kernel_regex))
        res[counter] = {"dispatches": len(vals), "kib_per_dispatch": sum(vals) / len(vals),
                        "kib_for_1GiB": kib_1gib, "factor": 1048576.0 / kib_1gib}
    line = None
    with open(bench_json) as fh:
        for ln in fh:
            ln = ln.strip()
            if ln.startswith("{"):
                line = json.loads(ln)
    if line is None:
        raise ValueError("no benchmark line in %s" % bench_json)
    alg = line[roofline_key]["algorithmic_bytes_per_launch"]
    measured = sum(res[c]["kib_per_dispatch"] * res[c]["factor"] * 1024.0 for c in res)
    key = next((k for k in SOURCES if k in kernel_regex), None)
    return {"kernel_regex": kernel_regex, "source_hash": source_hash(SOURCES[key]) if key else None,
            "counters": res, "bytes_per_launch": measured, "algorithmic_bytes_per_launch": alg,
            "bytes_per_algorithmic_byte": measured / alg}


BF16_DENSE_PEAK = 2.5e15     # flop/s, MI355X dense BF16 matrix cores


def mfma(kernel_regex: str, directory: str) -> str:
    """Executed BF16 MFMA flops of the matching launches in the timed region over their summed time."""
    pat = re.compile(kernel_regex)
    disp = OrderedDict()
    for path in _find(directory, "counter_collection.csv"):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                k = (_col(r.keys(), "dispatch_id", "dispatch"), _col(r.keys(), "kernel_name"),
                     _col(r.keys(), "counter_name"), _col(r.keys(), "counter_value", "value"),
                     _col(r.keys(), "start_timestamp"), _col(r.keys(), "end_timestamp"))
                d = disp.setdefault(int(r[k[0]]), {"name": r[k[1]], "t": (int(r[k[4]]), int(r[k[5]])), "mops": 0.0})
                if r[k[2]] == "SQ_INSTS_VALU_MFMA_MOPS_BF16":
                    d["mops"] += float(r[k[3]])    # rows of one dispatch (hardware instances) are summed
    rows = [(i, d["name"], d) for i, d in sorted(disp.items())]
    timed = timed_region(rows, lambda r: r[1])
    sel = [d for _, name, d in timed if pat.search(name)]
    if not sel:
        raise ValueError("no dispatch matching %r in the timed region" % kernel_regex)
    secs = sum((d["t"][1] - d["t"][0]) * 1e-9 for d in sel)
    flops = sum(d["mops"] * 512.0 for d in sel)
    rate = flops / secs
    return ("# executed BF16 MFMA work of %r in the timed region\n"
            "launches %d\nkernel time %.4f s\nBF16 MFMA flops executed %.4e\n"
            "rate %.1f TFLOP/s = %.3f of the %.1f PFLOP/s dense peak\n"
            % (kernel_regex, len(sel), secs, flops, rate / 1e12, rate / BF16_DENSE_PEAK, BF16_DENSE_PEAK / 1e15))


def main(argv):
    if len(argv) >= 2 and argv[0] == "trace":
        text = trace_summary(argv[1])
        if len(argv) > 2:
            with open(argv[2], "w") as fh:
                fh.write(text)
        print(text)
        return 0
    if len(argv) == 7 and argv[0] == "traffic":
        rec = traffic(*argv[1:6])
        with open(argv[6], "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec, indent=1))
        return 0
    if len(argv) >= 3 and argv[0] == "mfma":
        text = mfma(argv[1], argv[2])
        if len(argv) > 3:
            with open(argv[3], "w") as fh:
                fh.write(text)
        print(text)
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
