"""Summaries of rocprofv3 CSV output for the library's kernels.

Modes, each printing a short text report:

  python -m paper_1703_05638_amd.profile_summary stats DIR REGEX
      kernel-trace statistics (``*_kernel_stats.csv``): the kernels by total
      time and the line of the kernel matching REGEX.

  python -m paper_1703_05638_amd.profile_summary busy DIR MARKER_REGEX
      kernel trace (``*_kernel_trace.csv``): the run cut into windows that
      end where a kernel matching MARKER_REGEX ends (one per bench step
      when the marker runs once per step); per window the wall time, the
      time at least one kernel ran (union of the kernel intervals, all
      queues), and the idle gaps longer than 50 us by count and sum; then,
      over all windows after the first, the kernels that most often end
      right before such a gap (what the device waited after).

  python -m paper_1703_05638_amd.profile_summary traffic FETCH_DIR WRITE_DIR REGEX COPY_REGEX COPY_BYTES
      counter collection (``*_counter_collection.csv``) of two runs, one with
      FETCH_SIZE and one with WRITE_SIZE (KiB per dispatch).  A plain copy
      kernel that moves COPY_BYTES in and COPY_BYTES out gives one scale
      factor per counter (counter reading / true bytes); the matched kernel's
      average readings per dispatch are divided by them.  The report records
      a digest of the kernel's source so that a reader can tell when the
      figure no longer describes the kernel.

  python -m paper_1703_05638_amd.profile_summary counters DIR 'REGEX[;REGEX...]'
      counter collection (``*_counter_collection.csv``) of one --pmc run: per
      kernel regex the number of dispatches and the sum of every collected
      counter over them.
"""
import csv
import glob
import hashlib
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))


# source regions (first and last marker in kernels.hip) whose digest a
# traffic report records, by the kernel-name prefix the report matches
KERNEL_SOURCES = {
    "k_cheb": ("void k_cheb(", "template void mg_smooth_step<float>"),
    "k_mg": ("__device__ inline void strip_of(", "template void mg_up<float>"),
    "k_gram": ("// FP64 Gram on the matrix cores.", "void sum_partials("),
    "k_proj": ("// FP64 projection on the matrix cores,", "template void proj<float>("),
    "k_stencil": ("__device__ inline void stencil_strip_body", "// Autotuner of the stencil strip height"),
    "k_cd": ("// Convection-diffusion with the wind along x2 (Sec. 6.3)", "void tridiag_x2(hipStream_t st"),
}


def _source_key(regex):
    for key in ("k_gram", "k_proj", "k_mg", "k_stencil"):
        if key in regex:
            return key
    if any(k in regex for k in ("k_sine", "k_tridiag", "k_cd_")):
        return "k_cd"
    return "k_cheb"


def source_digest(key="k_cheb"):
    """sha256 (16 hex digits) of a kernel's source region in kernels.hip."""
    src = open(os.path.join(ROOT, "csrc", "kernels.hip")).read()
    first, last = KERNEL_SOURCES[key]
    a = src.index(first)
    b = src.index(last)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def _rows(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit("no *%s under %s" % (suffix, d))
    out = []
    for f in files:
        with open(f, newline="") as fh:
            out.extend(csv.DictReader(fh))
    return out


def stats(d, regex):
    rows = _rows(d, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    pat = re.compile(regex)
    print("%-60s %10s %14s %12s %7s" % ("kernel", "calls", "total_ms", "avg_us", "pct"))
    for r in rows[:25]:
        print("%-60s %10s %14.3f %12.3f %7.2f" % (r["Name"][:60], r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                  float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    for r in rows:
        if pat.search(r["Name"]):
            print("matched: %s calls=%s avg_us=%.3f total_ms=%.3f" % (r["Name"], r["Calls"], float(r["AverageNs"]) / 1e3,
                                                                      float(r["TotalDurationNs"]) / 1e6))


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names[0])


def busy(d, marker):
    rows = _rows(d, "kernel_trace.csv")
    ks = []
    for r in rows:
        name = _col(r, "Kernel_Name", "KernelName", "Name")
        ks.append((int(_col(r, "Start_Timestamp", "BeginNs", "Start")), int(_col(r, "End_Timestamp", "EndNs", "End")),
                   name))
    ks.sort()
    pat = re.compile(marker)
    cuts = sorted(e for b, e, n in ks if pat.search(n))
    if not ks:
        raise SystemExit("empty kernel trace")
    edges = [ks[0][0]] + cuts
    print("%-8s %12s %12s %8s %9s %12s %12s" % ("window", "wall_ms", "busy_ms", "busy", "kernels", "gaps>50us",
                                                 "gap_sum_ms"))
    after = {}
    for w in range(len(edges) - 1):
        lo, hi = edges[w], edges[w + 1]
        inside = [(max(b, lo), min(e, hi), n) for b, e, n in ks if e > lo and b < hi]
        busy_ns, cur_b, cur_e, cur_n, ngap, gap_ns = 0, None, None, "", 0, 0
        for b, e, n in inside:
            if cur_e is None or b > cur_e:
                if cur_e is not None:
                    busy_ns += cur_e - cur_b
                    if b - cur_e > 50000:
                        ngap += 1
                        gap_ns += b - cur_e
                        if w > 0:
                            key = cur_n.split("(")[0][:70]
                            c, t = after.get(key, (0, 0))
                            after[key] = (c + 1, t + b - cur_e)
                cur_b, cur_e, cur_n = b, e, n
            else:
                if e >= cur_e:
                    cur_n = n
                cur_e = max(cur_e, e)
        if cur_e is not None:
            busy_ns += cur_e - cur_b
        wall = hi - lo
        print("%-8d %12.1f %12.1f %8.3f %9d %12d %12.1f" % (w, wall / 1e6, busy_ns / 1e6, busy_ns / max(wall, 1),
                                                          len(inside), ngap, gap_ns / 1e6))
    if after:
        print("gaps > 50 us after windows 1.. by the kernel ending before them:")
        print("%-72s %8s %12s" % ("kernel", "gaps", "sum_ms"))
        for key, (c, t) in sorted(after.items(), key=lambda kv: -kv[1][1])[:12]:
            print("%-72s %8d %12.1f" % (key, c, t / 1e6))


def _per_dispatch(rows, regex, counter):
    pat = re.compile(regex)
    acc = {}
    for r in rows:
        if r["Counter_Name"] != counter or not pat.search(r["Kernel_Name"]):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    return list(acc.values())


def traffic(fetch_dir, write_dir, regex, copy_regex, copy_bytes):
    fr = _rows(fetch_dir, "counter_collection.csv")
    wr = _rows(write_dir, "counter_collection.csv")
    kf = _per_dispatch(fr, regex, "FETCH_SIZE")
    kw = _per_dispatch(wr, regex, "WRITE_SIZE")
    cf = _per_dispatch(fr, copy_regex, "FETCH_SIZE")
    cw = _per_dispatch(wr, copy_regex, "WRITE_SIZE")
    if not (kf and kw and cf and cw):
        raise SystemExit("missing dispatches: kernel %d/%d copy %d/%d" % (len(kf), len(kw), len(cf), len(cw)))
    # each counter is scaled by what it reads for the copy (which moves
    # copy_bytes in and copy_bytes out)
    f_fetch = statistics.median(cf) * 1024.0 / copy_bytes
    f_write = statistics.median(cw) * 1024.0 / copy_bytes
    per_launch = (statistics.mean(kf) / f_fetch + statistics.mean(kw) / f_write) * 1024.0
    print("kernel_regex: %s" % regex)
    print("kernel_source_sha256_16: %s" % source_digest(_source_key(regex)))
    print("dispatches_fetch: %d" % len(kf))
    print("dispatches_write: %d" % len(kw))
    print("fetch_kib_per_dispatch_mean: %.3f" % statistics.mean(kf))
    print("write_kib_per_dispatch_mean: %.3f" % statistics.mean(kw))
    print("copy_regex: %s" % copy_regex)
    print("copy_bytes_each_way: %d" % copy_bytes)
    print("copy_fetch_kib_median: %.3f" % statistics.median(cf))
    print("copy_write_kib_median: %.3f" % statistics.median(cw))
    print("fetch_scale_factor: %.6f" % f_fetch)
    print("write_scale_factor: %.6f" % f_write)
    print("traffic_bytes_per_launch: %.1f" % per_launch)


def read_traffic(path):
    """traffic_bytes_per_launch from a committed report, or None when the report
    is absent or the kernel's source has changed since it was taken."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    key = _source_key(vals.get("kernel_regex", ""))
    if vals.get("kernel_source_sha256_16") != source_digest(key):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def counters(d, regexes):
    """Per kernel (one regex each, separated by ';'): dispatches and the sum
    of every counter of a rocprofv3 --pmc run over them."""
    rows = _rows(d, "counter_collection.csv")
    names = sorted({r["Counter_Name"] for r in rows})
    for regex in regexes.split(";"):
        pat = re.compile(regex)
        n = len({r.get("Dispatch_Id") or r.get("Correlation_Id") for r in rows if pat.search(r["Kernel_Name"])})
        print("%s: dispatches %d" % (regex, n))
        for c in names:
            print("  %s sum %.6e" % (c, sum(_per_dispatch(rows, regex, c))))


if __name__ == "__main__":
    if len(sys.argv) >= 4 and sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3])
    elif len(sys.argv) >= 4 and sys.argv[1] == "busy":
        busy(sys.argv[2], sys.argv[3])
    elif len(sys.argv) >= 4 and sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3])
    elif len(sys.argv) >= 7 and sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], int(sys.argv[6]))
    else:
        raise SystemExit(__doc__)
