"""Summaries of rocprofv3 result databases (kernel times and counters).

    python3 -m paper_2307_11447_amd.rocprof_summary stats RUN_results.db
        per-kernel calls, total, average, min and max duration
    python3 -m paper_2307_11447_amd.rocprof_summary shapes RUN_results.db KERNEL
        the same per launch shape (grid size) of the kernels matching KERNEL
    python3 -m paper_2307_11447_amd.rocprof_summary counters RUN_results.db ...
        per-kernel mean of every collected hardware counter
    python3 -m paper_2307_11447_amd.rocprof_summary traffic KERNEL FETCH.db WRITE.db COPYF.db COPYW.db MIB
        HBM bytes per launch of KERNEL from FETCH_SIZE / WRITE_SIZE runs,
        each scaled by what the same counter reports for the stream-copy probe
        (bench.py --copy-probe MIB), which reads MIB and writes MIB mebibytes

The traffic summary also records the SHA-256 of the kernel sources, so a
reader can tell whether the counters still describe the current kernels.
"""
import collections
import hashlib
import os
import sqlite3
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(PKG, "csrc", f) for f in ("h4d_device.hpp", "h4d_kernels.hpp")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stats(path: str) -> str:
    db = sqlite3.connect(path)
    rows = list(db.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc"))
    tot = sum(r[2] for r in rows) or 1
    out = [f"{'kernel':64s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}"]
    for name, n, s, a, mn, mx in rows:
        out.append(f"{name[:64]:64s} {n:7d} {s / 1e6:10.3f} {a / 1e3:9.2f} {mn / 1e3:8.2f} {mx / 1e3:8.2f} "
                   f"{100 * s / tot:6.2f}")
    span = list(db.execute("select min(start), max(end) from kernels"))[0]
    if span[0] is not None:
        out.append(f"kernel span {(span[1] - span[0]) / 1e6:.3f} ms, kernels busy {tot / 1e6:.3f} ms")
    return "\n".join(out)


def _grid_column(db) -> str:
    cols = [r[1] for r in db.execute("pragma table_info(kernels)")]
    for c in ("grid_size", "grid_x", "grid_size_x"):
        if c in cols:
            return c
    grid = [c for c in cols if "grid" in c.lower()]
    if not grid:
        raise SystemExit(f"no grid column among {cols}")
    return grid[0]


def shapes(path: str, kernel_substr: str) -> str:
    """Per launch shape (grid size) of the kernels whose name contains
    kernel_substr: calls, total, average, min and max duration."""
    db = sqlite3.connect(path)
    g = _grid_column(db)
    rows = list(db.execute(
        f"select name, {g}, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        f"from kernels where instr(name, ?) > 0 group by name, {g} order by sum(duration) desc", (kernel_substr,)))
    out = [f"{'kernel':48s} {g:>12s} {'calls':>8s} {'total_ms':>10s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s}"]
    for name, grid, n, s, a, mn, mx in rows:
        out.append(f"{name[:48]:48s} {grid!s:>12s} {n:8d} {s / 1e6:10.3f} {a / 1e3:9.2f} {mn / 1e3:8.2f} {mx / 1e3:8.2f}")
    return "\n".join(out)


def counter_means(path: str) -> dict:
    db = sqlite3.connect(path)
    agg = collections.defaultdict(list)
    for name, cname, val in db.execute("select kernel_name, counter_name, value from counters_collection"):
        agg[(name, cname)].append(val)
    return {k: (sum(v) / len(v), len(v)) for k, v in agg.items()}


def counters(paths) -> str:
    out = []
    for p in paths:
        out.append(f"# {p}")
        for (name, cname), (mean, n) in sorted(counter_means(p).items(), key=lambda kv: -kv[1][0] * kv[1][1]):
            out.append(f"{name[:60]:60s} {cname:18s} launches={n:6d} mean={mean:16.2f}")
    return "\n".join(out)


def _mean_for(path, kernel_substr, counter):
    vals = [(m, n) for (name, c), (m, n) in counter_means(path).items() if kernel_substr in name and c == counter]
    if not vals:
        raise SystemExit(f"no {counter} for a kernel matching {kernel_substr!r} in {path}")
    tot = sum(m * n for m, n in vals)
    cnt = sum(n for m, n in vals)
    return tot / cnt, cnt


def traffic(kernel, fetch_db, write_db, copy_fetch_db, copy_write_db, copy_mib) -> str:
    f_kib, nf = _mean_for(fetch_db, kernel, "FETCH_SIZE")
    w_kib, nw = _mean_for(write_db, kernel, "WRITE_SIZE")
    cf_kib, _ = _mean_for(copy_fetch_db, "k_stream_copy", "FETCH_SIZE")
    cw_kib, _ = _mean_for(copy_write_db, "k_stream_copy", "WRITE_SIZE")
    true_kib = float(copy_mib) * 1024.0
    fs, ws = true_kib / cf_kib, true_kib / cw_kib
    bytes_per_launch = (f_kib * fs + w_kib * ws) * 1024.0
    lines = [
        f"kernel: {kernel}",
        f"kernel_source_sha256: {kernel_source_hash()}",
        f"fetch_kib_per_launch: {f_kib:.2f} (mean over {nf} launches)",
        f"write_kib_per_launch: {w_kib:.2f} (mean over {nw} launches)",
        f"copy_probe_kib_read_and_written: {true_kib:.0f}",
        f"copy_probe_fetch_kib: {cf_kib:.2f}",
        f"copy_probe_write_kib: {cw_kib:.2f}",
        f"fetch_scale: {fs:.4f}",
        f"write_scale: {ws:.4f}",
        f"traffic_bytes_per_launch: {bytes_per_launch:.0f}",
    ]
    return "\n".join(lines)


def main(argv):
    if len(argv) < 2:
        print(__doc__)
        return 2
    mode = argv[0]
    if mode == "stats":
        print(stats(argv[1]))
    elif mode == "shapes" and len(argv) == 3:
        print(shapes(argv[1], argv[2]))
    elif mode == "counters":
        print(counters(argv[1:]))
    elif mode == "traffic" and len(argv) == 7:
        print(traffic(*argv[1:]))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
