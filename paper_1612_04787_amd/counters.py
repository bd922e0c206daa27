"""Summaries of rocprofv3 output for the library's kernels.

  python -m paper_1612_04787_amd.counters stats  KERNEL_STATS_CSV
  python -m paper_1612_04787_amd.counters pmc    COUNTER_COLLECTION_CSV [--largest-grid]
  python -m paper_1612_04787_amd.counters traffic FETCH_CSV WRITE_CSV [--copy-bytes B]
  python -m paper_1612_04787_amd.counters lds    COUNTER_COLLECTION_CSV [--cus 256]

`stats` condenses a `--kernel-trace --stats` run to one line per kernel
(calls, average and total duration).  `pmc` averages every counter per
dispatch of each kernel.  `traffic` turns one FETCH_SIZE run and one
WRITE_SIZE run (KiB per dispatch; each kernel's largest-grid dispatches)
into HBM bytes per launch, each scaled by
the factor that makes the same counter read exactly `copy-bytes` for a plain
device-to-device copy of that size launched in the same program, and records
the digest of the kernel sources the numbers belong to.  `lds` turns one run of
SQ_INSTS_LDS_LOAD_BANDWIDTH, SQ_INSTS_LDS_STORE_BANDWIDTH (64-byte units moved
by LDS loads and stores), SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT and
GRBM_GUI_ACTIVE into LDS bytes per launch, the LDS busy fraction and the bank
conflict cycles per active cycle, with the source digest.

Kernel names are shortened to `name<N>` (the first template argument is the
window size), the form the library's own HIP-event timer uses; the instances
of the pruned inverse (a search radius) become `name_pruned<N>`, those of the
Pearson mode `name_pearson<N>`.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def _code_only(text: str) -> bytes:
    """The source without its comments and blank lines (comments change
    nothing the counters measure)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = [ln.strip() for ln in text.splitlines()]
    return "\n".join(ln for ln in lines if ln).encode()


def source_digest() -> str:
    """SHA-256 over the code of the library's HIP sources and headers (sorted
    by name), comments and blank lines left out."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp", ".h")):
            h.update(f.encode())
            with open(os.path.join(CSRC, f), encoding="utf-8") as fh:
                h.update(_code_only(fh.read()))
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "swift.h")
    if os.path.exists(inc):
        with open(inc, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()))
    return h.hexdigest()


def short_name(full: str) -> str | None:
    m = re.search(r"swift::k_bwd_(col|row|fin)<(\d+), true(, (true|false))?>", full)
    if m:  # centroid-Jacobian instance of the adjoint kernels
        return "k_cj_%s<%s>" % (m.group(1), m.group(2))
    m = re.search(r"swift::(k_row_fwd)<(\d+)(, \d+)+, true>", full)
    if m:  # Pearson instance of the forward row pass
        return "%s_pearson<%s>" % (m.group(1), m.group(2))
    m = re.search(r"swift::(k_row_inv)<(\d+), \d+, true, true>", full)
    if m:  # Pearson instance of the inverse row pass
        return "%s_pearson<%s>" % (m.group(1), m.group(2))
    m = re.search(r"swift::(k_col_pair|k_col|k_row_inv)<(\d+)(, \d+)?, true(, false)?>", full)
    if m:  # pruned-inverse instance (a search radius)
        return "%s_pruned<%s>" % (m.group(1), m.group(2))
    m = re.search(r"swift::(k_\w+)<(\d+)", full)
    if m:
        return "%s<%s>" % (m.group(1), m.group(2))
    m = re.search(r"swift::(k_\w+)<(true|false)>\(", full)
    if m:
        return "%s<%s>" % (m.group(1), m.group(2))
    m = re.search(r"swift::(k_\w+)\(", full)
    if m:
        return m.group(1)
    if "copyBuffer" in full or ("elementwise" in full and "copy" in full.lower()):
        return "copy:" + full.split("(")[0][-60:]
    return None


def _rows(path):
    with open(path, newline="") as f:
        yield from csv.DictReader(f)


def stats(path):
    out = []
    for r in _rows(path):
        name = short_name(r.get("Name", "") or r.get("Kernel_Name", ""))
        if not name:
            continue
        calls = int(r["Calls"])
        tot = float(r["TotalDurationNs"])
        out.append((name, calls, tot / calls, tot))
    out.sort(key=lambda x: -x[3])
    lines = ["%-26s %7s %12s %12s" % ("kernel", "calls", "avg_ms", "total_ms")]
    for name, calls, avg, tot in out:
        lines.append("%-26s %7d %12.4f %12.3f" % (name, calls, avg / 1e6, tot / 1e6))
    return "\n".join(lines)


def grids(path):
    """Kernel trace (run_kernel_trace.csv) summed per kernel and launch size:
    a kernel launched at several batch sizes gets one line per grid."""
    acc = collections.defaultdict(list)
    for r in _rows(path):
        name = short_name(r.get("Kernel_Name", ""))
        if not name:
            continue
        grid = int(float(r.get("Grid_Size_X", r.get("Grid_Size", 0)) or 0))
        wg = int(float(r.get("Workgroup_Size_X", r.get("Workgroup_Size", 0)) or 0))
        dur = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
        acc[(name, grid // wg if wg else grid)].append(dur)
    out = sorted(((k[0], k[1], len(v), sum(v) / len(v), sum(v)) for k, v in acc.items()), key=lambda x: -x[4])
    lines = ["%-26s %10s %7s %12s %12s" % ("kernel", "workgroups", "calls", "avg_ms", "total_ms")]
    for name, g, calls, avg, tot in out:
        lines.append("%-26s %10d %7d %12.4f %12.3f" % (name, g, calls, avg / 1e6, tot / 1e6))
    return "\n".join(lines)


def per_kernel_counters(path, largest_grid=False):
    """{kernel: {counter: [value per dispatch]}}; with largest_grid only the
    dispatches of each kernel's largest grid (the production batch, not the
    smaller set-up or tuning launches of the same kernel)."""
    rows = []
    for r in _rows(path):
        name = short_name(r.get("Kernel_Name", ""))
        if name:
            rows.append((name, int(float(r.get("Grid_Size", 0) or 0)), r["Counter_Name"],
                         float(r["Counter_Value"])))
    top = collections.defaultdict(int)
    for name, grid, _, _ in rows:
        top[name] = max(top[name], grid)
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for name, grid, ctr, val in rows:
        if largest_grid and not name.startswith("copy:") and grid != top[name]:
            continue
        acc[name][ctr].append(val)
    return acc


def pmc(path, largest_grid=False):
    acc = per_kernel_counters(path, largest_grid)
    lines = []
    for name in sorted(acc):
        lines.append(name)
        for c, vals in sorted(acc[name].items()):
            lines.append("    %-28s dispatches=%-5d mean=%.6g min=%.6g max=%.6g"
                         % (c, len(vals), sum(vals) / len(vals), min(vals), max(vals)))
    return "\n".join(lines)


def traffic(fetch_csv, write_csv, copy_bytes, ref_kernel=None, ref_bytes=None):
    """Bytes read and written per launch from FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch), each scaled so that a reference reads (writes) exactly its
    known bytes: the program's largest device-to-device copy of `copy_bytes`,
    or with ref_kernel a kernel of the library that reads and writes
    `ref_bytes` each per launch.  On this GPU FETCH_SIZE can count half the
    bytes of 128-byte requests, and which request size a copy uses varies, so
    the reference should issue requests like the kernels it calibrates."""
    f = per_kernel_counters(fetch_csv, largest_grid=True)
    w = per_kernel_counters(write_csv, largest_grid=True)

    def mean(d, name, ctr):
        v = d.get(name, {}).get(ctr, [])
        return sum(v) / len(v) if v else None

    def full(d, name, ctr):
        # the reference's full-size launches: a program may also launch it on
        # fewer sections with the same grid
        v = d.get(name, {}).get(ctr, [])
        top = [x for x in v if x >= 0.9 * max(v)] if v else []
        return sum(top) / len(top) if top else None

    if ref_kernel:
        cf, cw = full(f, ref_kernel, "FETCH_SIZE"), full(w, ref_kernel, "WRITE_SIZE")
        if cf is None or cw is None:
            raise SystemExit("no %s in the counter files" % ref_kernel)
        kf = ref_bytes / (cf * 1024.0)
        kw = ref_bytes / (cw * 1024.0)
        head = "calibration: %s reads and writes %d bytes per launch: FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB" % (
            ref_kernel, ref_bytes, cf, cw)
    else:
        copies = [k for k in f if k.startswith("copy:")]
        if not copies:
            raise SystemExit("no copy kernel in %s: run the program with its calibration copy" % fetch_csv)
        # the calibration copy is the largest copy dispatch
        cf = max(max(f[k]["FETCH_SIZE"]) for k in copies)
        cw = max(max(w[k]["WRITE_SIZE"]) for k in copies if k in w)
        kf = copy_bytes / (cf * 1024.0)
        kw = copy_bytes / (cw * 1024.0)
        head = "calibration: %d-byte copy reads FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB" % (copy_bytes, cf, cw)
    lines = [head, "scale_fetch %.4f" % kf, "scale_write %.4f" % kw, "source_digest %s" % source_digest(),
             "%-26s %16s %16s %16s" % ("kernel", "read_B/launch", "write_B/launch", "traffic_B/launch")]
    for name in sorted(k for k in f if not k.startswith("copy:")):
        fr, wr = mean(f, name, "FETCH_SIZE"), mean(w, name, "WRITE_SIZE")
        if fr is None or wr is None:
            continue
        rb, wb = fr * 1024.0 * kf, wr * 1024.0 * kw
        lines.append("%-26s %16.4g %16.4g %16.4g" % (name, rb, wb, rb + wb))
    return "\n".join(lines)


def lds(path, cus=256):
    d = per_kernel_counters(path, largest_grid=True)

    def mean(name, ctr):
        v = d[name].get(ctr, [])
        return sum(v) / len(v) if v else None

    lines = ["source_digest %s" % source_digest(),
             "%-26s %16s %16s %16s %10s %12s" % ("kernel", "lds_read_B", "lds_write_B", "lds_B/launch", "lds_busy",
                                                   "bank_confl")]
    for name in sorted(k for k in d if not k.startswith("copy:")):
        ld, st = mean(name, "SQ_INSTS_LDS_LOAD_BANDWIDTH"), mean(name, "SQ_INSTS_LDS_STORE_BANDWIDTH")
        act, bc, gui = mean(name, "SQ_LDS_IDX_ACTIVE"), mean(name, "SQ_LDS_BANK_CONFLICT"), mean(name, "GRBM_GUI_ACTIVE")
        if ld is None or st is None:
            continue
        busy = act / (gui * cus) if act is not None and gui else float("nan")
        conf = bc / (act - bc) if act is not None and bc is not None and act > bc else float("nan")
        lines.append("%-26s %16.4g %16.4g %16.4g %10.3f %12.3f" % (name, ld * 64.0, st * 64.0, (ld + st) * 64.0, busy,
                                                                   conf))
    return "\n".join(lines)


def read_lds(path, kernel):
    """(LDS bytes per launch of `kernel`, busy fraction, digest) from an `lds`
    summary, or (None, None, None)."""
    if not os.path.exists(path):
        return None, None, None
    digest, val, busy = None, None, None
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 2 and parts[0] == "source_digest":
                digest = parts[1]
            if len(parts) == 6 and parts[0] == kernel:
                try:
                    val, busy = float(parts[3]), float(parts[4])
                except ValueError:
                    pass
    return val, busy, digest


def read_traffic(path, kernel):
    """(traffic bytes per launch of `kernel`, digest) from a `traffic` summary,
    or (None, None) if the file or the kernel is absent."""
    if not os.path.exists(path):
        return None, None
    digest, val = None, None
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 2 and parts[0] == "source_digest":
                digest = parts[1]
            if len(parts) == 4 and parts[0] == kernel:
                try:
                    val = float(parts[3])
                except ValueError:
                    pass
    return val, digest


def main(argv=None):
    ap = argparse.ArgumentParser(description="rocprofv3 summaries for the library's kernels")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a = sub.add_parser("grids")
    a.add_argument("csv")
    a = sub.add_parser("pmc")
    a.add_argument("csv")
    a.add_argument("--largest-grid", action="store_true", help="only each kernel's largest-grid dispatches")
    a = sub.add_parser("traffic")
    a.add_argument("fetch_csv")
    a.add_argument("write_csv")
    a.add_argument("--copy-bytes", type=int, default=1 << 30)
    a.add_argument("--ref-kernel", default=None, help="calibrate against this kernel instead of the copy")
    a.add_argument("--ref-bytes", type=int, default=1 << 30, help="bytes the reference kernel reads and writes")
    a = sub.add_parser("lds")
    a.add_argument("csv")
    a.add_argument("--cus", type=int, default=256)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print(stats(args.csv))
    elif args.cmd == "grids":
        print(grids(args.csv))
    elif args.cmd == "pmc":
        print(pmc(args.csv, args.largest_grid))
    elif args.cmd == "lds":
        print(lds(args.csv, args.cus))
    else:
        print(traffic(args.fetch_csv, args.write_csv, args.copy_bytes, args.ref_kernel, args.ref_bytes))


if __name__ == "__main__":
    sys.exit(main())
