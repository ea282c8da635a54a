"""Text summaries of rocprofv3 output (CSV format) for the profiles folder.

    python -m paper_2402_17794_amd.prof_summary kernels DIR --title T --command C
        per-kernel call count and duration (from *_kernel_stats.csv), for the
        library's kernels and the calibration copy.

    python -m paper_2402_17794_amd.prof_summary traffic FETCH_DIR WRITE_DIR --kernel SUBSTR
            --title T --command C [--region product|dual]
        HBM traffic per dispatch of the kernel whose name contains SUBSTR,
        from a FETCH_SIZE run and a WRITE_SIZE run (*_counter_collection.csv).
        Both counters are scaled by what they read for the plain copy of
        CALIB_BYTES that bench.py issues (a same-type tensor copy, which the
        runtime runs as its blit kernel; bytes moved are known exactly:
        CALIB_BYTES read, CALIB_BYTES written).  It is the copy dispatch with
        the largest grid.  The output also records a hash of the product
        kernel's source, so a reader can tell when the kernel has changed since
        the counters were taken.
"""

import argparse
import csv
import glob
import hashlib
import os
import sys

CALIB_BYTES = 256 << 20                     # the calibration copy in bench.py
CALIB_NAME = "__amd_rocclr_copyBuffer"
PKG = os.path.dirname(os.path.abspath(__file__))
GEMM_HEADERS = ("csrc/common.hpp", "csrc/philox.hpp")
REGIONS = {
    "product": ("// ---- product kernel (begin) ----", "// ---- product kernel (end) ----"),
    "dual": ("// ---- two-sided sketch of the single-pass Algorithm 6 (begin) ----",
             "// ---- two-sided sketch (end) ----"),
}


def gemm_source_hash(region="product"):
    """Hash of a product kernel's device source (the marked region of
    csrc/gemm.hip, `product` for the products of Algorithm 4, `dual` for the
    two-sided sketch, and the device headers they use); host-side launch
    code of the products is outside it."""
    begin, end = REGIONS[region]
    h = hashlib.sha256()
    src = open(os.path.join(PKG, "csrc/gemm.hip")).read()
    h.update(src[src.index(begin):src.index(end)].encode())
    for f in GEMM_HEADERS:
        with open(os.path.join(PKG, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _one(pattern):
    files = sorted(glob.glob(pattern))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    return files[0]


def _is_calib(name):
    return CALIB_NAME in name


def kernels(args):
    rows = list(csv.DictReader(open(_one(os.path.join(args.dir, "*kernel_stats.csv")))))
    print(f"# rocprofv3 kernel summary: {args.title}")
    print("#")
    print("# command (repo root):")
    print(f"#   {args.command}")
    print("# durations per dispatch; only the library's kernels (and the calibration copy) are listed.")
    print()
    print(f"{'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'total_ms':>10}  kernel")
    for r in rows:
        name = r["Name"]
        if "rsvd::" not in name and not _is_calib(name):
            continue
        label = "runtime copy kernel (incl. the 256 MiB calibration copy)" if _is_calib(name) else name
        print(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:10.2f} "
              f"{float(r['MaxNs']) / 1e3:10.2f} {float(r['TotalDurationNs']) / 1e6:10.3f}  {label[:150]}")


def _counter_means(d, counter):
    """{kernel name: (mean counter value, dispatches)}; the calibration copy
    is keyed CALIB_NAME and restricted to its largest-grid dispatches."""
    rows = [r for r in csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv"))))
            if r["Counter_Name"] == counter]
    big = max([int(r["Grid_Size"]) for r in rows if _is_calib(r["Kernel_Name"])] or [0])
    acc = {}
    for r in rows:
        name = r["Kernel_Name"]
        if _is_calib(name):
            if int(r["Grid_Size"]) != big:
                continue
            name = CALIB_NAME
        s, n = acc.get(name, (0.0, 0))
        acc[name] = (s + float(r["Counter_Value"]), n + 1)
    return {k: (s / n, n) for k, (s, n) in acc.items()}


def traffic(args):
    fetch = _counter_means(args.fetch_dir, "FETCH_SIZE")
    write = _counter_means(args.write_dir, "WRITE_SIZE")
    cal_f = [v for k, v in fetch.items() if _is_calib(k)]
    cal_w = [v for k, v in write.items() if _is_calib(k)]
    if not cal_f or not cal_w:
        raise SystemExit("calibration copy not found in the counter runs")
    f_scale = CALIB_BYTES / (cal_f[0][0] * 1024.0)
    w_scale = CALIB_BYTES / (cal_w[0][0] * 1024.0)
    ks = [k for k in fetch if args.kernel in k]
    if len(ks) != 1:
        raise SystemExit(f"kernel pattern {args.kernel!r} matches {len(ks)} kernels")
    k = ks[0]
    fb = fetch[k][0] * 1024.0 * f_scale
    wb = write[k][0] * 1024.0 * w_scale
    print(f"# rocprofv3 HBM traffic: {args.title}")
    print("#")
    print("# commands (repo root), one counter per run:")
    for c in args.command:
        print(f"#   {c}")
    print(f"# calibration: plain copy of {CALIB_BYTES} bytes read + {CALIB_BYTES} bytes written "
          f"({cal_f[0][1]} dispatches);")
    print(f"#   FETCH_SIZE read {cal_f[0][0]:.0f} KiB -> scale {f_scale:.4f}; "
          f"WRITE_SIZE read {cal_w[0][0]:.0f} KiB -> scale {w_scale:.4f}")
    print(f"kernel: {k}")
    print(f"dispatches: {fetch[k][1]} (fetch run), {write[k][1]} (write run)")
    print(f"fetch_kib_per_dispatch: {fetch[k][0]:.1f}")
    print(f"write_kib_per_dispatch: {write[k][0]:.1f}")
    print(f"fetch_bytes_scaled: {fb:.6e}")
    print(f"write_bytes_scaled: {wb:.6e}")
    print(f"traffic_bytes_per_launch: {fb + wb:.6e}")
    print(f"gemm_source_hash: {gemm_source_hash(args.region)}")


def read_traffic(path):
    """(bytes per launch, source hash) from a traffic summary, or None."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    try:
        return float(vals["traffic_bytes_per_launch"]), vals["gemm_source_hash"]
    except KeyError:
        return None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    a = sub.add_parser("kernels")
    a.add_argument("dir")
    a.add_argument("--title", required=True)
    a.add_argument("--command", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--kernel", required=True)
    b.add_argument("--title", required=True)
    b.add_argument("--command", action="append", required=True)
    b.add_argument("--region", default="product", choices=sorted(REGIONS),
                   help="source region whose hash is recorded (product: Algorithm 4 products, dual: two-sided sketch)")
    args = ap.parse_args(argv)
    (kernels if args.mode == "kernels" else traffic)(args)


if __name__ == "__main__":
    sys.exit(main())
