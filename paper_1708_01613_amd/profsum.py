"""Summaries of rocprofv3 CSV output for the profiles kept with the library.

  python -m paper_1708_01613_amd.profsum stats DIR [--top N]
      Markdown table of the kernels in DIR/*kernel_stats.csv (a
      `rocprofv3 --kernel-trace --stats --output-format csv` run).

  python -m paper_1708_01613_amd.profsum traffic FETCH_DIR WRITE_DIR --kernel NAME
      HBM bytes per dispatch of the kernels whose name starts with NAME, from
      two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of a program
      that also copies a buffer of --copy-bytes bytes device to device
      (bench.py's copy-ceiling measurement does, 1 GiB, with the library's
      k_copy16).  Each counter is scaled by the factor that makes it read the
      known size for that copy (every k_copy16 dispatch, or else the
      largest-grid __amd_rocclr_copyBuffer dispatches).
"""
import argparse
import csv
import glob
import os
import sys


def _csv(d, suffix):
    hits = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not hits:
        sys.exit(f"no *{suffix} under {d}")
    with open(hits[0]) as fh:
        return list(csv.DictReader(fh))


def stats(d, top):
    rows = sorted(_csv(d, "kernel_stats.csv"), key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def _per_dispatch(rows, counter):
    """{dispatch id: (kernel name, grid size, summed counter value)}"""
    acc = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        k = r["Dispatch_Id"]
        name, grid, v = acc.get(k, (r["Kernel_Name"], int(r["Grid_Size"]), 0.0))
        acc[k] = (name, grid, v + float(r["Counter_Value"]))
    return acc


def _scaled(d, counter, kernel, copy_bytes):
    disp = _per_dispatch(_csv(d, "counter_collection.csv"), counter)
    cal = [v for n, _, v in disp.values() if "k_copy16" in n]
    if not cal:
        copies = [(g, v) for n, g, v in disp.values() if n.startswith("__amd_rocclr_copyBuffer")]
        if not copies:
            sys.exit(f"{d}: no copy dispatches to calibrate {counter}")
        gmax = max(g for g, _ in copies)
        cal = [v for g, v in copies if g == gmax]
    factor = copy_bytes / (sum(cal) / len(cal) * 1024.0)
    vals = [v for n, _, v in disp.values() if n.startswith(kernel)]
    if not vals:
        sys.exit(f"{d}: no dispatches of {kernel}")
    return sum(vals) / len(vals) * 1024.0 * factor, factor, len(vals), len(cal)


def traffic(fetch_dir, write_dir, kernel, copy_bytes, updates):
    rd, fr, nr, cr = _scaled(fetch_dir, "FETCH_SIZE", kernel, copy_bytes)
    wr, fw, nw, cw = _scaled(write_dir, "WRITE_SIZE", kernel, copy_bytes)
    out = [f"- kernel: `{kernel}`",
           f"- dispatches averaged: {nr} (FETCH_SIZE run), {nw} (WRITE_SIZE run)",
           f"- copy calibration: {copy_bytes} B device-to-device copy, {cr} / {cw} dispatches; "
           f"FETCH_SIZE x {fr:.3f}, WRITE_SIZE x {fw:.3f}",
           f"- hbm_read_bytes_per_launch: {rd:.0f}",
           f"- hbm_write_bytes_per_launch: {wr:.0f}",
           f"- hbm_bytes_per_launch: {rd + wr:.0f}"]
    if updates:
        out.append(f"- hbm_bytes_per_update: {(rd + wr) / updates:.2f} (over {updates} lattice updates per launch)")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--top", type=int, default=25)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--updates", type=int, default=0)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats(a.dir, a.top))
    else:
        print(traffic(a.fetch_dir, a.write_dir, a.kernel, a.copy_bytes, a.updates))


if __name__ == "__main__":
    main()
