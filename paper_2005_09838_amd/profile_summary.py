"""Condense rocprofv3 CSV output into the short text summaries kept with the measurements.

  python -m paper_2005_09838_amd.profile_summary stats DIR --command CMD --out FILE
      kernel table (calls, mean / min / max duration, share of GPU time) from the
      *kernel_stats.csv that `rocprofv3 --kernel-trace --stats --output-format csv` wrote.

  python -m paper_2005_09838_amd.profile_summary traffic --fetch DIR --write DIR
         --copy-fetch DIR --copy-write DIR --kernel NAME --copy-bytes N --stage S
         --precision P --workload W --algorithmic-bytes B --command CMD --out FILE
      HBM traffic of one kernel per launch: the mean FETCH_SIZE and WRITE_SIZE per dispatch
      (KiB) of the kernel, each scaled by the ratio of the known bytes of a plain copy
      kernel to what the same counter reads for it.  The summary records the SHA-256 of the
      kernel sources it was taken from, so a later reader can tell whether it still applies.

  python -m paper_2005_09838_amd.profile_summary all-traffic --fetch DIR --write DIR
         --copy-fetch DIR --copy-write DIR --copy-bytes N --per-iteration PATTERN ...
         --algorithmic-bytes B --title T --command CMD --out FILE
      the same scaled counter bytes for every kernel of a run, and their sum over the kernels
      launched once per iteration (the PATTERN list), against the iteration's algorithmic bytes.

  python -m paper_2005_09838_amd.profile_summary mfma --counters DIR --stats DIR
         --title T --command CMD --out FILE
      matrix-core use per kernel from a run that collected SQ_INSTS_VALU_MFMA_MOPS_F32,
      SQ_INSTS_VALU_MFMA_MOPS_F64, SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE: flops per
      dispatch (each MOPS unit is 512 flops), the rate over the kernel's mean duration from a
      kernel-trace run against the dense peak of its type, and the matrix-core busy share
      (busy cycles over that duration's cycles at 2.4 GHz times the chip's 1024 SIMDs).

  python -m paper_2005_09838_amd.profile_summary timeline DIR --anchor NAME
         --per-iteration PATTERN ... --title T --command CMD --out FILE
      the kernels of one iteration in start order, from the *kernel_trace.csv of a
      kernel-trace run: the windows between consecutive starts of the anchor kernel that
      hold each PATTERN once (graph-replayed iterations), and per kernel the median start,
      end and duration relative to the window's start, with the idle time before it.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import statistics
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def source_digest() -> str:
    """SHA-256 over the library's kernel sources (the generated tube transforms excluded)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name == "tube_dft_gen.h" or not name.endswith((".hip", ".cpp", ".h", ".py")):
            continue
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _find(directory: str, suffix: str) -> list[str]:
    """The newest *suffix file under directory (one profiled process per directory)."""
    out = glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)
    if not out:
        raise SystemExit(f"no *{suffix} under {directory}")
    return [max(out, key=os.path.getmtime)]


def _short(name: str) -> str:
    """Drop the argument list and namespace of a demangled kernel name."""
    base = name.split("(")[0].strip()
    if base.startswith("void "):
        base = base[5:]
    return base.replace("tctf::", "")


def kernel_stats(directory: str):
    rows = []
    for path in _find(directory, "kernel_stats.csv"):
        with open(path) as f:
            rows += list(csv.DictReader(f))
    return rows


def write_stats(directory: str, command: str, out: str) -> None:
    rows = kernel_stats(directory)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["rocprofv3 kernel statistics", f"command: {command}", "",
             f"{'kernel':58s} {'calls':>7s} {'mean_us':>9s} {'min_us':>9s} {'max_us':>9s} {'share%':>7s}"]
    for r in rows:
        lines.append(f"{_short(r['Name'])[:58]:58s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['MinNs']) / 1e3:9.2f} {float(r['MaxNs']) / 1e3:9.2f} {float(r['Percentage']):7.2f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def counter_means(directory: str, counter: str):
    """{kernel name: (mean counter value per dispatch, dispatches)}."""
    vals = defaultdict(list)
    for path in _find(directory, "counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") == counter:
                    vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (statistics.fmean(v), len(v)) for k, v in vals.items()}


def _pick(means, pattern: str):
    """The kernel whose name contains `pattern` with the most dispatches."""
    cands = [(n, k, m) for k, (m, n) in means.items() if pattern in k]
    if not cands:
        raise SystemExit(f"no dispatch of a kernel matching {pattern!r}")
    n, k, m = max(cands)
    return k, m, n


def write_traffic(a) -> None:
    kib = 1024.0
    fk, fetch, fn = _pick(counter_means(a.fetch, "FETCH_SIZE"), a.kernel)
    wk, write, wn = _pick(counter_means(a.write, "WRITE_SIZE"), a.kernel)
    _, cfetch, _ = _pick(counter_means(a.copy_fetch, "FETCH_SIZE"), a.copy_kernel)
    _, cwrite, _ = _pick(counter_means(a.copy_write, "WRITE_SIZE"), a.copy_kernel)
    f_fetch = a.copy_bytes / (cfetch * kib)
    f_write = a.copy_bytes / (cwrite * kib)
    fetch_b = fetch * kib * f_fetch
    write_b = write * kib * f_write
    lines = [
        f"HBM traffic of the {a.stage} kernel ({a.precision}) at {a.workload}",
        f"kernel: {_short(fk)}",
        f"source_sha256: {source_digest()}",
        f"fetch_kib_per_dispatch: {fetch:.1f}",
        f"fetch_dispatches: {fn}",
        f"write_kib_per_dispatch: {write:.1f}",
        f"write_dispatches: {wn}",
        f"copy_fetch_kib_per_dispatch: {cfetch:.1f}",
        f"copy_write_kib_per_dispatch: {cwrite:.1f}",
        f"copy_bytes_each_way: {a.copy_bytes}",
        f"fetch_scale: {f_fetch:.4f}",
        f"write_scale: {f_write:.4f}",
        f"fetch_bytes_per_launch: {fetch_b:.0f}",
        f"write_bytes_per_launch: {write_b:.0f}",
        f"traffic_bytes_per_launch: {fetch_b + write_b:.0f}",
        f"algorithmic_bytes_per_launch: {a.algorithmic_bytes}",
        f"traffic_over_algorithmic: {(fetch_b + write_b) / a.algorithmic_bytes:.3f}",
        "commands:",
    ] + [f"  {c}" for c in a.command]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _scales(a):
    kib = 1024.0
    _, cfetch, _ = _pick(counter_means(a.copy_fetch, "FETCH_SIZE"), a.copy_kernel)
    _, cwrite, _ = _pick(counter_means(a.copy_write, "WRITE_SIZE"), a.copy_kernel)
    return cfetch, cwrite, a.copy_bytes / (cfetch * kib), a.copy_bytes / (cwrite * kib)


def write_all_traffic(a) -> None:
    kib = 1024.0
    fetch = counter_means(a.fetch, "FETCH_SIZE")
    write = counter_means(a.write, "WRITE_SIZE")
    cfetch, cwrite, f_fetch, f_write = _scales(a)
    lines = [a.title, f"source_sha256: {source_digest()}",
             f"copy kernel: {a.copy_bytes:.0f} bytes each way; counter reads fetch {cfetch:.1f} KiB, "
             f"write {cwrite:.1f} KiB; scales {f_fetch:.4f} (fetch), {f_write:.4f} (write)", "",
             f"{'kernel':44s} {'dispatches':>10s} {'fetch_MB':>9s} {'write_MB':>9s} {'total_MB':>9s}"]
    total = 0.0
    rows = []
    for k in sorted(set(fetch) & set(write)):
        fb = fetch[k][0] * kib * f_fetch / 1e6
        wb = write[k][0] * kib * f_write / 1e6
        rows.append((fb + wb, k, fb, wb, fetch[k][1]))
    rows.sort(reverse=True)
    for t, k, fb, wb, n in rows:
        lines.append(f"{_short(k)[:44]:44s} {n:10d} {fb:9.2f} {wb:9.2f} {t:9.2f}")
    picked = []
    for pat in a.per_iteration:
        cands = [r for r in rows if pat in r[1]]
        if not cands:
            raise SystemExit(f"no kernel matching {pat!r}")
        best = max(cands, key=lambda r: r[4])
        picked.append(best)
        total += best[0]
    lines += ["", "once per iteration: " + ", ".join(_short(r[1]) for r in picked),
              f"counter_bytes_per_iteration_MB: {total:.2f}",
              f"algorithmic_bytes_per_iteration_MB: {a.algorithmic_bytes / 1e6:.2f}",
              f"counter_over_algorithmic: {total * 1e6 / a.algorithmic_bytes:.3f}", "commands:"]
    lines += [f"  {c}" for c in a.command]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


MFMA_PEAK_TFLOPS = {"F32": 157.3, "F64": 78.6, "BF16": 2500.0}
SIMDS = 1024          # 256 compute units x 4 SIMDs
CLOCK_HZ = 2.4e9      # peak engine clock


def write_mfma(a) -> None:
    f32 = counter_means(a.counters, "SQ_INSTS_VALU_MFMA_MOPS_F32")
    f64 = counter_means(a.counters, "SQ_INSTS_VALU_MFMA_MOPS_F64")
    bf16 = counter_means(a.counters, "SQ_INSTS_VALU_MFMA_MOPS_BF16")
    busy = counter_means(a.counters, "SQ_VALU_MFMA_BUSY_CYCLES")
    dur_ns = {r["Name"]: float(r["AverageNs"]) for r in kernel_stats(a.stats)}
    lines = [a.title, f"source_sha256: {source_digest()}", "",
             f"{'kernel':40s} {'disp':>5s} {'GFLOP_f32':>9s} {'GFLOP_f64':>9s} {'GFLOP_bf16':>10s} {'mean_us':>8s} "
             f"{'TFLOP/s':>8s} {'of_peak':>8s} {'busy%':>6s}"]
    rows = []
    for k in set(f32) | set(f64) | set(bf16):
        fl = {t: c.get(k, (0.0, 0))[0] * 512 / 1e9 for t, c in (("F32", f32), ("F64", f64), ("BF16", bf16))}
        tot = sum(fl.values())
        if tot == 0.0 or k not in dur_ns:
            continue
        ns = dur_ns[k]
        rate_tf = tot / ns * 1e6   # GFLOP per ns = 1e6 TFLOP/s
        # the time the flops would take at each type's dense peak, summed, against the duration
        peak_us = sum(fl[t] * 1e9 / (MFMA_PEAK_TFLOPS[t] * 1e12) for t in fl) * 1e6
        frac = peak_us / (ns / 1e3)
        util = 100.0 * busy.get(k, (0.0, 0))[0] / (ns * 1e-9 * CLOCK_HZ * SIMDS)
        disp = max(c.get(k, (0.0, 0))[1] for c in (f32, f64, bf16))
        rows.append((tot, f"{_short(k)[:40]:40s} {disp:5d} {fl['F32']:9.4f} {fl['F64']:9.4f} {fl['BF16']:10.4f} "
                          f"{ns / 1e3:8.2f} {rate_tf:8.2f} {frac:8.4f} {util:6.2f}"))
    rows.sort(reverse=True)
    lines += [r[1] for r in rows]
    lines += ["",
              "GFLOP: SQ_INSTS_VALU_MFMA_MOPS_* x 512 per dispatch (counter run); mean_us: the kernel's",
              "mean duration in the kernel-trace run; of_peak: the time the flops take at the dense MFMA",
              "peaks (FP32 157.3, FP64 78.6, BF16 2500 TFLOP/s) over that duration; busy%:",
              "SQ_VALU_MFMA_BUSY_CYCLES over mean duration x 2.4 GHz x 1024 SIMDs",
              "(GRBM_GUI_ACTIVE of a counter-run dispatch includes the profiler's serialisation, so it",
              "is not used as the denominator)",
              "commands:"] + [f"  {c}" for c in a.command]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def write_timeline(a) -> None:
    path = glob.glob(os.path.join(a.directory, "**", "*kernel_trace.csv"), recursive=True)[0]
    with open(path) as f:
        rows = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in csv.DictReader(f)]
    rows.sort()
    starts = [i for i, r in enumerate(rows) if a.anchor in r[2]]
    windows = []
    for i0, i1 in zip(starts, starts[1:]):
        ker = rows[i0:i1]
        picked = []
        for pat in a.per_iteration:
            hits = [k for k in ker if pat in k[2]]
            if len(hits) != 1:
                break
            picked.append(hits[0])
        else:
            if len(ker) == len(a.per_iteration):
                windows.append((rows[i1][0] - rows[i0][0], rows[i0][0], picked))
    if not windows:
        raise SystemExit("no iteration window holds every pattern once")
    period = statistics.median(w[0] for w in windows)
    windows = [w for w in windows if abs(w[0] - period) <= 0.2 * period]
    lines = [a.title, f"source_sha256: {source_digest()}",
             f"iterations: {len(windows)} (graph-replayed windows between starts of {a.anchor})",
             f"median period_us: {period / 1000:.2f}", "",
             f"{'kernel':32s} {'start_us':>9s} {'end_us':>9s} {'dur_us':>8s} {'idle_before_us':>15s}"]
    med = []
    for j in range(len(a.per_iteration)):
        st = statistics.median((w[2][j][0] - w[1]) / 1000 for w in windows)
        en = statistics.median((w[2][j][1] - w[1]) / 1000 for w in windows)
        med.append((st, en, _short(windows[0][2][j][2])))
    med.sort()
    busy_end = 0.0
    for st, en, name in med:
        lines.append(f"{name[:32]:32s} {st:9.2f} {en:9.2f} {en - st:8.2f} {max(0.0, st - busy_end):15.2f}")
        busy_end = max(busy_end, en)
    lines.append(f"{'(next iteration)':32s} {period / 1000:9.2f} {'':9s} {'':8s} "
                 f"{max(0.0, period / 1000 - busy_end):15.2f}")
    lines += ["", "idle_before_us: from the latest end among the earlier kernels to this start (0 when they overlap)",
              "commands:"] + [f"  {c}" for c in a.command]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("directory")
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "kernel", "stage", "precision", "workload", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-kernel", default="elementwise")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--algorithmic-bytes", type=float, required=True)
    t.add_argument("--command", action="append", required=True)
    t = sub.add_parser("all-traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "title", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-kernel", default="elementwise")
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--algorithmic-bytes", type=float, required=True)
    t.add_argument("--per-iteration", nargs="+", required=True)
    t.add_argument("--command", action="append", required=True)
    m = sub.add_parser("mfma")
    for k in ("counters", "stats", "title", "out"):
        m.add_argument("--" + k, required=True)
    m.add_argument("--command", action="append", required=True)
    tl = sub.add_parser("timeline")
    tl.add_argument("directory")
    for k in ("anchor", "title", "out"):
        tl.add_argument("--" + k, required=True)
    tl.add_argument("--per-iteration", nargs="+", required=True)
    tl.add_argument("--command", action="append", required=True)
    a = ap.parse_args()
    if a.what == "stats":
        write_stats(a.directory, a.command, a.out)
    elif a.what == "traffic":
        write_traffic(a)
    elif a.what == "all-traffic":
        write_all_traffic(a)
    elif a.what == "timeline":
        write_timeline(a)
    else:
        write_mfma(a)


if __name__ == "__main__":
    main()
