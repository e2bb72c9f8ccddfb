"""Summaries of rocprofv3 CSV output for the kernels of this library.

Four summaries, all short markdown files:

* ``stats``: the ``*_kernel_stats.csv`` of a ``--kernel-trace --stats -f csv`` run, as a table of
  calls / total / average per kernel.
* ``traffic``: HBM bytes per dispatch of one kernel from two ``--pmc`` runs (``FETCH_SIZE``, then
  ``WRITE_SIZE``, each in KiB per dispatch), each scaled by what the same counter reads for a plain
  copy-like kernel of known size run in the same process (1 GiB read and 1 GiB written). The result
  is embedded as a JSON block tagged with the SHA-256 of the kernel source it was measured on, so a
  reader can tell when the numbers have gone stale.
* ``counters``: per-dispatch means of any ``--pmc`` counters (several CSVs, one per pass) for each
  kernel, with the ratios that say where a kernel's waves spend their time.
* ``busy``: from the ``*_kernel_trace.csv`` of a ``--kernel-trace -f csv`` run, the share of each
  time bin during which at least one kernel ran, and the idle gaps longer than a threshold (where
  the device waited for the host).

  python -m paper_2604_11659_amd.profiling stats CSV --title T --command C --out FILE
  python -m paper_2604_11659_amd.profiling traffic FETCH_CSV WRITE_CSV --kernel REGEX --label NAME \
      --calib REGEX --calib-bytes 1073741824 --title T --command C --out FILE
  python -m paper_2604_11659_amd.profiling counters CSV [CSV ...] --kernel REGEX --title T --command C --out FILE
  python -m paper_2604_11659_amd.profiling busy TRACE_CSV [--bin-ms 100] [--gap-ms 5] [--active 0.5] --title T --command C --out FILE
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hip")
TRAFFIC_TAG = "fhe-traffic"


def kernel_source_sha256(path: str = KERNEL_SOURCE) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def short_name(name: str) -> str:
    n = name.replace("fhe::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", n).strip()


def stats_markdown(csv_path: str, title: str, command: str, note: str = "") -> str:
    rows = list(csv.DictReader(open(csv_path)))
    total = sum(int(r["TotalDurationNs"]) for r in rows)
    out = [f"# {title}", ""]
    if note:
        out += [note, ""]
    out += ["Command (from the repository root):", "", "```", command, "```", "",
            f"Total kernel time: {total / 1e9:.3f} s over {sum(int(r['Calls']) for r in rows)} dispatches.", "",
            "| kernel | calls | total (ms) | avg (us) | % |", "|---|---|---|---|---|"]
    for r in rows:
        if float(r["Percentage"]) < 0.05:
            continue
        out.append(f"| `{short_name(r['Kernel_Name'] if 'Kernel_Name' in r else r['Name'])}` | {r['Calls']} | "
                   f"{int(r['TotalDurationNs']) / 1e6:.1f} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def _per_kernel(csv_path: str, counter: str) -> dict[str, list[float]]:
    agg: dict[str, list[float]] = defaultdict(list)
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return agg


def _pick(agg: dict[str, list[float]], regex: str) -> list[float]:
    vals: list[float] = []
    for name, v in agg.items():
        if re.search(regex, name):
            vals += v
    return vals


def traffic(fetch_csv: str, write_csv: str, kernel: str, calib: str, calib_bytes: float) -> dict:
    """Calibrated HBM bytes per dispatch of the kernels matching `kernel`."""
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")
    fk, wk = _pick(f, kernel), _pick(w, kernel)
    fc, wc = _pick(f, calib), _pick(w, calib)
    if not fk or not wk or not fc or not wc:
        raise SystemExit("kernel or calibration kernel missing from the counter files")
    # the calibration kernel reads and writes calib_bytes; counters are in KiB
    f_scale = calib_bytes / (max(fc) * 1024.0)
    w_scale = calib_bytes / (max(wc) * 1024.0)
    fetch = sum(fk) / len(fk) * 1024.0 * f_scale
    write = sum(wk) / len(wk) * 1024.0 * w_scale
    return {"dispatches": len(fk), "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
            "bytes_per_launch": fetch + write, "fetch_scale": f_scale, "write_scale": w_scale,
            "raw_fetch_kib_per_launch": sum(fk) / len(fk), "raw_write_kib_per_launch": sum(wk) / len(wk)}


def traffic_markdown(t: dict, label: str, title: str, command: str, note: str = "") -> str:
    block = dict(t, kernel=label, source_sha256=kernel_source_sha256())
    out = [f"# {title}", ""]
    if note:
        out += [note, ""]
    out += ["Commands (from the repository root; one counter per run):", "", "```", command, "```", "",
            f"* FETCH_SIZE scale (1 GiB copy-like kernel): x{t['fetch_scale']:.3f}; "
            f"WRITE_SIZE scale: x{t['write_scale']:.3f}",
            f"* `{label}`: {t['dispatches']} dispatches; per dispatch "
            f"{t['fetch_bytes_per_launch'] / 1e9:.3f} GB read + {t['write_bytes_per_launch'] / 1e9:.3f} GB written "
            f"= {t['bytes_per_launch'] / 1e9:.3f} GB (raw {t['raw_fetch_kib_per_launch']:.0f} KiB fetched, "
            f"{t['raw_write_kib_per_launch']:.0f} KiB written)", "",
            f"```{TRAFFIC_TAG}", json.dumps(block, indent=1), "```", ""]
    return "\n".join(out)


def counters_markdown(csv_paths: list[str], kernel: str, title: str, command: str, note: str = "") -> str:
    """Per-dispatch means of every counter in the CSVs for the kernels matching `kernel`."""
    agg: dict[str, dict[str, list[float]]] = defaultdict(lambda: defaultdict(list))
    for path in csv_paths:
        for r in csv.DictReader(open(path)):
            if re.search(kernel, r["Kernel_Name"]):
                agg[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for cs in agg.values() for c in cs})
    out = [f"# {title}", ""]
    if note:
        out += [note, ""]
    out += ["Commands (from the repository root; one run per counter set):", "", "```", command, "```", "",
            "Per-dispatch means (counters as the device reports them, summed over its units):", "",
            "| kernel | dispatches | " + " | ".join(names) + " |", "|---" * (len(names) + 2) + "|"]
    for k, cs in sorted(agg.items()):
        n = max(len(v) for v in cs.values())
        out.append(f"| `{k}` | {n} | " + " | ".join(
            f"{sum(cs[c]) / len(cs[c]):.4g}" if cs.get(c) else "" for c in names) + " |")
    ratios = [("SQ_INSTS_VALU", "SQ_WAVES", "VALU instructions per wave"),
              ("SQ_INSTS_LDS", "SQ_WAVES", "LDS instructions per wave"),
              ("SQ_INSTS_VMEM_RD", "SQ_WAVES", "vector memory reads per wave"),
              ("SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES", "share of wave cycles waiting on a dependency (s_waitcnt)"),
              ("SQ_WAIT_ANY", "SQ_WAVE_CYCLES", "share of wave cycles waiting on anything"),
              ("SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES", "share of wave cycles issuing VALU"),
              ("SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS", "LDS bank-conflict cycles per LDS-active cycle")]
    rows = []
    for k, cs in sorted(agg.items()):
        vals = []
        for a, b, _ in ratios:
            if cs.get(a) and cs.get(b) and sum(cs[b]):
                vals.append(f"{sum(cs[a]) / sum(cs[b]):.3g}")
            else:
                vals.append("")
        rows.append(f"| `{k}` | " + " | ".join(vals) + " |")
    out += ["", "| kernel | " + " | ".join(t for _, _, t in ratios) + " |", "|---" * (len(ratios) + 1) + "|", *rows]
    return "\n".join(out) + "\n"


def busy_intervals(csv_path: str) -> list[list[int]]:
    """Union of the kernels' [start, end) intervals (ns), in time order."""
    spans = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in csv.DictReader(open(csv_path)))
    merged: list[list[int]] = []
    for s, e in spans:
        if merged and s <= merged[-1][1]:
            merged[-1][1] = max(merged[-1][1], e)
        else:
            merged.append([s, e])
    return merged


def busy_bins(merged: list[list[int]], bin_ns: float) -> list[float]:
    """Share of each bin of `bin_ns` (from the first kernel's start) covered by `merged`."""
    t0 = merged[0][0]
    nb = int((merged[-1][1] - t0) // bin_ns) + 1
    cover = [0.0] * nb
    for s, e in merged:
        a, b = s - t0, e - t0
        while a < b:
            k = int(a // bin_ns)
            edge = min(b, (k + 1) * bin_ns)
            cover[k] += edge - a
            a = edge
    return [c / bin_ns for c in cover]


def busy_markdown(csv_path: str, title: str, command: str, note: str = "", bin_ms: float = 100.0,
                  gap_ms: float = 5.0, active: float = 0.5) -> str:
    """Busy share per bin over the whole trace; the compute phase is the stretch from the first to the
    last bin at least `active` busy, and its idle gaps longer than `gap_ms` are listed."""
    merged = busy_intervals(csv_path)
    bin_ns = bin_ms * 1e6
    bins = busy_bins(merged, bin_ns)
    t0, t1 = merged[0][0], merged[-1][1]
    busy_ns = sum(e - s for s, e in merged)
    hot = [i for i, b in enumerate(bins) if b >= active]
    out = [f"# {title}", ""]
    if note:
        out += [note, ""]
    out += ["Commands (from the repository root):", "", "```", command, "```", "",
            f"Span from the first kernel's start to the last kernel's end: {(t1 - t0) / 1e9:.3f} s; at least one "
            f"kernel running {busy_ns / 1e9:.3f} s of it ({busy_ns / (t1 - t0):.3f}).", "",
            f"Share of each {bin_ms:g} ms bin with a kernel running:", "", "```"]
    for i in range(0, len(bins), 20):
        out.append(f"{i * bin_ms / 1e3:7.1f} s  " + " ".join(f"{b:.2f}" for b in bins[i:i + 20]))
    out += ["```", ""]
    if not hot:
        return "\n".join(out + [f"No bin is {active:g} busy.", ""])
    wa, wb = t0 + hot[0] * bin_ns, t0 + (hot[-1] + 1) * bin_ns
    in_w = sum(max(0.0, min(e, wb) - max(s, wa)) for s, e in merged)
    gaps = [(merged[i][1] - t0, merged[i + 1][0] - merged[i][1]) for i in range(len(merged) - 1)
            if merged[i + 1][0] - merged[i][1] > gap_ms * 1e6 and wa <= merged[i][1] and merged[i + 1][0] <= wb]
    out += [f"Compute phase (from the first to the last bin at least {active:g} busy): "
            f"{(wa - t0) / 1e9:.1f}-{(wb - t0) / 1e9:.1f} s, a kernel running {in_w / (wb - wa):.4f} of it. "
            f"Idle gaps longer than {gap_ms:g} ms inside it (start from the first kernel, length):", ""]
    out += [f"* {g0 / 1e9:.3f} s: {g / 1e6:.1f} ms" for g0, g in gaps] or ["* none"]
    return "\n".join(out) + "\n"


def load_traffic(profiles_dir: str, label: str) -> dict | None:
    """The traffic block for `label` measured on the current kernel source, if any."""
    if not os.path.isdir(profiles_dir):
        return None
    sha = kernel_source_sha256()
    for fn in sorted(os.listdir(profiles_dir)):
        if not fn.endswith(".md"):
            continue
        text = open(os.path.join(profiles_dir, fn)).read()
        for m in re.finditer(r"```" + TRAFFIC_TAG + r"\n(.*?)\n```", text, re.S):
            try:
                block = json.loads(m.group(1))
            except json.JSONDecodeError:
                continue
            if block.get("kernel") == label and block.get("source_sha256") == sha:
                return dict(block, file=fn)
    return None


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--kernel", required=True)
    t.add_argument("--label", required=True)
    t.add_argument("--calib", required=True)
    t.add_argument("--calib-bytes", type=float, default=float(1 << 30))
    c = sub.add_parser("counters")
    c.add_argument("csvs", nargs="+")
    c.add_argument("--kernel", required=True)
    b = sub.add_parser("busy")
    b.add_argument("csv")
    b.add_argument("--bin-ms", type=float, default=100.0)
    b.add_argument("--gap-ms", type=float, default=5.0)
    b.add_argument("--active", type=float, default=0.5)
    for p in (s, t, c, b):
        p.add_argument("--title", required=True)
        p.add_argument("--command", required=True)
        p.add_argument("--note", default="")
        p.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        text = stats_markdown(a.csv, a.title, a.command, a.note)
    elif a.cmd == "counters":
        text = counters_markdown(a.csvs, a.kernel, a.title, a.command, a.note)
    elif a.cmd == "busy":
        text = busy_markdown(a.csv, a.title, a.command, a.note, a.bin_ms, a.gap_ms, a.active)
    else:
        text = traffic_markdown(traffic(a.fetch_csv, a.write_csv, a.kernel, a.calib, a.calib_bytes), a.label,
                                a.title, a.command, a.note)
    with open(a.out, "w") as f:
        f.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
