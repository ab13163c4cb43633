"""Summaries of rocprofv3 output for the Trotter-step kernels (measurement).

Reads the CSV files that rocprofv3 writes (`--kernel-trace --stats`,
`--pmc ...`) and prints Markdown tables: per-kernel call counts and average
durations, HBM traffic per dispatch from FETCH_SIZE / WRITE_SIZE scaled by
a plain device copy and fill of known size measured in the same run, and
VALU / LDS / memory instruction counts with the VALU issue time they imply
(a wave64 VALU instruction occupies its SIMD for 4 cycles on CDNA).
Optionally writes the traffic table the benchmark reads (profiles/traffic.json).

    python -m paper_2409_12240_amd.rocprof_summary --stats DIR --fetch DIR --write DIR --sq DIR
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

KERNELS = {
    "k_simple_update": "simple_update",
    "k_bp_class": "bp_sweep",
    "k_canonicalise": "canonicalise",
    "k_gauge_apply": "gauge_apply",
    "k16_su_qr": "simple_update",
    "k16_su_core": "simple_update",
    "k16_su_apply": "simple_update",
    "k16_bp_class": "bp_sweep",
    "k16_canonicalise": "canonicalise",
    "k16_gauge_apply": "gauge_apply",
}
SIMDS = 256 * 4            # MI355X: 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def source_sha256() -> str:
    """Hash of the kernel sources (the chi <= 8 and chi = 16 kernels and the
    device helpers they include): profile records are valid only for this
    source."""
    h = hashlib.sha256()
    for name in ("gtqa_kernels.hip", "gtqa_device.h", "gtqa_wide.hip"):
        with open(os.path.join(ROOT, "paper_2409_12240_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _csv(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return list(csv.DictReader(open(hits[0])))


def stats_table(d):
    rows = _csv(d, "kernel_stats.csv")
    out = ["| Kernel | Calls | Average (us) | Share |", "|---|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["Percentage"]))[:12]:
        out.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.1f}% |")
    return "\n".join(out)


def _per_kernel(rows, counter, last=None):
    acc = collections.defaultdict(list)
    for r in rows:
        if r["Counter_Name"] == counter:
            acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (v[-last:] if last else v) for k, v in acc.items()}


def _calib(per, needle):
    """Counter value of the calibration kernel: the largest single dispatch
    among kernels whose name contains `needle` (copy / fill of 1 GiB)."""
    best = 0.0
    for k, v in per.items():
        if needle in k.lower():
            best = max(best, max(v))
    return best


def is_companion(name: str) -> bool:
    """A kernel that runs beside its stage's main launch rather than instead
    of it: the simple update's every-pair redo launch (FIX = true), and at
    chi = 16 the core SVD and the Q application after the QR launch."""
    if "k16_su_core" in name or "k16_su_apply" in name:
        return True
    return "k_simple_update<" in name and name.split(">")[0].rstrip().endswith("true")


def traffic_table(fetch_dir, write_dir, calib_bytes, items, last=200, chi=4, precision="mixed", calls=None):
    fr = _csv(fetch_dir, "counter_collection.csv")
    wr = _csv(write_dir, "counter_collection.csv")
    fper = _per_kernel(fr, "FETCH_SIZE")
    wper = _per_kernel(wr, "WRITE_SIZE")
    fcal = _calib(fper, "copy")
    wcal = _calib(wper, "fill")
    fscale = calib_bytes / 1024.0 / fcal if fcal else None
    wscale = calib_bytes / 1024.0 / wcal if wcal else None
    lines = [f"Calibration in the same runs: a {calib_bytes / 2**30:g} GiB device copy reads as {fcal:.0f} KiB "
             f"in FETCH_SIZE (scale {fscale:.3f}); a fill of the same size writes {wcal:.0f} KiB in WRITE_SIZE "
             f"(scale {wscale:.3f}).  Means over the last {last} dispatches of each kernel.", "",
             "| Kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | Traffic (MB, scaled) |", "|---|---:|---:|---:|"]
    rec = []
    sha = source_sha256()
    for name in sorted(fper):
        stage = next((s for k, s in KERNELS.items() if k in name), None)
        if stage is None or name not in wper:
            continue
        f = fper[name][-last:]
        w = wper[name][-last:]
        fk, wk = sum(f) / len(f), sum(w) / len(w)
        tb = (fk * fscale + wk * wscale) * 1024.0
        lines.append(f"| `{name[:80]}` | {fk:.0f} | {wk:.0f} | {tb / 1e6:.1f} |")
        rec.append({"kernel": name, "stage": stage, "chi": chi, "precision": precision,
                    "items_per_launch": items.get(stage), "source_sha256": sha, "dispatches": len(f),
                    "fetch_kib": fk, "write_kib": wk, "traffic_bytes_per_launch": round(tb),
                    "calls": (calls or {}).get(name), "companion": is_companion(name)})
    return "\n".join(lines), {"fetch_scale": fscale, "write_scale": wscale, "kernels": rec}


def sq_records(sq_dir, durations_us, last=100, chi=4, precision="mixed"):
    """Per-kernel mean SQ counts and the VALU issue time they imply."""
    rows = _csv(sq_dir, "counter_collection.csv")
    cols = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"]
    per = {c: _per_kernel(rows, c, last) for c in cols}
    out = []
    for n in sorted({r["Kernel_Name"] for r in rows}):
        stage = next((s for k, s in KERNELS.items() if k in n), None)
        if stage is None:
            continue
        m = {c: (sum(per[c][n]) / len(per[c][n]) if per[c].get(n) else 0.0) for c in cols}
        issue_us = m["SQ_INSTS_VALU"] * 4 / SIMDS / CLOCK_HZ * 1e6
        dur = next((v for k, v in durations_us.items() if k == n), None)
        out.append({"kernel": n, "stage": stage, "chi": chi, "precision": precision, **{c.lower(): m[c] for c in cols},
                    "valu_issue_us": issue_us, "duration_us": dur,
                    "valu_busy": (issue_us / dur) if dur else None})
    return out


def sq_table(sq_dir, durations_us, last=100):
    rows = _csv(sq_dir, "counter_collection.csv")
    names = sorted({r["Kernel_Name"] for r in rows})
    cols = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"]
    per = {c: _per_kernel(rows, c, last) for c in cols}
    out = ["| Kernel | Waves | VALU / wave | LDS / wave | SALU / wave | VMEM rd+wr / wave | VALU issue (us) | "
           "Duration (us) | VALU busy |", "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for n in names:
        if not any(k in n for k in KERNELS):
            continue
        m = {c: (sum(per[c][n]) / len(per[c][n]) if per[c].get(n) else 0.0) for c in cols}
        waves = m["SQ_WAVES"] or 1.0
        issue_us = m["SQ_INSTS_VALU"] * 4 / SIMDS / CLOCK_HZ * 1e6
        dur = next((v for k, v in durations_us.items() if k == n), None)
        busy = f"{issue_us / dur:.0%}" if dur else "n/a"
        out.append(f"| `{n[:70]}` | {m['SQ_WAVES']:.0f} | {m['SQ_INSTS_VALU'] / waves:.0f} | "
                   f"{m['SQ_INSTS_LDS'] / waves:.0f} | {m['SQ_INSTS_SALU'] / waves:.0f} | "
                   f"{(m['SQ_INSTS_VMEM_RD'] + m['SQ_INSTS_VMEM_WR']) / waves:.1f} | {issue_us:.1f} | "
                   f"{dur if dur is None else round(dur, 1)} | {busy} |")
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--stats")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--sq")
    ap.add_argument("--calib-mib", type=int, default=1024)
    ap.add_argument("--items", type=str, default="simple_update=96000,bp_sweep=96000,canonicalise=384000,"
                                                  "gauge_apply=256000")
    ap.add_argument("--traffic-json", type=str, default=None)
    ap.add_argument("--append", action="store_true",
                    help="add this run's records to an existing --traffic-json instead of replacing it")
    ap.add_argument("--chi", type=int, default=4)
    ap.add_argument("--precision", type=str, default="mixed")
    a = ap.parse_args(argv)
    items = {k: int(v) for k, v in (x.split("=") for x in a.items.split(","))}
    durations, calls = {}, {}
    if a.stats:
        print("## Kernel time\n")
        print(stats_table(a.stats))
        for r in _csv(a.stats, "kernel_stats.csv"):
            durations[r["Name"]] = float(r["AverageNs"]) / 1e3
            calls[r["Name"]] = int(r["Calls"])
        print()
    if a.fetch and a.write:
        print("## HBM traffic per dispatch\n")
        txt, rec = traffic_table(a.fetch, a.write, a.calib_mib << 20, items, chi=a.chi, precision=a.precision,
                                 calls=calls)
        print(txt)
        print()
        if a.traffic_json:
            rec["note"] = ("HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE passes, scaled by a "
                           "device copy (FETCH) and fill (WRITE) of known size measured in the same runs; valid "
                           "only for the kernel source with this sha256")
            if a.append and os.path.exists(a.traffic_json):
                with open(a.traffic_json) as fh:
                    old = json.load(fh)
                old["kernels"] = old.get("kernels", []) + rec["kernels"]
                rec = old
            with open(a.traffic_json, "w") as fh:
                json.dump(rec, fh, indent=1)
    if a.sq:
        print("## Instruction counts (SQ counters)\n")
        print(sq_table(a.sq, durations))
        if a.traffic_json:
            with open(a.traffic_json) as fh:
                rec = json.load(fh)
            rec["sq"] = (rec.get("sq", []) if a.append else []) + sq_records(a.sq, durations, chi=a.chi,
                                                                             precision=a.precision)
            with open(a.traffic_json, "w") as fh:
                json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
