"""HBM bytes per launch of the heavy-row kernels from rocprofv3 counters.

Two counter runs of the headline bench command, one with FETCH_SIZE and one
with WRITE_SIZE (KiB per dispatch), and the same two counters over a plain
elementwise kernel that reads and writes a known number of bytes
(`bench.py --copy-calibration`: torch.neg over 1 GiB of float32).  The
copy kernel's reading fixes one scale factor per counter; each kernel's
bytes per launch are the mean over its dispatches (after `--skip` leading
ones) of fetch * factor + write * factor.  Writes hbm_traffic_gfx950.json
next to this file, stamped with the digest of the HIP sources (bench.py
reports the figure only while the sources are unchanged), and prints a
markdown table of the readings.

    python paper_2509_18024_amd/tuning/traffic_digest.py --fetch DIR --write DIR \\
        --copy-fetch DIR --copy-write DIR --skip 4 --kernels k_heavy_select k_heavy_gram_x6
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "hbm_traffic_gfx950.json")
COPY_BYTES = 1 << 30  # bytes read and written by one calibration launch


def readings(directory: str, counter: str) -> dict:
    """Kernel short name -> counter values per dispatch (KiB), in dispatch order."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {directory}")
    rows = []
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    rows.append(r)
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    out: dict = {}
    for r in rows:
        m = re.search(r"(k_[A-Za-z0-9_]+)", r["Kernel_Name"])
        name = m.group(1) if m else ("elementwise" if "elementwise" in r["Kernel_Name"] else r["Kernel_Name"])
        out.setdefault(name, []).append(float(r["Counter_Value"]))
    return out


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--skip", type=int, default=0, help="leading dispatches of each kernel to leave out")
    ap.add_argument("--kernels", nargs="+", default=["k_heavy_select", "k_heavy_gram_x6"])
    ap.add_argument("--workload", default="c3_batched core r=1/10 fp32")
    ap.add_argument("--out", default=OUT, help="digest file (default: next to this script)")
    args = ap.parse_args()

    sys.path.insert(0, ROOT)
    from bench import kernel_source_digest

    cf = readings(args.copy_fetch, "FETCH_SIZE").get("elementwise", [])
    cw = readings(args.copy_write, "WRITE_SIZE").get("elementwise", [])
    if not cf or not cw:
        raise SystemExit("no elementwise dispatch in the calibration runs")
    kib = COPY_BYTES / 1024.0
    ff = kib / (sum(cf) / len(cf))
    fw = kib / (sum(cw) / len(cw))
    fetch = readings(args.fetch, "FETCH_SIZE")
    write = readings(args.write, "WRITE_SIZE")
    digest = {"workload": args.workload, "source_sha256": kernel_source_digest(), "fetch_factor": ff,
              "write_factor": fw, "kernels": {}}
    lines = ["| Quantity | Value |", "|---|---|",
             f"| copy kernel FETCH_SIZE per launch (KiB) | {sum(cf) / len(cf):.0f} (true {kib:.0f}) -> factor {ff:.4f} |",
             f"| copy kernel WRITE_SIZE per launch (KiB) | {sum(cw) / len(cw):.0f} (true {kib:.0f}) -> factor {fw:.4f} |"]
    for k in args.kernels:
        fv = fetch.get(k, [])[args.skip:]
        wv = write.get(k, [])[args.skip:]
        if not fv or not wv or len(fv) != len(wv):
            raise SystemExit(f"{k}: dispatch counts differ or are missing ({len(fv)} fetch, {len(wv)} write)")
        fb = sum(fv) / len(fv) * 1024.0 * ff
        wb = sum(wv) / len(wv) * 1024.0 * fw
        digest["kernels"][k] = {"hbm_bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb,
                                "write_bytes_per_launch": wb, "dispatches": len(fv),
                                "summary": f"profiles/hbm_traffic_{k}_c3_core_r10.md"}
        lines.append(f"| `{k}` FETCH_SIZE per dispatch (KiB) | {' / '.join(f'{v:.0f}' for v in fv)} |")
        lines.append(f"| `{k}` WRITE_SIZE per dispatch (KiB) | {' / '.join(f'{v:.0f}' for v in wv)} |")
        lines.append(f"| `{k}` scaled HBM bytes per launch (mean over {len(fv)} dispatches) | "
                     f"{(fb + wb) / 1e9:.3f} GB (fetch {fb / 1e9:.3f} + write {wb / 1e9:.3f}) |")
    with open(args.out, "w") as f:
        json.dump(digest, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
