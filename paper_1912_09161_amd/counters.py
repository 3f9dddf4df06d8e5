"""HBM traffic per launch from rocprofv3 hardware-counter runs.

Input: the counter_collection.csv files of two `rocprofv3 --pmc` runs of
bench.py (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) made with
`--copy-mb M`, which ends with four device-to-device copies of M MiB.  The
copies calibrate the counters: factor = bytes moved / bytes counted.

Output: per kernel and per stage (cluster, find_tracks, fit) the calibrated
HBM bytes per launch (one launch = one step of the benchmark), tagged with the
digest of the kernel sources they were measured on, as JSON.

    python -m paper_1912_09161_amd.counters FETCH.csv WRITE.csv COPY_MB OUT.json
"""
from __future__ import annotations

import csv
import json
import sys
from collections import defaultdict

STAGE_OF = [("k_offsets", "cluster"), ("k_validate", "cluster"), ("k_small", "cluster"), ("k_mid", "cluster"),
            ("k_finalize", "cluster"), ("k_clear_counts", "find_tracks"), ("k_phi_tables", "find_tracks"),
            ("k_find", "find_tracks"),
            ("k_fit", "fit")]


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def _short(name: str) -> str:
    n = name.split("(")[0].replace("void ", "")
    return n.split("::")[-1] if "::" in n else n


def summarize(fetch_csv: str, write_csv: str, copy_mb: int) -> dict:
    from .build import source_digest
    out = {"source_digest": source_digest(), "copy_mb": copy_mb}
    per = {}
    for label, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _rows(path)
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        big = max(int(r["Grid_Size"]) for r in copies)
        cal = [float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == big]
        counted = sum(cal) / len(cal) * 1024.0
        factor = (copy_mb << 20) / counted
        out[f"{label}_factor"] = round(factor, 4)
        out[f"{label}_copy_counted_bytes"] = round(counted)
        k = defaultdict(float)
        n = defaultdict(int)
        for r in rows:
            name = _short(r["Kernel_Name"])
            if not name.startswith("k_"):
                continue
            k[name] += float(r["Counter_Value"]) * 1024.0 * factor
            n[name] += 1
        per[label] = (k, n)
    steps = max(per["fetch"][1].get("k_validate", 0), 1)
    kernels = {}
    stages = defaultdict(float)
    for name in sorted(set(per["fetch"][0]) | set(per["write"][0])):
        fb = per["fetch"][0].get(name, 0.0) / steps
        wb = per["write"][0].get(name, 0.0) / steps
        kernels[name] = dict(fetch_bytes_per_launch=round(fb), write_bytes_per_launch=round(wb),
                             dispatches_per_launch=per["fetch"][1].get(name, 0) / steps)
        for prefix, stage in STAGE_OF:
            if name.startswith(prefix):
                stages[stage] += fb + wb
                break
    out["steps"] = steps
    out["kernels"] = kernels
    out["stage_bytes_per_launch"] = {s: round(v) for s, v in stages.items()}
    return out


if __name__ == "__main__":
    fetch, write, mb, dst = sys.argv[1], sys.argv[2], int(sys.argv[3]), sys.argv[4]
    res = summarize(fetch, write, mb)
    with open(dst, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res["stage_bytes_per_launch"]), res["fetch_factor"], res["write_factor"])
