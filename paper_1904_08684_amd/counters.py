"""HBM traffic records from rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE,
KiB per dispatch, one counter per run), scaled by what the same counters read
for a plain device copy of known size in the same run.

    python -m paper_1904_08684_amd.counters fused --fetch F.csv --write W.csv \\
        --n 513 --copy-mib 2048 --out profiles/gs_fused_513cubed_counters.json
    python -m paper_1904_08684_amd.counters vcycle --fetch F.csv --write W.csv \\
        --n 513 --cycles 16 --calib profiles/gs_fused_513cubed_counters.json \\
        --out profiles/vcycle_513cubed_fp64_traffic.json

F.csv / W.csv are the counter_collection CSVs of runs of
`paper_1904_08684_amd.kbench --ops smooth,copy` (fused) or of
`bench.py --steps 1 --warmup 0 --no-mixed --no-serve --no-configs
--no-cpu-baseline` (vcycle: every dispatch of its two solves, calibrated
by the fused record's copy).  The records carry the hash of the
dominant kernel's source (bench.kernel_source_hash), and bench.py reports
their traffic only while that hash is unchanged.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

COPY_KERNEL = "copyBuffer"      # the runtime's device-to-device copy kernel
SETUP_KERNELS = ("k_pack", "k_unpack", "k_zero", "k_copy", "elementwise", "copyBuffer", "fill", "distribution")


def read(path: str, counter: str):
    """{dispatch id: (kernel name, grid size, value)} for one counter."""
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            name, grid = r["Kernel_Name"], int(r["Grid_Size"])
            v = float(r["Counter_Value"])
            if d in out:
                v += out[d][2]
            out[d] = (name, grid, v)
    return out


def short(name: str) -> str:
    """Kernel name without namespaces and argument list."""
    base = name.replace("(anonymous namespace)::", "").split("(")[0]
    for pre in ("void ", "mg::"):
        base = base.replace(pre, "")
    return base.strip()


def calibrate(rows, nbytes: int) -> float:
    """bytes per counted KiB, from the largest copy dispatch of nbytes bytes."""
    vals = [v for (name, _, v) in rows.values() if COPY_KERNEL in name]
    if not vals:
        raise SystemExit("no copy dispatch in the run to calibrate against")
    return nbytes / max(vals)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("fused", "vcycle"))
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--n", type=int, default=513)
    ap.add_argument("--copy-mib", type=int, default=2048)
    ap.add_argument("--cycles", type=int, default=16, help="V-cycles in the run (vcycle mode)")
    ap.add_argument("--calib", help="a record whose copy calibration to reuse when the run has no copy")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    sys.path.insert(0, ROOT)
    import bench

    fetch = read(a.fetch, "FETCH_SIZE")
    write = read(a.write, "WRITE_SIZE")
    nbytes = a.copy_mib << 20
    if a.calib:
        cal = json.load(open(a.calib))["copy_calibration"]
        nbytes, fsc, wsc = cal["bytes_read_and_written"], cal["fetch_bytes_per_kib"], cal["write_bytes_per_kib"]
    else:
        fsc, wsc = calibrate(fetch, nbytes), calibrate(write, nbytes)
    unknowns = (a.n - 2) ** 3
    rec = {"kernel_source_sha256_16": bench.kernel_source_hash(),
           "copy_calibration": {"bytes_read_and_written": nbytes, "fetch_bytes_per_kib": fsc,
                                "write_bytes_per_kib": wsc}}
    if a.mode == "fused":
        # the finest level's fused pass: the launches with the largest grid
        def pick(rows):
            tb = [(g, v) for (name, g, v) in rows.values() if "k_node_gs_tb<double, 6" in name]
            gmax = max(g for g, _ in tb)
            return [v for g, v in tb if g == gmax]
        fv, wv = pick(fetch), pick(write)
        rec.update({
            "kernel": f"k_node_gs_tb<double, 6, 3, 12, 6, true, true> (finest-level FP64 fused pass of three "
                      f"red-black sweeps, {a.n}^3)",
            "launches": len(fv),
            "fetch_size_kib_raw_avg": sum(fv) / len(fv),
            "write_size_kib_raw_avg": sum(wv) / len(wv),
            "hbm_fetch_bytes_per_launch": fsc * sum(fv) / len(fv),
            "hbm_write_bytes_per_launch": wsc * sum(wv) / len(wv),
            "algorithmic_bytes_per_launch": 20.0 * unknowns,
            "algorithmic_read_bytes_per_launch": 12.0 * unknowns,
            "algorithmic_write_bytes_per_launch": 8.0 * unknowns})
        rec["hbm_bytes_per_launch"] = rec["hbm_fetch_bytes_per_launch"] + rec["hbm_write_bytes_per_launch"]
    else:
        per = defaultdict(lambda: {"launches": 0, "fetch_bytes_per_cycle": 0.0, "write_bytes_per_cycle": 0.0})
        for rows, key, sc in ((fetch, "fetch_bytes_per_cycle", fsc), (write, "write_bytes_per_cycle", wsc)):
            for name, _, v in rows.values():
                if any(k in name for k in SETUP_KERNELS):
                    continue
                e = per[short(name)]
                e[key] += sc * v / a.cycles
                if key == "fetch_bytes_per_cycle":
                    e["launches"] += 1
        fb = sum(e["fetch_bytes_per_cycle"] for e in per.values())
        wb = sum(e["write_bytes_per_cycle"] for e in per.values())
        rec.update({"cycles_measured": a.cycles, "hbm_bytes_per_cycle": fb + wb, "fetch_bytes_per_cycle": fb,
                    "write_bytes_per_cycle": wb,
                    "plain_sequence_compulsory_bytes_per_cycle": 194.0 * 8.0 / 7.0 * unknowns,
                    "per_kernel": dict(sorted(per.items(), key=lambda kv: -kv[1]["fetch_bytes_per_cycle"]))})
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({k: v for k, v in rec.items() if k != "per_kernel"}))


if __name__ == "__main__":
    main()
