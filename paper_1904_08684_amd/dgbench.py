"""DG volume-term benchmark: one launch of the quadrature-free element
integrals over a jittered split-quad mesh, timed with HIP events.

    python -m paper_1904_08684_amd.dgbench --nx 1024 --k 3 --reps 20

Prints one JSON line.  Bytes count the compulsory traffic (coefficients of
five fields, the map, the bathymetry in; three fields out: (5K + 5 + 3K) x
8 B per element); flops count the evaluated form, 8 K^3 + 30 K^2 + 15 K per
element (four multiply-adds per (p, i, m), the two-function terms and the
per-element set-up).
"""
from __future__ import annotations

import argparse
import json


def flops_per_element(K: int) -> int:
    return 8 * K ** 3 + 30 * K * K + 15 * K


def bytes_per_element(K: int) -> int:
    return (5 * K + 5 + 3 * K) * 8


def run(nx: int, k: int, reps: int):
    import numpy as np
    import torch

    from paper_1904_08684_amd import mg
    from paper_1904_08684_amd import workloads as W

    K = mg.DG_K[k]
    B = W.dg_mesh(nx, nx)
    ne = B.shape[1]
    c, u, hb = W.dg_fields(K, ne)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    c, u, B, hb = dev(c), dev(u), dev(B), dev(hb)
    out = torch.empty((3 * K, ne), dtype=torch.float64, device="cuda")
    op = mg.DGVolume(k)
    op(c, u, B, hb, 9.81, out)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        op(c, u, B, hb, 9.81, out)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    fl = flops_per_element(K) * ne
    by = bytes_per_element(K) * ne
    return {"elements": ne, "k": k, "ms": ms, "gflops": fl / (ms * 1e-3) / 1e9, "GBps": by / (ms * 1e-3) / 1e9,
            "frac_fp64_vector": fl / (ms * 1e-3) / 78.6e12, "frac_hbm": by / (ms * 1e-3) / 8e12}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--k", type=int, default=3)
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args(argv)
    print(json.dumps(run(a.nx, a.k, a.reps)), flush=True)


if __name__ == "__main__":
    main()
