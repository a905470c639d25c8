"""Kernel micro-benchmark: repeated finest-level red-black half-sweeps of the
3-D Poisson problem through the C ABI, and plain torch copy / triad kernels
of known size for the attainable-bandwidth reference and for calibrating
rocprofv3 FETCH_SIZE / WRITE_SIZE counters.

    python -m paper_1904_08684_amd.kbench --n 513 --reps 20 [--prec 1]

Prints one JSON line.  Sweep GB/s counts the compulsory bytes of a
half-sweep: the other colour and f of the updated colour are read, the
updated colour is written (3 x 4 B or 3 x 8 B per updated point).
"""
from __future__ import annotations

import argparse
import json
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=513)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--prec", type=int, default=0, help="0 FP64 hierarchy, 1 FP32 hierarchy")
    ap.add_argument("--copy-mib", type=int, default=2048)
    ap.add_argument("--ops", default="gs,smooth,residual,restrict,resrestrict,prolong,copy",
                    help="comma list of gs, smooth, residual, restrict, resrestrict, prolong, copy")
    ap.add_argument("--nu", type=int, default=3, help="sweeps of the smooth op (one fused pass up to 3)")
    a = ap.parse_args(argv)

    import torch

    from paper_1904_08684_amd import mg
    from paper_1904_08684_amd import workloads as W

    torch.cuda.set_device(0)
    ops = set(a.ops.split(","))
    out = {"n": a.n, "prec": a.prec, "reps": a.reps}
    n = a.n
    unknowns = (n - 2) ** 3
    es = 8 if a.prec == 0 else 4
    if ops & {"gs", "smooth", "residual", "restrict", "resrestrict", "prolong"}:
        s = mg.Solver(3, n, smoother=mg.MG_RBGS, nu1=a.nu, nu2=a.nu,
                      precision=mg.MG_MIXED if a.prec else mg.MG_FP64)
        u = W.interior_uniform(n, 3, 11)
        f = W.interior_uniform(n, 3, 12)
        s.level_set(0, mg.MG_FIELD_U, u, a.prec)
        s.level_set(0, mg.MG_FIELD_F, f, a.prec)
        s.level_set(0, mg.MG_FIELD_R, f, a.prec)
        del u, f
        print(f"# kbench n={n} prec={a.prec}", file=sys.stderr, flush=True)

        def timed(kclass, fn, level=0):
            fn()
            s.profile(True)
            for _ in range(a.reps):
                fn()
            cnt, ms = s.profile_read(kclass, level)
            s.profile(False)
            return ms / cnt

        if "gs" in ops:
            def sweep():
                s.apply(mg.MG_OP_GS_RED, 0, a.prec)
                s.apply(mg.MG_OP_GS_BLACK, 0, a.prec)
            t = timed(mg.MG_K_SMOOTH, sweep)
            out["gs_half_sweep_ms"] = t
            out["gs_half_sweep_GBps"] = 3 * es * unknowns / 2 / (t * 1e-3) / 1e9
        if "smooth" in ops:
            # nu red-black sweeps as the pre-smoothing runs them; a fused pass
            # reads one colour of u and both of f and writes both colours of u
            t = timed(mg.MG_K_SMOOTH, lambda: s.apply(mg.MG_OP_PRESMOOTH, 0, a.prec))
            out["smooth_nu"] = a.nu
            out["smooth_ms"] = t
            out["smooth_GBps"] = 2.5 * es * unknowns / (t * 1e-3) / 1e9
            out["smooth_halfsweep_equiv_GBps"] = 2 * a.nu * 1.5 * es * unknowns / (t * 1e-3) / 1e9
        if "residual" in ops:
            t = timed(mg.MG_K_RESIDUAL, lambda: s.apply(mg.MG_OP_RESIDUAL, 0, a.prec))
            out["residual_ms"] = t
            out["residual_GBps"] = 3 * es * unknowns / (t * 1e-3) / 1e9
        if "restrict" in ops:
            t = timed(mg.MG_K_RESTRICT, lambda: s.apply(mg.MG_OP_RESTRICT, 0, a.prec))
            out["restrict_ms"] = t
            out["restrict_GBps"] = es * unknowns * (1 + 1 / 8) / (t * 1e-3) / 1e9
        if "resrestrict" in ops:
            t = timed(mg.MG_K_RESTRICT, lambda: s.apply(mg.MG_OP_RESIDUAL_RESTRICT, 0, a.prec))
            out["residual_restrict_ms"] = t
            out["residual_restrict_GBps"] = es * unknowns * (2 + 1 / 8) / (t * 1e-3) / 1e9
        if "prolong" in ops:
            t = timed(mg.MG_K_PROLONG, lambda: s.apply(mg.MG_OP_PROLONG, 0, a.prec))
            out["prolong_ms"] = t
            out["prolong_GBps"] = es * unknowns * (2 + 1 / 8) / (t * 1e-3) / 1e9
        s.close()
    if "copy" in ops:
        nel = a.copy_mib * (1 << 20) // 8
        x = torch.rand(nel, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        z = torch.rand(nel, dtype=torch.float64, device="cuda")
        st = torch.cuda.current_stream()

        def ev_time(fn):
            fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(a.reps):
                fn()
            e1.record(st)
            e1.synchronize()
            return e0.elapsed_time(e1) / a.reps

        t = ev_time(lambda: y.copy_(x))
        out["copy_bytes_each_way"] = nel * 8
        out["copy_ms"] = t
        out["copy_GBps"] = 2 * nel * 8 / (t * 1e-3) / 1e9
        t = ev_time(lambda: torch.add(x, z, alpha=0.5, out=y))
        out["triad_ms"] = t
        out["triad_GBps"] = 3 * nel * 8 / (t * 1e-3) / 1e9
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
