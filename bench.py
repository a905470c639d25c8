#!/usr/bin/env python3
"""Benchmark: 3-D Poisson, 7-point stencil, 513^3 nodes (8 levels, 3^3
coarsest unknowns), red-black Gauss-Seidel V(3,3), full weighting,
trilinear interpolation, solved to relative residual 1e-10 in FP64 on one
MI355X.  One step = one complete solve from u = 0 on a resident seeded
right-hand side.  The same solve in mixed precision (single-precision
V-cycles inside FP64 iterative refinement) is timed beside it.

Prints one JSON line.  ``value`` is V-cycle MLUpS of the FP64 solve
(finest interior unknowns x V-cycles / time).  ``roofline`` covers the
dominant kernel (the finest-level fused pass of three red-black sweeps).
The timed solves replay each iteration from a captured HIP graph; events
recorded by graph nodes give no elapsed times on this runtime, so the
kernel durations come from HIP events on the library's stream over the same
solves repeated right after with profiling on (launches issued one by one).
``vcycle_roofline`` relates a whole V-cycle to the compulsory HBM bytes of
the plain (unfused) operation sequence: 222 B per finest unknown in FP64.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "V-cycle MLUpS & HBM GB/s to 1e-10 residual, FP64 vs mixed; solves/s + p99"


def _definition(text: str, signature: str) -> str:
    """The text of the definition that contains `signature`, from the line it
    starts on to its matching closing brace."""
    i = text.index(signature)
    i = text.rfind("\n", 0, i) + 1
    j = text.index("{", i)
    depth = 0
    for k in range(j, len(text)):
        depth += {"{": 1, "}": -1}.get(text[k], 0)
        if depth == 0:
            return text[i:k + 1]
    raise ValueError(signature)


def kernel_source_hash() -> str:
    """Hash of the source that determines the dominant kernel's memory
    traffic: the fused-pass kernel, its helpers, its launch shapes and its
    tiling (so the committed counter records stay valid across unrelated
    edits of the kernel file, and lapse when any of these change)."""
    csrc = os.path.join(ROOT, "paper_1904_08684_amd", "csrc")
    kern = open(os.path.join(csrc, "mg_kernels.hip")).read()
    internal = open(os.path.join(csrc, "mg_internal.h")).read()
    parts = [_definition(kern, sig) for sig in (
        "__global__ __launch_bounds__(64 * NW) void k_node_gs_tb(",
        "__device__ __forceinline__ double div6(double a)",
        "__device__ __forceinline__ T buf_load(",
        "static void gs_tb_launch(",
        "static hipError_t gs_tb_t(")]
    parts.append(_definition(internal, "static inline TbSpace make_tbspace("))
    return hashlib.sha256("\n".join(parts).encode()).hexdigest()[:16]


def traffic_record(n: int):
    """HBM bytes of the dominant kernel from committed rocprofv3 counter runs,
    valid only while the kernel source is unchanged."""
    path = os.path.join(ROOT, "profiles", f"gs_fused_{n}cubed_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec


def vcycle_traffic_record(n: int):
    """Measured HBM bytes per V-cycle (all kernels of a solve) from the
    committed rocprofv3 counter runs, valid only while the kernel source is
    unchanged."""
    path = os.path.join(ROOT, "profiles", f"vcycle_{n}cubed_fp64_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(n_sample: int = 257):
    """The oracle (plain NumPy FP64, one core) timed on bounded samples of the
    workloads: one V(3,3)-cycle of the 3-D Poisson problem at n_sample^3 (the
    reported value), and beside it the 2-D 129^2 case's ten Jacobi V(2,2)
    cycles, one single-precision refinement step of the mixed solve
    (float32-emulating cycle) at n_sample^3, and one V(3,3)-cycle of the
    variable-coefficient cell problem at 128^3 cells (about 15 s in all)."""
    import numpy as np
    from oracle import cycle
    from paper_1904_08684_amd import workloads as W
    host = f"NumPy single thread on {cpu_model()}, {os.cpu_count()} host CPUs"

    def timed(fn):
        t = time.perf_counter()
        fn()
        return time.perf_counter() - t

    f = W.interior_uniform(n_sample, 3, W.SEED_F_3D)
    h = cycle.build_hierarchy(cycle.Params(centering="node", dim=3, n=n_sample, smoother="rbgs", nu1=3, nu2=3))
    dt = timed(lambda: cycle.vcycle(h, np.zeros_like(f), f))
    dt_mx = timed(lambda: cycle.mixed_solve(h, f, tol=0.0, max_outer=1))
    n2 = 129
    f2 = W.sine_rhs_2d(n2)
    u2 = W.interior_uniform(n2, 2, W.SEED_U0_2D)
    h2 = cycle.build_hierarchy(cycle.Params(centering="node", dim=2, n=n2, smoother="jacobi", omega=0.8,
                                            nu1=2, nu2=2))
    dt2 = timed(lambda: cycle.cycles(h2, f2, u2, 10))
    nc = 128
    kc = W.varcoef_k(nc, 3)
    fc = W.normal_zero_mean(nc, 3, W.SEED_F_VARCOEF)
    hc = cycle.build_hierarchy(cycle.Params(centering="cell", dim=3, n=nc, coarsest=4, smoother="rbgs",
                                            nu1=3, nu2=3, k=kc))
    dtc = timed(lambda: cycle.vcycle(hc, np.zeros_like(fc), fc))
    m = (n_sample - 2) ** 3
    return {"value": m / dt / 1e6, "unit": "MLUpS", "cores": 1, "kind": "oracle",
            "sample": f"one V(3,3) RB-GS cycle of the 3-D Poisson problem at {n_sample}^3 nodes ({dt:.1f} s, {host})",
            "others": {
                "poisson2d_129_jacobi_10cycles": {"ms_per_cycle": round(1e2 * dt2, 2),
                                                  "mlups": round(127 ** 2 * 10 / dt2 / 1e6, 2)},
                f"mixed_refinement_step_{n_sample}": {"s": round(dt_mx, 2), "mlups": round(m / dt_mx / 1e6, 2),
                                                      "note": "FP64 residual + float32-emulating V(3,3) cycle"},
                "varcoef_cell_128_cycle": {"s": round(dtc, 2), "mlups": round(nc ** 3 / dtc / 1e6, 2)},
                "full_513_solve_estimate_s": round(8 * 511 ** 3 / (m / dt), 1)}}


def best_of(torch, run, reset=None, reps: int = 3):
    """Warm-up call, then the fastest of `reps` timed calls (device work
    included: synchronised on both sides); returns (seconds, last result)."""
    if reset:
        reset()
    run()
    torch.cuda.synchronize()
    best, out = float("inf"), None
    for _ in range(reps):
        if reset:
            reset()
        t = time.perf_counter()
        out = run()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best, out


CONFIG_GROUPS = ("poisson2d", "varcoef", "cycles", "fmg", "dg")


def other_configs(mg, W, torch, np, groups=CONFIG_GROUPS):
    """The 2-D 129^2 Jacobi case (10 V(2,2) cycles, latency bound), the
    256^3-cell variable-coefficient case (FP64 and mixed to 1e-10, FP64 with
    zero-flux walls, and CG preconditioned by the cycle), W- and F-cycle
    solves of the 513^3 Poisson problem, damped-Jacobi cycles with
    rediscretised and Galerkin coarse operators, CG with the V-cycle as
    preconditioner, full multigrid on a 513^3 problem with a closed-form
    discrete solution, and the DG scheme's volume terms, velocity
    projection, edge terms, whole right-hand side and SSP-RK3 step."""
    res = {}

    def solve_entry(s, rhs, tol=1e-10):
        s.set_rhs(rhs)
        dt, (code, cyc, rel) = best_of(torch, lambda: s.solve(tol), lambda: s.set_initial(None))
        return dt, code, cyc, rel

    def pcg_entry(s, rhs, tol=1e-10):
        s.set_rhs(rhs)
        dt, (code, its, rel) = best_of(torch, lambda: s.pcg(tol, 40), lambda: s.set_initial(None))
        return dt, code, its, rel

    if "poisson2d" in groups:
        # 2-D 129^2, ten damped-Jacobi V(2,2) cycles from the seeded start
        n = 129
        s = mg.Solver(2, n, smoother=mg.MG_JACOBI, omega=0.8, nu1=2, nu2=2)
        s.set_rhs(W.sine_rhs_2d(n))
        u0 = W.interior_uniform(n, 2, W.SEED_U0_2D)
        dt, _ = best_of(torch, lambda: s.vcycle(10), lambda: s.set_initial(u0), reps=20)
        res["poisson2d_129_jacobi_10cycles"] = {"ms_per_10_cycles": round(1e3 * dt, 3),
                                                "us_per_cycle": round(1e5 * dt, 2),
                                                "mlups": round(127 ** 2 * 10 / dt / 1e6, 1)}
        s.close()

    if "varcoef" in groups:
        # 256^3 cells, variable coefficient
        N = 256
        k = torch.from_numpy(W.varcoef_k(N, 3)).cuda()
        f = torch.from_numpy(W.normal_zero_mean(N, 3, W.SEED_F_VARCOEF)).cuda()
        sols = {}
        for prec, name in ((mg.MG_FP64, "fp64"), (mg.MG_MIXED, "mixed")):
            s = mg.Solver(3, N, centering=mg.MG_CELL, smoother=mg.MG_RBGS, nu1=3, nu2=3, k=k, precision=prec)
            dt, code, cyc, rel = solve_entry(s, f)
            res[f"varcoef_cell_256_{name}"] = {"ms_to_1e-10": round(1e3 * dt, 3), "cycles": cyc, "relres": rel,
                                               "status": code, "mlups": round(N ** 3 * cyc / dt / 1e6, 1)}
            sols[name] = torch.empty((N, N, N), dtype=torch.float64, device="cuda")
            s.solution(sols[name])
            s.close()
        res["varcoef_cell_256_mixed"]["max_rel_diff_vs_fp64_solution"] = float(
            (sols["mixed"] - sols["fp64"]).abs().max() / sols["fp64"].abs().max())
        # the same problem with zero-flux walls (projected right-hand side, zero-mean solution)
        s = mg.Solver(3, N, centering=mg.MG_CELL, smoother=mg.MG_RBGS, nu1=3, nu2=3, k=k, bc=mg.MG_NEUMANN0)
        dt, code, cyc, rel = solve_entry(s, f)
        res["varcoef_cell_256_neumann_fp64"] = {"ms_to_1e-10": round(1e3 * dt, 3), "cycles": cyc, "relres": rel,
                                                "status": code, "mlups": round(N ** 3 * cyc / dt / 1e6, 1)}
        s.close()
        # the same problem by CG preconditioned with the symmetric V(3,3)-cycle
        s = mg.Solver(3, N, centering=mg.MG_CELL, smoother=mg.MG_RBGS, nu1=3, nu2=3, post_order=1, k=k, krylov=1)
        dt, code, its, rel = pcg_entry(s, f)
        u = torch.empty((N, N, N), dtype=torch.float64, device="cuda")
        s.solution(u)
        res["varcoef_cell_256_pcg_fp64"] = {"ms_to_1e-10": round(1e3 * dt, 3), "iterations": its,
                                            "relres": rel, "status": code,
                                            "max_rel_diff_vs_fp64_solution": float(
                                                (u - sols["fp64"]).abs().max() / sols["fp64"].abs().max())}
        s.close()
        sols = u = k = f = None

    if "cycles" in groups:
        # 513^3 Poisson: W- and F-cycles, damped-Jacobi cycles with both coarse
        # operators, and CG preconditioned by the symmetric V(3,3)-cycle
        n = 513
        f3 = torch.from_numpy(W.interior_uniform(n, 3, W.SEED_F_3D)).cuda()
        for code_c, name in ((mg.MG_CYCLE_W, "W"), (mg.MG_CYCLE_F, "F")):
            s = mg.Solver(3, n, smoother=mg.MG_RBGS, nu1=3, nu2=3, cycle=code_c)
            dt, code, cyc, rel = solve_entry(s, f3)
            res[f"poisson3d_513_{name}cycle_fp64"] = {"ms_to_1e-10": round(1e3 * dt, 3), "cycles": cyc, "relres": rel,
                                                     "status": code, "ms_per_cycle": round(1e3 * dt / cyc, 3)}
            s.close()
        for cop, name in ((mg.MG_COARSE_REDISCRETISE, "rediscretised"), (mg.MG_COARSE_GALERKIN, "galerkin")):
            s = mg.Solver(3, n, smoother=mg.MG_JACOBI, omega=0.8, nu1=2, nu2=2, coarse_op=cop)
            dt, code, cyc, rel = solve_entry(s, f3)
            res[f"poisson3d_513_jacobi_{name}_fp64"] = {"ms_to_1e-10": round(1e3 * dt, 3), "cycles": cyc,
                                                         "relres": rel, "status": code,
                                                         "ms_per_cycle": round(1e3 * dt / cyc, 3)}
            s.close()
        s = mg.Solver(3, n, smoother=mg.MG_RBGS, nu1=3, nu2=3, post_order=1, krylov=1)
        dt, code, its, rel = pcg_entry(s, f3)
        res["poisson3d_513_pcg_vcycle_fp64"] = {"ms_to_1e-10": round(1e3 * dt, 3), "iterations": its, "relres": rel,
                                                "status": code, "ms_per_iteration": round(1e3 * dt / its, 3)}
        s.close()
        f3 = None

    if "fmg" in groups:
        # full multigrid on the sine problem, whose discrete solution is known in
        # closed form: one pass with two V(3,3)-cycles per level
        n = 513
        ue = torch.from_numpy(W.sine_mode(n, 3)).cuda()
        fs = 3 * np.pi ** 2 * ue
        s = mg.Solver(3, n, smoother=mg.MG_RBGS, nu1=3, nu2=3)
        s.set_rhs(fs)
        dt, _ = best_of(torch, lambda: s.fmg(2))
        u = torch.empty_like(fs)
        s.solution(u)
        hh = 1.0 / (n - 1)
        ch = (np.pi * hh / 2) ** 2 / np.sin(np.pi * hh / 2) ** 2
        res["fmg_513_sine_fp64"] = {"ms": round(1e3 * dt, 3), "cycles_per_level": 2,
                                    "algebraic_over_discretisation_error": float((u - ch * ue).abs().max()) / abs(ch - 1.0),
                                    "relres": s.residual_norm() / float(torch.linalg.vector_norm(fs[1:-1, 1:-1, 1:-1]))}
        s.close()
        u = ue = fs = None

    # the quadrature-free DG shallow-water scheme on 2 x 1024^2 perturbed
    # split-quad triangles, orders 1-3: each term, the right-hand side and an
    # SSP-RK3 step (HIP events)
    if "dg" in groups:
        from paper_1904_08684_amd import dgbench
        for op, name in (("volume", "dg_volume_terms"), ("projection", "dg_velocity_projection"),
                         ("edges", "dg_edge_terms"), ("rhs", "dg_rhs"), ("step", "dg_ssp_rk3_step")):
            for kk in (1, 2, 3):
                r = dgbench.run(1024, kk, 20, op)
                res[f"{name}_k{kk}_2M_elements"] = {
                    "ms": round(r["ms"], 4), "elements": r["elements"], "gflops": round(r["gflops"], 1),
                    "GBps": round(r["GBps"], 1), "frac_fp64_vector_peak": round(r["frac_fp64_vector"], 3),
                    "frac_hbm_peak": round(r["frac_hbm"], 3)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=513)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--configs", default=",".join(CONFIG_GROUPS),
                    help="comma list of the other configurations to run: " + ", ".join(CONFIG_GROUPS))
    ap.add_argument("--serve-count", type=int, default=4096)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1904_08684_amd import mg
    from paper_1904_08684_amd import workloads as W

    torch.cuda.set_device(0)
    n = args.n
    unknowns = (n - 2) ** 3
    print(f"# bench: {n}^3 FP64 setup", file=sys.stderr, flush=True)
    f = W.interior_uniform(n, 3, W.SEED_F_3D)
    f_dev = torch.from_numpy(f).cuda()
    del f

    def run(precision):
        s = mg.Solver(3, n, smoother=mg.MG_RBGS, nu1=3, nu2=3, precision=precision)
        s.set_rhs(f_dev)
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            s.set_initial(None)
            code, cyc, rel = s.solve(args.tol)
            assert code == mg.MG_OK, (code, rel)
        times, cycles, rels = [], [], []
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for _ in range(args.steps):
            t0 = time.perf_counter()
            s.set_initial(None)
            code, cyc, rel = s.solve(args.tol)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            assert code == mg.MG_OK, (code, rel)
            cycles.append(cyc)
            rels.append(rel)
        total = time.perf_counter() - t_all
        graphs = s.graph_launches()
        u_out = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        s.solution(u_out)
        # the same solves with per-kernel HIP events
        s.profile(True)
        t_prof = time.perf_counter()
        for _ in range(args.steps):
            s.set_initial(None)
            code, cyc, rel = s.solve(args.tol)
            assert code == mg.MG_OK, (code, rel)
        torch.cuda.synchronize()
        t_prof = time.perf_counter() - t_prof
        prof = {}
        for name, kc in (("smooth", mg.MG_K_SMOOTH), ("residual", mg.MG_K_RESIDUAL),
                         ("restrict", mg.MG_K_RESTRICT), ("prolong", mg.MG_K_PROLONG),
                         ("coarse", mg.MG_K_COARSE), ("reduce", mg.MG_K_REDUCE), ("cast", mg.MG_K_CAST),
                         ("update", mg.MG_K_UPDATE), ("copy", mg.MG_K_COPY)):
            cnt, ms = s.profile_read(kc, -1)
            if cnt:
                prof[name] = {"launches": cnt, "ms": round(ms, 3)}
        c0, ms0 = s.profile_read(mg.MG_K_SMOOTH, 0)
        s.profile(False)
        s.close()
        return {"total": total, "times": times, "cycles": cycles, "rels": rels, "prof": prof, "u": u_out,
                "fine_smooth": (c0, ms0), "graph_replays": graphs, "profiled_ms_per_solve": 1e3 * t_prof / args.steps}

    r64 = run(mg.MG_FP64)
    ms_step = 1e3 * r64["total"] / args.steps
    cyc_total = sum(r64["cycles"])
    mlups = unknowns * cyc_total / r64["total"] / 1e6
    c0, ms0 = r64["fine_smooth"]
    avg_ms = ms0 / c0
    # Algorithmic bytes of one fused pass of three red-black sweeps on the
    # finest level, two models: the per-sweep unit of the method (read u and
    # f, write u: 24 B per unknown per sweep, x 3 sweeps), and the pass's own
    # compulsory traffic (one colour of the iterate and both colours of f
    # read, both colours of the new iterate written: (4 + 8 + 8) B per
    # unknown in FP64).  `achieved` and `frac` use the per-sweep unit.
    bytes_per_launch = 3 * 24.0 * unknowns
    pass_bytes = 20.0 * unknowns
    secs = avg_ms * 1e-3
    achieved = bytes_per_launch / secs / 1e9
    traf = traffic_record(n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (traf["hbm_bytes_per_launch"] if traf else None),
                "kernel": "finest-level fused pass of three red-black GS sweeps (k_node_gs_tb<double, 6, 3, 12, 6, true, true>)",
                "avg_launch_ms": round(avg_ms, 4), "launches": c0,
                "timing": "HIP events, profiled repetition of the timed solves",
                "algorithmic_bytes_per_launch": bytes_per_launch,
                "byte_models": {
                    "per_sweep_24B_x3": {"bytes_per_launch": bytes_per_launch, "GBps": round(achieved, 1),
                                         "frac": round(achieved / HBM_PEAK_GBS, 4)},
                    "fused_pass_compulsory_20B": {"bytes_per_launch": pass_bytes,
                                                  "GBps": round(pass_bytes / secs / 1e9, 1),
                                                  "frac": round(pass_bytes / secs / 1e9 / HBM_PEAK_GBS, 4)},
                    "measured_counters": ({"bytes_per_launch": traf["hbm_bytes_per_launch"],
                                           "GBps": round(traf["hbm_bytes_per_launch"] / secs / 1e9, 1),
                                           "frac": round(traf["hbm_bytes_per_launch"] / secs / 1e9 / HBM_PEAK_GBS, 4)}
                                          if traf else None)}}
    # whole V-cycle against the plain operation sequence: per level 2 (nu1 + nu2)
    # half-sweeps x 12 B, residual 24 B, restriction 9 B, interpolation and
    # correction 17 B per unknown (194 B), summed over levels (x 8/7)
    vc_bytes = 194.0 * 8.0 / 7.0 * unknowns
    vc_ms = 1e3 * r64["total"] / cyc_total
    vtr = vcycle_traffic_record(n)
    vcycle_roofline = {"bound": "hbm", "unfused_compulsory_bytes_per_cycle": round(vc_bytes),
                       "ms_per_cycle": round(vc_ms, 4),
                       "traffic_per_cycle": (round(vtr["hbm_bytes_per_cycle"]) if vtr else None),
                       "achieved": round(vc_bytes / (vc_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(vc_bytes / (vc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    out = {"metric": METRIC, "value": round(mlups, 1), "unit": "MLUpS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded U[-1,1] right-hand side, u0 = 0)",
           "config": {"workload": f"3-D Poisson 7-point, {n}^3 nodes, 8 levels, RB-GS V(3,3), full weighting, "
                                  f"trilinear, 3^3 coarsest Cholesky, to relres {args.tol:g}",
                      "n": n, "unknowns": unknowns, "tol": args.tol,
                      "cycles_per_solve": r64["cycles"][0], "final_relres": r64["rels"][-1],
                      "graph_replays": r64["graph_replays"],
                      "median_ms_per_solve": round(1e3 * float(np.median(r64["times"])), 3),
                      "profiled_ms_per_solve": round(r64["profiled_ms_per_solve"], 3)},
           "roofline": roofline,
           "vcycle_roofline": vcycle_roofline,
           "kernel_ms_total": r64["prof"]}
    if not args.no_mixed:
        print("# bench: mixed precision", file=sys.stderr, flush=True)
        rmx = run(mg.MG_MIXED)
        ms_mx = 1e3 * rmx["total"] / args.steps
        # the FP64 GPU path matches the oracle per iterate (tests); the mixed
        # result's error is stated against the converged FP64 solution
        err = float((rmx["u"] - r64["u"]).abs().max() / r64["u"].abs().max())
        out["mixed"] = {"ms_per_solve": round(ms_mx, 3), "refinement_steps": rmx["cycles"][0],
                        "median_ms_per_solve": round(1e3 * float(np.median(rmx["times"])), 3),
                        "final_relres": rmx["rels"][-1], "max_rel_diff_vs_fp64_solution": err,
                        "mlups": round(unknowns * sum(rmx["cycles"]) / rmx["total"] / 1e6, 1),
                        "speedup_vs_fp64_time_to_tol": round(ms_step / ms_mx, 3),
                        "kernel_ms_total": rmx["prof"]}
    out["solves_per_s_fp64"] = round(args.steps / r64["total"], 3)
    r64 = rmx = None
    torch.cuda.empty_cache()
    if not args.no_configs:
        out["other_configs"] = other_configs(mg, W, torch, np, tuple(args.configs.split(",")))
    if not args.no_serve:
        print("# bench: served stream", file=sys.stderr, flush=True)
        from paper_1904_08684_amd import serve_bench
        f_dev = None
        torch.cuda.empty_cache()
        sv = serve_bench.main(["--count", str(args.serve_count), "--sweep", "0.25,0.5,1.0,1.2"], emit=False)
        out["serve"] = {"workload": sv["workload"], "solves_per_s": round(sv["open_loop"]["solves_per_s"], 1),
                        "p50_ms": round(sv["open_loop"]["p50_ms"], 3), "p99_ms": round(sv["open_loop"]["p99_ms"], 3),
                        "rate_per_s": round(sv["rate_per_s"], 1),
                        "saturation_solves_per_s": round(sv["saturation"]["solves_per_s"], 1),
                        "fifo_fp64_one_at_a_time": {k: round(v, 3) for k, v in sv["fifo_fp64_one_at_a_time"].items()},
                        "speedup_solves_per_s": round(sv["speedup_solves_per_s"], 2), "server": sv["server"],
                        "batched_bytes": {"saturation_mb_per_round": round(sv["saturation"]["algorithmic_mb_per_round"], 2),
                                          "saturation_GBps_over_makespan":
                                              round(sv["saturation"]["algorithmic_GBps_over_makespan"], 1),
                                          "open_loop_GBps_over_makespan":
                                              round(sv["open_loop"]["algorithmic_GBps_over_makespan"], 1),
                                          "peak_GBps": HBM_PEAK_GBS},
                        "load_sweep": [{k: round(v, 3) for k, v in row.items()} for row in sv["load_sweep"]]}
    if not args.no_cpu_baseline:
        print("# bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
