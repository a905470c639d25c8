"""Served-stream benchmark: Poisson solve requests of mixed sizes through the
continuously batched server, against the plain FP64 path serving the same
trace one request at a time.

Workload: `count` requests, sizes uniform over 2-D {65^2, 129^2, 257^2,
513^2, 1025^2} and 3-D {33^3, 65^3, 129^3} nodes, right-hand sides
U[-1, 1] on interior nodes drawn on the GPU from a per-request seeded
generator (seed 1000 + id), each solved to relative residual 1e-8 in mixed
precision (2-D: damped Jacobi V(2,2), 3-D: red-black GS V(3,3)).  The
saturation rate is measured with every request present at t = 0; the open
loop then runs exponential arrivals at `load` x saturation.

    python -m paper_1904_08684_amd.serve_bench --count 4096
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def percentile(vals, q):
    """Nearest-rank percentile."""
    s = sorted(vals)
    if not s:
        return float("nan")
    k = max(1, int(-(-q * len(s) // 100)))
    return s[min(k, len(s)) - 1]


def make_inputs(reqs, torch):
    fs, us = [], []
    g = torch.Generator(device="cuda")
    for r in reqs:
        g.manual_seed(1000 + r.rid)
        shape = (r.n,) * r.dim
        fs.append(torch.rand(shape, generator=g, dtype=torch.float64, device="cuda") * 2.0 - 1.0)
        us.append(torch.empty(shape, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    return fs, us


def method(mg, dim):
    return (mg.MG_JACOBI, 2, 2) if dim == 2 else (mg.MG_RBGS, 3, 3)


def run_server(mg, srv, reqs, fs, us, tol, arrivals):
    """Drive the server over a trace; arrivals[i] = offset in seconds (0 = at start)."""
    n = len(reqs)
    order = sorted(range(n), key=lambda i: arrivals[i])
    st0 = srv.stats()
    t0 = srv.clock()
    nxt = 0
    done = {}
    while len(done) < n:
        now = srv.clock() - t0
        while nxt < n and arrivals[order[nxt]] <= now:
            i = order[nxt]
            r = reqs[i]
            sm, nu1, nu2 = method(mg, r.dim)
            code = srv.submit(i, r.dim, r.n, fs[i], us[i], tol, sm, nu1, nu2, t_arrive=t0 + arrivals[i])
            if code != mg.MG_OK:
                raise RuntimeError(f"submit {i}: {code}")
            nxt += 1
        in_flight, queued = srv.step()
        for res in srv.poll():
            done[res["id"]] = res
        if in_flight == 0 and queued == 0 and nxt < n:
            wait = t0 + arrivals[order[nxt]] - srv.clock()
            if wait > 0:
                time.sleep(min(wait, 0.01))
    lat = [1e3 * (r["t_done"] - r["t_arrive"]) for r in done.values()]
    t_first = min(r["t_arrive"] for r in done.values())
    t_last = max(r["t_done"] for r in done.values())
    bad = [r for r in done.values() if r["status"] != mg.MG_OK]
    st1 = srv.stats()
    nbytes = st1["algorithmic_bytes"] - st0["algorithmic_bytes"]
    rounds = max(1, st1["rounds"] - st0["rounds"])
    # the batched launches' compulsory bytes (each op's reads and writes once),
    # per round and as a rate over the pass (a lower bound on k_batch's rate:
    # the pass also holds the host's round trips and idle gaps)
    return {"requests": n, "solves_per_s": n / (t_last - t_first), "p50_ms": percentile(lat, 50),
            "p99_ms": percentile(lat, 99), "mean_steps": sum(r["steps"] for r in done.values()) / n,
            "max_relres": max(r["relres"] for r in done.values()), "failed": len(bad),
            "makespan_s": t_last - t_first, "rounds": rounds, "algorithmic_gb": nbytes / 1e9,
            "algorithmic_mb_per_round": nbytes / rounds / 1e6,
            "algorithmic_GBps_over_makespan": nbytes / 1e9 / (t_last - t_first)}


def run_fifo_fp64(mg, reqs, fs, us, tol, arrivals, limit, torch):
    """The plain FP64 path, one request at a time in arrival order (the same
    arrival trace as the open-loop server run), one resident context per
    size class."""
    idx = sorted(range(len(reqs)), key=lambda i: arrivals[i])[:limit]
    solvers = {}
    for i in idx:
        r = reqs[i]
        key = (r.dim, r.n)
        if key not in solvers:
            sm, nu1, nu2 = method(mg, r.dim)
            solvers[key] = mg.Solver(r.dim, r.n, smoother=sm, nu1=nu1, nu2=nu2, precision=mg.MG_FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, t_last = [], t0
    for i in idx:
        r = reqs[i]
        arr = t0 + arrivals[i]
        while time.perf_counter() < arr:
            pass
        s = solvers[(r.dim, r.n)]
        s.set_rhs(fs[i])
        s.set_initial(None)
        code, cyc, rel = s.solve(tol)
        s.solution(us[i])
        torch.cuda.synchronize()
        t_last = time.perf_counter()
        lat.append(1e3 * (t_last - arr))
    for s in solvers.values():
        s.close()
    n = len(idx)
    first = t0 + min(arrivals[i] for i in idx)
    return {"requests": n, "solves_per_s": n / (t_last - first), "p50_ms": percentile(lat, 50),
            "p99_ms": percentile(lat, 99)}


def main(argv=None, emit=True):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--slots", type=int, default=512)
    ap.add_argument("--arena-gb", type=float, default=48.0)
    ap.add_argument("--fifo-count", type=int, default=0,
                    help="requests of the trace the FIFO baseline serves (0: all, the same trace)")
    ap.add_argument("--sweep", default="", help="comma list of further loads (x saturation) to run open loop")
    a = ap.parse_args(argv)

    import torch

    from paper_1904_08684_amd import mg
    from paper_1904_08684_amd import workloads as W

    torch.cuda.set_device(0)
    reqs = W.request_stream(a.count, 1.0)        # sizes; arrival times are rescaled below
    unit = [r.t_arrive for r in reqs]            # arrivals at rate 1 / s
    print(f"# serve: generating {a.count} right-hand sides", file=sys.stderr, flush=True)
    fs, us = make_inputs(reqs, torch)
    srv = mg.Server(int(a.arena_gb * (1 << 30)), max_slots=a.slots)
    # a first full pass builds the resident hierarchies (as a long-running
    # server would already hold them); the measured passes reuse them
    print("# serve: warm-up pass", file=sys.stderr, flush=True)
    warm = run_server(mg, srv, reqs, fs, us, a.tol, [0.0] * a.count)
    print("# serve: saturation (all requests at t = 0)", file=sys.stderr, flush=True)
    sat = run_server(mg, srv, reqs, fs, us, a.tol, [0.0] * a.count)
    rate = a.load * sat["solves_per_s"]
    arrivals = [t / rate for t in unit]
    print(f"# serve: open loop at {rate:.0f} req/s", file=sys.stderr, flush=True)
    opn = run_server(mg, srv, reqs, fs, us, a.tol, arrivals)
    sweep = []
    for ld in [float(x) for x in a.sweep.split(",") if x]:
        r = ld * sat["solves_per_s"]
        print(f"# serve: open loop at {ld:g} x saturation ({r:.0f} req/s)", file=sys.stderr, flush=True)
        res = run_server(mg, srv, reqs, fs, us, a.tol, [t / r for t in unit])
        sweep.append({"load": ld, "rate_per_s": r, "solves_per_s": res["solves_per_s"], "p50_ms": res["p50_ms"],
                      "p99_ms": res["p99_ms"], "failed": res["failed"]})
    st = srv.stats()
    srv.close()
    print("# serve: FIFO FP64 baseline", file=sys.stderr, flush=True)
    fifo = run_fifo_fp64(mg, reqs, fs, us, a.tol, arrivals, a.fifo_count or a.count, torch)
    out = {"workload": f"{a.count} Poisson solve requests, 2-D 65^2..1025^2 and 3-D 33^3..129^3 nodes, "
                       f"mixed precision to relres {a.tol:g}",
           "cold_start": warm, "saturation": sat, "rate_per_s": rate, "load": a.load, "open_loop": opn,
           "fifo_fp64_one_at_a_time": fifo,
           "speedup_solves_per_s": opn["solves_per_s"] / fifo["solves_per_s"],
           "load_sweep": sweep,
           "server": {"max_slots": a.slots, "arena_gb": a.arena_gb, "rounds": st["rounds"],
                      "launches": st["launches"], "hierarchies_built": st["hierarchies_built"],
                      "arena_peak_gb": st["arena_peak_bytes"] / (1 << 30)}}
    if emit:
        print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
