"""The continuously batched solve server: each result is bitwise the same
alone and in a mix (with arrivals while others are in flight), meets its
tolerance by the oracle's own residual, matches the oracle's mixed-precision
solve, and admission respects the HBM budget."""
import numpy as np
import pytest

from oracle import cycle
from paper_1904_08684_amd import workloads as W

pytestmark = pytest.mark.gpu

# (dim, n): 2-D requests use damped Jacobi V(2,2), 3-D requests red-black GS V(3,3)
MIX = [(2, 65), (3, 33), (2, 129), (3, 65), (2, 257), (3, 17), (2, 33), (3, 33)]
# the largest served classes: 3-D 129^3 runs the column-marching batched
# smoother and residuals, 2-D 1025^2 the row-marching ones on every level
# from 1025^2 down to 129^2
LARGE = [(3, 129), (2, 1025), (3, 65), (2, 513), (3, 129), (2, 257)]


def method(dim):
    from paper_1904_08684_amd import mg
    return (mg.MG_JACOBI, 2, 2) if dim == 2 else (mg.MG_RBGS, 3, 3)


def make_inputs(torch, reqs):
    fs, us = [], []
    for rid, (d, n) in enumerate(reqs):
        fs.append(torch.from_numpy(W.interior_uniform(n, d, W.SEED_REQUEST_BASE + rid)).cuda())
        us.append(torch.zeros((n,) * d, dtype=torch.float64, device="cuda"))
    return fs, us


def run(mg, torch, reqs, order, arena=1 << 30, slots=64, stagger=False, tol=1e-8):
    srv = mg.Server(arena, max_slots=slots)
    fs, us = make_inputs(torch, reqs)
    pending = list(order)
    results = {}
    # with stagger, requests arrive two at a time while earlier ones are in flight
    while pending or len(results) < len(order):
        batch = pending[:2] if stagger else pending
        for rid in batch:
            d, n = reqs[rid]
            sm, nu1, nu2 = method(d)
            assert srv.submit(rid, d, n, fs[rid], us[rid], tol, sm, nu1, nu2) == mg.MG_OK
        pending = pending[len(batch):]
        srv.step()
        for r in srv.poll():
            results[r["id"]] = r
    torch.cuda.synchronize()
    st = srv.stats()
    sols = {rid: us[rid].cpu().numpy() for rid in order}
    srv.close()
    return results, sols, st


def oracle_check(mg, res, sols, reqs, rids):
    for rid in rids:
        d, n = reqs[rid]
        f = W.interior_uniform(n, d, W.SEED_REQUEST_BASE + rid)
        sm = "jacobi" if d == 2 else "rbgs"
        nu = 2 if d == 2 else 3
        h = cycle.build_hierarchy(cycle.Params(centering="node", dim=d, n=n, smoother=sm, nu1=nu, nu2=nu))
        u = sols[rid]
        rel = cycle.residual_norm(h, u, f) / cycle.residual_norm(h, np.zeros_like(f), f)
        u_ref, hist = cycle.mixed_solve(h, f, tol=1e-8)
        diff = np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref))
        print(f"request {rid} {d}d n={n}: steps {res[rid]['steps']} (oracle {len(hist) - 1}) "
              f"relres {res[rid]['relres']:.3e} cpu {rel:.3e} vs oracle {diff:.2e}", flush=True)
        assert res[rid]["status"] == mg.MG_OK and rel <= 1e-8
        assert abs(rel - res[rid]["relres"]) <= 1e-6 * rel
        assert res[rid]["steps"] == len(hist) - 1
        assert diff <= 1e-9


def test_alone_equals_in_mix_bitwise(mg):
    import torch
    reqs = MIX
    alone_res, alone_sol = {}, {}
    for rid in range(len(reqs)):
        r, s, _ = run(mg, torch, reqs, [rid])
        alone_res.update(r)
        alone_sol.update(s)
    mix_res, mix_sol, st = run(mg, torch, reqs, list(range(len(reqs)))[::-1], stagger=True)
    for rid in range(len(reqs)):
        assert alone_res[rid]["status"] == mg.MG_OK
        assert mix_res[rid]["steps"] == alone_res[rid]["steps"]
        assert np.array_equal(mix_sol[rid], alone_sol[rid]), rid
        assert mix_res[rid]["relres"] == alone_res[rid]["relres"]
    print("mix stats", st, flush=True)
    assert st["completed"] == len(reqs) and st["rounds"] > 0


def test_results_meet_tolerance_and_match_oracle(mg):
    import torch
    reqs = MIX[:6]
    res, sols, _ = run(mg, torch, reqs, list(range(len(reqs))))
    oracle_check(mg, res, sols, reqs, range(len(reqs)))


def test_small_budget_admits_within_footprint(mg):
    """An arena that holds about two hierarchies: requests queue, the arena is
    never overcommitted, hierarchies are evicted and rebuilt, all finish."""
    import torch
    reqs = [(3, 65), (2, 257), (3, 65), (3, 33), (2, 257), (3, 65)]
    fp = max(mg.server_footprint(d, n, *method(d)) for d, n in reqs)
    arena = 2 * fp + (1 << 20)
    res, sols, st = run(mg, torch, reqs, list(range(len(reqs))), arena=arena, slots=8)
    assert all(r["status"] == mg.MG_OK for r in res.values())
    assert st["arena_peak_bytes"] <= arena
    assert st["evictions"] >= 1
    # same answers as with a roomy arena
    res2, sols2, _ = run(mg, torch, reqs, list(range(len(reqs))))
    for rid in range(len(reqs)):
        assert np.array_equal(sols[rid], sols2[rid])


def test_queue_limit_and_invalid_requests(mg):
    import torch
    srv = mg.Server(256 << 20, max_slots=2, max_queue=3)
    f = torch.zeros((17,) * 3, dtype=torch.float64, device="cuda")
    u = torch.zeros_like(f)
    codes = [srv.submit(i, 3, 17, f, u, 1e-8, mg.MG_RBGS, 3, 3) for i in range(4)]
    assert codes[:3] == [mg.MG_OK] * 3 and codes[3] == mg.MG_EBUSY
    assert srv.submit(9, 3, 18, f, u, 1e-8) == mg.MG_EINVAL
    # served requests are V-cycles
    r = mg.mg_request()
    r.id, r.grid, r.tol = 11, mg.make_grid(3, 17), 1e-8
    r.opts = mg.make_opts(mg.MG_RBGS, 0.8, 3, 3, mg.MG_MIXED, 50, 0, mg.MG_CYCLE_W)
    r.f, r.u_out = f.data_ptr(), u.data_ptr()
    assert mg.mg_server_submit(srv.h, mg.C.byref(r), None) == mg.MG_EINVAL
    big = mg.server_footprint(3, 257, mg.MG_RBGS, 3, 3)
    assert big > (256 << 20)
    fb = torch.zeros((2, 2), dtype=torch.float64, device="cuda")
    assert srv.submit(10, 3, 257, fb, fb, 1e-8, mg.MG_RBGS, 3, 3) == mg.MG_ENOMEM
    done = []
    while len(done) < 3:
        srv.step()
        done += srv.poll()
    assert all(r["status"] == mg.MG_OK for r in done)
    # zero right-hand side: converged at once with a zero solution
    u.fill_(1.0)
    assert srv.submit(20, 3, 17, f, u, 1e-8, mg.MG_RBGS, 3, 3) == mg.MG_OK
    out = []
    while not out:
        srv.step()
        out = srv.poll()
    torch.cuda.synchronize()
    assert out[0]["status"] == mg.MG_OK and float(u.abs().max()) == 0.0
    srv.close()


def test_tickets_and_latency_accounting_on_the_supplied_clock(mg):
    """Tickets are issued 0, 1, 2, ... in submission order and come back in
    the results; a result keeps the arrival time the caller supplied (here
    0.25 s before submission, and one at submission), is admitted no
    earlier than it was submitted and finishes after admission, so
    t_done - t_arrive counts the time before submission too."""
    import torch
    srv = mg.Server(512 << 20, max_slots=4)
    reqs = [(3, 33), (2, 65), (3, 17), (2, 129), (3, 33)]
    fs, us = make_inputs(torch, reqs)
    tickets, submitted, arrive = {}, {}, {}
    for rid, (d, n) in enumerate(reqs):
        sm, nu1, nu2 = method(d)
        now = srv.clock()
        arrive[rid] = now - 0.25 if rid % 2 == 0 else now
        submitted[rid] = now
        assert srv.submit(rid, d, n, fs[rid], us[rid], 1e-8, sm, nu1, nu2, t_arrive=arrive[rid]) == mg.MG_OK
        tickets[rid] = srv.last_ticket
    assert [tickets[i] for i in range(len(reqs))] == list(range(len(reqs)))
    done = {}
    while len(done) < len(reqs):
        srv.step()
        for r in srv.poll():
            done[r["id"]] = r
    srv.close()
    for rid, r in done.items():
        assert r["status"] == mg.MG_OK and r["ticket"] == tickets[rid]
        assert r["t_arrive"] == arrive[rid]
        assert submitted[rid] <= r["t_admit"] <= r["t_done"]
        lat = r["t_done"] - r["t_arrive"]
        assert lat >= (0.25 if rid % 2 == 0 else 0.0)
        print(f"request {rid} ticket {r['ticket']}: latency {1e3 * lat:.2f} ms, queued "
              f"{1e3 * (r['t_admit'] - r['t_arrive']):.2f} ms", flush=True)


def test_cancellation_and_deadlines(mg):
    """A queued request cancelled at once and one in flight cancelled before
    the next round come back MG_ECANCELED with u_out untouched; a request
    queued past its deadline is retired unadmitted, and one that cannot
    reach its tolerance is retired MG_ETIMEDOUT at the first round ending
    after its deadline, with its iterate so far; the rest converge; unknown
    and finished tickets are refused."""
    import torch
    srv = mg.Server(512 << 20, max_slots=2)
    reqs = [(3, 33)] * 5
    fs, us = make_inputs(torch, reqs)
    sm, nu1, nu2 = method(3)
    now = srv.clock()
    dl = {2: now + 0.2, 3: 1e-9}          # request 3: a deadline already past
    tickets = []
    for rid in range(5):
        tol, steps = (1e-30, 100000) if rid == 2 else (1e-8, 50)
        assert srv.submit(rid, 3, 33, fs[rid], us[rid], tol, sm, nu1, nu2, max_steps=steps,
                          deadline=dl.get(rid, 0.0)) == mg.MG_OK
        tickets.append(srv.last_ticket)
    assert srv.cancel(tickets[4]) == mg.MG_OK              # still queued
    done = {r["id"]: r for r in srv.poll()}
    assert done[4]["status"] == mg.MG_ECANCELED and done[4]["steps"] == 0
    srv.step()                                               # requests 0 and 1 run one round
    assert srv.cancel(tickets[1]) == mg.MG_OK              # in flight
    assert srv.cancel(99) != mg.MG_OK
    while len(done) < 5:
        srv.step()
        for r in srv.poll():
            done[r["id"]] = r
    assert srv.cancel(tickets[0]) != mg.MG_OK              # finished
    srv.close()
    torch.cuda.synchronize()
    assert done[0]["status"] == mg.MG_OK and done[0]["relres"] <= 1e-8
    assert done[1]["status"] == mg.MG_ECANCELED and done[1]["steps"] == 1
    assert done[3]["status"] == mg.MG_ETIMEDOUT and done[3]["steps"] == 0
    assert done[2]["status"] == mg.MG_ETIMEDOUT and done[2]["steps"] >= 1 and 0.0 < done[2]["relres"] < 1e-6
    assert done[2]["t_done"] >= dl[2]
    for rid in (1, 3, 4):
        assert float(us[rid].abs().max()) == 0.0
    assert float(us[2].abs().max()) > 0.0 and float(us[0].abs().max()) > 0.0
    for rid in range(5):
        assert done[rid]["ticket"] == tickets[rid]
        print(f"request {rid}: status {done[rid]['status']} steps {done[rid]['steps']} "
              f"relres {done[rid]['relres']:.3e}", flush=True)


def test_largest_classes_alone_equal_mix_and_match_oracle(mg):
    """3-D 129^3 and 2-D 1025^2 / 513^2 requests (the marching batched ops)
    beside smaller ones: each result bitwise the same alone and in a
    staggered mix, within 1e-9 of the oracle's mixed-precision solve with
    the same step count, and its residual recomputed by the oracle."""
    import torch
    reqs = LARGE
    alone_res, alone_sol = {}, {}
    for rid in range(len(reqs)):
        print(f"alone: request {rid} {reqs[rid]}", flush=True)
        r, s, _ = run(mg, torch, reqs, [rid])
        alone_res.update(r)
        alone_sol.update(s)
    mix_res, mix_sol, st = run(mg, torch, reqs, [1, 0, 3, 2, 5, 4], stagger=True)
    for rid in range(len(reqs)):
        assert alone_res[rid]["status"] == mg.MG_OK
        assert mix_res[rid]["steps"] == alone_res[rid]["steps"]
        assert np.array_equal(mix_sol[rid], alone_sol[rid]), rid
        assert mix_res[rid]["relres"] == alone_res[rid]["relres"]
    print("mix stats", st, flush=True)
    oracle_check(mg, mix_res, mix_sol, reqs, [0, 1, 3, 4])
