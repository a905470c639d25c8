"""The solve server's scheduler on the CPU: mg_server_create_hosted runs the
same queue, footprint admission, hierarchy reuse and eviction, rounds,
deadlines and cancellation as the device server, with each round's
refinement steps done by an executor built here from the oracle's
primitives (FP64 residual, power-of-two scale, single-precision V-cycle,
update: the steps of the oracle's mixed-precision refinement).  Every
request's result must equal the oracle's mixed solve of that request run
alone, whatever else is queued or in flight."""
import ctypes as C
import time

import numpy as np
import pytest

from oracle import cycle
from paper_1904_08684_amd import workloads as W

MIX = [(2, 17), (3, 9), (2, 33), (3, 17), (2, 65), (2, 17), (3, 9), (2, 33)]
TOL = 1e-8


@pytest.fixture(scope="module")
def mg():
    """The library's binding: the hosted server makes no device call."""
    from paper_1904_08684_amd import mg as _mg
    return _mg


def method(mg, dim):
    return ("jacobi", mg.MG_JACOBI, 2, 2) if dim == 2 else ("rbgs", mg.MG_RBGS, 3, 3)


def params(dim, n, smoother, nu1, nu2):
    return cycle.Params(centering="node", dim=dim, n=n, smoother=smoother, omega=0.8, nu1=nu1, nu2=nu2)


def view(addr, dim, n):
    return np.ctypeslib.as_array((C.c_double * (n ** dim)).from_address(addr)).reshape((n,) * dim)


class OracleExecutor:
    """Hierarchies per slot; per request its iterate, the residual after
    its last step and that residual's largest magnitude."""

    def __init__(self, fail_on_step=None):
        self.hier = {}
        self.state = {}
        self.built = []
        self.released = []
        self.fail_on_step = fail_on_step

    def build(self, slot, r):
        dim, n = r.grid.dim, r.grid.n[0]
        sm = "jacobi" if r.opts.smoother == 0 else "rbgs"
        self.hier[slot] = cycle.build_hierarchy(params(dim, n, sm, r.opts.nu1, r.opts.nu2))
        self.built.append((slot, dim, n))

    def step(self, slots, first, reqs):
        if self.fail_on_step is not None and self.fail_on_step(reqs):
            raise RuntimeError("executor failure requested by the test")
        out = []
        for slot, fresh, r in zip(slots, first, reqs):
            h = self.hier[slot]
            dim, n = r.grid.dim, r.grid.n[0]
            init = 0.0
            if fresh:
                f = view(r.f, dim, n).copy()
                u = np.zeros_like(f)
                res = cycle.residual(h, 0, u, f)
                ru = np.asarray(cycle.unknowns(h, res))
                init = float(np.sum(ru * ru))
                st = {"f": f, "u": u, "r": res, "m": float(np.max(np.abs(ru))), "m_prev": None}
                self.state[r.id] = st
            st = self.state[r.id]
            if not np.isfinite(st["m"]):
                # (the oracle's coarse solve refuses non-finite data: report it)
                out.append((init, float("nan")))
                continue
            # sigma from the previous step's residual (the first step's from its own)
            sigma = cycle.pow2_scale(st["m"] if st["m_prev"] is None else st["m_prev"])
            st["m_prev"] = st["m"]
            r32 = (st["r"] / sigma).astype(np.float32)
            c = cycle.vcycle(h, np.zeros_like(r32), r32)
            st["u"] = st["u"] + sigma * c.astype(np.float64)
            st["r"] = cycle.residual(h, 0, st["u"], st["f"])
            ru = np.asarray(cycle.unknowns(h, st["r"]))
            st["m"] = float(np.max(np.abs(ru)))
            out.append((init, float(np.sum(ru * ru))))
        return out

    def finish(self, slot, r):
        view(r.u_out, r.grid.dim, r.grid.n[0])[...] = self.state[r.id]["u"]

    def release(self, slot):
        self.released.append(slot)
        self.hier.pop(slot, None)


def inputs(reqs):
    fs = [np.ascontiguousarray(W.interior_uniform(n, d, W.SEED_REQUEST_BASE + rid)) for rid, (d, n) in enumerate(reqs)]
    us = [np.full((n,) * d, -7.0) for d, n in reqs]   # untouched entries stay -7
    return fs, us


def submit(mg, srv, rid, reqs, fs, us, **kw):
    d, n = reqs[rid]
    _, sm, nu1, nu2 = method(mg, d)
    return srv.submit(rid, d, n, fs[rid], us[rid], TOL, sm, nu1, nu2, **kw)


def drain(srv, results, limit=200):
    for _ in range(limit):
        a, q = srv.step()
        for r in srv.poll():
            results[r["id"]] = r
        if a == 0 and q == 0:
            return
    raise AssertionError("server did not drain")


def oracle_alone(mg, reqs, fs, rid):
    d, n = reqs[rid]
    sm, _, nu1, nu2 = method(mg, d)
    h = cycle.build_hierarchy(params(d, n, sm, nu1, nu2))
    return cycle.mixed_solve(h, fs[rid], tol=TOL, max_outer=50)


def test_mix_equals_the_oracle_alone(mg):
    """Requests arriving two per round into a running mix: each result (its
    iterate bitwise, steps, relres) equals the oracle's mixed solve alone;
    hierarchies of a shape are reused; tickets follow submission order and
    the clock stamps are ordered."""
    ex = OracleExecutor()
    srv = mg.HostedServer(ex, 1 << 30, max_slots=3)
    fs, us = inputs(MIX)
    results, tickets = {}, []
    pending = list(range(len(MIX)))
    while pending:
        for rid in pending[:2]:
            assert submit(mg, srv, rid, MIX, fs, us) == mg.MG_OK
            tickets.append(srv.last_ticket)
        pending = pending[2:]
        srv.step()
        for r in srv.poll():
            results[r["id"]] = r
    drain(srv, results)
    st = srv.stats()
    srv.close()
    assert tickets == list(range(len(MIX)))
    for rid in range(len(MIX)):
        r = results[rid]
        u, hist = oracle_alone(mg, MIX, fs, rid)
        assert r["status"] == mg.MG_OK and r["ticket"] == rid
        assert r["steps"] == len(hist) - 1 and r["relres"] == hist[-1]
        assert np.array_equal(us[rid], u), rid
        assert r["t_arrive"] <= r["t_admit"] <= r["t_done"]
    # eight requests of five shapes, at most three in flight
    assert st["completed"] == len(MIX) and st["admitted"] == len(MIX)
    assert st["hierarchies_built"] < len(MIX)
    assert st["rounds"] > 0 and st["launches"] == 0


def test_admission_respects_the_budget_and_evicts_idle_hierarchies(mg):
    """With room for only the largest hierarchy plus a little, shapes take
    turns: the arena never exceeds its budget, idle hierarchies are evicted
    least recently used first, and every result still equals the oracle's."""
    reqs = [(2, 65), (3, 17), (2, 33), (2, 65), (3, 17)]
    fp = {(d, n): mg.server_footprint(d, n, *method(mg, d)[1:]) for d, n in set(reqs)}
    budget = max(fp.values()) + min(fp.values())
    ex = OracleExecutor()
    srv = mg.HostedServer(ex, budget, max_slots=4)
    fs, us = inputs(reqs)
    for rid in range(len(reqs)):
        assert submit(mg, srv, rid, reqs, fs, us) == mg.MG_OK
    results = {}
    drain(srv, results)
    st = srv.stats()
    srv.close()
    assert st["arena_peak_bytes"] <= budget
    assert st["evictions"] > 0 and len(ex.released) == st["evictions"]
    for rid in range(len(reqs)):
        u, hist = oracle_alone(mg, reqs, fs, rid)
        assert results[rid]["status"] == mg.MG_OK
        assert np.array_equal(us[rid], u)


def test_request_larger_than_the_arena_is_refused(mg):
    fp = mg.server_footprint(3, 17, mg.MG_RBGS, 3, 3)
    srv = mg.HostedServer(OracleExecutor(), fp - 4096, max_slots=2)
    fs, us = inputs([(3, 17)])
    assert submit(mg, srv, 0, [(3, 17)], fs, us) == mg.MG_ENOMEM
    assert srv.stats()["queued"] == 0
    srv.close()


def test_cancellation_and_deadlines(mg):
    """One slot: request 0 runs, 1 is cancelled while queued, 2 waits past
    its deadline, 3 is cancelled in flight, 4 runs out of time in flight.
    Retired-unadmitted requests leave u_out untouched; a request past its
    deadline in flight returns its iterate so far."""
    reqs = [(2, 33), (2, 33), (2, 33), (2, 33), (3, 17)]
    ex = OracleExecutor()
    srv = mg.HostedServer(ex, 1 << 30, max_slots=1)
    fs, us = inputs(reqs)
    tk = {}
    for rid in range(3):
        dl = srv.clock() + 0.05 if rid == 2 else 0.0
        assert submit(mg, srv, rid, reqs, fs, us, deadline=dl) == mg.MG_OK
        tk[rid] = srv.last_ticket
    assert srv.cancel(tk[1]) == mg.MG_OK
    assert srv.cancel(tk[1]) == mg.MG_EINVAL          # already finished
    time.sleep(0.06)
    results = {}
    drain(srv, results)
    assert results[1]["status"] == mg.MG_ECANCELED and results[1]["steps"] == 0
    assert results[2]["status"] == mg.MG_ETIMEDOUT and results[2]["steps"] == 0
    assert np.all(us[1] == -7.0) and np.all(us[2] == -7.0)
    assert results[0]["status"] == mg.MG_OK
    # in flight: cancelled after its first round
    assert submit(mg, srv, 3, reqs, fs, us) == mg.MG_OK
    srv.step()
    assert srv.cancel(srv.last_ticket) == mg.MG_OK
    drain(srv, results)
    assert results[3]["status"] == mg.MG_ECANCELED and results[3]["steps"] == 1
    # in flight past its deadline: retired after the round that crosses it,
    # with the iterate of its two steps
    assert submit(mg, srv, 4, reqs, fs, us, deadline=srv.clock() + 0.05) == mg.MG_OK
    srv.step()
    time.sleep(0.06)
    drain(srv, results)
    srv.close()
    r = results[4]
    assert r["status"] == mg.MG_ETIMEDOUT and r["steps"] == 2
    ref = OracleExecutor()
    q = _req(mg, reqs[4], fs[4], 4)
    ref.build(0, q)
    (init, _), = ref.step([0], [1], [q])
    (_, last), = ref.step([0], [0], [q])
    assert np.array_equal(us[4], ref.state[4]["u"])
    assert r["relres"] == np.sqrt(last) / np.sqrt(init)


def _req(mg, shape, f, rid):
    d, n = shape
    sm, smc, nu1, nu2 = method(mg, d)
    r = mg.mg_request()
    r.id = rid
    r.grid = mg.make_grid(d, n)
    r.opts = mg.make_opts(smc, 0.8, nu1, nu2, mg.MG_MIXED, 50)
    r.f = f.ctypes.data
    return r


def test_nonfinite_rhs_and_executor_failure(mg):
    """A NaN in the right-hand side retires the request with MG_ENONFINITE
    after its first round; an executor failure aborts the round and is
    reported by mg_server_step."""
    reqs = [(2, 17), (2, 17)]
    fs, us = inputs(reqs)
    fs[0][5, 5] = np.nan
    srv = mg.HostedServer(OracleExecutor(), 1 << 30, max_slots=2)
    assert submit(mg, srv, 0, reqs, fs, us) == mg.MG_OK
    results = {}
    with np.errstate(invalid="ignore"):
        drain(srv, results)
    srv.close()
    assert results[0]["status"] == mg.MG_ENONFINITE and results[0]["steps"] == 1
    ex = OracleExecutor(fail_on_step=lambda reqs: any(r.id == 1 for r in reqs))
    srv = mg.HostedServer(ex, 1 << 30, max_slots=2)
    assert submit(mg, srv, 1, reqs, fs, us) == mg.MG_OK
    with pytest.raises(mg.MGError) as e:
        srv.step()
    assert e.value.code == mg.MG_EDEVICE and isinstance(srv.callback_error, RuntimeError)
    srv.close()
