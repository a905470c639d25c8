"""Pins for the oracle's V-cycle, solve and mixed-precision refinement:
textbook two-grid factors, direct solves and closed forms."""
import json
import os

import numpy as np
import pytest

from oracle import cell, cycle, node
from paper_1904_08684_amd import workloads as W
from tests.test_oracle_node import dst_solve

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lfa_2d_rbgs.json")))


def two_grid_matrix(p: cycle.Params):
    """Dense two-grid iteration matrix (f = 0) of the oracle's cycle with an
    exact coarse solve, built by applying one cycle to unit vectors."""
    q = cycle.Params(**{**p.__dict__, "coarsest": (p.n + 1) // 2})
    h = cycle.build_hierarchy(q)
    assert h.levels == 2
    n, d = p.n, p.dim
    m = (n - 2) ** d
    M = np.zeros((m, m))
    f = np.zeros((n,) * d)
    c = node.interior(d)
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1
        u = np.zeros((n,) * d)
        u[c] = e.reshape((n - 2,) * d)
        M[:, j] = cycle.vcycle(h, u, f)[c].reshape(-1)
    return M


def spectral_radius(M):
    return float(np.max(np.abs(np.linalg.eigvals(M))))


@pytest.mark.parametrize("nu", [1, 2])
def test_two_grid_rbgs_matches_lfa(nu):
    p = cycle.Params(centering="node", dim=2, n=33, smoother="rbgs", nu1=nu, nu2=nu)
    rho = spectral_radius(two_grid_matrix(p))
    ref = GOLD["rho_two_grid"][str(2 * nu)]
    assert abs(rho - ref) / ref < 0.05, (rho, ref)


def test_two_grid_jacobi_near_smoothing_bound():
    """omega-Jacobi V(2,2): the two-grid factor is close to mu^4 = 0.1296."""
    p = cycle.Params(centering="node", dim=2, n=33, smoother="jacobi", omega=0.8, nu1=2, nu2=2)
    rho = spectral_radius(two_grid_matrix(p))
    mu = GOLD["smoothing_factor_omega_jacobi"]["mu"]
    assert mu ** 4 * 0.95 < rho < mu ** 4 * 1.15, rho


def _vcycle_factor(p, cycles_=10):
    """Asymptotic V-cycle factor by power iteration with f = 0."""
    h = cycle.build_hierarchy(p)
    e = W.interior_uniform(p.n, p.dim, 77)
    f = np.zeros_like(e)
    c = node.interior(p.dim)
    nrm = [np.linalg.norm(e[c])]
    for _ in range(cycles_):
        e = cycle.vcycle(h, e, f)
        nrm.append(np.linalg.norm(e[c]))
    return (nrm[-1] / nrm[-4]) ** (1 / 3)


def test_vcycle_factor_2d_rbgs_h_independent():
    """The V(2,2) factor stays within 1.5x the two-grid LFA value and does not
    grow under refinement."""
    rates = []
    for n in (33, 65, 129):
        p = cycle.Params(centering="node", dim=2, n=n, smoother="rbgs", nu1=2, nu2=2)
        rates.append(_vcycle_factor(p, 12))
    assert max(rates) <= 1.5 * GOLD["rho_two_grid"]["4"], rates
    assert max(rates) - min(rates) < 0.01, rates


def test_vcycle_factor_3d_rbgs():
    p = cycle.Params(centering="node", dim=3, n=33, smoother="rbgs", nu1=3, nu2=3)
    rate = _vcycle_factor(p, 10)
    assert rate < 0.09, rate


def test_two_grid_3d_rbgs_power_iteration():
    """3-D RB-GS V(3,3) two-grid factor at n = 17, by power iteration."""
    p = cycle.Params(centering="node", dim=3, n=17, smoother="rbgs", nu1=3, nu2=3, coarsest=9)
    h = cycle.build_hierarchy(p)
    assert h.levels == 2
    e = W.interior_uniform(17, 3, 5)
    f = np.zeros_like(e)
    norms = [np.linalg.norm(e)]
    for _ in range(25):
        e = cycle.vcycle(h, e, f)
        norms.append(np.linalg.norm(e))
    rho = (norms[-1] / norms[-6]) ** 0.2
    assert 0.03 < rho < 0.08, rho


@pytest.mark.parametrize("d,n,smoother", [(2, 17, "jacobi"), (2, 33, "rbgs"), (3, 9, "rbgs"), (3, 17, "jacobi")])
def test_vcycles_converge_to_dense_solution(d, n, smoother):
    p = cycle.Params(centering="node", dim=d, n=n, smoother=smoother, nu1=2, nu2=2)
    h = cycle.build_hierarchy(p)
    f = W.interior_uniform(n, d, 40)
    A = node.dense_matrix(n, d)
    c = node.interior(d)
    ud = np.linalg.solve(A, f[c].reshape(-1))
    u = np.zeros_like(f)
    for _ in range(50):
        u = cycle.vcycle(h, u, f)
    assert np.linalg.norm(u[c].reshape(-1) - ud) <= 1e-13 * np.linalg.norm(ud) * 10


def test_coarse_solve_is_exact():
    for d in (2, 3):
        p = cycle.Params(centering="node", dim=d, n=5, smoother="rbgs")
        h = cycle.build_hierarchy(p)
        assert h.levels == 1
        f = W.interior_uniform(5, d, 9)
        e = cycle.coarse_solve(h, f)
        assert np.max(np.abs(node.residual(e, f))) < 1e-13 * np.max(np.abs(f)) * 16
        assert np.max(np.abs(e - dst_solve(f))) < 1e-16 * 100


def test_c0_solution_closed_form():
    """The oracle's C0 solve reaches c_h sin(pi x) sin(pi y)."""
    n = 129
    p = cycle.Params(centering="node", dim=2, n=n, smoother="jacobi", omega=0.8, nu1=2, nu2=2)
    h = cycle.build_hierarchy(p)
    ch = (np.pi / 256) ** 2 / np.sin(np.pi / 256) ** 2
    u, hist, _ = cycle.solve(h, W.sine_rhs_2d(n), W.interior_uniform(n, 2, 0), tol=1e-13, max_cycles=40)
    assert hist[-1] <= 1e-13
    assert np.max(np.abs(u - ch * W.sine_mode(n, 2))) < 5e-12


def test_3d_solve_matches_dst():
    n = 33
    p = cycle.Params(centering="node", dim=3, n=n, smoother="rbgs", nu1=3, nu2=3)
    h = cycle.build_hierarchy(p)
    f = W.interior_uniform(n, 3, 1)
    u, hist, _ = cycle.solve(h, f, tol=1e-10)
    assert hist[-1] <= 1e-10 and len(hist) - 1 <= 12
    ud = dst_solve(f)
    kappa = 4 * (n - 1) ** 2 / (3 * np.pi ** 2) * 3
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) <= kappa * 1e-10


def test_mixed_precision_reaches_fp64_tolerance():
    n = 33
    p = cycle.Params(centering="node", dim=3, n=n, smoother="rbgs", nu1=3, nu2=3)
    h = cycle.build_hierarchy(p)
    f = W.interior_uniform(n, 3, 1)
    u, hist = cycle.mixed_solve(h, f, tol=1e-10)
    # recompute the final residual independently of the solver's own bookkeeping
    rel = np.linalg.norm(node.residual(u, f)) / np.linalg.norm(f)
    assert rel <= 1e-10 and abs(rel - hist[-1]) <= 1e-3 * rel
    ud = dst_solve(f)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-8
    # the refinement contracts like the FP64 cycle (single precision is not the bottleneck)
    rates = [hist[i + 1] / hist[i] for i in range(1, len(hist) - 1)]
    assert max(rates) < 0.15


def test_float32_cycle_stays_in_float32_and_tracks_fp64():
    n = 17
    p = cycle.Params(centering="node", dim=3, n=n, smoother="rbgs", nu1=3, nu2=3)
    h = cycle.build_hierarchy(p)
    f = W.interior_uniform(n, 3, 2)
    c32 = cycle.vcycle(h, np.zeros(f.shape, np.float32), f.astype(np.float32))
    c64 = cycle.vcycle(h, np.zeros_like(f), f)
    assert c32.dtype == np.float32
    assert np.max(np.abs(c32 - c64)) <= 1e-5 * np.max(np.abs(c64))


def test_refinement_scale_is_immaterial_in_range_and_keeps_tiny_residuals():
    """Every operation of the single-precision cycle commutes with a power of
    two, so the refinement iterates are bitwise the same whether the scale
    comes from the previous or the current residual; and scaling f by 2^-140
    (its residuals lie below FP32's smallest normal, about 1.2e-38, so an
    unscaled float32 cycle would flush them) scales the solution by exactly
    2^-140, which holds only if the scale is applied."""
    n = 17
    p = cycle.Params(centering="node", dim=3, n=n, smoother="rbgs", nu1=3, nu2=3)
    h = cycle.build_hierarchy(p)
    f = W.interior_uniform(n, 3, 1)
    u_prev, hist_prev = cycle.mixed_solve(h, f, tol=1e-10, scale="previous")
    u_cur, hist_cur = cycle.mixed_solve(h, f, tol=1e-10, scale="current")
    assert np.array_equal(u_prev, u_cur) and hist_prev == hist_cur
    tiny = 2.0 ** -140
    u_tiny, hist_tiny = cycle.mixed_solve(h, f * tiny, tol=1e-10)
    assert np.array_equal(u_tiny, u_prev * tiny)
    assert np.allclose(hist_tiny, hist_prev, rtol=0, atol=0)
    # without the scale the same steps lose the residual to underflow
    r32 = (node.residual(np.zeros_like(f), f * tiny)).astype(np.float32)
    assert np.count_nonzero(r32) < np.count_nonzero(f)


def test_pow2_scale():
    for v in (1.0, 0.75, 3.0, 1e-300, 5e300, 2.0 ** -20):
        s = cycle.pow2_scale(v)
        assert s <= v < 2 * s and np.log2(s) == np.floor(np.log2(s))


# ------------------------------------------------------------ W- and F-cycles

@pytest.mark.parametrize("n", [33, 65, 129])
def test_cycle_types_visit_the_coarsest_level_as_defined(n):
    """gamma = 2 doubles the visits of every level below the second-coarsest,
    and the F-cycle adds one visit per level: per cycle the coarsest solve runs
    1 (V), 2^(L-2) (W) and L-1 (F) times for L levels."""
    for kind, count in (("V", lambda L: 1), ("W", lambda L: 2 ** (L - 2)), ("F", lambda L: L - 1)):
        h = cycle.build_hierarchy(cycle.Params(centering="node", dim=2, n=n, smoother="rbgs", nu1=1, nu2=1,
                                               cycle=kind))
        u = W.interior_uniform(n, 2, 5)
        cycle.vcycle(h, u, np.zeros_like(u))
        assert h.coarse_solves == count(h.levels), (kind, h.levels, h.coarse_solves)


def test_cycle_types_agree_on_two_levels():
    """With one level above the exact coarsest solve, V, W and F are the same
    two-grid cycle, bit for bit."""
    n = 9
    f = W.interior_uniform(n, 2, 3)
    u0 = W.interior_uniform(n, 2, 4)
    out = []
    for kind in ("V", "W", "F"):
        h = cycle.build_hierarchy(cycle.Params(centering="node", dim=2, n=n, smoother="rbgs", nu1=2, nu2=2,
                                               cycle=kind))
        assert h.levels == 2
        out.append(cycle.vcycle(h, u0, f))
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


@pytest.mark.parametrize("nu", [1, 2])
def test_w_and_f_cycles_reach_the_two_grid_factor(nu):
    """A W-cycle (and an F-cycle) recovers the two-grid convergence factor
    within the LFA's accuracy on a 5-level hierarchy, where the V-cycle is
    slower."""
    ref = GOLD["rho_two_grid"][str(2 * nu)]
    fac = {}
    for kind in ("V", "W", "F"):
        fac[kind] = _vcycle_factor(cycle.Params(centering="node", dim=2, n=65, smoother="rbgs", nu1=nu, nu2=nu,
                                                cycle=kind), cycles_=12)
    for kind in ("W", "F"):
        assert ref / 1.35 < fac[kind] < ref * 1.35, (kind, fac, ref)
    assert fac["V"] > 1.2 * fac["W"], fac


@pytest.mark.parametrize("kind", ["W", "F"])
def test_w_and_f_cycles_converge_to_dense_solution(kind):
    n = 17
    f = W.interior_uniform(n, 2, 9)
    h = cycle.build_hierarchy(cycle.Params(centering="node", dim=2, n=n, smoother="rbgs", nu1=2, nu2=2,
                                           cycle=kind))
    u, hist, _ = cycle.solve(h, f, tol=1e-14, max_cycles=40)
    A = node.dense_matrix(n, 2)
    c = node.interior(2)
    ud = np.linalg.solve(A, f[c].reshape(-1))
    assert np.max(np.abs(u[c].reshape(-1) - ud)) <= 1e-12 * np.max(np.abs(ud))


# ------------------------------------------------------------------ full multigrid

def _fmg_errors(dim, n, sm, nu, cpl):
    """FMG on -Lap u = dim pi^2 prod sin(pi x): returns the algebraic error
    max |u_fmg - u_h| over the discretisation error max |u_h - u|, where the
    discrete solution is u_h = c_h u with c_h = (pi h / 2)^2 / sin^2(pi h / 2)
    in closed form."""
    h = cycle.build_hierarchy(cycle.Params(centering="node", dim=dim, n=n, smoother=sm, nu1=nu, nu2=nu))
    ue = W.sine_mode(n, dim)
    f = dim * np.pi ** 2 * ue
    hh = 1.0 / (n - 1)
    ch = (np.pi * hh / 2) ** 2 / np.sin(np.pi * hh / 2) ** 2
    u = cycle.fmg(h, f, cpl)
    return np.max(np.abs(u - ch * ue)) / abs(ch - 1.0)


def test_fmg_reaches_discretisation_accuracy_2d():
    """One FMG pass with one RB-GS V(2,2)-cycle per level leaves an algebraic
    error below the discretisation error, independently of h."""
    r = [_fmg_errors(2, n, "rbgs", 2, 1) for n in (33, 65, 129, 257)]
    assert max(r) < 1.0 and max(r) / min(r) < 1.1, r


def test_fmg_reaches_discretisation_accuracy_3d():
    """3-D, RB-GS V(3,3), two cycles per level: algebraic error at most 0.15 of
    the discretisation error on every grid."""
    r = [_fmg_errors(3, n, "rbgs", 3, 2) for n in (17, 33, 65)]
    assert max(r) < 0.15, r


def test_fmg_more_cycles_approach_the_discrete_solution():
    r = [_fmg_errors(2, 65, "jacobi", 2, c) for c in (1, 2, 3)]
    assert r[0] > r[1] > r[2], r


# ----------------------------------------------- multigrid-preconditioned CG

def test_vcycle_preconditioner_symmetric_with_reversed_post_order():
    """b . M a = a . M b for the V(2,2) cycle from zero when post-smoothing runs
    the colours in reverse (black, red); with red-first post-smoothing it is
    not symmetric."""
    gaps = {}
    for post in ((1, 0), (0, 1)):
        h = cycle.build_hierarchy(cycle.Params(centering="node", dim=2, n=17, smoother="rbgs", nu1=2, nu2=2,
                                               post_order=post))
        a = W.interior_uniform(17, 2, 1)
        b = W.interior_uniform(17, 2, 2)
        ma = cycle.vcycle(h, np.zeros_like(a), a)
        mb = cycle.vcycle(h, np.zeros_like(b), b)
        gaps[post] = abs(cycle.dot(h, b, ma) - cycle.dot(h, a, mb)) / abs(cycle.dot(h, b, ma))
    assert gaps[(1, 0)] < 1e-14 and gaps[(0, 1)] > 1e-6, gaps


def test_plain_cg_terminates_within_m_steps():
    n = 9
    h = cycle.build_hierarchy(cycle.Params(centering="node", dim=2, n=n, smoother="rbgs", nu1=1, nu2=1,
                                           post_order=(1, 0)))
    f = W.interior_uniform(n, 2, 3)
    u, hist = cycle.pcg(h, f, tol=1e-13, max_it=200, precondition=False)
    assert len(hist) - 1 <= (n - 2) ** 2 and hist[-1] <= 1e-13


@pytest.mark.parametrize("centering", ["node", "cell"])
def test_pcg_reaches_dense_solution(centering):
    if centering == "node":
        n = 17
        p = cycle.Params(centering="node", dim=2, n=n, smoother="rbgs", nu1=2, nu2=2, post_order=(1, 0))
        f = W.interior_uniform(n, 2, 9)
        A = node.dense_matrix(n, 2)
        c = node.interior(2)
    else:
        n = 8
        k = W.varcoef_k(n, 3)
        p = cycle.Params(centering="cell", dim=3, n=n, coarsest=4, smoother="rbgs", nu1=2, nu2=2,
                         post_order=(1, 0), k=k)
        f = W.normal_zero_mean(n, 3, 9)
        h0 = cycle.build_hierarchy(p)
        A = cell.dense_matrix(h0.beta[0], n, 3)
        c = (slice(None),) * 3
    h = cycle.build_hierarchy(p)
    u, hist = cycle.pcg(h, f, tol=1e-14, max_it=60)
    ud = np.linalg.solve(A, f[c].reshape(-1))
    assert np.max(np.abs(u[c].reshape(-1) - ud)) <= 1e-12 * np.max(np.abs(ud))


def test_pcg_needs_fewer_iterations_than_stationary_cycles():
    n = 33
    h = cycle.build_hierarchy(cycle.Params(centering="node", dim=3, n=n, smoother="rbgs", nu1=2, nu2=2,
                                           post_order=(1, 0)))
    f = W.interior_uniform(n, 3, 1)
    _, hp = cycle.pcg(h, f, tol=1e-10)
    _, hm, _ = cycle.solve(h, f, tol=1e-10)
    assert len(hp) < len(hm), (len(hp), len(hm))
