"""Pins for the node-centred oracle: each check compares the oracle with
something other than itself (closed forms, brute-force loops on tiny grids,
exact identities of the textbook operators, library direct solves)."""
import itertools

import numpy as np
import pytest
import scipy.fft

from oracle import node
from paper_1904_08684_amd import workloads as W


def coords(n):
    return np.arange(n) / (n - 1)


# ---------------------------------------------------------------- operator
@pytest.mark.parametrize("d,n,ks", [(2, 17, (1, 1)), (2, 33, (3, 5)), (3, 9, (1, 2, 3)), (3, 17, (2, 1, 7))])
def test_operator_sine_eigenvector(d, n, ks):
    """A sin(k pi x)... = (4/h^2) sum_a sin^2(k_a pi h / 2) * the same mode."""
    h = 1.0 / (n - 1)
    u = W.sine_mode(n, d, ks)
    lam = 4.0 / h ** 2 * sum(np.sin(k * np.pi * h / 2) ** 2 for k in ks)
    Au = node.apply_A(u)
    c = node.interior(d)
    assert np.max(np.abs(Au[c] - lam * u[c])) <= 1e-12 * lam


@pytest.mark.parametrize("d", [2, 3])
def test_operator_exact_on_quadratic(d):
    """-Laplace(-x^2/2) = 1 and the 2nd difference is exact on quadratics."""
    n = 9
    x = coords(n)
    shape = [1] * d
    shape[-1] = n
    u = np.broadcast_to(-0.5 * x.reshape(shape) ** 2, (n,) * d).copy()
    Au = node.apply_A(u)
    assert np.allclose(Au[node.interior(d)], 1.0, rtol=0, atol=1e-11)


@pytest.mark.parametrize("d,n", [(2, 9), (3, 5)])
def test_operator_matches_brute_force_and_is_symmetric(d, n):
    A = node.dense_matrix(n, d)
    # brute force: A_ij = 2d s on the diagonal, -s for each axis neighbour
    s = (n - 1) ** 2
    pts = list(itertools.product(range(1, n - 1), repeat=d))
    B = np.zeros_like(A)
    for i, p in enumerate(pts):
        for j, q in enumerate(pts):
            diff = [abs(a - b) for a, b in zip(p, q)]
            if sum(diff) == 0:
                B[i, j] = 2 * d * s
            elif sum(diff) == 1:
                B[i, j] = -s
    assert np.array_equal(A, B)
    assert np.array_equal(A, A.T)
    assert np.all(np.linalg.eigvalsh(A) > 0)


# ---------------------------------------------------------------- Jacobi
@pytest.mark.parametrize("ks", [(1, 1), (3, 7), (15, 15), (8, 2)])
def test_jacobi_fourier_amplification(ks):
    """One damped-Jacobi sweep multiplies an error mode sin(k pi x) sin(l pi y)
    by 1 - omega (1 - (cos k pi h + cos l pi h) / 2)."""
    n, omega = 17, 0.8
    h = 1.0 / (n - 1)
    e = W.sine_mode(n, 2, ks)
    out = node.jacobi(e, np.zeros_like(e), omega)
    g = 1 - omega * (1 - (np.cos(ks[0] * np.pi * h) + np.cos(ks[1] * np.pi * h)) / 2)
    assert np.max(np.abs(out - g * e)) <= 1e-14


def test_jacobi_smoothing_factor_matches_lfa():
    """max over high frequencies of |Jacobi amplification| = 0.6 at omega = 0.8."""
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lfa_2d_rbgs.json")))
    om = gold["smoothing_factor_omega_jacobi"]["omega"]
    th = np.linspace(-np.pi, np.pi, 513)
    T1, T2 = np.meshgrid(th, th)
    high = np.maximum(np.abs(T1), np.abs(T2)) >= np.pi / 2
    amp = np.abs(1 - om * (1 - (np.cos(T1) + np.cos(T2)) / 2))
    # the oracle's amplification equals this symbol on every representable mode
    n = 33
    h = 1.0 / (n - 1)
    worst = 0.0
    for k in range(1, n - 1):
        for l in range(1, n - 1):
            if max(k, l) >= (n - 1) // 2:
                e = W.sine_mode(n, 2, (k, l))
                out = node.jacobi(e, np.zeros_like(e), om)
                c = node.interior(2)
                ratio = np.linalg.norm(out[c]) / np.linalg.norm(e[c])
                worst = max(worst, ratio)
    assert abs(amp[high].max() - gold["smoothing_factor_omega_jacobi"]["mu"]) < 1e-12
    assert abs(worst - gold["smoothing_factor_omega_jacobi"]["mu"]) < 0.02


# ---------------------------------------------------------------- RB-GS
def _gs_brute(u, f, colour):
    """Lexicographic loop over the nodes of one colour (pure Python)."""
    d = u.ndim
    n = u.shape[0]
    s = float((n - 1) ** 2)
    u = u.copy()
    for p in itertools.product(range(1, n - 1), repeat=d):
        if sum(p) % 2 != colour:
            continue
        nb = 0.0
        for ax in reversed(range(d)):
            for sh in (-1, 1):
                q = list(p)
                q[ax] += sh
                nb = nb + u[tuple(q)]
        u[p] = (f[p] / s + nb) / (2 * d)
    return u


@pytest.mark.parametrize("d,n", [(2, 9), (2, 17), (3, 9)])
def test_rbgs_equals_lexicographic_colour_loops(d, n):
    rng = np.random.default_rng(5)
    u = W.interior_uniform(n, d, 11)
    f = W.interior_uniform(n, d, 12) * 50
    ref = _gs_brute(_gs_brute(u, f, 0), f, 1)
    got = node.rbgs(u, f)
    assert np.array_equal(got, ref)
    del rng


@pytest.mark.parametrize("d,n", [(2, 17), (3, 17)])
def test_rbgs_colour_residual_invariant(d, n):
    """After the red half-sweep the residual vanishes at red nodes; after the
    black half-sweep it vanishes at black nodes (up to rounding)."""
    u = W.interior_uniform(n, d, 3)
    f = W.interior_uniform(n, d, 4) * 100
    c = node.interior(d)
    node.gs_colour(u, f, 0)
    r = node.residual(u, f)[c]
    red = node.colour_mask(n, d, 0)
    assert np.max(np.abs(r[red])) < 1e-9 * np.max(np.abs(r[~red]))
    node.gs_colour(u, f, 1)
    r = node.residual(u, f)[c]
    assert np.max(np.abs(r[~red])) < 1e-9 * np.max(np.abs(r[red]))


def test_rbgs_fixed_point_is_discrete_solution():
    n, d = 9, 2
    f = W.interior_uniform(n, d, 8)
    A = node.dense_matrix(n, d)
    c = node.interior(d)
    u = np.zeros_like(f)
    u[c] = np.linalg.solve(A, f[c].reshape(-1)).reshape((n - 2,) * d)
    assert np.max(np.abs(node.rbgs(u, f) - u)) < 1e-14


# ---------------------------------------------------------------- transfers
def _restriction_matrix(n, d):
    nc = (n + 1) // 2
    m, mc = (n - 2) ** d, (nc - 2) ** d
    R = np.zeros((mc, m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1
        r = np.zeros((n,) * d)
        r[node.interior(d)] = e.reshape((n - 2,) * d)
        R[:, j] = node.restrict_fw(r)[node.interior(d)].reshape(-1)
    return R


def _prolongation_matrix(n, d):
    nc = (n + 1) // 2
    m, mc = (n - 2) ** d, (nc - 2) ** d
    P = np.zeros((m, mc))
    for j in range(mc):
        e = np.zeros(mc)
        e[j] = 1
        ec = np.zeros((nc,) * d)
        ec[node.interior(d)] = e.reshape((nc - 2,) * d)
        P[:, j] = node.prolong_linear(ec)[node.interior(d)].reshape(-1)
    return P


@pytest.mark.parametrize("d,n", [(2, 9), (2, 17), (3, 9)])
def test_prolongation_is_2d_times_restriction_transpose(d, n):
    R = _restriction_matrix(n, d)
    P = _prolongation_matrix(n, d)
    assert np.array_equal(P, (2 ** d) * R.T)


@pytest.mark.parametrize("d,n", [(2, 17), (3, 9)])
def test_restriction_brute_force_weights(d, n):
    """f_c[I] = sum over the 3^d neighbours of 2I of prod (2-|o|)/4 r[2I+o]."""
    r = W.interior_uniform(n, d, 21)
    fc = node.restrict_fw(r)
    nc = (n + 1) // 2
    for I in itertools.product(range(1, nc - 1), repeat=d):
        acc = 0.0
        for o in itertools.product((-1, 0, 1), repeat=d):
            w = np.prod([2 - abs(k) for k in o]) / 4 ** d
            acc += w * r[tuple(2 * i + k for i, k in zip(I, o))]
        assert abs(fc[I] - acc) <= 1e-15
    # constants on the interior map to constants away from the boundary ring
    ones = np.zeros((n,) * d)
    ones[node.interior(d)] = 1.0
    fc1 = node.restrict_fw(ones)
    inner = (slice(2, -2),) * d
    assert np.all(fc1[inner] == 1.0)


@pytest.mark.parametrize("d,nc", [(2, 5), (2, 9), (3, 5)])
def test_prolongation_reproduces_multilinear_functions(d, nc):
    """Linear interpolation is exact for functions linear in each coordinate."""
    xc = np.arange(nc) / (nc - 1)
    nf = 2 * nc - 1
    xf = np.arange(nf) / (nf - 1)

    def g(*xs):
        out = 1.0
        for a, x in enumerate(xs):
            out = out * (0.3 + (a + 1) * x)
        return out + 0.7 * xs[-1]

    ec = g(*np.meshgrid(*([xc] * d), indexing="ij"))
    ef = g(*np.meshgrid(*([xf] * d), indexing="ij"))
    assert np.max(np.abs(node.prolong_linear(ec) - ef)) < 1e-14


# ---------------------------------------------------------------- direct solves
def dst_solve(f):
    """Exact discrete Poisson solution by the type-I sine transform."""
    n = f.shape[0]
    d = f.ndim
    h = 1.0 / (n - 1)
    k = np.arange(1, n - 1)
    lam1 = 4.0 / h ** 2 * np.sin(k * np.pi * h / 2) ** 2
    lam = np.zeros((n - 2,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = n - 2
        lam = lam + lam1.reshape(shape)
    c = node.interior(d)
    fh = scipy.fft.dstn(f[c], type=1, norm="ortho")
    u = np.zeros_like(f)
    u[c] = scipy.fft.idstn(fh / lam, type=1, norm="ortho")
    return u


@pytest.mark.parametrize("d,n", [(2, 9), (3, 5), (3, 9)])
def test_dst_agrees_with_dense_solve(d, n):
    f = W.interior_uniform(n, d, 31)
    A = node.dense_matrix(n, d)
    c = node.interior(d)
    ud = np.linalg.solve(A, f[c].reshape(-1)).reshape((n - 2,) * d)
    assert np.max(np.abs(dst_solve(f)[c] - ud)) < 1e-14 * np.max(np.abs(ud)) * 10


def test_c0_discrete_solution_closed_form():
    """For f = 2 pi^2 sin(pi x) sin(pi y) the discrete solution is
    c_h sin(pi x) sin(pi y), c_h = (pi h / 2)^2 / sin^2(pi h / 2)."""
    n = 129
    h = 1.0 / 128
    ch = (np.pi * h / 2) ** 2 / np.sin(np.pi * h / 2) ** 2
    assert abs(ch - 1.0000502009159198) < 1e-15
    u = dst_solve(W.sine_rhs_2d(n))
    assert np.max(np.abs(u - ch * W.sine_mode(n, 2))) < 1e-13
