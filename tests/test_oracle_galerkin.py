"""Pins of the oracle's Galerkin coarse operators (node grids): the textbook
nine-point stencil in 2-D, the tensor-product closed form on every level
computed in exact rational arithmetic, the projection property of the
Galerkin coarse-grid correction, and the solution of a Galerkin V-cycle."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import cycle, galerkin, node
from paper_1904_08684_amd import workloads as W


def test_2d_galerkin_of_five_point_laplacian_is_the_nine_point_stencil():
    n = 33
    W0 = galerkin.laplacian_stencil(n, 2)
    W1 = galerkin.coarse_stencil(W0)
    H = 2.0 / (n - 1)
    want = np.array([[-1, -2, -1], [-2, 12, -2], [-1, -2, -1]]) / (4 * H * H)
    assert np.max(np.abs(W1 - want)) <= 1e-12 * 12 / (4 * H * H)


def galerkin_1d(S):
    """R1 S P1 for a 3-point 1-D stencil S, exactly, from dense 1-D matrices:
    R1 = [1 2 1] / 4 at the coarse nodes, P1 = linear interpolation."""
    nc, nf = 7, 13
    R = [[Fraction(0)] * nf for _ in range(nc)]
    for I in range(1, nc - 1):
        for o, w in ((-1, Fraction(1, 4)), (0, Fraction(1, 2)), (1, Fraction(1, 4))):
            R[I][2 * I + o] = w
    P = [[Fraction(0)] * nc for _ in range(nf)]
    for J in range(nc):
        P[2 * J][J] = Fraction(1)
        if 2 * J - 1 >= 0:
            P[2 * J - 1][J] = Fraction(1, 2)
        if 2 * J + 1 < nf:
            P[2 * J + 1][J] = Fraction(1, 2)
    A = [[Fraction(0)] * nf for _ in range(nf)]
    for i in range(1, nf - 1):
        for o in (-1, 0, 1):
            A[i][i + o] = S[o + 1]
    AP = [[sum(A[i][k] * P[k][j] for k in range(nf)) for j in range(nc)] for i in range(nf)]
    RAP = [[sum(R[i][k] * AP[k][j] for k in range(nf)) for j in range(nc)] for i in range(nc)]
    return [RAP[3][2], RAP[3][3], RAP[3][4]]


@pytest.mark.parametrize("d,n,levels", [(2, 65, 4), (3, 33, 3)])
def test_galerkin_stencils_match_the_tensor_product_closed_form(d, n, levels):
    """A = s sum_a T_a (x) M_b (x) ...: with T = [-1 2 -1], M = [0 1 0] on the
    finest level, R A P is again such a sum with T <- R1 T P1, M <- R1 M P1
    (the transfers are tensor products), computed here exactly."""
    s = Fraction((n - 1) ** 2)
    T = [-s, 2 * s, -s]
    M = [Fraction(0), Fraction(1), Fraction(0)]
    Wl = galerkin.laplacian_stencil(n, d)
    for _ in range(levels):
        T, M = galerkin_1d(T), galerkin_1d(M)
        Wl = galerkin.coarse_stencil(Wl)
        want = np.zeros((3,) * d)
        for o in itertools.product(range(3), repeat=d):
            acc = Fraction(0)
            for a in range(d):
                t = T[o[a]]
                for b in range(d):
                    if b != a:
                        t = t * M[o[b]]
                acc += t
            want[o] = float(acc)
        assert np.max(np.abs(Wl - want)) <= 1e-12 * np.max(np.abs(want))
        # symmetric, rows sum to zero (constants are not touched inside)
        assert np.allclose(Wl, Wl[::-1, ::-1] if d == 2 else Wl[::-1, ::-1, ::-1], rtol=0, atol=1e-9)
        assert abs(Wl.sum()) <= 1e-12 * np.max(np.abs(Wl))


@pytest.mark.parametrize("d,n", [(2, 17), (3, 9)])
def test_galerkin_coarse_grid_correction_annihilates_the_restricted_residual(d, n):
    """With A_c = R A P and an exact coarse solve the corrected residual
    satisfies R r = 0 (the correction is a projection); the rediscretised
    coarse operator does not have this property."""
    f = W.interior_uniform(n, d, 5)
    u = W.interior_uniform(n, d, 6)
    nc = (n + 1) // 2
    c = node.interior(d)
    W0 = galerkin.laplacian_stencil(n, d)
    for Ac, galer in ((galerkin.dense_matrix(galerkin.coarse_stencil(W0), nc), True),
                      (node.dense_matrix(nc, d), False)):
        fc = node.restrict_fw(node.residual(u, f))
        ec = np.zeros((nc,) * d)
        ec[c] = np.linalg.solve(Ac, fc[c].reshape(-1)).reshape((nc - 2,) * d)
        rc = node.restrict_fw(node.residual(node.correct(u, ec), f))
        rel = np.max(np.abs(rc)) / np.max(np.abs(fc))
        assert (rel <= 1e-12) if galer else (rel > 1e-3), (galer, rel)


def test_galerkin_vcycle_reaches_the_dense_solution():
    n = 17
    d = 3
    f = W.interior_uniform(n, d, 7)
    p = cycle.Params(centering="node", dim=d, n=n, smoother="jacobi", omega=0.8, nu1=2, nu2=2,
                     coarse_op="galerkin")
    h = cycle.build_hierarchy(p)
    u, hist, _ = cycle.solve(h, f, tol=1e-13, max_cycles=60)
    c = node.interior(d)
    ud = np.linalg.solve(node.dense_matrix(n, d), f[c].reshape(-1))
    assert np.max(np.abs(u[c].reshape(-1) - ud)) <= 1e-11 * np.max(np.abs(ud))
    rates = [hist[i + 1] / hist[i] for i in range(1, len(hist) - 1)]
    assert max(rates) < 0.35, rates


def test_galerkin_needs_node_grids_and_jacobi():
    for kw in ({"centering": "cell", "n": 16, "coarsest": 4, "smoother": "jacobi"},
               {"centering": "node", "n": 17, "smoother": "rbgs"}):
        with pytest.raises(ValueError):
            cycle.build_hierarchy(cycle.Params(dim=2, coarse_op="galerkin", **kw))


def galerkin_symbol(T, M, thetas):
    """Eigenvalue of the tensor-product stencil sum_a T_a (x) M_b (x) ... on the
    sine mode with angles thetas (one per axis): a symmetric 3-point 1-D
    stencil S acts on sin(j theta) as S[1] + 2 S[0] cos(theta)."""
    t = [float(T[1]) + 2 * float(T[0]) * np.cos(th) for th in thetas]
    m = [float(M[1]) + 2 * float(M[0]) * np.cos(th) for th in thetas]
    lam = 0.0
    for a in range(len(thetas)):
        term = t[a]
        for b in range(len(thetas)):
            if b != a:
                term *= m[b]
        lam += term
    return lam


@pytest.mark.parametrize("omega", [0.5, 0.8])
@pytest.mark.parametrize("d,n,level,ks", [(2, 33, 1, (1, 1)), (2, 33, 1, (5, 12)), (2, 65, 2, (3, 14)),
                                          (3, 17, 1, (1, 2, 3)), (3, 33, 2, (7, 1, 4))])
def test_galerkin_jacobi_fourier_amplification(omega, d, n, level, ks):
    """On a Galerkin level the stencil is a constant tensor product
    s sum_a T_a (x) M_b (x) ... (T, M the exact 1-D Galerkin products of
    [-1 2 -1] and [0 1 0]), so the sine modes of that level are eigenvectors
    and one damped-Jacobi sweep with f = 0 multiplies them by exactly
    1 - omega lam / W_centre, lam the stencil's symbol.  The stencil fed to
    the sweep is the closed form built here, not the oracle's R A P."""
    s = Fraction((n - 1) ** 2)
    T = [-s, 2 * s, -s]
    M = [Fraction(0), Fraction(1), Fraction(0)]
    for _ in range(level):
        T, M = galerkin_1d(T), galerkin_1d(M)
    Wl = np.zeros((3,) * d)
    for o in itertools.product(range(3), repeat=d):
        acc = Fraction(0)
        for a in range(d):
            t = T[o[a]]
            for b in range(d):
                if b != a:
                    t = t * M[o[b]]
            acc += t
        Wl[o] = float(acc)
    nl = (n - 1) // 2 ** level + 1
    H = 1.0 / (nl - 1)
    v = W.sine_mode(nl, d, ks)
    out = galerkin.jacobi(v, np.zeros_like(v), Wl, omega)
    lam = galerkin_symbol(T, M, [k * np.pi * H for k in ks])
    centre = float(d * T[1] * M[1] ** (d - 1))
    g = 1 - omega * lam / centre
    assert np.max(np.abs(out - g * v)) <= 1e-13
    if d == 2 and level == 1:
        # the textbook nine-point stencil: symbol (3 - c_k - c_l - c_k c_l) / H^2, centre 3 / H^2
        ck, cl = np.cos(ks[0] * np.pi * H), np.cos(ks[1] * np.pi * H)
        assert abs(g - (1 - omega * (3 - ck - cl - ck * cl) / 3)) <= 1e-14
