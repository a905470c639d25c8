"""Pins of the oracle's DG element integrals: the quadrature rule against the
closed-form monomial integrals of the reference triangle, orthonormality of
the paper's basis, the hand-written gradients against finite differences,
and the volume integrals of constant fields against the boundary integrals
the divergence theorem turns them into (1-D Gauss rule on the three edges)."""
import math

import numpy as np
import pytest

from oracle import dg


def test_triangle_rule_integrates_monomials_exactly():
    X, Y, Wt = dg.triangle_rule()
    for a in range(13):
        for b in range(13 - a):
            want = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(np.sum(Wt * X ** a * Y ** b) - want) <= 1e-15 + 1e-13 * want


def test_basis_is_orthonormal_on_the_reference_triangle():
    X, Y, Wt = dg.triangle_rule()
    P = np.array(dg.basis(X, Y))
    M = (P * Wt) @ P.T
    assert np.max(np.abs(M - np.eye(10))) <= 1e-13


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.uniform(0.05, 0.45, 20)
    y = rng.uniform(0.05, 0.45, 20)
    h = 1e-6
    gx, gy = dg.basis_grad(x, y)
    for p in range(10):
        fx = (np.asarray(dg.basis(x + h, y)[p]) - np.asarray(dg.basis(x - h, y)[p])) / (2 * h)
        fy = (np.asarray(dg.basis(x, y + h)[p]) - np.asarray(dg.basis(x, y - h)[p])) / (2 * h)
        assert np.max(np.abs(gx[p] - fx)) <= 1e-6 * (1 + np.max(np.abs(fx)))
        assert np.max(np.abs(gy[p] - fy)) <= 1e-6 * (1 + np.max(np.abs(fy)))


def edge_integrals(k, B, a1, Ac):
    """sum over edges of int phi_ep (A_j . n) ds for a constant flux tensor Ac
    (3 x 2), with a 1-D Gauss rule and outward normals (counter-clockwise)."""
    K = dg.K_OF[k]
    det = B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]
    verts = [a1, a1 + B[:, 0], a1 + B[:, 1]]
    t, w = np.polynomial.legendre.leggauss(6)
    s = (t + 1) / 2
    out = np.zeros((3, K))
    for q in range(3):
        p0, p1 = verts[q], verts[(q + 1) % 3]
        d = p1 - p0
        L = np.hypot(d[0], d[1])
        n = np.array([d[1], -d[0]]) / L               # outward for counter-clockwise vertices
        pts = p0[None, :] + s[:, None] * d[None, :]
        ref = np.linalg.solve(B, (pts - a1).T)        # reference coordinates
        phi = np.array(dg.basis(ref[0], ref[1]))[:K] / math.sqrt(abs(det))
        for j in range(3):
            out[j] += (phi * (w / 2 * L)).sum(axis=1) * (Ac[j] @ n)
    return out


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_constant_fields_reduce_to_boundary_integrals(k):
    """A constant flux tensor has no divergence: (A, grad phi)_Omega equals
    the boundary integral of phi A n, for every element shape and order."""
    rng = np.random.default_rng(10 + k)
    K = dg.K_OF[k]
    g = 9.81
    for _ in range(4):
        a1 = rng.uniform(-1, 1, 2)
        B = np.array([[1.0, 0.3], [0.1, 0.9]]) * rng.uniform(0.2, 2.0) + rng.uniform(-0.1, 0.1, (2, 2))
        assert np.linalg.det(B) > 0
        det = np.linalg.det(B)
        xi, U, V, u0, v0 = rng.uniform(-1, 1, 5)
        hb = rng.uniform(1.0, 5.0)
        c = np.zeros((3, K))
        u = np.zeros((2, K))
        unit = math.sqrt(abs(det)) / math.sqrt(2.0)    # coefficient of the constant 1
        c[:, 0] = np.array([xi, U, V]) * unit
        u[:, 0] = np.array([u0, v0]) * unit
        E = dg.volume_integrals(k, c, u, B, hb, g)
        pres = 0.5 * g * xi * ((xi + hb) + hb)
        Ac = np.array([[U, V], [U * u0 + pres, U * v0], [V * u0, V * v0 + pres]])
        want = edge_integrals(k, B, a1, Ac)
        assert np.max(np.abs(E - want)) <= 1e-12 * (1 + np.max(np.abs(want)))
        assert np.max(np.abs(E[:, 0])) <= 1e-13 * (1 + np.max(np.abs(E)))   # constant test function


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_projection_of_constant_depth_divides(k):
    """With xi = 0 the depth is the constant h_b, the weighted mass matrix is
    h_b times the identity (orthonormal basis) and u = q / h_b."""
    rng = np.random.default_rng(20 + k)
    K = dg.K_OF[k]
    B = np.array([[0.7, 0.2], [-0.1, 0.8]])
    c = np.zeros((3, K))
    c[1:] = rng.normal(size=(2, K))
    u = dg.velocity_projection(k, c, B, 2.5)
    assert np.max(np.abs(u - c[1:] / 2.5)) <= 1e-13


@pytest.mark.parametrize("k", [1, 2, 3])
def test_projection_recovers_a_constant_velocity(k):
    """q = H u0 with a linear depth H and a constant velocity u0 lies in P^k,
    so the projection returns exactly u0 (only the constant mode)."""
    rng = np.random.default_rng(30 + k)
    K = dg.K_OF[k]
    B = np.array([[0.9, 0.3], [0.2, 1.1]])
    det = np.linalg.det(B)
    hb = 3.0
    c = np.zeros((3, K))
    c[0, :3] = rng.normal(0.0, 0.2, 3)                  # linear surface elevation
    u0 = np.array([0.7, -0.4])
    unit = math.sqrt(abs(det)) / math.sqrt(2.0)         # coefficient of the constant 1
    H = c[0].copy()
    H[0] += hb * unit
    c[1] = u0[0] * H                                    # U = u0 H, V = v0 H: in P^1
    c[2] = u0[1] * H
    u = dg.velocity_projection(k, c, B, hb)
    want = np.zeros((2, K))
    want[:, 0] = u0 * unit
    assert np.max(np.abs(u - want)) <= 1e-12
