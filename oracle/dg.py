"""Element integrals of the quadrature-free DG discretisation of the shallow
water equations (the paper's Sec. 2.2: the volume terms
(A~(c, u), grad(phi e_j)) over one triangle, equations mass_basis and
momentum_basis_u), evaluated here by their plain definition: numerical
quadrature on the physical triangle of the pointwise flux tensor times the
gradient of the test function.  The GPU library evaluates the same numbers
through the algebraic (quadrature-free) form with precomputed reference
integrals; the two routes share nothing but the basis polynomials, which the
paper lists.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (readings):
* Reference triangle {(0,0), (1,0), (0,1)}; F_e(x^) = B_e x^ + a_e1 with
  B_e = [a_e2 - a_e1, a_e3 - a_e1] (columns), det B_e != 0 (either
  orientation; the physical integrals are taken as they are).
* The element basis is phi_ei = |det B_e|^(-1/2) phi^_i o F_e^-1, orthonormal
  on the element: the factors 1/|det B_e| and 1/|det B_e|^(3/2) of the
  paper's algebraic forms imply this scaling.
* Flux tensor rows (with H = xi + h_b, h_b constant on the element):
  (U, V), (U u + g xi (H + h_b) / 2, U v), (V u, V v + g xi (H + h_b) / 2);
  c = (xi, U, V) and u = (u, v) are DG fields with K(k) coefficients each.
* Output E[j, p] = (A~, grad(phi_ep e_j))_{Omega_e}, j = 1, 2, 3.
"""
from __future__ import annotations

import math

import numpy as np

K_OF = {0: 1, 1: 3, 2: 6, 3: 10}


def basis(x, y):
    """The ten orthonormal polynomials on the reference triangle listed in the
    paper (P^0: 1, P^1: 2-3, P^2: 4-6, P^3: 7-10), evaluated at (x, y)."""
    s = math.sqrt
    return [
        s(2.0) + 0.0 * x,
        2.0 - 6.0 * x,
        s(12.0) * (1.0 - x - 2.0 * y),
        s(6.0) * (1.0 - 8.0 * x + 10.0 * x ** 2),
        s(3.0) * (-1.0 - 4.0 * x + 5.0 * x ** 2 + 12.0 * y - 15.0 * y ** 2),
        s(45.0) * (1.0 - 4.0 * x + 3.0 * x ** 2 - 4.0 * y + 8.0 * x * y + 3.0 * y ** 2),
        s(8.0) * (-1.0 + 15.0 * x - 45.0 * x ** 2 + 35.0 * x ** 3),
        s(24.0) * (-1.0 + 13.0 * x - 33.0 * x ** 2 + 21.0 * x ** 3 + 2.0 * y - 24.0 * x * y + 42.0 * x ** 2 * y),
        s(40.0) * (-1.0 + 9.0 * x - 15.0 * x ** 2 + 7.0 * x ** 3 + 6.0 * y - 48.0 * x * y + 42.0 * x ** 2 * y
                   - 6.0 * y ** 2 + 42.0 * x * y ** 2),
        s(56.0) * (-1.0 + 3.0 * x - 3.0 * x ** 2 + x ** 3 + 12.0 * y - 24.0 * x * y + 12.0 * x ** 2 * y
                   - 30.0 * y ** 2 + 30.0 * x * y ** 2 + 20.0 * y ** 3),
    ]


def basis_grad(x, y):
    """Reference gradients (d/dx^1, d/dx^2) of the ten polynomials, written
    out by differentiating each term."""
    s = math.sqrt
    z = 0.0 * x
    gx = [
        z,
        -6.0 + z,
        -s(12.0) + z,
        s(6.0) * (-8.0 + 20.0 * x),
        s(3.0) * (-4.0 + 10.0 * x),
        s(45.0) * (-4.0 + 6.0 * x + 8.0 * y),
        s(8.0) * (15.0 - 90.0 * x + 105.0 * x ** 2),
        s(24.0) * (13.0 - 66.0 * x + 63.0 * x ** 2 - 24.0 * y + 84.0 * x * y),
        s(40.0) * (9.0 - 30.0 * x + 21.0 * x ** 2 - 48.0 * y + 84.0 * x * y + 42.0 * y ** 2),
        s(56.0) * (3.0 - 6.0 * x + 3.0 * x ** 2 - 24.0 * y + 24.0 * x * y + 30.0 * y ** 2),
    ]
    gy = [
        z,
        z,
        -2.0 * s(12.0) + z,
        z,
        s(3.0) * (12.0 - 30.0 * y),
        s(45.0) * (-4.0 + 8.0 * x + 6.0 * y),
        z,
        s(24.0) * (2.0 - 24.0 * x + 42.0 * x ** 2),
        s(40.0) * (6.0 - 48.0 * x + 42.0 * x ** 2 - 12.0 * y + 84.0 * x * y),
        s(56.0) * (12.0 - 24.0 * x + 12.0 * x ** 2 - 60.0 * y + 60.0 * x * y + 60.0 * y ** 2),
    ]
    return gx, gy


def triangle_rule(n: int = 7):
    """Collapsed (Duffy) tensor Gauss-Legendre rule on the reference triangle:
    x = a, y = (1 - a) b with a, b Gauss points on [0, 1] and weight
    w_a w_b (1 - a); exact for polynomials of degree <= 2 n - 2."""
    t, w = np.polynomial.legendre.leggauss(n)
    a = (t + 1.0) / 2.0
    wa = w / 2.0
    X, Y, Wt = [], [], []
    for i in range(n):
        for j in range(n):
            X.append(a[i])
            Y.append((1.0 - a[i]) * a[j])
            Wt.append(wa[i] * wa[j] * (1.0 - a[i]))
    return np.array(X), np.array(Y), np.array(Wt)


def volume_integrals(k: int, c: np.ndarray, u: np.ndarray, B: np.ndarray, hb: float, g: float) -> np.ndarray:
    """E[j, p] for one element: c (3, K) and u (2, K) coefficients, B (2, 2),
    bathymetry hb, gravity g.  Quadrature on the physical element."""
    K = K_OF[k]
    X, Y, Wt = triangle_rule()
    phi = np.array(basis(X, Y))[:K]                  # (K, Q)
    gx, gy = basis_grad(X, Y)
    gx, gy = np.array(gx)[:K], np.array(gy)[:K]
    det = B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]
    sc = abs(det) ** -0.5
    # physical gradients: grad phi = |det|^-1/2 B^-T grad^ phi^
    Binv = np.linalg.inv(B)
    dx1 = sc * (Binv[0, 0] * gx + Binv[1, 0] * gy)
    dx2 = sc * (Binv[0, 1] * gx + Binv[1, 1] * gy)
    ph = sc * phi
    xi, U, V = (c[j] @ ph for j in range(3))         # field values at the points
    uu, vv = (u[j] @ ph for j in range(2))
    pres = 0.5 * g * xi * ((xi + hb) + hb)
    A = [(U, V), (U * uu + pres, U * vv), (V * uu, V * vv + pres)]
    w = Wt * abs(det)
    E = np.zeros((3, K))
    for j in range(3):
        E[j] = (dx1 * (w * A[j][0])).sum(axis=1) + (dx2 * (w * A[j][1])).sum(axis=1)
    return E


def velocity_projection(k: int, c: np.ndarray, B: np.ndarray, hb: float) -> np.ndarray:
    """The velocity u = (u, v) of one element from (u H, psi) = (q, psi) for
    every test function psi of the element (the paper's variational_disc_2),
    H = xi + h_b, q = (U, V): assemble the H-weighted mass matrix and the
    right-hand sides by quadrature on the physical element and solve.
    Returns the coefficients (2, K)."""
    K = K_OF[k]
    X, Y, Wt = triangle_rule()
    det = B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]
    ph = abs(det) ** -0.5 * np.array(basis(X, Y))[:K]
    w = Wt * abs(det)
    H = c[0] @ ph + hb
    M = (ph * (w * H)) @ ph.T
    rhs = np.stack([(ph * (w * (c[j] @ ph))).sum(axis=1) for j in (1, 2)], axis=1)
    return np.linalg.solve(M, rhs).T


# ------------------------------------------------------------ edge terms
# Local edges of the reference triangle, counter-clockwise: q0 (0,0)->(1,0),
# q1 (1,0)->(0,1), q2 (0,1)->(0,0).
REF_VERTS = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])


def element_vertices(B: np.ndarray, a1: np.ndarray):
    return [a1, a1 + B[:, 0], a1 + B[:, 1]]


def eval_fields(k: int, coef: np.ndarray, B: np.ndarray, rel: np.ndarray) -> np.ndarray:
    """Values of the fields with coefficients coef (nf, K) on the element
    with map B at the points rel (P, 2), given relative to the element's
    first vertex (relative coordinates keep small elements accurate)."""
    K = K_OF[k]
    det = B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]
    ref = np.linalg.solve(B, rel.T)
    ph = abs(det) ** -0.5 * np.array(basis(ref[0], ref[1]))[:K]
    return coef @ ph


def mean_state(k: int, c: np.ndarray, u: np.ndarray, B: np.ndarray, hb: float):
    """Element means of the velocity and of the depth: the constant mode's
    coefficient times the value of phi_e1, sqrt(2 / |det B_e|)."""
    det = B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]
    v1 = math.sqrt(2.0 / abs(det))
    return u[:, 0] * v1, c[0, 0] * v1 + hb


def flux_tensor(xi, U, V, uu, vv, hb, g):
    pres = 0.5 * g * xi * ((xi + hb) + hb)
    return [(U, V), (U * uu + pres, U * vv), (V * uu, V * vv + pres)]


def edge_integrals_lf(k, own, nbrs, g):
    """Interior-edge terms of one element: for every local edge q with a
    neighbour, int_E F_j phi_ep ds with the Lax-Friedrichs flux
    F = (A(c-, u-) n + A(c+, u+) n) / 2 + lambda_E (c- - c+) / 2, lambda_E
    = max over both sides of |u_mean . n| + sqrt(g H_mean) (constant on the
    edge), n the unit outward normal.  own = (c, u, B, a1, hb); nbrs[q] =
    the neighbour's (c, u, B, a1, hb) or None on the boundary.  Gauss rule
    on the physical edge.  Returns (3, K)."""
    K = K_OF[k]
    c, u, B, a1, hb = own
    V = element_vertices(B, np.zeros(2))            # relative to a1
    t, w = np.polynomial.legendre.leggauss(8)
    s = (t + 1.0) / 2.0
    out = np.zeros((3, K))
    for q in range(3):
        if nbrs[q] is None:
            continue
        cn, un, Bn, a1n, hbn = nbrs[q]
        p0, p1 = V[q], V[(q + 1) % 3]
        d = p1 - p0
        L = math.hypot(d[0], d[1])
        n = np.array([d[1], -d[0]]) / L
        pts = p0[None, :] + s[:, None] * d[None, :]
        fm = eval_fields(k, np.vstack([c, u]), B, pts)
        fp = eval_fields(k, np.vstack([cn, un]), Bn, (a1 - a1n)[None, :] + pts)
        um, Hm = mean_state(k, c, u, B, hb)
        up, Hp = mean_state(k, cn, un, Bn, hbn)
        lam = max(abs(um @ n) + math.sqrt(g * Hm), abs(up @ n) + math.sqrt(g * Hp))
        Am = flux_tensor(fm[0], fm[1], fm[2], fm[3], fm[4], hb, g)
        Ap = flux_tensor(fp[0], fp[1], fp[2], fp[3], fp[4], hbn, g)
        ph = eval_fields(k, np.eye(K), B, pts)              # the element's basis at the points
        for j in range(3):
            F = 0.5 * ((Am[j][0] * n[0] + Am[j][1] * n[1]) + (Ap[j][0] * n[0] + Ap[j][1] * n[1])) \
                + 0.5 * lam * (fm[j] - fp[j])
            out[j] += (ph * (F * w / 2.0 * L)).sum(axis=1)
    return out
