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
* Flux tensor rows (with H = xi + h_b):
  (U, V), (U u + g xi (H + h_b) / 2, U v), (V u, V v + g xi (H + h_b) / 2);
  c = (xi, U, V) and u = (u, v) are DG fields with K(k) coefficients each,
  and the bathymetry h_b is one of order max(k, 1) (KB(k) = 3, 3, 6, 10
  coefficients): the paper's algebraic form, which takes h_b out of the
  integral, is the case of a field with only the constant mode, and a
  linear h_b (the convergence test of Sec. 3.1) is exact for every k.  At
  k = 0 a piecewise-constant h_b would not do: the pressure flux jumps with
  h_b across the edges while g xi grad h_b vanishes inside the elements, an
  O(1) force wherever xi != 0.
* Output E[j, p] = (A~, grad(phi_ep e_j))_{Omega_e}, j = 1, 2, 3.
* The semi-discrete system (the paper's variational_disc_1 with the source
  r(c) of eq:def_r and a body force): with the orthonormal element basis the
  mass matrix is the identity and
      dc/dt = E - S + R + F,
  S the edge terms, R = (r(c), phi_ep e_j).  Time stepping: the three-stage
  strong-stability-preserving Runge-Kutta method of Shu and Osher (the
  paper names no integrator).
"""
from __future__ import annotations

import math

import numpy as np

K_OF = {0: 1, 1: 3, 2: 6, 3: 10}
KB_OF = {0: 3, 1: 3, 2: 6, 3: 10}     # coefficients of the bathymetry


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


def constant_field(k: int, value: float, B: np.ndarray) -> np.ndarray:
    """Coefficients (K,) of the constant `value` on the element with map B:
    value / phi_e1 = value sqrt(|det B| / 2) on the constant mode."""
    det = B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]
    out = np.zeros(K_OF[k])
    out[0] = value * math.sqrt(abs(det) / 2.0)
    return out


def volume_integrals(k: int, c: np.ndarray, u: np.ndarray, B: np.ndarray, hb: np.ndarray, g: float) -> np.ndarray:
    """E[j, p] for one element: c (3, K) and u (2, K) coefficients, B (2, 2),
    bathymetry coefficients hb (any number of them, up to 10), gravity g.
    Quadrature on the physical element."""
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
    hbv = hb @ (sc * np.array(basis(X, Y))[:len(hb)])
    pres = 0.5 * g * xi * ((xi + hbv) + hbv)
    A = [(U, V), (U * uu + pres, U * vv), (V * uu, V * vv + pres)]
    w = Wt * abs(det)
    E = np.zeros((3, K))
    for j in range(3):
        E[j] = (dx1 * (w * A[j][0])).sum(axis=1) + (dx2 * (w * A[j][1])).sum(axis=1)
    return E


def velocity_projection(k: int, c: np.ndarray, B: np.ndarray, hb: np.ndarray) -> np.ndarray:
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
    H = c[0] @ ph + hb @ (abs(det) ** -0.5 * np.array(basis(X, Y))[:len(hb)])
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
    K = coef.shape[1]              # the fields' own number of coefficients
    det = B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]
    ref = np.linalg.solve(B, rel.T)
    ph = abs(det) ** -0.5 * np.array(basis(ref[0], ref[1]))[:K]
    return coef @ ph


def mean_state(k: int, c: np.ndarray, u: np.ndarray, B: np.ndarray, hb: np.ndarray):
    """Element means of the velocity and of the depth: the constant mode's
    coefficient times the value of phi_e1, sqrt(2 / |det B_e|)."""
    det = B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]
    v1 = math.sqrt(2.0 / abs(det))
    return u[:, 0] * v1, (c[0, 0] + hb[0]) * v1


def flux_tensor(xi, U, V, uu, vv, hbv, g):
    """Rows of the flux tensor from point values (hbv: the bathymetry)."""
    pres = 0.5 * g * xi * ((xi + hbv) + hbv)
    return [(U, V), (U * uu + pres, U * vv), (V * uu, V * vv + pres)]


class Ghost:
    """A prescribed exterior state on a domain-boundary edge (Dirichlet
    data): coefficients cb (3, K) and ub (2, K) of polynomials in the basis
    of the element that owns the edge, whose traces on the edge are the
    exterior values; the exterior bathymetry is the element's own."""

    def __init__(self, cb: np.ndarray, ub: np.ndarray):
        self.cb, self.ub = cb, ub


def edge_integrals_lf(k, own, nbrs, g):
    """Interior-edge terms of one element: for every local edge q with a
    neighbour, int_E F_j phi_ep ds with the Lax-Friedrichs flux
    F = (A(c-, u-) n + A(c+, u+) n) / 2 + lambda_E (c- - c+) / 2, lambda_E
    = max over both sides of |u_mean . n| + sqrt(g H_mean) (constant on the
    edge), n the unit outward normal.  own = (c, u, B, a1, hb); nbrs[q] =
    the neighbour's (c, u, B, a1, hb), a Ghost (prescribed exterior state;
    its mean state enters lambda_E like a neighbour's), or None (no term).
    Gauss rule on the physical edge.  Returns (3, K)."""
    K = K_OF[k]
    c, u, B, a1, hb = own
    V = element_vertices(B, np.zeros(2))            # relative to a1
    t, w = np.polynomial.legendre.leggauss(8)
    s = (t + 1.0) / 2.0
    out = np.zeros((3, K))
    for q in range(3):
        if nbrs[q] is None:
            continue
        if isinstance(nbrs[q], Ghost):      # exterior polynomials on this element
            cn, un, Bn, a1n, hbn = nbrs[q].cb, nbrs[q].ub, B, a1, hb
        else:
            cn, un, Bn, a1n, hbn = nbrs[q]
        p0, p1 = V[q], V[(q + 1) % 3]
        d = p1 - p0
        L = math.hypot(d[0], d[1])
        n = np.array([d[1], -d[0]]) / L
        pts = p0[None, :] + s[:, None] * d[None, :]
        fm = np.vstack([eval_fields(k, np.vstack([c, u]), B, pts), eval_fields(k, hb[None, :], B, pts)])
        fp = np.vstack([eval_fields(k, np.vstack([cn, un]), Bn, (a1 - a1n)[None, :] + pts),
                        eval_fields(k, hbn[None, :], Bn, (a1 - a1n)[None, :] + pts)])
        um, Hm = mean_state(k, c, u, B, hb)
        up, Hp = mean_state(k, cn, un, Bn, hbn)
        lam = max(abs(um @ n) + math.sqrt(g * Hm), abs(up @ n) + math.sqrt(g * Hp))
        Am = flux_tensor(fm[0], fm[1], fm[2], fm[3], fm[4], fm[5], g)
        Ap = flux_tensor(fp[0], fp[1], fp[2], fp[3], fp[4], fp[5], g)
        ph = eval_fields(k, np.eye(K), B, pts)              # the element's basis at the points
        for j in range(3):
            F = 0.5 * ((Am[j][0] * n[0] + Am[j][1] * n[1]) + (Ap[j][0] * n[0] + Ap[j][1] * n[1])) \
                + 0.5 * lam * (fm[j] - fp[j])
            out[j] += (ph * (F * w / 2.0 * L)).sum(axis=1)
    return out


# ------------------------------------------------ source terms, the system
def source_integrals(k: int, c: np.ndarray, B: np.ndarray, hb: np.ndarray, g: float, tau: float,
                     fc: float) -> np.ndarray:
    """R[j, p] = (r(c), phi_ep e_j) for one element with the paper's source
    (eq:def_r without the body force): r = (0, -tau U + fc V + g xi dh_b/dx,
    -tau V - fc U + g xi dh_b/dy), tau and fc constants.  Quadrature on the
    physical element; returns (3, K)."""
    K = K_OF[k]
    X, Y, Wt = triangle_rule()
    det = B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]
    sc = abs(det) ** -0.5
    ph = sc * np.array(basis(X, Y))[:K]
    gx, gy = basis_grad(X, Y)
    Binv = np.linalg.inv(B)
    dx1 = sc * (Binv[0, 0] * np.array(gx)[:K] + Binv[1, 0] * np.array(gy)[:K])
    dx2 = sc * (Binv[0, 1] * np.array(gx)[:K] + Binv[1, 1] * np.array(gy)[:K])
    xi, U, V = (c[j] @ ph for j in range(3))
    nb_ = len(hb)
    bx = sc * (Binv[0, 0] * np.array(gx)[:nb_] + Binv[1, 0] * np.array(gy)[:nb_])
    by = sc * (Binv[0, 1] * np.array(gx)[:nb_] + Binv[1, 1] * np.array(gy)[:nb_])
    hx, hy = hb @ bx, hb @ by
    r = [0.0 * xi, -tau * U + fc * V + g * xi * hx, -tau * V - fc * U + g * xi * hy]
    w = Wt * abs(det)
    return np.array([(ph * (w * r[j])).sum(axis=1) for j in range(3)])


def mesh_rhs(k: int, B: np.ndarray, a1: np.ndarray, nbr: np.ndarray, c: np.ndarray, u: np.ndarray,
             hb: np.ndarray, g: float, tau: float = 0.0, fc: float = 0.0, F=None, cb=None, ub=None) -> np.ndarray:
    """dc/dt = E - S + R + F of the semi-discrete system on a mesh: B (4, ne)
    rows B11, B12, B21, B22; a1 (2, ne) first vertices; nbr (3, ne) the
    element across each local edge, -1 for no term and -2 - b for the
    prescribed exterior state b (cb (3K, nb), ub (2K, nb)); c (3K, ne), u
    (2K, ne), hb (KB, ne) coefficients; F (3K, ne) or None.  Returns (3K, ne)."""
    K = K_OF[k]
    ne = B.shape[1]

    def state(e):
        Be = np.array([[B[0, e], B[1, e]], [B[2, e], B[3, e]]])
        return c[:, e].reshape(3, K), u[:, e].reshape(2, K), Be, a1[:, e], hb[:, e]

    out = np.zeros((3 * K, ne))
    for e in range(ne):
        own = state(e)
        nbrs = []
        for q in range(3):
            f = int(nbr[q, e])
            if f >= 0:
                nbrs.append(state(f))
            elif f <= -2:
                b = -2 - f
                nbrs.append(Ghost(cb[:, b].reshape(3, K), ub[:, b].reshape(2, K)))
            else:
                nbrs.append(None)
        E = volume_integrals(k, own[0], own[1], own[2], own[4], g)
        S = edge_integrals_lf(k, own, nbrs, g)
        R = source_integrals(k, own[0], own[2], own[4], g, tau, fc)
        out[:, e] = (E - S + R).reshape(-1)
    if F is not None:
        out += F
    return out


def mesh_velocity(k: int, B: np.ndarray, c: np.ndarray, hb: np.ndarray) -> np.ndarray:
    """The velocity projection on every element, (2K, ne)."""
    K = K_OF[k]
    out = np.zeros((2 * K, B.shape[1]))
    for e in range(B.shape[1]):
        Be = np.array([[B[0, e], B[1, e]], [B[2, e], B[3, e]]])
        out[:, e] = velocity_projection(k, c[:, e].reshape(3, K), Be, hb[:, e]).reshape(-1)
    return out


# stage times (fractions of dt) and the convex weights of the three stages
SSP3_TIMES = (0.0, 1.0, 0.5)


def ssp_rk3_step(k: int, B, a1, nbr, c, hb, dt: float, g: float, tau: float = 0.0, fc: float = 0.0,
                 F3=None, cb3=None, ub3=None):
    """One step of the three-stage SSP Runge-Kutta method (Shu and Osher):
        c1 = c + dt L(c),  c2 = 3/4 c + 1/4 (c1 + dt L(c1)),
        c3 = 1/3 c + 2/3 (c2 + dt L(c2)),
    L the semi-discrete right-hand side with the velocity projected from the
    stage state first; F3[s], cb3[s], ub3[s] the body force and exterior
    states at the stage times t + SSP3_TIMES[s] dt (None: none)."""
    pick = lambda a, s: None if a is None else a[s]
    weights = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))
    y = c
    for s_ in range(3):
        u = mesh_velocity(k, B, y, hb)
        L = mesh_rhs(k, B, a1, nbr, y, u, hb, g, tau, fc, pick(F3, s_), pick(cb3, s_), pick(ub3, s_))
        a, b = weights[s_]
        y = a * c + b * (y + dt * L)
    return y
