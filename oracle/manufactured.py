"""The manufactured solution of the paper's convergence test (Sec. 3.1,
randomly perturbed regular mesh of [0, 1000]^2): exact surface elevation and
depth-integrated velocity, the linear bathymetry, and the body force F that
makes them solve the shallow water equations (eq:def_A, eq:def_r with
tau_bf = f_c = 0, which the test does not state), written out by hand with
the chain rule.  Also the L2 projection of a function onto the element basis
and the L2 error of a DG field, both by quadrature on the physical elements.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With theta = pi (x1 + x2 + C_t t) / 600 (x1, x2 the coordinates):
    xi = 2 + y_a - 2 C_a sin theta,  U = 2 y_a + C_a C_t sin theta,
    V = y_a + C_a C_t sin theta,     h_b = 1 + x1 / 1000 + 2 x2 / 1000,
C_a = C_t = 0.2, y_a = 0.3 as in the paper.  The mass equation holds
without a force (d xi/dt + dU/dx1 + dV/dx2 = 0); the momentum force is
    F = dq/dt + div(q q^T / H) + g H grad xi,  H = h_b + xi.
"""
from __future__ import annotations

import math

import numpy as np

from . import dg

C_A, C_T, Y_A = 0.2, 0.2, 0.3
G = 9.81
KAPPA = math.pi / 600.0


def theta(x, y, t):
    return KAPPA * (x + y + C_T * t)


def exact(x, y, t):
    """(xi, U, V) at points (x, y) and time t."""
    s = np.sin(theta(x, y, t))
    return 2.0 + Y_A - 2.0 * C_A * s, 2.0 * Y_A + C_A * C_T * s, Y_A + C_A * C_T * s


def bathymetry(x, y):
    return 1.0 + x / 1000.0 + 2.0 * y / 1000.0


def forcing(x, y, t):
    """(F_U, F_V) of the momentum equations (F_xi = 0)."""
    co = np.cos(theta(x, y, t))
    xi, U, V = exact(x, y, t)
    H = bathymetry(x, y) + xi
    # first derivatives (d/dx1 and d/dx2 of theta are both KAPPA)
    xi_x = xi_y = -2.0 * C_A * KAPPA * co
    U_x = U_y = V_x = V_y = C_A * C_T * KAPPA * co
    U_t = V_t = C_A * C_T * C_T * KAPPA * co
    H_x = 1.0 / 1000.0 + xi_x
    H_y = 2.0 / 1000.0 + xi_y
    d_uu_x = 2.0 * U * U_x / H - U * U * H_x / H ** 2          # d/dx1 (U^2 / H)
    d_uv_y = (U_y * V + U * V_y) / H - U * V * H_y / H ** 2    # d/dx2 (U V / H)
    d_uv_x = (U_x * V + U * V_x) / H - U * V * H_x / H ** 2    # d/dx1 (U V / H)
    d_vv_y = 2.0 * V * V_y / H - V * V * H_y / H ** 2          # d/dx2 (V^2 / H)
    return U_t + d_uu_x + d_uv_y + G * H * xi_x, V_t + d_uv_x + d_vv_y + G * H * xi_y


def element_points(B: np.ndarray, a1: np.ndarray, e: int, n: int = 8):
    """Quadrature points (x, y), weights (physical) and the element's basis
    values (K_max, Q) on element e of a mesh (B (4, ne), a1 (2, ne))."""
    X, Y, Wt = dg.triangle_rule(n)
    Be = np.array([[B[0, e], B[1, e]], [B[2, e], B[3, e]]])
    det = Be[0, 0] * Be[1, 1] - Be[0, 1] * Be[1, 0]
    x = a1[0, e] + Be[0, 0] * X + Be[0, 1] * Y
    y = a1[1, e] + Be[1, 0] * X + Be[1, 1] * Y
    ph = abs(det) ** -0.5 * np.array(dg.basis(X, Y))
    return x, y, Wt * abs(det), ph


def project(k: int, B: np.ndarray, a1: np.ndarray, fn) -> np.ndarray:
    """L2 projection of fn(x, y) -> list of arrays (nf of them) onto P^k of
    every element: coefficients (nf K, ne), field-major (the element basis
    is orthonormal, so a coefficient is the integral of fn times phi_ep)."""
    K = dg.K_OF[k]
    ne = B.shape[1]
    rows = None
    for e in range(ne):
        x, y, w, ph = element_points(B, a1, e)
        vals = fn(x, y)
        if rows is None:
            rows = np.zeros((len(vals) * K, ne))
        for j, v in enumerate(vals):
            rows[j * K:(j + 1) * K, e] = (ph[:K] * (w * v)).sum(axis=1)
    return rows


def l2_errors(k: int, B: np.ndarray, a1: np.ndarray, c: np.ndarray, fn) -> np.ndarray:
    """L2 norms over the mesh of (DG field - fn) for each of the nf fields of
    c (nf K, ne)."""
    K = dg.K_OF[k]
    nf = c.shape[0] // K
    acc = np.zeros(nf)
    for e in range(B.shape[1]):
        x, y, w, ph = element_points(B, a1, e)
        vals = fn(x, y)
        for j in range(nf):
            d = c[j * K:(j + 1) * K, e] @ ph[:K] - vals[j]
            acc[j] += np.sum(w * d * d)
    return np.sqrt(acc)


def velocity(x, y, t):
    """Exact (u, v) = q / H."""
    xi, U, V = exact(x, y, t)
    H = bathymetry(x, y) + xi
    return U / H, V / H


def stage_data(k: int, B: np.ndarray, a1: np.ndarray, be: np.ndarray, t: float):
    """Body force (3K, ne) and exterior states of the boundary edges at time
    t: cb (3K, nb) and ub (2K, nb), the projections of the exact (xi, U, V)
    and (u, v) onto P^k of the element that owns each boundary edge."""
    K = dg.K_OF[k]
    F = project(k, B, a1, lambda x, y: (0.0 * x,) + tuple(forcing(x, y, t)))
    own = np.unique(be)
    cpr = project(k, B[:, own], a1[:, own], lambda x, y: exact(x, y, t))
    upr = project(k, B[:, own], a1[:, own], lambda x, y: velocity(x, y, t))
    pos = {int(e): i for i, e in enumerate(own)}
    idx = np.array([pos[int(e)] for e in be], dtype=np.int64)
    return F, cpr[:, idx], upr[:, idx]
