"""Galerkin coarse operators for node grids: A_{l+1} = R A_l P with R the
full weighting and P the (bi/tri)linear interpolation of ``node`` (the
Galerkin coarse-grid operator of Trottenberg et al., *Multigrid*), in place of the
rediscretised 5/7-point stencil.  For the constant-coefficient Laplacian
every coarse operator is a constant 3^d-point stencil (9 points in 2-D,
27 in 3-D) over the interior nodes, with zero boundary nodes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A stencil is an array W of shape (3,)*d indexed by offset + 1 along the
array axes [z, y, x] (or [y, x]); (A u)_i = sum_o W[o] u[i + o], summed in
itertools.product order over the offsets (z offset slowest, x fastest),
each term W[o] * u[i + o] rounded before it is added.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import node


def laplacian_stencil(n: int, d: int) -> np.ndarray:
    """The 5-point (2-D) / 7-point (3-D) stencil of ``node`` as a 3^d array:
    2d s at the centre, -s at the 2d axis neighbours, s = (n - 1)^2."""
    s = float((n - 1) ** 2)
    W = np.zeros((3,) * d)
    W[(1,) * d] = 2 * d * s
    for ax in range(d):
        for sh in (0, 2):
            o = [1] * d
            o[ax] = sh
            W[tuple(o)] = -s
    return W


def coarse_stencil(W: np.ndarray) -> np.ndarray:
    """R A P for the constant stencil W: column J of R A P is R (A (P e_J));
    taken for a coarse node far enough from the boundary that no stencil is
    truncated, its entries at J + o are the coarse stencil (R A P is
    symmetric, so columns are rows)."""
    d = W.ndim
    nc = 7
    ec = np.zeros((nc,) * d)
    ec[(3,) * d] = 1.0
    v = node.prolong_linear(ec)
    w = apply(v, W)
    col = node.restrict_fw(w)
    return col[tuple(slice(2, 5) for _ in range(d))].copy()


def apply(u: np.ndarray, W: np.ndarray) -> np.ndarray:
    """A u at interior nodes for the stencil W; 0 on the boundary."""
    d = u.ndim
    n = u.shape[0]
    acc = None
    for o in itertools.product((-1, 0, 1), repeat=d):
        view = u[tuple(slice(1 + k, n - 1 + k) for k in o)]
        term = W[tuple(k + 1 for k in o)] * view
        acc = term if acc is None else acc + term
    out = np.zeros_like(u)
    out[node.interior(d)] = acc
    return out


def residual(u: np.ndarray, f: np.ndarray, W: np.ndarray) -> np.ndarray:
    """r = f - A u on interior nodes, 0 on the boundary."""
    d = u.ndim
    c = node.interior(d)
    r = np.zeros_like(u)
    r[c] = f[c] - apply(u, W)[c]
    return r


def jacobi(u: np.ndarray, f: np.ndarray, W: np.ndarray, omega) -> np.ndarray:
    """One damped-Jacobi sweep: u' = u + (omega r) / W_centre."""
    d = u.ndim
    c = node.interior(d)
    r = residual(u, f, W)
    out = u.copy()
    out[c] = u[c] + (u.dtype.type(omega) * r[c]) / W[(1,) * d]
    return out


def dense_matrix(W: np.ndarray, n: int) -> np.ndarray:
    """Dense A over the (n - 2)^d interior unknowns (C order), column by
    column by applying the stencil to unit vectors."""
    d = W.ndim
    m = (n - 2) ** d
    A = np.zeros((m, m))
    c = node.interior(d)
    for j in range(m):
        e = np.zeros((n,) * d)
        unit = np.zeros(m)
        unit[j] = 1.0
        e[c] = unit.reshape((n - 2,) * d)
        A[:, j] = apply(e, W)[c].reshape(-1)
    return A
