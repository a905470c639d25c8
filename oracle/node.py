"""Node-centred Poisson operators on [0, 1]^d with zero Dirichlet boundary.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid: n = 2^L + 1 nodes per axis, h = 1/(n-1), x_i = i h; arrays have shape
(n,)*d indexed [z, y, x] (3-D) or [y, x] (2-D).  Boundary nodes are not
unknowns; their entries are whatever the array holds (zero in every solve,
the paper's Sec. 2.1 assumes Dirichlet data) and are never written here.

Every function is dtype-generic: float64 arrays give the FP64 method, float32
arrays give the single-precision inner cycle with each operation rounded to
float32.
"""
from __future__ import annotations

import itertools

import numpy as np


def interior(d: int):
    return (slice(1, -1),) * d


def scale(n: int, dtype) -> np.generic:
    """s = 1/h^2 = (n-1)^2, an exact integer (a power of two for n = 2^L + 1)."""
    return np.dtype(dtype).type((n - 1) ** 2)


def _shift(u: np.ndarray, ax: int, sh: int) -> np.ndarray:
    """View of u at interior index + sh along array axis ax."""
    n = u.shape[ax]
    sl = list(interior(u.ndim))
    sl[ax] = slice(1 + sh, n - 1 + sh)
    return u[tuple(sl)]


def neighbour_sum(u: np.ndarray) -> np.ndarray:
    """Sum of the 2d axis neighbours at interior nodes, accumulated in the
    order x-, x+, y-, y+, z-, z+ (x is the last array axis)."""
    d = u.ndim
    acc = None
    for ax in reversed(range(d)):
        for sh in (-1, 1):
            t = _shift(u, ax, sh)
            acc = t.copy() if acc is None else acc + t
    return acc


def apply_A(u: np.ndarray) -> np.ndarray:
    """(A u)_i = (2d u_i - sum of neighbours) * s at interior nodes; 0 on the
    boundary.  This is the 5-point (2-D) / 7-point (3-D) stencil."""
    d = u.ndim
    s = scale(u.shape[0], u.dtype)
    two_d = u.dtype.type(2 * d)
    out = np.zeros_like(u)
    out[interior(d)] = (two_d * u[interior(d)] - neighbour_sum(u)) * s
    return out


def residual(u: np.ndarray, f: np.ndarray) -> np.ndarray:
    """r = f - A u on interior nodes, 0 on the boundary."""
    d = u.ndim
    s = scale(u.shape[0], u.dtype)
    two_d = u.dtype.type(2 * d)
    r = np.zeros_like(u)
    c = interior(d)
    r[c] = f[c] - (two_d * u[c] - neighbour_sum(u)) * s
    return r


def jacobi(u: np.ndarray, f: np.ndarray, omega) -> np.ndarray:
    """One damped-Jacobi sweep, all interior nodes at once:
    u' = u + (omega * r) / (2d s),  r = f - A u."""
    d = u.ndim
    t = u.dtype.type
    s = scale(u.shape[0], u.dtype)
    diag = t(2 * d) * s
    r = residual(u, f)
    out = u.copy()
    c = interior(d)
    out[c] = u[c] + (t(omega) * r[c]) / diag
    return out


def colour_mask(n: int, d: int, colour: int) -> np.ndarray:
    """Boolean mask over the interior nodes: True where the index sum
    (counted with boundary index 0) has parity ``colour`` (0 = red, 1 = black)."""
    idx = np.indices((n - 2,) * d).sum(axis=0) + d   # interior index = k + 1 per axis
    return (idx % 2) == colour


def gs_colour(u: np.ndarray, f: np.ndarray, colour: int) -> None:
    """Gauss-Seidel update of all nodes of one colour, in place:
    u_i <- (f_i / s + sum of neighbours) / (2d).

    All neighbours of a node have the other colour, so updating every node
    of one colour from the current array at once is exactly the sequential
    colour sweep."""
    d = u.ndim
    t = u.dtype.type
    s = scale(u.shape[0], u.dtype)
    c = interior(d)
    new = (f[c] / s + neighbour_sum(u)) / t(2 * d)
    m = colour_mask(u.shape[0], d, colour)
    view = u[c]
    view[m] = new[m]


def rbgs(u: np.ndarray, f: np.ndarray, order=(0, 1)) -> np.ndarray:
    """One red-black Gauss-Seidel sweep (red = even index sum first)."""
    out = u.copy()
    for colour in order:
        gs_colour(out, f, colour)
    return out


def restrict_fw(r: np.ndarray) -> np.ndarray:
    """Full weighting: f_c[I] = sum_{o in {-1,0,1}^d} w_o r[2I + o] at interior
    coarse nodes, w_o = prod_a (2 - |o_a|) / 4^d (the [1 2 1]/4 tensor
    stencil).  Terms are accumulated in itertools.product order over the
    array axes (z offset slowest, x offset fastest).  Coarse boundary = 0."""
    d = r.ndim
    n = r.shape[0]
    nc = (n + 1) // 2
    t = r.dtype.type
    fc = np.zeros((nc,) * d, dtype=r.dtype)
    acc = None
    for o in itertools.product((-1, 0, 1), repeat=d):
        w = t(np.prod([2 - abs(k) for k in o])) / t(4 ** d)
        sl = tuple(slice(2 + k, n - 2 + k, 2) for k in o)
        term = w * r[sl]
        acc = term if acc is None else acc + term
    fc[interior(d)] = acc
    return fc


def prolong_linear(ec: np.ndarray) -> np.ndarray:
    """(Bi/tri)linear interpolation from a coarse node grid (n_c per axis) to
    the fine grid (2 n_c - 1 per axis), as the tensor product of the 1-D
    rule (even fine node = coarse value, odd fine node = half the sum of the
    two coarse neighbours), applied along x first, then y, then z."""
    d = ec.ndim
    t = ec.dtype.type
    half = t(0.5)
    e = ec
    for ax in reversed(range(d)):
        nc = e.shape[ax]
        nf = 2 * nc - 1
        shape = list(e.shape)
        shape[ax] = nf
        out = np.zeros(shape, dtype=e.dtype)
        ev = [slice(None)] * d
        ev[ax] = slice(0, nf, 2)
        out[tuple(ev)] = e
        od = [slice(None)] * d
        od[ax] = slice(1, nf, 2)
        lo = [slice(None)] * d
        lo[ax] = slice(0, nc - 1)
        hi = [slice(None)] * d
        hi[ax] = slice(1, nc)
        out[tuple(od)] = half * (e[tuple(lo)] + e[tuple(hi)])
        e = out
    return e


def correct(u: np.ndarray, ec: np.ndarray) -> np.ndarray:
    """u + P e_c on interior nodes (the boundary of P e_c is zero)."""
    e = prolong_linear(ec)
    out = u.copy()
    c = interior(u.ndim)
    out[c] = u[c] + e[c]
    return out


def dense_matrix(n: int, d: int, dtype=np.float64) -> np.ndarray:
    """Dense A over the (n-2)^d interior unknowns (C order), assembled column
    by column by applying ``apply_A`` to unit vectors."""
    m = (n - 2) ** d
    A = np.zeros((m, m), dtype=dtype)
    c = interior(d)
    for j in range(m):
        unit = np.zeros(m, dtype=dtype)
        unit[j] = 1
        e = np.zeros((n,) * d, dtype=dtype)
        e[c] = unit.reshape((n - 2,) * d)
        A[:, j] = apply_A(e)[c].reshape(-1)
    return A
