"""Cell-centred variable-coefficient diffusion -div(k grad u) = f on [0, 1]^d
with zero Dirichlet walls or homogeneous Neumann walls (zero flux).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Grid: N = 2^L cells per axis (times the coarsest size), h = 1/N, centres
(i + 1/2) h; arrays of shape (N,)*d indexed [z, y, x].  The coefficient is
carried by the faces, as ExaSlang's ``StencilField`` carries per-point stencil
coefficients: for array axis a, ``beta[a]`` has N+1 entries along a (face i
lies between cells i-1 and i; faces 0 and N are walls) and N along the other
axes.

Operator (finite volumes, two-point fluxes):
    (A u)_i = s * (diag_i * u_i - off_i),   s = 1/h^2 = N^2,
    diag_i  = sum over the 2d faces of w_f * beta_f   (w_f = 2 on a wall),
    off_i   = sum over interior faces of beta_f * u_neighbour.
A Dirichlet wall face uses the mirror ghost u_g = -u_i (zero value on the
wall), which is what the weight 2 and the missing off-diagonal term express.
A Neumann wall face uses the even ghost u_g = u_i: its flux vanishes, so it
has weight 0 and again no off-diagonal term; the operator then annihilates
constants and the problem is solvable for right-hand sides of zero mean
(a singular compatible system; the solution is fixed by zero mean).  Face
sums run in the order x-, x+, y-, y+, z-, z+.  Functions taking ``bc`` accept
"dirichlet" (default) or "neumann".
"""
from __future__ import annotations

import itertools

import numpy as np


def scale(N: int, dtype) -> np.generic:
    """s = 1/h^2 = N^2, an exact integer."""
    return np.dtype(dtype).type(N * N)


def _sl(d, ax, s):
    out = [slice(None)] * d
    out[ax] = s
    return tuple(out)


def harmonic_faces(k: np.ndarray) -> list[np.ndarray]:
    """Face coefficients from cell values k (FP64):
    interior face: 2 k_a k_b / (k_a + k_b), evaluated as ((2 k_a) k_b) / (k_a + k_b)
    with k_a the lower cell; wall face: k of the adjacent cell.
    Returns [beta_axis0, beta_axis1, ...] in array-axis order."""
    d = k.ndim
    N = k.shape[0]
    out = []
    for ax in range(d):
        shape = list(k.shape)
        shape[ax] = N + 1
        b = np.empty(shape, dtype=np.float64)
        ka = k[_sl(d, ax, slice(0, N - 1))]
        kb = k[_sl(d, ax, slice(1, N))]
        b[_sl(d, ax, slice(1, N))] = ((2.0 * ka) * kb) / (ka + kb)
        b[_sl(d, ax, 0)] = k[_sl(d, ax, 0)]
        b[_sl(d, ax, N)] = k[_sl(d, ax, N - 1)]
        out.append(b)
    return out


def coarsen_faces(beta: list[np.ndarray]) -> list[np.ndarray]:
    """Coarse face coefficient = mean of the 2^(d-1) fine faces that tile the
    coarse face: coarse face I along axis a is fine face 2I along a, and the
    fine index pairs (2J, 2J+1) along every other axis.  The sum runs in
    itertools.product order over the other axes, then is scaled by 1/2^(d-1)."""
    d = beta[0].ndim
    out = []
    for ax in range(d):
        b = beta[ax]
        N = b.shape[(ax + 1) % d]          # cells along another axis
        Nc = N // 2
        others = [a for a in range(d) if a != ax]
        acc = None
        for o in itertools.product((0, 1), repeat=d - 1):
            sl = [slice(None)] * d
            sl[ax] = slice(0, b.shape[ax], 2)
            for a, off in zip(others, o):
                sl[a] = slice(off, 2 * Nc, 2)
            term = b[tuple(sl)]
            acc = term.copy() if acc is None else acc + term
        out.append(acc * (1.0 / 2 ** (d - 1)))
    return out


def _face_terms(u: np.ndarray, beta: list[np.ndarray]):
    """Yield, per face in the order x-, x+, y-, y+, z-, z+:
    (beta_f over cells, wall mask over cells, neighbour values with 0 at walls)."""
    d = u.ndim
    N = u.shape[0]
    for ax in reversed(range(d)):
        b = beta[ax]
        for side in (-1, 1):
            if side < 0:
                bf = b[_sl(d, ax, slice(0, N))]
                wall = np.zeros(u.shape, dtype=bool)
                wall[_sl(d, ax, 0)] = True
                nb = np.zeros_like(u)
                nb[_sl(d, ax, slice(1, N))] = u[_sl(d, ax, slice(0, N - 1))]
            else:
                bf = b[_sl(d, ax, slice(1, N + 1))]
                wall = np.zeros(u.shape, dtype=bool)
                wall[_sl(d, ax, N - 1)] = True
                nb = np.zeros_like(u)
                nb[_sl(d, ax, slice(0, N - 1))] = u[_sl(d, ax, slice(1, N))]
            yield bf, wall, nb


WALL_WEIGHT = {"dirichlet": 2, "neumann": 0}


def diagonal(beta: list[np.ndarray], shape, dtype, bc: str = "dirichlet") -> np.ndarray:
    """diag_i = sum over faces of w_f beta_f, w_f = 1 inside and on walls 2
    (Dirichlet) or 0 (Neumann)."""
    t = np.dtype(dtype).type
    w = t(WALL_WEIGHT[bc])
    dummy = np.zeros(shape, dtype=dtype)
    acc = None
    for bf, wall, _ in _face_terms(dummy, beta):
        term = np.where(wall, w * bf, bf).astype(dtype)
        acc = term if acc is None else acc + term
    return acc


def off_sum(u: np.ndarray, beta: list[np.ndarray]) -> np.ndarray:
    """off_i = sum over faces of beta_f * u_neighbour (the neighbour is 0 at walls)."""
    acc = None
    for bf, _, nb in _face_terms(u, beta):
        term = bf * nb
        acc = term if acc is None else acc + term
    return acc


def apply_A(u: np.ndarray, beta: list[np.ndarray], bc: str = "dirichlet") -> np.ndarray:
    s = scale(u.shape[0], u.dtype)
    return (diagonal(beta, u.shape, u.dtype, bc) * u - off_sum(u, beta)) * s


def residual(u: np.ndarray, f: np.ndarray, beta: list[np.ndarray], bc: str = "dirichlet") -> np.ndarray:
    """r = f - (diag u - off) s."""
    s = scale(u.shape[0], u.dtype)
    return f - (diagonal(beta, u.shape, u.dtype, bc) * u - off_sum(u, beta)) * s


def jacobi(u, f, beta, omega, bc: str = "dirichlet"):
    """u' = u + (omega r) / (diag s)."""
    t = u.dtype.type
    s = scale(u.shape[0], u.dtype)
    r = residual(u, f, beta, bc)
    return u + (t(omega) * r) / (diagonal(beta, u.shape, u.dtype, bc) * s)


def colour_mask(N: int, d: int, colour: int) -> np.ndarray:
    return (np.indices((N,) * d).sum(axis=0) % 2) == colour


def gs_colour(u, f, beta, colour, bc: str = "dirichlet") -> None:
    """In place: u_i <- (f_i / s + off_i) / diag_i on cells of one colour."""
    s = scale(u.shape[0], u.dtype)
    new = (f / s + off_sum(u, beta)) / diagonal(beta, u.shape, u.dtype, bc)
    m = colour_mask(u.shape[0], u.ndim, colour)
    u[m] = new[m]


def rbgs(u, f, beta, order=(0, 1), bc: str = "dirichlet"):
    out = u.copy()
    for c in order:
        gs_colour(out, f, beta, c, bc)
    return out


def project_mean(a: np.ndarray) -> np.ndarray:
    """a minus its arithmetic mean over all cells: the component of a
    orthogonal to the constants, the null space of the Neumann operator."""
    return a - a.dtype.type(np.sum(a, dtype=np.float64) / a.size)


def restrict_mean(r: np.ndarray) -> np.ndarray:
    """f_c[I] = (sum over the 2^d children 2I + o, o in {0,1}^d) / 2^d,
    summed in itertools.product order."""
    d = r.ndim
    N = r.shape[0]
    acc = None
    for o in itertools.product((0, 1), repeat=d):
        term = r[tuple(slice(k, N, 2) for k in o)]
        acc = term.copy() if acc is None else acc + term
    return acc * r.dtype.type(1.0 / 2 ** d)


def prolong_trilinear(ec: np.ndarray, bc: str = "dirichlet") -> np.ndarray:
    """Cell-centred (bi/tri)linear interpolation, the tensor product of the 1-D
    rule fine(2I) = 3/4 e[I] + 1/4 e[I-1], fine(2I+1) = 3/4 e[I] + 1/4 e[I+1]
    with ghosts beyond the walls: e[-1] = -e[0], e[Nc] = -e[Nc-1] (Dirichlet,
    odd mirror) or e[-1] = e[0], e[Nc] = e[Nc-1] (Neumann, even mirror);
    applied along x first, then y, then z.  In 3-D the weights are 27, 9, 3, 1
    over 64."""
    d = ec.ndim
    t = ec.dtype.type
    a, b = t(0.75), t(0.25)
    sg = t(-1) if bc == "dirichlet" else t(1)
    e = ec
    for ax in reversed(range(d)):
        Nc = e.shape[ax]
        lo = np.concatenate([sg * e[_sl(d, ax, slice(0, 1))], e[_sl(d, ax, slice(0, Nc - 1))]], axis=ax)
        hi = np.concatenate([e[_sl(d, ax, slice(1, Nc))], sg * e[_sl(d, ax, slice(Nc - 1, Nc))]], axis=ax)
        shape = list(e.shape)
        shape[ax] = 2 * Nc
        out = np.empty(shape, dtype=e.dtype)
        out[_sl(d, ax, slice(0, 2 * Nc, 2))] = a * e + b * lo
        out[_sl(d, ax, slice(1, 2 * Nc, 2))] = a * e + b * hi
        e = out
    return e


def correct(u, ec, bc: str = "dirichlet"):
    return u + prolong_trilinear(ec, bc)


def dense_matrix(beta: list[np.ndarray], N: int, d: int, bc: str = "dirichlet") -> np.ndarray:
    """Dense FP64 A over the N^d cells (C order), column by column from unit vectors."""
    m = N ** d
    A = np.zeros((m, m))
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        A[:, j] = apply_A(e.reshape((N,) * d), beta, bc).reshape(-1)
    return A
