"""Seeded synthetic inputs for the multigrid workloads.

This module only draws and samples inputs: right-hand sides, initial guesses,
coefficient fields and request arrival traces.  It holds none of the solver's
arithmetic (no operator, smoother, transfer or norm) so that both the GPU
library's tests and the CPU oracle can be fed the very same arrays.

Everything is NumPy float64 on the host, C order, x fastest
(``a[z, y, x]`` in 3-D, ``a[y, x]`` in 2-D).  Node grids hold the boundary
nodes (always zero); cell grids hold only cells.

Seeds follow one fixed scheme: 0 for the 2-D initial guess, 1 for the 3-D
Poisson right-hand side, 2 for the variable-coefficient right-hand side,
3 and 4 for the request stream's arrivals and size classes, 1000 + id for
request right-hand sides.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_U0_2D = 0
SEED_F_3D = 1
SEED_F_VARCOEF = 2
SEED_ARRIVALS = 3
SEED_SIZES = 4
SEED_REQUEST_BASE = 1000


def node_coords(n: int) -> np.ndarray:
    """Node positions x_i = i*h, h = 1/(n-1), on [0, 1]."""
    return np.arange(n, dtype=np.float64) / (n - 1)


def cell_coords(N: int) -> np.ndarray:
    """Cell-centre positions (i + 1/2)*h, h = 1/N, on [0, 1]."""
    return (np.arange(N, dtype=np.float64) + 0.5) / N


def interior_uniform(n: int, dim: int, seed: int, lo=-1.0, hi=1.0) -> np.ndarray:
    """Node array of shape (n,)*dim: U[lo, hi] on interior nodes, 0 on the boundary."""
    rng = np.random.default_rng(seed)
    a = np.zeros((n,) * dim, dtype=np.float64)
    a[(slice(1, -1),) * dim] = rng.uniform(lo, hi, size=(n - 2,) * dim)
    return a


def sine_rhs_2d(n: int) -> np.ndarray:
    """f = 2 pi^2 sin(pi x) sin(pi y) sampled at the nodes of an n x n grid
    (boundary samples are zero up to rounding; they are set to exactly 0)."""
    x = node_coords(n)
    s = np.sin(np.pi * x)
    f = 2.0 * np.pi ** 2 * np.outer(s, s)
    f[0, :] = f[-1, :] = f[:, 0] = f[:, -1] = 0.0
    return f


def sine_mode(n: int, dim: int, ks=None) -> np.ndarray:
    """Product over array axes a of sin(ks[a] * pi * x_a) at the nodes; the
    boundary samples are set to exactly 0."""
    ks = ks or (1,) * dim
    x = node_coords(n)
    out = np.ones((n,) * dim)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = n
        out = out * np.sin(ks[ax] * np.pi * x).reshape(shape)
    for ax in range(dim):
        idx = [slice(None)] * dim
        idx[ax] = 0
        out[tuple(idx)] = 0.0
        idx[ax] = -1
        out[tuple(idx)] = 0.0
    return out


def varcoef_k(N: int, dim: int = 3) -> np.ndarray:
    """k = exp(0.5 * prod_a sin(2 pi x_a)) at the N^dim cell centres."""
    x = cell_coords(N)
    s = np.sin(2.0 * np.pi * x)
    prod = np.ones((1,) * dim)
    for ax in range(dim):
        shape = [1] * dim
        shape[ax] = N
        prod = prod * s.reshape(shape)
    return np.exp(0.5 * np.broadcast_to(prod, (N,) * dim))


def normal_zero_mean(N: int, dim: int, seed: int) -> np.ndarray:
    """N(0, 1) samples on N^dim cells, shifted to zero mean."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(size=(N,) * dim)
    return f - f.mean()


# --------------------------------------------------------------------------
# Request stream for the served workload
# --------------------------------------------------------------------------
SERVE_CLASSES = (
    (2, 65), (2, 129), (2, 257), (2, 513), (2, 1025),
    (3, 33), (3, 65), (3, 129),
)


@dataclass(frozen=True)
class Request:
    rid: int
    dim: int
    n: int
    t_arrive: float   # seconds from the start of the stream

    def rhs(self) -> np.ndarray:
        return interior_uniform(self.n, self.dim, SEED_REQUEST_BASE + self.rid)


def request_stream(count: int, rate_per_s: float, classes=SERVE_CLASSES,
                   seed_arrivals: int = SEED_ARRIVALS,
                   seed_sizes: int = SEED_SIZES) -> list[Request]:
    """Poisson arrivals (exponential gaps at ``rate_per_s``) with size classes
    drawn uniformly from ``classes``."""
    ra = np.random.default_rng(seed_arrivals)
    rs = np.random.default_rng(seed_sizes)
    gaps = ra.exponential(1.0 / rate_per_s, size=count) if rate_per_s > 0 else np.zeros(count)
    t = np.cumsum(gaps) - gaps[0] if count else gaps
    cls = rs.integers(0, len(classes), size=count)
    out = []
    for i in range(count):
        d, n = classes[int(cls[i])]
        out.append(Request(i, d, n, float(t[i])))
    return out


def cell_uniform(N: int, dim: int, seed: int, lo=-1.0, hi=1.0) -> np.ndarray:
    """U[lo, hi] samples on N^dim cells."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(N,) * dim)


# ------------------------------------------------ DG element workloads
SEED_DG_MESH = 20
SEED_DG_FIELDS = 21


def _square_index(i, j, nx: int, ny: int, tile: int):
    """Index of square (i, j) in the element numbering: i ny + j, or with
    tile > 0 tile by tile (tiles of tile x tile squares, ordered like the
    squares, and the squares of a tile in that order inside it), which keeps
    most edge neighbours within a few hundred indices."""
    if tile <= 0:
        return i * ny + j
    if nx % tile or ny % tile:
        raise ValueError("tile must divide nx and ny")
    return ((i // tile) * (ny // tile) + j // tile) * tile * tile + (i % tile) * tile + j % tile


def dg_mesh(nx: int, ny: int, seed: int = SEED_DG_MESH, jitter: float = 0.2, with_origin: bool = False,
            length: float = 1.0, tile: int = 0):
    """Affine maps of a split-quad triangulation of the square [0, length]^2
    (the convergence test's domain is [0, 1000]^2): nx x ny
    squares, each cut along one diagonal into two counter-clockwise
    triangles, interior vertices moved by up to `jitter` of a cell width (the
    randomly perturbed regular mesh of the paper's convergence test moves
    them by up to 20 % of the edge length), so that every element has its
    own map.  Returns B (4, 2 nx ny) with rows B11, B12, B21, B22 of
    B_e = [a_e2 - a_e1, a_e3 - a_e1] (and a_e1 (2, 2 nx ny) with_origin).
    Elements: the lower-right triangles (p00, p10, p11) of squares (i, j) at
    i ny + j (or the tiled index of _square_index), then the upper-left ones
    (p00, p11, p01) in the same order."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, length, nx + 1)
    ys = np.linspace(0.0, length, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    d = jitter * min(length / nx, length / ny)
    X[1:-1, 1:-1] += rng.uniform(-d, d, (nx - 1, ny - 1))
    Y[1:-1, 1:-1] += rng.uniform(-d, d, (nx - 1, ny - 1))
    p00 = np.stack([X[:-1, :-1], Y[:-1, :-1]], -1).reshape(-1, 2)
    p10 = np.stack([X[1:, :-1], Y[1:, :-1]], -1).reshape(-1, 2)
    p01 = np.stack([X[:-1, 1:], Y[:-1, 1:]], -1).reshape(-1, 2)
    p11 = np.stack([X[1:, 1:], Y[1:, 1:]], -1).reshape(-1, 2)
    if tile > 0:
        i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
        order = np.empty(nx * ny, dtype=np.int64)
        order[_square_index(i.ravel(), j.ravel(), nx, ny, tile)] = i.ravel() * ny + j.ravel()
        p00, p10, p01, p11 = p00[order], p10[order], p01[order], p11[order]
    # lower-right (p00, p10, p11) and upper-left (p00, p11, p01) triangles
    a1 = np.concatenate([p00, p00])
    a2 = np.concatenate([p10, p11])
    a3 = np.concatenate([p11, p01])
    e2, e3 = a2 - a1, a3 - a1
    B = np.ascontiguousarray(np.stack([e2[:, 0], e3[:, 0], e2[:, 1], e3[:, 1]]))
    return (B, np.ascontiguousarray(a1.T)) if with_origin else B


def dg_mesh_neighbours(nx: int, ny: int, tile: int = 0):
    """Edge neighbours of the elements of dg_mesh(nx, ny, tile=tile):
    nbr[q][e] is the element across local edge q of e (q0: a1->a2, q1:
    a2->a3, q2: a3->a1), -1 on the domain boundary, and nq[q][e] that
    element's local index of the shared edge (int32 arrays (3, 2 nx ny))."""
    half = nx * ny
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    i, j = i.ravel(), j.ravel()

    def sq(a, b):
        return _square_index(a, b, nx, ny, tile)

    lr = sq(i, j)                       # lower-right of square (i, j)
    ul = half + lr                      # upper-left of square (i, j)
    nbr = np.full((3, 2 * half), -1, dtype=np.int32)
    nq = np.full((3, 2 * half), -1, dtype=np.int32)
    # lower-right: q0 bottom -> upper-left of (i, j-1) edge q1; q1 right ->
    # upper-left of (i+1, j) edge q2; q2 diagonal -> upper-left of (i, j) edge q0
    m = j > 0
    nbr[0, lr[m]] = half + sq(i[m], j[m] - 1)
    nq[0, lr[m]] = 1
    m = i < nx - 1
    nbr[1, lr[m]] = half + sq(i[m] + 1, j[m])
    nq[1, lr[m]] = 2
    nbr[2, lr] = ul
    nq[2, lr] = 0
    # upper-left: q0 diagonal -> lower-right of (i, j) edge q2; q1 top ->
    # lower-right of (i, j+1) edge q0; q2 left -> lower-right of (i-1, j) edge q1
    nbr[0, ul] = lr
    nq[0, ul] = 2
    m = j < ny - 1
    nbr[1, ul[m]] = sq(i[m], j[m] + 1)
    nq[1, ul[m]] = 0
    m = i > 0
    nbr[2, ul[m]] = sq(i[m] - 1, j[m])
    nq[2, ul[m]] = 1
    return nbr, nq


def dg_fields(K: int, B: np.ndarray, seed: int = SEED_DG_FIELDS):
    """Coefficients of (xi, U, V), (u, v) and the bathymetry h_b, (3K, ne),
    (2K, ne) and (KB, ne) (KB = max(K, 3): the bathymetry is at least
    linear), for the elements with maps B (4, ne).  Physical
    values: xi ~ N(0, 0.1) (so that the depth xi + h_b stays positive), U,
    V, u, v ~ N(0, 1) for the element mean, a tenth of that for each higher
    mode; h_b with a mean U[1, 5] and higher modes N(0, 0.02); a coefficient
    is the physical amplitude times sqrt(|det B_e| / 2), the factor of the
    orthonormal element basis."""
    rng = np.random.default_rng(seed)
    ne = B.shape[1]
    unit = np.sqrt(np.abs(B[0] * B[3] - B[1] * B[2]) / 2.0)
    scale = np.full((K, 1), 0.1)
    scale[0] = 1.0
    amp = np.array([0.1, 1.0, 1.0])[:, None, None]
    c = rng.normal(0.0, 1.0, (3, K, ne)) * scale * amp * unit
    u = rng.normal(0.0, 1.0, (2, K, ne)) * scale * unit
    KB = max(K, 3)
    hb = np.empty((KB, ne))
    hb[0] = rng.uniform(1.0, 5.0, ne)
    hb[1:] = rng.normal(0.0, 0.02, (KB - 1, ne))
    hb *= unit
    return (np.ascontiguousarray(c.reshape(3 * K, ne)), np.ascontiguousarray(u.reshape(2 * K, ne)),
            np.ascontiguousarray(hb))


def dg_boundary_ghosts(nbr: np.ndarray):
    """Number the domain-boundary edges of a neighbour table (entries -1):
    returns a copy of nbr with -2 - b at boundary edge b, and the element
    and local edge of every boundary edge (be, bq int32 (nb,)), in the order
    of the element index, then the local edge."""
    nbr = np.array(nbr, dtype=np.int32, copy=True)
    q, e = np.nonzero(nbr.T == -1)[1], np.nonzero(nbr.T == -1)[0]
    b = np.arange(e.size, dtype=np.int32)
    nbr[q, e] = -2 - b
    return nbr, e.astype(np.int32), q.astype(np.int32)
