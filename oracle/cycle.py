"""Level hierarchy, coarsest-level direct solve, multigrid cycles (V, W, F),
solve to tolerance and mixed-precision iterative refinement.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The V-cycle is the textbook recursion (Trottenberg et al., *Multigrid*,
Sec. 2.4, gamma = 1): on level l, smooth nu1 times, restrict the residual to
the right-hand side of level l+1, start level l+1 from zero, recurse, add the
interpolated correction, smooth nu2 times; on the coarsest level solve
exactly.  The W-cycle (gamma = 2) visits level l+1 twice, the second visit
continuing from the first one's result; the F-cycle visits it with an
F-cycle from zero followed by a V-cycle (Trottenberg et al., Sec. 2.4.2).
A level directly above the coarsest is visited once in every type, since
the coarsest solve is exact.  Coarse operators are rediscretised (the same stencil with the
coarse mesh width), matching ExaSlang's per-level ``Stencil`` declarations.
The coarsest solve is always FP64: a dense Cholesky factorisation of the
coarsest matrix followed by two triangular solves, with float32 right-hand
sides upcast and the result downcast.

``solve`` repeats cycles until ||r_k|| / ||r_0|| <= tol (the ExaSlang
``repeat ... until`` form), with the unweighted 2-norm over the unknowns.

Galerkin coarse operators (``coarse_op="galerkin"``, node grids with damped
Jacobi smoothing): every coarser level uses A_{l+1} = R A_l P (``galerkin``)
for its smoothing, residual and coarsest solve, the finest level keeps the
5/7-point stencil.

Cell grids with Neumann walls (``bc="neumann"``): the right-hand side is
projected to zero mean when a solve starts and after every restriction, the
coarsest level is solved by the minimum-norm least-squares solution (the
zero-mean solution of the singular consistent system), interpolation uses
even ghosts, and the finest iterate is projected to zero mean after every
cycle, which fixes the constant the operator cannot see.

``mixed_solve`` is FP64 iterative refinement around single-precision
V-cycles: r_k = f - A u_k in FP64, c = V32(0, fl32(r_k / sigma_k)),
u_{k+1} = u_k + sigma_k * fl64(c), with the power-of-two scale
sigma_k = 2^floor(log2 m_k), m_k the largest |r| of the previous step's
residual r_{k-1} (of r_0 itself in the first step).  A power-of-two scale
adds no rounding, and every operation of the single-precision cycle commutes
with it, so away from FP32 underflow and overflow the iterates do not depend
on which power of two is taken; the scale only keeps the single-precision
values in range when the residual is tiny or huge.  Taking the previous
residual's maximum lets an implementation scale the residual while it is
formed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

from . import cell, galerkin, node


@dataclass
class Params:
    centering: str = "node"          # "node" or "cell"
    dim: int = 2
    n: int = 129                     # nodes per axis (node) or cells per axis (cell), finest
    coarsest: int = 5                # 5 nodes (3^d unknowns) or 4 cells
    smoother: str = "jacobi"         # "jacobi" or "rbgs"
    omega: float = 0.8
    nu1: int = 2
    nu2: int = 2
    post_order: tuple = (0, 1)       # colour order of post-smoothing sweeps
    k: np.ndarray | None = None      # cell coefficients (cell grids); None = 1
    cycle: str = "V"                 # "V", "W" or "F"
    bc: str = "dirichlet"            # "dirichlet", or "neumann" (cell grids)
    coarse_op: str = "rediscretise"  # or "galerkin" (node grids, Jacobi): A_{l+1} = R A_l P


@dataclass
class Hierarchy:
    p: Params
    sizes: list
    beta: list = field(default_factory=list)       # per level, FP64 face lists (cell only)
    chol: np.ndarray | None = None                  # FP64 lower Cholesky factor, coarsest
    dense: np.ndarray | None = None                 # FP64 coarsest matrix (Neumann: singular)
    W: list = field(default_factory=list)           # Galerkin: 3^d stencil per level
    _beta_cache: dict = field(default_factory=dict)
    coarse_solves: int = 0                          # coarsest solves performed (instrumentation)

    @property
    def levels(self) -> int:
        return len(self.sizes)

    def beta_as(self, lvl: int, dtype):
        key = (lvl, np.dtype(dtype).str)
        if key not in self._beta_cache:
            self._beta_cache[key] = [b.astype(dtype) for b in self.beta[lvl]]
        return self._beta_cache[key]


def ladder(p: Params) -> list:
    sizes = [p.n]
    n = p.n
    while n > p.coarsest:
        if p.centering == "node":
            if (n - 1) % 2:
                raise ValueError(f"node size {n} cannot be coarsened 2:1")
            n = (n - 1) // 2 + 1
        else:
            if n % 2:
                raise ValueError(f"cell count {n} cannot be coarsened 2:1")
            n //= 2
        sizes.append(n)
    if n != p.coarsest:
        raise ValueError(f"ladder from {p.n} misses the coarsest size {p.coarsest}")
    return sizes


def neumann(h: Hierarchy) -> bool:
    return h.p.bc == "neumann"


def build_hierarchy(p: Params) -> Hierarchy:
    if p.bc not in ("dirichlet", "neumann") or (p.bc == "neumann" and p.centering != "cell"):
        raise ValueError(f"boundary {p.bc!r} with {p.centering} centring")
    if p.coarse_op not in ("rediscretise", "galerkin") or (
            p.coarse_op == "galerkin" and (p.centering != "node" or p.smoother != "jacobi")):
        raise ValueError(f"coarse operator {p.coarse_op!r} with {p.centering} centring and {p.smoother}")
    h = Hierarchy(p, ladder(p))
    if p.centering == "cell":
        k = p.k if p.k is not None else np.ones((p.n,) * p.dim)
        h.beta.append(cell.harmonic_faces(np.asarray(k, dtype=np.float64)))
        for _ in h.sizes[1:]:
            h.beta.append(cell.coarsen_faces(h.beta[-1]))
        A = cell.dense_matrix(h.beta[-1], h.sizes[-1], p.dim, p.bc)
    elif p.coarse_op == "galerkin":
        h.W.append(galerkin.laplacian_stencil(p.n, p.dim))
        for _ in h.sizes[1:]:
            h.W.append(galerkin.coarse_stencil(h.W[-1]))
        A = galerkin.dense_matrix(h.W[-1], h.sizes[-1])
    else:
        A = node.dense_matrix(h.sizes[-1], p.dim)
    h.dense = A
    if p.bc == "dirichlet":
        h.chol = np.linalg.cholesky(A)
    return h


# ---------------------------------------------------------------- level ops
def galerkin_level(h: Hierarchy, lvl: int) -> bool:
    """Coarse levels of a Galerkin hierarchy carry R A P stencils; the finest
    keeps the 5/7-point operator."""
    return h.p.coarse_op == "galerkin" and lvl > 0


def residual(h: Hierarchy, lvl: int, u, f):
    if galerkin_level(h, lvl):
        return galerkin.residual(u, f, h.W[lvl])
    if h.p.centering == "node":
        return node.residual(u, f)
    return cell.residual(u, f, h.beta_as(lvl, u.dtype), h.p.bc)


def unknowns(h: Hierarchy, a):
    """The entries of a level array that are unknowns (flattened view)."""
    if h.p.centering == "node":
        return a[node.interior(a.ndim)]
    return a


def smooth(h: Hierarchy, lvl: int, u, f, sweeps: int, order=(0, 1)):
    p = h.p
    for _ in range(sweeps):
        if galerkin_level(h, lvl):
            u = galerkin.jacobi(u, f, h.W[lvl], p.omega)
        elif p.centering == "node":
            u = node.jacobi(u, f, p.omega) if p.smoother == "jacobi" else node.rbgs(u, f, order)
        else:
            b = h.beta_as(lvl, u.dtype)
            u = (cell.jacobi(u, f, b, p.omega, p.bc) if p.smoother == "jacobi"
                 else cell.rbgs(u, f, b, order, p.bc))
    return u


def restrict(h: Hierarchy, r):
    """Transfer of a residual to the next coarser right-hand side (zero mean
    with Neumann walls)."""
    if h.p.centering == "node":
        return node.restrict_fw(r)
    fc = cell.restrict_mean(r)
    return cell.project_mean(fc) if neumann(h) else fc


def prolong_correct(h: Hierarchy, u, ec):
    return node.correct(u, ec) if h.p.centering == "node" else cell.correct(u, ec, h.p.bc)


def coarse_solve(h: Hierarchy, fc):
    """Exact coarsest solve in FP64 via the stored Cholesky factor L:
    L y = b, L^T x = y; float32 inputs are upcast and the result downcast."""
    h.coarse_solves += 1
    b = np.asarray(unknowns(h, fc), dtype=np.float64).reshape(-1)
    if neumann(h):
        # minimum-norm least-squares solution of the singular system
        x = np.linalg.lstsq(h.dense, b, rcond=None)[0]
    else:
        y = scipy.linalg.solve_triangular(h.chol, b, lower=True)
        x = scipy.linalg.solve_triangular(h.chol.T, y, lower=False)
    out = np.zeros(fc.shape, dtype=fc.dtype)
    if h.p.centering == "node":
        out[node.interior(fc.ndim)] = x.reshape((fc.shape[0] - 2,) * fc.ndim).astype(fc.dtype)
    else:
        out[...] = x.reshape(fc.shape).astype(fc.dtype)
    return out


def vcycle(h: Hierarchy, u, f, lvl: int = 0):
    """One (nu1, nu2)-cycle of type h.p.cycle on level lvl; returns the new
    iterate (the name is kept for the default V-cycle)."""
    return mg_cycle(h, u, f, lvl, h.p.cycle)


def mg_cycle(h: Hierarchy, u, f, lvl: int, kind: str):
    p = h.p
    if lvl == h.levels - 1:
        return coarse_solve(h, f)
    u = smooth(h, lvl, u, f, p.nu1, (0, 1))
    r = residual(h, lvl, u, f)
    fc = restrict(h, r)
    uc = np.zeros_like(fc)
    uc = mg_cycle(h, uc, fc, lvl + 1, kind)
    if lvl + 1 < h.levels - 1:
        if kind == "W":
            uc = mg_cycle(h, uc, fc, lvl + 1, "W")
        elif kind == "F":
            uc = mg_cycle(h, uc, fc, lvl + 1, "V")
    u = prolong_correct(h, u, uc)
    u = smooth(h, lvl, u, f, p.nu2, p.post_order)
    if lvl == 0 and neumann(h):
        u = cell.project_mean(u)
    return u


def start_rhs(h: Hierarchy, f):
    """The right-hand side a solve starts from: zero mean with Neumann walls."""
    return cell.project_mean(f) if neumann(h) else f


def fmg(h: Hierarchy, f, cycles_per_level: int = 1):
    """Full multigrid (Trottenberg et al., Sec. 2.6): the right-hand side is
    restricted to every level by the transfer operator of the cycle, the
    coarsest level is solved exactly, and each finer level starts from the
    interpolated coarser solution (multilinear interpolation, the cycle's
    own) and applies cycles_per_level cycles of type h.p.cycle.  Returns the
    finest iterate."""
    fs = [start_rhs(h, f)]
    for _ in range(1, h.levels):
        fs.append(restrict(h, fs[-1]))
    u = coarse_solve(h, fs[-1])
    for lvl in range(h.levels - 2, -1, -1):
        u = prolong_correct(h, np.zeros_like(fs[lvl]), u)
        for _ in range(cycles_per_level):
            u = mg_cycle(h, u, fs[lvl], lvl, h.p.cycle)
    return u


def apply_operator(h: Hierarchy, u):
    """A u on the finest level (0 on node boundaries)."""
    return -residual(h, 0, u, np.zeros_like(u))


def dot(h: Hierarchy, a, b) -> float:
    """Euclidean inner product over the finest level's unknowns."""
    ua = np.asarray(unknowns(h, a), dtype=np.float64)
    ub = np.asarray(unknowns(h, b), dtype=np.float64)
    return float(np.sum(ua * ub))


def pcg(h: Hierarchy, f, u0=None, tol=1e-10, max_it=100, precondition=True):
    """Conjugate gradients for A u = f preconditioned by one cycle from zero
    (Trottenberg et al., Sec. 7.8; Saad, Iterative Methods for Sparse Linear
    Systems, Alg. 9.1).  The cycle is a symmetric positive definite
    preconditioner when nu1 = nu2 and post-smoothing is the adjoint of
    pre-smoothing (red-black GS: the reverse colour order).  With
    precondition=False it is plain CG.  Returns (u, relres history)."""
    if neumann(h):
        raise ValueError("the Krylov solver is for Dirichlet problems")
    u = np.zeros_like(f) if u0 is None else u0.copy()
    r = residual(h, 0, u, f)
    prec = (lambda v: vcycle(h, np.zeros_like(v), v)) if precondition else (lambda v: v.copy())
    z = prec(r)
    p = z.copy()
    rho = dot(h, r, z)
    r0 = np.sqrt(dot(h, r, r))
    hist = [1.0]
    for _ in range(max_it):
        if r0 == 0.0 or hist[-1] <= tol:
            break
        q = apply_operator(h, p)
        alpha = rho / dot(h, p, q)
        u = u + alpha * p
        r = r - alpha * q
        hist.append(np.sqrt(dot(h, r, r)) / r0)
        if hist[-1] <= tol:
            break
        z = prec(r)
        rho_new = dot(h, r, z)
        p = z + (rho_new / rho) * p
        rho = rho_new
    return u, hist


def residual_norm(h: Hierarchy, u, f) -> float:
    r = residual(h, 0, u, f)
    ru = np.asarray(unknowns(h, r), dtype=np.float64)
    return float(np.sqrt(np.sum(ru * ru)))


def solve(h: Hierarchy, f, u0=None, tol=1e-10, max_cycles=100, record_iterates=False):
    """V-cycles from u0 until ||r|| / ||r0|| <= tol.  Returns
    (u, relres history including the initial 1.0, iterates or None)."""
    f = start_rhs(h, f)
    u = np.zeros_like(f) if u0 is None else u0.copy()
    r0 = residual_norm(h, u, f)
    hist = [1.0]
    its = [] if record_iterates else None
    for _ in range(max_cycles):
        if r0 == 0.0 or hist[-1] <= tol:
            break
        u = vcycle(h, u, f)
        if its is not None:
            its.append(u.copy())
        hist.append(residual_norm(h, u, f) / r0)
    return u, hist, its


def cycles(h: Hierarchy, f, u0, k: int):
    """Exactly k V-cycles from u0; returns the list of iterates u^1..u^k."""
    f = start_rhs(h, f)
    u = u0.copy()
    out = []
    for _ in range(k):
        u = vcycle(h, u, f)
        out.append(u.copy())
    return out


def pow2_scale(maxabs: float) -> float:
    """2^floor(log2 maxabs) for maxabs > 0 (frexp gives maxabs = m 2^e, m in [0.5, 1))."""
    _, e = np.frexp(maxabs)
    return float(np.ldexp(1.0, int(e) - 1))


def mixed_solve(h: Hierarchy, f, tol=1e-10, max_outer=100, inner=np.float32, scale="previous"):
    """FP64 iterative refinement with single-precision V-cycles, from u = 0.
    scale: "previous" (sigma_k from the previous step's residual, the first
    step's from its own) or "current" (sigma_k from r_k itself).
    Returns (u, relres history ||r_k|| / ||f||)."""
    if neumann(h):
        raise ValueError("mixed-precision refinement is for Dirichlet problems")
    u = np.zeros_like(f, dtype=np.float64)
    hist = []
    r0 = None
    m_prev = None
    for _ in range(max_outer + 1):
        r = residual(h, 0, u, f)
        ru = np.asarray(unknowns(h, r))
        nrm = float(np.sqrt(np.sum(ru * ru)))
        m_cur = float(np.max(np.abs(ru)))
        if r0 is None:
            r0 = nrm
        hist.append(nrm / r0 if r0 else 0.0)
        if r0 == 0.0 or hist[-1] <= tol or len(hist) > max_outer:
            break
        sigma = pow2_scale(m_cur if (scale == "current" or m_prev is None) else m_prev)
        m_prev = m_cur
        r32 = (r / sigma).astype(inner)
        c = vcycle(h, np.zeros_like(r32), r32)
        u = u + sigma * c.astype(np.float64)
    return u, hist
