"""The convergence test of the paper's Sec. 3.1 on the GPU: the manufactured
solution on a randomly perturbed split-quad mesh of [0, 1000]^2, stepped
with the library's SSP-RK3 step (dg_ssp_rk3_step), and the L2 errors of
xi, U and V at the final time.

The test problem's data (the exact fields, the body force that makes them a
solution, and the exterior states on the boundary) are inputs of the solver,
not part of the method: this module evaluates them with torch on the device
at the points of a collapsed Gauss rule on every element and L2-projects
them with the library's own basis values (dg_basis_values).  Every step of
the scheme itself runs in the library's kernels.

With theta = pi (x1 + x2 + C_t t) / 600 the exact fields are
    xi = 2 + y_a - 2 C_a sin theta,  U = 2 y_a + C_a C_t sin theta,
    V = y_a + C_a C_t sin theta,     h_b = 1 + x1 / 1000 + 2 x2 / 1000,
with C_a = C_t = 0.2, y_a = 0.3; the mass equation holds as it is and the
momentum equations get the force
    F = dq/dt + div(q q^T / H) + g H grad xi  (tau_bf = f_c = 0).
"""
from __future__ import annotations

import math

import numpy as np

from . import mg
from . import workloads as W

C_A, C_T, Y_A = 0.2, 0.2, 0.3
GRAV = 9.81
KAPPA = math.pi / 600.0
LENGTH = 1000.0


def collapsed_gauss(n: int):
    """Points and weights of the n x n collapsed Gauss-Legendre rule on the
    reference triangle (Duffy map x = a, y = (1 - a) b; exact to degree
    2 n - 2)."""
    t, w = np.polynomial.legendre.leggauss(n)
    s, ws = 0.5 * (t + 1.0), 0.5 * w
    A, Bq = np.meshgrid(s, s, indexing="ij")
    WA, WB = np.meshgrid(ws, ws, indexing="ij")
    return A.ravel(), ((1.0 - A) * Bq).ravel(), (WA * WB * (1.0 - A)).ravel()


class Problem:
    """The test on an nx x nx split-quad mesh (2 nx^2 elements) at order k."""

    def __init__(self, k: int, nx: int, device: str = "cuda", seed: int = W.SEED_DG_MESH, quad: int = 8,
                 with_system: bool = True, g: float = GRAV):
        import torch
        self.k, self.K, self.nx, self.g = k, mg.DG_K[k], nx, g
        B, a1 = W.dg_mesh(nx, nx, seed=seed, with_origin=True, length=LENGTH)
        nbr, nq = W.dg_mesh_neighbours(nx, nx)
        nbr, be, _ = W.dg_boundary_ghosts(nbr)
        self.ne, self.nb = B.shape[1], be.size
        X, Y, Wq = collapsed_gauss(quad)
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.phi = torch.tensor(mg.dg_basis(k, X, Y), **f64)                 # (K, Q)
        self.phib = torch.tensor(mg.dg_basis(max(k, 1), X, Y), **f64)       # (KB, Q): h_b is linear
        self.wq = torch.tensor(Wq, **f64)
        Bt = torch.tensor(B, **f64)
        At = torch.tensor(a1, **f64)
        Xt, Yt = torch.tensor(X, **f64), torch.tensor(Y, **f64)
        self.x = At[0][:, None] + Bt[0][:, None] * Xt[None, :] + Bt[1][:, None] * Yt[None, :]   # (ne, Q)
        self.y = At[1][:, None] + Bt[2][:, None] * Xt[None, :] + Bt[3][:, None] * Yt[None, :]
        self.sq = torch.sqrt(torch.abs(Bt[0] * Bt[3] - Bt[1] * Bt[2]))     # |det B_e|^(1/2)
        self.be = torch.tensor(be.astype(np.int64), device=dev)
        hb = ((1.0 + self.x / 1000.0 + 2.0 * self.y / 1000.0) * self.wq) @ self.phib.T
        hb = hb.T * self.sq
        self.hb = hb
        self.system = None if not with_system else mg.DGSystem(k, Bt.contiguous(), hb.contiguous(),
                                  torch.tensor(nbr, dtype=torch.int32, device=dev),
                                  torch.tensor(nq, dtype=torch.int32, device=dev), nb=self.nb, g=g)

    # -------------------------------------------------- the test problem's data
    def project(self, vals):
        """Coefficients (K, ne) of the L2 projection of point values (ne, Q):
        int f phi_ep = |det B_e|^(1/2) sum_q w_q f_q phi^_p(q)."""
        return ((vals * self.wq) @ self.phi.T).T * self.sq

    def fields(self, t: float):
        """Exact xi, U, V and the depth H at the points, (ne, Q) each."""
        import torch
        s = torch.sin(KAPPA * (self.x + self.y + C_T * t))
        xi = 2.0 + Y_A - 2.0 * C_A * s
        U = 2.0 * Y_A + C_A * C_T * s
        V = Y_A + C_A * C_T * s
        H = 1.0 + self.x / 1000.0 + 2.0 * self.y / 1000.0 + xi
        return xi, U, V, H

    def force(self, t: float):
        """The momentum force (F_U, F_V) at the points: quotient rule on
        q q^T / H, with every first derivative of the sine's argument
        equal to KAPPA in x1 and x2 and KAPPA C_t in t."""
        import torch
        xi, U, V, H = self.fields(t)
        d = KAPPA * torch.cos(KAPPA * (self.x + self.y + C_T * t))
        dxi = -2.0 * C_A * d                 # d xi / dx1 = d xi / dx2
        dq = C_A * C_T * d                   # dU/dx_l = dV/dx_l
        dqt = C_A * C_T * C_T * d            # dU/dt = dV/dt
        Hx, Hy = 1.0 / 1000.0 + dxi, 2.0 / 1000.0 + dxi
        H2 = H * H
        FU = dqt + (2.0 * U * dq * H - U * U * Hx) / H2 + ((dq * V + U * dq) * H - U * V * Hy) / H2 + self.g * H * dxi
        FV = dqt + ((dq * V + U * dq) * H - U * V * Hx) / H2 + (2.0 * V * dq * H - V * V * Hy) / H2 + self.g * H * dxi
        return FU, FV

    def state(self, t: float):
        """Coefficients of the projected exact state c (3K, ne) and velocity
        u = q / H (2K, ne) at time t."""
        import torch
        xi, U, V, H = self.fields(t)
        c = torch.cat([self.project(xi), self.project(U), self.project(V)])
        u = torch.cat([self.project(U / H), self.project(V / H)])
        return c.contiguous(), u.contiguous()

    def stage_data(self, t: float):
        """Body force (3K, ne) and the exterior states of the boundary edges
        (3K, nb), (2K, nb) at time t: the projections of the exact fields onto
        the element that owns each boundary edge."""
        import torch
        FU, FV = self.force(t)
        F = torch.cat([torch.zeros(self.K, self.ne, dtype=FU.dtype, device=FU.device),
                       self.project(FU), self.project(FV)])
        c, u = self.state(t)
        return F, c[:, self.be], u[:, self.be]

    # ----------------------------------------------------------- the run
    def initial(self):
        c, _ = self.state(0.0)
        return c

    def run(self, t_end: float, dt: float, c=None):
        """Steps of dt from t = 0 (or from c at t = 0) to t_end; returns the
        final coefficients (3K, ne) and the number of steps."""
        import torch
        steps = int(round(t_end / dt))
        if abs(steps * dt - t_end) > 1e-9 * max(1.0, t_end):
            raise ValueError("t_end must be a whole number of steps")
        c = self.initial() if c is None else c
        u = torch.empty(2 * self.K, self.ne, dtype=torch.float64, device=c.device)
        times = (0.0, 1.0, 0.5)
        carry = None                      # the data at t + dt opens the next step
        for n in range(steps):
            t = n * dt
            data = [carry if (s == 0.0 and carry is not None) else self.stage_data(t + s * dt) for s in times]
            carry = data[1]
            F3 = torch.stack([d[0] for d in data]).contiguous()
            cb3 = torch.stack([d[1] for d in data]).contiguous()
            ub3 = torch.stack([d[2] for d in data]).contiguous()
            self.system.step(c, u, dt, cb3, ub3, F3)
        return c, steps

    def errors(self, c, t: float):
        """L2 errors (over the mesh) of xi, U, V of the DG state c at time t."""
        import torch
        xi, U, V, _ = self.fields(t)
        out = []
        for j, f in enumerate((xi, U, V)):
            vals = (c[j * self.K:(j + 1) * self.K].T @ self.phi) / self.sq[:, None]    # (ne, Q)
            d = vals - f
            out.append(math.sqrt(float(torch.sum((d * d * self.wq) * (self.sq * self.sq)[:, None]))))
        return out


# the largest |u . n| + sqrt(g H) of the exact solution: H <= 4 + 2.7,
# |u| <= 0.64 / 2.9
WAVE_SPEED = 8.5


def stable_dt(k: int, nx: int, t_end: float, dt_max: float = 0.5, cfl: float = 0.25, g: float = GRAV):
    """The paper's step (0.5), or less where the explicit scheme needs it:
    lambda dt (2k + 1) / h <= cfl with h the square's side (runs at 0.4 and
    above blew up); returns (dt, steps) with steps dt = t_end.  For another
    g the wave speed bound is 0.25 + sqrt(6.7 g) (H <= 6.7)."""
    h = LENGTH / nx
    speed = WAVE_SPEED if g == GRAV else 0.25 + math.sqrt(6.7 * g)
    dt = min(dt_max, cfl * h / (speed * (2 * k + 1)))
    steps = int(math.ceil(t_end / dt - 1e-9))
    return t_end / steps, steps


def table(orders=(0, 1, 2, 3), levels=None, t_end: float = 1500.0, dt: float = 0.5, device: str = "cuda"):
    """Errors and experimental orders of convergence for the meshes of the
    paper's table (nx = 4, 8, ... squares per side: 32, 128, ... elements).
    levels maps k to the list of nx; returns {k: [(ne, err_xi, err_U,
    err_V), ...]}."""
    levels = levels or {0: [4, 8, 16, 32, 64, 128], 1: [4, 8, 16, 32, 64], 2: [4, 8, 16, 32],
                        3: [4, 8, 16, 32]}
    out = {}
    for k in orders:
        rows = []
        for nx in levels[k]:
            pr = Problem(k, nx, device=device)
            c, _ = pr.run(t_end, stable_dt(k, nx, t_end, dt)[0])
            rows.append((pr.ne, *pr.errors(c, t_end)))
        out[k] = rows
    return out


def main(argv=None):
    """python -m paper_1904_08684_amd.convergence [--orders 0 1 2 3] [--t-end 1500] [--dt 0.5]
    prints one JSON line per run (k, elements, errors, EOC against the
    previous mesh) as it finishes."""
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser()
    ap.add_argument("--orders", type=int, nargs="+", default=[0, 1, 2, 3])
    ap.add_argument("--t-end", type=float, default=1500.0)
    ap.add_argument("--dt", type=float, default=0.5)
    ap.add_argument("--max-nx", type=int, default=128)
    ap.add_argument("--g", type=float, default=GRAV, help="gravitational acceleration (the paper states none)")
    ap.add_argument("--exact-dt", action="store_true", help="step with --dt on every mesh, no stability cap")
    a = ap.parse_args(argv)
    levels = {0: [4, 8, 16, 32, 64, 128], 1: [4, 8, 16, 32, 64], 2: [4, 8, 16, 32], 3: [4, 8, 16, 32]}
    for k in a.orders:
        prev = None
        for nx in levels[k]:
            if nx > a.max_nx:
                break
            dt, steps = (a.dt, int(round(a.t_end / a.dt))) if a.exact_dt else stable_dt(k, nx, a.t_end, a.dt, g=a.g)
            print(f"# k={k} nx={nx}: {2 * nx * nx} elements, {steps} steps of {dt:.4g}, g = {a.g:g}", flush=True)
            t0 = time.perf_counter()
            pr = Problem(k, nx, g=a.g)
            c, steps = pr.run(a.t_end, dt)
            err = pr.errors(c, a.t_end)
            eoc = None if prev is None else [round(math.log2(p / e), 2) for p, e in zip(prev, err)]
            print(json.dumps({"k": k, "g": a.g, "elements": pr.ne, "steps": steps, "dt": dt, "err_xi": err[0],
                              "err_U": err[1],
                              "err_V": err[2], "eoc": eoc, "seconds": round(time.perf_counter() - t0, 2)}),
                  flush=True)
            prev = err


if __name__ == "__main__":
    main()
