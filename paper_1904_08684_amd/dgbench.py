"""DG benchmark: one launch of the quadrature-free volume terms, of the
velocity projection or of the edge terms, one evaluation of the whole
right-hand side, or one SSP-RK3 step, over a perturbed split-quad mesh
(boundary edges with prescribed exterior states), timed with HIP events.
The elements are numbered row by row (each half of the triangles in the
same order); --tile T numbers the squares in T x T tiles instead, which
keeps most edge neighbours within a block or two (measured: no faster,
the edge pass fetched 6.6 against 6.1 GB per launch at order 3).

    python -m paper_1904_08684_amd.dgbench --nx 1024 --k 3 --reps 20 [--op projection|edges|rhs|step] [--tile 0]

Prints one JSON line.  Bytes count the compulsory traffic per element (8 B
a double).  Volume terms: five fields, the map and the bathymetry in, three
fields out, 5K + 4 + K + 3K doubles; flops of the evaluated form,
8 K^3 + 30 K^2 + 15 K (four multiply-adds per (p, i, m), the two-function
terms and the set-up).  Projection: three fields, the map and the
bathymetry in, two out, 3K + 4 + K + 2K doubles; flops K^2 (K + 1) for the
weighted mass matrix, K^3 / 3 for its factorisation and 4 K^2 for the two
solves.  Edge terms: the element's fields, map and bathymetry, the
neighbour indices (24 B), three fields out (neighbours' data counted once,
as it is every element's own); flops of the Legendre-trace form,
6 (8 K NT + 2 KB NB + 9 NT^2 NB + 3 K NT) with NT = k + 1 and
NB = max(k, 1) + 1 (three edges; traces of both sides, trace products,
the map back to the test functions; a multiply-add counts two).  Right-hand side: both, with the
edge pass reading back what the volume pass wrote, and the bathymetry
source (4 K^3 more flops).  Step: three projections and right-hand sides,
the copy of the state (2 x 3K doubles) and three stage combinations (4 x 3K
doubles each).
"""
from __future__ import annotations

import argparse
import json


def flops_per_element(K: int) -> int:
    return 8 * K ** 3 + 30 * K * K + 15 * K


def bytes_per_element(K: int) -> int:
    return (5 * K + 4 + K + 3 * K) * 8


def projection_flops(K: int) -> int:
    return K * K * (K + 1) + K ** 3 // 3 + 4 * K * K


def projection_bytes(K: int) -> int:
    return (3 * K + 4 + K + 2 * K) * 8


def edge_flops(K: int) -> int:
    # per edge: the Legendre traces of both sides (four fields of K and the
    # bathymetry's KB coefficients), the three trace products against the
    # dense (NT, NT, NB) integrals, and the map back to the K test functions
    NT = {1: 1, 3: 2, 6: 3, 10: 4}[K]
    NB = max(NT, 2)
    KB = max(K, 3)
    return 3 * 2 * (8 * K * NT + 2 * KB * NB + 9 * NT * NT * NB + 3 * K * NT)


def edge_bytes(K: int) -> int:
    return (5 * K + 4 + K) * 8 + 24 + 3 * K * 8


def rhs_flops(K: int) -> int:
    return flops_per_element(K) + 4 * K ** 3 + edge_flops(K)


def rhs_bytes(K: int) -> int:
    return bytes_per_element(K) + edge_bytes(K) + 3 * K * 8


def step_flops(K: int) -> int:
    return 3 * (projection_flops(K) + rhs_flops(K) + 3 * 3 * K)


def step_bytes(K: int) -> int:
    return 3 * (projection_bytes(K) + rhs_bytes(K) + 4 * 3 * K * 8) + 2 * 3 * K * 8


def run(nx: int, k: int, reps: int, op: str = "volume", tile: int = 0):
    import numpy as np
    import torch

    from paper_1904_08684_amd import mg
    from paper_1904_08684_amd import workloads as W

    K = mg.DG_K[k]
    tile = tile if tile > 0 and nx % tile == 0 else 0
    B = W.dg_mesh(nx, nx, tile=tile)
    ne = B.shape[1]
    c, u, hb = W.dg_fields(K, B)
    nbr, nq = W.dg_mesh_neighbours(nx, nx, tile=tile)
    nbr, be, _ = W.dg_boundary_ghosts(nbr)
    cb, ub, _ = W.dg_fields(K, B[:, be], seed=W.SEED_DG_FIELDS + 1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    c, u, B, hb, nbr, nq, cb, ub = (dev(a) for a in (c, u, B, hb, nbr, nq, cb, ub))
    if op == "volume":
        out = torch.empty((3 * K, ne), dtype=torch.float64, device="cuda")
        kern = mg.DGVolume(k)
        call = lambda: kern(c, u, B, hb, 9.81, out)
        fl, by = flops_per_element(K) * ne, bytes_per_element(K) * ne
    elif op == "projection":
        kern = mg.DGProjection(k)
        call = lambda: kern(c, B, hb, u)
        fl, by = projection_flops(K) * ne, projection_bytes(K) * ne
    elif op == "edges":
        out = torch.empty((3 * K, ne), dtype=torch.float64, device="cuda")
        kern = mg.DGEdges(k)
        call = lambda: kern(c, u, B, hb, nbr, nq, 9.81, out, cb, ub)
        fl, by = edge_flops(K) * ne, edge_bytes(K) * ne
    elif op == "rhs":
        out = torch.empty((3 * K, ne), dtype=torch.float64, device="cuda")
        system = mg.DGSystem(k, B, hb, nbr, nq, nb=be.size)
        call = lambda: system.rhs(c, u, out, cb, ub)
        fl, by = rhs_flops(K) * ne, rhs_bytes(K) * ne
    else:
        # a step of dt small enough for the random fields to stay physical
        system = mg.DGSystem(k, B, hb, nbr, nq, nb=be.size)
        cb3, ub3 = cb.expand(3, -1, -1).contiguous(), ub.expand(3, -1, -1).contiguous()
        call = lambda: system.step(c, u, 1e-6, cb3, ub3)
        fl, by = step_flops(K) * ne, step_bytes(K) * ne
    call()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        call()
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"op": op, "elements": ne, "k": k, "tile": tile, "ms": ms, "gflops": fl / (ms * 1e-3) / 1e9,
            "GBps": by / (ms * 1e-3) / 1e9, "frac_fp64_vector": fl / (ms * 1e-3) / 78.6e12,
            "frac_hbm": by / (ms * 1e-3) / 8e12}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--k", type=int, default=3)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--op", default="volume", choices=("volume", "projection", "edges", "rhs", "step"))
    ap.add_argument("--tile", type=int, default=0, help="squares per tile side of the element numbering (0: rows)")
    a = ap.parse_args(argv)
    print(json.dumps(run(a.nx, a.k, a.reps, a.op, a.tile)), flush=True)


if __name__ == "__main__":
    main()
