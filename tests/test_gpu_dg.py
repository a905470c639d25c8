"""GPU parity of the DG volume terms (quadrature-free algebraic form, one
thread per element) with the oracle's quadrature on the physical element:
every element of small meshes for orders 0-3, and sampled elements of a
2 x 1000 x 1000 mesh (a ragged last block)."""
import numpy as np
import pytest

from oracle import dg
from paper_1904_08684_amd import workloads as W

pytestmark = pytest.mark.gpu

G_GRAV = 9.81
TOL = 1e-12   # relative to the largest |E| of the element and equation


def run(mg, k, nx, ny):
    import torch
    K = dg.K_OF[k]
    B = W.dg_mesh(nx, ny)
    ne = B.shape[1]
    c, u, hb = W.dg_fields(K, B)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = torch.full((3 * K, ne), float("nan"), dtype=torch.float64, device="cuda")
    mg.DGVolume(k)(dev(c), dev(u), dev(B), dev(hb), G_GRAV, out)
    torch.cuda.synchronize()
    return B, c, u, hb, out.cpu().numpy()


def check(k, B, c, u, hb, out, elems):
    K = dg.K_OF[k]
    worst = 0.0
    for e in elems:
        Be = np.array([[B[0, e], B[1, e]], [B[2, e], B[3, e]]])
        ref = dg.volume_integrals(k, c[:, e].reshape(3, K), u[:, e].reshape(2, K), Be, hb[e], G_GRAV)
        got = out[:, e].reshape(3, K)
        for j in range(3):
            scale = max(np.max(np.abs(ref[j])), 1e-300)
            worst = max(worst, float(np.max(np.abs(got[j] - ref[j])) / scale))
    return worst


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_small_mesh_every_element(mg, k):
    B, c, u, hb, out = run(mg, k, 8, 8)
    worst = check(k, B, c, u, hb, out, range(B.shape[1]))
    print(f"DG k={k} 128 elements: worst relative difference {worst:.2e}", flush=True)
    assert np.all(np.isfinite(out)) and worst <= TOL


def test_full_size_sampled(mg):
    k = 3
    B, c, u, hb, out = run(mg, k, 1000, 1000)
    ne = B.shape[1]
    rng = np.random.default_rng(5)
    elems = np.concatenate([rng.integers(0, ne, 300), np.arange(ne - 64, ne)])
    worst = check(k, B, c, u, hb, out, elems)
    print(f"DG k=3 {ne} elements: {len(elems)} sampled, worst relative difference {worst:.2e}", flush=True)
    assert np.all(np.isfinite(out)) and worst <= TOL


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_velocity_projection(mg, k):
    """The per-element solve of (u H, psi) = (q, psi) against the oracle's
    quadrature-assembled system, every element of a small mesh and sampled
    elements of a 2M-element mesh (ragged last block)."""
    import torch
    K = dg.K_OF[k]
    for nx, sample in ((8, None), (1000, 300)):
        B = W.dg_mesh(nx, nx)
        ne = B.shape[1]
        c, _, hb = W.dg_fields(K, B)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        u = torch.full((2 * K, ne), float("nan"), dtype=torch.float64, device="cuda")
        mg.DGProjection(k)(dev(c), dev(B), dev(hb), u)
        torch.cuda.synchronize()
        got = u.cpu().numpy()
        if sample is None:
            elems = range(ne)
        else:
            rng = np.random.default_rng(6)
            elems = np.concatenate([rng.integers(0, ne, sample), np.arange(ne - 64, ne)])
        worst = 0.0
        for e in elems:
            Be = np.array([[B[0, e], B[1, e]], [B[2, e], B[3, e]]])
            ref = dg.velocity_projection(k, c[:, e].reshape(3, K), Be, hb[e])
            worst = max(worst, float(np.max(np.abs(got[:, e].reshape(2, K) - ref)) / np.max(np.abs(ref))))
        print(f"DG projection k={k} {ne} elements: worst relative difference {worst:.2e}", flush=True)
        assert np.all(np.isfinite(got)) and worst <= TOL


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_edge_terms(mg, k):
    """Interior-edge Lax-Friedrichs terms against the oracle's edge
    quadrature: every element of an 8 x 8 split-quad mesh (boundary edges
    skipped), sampled elements of a 2M-element mesh."""
    import torch
    K = dg.K_OF[k]
    for nx, sample in ((8, None), (1000, 200)):
        B, a1 = W.dg_mesh(nx, nx, with_origin=True)
        nbr, nq = W.dg_mesh_neighbours(nx, nx)
        ne = B.shape[1]
        c, u, hb = W.dg_fields(K, B)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        out = torch.full((3 * K, ne), float("nan"), dtype=torch.float64, device="cuda")
        mg.DGEdges(k)(dev(c), dev(u), dev(B), dev(hb), dev(nbr), dev(nq), G_GRAV, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))

        def state(e):
            Be = np.array([[B[0, e], B[1, e]], [B[2, e], B[3, e]]])
            return c[:, e].reshape(3, K), u[:, e].reshape(2, K), Be, a1[:, e], hb[e]
        if sample is None:
            elems = range(ne)
        else:
            rng = np.random.default_rng(7)
            elems = np.concatenate([rng.integers(0, ne, sample), np.arange(ne - 32, ne)])
        worst = 0.0
        for e in elems:
            nbrs = [state(int(nbr[q, e])) if nbr[q, e] >= 0 else None for q in range(3)]
            ref = dg.edge_integrals_lf(k, state(e), nbrs, G_GRAV)
            got_e = got[:, e].reshape(3, K)
            # relative to the element's largest term: the three rows differ in
            # size (the pressure terms g h_b xi dominate the momentum rows)
            worst = max(worst, float(np.max(np.abs(got_e - ref)) / max(np.max(np.abs(ref)), 1e-300)))
        print(f"DG edge terms k={k} {ne} elements: worst relative difference {worst:.2e}", flush=True)
        assert worst <= TOL
