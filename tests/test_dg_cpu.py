"""Host side of the DG volume terms: the library's exact reference integrals
against the oracle's quadrature of the same products (no GPU needed)."""
import numpy as np
import pytest

from oracle import dg


@pytest.fixture(scope="module")
def mg():
    from paper_1904_08684_amd import mg as _mg
    return _mg


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_reference_integrals_match_quadrature(mg, k):
    """Tables of order max(k, 1) (the bathymetry is at least linear)."""
    G, H = mg.dg_reference(k)
    K = dg.KB_OF[k]
    X, Y, Wt = dg.triangle_rule()
    phi = np.array(dg.basis(X, Y))[:K]
    gx, gy = dg.basis_grad(X, Y)
    d = [np.array(gx)[:K], np.array(gy)[:K]]
    for l in range(2):
        Gq = (d[l] * Wt) @ phi.T
        Hq = np.einsum("pq,iq,mq->pim", d[l] * Wt, phi, phi)
        assert np.max(np.abs(G[l] - Gq)) <= 1e-12
        assert np.max(np.abs(H[l] - Hq)) <= 1e-12


def test_reference_sizes_and_bad_orders(mg):
    assert [mg.dg_reference_size(k) for k in range(4)] == [2 * K * K + 2 * K ** 3 for K in (3, 3, 6, 10)]
    assert mg.dg_reference_size(4) == 0 and mg.dg_reference_size(-1) == 0
    assert mg.dg_reference_integrals(4, None) == mg.MG_EINVAL
    assert mg.dg_volume_integrals(5, 10, None, None, None, None, 9.81, None, None, None) == mg.MG_EINVAL
    assert mg.dg_volume_integrals(3, -1, None, None, None, None, 9.81, None, None, None) == mg.MG_EINVAL
    assert mg.dg_volume_integrals(3, 0, None, None, None, None, 9.81, None, None, None) == mg.MG_OK


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_product_integrals_match_quadrature(mg, k):
    T = mg.dg_products(k)
    K = dg.K_OF[k]
    X, Y, Wt = dg.triangle_rule()
    phi = np.array(dg.basis(X, Y))[:K]
    Tq = np.einsum("pq,iq,mq->pim", phi * Wt, phi, phi)
    assert np.max(np.abs(T - Tq)) <= 1e-12
    assert mg.dg_product_size(k) == K ** 3
    assert mg.dg_velocity_projection(k, -1, None, None, None, None, None, None) == mg.MG_EINVAL


def _shifted_legendre(n, s):
    return [np.ones_like(s), 2 * s - 1, 6 * s * s - 6 * s + 1, 20 * s ** 3 - 30 * s * s + 12 * s - 1][:n]


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_edge_trace_table_matches_quadrature(mg, k):
    """C[q][i][a] = (2a + 1) int_0^1 phi^_i(edge q at s) P_a(s) ds against
    Gauss quadrature of the oracle's basis, and the expansion reproduces
    the traces (they have degree max(k, 1))."""
    KB, NB = dg.KB_OF[k], mg.DG_NB[k]
    C = mg.dg_edge_table(k)["C"]
    t, w = np.polynomial.legendre.leggauss(8)
    s = (t + 1.0) / 2.0
    w = w / 2.0
    lin = {0: (0, 1, 0, 0), 1: (1, -1, 0, 1), 2: (0, 0, 1, -1)}
    P = np.array(_shifted_legendre(NB, s))
    for q in range(3):
        x0, xs, y0, ys = lin[q]
        tr = np.array(dg.basis(x0 + xs * s, y0 + ys * s))[:KB]
        want = (tr * w) @ P.T * (2 * np.arange(NB) + 1)
        assert np.max(np.abs(C[q] - want)) <= 1e-12
        assert np.max(np.abs(C[q] @ P - tr)) <= 1e-12
    assert mg.dg_edge_table_size(k) == 3 * KB * NB


@pytest.mark.parametrize("k", [1, 3])
def test_edge_trace_factorisation_gives_the_triple_product_integrals(mg, k):
    """The edge kernel's factorised form: int phi^_p(q, s) phi^_i(q', s')
    phi^_m(q', s') ds with s' = s (own edge) or 1 - s (a neighbour's edge,
    odd Legendre coefficients negated) equals
    sum_abc C[q][p][a] C'[i][b] C'[m][c] int P_a P_b P_c, the last by
    Gauss quadrature here."""
    K, NB = dg.K_OF[k], mg.DG_NB[k]
    C = mg.dg_edge_table(k)["C"]
    t, w = np.polynomial.legendre.leggauss(10)
    s = (t + 1.0) / 2.0
    w = w / 2.0
    P = np.array(_shifted_legendre(NB, s))
    L3 = np.einsum("aq,bq,cq->abc", P * w, P, P)
    lin = {0: (0, 1, 0, 0), 1: (1, -1, 0, 1), 2: (0, 0, 1, -1)}
    flip = (-1.0) ** np.arange(NB)

    def trace(q, back):
        x0, xs, y0, ys = lin[q]
        ss = 1.0 - s if back else s
        return np.array(dg.basis(x0 + xs * ss, y0 + ys * ss))[:K]
    for q in range(3):
        own = trace(q, False)
        for r in (None, 0, 1, 2):
            other = own if r is None else trace(r, True)
            want = np.einsum("pq,iq,mq->pim", own * w, other, other)
            Co = C[q, :K] if r is None else C[r, :K] * flip
            got = np.einsum("pa,ib,mc,abc->pim", C[q, :K], Co, Co, L3)
            assert np.max(np.abs(got - want)) <= 1e-11


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_basis_values_match_the_papers_polynomials(mg, k):
    """The library's host evaluation of the reference basis (used by the
    convergence test's projections) against the oracle's transcription of
    the paper's ten polynomials."""
    rng = np.random.default_rng(8)
    x = rng.uniform(0.0, 1.0, 40)
    y = rng.uniform(0.0, 1.0, 40) * (1.0 - x)
    want = np.array(dg.basis(x, y))[:mg.DG_K[k]]
    assert np.max(np.abs(mg.dg_basis(k, x, y) - want)) <= 1e-13


def test_system_entry_points_reject_bad_arguments(mg):
    """Argument checks that return before any device work."""
    E = mg.MG_EINVAL
    n = None
    # bad order, negative sizes, prescribed states without arrays, non-finite dt
    assert mg.dg_rhs(4, 10, n, n, n, n, n, n, 0, n, n, 9.81, 0.0, 0.0, n, n, n, n, n) == E
    assert mg.dg_rhs(1, -1, n, n, n, n, n, n, 0, n, n, 9.81, 0.0, 0.0, n, n, n, n, n) == E
    assert mg.dg_rhs(1, 0, n, n, n, n, n, n, 5, n, n, 9.81, 0.0, 0.0, n, n, n, n, n) == E
    assert mg.dg_rhs(1, 0, n, n, n, n, n, n, -1, n, n, 9.81, 0.0, 0.0, n, n, n, n, n) == E
    assert mg.dg_rhs(1, 0, n, n, n, n, n, n, 0, n, n, 9.81, 0.0, 0.0, n, n, n, n, n) == mg.MG_OK
    assert mg.dg_rhs(1, 10, n, n, n, n, n, n, 0, n, n, 9.81, 0.0, 0.0, n, n, n, n, n) == E
    assert mg.dg_edge_terms(2, 0, n, n, n, n, n, n, 3, n, n, 9.81, n, n, n) == E
    assert mg.dg_edge_terms(2, 0, n, n, n, n, n, n, 0, n, n, 9.81, n, n, n) == mg.MG_OK
    step = lambda k, ne, nb, dt: mg.dg_ssp_rk3_step(k, ne, n, n, n, n, n, n, n, nb, n, n, 9.81, 0.0, 0.0,
                                                    n, n, n, n, dt, n)
    assert step(3, 0, 0, float("nan")) == E
    assert step(3, 0, 2, 0.5) == E
    assert step(7, 0, 0, 0.5) == E
    assert step(3, 0, 0, 0.5) == mg.MG_OK
    assert step(3, 5, 0, 0.5) == E
    assert mg.dg_basis_values(9, 3, n, n, n) == E


@pytest.mark.parametrize("nx,ny,tile", [(3, 4, 0), (5, 5, 0), (8, 12, 4)])
def test_mesh_neighbours_match_the_geometry(nx, ny, tile):
    """The split-quad mesh's neighbour table (row-wise and tiled numbering):
    every element is counter-clockwise, edge q of e (vertex q to q + 1) is
    edge nq of its neighbour traversed backwards, the relation is symmetric,
    and the 2 (nx + ny) boundary edges are the ones without a neighbour."""
    from paper_1904_08684_amd import workloads as W
    B, a1 = W.dg_mesh(nx, ny, with_origin=True, tile=tile)
    nbr, nq = W.dg_mesh_neighbours(nx, ny, tile=tile)
    assert np.all(B[0] * B[3] - B[1] * B[2] > 0)

    def verts(e):
        return [a1[:, e], a1[:, e] + B[[0, 2], e], a1[:, e] + B[[1, 3], e]]
    for e in range(B.shape[1]):
        for q in range(3):
            f, r = int(nbr[q, e]), int(nq[q, e])
            if f < 0:
                continue
            P, Q = verts(e), verts(f)
            assert np.allclose(P[q], Q[(r + 1) % 3]) and np.allclose(P[(q + 1) % 3], Q[r])
            assert nbr[r, f] == e and nq[r, f] == q
    assert int((nbr < 0).sum()) == 2 * (nx + ny)


def test_tiled_numbering_is_a_relabelling():
    """The tiled numbering holds the same elements (maps and origins) as the
    row-wise one, the halves in the same order, and a relabelled neighbour
    table."""
    from paper_1904_08684_amd import workloads as W
    nx, ny, t = 8, 12, 4
    B0, o0 = W.dg_mesh(nx, ny, with_origin=True)
    B1, o1 = W.dg_mesh(nx, ny, with_origin=True, tile=t)
    n0, _ = W.dg_mesh_neighbours(nx, ny)
    n1, _ = W.dg_mesh_neighbours(nx, ny, tile=t)
    half = nx * ny
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    new = W._square_index(i.ravel(), j.ravel(), nx, ny, t)
    perm = np.concatenate([new, half + new])          # row-wise index -> tiled index
    assert sorted(perm.tolist()) == list(range(2 * half))
    np.testing.assert_array_equal(B1[:, perm], B0)
    np.testing.assert_array_equal(o1[:, perm], o0)
    relab = np.where(n0 >= 0, perm[np.maximum(n0, 0)], -1)
    np.testing.assert_array_equal(n1[:, perm], relab)
