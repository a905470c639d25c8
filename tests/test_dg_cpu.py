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


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_edge_tables_match_quadrature(mg, k):
    """The exact edge integrals (own edge, and the neighbour's edge traversed
    backwards) against Gauss quadrature of the oracle's basis; tables of
    order max(k, 1)."""
    K = dg.KB_OF[k]
    T = mg.dg_edge_table(k)
    t, w = np.polynomial.legendre.leggauss(8)
    s = (t + 1.0) / 2.0
    w = w / 2.0
    lin = {0: (0, 1, 0, 0), 1: (1, -1, 0, 1), 2: (0, 0, 1, -1)}

    def at(q, back):
        x0, xs, y0, ys = lin[q]
        ss = 1.0 - s if back else s
        return np.array(dg.basis(x0 + xs * ss, y0 + ys * ss))[:K]
    for q in range(3):
        ph = at(q, False)
        assert np.max(np.abs(T["O2"][q] - (ph * w) @ ph.T)) <= 1e-12
        assert np.max(np.abs(T["O3"][q] - np.einsum("pq,iq,mq->pim", ph * w, ph, ph))) <= 1e-12
        for r in range(3):
            pb = at(r, True)
            assert np.max(np.abs(T["N2"][q, r] - (ph * w) @ pb.T)) <= 1e-12
            assert np.max(np.abs(T["N3"][q, r] - np.einsum("pq,iq,mq->pim", ph * w, pb, pb))) <= 1e-12
    assert mg.dg_edge_table_size(k) == 12 * K * K + 12 * K ** 3


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
