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
    G, H = mg.dg_reference(k)
    K = dg.K_OF[k]
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
    assert [mg.dg_reference_size(k) for k in range(4)] == [2 * K * K + 2 * K ** 3 for K in (1, 3, 6, 10)]
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
    backwards) against Gauss quadrature of the oracle's basis."""
    K = dg.K_OF[k]
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
