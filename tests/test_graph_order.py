"""Nested-bisection ordering of a general sparse graph (host, CPU): a
permutation, blocks of at most B at one uniform depth, the path graph cut
into intervals, and the analysis with pairs of blocks (J = 2) bit-exact with
the oracle's symbolic levels."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import problems


def _cae():
    import paper_1603_09133_amd as cae
    cae.lib()
    return cae


@pytest.mark.parametrize("B", [4, 16, 64])
def test_graph_order_blocks_and_permutation(B):
    cae = _cae()
    A = problems.disk_laplacian(40)
    ip, ix, _ = problems.to_csr_arrays(A)
    perm, bp = cae.graph_order(ip, ix, B)
    n = A.shape[0]
    assert np.array_equal(np.sort(perm), np.arange(n))
    sizes = np.diff(bp)
    assert sizes.max() <= B and sizes.min() >= 1
    nb = len(sizes)
    assert nb & (nb - 1) == 0                       # uniform depth
    assert nb >= -(-n // B)


def test_graph_order_cuts_a_path_into_intervals():
    cae = _cae()
    n = 100
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    A.sort_indices()
    ip, ix, _ = problems.to_csr_arrays(A)
    perm, bp = cae.graph_order(ip, ix, 16)
    for k in range(len(bp) - 1):
        blk = np.sort(perm[bp[k]:bp[k + 1]])
        assert np.all(np.diff(blk) == 1)


@pytest.mark.parametrize("order", ["paper", "multicolour"])
def test_graph_ordered_analysis_matches_oracle(order):
    cae = _cae()
    A = problems.disk_laplacian(30)
    ip, ix, _ = problems.to_csr_arrays(A)
    perm, bp = cae.graph_order(ip, ix, 16)
    an = cae.Analysis(ip, ix, perm, bp, None, order=cae.ORDER_PAPER if order == "paper" else cae.ORDER_MULTICOLOUR,
                      ndim=1)
    M = len(bp) - 1
    pairs = oracle.level1_pattern(ip, ix, perm, bp)
    for lvl in range(an.nlevels()):
        arr = an.level_arrays(lvl)
        inf = an.level_info(lvl)
        assert inf["M"] == M
        ad = oracle.adjacency(M, pairs)
        orc_order = oracle.element_order(ad, order, None)
        assert np.array_equal(arr["order"], np.asarray(orc_order))
        far, farp, removed = oracle.simulate_level(M, pairs, orc_order)
        assert sorted(map(tuple, arr["far_pairs"].tolist())) == sorted(map(tuple, farp))
        if M == 1:
            break
        parent, _ = oracle.coarsen(None, M, 2)
        assert np.array_equal(arr["parent"], parent)
        pairs = oracle.coarse_pattern(parent, oracle.live_pairs(sorted(set(map(tuple, pairs)) | set(farp)), removed))
        M = int(parent.max()) + 1
    an.close()
