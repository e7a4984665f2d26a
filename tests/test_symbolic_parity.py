"""The C ABI library loads, exports every declared symbol, and its host
symbolic analysis is bit-exact with the oracle's (CPU only, no GPU call):
permutation and blocks, close pattern, elimination order, created far
blocks, removed blocks and coarsening of every level; the dependency waves
keep the order of every pair of steps at block-graph distance <= 2."""
import os
import re

import numpy as np
import pytest

import problems
import oracle
from oracle import symbolic as osym

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1603_09133_amd", "libcae.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcae.so not built")


def test_exports_every_declared_symbol():
    import ctypes
    hdr = open(os.path.join(ROOT, "include", "cae.h")).read()
    names = set(re.findall(r"(?:int|void|char\s*\*)\s+(cae_[a-z_0-9]+)\s*\(", hdr))
    L = ctypes.CDLL(LIB)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert {"cae_factor_numeric", "cae_apply_precond", "cae_pcg_solve", "cae_analyze"} <= names


GRIDS = [((64, 64), (4, 4)), ((18, 13), (4, 4)), ((40, 24), (8, 8)), ((8, 8, 8), (2, 2, 2)),
         ((7, 9, 6), (2, 2, 2)), ((12, 12, 12), (4, 4, 4))]


@pytest.mark.parametrize("dims,patch", GRIDS)
def test_grid_order_bit_exact(dims, patch):
    import paper_1603_09133_amd as cae
    perm, bp, co = cae.grid_order(dims, patch)
    operm, obp, oco = oracle.grid_order(dims, patch)
    assert np.array_equal(perm, operm) and np.array_equal(bp, obp) and np.array_equal(co, oco)


def _oracle_levels(csr, perm, bp, co, order):
    """Structural levels by the oracle's own symbolic functions."""
    pairs = osym.level1_pattern(*csr[:2], perm, bp)
    M = len(bp) - 1
    coords = co
    out = []
    while True:
        adj = osym.adjacency(M, pairs)
        ordl = osym.element_order(adj, order, coords) if M > 1 else [0]
        _, far, removed = osym.simulate_level(M, pairs, ordl)
        lev = dict(M=M, close=pairs, order=ordl, far=far, removed=removed)
        out.append(lev)
        if M == 1:
            break
        parent, coords = osym.coarsen(coords)
        lev["parent"] = parent
        pairs = osym.coarse_pattern(parent, osym.live_pairs(sorted(set(pairs) | set(far)), removed))
        M = int(parent.max()) + 1
    return out


@pytest.mark.parametrize("dims,patch", GRIDS)
@pytest.mark.parametrize("order", ["paper", "multicolour"])
def test_levels_bit_exact(dims, patch, order):
    import paper_1603_09133_amd as cae
    A = problems.laplacian(dims)
    csr = problems.to_csr_arrays(A)
    perm, bp, co = cae.grid_order(dims, patch)
    an = cae.Analysis(csr[0], csr[1], perm, bp, co,
                      order=cae.ORDER_PAPER if order == "paper" else cae.ORDER_MULTICOLOUR)
    ref = _oracle_levels(csr, perm.astype(np.int64), bp.astype(np.int64), co.astype(np.int64), order)
    assert an.nlevels() == len(ref)
    for l, lev in enumerate(ref):
        arr = an.level_arrays(l)
        assert an.level_info(l)["M"] == lev["M"]
        assert [tuple(x) for x in arr["close_pairs"].tolist()] == [tuple(map(int, p)) for p in lev["close"]]
        assert arr["order"].tolist() == list(lev["order"])
        assert [tuple(x) for x in arr["far_pairs"].tolist()] == [tuple(map(int, p)) for p in lev["far"]]
        assert set(np.nonzero(arr["removed"])[0].tolist()) == set(lev["removed"])
        if "parent" in lev:
            assert arr["parent"].tolist() == lev["parent"].tolist()
        # waves: steps within distance 2 keep their order and differ in wave
        M = lev["M"]
        adj = osym.adjacency(M, lev["close"])
        d2 = osym.distance2_sets(adj)
        pos = {b: k for k, b in enumerate(lev["order"])}
        w = arr["wave"]
        for i in range(M):
            for j in d2[i]:
                if pos[j] < pos[i]:
                    assert w[j] < w[i]


def test_uniform_blocks_and_errors():
    import paper_1603_09133_amd as cae
    A = problems.laplacian((10, 10))
    csr = problems.to_csr_arrays(A)
    an = cae.Analysis(csr[0], csr[1], np.arange(100), None, None, B=7, order=cae.ORDER_PAPER)
    assert an.level_info(0)["M"] == 15
    with pytest.raises(cae.CAEError):
        cae.Analysis(csr[0], csr[1], np.zeros(100), None, None, B=7)        # not a permutation
    with pytest.raises(cae.CAEError):
        cae.Analysis(csr[0], csr[1], np.arange(100), [0, 50, 99], None)      # blocks do not span n


@pytest.mark.parametrize("dims,patch", [((16, 16, 16), (4, 4, 4)), ((12, 10), (4, 4)), ((10, 9, 7), (2, 2, 2))])
def test_pairs_coarsening_matches_oracle(dims, patch):
    """Coarsening by pairs along the Morton curve (axes in turn): parents and
    levels bit-exact with the oracle's twin."""
    import paper_1603_09133_amd as cae
    A = problems.laplacian(dims)
    ip, ix, _ = problems.to_csr_arrays(A)
    perm, bp, co = osym.grid_order(dims, patch)
    an = cae.Analysis(ip, ix, perm, bp, co, order=cae.ORDER_PAPER, coarsen="pairs")
    coords = np.asarray(co)
    M = len(bp) - 1
    pairs = osym.level1_pattern(ip, ix, perm, bp)
    for lvl in range(an.nlevels()):
        arr = an.level_arrays(lvl)
        order = osym.element_order(osym.adjacency(M, pairs), "paper", coords)
        assert np.array_equal(arr["order"], np.asarray(order))
        far, farp, removed = osym.simulate_level(M, pairs, order)
        if M == 1:
            break
        parent, coords = osym.coarsen(coords, M, None, axis=lvl % coords.shape[1])
        assert np.array_equal(arr["parent"], parent), lvl
        pairs = osym.coarse_pattern(parent, osym.live_pairs(sorted(set(map(tuple, pairs)) | set(farp)), removed))
        M = int(parent.max()) + 1
    an.close()
