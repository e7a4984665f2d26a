"""Joining independent problems into one analysis (host side, CPU): the
joint blocks keep every problem's Morton order, the analysis accepts the
joint coordinates, no close or far pair couples two problems, and the
symbolic levels equal the oracle's on the joint problem."""
import numpy as np
import pytest

import oracle
import problems


def _batch():
    from paper_1603_09133_amd import batched
    mats, dims, patches = [], [], []
    for kind, side in [(0, 24), (1, 8), (0, 17), (1, 6), (0, 32)]:
        d = (side, side) if kind == 0 else (side, side, side)
        mats.append(problems.laplacian(d))
        dims.append(d)
        patches.append((4, 4) if kind == 0 else (2, 2, 2))
    return batched.assemble(mats, dims, patches)


def test_joint_problem_is_block_diagonal_and_morton_ordered():
    import paper_1603_09133_amd as cae
    A, perm, bp, co, off = _batch()
    assert A.shape[0] == off[-1]
    # the permutation maps every block into one problem's rows
    which = np.searchsorted(off, perm, side="right") - 1
    for k in range(len(bp) - 1):
        assert len(set(which[bp[k]:bp[k + 1]])) == 1
    an = cae.Analysis(*problems.to_csr_arrays(A)[:2], perm, bp, co)
    info = an.level_info(0)
    assert info["M"] == len(bp) - 1
    arr = an.level_arrays(0)
    blk_prob = np.array([which[bp[k]] for k in range(len(bp) - 1)])
    for p, q in np.concatenate([arr["close_pairs"], arr["far_pairs"]]):
        assert blk_prob[p] == blk_prob[q]
    an.close()


def test_joint_symbolic_matches_oracle():
    import paper_1603_09133_amd as cae
    A, perm, bp, co, off = _batch()
    ip, ix, _ = problems.to_csr_arrays(A)
    an = cae.Analysis(ip, ix, perm, bp, co)
    ad = oracle.adjacency(len(bp) - 1, oracle.level1_pattern(ip, ix, perm, bp))
    order = oracle.element_order(ad, "multicolour", co)
    arr = an.level_arrays(0)
    assert np.array_equal(arr["order"], np.asarray(order))
    an.close()
