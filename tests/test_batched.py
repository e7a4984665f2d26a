"""Joining independent problems into one analysis (host side, CPU,
``cae_analyze_batched``): the joint blocks keep every problem's Morton order,
problem by problem; no close or far pair couples two problems; the analysis
equals that of the joint matrix assembled here from the documented rule (block
diagonal, rows stacked, block coordinates offset by the problem index's
binary digits dealt to the three axes above 8 bits); and the symbolic order
equals the oracle's on the joint problem."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import problems

SPEC = [(0, 24, (4, 4)), (1, 8, (2, 2, 2)), (0, 17, (4, 4)), (1, 6, (2, 2, 2)), (0, 32, (4, 4))]


def _mats():
    mats, dims, patches = [], [], []
    for kind, side, patch in SPEC:
        d = (side, side) if kind == 0 else (side, side, side)
        mats.append(problems.laplacian(d).tocsr())
        dims.append(d)
        patches.append(patch)
    return mats, dims, patches


def _offset(t):
    out = [0, 0, 0]
    bit = 0
    while t >> bit:
        out[bit % 3] |= ((t >> bit) & 1) << (bit // 3)
        bit += 1
    return [o << 8 for o in out]


def _joint_here(mats, dims, patches):
    """The joint problem assembled in the test from the documented rule."""
    import paper_1603_09133_amd as cae
    perms, bps, cos, off = [], [], [], [0]
    for t, (A, d, patch) in enumerate(zip(mats, dims, patches)):
        p, bp, co = cae.grid_order(d, patch)
        co = np.concatenate([co, np.zeros((co.shape[0], 3 - co.shape[1]), np.int32)], axis=1)
        perms.append(p.astype(np.int64) + off[-1])
        bps.append(bp[:-1].astype(np.int64) + off[-1])
        cos.append(co + np.array(_offset(t), np.int32))
        off.append(off[-1] + A.shape[0])
    A = sp.block_diag(mats, format="csr")
    A.sort_indices()
    return (A, np.concatenate(perms).astype(np.int32),
            np.concatenate(bps + [np.array([off[-1]])]).astype(np.int32), np.concatenate(cos).astype(np.int32),
            np.array(off, np.int64))


def test_joint_problem_is_block_diagonal_and_morton_ordered():
    from paper_1603_09133_amd import batched
    mats, dims, patches = _mats()
    an = batched.analyze(mats, dims, patches)
    off = an.batch_rows()
    assert np.array_equal(off, np.concatenate([[0], np.cumsum([m.shape[0] for m in mats])]))
    perm, bp = an.perm()
    which = np.searchsorted(off, perm, side="right") - 1
    blk_prob = np.array([which[bp[k]] for k in range(len(bp) - 1)])
    for k in range(len(bp) - 1):
        assert len(set(which[bp[k]:bp[k + 1]])) == 1
    # problem by problem, in problem order
    assert np.all(np.diff(blk_prob) >= 0)
    for lev in range(an.nlevels()):
        arr = an.level_arrays(lev)
        if lev == 0:
            for p, q in np.concatenate([arr["close_pairs"], arr["far_pairs"]]):
                assert blk_prob[p] == blk_prob[q]
    an.close()


def test_batched_analysis_equals_the_documented_assembly():
    import paper_1603_09133_amd as cae
    from paper_1603_09133_amd import batched
    mats, dims, patches = _mats()
    an = batched.analyze(mats, dims, patches)
    A, perm, bp, co, off = _joint_here(mats, dims, patches)
    ip, ix, _ = problems.to_csr_arrays(A)
    ref = cae.Analysis(ip, ix, perm, bp, co)
    p1, b1 = an.perm()
    assert np.array_equal(p1, perm) and np.array_equal(b1, bp)
    assert an.nlevels() == ref.nlevels()
    for lev in range(ref.nlevels()):
        assert an.level_info(lev) == ref.level_info(lev), lev
        x, y = an.level_arrays(lev), ref.level_arrays(lev)
        for k in x:
            assert np.array_equal(x[k], y[k]), (lev, k)
    an.close()
    ref.close()


def test_joint_symbolic_matches_oracle():
    from paper_1603_09133_amd import batched
    mats, dims, patches = _mats()
    an = batched.analyze(mats, dims, patches)
    A, perm, bp, co, off = _joint_here(mats, dims, patches)
    ip, ix, _ = problems.to_csr_arrays(A)
    ad = oracle.adjacency(len(bp) - 1, oracle.level1_pattern(ip, ix, perm, bp))
    order = oracle.element_order(ad, "multicolour", co)
    arr = an.level_arrays(0)
    assert np.array_equal(arr["order"], np.asarray(order))
    an.close()


def test_batched_analysis_rejects_bad_problems():
    import paper_1603_09133_amd as cae
    from paper_1603_09133_amd import batched
    mats, dims, patches = _mats()
    with pytest.raises(cae.CAEError, match="problem 1"):
        batched.analyze(mats[:2], [dims[0], (9, 9, 9)], patches[:2])   # n is not the product of dims
    big = problems.laplacian((1100, 4)).tocsr()
    with pytest.raises(cae.CAEError, match="256 patches"):
        batched.analyze([big], [(1100, 4)], [(4, 4)])


def test_analysis_of_one_matrix_reports_one_problem():
    import paper_1603_09133_amd as cae
    A = problems.laplacian((16, 16))
    ip, ix, _ = problems.to_csr_arrays(A)
    perm, bp, co = cae.grid_order((16, 16), (4, 4))
    an = cae.Analysis(ip, ix, perm, bp, co)
    assert an.batch_rows().tolist() == [0, A.shape[0]]
    an.close()
