"""Pins of the FP64 oracle against facts that the paper and the mathematics
fix, independently of the oracle's own code.

* Frobenius identity: every step is an exact orthogonal change of basis
  (eq. (q)) followed by an exact block elimination (eq. (sm_L)); the only
  inexact operation is dropping the symmetric pair (E_i, E_i^T) (eq. (rreav)).
  The dropped pairs of different steps and levels occupy disjoint entries in
  the final coordinates, so ||A0 - M||_F^2 = 2 sum_i ||E_i||_F^2 exactly.
* eps = 0 keeps every nonzero singular value: M = A0 (Section 2.3 with E=0).
* A block-tridiagonal ordering has no far blocks: CE is textbook block
  Cholesky (eq. (bl_chol)), so L must equal the dense Cholesky factor.
* The rank rule (Remark 2.1, CE(eps)): sigma_{r+1} <= theta < sigma_r, checked
  with eigenvalues of F F^T rather than the SVD the oracle calls.
* Scale invariance, monotonicity in eps, the apply as the inverse of the
  product (Proposition 2.2), PCG with an exact preconditioner, and CG's
  Chebyshev bound with the closed-form spectrum of the Laplacian.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import problems
from oracle import (CEOptions, NotSPD, ce_dense, ce_factor, ce_multiply, ce_solve,
                    grid_order, level1_pattern, pcg, simulate_level, coarsen,
                    coarse_pattern, adjacency, colour_order, live_pairs)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(dims, patch):
    A = problems.laplacian(dims)
    ip, ix, dv = problems.to_csr_arrays(A)
    perm, bp, co = grid_order(dims, patch)
    return A, (ip, ix, dv), perm, bp, co


def _A0(A, perm):
    return A[perm][:, perm].toarray()


CASES = [
    ((16, 16), (4, 4)),
    ((18, 13), (4, 4)),          # ragged: partial patches on both axes
    ((8, 8, 8), (2, 2, 2)),
    ((7, 9, 6), (2, 2, 2)),      # ragged 3D
]


@pytest.mark.parametrize("dims,patch", CASES)
@pytest.mark.parametrize("eps", [1e-2, 1e-5])
@pytest.mark.parametrize("order", ["paper", "multicolour"])
def test_frobenius_identity(dims, patch, eps, order):
    A, csr, perm, bp, co = _setup(dims, patch)
    f = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, order=order, coarse_max_dim=0))
    M = ce_dense(f)
    err = np.linalg.norm(A.toarray() - M)
    pred = math.sqrt(2.0 * f.dropped())
    assert abs(err - pred) <= 1e-8 * pred + 1e-13 * np.linalg.norm(A.toarray()), (err, pred)
    assert len(f.levels) >= 2
    # something was compressed and something was dropped
    assert pred > 0.0


@pytest.mark.parametrize("dims,patch", CASES[:3])
def test_eps_zero_is_exact(dims, patch):
    A, csr, perm, bp, co = _setup(dims, patch)
    f = ce_factor(*csr, perm, bp, co, CEOptions(eps=0.0, coarse_max_dim=0))
    Ad = A.toarray()
    M = ce_dense(f)
    assert np.linalg.norm(Ad - M) <= 1e-13 * np.linalg.norm(Ad)
    b = problems.rhs_uniform(A.shape[0], 0)
    x = ce_solve(f, b)
    xs = np.linalg.solve(Ad, b)
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
    # log det M = 2 sum log diag(L) (Q orthogonal) equals log det A
    ld = 2.0 * sum(np.log(np.diag(L)).sum() for lf in f.levels for L in lf.Lnn if L.size)
    ld += 2.0 * np.log(np.diag(f.coarse_L)).sum()
    sign, ref = np.linalg.slogdet(Ad)
    assert sign > 0 and abs(ld - ref) <= 1e-12 * abs(ref)


def test_block_tridiagonal_order_is_textbook_cholesky():
    """Patches that are whole grid rows give a block-tridiagonal A0 whose
    rows have no far blocks: every step is a full block Cholesky step."""
    n = 12
    A, csr, perm, bp, co = _setup((n, n), (n, 1))
    assert np.array_equal(perm, np.arange(n * n))      # lexicographic rows
    f = ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-3, coarse_max_dim=0))
    lf = f.levels[0]
    # far blocks only couple to fully eliminated rows: they are structurally
    # present but numerically empty, so nothing is ever kept
    assert np.all(lf.r == 0)
    assert all(float(np.max(s, initial=0.0)) == 0.0 for s in lf.sigma)
    L = np.zeros((n * n, n * n))
    for i in lf.order:
        s = slice(bp[i], bp[i + 1])
        L[s, s] = lf.Lnn[i]
        for x, p in lf.panel[i].items():
            if x != i:
                L[bp[x]:bp[x + 1], s] = p
    Lref = np.linalg.cholesky(_A0(A, perm))
    assert np.linalg.norm(L - Lref) <= 1e-13 * np.linalg.norm(Lref)
    assert f.coarse_L.shape == (0, 0)


@pytest.mark.parametrize("dims,patch,eps", [((16, 16), (4, 4), 1e-4), ((8, 8, 8), (2, 2, 2), 1e-3)])
def test_rank_rule_against_gram_eigenvalues(dims, patch, eps):
    A, csr, perm, bp, co = _setup(dims, patch)
    f = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, coarse_max_dim=0, keep_far_rows=True))
    th = f.theta
    nchecked = 0
    for lf in f.levels:
        for i in range(lf.M):
            F = lf.F[i]
            if F is None or F.shape[1] == 0:
                assert lf.r[i] == 0
                continue
            b = F.shape[0]
            ev = np.sort(np.linalg.eigvalsh(F @ F.T))[::-1]
            sig = np.sqrt(np.clip(ev, 0.0, None))
            r = lf.r[i]
            tol = 1e-7 * sig[0]
            if r > 0:
                assert sig[r - 1] > th - tol
            if r < b:
                assert sig[r] <= th + tol
            # dropped part: trailing rows of U^T F
            E = (lf.U[i].T @ F)[r:]
            assert abs(np.sum(E ** 2) - lf.e[i]) <= 1e-10 * max(np.sum(F ** 2), 1e-300)
            if E.size:
                assert np.linalg.norm(E, 2) <= th * (1 + 1e-8) + 1e-14 * sig[0]
            nchecked += 1
    assert nchecked > 10


def test_scale_invariance():
    A, csr, perm, bp, co = _setup((16, 16), (4, 4))
    c = 37.5
    f1 = ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-4, coarse_max_dim=0))
    f2 = ce_factor(csr[0], csr[1], c * csr[2], perm, bp, co, CEOptions(eps=1e-4, coarse_max_dim=0))
    for r1, r2 in zip(f1.ranks(), f2.ranks()):
        assert np.array_equal(r1, r2)
    M1, M2 = ce_dense(f1), ce_dense(f2)
    assert np.linalg.norm(M2 - c * M1) <= 1e-12 * np.linalg.norm(M2)


def test_monotone_in_eps():
    A, csr, perm, bp, co = _setup((24, 24), (4, 4))
    Ad = A.toarray()
    errs, kept = [], []
    for eps in [1e-2, 1e-4, 1e-6, 1e-8]:
        f = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, coarse_max_dim=0))
        errs.append(np.linalg.norm(Ad - ce_dense(f)))
        kept.append(sum(int(r.sum()) for r in f.ranks()))
    assert all(errs[k + 1] < errs[k] for k in range(3)), errs
    assert all(kept[k + 1] >= kept[k] for k in range(3)), kept


@pytest.mark.parametrize("order", ["paper", "multicolour"])
def test_solve_inverts_multiply(order):
    A, csr, perm, bp, co = _setup((20, 17), (4, 4))
    f = ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-3, order=order, coarse_max_dim=40))
    X = np.random.default_rng(12345).standard_normal((A.shape[0], 3))
    Y = ce_multiply(f, X)
    Z = ce_solve(f, Y)
    assert np.linalg.norm(Z - X) <= 1e-11 * np.linalg.norm(X)
    # the dense M agrees with the multiply and is symmetric positive definite
    M = ce_dense(f)
    assert np.linalg.norm(M - M.T) <= 1e-14 * np.linalg.norm(M)
    assert np.linalg.eigvalsh(M).min() > 0


def test_pcg_exact_preconditioner_one_iteration():
    A, csr, perm, bp, co = _setup((16, 16), (4, 4))
    f = ce_factor(*csr, perm, bp, co, CEOptions(eps=0.0, coarse_max_dim=0))
    b = problems.rhs_uniform(A.shape[0], 0)
    x, it, rel = pcg(A, b, lambda r: ce_solve(f, r), tol=1e-10)
    assert it == 1 and rel <= 1e-10


def test_cg_chebyshev_bound():
    n = 30
    A = problems.laplacian((n, n))
    lmin = 4 - 4 * math.cos(math.pi / (n + 1))
    lmax = 4 + 4 * math.cos(math.pi / (n + 1))
    ev = np.linalg.eigvalsh(A.toarray())
    assert abs(ev[0] - lmin) < 1e-12 and abs(ev[-1] - lmax) < 1e-12
    kappa = lmax / lmin
    rho = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    b = problems.rhs_uniform(n * n, 0)
    xs = np.linalg.solve(A.toarray(), b)
    e0 = math.sqrt(xs @ (A @ xs))
    for k in [5, 20, 40]:
        x, it, _ = pcg(A, b, lambda r: r, tol=0.0, maxit=k)
        ek = math.sqrt((x - xs) @ (A @ (x - xs)))
        assert it == k
        assert ek <= 2 * rho ** k * e0 * (1 + 1e-9)


def test_ce_preconditioner_beats_cg_and_improves_with_eps():
    A, csr, perm, bp, co = _setup((48, 48), (4, 4))
    b = problems.rhs_uniform(A.shape[0], 0)
    _, it_none, _ = pcg(A, b, lambda r: r, tol=1e-8)
    its = []
    for eps in [1e-1, 1e-3, 1e-6]:
        f = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps))
        _, it, rel = pcg(A, b, lambda r: ce_solve(f, r), tol=1e-8)
        assert rel <= 1e-8
        its.append(it)
    assert its[0] < it_none
    assert its[0] >= its[1] >= its[2]


def test_indefinite_matrix_reports_not_spd():
    A, csr, perm, bp, co = _setup((8, 8), (4, 4))
    bad = csr[2].copy()
    bad[csr[1] == np.repeat(np.arange(64), np.diff(csr[0]))] -= 5.0     # shift the diagonal
    with pytest.raises(NotSPD):
        ce_factor(csr[0], csr[1], bad, perm, bp, co, CEOptions(eps=1e-6, coarse_max_dim=0))


# ----------------------------------------------------------- symbolic ----

def test_morton_patch_order_small():
    perm, bp, co = grid_order((4, 4), (2, 2))
    # patches (0,0),(1,0),(0,1),(1,1) in Z order; points x fastest inside
    assert perm.tolist() == [0, 1, 4, 5, 2, 3, 6, 7, 8, 9, 12, 13, 10, 11, 14, 15]
    assert bp.tolist() == [0, 4, 8, 12, 16]
    assert co.tolist() == [[0, 0], [1, 0], [0, 1], [1, 1]]
    perm3, bp3, co3 = grid_order((2, 2, 2), (1, 1, 1))
    assert perm3.tolist() == list(range(8))         # Z order of 2x2x2 = natural order


def _far_superset_count_2d(n):
    # distance-2 pairs of the n x n grid graph: offsets (2,0),(0,2),(1,1),(1,-1)
    return 2 * n * (n - 2) + 2 * (n - 1) ** 2


@pytest.mark.parametrize("order", ["paper", "multicolour"])
def test_level_counts_64x64(order):
    """Per-level block counts on the 64x64 grid with 4x4 patches: the close
    pattern is the 5-point graph of the patch grid at level 1 and the 9-point
    graph after squaring and coarsening (Proposition on tensor grids)."""
    A, csr, perm, bp, co = _setup((64, 64), (4, 4))
    pairs = level1_pattern(*csr[:2], perm, bp)
    M = 256
    assert len(pairs) == 2 * 16 * 15
    coords = co
    # close pairs of the 5-point (level 1) and at most the 9-point graph later
    bound_close = [480, 210, 42, 6]
    Ms = [M]
    for lev in range(4):
        assert len(pairs) == bound_close[lev] if lev == 0 else len(pairs) <= bound_close[lev]
        adj = adjacency(M, pairs)
        order_l = list(range(M)) if order == "paper" else colour_order(adj, coords)[0]
        _, far, removed = simulate_level(M, pairs, order_l)
        # far pattern is inside pattern(A^2) \ pattern(A)
        d2 = set()
        for i in range(M):
            for c in adj[i]:
                for d in adj[c]:
                    if d != i and d not in adj[i]:
                        d2.add((min(i, d), max(i, d)))
        assert set(far) <= d2
        if lev == 0:
            assert len(d2) == _far_superset_count_2d(16) == 898
        prev = np.asarray(coords)
        parent, coords = coarsen(coords)
        # every super-block joins exactly the 2^2 Morton siblings: the blocks
        # whose patch coordinates agree after dropping the lowest bit
        for P in range(int(parent.max()) + 1):
            kids = np.flatnonzero(parent == P)
            assert len(kids) == 4 and np.all(np.diff(kids) == 1)
            assert np.all((prev[kids] >> 1) == coords[P])
            assert sorted(map(tuple, prev[kids] & 1)) == [(0, 0), (0, 1), (1, 0), (1, 1)]
        pairs = coarse_pattern(parent, live_pairs(sorted(set(pairs) | set(far)), removed))
        M = int(parent.max()) + 1
        Ms.append(M)
    # 16^2 patches -> 8^2 -> 4^2 -> 2^2 -> 1 (J = 4 siblings per level)
    assert Ms == [256, 64, 16, 4, 1]


def test_far_blocks_are_in_block_pattern_of_A_squared():
    """Brute force: the far blocks lie in bsp(A0)^2 minus bsp(A0), the
    block pattern of A0 squared as a boolean matrix product (the remark
    after eq. (sm_L) and the bound bsp(A1) <= bsp(A0^2) of Section 2.5)."""
    A, csr, perm, bp, co = _setup((16, 16), (4, 4))
    f = ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-6, coarse_max_dim=0))
    A0 = _A0(A, perm)
    M = len(bp) - 1
    Bp = np.zeros((M, M), dtype=np.int64)
    for p in range(M):
        for q in range(M):
            Bp[p, q] = int(np.any(A0[bp[p]:bp[p + 1], bp[q]:bp[q + 1]] != 0))
    B2 = (Bp @ Bp) > 0
    for p, q in f.levels[0].far_pairs:
        assert B2[p, q] and not Bp[p, q]
    # eq. (L): the factor of level 1 has at most 2 #blocks(A0) nonzero blocks
    nblk_A0 = int(Bp.sum())
    nblk_L1 = sum(1 + len([x for x in f.levels[0].panel[i] if x != i]) for i in range(M))
    assert nblk_L1 <= 2 * nblk_A0
    # bsp(A1) <= bsp(A0^2): blocks of the remainder (level-1 indices) couple
    # only pairs that are in the pattern of A0^2
    for p, q in f.levels[0].far_pairs + f.levels[0].close_pairs:
        assert B2[p, q]


def test_four_node_example():
    g = json.load(open(os.path.join(GOLDEN, "four_node_example.json")))
    nb, B = g["blocks"], 3
    rng = np.random.default_rng(7)
    N = nb * B
    A0 = np.zeros((N, N))
    for a, c in g["edges_1based"]:
        blk = rng.uniform(-0.3, 0.3, (B, B))
        A0[(a - 1) * B:a * B, (c - 1) * B:c * B] = blk
        A0[(c - 1) * B:c * B, (a - 1) * B:a * B] = blk.T
    A0 += np.diag(np.full(N, 4.0))
    S = sp.csr_matrix(A0)
    S.sort_indices()
    bp = np.arange(0, N + 1, B)
    f = ce_factor(S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data, np.arange(N),
                  bp, None, CEOptions(eps=1e-12, coarse_max_dim=0, max_levels=1), J=4)
    lf = f.levels[0]
    assert [[p + 1, q + 1] for p, q in lf.far_pairs] == g["far_edges_after_pass_1based"]
    for blk in g["blocks_with_empty_far_row_1based"]:
        assert lf.r[blk - 1] == 0
    # remainder: only blocks 2 and 4 keep unknowns, coupled through the far block
    assert lf.r[1] > 0 and lf.r[3] > 0
    # ||A0 - M|| = sqrt(2 sum e)
    M = ce_dense(f)
    assert abs(np.linalg.norm(A0 - M) - math.sqrt(2 * f.dropped())) <= 1e-12


def _biharmonic(n):
    L = problems.laplacian((n, n))
    B = (L @ L).tocsr()
    B.sort_indices()
    return B


def test_compensation_keeps_m_minus_a_psd_and_prevents_breakdown():
    """Diagonal compensation adds, per dropped far block E, the positive
    semidefinite [[e I, -E], [-E^T, e I]] (e = ||E||_F >= ||E||_2) to A0, so
    M - A0 is positive semidefinite and no pivot can fail.  The biharmonic
    operator (not an M-matrix) breaks the plain method at eps = 1e-3."""
    B = _biharmonic(32)
    csr = problems.to_csr_arrays(B)
    perm, bp, co = oracle.grid_order((32, 32), (4, 4))
    with pytest.raises(oracle.NotSPD):
        ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-3, order="multicolour", coarse_max_dim=0))
    f = ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-3, order="multicolour", coarse_max_dim=0, compensate=True))
    M = ce_dense(f)
    Bd = B.toarray()
    assert np.linalg.eigvalsh(M - Bd)[0] >= -1e-12 * np.linalg.norm(Bd)
    assert np.linalg.norm(M - Bd) > 0
    b = problems.rhs_uniform(B.shape[0])
    _, it, rel = oracle.pcg(B, b, lambda r: ce_solve(f, r), tol=1e-8)
    assert rel <= 1e-8 and it < 100


def test_compensation_vanishes_at_eps_zero():
    B = _biharmonic(16)
    csr = problems.to_csr_arrays(B)
    perm, bp, co = oracle.grid_order((16, 16), (4, 4))
    f = ce_factor(*csr, perm, bp, co, CEOptions(eps=0.0, order="multicolour", coarse_max_dim=0, compensate=True))
    assert np.linalg.norm(ce_dense(f) - B.toarray()) <= 1e-12 * np.linalg.norm(B.toarray())
