"""A batch of independent problems factored in one joint analysis equals the
problems factored one by one with the same threshold theta = eps * max diag
of the joint matrix (block-diagonal independence, FP64, M X per problem to
1e-10), and each problem's block of the joint factor equals the FP64
oracle's factorization of that problem (M X to 1e-10 where every block has
at most 128 unknowns; 5e-8 for a 3D problem whose second level holds blocks
of up to 215 unknowns, whose compression decides the kept subspace from the
Gram matrix with the pivots stopped at a trailing energy of (theta/32)^2, a
perturbation of the kept subspaces of that order over the spectral gap
(measured 1.1e-8)); every problem's PCG
residual reaches the tolerance in an independent PCG per problem, and the
autotuner picks and caches a patch shape."""
import json

import numpy as np
import pytest

import oracle
import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cae():
    import paper_1603_09133_amd as cae
    cae.lib()
    return cae


def test_batch_equals_individual_factorizations():
    cae = _cae()
    from paper_1603_09133_amd import batched
    spec = [(0, 40, (8, 8)), (1, 12, (4, 4, 4)), (0, 33, (4, 4)), (1, 8, (2, 2, 4)), (0, 64, (8, 8)),
            (1, 20, (4, 4, 4))]
    mats, dims, patches = [], [], []
    for kind, side, patch in spec:
        d = (side, side) if kind == 0 else (side,) * 3
        mats.append(problems.laplacian(d))
        dims.append(d)
        patches.append(patch)
    eps = 1e-6
    # both run every level down to one block in the block order of Algorithm 2
    # (the multicolour order of a 2D problem differs once it sits among 3D
    # ones), so every problem sees the same compressions; the joint analysis
    # only adds exact eliminations of single-block problems
    bt = batched.Batch(mats, dims, patches, eps, precision=cae.FP64, order=cae.ORDER_PAPER, coarse_max_dim=0)
    bt.factorize()
    N = int(bt.row_off[-1])
    X = np.random.default_rng(12345).standard_normal((N, 3))
    MX = bt.factor.multiply(torch.from_numpy(np.ascontiguousarray(X.T)).cuda()).cpu().numpy().T
    tau = max(A.diagonal().max() for A in mats)
    for t, (A, d, patch) in enumerate(zip(mats, dims, patches)):
        s = slice(bt.row_off[t], bt.row_off[t + 1])
        perm, bp, co = cae.grid_order(d, patch)
        ip, ix, dv = problems.to_csr_arrays(A)
        an = cae.Analysis(ip, ix, perm, bp, co, order=cae.ORDER_PAPER)
        # the joint threshold is eps * max diag of the joint matrix
        eps_t = eps * tau / A.diagonal().max()
        f = cae.Factor(an, torch.from_numpy(dv).cuda(), eps_t, precision=cae.FP64, coarse_max_dim=0)
        Mt = f.multiply(torch.from_numpy(np.ascontiguousarray(X[s].T)).cuda()).cpu().numpy().T
        assert np.linalg.norm(MX[s] - Mt) <= 1e-10 * np.linalg.norm(Mt), t
        bmax = max(int(f.sizes(l).max()) for l in range(f.stats()["nlevels"]))
        f.close()
        an.close()
        fo = oracle.ce_factor(ip, ix, dv, perm.astype(np.int64), bp.astype(np.int64), co.astype(np.int64),
                              oracle.CEOptions(eps=eps_t, order="paper", coarse_max_dim=0))
        Mo = oracle.ce_multiply(fo, X[s])
        err = np.linalg.norm(MX[s] - Mo) / np.linalg.norm(Mo)
        print(f"problem {t} ({d}, largest block {bmax}): joint factor vs oracle {err:.2e}")
        assert err <= (1e-10 if bmax <= 128 else 5e-8), (t, err)
    B = torch.from_numpy(np.ascontiguousarray(problems.rhs_normal(N, 4, seed=1).T)).cuda()
    x, it, rel = bt.pcg(B, rtol=1e-10)
    assert it.shape == (len(mats), 4)
    res = bt.problem_residuals(B, x)
    # every (problem, column) stops at its own residual: the true residual
    # over the problem's rows is at the tolerance (up to the gap between the
    # recurrence and the true residual)
    assert res.max() <= 2e-10, res.max()
    assert np.allclose(rel, res, rtol=1e-3, atol=1e-14)
    bt.close()


def test_batched_pcg_runs_each_problem_as_alone():
    """cae_factor_batched equals the numeric factorization of the batched
    analysis with stacked values (M X bitwise), and cae_pcg_solve_batched
    gives every problem the iteration count of a PCG on that problem alone
    with its own factor (the joint factor's blocks equal the individual
    factors to rounding; the count may move by one at the stopping test)."""
    cae = _cae()
    from paper_1603_09133_amd import batched
    spec = [(0, 48, (8, 8)), (1, 16, (4, 4, 4)), (0, 20, (4, 4)), (1, 12, (2, 2, 4)), (0, 64, (8, 8))]
    mats, dims, patches = [], [], []
    for kind, side, patch in spec:
        d = (side, side) if kind == 0 else (side,) * 3
        mats.append(problems.laplacian(d).tocsr())
        dims.append(d)
        patches.append(patch)
    eps = 1e-4
    # every level down to one block in the block order of Algorithm 2, alone
    # and in the batch, so both see the same compressions
    kw = dict(precision=cae.FP64, coarse_max_dim=0)
    bt = batched.Batch(mats, dims, patches, eps, order=cae.ORDER_PAPER, **kw)
    f = bt.factorize()
    N = int(bt.row_off[-1])
    an = batched.analyze(mats, dims, patches, order=cae.ORDER_PAPER)
    g = cae.Factor(an, batched.stacked_values(mats), eps, **kw)
    X = torch.from_numpy(np.random.default_rng(7).standard_normal((2, N))).cuda()
    assert torch.equal(f.multiply(X), g.multiply(X))
    g.close()
    B = torch.from_numpy(np.ascontiguousarray(problems.rhs_normal(N, 3, seed=5).T)).cuda()
    x, it, rel = bt.pcg(B, rtol=1e-8)
    tau = max(A.diagonal().max() for A in mats)
    for t, (A, d, patch) in enumerate(zip(mats, dims, patches)):
        s = slice(bt.row_off[t], bt.row_off[t + 1])
        perm, bp, co = cae.grid_order(d, patch)
        ip, ix, dv = problems.to_csr_arrays(A)
        a1 = cae.Analysis(ip, ix, perm, bp, co, order=cae.ORDER_PAPER)
        f1 = cae.Factor(a1, torch.from_numpy(dv).cuda(), eps * tau / A.diagonal().max(), **kw)
        _, it1, rel1 = f1.pcg(B[:, s].contiguous(), rtol=1e-8)
        print(f"problem {t} {d}: batched {it[t].tolist()} alone {it1.tolist()}")
        assert np.all(np.abs(it[t] - it1) <= 1), (t, it[t], it1)
        assert rel[t].max() <= 1.001e-8
        f1.close()
        a1.close()
    # a handle of one matrix has no problems to run apart
    ip, ix, dv = problems.to_csr_arrays(mats[0])
    perm, bp, co = cae.grid_order(dims[0], patches[0])
    a1 = cae.Analysis(ip, ix, perm, bp, co)
    f1 = cae.Factor(a1, torch.from_numpy(dv).cuda(), eps, precision=cae.FP64)
    with pytest.raises(cae.CAEError, match="batch"):
        f1.row_off = np.array([0, mats[0].shape[0]])
        f1.pcg_batched(B[:, :mats[0].shape[0]].contiguous())
    f1.close()
    a1.close()
    bt.close()


def test_autotune_caches_a_choice(tmp_path):
    _cae()
    from paper_1603_09133_amd import batched
    cache = str(tmp_path / "tune.json")
    p = batched.autotune(2, 64, lambda s: problems.laplacian((s, s)), cache=cache)
    assert p in [tuple(c) for c in batched.CANDIDATES[2]]
    table = json.load(open(cache))
    assert len(table) == 1 and list(table.values())[0]["patch"] == list(p)
    assert batched.autotune(2, 64, lambda s: problems.laplacian((s, s)), cache=cache) == p
