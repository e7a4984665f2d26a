"""GPU solvers on the paper's own problem (3D anisotropic diffusion, B = 8):
MINRES parity with the oracle's MINRES, CE(eps) as a direct solver (the
paper's Table 1 trend) and the iteration counts of MINRES/PCG with CE(eps) and
CE(r) against the grid size (the paper's Table 2 trend).

The trends are qualitative (the paper's absolute numbers come from another
threshold scaling and machine): eta decreases and memory grows as eps
shrinks; CE(1e-3) iterations stay flat in N; CE(r=4) needs more iterations.
"""
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


def _e1(dims):
    A = problems.anisotropic_diffusion_3d(dims)
    csr = problems.to_csr_arrays(A)
    perm, bp, co = oracle.grid_order(dims, (2, 2, 2))
    return A, csr, perm, bp, co


@pytest.mark.parametrize("mode", ["eps", "r4"])
def test_minres_parity_with_oracle(mode):
    cae = _cae()
    dims = (16, 16, 8)
    A, csr, perm, bp, co = _e1(dims)
    if mode == "eps":
        o = oracle.CEOptions(eps=1e-3, order="multicolour", coarse_max_dim=0)
        kw = dict(eps=1e-3)
    else:
        o = oracle.CEOptions(eps=0.0, rank_mode="fixed", fixed_rank=4, order="multicolour", coarse_max_dim=0)
        kw = dict(eps=0.0, rank_mode=cae.RANK_FIXED, fixed_rank=4)
    fo = oracle.ce_factor(*csr, perm, bp, co, o)
    b = problems.rhs_ones(A.shape[0])
    xo, ito, relo = oracle.minres(A, b, lambda r: oracle.ce_solve(fo, r), tol=1e-10)
    an = cae.Analysis(csr[0], csr[1], perm, bp, co, order=cae.ORDER_MULTICOLOUR)
    vals = torch.from_numpy(csr[2]).cuda()
    f = cae.Factor(an, vals, kw.pop("eps"), precision=cae.FP64, coarse_max_dim=0, **kw)
    xg, itg, relg = f.minres(torch.from_numpy(b).cuda(), rtol=1e-10)
    assert f.converged
    assert int(itg[0]) == ito, (int(itg[0]), ito)
    xg = xg.cpu().numpy()
    assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)
    assert relg[0] <= 1e-8 and relo <= 1e-8
    # multi-RHS: every column is an independent MINRES
    B = np.stack([b, problems.rhs_uniform(A.shape[0], seed=4)], axis=1)
    Xg, itg2, _ = f.minres(torch.from_numpy(np.ascontiguousarray(B.T)).cuda(), rtol=1e-10)
    x1, it1, _ = oracle.minres(A, B[:, 1], lambda r: oracle.ce_solve(fo, r), tol=1e-10)
    assert int(itg2[0]) == ito and int(itg2[1]) == it1
    assert np.linalg.norm(Xg[1].cpu().numpy() - x1) <= 1e-8 * np.linalg.norm(x1)
    f.close()
    an.close()


def test_direct_solver_matches_oracle():
    cae = _cae()
    dims = (16, 16, 8)
    A, csr, perm, bp, co = _e1(dims)
    b = problems.rhs_ones(A.shape[0])
    an = cae.Analysis(csr[0], csr[1], perm, bp, co, order=cae.ORDER_MULTICOLOUR)
    vals = torch.from_numpy(csr[2]).cuda()
    for eps in (1e-2, 1e-5):
        fo = oracle.ce_factor(*csr, perm, bp, co, oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=0))
        xo = oracle.ce_solve(fo, b)
        f = cae.Factor(an, vals, eps, precision=cae.FP64, coarse_max_dim=0)
        xg = f.solve(torch.from_numpy(b).cuda()).cpu().numpy()
        assert np.linalg.norm(xg - xo) <= 1e-9 * np.linalg.norm(xo), eps
        f.close()
    an.close()


def test_direct_solver_table1_trend():
    from paper_1603_09133_amd import experiments
    res = experiments.table_direct(N=8192)
    rows = res["rows"]
    print(res)
    etas = [r["eta"] for r in rows]
    mem = [r["factor_MB"] for r in rows]
    assert res["reference_relres"] <= 1e-12
    assert all(e2 < e1 for e1, e2 in zip(etas, etas[1:])), etas
    assert all(m2 >= m1 for m1, m2 in zip(mem, mem[1:])), mem
    assert etas[-1] < 1e-5


def test_iterations_table2_trend():
    """The paper's Table 2 sizes, N = 8192 .. 131072 (its own problem and
    preconditioners): CE(1e-3) iterations stay flat, CE(r = 4) needs more and
    grows mildly."""
    from paper_1603_09133_amd import experiments
    res = experiments.table_iterations(Ns=(8192, 16384, 32768, 65536, 131072))
    print(res)
    eps_it = [r["ce_eps_1e-3"]["minres"] for r in res["rows"]]
    r_it = [r["ce_r_4"]["minres"] for r in res["rows"]]
    for r in res["rows"]:
        for k in ("ce_eps_1e-3", "ce_r_4"):
            assert r[k]["minres_relres"] <= 1e-8 and r[k]["pcg_relres"] <= 1e-8
    assert max(eps_it) <= 12 and max(eps_it) - min(eps_it) <= 3, eps_it
    assert all(a > b for a, b in zip(r_it, eps_it)), (r_it, eps_it)
    assert r_it[-1] <= 3 * r_it[0], r_it
