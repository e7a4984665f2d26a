"""The C ABI's factor-level entry points beyond analyze / numeric: the
caller-provided workspace (cae_workspace_query, cae_options_t.workspace), the
one-call cae_factor, and cae_export_factor, each through ctypes on the GPU and
checked against the two-step factorization or the oracle (statement of the
problem of Section 2; Algorithm 1's outputs; Proposition 2.1)."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import problems

pytestmark = pytest.mark.gpu


def _cae():
    import paper_1603_09133_amd as cae
    return cae


def _probe(f, n, k=4):
    X = np.random.default_rng(12345).standard_normal((n, k))
    Xg = torch.from_numpy(np.ascontiguousarray(X.T)).cuda()
    return f.multiply(Xg).cpu().numpy().T


@pytest.mark.parametrize("precision", [0, 1])
def test_workspace_factor_equals_library_memory(precision):
    """A factorization carved from a caller's arena of the queried size is
    bitwise the one made with the library's own memory; an arena one byte
    short of the query is refused with CAE_ENOMEM (and names the bytes)."""
    cae = _cae()
    dims, patch = (96, 80), (8, 8)
    A = problems.laplacian(dims)
    ip, ix, dv = problems.to_csr_arrays(A)
    perm, bp, co = cae.grid_order(dims, patch)
    an = cae.Analysis(ip, ix, perm, bp, co)
    vals = torch.from_numpy(dv).cuda()
    need = cae.workspace_bytes(an, vals, 1e-6, precision=precision)
    assert need > 0
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    arena = ws[off:off + need]
    fw = cae.Factor(an, vals, 1e-6, precision=precision, workspace=arena)
    fl = cae.Factor(an, vals, 1e-6, precision=precision)
    n = A.shape[0]
    assert np.array_equal(_probe(fw, n), _probe(fl, n))
    b = torch.from_numpy(problems.rhs_normal(n, 2, seed=4).T.copy()).cuda()
    _, itw, relw = fw.pcg(b, rtol=1e-10)
    _, itl, rell = fl.pcg(b, rtol=1e-10)
    assert itw.tolist() == itl.tolist() and np.array_equal(relw, rell)
    with pytest.raises(cae.CAEError) as ei:
        cae.Factor(an, vals, 1e-6, precision=precision, workspace=ws[off:off + need - 256])
    assert ei.value.code == -2 and "too small" in str(ei.value)
    fw.close()
    fl.close()


def test_one_call_factor_equals_two_step():
    cae = _cae()
    dims, patch = (72, 64), (8, 8)
    A = problems.laplacian(dims)
    ip, ix, dv = problems.to_csr_arrays(A)
    perm, bp, co = cae.grid_order(dims, patch)
    f1 = cae.OneCallFactor(ip, ix, dv, perm, bp, co, 1e-6)
    an = cae.Analysis(ip, ix, perm, bp, co)
    f2 = cae.Factor(an, torch.from_numpy(dv).cuda(), 1e-6)
    n = A.shape[0]
    assert np.array_equal(_probe(f1, n), _probe(f2, n))
    b = torch.from_numpy(problems.rhs_uniform(n, 0)).cuda()
    _, it, rel = f1.pcg(b, rtol=1e-10)
    assert f1.converged and rel[0] <= 1e-10
    f1.close()
    f2.close()


def test_export_matches_handle_and_oracle(tmp_path):
    """The exported factor (FP64): ranks and sizes as the handle reports them,
    orthogonal bases, -A_K^{-1} the inverse of the exported remainder, and at
    level 1 the kept subspace of every compressed block equal to the oracle's
    (projectors U_b U_b^T, within the SVD's perturbation bound u sigma_1 / gap)."""
    cae = _cae()
    dims, patch, eps = (48, 40), (8, 8), 1e-6
    A = problems.laplacian(dims)
    ip, ix, dv = problems.to_csr_arrays(A)
    perm, bp, co = cae.grid_order(dims, patch)
    an = cae.Analysis(ip, ix, perm, bp, co)
    f = cae.Factor(an, torch.from_numpy(dv).cuda(), eps, coarse_max_dim=300)
    path = tmp_path / "factor.bin"
    f.export(path)
    ex = cae.read_export(path)
    st = f.stats()
    assert ex["K"] == st["nlevels"] and ex["coarse_dim"] == st["coarse_dim"] and ex["esize"] == 8
    assert np.array_equal(ex["perm"], an.perm()[0])
    for l, lv in enumerate(ex["levels"]):
        assert np.array_equal(lv["ranks"], f.ranks(l))
        assert np.array_equal(lv["sizes"], f.sizes(l))
        for i, b in enumerate(lv["sizes"]):
            U = lv["U"][lv["u_off"][i]:lv["u_off"][i + 1]].reshape(b, b)
            assert np.abs(U.T @ U - np.eye(b)).max() <= 1e-12
    d = ex["coarse_dim"]
    assert d > 0
    assert np.abs(-ex["neg_inv_A_K"] @ ex["A_K"] - np.eye(d)).max() <= 1e-9
    fo = oracle.ce_factor(ip, ix, dv, perm.astype(np.int64), bp.astype(np.int64), co.astype(np.int64),
                          oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=300))
    lv, lo = ex["levels"][0], fo.levels[0]
    checked = 0
    for i, b in enumerate(lv["sizes"]):
        r = int(lv["ranks"][i])
        assert r == int(lo.r[i])
        sig = np.asarray(lo.sigma[i])
        if r == 0 or r == b or sig[0] == 0:
            continue
        U = lv["U"][lv["u_off"][i]:lv["u_off"][i + 1]].reshape(b, b)
        Pg = U[:, :r] @ U[:, :r].T
        Uo = lo.U[i]
        Po = Uo[:, :r] @ Uo[:, :r].T
        gap = sig[r - 1] - (sig[r] if r < len(sig) else 0.0)
        assert np.abs(Pg - Po).max() <= 64 * np.finfo(float).eps * sig[0] / gap + 1e-13, (i, r)
        checked += 1
    assert checked > 10
    f.close()
