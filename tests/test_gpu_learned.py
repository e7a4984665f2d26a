"""GPU learned-rank compression against the oracle, through the C ABI.

* features recorded by an exact GPU factorization equal the oracle's
  features of the same steps (FP64 factor, to FP32 rounding of the record;
  the norm features of far rows at rounding level are not compared), labels
  (the sketch width an ideal sketch needs to pass the check) agree;
* the FP32 MLP gradient equals the oracle's FP64 gradient to FP32
  tolerance; the prediction equals the oracle's forward pass;
* a predictor that always asks for the full width reproduces the exact
  CE(eps) oracle (ranks and M X to 1e-10); with a real predictor the GPU
  factor satisfies the Frobenius identity of its own drops, stays within the
  drop bounds of the exact factor and keeps PCG convergence (element parity
  with the oracle's learned run is not defined: the sketch of F_i depends on
  the basis chosen inside processed neighbours' kept subspaces);
* training on one problem's records lowers the loss and the rejection rate
  on another problem, and the PCG iteration count stays within one of the
  exact compression.
"""
import numpy as np
import pytest

import oracle
import problems
from oracle import learned as L

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cae():
    import paper_1603_09133_amd as cae
    cae.lib()
    return cae


def _setup(dims, patch, A=None):
    if A is None:
        A = problems.laplacian(dims)
    csr = problems.to_csr_arrays(A)
    perm, bp, co = oracle.grid_order(dims, patch)
    return A, csr, perm, bp, co


def test_recorded_features_match_oracle():
    cae = _cae()
    from paper_1603_09133_amd import learned
    A, csr, perm, bp, co = _setup((32, 32), (4, 4))
    eps = 1e-6
    fo = oracle.ce_factor(*csr, perm, bp, co,
                          oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=0, record_features=True))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    vals = torch.from_numpy(csr[2]).cuda()
    rec = learned.record(an, vals, eps, coarse_max_dim=0).cpu().numpy()
    row = 0
    nchk = 0
    for lv in fo.levels:
        for i in range(lv.M):
            x = lv.features[i]
            g = rec[row + i]
            if x is None:
                assert g[16] < 0
                continue
            nchk += 1
            # label: the sketch width an ideal sketch needs (a borderline tail may move it by one)
            assert abs(g[16] * lv.sizes[i] - lv.label[i]) <= 1.0 + 1e-4, (row, i, g[16] * lv.sizes[i], lv.label[i])
            # a far row at rounding level (||F|| < 1e-12 tau) is noise: only
            # its structural features are defined
            noise = x[5] < np.log10(1e-12 / eps)
            for k in range(16):
                if noise and 5 <= k <= 11:
                    continue
                assert abs(g[k] - np.float32(x[k])) <= 1e-6 * max(1.0, abs(x[k])), (row, i, k, g[k], x[k])
        row += lv.M
    assert nchk > 50


def test_mlp_gradient_and_prediction_match_oracle():
    cae = _cae()
    from paper_1603_09133_amd import learned
    rng = np.random.default_rng(4)
    n = 300
    X = rng.standard_normal((n, 16)) * 2.0
    y = rng.random(n)
    rec = np.concatenate([X, y[:, None]], axis=1).astype(np.float32)
    rec[::7, 16] = -1.0          # rows that are not samples
    p = L.init_params(3)
    p[L.OFF_MEAN:L.OFF_STD] = rng.standard_normal(16).astype(np.float32) * 0.2
    p[L.OFF_STD:L.OFF_W1] = (1.0 + rng.random(16)).astype(np.float32)
    pg = torch.from_numpy(p).cuda()
    rg = torch.from_numpy(rec).cuda()
    loss_g, grad_g = learned.loss_grad(pg, rg)
    keep = rec[:, 16] >= 0
    loss_o, grad_o = L.mlp_loss_grad(p, rec[keep, :16].astype(np.float64), rec[keep, 16].astype(np.float64))
    assert abs(loss_g - loss_o) <= 1e-5 * max(1.0, loss_o)
    gg = grad_g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gg - grad_o) <= 1e-4 * np.linalg.norm(grad_o)
    z = learned.predict(pg, rg).cpu().numpy()
    zo = L.mlp_forward(p, rec[:, :16].astype(np.float64))
    assert np.max(np.abs(z - zo)) <= 1e-5 * max(1.0, np.max(np.abs(zo)))


def _dense_M(f, n):
    E = torch.eye(n, dtype=torch.float64, device="cuda")
    return f.multiply(E).cpu().numpy().T


@pytest.mark.parametrize("dims,patch,eps", [((32, 32), (4, 4), 1e-6), ((24, 20), (4, 4), 1e-3),
                                            ((8, 8, 8), (2, 2, 2), 1e-4)])
def test_learned_with_full_sketch_equals_exact(dims, patch, eps):
    """A predictor that always answers k = b sketches the whole range of F_i:
    every sketch is accepted and the kept subspaces are the exact ones, so
    ranks and M equal the exact CE(eps) oracle (M does not depend on the
    basis chosen inside a kept subspace)."""
    cae = _cae()
    A, csr, perm, bp, co = _setup(dims, patch)
    fo = oracle.ce_factor(*csr, perm, bp, co, oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=0))
    p = L.init_params(0)
    p[L.OFF_W3:L.OFF_B3] = 0.0
    p[L.OFF_B3] = 1.0
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    vals = torch.from_numpy(csr[2]).cuda()
    f = cae.Factor(an, vals, eps, precision=cae.FP64, coarse_max_dim=0, rank_mode=cae.RANK_LEARNED,
                   mlp_params=torch.from_numpy(p).cuda(), seed=7)
    st = f.stats()
    assert st["sketch_rejected"] == 0 and st["sketch_accepted"] > 0
    for l, lv in enumerate(fo.levels):
        rg = f.ranks(l)
        for i in np.nonzero(rg != lv.r)[0]:
            s = lv.sigma[i]
            k = min(rg[i], lv.r[i])
            assert abs(s[k] - fo.theta) <= 1e-8 * max(s[0], 1e-300), (l, i, rg[i], lv.r[i])
    X = np.random.default_rng(12345).standard_normal((A.shape[0], 8))
    MX = f.multiply(torch.from_numpy(np.ascontiguousarray(X.T)).cuda()).cpu().numpy().T
    MXo = oracle.ce_multiply(fo, X)
    assert np.linalg.norm(MX - MXo) <= 1e-10 * np.linalg.norm(MXo)
    f.close()
    an.close()


@pytest.mark.parametrize("dims,patch,eps", [((32, 32), (4, 4), 1e-6), ((24, 20), (4, 4), 1e-3),
                                            ((8, 8, 8), (2, 2, 2), 1e-4)])
def test_learned_factor_invariants(dims, patch, eps):
    """With a real (untrained) predictor the sketches differ from the oracle's
    (a processed neighbour's kept basis, and so F_i, is defined only up to a
    rotation), so the GPU factor is checked by what must hold for any valid
    CE(eps) factorization: the Frobenius identity ||A0 - M||_F^2 = 2 sum e_i
    of its own factor, every step counted once, M within the two drop bounds
    of the exact factor, and PCG convergence."""
    cae = _cae()
    A, csr, perm, bp, co = _setup(dims, patch)
    p = L.init_params(0)
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    vals = torch.from_numpy(csr[2]).cuda()
    fe = cae.Factor(an, vals, eps, precision=cae.FP64, coarse_max_dim=0)
    f = cae.Factor(an, vals, eps, precision=cae.FP64, coarse_max_dim=0, rank_mode=cae.RANK_LEARNED,
                   mlp_params=torch.from_numpy(p).cuda(), seed=7)
    st, ste = f.stats(), fe.stats()
    assert st["sketch_accepted"] + st["sketch_rejected"] == st["compressions"] or st["compressions"] == 0
    assert st["sketch_accepted"] > 0
    n = A.shape[0]
    A0 = A.toarray()
    M, Me = _dense_M(f, n), _dense_M(fe, n)
    err2 = np.linalg.norm(A0 - M) ** 2
    # a sketch's e_i = ||F_i||^2 - ||B||^2 + sum of dropped sigma(B)^2 cancels:
    # allow 64 u ||F_i||_F^2 per step, with the far-row energies of the exact run
    fo = oracle.ce_factor(*csr, perm, bp, co, oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=0,
                                                                keep_far_rows=True))
    far2 = sum(float(np.sum(F * F)) for lv in fo.levels for F in lv.F if F is not None)
    slack = 2 * 64 * np.finfo(float).eps * 4 * far2
    assert abs(err2 - 2 * st["dropped_sq"]) <= 1e-8 * err2 + slack, (err2, 2 * st["dropped_sq"], slack)
    assert np.linalg.norm(M - Me) <= np.sqrt(2 * st["dropped_sq"]) + np.sqrt(2 * ste["dropped_sq"]) + 1e-12 * n
    b = torch.from_numpy(problems.rhs_uniform(n, seed=0)).cuda()
    _, it, rel = f.pcg(b, rtol=1e-10)
    _, ite, _ = fe.pcg(b, rtol=1e-10)
    assert f.converged and rel[0] <= 1e-9
    assert it[0] <= ite[0] + 3
    f.close()
    fe.close()
    an.close()


def test_training_lowers_rejections_and_keeps_iterations():
    """Records from exact FP32 factorizations of a few 2D problems (Laplacian
    and diffusion with a random coefficient, other seeds) train the
    predictor; on a held-out coefficient field the trained predictor is
    rejected less often than the untrained one, and PCG needs at most one
    iteration more than with the exact compression."""
    cae = _cae()
    from paper_1603_09133_amd import learned
    eps = 1e-6
    recs = []
    train_mats = [problems.laplacian((128, 128))] + [problems.grf_diffusion_2d(128, seed=s)[0] for s in (11, 12, 13)]
    for Am in train_mats:
        A, csr, perm, bp, co = _setup((128, 128), (8, 8), A=Am)
        an = cae.Analysis(csr[0], csr[1], perm, bp, co)
        recs.append(learned.record(an, torch.from_numpy(csr[2]).cuda(), eps, precision=cae.FP32))
        an.close()
    p0 = learned.init_params(1)
    l0, _ = learned.loss_grad(p0, torch.cat(recs))
    params, loss = learned.train(recs, epochs=800, lr=1e-3, params=p0.clone())
    assert loss < 0.2 * l0
    Ag, _ = problems.grf_diffusion_2d(128, seed=2)
    A, csr, perm, bp, co = _setup((128, 128), (8, 8), A=Ag)
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    vals = torch.from_numpy(csr[2]).cuda()
    b = torch.from_numpy(problems.rhs_normal(A.shape[0], 4, seed=1).T.copy()).cuda()
    fe = cae.Factor(an, vals, eps, precision=cae.FP32)
    _, it_e, _ = fe.pcg(b, rtol=1e-8)
    fe.close()
    res = {}
    for name, pp in (("init", p0), ("trained", params)):
        f = cae.Factor(an, vals, eps, precision=cae.FP32, rank_mode=cae.RANK_LEARNED, mlp_params=pp, seed=5)
        st = f.stats()
        _, it, rel = f.pcg(b, rtol=1e-8)
        assert f.converged and np.all(rel <= 1.0001e-8)
        res[name] = (st["sketch_rejected"] / max(1, st["sketch_accepted"] + st["sketch_rejected"]), it)
        f.close()
    print(res, it_e)
    assert res["trained"][0] < res["init"][0]
    assert res["trained"][0] < 0.3
    assert np.all(res["trained"][1] <= it_e + 1)
    an.close()


def test_learned_cap_wide_equals_exact_and_trained_keeps_exact_ranks():
    """LEARNED_CAP (the MLP's width caps the pivoted Cholesky of the far rows'
    Gram matrices, FP32 factor): a predictor that asks for the full width
    gives bitwise the exact factor; a trained predictor caps most steps, and
    every kept capped step has the exact rank (the acceptance test bounds
    sigma_{r+1} by theta), so level 1, whose far rows are the exact
    factorization's, has the exact ranks wherever no singular value lies at
    the FP32 rounding level of theta; PCG needs at most one iteration more.
    The 3D problem with sibling coarsening holds blocks of up to 215
    unknowns at level 2 (the big-block compression capped as well)."""
    cae = _cae()
    from paper_1603_09133_amd import learned
    eps = 1e-4
    A, csr, perm, bp, co = _setup((20, 20, 20), (4, 4, 4))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    vals = torch.from_numpy(csr[2]).cuda()
    n = A.shape[0]
    X = torch.from_numpy(np.random.default_rng(12345).standard_normal((4, n))).cuda()
    fe = cae.Factor(an, vals, eps, precision=cae.FP32, coarse_max_dim=0)
    Me = fe.multiply(X).cpu().numpy()
    # width = b: the cap never binds
    wide = learned.init_params(3)
    wide[cae._lib.lib().cae_mlp_param_count() - 1] = 1e3
    fw = cae.Factor(an, vals, eps, precision=cae.FP32, coarse_max_dim=0, rank_mode=cae.RANK_LEARNED_CAP,
                    mlp_params=wide)
    assert np.array_equal(fw.multiply(X).cpu().numpy(), Me)
    fw.close()
    # trained on the records of a 24^3 problem
    A2, csr2, p2, b2, c2 = _setup((24, 24, 24), (4, 4, 4))
    an2 = cae.Analysis(csr2[0], csr2[1], p2, b2, c2)
    rec = learned.record(an2, torch.from_numpy(csr2[2]).cuda(), eps, precision=cae.FP32, coarse_max_dim=0)
    an2.close()
    params, _ = learned.train(rec, epochs=600, lr=1e-3)
    f = cae.Factor(an, vals, eps, precision=cae.FP32, coarse_max_dim=0, rank_mode=cae.RANK_LEARNED_CAP,
                   mlp_params=params)
    st = f.stats()
    print("capped steps kept / redone:", st["sketch_accepted"], st["sketch_rejected"])
    assert st["sketch_accepted"] > st["sketch_rejected"]
    fo = oracle.ce_factor(*csr, perm, bp, co, oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=0))
    rg, lf = f.ranks(0), fo.levels[0]
    for i in np.nonzero(rg != lf.r)[0]:
        s = lf.sigma[i]
        k = min(rg[i], lf.r[i])
        assert abs(s[k] - fo.theta) <= 1e-5 * s[0], (i, rg[i], lf.r[i])
    b = torch.from_numpy(problems.rhs_normal(n, 2, seed=4).T.copy()).cuda()
    _, it_e, _ = fe.pcg(b, rtol=1e-8)
    _, it, rel = f.pcg(b, rtol=1e-8)
    assert f.converged and np.all(rel <= 1.0001e-8)
    assert np.all(it <= it_e + 1)
    f.close()
    fe.close()
    an.close()


def test_c3_arithmetic_against_oracle():
    """The mixed-precision arithmetic of the 128^3 workload on a 20^3 grid:
    FP32 factor with BF16-input Schur products, learned ranks by the capped
    rank-revealing factorization, sibling coarsening (blocks of up to 215
    unknowns at level 2).  Against the FP64 oracle's exact CE(eps): M X within
    the BF16 input rounding bound (2e-3, as for the exact-rank BF16 factor),
    and PCG to 1e-8 converges in at most a few iterations more."""
    cae = _cae()
    from paper_1603_09133_amd import learned
    eps = 1e-4
    A2, csr2, p2, b2, c2 = _setup((24, 24, 24), (4, 4, 4))
    an2 = cae.Analysis(csr2[0], csr2[1], p2, b2, c2)
    rec = learned.record(an2, torch.from_numpy(csr2[2]).cuda(), eps, precision=cae.FP32, coarse_max_dim=0)
    an2.close()
    params, _ = learned.train(rec, epochs=600, lr=1e-3)
    A, csr, perm, bp, co = _setup((20, 20, 20), (4, 4, 4))
    fo = oracle.ce_factor(*csr, perm, bp, co, oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=0))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    f = cae.Factor(an, torch.from_numpy(csr[2]).cuda(), eps, precision=cae.FP32_BF16, coarse_max_dim=0,
                   rank_mode=cae.RANK_LEARNED_CAP, mlp_params=params)
    assert max(int(f.sizes(l).max()) for l in range(f.stats()["nlevels"])) > 128
    X = np.random.default_rng(12345).standard_normal((A.shape[0], 8))
    Mo = oracle.ce_multiply(fo, X)
    Mg = f.multiply(torch.from_numpy(np.ascontiguousarray(X.T)).cuda()).cpu().numpy().T
    err = np.linalg.norm(Mg - Mo) / np.linalg.norm(Mo)
    print(f"FP32/BF16 + learned caps probe error vs oracle: {err:.3e}")
    assert err <= 2e-3
    b = problems.rhs_normal(A.shape[0], 1, seed=0)[:, 0]
    _, it, rel = f.pcg(torch.from_numpy(b.copy()).cuda(), rtol=1e-8)
    _, ito, _ = oracle.pcg(A, b, lambda r: oracle.ce_solve(fo, r), tol=1e-8)
    assert f.converged and rel[0] <= 1.0001e-8
    assert it[0] <= ito + 6, (it[0], ito)
    f.close()
    an.close()
