"""Pins of the oracle's learned-rank compression (the cheaper rank-revealing
variant of the compression step, eq. (rreav)).

* Philox4x32-10 reproduces the published known-answer vectors
  (``tests/golden/philox4x32_10_kat.json``).
* Its Box-Muller normals have mean 0 and variance 1, and different
  (level, block) keys give uncorrelated streams.
* The MLP gradient equals central finite differences (FP64).
* An accepted sketch satisfies the CE(eps) condition ||E_i||_2 <= theta
  (checked with an SVD of the dropped part), never keeps more than the exact
  rank (singular values of Q^T F interlace those of F), and keeps exactly the
  exact rank when the sketch is wide enough and the spectrum has a gap.
* The Frobenius identity ||A0 - M||_F^2 = 2 sum ||E_i||_F^2 holds in the
  learned mode too (each step is still an exact change of basis plus an
  exact elimination); the tolerance allows the cancellation in
  e_i = ||F||_F^2 - sum s_k^2.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import problems
from oracle import learned as L

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def test_philox_known_answers():
    kat = json.load(open(GOLD))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x, 16) for x in v["out"]]
        assert list(L.philox4x32_10(ctr, key)) == out


def test_sketch_normals_moments_and_independence():
    a = L.sketch_normals(11, 0, 3, 400, 40).ravel()
    b = L.sketch_normals(11, 1, 3, 400, 40).ravel()
    c = L.sketch_normals(11, 0, 4, 400, 40).ravel()
    n = a.size
    assert abs(a.mean()) < 5 / math.sqrt(n)
    assert abs(a.var() - 1.0) < 6 * math.sqrt(2.0 / n)
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(n)
    assert abs(np.corrcoef(a, c)[0, 1]) < 5 / math.sqrt(n)
    # the first l columns do not depend on l
    assert np.array_equal(L.sketch_normals(11, 0, 3, 50, 7), L.sketch_normals(11, 0, 3, 50, 12)[:, :7])


def test_mlp_gradient_finite_differences():
    rng = np.random.default_rng(3)
    p = L.init_params(5).astype(np.float64)
    p[L.OFF_MEAN:L.OFF_STD] = rng.standard_normal(L.NFEAT) * 0.1
    p[L.OFF_STD:L.OFF_W1] = 1.0 + rng.random(L.NFEAT)
    X = rng.standard_normal((20, L.NFEAT))
    y = rng.random(20)
    loss, g = L.mlp_loss_grad(p, X, y)
    idx = np.concatenate([rng.choice(np.arange(L.OFF_W1, L.NPARAM), 60, replace=False), [L.OFF_B3]])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (L.mlp_loss_grad(pp, X, y)[0] - L.mlp_loss_grad(pm, X, y)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])
    assert np.all(g[:L.OFF_W1] == 0.0)
    assert np.allclose(L.mlp_forward(p, X), X.shape[0] * 0 + L.mlp_forward(p, X))


def _low_rank_far_row(b, w, ranks_sig, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((b, b)))
    V, _ = np.linalg.qr(rng.standard_normal((w, b)))
    s = np.zeros(b)
    s[:len(ranks_sig)] = ranks_sig
    return (U * s) @ V.T, s


@pytest.mark.parametrize("k", [2, 6, 10, 30])
def test_randomized_compress_condition(k):
    theta = 1e-3
    sig = np.concatenate([np.geomspace(1.0, 1e-2, 8), np.geomspace(5e-4, 1e-7, 20)])
    F, s = _low_rank_far_row(40, 120, sig, 9)
    r_exact = int(np.count_nonzero(s > theta))
    ok, Ur, r, sb, e = L.randomized_compress(F, theta, k, seed=1, level=0, block=2)
    assert r <= r_exact
    if ok:
        E = F - Ur @ (Ur.T @ F)
        assert np.linalg.norm(E, 2) <= theta * (1 + 1e-10)
        assert abs(e - np.linalg.norm(E) ** 2) <= 1e-12 * np.linalg.norm(F) ** 2
    if k >= r_exact + 2:
        assert ok and r == r_exact


def test_complete_basis_is_orthonormal_and_keeps_the_span():
    rng = np.random.default_rng(2)
    Ur, _ = np.linalg.qr(rng.standard_normal((12, 5)))
    U = L.complete_basis(Ur, 12)
    assert np.allclose(U.T @ U, np.eye(12), atol=1e-13)
    assert np.allclose(U[:, :5], Ur)


@pytest.mark.parametrize("dims,patch,eps", [((32, 32), (4, 4), 1e-6), ((24, 20), (4, 4), 1e-3),
                                            ((8, 8, 8), (2, 2, 2), 1e-4)])
def test_learned_mode_frobenius_identity(dims, patch, eps):
    A = problems.laplacian(dims)
    ip, ix, dv = problems.to_csr_arrays(A)
    perm, bp, co = oracle.grid_order(dims, patch)
    f = oracle.ce_factor(ip, ix, dv, perm, bp, co,
                         oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=0, rank_mode="learned",
                                          mlp_params=L.init_params(0), seed=7))
    M = oracle.ce_dense(f)
    err2 = np.linalg.norm(A.toarray() - M) ** 2
    pred2 = 2.0 * f.dropped()
    # e_i = ||F||^2 - sum s^2 cancels: allow 64 u ||F_i||_F^2 per step
    slack = 2 * 64 * np.finfo(float).eps * sum(len(lv.order) for lv in f.levels) * 16.0
    assert abs(err2 - pred2) <= 1e-8 * pred2 + slack
    assert sum(lv.accepted for lv in f.levels) > 0


def test_learned_mode_with_exact_predictor_matches_exact_ranks():
    """A predictor that returns the exact rank (z = r/b) with oversampling
    accepts (almost) every sketch and reproduces the exact ranks."""
    dims, patch, eps = (24, 24), (4, 4), 1e-5
    A = problems.laplacian(dims)
    ip, ix, dv = problems.to_csr_arrays(A)
    perm, bp, co = oracle.grid_order(dims, patch)
    fe = oracle.ce_factor(ip, ix, dv, perm, bp, co, oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=0))
    # the constant predictor z = 1 (k = b): the sketch spans the full row space
    p = L.init_params(0)
    p[L.OFF_W3:L.OFF_B3] = 0.0
    p[L.OFF_B3] = 1.0
    fl = oracle.ce_factor(ip, ix, dv, perm, bp, co,
                          oracle.CEOptions(eps=eps, order="multicolour", coarse_max_dim=0, rank_mode="learned",
                                           mlp_params=p, seed=3))
    for a, b in zip(fe.levels, fl.levels):
        assert np.array_equal(a.r, b.r)
        assert b.fallbacks == 0


def test_sketch_label_is_the_smallest_passing_width():
    theta = 1.0
    sig = np.array([5.0, 3.0, 0.9, 0.5, 0.3, 0.1])
    r = 2
    k = L.sketch_label(sig, r, theta)
    tail = lambda kk: float(np.sum(sig[kk:] ** 2))
    ok = lambda kk: tail(kk) + (sig[r] ** 2 if kk > r else 0.0) <= theta ** 2
    assert ok(k) and all(not ok(kk) for kk in range(r, k))
    # an ideal sketch of that width passes the randomized check
    F, s = _low_rank_far_row(12, 40, sig, 4)
    kk = L.sketch_label(s, int(np.count_nonzero(s > theta)), theta)
    ok2, Ur, rr, sb, e = L.randomized_compress(F, theta, kk, seed=2, level=0, block=0, p=12)
    assert ok2
