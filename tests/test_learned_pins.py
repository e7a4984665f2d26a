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
    # the loss evaluates the same network as the forward pass: zero at the
    # forward pass's own outputs, 0.5 mean(z^2) against zero targets
    z = L.mlp_forward(p, X)
    assert L.mlp_loss_grad(p, X, z)[0] == 0.0
    assert abs(L.mlp_loss_grad(p, X, np.zeros(20))[0] - 0.5 * np.mean(z * z)) <= 1e-14 * np.mean(z * z)


def _hand_network():
    """A network with a handful of nonzero parameters whose output is worked
    out by hand below (normalisation (x - mean) / std, then W1 indexed
    [hidden][feature], ReLU, W2 indexed [out][in], ReLU, w3, b3)."""
    p = np.zeros(L.NPARAM, dtype=np.float32)
    p[L.OFF_STD:L.OFF_W1] = 1.0
    p[L.OFF_MEAN + 3], p[L.OFF_STD + 3] = 1.0, 2.0
    p[L.OFF_MEAN + 7], p[L.OFF_STD + 7] = -2.0, 0.5
    W1 = lambda h, f: L.OFF_W1 + h * L.NFEAT + f
    p[W1(0, 3)] = 1.0
    p[W1(1, 7)] = -1.0
    p[W1(2, 3)] = 1.0
    p[W1(2, 7)] = 1.0
    p[L.OFF_B1 + 0], p[L.OFF_B1 + 1], p[L.OFF_B1 + 2] = 0.5, 0.25, -1.0
    W2 = lambda o, i: L.OFF_W2 + o * L.H + i
    p[W2(0, 0)], p[W2(0, 1)], p[W2(1, 0)], p[W2(5, 2)] = 2.0, 3.0, 1.0, 4.0
    p[L.OFF_B2 + 1] = -1.0
    p[L.OFF_W3 + 0], p[L.OFF_W3 + 1], p[L.OFF_W3 + 5] = 1.0, 10.0, -0.5
    p[L.OFF_B3] = 0.125
    return p


def test_mlp_forward_hand_worked_network():
    """Input 1: x3 = 5, x7 = -1.5 -> normalised 2, 1 -> hidden-1 (2.5, 0, 2)
    -> hidden-2 h0 = 2*2.5 = 5, h1 = 2.5 - 1 = 1.5, h5 = 4*2 = 8 -> z = 5 +
    15 - 4 + 0.125 = 16.125.  Input 2: x3 = -3, x7 = -2.25 -> normalised -2,
    -0.5 -> hidden-1 (0, 0.75, 0) -> hidden-2 h0 = 2.25 -> z = 2.375.  The
    other features carry zero weights."""
    p = _hand_network()
    X = np.full((2, L.NFEAT), 7.0)
    X[0, 3], X[0, 7] = 5.0, -1.5
    X[1, 3], X[1, 7] = -3.0, -2.25
    assert np.array_equal(L.mlp_forward(p, X), np.array([16.125, 2.375]))


def test_features_of_a_constructed_far_row():
    """A 4 x 6 far row of three far blocks of widths 2, 3, 1 with squared
    Frobenius norms 8 (all ones), 9 (one entry 3) and 0.01 (one entry 0.1):
    the whole row has ||F||_F^2 = 17.01, the largest block norm is 3 and two
    of the three blocks exceed theta = 0.5.  The expected features are the
    definitions evaluated on these norms (not on F)."""
    F = np.zeros((4, 6))
    F[:, 0:2] = 1.0
    F[0, 2] = 3.0
    F[2, 5] = 0.1
    x = L.features(F, 0.5, level=2, nclose=5, nfar=3, nfar_proc=2, proc_rank_sum=6, proc_size_sum=8,
                   widths=[2, 3, 1])
    fro = math.sqrt(17.01)
    want = [math.log2(5), math.log2(7), 2, 3, 5,
            math.log10(fro / 0.5), math.log10(fro / 2 / 0.5), math.log10(6.0), math.log10(fro / math.sqrt(6) / 0.5),
            2 / 3, (64 + 81 + 1e-4) / 17.01 ** 2, 17.01 / 27, 2 / 3, 0.75, 4 / 64, 1.0]
    assert np.allclose(x, want, rtol=1e-13, atol=1e-15)
    # invariant under orthogonal changes of basis inside a far block's
    # columns and inside the rows (kept bases are defined up to rotations)
    rng = np.random.default_rng(0)
    Qr, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    Qa, _ = np.linalg.qr(rng.standard_normal((2, 2)))
    Qb, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    G = Qr @ F
    G[:, 0:2] = G[:, 0:2] @ Qa
    G[:, 2:5] = G[:, 2:5] @ Qb
    y = L.features(G, 0.5, level=2, nclose=5, nfar=3, nfar_proc=2, proc_rank_sum=6, proc_size_sum=8,
                   widths=[2, 3, 1])
    assert np.allclose(y, x, rtol=1e-12, atol=1e-13)
    # a row far below theta clips its logarithms at -30
    z = L.features(F * 1e-40, 0.5, 2, 5, 3, 2, 6, 8, widths=[2, 3, 1])
    assert z[5] == z[6] == z[7] == z[8] == -30.0


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
