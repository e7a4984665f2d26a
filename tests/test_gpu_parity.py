"""GPU parity: the HIP factorization against the FP64 oracle, element by
element on the same seeded inputs, through the C ABI.

Tolerances (FP64 path, readings of the parity bar):
* ranks of every level equal (a mismatch is allowed only where the oracle's
  singular value lies within 1e-10 sigma_1 of the threshold);
* M X with eight N(0,1) probes (default_rng(12345)):
  ||(M_gpu - M_orc) X||_F <= 1e-12 ||M_orc X||_F;
* sum of ||E_i||_F^2 within 1e-10 relative;
* M^{-1} X within 1e-10 relative (amplified by the condition number);
* PCG iteration counts equal.
"""
import math

import numpy as np
import pytest

import problems
import oracle
from oracle import CEOptions, ce_factor, ce_multiply, ce_solve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cae():
    import paper_1603_09133_amd as cae
    cae.lib()
    return cae


def _probes(N, k=8):
    return np.random.default_rng(12345).standard_normal((N, k))


def _setup(dims, patch, A=None):
    if A is None:
        A = problems.laplacian(dims)
    csr = problems.to_csr_arrays(A)
    perm, bp, co = oracle.grid_order(dims, patch)
    return A, csr, perm, bp, co


def _gpu_factor(cae, csr, perm, bp, co, eps, order, precision=0, coarse=2048, rank_mode=0, fixed_rank=0):
    an = cae.Analysis(csr[0], csr[1], perm, bp, co,
                      order=cae.ORDER_PAPER if order == "paper" else cae.ORDER_MULTICOLOUR)
    vals = torch.from_numpy(csr[2]).cuda()
    f = cae.Factor(an, vals, eps, precision=precision, coarse_max_dim=coarse, rank_mode=rank_mode,
                   fixed_rank=fixed_rank)
    return an, f


def _to_gpu_cols(X):
    return torch.from_numpy(np.ascontiguousarray(X.T)).cuda()


def _from_gpu_cols(T):
    return T.cpu().numpy().T


def _check_ranks(f, fo):
    for l, lf in enumerate(fo.levels):
        rg = f.ranks(l)
        bad = np.nonzero(rg != lf.r)[0]
        for i in bad:
            s = lf.sigma[i]
            k = min(rg[i], lf.r[i])
            assert abs(s[k] - fo.theta) <= 1e-10 * s[0], (l, i, rg[i], lf.r[i])


CASES = [
    ((16, 16), (4, 4), 1e-4, "paper", 0),
    ((16, 16), (4, 4), 1e-4, "multicolour", 0),
    ((18, 13), (4, 4), 1e-5, "multicolour", 0),
    ((40, 24), (8, 8), 1e-6, "multicolour", 0),
    ((40, 24), (8, 8), 1e-6, "paper", 100),
    ((8, 8, 8), (2, 2, 2), 1e-3, "multicolour", 0),
    ((7, 9, 6), (2, 2, 2), 1e-4, "paper", 0),
    ((64, 64), (4, 4), 1e-8, "multicolour", 2048),
    ((64, 64), (4, 4), 1e-8, "paper", 0),
]


@pytest.mark.parametrize("dims,patch,eps,order,coarse", CASES)
def test_factor_matches_oracle_fp64(dims, patch, eps, order, coarse):
    cae = _cae()
    A, csr, perm, bp, co = _setup(dims, patch)
    print(f"case dims={dims} patch={patch} eps={eps} order={order} coarse={coarse}", flush=True)
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, order=order, coarse_max_dim=coarse))
    an, f = _gpu_factor(cae, csr, perm, bp, co, eps, order, coarse=coarse)
    st = f.stats()
    assert st["nlevels"] == len(fo.levels)
    assert st["coarse_dim"] == fo.coarse_L.shape[0]
    _check_ranks(f, fo)
    for l, lf in enumerate(fo.levels):
        assert np.array_equal(f.sizes(l), lf.sizes)
    assert abs(st["tau"] - float(A.diagonal().max())) == 0.0
    X = _probes(A.shape[0])
    Mo = ce_multiply(fo, X)
    Mg = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    assert np.linalg.norm(Mg - Mo) <= 1e-12 * np.linalg.norm(Mo)
    Zo = ce_solve(fo, X)
    Zg = _from_gpu_cols(f.apply(_to_gpu_cols(X)))
    assert np.linalg.norm(Zg - Zo) <= 1e-10 * np.linalg.norm(Zo)
    # sum of ||E_i||^2: a backward-stable SVD (LAPACK's and the one-sided
    # Jacobi alike) gives every singular value to within c*u*sigma_1 absolutely,
    # so |delta e_i| <= 2 c u sigma_1(F_i) sum_{k>r} sigma_k <= 2 c u sigma_1 sqrt(b e_i)
    d_o = fo.dropped()
    u = np.finfo(float).eps
    bound = sum(2 * 64 * u * lf.sigma[i][0] * math.sqrt(lf.sizes[i] * lf.e[i])
                for lf in fo.levels for i in range(lf.M) if lf.sigma[i].size)
    assert abs(st["dropped_sq"] - d_o) <= 1e-10 * d_o + bound


@pytest.mark.parametrize("dims,patch,eps,order,coarse,prec", [
    ((40, 24), (8, 8), 1e-6, "multicolour", 0, "fp64"),
    ((7, 9, 6), (2, 2, 2), 1e-4, "paper", 0, "fp64"),
    ((64, 64), (4, 4), 1e-8, "multicolour", 2048, "fp64"),
    ((40, 24), (8, 8), 1e-6, "multicolour", 0, "fp32"),
])
def test_apply_one_workgroup_per_step_matches_oracle(dims, patch, eps, order, coarse, prec):
    """Both forms of the apply's close-block updates against the oracle's
    M^{-1} X: one workgroup per step (apply_split_steps = 0, the form large
    waves take) and one per (step, close block) (apply_split_steps large,
    every wave); FP64 to the parity bar, FP32 within 1e-3 (the FP32 factor's
    1e-7 probe error times the preconditioner's condition), and the two forms
    within rounding of each other (only the order of FP64 sums differs)."""
    cae = _cae()
    A, csr, perm, bp, co = _setup(dims, patch)
    print(f"case dims={dims} patch={patch} eps={eps} order={order} coarse={coarse} {prec}", flush=True)
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, order=order, coarse_max_dim=coarse))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co,
                      order=cae.ORDER_PAPER if order == "paper" else cae.ORDER_MULTICOLOUR)
    vals = torch.from_numpy(csr[2]).cuda()
    precision = cae.FP64 if prec == "fp64" else cae.FP32
    X = _probes(A.shape[0])
    Zo = ce_solve(fo, X)
    Z = {}
    for split in (0, 1 << 30):
        f = cae.Factor(an, vals, eps, precision=precision, coarse_max_dim=coarse, apply_split_steps=split)
        Z[split] = _from_gpu_cols(f.apply(_to_gpu_cols(X)))
        f.close()
    tol = 1e-10 if prec == "fp64" else 1e-3
    for split, Zg in Z.items():
        assert np.linalg.norm(Zg - Zo) <= tol * np.linalg.norm(Zo), split
    assert np.linalg.norm(Z[0] - Z[1 << 30]) <= 1e-12 * np.linalg.norm(Z[0])


def test_eps_zero_exact_and_frobenius_identity_on_gpu():
    cae = _cae()
    A, csr, perm, bp, co = _setup((20, 20), (4, 4))
    Ad = A.toarray()
    an, f0 = _gpu_factor(cae, csr, perm, bp, co, 0.0, "multicolour", coarse=0)
    I = np.eye(A.shape[0])
    M0 = _from_gpu_cols(f0.multiply(_to_gpu_cols(I)))
    assert np.linalg.norm(M0 - Ad) <= 1e-13 * np.linalg.norm(Ad)
    an, f = _gpu_factor(cae, csr, perm, bp, co, 1e-3, "multicolour", coarse=0)
    M = _from_gpu_cols(f.multiply(_to_gpu_cols(I)))
    pred = math.sqrt(2 * f.stats()["dropped_sq"])
    assert pred > 0
    assert abs(np.linalg.norm(Ad - M) - pred) <= 1e-8 * pred + 1e-13 * np.linalg.norm(Ad)


@pytest.mark.parametrize("order", ["paper", "multicolour"])
def test_pcg_iterations_match_oracle(order):
    cae = _cae()
    A, csr, perm, bp, co = _setup((64, 64), (4, 4))
    b = problems.rhs_uniform(A.shape[0], 0)
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-8, order=order))
    _, it_o, rel_o = oracle.pcg(A, b, lambda r: ce_solve(fo, r), tol=1e-10)
    an, f = _gpu_factor(cae, csr, perm, bp, co, 1e-8, order)
    x, it, rel = f.pcg(torch.from_numpy(b).cuda(), rtol=1e-10, maxit=1000)
    assert f.converged
    assert int(it[0]) == it_o
    xr = x.cpu().numpy()
    assert np.linalg.norm(b - A @ xr) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)
    assert abs(rel[0] - np.linalg.norm(b - A @ xr) / np.linalg.norm(b)) <= 1e-3 * rel[0] + 1e-16


def test_multi_rhs_pcg_and_fp32_factor():
    cae = _cae()
    A, csr, perm, bp, co = _setup((48, 40), (8, 8))
    B = problems.rhs_normal(A.shape[0], 4, seed=1)
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-6, order="multicolour"))
    its_o = [oracle.pcg(A, B[:, k], lambda r: ce_solve(fo, r), tol=1e-8)[1] for k in range(4)]
    an, f = _gpu_factor(cae, csr, perm, bp, co, 1e-6, "multicolour")
    x, it, rel = f.pcg(_to_gpu_cols(B), rtol=1e-8)
    assert it.tolist() == its_o
    assert np.all(rel <= 1.0001e-8)
    # the FP32 factor with every level compressed (no dense remainder, which
    # would hold the whole 1920-unknown matrix in FP64)
    fo0 = ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-6, order="multicolour", coarse_max_dim=0))
    its_o0 = [oracle.pcg(A, B[:, k], lambda r: ce_solve(fo0, r), tol=1e-8)[1] for k in range(4)]
    an, f32 = _gpu_factor(cae, csr, perm, bp, co, 1e-6, "multicolour", precision=cae.FP32, coarse=0)
    assert f32.stats()["nlevels"] >= 2
    X = _probes(A.shape[0])
    Mo = ce_multiply(fo0, X)
    M32 = _from_gpu_cols(f32.multiply(_to_gpu_cols(X)))
    err32 = np.linalg.norm(M32 - Mo) / np.linalg.norm(Mo)
    print(f"fp32 factor probe error vs oracle: {err32:.3e}")
    assert err32 <= 1e-5
    x, it32, rel32 = f32.pcg(_to_gpu_cols(B), rtol=1e-8)
    assert np.all(rel32 <= 1.0001e-8)
    assert np.all(it32 <= np.array(its_o0) + 1)


def test_fp32_factor_with_blocks_above_64():
    """FP32 factor of a 3D Laplacian whose second level holds blocks of 65..128
    unknowns (the Gram compression's two-coordinates-per-lane instance):
    probe error against the FP64 oracle within the FP32 bound, and the ranks
    of that level equal to the oracle's wherever the oracle's singular values
    are not within the FP32 rounding level of the threshold."""
    cae = _cae()
    dims, patch, eps = (16, 16, 16), (2, 2, 4), 1e-4
    A, csr, perm, bp, co = _setup(dims, patch)
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, order="multicolour", coarse_max_dim=0))
    an, f = _gpu_factor(cae, csr, perm, bp, co, eps, "multicolour", precision=cae.FP32, coarse=0)
    big = [l for l in range(len(fo.levels)) if 64 < int(f.sizes(l).max()) <= 128 and fo.levels[l].sigma]
    assert big, "no level with blocks of 65..128 unknowns"
    for l in big:
        rg, lf = f.ranks(l), fo.levels[l]
        for i in np.nonzero(rg != lf.r)[0]:
            s = lf.sigma[i]
            k = min(rg[i], lf.r[i])
            assert abs(s[k] - fo.theta) <= 1e-5 * s[0], (l, i, rg[i], lf.r[i])
    X = _probes(A.shape[0])
    Mo = ce_multiply(fo, X)
    M32 = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    err = np.linalg.norm(M32 - Mo) / np.linalg.norm(Mo)
    print(f"fp32 (b <= 128) probe error vs oracle: {err:.3e}")
    assert err <= 1e-5


_BIG = {}


def _big_oracle():
    """The oracle's factor of the 20^3 Laplacian with sibling coarsening (its
    second level holds blocks of up to 215 unknowns), computed once."""
    if not _BIG:
        dims, patch, eps = (20, 20, 20), (4, 4, 4), 1e-4
        A, csr, perm, bp, co = _setup(dims, patch)
        fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, order="multicolour", coarse_max_dim=0,
                                                     keep_far_rows=True))
        _BIG.update(A=A, csr=csr, perm=perm, bp=bp, co=co, eps=eps, fo=fo, Mo=oracle.ce_dense(fo))
    return _BIG


def _dense_M(f, n, chunk=2000):
    cols = []
    for c0 in range(0, n, chunk):
        E = torch.zeros((min(chunk, n - c0), n), dtype=torch.float64, device="cuda")
        E[torch.arange(E.shape[0]), torch.arange(c0, c0 + E.shape[0])] = 1.0
        cols.append(f.multiply(E).cpu().numpy())
    return np.concatenate(cols, axis=0).T


@pytest.mark.parametrize("prec,cap", [("fp32", 0), ("fp32", 1), ("fp32", 24), ("fp32", 12), ("fp64", 24),
                                      ("fp64", 12)])
def test_factor_with_blocks_above_128(prec, cap):
    """Factor of a 3D Laplacian with the paper's coarsening (the eight Morton
    siblings join, Section 2.5): the second level holds blocks of up to 215
    unknowns, which take the big-block kernels (Gram tiles on the FP64 matrix
    cores, pivoted Cholesky, Jacobi on X X^T, reflectors).

    Default cap, and cap 1 (which sends every big step of rank above 1 to an
    uncapped pivoted Cholesky): probe error against the FP64 oracle within
    the FP32 bound, every level's ranks equal to the oracle's wherever the
    oracle's singular values are not within the FP32 rounding level of the
    threshold, and every step's dropped energy equal to the oracle's.

    A pivot cap below the default truncates the pivoted Cholesky, so that the
    other ways of settling a rank run too: the Frobenius bound, the spectral
    certificate by repeated squaring, and the uncapped pivoted Cholesky (each
    asserted to occur for some cap).  A truncated step keeps the Ritz basis of its pivoted
    rows instead of the exact singular vectors -- another valid CE(eps) basis
    with the same rank -- so the later far rows, and near-threshold ranks
    after it, differ from the oracle's.  Such a factor is checked by what
    holds for any CE(eps) factorization: the ranks of the levels before the
    first big one equal the oracle's; the Frobenius identity ||A0 - M||_F^2 =
    2 sum e_i of its own drops; M within the two drop bounds of the oracle's
    M; PCG iterations."""
    cae = _cae()
    d = _big_oracle()
    A, csr, perm, bp, co, eps, fo = (d[k] for k in ("A", "csr", "perm", "bp", "co", "eps", "fo"))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co, order=cae.ORDER_MULTICOLOUR)
    vals = torch.from_numpy(csr[2]).cuda()
    f = cae.Factor(an, vals, eps, precision=cae.FP32 if prec == "fp32" else cae.FP64, coarse_max_dim=0,
                   big_pivot_cap=cap)
    st = f.stats()
    K = min(st["nlevels"], len(fo.levels))
    # the levels whose blocks are those of the oracle (a different rank
    # changes the sizes of the levels after it)
    same = []
    for l in range(K):
        if len(f.sizes(l)) != len(fo.levels[l].sizes) or not np.array_equal(f.sizes(l), fo.levels[l].sizes):
            break
        same.append(l)
    big = [l for l in same if int(f.sizes(l).max()) > 128 and fo.levels[l].sigma]
    first_big = min(big) if big else K
    nbig = 0
    rank_diff = []
    for l in same:
        rg, sz, lf = f.ranks(l), f.sizes(l), fo.levels[l]
        for i in np.nonzero(rg != lf.r)[0]:
            s = lf.sigma[i]
            k = min(rg[i], lf.r[i])
            rank_diff.append((l, int(i), int(rg[i]), int(lf.r[i]), float(s[k] / fo.theta)))
    for l in range(K):
        sz = f.sizes(l)
        nbig += int(np.count_nonzero(sz > 128))
    cls = [st[k] for k in ("big_untruncated", "big_frobenius", "big_certified", "big_uncapped")]
    X = _probes(A.shape[0])
    Mo = ce_multiply(fo, X)
    Mg = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    err = np.linalg.norm(Mg - Mo) / np.linalg.norm(Mo)
    ed_o = sum(float(np.sum(l.e)) for l in fo.levels)
    # per-step dropped energy against the oracle's, on the levels whose far
    # rows are the oracle's (before the first big level; every level for the
    # exact caps); the worst step relative to the level's total
    th2 = fo.theta ** 2
    worst = []
    for l in same:
        if cap not in (0, 1) and l >= first_big:
            break
        dg, do = f.drops(l), np.asarray(fo.levels[l].e)
        k = int(np.argmax(np.abs(dg - do)))
        worst.append((l, k, int(f.sizes(l)[k]), float(dg[k] / th2), float(do[k] / th2)))
    print(f"{prec} cap {cap}: levels with the oracle's blocks {same}, first big {first_big}, blocks above 128 "
          f"{nbig}, untruncated/Frobenius/certified/uncapped {cls}, probe error vs oracle {err:.3e}, dropped "
          f"energy {st['dropped_sq']:.6e} vs oracle {ed_o:.6e}, rank differences (level, block, gpu, oracle, "
          f"sigma/theta) {rank_diff[:8]}, worst step drop (level, block, b, gpu/theta^2, oracle/theta^2) {worst}")
    assert big, "no level with blocks above 128 unknowns"
    assert 0 < sum(cls) <= nbig
    # (in units of theta^2) FP64: a big step's pivoted Cholesky stops once the
    # trailing energy is below (theta / 32)^2, which its dropped energy may
    # miss; FP32: the far row's entries carry the rounding of the FP32 factor
    # so far (about u_32 times the Schur terms that formed them, ~1e-5 in
    # ||dF||_2 against theta = 6e-4), which moves a dropped sigma^2 near
    # theta^2 by a few per cent
    for l, k, b, eg, eo in worst:
        tol = 0.1 + 2e-2 * eo if prec == "fp32" else 1e-6 * eo + (1.0 / 1024 if b > 128 else 1e-12)
        assert abs(eg - eo) <= tol, (l, k, b, eg, eo)
    if cap in (0, 1):
        if cap == 0:
            assert cls[1:] == [0, 0, 0]
        else:
            assert cls[3] > 0
        assert len(same) == K == len(fo.levels)
        # every block above 128 unknowns with a far row is counted once
        assert sum(cls) == sum(1 for lf in fo.levels for i, F in enumerate(lf.F)
                               if lf.sizes[i] > 128 and F is not None and F.shape[1] > 0)
        for l, i, rg_i, ro_i, q in rank_diff:
            assert abs(q - 1.0) <= 1e-5 * fo.levels[l].sigma[i][0] / fo.theta, (l, i, rg_i, ro_i)
        # FP32: the rounding of the far rows; FP64: the pivoted Cholesky stops
        # once the trailing energy is below (theta / 32)^2, which moves the
        # basis by O(that / gap) -- measured 1e-8
        assert err <= (1e-5 if prec == "fp32" else 1e-7)
        # every dropped sigma (<= theta) of an FP32 far row is perturbed by
        # about u_32 ||F_i||, so sigma^2 by about 2 theta u_32 ||F_i||:
        # relative to the total, ~2 u_32 ||F|| / theta (a few 1e-3 here)
        assert abs(st["dropped_sq"] - ed_o) <= 1e-2 * ed_o
    else:
        if cap == 24:
            assert cls[2] > 0
        if cap == 12:
            assert cls[3] > 0
        n = A.shape[0]
        A0 = A.toarray()
        M = _dense_M(f, n)
        Mo_d = d["Mo"]
        err2 = np.linalg.norm(A0 - M) ** 2
        dM = np.linalg.norm(M - Mo_d)
        bound = np.sqrt(2 * st["dropped_sq"]) + np.sqrt(2 * ed_o)
        b = torch.from_numpy(problems.rhs_uniform(n, seed=0)).cuda()
        _, it, rel = f.pcg(b, rtol=1e-10)
        _, it_o, _ = oracle.pcg(A, problems.rhs_uniform(n, seed=0), lambda r: ce_solve(fo, r), tol=1e-10)
        print(f"   ||A0 - M||_F^2 {err2:.6e} vs 2 sum e_i {2 * st['dropped_sq']:.6e}; ||M - M_orc||_F {dM:.3e} "
              f"<= {bound:.3e}; PCG {int(it[0])} vs oracle {it_o}")
        for l, i, rg_i, ro_i, q in rank_diff:
            if l < first_big:
                assert abs(q - 1.0) <= 1e-5 * fo.levels[l].sigma[i][0] / fo.theta, (l, i, rg_i, ro_i)
        # the identity to rounding, but for the (theta / 32)^2 a big step's
        # dropped energy may miss; FP32: M's entries also carry the FP32
        # rounding of the factor (u_32 ||A||_F per entry block), against
        # ||A0 - M||_F of about sqrt(2 sum e_i)
        tol = 1e-8 if prec == "fp64" else 3e-2
        assert abs(err2 - 2 * st["dropped_sq"]) <= tol * err2 + 2 * nbig * th2 / 1024
        assert dM <= bound * (1 + 1e-6) + 1e-6 * np.linalg.norm(A0)
        assert f.converged and rel[0] <= 1e-9
        assert int(it[0]) <= it_o + 1
    f.close()
    an.close()


def test_random_coefficient_diffusion_fp32_matches_oracle():
    """The 2D diffusion with a log-normal random coefficient (the 2048^2
    workload's matrix family, here on 128^2: k = exp(GRF), harmonic-mean
    faces, 8 x 8 patches, eps = 1e-5): the FP32 factor against the FP64
    oracle, probe error within the FP32 bound, level-1 ranks equal except at
    FP32-level ties, and PCG to 1e-8 in at most one iteration more."""
    cae = _cae()
    Ag, _ = problems.grf_diffusion_2d(128)
    A, csr, perm, bp, co = _setup((128, 128), (8, 8), A=Ag)
    eps = 1e-5
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, order="multicolour"))
    an, f = _gpu_factor(cae, csr, perm, bp, co, eps, "multicolour", precision=cae.FP32)
    rg, lf = f.ranks(0), fo.levels[0]
    for i in np.nonzero(rg != lf.r)[0]:
        sv = lf.sigma[i]
        k = min(rg[i], lf.r[i])
        assert abs(sv[k] - fo.theta) <= 1e-5 * sv[0], (i, rg[i], lf.r[i])
    X = _probes(A.shape[0])
    Mo = ce_multiply(fo, X)
    M32 = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    err = np.linalg.norm(M32 - Mo) / np.linalg.norm(Mo)
    print(f"random-coefficient fp32 probe error vs oracle: {err:.3e}")
    assert err <= 1e-5
    B = problems.rhs_normal(A.shape[0], 2, seed=2)
    its_o = [oracle.pcg(A, B[:, k], lambda r: ce_solve(fo, r), tol=1e-8)[1] for k in range(2)]
    _, it, rel = f.pcg(_to_gpu_cols(B), rtol=1e-8)
    assert f.converged and np.all(rel <= 1.0001e-8)
    assert np.all(it <= np.array(its_o) + 1), (it, its_o)
    f.close()
    an.close()


def test_solver_apply_graph_replays_equal_eager_launches():
    """The iterative solvers replay the captured apply graph: three PCG solves
    on one handle (the later ones replaying the graph captured by the first,
    with the solver's own eager kernels, host reads and synchronisations in
    between) and a MINRES solve (two captured inputs alternating) give
    bitwise the iterates of a handle that launches the apply kernels one by
    one (the same kernels in the same order)."""
    cae = _cae()
    A, csr, perm, bp, co = _setup((96, 80), (8, 8))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    vals = torch.from_numpy(csr[2]).cuda()
    fg = cae.Factor(an, vals, 1e-4, precision=cae.FP32, coarse_max_dim=0)
    fe = cae.Factor(an, vals, 1e-4, precision=cae.FP32, coarse_max_dim=0, graphs=False)
    B1 = problems.rhs_normal(A.shape[0], 4, seed=5)
    B2 = problems.rhs_normal(A.shape[0], 4, seed=6)
    for B in (B1, B2, B1):
        xg, itg, relg = fg.pcg(_to_gpu_cols(B), rtol=1e-10)
        xe, ite, rele = fe.pcg(_to_gpu_cols(B), rtol=1e-10)
        assert itg.tolist() == ite.tolist()
        assert np.array_equal(_from_gpu_cols(xg), _from_gpu_cols(xe))
        assert np.all(relg <= 1.0001e-10)
    xg, itg, relg = fg.minres(_to_gpu_cols(B2), rtol=1e-8)
    xe, ite, rele = fe.minres(_to_gpu_cols(B2), rtol=1e-8)
    assert itg.tolist() == ite.tolist()
    assert np.array_equal(_from_gpu_cols(xg), _from_gpu_cols(xe))


def test_graphs_dropped_when_work_vectors_grow():
    """A captured solver apply holds the addresses of the handle's work
    vectors.  An apply with more right-hand sides releases and reallocates
    them (the old blocks go back to the device cache, where another
    factorization can take them); the next PCG must capture afresh instead of
    replaying into released memory, and stay bitwise equal to eager launches."""
    cae = _cae()
    A, csr, perm, bp, co = _setup((96, 80), (8, 8))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    vals = torch.from_numpy(csr[2]).cuda()
    fg = cae.Factor(an, vals, 1e-3, precision=cae.FP32, coarse_max_dim=0)
    fe = cae.Factor(an, vals, 1e-3, precision=cae.FP32, coarse_max_dim=0, graphs=False)
    b = _to_gpu_cols(problems.rhs_normal(A.shape[0], 1, seed=7))
    xg, itg, _ = fg.pcg(b, rtol=1e-11)
    assert int(itg[0]) > 4   # enough applies to capture and replay a graph
    fg.apply(_to_gpu_cols(problems.rhs_normal(A.shape[0], 16, seed=8)))
    other = cae.Factor(an, vals, 1e-5, precision=cae.FP32, coarse_max_dim=0)
    other.apply(_to_gpu_cols(problems.rhs_normal(A.shape[0], 16, seed=9)))
    for f in (fg, fe):
        f.pcg(b, rtol=1e-11)
    xg, itg, relg = fg.pcg(b, rtol=1e-11)
    xe, ite, rele = fe.pcg(b, rtol=1e-11)
    other.close()
    assert itg.tolist() == ite.tolist()
    assert np.array_equal(_from_gpu_cols(xg), _from_gpu_cols(xe))
    assert np.all(relg <= 1.0001e-11)


def test_solvers_report_no_convergence_at_maxit():
    """maxit = 1 on a system that needs more iterations: PCG and MINRES
    return CAE_ENOCONV through the C ABI (the iterate of the last iteration
    is kept, iters = maxit, the true residual is reported)."""
    import ctypes as C
    cae = _cae()
    A, csr, perm, bp, co = _setup((64, 48), (8, 8))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    f = cae.Factor(an, torch.from_numpy(csr[2]).cuda(), 1e-2, coarse_max_dim=0)
    n = A.shape[0]
    b = _to_gpu_cols(problems.rhs_normal(n, 2, seed=3))
    x = torch.empty_like(b)
    it = np.zeros(2, np.int32)
    rel = np.zeros(2)
    for fn in (cae.lib().cae_pcg_solve, cae.lib().cae_minres_solve):
        rc = fn(f._h, 2, b.data_ptr(), n, x.data_ptr(), n, C.c_double(1e-12), 1, it.ctypes.data, rel.ctypes.data)
        assert rc == -4, rc
        assert b"did not converge" in cae.lib().cae_last_error(None)
        assert b"did not converge" in cae.lib().cae_last_error(f._h)   # kept with the handle too
        assert it.tolist() == [1, 1]
        assert np.all(rel > 1e-12) and np.all(rel < 1.0)
    xx, it2, rel2 = f.pcg(b, rtol=1e-12, maxit=1)
    assert not f.converged and it2.tolist() == [1, 1]


def test_indefinite_matrix_reports_not_spd():
    cae = _cae()
    A, csr, perm, bp, co = _setup((16, 16), (4, 4))
    vals = csr[2].copy()
    rows = np.repeat(np.arange(256), np.diff(csr[0]))
    vals[csr[1] == rows] -= 5.0
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    with pytest.raises(cae.CAEError) as e:
        cae.Factor(an, torch.from_numpy(vals).cuda(), 1e-6, coarse_max_dim=0)
    assert e.value.code == -3


@pytest.mark.parametrize("dims,late", [((16, 16), False), ((16, 16), True), ((12, 9), True)])
def test_indefinite_dense_remainder_reports_not_spd(dims, late):
    """A matrix that goes whole into the dense remainder (no level is
    factored) and is indefinite: the pivot inverses of the Gauss-Jordan sweep
    meet a non-positive pivot -- in the first 64-unknown panel (its own
    kernel; every diagonal shifted) or only in a later one (inverted inside
    the previous panel's update; diagonals shifted from the second panel
    on) -- and the factorization reports CAE_ENOTSPD; the unshifted matrix
    factors and solves."""
    cae = _cae()
    A, csr, perm, bp, co = _setup(dims, (4, 4))
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(csr[0]))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    vals = csr[2].copy()
    shift = np.ones(n, bool)
    if late:
        shift[:] = False
        shift[np.asarray(perm)[64:]] = True   # unknowns after the first panel of the level order
    vals[(csr[1] == rows) & shift[rows]] -= 5.0
    with pytest.raises(cae.CAEError) as e:
        cae.Factor(an, torch.from_numpy(vals).cuda(), 1e-6, coarse_max_dim=4096)
    assert e.value.code == -3
    f = cae.Factor(an, torch.from_numpy(csr[2]).cuda(), 1e-6, coarse_max_dim=4096)
    assert f.stats()["nlevels"] == 0 and f.stats()["coarse_dim"] == n
    X = _probes(n, 2)
    Z = _from_gpu_cols(f.apply(_to_gpu_cols(X)))
    Ad = A.toarray()
    assert np.linalg.norm(Ad @ Z - X) <= 1e-12 * np.linalg.norm(X) * np.linalg.cond(Ad)


def test_fixed_rank_mode_matches_oracle():
    """CE(r) element parity where every kept subspace is unique (r = 3 on
    4x4 patches: the smallest relative gap sigma_r - sigma_{r+1} is 4e-4)."""
    cae = _cae()
    A, csr, perm, bp, co = _setup((32, 32), (4, 4))
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=0.0, rank_mode="fixed", fixed_rank=3, order="multicolour",
                                                 coarse_max_dim=0))
    an, f = _gpu_factor(cae, csr, perm, bp, co, 0.0, "multicolour", coarse=0, rank_mode=1, fixed_rank=3)
    for l, lf in enumerate(fo.levels):
        assert np.array_equal(f.ranks(l), lf.r)
    X = _probes(A.shape[0])
    Mo = ce_multiply(fo, X)
    Mg = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    assert np.linalg.norm(Mg - Mo) <= 1e-12 * np.linalg.norm(Mo)


def test_fixed_rank_paper_parameters_converge():
    """CE(r) with the paper's recommended r = 4 = B/2 on B = 8 patches: the
    kept subspace is not unique at every step (tied zero singular values), so
    the check is the Frobenius identity of the GPU factor and PCG."""
    cae = _cae()
    A, csr, perm, bp, co = _setup((24, 24), (4, 2))
    an, f = _gpu_factor(cae, csr, perm, bp, co, 0.0, "multicolour", coarse=0, rank_mode=1, fixed_rank=4)
    Ad = A.toarray()
    M = _from_gpu_cols(f.multiply(_to_gpu_cols(np.eye(A.shape[0]))))
    pred = math.sqrt(2 * f.stats()["dropped_sq"])
    assert abs(np.linalg.norm(Ad - M) - pred) <= 1e-8 * pred + 1e-13 * np.linalg.norm(Ad)
    b = problems.rhs_uniform(A.shape[0], 0)
    x, it, rel = f.pcg(torch.from_numpy(b).cuda(), rtol=1e-8)
    assert f.converged and rel[0] <= 1.0001e-8


@pytest.mark.parametrize("dims,patch,eps", [((40, 24), (8, 8), 1e-6), ((8, 8, 8), (2, 2, 2), 1e-4)])
def test_bf16_schur_factor(dims, patch, eps):
    """FP32 factor with BF16-input Schur products (FP32 accumulation on the
    matrix cores): M stays within BF16 rounding of the FP64 oracle (each
    product entry carries a relative error of about 2^-8 of its inputs),
    eps = 0 gives A within that rounding, and PCG to 1e-8 converges with at
    most a few iterations more than the FP64 factor."""
    cae = _cae()
    A, csr, perm, bp, co = _setup(dims, patch)
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, order="multicolour", coarse_max_dim=0))
    an, f = _gpu_factor(cae, csr, perm, bp, co, eps, "multicolour", precision=cae.FP32_BF16, coarse=0)
    X = _probes(A.shape[0])
    MX = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    MXo = ce_multiply(fo, X)
    rel = np.linalg.norm(MX - MXo) / np.linalg.norm(MXo)
    assert rel <= 2e-3, rel
    b = problems.rhs_uniform(A.shape[0], seed=0)
    _, it, relr = f.pcg(torch.from_numpy(b).cuda(), rtol=1e-8)
    _, ito, _ = oracle.pcg(A, b, lambda r: ce_solve(fo, r), tol=1e-8)
    assert f.converged and relr[0] <= 1.0001e-8
    assert it[0] <= ito + 6, (it[0], ito)
    f.close()
    f0 = cae.Factor(an, torch.from_numpy(csr[2]).cuda(), 0.0, precision=cae.FP32_BF16, coarse_max_dim=0)
    A0X = A @ X
    M0X = _from_gpu_cols(f0.multiply(_to_gpu_cols(X)))
    assert np.linalg.norm(M0X - A0X) <= 2e-3 * np.linalg.norm(A0X)
    f0.close()
    an.close()


def test_bf16_schur_factor_with_blocks_above_128():
    """The configured 3D arithmetic (FP32 factor, BF16-input Schur products)
    on the 20^3 Laplacian with sibling coarsening, whose second level holds
    blocks of up to 215 unknowns (the big-block Schur kernel on BF16 matrix
    cores): M within the BF16 bar of the FP64 oracle, every block above 128
    unknowns compressed, and PCG to 1e-8 within a few iterations of the
    oracle's."""
    cae = _cae()
    d = _big_oracle()
    A, csr, perm, bp, co, eps, fo = (d[k] for k in ("A", "csr", "perm", "bp", "co", "eps", "fo"))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co, order=cae.ORDER_MULTICOLOUR)
    f = cae.Factor(an, torch.from_numpy(csr[2]).cuda(), eps, precision=cae.FP32_BF16, coarse_max_dim=0)
    st = f.stats()
    X = _probes(A.shape[0])
    MX = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    MXo = ce_multiply(fo, X)
    rel = np.linalg.norm(MX - MXo) / np.linalg.norm(MXo)
    b = problems.rhs_uniform(A.shape[0], seed=0)
    _, it, relr = f.pcg(torch.from_numpy(b).cuda(), rtol=1e-8)
    _, ito, _ = oracle.pcg(A, b, lambda r: ce_solve(fo, r), tol=1e-8)
    nbig = sum(st[k] for k in ("big_untruncated", "big_frobenius", "big_certified", "big_uncapped"))
    print(f"bf16 (b > 128): probe error vs oracle {rel:.3e}, big compressions {nbig}, PCG {int(it[0])} vs {ito}")
    assert nbig > 0
    assert rel <= 2e-3, rel
    assert f.converged and relr[0] <= 1.0001e-8
    assert it[0] <= ito + 6, (it[0], ito)
    f.close()
    an.close()


def test_compensation_matches_oracle_and_prevents_breakdown():
    """Diagonal compensation on the biharmonic operator, which breaks the
    plain method at eps = 1e-3: the GPU reports CAE_ENOTSPD without it, and
    with it matches the oracle's compensated factor (M X to 1e-10, FP64) and
    converges in PCG."""
    cae = _cae()
    L = problems.laplacian((32, 32))
    B = (L @ L).tocsr()
    B.sort_indices()
    A, csr, perm, bp, co = _setup((32, 32), (4, 4), A=B)
    an = cae.Analysis(csr[0], csr[1], perm, bp, co)
    vals = torch.from_numpy(csr[2]).cuda()
    with pytest.raises(cae.CAEError) as ei:
        cae.Factor(an, vals, 1e-3, precision=cae.FP64, coarse_max_dim=0)
    assert ei.value.code == -3
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=1e-3, order="multicolour", coarse_max_dim=0, compensate=True))
    f = cae.Factor(an, vals, 1e-3, precision=cae.FP64, coarse_max_dim=0, compensate=True)
    X = _probes(A.shape[0])
    MX = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    MXo = ce_multiply(fo, X)
    assert np.linalg.norm(MX - MXo) <= 1e-10 * np.linalg.norm(MXo)
    b = problems.rhs_uniform(A.shape[0], seed=0)
    _, it, rel = f.pcg(torch.from_numpy(b).cuda(), rtol=1e-8)
    assert f.converged and rel[0] <= 1.0001e-8
    f.close()
    f32 = cae.Factor(an, vals, 1e-3, precision=cae.FP32, coarse_max_dim=0, compensate=True)
    _, it32, rel32 = f32.pcg(torch.from_numpy(b).cuda(), rtol=1e-8)
    assert f32.converged
    f32.close()
    an.close()


@pytest.mark.parametrize("eps,order", [(1e-6, "multicolour"), (1e-4, "paper")])
def test_general_sparse_graph_ordering(eps, order):
    """An irregular domain (the grid nodes inside a disk) ordered by nested
    bisection of its graph, blocks of at most 32, pairs of blocks coarsened
    (no coordinates): GPU factor against the oracle on the same ordering."""
    cae = _cae()
    A = problems.disk_laplacian(44)
    csr = problems.to_csr_arrays(A)
    perm, bp = cae.graph_order(csr[0], csr[1], 32)
    fo = ce_factor(*csr, perm, bp, None, CEOptions(eps=eps, order=order, coarse_max_dim=0), J=2)
    an = cae.Analysis(csr[0], csr[1], perm, bp, None,
                      order=cae.ORDER_PAPER if order == "paper" else cae.ORDER_MULTICOLOUR, ndim=1)
    f = cae.Factor(an, torch.from_numpy(csr[2]).cuda(), eps, precision=cae.FP64, coarse_max_dim=0)
    _check_ranks(f, fo)
    X = _probes(A.shape[0])
    MX = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    MXo = ce_multiply(fo, X)
    assert np.linalg.norm(MX - MXo) <= 1e-12 * np.linalg.norm(MXo)
    b = problems.rhs_uniform(A.shape[0], seed=0)
    _, it, rel = f.pcg(torch.from_numpy(b).cuda(), rtol=1e-10)
    _, ito, _ = oracle.pcg(A, b, lambda r: ce_solve(fo, r), tol=1e-10)
    assert it[0] == ito and rel[0] <= 1e-9
    f.close()
    an.close()


@pytest.mark.parametrize("dims,patch,eps", [((16, 16, 16), (4, 4, 4), 1e-4), ((40, 24), (8, 8), 1e-6)])
def test_pairs_coarsening_matches_oracle(dims, patch, eps):
    """Coarsening by pairs along the Morton curve: GPU factor against the
    oracle with the same coarsening (ranks, M X to 1e-12)."""
    cae = _cae()
    A, csr, perm, bp, co = _setup(dims, patch)
    fo = ce_factor(*csr, perm, bp, co, CEOptions(eps=eps, order="multicolour", coarse_max_dim=256, coarsen="pairs"))
    an = cae.Analysis(csr[0], csr[1], perm, bp, co, order=cae.ORDER_MULTICOLOUR, coarsen="pairs")
    f = cae.Factor(an, torch.from_numpy(csr[2]).cuda(), eps, precision=cae.FP64, coarse_max_dim=256)
    _check_ranks(f, fo)
    X = _probes(A.shape[0])
    MX = _from_gpu_cols(f.multiply(_to_gpu_cols(X)))
    assert np.linalg.norm(MX - ce_multiply(fo, X)) <= 1e-12 * np.linalg.norm(MX)
    f.close()
    an.close()
