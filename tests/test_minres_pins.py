"""Pins of the oracle's MINRES and of the paper's Section 3 problem.

MINRES is fixed by its definition: the k-th iterate minimises the residual
norm over a Krylov space.  Brute force on small matrices (explicit Krylov
basis, least squares) pins the recurrences of ``oracle.minres``:
* without preconditioner: x_k = argmin_{x in K_k(A, b)} ||b - A x||_2;
* with an SPD preconditioner P = M^{-1}:
  x_k = argmin_{x in K_k(P A, P b)} ||b - A x||_P  (||r||_P^2 = r^T P r).
"""
import numpy as np
import pytest

import oracle
import problems


def _spd(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def _krylov_argmin(A, b, P, k):
    """argmin over K_k(P A, P b) of ||b - A x||_P, by an orthonormal basis."""
    z = P @ b
    K = [z]
    for _ in range(k - 1):
        K.append(P @ (A @ K[-1]))
    Qk, _ = np.linalg.qr(np.stack(K, axis=1))
    C = np.linalg.cholesky(P).T                      # P = C^T C
    c, *_ = np.linalg.lstsq(C @ A @ Qk, C @ b, rcond=None)
    return Qk @ c


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_minres_unpreconditioned_is_krylov_least_squares(k):
    A = _spd(30, 1)
    b = np.random.default_rng(2).standard_normal(30)
    x, it, _ = oracle.minres(A, b, lambda r: r, tol=0.0, maxit=k)
    assert it == k
    xr = _krylov_argmin(A, b, np.eye(30), k)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_minres_preconditioned_is_krylov_least_squares(k):
    A = _spd(25, 3, cond=200.0)
    P = _spd(25, 4, cond=10.0)
    b = np.random.default_rng(5).standard_normal(25)
    x, it, _ = oracle.minres(A, b, lambda r: P @ r, tol=0.0, maxit=k)
    assert it == k
    xr = _krylov_argmin(A, b, P, k)
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)


def test_minres_stopping_norm_and_exact_preconditioner():
    A = _spd(40, 6, cond=1e3)
    b = np.random.default_rng(7).standard_normal(40)
    P = np.linalg.inv(A)
    # M = A: the preconditioned operator is the identity, one iteration is exact
    x, it, rel = oracle.minres(A, b, lambda r: P @ r, tol=1e-12, maxit=10)
    assert it == 1 and rel < 1e-10
    # the monitored phibar is the P-norm of the true residual
    Pd = _spd(40, 8, cond=5.0)
    x, it, rel = oracle.minres(A, b, lambda r: Pd @ r, tol=1e-6, maxit=200)
    r = b - A @ x
    beta1 = np.sqrt(b @ Pd @ b)
    assert np.sqrt(r @ Pd @ r) <= 1e-6 * beta1 * (1 + 1e-6)
    x2, it2, _ = oracle.minres(A, b, lambda r: Pd @ r, tol=1e-6, maxit=it - 1)
    r2 = b - A @ x2
    assert np.sqrt(r2 @ Pd @ r2) > 1e-6 * beta1


def test_minres_agrees_with_cg_on_spd_in_the_limit():
    A = problems.laplacian((12, 12)).toarray()
    b = problems.rhs_uniform(144, seed=0)
    x, it, rel = oracle.minres(A, b, lambda r: r, tol=1e-12, maxit=500)
    assert rel < 1e-10
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-9 * np.linalg.norm(x)


def test_aniso_rectangular_grid_reduces_to_cubic_and_is_spd():
    A = problems.anisotropic_diffusion_3d(5)
    B = problems.anisotropic_diffusion_3d((5, 5, 5))
    assert (A != B).nnz == 0
    C = problems.anisotropic_diffusion_3d((6, 4, 3)).toarray()
    assert np.abs(C - C.T).max() == 0.0
    assert np.linalg.eigvalsh(C).min() > 0
    # 7-point pattern: at most 7 entries per row, constant-k limit is the Laplacian scaled by h^2
    assert max(np.count_nonzero(row) for row in C) <= 7
