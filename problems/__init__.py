"""Seeded synthetic SPD problems and right-hand sides.

This module is shared by the FP64 oracle (``oracle/``) and the GPU path
(``paper_1603_09133_amd``).  It holds none of the factorization's arithmetic:
it only builds the sparse test matrices and the random right-hand sides that
both sides consume, in the natural grid ordering (x fastest).

Matrices (all symmetric positive definite, homogeneous Dirichlet boundary,
boundary nodes are not unknowns, mesh factor h^2 removed):

* ``laplacian(dims)``: 2D 5-point (diagonal 4, off-diagonal -1) or 3D
  7-point (diagonal 6, off-diagonal -1) stencil on an ``dims`` grid.
* ``grf_diffusion_2d(n, ...)``: 2D ``-div(k grad u)`` with the 5-point
  harmonic-mean stencil and ``k = exp(g)``, ``g`` a Gaussian random field with
  squared-exponential covariance, sampled exactly through the separable
  Kronecker factorisation of the covariance.
* ``anisotropic_diffusion_3d(n)``: the paper's test problem of Section 3:
  3D ``div(k grad u)`` on the unit cube with ``k = diag(x1^2+0.5, x2^2+0.5,
  x3^2+0.5)`` (equidistant grid, face-centred coefficients).

CSR arrays are returned as ``(indptr int64, indices int32, data float64)``
with sorted column indices and an explicit diagonal.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

__all__ = [
    "laplacian",
    "grf_diffusion_2d",
    "anisotropic_diffusion_3d",
    "to_csr_arrays",
    "rhs_uniform",
    "rhs_normal",
    "batched_problem_draws",
]


def to_csr_arrays(A: sp.spmatrix):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return (A.indptr.astype(np.int64), A.indices.astype(np.int32),
            A.data.astype(np.float64))


def _tridiag(n: int) -> sp.csr_matrix:
    e = np.ones(n)
    return sp.diags([-e[:-1], 2.0 * e, -e[:-1]], [-1, 0, 1], format="csr")


def laplacian(dims) -> sp.csr_matrix:
    """Unscaled Dirichlet Laplacian on a tensor grid ``dims`` (x fastest)."""
    dims = tuple(int(d) for d in dims)
    if len(dims) not in (1, 2, 3) or min(dims) < 1:
        raise ValueError("dims must hold 1..3 positive sizes")
    N = int(np.prod(dims))
    A = sp.csr_matrix((N, N))
    for k, nk in enumerate(dims):
        # axis k varies with stride prod(dims[:k]); kron order is slowest-first.
        mats = []
        for j in reversed(range(len(dims))):
            mats.append(_tridiag(dims[j]) if j == k else sp.identity(dims[j], format="csr"))
        T = mats[0]
        for m in mats[1:]:
            T = sp.kron(T, m, format="csr")
        A = A + T
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A


def _grf_2d(n: int, length: float, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Exact sample of a 2D GRF on nodes x_i=(i+1)/(n+1), covariance
    sigma^2 exp(-|x-y|^2/(2 length^2)) = C1 (x) C1, via g = S Xi S^T."""
    x = (np.arange(n) + 1.0) / (n + 1.0)
    C1 = np.exp(-((x[:, None] - x[None, :]) ** 2) / (2.0 * length ** 2))
    lam, V = np.linalg.eigh(C1)
    S = V * np.sqrt(np.clip(lam, 0.0, None))[None, :]
    Xi = rng.standard_normal((n, n))
    g = sigma * (S @ Xi @ S.T)      # g[iy, ix]
    return g


def grf_diffusion_2d(n: int, length: float = 0.05, sigma: float = 1.0,
                     rng: np.random.Generator | None = None, seed: int = 2):
    """2D -div(k grad u), 5-point harmonic-mean stencil, k = exp(GRF).

    Returns ``(A, rng)``: the CSR matrix and the generator, positioned after
    the field draw so that the caller can draw the right-hand sides from it.
    Face coefficient between nodes p, q is 2 k_p k_q / (k_p + k_q); a face to
    the Dirichlet boundary uses k_p.  The diagonal is the sum of the 4 faces.
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    k = np.exp(_grf_2d(n, length, sigma, rng))     # k[iy, ix]
    kx = 2.0 * k[:, :-1] * k[:, 1:] / (k[:, :-1] + k[:, 1:])   # faces between ix, ix+1
    ky = 2.0 * k[:-1, :] * k[1:, :] / (k[:-1, :] + k[1:, :])   # faces between iy, iy+1
    diag = np.zeros((n, n))
    diag[:, :-1] += kx
    diag[:, 1:] += kx
    diag[:-1, :] += ky
    diag[1:, :] += ky
    # boundary faces: use k_p
    diag[:, 0] += k[:, 0]
    diag[:, -1] += k[:, -1]
    diag[0, :] += k[0, :]
    diag[-1, :] += k[-1, :]
    idx = np.arange(n * n).reshape(n, n)
    rows = [idx.ravel(), idx[:, :-1].ravel(), idx[:, 1:].ravel(), idx[:-1, :].ravel(), idx[1:, :].ravel()]
    cols = [idx.ravel(), idx[:, 1:].ravel(), idx[:, :-1].ravel(), idx[1:, :].ravel(), idx[:-1, :].ravel()]
    vals = [diag.ravel(), -kx.ravel(), -kx.ravel(), -ky.ravel(), -ky.ravel()]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n * n, n * n))
    A.sort_indices()
    return A, rng


def anisotropic_diffusion_3d(n) -> sp.csr_matrix:
    """The paper's Section 3 problem, div(k grad u)=f on [0,1]^3, Dirichlet,
    k = diag(x1^2+0.5, x2^2+0.5, x3^2+0.5), on the equidistant interior grid
    ``n`` (an int for n^3, or ``(n1, n2, n3)``, x fastest; spacing h_a =
    1/(n_a+1) per axis).  Written with the sign that makes the matrix SPD;
    face coefficients are evaluated at face midpoints and axis a carries
    k_a / h_a^2, scaled by h_1^2 (so h^2 is removed on a cubic grid)."""
    dims = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    nx, ny, nz = dims
    N = nx * ny * nz
    idx = np.arange(N).reshape(nz, ny, nx)        # idx[z, y, x]
    diag = np.zeros((nz, ny, nx))
    rows, cols, vals = [], [], []
    h1 = 1.0 / (nx + 1)
    for axis, na in ((2, nx), (1, ny), (0, nz)):
        h = 1.0 / (na + 1)
        faces = (np.arange(na + 1) + 0.5) * h      # midpoints between nodes i-1..i (i=0..na)
        kf = (faces ** 2 + 0.5) * (h1 / h) ** 2    # coefficient of the matching axis
        # coefficient on the face between node i and i+1 along the axis: kf[i+1]
        c = kf[1:-1]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, na - 1)
        hi[axis] = slice(1, na)
        shp = [1, 1, 1]
        shp[axis] = na - 1
        cc = np.broadcast_to(c.reshape(shp), idx[tuple(lo)].shape)
        diag[tuple(lo)] += cc
        diag[tuple(hi)] += cc
        rows += [idx[tuple(lo)].ravel(), idx[tuple(hi)].ravel()]
        cols += [idx[tuple(hi)].ravel(), idx[tuple(lo)].ravel()]
        vals += [-cc.ravel(), -cc.ravel()]
        # boundary faces
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = 0
        last[axis] = na - 1
        diag[tuple(first)] += kf[0]
        diag[tuple(last)] += kf[na]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    A.sort_indices()
    return A


def rhs_ones(N: int) -> np.ndarray:
    """The paper's right-hand side f = 1 (with the h^2 of the stencil removed,
    a constant vector)."""
    return np.ones(N, dtype=np.float64)


def disk_laplacian(n: int) -> sp.csr_matrix:
    """5-point Laplacian (4/-1, Dirichlet) on the nodes of an n x n grid that
    lie inside the inscribed disk: an irregular domain without a tensor-grid
    block structure (for graph orderings)."""
    c = (n - 1) / 2.0
    yy, xx = np.mgrid[0:n, 0:n]
    inside = (xx - c) ** 2 + (yy - c) ** 2 <= (n / 2.0) ** 2
    idx = -np.ones((n, n), dtype=np.int64)
    idx[inside] = np.arange(int(inside.sum()))
    rows, cols, vals = [], [], []
    N = int(inside.sum())
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(np.full(N, 4.0))
    for dy, dx in ((0, 1), (1, 0)):
        a = idx[: n - dy, : n - dx]
        b = idx[dy:, dx:]
        m = (a >= 0) & (b >= 0)
        rows += [a[m], b[m]]
        cols += [b[m], a[m]]
        vals += [-np.ones(m.sum()), -np.ones(m.sum())]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    A.sort_indices()
    return A


def rhs_uniform(N: int, seed: int = 0) -> np.ndarray:
    """One RHS, i.i.d. U(-1, 1)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, N)


def rhs_normal(N: int, nrhs: int, seed: int | None = None,
               rng: np.random.Generator | None = None) -> np.ndarray:
    """``nrhs`` right-hand sides, i.i.d. N(0,1), column-major ``(N, nrhs)``;
    column k is row k of ``standard_normal((nrhs, N))``."""
    if rng is None:
        rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((nrhs, N)).T)


def batched_problem_draws(nprob: int = 256, seed: int = 3):
    """Draws for the batch of uneven problems: kind (0 = 2D, 1 = 3D), then one
    side per problem (2D: [64, 512], 3D: [16, 64]), in this order."""
    rng = np.random.default_rng(seed)
    kind = rng.integers(0, 2, nprob)
    sides = np.array([rng.integers(64, 513) if k == 0 else rng.integers(16, 65) for k in kind])
    return kind, sides, rng
