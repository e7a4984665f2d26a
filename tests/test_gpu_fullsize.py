"""The headline workload at its full size, in the launch configuration the
benchmark times: 2D 5-point Laplacian 1024 x 1024 (N = 1048576), 8 x 8
Morton patches (B = 64), eps = 1e-6, multicolour order, dense remainder up to
2048 unknowns, FP64 and FP32 factors.  The oracle cannot factor a million
unknowns in a test, so the GPU factor is checked through properties that hold
at any size:

* M^{-1} (M X) = X: to rounding for the FP64 factor; for the FP32 factor to
  about 1e-5, since the apply uses the stored L_nn^{-1}, itself rounded to
  FP32, which inverts the stored L_nn only to FP32 rounding times its
  condition;
* M^{-1} is symmetric: x^T M^{-1} y = y^T M^{-1} x;
* ||A0 - M||_F^2 = 2 sum_i ||E_i||_F^2 (FP64 factor; the identity of the
  dropped blocks that the small-grid test checks exactly), estimated with
  Gaussian probes: E ||(A0 - M) x||^2 = ||A0 - M||_F^2 for x ~ N(0, I);
* PCG (FP64) reaches 1e-8 on 16 right-hand sides N(0,1) seed 1, the true
  residual recomputed on the host, with the FP32 factor in no more iterations
  than the FP64 factor.
"""
import numpy as np
import pytest

import problems

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cols(X):
    return torch.from_numpy(np.ascontiguousarray(X.T)).cuda()


def _np(T):
    return T.cpu().numpy().T


def test_laplacian_1024_full_size_properties():
    import paper_1603_09133_amd as cae
    cae.lib()
    dims, patch, eps = (1024, 1024), (8, 8), 1e-6
    A = problems.laplacian(dims)
    ip, ix, dv = problems.to_csr_arrays(A)
    perm, bp, co = cae.grid_order(dims, patch)
    an = cae.Analysis(ip, ix, perm, bp, co)
    vals = torch.from_numpy(dv).cuda()
    N = A.shape[0]
    rng = np.random.default_rng(12345)
    X = rng.standard_normal((N, 8))
    AX = A @ X
    B = problems.rhs_normal(N, 16, seed=1)
    iters = {}
    for name, prec in (("fp64", cae.FP64), ("fp32", cae.FP32)):
        print(f"factor {name}", flush=True)
        f = cae.Factor(an, vals, eps, precision=prec)
        st = f.stats()
        MX = _np(f.multiply(_cols(X)))
        Z = _np(f.apply(_cols(MX)))
        err = np.linalg.norm(Z - X) / np.linalg.norm(X)
        print(f"{name}: levels {st['nlevels']}, coarse {st['coarse_dim']}, |M^-1 M X - X| / |X| = {err:.2e}",
              flush=True)
        assert err <= (1e-9 if name == "fp64" else 1e-4)
        W = _np(f.apply(_cols(X[:, :2])))
        s01, s10 = X[:, 0] @ W[:, 1], X[:, 1] @ W[:, 0]
        assert abs(s01 - s10) <= 1e-10 * np.linalg.norm(X[:, 0]) * np.linalg.norm(W[:, 1])
        if name == "fp64":
            est = np.mean(np.sum((AX - MX) ** 2, axis=0))
            pred = 2.0 * st["dropped_sq"]
            print(f"probe estimate of ||A0 - M||_F^2 {est:.4e}, 2 sum ||E_i||^2 {pred:.4e}", flush=True)
            assert pred > 0 and abs(est / pred - 1.0) <= 0.1
        x, it, rel = f.pcg(_cols(B), rtol=1e-8, maxit=1000)
        assert f.converged
        xs = _np(x)
        true_rel = np.linalg.norm(B - A @ xs, axis=0) / np.linalg.norm(B, axis=0)
        print(f"{name}: PCG iterations {sorted(set(it.tolist()))}, true relative residual max {true_rel.max():.2e}",
              flush=True)
        assert np.all(rel <= 1.0001e-8) and np.all(true_rel <= 2e-8)
        iters[name] = it
        f.close()
    assert np.all(iters["fp32"] <= iters["fp64"])
