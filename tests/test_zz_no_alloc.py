"""The allocation-free apply (cae_apply_precond_noalloc) against the apply
that uses the handle's own work vectors (cae_apply_precond), through the C
ABI: two calls in a row, the second on a smaller problem with fewer
right-hand sides, both equal to the ordinary apply to the parity bar of the
apply (1e-10 relative; the kernels are the same, so in fact bitwise); and a
call whose work vectors exceed the scratch array is refused before anything
is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

import problems

pytestmark = pytest.mark.gpu


def _factor(cae, dims, patch, eps, precision):
    A = problems.laplacian(dims)
    ip, ix, dv = problems.to_csr_arrays(A)
    perm, bp, co = cae.grid_order(dims, patch)
    an = cae.Analysis(ip, ix, perm, bp, co)
    return A.shape[0], an, cae.Factor(an, torch.from_numpy(dv).cuda(), eps, precision=precision)


def _both(cae, f, n, nrhs, seed):
    r = torch.from_numpy(np.ascontiguousarray(problems.rhs_normal(n, nrhs, seed=seed).T)).cuda()
    z_ref = torch.full_like(r, np.nan)
    z_new = torch.full_like(r, np.nan)
    L = cae.lib()
    cae.check(L.cae_apply_precond(f._h, nrhs, r.data_ptr(), n, z_ref.data_ptr(), n))
    cae.check(L.cae_apply_precond_noalloc(f._h, nrhs, r.data_ptr(), n, z_new.data_ptr(), n, None))
    torch.cuda.synchronize()
    return z_ref.cpu().numpy(), z_new.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_apply_equals_apply_two_calls(precision):
    import paper_1603_09133_amd as cae
    n1, an1, f1 = _factor(cae, (96, 80), (8, 8), 1e-6, precision)
    n2, an2, f2 = _factor(cae, (40, 36), (4, 4), 1e-4, precision)
    try:
        for f, n, nrhs, seed in ((f1, n1, 5, 11), (f2, n2, 2, 12)):
            z_ref, z_new = _both(cae, f, n, nrhs, seed)
            assert np.all(np.isfinite(z_new))
            err = np.linalg.norm(z_new - z_ref) / np.linalg.norm(z_ref)
            print(f"n={n} nrhs={nrhs}: relative difference {err:.3e}")
            assert err <= 1e-10
            assert np.array_equal(z_new, z_ref)
    finally:
        f1.close()
        f2.close()
        an1.close()
        an2.close()


def test_noalloc_apply_refuses_work_beyond_its_scratch():
    import paper_1603_09133_amd as cae
    n, an, f = _factor(cae, (64, 64), (8, 8), 1e-6, 0)
    try:
        nrhs = 2048   # level vectors of about 2 n nrhs doubles: more than 64 MiB
        r = torch.zeros((nrhs, n), dtype=torch.float64, device="cuda")
        z = torch.full_like(r, 7.0)
        rc = cae.lib().cae_apply_precond_noalloc(f._h, nrhs, r.data_ptr(), n, z.data_ptr(), n, None)
        torch.cuda.synchronize()
        assert rc == cae._lib.CAE_EINVAL
        assert b"limit is" in cae.lib().cae_last_error(None)
        assert bool(torch.all(z == 7.0))   # nothing was enqueued
        # a size within the limit still works after the refusal
        z_ref, z_new = _both(cae, f, n, 3, 13)
        assert np.array_equal(z_new, z_ref)
    finally:
        f.close()
        an.close()
