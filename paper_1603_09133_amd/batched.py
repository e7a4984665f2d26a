"""Many independent problems in one factorization, and the choice of the
block size B per problem class (autotuner).

The problems are joined into one block-diagonal matrix.  Each keeps its own
Morton patch order; problem t is placed at block coordinates offset by
``t``'s own Morton digits above the problem's coordinate bits, so the joint
Morton order is problem by problem and the coarsening never joins blocks of
two problems before each has been reduced to one block.  Every dependency
wave of the joint analysis therefore holds the independent steps of all
problems: one launch per wave serves the whole batch.  Right-hand sides of
problem t occupy its rows of every joint column.

The autotuner times factorization + PCG on a sample of each problem class
for every candidate patch shape and caches the fastest per (GPU arch, class)
in a JSON file.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import scipy.sparse as sp

from . import FP32, ORDER_MULTICOLOUR, Analysis, Factor, grid_order

CANDIDATES = {2: [(8, 8), (4, 4)], 3: [(4, 4, 4), (2, 2, 4)]}
SHIFT = 8   # coordinate bits reserved per problem and axis


def _spread3(t):
    """Split t into three integers whose Morton interleave is t."""
    out = [0, 0, 0]
    bit = 0
    while t >> bit:
        out[bit % 3] |= ((t >> bit) & 1) << (bit // 3)
        bit += 1
    return out


def assemble(mats, dims_list, patches):
    """Join problems (CSR matrices on tensor grids ``dims_list``, patch shapes
    ``patches``) into one.  Returns ``(A, perm, block_ptr, coords, row_off)``:
    the block-diagonal CSR matrix, the joint permutation, blocks and 3D block
    coordinates, and the first row of every problem."""
    perms, bps, cos, offs = [], [], [], [0]
    nb = 0
    for t, (A, dims, patch) in enumerate(zip(mats, dims_list, patches)):
        p, bp, co = grid_order(dims, patch)
        if co.shape[1] < 3:
            co = np.concatenate([co, np.zeros((co.shape[0], 3 - co.shape[1]), np.int32)], axis=1)
        if co.max() >= (1 << SHIFT):
            raise ValueError("problem too large for the coordinate budget")
        sx, sy, sz = _spread3(t)
        co = co + np.array([sx << SHIFT, sy << SHIFT, sz << SHIFT], np.int32)
        perms.append(p.astype(np.int64) + offs[-1])
        bps.append(bp[:-1].astype(np.int64) + offs[-1])
        cos.append(co)
        offs.append(offs[-1] + A.shape[0])
        nb += len(bp) - 1
    A = sp.block_diag(mats, format="csr")
    A.sort_indices()
    perm = np.concatenate(perms).astype(np.int32)
    block_ptr = np.concatenate(bps + [np.array([offs[-1]])]).astype(np.int32)
    coords = np.concatenate(cos).astype(np.int32)
    return A, perm, block_ptr, coords, np.array(offs, np.int64)


def _cache_path(path=None):
    if path:
        return path
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_1603_09133_amd", "autotune.json")


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def autotune(ndim, side, make_matrix, eps=1e-6, precision=FP32, cache=None, nrhs=4, sample_side=None,
             candidates=None):
    """Patch shape for problems of dimension ``ndim`` and the size class of
    ``side``: the cached choice, else the fastest candidate measured on a
    sample problem (``make_matrix(side) -> CSR``)."""
    import torch

    import problems
    cls = f"{ndim}d-{int(np.ceil(np.log2(max(side, 2))))}"
    key = f"{_arch()}/{cls}/eps{eps:g}/p{precision}"
    path = _cache_path(cache)
    table = {}
    if os.path.exists(path):
        with open(path) as fh:
            table = json.load(fh)
    if key in table:
        return tuple(table[key]["patch"])
    s = sample_side or side
    A = make_matrix(s)
    ip, ix, dv = problems.to_csr_arrays(A)
    dims = (s,) * ndim
    vals = torch.from_numpy(dv).cuda()
    b = torch.from_numpy(np.ascontiguousarray(problems.rhs_normal(A.shape[0], nrhs, seed=0).T)).cuda()
    best, best_t = None, np.inf
    times = {}
    for patch in candidates or CANDIDATES[ndim]:
        perm, bp, co = grid_order(dims, patch)
        an = Analysis(ip, ix, perm, bp, co, order=ORDER_MULTICOLOUR)
        ts = []
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f = Factor(an, vals, eps, precision=precision)
            f.pcg(b, rtol=1e-8)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            f.close()
        an.close()
        times[str(patch)] = min(ts)
        if min(ts) < best_t:
            best, best_t = patch, min(ts)
    table[key] = {"patch": list(best), "times_s": times}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1)
    return tuple(best)


class Batch:
    """Factorization and PCG of many independent problems at once."""

    def __init__(self, mats, dims_list, patches, eps, precision=FP32, order=ORDER_MULTICOLOUR, **factor_kw):
        import torch
        import problems
        self.A, perm, bp, co, self.row_off = assemble(mats, dims_list, patches)
        ip, ix, dv = problems.to_csr_arrays(self.A)
        self.analysis = Analysis(ip, ix, perm, bp, co, order=order)
        self.vals = torch.from_numpy(dv).cuda()
        self.eps, self.precision, self.kw = eps, precision, factor_kw
        self.factor = None

    def factorize(self):
        if self.factor is not None:
            self.factor.close()
        self.factor = Factor(self.analysis, self.vals, self.eps, precision=self.precision, **self.kw)
        return self.factor

    def pcg(self, B, rtol=1e-8, maxit=1000):
        """B: (nrhs, N) CUDA tensor of the joint right-hand sides."""
        return self.factor.pcg(B, rtol=rtol, maxit=maxit)

    def problem_residuals(self, B, X):
        """Relative residual of every problem and column (host check)."""
        Bh, Xh = B.cpu().numpy(), X.cpu().numpy()
        R = Bh - (self.A @ Xh.T).T
        out = np.zeros((len(self.row_off) - 1, Bh.shape[0]))
        for t in range(len(self.row_off) - 1):
            s = slice(self.row_off[t], self.row_off[t + 1])
            out[t] = np.linalg.norm(R[:, s], axis=1) / np.maximum(np.linalg.norm(Bh[:, s], axis=1), 1e-300)
        return out

    def close(self):
        if self.factor is not None:
            self.factor.close()
            self.factor = None
        self.analysis.close()
