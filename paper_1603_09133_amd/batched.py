"""Many independent problems in one factorization, and the choice of the
block size B per problem class (autotuner).

The joint problem is assembled by the library (``cae_analyze_batched``,
``cae_factor_batched``): the problems form one block-diagonal matrix, each
keeps its own Morton patch order, and problem t's block coordinates are
offset by t's binary digits above the problem's own coordinate bits, so the
joint Morton order runs problem by problem and the coarsening never joins
blocks of two problems before each has been reduced to one block.  Every
dependency wave of the joint analysis therefore holds the independent steps
of all problems: one launch per wave serves the whole batch.  Right-hand
sides of problem t occupy its rows of every joint column, and
``cae_pcg_solve_batched`` runs an independent PCG per problem.

The autotuner times factorization + PCG on a sample of each problem class
for every candidate patch shape and caches the fastest per (GPU arch, class)
in a JSON file.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import time

import numpy as np

from . import FP32, ORDER_MULTICOLOUR, Analysis, Factor, _lib, _options, grid_order
from ._lib import check, lib, ptr

CANDIDATES = {2: [(8, 8), (4, 4)], 3: [(4, 4, 4), (2, 2, 4)]}


def _problems(mats, dims_list, patches, vals=None):
    """ctypes array of ``cae_problem_t`` and the host arrays it points to."""
    arr = (_lib.Problem * len(mats))()
    keep = []
    for t, (A, dims, patch) in enumerate(zip(mats, dims_list, patches)):
        ip = np.ascontiguousarray(A.indptr, dtype=np.int64)
        ix = np.ascontiguousarray(A.indices, dtype=np.int32)
        keep += [ip, ix]
        P = arr[t]
        P.n = A.shape[0]
        P.row_ptr, P.col_idx = ip.ctypes.data, ix.ctypes.data
        P.vals = None if vals is None else vals[t].data_ptr()
        P.ndim = len(dims)
        for a in range(3):
            P.dims[a] = int(dims[a]) if a < len(dims) else 1
            P.patch[a] = int(patch[a]) if a < len(patch) else (1 if len(patch) else 0)
    return arr, keep


def analyze(mats, dims_list, patches, order=ORDER_MULTICOLOUR, coarsen="siblings"):
    """Joint symbolic analysis of the problems (CSR matrices with sorted
    columns on tensor grids ``dims_list``, patch shapes ``patches``):
    ``cae_analyze_batched``, host only."""
    arr, keep = _problems(mats, dims_list, patches)
    o = _options(order=order)
    o.coarsen = {"siblings": 0, "pairs": 1}[coarsen]
    h = C.c_void_p()
    check(lib().cae_analyze_batched(len(mats), arr, C.byref(o), C.byref(h)))
    return Analysis._adopt(h, int(sum(A.shape[0] for A in mats)), order)


def stacked_values(mats, device="cuda"):
    """The problems' CSR values stacked in the joint order (FP64 tensor)."""
    import torch
    return torch.from_numpy(np.concatenate([np.asarray(A.data, dtype=np.float64) for A in mats])).to(device)


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
    """Factorization and PCG of many independent problems at once
    (``cae_factor_batched`` and ``cae_pcg_solve_batched``)."""

    def __init__(self, mats, dims_list, patches, eps, precision=FP32, order=ORDER_MULTICOLOUR, **factor_kw):
        import torch
        self.mats = [m.tocsr() for m in mats]
        for m in self.mats:
            m.sort_indices()
        self.dims_list, self.patches = list(dims_list), list(patches)
        self.row_off = np.concatenate([[0], np.cumsum([m.shape[0] for m in self.mats])]).astype(np.int64)
        self.vals = [torch.from_numpy(np.asarray(m.data, dtype=np.float64)).cuda() for m in self.mats]
        self.eps, self.precision, self.order, self.kw = eps, precision, order, factor_kw
        self.factor = None

    def factorize(self):
        if self.factor is not None:
            self.factor.close()
        arr, keep = _problems(self.mats, self.dims_list, self.patches, self.vals)
        f = Factor.__new__(Factor)
        f.analysis, f.n, f._stream, f.row_off = None, int(self.row_off[-1]), None, self.row_off
        f._keep = (self.kw.get("mlp_params"), self.kw.get("record"), self.kw.get("workspace"))
        f._opts = _options(order=self.order, precision=self.precision, **self.kw)
        h = C.c_void_p()
        check(lib().cae_factor_batched(len(self.mats), arr, float(self.eps), C.byref(f._opts), C.byref(h)))
        f._h = h
        self.factor = f
        return f

    def pcg(self, B, rtol=1e-8, maxit=1000):
        """B: (nrhs, N) CUDA tensor of the joint right-hand sides; an
        independent PCG per problem.  Returns ``(X, iters, relres)`` with
        per-(problem, column) ``iters`` and ``relres``."""
        return self.factor.pcg_batched(B, rtol=rtol, maxit=maxit)

    def problem_residuals(self, B, X):
        """Relative residual of every problem and column (host check)."""
        Bh, Xh = B.cpu().numpy(), X.cpu().numpy()
        out = np.zeros((len(self.mats), Bh.shape[0]))
        for t, A in enumerate(self.mats):
            s = slice(self.row_off[t], self.row_off[t + 1])
            R = Bh[:, s] - (A @ Xh[:, s].T).T
            out[t] = np.linalg.norm(R, axis=1) / np.maximum(np.linalg.norm(Bh[:, s], axis=1), 1e-300)
        return out

    def close(self):
        if self.factor is not None:
            self.factor.close()
            self.factor = None
