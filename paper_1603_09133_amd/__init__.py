"""Compress-and-eliminate (CE) approximate block Cholesky on MI355X.

Thin Python layer over the C ABI of ``libcae.so`` (``include/cae.h``):

* :func:`grid_order` -- Morton patch permutation of a tensor grid;
* :class:`Analysis` -- host symbolic analysis (patterns, orders, waves);
* :class:`Factor` -- GPU factorization ``A ~ Q^T L L^T Q`` with
  :meth:`Factor.apply` (``M^{-1}``), :meth:`Factor.multiply` (``M``) and
  :meth:`Factor.pcg` (FP64 PCG preconditioned by ``M^{-1}``).

Vectors are PyTorch FP64 tensors on the GPU of shape ``(N,)`` or
``(nrhs, N)`` (one right-hand side per row, i.e. column-major ``N x nrhs``).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (CAEError, FP32, FP32_BF16, FP64, ORDER_MULTICOLOUR, ORDER_PAPER, RANK_EPS, RANK_FIXED, RANK_LEARNED,
                   RANK_LEARNED_CAP,
                   RECORD_WIDTH, check, lib, ptr)

__all__ = ["grid_order", "graph_order", "Analysis", "Factor", "CAEError", "FP64", "FP32", "FP32_BF16", "ORDER_PAPER",
           "ORDER_MULTICOLOUR", "RANK_EPS", "RANK_FIXED", "RANK_LEARNED", "RECORD_WIDTH", "lib"]


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _i64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def grid_order(dims, patch):
    """Morton patch permutation: returns ``perm`` (new -> old), ``block_ptr``
    and the patch ``coords`` (int32 NumPy arrays)."""
    nd = len(dims)
    d, p = _i32(dims), _i32(patch)
    nb = C.c_int32()
    check(lib().cae_grid_order(nd, ptr(d), ptr(p), None, None, None, C.byref(nb)))
    n = int(np.prod(d.astype(np.int64)))
    perm = np.empty(n, np.int32)
    bp = np.empty(nb.value + 1, np.int32)
    co = np.empty((nb.value, nd), np.int32)
    check(lib().cae_grid_order(nd, ptr(d), ptr(p), ptr(perm), ptr(bp), ptr(co), C.byref(nb)))
    return perm, bp, co


def graph_order(indptr, indices, B):
    """Nested-bisection permutation of a general sparse graph: returns
    ``perm`` (new -> old) and ``block_ptr`` (blocks of at most ``B``); analyse
    with ``coords=None`` and ``J=2`` (``Analysis(..., coords=None, ndim=1)``)."""
    ip, ix = _i64(indptr), _i32(indices)
    n = len(ip) - 1
    nb = C.c_int32()
    check(lib().cae_graph_order(n, ptr(ip), ptr(ix), int(B), None, None, C.byref(nb)))
    perm = np.empty(n, np.int32)
    bp = np.empty(nb.value + 1, np.int32)
    check(lib().cae_graph_order(n, ptr(ip), ptr(ix), int(B), ptr(perm), ptr(bp), C.byref(nb)))
    return perm, bp


def _options(order=ORDER_MULTICOLOUR, precision=FP64, rank_mode=RANK_EPS, fixed_rank=0, max_levels=0,
             coarse_max_dim=2048, stream=None, timing=False, mlp_params=None, seed=0, record=None,
             compensate=False, graphs=True, apply_split_steps=None, workspace=None, big_pivot_cap=0):
    o = _lib.Options()
    lib().cae_default_options(C.byref(o))
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.compensate = 1 if compensate else 0
    o.graphs = 1 if graphs else 0
    if apply_split_steps is not None:
        o.apply_split_steps = int(apply_split_steps)
    o.mlp_params = None if mlp_params is None else mlp_params.data_ptr()
    o.seed = int(seed)
    o.record = None if record is None else record.data_ptr()
    o.record_cap = 0 if record is None else record.shape[0]
    o.order = order
    o.precision = precision
    o.rank_mode = rank_mode
    o.fixed_rank = fixed_rank
    o.max_levels = max_levels
    o.coarse_max_dim = coarse_max_dim
    o.stream = stream
    o.timing = 1 if timing else 0
    o.big_pivot_cap = int(big_pivot_cap)
    return o


class Analysis:
    """Symbolic analysis of a CSR pattern with a permutation and blocks."""

    def __init__(self, indptr, indices, perm, block_ptr=None, coords=None, B=0, order=ORDER_MULTICOLOUR,
                 ndim=None, coarsen="siblings"):
        """Without ``coords`` consecutive groups of ``2**ndim`` blocks form the
        next level (``ndim=1``: pairs, as for :func:`graph_order`).  With
        coordinates, ``coarsen="siblings"`` joins the 2^d Morton siblings,
        ``"pairs"`` joins pairs along the Morton curve (axes in turn)."""
        self._ip, self._ix = _i64(indptr), _i32(indices)
        self._perm = _i32(perm)
        n = len(self._ip) - 1
        bp = None if block_ptr is None else _i32(block_ptr)
        co = None if coords is None else _i32(coords)
        if co is not None:
            ndim = co.shape[1] if co.ndim == 2 else 1
        elif ndim is None:
            ndim = 0
        nb = 0 if bp is None else len(bp) - 1
        self.order = order
        self.n = n
        o = _options(order=order)
        o.coarsen = {"siblings": 0, "pairs": 1}[coarsen]
        h = C.c_void_p()
        check(lib().cae_analyze(n, ptr(self._ip), ptr(self._ix), ptr(self._perm), ptr(bp), nb, int(B), ptr(co),
                                ndim, C.byref(o), C.byref(h)))
        self._h = h

    @classmethod
    def _adopt(cls, h, n, order, keep=()):
        """Wrap an analysis handle made by another entry point (owned)."""
        self = cls.__new__(cls)
        self._h, self.n, self.order, self._keep = h, n, order, keep
        return self

    @property
    def handle(self):
        return self._h

    def batch_rows(self):
        """First row of every problem of a batched analysis (``nprob + 1``
        entries; one problem for an analysis of one matrix)."""
        k = C.c_int32()
        check(lib().cae_analysis_batch_rows(self._h, C.byref(k), None))
        out = np.empty(k.value + 1, np.int64)
        check(lib().cae_analysis_batch_rows(self._h, C.byref(k), ptr(out)))
        return out

    def nlevels(self):
        v = C.c_int32()
        check(lib().cae_analysis_levels(self._h, C.byref(v)))
        return v.value

    def level_info(self, level):
        info = _lib.LevelInfo()
        check(lib().cae_analysis_level_info(self._h, level, C.byref(info)))
        return {k: getattr(info, k) for k, _ in _lib.LevelInfo._fields_}

    def level_arrays(self, level):
        inf = self.level_info(level)
        M = inf["M"]
        order = np.empty(M, np.int32)
        wave = np.empty(M, np.int32)
        cp = np.empty((inf["nclose"], 2), np.int32)
        fp = np.empty((inf["nfar"], 2), np.int32)
        rem = np.empty(M, np.uint8)
        par = np.empty(M, np.int32)
        check(lib().cae_analysis_level_arrays(self._h, level, ptr(order), ptr(wave), ptr(cp), ptr(fp), ptr(rem),
                                              ptr(par)))
        return dict(order=order, wave=wave, close_pairs=cp, far_pairs=fp, removed=rem, parent=par)

    def perm(self):
        perm = np.empty(self.n, np.int32)
        nb = self.level_info(0)["M"]
        bp = np.empty(nb + 1, np.int32)
        check(lib().cae_analysis_perm(self._h, ptr(perm), ptr(bp)))
        return perm, bp

    def close(self):
        if getattr(self, "_h", None):
            lib().cae_analysis_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _as_cols(t):
    """(N,) or (nrhs, N) tensor -> (tensor (nrhs, N) contiguous, nrhs, squeeze)."""
    if t.dim() == 1:
        return t.reshape(1, -1).contiguous(), 1, True
    return t.contiguous(), t.shape[0], False


class Factor:
    """CE factorization on the GPU (``cae_factor_numeric``)."""

    def __init__(self, analysis: Analysis, vals, eps, precision=FP64, rank_mode=RANK_EPS, fixed_rank=0,
                 max_levels=0, coarse_max_dim=2048, stream=None, timing=False, mlp_params=None, seed=0,
                 record=None, compensate=False, graphs=True, apply_split_steps=None, workspace=None,
                 big_pivot_cap=0):
        """``rank_mode=RANK_LEARNED`` needs ``mlp_params`` (float32 CUDA tensor of
        ``learned.param_count()`` entries); ``record`` (float32 CUDA tensor of
        shape ``(rows, RECORD_WIDTH)``) receives the training records;
        ``graphs=False`` makes the iterative solvers launch the apply kernels
        one by one instead of replaying a captured HIP graph;
        ``apply_split_steps`` overrides the wave size below which the apply
        updates close blocks one workgroup per (step, block) (0 = never);
        ``workspace`` (a 256-byte aligned CUDA tensor of at least
        :func:`workspace_bytes` bytes, kept alive by the factor) holds every
        device buffer of the numeric factorization; ``big_pivot_cap`` (1..128,
        0 = 128) bounds the pivoted Cholesky of blocks above 128 unknowns."""
        import torch
        if not (isinstance(vals, torch.Tensor) and vals.is_cuda and vals.dtype == torch.float64):
            raise TypeError("vals must be a float64 CUDA tensor")
        for t in (mlp_params, record):
            if t is not None and not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
                                      and t.is_contiguous()):
                raise TypeError("mlp_params / record must be contiguous float32 CUDA tensors")
        self.analysis = analysis
        self.n = analysis.n
        self._stream = stream
        self._keep = (mlp_params, record, workspace)
        sptr = None if stream is None else stream.cuda_stream
        self._opts = _options(order=analysis.order, precision=precision, rank_mode=rank_mode,
                              fixed_rank=fixed_rank, max_levels=max_levels, coarse_max_dim=coarse_max_dim,
                              stream=sptr, timing=timing, mlp_params=mlp_params, seed=seed, record=record,
                              compensate=compensate, graphs=graphs, apply_split_steps=apply_split_steps,
                              workspace=workspace, big_pivot_cap=big_pivot_cap)
        h = C.c_void_p()
        self._vals = vals.contiguous()
        check(lib().cae_factor_numeric(analysis.handle, self._vals.data_ptr(), float(eps), C.byref(self._opts),
                                       C.byref(h)))
        self._h = h

    def stats(self):
        s = _lib.Stats()
        check(lib().cae_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _lib.Stats._fields_}

    def level_ms(self):
        """Host wall time of every factored level and of the dense remainder
        (``cae_get_level_ms``, K + 1 values)."""
        K = self.stats()["nlevels"]
        out = []
        for l in range(K + 1):
            v = C.c_double()
            check(lib().cae_get_level_ms(self._h, l, C.byref(v)))
            out.append(v.value)
        return out

    def ranks(self, level):
        M = self.analysis.level_info(level)["M"]
        out = np.empty(M, np.int32)
        check(lib().cae_get_ranks(self._h, level, ptr(out)))
        return out

    def sizes(self, level):
        M = self.analysis.level_info(level)["M"]
        out = np.empty(M, np.int32)
        check(lib().cae_get_sizes(self._h, level, ptr(out)))
        return out

    def drops(self, level):
        """``||E_i||_F^2`` of every step of a factored level (``cae_get_drops``)."""
        M = self.analysis.level_info(level)["M"]
        out = np.empty(M, np.float64)
        check(lib().cae_get_drops(self._h, level, ptr(out)))
        return out

    def apply(self, r):
        """``M^{-1} r``."""
        import torch
        rr, k, sq = _as_cols(r)
        z = torch.empty_like(rr)
        check(lib().cae_apply_precond(self._h, k, rr.data_ptr(), self.n, z.data_ptr(), self.n))
        return z.reshape(-1) if sq else z

    def multiply(self, x):
        """``M x`` with the stored factor."""
        import torch
        xx, k, sq = _as_cols(x)
        y = torch.empty_like(xx)
        check(lib().cae_apply_factor(self._h, k, xx.data_ptr(), self.n, y.data_ptr(), self.n))
        return y.reshape(-1) if sq else y

    def pcg(self, b, rtol=1e-8, maxit=1000, x=None):
        """FP64 PCG; returns ``(x, iters, relres)``; raises on non-convergence
        unless ``maxit`` is reached on purpose (``CAE_ENOCONV`` is returned as
        ``converged = False`` in the third element's companion)."""
        import torch
        bb, k, sq = _as_cols(b)
        if x is None:
            x = torch.empty_like(bb)
        it = np.zeros(k, np.int32)
        rel = np.zeros(k, np.float64)
        rc = check(lib().cae_pcg_solve(self._h, k, bb.data_ptr(), self.n, x.data_ptr(), self.n, float(rtol),
                                       int(maxit), ptr(it), ptr(rel)), allow=(_lib.CAE_ENOCONV,))
        self.converged = rc == _lib.CAE_OK
        return (x.reshape(-1) if sq else x), it, rel

    def pcg_batched(self, b, rtol=1e-8, maxit=1000, x=None):
        """Independent FP64 PCG on every problem of a batched factor
        (``cae_pcg_solve_batched``); returns ``(x, iters, relres)`` with
        ``iters`` and ``relres`` of shape ``(nprob, nrhs)``."""
        import torch
        bb, k, sq = _as_cols(b)
        if x is None:
            x = torch.empty_like(bb)
        nprob = len(self._rows()) - 1
        it = np.zeros((nprob, k), np.int32)
        rel = np.zeros((nprob, k), np.float64)
        rc = check(lib().cae_pcg_solve_batched(self._h, k, bb.data_ptr(), self.n, x.data_ptr(), self.n, float(rtol),
                                               int(maxit), ptr(it), ptr(rel)), allow=(_lib.CAE_ENOCONV,))
        self.converged = rc == _lib.CAE_OK
        return (x.reshape(-1) if sq else x), it, rel

    def _rows(self):
        return self.row_off if getattr(self, "row_off", None) is not None else self.analysis.batch_rows()

    def minres(self, b, rtol=1e-10, maxit=1000, x=None):
        """FP64 preconditioned MINRES (``cae_minres_solve``); returns ``(x, iters,
        relres)`` with the true relative residual at exit."""
        import torch
        bb, k, sq = _as_cols(b)
        if x is None:
            x = torch.empty_like(bb)
        it = np.zeros(k, np.int32)
        rel = np.zeros(k, np.float64)
        rc = check(lib().cae_minres_solve(self._h, k, bb.data_ptr(), self.n, x.data_ptr(), self.n, float(rtol),
                                          int(maxit), ptr(it), ptr(rel)), allow=(_lib.CAE_ENOCONV,))
        self.converged = rc == _lib.CAE_OK
        return (x.reshape(-1) if sq else x), it, rel

    def export(self, path):
        """Write the factor to ``path`` (``cae_export_factor``); read it back
        with :func:`read_export`."""
        check(lib().cae_export_factor(self._h, str(path).encode()))

    def solve(self, b):
        """Direct approximate solve ``x = M^{-1} b`` (CE(eps) used as a direct
        solver, no Krylov iterations)."""
        return self.apply(b)

    def close(self):
        if getattr(self, "_h", None):
            lib().cae_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(analysis: Analysis, vals, eps, **opts):
    """Device bytes a :class:`Factor` of these values and options takes from a
    ``workspace`` (``cae_workspace_query``: the factorization is run once with
    the library's own memory and counted)."""
    o = _options(order=analysis.order, **opts)
    nb = C.c_size_t()
    check(lib().cae_workspace_query(analysis.handle, vals.data_ptr(), float(eps), C.byref(o), C.byref(nb)))
    return nb.value


class OneCallFactor(Factor):
    """``cae_factor``: analysis and numeric factorization in one call from a
    host CSR matrix (the handle owns its analysis)."""

    def __init__(self, indptr, indices, data, perm, block_ptr, coords, eps, order=ORDER_MULTICOLOUR,
                 precision=FP64, coarse_max_dim=2048, workspace=None):
        ip, ix = _i64(indptr), _i32(indices)
        dv = np.ascontiguousarray(data, dtype=np.float64)
        pm, bp, co = _i32(perm), _i32(block_ptr), _i32(coords)
        ndim = co.shape[1] if co.ndim == 2 else 1
        self.analysis = None
        self.n = len(ip) - 1
        self._stream = None
        self._keep = (workspace,)
        self._opts = _options(order=order, precision=precision, coarse_max_dim=coarse_max_dim, workspace=workspace)
        h = C.c_void_p()
        check(lib().cae_factor(self.n, ptr(ip), ptr(ix), ptr(dv), ptr(pm), ptr(bp), len(bp) - 1, 0, ptr(co), ndim,
                               float(eps), C.byref(self._opts), C.byref(h)))
        self._h = h


def read_export(path):
    """Parse a file written by ``cae_export_factor`` into NumPy arrays (the
    layout is documented with ``cae_export_factor`` in ``include/cae.h``)."""
    buf = open(path, "rb").read()
    pos = 0

    def take(dtype, count):
        nonlocal pos
        a = np.frombuffer(buf, dtype=dtype, count=count, offset=pos)
        pos += a.nbytes
        return a.copy()

    if buf[:8] != b"CAEFACT1":
        raise ValueError("not a CAE factor export")
    pos = 8
    esize, K = take(np.int32, 2)
    n, coarse_dim = take(np.int64, 2)
    tau = float(take(np.float64, 1)[0])
    T = np.float64 if esize == 8 else np.float32
    out = {"esize": int(esize), "K": int(K), "n": int(n), "coarse_dim": int(coarse_dim), "tau": tau,
           "perm": take(np.int32, n), "levels": []}
    for _ in range(K):
        M, ns = take(np.int32, 2)
        lv = {"sizes": take(np.int32, M), "ranks": take(np.int32, M), "slot_p": take(np.int32, ns),
              "slot_q": take(np.int32, ns), "slot_off": take(np.int64, ns + 1)}
        lv["arena"] = take(T, int(lv["slot_off"][-1]))
        lv["u_off"] = take(np.int64, M + 1)
        lv["U"] = take(T, int(lv["u_off"][-1]))
        lv["Li"] = take(T, int(lv["u_off"][-1]))
        lv["parent"] = take(np.int32, M)
        lv["off_in_parent"] = take(np.int32, M)
        lv["order"] = take(np.int32, M)
        out["levels"].append(lv)
    d = int(coarse_dim)
    out["A_K"] = take(np.float64, d * d).reshape(d, d)
    out["neg_inv_A_K"] = take(np.float64, d * d).reshape(d, d)
    if pos != len(buf):
        raise ValueError("trailing bytes in the export")
    return out
