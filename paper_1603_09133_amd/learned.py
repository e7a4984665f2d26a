"""Learned ranks for the compression step: training records, the MLP and its
training, all through the C ABI (``cae_mlp_*``) on the GPU.

Typical use::

    rec = learned.record(analysis, vals, eps)          # exact factorization, records per step
    params = learned.train(rec, epochs=2000)           # Adam on 0.5 mean (z - r/b)^2
    f = Factor(analysis, vals, eps, rank_mode=RANK_LEARNED, mlp_params=params, seed=1)

Records are rows of 16 far-row features and the label r_i / b_i (negative:
no compression at that step).  Blocks larger than 64 always take the exact
compression and give no records.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import RECORD_WIDTH, check, lib


def param_count():
    return int(lib().cae_mlp_param_count())


def init_params(seed=0, device="cuda"):
    """He-initialised weights, identity feature normalisation, output bias
    0.5 (half the block kept)."""
    import torch
    n_in, h = 16, 64
    rng = np.random.default_rng(seed)
    p = np.zeros(param_count(), dtype=np.float32)
    p[16:32] = 1.0
    o = 32
    p[o:o + h * n_in] = rng.standard_normal(h * n_in) * np.sqrt(2.0 / n_in)
    o += h * n_in + h
    p[o:o + h * h] = rng.standard_normal(h * h) * np.sqrt(2.0 / h)
    o += h * h + h
    p[o:o + h] = rng.standard_normal(h) * np.sqrt(1.0 / h)
    p[o + h] = 0.5
    return torch.from_numpy(p).to(device)


def record(analysis, vals, eps, precision=0, rows=None, **factor_kw):
    """Run an exact CE(eps) factorization that writes one record per block
    and level; returns the used rows (float32 CUDA tensor, RECORD_WIDTH wide)."""
    import torch

    from . import Factor
    if rows is None:
        rows = sum(analysis.level_info(l)["M"] for l in range(analysis.nlevels()))
    rec = torch.full((max(rows, 1), RECORD_WIDTH), -1.0, dtype=torch.float32, device="cuda")
    f = Factor(analysis, vals, eps, precision=precision, record=rec, **factor_kw)
    used = f.stats()["record_rows"]
    f.close()
    return rec[:used].contiguous()


def train(records, epochs=2000, lr=1e-3, params=None, seed=0, stream=None):
    """Adam on the records from ``params`` (default :func:`init_params`);
    returns ``(params, final_loss)``."""
    import torch
    if params is None:
        params = init_params(seed)
    params = params.contiguous()
    recs = torch.cat(records) if isinstance(records, (list, tuple)) else records
    recs = recs.contiguous()
    loss = C.c_float()
    check(lib().cae_mlp_train(recs.data_ptr(), recs.shape[0], params.data_ptr(), int(epochs), float(lr),
                              C.byref(loss), None if stream is None else stream.cuda_stream))
    return params, float(loss.value)


def loss_grad(params, records):
    """FP32 loss and gradient at ``params`` (GPU)."""
    import torch
    g = torch.empty_like(params)
    loss = C.c_float()
    check(lib().cae_mlp_loss_grad(params.data_ptr(), records.data_ptr(), records.shape[0], g.data_ptr(),
                                  C.byref(loss), None))
    return float(loss.value), g


def predict(params, records):
    """z for every record (FP64 arithmetic on the device, returned as float32)."""
    import torch
    z = torch.empty(records.shape[0], dtype=torch.float32, device=records.device)
    check(lib().cae_mlp_predict(params.data_ptr(), records.data_ptr(), records.shape[0], z.data_ptr(), None))
    return z
