"""Oracle, learned-rank compression: counter-based Gaussian sketch, far-row
features, a small MLP that predicts the rank, and the randomized range finder
with its a-posteriori check and exact fallback.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  Shares no code
with the GPU path.

The paper names a cheaper rank-revealing factorization as the way to speed up
the compression (conclusion); this is that variant:

1. 16 features of the far row ``F_i`` (``b x w``) and of its step, all
   invariant under rotations inside a far block's columns;
2. an MLP 16 -> 64 -> 64 -> 1 (ReLU), evaluated in FP64 on FP32 parameters,
   predicts ``z ~ r_i / b_i``; ``k = clamp(ceil(b z), 0, b)``;
3. sketch ``Y = F Omega`` with ``l = min(k + p, b, w)`` Gaussian columns drawn
   by Philox4x32-10 keyed by ``(seed, level, block)``; ``Q = orth(Y)``;
4. ``B = Q^T F``, its SVD ``B = Ub S Vb^T``; ``r = #{s > theta}``; kept basis
   ``Q Ub[:, :r]``;
5. accept when ``||F - Q Q^T F||_F^2 + s_{r+1}^2 <= theta^2`` (this bounds
   the spectral norm of the dropped part ``E_i`` by ``theta``, the CE(eps)
   condition of eq. (rreav) in its spectral reading); otherwise the exact
   SVD path is taken.
"""
from __future__ import annotations

import numpy as np

NFEAT = 16
H = 64
OVERSAMPLE = 8

# parameter layout (float32): mean[16], std[16], W1[64x16], b1[64], W2[64x64], b2[64], w3[64], b3[1]
OFF_MEAN = 0
OFF_STD = OFF_MEAN + NFEAT
OFF_W1 = OFF_STD + NFEAT
OFF_B1 = OFF_W1 + H * NFEAT
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
NPARAM = OFF_B3 + 1

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): four
    32-bit counter words, two key words; returns four 32-bit words."""
    c0, c1, c2, c3 = (int(v) & _MASK for v in ctr)
    k0, k1 = (int(v) & _MASK for v in key)
    for rnd in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK
        hi1, lo1 = p1 >> 32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK, lo1, (hi0 ^ c3 ^ k1) & _MASK, lo0
        if rnd < 9:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def sketch_normals(seed, level, block, w, l):
    """Omega (w x l): entry (m, j) comes from the Philox output for counter
    (m, j >> 1, block, level) and key (seed low, seed high): two 53-bit
    uniforms from words (0, 1) and (2, 3), Box-Muller, cosine for even j and
    sine for odd j."""
    key = (seed & _MASK, (seed >> 32) & _MASK)
    Om = np.zeros((w, l))
    for m in range(w):
        for jp in range((l + 1) // 2):
            x0, x1, x2, x3 = philox4x32_10((m, jp, block, level), key)
            ua = ((x0 >> 5) * 67108864.0 + (x1 >> 6) + 0.5) / 9007199254740992.0
            ub = ((x2 >> 5) * 67108864.0 + (x3 >> 6) + 0.5) / 9007199254740992.0
            rad = np.sqrt(-2.0 * np.log(ua))
            Om[m, 2 * jp] = rad * np.cos(2.0 * np.pi * ub)
            if 2 * jp + 1 < l:
                Om[m, 2 * jp + 1] = rad * np.sin(2.0 * np.pi * ub)
    return Om


def _clog10(v, theta):
    return float(np.clip(np.log10(max(v, 1e-300) / theta), -30.0, 30.0))


def features(F, theta, level, nclose, nfar, nfar_proc, proc_rank_sum, proc_size_sum, widths=None):
    """The 16 features of a far row F (b x w, live columns only, far blocks of
    the given ``widths`` side by side) and its step.  Every feature is
    invariant under orthogonal changes of basis inside a far block's columns
    and inside the rows (kept bases are defined only up to such rotations,
    and at coarser levels the rows themselves are children's kept bases):
    Frobenius norms of the row and of its far blocks, widths and counts."""
    b, w = F.shape
    widths = [w] if widths is None else list(widths)
    rn = np.sqrt(np.sum(F * F, axis=1)) if w > 0 else np.zeros(b)
    edges = np.concatenate([[0], np.cumsum(widths)]).astype(int)
    bn = np.array([np.sqrt(np.sum(F[:, edges[k]:edges[k + 1]] ** 2)) for k in range(len(widths))])
    fro2 = float(np.sum(rn * rn))
    bmax = float(bn.max()) if len(bn) else 0.0
    x = np.zeros(NFEAT)
    x[0] = np.log2(b + 1.0)
    x[1] = np.log2(w + 1.0)
    x[2] = level
    x[3] = nfar
    x[4] = nclose
    x[5] = _clog10(np.sqrt(fro2), theta)
    x[6] = _clog10(np.sqrt(fro2 / max(b, 1)), theta)
    x[7] = _clog10(bmax, theta)
    x[8] = _clog10(np.sqrt(fro2 / max(w, 1)), theta)
    x[9] = np.count_nonzero(bn > theta) / max(len(bn), 1)
    x[10] = float(np.sum(bn ** 4)) / (fro2 * fro2) if fro2 > 0 else 0.0
    x[11] = fro2 / (bmax * bmax * len(bn)) if bmax > 0 else 0.0
    x[12] = nfar_proc / max(nfar, 1)
    x[13] = proc_rank_sum / proc_size_sum if proc_size_sum > 0 else 0.0
    x[14] = b / 64.0
    x[15] = 1.0
    return x


def init_params(seed=0):
    """He-initialised parameters, identity feature normalisation."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM, dtype=np.float32)
    p[OFF_STD:OFF_STD + NFEAT] = 1.0
    p[OFF_W1:OFF_B1] = rng.standard_normal(H * NFEAT) * np.sqrt(2.0 / NFEAT)
    p[OFF_W2:OFF_B2] = rng.standard_normal(H * H) * np.sqrt(2.0 / H)
    p[OFF_W3:OFF_B3] = rng.standard_normal(H) * np.sqrt(1.0 / H)
    p[OFF_B3] = 0.5
    return p


def _unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return (p[OFF_MEAN:OFF_STD], p[OFF_STD:OFF_W1], p[OFF_W1:OFF_B1].reshape(H, NFEAT), p[OFF_B1:OFF_W2],
            p[OFF_W2:OFF_B2].reshape(H, H), p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3])


def mlp_forward(p, X):
    """z for each row of X (n x 16), FP64 arithmetic on the FP32 parameters."""
    mu, sd, W1, b1, W2, b2, w3, b3 = _unpack(p)
    Xn = (np.atleast_2d(X) - mu) / sd
    h1 = np.maximum(Xn @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ w3 + b3


def mlp_loss_grad(p, X, y):
    """Mean squared error 0.5 mean((z - y)^2) and its gradient with respect to
    the trainable parameters (the normalisation entries get zero), FP64."""
    mu, sd, W1, b1, W2, b2, w3, b3 = _unpack(p)
    X = np.atleast_2d(X)
    n = X.shape[0]
    Xn = (X - mu) / sd
    a1 = Xn @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    d = (z - y) / n
    loss = 0.5 * float(np.sum((z - y) ** 2)) / n
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = h2.T @ d
    g[OFF_B3] = d.sum()
    dh2 = np.outer(d, w3) * (a2 > 0)
    g[OFF_W2:OFF_B2] = (dh2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (a1 > 0)
    g[OFF_W1:OFF_B1] = (dh1.T @ Xn).ravel()
    g[OFF_B1:OFF_W2] = dh1.sum(axis=0)
    return loss, g


def sketch_label(sig, r, theta):
    """Training target of the predictor: the smallest sketch width k >= r with
    which an ideal sketch (the top k singular directions) passes the check,
    sum_{j >= k} sigma_j^2 + (sigma_r^2 if k > r) <= theta^2 (sigma sorted
    descending, 0-based)."""
    s2 = np.asarray(sig, dtype=np.float64) ** 2
    n = len(s2)
    sr2 = s2[r] if r < n else 0.0
    kf = n
    tail = 0.0
    for k in range(n, r - 1, -1):
        if k < n:
            tail += s2[k]
        if tail + (sr2 if k > r else 0.0) <= theta * theta:
            kf = k
    return max(kf, r)


def predicted_rank(z, b):
    return int(min(max(int(np.ceil(b * z)), 0), b))


def randomized_compress(F, theta, k, seed, level, block, p=OVERSAMPLE):
    """Steps 3-5 of the module docstring.  Returns ``(accepted, U_kept (b x r),
    r, s (singular values of B), e = ||F||_F^2 - sum_{k<r} s_k^2)``."""
    b, w = F.shape
    l = min(k + p, b, w)
    if l <= 0:
        return False, None, 0, np.zeros(0), 0.0
    Om = sketch_normals(seed, level, block, w, l)
    Y = F @ Om
    Q, _ = np.linalg.qr(Y)
    B = Q.T @ F
    Ub, s, _ = np.linalg.svd(B, full_matrices=True)
    r = int(np.count_nonzero(s > theta))
    fro2 = float(np.sum(F * F))
    out2 = max(fro2 - float(np.sum(B * B)), 0.0)
    nxt = float(s[r] ** 2) if r < len(s) else 0.0
    accepted = out2 + nxt <= theta * theta
    e = max(fro2 - float(np.sum(s[:r] ** 2)), 0.0)
    return accepted, Q @ Ub[:, :r], r, s, e


def complete_basis(Ur, b):
    """An orthonormal b x b matrix whose leading columns span Ur (b x r)."""
    r = Ur.shape[1]
    if r == 0:
        return np.eye(b)
    Qf, _ = np.linalg.qr(np.hstack([Ur, np.eye(b)]))
    Qf = Qf[:, :b]
    # the first r columns span Ur; rotate them to Ur exactly
    Qf[:, :r] = Ur
    rest = Qf[:, r:] - Ur @ (Ur.T @ Qf[:, r:])
    rest, _ = np.linalg.qr(rest)
    return np.hstack([Ur, rest])
