"""Oracle, numeric part: the compress-and-eliminate (CE) factorization in FP64.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU path; the GPU path never calls it.

The factorization follows the paper's Algorithm 1 (levels) and Algorithm 2
(one level) step by step, strictly sequentially, with NumPy/SciPy dense
routines (SVD, Cholesky, triangular solve, matrix product) as the steps:

for every block row ``i`` of the level, in the elimination order:

1. far row ``F_i``: the far blocks of row ``i`` side by side, each with its
   full block width (Section 2.2, the row split ``[D_i C_i F_i 0]``);
2. compression (eq. (rreav), Remark 2.1): ``F_i = U S V^T``;
   CE(eps) keeps the ``r_i`` singular values ``> theta = eps * max diag(A0)``
   (spectral norm of the dropped part ``E_i``), CE(r) keeps ``min(r, b_i)``;
   an empty far row keeps nothing (``r_i = 0``, ``U_i = I``: the first-row
   elimination of Section 2.1);
3. rotation (eq. (q)): row and column ``i`` become ``U_i^T (.)`` and
   ``(.) U_i``; the stored factor rows of block ``i`` are rotated the same way
   (eq. (big_L)); the trailing ``b_i - r_i`` rows of the rotated far blocks
   (``E_i``) are set to zero, with their symmetric columns;
4. elimination of the sub-row ``S_i`` (the trailing ``b_i - r_i`` rotated
   rows): Cholesky of its diagonal block, ``L_i = S_i^T L^{-T}`` (eq. (sm_L)),
   Schur complement into the close neighbours, which creates the far blocks.

After a level the remaining (basis) unknowns of ``2^d`` Morton siblings form
one super-block of the next level (Section 2.5, eq. (bsp)); when one block is
left or the remaining dimension is small the remainder is factored by a
dense Cholesky (Section 2.6, Algorithm 1, Proposition 2.1).  The solve is
``x = Q^T L^{-T} L^{-1} Q b`` (Proposition 2.2).

Readings where the paper is silent (the same ones the GPU path implements):
the norm of ``E_i`` is the spectral norm and the threshold is absolute,
scaled by ``max diag(A0)``; the basis is the leading ``r_i`` singular
directions; close blocks of a level are the structural pattern of its
matrix; a level stops when one block remains or its dimension is at most
``coarse_max_dim``.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import time

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import learned as lrn
from . import symbolic as sym

__all__ = ["NotSPD", "CEOptions", "LevelFactor", "CEFactor", "ce_factor",
           "ce_solve", "ce_multiply", "ce_dense", "pcg"]


class NotSPD(RuntimeError):
    """A pivot block of an elimination step is not positive definite."""

    def __init__(self, level, block, msg=""):
        super().__init__(f"non-SPD pivot at level {level}, block {block} {msg}")
        self.level = level
        self.block = block


@dataclass
class CEOptions:
    eps: float = 1e-8
    rank_mode: str = "eps"          # 'eps' = CE(eps), 'fixed' = CE(r), 'learned' = CE(eps) by sketch
    fixed_rank: int = 0
    mlp_params: object = None       # learned: FP32 parameter vector of the rank MLP
    seed: int = 0                   # learned: Philox key of the sketches
    record_features: bool = False   # compute the learned-mode features in any mode (tests only)
    compensate: bool = False        # add |E_i| to the diagonals (keeps M - A0 positive semidefinite)
    coarsen: str = "siblings"       # 'siblings' (2^d Morton siblings) | 'pairs' (along the Morton curve)
    order: str = "paper"            # 'paper' | 'multicolour'
    coarse_max_dim: int = 2048
    max_levels: int = 0             # 0 = no limit
    keep_far_rows: bool = False     # record F_i of every step (tests only)
    dense_remainder: bool = True    # False: stop after the levels (bounded timing samples only)
    max_steps: int = 0              # > 0: only the first max_steps steps of level 1 and nothing
                                    # after them (bounded timing samples only)


@dataclass
class LevelFactor:
    M: int
    sizes: np.ndarray               # b_i
    order: list
    close_pairs: list               # structural pattern at level start
    far_pairs: list = field(default_factory=list)   # created during the level
    removed: set = field(default_factory=set)       # eliminated whole (empty far row)
    U: list = field(default_factory=list)
    r: np.ndarray = None
    e: np.ndarray = None            # squared Frobenius norm of dropped E_i
    sigma: list = field(default_factory=list)       # singular values of F_i
    F: list = field(default_factory=list)           # far rows, when kept
    Lnn: list = field(default_factory=list)
    panel: list = field(default_factory=list)       # dict x -> rows_x x n_i
    parent: np.ndarray = None
    min_pivot: float = np.inf
    seconds: float = 0.0            # wall time of the level (timing of bounded samples)
    features: list = field(default_factory=list)    # learned: features of every compressed step
    exact_rank: list = field(default_factory=list)  # learned: the exact-SVD rank of that step
    label: list = field(default_factory=list)       # learned: sketch width an ideal sketch needs
    accepted: int = 0               # learned: sketches accepted
    fallbacks: int = 0              # learned: steps that took the exact SVD


@dataclass
class CEFactor:
    N: int
    perm: np.ndarray
    block_ptr: np.ndarray
    theta: float
    levels: list
    coarse_L: np.ndarray
    coarse_sizes: np.ndarray        # block sizes of the remainder, in order

    def ranks(self):
        return [lf.r.copy() for lf in self.levels]

    def dropped(self):
        """Sum over all steps of ||E_i||_F^2."""
        return float(sum(lf.e.sum() for lf in self.levels))


class _Blocks:
    """Symmetric block storage: canonical key (p, q) with p <= q."""

    def __init__(self):
        self.d = {}

    def has(self, p, q):
        return (min(p, q), max(p, q)) in self.d

    def get(self, p, q):
        """View of block (p, q) as rows of p, columns of q (writes go through)."""
        if p <= q:
            return self.d[(p, q)]
        return self.d[(q, p)].T

    def put(self, p, q, X):
        if p <= q:
            self.d[(p, q)] = X
        else:
            self.d[(q, p)] = np.ascontiguousarray(X.T)


def _level1_blocks(A0: sp.csr_matrix, block_ptr):
    """Dense copies of the nonzero blocks of A0 (blocks (p, q), p <= q): the
    entries are grouped by block, then each group is added into its block."""
    coo = A0.tocoo()
    M = len(block_ptr) - 1
    owner = np.repeat(np.arange(M), np.diff(block_ptr))
    bi, bj = owner[coo.row], owner[coo.col]
    keep = bi <= bj
    bi, bj, rows, cols, vals = bi[keep], bj[keep], coo.row[keep], coo.col[keep], coo.data[keep]
    li, lj = rows - block_ptr[bi], cols - block_ptr[bj]
    W = _Blocks()
    sizes = np.diff(block_ptr)
    key = bi.astype(np.int64) * M + bj
    order = np.argsort(key, kind="stable")
    key, li, lj, vals = key[order], li[order], lj[order], vals[order]
    starts = np.flatnonzero(np.r_[True, key[1:] != key[:-1]])
    ends = np.r_[starts[1:], len(key)]
    for s0, s1 in zip(starts, ends):
        p, q = int(key[s0] // M), int(key[s0] % M)
        X = np.zeros((sizes[p], sizes[q]))
        np.add.at(X, (li[s0:s1], lj[s0:s1]), vals[s0:s1])
        W.put(p, q, X)
    for p in range(M):
        if not W.has(p, p):
            W.put(p, p, np.zeros((sizes[p], sizes[p])))
    return W


def _rank(sig_full, theta, opts: CEOptions, has_far: bool, b: int):
    if not has_far:
        return 0
    if opts.rank_mode in ("eps", "learned"):
        return int(np.count_nonzero(sig_full > theta))
    if opts.rank_mode == "fixed":
        return int(min(opts.fixed_rank, b))
    raise ValueError(opts.rank_mode)


def _factor_level(level_no, sizes, W: _Blocks, close_pairs, order, theta, opts):
    """Algorithm 2 on one level; updates W in place."""
    M = len(sizes)
    close = sym.adjacency(M, close_pairs)
    far = [set() for _ in range(M)]
    lf = LevelFactor(M=M, sizes=np.asarray(sizes), order=list(order), close_pairs=list(close_pairs))
    lf.U = [None] * M
    lf.r = np.zeros(M, dtype=np.int64)
    lf.e = np.zeros(M)
    lf.sigma = [None] * M
    lf.F = [None] * M
    lf.Lnn = [None] * M
    lf.panel = [None] * M
    lrows = [[] for _ in range(M)]      # steps whose stored panel has rows of block c
    removed = set()
    pos = {blk: k for k, blk in enumerate(order)}
    lf.features = [None] * M
    lf.exact_rank = [None] * M
    lf.label = [None] * M
    for step_no, i in enumerate(order):
        if opts.max_steps and step_no >= opts.max_steps:
            break
        b = int(sizes[i])
        fl = sorted(far[i])
        # 1. far row F_i (full block widths; eliminated columns are zero)
        F = np.hstack([W.get(i, l) for l in fl]) if fl else np.zeros((b, 0))
        # 2. compression
        if F.shape[1] > 0 and b > 0:
            Uf, s, _ = np.linalg.svd(F, full_matrices=True)
            sig = np.zeros(b)
            sig[:len(s)] = s
        else:
            Uf, sig = np.eye(b), np.zeros(b)
        r = _rank(sig, theta, opts, len(fl) > 0 and F.shape[1] > 0, b)
        U = Uf if (len(fl) > 0 and F.shape[1] > 0) else np.eye(b)
        e_i = float(np.sum(sig[r:] ** 2))
        if (opts.rank_mode == "learned" or opts.record_features) and fl and b > 0:
            # live columns only: a processed far neighbour keeps its r_l basis columns
            proc = [l for l in fl if pos[l] < pos[i]]
            wl = [int(lf.r[l]) if pos[l] < pos[i] else int(sizes[l]) for l in fl]
            F_live = np.hstack([W.get(i, l)[:, :wd] for l, wd in zip(fl, wl)])
            x = lrn.features(F_live, theta, level_no - 1, len(close[i]), len(fl), len(proc),
                             float(sum(lf.r[l] for l in proc)), float(sum(int(sizes[l]) for l in proc)), wl)
            lf.features[i] = x
            lf.exact_rank[i] = r
            lf.label[i] = lrn.sketch_label(sig, r, theta)
        if opts.rank_mode == "learned" and fl and b > 0:
            if F_live.shape[1] > 0:
                k = lrn.predicted_rank(float(lrn.mlp_forward(opts.mlp_params, x)[0]), b)
                ok, Ur, rr, sb, e = lrn.randomized_compress(F_live, theta, k, opts.seed, level_no - 1, i)
            else:
                ok, Ur, rr, sb, e = True, np.zeros((b, 0)), 0, np.zeros(0), 0.0
            if ok:
                U = lrn.complete_basis(Ur, b)
                r = rr
                sig = np.zeros(b)
                sig[:min(len(sb), b)] = sb[:b]
                e_i = e
                lf.accepted += 1
            else:
                lf.fallbacks += 1
        if not fl:
            removed.add(i)          # eliminated whole; leaves the graph
        lf.U[i], lf.r[i], lf.sigma[i] = U, r, sig
        if opts.keep_far_rows:
            lf.F[i] = F.copy()
        lf.e[i] = e_i
        # 3. rotation of row/column i, of the stored factor rows of i, drop E_i
        for x in sorted(close[i] | far[i]):
            blk = W.get(i, x)
            blk[...] = U.T @ blk
        D = W.get(i, i)
        D[...] = U.T @ D @ U
        for k in lrows[i]:
            lf.panel[k][i] = U.T @ lf.panel[k][i]
        for l in fl:
            blk = W.get(i, l)
            if opts.compensate and b - r > 0:
                # diagonal compensation of the dropped block E_il (robustness
                # option, not in the paper): its Frobenius norm e is added to
                # the diagonal of i's eliminated rows and of l's live columns,
                # so M - A0 gains [[e I, -E], [-E^T, e I]], positive
                # semidefinite because ||E||_2 <= e; e and the identities do
                # not depend on the bases chosen inside the subspaces
                wl = int(lf.r[l]) if pos[l] < pos[i] else int(sizes[l])
                eF = float(np.linalg.norm(blk[r:, :wl]))
                Dl = W.get(l, l)
                D[np.arange(r, b), np.arange(r, b)] += eF
                Dl[np.arange(wl), np.arange(wl)] += eF
            blk[r:, :] = 0.0
        # 4. elimination of the trailing b - r rotated rows
        n = slice(r, b)
        kb = slice(0, r)
        group = [i] + sorted(close[i])
        if b - r > 0:
            S = D[n, n]
            try:
                Lnn = np.linalg.cholesky(S)
            except np.linalg.LinAlgError:
                raise NotSPD(level_no, i)
            lf.min_pivot = min(lf.min_pivot, float(np.min(np.diag(Lnn))))
            pan = {i: sla.solve_triangular(Lnn, D[n, kb], lower=True).T}
            for c in group[1:]:
                pan[c] = sla.solve_triangular(Lnn, W.get(i, c)[n, :], lower=True).T
        else:
            Lnn = np.zeros((0, 0))
            pan = {i: np.zeros((r, 0))}
            for c in group[1:]:
                pan[c] = np.zeros((int(sizes[c]), 0))
        # Schur complement (and structural creation of far blocks)
        for ia, a in enumerate(group):
            for c in group[ia:]:
                if a != c and not W.has(a, c):
                    if a in removed or c in removed:
                        continue
                    W.put(a, c, np.zeros((int(sizes[a]), int(sizes[c]))))
                    far[a].add(c)
                    far[c].add(a)
                if b - r == 0:
                    continue
                upd = pan[a] @ pan[c].T
                tgt = W.get(a, c)
                ra = kb if a == i else slice(None)
                rc = kb if c == i else slice(None)
                tgt[ra, rc] -= upd
        # the eliminated sub-row and sub-column are now zero
        D[n, :] = 0.0
        D[:, n] = 0.0
        for c in group[1:]:
            W.get(i, c)[n, :] = 0.0
        lf.Lnn[i] = Lnn
        lf.panel[i] = pan
        for c in group[1:]:
            lrows[c].append(i)
    lf.far_pairs = sorted((p, q) for p in range(M) for q in far[p] if p < q)
    lf.removed = removed
    return lf


def _next_level(sizes, r, W: _Blocks, parent, Mn, removed):
    """Remainder of a level on the basis unknowns, grouped by parent."""
    M = len(sizes)
    nsz = np.zeros(Mn, dtype=np.int64)
    off = np.zeros(M, dtype=np.int64)          # offset of child's basis inside parent
    for c in range(M):
        off[c] = nsz[parent[c]]
        nsz[parent[c]] += r[c]
    Wn = _Blocks()
    for P in range(Mn):
        Wn.put(P, P, np.zeros((nsz[P], nsz[P])))
    for (p, q), X in W.d.items():
        if p in removed or q in removed:
            continue
        P, Q = parent[p], parent[q]
        sub = X[:r[p], :r[q]]
        if not Wn.has(P, Q):
            Wn.put(P, Q, np.zeros((nsz[P], nsz[Q])))
        T = Wn.get(P, Q)
        T[off[p]:off[p] + r[p], off[q]:off[q] + r[q]] = sub
        if P == Q and p != q:
            T[off[q]:off[q] + r[q], off[p]:off[p] + r[p]] = sub.T
    return nsz, Wn


def ce_factor(indptr, indices, data, perm, block_ptr, coords, opts: CEOptions, J=None):
    """CE factorization ``A ~ Q^T L L^T Q`` of the CSR matrix (Algorithm 1).

    ``perm`` maps new to old indices (``A0 = A[perm][:, perm]``), ``block_ptr``
    gives the level-1 blocks of ``A0`` and ``coords`` their Morton
    coordinates (or ``None``: consecutive groups of ``J`` blocks are joined).
    """
    N = len(perm)
    A = sp.csr_matrix((data, indices, indptr), shape=(N, N))
    perm = np.asarray(perm)
    block_ptr = np.asarray(block_ptr)
    A0 = A[perm][:, perm].tocsr()
    tau = float(A0.diagonal().max())
    theta = opts.eps * tau
    sizes = np.diff(block_ptr)
    W = _level1_blocks(A0, block_ptr)
    close_pairs = sym.level1_pattern(indptr, indices, perm, block_ptr)
    if J is None and coords is not None:
        J = 2 ** np.asarray(coords).shape[1]
    levels = []
    level_no = 1
    while True:
        M = len(sizes)
        dim = int(np.sum(sizes))
        if M <= 1 or dim <= opts.coarse_max_dim or (opts.max_levels and level_no > opts.max_levels):
            break
        adj = sym.adjacency(M, close_pairs)
        order = sym.element_order(adj, opts.order, coords)
        t_level = time.perf_counter()
        lf = _factor_level(level_no, sizes, W, close_pairs, order, theta, opts)
        lf.seconds = time.perf_counter() - t_level
        if opts.max_steps:
            levels.append(lf)
            return CEFactor(N=N, perm=perm, block_ptr=block_ptr, theta=theta, levels=levels,
                            coarse_L=None, coarse_sizes=np.asarray(sizes))
        axis = None
        if opts.coarsen == "pairs" and coords is not None:
            axis = (level_no - 1) % np.asarray(coords).shape[1]
        parent, coords = sym.coarsen(coords, M, J, axis=axis)
        Mn = int(parent.max()) + 1
        lf.parent = parent
        levels.append(lf)
        all_pairs = sym.live_pairs(sorted(set(close_pairs) | set(lf.far_pairs)), lf.removed)
        close_pairs = sym.coarse_pattern(parent, all_pairs)
        sizes, W = _next_level(sizes, lf.r, W, parent, Mn, lf.removed)
        level_no += 1
    if not opts.dense_remainder:
        return CEFactor(N=N, perm=perm, block_ptr=block_ptr, theta=theta, levels=levels,
                        coarse_L=None, coarse_sizes=np.asarray(sizes))
    # dense Cholesky of the remainder
    offs = np.concatenate([[0], np.cumsum(sizes)])
    dim = int(offs[-1])
    AK = np.zeros((dim, dim))
    for (p, q), X in W.d.items():
        AK[offs[p]:offs[p + 1], offs[q]:offs[q + 1]] = X
        AK[offs[q]:offs[q + 1], offs[p]:offs[p + 1]] = X.T
    try:
        LK = np.linalg.cholesky(AK) if dim > 0 else np.zeros((0, 0))
    except np.linalg.LinAlgError:
        raise NotSPD(level_no, -1, "(coarse)")
    return CEFactor(N=N, perm=perm, block_ptr=block_ptr, theta=theta, levels=levels,
                    coarse_L=LK, coarse_sizes=np.asarray(sizes))


# ---------------------------------------------------------------- apply ----

def _split(vec, sizes):
    offs = np.concatenate([[0], np.cumsum(sizes)])
    return [vec[offs[k]:offs[k + 1]].copy() for k in range(len(sizes))]


def _children(parent, Mn):
    ch = [[] for _ in range(Mn)]
    for c, P in enumerate(parent):
        ch[P].append(c)
    return ch


def _to_next(lf, ys, Mn):
    ch = _children(lf.parent, Mn)
    return [np.concatenate([ys[c][:lf.r[c]] for c in ch[P]], axis=0) if ch[P]
            else np.zeros((0,) + ys[0].shape[1:]) for P in range(Mn)]


def _from_next(lf, zs, nxt, Mn):
    ch = _children(lf.parent, Mn)
    for P in range(Mn):
        o = 0
        for c in ch[P]:
            zs[c][:lf.r[c]] = nxt[P][o:o + lf.r[c]]
            o += lf.r[c]


def _next_sizes(f: CEFactor, lev):
    return f.levels[lev + 1].sizes if lev + 1 < len(f.levels) else f.coarse_sizes


def _solve_level(f: CEFactor, lev, ys):
    if lev == len(f.levels):
        v = np.concatenate(ys, axis=0)
        if v.shape[0]:
            v = sla.solve_triangular(f.coarse_L, v, lower=True)
            v = sla.solve_triangular(f.coarse_L.T, v, lower=False)
        return _split(v, f.coarse_sizes)
    lf = f.levels[lev]
    ys = [lf.U[i].T @ ys[i] for i in range(lf.M)]
    for i in lf.order:                              # forward, L^{-1}
        r, b = lf.r[i], lf.sizes[i]
        if b - r == 0:
            continue
        t = sla.solve_triangular(lf.Lnn[i], ys[i][r:], lower=True)
        ys[i][r:] = t
        for x, p in lf.panel[i].items():
            if x == i:
                ys[i][:r] -= p @ t
            else:
                ys[x] -= p @ t
    Mn = len(_next_sizes(f, lev))
    nxt = _solve_level(f, lev + 1, _to_next(lf, ys, Mn))
    zs = [y.copy() for y in ys]
    _from_next(lf, zs, nxt, Mn)
    for i in reversed(lf.order):                    # backward, L^{-T}
        r, b = lf.r[i], lf.sizes[i]
        if b - r == 0:
            continue
        t = ys[i][r:].copy()
        for x, p in lf.panel[i].items():
            t -= p.T @ (zs[i][:r] if x == i else zs[x])
        zs[i][r:] = sla.solve_triangular(lf.Lnn[i].T, t, lower=False)
    return [lf.U[i] @ zs[i] for i in range(lf.M)]


def _mul_level(f: CEFactor, lev, zs):
    if lev == len(f.levels):
        v = np.concatenate(zs, axis=0)
        if v.shape[0]:
            v = f.coarse_L @ (f.coarse_L.T @ v)
        return _split(v, f.coarse_sizes)
    lf = f.levels[lev]
    zs = [lf.U[i].T @ zs[i] for i in range(lf.M)]
    w = {}
    for i in lf.order:                              # w = Lcheck^T z
        r, b = lf.r[i], lf.sizes[i]
        if b - r == 0:
            continue
        wi = lf.Lnn[i].T @ zs[i][r:]
        for x, p in lf.panel[i].items():
            wi = wi + p.T @ (zs[i][:r] if x == i else zs[x])
        w[i] = wi
    Mn = len(_next_sizes(f, lev))
    nxt = _mul_level(f, lev + 1, _to_next(lf, zs, Mn))
    out = [np.zeros_like(z) for z in zs]
    _from_next(lf, out, nxt, Mn)
    for i, wi in w.items():                         # + Lcheck w
        r = lf.r[i]
        out[i][r:] += lf.Lnn[i] @ wi
        for x, p in lf.panel[i].items():
            if x == i:
                out[i][:r] += p @ wi
            else:
                out[x] += p @ wi
    return [lf.U[i] @ out[i] for i in range(lf.M)]


def _in_blocks(f: CEFactor, x):
    x0 = np.asarray(x, dtype=np.float64)[f.perm]
    sizes = f.levels[0].sizes if f.levels else f.coarse_sizes
    return _split(x0, sizes)


def _out_vec(f: CEFactor, blocks):
    v = np.concatenate(blocks, axis=0)
    out = np.empty_like(v)
    out[f.perm] = v
    return out


def ce_solve(f: CEFactor, b):
    """``M^{-1} b`` with ``M = Q^T L L^T Q`` (Proposition 2.2); ``b`` may be
    ``(N,)`` or ``(N, k)`` in the original ordering."""
    return _out_vec(f, _solve_level(f, 0, _in_blocks(f, b)))


def ce_multiply(f: CEFactor, x):
    """``M x`` with ``M = Q^T L L^T Q``."""
    return _out_vec(f, _mul_level(f, 0, _in_blocks(f, x)))


def ce_dense(f: CEFactor):
    """Dense ``M`` (small problems only)."""
    return ce_multiply(f, np.eye(f.N))


# ------------------------------------------------------------------ PCG ----

def pcg(A, b, apply_prec, tol=1e-8, maxit=1000):
    """Preconditioned conjugate gradients from ``x0 = 0`` for one column;
    stops when the recurrence residual satisfies ``||r|| <= tol ||b||``.
    Returns ``(x, iterations, ||b - A x|| / ||b||)``."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    z = apply_prec(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > tol * nb and it < maxit:
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if np.linalg.norm(r) <= tol * nb:
            break
        z = apply_prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, float(np.linalg.norm(b - A @ x) / nb)


def minres(A, b, apply_prec, tol=1e-10, maxit=1000):
    """Preconditioned MINRES from ``x0 = 0`` for one column (the Krylov method
    of the paper's Section 3; Paige-Saunders recurrences).  ``apply_prec`` is
    ``M^{-1}`` (symmetric positive definite).  The iterate ``x_k`` minimises
    ``||b - A x||_{M^{-1}}`` over the preconditioned Krylov space of
    dimension ``k``.  Stops when that norm (``phibar``) is at most
    ``tol * ||b||_{M^{-1}}``.  Returns ``(x, iterations, ||b - A x|| / ||b||)``.

    Steps per iteration: Lanczos ``v_k = y / beta_k``, ``y = A v_k -
    (beta_k / beta_{k-1}) r_{k-1}``, ``alpha_k = v_k^T y``, ``y -= (alpha_k /
    beta_k) r_k``, ``beta_{k+1} = sqrt(y^T M^{-1} y)``; the previous Givens
    rotation (cs, sn) acts on the new column of the tridiagonal matrix, a new
    rotation annihilates ``beta_{k+1}``; the search direction is the
    three-term combination ``w_k = (v_k - eps_k w_{k-2} - delta_k w_{k-1}) /
    gamma_k`` and ``x += phi_k w_k``."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    r1 = b.copy()
    y = apply_prec(r1)
    beta1 = float(np.sqrt(max(r1 @ y, 0.0)))
    if beta1 == 0.0:
        return x, 0, 0.0
    r2 = r1.copy()
    beta, oldb = beta1, 0.0
    dbar = epsln = 0.0
    phibar = beta1
    cs, sn = -1.0, 0.0
    w = np.zeros_like(b)
    w2 = np.zeros_like(b)
    it = 0
    while it < maxit:
        v = y / beta
        y = A @ v
        if it > 0:
            y = y - (beta / oldb) * r1
        alpha = float(v @ y)
        y = y - (alpha / beta) * r2
        r1, r2 = r2, y
        y = apply_prec(r2)
        oldb, beta = beta, float(np.sqrt(max(r2 @ y, 0.0)))
        oldeps = epsln
        delta = cs * dbar + sn * alpha
        gbar = sn * dbar - cs * alpha
        epsln = sn * beta
        dbar = -cs * beta
        gamma = max(np.hypot(gbar, beta), 1e-300)
        cs, sn = gbar / gamma, beta / gamma
        phi = cs * phibar
        phibar = sn * phibar
        w1, w2 = w2, w
        w = (v - oldeps * w1 - delta * w2) / gamma
        x = x + phi * w
        it += 1
        if phibar <= tol * beta1 or not beta > 0.0:
            break
    return x, it, float(np.linalg.norm(b - A @ x) / nb) if nb > 0 else 0.0
