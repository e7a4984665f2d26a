"""Oracle, integer part: initial permutation, block patterns, elimination
order and the structural simulation of one level.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU path.

Everything here is plain Python over integers, written for readability.

* Initial permutation ``A0 = P A P^T`` (Section 2, eq. (init_perm)): the grid
  is cut into patches of ``patch`` points; patches are visited in Z (Morton)
  order of their patch coordinates, points inside a patch lexicographically
  with x fastest.  One patch is one block of ``A0``.
* Close blocks are the nonzero blocks of the current level matrix
  (Section 2, definition of close/far before Section 2.1).
* Coarsening joins the ``J = 2^d`` Morton siblings of a level into one
  super-block (Section 2.5, eq. (bsp), and
  Section 2.8, Proposition 2.4 on tensor grids: at least two nodes per direction).
* Far blocks are created by the Schur complement of an elimination step
  between two close neighbours of the eliminated block that are not close to
  each other (eq. (A_st) and the remark after eq. (sm_L): the far pattern is
  contained in the pattern of A^2 minus that of A).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = [
    "morton_key", "grid_order", "level1_pattern", "coarsen", "coarse_pattern",
    "colour_order", "element_order", "simulate_level", "distance2_sets", "live_pairs",
]


def morton_key(coord) -> int:
    """Z-order key: bit b of axis k goes to bit ``b*ndim + k`` (x = axis 0)."""
    ndim = len(coord)
    key = 0
    for bit in range(21):
        for k in range(ndim):
            key |= ((int(coord[k]) >> bit) & 1) << (bit * ndim + k)
    return key


def grid_order(dims, patch):
    """Permutation for a tensor grid ``dims`` (natural order, x fastest).

    Returns ``perm`` (new -> old), ``block_ptr`` (len M+1) and ``coords``
    (M x ndim patch coordinates), with patches in Morton order.  Partial
    patches at the high end of an axis keep their smaller size.
    """
    dims = [int(d) for d in dims]
    patch = [int(p) for p in patch]
    ndim = len(dims)
    npatch = [math.ceil(dims[k] / patch[k]) for k in range(ndim)]
    coords = list(itertools.product(*[range(n) for n in npatch]))
    coords.sort(key=morton_key)
    strides = [1]
    for k in range(1, ndim):
        strides.append(strides[-1] * dims[k - 1])
    perm = []
    block_ptr = [0]
    for c in coords:
        rng = [range(c[k] * patch[k], min((c[k] + 1) * patch[k], dims[k])) for k in range(ndim)]
        # lexicographic inside the patch, x fastest: iterate slowest axis outermost
        for pt in itertools.product(*reversed(rng)):
            pt = pt[::-1]
            perm.append(sum(pt[k] * strides[k] for k in range(ndim)))
        block_ptr.append(len(perm))
    return (np.array(perm, dtype=np.int64), np.array(block_ptr, dtype=np.int64),
            np.array(coords, dtype=np.int64).reshape(len(coords), ndim))


def level1_pattern(indptr, indices, perm, block_ptr):
    """Close pairs (p, q), p < q, of ``A0 = P A P^T``: a block is close when
    it holds a structural nonzero of A."""
    N = len(perm)
    pos = np.empty(N, dtype=np.int64)
    pos[np.asarray(perm)] = np.arange(N)
    owner = np.repeat(np.arange(len(block_ptr) - 1, dtype=np.int64), np.diff(np.asarray(block_ptr)))
    rows = np.repeat(np.arange(N, dtype=np.int64), np.diff(np.asarray(indptr)))
    bi, bj = owner[pos[rows]], owner[pos[np.asarray(indices, dtype=np.int64)]]
    off = bi != bj
    lo, hi = np.minimum(bi[off], bj[off]), np.maximum(bi[off], bj[off])
    pairs = np.unique(np.stack([lo, hi], axis=1), axis=0)
    return [(int(p), int(q)) for p, q in pairs]


def adjacency(M, pairs):
    adj = [set() for _ in range(M)]
    for p, q in pairs:
        adj[p].add(q)
        adj[q].add(p)
    return adj


def coarsen(coords, M=None, J=None, axis=None):
    """Parent of every block: Morton siblings (coordinate >> 1) when
    coordinates are known, else consecutive groups of J blocks.  With
    ``axis`` only that coordinate is halved: pairs of blocks along the Morton
    curve (the lowest remaining bit of the Morton key).  Returns ``parent``
    (len M) and the parents' coordinates (or None)."""
    if coords is None:
        parent = np.arange(M) // J
        return parent, None
    coords = np.asarray(coords)
    if axis is None:
        pc = coords >> 1
    else:
        pc = coords.copy()
        pc[:, axis] >>= 1
    parent = np.empty(len(coords), dtype=np.int64)
    seen = {}
    out = []
    for i, c in enumerate(map(tuple, pc)):
        if c not in seen:
            seen[c] = len(out)
            out.append(c)
        parent[i] = seen[c]
    # children of one parent are consecutive in Morton order
    assert all(parent[i] <= parent[i + 1] for i in range(len(parent) - 1))
    return parent, np.array(out, dtype=np.int64).reshape(len(out), coords.shape[1])


def coarse_pattern(parent, pairs):
    """Pattern of the next level: super-blocks P != Q are close when any pair
    of their children holds a block (close or far) at the current level."""
    out = set()
    for p, q in pairs:
        P, Q = parent[p], parent[q]
        if P != Q:
            out.add((min(P, Q), max(P, Q)))
    return sorted(out)


def distance2_sets(adj):
    d2 = []
    for i in range(len(adj)):
        s = set(adj[i])
        for c in adj[i]:
            s |= adj[c]
        s.discard(i)
        d2.append(s)
    return d2


def lattice_colours(adj, coords):
    """Colouring by a lattice pattern of the block coordinates, when one is
    valid at distance 2 on this graph: (x + 2y) mod 5 and (x + 2y + 3z) mod 7
    for nearest-neighbour graphs, the product of (coordinate mod 3) for graphs
    inside the 3^d-point stencil; candidates are tried in this order."""
    if coords is None:
        return None
    coords = np.asarray(coords)
    ndim = coords.shape[1]
    if ndim == 1:
        cands = [("lin", (1,), 3)]
    elif ndim == 2:
        cands = [("lin", (1, 2), 5), ("prod", None, 3)]
    else:
        cands = [("lin", (1, 2, 3), 7), ("prod", None, 3)]
    d2 = distance2_sets(adj)
    for kind, a, q in cands:
        if kind == "lin":
            col = [int(sum(a[k] * int(c[k]) for k in range(ndim)) % q) for c in coords]
        else:
            col = [int(sum((int(c[k]) % q) * q ** k for k in range(ndim))) for c in coords]
        if all(col[i] != col[j] for i in range(len(adj)) for j in d2[i]):
            return col
    return None


def colour_order(adj, coords=None):
    """Multicolour order: blocks within graph distance 2 never share a colour;
    blocks are ordered by (colour, index).  The colouring is the lattice one
    when valid, else greedy in block index order.  Returns (order, colour)."""
    M = len(adj)
    colour = lattice_colours(adj, coords)
    if colour is None:
        d2 = distance2_sets(adj)
        colour = [-1] * M
        for i in range(M):
            used = {colour[j] for j in d2[i] if j < i}
            c = 0
            while c in used:
                c += 1
            colour[i] = c
    order = sorted(range(M), key=lambda i: (colour[i], i))
    return order, colour


def element_order(adj, kind: str, coords=None):
    """Elimination order of a level: 'paper' is the block order of the level
    (Algorithm 2 loops i = 1..M_j), 'multicolour' is :func:`colour_order`."""
    if kind == "paper":
        return list(range(len(adj)))
    if kind == "multicolour":
        return colour_order(adj, coords)[0]
    raise ValueError(kind)


def simulate_level(M, close_pairs, order):
    """Structural pass over one level in the given order.

    For every step ``i`` returns the far neighbours that exist when ``i`` is
    compressed (created by earlier steps), the set of far pairs that exist
    at the end of the level, and the removed blocks.  A block whose far row
    is empty when it is processed is eliminated entirely (the first-row
    elimination of Section 2.1) and leaves the graph, as node 1 does in the
    example of Section 2.4.  Step ``i`` creates the pairs among ``close(i)``
    that are neither close nor already far and whose blocks are not removed.
    """
    adj = adjacency(M, close_pairs)
    far = [set() for _ in range(M)]
    removed = set()
    far_at_step = {}
    for i in order:
        far_at_step[i] = sorted(far[i])
        if not far[i]:
            removed.add(i)
        group = sorted(adj[i])
        for a, c in itertools.combinations(group, 2):
            if a in removed or c in removed:
                continue
            if c not in adj[a] and c not in far[a]:
                far[a].add(c)
                far[c].add(a)
    far_pairs = sorted((p, q) for p in range(M) for q in far[p] if p < q)
    return far_at_step, far_pairs, removed


def live_pairs(pairs, removed):
    """Pairs of a level that carry unknowns into the next level."""
    return [(p, q) for p, q in pairs if p not in removed and q not in removed]
