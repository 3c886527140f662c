"""CPU reference octree: Morton keys, adaptive boxes and the four interaction
lists of the adaptive FMM (Carrier-Greengard-Rokhlin lists; list-3 and list-4
as described in Section 3.2 of the paper).  The GPU tree must match this
bit-exactly.

TEST INFRASTRUCTURE ONLY (see oracle/core.py).

Conventions (the paper leaves them open; these are the readings used):
  keys   -- 21 bits per axis: lo = per-axis minimum, S = largest extent
            (1 if zero), scale = 2^21 / S (one rounded division),
            q = min(2^21 - 1, floor((x - lo) * scale)) with a separate
            subtract and multiply (no fused multiply-add); bit b of q_x, q_y,
            q_z goes to key bit 3b, 3b+1, 3b+2.  Points sorted by (key, index).
  boxes  -- (level, prefix = key >> 3 (21 - level)); a box with more than
            leaf_cap points below level 21 is split into its non-empty
            children; boxes numbered by ascending (level, prefix).
  adj    -- distinct boxes, neither an ancestor of the other, whose closed
            cubes touch.
  U(B)   -- leaf B: B and every adjacent leaf.
  V(B)   -- level >= 2: children of the colleagues of parent(B) not adjacent
            to B.
  W(B)   -- leaf B: descendants C of B's colleagues with C not adjacent to B
            but parent(C) adjacent to B (list-3).
  X(B)   -- {C : B in W(C)} (list-4).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

MAXLEVEL = 21


def morton_keys(xyz):
    x = np.ascontiguousarray(xyz, dtype=np.float64)
    lo = x.min(axis=0)
    hi = x.max(axis=0)
    S = float((hi - lo).max())
    if S == 0.0:
        S = 1.0
    scale = 2097152.0 / S
    d = x - lo                    # one rounded subtraction
    q = np.floor(d * scale)       # one rounded multiplication
    q = np.minimum(q, 2097151.0).astype(np.int64)
    key = np.zeros(len(x), dtype=np.int64)
    for b in range(MAXLEVEL):
        for a in range(3):
            key |= ((q[:, a] >> b) & 1) << (3 * b + a)
    perm = np.lexsort((np.arange(len(x)), key))
    return key, perm, lo, scale


def deinterleave(prefix, level):
    ix = iy = iz = 0
    for b in range(level):
        ix |= ((prefix >> (3 * b)) & 1) << b
        iy |= ((prefix >> (3 * b + 1)) & 1) << b
        iz |= ((prefix >> (3 * b + 2)) & 1) << b
    return ix, iy, iz


@dataclass
class Tree:
    keys_sorted: np.ndarray
    perm: np.ndarray
    level: np.ndarray
    prefix: np.ndarray
    parent: np.ndarray
    child_begin: np.ndarray
    n_child: np.ndarray
    pt_begin: np.ndarray
    pt_end: np.ndarray
    anchor: np.ndarray      # [nb,3] integer anchors
    side: np.ndarray

    @property
    def nbox(self):
        return len(self.level)

    def is_leaf(self):
        return self.n_child == 0


def build_tree(xyz, leaf_cap: int) -> Tree:
    key, perm, _, _ = morton_keys(xyz)
    ks = key[perm]
    level, prefix, parent, cb, nc, pb, pe = [0], [0], [-1], [-1], [0], [0], [len(ks)]
    cur = [0]
    while cur:
        nxt = []
        for b in cur:
            l = level[b]
            if pe[b] - pb[b] > leaf_cap and l < MAXLEVEL:
                sh = 3 * (MAXLEVEL - l - 1)
                seg = ks[pb[b]:pe[b]] >> sh
                starts = np.nonzero(np.r_[True, seg[1:] != seg[:-1]])[0]
                ends = np.r_[starts[1:], len(seg)]
                cb[b] = len(level)
                nc[b] = len(starts)
                for s, e in zip(starts, ends):
                    level.append(l + 1)
                    prefix.append(int(seg[s]))
                    parent.append(b)
                    cb.append(-1)
                    nc.append(0)
                    pb.append(pb[b] + int(s))
                    pe.append(pb[b] + int(e))
                    nxt.append(len(level) - 1)
        cur = nxt
    level = np.array(level, np.int64)
    prefix = np.array(prefix, np.int64)
    anchor = np.array([deinterleave(int(p), int(l)) for p, l in zip(prefix, level)],
                      dtype=np.int64).reshape(-1, 3)
    side = np.left_shift(1, MAXLEVEL - level)
    anchor = anchor * side[:, None]
    return Tree(ks, perm, level, prefix, np.array(parent, np.int64),
                np.array(cb, np.int64), np.array(nc, np.int64),
                np.array(pb, np.int64), np.array(pe, np.int64), anchor, side)


def ancestor_matrix(t: Tree):
    """anc[A, B] = A is a proper ancestor of B."""
    la, lb = t.level[:, None], t.level[None, :]
    sh = np.clip(3 * (lb - la), 0, 63)
    return (la < lb) & ((t.prefix[None, :] >> sh) == t.prefix[:, None])


def adjacency_matrix(t: Tree, anc=None):
    if anc is None:
        anc = ancestor_matrix(t)
    a, s = t.anchor, t.side
    touch = np.ones((t.nbox, t.nbox), bool)
    for d in range(3):
        ai, bi = a[:, d][:, None], a[:, d][None, :]
        touch &= (ai <= bi + s[None, :]) & (bi <= ai + s[:, None])
    np.fill_diagonal(touch, False)
    return touch & ~anc & ~anc.T


@dataclass
class Lists:
    U: list
    V: list
    W: list
    X: list
    V_class: list


def offset_class(d):
    """Rank of offset d in [-3,3]^3 minus [-1,1]^3, lexicographic (dx,dy,dz)."""
    r = 0
    for dx in range(-3, 4):
        for dy in range(-3, 4):
            for dz in range(-3, 4):
                if max(abs(dx), abs(dy), abs(dz)) <= 1:
                    continue
                if (dx, dy, dz) == tuple(d):
                    return r
                r += 1
    raise ValueError(d)


def build_lists(t: Tree) -> Lists:
    anc = ancestor_matrix(t)
    adj = adjacency_matrix(t, anc)
    nb = t.nbox
    leaf = t.is_leaf()
    same = t.level[:, None] == t.level[None, :]
    coll = adj & same
    U, V, W, X, VC = [], [], [], [], []
    for B in range(nb):
        if leaf[B]:
            u = np.nonzero(adj[B] & leaf)[0].tolist()
            U.append(sorted([B] + u))
        else:
            U.append([])
        v = []
        if t.level[B] >= 2:
            pcol = np.nonzero(coll[t.parent[B]])[0]
            cand = np.nonzero(np.isin(t.parent, pcol))[0]
            v = sorted(c for c in cand.tolist() if not adj[B, c])
        V.append(v)
        VC.append([offset_class((t.anchor[c] - t.anchor[B]) // t.side[B]) for c in v])
        w = []
        if leaf[B]:
            cols = np.nonzero(coll[B])[0]
            desc = np.any(anc[cols], axis=0) if len(cols) else np.zeros(nb, bool)
            for c in np.nonzero(desc)[0].tolist():
                if not adj[B, c] and adj[B, t.parent[c]]:
                    w.append(c)
        W.append(sorted(w))
    X = [[] for _ in range(nb)]
    for C in range(nb):
        for B in W[C]:
            X[B].append(C)
    X = [sorted(x) for x in X]
    return Lists(U, V, W, X, VC)
