"""Pins for the CPU reference octree (Morton keys, boxes, adaptive FMM lists):
hand-worked keys, structural invariants and brute-force coverage of every
(target, source) point pair."""
import numpy as np
import pytest

from oracle import tree as T


def test_hand_worked_keys():
    pts = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.5, 0.0, 0.0],
                    [0.0, 0.5, 0.0], [0.0, 0.0, 0.25], [0.75, 0.75, 0.75]])
    key, perm, lo, scale = T.morton_keys(pts)
    assert scale == 2097152.0 and (lo == 0).all()
    assert key[0] == 0
    assert key[1] == (1 << 63) - 1                 # clamped to 2^21-1 per axis
    assert key[2] == 1 << 60                        # q_x = 2^20 -> bit 3*20
    assert key[3] == 1 << 61
    assert key[4] == 1 << 59                        # q_z = 2^19 -> bit 3*19+2
    assert key[5] == (7 << 60) | (7 << 57)
    assert list(perm) == [0, 4, 2, 3, 5, 1]


def test_sort_is_stable_on_equal_keys():
    pts = np.array([[0.0, 0, 0], [1, 1, 1], [0, 0, 0], [0, 0, 0]])
    key, perm, _, _ = T.morton_keys(pts)
    assert list(perm) == [0, 2, 3, 1]


def _clustered(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n // 2, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)           # sphere surface
    b = rng.normal(scale=0.05, size=(n - n // 2, 3)) + rng.uniform(-1, 1, 3)
    return np.vstack([a, b])


@pytest.mark.parametrize("n,cap,seed", [(300, 8, 1), (1500, 16, 2), (3000, 32, 3)])
def test_tree_invariants(n, cap, seed):
    x = _clustered(n, seed)
    t = T.build_tree(x, cap)
    assert t.pt_begin[0] == 0 and t.pt_end[0] == n
    order = np.lexsort((t.prefix, t.level))
    assert (order == np.arange(t.nbox)).all()            # numbered by (level, prefix)
    for b in range(t.nbox):
        if t.n_child[b]:
            ch = np.arange(t.child_begin[b], t.child_begin[b] + t.n_child[b])
            assert (t.parent[ch] == b).all()
            assert t.pt_begin[ch[0]] == t.pt_begin[b] and t.pt_end[ch[-1]] == t.pt_end[b]
            assert (t.pt_begin[ch[1:]] == t.pt_end[ch[:-1]]).all()
            assert ((t.prefix[ch] >> 3) == t.prefix[b]).all()
            assert t.pt_end[b] - t.pt_begin[b] > cap
        else:
            assert t.pt_end[b] - t.pt_begin[b] <= cap or t.level[b] == 21
            assert t.pt_end[b] > t.pt_begin[b]


@pytest.mark.parametrize("n,cap,seed", [(200, 4, 4), (1200, 12, 5), (4000, 24, 6)])
def test_lists_cover_every_pair_exactly_once(n, cap, seed):
    x = _clustered(n, seed)
    t = T.build_tree(x, cap)
    L = T.build_lists(t)
    leaf = t.is_leaf()
    box_of = np.zeros(n, np.int64)
    for b in np.nonzero(leaf)[0]:
        box_of[t.pt_begin[b]:t.pt_end[b]] = b
    cover = np.zeros((t.nbox, n), np.int64)             # per target leaf: source hits
    for B in np.nonzero(leaf)[0]:
        for C in L.U[B] + L.W[B]:
            cover[B, t.pt_begin[C]:t.pt_end[C]] += 1
        A = B
        while A >= 0:
            for C in L.X[A]:
                cover[B, t.pt_begin[C]:t.pt_end[C]] += 1
            for C in L.V[A]:
                cover[B, t.pt_begin[C]:t.pt_end[C]] += 1
            A = t.parent[A]
    assert (cover[leaf] == 1).all()
    # structural facts
    adj = T.adjacency_matrix(t)
    assert (adj == adj.T).all()
    assert max(len(v) for v in L.V) <= 189
    for B in range(t.nbox):
        assert len(L.V[B]) == len(L.V_class[B])
        assert all(0 <= c < 316 for c in L.V_class[B])
        for lst in (L.U[B], L.V[B], L.W[B], L.X[B]):
            assert lst == sorted(lst)
        for C in L.X[B]:
            assert leaf[C]


@pytest.mark.parametrize("n,cap,seed", [(200, 4, 4), (1200, 12, 5), (4000, 24, 6)])
def test_direct_pairs_decompose_into_symmetric_tasks(n, cap, seed):
    """The direct (P2P) point pairs of the U, W and X lists are symmetric, so
    each unordered pair of point sets can be evaluated once: a leaf's own
    points (one way, p != t), the leaves of U(B) after B and the boxes of
    W(B), each credited both ways, give every ordered pair of U(B) u W(B) u
    X(A) (A = B and its ancestors) exactly once."""
    x = _clustered(n, seed)
    t = T.build_tree(x, cap)
    L = T.build_lists(t)
    leaf = np.nonzero(t.is_leaf())[0]
    direct = np.zeros((n, n), np.int64)        # the lists' ordered pairs
    tasks = np.zeros((n, n), np.int64)         # the symmetric tasks' ordered pairs
    for B in leaf:
        P = slice(t.pt_begin[B], t.pt_end[B])
        srcs = set(L.U[B]) | set(L.W[B])
        A = B
        while A >= 0:
            srcs |= set(L.X[A])
            A = t.parent[A]
        for C in srcs:
            direct[P, t.pt_begin[C]:t.pt_end[C]] += 1
        tasks[P, P] += 1
        for C in [c for c in L.U[B] if c > B] + list(L.W[B]):
            S = slice(t.pt_begin[C], t.pt_end[C])
            tasks[P, S] += 1
            tasks[S, P] += 1
    np.fill_diagonal(direct, 0)
    np.fill_diagonal(tasks, 0)
    assert direct.max() == 1 and tasks.max() == 1
    assert (direct == tasks).all()
    assert (direct == direct.T).all()


def test_offset_class_ranking():
    assert T.offset_class((-3, -3, -3)) == 0
    assert T.offset_class((3, 3, 3)) == 315
    assert T.offset_class((-3, -3, -2)) == 1
