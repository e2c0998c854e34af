"""The setup's symbolic analysis (hc_test_symbolic, host only): the
approximate minimum degree order, its elimination tree, column counts,
fundamental supernodes and level sets, checked against the definitions by
brute-force graph elimination on small graphs: eliminating vertex v joins
its remaining neighbours into a clique; the factor's column for v holds v and
those neighbours; the tree parent of v is the first of them eliminated."""
import numpy as np
import pytest

from paper_2412_19027_amd import hipcone as HC


def csr(n, edges):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    ptr = np.zeros(n + 1, np.int64)
    for i in range(n):
        ptr[i + 1] = ptr[i] + len(adj[i])
    flat = np.array([j for i in range(n) for j in sorted(adj[i])], np.int32)
    return ptr, flat, adj


def eliminate(n, adj, order):
    """Brute force: per position the factor column's row positions, and the tree."""
    pos = {v: k for k, v in enumerate(order)}
    nb = [set(a) for a in adj]
    cols, parent = [], []
    for k, v in enumerate(order):
        rest = {pos[u] for u in nb[v]}
        cols.append(rest)
        parent.append(min(rest) if rest else -1)
        for a in nb[v]:
            nb[a] |= nb[v] - {a}
            nb[a].discard(v)
        nb[v] = set()
    return cols, parent


def random_graph(rng, n, p):
    return [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]


def grid(r, c):
    idx = lambda i, j: i * c + j
    e = []
    for i in range(r):
        for j in range(c):
            if i + 1 < r:
                e.append((idx(i, j), idx(i + 1, j)))
            if j + 1 < c:
                e.append((idx(i, j), idx(i, j + 1)))
    return e


def check(n, edges):
    ptr, flat, adj = csr(n, edges)
    out = HC.symbolic(n, ptr, flat)
    order = out["order"]
    assert sorted(order.tolist()) == list(range(n))          # a permutation
    cols, parent = eliminate(n, adj, order.tolist())
    assert out["parent"].tolist() == parent                    # elimination tree
    assert out["count"].tolist() == [1 + len(c) for c in cols]  # column counts
    for k, p in enumerate(parent):                             # postordered: parent after child
        assert p == -1 or p > k
    # subtrees contiguous: each subtree ends at its root
    size = [1] * n
    for k in range(n):
        if parent[k] >= 0:
            size[parent[k]] += size[k]
    for k in range(n):
        first = k - size[k] + 1
        assert all(first <= d <= k for d in range(first, k + 1) if d >= 0)
        for d in range(first, k):
            a = d
            while a != -1 and a < k:
                a = parent[a]
            assert a == k
    # fundamental supernodes
    f, sp, sl = out["sn_first"], out["sn_parent"], out["sn_level"]
    assert f[0] == 0 and f[-1] == n and np.all(np.diff(f) > 0)
    sn_of = np.repeat(np.arange(len(f) - 1), np.diff(f))
    for k in range(n - 1):
        same = sn_of[k] == sn_of[k + 1]
        fund = parent[k] == k + 1 and sum(1 for c in range(n) if parent[c] == k + 1) == 1 \
            and out["count"][k] == out["count"][k + 1] + 1
        assert same == fund, k
    for t in range(len(sp)):
        last = f[t + 1] - 1
        assert sp[t] == (sn_of[parent[last]] if parent[last] >= 0 else -1)
        kids = [u for u in range(len(sp)) if sp[u] == t]
        assert sl[t] == (1 + max(sl[u] for u in kids) if kids else 0)
    assert out["nlevels"] == (1 + max(sl) if len(sl) else 0)
    return out


@pytest.mark.parametrize("seed", range(12))
def test_symbolic_random_graphs(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    check(n, random_graph(rng, n, float(rng.choice([0.03, 0.08, 0.2, 0.5]))))


def test_symbolic_special_graphs():
    # path: no fill, n - 1 off-diagonal entries in the factor
    out = check(30, [(i, i + 1) for i in range(29)])
    assert out["count"].sum() == 2 * 30 - 1
    # star: the centre goes once at most one leaf is left (no fill)
    out = check(25, [(0, j) for j in range(1, 25)])
    assert 0 in out["order"][-2:].tolist() and out["count"].sum() == 2 * 25 - 1
    # clique: one supernode
    out = check(12, [(i, j) for i in range(12) for j in range(i + 1, 12)])
    assert len(out["sn_parent"]) == 1 and out["nlevels"] == 1
    # disconnected pieces and isolated vertices: a forest
    out = check(20, [(0, 1), (1, 2), (5, 6), (6, 7), (7, 5), (10, 11)])
    assert (out["parent"] == -1).sum() == 12 + 3   # 12 isolated vertices, 3 pieces
    check(0, [])
    check(1, [])


def test_symbolic_fill_against_natural_order():
    """A 16 x 16 grid: the minimum degree order creates far less fill than the
    row-by-row order (a band of half-width 16)."""
    n = 256
    edges = grid(16, 16)
    ptr, flat, adj = csr(n, edges)
    out = check(n, edges)
    cols_nat, _ = eliminate(n, adj, list(range(n)))
    nat = sum(1 + len(c) for c in cols_nat)
    assert out["count"].sum() < 0.8 * nat, (out["count"].sum(), nat)


def test_symbolic_rejects_malformed():
    with pytest.raises(HC.HipconeError) as e:
        HC.symbolic(3, np.array([0, 1, 2, 1]), np.array([1, 0], np.int32))
    assert e.value.code == -3
    with pytest.raises(HC.HipconeError) as e:
        HC.symbolic(2, np.array([0, 1, 2]), np.array([1, 5], np.int32))
    assert e.value.code == -3


def test_setup_leaf_blocks_from_the_elimination_tree():
    """hc_setup's two-level split (host only): the non-tail columns of an MPC
    request form one chain-like component of more than 32 columns; the setup
    orders it, takes subtrees of at most 32 columns of its elimination tree as
    leaf blocks and puts the rest in the tail.  The logistic regression's
    per-sample components are whole subtrees (one leaf each)."""
    from paper_2412_19027_amd import workloads as W
    p = W.mpc_socp(7, 4)
    a = HC.analyze(p)
    assert a["sym_split_columns"] == p.n
    assert a["n_leaves"] >= 1 and a["leaf_columns"] <= 32 * a["n_leaves"]
    assert a["n_ordered"] + a["leaf_columns"] == p.n
    assert a["sym_supernodes"] >= 1 and a["sym_levels"] >= 2 and a["sym_nnz_l"] >= p.n
    q = W.logreg_exp(0, samples=300, features=20)
    b = HC.analyze(q)
    assert b["n_leaves"] == 300 + 20 and b["n_ordered"] == 20
    assert b["sym_split_columns"] == b["leaf_columns"] and b["sym_levels"] == 1
