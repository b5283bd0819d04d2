"""Pins for the oracle's bounds, X0 map, graphs and partitions (brute force, closed
forms, invariants).  CPU only."""
import numpy as np
import pytest

from oracle.bounds import gershgorin, x0_values, ell_to_dense
from oracle.graph import (graph_x2, graph_x2_dense, graph_pattern, graph_dprev,
                          graph_dprev_symbolic, csr_from_edges)
from oracle.partition import block_cores, halo_subgraphs, partition, bfs_order


def _csr_sets(rp, cl):
    return [set(cl[rp[i]:rp[i + 1]].tolist()) for i in range(len(rp) - 1)]


def test_gershgorin_hand_example():
    # H = [[1, -2, 0], [-2, 3, 0.5], [0, 0.5, -1]]
    col = np.array([[0, 1, -1], [0, 1, 2], [1, 2, -1]], dtype=np.int32)
    val = np.array([[1.0, -2.0, 0.0], [-2.0, 3.0, 0.5], [0.5, -1.0, 0.0]])
    emin, emax = gershgorin(col, val)
    # discs: 1 +- 2, 3 +- 2.5, -1 +- 0.5
    assert (emin, emax) == (-1.5, 5.5)
    x0 = x0_values(col, val, emin, emax)
    X = ell_to_dense(col, x0)
    assert np.array_equal(X, (5.5 * np.eye(3) - ell_to_dense(col, val)) / 7.0)


def test_gershgorin_contains_spectrum(model_cache):
    m = model_cache("n1024")
    emin, emax = gershgorin(m["H_col"], m["H_val"])
    w = np.linalg.eigvalsh(ell_to_dense(m["H_col"], m["H_val"]))
    assert emin <= w[0] and w[-1] <= emax
    X0 = ell_to_dense(m["H_col"], x0_values(m["H_col"], m["H_val"], emin, emax))
    wx = np.linalg.eigvalsh(X0)
    assert wx[0] >= -1e-12 and wx[-1] <= 1 + 1e-12


def test_gershgorin_diagonal_matrix():
    col = np.arange(5, dtype=np.int32)[:, None]
    val = np.array([[3.0], [-1.0], [2.5], [0.0], [7.0]])
    assert gershgorin(col, val) == (-1.0, 7.0)


def _brute_x2_graph(H_col, H_val, tau):
    """Pure-Python triple loop: bounds, X0 and the canonical X0^2, Python floats."""
    N, W = H_col.shape
    H = [[0.0] * N for _ in range(N)]
    pat = [set() for _ in range(N)]
    for i in range(N):
        for t in range(W):
            j = int(H_col[i, t])
            if j >= 0:
                H[i][j] = float(H_val[i, t])
                pat[i].add(j)
    lo, hi = [], []
    for i in range(N):
        r = 0.0
        for j in sorted(pat[i]):
            if j != i:
                r = r + abs(H[i][j])
        lo.append(H[i][i] - r)
        hi.append(H[i][i] + r)
    emin, emax = min(lo), max(hi)
    d = emax - emin
    X = [[((emax if i == j else 0.0) - H[i][j]) / d if j in pat[i] else 0.0 for j in range(N)]
         for i in range(N)]
    edges = set()
    for i in range(N):
        hop2 = set()
        for k in pat[i]:
            hop2 |= pat[k]
        for j in range(N):
            acc = 0.0
            for k in range(N):
                acc = acc + X[i][k] * X[k][j]
            if (j in hop2 and abs(acc) >= tau) or i == j:
                edges.add((i, j))
                edges.add((j, i))
    r = np.array([e[0] for e in edges])
    c = np.array([e[1] for e in edges])
    return csr_from_edges(N, r, c)


@pytest.mark.parametrize("tau", [1e-2, 1e-3, 1e-5, 0.0])
def test_x2_graph_bit_exact_vs_triple_loop(model_cache, tau):
    m = model_cache("tiny48")
    rp, cl = graph_x2(m["H_col"], m["H_val"], tau)
    brp, bcl = _brute_x2_graph(m["H_col"], m["H_val"], tau)
    assert np.array_equal(rp, brp) and np.array_equal(cl, bcl)


def test_x2_graph_sparse_equals_dense(model_cache):
    m = model_cache("small256")
    for tau in (1e-3, 1e-5):
        a = graph_x2(m["H_col"], m["H_val"], tau)
        b = graph_x2_dense(m["H_col"], m["H_val"], tau)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_x2_graph_invariants(model_cache):
    m = model_cache("small256")
    N = m["N"]
    prev = None
    for tau in (1e-2, 1e-3, 1e-4, 1e-5):
        rp, cl = graph_x2(m["H_col"], m["H_val"], tau)
        sets = _csr_sets(rp, cl)
        assert all(i in sets[i] for i in range(N)), "self-loops"
        assert all(i in sets[j] for i in range(N) for j in sets[i]), "symmetric"
        for i in range(N):
            assert np.all(np.diff(cl[rp[i]:rp[i + 1]]) > 0), "sorted, unique"
        if prev is not None:
            assert all(prev[i] <= sets[i] for i in range(N)), "monotone in tau"
        prev = sets


def test_pattern_and_dprev_rules(model_cache):
    m = model_cache("tiny48")
    N = m["N"]
    H = ell_to_dense(m["H_col"], m["H_val"])
    rp, cl = graph_pattern(m["H_col"], m["H_val"], 0.01)
    want = (np.abs(H) >= 0.01) | np.eye(N, dtype=bool)
    want |= want.T
    got = np.zeros((N, N), dtype=bool)
    for i in range(N):
        got[i, cl[rp[i]:rp[i + 1]]] = True
    assert np.array_equal(got, want)
    # previous D as column-ELL: a random sparse matrix
    rng = np.random.default_rng(5)
    Dd = np.where(rng.random((N, N)) < 0.1, rng.normal(0, 1e-3, (N, N)), 0.0)
    Dc = np.full((N, N), -1, dtype=np.int32)
    Dv = np.zeros((N, N))
    for i in range(N):
        rows = np.nonzero(Dd[:, i])[0]
        Dc[i, :len(rows)] = rows
        Dv[i, :len(rows)] = Dd[rows, i]
    rp2, cl2 = graph_dprev(m["H_col"], m["H_val"], Dc, Dv, 1e-3, 1e-4)
    x2 = _csr_sets(*graph_x2(m["H_col"], m["H_val"], 1e-3))
    got2 = _csr_sets(rp2, cl2)
    for i in range(N):
        exp = set(x2[i]) | set(np.nonzero(np.abs(Dd[i, :]) >= 1e-4)[0].tolist()) \
            | set(np.nonzero(np.abs(Dd[:, i]) >= 1e-4)[0].tolist())
        assert got2[i] == exp
    # Eq. 8 symbolic: paths of length two
    rp3, cl3 = graph_dprev_symbolic(m["H_col"], Dc, Dv, 1e-4)
    P = (np.abs(Dd) >= 1e-4) | (H != 0) | np.eye(N, dtype=bool)
    P |= P.T
    S = np.zeros((N, N), dtype=bool)
    for i in range(N):
        for k in range(N):
            if P[i, k]:
                S[i] |= P[k]
    got3 = np.zeros((N, N), dtype=bool)
    for i in range(N):
        got3[i, cl3[rp3[i]:rp3[i + 1]]] = True
    assert np.array_equal(got3, S)


def test_block_cores():
    assert block_cores(10, 4).tolist() == [0, 4, 8, 10]
    assert block_cores(8, 4).tolist() == [0, 4, 8]
    assert block_cores(3, 16).tolist() == [0, 3]


def test_halo_brute_force(model_cache):
    m = model_cache("small256")
    rp, cl = graph_x2(m["H_col"], m["H_val"], 1e-3)
    sets = _csr_sets(rp, cl)
    for cs in (1, 8, 16, 37):
        core_ptr, core_v, sub_ptr, sub_idx = partition(rp, cl, cs)
        for s in range(len(core_ptr) - 1):
            core = list(range(core_ptr[s], core_ptr[s + 1]))
            halo = set()
            for v in core:
                halo |= sets[v]
            halo -= set(core)
            want = core + sorted(halo)
            assert sub_idx[sub_ptr[s]:sub_ptr[s + 1]].tolist() == want


def test_bfs_partition_invariants(model_cache):
    m = model_cache("small256")
    rp, cl = graph_x2(m["H_col"], m["H_val"], 1e-3)
    order = bfs_order(rp, cl)
    N = m["N"]
    assert np.array_equal(np.sort(order), np.arange(N))
    core_ptr, core_v, sub_ptr, sub_idx = partition(rp, cl, 16, "bfs")
    assert np.array_equal(np.sort(core_v), np.arange(N)), "cores disjoint and covering"
    sets = _csr_sets(rp, cl)
    for s in range(len(core_ptr) - 1):
        sub = sub_idx[sub_ptr[s]:sub_ptr[s + 1]]
        k = core_ptr[s + 1] - core_ptr[s]
        core = sub[:k]
        assert np.array_equal(core, core_v[core_ptr[s]:core_ptr[s + 1]])
        assert np.all(np.diff(core) > 0) and np.all(np.diff(sub[k:]) > 0)
        closed = set()
        for v in core:
            closed |= sets[v]
        assert closed | set(core.tolist()) == set(sub.tolist()), "closed under one hop"


def test_rcut_graph_against_kdtree():
    """RCUT graph: the site pairs within r_cut found by scipy's periodic KD-tree (an
    independent search), expanded to orbitals, plus every same-site pair."""
    from scipy.spatial import cKDTree
    from oracle.graph import graph_rcut
    from synth import make_model
    m = make_model("small256")
    pos, L = m["pos"], m["L"]
    for rc in (3.0, 5.5):
        rp, col = graph_rcut(pos, L, rc, 2)
        pairs = cKDTree(pos, boxsize=L).query_pairs(rc, output_type="ndarray")
        n = len(pos)
        site_adj = [set([a]) for a in range(n)]
        for a, b in pairs:
            site_adj[a].add(b)
            site_adj[b].add(a)
        for i in range(2 * n):
            got = set(col[rp[i]:rp[i + 1]].tolist())
            want = {2 * b + q for b in site_adj[i // 2] for q in (0, 1)}
            assert got == want, (rc, i)
        assert np.all(np.diff(col[rp[0]:rp[1]]) > 0)
