"""Multilevel communities for the cores (oracle; test infrastructure only).

The paper takes its communities from a multilevel graph partitioner and prices a partition by
the dense work of its subgraphs, sum over cores of (|core| + |halo|)^3 (cost discussion after
Eq. 6; communities, obs. vi-vii).  This is the plain statement of the partitioner the library
implements, step by step, so that the library's cores can be checked index for index:

1. Edge weights on the input graph (self loops dropped): the number of common closed
   neighbours of the two ends, i.e. (A A)_uv for the 0/1 adjacency A with its diagonal.
2. Coarsening by heavy-edge matching until no pair can be matched.  Level l visits vertices
   in the order of SplitMix64((l << 32) | v) (ties by v); an unmatched vertex takes the
   unmatched neighbour maximising (edge weight, -vertex weight, -index) among those whose
   joint weight is at most max(1, cap // 4); pairs become coarse vertices numbered by their
   smaller member, with summed vertex weights and summed edge weights (self loops dropped).
3. On the coarsest graph, parts are grown: seeds in breadth-first order (components by their
   smallest vertex, neighbours ascending); a part repeatedly takes the unassigned vertex
   maximising (summed edge weight to the part, -vertex weight, -index) that keeps it within
   cap.
4. The parts are projected back to the input graph; non-empty parts in ascending order of
   their smallest vertex, vertices ascending.
The cost returned is sum (k_p + h_p)^3, k_p the core size and h_p the number of vertices
outside p adjacent to p.  The on-the-fly update carries given cores to a new graph on the same
vertices (renumbered as in step 4) and returns their cost there.

Pins (tests): every vertex in exactly one core of at most cap vertices; the reported cost
equals sum (|core| + |halo|)^3 recomputed from the halos; hand-checkable graphs (disjoint
cliques of cap vertices are found exactly, a path is cut into consecutive runs); the cores do
not depend on the vertex numbering of a clique graph; a spatial model gets cheaper cores than
blocks of its sorted vertex order, and a random relabelling of it gets cores of about the same
cost.
"""
import numpy as np
import scipy.sparse as sp

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output function (Steele, Lea and Flood, 2014) of a 64-bit counter."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def visit_order(n: int, level: int):
    return sorted(range(n), key=lambda v: (splitmix64((level << 32) | v), v))


def common_neighbour_weights(row_ptr, col):
    """Adjacency lists without self loops and their weights (A A)_uv, A with its diagonal."""
    n = len(row_ptr) - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    A = sp.csr_matrix((np.ones(len(col), dtype=np.int64), (rows, np.asarray(col))), shape=(n, n))
    A = ((A + sp.identity(n, dtype=np.int64, format="csr")) > 0).astype(np.int64)
    AA = (A @ A).tocsr()
    adj, ew = [], []
    for u in range(n):
        row = dict(zip(AA.indices[AA.indptr[u]:AA.indptr[u + 1]].tolist(),
                       AA.data[AA.indptr[u]:AA.indptr[u + 1]].tolist()))
        nb = [int(v) for v in col[row_ptr[u]:row_ptr[u + 1]] if v != u]
        adj.append(nb)
        ew.append([row[v] for v in nb])
    return adj, ew


def coarsen(adj, ew, vw, cap, level):
    """One heavy-edge matching level; None when no pair was matched, else
    (cmap, coarse adj, coarse ew, coarse vw)."""
    n = len(adj)
    match = [-1] * n
    any_pair = False
    for v in visit_order(n, level):
        if match[v] >= 0:
            continue
        best, key = -1, None
        for u, w in zip(adj[v], ew[v]):
            if match[u] >= 0 or vw[u] + vw[v] > cap:
                continue
            k = (w, -vw[u], -u)
            if key is None or k > key:
                best, key = u, k
        if best >= 0:
            match[v], match[best] = best, v
            any_pair = True
        else:
            match[v] = v
    if not any_pair:
        return None
    cmap = [-1] * n
    nc = 0
    for v in range(n):
        if cmap[v] < 0:
            cmap[v] = cmap[match[v]] = nc
            nc += 1
    cvw = [0] * nc
    for v in range(n):
        cvw[cmap[v]] += vw[v]
    cadj, cew = [[] for _ in range(nc)], [[] for _ in range(nc)]
    for v in range(n):
        c = cmap[v]
        if min(v, match[v]) != v:
            continue
        acc = {}
        for x in {v, match[v]}:
            for u, w in zip(adj[x], ew[x]):
                cu = cmap[u]
                if cu != c:
                    acc[cu] = acc.get(cu, 0) + w
        for cu in sorted(acc):
            cadj[c].append(cu)
            cew[c].append(acc[cu])
    return cmap, cadj, cew, cvw


def bfs_order(adj):
    n = len(adj)
    seen = [False] * n
    order = []
    for s0 in range(n):
        if seen[s0]:
            continue
        seen[s0] = True
        queue = [s0]
        head = 0
        while head < len(queue):
            v = queue[head]
            head += 1
            order.append(v)
            for u in adj[v]:
                if not seen[u]:
                    seen[u] = True
                    queue.append(u)
    return order


def grow_parts(adj, ew, vw, cap):
    n = len(adj)
    part = [-1] * n
    np_ = 0
    for seed in bfs_order(adj):
        if part[seed] >= 0:
            continue
        p = np_
        np_ += 1
        weight = 0
        conn = {}
        v = seed
        while True:
            part[v] = p
            weight += vw[v]
            for u, w in zip(adj[v], ew[v]):
                if part[u] < 0:
                    conn[u] = conn.get(u, 0) + w
            best, key = -1, None
            for u, cu in conn.items():
                if part[u] >= 0 or weight + vw[u] > cap:
                    continue
                k = (cu, -vw[u], -u)
                if key is None or k > key:
                    best, key = u, k
            if best < 0:
                break
            v = best
    return part


def subgraph_cost(adj, part, n_parts):
    """sum over parts of (k_p + h_p)^3."""
    k = [0] * n_parts
    halo = [set() for _ in range(n_parts)]
    for u in range(len(adj)):
        k[part[u]] += 1
        for x in adj[u]:
            if part[x] != part[u]:
                halo[part[x]].add(u)
    return sum((k[p] + len(halo[p])) ** 3 for p in range(n_parts))


def _emit(part, n):
    members = {}
    for v in range(n):
        members.setdefault(part[v], []).append(v)
    cores = sorted(members.values(), key=lambda c: c[0])
    core_ptr = np.zeros(len(cores) + 1, dtype=np.int32)
    core_ptr[1:] = np.cumsum([len(c) for c in cores])
    core_vtx = np.concatenate([np.array(c, dtype=np.int32) for c in cores])
    return core_ptr, core_vtx


def partition_multilevel(row_ptr, col, cap: int):
    """(core_ptr, core_vertices, cost) of the multilevel cores of at most ``cap`` vertices."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = len(row_ptr) - 1
    adj0, ew0 = common_neighbour_weights(row_ptr, col)
    levels = [(adj0, ew0, [1] * n)]
    cmaps = []
    ccap = max(1, cap // 4)
    level = 0
    while True:
        adj, ew, vw = levels[-1]
        r = coarsen(adj, ew, vw, ccap, level)
        if r is None:
            break
        cmap, cadj, cew, cvw = r
        cmaps.append(cmap)
        levels.append((cadj, cew, cvw))
        level += 1
    part = grow_parts(*levels[-1], cap)
    n_parts = max(part) + 1
    for l in range(len(levels) - 2, -1, -1):
        part = [part[cmaps[l][v]] for v in range(len(levels[l][0]))]
    cost = subgraph_cost(adj0, part, n_parts)
    core_ptr, core_vtx = _emit(part, n)
    return core_ptr, core_vtx, int(cost)


def partition_update(row_ptr, col, prev_core_ptr, prev_core_vtx):
    """Given cores carried to a new graph on the same vertices (on-the-fly update between MD
    steps): (core_ptr, core_vertices, cost on the new graph)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = len(row_ptr) - 1
    adj = [[int(v) for v in col[row_ptr[u]:row_ptr[u + 1]] if v != u] for u in range(n)]
    n_parts = len(prev_core_ptr) - 1
    part = [-1] * n
    for p in range(n_parts):
        for i in range(prev_core_ptr[p], prev_core_ptr[p + 1]):
            part[int(prev_core_vtx[i])] = p
    cost = subgraph_cost(adj, part, n_parts)
    core_ptr, core_vtx = _emit(part, n)
    return core_ptr, core_vtx, int(cost)
