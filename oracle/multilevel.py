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
4. From the coarsest level down to the input graph (the partition projected at each step),
   up to 4 passes: each vertex in ascending order moves to the neighbouring part with the
   largest positive gain in edge weight to it (ties: smaller part index) if that part has room.
5. On the input graph, up to 4 passes: each vertex in ascending order considers its three most
   tied neighbouring parts with room (by summed edge weight to them, ties by smaller index) and
   moves to the first of them that lowers sum (k_p + h_p)^3 most (strictly), k_p the core size
   and h_p the number of vertices outside p adjacent to p.
6. Non-empty parts in ascending order of their smallest vertex, vertices ascending.

Pins (tests): every vertex in exactly one core of at most cap vertices; the reported cost
equals sum (|core| + |halo|)^3 recomputed from the halos; hand-checkable graphs (disjoint
cliques of cap vertices are found exactly, a path is cut into consecutive runs); the cores do
not depend on the vertex numbering of a clique graph; a random relabelling of a spatial model
gives cores of about the same cost.
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


def refine_cut(adj, ew, vw, part, pw, cap, passes=4):
    for _ in range(passes):
        moved = 0
        for v in range(len(adj)):
            a = part[v]
            conn = {}
            for u, w in zip(adj[v], ew[v]):
                conn[part[u]] = conn.get(part[u], 0) + w
            own = conn.get(a, 0)
            best, key = -1, None
            for b, cb in conn.items():
                if b == a or pw[b] + vw[v] > cap:
                    continue
                gain = cb - own
                if gain > 0 and (key is None or (gain, -b) > key):
                    best, key = b, (gain, -b)
            if best >= 0:
                part[v] = best
                pw[a] -= vw[v]
                pw[best] += vw[v]
                moved += 1
        if not moved:
            break


def refine_cost(adj, ew, part, n_parts, cap, passes=4):
    """Moves lowering sum (k_p + h_p)^3; returns the final cost."""
    n = len(adj)
    cnt = [dict() for _ in range(n)]   # cnt[u][p]: neighbours of u in part p
    for u in range(n):
        for x in adj[u]:
            cnt[u][part[x]] = cnt[u].get(part[x], 0) + 1
    k = [0] * n_parts
    h = [0] * n_parts
    for v in range(n):
        k[part[v]] += 1
    for u in range(n):
        for p, c in cnt[u].items():
            if c > 0 and p != part[u]:
                h[p] += 1
    cost = sum((k[p] + h[p]) ** 3 for p in range(n_parts))
    for _ in range(passes):
        moved = 0
        for v in range(n):
            a = part[v]
            dha = 1 if cnt[v].get(a, 0) > 0 else 0
            for u in adj[v]:
                if part[u] != a and cnt[u].get(a, 0) == 1:
                    dha -= 1
            conn = {}
            for u, w in zip(adj[v], ew[v]):
                if part[u] != a:
                    conn[part[u]] = conn.get(part[u], 0) + w
            cands = sorted((b for b in conn if k[b] + 1 <= cap), key=lambda b: (-conn[b], b))[:3]
            before_a = (k[a] + h[a]) ** 3
            after_a = (k[a] - 1 + h[a] + dha) ** 3
            best, best_d, best_dhb = -1, 0, 0
            for b in cands:
                dhb = -1 if cnt[v].get(b, 0) > 0 else 0
                for u in adj[v]:
                    if part[u] != b and cnt[u].get(b, 0) == 0:
                        dhb += 1
                d = after_a - before_a + (k[b] + 1 + h[b] + dhb) ** 3 - (k[b] + h[b]) ** 3
                if d < best_d:
                    best, best_d, best_dhb = b, d, dhb
            if best < 0:
                continue
            for u in adj[v]:
                cnt[u][a] -= 1
                if cnt[u][a] == 0:
                    del cnt[u][a]
                cnt[u][best] = cnt[u].get(best, 0) + 1
            h[a] += dha
            h[best] += best_dhb
            k[a] -= 1
            k[best] += 1
            part[v] = best
            cost += best_d
            moved += 1
        if not moved:
            break
    return cost


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
    for l in range(len(levels) - 1, -1, -1):
        if l < len(levels) - 1:
            part = [part[cmaps[l][v]] for v in range(len(levels[l][0]))]
        adj, ew, vw = levels[l]
        pw = [0] * n_parts
        for v in range(len(adj)):
            pw[part[v]] += vw[v]
        refine_cut(adj, ew, vw, part, pw, cap)
    cost = refine_cost(adj0, ew0, part, n_parts, cap)
    members = {}
    for v in range(n):
        members.setdefault(part[v], []).append(v)
    cores = sorted(members.values(), key=lambda c: c[0])
    core_ptr = np.zeros(len(cores) + 1, dtype=np.int32)
    core_ptr[1:] = np.cumsum([len(c) for c in cores])
    core_vtx = np.concatenate([np.array(c, dtype=np.int32) for c in cores])
    return core_ptr, core_vtx, int(cost)


def partition_update(row_ptr, col, cap: int, prev_core_ptr, prev_core_vtx):
    """The previous cores carried to a new graph on the same vertices and improved by step 5
    alone (on-the-fly update between MD steps): (core_ptr, core_vertices, cost)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = len(row_ptr) - 1
    adj0, ew0 = common_neighbour_weights(row_ptr, col)
    n_parts = len(prev_core_ptr) - 1
    part = [-1] * n
    for p in range(n_parts):
        for i in range(prev_core_ptr[p], prev_core_ptr[p + 1]):
            part[int(prev_core_vtx[i])] = p
    cost = refine_cost(adj0, ew0, part, n_parts, cap)
    members = {}
    for v in range(n):
        members.setdefault(part[v], []).append(v)
    cores = sorted(members.values(), key=lambda c: c[0])
    core_ptr = np.zeros(len(cores) + 1, dtype=np.int32)
    core_ptr[1:] = np.cumsum([len(c) for c in cores])
    core_vtx = np.concatenate([np.array(c, dtype=np.int32) for c in cores])
    return core_ptr, core_vtx, int(cost)
