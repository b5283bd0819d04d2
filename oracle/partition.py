"""Cores (communities) and core+halo subgraphs (oracle).

Eq. 6: for a core vertex i, the subgraph s^i holds i and every vertex directly
connected to i in S (its halo); column i of the thresholded polynomial equals the
column of i in the dense polynomial of the principal submatrix x[s^i].  Obs. vi lets
a core be a set of vertices (a community): the subgraph of a core C is C together
with every vertex outside C adjacent to some vertex of C.

Layout (bit-exact on the GPU):
  core_ptr  int32 [n_sub + 1]   core c is vertices core_ptr[c] .. core_ptr[c+1]-1
  sub_ptr   int32 [n_sub + 1]   offsets into sub_idx
  sub_idx   int32 [sum n_s]     per subgraph: core vertices ascending, then halo ascending

Partitions: BLOCK = contiguous runs of ``core_size`` vertices in vertex order (the
generator emits spatially sorted vertices, so blocks are compact communities);
BFS = the same blocks cut from a deterministic breadth-first (Cuthill-McKee) order;
MULTILEVEL = communities of at most ``core_size`` vertices (oracle/multilevel.py).
"""
import numpy as np


def block_cores(N: int, core_size: int) -> np.ndarray:
    """core_ptr of contiguous blocks (the last one may be short)."""
    n_sub = (N + core_size - 1) // core_size
    ptr = np.minimum(np.arange(n_sub + 1, dtype=np.int64) * core_size, N)
    return ptr.astype(np.int32)


def bfs_order(row_ptr: np.ndarray, col: np.ndarray) -> np.ndarray:
    """Cuthill-McKee order: repeatedly start at the lowest-numbered unvisited vertex
    of minimum degree, visit neighbours in ascending (degree, index) order."""
    N = len(row_ptr) - 1
    deg = np.diff(row_ptr)
    seen = np.zeros(N, dtype=bool)
    order = []
    by_deg = np.lexsort((np.arange(N), deg))
    for start in by_deg:
        if seen[start]:
            continue
        seen[start] = True
        queue = [int(start)]
        head = 0
        while head < len(queue):
            v = queue[head]
            head += 1
            order.append(v)
            nb = col[row_ptr[v]:row_ptr[v + 1]]
            nb = nb[~seen[nb]]
            nb = nb[np.lexsort((nb, deg[nb]))]
            seen[nb] = True
            queue.extend(int(x) for x in nb)
    return np.asarray(order, dtype=np.int32)


def core_lists(N: int, core_size: int, order: np.ndarray | None = None):
    """Vertex lists of the cores, each ascending."""
    ptr = block_cores(N, core_size)
    seq = np.arange(N, dtype=np.int32) if order is None else np.asarray(order, dtype=np.int32)
    return ptr, [np.sort(seq[ptr[c]:ptr[c + 1]]) for c in range(len(ptr) - 1)]


def halo_subgraphs(row_ptr: np.ndarray, col: np.ndarray, cores):
    """sub_ptr, sub_idx for the given core vertex lists (each ascending)."""
    subs = []
    for C in cores:
        nb = np.concatenate([col[row_ptr[v]:row_ptr[v + 1]] for v in C]) if len(C) else \
            np.zeros(0, dtype=np.int32)
        halo = np.setdiff1d(np.unique(nb), C)
        subs.append(np.concatenate([C, halo]).astype(np.int32))
    sub_ptr = np.zeros(len(subs) + 1, dtype=np.int64)
    np.cumsum([len(s) for s in subs], out=sub_ptr[1:])
    sub_idx = np.concatenate(subs) if subs else np.zeros(0, dtype=np.int32)
    return sub_ptr.astype(np.int32), sub_idx.astype(np.int32)


def partition(row_ptr, col, core_size: int, method: str = "block"):
    """(core_ptr, core_vertices, sub_ptr, sub_idx).  core_vertices lists each core's
    vertices in the same order as the first entries of its subgraph."""
    N = len(row_ptr) - 1
    if method == "multilevel":
        from oracle.multilevel import partition_multilevel
        ptr, cv, _ = partition_multilevel(row_ptr, col, core_size)
        cores = [cv[ptr[c]:ptr[c + 1]] for c in range(len(ptr) - 1)]
        sub_ptr, sub_idx = halo_subgraphs(row_ptr, col, cores)
        return ptr, cv, sub_ptr, sub_idx
    order = None if method == "block" else bfs_order(row_ptr, col)
    ptr, cores = core_lists(N, core_size, order)
    sub_ptr, sub_idx = halo_subgraphs(row_ptr, col, cores)
    core_vertices = np.concatenate(cores).astype(np.int32) if cores else np.zeros(0, np.int32)
    return ptr, core_vertices, sub_ptr, sub_idx
