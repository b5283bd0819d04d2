"""Data-dependency graphs S (oracle).

Eq. 2 defines S_tau: a vertex per row of X and an edge (i, j) when the magnitude of
some term T^(n)(X)_ij of the expansion reaches tau (the printed inequality lacks the
absolute value; the text says "magnitude", so |.| >= tau is used).  Obs. viii allows
any graph, and the paper estimates S from an approximate prior density matrix
(paragraph after Eq. 7) or, in MD, from Eq. 8.

Graph rules implemented here (all include every self-loop, because T^(0) = I puts
vertex i in its own subgraph, Eqs. 5-6, and all are symmetrised by union):
  X2        S = {(i, j) : j two hops from i in pattern(H), |(X0^2)_ij| >= tau}
  PATTERN   S = {(i, j) : |A_ij| >= tau}
  DPREV     S = {|D_prev_ij| >= tau_d}  U  X2(H, tau)          (adaptive MD graph)
  DPREV_SYMBOLIC   Eq. 8 with eps = 0: paths of length two in
            pattern(|D_prev| >= tau_d) U pattern(H)
  RCUT      the divide-and-conquer comparison (Fig. 5): orbitals i, j adjacent when the
            minimum-image distance of their sites is below r_cut (periodic cube of edge L).
            Canonical distance: per axis d = x_j - x_i, d = d - L * rint(d / L); r2 summed
            x, y, z in that order; edge iff r2 < r_cut * r_cut (every operation rounded
            separately, so the GPU reproduces it bit for bit).

Canonical X0^2 entry (bit-exact on the GPU): (X0^2)_ij = sum over k in
row_i intersect row_j of x0_ik * x0_kj, accumulated sequentially in ascending k,
every product and sum rounded separately (no fused multiply-add).  Adding the
zero products of a dense ascending-k sum leaves every partial sum unchanged, so
the dense and sparse forms agree bit for bit; the tests pin one to the other and
both to a pure-Python triple loop.
"""
import numpy as np

from .bounds import gershgorin, x0_values


def csr_from_edges(N: int, rows: np.ndarray, cols: np.ndarray):
    """Sorted, duplicate-free CSR (int32 row_ptr [N+1], int32 col) of an edge list."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = np.unique(rows * N + cols)
    r = key // N
    c = key % N
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=N), out=row_ptr[1:])
    return row_ptr.astype(np.int32), c.astype(np.int32)


def symmetrise(N: int, row_ptr: np.ndarray, col: np.ndarray):
    """Union of S and its transpose, with every self-loop added."""
    r = np.repeat(np.arange(N), np.diff(row_ptr))
    rows = np.concatenate([r, col, np.arange(N)])
    cols = np.concatenate([col, r, np.arange(N)])
    return csr_from_edges(N, rows, cols)


def x2_rows(H_col: np.ndarray, x0: np.ndarray, rows: np.ndarray, chunk: int = 128):
    """Canonical (X0^2)_ij for every j two hops from each i in ``rows``.

    Yields (i_block, acc, touched): acc[r, j] is the sequential ascending-k sum for
    row rows[r] (a dense row of length N, plus one dummy column for padding), and
    touched marks the two-hop candidates.
    """
    N, W = H_col.shape
    hc = np.where(H_col >= 0, H_col, N)          # padding -> dummy column N
    for s in range(0, len(rows), chunk):
        blk = np.asarray(rows[s:s + chunk])
        m = len(blk)
        acc = np.zeros((m, N + 1))
        touched = np.zeros((m, N + 1), dtype=bool)
        rr = np.arange(m)[:, None]
        for t in range(W):
            k = H_col[blk, t]
            ok = k >= 0
            if not ok.any():
                continue
            kk = np.where(ok, k, 0)
            # row k of X0 scaled by x0_ik, added at columns of row k (unique per row)
            prod = x0[blk, t][:, None] * x0[kk]
            cols = np.where(ok[:, None], hc[kk], N)
            acc[rr, cols] = acc[rr, cols] + prod
            touched[rr, cols] = True
        yield blk, acc[:, :N], touched[:, :N]


def graph_x2(H_col, H_val, tau, emin=None, emax=None, rows=None):
    """X2 graph (CSR).  With ``rows`` given, only those rows' edge lists are
    returned, as a list of int32 arrays (used to sample large systems)."""
    if emin is None or emax is None:
        emin, emax = gershgorin(H_col, H_val)
    x0 = x0_values(H_col, H_val, emin, emax)
    N = H_col.shape[0]
    want = np.arange(N) if rows is None else np.asarray(rows)
    er, ec = [], []
    lists = []
    for blk, acc, touched in x2_rows(H_col, x0, want):
        keep = touched & (np.abs(acc) >= tau)
        keep[np.arange(len(blk)), blk] = True
        rr, cc = np.nonzero(keep)
        if rows is None:
            er.append(blk[rr])
            ec.append(cc)
        else:
            for r in range(len(blk)):
                lists.append(np.nonzero(keep[r])[0].astype(np.int32))
    if rows is not None:
        return lists
    rp, cl = csr_from_edges(N, np.concatenate(er), np.concatenate(ec))
    return symmetrise(N, rp, cl)


def x2_dense_canonical(X0: np.ndarray) -> np.ndarray:
    """Dense X0 @ X0 summed sequentially in ascending k with separate rounding."""
    acc = np.zeros_like(X0)
    for k in range(X0.shape[0]):
        acc = acc + np.multiply.outer(X0[:, k], X0[k, :])
    return acc


def pattern_matrix(col: np.ndarray, n_cols: int) -> np.ndarray:
    N = col.shape[0]
    P = np.zeros((N, n_cols), dtype=bool)
    r, t = np.nonzero(col >= 0)
    P[r, col[r, t]] = True
    return P


def graph_x2_dense(H_col, H_val, tau, emin=None, emax=None):
    """Dense form of the X2 rule (small N): the brute-force counterpart of graph_x2."""
    from .bounds import ell_to_dense
    if emin is None or emax is None:
        emin, emax = gershgorin(H_col, H_val)
    N = H_col.shape[0]
    X0 = ell_to_dense(H_col, x0_values(H_col, H_val, emin, emax))
    P = pattern_matrix(H_col, N).astype(np.int64)
    two_hop = (P @ P) > 0
    keep = two_hop & (np.abs(x2_dense_canonical(X0)) >= tau)
    keep |= np.eye(N, dtype=bool)
    keep |= keep.T
    r, c = np.nonzero(keep)
    return csr_from_edges(N, r, c)


def graph_pattern(A_col, A_val, tau):
    """PATTERN rule: |A_ij| >= tau, plus self-loops, symmetrised."""
    N = A_col.shape[0]
    r, t = np.nonzero((A_col >= 0) & (np.abs(A_val) >= tau))
    rp, cl = csr_from_edges(N, r, A_col[r, t])
    return symmetrise(N, rp, cl)


def graph_dprev(H_col, H_val, Dp_col, Dp_val, tau, tau_d, emin=None, emax=None):
    """Adaptive MD graph: entries of the previous D (column-ELL: row i of the arrays
    is column i of D) with |D_ri| >= tau_d, united with the X2 graph of the new H."""
    N = H_col.shape[0]
    rp, cl = graph_x2(H_col, H_val, tau, emin, emax)
    r0 = np.repeat(np.arange(N), np.diff(rp))
    i, t = np.nonzero((Dp_col >= 0) & (np.abs(Dp_val) >= tau_d))
    rows = np.concatenate([r0, Dp_col[i, t]])
    cols = np.concatenate([cl, i])
    rp2, cl2 = csr_from_edges(N, rows, cols)
    return symmetrise(N, rp2, cl2)


def graph_dprev_symbolic(H_col, Dp_col, Dp_val, tau_d):
    """Eq. 8 with eps = 0 (symbolic square): paths of length two in the union of
    pattern(H) and the previous D thresholded at tau_d.  Dense; small N only."""
    N = H_col.shape[0]
    P = pattern_matrix(H_col, N)
    i, t = np.nonzero((Dp_col >= 0) & (np.abs(Dp_val) >= tau_d))
    P[Dp_col[i, t], i] = True
    P |= np.eye(N, dtype=bool)
    P |= P.T
    Pi = P.astype(np.int64)
    S = (Pi @ Pi) > 0
    r, c = np.nonzero(S | S.T)
    return csr_from_edges(N, r, c)


def graph_rcut(pos: np.ndarray, L: float, r_cut: float, orbs_per_site: int = 2):
    """RCUT graph over orbitals (orbital o of site a is a * orbs_per_site + o)."""
    n_sites = pos.shape[0]
    m = int(orbs_per_site)
    rows, cols = [], []
    rc2 = r_cut * r_cut
    for a in range(n_sites):
        d = pos - pos[a]
        d = d - L * np.rint(d / L)
        r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        nb = np.nonzero(r2 < rc2)[0]
        for o in range(m):
            i = a * m + o
            for q in range(m):
                rows.append(np.full(len(nb), i))
                cols.append(nb * m + q)
    N = n_sites * m
    return csr_from_edges(N, np.concatenate(rows), np.concatenate(cols))
