"""Partitioned SP2 density matrix: the parity reference (oracle).

The method (Eq. 6, obs. ix-x and the SP2 paragraph after Eq. 7): every subgraph
expansion applies the same recursive sequence of second-order maps
X <- X^2 or X <- 2X - X^2 to its own dense principal submatrix x[s] of X0, and the
core columns of the results are assembled, column by column, into D = P_tau(X0)
(obs. i: the assembly is not symmetric).  The branch of each step is chosen
globally from the traces summed over every subgraph's core columns, so that the
assembled D carries the requested occupation.

Readings taken where the paper is silent (it cites SP2 without restating it):
  * start X0 = (e_max I - H)/(e_max - e_min) with global Gershgorin bounds;
  * t1 = sum over subgraphs s, over core rows j of x_s[j, j]; t2 the same over
    S_s = x_s^2; both summed sequentially, s outer, j inner;
  * stop rule: e = |t1 - t2| <= idem_tol ends the loop before the update, so D is
    the current X (its square only served the test);
  * branch: b = 0 (X <- X^2) if |t2 - n_occ| < |2 t1 - t2 - n_occ|, else
    b = 1 (X <- 2X - X^2); a tie goes to 2X - X^2;
  * replay: a given branch sequence is applied step by step and the loop stops
    when it is exhausted (the paper's pre-determined sequence, MD section);
  * optional trailing McWeeny steps X <- 3X^2 - 2X^3.
The whole-matrix thresholded SP2 (the paper's thresholded sparse-algebra
comparison, Fig. 3) uses the same rules on the full matrix and zeroes every entry
of magnitude below tau after each update.

Pins (tests): one subgraph holding every vertex equals dense SP2 and the
eigensolver's projector; a diagonal H gives the exact occupation projector;
Eq. 6 against the whole-matrix masked polynomial; Tr D = n_occ at convergence.
"""
import numpy as np

from .bounds import gershgorin, x0_values, ell_to_dense
from .graph import graph_x2
from .partition import partition


def default_idem_tol(N: int) -> float:
    return 1e-10 * N / 1024.0


def gather(H_col: np.ndarray, x0: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Dense principal submatrix x0[s, s] from the ELL entries of X0."""
    N = H_col.shape[0]
    n = len(s)
    loc = np.full(N + 1, -1, dtype=np.int64)
    loc[s] = np.arange(n)
    hc = np.where(H_col[s] >= 0, H_col[s], N)
    lj = loc[hc]
    x = np.zeros((n, n))
    a, t = np.nonzero(lj >= 0)
    x[a, lj[a, t]] = x0[s][a, t]
    return x


def sp2_partitioned(blocks, core_counts, n_occ, idem_tol, max_iter=100, branch_in=None,
                    n_refine=0, keep_tape=False, consume=False, low_memory=False):
    """Run the shared SP2 sequence on every block (list of dense symmetric arrays,
    core rows first).  Returns (blocks, info).  With ``consume`` the given list is emptied
    and its arrays are used directly (they are never written), to bound memory.  With
    ``low_memory`` the traces of X^2 are taken from its core diagonal alone (a dot product per
    entry) and X^2 is recomputed block by block for the update, so one copy of the blocks
    is held; the diagonal dot products may round differently from the full product, which
    only matters at the last bit of the traces."""
    if consume:
        xs = list(blocks)
        blocks.clear()
    else:
        xs = [np.array(b, dtype=np.float64, copy=True) for b in blocks]
    branches, margins, traces = [], [], []
    tape = [list(xs)] if keep_tape else None
    converged = False
    last_e = np.inf
    it = 0
    while True:
        if low_memory:
            # only the core diagonals of the squares are needed before the branch is known;
            # the squares are recomputed for the update, one block at a time
            S = [np.einsum("ij,ji->i", x[:k], x[:, :k]) for x, k in zip(xs, core_counts)]
        else:
            S = [x @ x for x in xs]
        t1 = 0.0
        t2 = 0.0
        for x, s, k in zip(xs, S, core_counts):
            for j in range(k):
                t1 += x[j, j]
                t2 += s[j] if low_memory else s[j, j]
        e = abs(t1 - t2)
        traces.append((t1, t2))
        last_e = e
        if branch_in is None:
            if e <= idem_tol:
                converged = True
                break
            if it >= max_iter:
                break
            d_sq = abs(t2 - n_occ)
            d_lin = abs(2.0 * t1 - t2 - n_occ)
            b = 0 if d_sq < d_lin else 1
            margins.append(abs(d_sq - d_lin))
        else:
            if it >= len(branch_in):
                converged = e <= idem_tol
                break
            b = int(branch_in[it])
            d_sq = abs(t2 - n_occ)
            d_lin = abs(2.0 * t1 - t2 - n_occ)
            margins.append(abs(d_sq - d_lin))
        branches.append(b)
        if low_memory:
            for q in range(len(xs)):
                sq = xs[q] @ xs[q]
                xs[q] = sq if b == 0 else np.subtract(2.0 * xs[q], sq, out=sq)
        else:
            if b == 1:
                for x, s in zip(xs, S):
                    np.subtract(2.0 * x, s, out=s)   # s <- 2x - s, the same rounding as 2x - s
            xs = S
        if keep_tape:
            tape.append(list(xs))
        it += 1
    for _ in range(n_refine):
        xs = [3.0 * (x @ x) - 2.0 * ((x @ x) @ x) for x in xs]
    info = {"iters": len(branches), "converged": converged, "branch": branches,
            "traces": traces, "margins": margins,
            "min_margin": float(min(margins)) if margins else np.inf,
            "idem": last_e, "tape": tape}
    return xs, info


def scatter_columns(xs, sub_ptr, sub_idx, core_counts, N: int, width: int | None = None):
    """Column-ELL D: row i of the arrays holds column i of D, entries sorted by global
    row index (padding col = -1, val = 0).  Column i comes from the column of i in its
    subgraph's block."""
    n_sub = len(sub_ptr) - 1
    if width is None:
        width = int(np.max(np.diff(sub_ptr))) if n_sub else 0
    D_col = np.full((N, width), -1, dtype=np.int32)
    D_val = np.zeros((N, width))
    for s in range(n_sub):
        idx = sub_idx[sub_ptr[s]:sub_ptr[s + 1]]
        order = np.argsort(idx, kind="stable")
        n = len(idx)
        for j in range(core_counts[s]):
            i = idx[j]
            D_col[i, :n] = idx[order]
            D_val[i, :n] = xs[s][order, j]
    return D_col, D_val


def density_partitioned(H_col, H_val, n_occ, tau, core_size, method="block", idem_tol=None,
                        max_iter=100, branch_in=None, n_refine=0, graph=None, keep_tape=False,
                        low_memory=False):
    """The whole partitioned method: bounds, X2 graph, partition, gather, SP2, scatter."""
    N = H_col.shape[0]
    if idem_tol is None:
        idem_tol = default_idem_tol(N)
    emin, emax = gershgorin(H_col, H_val)
    if graph is None:
        graph = graph_x2(H_col, H_val, tau, emin, emax)
    row_ptr, col = graph
    core_ptr, core_vertices, sub_ptr, sub_idx = partition(row_ptr, col, core_size, method)
    x0 = x0_values(H_col, H_val, emin, emax)
    subs = [sub_idx[sub_ptr[s]:sub_ptr[s + 1]] for s in range(len(sub_ptr) - 1)]
    blocks = [gather(H_col, x0, s) for s in subs]
    core_counts = np.diff(core_ptr)
    blocks0 = list(blocks) if keep_tape else None
    xs, info = sp2_partitioned(blocks, core_counts, n_occ, idem_tol, max_iter, branch_in,
                               n_refine, keep_tape, consume=True, low_memory=low_memory)
    D_col, D_val = scatter_columns(xs, sub_ptr, sub_idx, core_counts, N)
    info.update(emin=emin, emax=emax, row_ptr=row_ptr, col=col, core_ptr=core_ptr,
                core_vertices=core_vertices, sub_ptr=sub_ptr, sub_idx=sub_idx,
                trace=float(sum(D_val[i][D_col[i] == i].sum() for i in range(N))),
                blocks0=blocks0)
    return D_col, D_val, info


def sp2_dense(X0: np.ndarray, n_occ, idem_tol, max_iter=100, tau=0.0, stall_stop=False):
    """Whole-matrix SP2 on a dense X0; with tau > 0 every entry of magnitude below tau
    is zeroed after each update (the thresholded sparse-algebra expansion).  With
    ``stall_stop`` the expansion also ends once e_n = |t1 - t2| stops decreasing (after at least
    ten steps, e_n > e_{n-2}): thresholding perturbs every step, so e_n settles at a floor
    above a tight idem_tol, as rounding does for a low-precision expansion."""
    N = X0.shape[0]
    x = np.array(X0, dtype=np.float64, copy=True)
    branches, traces = [], []
    converged = False
    stalled = False
    for it in range(max_iter + 1):
        s = x @ x
        t1 = 0.0
        t2 = 0.0
        for j in range(N):
            t1 += x[j, j]
            t2 += s[j, j]
        traces.append((t1, t2))
        if abs(t1 - t2) <= idem_tol:
            converged = True
            break
        if stall_stop and it >= 9 and abs(t1 - t2) > abs(traces[-3][0] - traces[-3][1]):
            stalled = True
            break
        if it == max_iter:
            break
        b = 0 if abs(t2 - n_occ) < abs(2.0 * t1 - t2 - n_occ) else 1
        branches.append(b)
        x = s if b == 0 else 2.0 * x - s
        if tau > 0.0:
            x[np.abs(x) < tau] = 0.0
    return x, {"iters": len(branches), "converged": converged, "stalled": stalled,
               "branch": branches, "traces": traces}


def x0_dense(H_col, H_val, emin=None, emax=None):
    if emin is None or emax is None:
        emin, emax = gershgorin(H_col, H_val)
    return ell_to_dense(H_col, x0_values(H_col, H_val, emin, emax))
