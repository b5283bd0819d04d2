"""Spectral bounds and the SP2 start map (oracle).

SP2 (the recursive zero-temperature expansion the paper uses, Results section, the
paragraph after Eq. 7) starts from X0 = (e_max I - H) / (e_max - e_min), which maps
the spectrum of H into [0, 1] with occupied states near 1.  The bounds are the
Gershgorin discs of H.  Because the same global bounds are used for every principal
submatrix, every subgraph expansion starts from exactly the entries of X0
(Cauchy interlacing keeps each submatrix spectrum inside [e_min, e_max]).

Canonical evaluation (so that the GPU reproduces every bit): the off-diagonal
absolute row sum is accumulated sequentially in ascending column order, the
Gershgorin ends are diag - R and diag + R, and x0 is one IEEE subtraction followed
by one IEEE division by (e_max - e_min).

Pins: spectrum of H inside [e_min, e_max] (eigensolver); a diagonal H gives its
own min / max; a hand 3x3 example.
"""
import numpy as np


def gershgorin(H_col: np.ndarray, H_val: np.ndarray):
    """(e_min, e_max) of the ELL matrix: min_i (h_ii - R_i), max_i (h_ii + R_i),
    R_i = sum_{j != i} |h_ij| in ascending column order."""
    N, W = H_col.shape
    rows = np.arange(N)
    acc = np.zeros(N)
    diag = np.zeros(N)
    for t in range(W):
        c = H_col[:, t]
        on = c == rows
        off = (c >= 0) & ~on
        acc = acc + np.where(off, np.abs(H_val[:, t]), 0.0)
        diag = np.where(on, H_val[:, t], diag)
    return float(np.min(diag - acc)), float(np.max(diag + acc))


def x0_values(H_col: np.ndarray, H_val: np.ndarray, emin: float, emax: float) -> np.ndarray:
    """Entries of X0 = (e_max I - H) / (e_max - e_min) on H's ELL pattern."""
    N = H_col.shape[0]
    rows = np.arange(N)[:, None]
    denom = emax - emin
    num = np.where(H_col == rows, emax - H_val, 0.0 - H_val)
    return np.where(H_col >= 0, num / denom, 0.0)


def ell_to_dense(col: np.ndarray, val: np.ndarray, n_cols: int | None = None) -> np.ndarray:
    """Dense matrix from row-major ELL arrays (padding col = -1 ignored)."""
    N, W = col.shape
    n_cols = N if n_cols is None else n_cols
    A = np.zeros((N, n_cols))
    r, t = np.nonzero(col >= 0)
    A[r, col[r, t]] = val[r, t]
    return A
