"""Eq. 3-6: thresholded whole-matrix polynomial vs subgraph polynomials (oracle).

Eq. 3 thresholds a matrix on the edges of a graph, Eq. 4 defines the thresholded
polynomial, Eq. 5 evaluates it by a linear recurrence in which every product with X
is thresholded, and Eq. 6 states that column i of the result equals the column of i
in the dense polynomial of the principal submatrix of the subgraph of i.  With
communities (obs. vi) the column mask of column i is the vertex set of the subgraph
of the core holding i; every such mask contains i itself.

These functions evaluate both sides independently: the left side on the full N x N
matrix with a column mask applied after every product, the right side per subgraph
on small dense blocks.  They are used only to pin the partitioned SP2 oracle.
"""
import numpy as np


def column_mask(N: int, sub_ptr, sub_idx, core_vertices_per_sub) -> np.ndarray:
    """R[r, i] = True iff vertex r belongs to the subgraph of the core holding i."""
    R = np.zeros((N, N), dtype=bool)
    for s in range(len(sub_ptr) - 1):
        rows = sub_idx[sub_ptr[s]:sub_ptr[s + 1]]
        for i in core_vertices_per_sub[s]:
            R[rows, i] = True
    return R


def sp2_power_coefficients(branches) -> list:
    """Ascending power coefficients (exact integers) of the composed SP2 map for a
    branch sequence: p <- p^2 (b = 0) or p <- 2p - p^2 (b = 1), starting at p = x."""
    p = [0, 1]
    for b in branches:
        sq = [0] * (2 * len(p) - 1)
        for i, a in enumerate(p):
            if a:
                for j, c in enumerate(p):
                    sq[i + j] += a * c
        if b == 0:
            p = sq
        else:
            p = [2 * (p[k] if k < len(p) else 0) - sq[k] for k in range(len(sq))]
    while len(p) > 1 and p[-1] == 0:
        p.pop()
    return p


def masked_horner(X: np.ndarray, coeffs, R: np.ndarray) -> np.ndarray:
    """Eq. 5 in Horner form: B <- c_M I; B <- floor(X B)_R + c_k I for k = M-1 .. 0."""
    N = X.shape[0]
    I = np.eye(N)
    B = float(coeffs[-1]) * I
    for c in reversed(coeffs[:-1]):
        B = np.where(R, X @ B, 0.0) + float(c) * I
    return B


def dense_horner(x: np.ndarray, coeffs) -> np.ndarray:
    n = x.shape[0]
    I = np.eye(n)
    B = float(coeffs[-1]) * I
    for c in reversed(coeffs[:-1]):
        B = x @ B + float(c) * I
    return B


def masked_chebyshev(X: np.ndarray, coeffs, R: np.ndarray) -> np.ndarray:
    """Sum_n c_n T_n with T_0 = I, T_1 = floor(X T_0)_R,
    T_n = 2 floor(X T_{n-1})_R - T_{n-2} (Eq. 4 with the Chebyshev recurrence)."""
    N = X.shape[0]
    T0 = np.eye(N)
    P = coeffs[0] * T0
    if len(coeffs) == 1:
        return P
    T1 = np.where(R, X @ T0, 0.0)
    P = P + coeffs[1] * T1
    for c in coeffs[2:]:
        T2 = 2.0 * np.where(R, X @ T1, 0.0) - T0
        P = P + c * T2
        T0, T1 = T1, T2
    return P


def dense_chebyshev(x: np.ndarray, coeffs) -> np.ndarray:
    n = x.shape[0]
    T0 = np.eye(n)
    P = coeffs[0] * T0
    if len(coeffs) == 1:
        return P
    T1 = x.copy()
    P = P + coeffs[1] * T1
    for c in coeffs[2:]:
        T2 = 2.0 * (x @ T1) - T0
        P = P + c * T2
        T0, T1 = T1, T2
    return P


def assemble_columns(N: int, blocks, sub_ptr, sub_idx, core_counts) -> np.ndarray:
    """Dense N x N matrix whose column i is the column of i in its subgraph block."""
    out = np.zeros((N, N))
    for s, blk in enumerate(blocks):
        rows = sub_idx[sub_ptr[s]:sub_ptr[s + 1]]
        for j in range(core_counts[s]):
            out[rows, rows[j]] = blk[:, j]
    return out
