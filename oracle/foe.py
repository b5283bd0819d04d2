"""Finite-temperature Fermi-operator expansion on the subgraph partition (oracle).

Eq. 7 writes the density matrix at inverse temperature beta and chemical potential mu as
the Fermi function of H, expanded in Chebyshev polynomials T_n of H; Eq. 4-5 build the
T_n by a linear recurrence and Eq. 6 evaluates the expansion per subgraph: every core
column of D is the matching column of the same polynomial applied to the dense principal
submatrix of its subgraph.  The coefficients are the same for every subgraph.

Readings (the paper leaves these open):
  * spectral map: Ht = (2 H - (e_max + e_min) I) / (e_max - e_min) with the global
    Gershgorin bounds, so every block's spectrum lies in [-1, 1] (Cauchy interlacing);
    energies map back by e(x) = (e_max + e_min)/2 + x (e_max - e_min)/2;
  * coefficients: Chebyshev-Gauss quadrature with K nodes theta_k = pi (k + 1/2) / K,
        c_n = (2 - delta_n0) / K * sum_k f(e(cos theta_k)) cos(n theta_k),
    K = max(4 (M + 1), 1024) unless given; f(e) = 1 / (1 + exp(beta (e - mu)));
  * recurrence: T_0 = I, T_1 = Ht, T_{n+1} = 2 Ht T_n - T_{n-1}; D_s = sum_{n<=M} c_n T_n;
  * graph and partition: the same as the zero-temperature path (the X0^2 estimate of
    Eq. 2 and block cores; obs. viii allows any graph);
  * mu (when not given): the value for which the summed core traces of the blocks,
    sum_n c_n(mu) t_n with t_n = sum_s sum_{j < k_s} T_n[s][j, j], equal n_occ;
    found by a bracketing root finder on [e_min, e_max].

Pins (tests): the coefficient rule reproduces a polynomial's Chebyshev coefficients exactly
and those of exp(x) in closed form (modified Bessel functions); one subgraph holding every
vertex equals V f(lambda) V^T from the eigensolver within the coefficient tail; a diagonal H
gives f(h_ii); the partitioned result equals the whole-matrix column-masked recurrence
(Eq. 4-6); the solved mu reproduces n_occ and lies in the gap at large beta.
"""
import numpy as np
from scipy.optimize import brentq
from scipy.special import expit

from .bounds import gershgorin, x0_values
from .graph import graph_x2
from .partition import partition
from .sp2 import gather


def default_nodes(order: int) -> int:
    return max(4 * (order + 1), 1024)


def chebyshev_coefficients(g, order: int, n_nodes: int | None = None) -> np.ndarray:
    """c_0 .. c_order of g on [-1, 1] by K-node Chebyshev-Gauss quadrature."""
    K = default_nodes(order) if n_nodes is None else int(n_nodes)
    theta = np.pi * (np.arange(K) + 0.5) / K
    gx = g(np.cos(theta))
    n = np.arange(order + 1)
    c = (np.cos(np.outer(n, theta)) @ gx) * (2.0 / K)
    c[0] *= 0.5
    return c


def fermi(e, beta: float, mu: float):
    return expit(-beta * (np.asarray(e, dtype=np.float64) - mu))


def fermi_coefficients(emin, emax, beta, mu, order, n_nodes=None) -> np.ndarray:
    mid, half = 0.5 * (emax + emin), 0.5 * (emax - emin)
    return chebyshev_coefficients(lambda x: fermi(mid + half * x, beta, mu), order, n_nodes)


def ht_block(H_col, H_val, s, emin, emax) -> np.ndarray:
    """Dense principal submatrix of Ht = (2 H - (e_max + e_min) I)/(e_max - e_min)."""
    h = gather(H_col, H_val, s)
    n = h.shape[0]
    return (2.0 * h - (emax + emin) * np.eye(n)) / (emax - emin)


def chebyshev_terms(ht: np.ndarray, order: int):
    """Yield T_0 .. T_order of the block (the recurrence of Eq. 5, dense)."""
    n = ht.shape[0]
    t0 = np.eye(n)
    yield t0
    if order == 0:
        return
    t1 = ht.copy()
    yield t1
    for _ in range(order - 1):
        t2 = 2.0 * (ht @ t1) - t0
        yield t2
        t0, t1 = t1, t2


def foe_block(ht: np.ndarray, coeffs) -> np.ndarray:
    """sum_n c_n T_n(ht)."""
    D = np.zeros_like(ht)
    for c, t in zip(coeffs, chebyshev_terms(ht, len(coeffs) - 1)):
        D += c * t
    return D


def core_traces(ht: np.ndarray, k: int, order: int) -> np.ndarray:
    """t_n = sum_{j < k} T_n[j, j] for n = 0 .. order."""
    return np.array([np.trace(t[:k, :k]) for t in chebyshev_terms(ht, order)])


def solve_mu(traces, emin, emax, beta, order, n_occ, n_nodes=None) -> float:
    """mu with sum_n c_n(mu) t_n = n_occ (the summed core traces)."""
    def excess(mu):
        return float(fermi_coefficients(emin, emax, beta, mu, order, n_nodes) @ traces) - n_occ
    return brentq(excess, emin, emax, xtol=1e-14, rtol=4 * np.finfo(float).eps, maxiter=500)


def foe_partitioned(H_col, H_val, tau, core_size, beta, order, mu=None, n_occ=None,
                    n_nodes=None, subgraphs=None, method="block"):
    """Core columns of the partitioned Fermi-operator expansion.

    Returns (cols, info): cols maps every core vertex i of the computed subgraphs to
    (rows, values) of column i of D; info holds mu, the coefficients, the bounds, the
    partition and the summed core traces t_n (only when every subgraph is computed).
    With ``subgraphs`` (a list of subgraph indices; needs ``mu``) only those are computed."""
    emin, emax = gershgorin(H_col, H_val)
    rp, col = graph_x2(H_col, H_val, tau, emin, emax)
    core_ptr, _, sub_ptr, sub_idx = partition(rp, col, core_size, method)
    n_sub = len(core_ptr) - 1
    core_counts = np.diff(core_ptr)
    picks = range(n_sub) if subgraphs is None else subgraphs
    blocks = {s: ht_block(H_col, H_val, sub_idx[sub_ptr[s]:sub_ptr[s + 1]], emin, emax)
              for s in picks}
    traces = None
    if subgraphs is None:
        traces = np.zeros(order + 1)
        for s in range(n_sub):
            traces += core_traces(blocks[s], int(core_counts[s]), order)
    if mu is None:
        if traces is None or n_occ is None:
            raise ValueError("solving for mu needs n_occ and every subgraph")
        mu = solve_mu(traces, emin, emax, beta, order, n_occ, n_nodes)
    coeffs = fermi_coefficients(emin, emax, beta, mu, order, n_nodes)
    cols = {}
    for s in picks:
        D = foe_block(blocks[s], coeffs)
        rows = sub_idx[sub_ptr[s]:sub_ptr[s + 1]]
        for j in range(int(core_counts[s])):
            cols[int(rows[j])] = (rows, D[:, j].copy())
    info = {"mu": mu, "coeffs": coeffs, "emin": emin, "emax": emax, "traces": traces,
            "core_ptr": core_ptr, "sub_ptr": sub_ptr, "sub_idx": sub_idx}
    return cols, info


def columns_to_ell(cols, N: int, width: int):
    """Column-ELL arrays (row i = column i of D, rows ascending, padding -1 / 0)."""
    D_col = np.full((N, width), -1, dtype=np.int32)
    D_val = np.zeros((N, width))
    for i, (rows, vals) in cols.items():
        order = np.argsort(rows, kind="stable")
        D_col[i, :len(rows)] = rows[order]
        D_val[i, :len(rows)] = vals[order]
    return D_col, D_val
