"""Pins for the finite-temperature Fermi-operator expansion oracle: closed-form Chebyshev
coefficients, the eigensolver, a diagonal H, the Eq. 4-6 equivalence and the occupation.
CPU only."""
import numpy as np
import pytest
from scipy.special import iv

from synth import make_model
from oracle.bounds import gershgorin, ell_to_dense
from oracle.equivalence import column_mask
from oracle.foe import (chebyshev_coefficients, fermi, fermi_coefficients, foe_block,
                        foe_partitioned, columns_to_ell, ht_block)
from oracle.graph import graph_x2
from oracle.partition import partition
from oracle.metrics import column_ell_to_dense


def test_coefficients_of_a_polynomial_are_exact():
    # 2 + T_3(x) = 2 + 4x^3 - 3x
    c = chebyshev_coefficients(lambda x: 2.0 + 4.0 * x**3 - 3.0 * x, 8, n_nodes=64)
    want = np.zeros(9)
    want[0], want[3] = 2.0, 1.0
    assert np.abs(c - want).max() < 1e-14


def test_coefficients_of_exp_are_bessel_values():
    # exp(x) = I_0(1) + 2 sum_{n>=1} I_n(1) T_n(x)
    c = chebyshev_coefficients(np.exp, 12)
    n = np.arange(13)
    want = 2.0 * iv(n, 1.0)
    want[0] = iv(0, 1.0)
    assert np.abs(c - want).max() < 1e-14


def test_fermi_function_limits():
    assert fermi(0.0, 10.0, 0.0) == 0.5
    assert fermi(-5.0, 10.0, 0.0) == pytest.approx(1.0, abs=1e-21)
    assert fermi(5.0, 10.0, 0.0) < 1e-21


def _tail(emin, emax, beta, mu, order):
    c = fermi_coefficients(emin, emax, beta, mu, 4 * order, n_nodes=16 * order)
    return float(np.abs(c[order + 1:]).sum())


def test_one_subgraph_equals_eigensolver():
    m = make_model("tiny48")
    N = m["N"]
    H = ell_to_dense(m["H_col"], m["H_val"])
    beta, order, mu = 4.0, 200, 0.1
    cols, info = foe_partitioned(m["H_col"], m["H_val"], 0.0, N, beta, order, mu=mu)
    assert len(info["core_ptr"]) == 2  # one subgraph holding every vertex
    D = np.zeros((N, N))
    for i, (rows, v) in cols.items():
        D[rows, i] = v
    w, V = np.linalg.eigh(H)
    ref = (V * fermi(w, beta, mu)) @ V.T
    bound = _tail(info["emin"], info["emax"], beta, mu, order) + 1e-13
    assert np.abs(D - ref).max() <= bound
    assert bound < 1e-9


def test_diagonal_hamiltonian_gives_fermi_values():
    h = np.array([-2.0, -0.5, 0.25, 1.0, 3.0])
    N = len(h)
    H_col = np.arange(N, dtype=np.int32)[:, None]
    H_val = h[:, None].copy()
    beta, order, mu = 3.0, 120, 0.0
    cols, info = foe_partitioned(H_col, H_val, 1e-5, 1, beta, order, mu=mu)
    got = np.array([cols[i][1][0] for i in range(N)])
    assert all(len(cols[i][0]) == 1 for i in range(N))
    bound = _tail(info["emin"], info["emax"], beta, mu, order) + 1e-14
    assert np.abs(got - fermi(h, beta, mu)).max() <= bound


def test_partitioned_equals_masked_whole_matrix():
    """Eq. 6: each core column of the subgraph expansions equals the column of the
    whole-matrix Chebyshev recurrence masked to that column's subgraph after every
    product (Eq. 4-5)."""
    m = make_model("small256")
    N = m["N"]
    beta, order, mu, tau, core = 6.0, 40, 0.0, 1e-3, 8
    cols, info = foe_partitioned(m["H_col"], m["H_val"], tau, core, beta, order, mu=mu)
    emin, emax = info["emin"], info["emax"]
    rp, col = graph_x2(m["H_col"], m["H_val"], tau, emin, emax)
    core_ptr, core_vtx, sub_ptr, sub_idx = partition(rp, col, core)
    cores = [core_vtx[core_ptr[s]:core_ptr[s + 1]] for s in range(len(core_ptr) - 1)]
    R = column_mask(N, sub_ptr, sub_idx, cores)
    Ht = (2.0 * ell_to_dense(m["H_col"], m["H_val"]) - (emax + emin) * np.eye(N)) / (emax - emin)
    c = info["coeffs"]
    T0 = np.eye(N)
    T1 = np.where(R, Ht @ T0, 0.0)
    ref = c[0] * T0 + c[1] * T1
    for cn in c[2:]:
        T2 = 2.0 * np.where(R, Ht @ T1, 0.0) - T0
        ref = ref + cn * T2
        T0, T1 = T1, T2
    D = np.zeros((N, N))
    for i, (rows, v) in cols.items():
        D[rows, i] = v
    assert np.abs(D - ref).max() < 1e-12


def test_solved_mu_gives_the_occupation_and_sits_in_the_gap():
    m = make_model("tiny48")
    N, n_occ = m["N"], m["n_occ"]
    H = ell_to_dense(m["H_col"], m["H_val"])
    w = np.linalg.eigvalsh(H)
    beta, order = 8.0, 400
    cols, info = foe_partitioned(m["H_col"], m["H_val"], 0.0, N, beta, order, n_occ=n_occ)
    tr = sum(v[list(rows).index(i)] for i, (rows, v) in cols.items())
    assert abs(tr - n_occ) < 1e-9
    assert w[n_occ - 1] < info["mu"] < w[n_occ]
    # the solved mu reproduces the occupation in the partitioned case too
    m2 = make_model("small256")
    cols2, info2 = foe_partitioned(m2["H_col"], m2["H_val"], 1e-5, 16, 6.0, 60,
                                   n_occ=m2["n_occ"])
    tr2 = sum(v[list(rows).index(i)] for i, (rows, v) in cols2.items())
    assert abs(tr2 - m2["n_occ"]) < 1e-9


def test_columns_to_ell_round_trip():
    m = make_model("small256")
    cols, info = foe_partitioned(m["H_col"], m["H_val"], 1e-5, 16, 6.0, 20, mu=0.0)
    width = int(np.diff(info["sub_ptr"]).max())
    D_col, D_val = columns_to_ell(cols, m["N"], width)
    D = column_ell_to_dense(D_col, D_val)
    for i, (rows, v) in cols.items():
        assert np.array_equal(D[rows, i], v)
