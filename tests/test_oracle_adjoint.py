"""Pins for the oracle's adjoint of Tr[D V]: central finite differences of the frozen
forward map, and the eigen-decomposition derivative of the exact projector.  CPU only."""
import numpy as np
import pytest

from synth import make_operator_v
from oracle.bounds import ell_to_dense
from oracle.sp2 import density_partitioned
from oracle.adjoint import trace_dv_and_grad, frozen_trace_dv, daleckii_krein_grad


@pytest.fixture(scope="module")
def run(model_cache):
    m = model_cache("small256")
    V = make_operator_v(m["H_col"], 51)
    Dc, Dv, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-4, 16,
                                       keep_tape=True)
    L, G = trace_dv_and_grad(m["H_col"], m["H_val"], V, m["n_occ"], info, None)
    return m, V, info, L, G, Dc, Dv


def test_trace_dv_matches_assembled_d(run):
    m, V, info, L, G, Dc, Dv = run
    from oracle.metrics import column_ell_to_dense
    D = column_ell_to_dense(Dc, Dv)
    Vd = ell_to_dense(m["H_col"], V)
    assert abs(L - float(np.sum(D * Vd.T))) < 1e-10


def test_adjoint_vs_central_differences(run):
    m, V, info, L, G, Dc, Dv = run
    rng = np.random.default_rng(53)
    gmax = np.abs(G).max()
    for _ in range(12):
        i = int(rng.integers(0, m["N"]))
        t = int(rng.integers(0, (m["H_col"][i] >= 0).sum()))
        j = int(m["H_col"][i, t])
        h = 1e-6
        fd = (frozen_trace_dv(m["H_col"], m["H_val"], V, info, i, j, h)
              - frozen_trace_dv(m["H_col"], m["H_val"], V, info, i, j, -h)) / (2 * h)
        tj = np.nonzero(m["H_col"][j] == i)[0][0]
        ad = G[i, t] + (G[j, tj] if i != j else 0.0)
        assert abs(fd - ad) <= max(1e-5 * gmax, 1e-7), (i, j, fd, ad)


def test_adjoint_gradient_is_symmetric(run):
    m, V, info, L, G, Dc, Dv = run
    Gd = ell_to_dense(m["H_col"], G)
    assert np.abs(Gd - Gd.T).max() < 1e-14


def test_whole_matrix_adjoint_equals_daleckii_krein(model_cache):
    """One subgraph holding every vertex: the SP2 adjoint is the derivative of the exact
    projector, which the eigen-decomposition gives in closed form."""
    m = model_cache("small256")
    V = make_operator_v(m["H_col"], 51)
    Dc, Dv, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-5, 10 ** 6,
                                       keep_tape=True)
    L, G = trace_dv_and_grad(m["H_col"], m["H_val"], V, m["n_occ"], info, None)
    H = ell_to_dense(m["H_col"], m["H_val"])
    Gdk = daleckii_krein_grad(H, ell_to_dense(m["H_col"], V), m["n_occ"])
    r, t = np.nonzero(m["H_col"] >= 0)
    assert np.abs(G[r, t] - Gdk[r, m["H_col"][r, t]]).max() < 1e-8
