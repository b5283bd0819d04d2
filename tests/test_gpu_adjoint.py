"""Adjoint of Tr[D V] on the GPU against the oracle's reverse recursion (GPU)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available()
    import paper_1603_00937_amd as gb
    return gb


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _grad_d(V, H_col, D_col):
    """dL/dD[r, i] = V[i, r] on D's column-ELL pattern (zero off V's pattern)."""
    N = H_col.shape[0]
    G = np.zeros(D_col.shape)
    for i in range(N):
        cols = H_col[i][H_col[i] >= 0]
        vals = V[i][:len(cols)]
        rows = D_col[i]
        pos = np.searchsorted(cols, rows)
        pos = np.minimum(pos, len(cols) - 1)
        hit = (rows >= 0) & (cols[pos] == rows)
        G[i, hit] = vals[pos[hit]]
    return G


@pytest.fixture(scope="module")
def case(model_cache):
    from synth import make_operator_v
    from oracle.sp2 import density_partitioned
    from oracle.adjoint import trace_dv_and_grad
    m = model_cache("small256")
    V = make_operator_v(m["H_col"], 51)
    Dc, Dv, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-4, 16,
                                       keep_tape=True)
    L, G = trace_dv_and_grad(m["H_col"], m["H_val"], V, m["n_occ"], info, None)
    return m, V, Dc, info, L, G


@pytest.mark.parametrize("stride", [0, 1, 3, 64])
def test_vjp_matches_oracle(gb, case, stride):
    m, V, Dc, info, L, G = case
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-4,
                                  core_size=16, keep_tape=True, tape_stride=stride)
    assert st["branch"] == info["branch"]
    assert np.array_equal(D_col.cpu().numpy(), Dc)
    GD = _grad_d(V, m["H_col"], Dc)
    GH = st["tape"].vjp(_dev(GD)).cpu().numpy()
    assert np.abs(GH - G).max() <= 1e-9 * max(1.0, np.abs(G).max())


def test_autograd_function(gb, case):
    import torch
    m, V, Dc, info, L, G = case
    Hv = _dev(m["H_val"]).requires_grad_(True)
    D_col, D_val, st = gb.density_with_grad(_dev(m["H_col"]), Hv, m["n_occ"], 1e-4, core_size=16)
    GD = _dev(_grad_d(V, m["H_col"], D_col.cpu().numpy()))
    loss = (D_val * GD).sum()
    loss.backward()
    assert abs(loss.item() - L) < 1e-9
    assert np.abs(Hv.grad.cpu().numpy() - G).max() <= 1e-9 * max(1.0, np.abs(G).max())


def test_dprev_graph_bit_exact(gb, model_cache):
    from oracle.graph import graph_dprev
    from oracle.sp2 import density_partitioned
    m = model_cache("small256")
    Dc, Dv, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-4, 16)
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), 1e-5, mode="dprev",
                       aux=(_dev(Dc), _dev(Dv)), tau_aux=1e-4)
    rp, cl = [t.cpu().numpy() for t in g.arrays()]
    orp, ocl = graph_dprev(m["H_col"], m["H_val"], Dc, Dv, 1e-5, 1e-4)
    assert np.array_equal(rp, orp) and np.array_equal(cl, ocl)
