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


def test_whole_matrix_adjoint_vs_daleckii_krein(gb, model_cache):
    """N = 1024 with one subgraph holding every vertex: the GPU adjoint of Tr[D V] equals the
    eigen-decomposition derivative of the exact projector."""
    from synth import make_operator_v
    from oracle.bounds import ell_to_dense
    from oracle.adjoint import daleckii_krein_grad
    m = model_cache("n1024")
    V = make_operator_v(m["H_col"], 51)
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                  core_size=4096, keep_tape=True)
    assert st["n_sub"] == 1 and st["converged"]
    Dc = D_col.cpu().numpy()
    GH = st["tape"].vjp(_dev(_grad_d(V, m["H_col"], Dc))).cpu().numpy()
    H = ell_to_dense(m["H_col"], m["H_val"])
    Gdk = daleckii_krein_grad(H, ell_to_dense(m["H_col"], V), m["n_occ"])
    r, t = np.nonzero(m["H_col"] >= 0)
    err = np.abs(GH[r, t] - Gdk[r, m["H_col"][r, t]]).max()
    print(f"DK max diff {err:.3e} (max |G| {np.abs(Gdk).max():.3f})")
    assert err < 1e-8


def test_fullsize_adjoint_vs_central_differences(gb):
    """N = 18000: the adjoint against central differences of the GPU forward map with the
    graph, partition, bounds and branch sequence frozen (h = 1e-6, 8 sampled entries)."""
    import torch
    from synth import make_model, make_operator_v
    m = make_model("n18000")
    V = make_operator_v(m["H_col"], 51)
    Hc, Hv = _dev(m["H_col"]), _dev(m["H_val"])
    g = gb.build_graph(Hc, Hv, 1e-5)
    p = gb.partition(g, 32)
    D_col, D_val, st = gb.density(Hc, Hv, m["n_occ"], 1e-5, partition=p, keep_tape=True)
    Dc = D_col.cpu().numpy()
    GDn = _grad_d(V, m["H_col"], Dc)
    GD = _dev(GDn)
    GH = st["tape"].vjp(GD).cpu().numpy()
    del st["tape"]
    br = st["branch"]
    emin, emax = st["emin"], st["emax"]

    def L_of(Hval):
        dc, dv, s2 = gb.density(Hc, _dev(Hval), m["n_occ"], 1e-5, partition=p, branch_in=br,
                                emin=emin, emax=emax, D=(D_col, torch.empty_like(D_val)))
        return float((dv * GD).sum())

    rng = np.random.default_rng(53)
    gmax = np.abs(GH).max()
    h = 1e-6
    for _ in range(8):
        i = int(rng.integers(0, m["N"]))
        t = int(rng.integers(0, (m["H_col"][i] >= 0).sum()))
        j = int(m["H_col"][i, t])
        tj = int(np.nonzero(m["H_col"][j] == i)[0][0])
        plus, minus = m["H_val"].copy(), m["H_val"].copy()
        plus[i, t] += h
        minus[i, t] -= h
        if i != j:
            plus[j, tj] += h
            minus[j, tj] -= h
        fd = (L_of(plus) - L_of(minus)) / (2 * h)
        ad = GH[i, t] + (GH[j, tj] if i != j else 0.0)
        print(f"({i},{j}) fd={fd:.9e} adjoint={ad:.9e}")
        assert abs(fd - ad) <= max(1e-5 * gmax, 1e-7)


def test_dprev_symbolic_graph_bit_exact(gb, model_cache):
    """Eq. 8 with eps = 0 (symbolic square of pattern(H) and the thresholded previous D)."""
    from oracle.graph import graph_dprev_symbolic
    from oracle.sp2 import density_partitioned
    m = model_cache("small256")
    Dc, Dv, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-3, 16)
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), 0.0, mode="dprev_symbolic",
                       aux=(_dev(Dc), _dev(Dv)), tau_aux=1e-2)
    rp, cl = [t.cpu().numpy() for t in g.arrays()]
    orp, ocl = graph_dprev_symbolic(m["H_col"], Dc, Dv, 1e-2)
    assert np.array_equal(rp, orp) and np.array_equal(cl, ocl)
