"""Pins for the partitioned SP2 oracle: exact special cases, the eigensolver, the
paper's Eq. 6 equivalence, the occupation and the accuracy trend.  CPU only."""
import numpy as np
import pytest

from synth import ModelSpec, make_model
from oracle.bounds import gershgorin, x0_values, ell_to_dense
from oracle.graph import graph_x2
from oracle.partition import partition
from oracle.sp2 import (gather, sp2_partitioned, sp2_dense, scatter_columns,
                        density_partitioned, x0_dense)
from oracle.exact import density_exact
from oracle.equivalence import (column_mask, sp2_power_coefficients, masked_horner,
                                dense_horner, masked_chebyshev, dense_chebyshev,
                                assemble_columns)
from oracle.metrics import column_ell_to_dense, errors

MID = ModelSpec(n_sites=256, seed=11, name="n512")


@pytest.fixture(scope="module")
def mid():
    return make_model(MID)


def test_exact_projector_invariants(model_cache):
    m = model_cache("n1024")
    H = ell_to_dense(m["H_col"], m["H_val"])
    D, w, gap = density_exact(H, m["n_occ"])
    assert abs(np.trace(D) - m["n_occ"]) < 1e-10
    assert np.abs(D @ D - D).max() < 1e-12
    assert np.abs(H @ D - D @ H).max() < 1e-12
    assert gap > 0.5


def test_branch_rule_hand_cases():
    # one 1x1 block, core 1: x = 0.6, n_occ = 1 -> t1 = .6, t2 = .36
    # |t2 - 1| = .64 > |2*.6 - .36 - 1| = .16 -> b = 1 (2x - x^2)
    xs, info = sp2_partitioned([np.array([[0.6]])], [1], 1, 1e-14, max_iter=1)
    assert info["branch"][0] == 1
    xs, info = sp2_partitioned([np.array([[0.6]])], [1], 0, 1e-14, max_iter=1)
    assert info["branch"][0] == 0
    # a tie (t1 = n_occ exactly, x = 0.5, n = 0.5 -> d_sq = .25, d_lin = .25) -> 1
    xs, info = sp2_partitioned([np.array([[0.5]])], [1], 0.5, 1e-14, max_iter=1)
    assert info["branch"][0] == 1


def test_scalar_sp2_matches_polynomial_composition():
    """The SP2 map after K steps is a polynomial of degree 2^K (expansion order over
    a billion after 30 steps, SP2 paragraph after Eq. 7); check the composed
    coefficients against the scalar recursion."""
    br = [0, 1, 1, 0, 1, 0]
    c = sp2_power_coefficients(br)
    assert len(c) - 1 == 2 ** len(br)
    from fractions import Fraction
    for num in range(0, 17):
        x = Fraction(num, 16)
        y = x
        for b in br:
            y = y * y if b == 0 else 2 * y - y * y
        assert sum(ck * x ** k for k, ck in enumerate(c)) == y   # exact rationals
    assert 2 ** 30 > 1e9


def test_diagonal_h_gives_exact_occupation():
    rng = np.random.default_rng(3)
    N = 40
    d = rng.permutation(np.linspace(-3, 3, N))
    col = np.arange(N, dtype=np.int32)[:, None]
    val = d[:, None]
    D_col, D_val, info = density_partitioned(col, val, 15, 1e-5, 4, idem_tol=1e-14)
    D = column_ell_to_dense(D_col, D_val)
    want = np.diag((d <= np.sort(d)[14]).astype(float))
    assert info["converged"]
    assert np.abs(D - want).max() < 1e-14


def test_complete_graph_equals_dense_sp2_and_eigensolver(mid):
    """One community holding every vertex: the partitioned method is whole-matrix
    dense SP2 (Results: one community costs O(N^3)); compare with diagonalisation."""
    m = mid
    N = m["N"]
    emin, emax = gershgorin(m["H_col"], m["H_val"])
    x0 = x0_values(m["H_col"], m["H_val"], emin, emax)
    blk = gather(m["H_col"], x0, np.arange(N, dtype=np.int32))
    assert np.array_equal(blk, x0_dense(m["H_col"], m["H_val"]))
    xs, info = sp2_partitioned([blk], [N], m["n_occ"], 1e-10)
    xd, infod = sp2_dense(blk, m["n_occ"], 1e-10)
    assert info["branch"] == infod["branch"]
    assert np.array_equal(xs[0], xd)
    D, w, gap = density_exact(ell_to_dense(m["H_col"], m["H_val"]), m["n_occ"])
    assert np.abs(xs[0] - D).max() < 1e-12


def test_block_diagonal_h_aligned_cores():
    """Disconnected blocks, one core per block: no halos, and the assembled D is the
    exact projector of the whole matrix."""
    rng = np.random.default_rng(8)
    nb, bs = 6, 10
    N = nb * bs
    H = np.zeros((N, N))
    for b in range(nb):
        A = rng.normal(0, 0.3, (bs, bs))
        A = (A + A.T) / 2 + np.diag(np.where(np.arange(bs) % 2 == 0, -1.5, 1.5))
        H[b * bs:(b + 1) * bs, b * bs:(b + 1) * bs] = A
    W = bs
    col = np.full((N, W), -1, dtype=np.int32)
    val = np.zeros((N, W))
    for i in range(N):
        nz = np.nonzero(H[i])[0]
        col[i, :len(nz)] = nz
        val[i, :len(nz)] = H[i, nz]
    n_occ = N // 2
    D_col, D_val, info = density_partitioned(col, val, n_occ, 0.0, bs, idem_tol=1e-12)
    assert np.diff(info["sub_ptr"]).tolist() == [bs] * nb
    D = column_ell_to_dense(D_col, D_val)
    De, w, gap = density_exact(H, n_occ)
    assert gap > 0.1
    assert np.abs(D - De).max() < 1e-10


def _setup(m, tau, core):
    N = m["N"]
    emin, emax = gershgorin(m["H_col"], m["H_val"])
    x0 = x0_values(m["H_col"], m["H_val"], emin, emax)
    rp, cl = graph_x2(m["H_col"], m["H_val"], tau, emin, emax)
    cp, cv, sp, si = partition(rp, cl, core)
    subs = [si[sp[s]:sp[s + 1]] for s in range(len(sp) - 1)]
    cores = [cv[cp[s]:cp[s + 1]] for s in range(len(cp) - 1)]
    blocks = [gather(m["H_col"], x0, s) for s in subs]
    return N, ell_to_dense(m["H_col"], x0), cp, sp, si, cores, blocks


@pytest.mark.parametrize("tau,core", [(1e-3, 1), (1e-3, 8), (1e-5, 16)])
def test_eq6_equivalence_sp2(model_cache, tau, core):
    """Eq. 6: the whole-matrix polynomial thresholded after every product (Eqs. 3-5,
    column mask of the core's subgraph) equals the column-assembled subgraph
    polynomials.  Three fixed SP2 steps (degree 8), then four (degree 16)."""
    m = model_cache("small256")
    N, X0, cp, sp, si, cores, blocks = _setup(m, tau, core)
    R = column_mask(N, sp, si, cores)
    kc = np.diff(cp)
    for br, tol in (([1, 0, 1], 1e-13), ([0, 1, 1, 0], 1e-12)):
        c = sp2_power_coefficients(br)
        left = masked_horner(X0, c, R)
        right_h = assemble_columns(N, [dense_horner(b, c) for b in blocks], sp, si, kc)
        xs, info = sp2_partitioned(blocks, kc, N // 2, 0.0, branch_in=br)
        right_sp2 = assemble_columns(N, xs, sp, si, kc)
        assert np.abs(left - right_h).max() < tol
        assert np.abs(left - right_sp2).max() < tol
    # without the mask (plain whole-matrix polynomial) the columns differ: the
    # thresholding is what the subgraphs reproduce
    if core == 1 and tau == 1e-3:
        full = dense_horner(X0, sp2_power_coefficients([1, 0, 1]))
        assert np.abs(full - left).max() > 1e-6


def test_eq6_equivalence_chebyshev(model_cache):
    m = model_cache("small256")
    N, X0, cp, sp, si, cores, blocks = _setup(m, 1e-3, 8)
    R = column_mask(N, sp, si, cores)
    kc = np.diff(cp)
    coeffs = np.polynomial.chebyshev.chebinterpolate(lambda t: 1.0 / (1.0 + np.exp(8 * t)), 40)
    I = np.eye(N)
    left = masked_chebyshev(2 * X0 - I, coeffs, R)
    right = assemble_columns(N, [dense_chebyshev(2 * b - np.eye(len(b)), coeffs) for b in blocks],
                             sp, si, kc)
    assert np.abs(left - right).max() < 1e-13


def test_partitioned_occupation_and_accuracy(mid):
    m = mid
    D_col, D_val, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-5, 16)
    assert info["converged"]
    # the assembled trace is the core-trace the loop drove to n_occ
    t1 = info["traces"][-1][0]
    assert abs(info["trace"] - t1) < 1e-9
    assert abs(info["trace"] - m["n_occ"]) < 1e-6
    H = ell_to_dense(m["H_col"], m["H_val"])
    De, w, gap = density_exact(H, m["n_occ"])
    err = errors(column_ell_to_dense(D_col, D_val), De, H, m["N"] // 2)
    assert err["max_abs"] < 2e-3
    # pattern of D = the subgraph rows of each column (obs. iv-v)
    sp, si, cp = info["sub_ptr"], info["sub_idx"], info["core_ptr"]
    for s in range(len(sp) - 1):
        rows = np.sort(si[sp[s]:sp[s + 1]])
        for i in range(cp[s], cp[s + 1]):
            assert np.array_equal(D_col[i, :len(rows)], rows)


def test_accuracy_improves_as_tau_decreases(mid):
    """Obs. ii: the error against the exact D does not grow as tau is lowered."""
    m = mid
    H = ell_to_dense(m["H_col"], m["H_val"])
    De, w, gap = density_exact(H, m["n_occ"])
    errs = []
    for tau in (1e-4, 1e-5, 1e-6):
        D_col, D_val, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], tau, 16)
        errs.append(np.abs(column_ell_to_dense(D_col, D_val) - De).max())
    assert errs[1] <= 1.1 * errs[0] and errs[2] <= 1.1 * errs[1]
    assert errs[2] < 0.2 * errs[0]


def test_whole_matrix_thresholded_sp2_tight_tau_is_exact(mid):
    """The paper's exact reference is thresholded sparse algebra at tau = 1e-12."""
    m = mid
    X0 = x0_dense(m["H_col"], m["H_val"])
    x, info = sp2_dense(X0, m["n_occ"], 1e-10, tau=1e-12)
    De, w, gap = density_exact(ell_to_dense(m["H_col"], m["H_val"]), m["n_occ"])
    assert info["converged"] and np.abs(x - De).max() < 1e-10


def test_replay_reproduces_run(model_cache):
    m = model_cache("small256")
    N, X0, cp, sp, si, cores, blocks = _setup(m, 1e-4, 16)
    kc = np.diff(cp)
    xs, info = sp2_partitioned(blocks, kc, m["n_occ"], 1e-10 * N / 1024)
    xr, infr = sp2_partitioned(blocks, kc, m["n_occ"], 1e-10 * N / 1024, branch_in=info["branch"])
    assert infr["branch"] == info["branch"]
    assert all(np.array_equal(a, b) for a, b in zip(xs, xr))


def test_mcweeny_refinement_restores_idempotency():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.normal(size=(30, 30)))
    P = Q[:, :12] @ Q[:, :12].T
    E = rng.normal(0, 1e-4, (30, 30))
    X = P + (E + E.T) / 2
    xs, info = sp2_partitioned([X], [30], 12, np.inf, n_refine=3)
    w = np.linalg.eigvalsh(xs[0])
    assert np.abs(np.minimum(np.abs(w), np.abs(w - 1))).max() < 1e-12


def test_scatter_sorted_column_ell():
    blocks = [np.arange(16.0).reshape(4, 4)]
    sub_ptr = np.array([0, 4])
    sub_idx = np.array([5, 2, 7, 0], dtype=np.int32)   # core {5, 2}? cores are first
    D_col, D_val = scatter_columns(blocks, sub_ptr, sub_idx, [2], 8, width=5)
    assert D_col[5].tolist() == [0, 2, 5, 7, -1]
    assert D_val[5].tolist() == [12.0, 4.0, 0.0, 8.0, 0.0]
    assert D_col[2].tolist() == [0, 2, 5, 7, -1]
    assert D_val[2].tolist() == [13.0, 5.0, 1.0, 9.0, 0.0]
    assert (D_col[0] == -1).all()


def test_low_memory_mode_matches(mid):
    """The low-memory oracle (traces from diagonal dot products, squares recomputed for the
    update) takes the same branches and returns the same D."""
    m = mid
    a = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-5, 16)
    b = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-5, 16, low_memory=True)
    assert a[2]["branch"] == b[2]["branch"]
    assert np.abs(a[1] - b[1]).max() < 1e-13


def test_metrics_hand_example():
    """Fig. 2 measures on a 2 x 2 case worked by hand.  diff = D - D_ref = [[.1, -.2],
    [-.1, -.1]] (not symmetric, so a transposed H changes the band energy): max-abs 0.2;
    Frobenius norm sqrt(.01 + .04 + .01 + .01) = sqrt(.07), per site (2 sites) sqrt(.07)/2;
    Tr[diff H] = sum_ij diff_ij H_ji = .1*1 - .2*3 - .1*2 - .1*4 = -1.1, per site 0.55
    (without the transpose it would be -1.0); Tr D = 1; D is idempotent."""
    D = np.array([[1.0, 0.0], [0.0, 0.0]])
    D_ref = np.array([[0.9, 0.2], [0.1, 0.1]])
    H = np.array([[1.0, 2.0], [3.0, 4.0]])
    e = errors(D, D_ref, H, 2)
    assert abs(e["max_abs"] - 0.2) < 1e-15
    assert abs(e["frob_per_site"] - np.sqrt(0.07) / 2) < 1e-15
    assert abs(e["eband_err_per_site"] - 0.55) < 1e-15
    assert e["trace"] == 1.0 and e["idem"] == 0.0


def test_core_columns_equal_whole_system_oracle(mid):
    """The oracle restricted to chosen cores (their subgraphs only, the whole run's branch
    sequence replayed) gives the whole-system oracle's D columns bit for bit."""
    from oracle.subgraphs import core_columns
    m = mid
    D_col, D_val, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-5, 16)
    cp = info["core_ptr"]
    picks = [0, 5, len(cp) - 2]
    cores = [np.arange(cp[c], cp[c + 1]) for c in picks]
    out = core_columns(m["H_col"], m["H_val"], m["n_occ"], 1e-5, cores, info["branch"])
    for verts, (rows, vals) in zip(cores, out):
        for c, v in enumerate(verts):
            assert np.array_equal(D_col[v, :len(rows)], rows)
            assert (D_col[v, len(rows):] == -1).all()
            assert np.array_equal(D_val[v, :len(rows)], vals[c])


def test_thresholded_sp2_stall_stop(mid):
    """With thresholding the idempotency measure stalls above a tight tolerance; the stall stop
    ends the expansion there, after at least ten steps, at an error against the eigensolver of
    the order of the threshold, while tau = 1e-12 still converges without it."""
    m = mid
    X0 = x0_dense(m["H_col"], m["H_val"])
    De, w, gap = density_exact(ell_to_dense(m["H_col"], m["H_val"]), m["n_occ"])
    x, info = sp2_dense(X0, m["n_occ"], 1e-12, tau=1e-5, stall_stop=True)
    e = [abs(a - b) for a, b in info["traces"]]
    assert info["stalled"] and not info["converged"] and info["iters"] >= 10
    assert e[-1] > e[-3]
    assert np.abs(x - De).max() < 1e-3
    x2, info2 = sp2_dense(X0, m["n_occ"], 1e-10, tau=1e-12, stall_stop=True)
    assert info2["converged"] and not info2["stalled"]
