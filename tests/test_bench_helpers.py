"""Host-side measures of the benchmark (CPU): |D^2 - D| on chosen columns of a column-ELL D and
the element-wise error against the oracle's columns, pinned to dense evaluations."""
import numpy as np

import bench


def _col_ell(D, width):
    """Column-ELL arrays of a dense matrix (row i of the arrays = column i of D, every nonzero
    and the diagonal kept, rows ascending)."""
    N = D.shape[0]
    dc = np.full((N, width), -1, dtype=np.int32)
    dv = np.zeros((N, width))
    for j in range(N):
        rows = np.nonzero((D[:, j] != 0) | (np.arange(N) == j))[0]
        dc[j, :len(rows)] = rows
        dv[j, :len(rows)] = D[rows, j]
    return dc, dv


def test_idempotency_matches_dense():
    rng = np.random.default_rng(3)
    N = 40
    Q, _ = np.linalg.qr(rng.normal(size=(N, N)))
    P = Q[:, :15] @ Q[:, :15].T
    P[np.abs(P) < 0.05] = 0.0          # a sparse, nearly idempotent, non-symmetric pattern
    P[3, 7] += 1e-3                      # and a non-symmetric entry
    dc, dv = _col_ell(P, N)
    cols = [np.array([0, 3, 7]), np.array([20, 21])]
    got = bench.idempotency(dc, dv, cols)
    E = (P @ P - P)[:, np.concatenate(cols)]
    assert abs(got["max_abs"] - np.abs(E).max()) < 1e-14
    assert abs(got["frobenius"] - np.linalg.norm(E)) < 1e-13
    assert got["columns"] == 5
    # an exact projector on its full pattern: zero up to rounding
    Pf = Q[:, :15] @ Q[:, :15].T
    dc, dv = _col_ell(Pf, N)
    assert bench.idempotency(dc, dv, cols)["max_abs"] < 1e-14


def test_d_errors_against_columns():
    rng = np.random.default_rng(4)
    N = 12
    D = rng.normal(size=(N, N)) * (rng.random((N, N)) < 0.4)
    dc, dv = _col_ell(D, N)
    rows = dc[2][dc[2] >= 0]
    # oracle columns for core {2} only (pattern of column 2), off by 1e-7 everywhere
    ref = [(np.array([2]), (rows, D[rows, 2][None, :] + 1e-7))]
    e = bench.d_errors(dc, dv, ref)
    assert e["pattern_equal"] and abs(e["max_abs"] - 1e-7) < 1e-12
    assert abs(e["frobenius"] - 1e-7 * np.sqrt(len(rows))) < 1e-12


def test_symmetric_square_flops():
    # n = 2: upper entries (0,0), (0,1), (1,1), 2n = 4 flops each = 12 = n^2 (n + 1)
    assert bench.sym_square_flops([2], 1) == 12.0
    assert bench.sym_square_flops([2, 3], 6) == 6 * (12.0 + 36.0)


def test_stage_hbm_bytes():
    """Gather: padded blocks (64-multiples) times the element size plus H's ELL; scatter: 20
    bytes per D entry (core columns times subgraph rows)."""
    import numpy as np
    import bench
    model = {"H_col": np.zeros((10, 3), np.int32)}
    out = bench.stage_hbm({"gather": 1.0, "scatter": 2.0}, np.array([65, 64]),
                          np.array([2, 3]), model, "fp16x3")
    assert out["gather_bytes"] == (128 * 128 + 64 * 64) * 4 + 30 * 12
    assert out["scatter_bytes"] == (2 * 65 + 3 * 64) * 20
    assert abs(out["gather"] - out["gather_bytes"] / 1e-3 / 1e9) < 1e-9
    fp64 = bench.stage_hbm({}, np.array([65]), np.array([2]), model, "fp64")
    assert fp64["gather_bytes"] == 128 * 128 * 8 + 30 * 12 and "gather" not in fp64
