"""Error measures (oracle).

Fig. 2 reports the density-matrix error as a Frobenius norm normalised per atom and
the band-energy error E_band = Tr[D H] per atom.  Max-abs is taken over the union of
the two patterns (a missing entry counts as 0).
"""
import numpy as np


def column_ell_to_dense(D_col: np.ndarray, D_val: np.ndarray) -> np.ndarray:
    """Dense D from column-ELL arrays (row i of the arrays = column i of D)."""
    N = D_col.shape[0]
    D = np.zeros((N, N))
    i, t = np.nonzero(D_col >= 0)
    D[D_col[i, t], i] = D_val[i, t]
    return D


def errors(D: np.ndarray, D_ref: np.ndarray, H: np.ndarray, n_sites: int) -> dict:
    diff = D - D_ref
    return {
        "max_abs": float(np.max(np.abs(diff))),
        "frob_per_site": float(np.linalg.norm(diff) / n_sites),
        "eband_err_per_site": float(abs(np.sum(diff * H.T)) / n_sites),
        "trace": float(np.trace(D)),
        "idem": float(np.max(np.abs(D @ D - D))),
    }
