"""Exact zero-temperature density matrix by dense diagonalisation (oracle).

D = theta(mu I - H) (SP2 paragraph after Eq. 7) is the projector onto the n_occ
lowest eigenvectors of H; the paper's own exact reference is a tightly thresholded
expansion (Results, Fig. 2 text), which agrees with this projector for a gapped H.

Pins: Tr D = n_occ, D^2 = D, [H, D] = 0 (checked in the tests to 1e-12).
"""
import numpy as np


def density_exact(H: np.ndarray, n_occ: int):
    """(D, eigenvalues, gap) for a dense symmetric H."""
    w, V = np.linalg.eigh(H)
    Vo = V[:, :n_occ]
    D = Vo @ Vo.T
    gap = float(w[n_occ] - w[n_occ - 1]) if 0 < n_occ < H.shape[0] else np.inf
    return D, w, gap


def frontier_levels(H: np.ndarray, n_occ: int):
    """(e_homo, e_lumo): the n_occ-th and (n_occ+1)-th eigenvalues of a dense symmetric H."""
    w = np.linalg.eigvalsh(H)
    return float(w[n_occ - 1]), float(w[n_occ])
