"""Pins for the pre-determined SP2 sequence (MD section): a sequence built from the
eigensolver's HOMO and LUMO replays to the eigensolver's projector, and the distances it
tracks are the actual eigenvalue images of the replayed iterates.  CPU only."""
import numpy as np
import pytest

from synth import make_model
from oracle.bounds import ell_to_dense, gershgorin
from oracle.exact import density_exact
from oracle.sequence import sequence_from_gap, propagate
from oracle.sp2 import sp2_partitioned


def _dense(name):
    m = make_model(name)
    H = ell_to_dense(m["H_col"], m["H_val"])
    lo, hi = gershgorin(m["H_col"], m["H_val"])
    X0 = (hi * np.eye(len(H)) - H) / (hi - lo)
    return m, H, X0, lo, hi


@pytest.mark.parametrize("name", ["tiny48", "small256"])
def test_sequence_from_exact_gap_gives_the_projector(name):
    m, H, X0, lo, hi = _dense(name)
    n = m["n_occ"]
    w = np.linalg.eigvalsh(H)
    seq = sequence_from_gap(lo, hi, w[n - 1], w[n])
    xs, info = sp2_partitioned([X0.copy()], [len(H)], n, 0.0, branch_in=seq)
    D, _, _ = density_exact(H, n)
    assert np.abs(xs[0] - D).max() < 1e-10
    assert abs(np.trace(xs[0]) - n) < 1e-9
    # no longer than the trace-driven expansion needs (plus one step)
    _, ref = sp2_partitioned([X0.copy()], [len(H)], n, 1e-10 * len(H) / 1024)
    assert len(seq) <= ref["iters"] + 1


def test_tracked_distances_are_eigenvalue_images():
    m, H, X0, lo, hi = _dense("tiny48")
    n = m["n_occ"]
    w, V = np.linalg.eigh(H)
    seq = sequence_from_gap(lo, hi, w[n - 1], w[n])[:6]
    u0 = 1.0 - (hi - w[n - 1]) / (hi - lo)
    v0 = (hi - w[n]) / (hi - lo)
    us, vs = propagate(u0, v0, seq)
    xs, _ = sp2_partitioned([X0.copy()], [len(H)], n, 0.0, branch_in=seq)
    X = xs[0]
    vh, vl = V[:, n - 1], V[:, n]
    assert abs((vh @ X @ vh) - (1.0 - us[-1])) < 1e-12
    assert abs((vl @ X @ vl) - vs[-1]) < 1e-12


def test_rule_and_errors():
    # e in [0, 1] maps to x = 1 - e: u = e_homo, v = 1 - e_lumo
    # v = 0.45 > u = 0.30 -> X^2 first; u = 0.45 > v = 0.40 -> 2X - X^2 first
    assert sequence_from_gap(0.0, 1.0, 0.30, 0.55)[0] == 0
    assert sequence_from_gap(0.0, 1.0, 0.45, 0.60)[0] == 1
    with pytest.raises(ValueError):
        sequence_from_gap(0.0, 1.0, 0.6, 0.4)
