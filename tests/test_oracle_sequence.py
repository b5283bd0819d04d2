"""Pins for the pre-determined SP2 sequence (MD section): a sequence built from the
eigensolver's HOMO and LUMO replays to the eigensolver's projector, and the distances it
tracks are the actual eigenvalue images of the replayed iterates.  Pins for the gap estimate
from an expansion's traces: the levels of two-level spectra (with multiplicities), the bracket
around the eigensolver's HOMO and LUMO for dense and partitioned expansions, and a sequence
from the estimate that replays to the projector.  CPU only."""
import itertools

import numpy as np
import pytest

from synth import make_model
from oracle.bounds import ell_to_dense, gershgorin
from oracle.exact import density_exact
from oracle.sequence import sequence_from_gap, propagate, estimate_gap, _g, _forward
from oracle.sp2 import sp2_partitioned, density_partitioned


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


def _diag_expansion(levels, n_occ, emin=-2.0, emax=2.0):
    """Dense SP2 of diag(levels), the bounds included as exact levels (they map to 1 and 0)."""
    h = np.array(list(levels) + [emin, emax])
    X0 = np.diag((emax - h) / (emax - emin))
    _, info = sp2_partitioned([X0], [len(h)], n_occ + 1, 1e-14)
    return info


@pytest.mark.parametrize("mh,ml,a,b", [(1, 1, -0.7, 0.4), (3, 2, -0.2, 0.5), (5, 7, 0.1, 0.15),
                                       (2, 1, 0.3, 0.35)])
def test_two_level_spectra(mh, ml, a, b):
    """One occupied level a (multiplicity mh) and one unoccupied level b (ml): the ratio
    estimates are the levels, whatever the multiplicities; the bounds sit between the levels
    and the gap centre, exact for a single state."""
    info = _diag_expansion([a] * mh + [b] * ml, mh)
    assert info["converged"]
    e = estimate_gap(info["traces"], info["branch"], mh + 1, -2.0, 2.0)
    assert abs(e["homo_ratio"] - a) < 1e-6 and abs(e["lumo_ratio"] - b) < 1e-6
    assert a - 1e-6 <= e["homo_bound"] < e["lumo_bound"] <= b + 1e-6
    if mh == 1:
        assert abs(e["homo_bound"] - a) < 1e-6
    if ml == 1:
        assert abs(e["lumo_bound"] - b) < 1e-6
    assert e["homo_bound"] - a < 0.03 and b - e["lumo_bound"] < 0.03


@pytest.mark.parametrize("mh,ml,a,b,floor", [(4, 1, -0.05, 0.3, 1e-3), (8, 1, -0.3, 0.1, 1e-2)])
def test_bound_keeps_the_cross_term(mh, ml, a, b, floor):
    """At an earlier iterate (a raised floor) the occupied side still adds sum u^2/2 to L; the
    bound includes it (as U^2/2) and stays at or below the lone LUMO."""
    info = _diag_expansion([a] * mh + [b] * ml, mh)
    e = estimate_gap(info["traces"], info["branch"], mh + 1, -2.0, 2.0, floor=floor)
    assert e["lumo_bound"] <= b + 1e-12
    assert e["homo_bound"] >= a - 1e-12


def test_ratio_function_rises_below_one():
    """The bisection assumes g(F(x))/g(x) < 1 exactly on an initial interval of (0, 1) and
    increases there, for every branch segment that squares the side (up to 6 steps here)."""
    xs = np.linspace(1e-6, 1.0 - 1e-9, 4001)
    for n in range(1, 7):
        for seg in itertools.product([0, 1], repeat=n):
            for side, sq in (("v", 0), ("u", 1)):
                if sq not in seg:
                    continue
                r = np.array([_g(_forward(x, seg, side)) / _g(x) for x in xs])
                k = int(np.argmin(r < 1.0)) if (r >= 1.0).any() else len(r)
                assert (r[k:] >= 1.0).all(), (seg, side)
                d = np.diff(r[:k])
                assert ((d > 0) | (r[1:k] < 1e-200)).all(), (seg, side)


def _check_bracket(e, w, n, lo, hi, width):
    W = hi - lo
    tol = 1e-6 * W
    assert e["homo_ratio"] - tol <= w[n - 1] <= e["homo_bound"] + tol
    assert e["lumo_bound"] - tol <= w[n] <= e["lumo_ratio"] + tol
    assert e["homo_bound"] - e["homo_ratio"] < width * W
    assert e["lumo_ratio"] - e["lumo_bound"] < width * W


@pytest.mark.parametrize("name", ["tiny48", "small256"])
def test_dense_expansion_brackets_homo_and_lumo(name):
    m, H, X0, lo, hi = _dense(name)
    n = m["n_occ"]
    w = np.linalg.eigvalsh(H)
    _, info = sp2_partitioned([X0.copy()], [len(H)], n, 1e-10 * len(H) / 1024)
    e = estimate_gap(info["traces"], info["branch"], n, lo, hi)
    _check_bracket(e, w, n, lo, hi, 0.03)


def test_partitioned_expansion_brackets_homo_and_lumo():
    m = make_model("small256")
    n = m["n_occ"]
    H = ell_to_dense(m["H_col"], m["H_val"])
    w = np.linalg.eigvalsh(H)
    _, _, info = density_partitioned(m["H_col"], m["H_val"], n, 1e-5, 16)
    lo, hi = info["emin"], info["emax"]
    e = estimate_gap(info["traces"], info["branch"], n, lo, hi)
    _check_bracket(e, w, n, lo, hi, 0.05)


def test_sequence_from_estimate_gives_the_projector():
    m, H, X0, lo, hi = _dense("small256")
    n = m["n_occ"]
    _, info = sp2_partitioned([X0.copy()], [len(H)], n, 1e-10 * len(H) / 1024)
    e = estimate_gap(info["traces"], info["branch"], n, lo, hi)
    seq = sequence_from_gap(lo, hi, e["homo_bound"], e["lumo_bound"])
    xs, _ = sp2_partitioned([X0.copy()], [len(H)], n, 0.0, branch_in=seq)
    D, _, _ = density_exact(H, n)
    assert np.abs(xs[0] - D).max() < 1e-10


def test_estimate_needs_usable_iterates():
    info = _diag_expansion([-0.7, 0.4], 1)
    # one step: no clean iterate with a squaring before it on both sides
    with pytest.raises(ValueError):
        estimate_gap(info["traces"][:2], info["branch"][:1], 2, -2.0, 2.0)
    # a floor above every sum
    with pytest.raises(ValueError):
        estimate_gap(info["traces"], info["branch"], 2, -2.0, 2.0, floor=1.0)


def test_n18000_traces_bracket_the_levels():
    """The full-size system: the oracle's recorded traces (stored run) bracket the HOMO and LUMO
    of its dense diagonalisation (stored), within 3 % of the spectral range."""
    import json
    import os
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    ref = json.load(open(os.path.join(gdir, "n18000_fp64_partitioned.json")))
    lv = json.load(open(os.path.join(gdir, "n18000_levels.json")))
    assert ref["H_sha256"] == lv["H_sha256"]
    tr = [(float.fromhex(a), float.fromhex(b)) for a, b in ref["traces"]]
    br = [int(c) for c in ref["branch"]]
    lo, hi = float.fromhex(ref["emin"]), float.fromhex(ref["emax"])
    e = estimate_gap(tr, br, ref["n_occ"], lo, hi)
    eh, el = float.fromhex(lv["e_homo"]), float.fromhex(lv["e_lumo"])
    W = hi - lo
    assert e["homo_ratio"] <= eh <= e["homo_bound"]
    assert e["lumo_bound"] <= el <= e["lumo_ratio"]
    assert e["homo_bound"] - e["homo_ratio"] < 0.04 * W
    assert e["lumo_ratio"] - e["lumo_bound"] < 0.04 * W
