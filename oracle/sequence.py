"""Pre-determined SP2 sequences from HOMO/LUMO estimates (oracle).

In MD the paper fixes the whole SP2 branch sequence of a step in advance, from the HOMO-LUMO gap
estimated at the previous step (MD section, following Rubensson and Niklasson's interior
eigenvalue estimates), so every subgraph expansion runs without exchanging traces.

Sequence from a gap.  In X0 = (e_max I - H)/(e_max - e_min) the HOMO maps to x_h and the LUMO to
x_l < x_h; their distances from the targets are u = 1 - x_h and v = x_l.  X <- X^2 squares v and
takes u to 2u - u^2; X <- 2X - X^2 squares u and takes v to 2v - v^2.  Each step takes the branch
that squares the larger of the two (X^2 when v > u, ties to 2X - X^2) and the sequence ends once
both are at most delta.  Applied to a matrix whose spectrum has no eigenvalue strictly inside
(e_homo, e_lumo) the sequence drives every eigenvalue to 0 or 1 and so yields the projector onto
the states below the gap.

Gap from an expansion's traces.  The MD section takes the next step's sequence from HOMO/LUMO
estimates made during the previous step's expansion (the interior-eigenvalue estimates of
Rubensson and Niklasson).  This estimator uses only the core traces t1 = Tr X_i and t2 = Tr X_i^2
that the trace rule already computes, so it costs no products.  With v_k = x_k for the
unoccupied and u_k = 1 - x_k for the occupied eigenvalues and g(x) = x - x^2/2,
  L_i = (t1 - t2 + t1 - n_occ)/2 = sum_unocc g(v_k) - sum_occ u_k^2/2,
  U_i = (t1 - t2 - t1 + n_occ)/2 = sum_occ g(u_k) - sum_unocc v_k^2/2.
Right after a step 2X - X^2 the u_k were just squared, so there L_i = sum_unocc g(v_k) up to
fourth order in u ("clean" iterates of the v side); right after a step X^2 the same holds for U_i.
Two estimates of the LUMO image v (the largest v_k) come from the clean iterates:
  bound: g(v) <= sum g(v_k) = L_i + sum u_k^2/2 <= L_i + U_i^2/2, so v <= g^-1(L_i + U_i^2/2),
         an image at or beyond the LUMO's, towards the gap centre;
  ratio: for two clean iterates i < j with a squaring of v between them, L_j/L_i is a
         g-weighted mean of g(F(v_k))/g(v_k) (F the composed branch maps, and g(F(v))/g(v)
         increases with v), at most that of the LUMO; solving g(F(v))/g(v) = L_j/L_i by
         bisection gives an image at or short of the LUMO's, away from the gap centre.
The two bracket the LUMO image; the U side brackets the HOMO the same way.  The inverse branch
maps (a squaring: d -> sqrt(d); the other branch: d -> d / (1 + sqrt(1 - d)) on the distance d)
take them back to step 0; every square root halves the relative error, so the latest clean
iterates whose sums are above a noise floor give the tightest bracket.  The default floor is
10 times the last iterate's |t1 - n_occ| + |t1 - t2| (the rounding and truncation level of
partitioned traces), and at least 1e-12 n_occ.  A sequence built from the bound is long enough
for the expansion the traces came from.

Pins (tests): a sequence from the eigensolver's HOMO and LUMO replays (dense SP2) to the
eigensolver's projector; the propagated distances match the images of those eigenvalues under
the composed polynomial; the bound and ratio estimates from an expansion's traces bracket the
eigensolver's HOMO and LUMO (two-level spectra with multiplicities, where both are within
rounding of the levels, dense models and partitioned ones) within a stated width, and a
sequence built from the bounds replays to the projector.
"""
import numpy as np


def sequence_from_gap(emin, emax, e_homo, e_lumo, delta=1e-12, max_len=127):
    """Branch list (0: X^2, 1: 2X - X^2) for the mapped HOMO/LUMO pair."""
    u = 1.0 - (emax - e_homo) / (emax - emin)
    v = (emax - e_lumo) / (emax - emin)
    if not (0.0 < v < 1.0 - u < 1.0):
        raise ValueError("need e_min < e_homo < e_lumo < e_max")
    out = []
    while (u > delta or v > delta) and len(out) < max_len:
        if v > u:
            out.append(0)
            u, v = 2.0 * u - u * u, v * v
        else:
            out.append(1)
            u, v = u * u, 2.0 * v - v * v
    return out


def propagate(u0, v0, branches):
    """(u_i, v_i) for i = 0 .. len(branches)."""
    us, vs = [u0], [v0]
    u, v = u0, v0
    for b in branches:
        if b == 0:
            u, v = 2.0 * u - u * u, v * v
        else:
            u, v = u * u, 2.0 * v - v * v
        us.append(u)
        vs.append(v)
    return np.array(us), np.array(vs)


def _forward(d, branches, side):
    """Distance d of an eigenvalue image from its target taken through the given branches."""
    for b in branches:
        squares = (b == 0) if side == "v" else (b == 1)
        d = d * d if squares else 2.0 * d - d * d
    return d


def _back_to_x0(d, branches, k, side):
    """Distance d at step k (side "v": from 0, "u": from 1) mapped back through
    branches[k-1], ..., branches[0] to the distance at step 0."""
    for b in reversed(branches[:k]):
        squares = (b == 0) if side == "v" else (b == 1)
        if squares:
            d = np.sqrt(d)          # this branch squared the distance
        else:
            d = d / (1.0 + np.sqrt(1.0 - d))   # this branch took d to 2d - d^2
    return d


def _g(x):
    return x - 0.5 * x * x


def _solve_ratio(rho, seg, side, n_bisect=200):
    """x in (0, 1) with g(F(x)) = rho g(x), F the maps of the branches in seg (bisection)."""
    lo, hi = 0.0, 1.0
    for _ in range(n_bisect):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if _g(_forward(mid, seg, side)) - rho * _g(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def default_floor(traces, n_occ):
    t1, t2 = traces[-1]
    return max(10.0 * (abs(t1 - n_occ) + abs(t1 - t2)), 1e-12 * n_occ)


def estimate_gap(traces, branches, n_occ, emin, emax, floor=None):
    """HOMO/LUMO estimates from the core traces of an SP2 expansion.

    traces: (t1_i, t2_i) for i = 0 .. len(branches) (entry i: the iterate before update i);
    branches[i]: update i (0: X^2, 1: 2X - X^2).  Returns a dict with the bounds
    ``homo_bound`` >= e_homo and ``lumo_bound`` <= e_lumo (between the levels and the gap centre),
    the ratio estimates ``homo_ratio`` <= e_homo and ``lumo_ratio`` >= e_lumo, the floor and
    the iterates used (bound, ratio pair).  Raises ValueError when a side has no clean iterate above the floor."""
    nb = len(branches)
    if len(traces) < nb + 1:
        raise ValueError("need the traces of every iterate up to the last update")
    traces = traces[:nb + 1]
    if floor is None or floor <= 0.0:
        floor = default_floor(traces, n_occ)
    t1 = np.array([t[0] for t in traces])
    t2 = np.array([t[1] for t in traces])
    A = t1 - t2
    B = t1 - n_occ
    sums = {"v": 0.5 * (A + B), "u": 0.5 * (A - B)}
    w = emax - emin
    out = {"floor": floor}
    for side, other in (("v", "u"), ("u", "v")):
        S, So = sums[side], sums[other]
        sq = 0 if side == "v" else 1          # the branch that squares this side
        clean = [i for i in range(1, nb + 1) if branches[i - 1] != sq]
        # bound: the latest clean iterate with its sum in (floor, 1/2)
        ib = None
        for i in clean:
            val = S[i] + 0.5 * So[i] * So[i]
            if S[i] > floor and val < 0.5:
                ib = i
        if ib is None:
            raise ValueError("no clean iterate above the noise floor")
        val = S[ib] + 0.5 * So[ib] * So[ib]
        d = 2.0 * val / (1.0 + np.sqrt(1.0 - 2.0 * val))      # g^-1(val)
        d_bound = _back_to_x0(d, branches, ib, side)
        # ratio: the latest pair of clean iterates with a squaring between, later sum > floor
        pair = None
        for a, i in enumerate(clean):
            for j in clean[a + 1:]:
                if sq in branches[i:j]:
                    if S[j] > floor and S[i] > S[j]:
                        pair = (i, j)
                    break
        if pair is None:
            raise ValueError("no pair of clean iterates above the noise floor")
        i, j = pair
        d = _solve_ratio(S[j] / S[i], branches[i:j], side)
        d_ratio = _back_to_x0(d, branches, i, side)
        if side == "v":
            out["lumo_bound"] = emax - d_bound * w
            out["lumo_ratio"] = emax - d_ratio * w
            out["lumo_iterates"] = (ib, i, j)
        else:
            out["homo_bound"] = emax - (1.0 - d_bound) * w
            out["homo_ratio"] = emax - (1.0 - d_ratio) * w
            out["homo_iterates"] = (ib, i, j)
    return out
