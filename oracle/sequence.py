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

Pins (tests): a sequence from the eigensolver's HOMO and LUMO replays (dense SP2) to the
eigensolver's projector; the propagated distances match the images of those eigenvalues under
the composed polynomial.
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
