"""The partitioned oracle restricted to chosen cores (test infrastructure).

Eq. 6 makes the columns of D that belong to one core a function of that core's subgraph
alone once the branch sequence is fixed: subgraphs interact only through the summed traces
that choose each branch (SP2 paragraph after Eq. 7; the same sequence is applied to every
subgraph, MD section).  With the sequence of a whole-system oracle run, the D columns of any
chosen cores therefore follow from those cores' subgraphs only: the X2 graph rows of the core
vertices, the halo (Eq. 6, obs. vi), the gather of x0[s] and the replayed SP2 steps.  This is
the arithmetic of ``sp2.density_partitioned`` applied to fewer subgraphs, which makes
element-by-element comparisons of whole subgraphs affordable at sizes where the full oracle
takes many minutes.

Pin (tests/test_oracle_sp2.py): on the N = 1024 system, the columns of every chosen core equal
the whole-system oracle's D bit for bit.
"""
import numpy as np

from .bounds import gershgorin, x0_values
from .graph import graph_x2
from .sp2 import gather, sp2_partitioned


def core_subgraph(H_col, H_val, tau, emin, emax, verts):
    """sub_idx of a core: its vertices in the given order, then the halo ascending (every vertex
    outside the core adjacent to a core vertex in the X2 graph at ``tau``)."""
    verts = np.asarray(verts, dtype=np.int32)
    rows = graph_x2(H_col, H_val, tau, emin, emax, rows=verts)
    halo = np.setdiff1d(np.unique(np.concatenate(rows)), verts)
    return np.concatenate([verts, halo]).astype(np.int32)


def core_columns(H_col, H_val, n_occ, tau, cores, branch, n_refine=0, emin=None, emax=None):
    """D columns of the given cores (a list of vertex arrays, each ascending) under a fixed
    branch sequence.  Returns a list of (rows, vals): rows int32 [n] = the subgraph's vertices
    ascending (the column-ELL row indices), vals float64 [k, n] with vals[c, a] = D[rows[a],
    core[c]] (the column-ELL values of the core vertices)."""
    if emin is None or emax is None:
        emin, emax = gershgorin(H_col, H_val)
    x0 = x0_values(H_col, H_val, emin, emax)
    subs, blocks, kc = [], [], []
    for verts in cores:
        sub = core_subgraph(H_col, H_val, tau, emin, emax, verts)
        subs.append(sub)
        blocks.append(gather(H_col, x0, sub))
        kc.append(len(verts))
    xs, _ = sp2_partitioned(blocks, kc, n_occ, 0.0, branch_in=[int(b) for b in branch],
                            n_refine=n_refine, consume=True)
    out = []
    for sub, x, k in zip(subs, xs, kc):
        order = np.argsort(sub, kind="stable")
        out.append((sub[order], np.ascontiguousarray(x[order, :k].T)))
    return out
