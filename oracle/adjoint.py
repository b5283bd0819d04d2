"""Reverse-mode derivative of L = Tr[D V] through the partitioned SP2 expansion (oracle).

Observables are traces with D (<A> = Tr[D A], end of the SP2 paragraph after Eq. 7).  The
derivative with respect to H follows the recursion backwards with the graph, the
partition, the spectral bounds and the branch sequence held fixed:
  * seed: for each subgraph, Gbar_K[a, j] = dL/dD[sub_a, sub_j] on its core columns j, 0 on
    the halo columns; only the symmetric part matters because every X_n is symmetric, so
    Gbar is symmetrised once and stays symmetric;
  * step X <- X^2:       Gbar <- Gbar X + X Gbar
    step X <- 2X - X^2:  Gbar <- 2 Gbar - (Gbar X + X Gbar)
  * start X0 = (e_max I - h)/(e_max - e_min): dL/dh = -Gbar_0 / (e_max - e_min);
  * assembly: the derivative for one ELL slot (i, j) of H is the sum over every subgraph
    holding both i and j of its entry, in ascending subgraph order.  It is the symmetric
    (per-slot) gradient: perturbing H_ij and H_ji together by h changes L by
    h (G_ij + G_ji).

Pins (tests): central finite differences of the frozen forward map; for the whole-matrix
expansion, the eigen-decomposition (Daleckii-Krein) derivative of the exact projector.
"""
import numpy as np

from .sp2 import sp2_partitioned


def seed_from_column_ell(G_col, G_val, sub_ptr, sub_idx, core_counts, sizes):
    """Gbar_K per subgraph from dL/dD given on D's column-ELL pattern."""
    out = []
    for s in range(len(sub_ptr) - 1):
        idx = sub_idx[sub_ptr[s]:sub_ptr[s + 1]]
        n = len(idx)
        loc = {int(v): a for a, v in enumerate(idx)}
        G = np.zeros((n, n))
        for j in range(core_counts[s]):
            i = int(idx[j])
            rows = G_col[i]
            for t in range(len(rows)):
                r = int(rows[t])
                if r >= 0 and r in loc:
                    G[loc[r], j] = G_val[i, t]
        out.append(0.5 * (G + G.T))
    return out


def reverse_sp2(tape, branches, seeds):
    """Gbar_0 per subgraph from the stored iterates X_0 .. X_K (tape[n][s])."""
    G = [g.copy() for g in seeds]
    for n in range(len(branches) - 1, -1, -1):
        X = tape[n]
        newG = []
        for g, x in zip(G, X):
            p = g @ x + x @ g
            newG.append(p if branches[n] == 0 else 2.0 * g - p)
        G = newG
    return G


def assemble_grad_h(H_col, G0, sub_ptr, sub_idx, emin, emax):
    """Per-slot symmetric gradient on H's ELL pattern."""
    N, W = H_col.shape
    G_H = np.zeros((N, W))
    scale = -1.0 / (emax - emin)
    for s in range(len(sub_ptr) - 1):
        idx = sub_idx[sub_ptr[s]:sub_ptr[s + 1]]
        loc = np.full(N, -1, dtype=np.int64)
        loc[idx] = np.arange(len(idx))
        rows = idx
        cols = H_col[rows]
        la = np.repeat(np.arange(len(idx))[:, None], W, axis=1)
        lb = np.where(cols >= 0, loc[np.where(cols >= 0, cols, 0)], -1)
        ok = lb >= 0
        r_a, t_a = np.nonzero(ok)
        G_H[rows[r_a], t_a] += scale * G0[s][la[r_a, t_a], lb[r_a, t_a]]
    return G_H


def trace_dv_and_grad(model_H_col, model_H_val, V_val, n_occ, info, blocks0):
    """L = Tr[D V] and its per-slot gradient for a partitioned run ``info`` (from
    oracle.sp2.density_partitioned with keep_tape=True)."""
    H_col = model_H_col
    sub_ptr, sub_idx, core_ptr = info["sub_ptr"], info["sub_idx"], info["core_ptr"]
    kc = np.diff(core_ptr)
    tape = info["tape"]
    XK = tape[-1]
    # dL/dD[r, i] = V[i, r] = V[r, i]; on D's pattern only the entries of V's pattern count
    seeds = []
    L = 0.0
    N = H_col.shape[0]
    for s in range(len(sub_ptr) - 1):
        idx = sub_idx[sub_ptr[s]:sub_ptr[s + 1]]
        n = len(idx)
        loc = np.full(N, -1, dtype=np.int64)
        loc[idx] = np.arange(n)
        G = np.zeros((n, n))
        for j in range(kc[s]):
            i = idx[j]
            c = H_col[i]
            ok = c >= 0
            la = loc[c[ok]]
            m = la >= 0
            G[la[m], j] = V_val[i][ok][m]
        L += float(np.sum(G * XK[s]))
        seeds.append(0.5 * (G + G.T))
    G0 = reverse_sp2(tape, info["branch"], seeds)
    return L, assemble_grad_h(H_col, G0, sub_ptr, sub_idx, info["emin"], info["emax"])


def frozen_trace_dv(H_col, H_val, V_val, info, i, j, h):
    """Tr[D V] after perturbing H_ij and H_ji by h, with graph, partition, bounds and branch
    sequence frozen.  Only subgraphs holding both i and j change; returns the change of L."""
    from .bounds import x0_values
    from .sp2 import gather
    sub_ptr, sub_idx, core_ptr = info["sub_ptr"], info["sub_idx"], info["core_ptr"]
    kc = np.diff(core_ptr)
    N, W = H_col.shape
    Hv = H_val.copy()
    ti = np.nonzero(H_col[i] == j)[0]
    tj = np.nonzero(H_col[j] == i)[0]
    Hv[i, ti] += h
    if i != j:
        Hv[j, tj] += h
    x0p = x0_values(H_col, Hv, info["emin"], info["emax"])
    x0o = x0_values(H_col, H_val, info["emin"], info["emax"])
    dL = 0.0
    for s in range(len(sub_ptr) - 1):
        idx = sub_idx[sub_ptr[s]:sub_ptr[s + 1]]
        if not (np.any(idx == i) and np.any(idx == j)):
            continue
        outs = []
        for x0 in (x0p, x0o):
            xs, _ = sp2_partitioned([gather(H_col, x0, idx)], [kc[s]], 0, 0.0,
                                    branch_in=info["branch"])
            outs.append(xs[0])
        n = len(idx)
        loc = np.full(N, -1, dtype=np.int64)
        loc[idx] = np.arange(n)
        G = np.zeros((n, n))
        for a in range(kc[s]):
            r = idx[a]
            c = H_col[r]
            ok = c >= 0
            la = loc[c[ok]]
            m = la >= 0
            G[la[m], a] = V_val[r][ok][m]
        dL += float(np.sum(G * (outs[0] - outs[1])))
    return dL


def daleckii_krein_grad(H, V, n_occ):
    """Symmetric gradient of Tr[D V] for the exact projector D (eigen-perturbation)."""
    w, P = np.linalg.eigh(H)
    Vt = P.T @ V @ P
    F = np.zeros_like(H)
    occ = np.arange(n_occ)
    vir = np.arange(n_occ, H.shape[0])
    F[np.ix_(vir, occ)] = 1.0 / (w[occ][None, :] - w[vir][:, None])
    F = F + F.T
    return P @ (Vt * F) @ P.T
