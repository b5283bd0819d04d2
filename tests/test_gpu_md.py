"""Adaptive graph along a displacement trajectory (GPU): each step derives the graph from the
previous step's D and the new H (the MD graph estimate after Eq. 8), and must match the oracle
bit for bit; D within 1e-9."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_three_md_steps_match_oracle():
    import torch
    import paper_1603_00937_amd as gb
    from synth import make_model, rebuild_hamiltonian, displace_sites
    from oracle.graph import graph_dprev
    from oracle.sp2 import density_partitioned
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    m = make_model("small256")
    rng = np.random.default_rng(52)
    tau, tau_d, core = 1e-5, 1e-4, 16
    oc, ov, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], tau, core)
    D_col, D_val, st = gb.density(dev(m["H_col"]), dev(m["H_val"]), m["n_occ"], tau, core_size=core)
    pos = m["pos"]
    for step in range(3):
        pos = displace_sites(pos, m["L"], 0.02, rng)
        m = rebuild_hamiltonian(m, pos)
        og = graph_dprev(m["H_col"], m["H_val"], oc, ov, tau, tau_d)
        oc, ov, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], tau, core, graph=og)
        g = gb.build_graph(dev(m["H_col"]), dev(m["H_val"]), tau, mode="dprev",
                           aux=(D_col, D_val), tau_aux=tau_d)
        rp, cl = [t.cpu().numpy() for t in g.arrays()]
        assert np.array_equal(rp, og[0]) and np.array_equal(cl, og[1]), step
        p = gb.partition(g, core)
        D_col, D_val, st = gb.density(dev(m["H_col"]), dev(m["H_val"]), m["n_occ"], tau,
                                      partition=p, core_size=core)
        assert st["branch"] == info["branch"], step
        assert np.array_equal(D_col.cpu().numpy(), oc)
        assert np.abs(D_val.cpu().numpy() - ov).max() <= 1e-9


def test_md_with_the_previous_sequence_replayed():
    """The MD section's pre-determined sequence: each step replays the branch sequence the
    previous step chose, with one X^2 / 2X - X^2 pair appended as a margin (no trace exchange
    during the expansion; the pair leaves a converged X unchanged).  The replay converges, matches
    the oracle's replay of the same sequence, and agrees with the trace-driven D of the same
    step to the accuracy of the stop rule."""
    import torch
    import paper_1603_00937_amd as gb
    from synth import make_model, rebuild_hamiltonian, displace_sites
    from oracle.graph import graph_dprev
    from oracle.sp2 import density_partitioned
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    m = make_model("small256")
    rng = np.random.default_rng(52)
    tau, tau_d, core = 1e-5, 1e-4, 16
    D_col, D_val, st = gb.density(dev(m["H_col"]), dev(m["H_val"]), m["n_occ"], tau, core_size=core)
    seq = st["branch"] + [0, 1]
    oc, ov = D_col.cpu().numpy(), D_val.cpu().numpy()
    pos = m["pos"]
    for step in range(3):
        pos = displace_sites(pos, m["L"], 0.02, rng)
        m = rebuild_hamiltonian(m, pos)
        og = graph_dprev(m["H_col"], m["H_val"], oc, ov, tau, tau_d)
        g = gb.build_graph(dev(m["H_col"]), dev(m["H_val"]), tau, mode="dprev",
                           aux=(D_col, D_val), tau_aux=tau_d)
        p = gb.partition(g, core)
        D_col, D_val, st = gb.density(dev(m["H_col"]), dev(m["H_val"]), m["n_occ"], tau,
                                      partition=p, branch_in=seq)
        rc, rv, rinfo = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], tau, core,
                                            graph=og, branch_in=seq)
        assert st["converged"], step
        assert np.array_equal(D_col.cpu().numpy(), rc)
        assert np.abs(D_val.cpu().numpy() - rv).max() <= 1e-9
        _, tv, tst = gb.density(dev(m["H_col"]), dev(m["H_val"]), m["n_occ"], tau, partition=p)
        assert np.abs(D_val.cpu().numpy() - tv.cpu().numpy()).max() <= 1e-7
        oc, ov = D_col.cpu().numpy(), D_val.cpu().numpy()
        seq = tst["branch"] + [0, 1]
