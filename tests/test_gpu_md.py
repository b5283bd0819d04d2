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


def _narrowed(est, margin=0.05):
    """The bound bracket narrowed towards its centre by `margin` of its width (room for the
    levels to move between steps)."""
    hb, lb = est["homo_bound"], est["lumo_bound"]
    return hb + margin * (lb - hb), lb - margin * (lb - hb)


def test_md_with_the_sequence_from_the_estimated_gap():
    """The MD section's pre-determined sequence from the previous step's HOMO/LUMO estimate:
    the host estimator on the GPU's traces equals the oracle's on the same traces, and each step
    replays the sequence built from the narrowed bounds with no trace rule.  The replay converges,
    matches the oracle's replay of the same sequence, and agrees with the trace-driven D."""
    import torch
    import paper_1603_00937_amd as gb
    from synth import make_model, rebuild_hamiltonian, displace_sites
    from oracle.graph import graph_dprev
    from oracle.sp2 import density_partitioned
    from oracle.sequence import estimate_gap
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    m = make_model("small256")
    rng = np.random.default_rng(52)
    tau, tau_d, core = 1e-5, 1e-4, 16
    n = m["n_occ"]
    D_col, D_val, st = gb.density(dev(m["H_col"]), dev(m["H_val"]), n, tau, core_size=core)
    oc, ov = D_col.cpu().numpy(), D_val.cpu().numpy()
    pos = m["pos"]
    for step in range(3):
        inp = gb.gap_inputs(st, n)
        est = gb.sp2_estimate_gap(**inp)
        ref = estimate_gap(list(zip(inp["t1"], inp["t2"])), inp["branch"], n, inp["emin"],
                           inp["emax"])
        for k in ("homo_bound", "lumo_bound", "homo_ratio", "lumo_ratio"):
            assert abs(est[k] - ref[k]) <= 1e-12 * (inp["emax"] - inp["emin"]), (step, k)
        pos = displace_sites(pos, m["L"], 0.02, rng)
        m = rebuild_hamiltonian(m, pos)
        Hc, Hv = dev(m["H_col"]), dev(m["H_val"])
        lo, hi = gb.spectral_bounds(Hc, Hv)
        seq = gb.sp2_sequence(lo, hi, *_narrowed(est))
        og = graph_dprev(m["H_col"], m["H_val"], oc, ov, tau, tau_d)
        g = gb.build_graph(Hc, Hv, tau, mode="dprev", aux=(D_col, D_val), tau_aux=tau_d)
        p = gb.partition(g, core)
        D_col, D_val, st = gb.density(Hc, Hv, n, tau, partition=p, branch_in=seq)
        print(f"step {step + 1}: gap bracket homo [{est['homo_ratio']:.4f}, {est['homo_bound']:.4f}]"
              f" lumo [{est['lumo_bound']:.4f}, {est['lumo_ratio']:.4f}] sequence {len(seq)}"
              f" converged {st['converged']}")
        assert st["converged"], step
        rc, rv, _ = density_partitioned(m["H_col"], m["H_val"], n, tau, core, graph=og,
                                        branch_in=seq)
        assert np.array_equal(D_col.cpu().numpy(), rc)
        assert np.abs(D_val.cpu().numpy() - rv).max() <= 1e-9
        _, tv, _ = gb.density(Hc, Hv, n, tau, partition=p)
        assert np.abs(D_val.cpu().numpy() - tv.cpu().numpy()).max() <= 1e-7
        oc, ov = D_col.cpu().numpy(), D_val.cpu().numpy()


def test_gap_bracket_from_gpu_traces_n1024(model_cache):
    """The bracket from the GPU expansion's traces holds the eigensolver's HOMO and LUMO."""
    import torch
    import paper_1603_00937_amd as gb
    from oracle.bounds import ell_to_dense
    m = model_cache("n1024")
    n = m["n_occ"]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    _, _, st = gb.density(dev(m["H_col"]), dev(m["H_val"]), n, 1e-5, core_size=16)
    est = gb.sp2_estimate_gap(**gb.gap_inputs(st, n))
    w = np.linalg.eigvalsh(ell_to_dense(m["H_col"], m["H_val"]))
    W = st["emax"] - st["emin"]
    print(f"n1024: homo {w[n - 1]:.5f} in [{est['homo_ratio']:.5f}, {est['homo_bound']:.5f}], "
          f"lumo {w[n]:.5f} in [{est['lumo_bound']:.5f}, {est['lumo_ratio']:.5f}]")
    assert est["homo_ratio"] - 1e-6 * W <= w[n - 1] <= est["homo_bound"] + 1e-6 * W
    assert est["lumo_bound"] - 1e-6 * W <= w[n] <= est["lumo_ratio"] + 1e-6 * W
    assert est["homo_bound"] - est["homo_ratio"] < 0.05 * W
    assert est["lumo_ratio"] - est["lumo_bound"] < 0.05 * W
