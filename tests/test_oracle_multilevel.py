"""Pins for the multilevel community oracle (cores of at most cap vertices aimed at the summed
cubed subgraph sizes), and the host entry point of the library against it index for index.
CPU only."""
import numpy as np
import pytest

from synth import make_model
from oracle.graph import graph_x2
from oracle.partition import halo_subgraphs, partition
from oracle.multilevel import partition_multilevel, splitmix64


def _csr(rows):
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate([np.sort(np.asarray(r, dtype=np.int32)) for r in rows])
    return rp, col


def _cost(rp, col, cp, cv):
    cores = [cv[cp[i]:cp[i + 1]] for i in range(len(cp) - 1)]
    sp, _ = halo_subgraphs(rp, col, cores)
    return int((np.diff(sp).astype(np.int64) ** 3).sum())


def _check_valid(n, cp, cv, cap):
    assert cp[0] == 0 and cp[-1] == n
    sizes = np.diff(cp)
    assert sizes.min() >= 1 and sizes.max() <= cap
    assert np.array_equal(np.sort(cv), np.arange(n))
    for i in range(len(cp) - 1):
        c = cv[cp[i]:cp[i + 1]]
        assert np.all(np.diff(c) > 0)
    firsts = [cv[cp[i]] for i in range(len(cp) - 1)]
    assert firsts == sorted(firsts)


def test_splitmix64_reference_values():
    # the published generator seeded with 0 yields these first outputs (state += golden gamma)
    g = 0x9E3779B97F4A7C15
    outs = [splitmix64((k * g) & ((1 << 64) - 1)) for k in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def _cliques(n_cliques, size, perm=None):
    n = n_cliques * size
    lab = np.arange(n) if perm is None else perm
    rows = [[] for _ in range(n)]
    for c in range(n_cliques):
        members = [int(lab[c * size + i]) for i in range(size)]
        for a in members:
            rows[a] = members
    return rows


@pytest.mark.parametrize("relabel", [False, True])
def test_disjoint_cliques_are_found(relabel):
    perm = np.random.default_rng(3).permutation(40) if relabel else None
    rp, col = _csr(_cliques(5, 8, perm))
    cp, cv, cost = partition_multilevel(rp, col, 8)
    _check_valid(40, cp, cv, 8)
    got = sorted(tuple(cv[cp[i]:cp[i + 1]]) for i in range(len(cp) - 1))
    lab = np.arange(40) if perm is None else perm
    want = sorted(tuple(sorted(int(lab[c * 8 + i]) for i in range(8))) for c in range(5))
    assert got == want
    assert cost == 5 * 8 ** 3      # no halos


def test_path_is_cut_into_runs():
    n = 30
    rows = [[j for j in (i - 1, i, i + 1) if 0 <= j < n] for i in range(n)]
    rp, col = _csr(rows)
    cp, cv, cost = partition_multilevel(rp, col, 6)
    _check_valid(n, cp, cv, 6)
    for i in range(len(cp) - 1):
        c = cv[cp[i]:cp[i + 1]]
        assert c[-1] - c[0] == len(c) - 1      # consecutive vertices
    assert cost == _cost(rp, col, cp, cv)


@pytest.mark.parametrize("name,cap", [("tiny48", 5), ("small256", 16), ("small256", 7)])
def test_valid_cores_and_reported_cost(name, cap):
    m = make_model(name)
    rp, col = graph_x2(m["H_col"], m["H_val"], 1e-5)
    cp, cv, cost = partition_multilevel(rp, col, cap)
    _check_valid(len(rp) - 1, cp, cv, cap)
    assert cost == _cost(rp, col, cp, cv)


def test_cheaper_than_blocks_and_independent_of_numbering():
    """On the N = 1024 model the communities cost less than blocks of the (already spatially
    sorted) vertex order, and a random relabelling of the graph costs about the same, where
    blocks of the relabelled order lose all locality."""
    m = make_model("n1024")
    rp, col = graph_x2(m["H_col"], m["H_val"], 1e-5)
    n = len(rp) - 1
    _, _, sp, _ = partition(rp, col, 16)
    block_cost = int((np.diff(sp).astype(np.int64) ** 3).sum())
    _, _, cost = partition_multilevel(rp, col, 16)
    assert cost < block_cost
    perm = np.random.default_rng(5).permutation(n)
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    rows = [inv[col[rp[perm[i]]:rp[perm[i] + 1]]] for i in range(n)]
    rp2, col2 = _csr(rows)
    _, _, cost2 = partition_multilevel(rp2, col2, 16)
    _, _, sp2, _ = partition(rp2, col2, 16)
    shuffled_block = int((np.diff(sp2).astype(np.int64) ** 3).sum())
    assert abs(cost2 - cost) < 0.1 * cost
    assert cost2 < shuffled_block


@pytest.mark.parametrize("name,cap", [("tiny48", 5), ("tiny48", 16), ("small256", 16),
                                      ("small256", 7), ("n1024", 32), ("n4096", 32)])
def test_library_host_entry_point_matches_oracle(name, cap):
    """n4096 is large enough for the library to build its coarse graphs on several threads."""
    import paper_1603_00937_amd as gb
    m = make_model(name)
    rp, col = graph_x2(m["H_col"], m["H_val"], 1e-5)
    ocp, ocv, ocost = partition_multilevel(rp, col, cap)
    ccp, ccv, ccost = gb.partition_host(rp, col, cap)
    assert np.array_equal(ocp, ccp) and np.array_equal(ocv, ccv)
    assert ocost == ccost


def test_library_host_buffers_reused_across_graphs():
    """The library keeps its coarse graphs and candidate lists between calls: calls on graphs
    of different sizes, in an order that shrinks and regrows them, each give the oracle's
    cores."""
    import paper_1603_00937_amd as gb
    graphs = {}
    for name in ("small256", "tiny48", "n1024", "small256"):
        if name not in graphs:
            m = make_model(name)
            rp, col = graph_x2(m["H_col"], m["H_val"], 1e-5)
            graphs[name] = (rp, col, partition_multilevel(rp, col, 16))
        rp, col, (ocp, ocv, ocost) = graphs[name]
        ccp, ccv, ccost = gb.partition_host(rp, col, 16)
        assert np.array_equal(ocp, ccp) and np.array_equal(ocv, ccv) and ocost == ccost, name
    gb.trim()  # releases the idle buffer sets; the next call allocates afresh
    rp, col, (ocp, ocv, ocost) = graphs["tiny48"]
    ccp, ccv, ccost = gb.partition_host(rp, col, 16)
    assert np.array_equal(ocp, ccp) and np.array_equal(ocv, ccv) and ocost == ccost


def test_library_host_concurrent_calls():
    """Calls from several host threads at once (one uses the library's worker pool, the others
    start threads of their own) each give the oracle's cores."""
    import threading
    import paper_1603_00937_amd as gb
    m = make_model("n1024")
    rp, col = graph_x2(m["H_col"], m["H_val"], 1e-5)
    ocp, ocv, ocost = partition_multilevel(rp, col, 32)
    results = [None] * 4

    def run(i):
        results[i] = gb.partition_host(rp, col, 32)

    threads = [threading.Thread(target=run, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for ccp, ccv, ccost in results:
        assert np.array_equal(ocp, ccp) and np.array_equal(ocv, ccv) and ocost == ccost


def test_library_host_entry_point_rejects_bad_arguments():
    import paper_1603_00937_amd as gb
    rp, col = _csr(_cliques(2, 4))
    with pytest.raises(gb.GbError):
        gb.partition_host(rp, col, 0)
    bad = col.copy()
    bad[3] = 99
    with pytest.raises(gb.GbError):
        gb.partition_host(rp, bad, 4)


def _displaced(name, steps=1, seed=52):
    from synth import displace_sites, rebuild_hamiltonian
    m = make_model(name)
    rng = np.random.default_rng(seed)
    pos = m["pos"]
    for _ in range(steps):
        pos = displace_sites(pos, m["L"], 0.02, rng)
        m = rebuild_hamiltonian(m, pos)
    return m


@pytest.mark.parametrize("start", ["multilevel", "block"])
def test_update_carries_the_cores(start):
    """Cores carried to the graph of a displaced system: the same vertex sets, their cost there
    recomputed from the halos, and the library's host entry point gives the same cores."""
    import paper_1603_00937_amd as gb
    from oracle.multilevel import partition_update
    m0 = make_model("small256")
    rp0, col0 = graph_x2(m0["H_col"], m0["H_val"], 1e-5)
    if start == "multilevel":
        pcp, pcv, _ = partition_multilevel(rp0, col0, 16)
    else:
        pcp, pcv, _, _ = partition(rp0, col0, 16)
    m1 = _displaced("small256", 3)
    rp1, col1 = graph_x2(m1["H_col"], m1["H_val"], 1e-5)
    cp, cv, cost = partition_update(rp1, col1, pcp, pcv)
    _check_valid(len(rp1) - 1, cp, cv, 16)
    before = sorted(tuple(pcv[pcp[i]:pcp[i + 1]]) for i in range(len(pcp) - 1))
    after = sorted(tuple(cv[cp[i]:cp[i + 1]]) for i in range(len(cp) - 1))
    assert before == after
    assert cost == _cost(rp1, col1, cp, cv)
    ccp, ccv, ccost = gb.partition_update_host(rp1, col1, pcp, pcv)
    assert np.array_equal(cp, ccp) and np.array_equal(cv, ccv) and cost == ccost


def test_update_rejects_a_bad_cover():
    import paper_1603_00937_amd as gb
    rp, col = _csr(_cliques(2, 4))
    with pytest.raises(gb.GbError):
        gb.partition_update_host(rp, col, np.array([0, 4, 8]), np.array([0, 1, 2, 3, 4, 5, 6, 6]))
    with pytest.raises(gb.GbError):
        gb.partition_update_host(rp, col, np.array([0, 4, 7]), np.arange(8))
