"""Full-size parity (GPU): the N = 18000 and N = 100000 systems in the configuration the
benchmark times, against oracle outputs stored by tests/golden/make_golden.py (graph,
partition and D pattern by SHA-256; D values on 4096 sampled entries)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name, method="block"):
    tag = "partitioned" if method == "block" else method
    path = os.path.join(GOLDEN, f"{name}_fp64_{tag}.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle run for {name}")
    return json.load(open(path))


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available()
    import paper_1603_00937_amd as gb
    return gb


def _run(gb, name, precision, launch_mode="batched", method="block", **kw):
    import torch
    from synth import make_model, ell_sha256
    ref = _golden(name, method)
    m = make_model(name)
    assert ell_sha256(m["H_col"], m["H_val"]) == ref["H_sha256"], "inputs differ from the oracle's"
    Hc = torch.from_numpy(m["H_col"]).cuda()
    Hv = torch.from_numpy(m["H_val"]).cuda()
    lo, hi = gb.spectral_bounds(Hc, Hv)
    assert (lo.hex(), hi.hex()) == (ref["emin"], ref["emax"])
    g = gb.build_graph(Hc, Hv, ref["tau"])
    rp, cl = [t.cpu().numpy() for t in g.arrays()]
    assert ell_sha256(rp, cl) == ref["graph_sha256"]
    p = gb.partition(g, ref["core_size"], method=method)
    cp, sp, si = [t.cpu().numpy() for t in p.arrays()]
    assert ell_sha256(cp, sp, si) == ref["partition_sha256"]
    D_col, D_val, st = gb.density(Hc, Hv, m["n_occ"], ref["tau"], partition=p,
                                  core_size=ref["core_size"], precision=precision,
                                  launch_mode=launch_mode, **kw)
    dc = D_col.cpu().numpy()
    dv = D_val.cpu().numpy()
    assert ell_sha256(dc) == ref["D_col_sha256"]
    err = max(abs(dv[r, s] - float.fromhex(v)) for r, s, v in ref["samples"])
    print(f"{name} {precision}: iters={st['iters']} err={err:.3e} trace={st['trace']:.9f} "
          f"idem_max={st['idem_max']:.2e} ms={st['ms']}")
    return ref, st, err


def test_n18000_fp64(gb):
    ref, st, err = _run(gb, "n18000", "fp64")
    assert "".join(map(str, st["branch"])) == ref["branch"]
    assert st["iters"] == ref["iters"] and st["converged"]
    assert err <= 1e-9
    assert abs(st["trace"] - ref["trace_D"]) < 1e-8


def test_n18000_bf16x6(gb):
    """Split-bf16 squares (six plane products) plus FP64 McWeeny refinement meet the 1e-6
    bar with margin."""
    ref, st, err = _run(gb, "n18000", "bf16x6")
    assert st["converged"]
    assert err <= 1e-6


def test_n18000_fp16x3(gb):
    """Split-fp16 squares (two planes of the pre-scaled iterate, three products) plus FP64
    McWeeny refinement meet the 1e-6 bar."""
    ref, st, err = _run(gb, "n18000", "fp16x3")
    assert st["converged"]
    assert err <= 1e-6


@pytest.mark.parametrize("first", [0, 3])
def test_n18000_fp32(gb, first):
    """FP32 MFMA squares (blocked summation per 32-k chunk) plus FP64 McWeeny refinement, with
    and without the first steps in FP64, meet the 1e-6 bar."""
    ref, st, err = _run(gb, "n18000", "fp32", n_fp64_first=first)
    assert st["converged"]
    assert err <= 1e-6


def test_n18000_multilevel_fp64(gb):
    """Multilevel communities (cores of at most 32): partition index for index, branches and D
    against the oracle's run on the same communities."""
    ref, st, err = _run(gb, "n18000", "fp64", method="multilevel")
    assert "".join(map(str, st["branch"])) == ref["branch"]
    assert st["iters"] == ref["iters"] and st["converged"]
    assert err <= 1e-9


def test_n18000_multilevel_bf16x6(gb):
    ref, st, err = _run(gb, "n18000", "bf16x6", method="multilevel")
    assert st["converged"]
    assert err <= 1e-6


def test_n100000_fp64(gb):
    ref, st, err = _run(gb, "n100000", "fp64")
    assert "".join(map(str, st["branch"])) == ref["branch"]
    assert st["iters"] == ref["iters"] and st["converged"]
    assert err <= 1e-9


def test_n100000_bf16x6(gb):
    ref, st, err = _run(gb, "n100000", "bf16x6")
    assert st["converged"]
    assert err <= 1e-6


def test_n100000_sampled_graph_partition_and_properties(gb):
    """N = 100000 (clustered): the graph rows and subgraphs of sampled cores against the
    oracle computed row by row, and properties of D that hold at any size."""
    import torch
    from synth import make_model
    from oracle.bounds import gershgorin
    from oracle.graph import graph_x2
    m = make_model("n100000")
    Hc = torch.from_numpy(m["H_col"]).cuda()
    Hv = torch.from_numpy(m["H_val"]).cuda()
    assert gb.spectral_bounds(Hc, Hv) == gershgorin(m["H_col"], m["H_val"])
    g = gb.build_graph(Hc, Hv, 1e-5)
    rp, cl = [t.cpu().numpy() for t in g.arrays()]
    p = gb.partition(g, 32)
    cp, sp, si = [t.cpu().numpy() for t in p.arrays()]
    rng = np.random.default_rng(7)
    cores = rng.choice(len(cp) - 1, size=6, replace=False)
    emin, emax = gershgorin(m["H_col"], m["H_val"])
    for c in cores:
        verts = np.arange(cp[c], cp[c + 1])
        rows = graph_x2(m["H_col"], m["H_val"], 1e-5, emin, emax, rows=verts)
        for v, r in zip(verts, rows):
            assert np.array_equal(cl[rp[v]:rp[v + 1]], r), v
        halo = np.setdiff1d(np.unique(np.concatenate(rows)), verts)
        assert np.array_equal(si[sp[c]:sp[c + 1]], np.concatenate([verts, halo]))
    sizes = np.diff(sp)
    print(f"n100000: n_sub={len(sizes)} sizes min/mean/max = {sizes.min()}/{sizes.mean():.0f}/"
          f"{sizes.max()}, graph nnz={g.nnz}")
    D_col, D_val, st = gb.density(Hc, Hv, m["n_occ"], 1e-5, partition=p, precision="bf16x6",
                                  check_idem=True)
    print(f"n100000 bf16x6: iters={st['iters']} trace={st['trace']:.6f} idem={st['idem']:.2e} "
          f"idem_max={st['idem_max']:.2e} refine={st['n_refine_done']} ms={st['ms']}")
    assert st["converged"]
    assert abs(st["trace"] - m["n_occ"]) < 1e-3
    assert st["idem_max"] < 1e-8
    dc = D_col.cpu().numpy()
    for c in cores[:2]:
        sub = np.sort(si[sp[c]:sp[c + 1]])
        for v in range(cp[c], cp[c + 1]):
            assert np.array_equal(dc[v, :len(sub)], sub)


def test_n18000_gap_bracket_from_gpu_traces(gb):
    """The HOMO/LUMO bracket from the GPU expansion's traces holds the dense diagonalisation's
    levels (stored) and equals the oracle estimator's on the same traces."""
    from oracle.sequence import estimate_gap
    ref, st, err = _run(gb, "n18000", "fp64")
    lv = json.load(open(os.path.join(GOLDEN, "n18000_levels.json")))
    inp = gb.gap_inputs(st, ref["n_occ"])
    est = gb.sp2_estimate_gap(**inp)
    o = estimate_gap(list(zip(inp["t1"], inp["t2"])), inp["branch"], ref["n_occ"], inp["emin"],
                     inp["emax"])
    W = inp["emax"] - inp["emin"]
    for k in ("homo_bound", "lumo_bound", "homo_ratio", "lumo_ratio"):
        assert abs(est[k] - o[k]) <= 1e-12 * W
    eh, el = float.fromhex(lv["e_homo"]), float.fromhex(lv["e_lumo"])
    print(f"n18000: homo {eh:.5f} in [{est['homo_ratio']:.5f}, {est['homo_bound']:.5f}], "
          f"lumo {el:.5f} in [{est['lumo_bound']:.5f}, {est['lumo_ratio']:.5f}]")
    assert est["homo_ratio"] <= eh <= est["homo_bound"]
    assert est["lumo_bound"] <= el <= est["lumo_ratio"]


def test_n100000_multilevel_fp64(gb):
    """The heterogeneous system on multilevel communities: partition index for index, branches
    and D against the oracle's run on the same communities."""
    ref, st, err = _run(gb, "n100000", "fp64", method="multilevel")
    assert "".join(map(str, st["branch"])) == ref["branch"]
    assert st["iters"] == ref["iters"] and st["converged"]
    assert err <= 1e-9


def test_n100000_multilevel_bf16x6(gb):
    ref, st, err = _run(gb, "n100000", "bf16x6", method="multilevel")
    assert st["converged"]
    assert err <= 1e-6


@pytest.mark.parametrize("name,method", [("n18000", "block"), ("n100000", "multilevel")])
def test_hash_vertex_sets_give_the_same_graph_and_partition(gb, name, method, monkeypatch):
    """The graph and halo kernels on LDS hash sets (forced here; the default above 2^17
    vertices) against the oracle's stored graph and partition: bit for bit."""
    import torch
    from synth import make_model, ell_sha256
    ref = _golden(name, method)
    m = make_model(name)
    Hc = torch.from_numpy(m["H_col"]).cuda()
    Hv = torch.from_numpy(m["H_val"]).cuda()
    monkeypatch.setenv("GB_VERTEX_SETS", "hash")
    g = gb.build_graph(Hc, Hv, ref["tau"])
    rp, cl = [t.cpu().numpy() for t in g.arrays()]
    assert ell_sha256(rp, cl) == ref["graph_sha256"]
    p = gb.partition(g, ref["core_size"], method=method)
    cp, sp, si = [t.cpu().numpy() for t in p.arrays()]
    assert ell_sha256(cp, sp, si) == ref["partition_sha256"]


def test_n500000_graph_and_halos_beyond_the_bitmaps(gb):
    """N = 500000 (250000 sites), past the n-bit LDS bitmaps: the graph rows and subgraphs of
    sampled cores against the oracle computed row by row, and the graph's symmetry."""
    import time
    import torch
    from synth import make_model
    from oracle.bounds import gershgorin
    from oracle.graph import graph_x2
    m = make_model("n500000")
    Hc = torch.from_numpy(m["H_col"]).cuda()
    Hv = torch.from_numpy(m["H_val"]).cuda()
    emin, emax = gershgorin(m["H_col"], m["H_val"])
    assert gb.spectral_bounds(Hc, Hv) == (emin, emax)
    torch.cuda.synchronize()
    t0 = time.time()
    g = gb.build_graph(Hc, Hv, 1e-5)
    p = gb.partition(g, 32)
    torch.cuda.synchronize()
    dt = time.time() - t0
    rp, cl = [t.cpu().numpy() for t in g.arrays()]
    cp, sp, si = [t.cpu().numpy() for t in p.arrays()]
    sizes = np.diff(sp)
    print(f"n500000: graph nnz {g.nnz}, {len(sizes)} subgraphs of {sizes.min()}..{sizes.max()} "
          f"vertices, graph + partition {dt * 1e3:.0f} ms")
    rng = np.random.default_rng(11)
    for c in rng.choice(len(cp) - 1, size=6, replace=False):
        verts = np.arange(cp[c], cp[c + 1])
        rows = graph_x2(m["H_col"], m["H_val"], 1e-5, emin, emax, rows=verts)
        for v, r in zip(verts, rows):
            assert np.array_equal(cl[rp[v]:rp[v + 1]], r), v
        halo = np.setdiff1d(np.unique(np.concatenate(rows)), verts)
        assert np.array_equal(si[sp[c]:sp[c + 1]], np.concatenate([verts, halo]))
    # symmetric: the transposed pattern equals the pattern
    r = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    a = np.sort(r.astype(np.int64) * (len(rp) - 1) + cl)
    b = np.sort(cl.astype(np.int64) * (len(rp) - 1) + r)
    assert np.array_equal(a, b)
