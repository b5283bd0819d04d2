"""Parity of the HIP path with the CPU oracle (GPU).

Index results (graph, partition, D pattern) must match bit for bit; FP64 D within 1e-9
max-abs with the identical branch sequence and iteration count."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FP64_TOL = 1e-9


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_1603_00937_amd as gb
    return gb


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(*ts):
    return [t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("name", ["tiny48", "small256", "n1024"])
def test_bounds_bit_exact(gb, model_cache, name):
    from oracle.bounds import gershgorin
    m = model_cache(name)
    lo, hi = gb.spectral_bounds(_dev(m["H_col"]), _dev(m["H_val"]))
    assert (lo, hi) == gershgorin(m["H_col"], m["H_val"])


@pytest.mark.parametrize("name,tau", [("tiny48", 1e-2), ("tiny48", 1e-3), ("tiny48", 0.0),
                                      ("small256", 1e-3), ("small256", 1e-5),
                                      ("n1024", 1e-5)])
def test_x2_graph_bit_exact(gb, model_cache, name, tau):
    from oracle.graph import graph_x2
    m = model_cache(name)
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), tau)
    rp, cl = _host(*g.arrays())
    orp, ocl = graph_x2(m["H_col"], m["H_val"], tau)
    assert np.array_equal(rp, orp) and np.array_equal(cl, ocl)


@pytest.mark.parametrize("sets", ["bitmap", "hash"])
@pytest.mark.parametrize("name,tau", [("tiny48", 1e-2), ("tiny48", 0.0), ("small256", 1e-5),
                                      ("n1024", 1e-5)])
def test_x2_graph_every_candidate_resummed(gb, model_cache, name, tau, sets, monkeypatch):
    """The X2 kernels sum the entries in any order and re-sum in ascending k the candidates
    whose decision that order could change; GB_X2_SUMS=ascending sends every candidate through
    that re-summation: the graph is still the oracle's bit for bit."""
    from oracle.graph import graph_x2
    m = model_cache(name)
    monkeypatch.setenv("GB_X2_SUMS", "ascending")
    monkeypatch.setenv("GB_VERTEX_SETS", sets)
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), tau)
    rp, cl = _host(*g.arrays())
    orp, ocl = graph_x2(m["H_col"], m["H_val"], tau)
    assert np.array_equal(rp, orp) and np.array_equal(cl, ocl)


@pytest.mark.parametrize("sets", ["bitmap", "hash"])
def test_x2_graph_threshold_on_an_entry(gb, model_cache, sets, monkeypatch):
    """tau set to the ascending-order value |(X0^2)_ij| of candidates (so the GPU's own sum,
    taken in another order, may land on either side of it), and to the next double above:
    the edge is kept at tau and dropped just above, as the oracle decides."""
    from oracle.bounds import gershgorin, x0_values
    from oracle.graph import graph_x2, x2_rows
    m = model_cache("small256")
    monkeypatch.setenv("GB_VERTEX_SETS", sets)
    emin, emax = gershgorin(m["H_col"], m["H_val"])
    x0 = x0_values(m["H_col"], m["H_val"], emin, emax)
    rows = np.array([3, 77, 200])
    (_, acc, touched), = list(x2_rows(m["H_col"], x0, rows, chunk=len(rows)))
    vals = []
    for r, i in enumerate(rows):
        cand = np.flatnonzero(touched[r])
        cand = cand[cand != i]
        a = np.abs(acc[r, cand])
        vals.append(float(np.sort(a)[len(a) // 2]))  # a mid-sized entry of the row
    for v in vals:
        for tau in (v, float(np.nextafter(v, np.inf))):
            g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), tau)
            rp, cl = _host(*g.arrays())
            orp, ocl = graph_x2(m["H_col"], m["H_val"], tau)
            assert np.array_equal(rp, orp) and np.array_equal(cl, ocl)


def test_pattern_graph_bit_exact(gb, model_cache):
    from oracle.graph import graph_pattern
    m = model_cache("small256")
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), 1e-3, mode="pattern")
    rp, cl = _host(*g.arrays())
    orp, ocl = graph_pattern(m["H_col"], m["H_val"], 1e-3)
    assert np.array_equal(rp, orp) and np.array_equal(cl, ocl)


@pytest.mark.parametrize("name,tau,core", [("tiny48", 1e-3, 1), ("small256", 1e-3, 8),
                                           ("small256", 1e-5, 37), ("n1024", 1e-5, 16),
                                           ("small256", 1e-5, 1000)])
def test_partition_bit_exact(gb, model_cache, name, tau, core):
    from oracle.graph import graph_x2
    from oracle.partition import partition
    m = model_cache(name)
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), tau)
    p = gb.partition(g, core)
    cp, sp, si = _host(*p.arrays())
    ocp, ocv, osp, osi = partition(*graph_x2(m["H_col"], m["H_val"], tau), core)
    assert np.array_equal(cp, ocp) and np.array_equal(sp, osp) and np.array_equal(si, osi)
    assert p.max_sub == int(np.diff(osp).max())


def _compare_density(gb, m, tau, core, **kw):
    from oracle.sp2 import density_partitioned
    oc, ov, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], tau, core,
                                       branch_in=kw.get("branch_in"))
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], tau,
                                  core_size=core, **kw)
    dc, dv = _host(D_col, D_val)
    assert st["branch"] == info["branch"]
    assert st["iters"] == info["iters"] and st["converged"] == info["converged"]
    assert np.array_equal(dc, oc)
    err = float(np.abs(dv - ov).max())
    assert err <= FP64_TOL, err
    return st, info, err


@pytest.mark.parametrize("br", [[0], [1], [1, 0, 1]])
def test_fixed_steps_match_oracle(gb, model_cache, br):
    """Replay of a short branch sequence: exercises gather, the squaring kernel (both
    branches), and scatter with no stop rule involved."""
    m = model_cache("small256")
    st, info, err = _compare_density(gb, m, 1e-5, 16, branch_in=br)
    assert err <= 1e-13


@pytest.mark.parametrize("name,tau,core", [("small256", 1e-5, 16), ("small256", 1e-3, 1),
                                           ("small256", 1e-4, 24)])
def test_density_fp64_matches_oracle(gb, model_cache, name, tau, core):
    _compare_density(gb, model_cache(name), tau, core)


def test_single_subgraph_is_dense_sp2(gb, model_cache):
    """core_size >= N: one block holding every vertex (whole-matrix dense SP2)."""
    from oracle.exact import density_exact
    from oracle.bounds import ell_to_dense
    m = model_cache("small256")
    st, info, err = _compare_density(gb, m, 1e-5, 4096)
    assert st["n_sub"] == 1


def test_density_n1024_golden(gb, model_cache):
    ref = json.load(open(os.path.join(GOLDEN, "n1024_fp64_partitioned.json")))
    from synth import ell_sha256
    m = model_cache("n1024")
    assert ell_sha256(m["H_col"], m["H_val"]) == ref["H_sha256"]
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], ref["tau"],
                                  core_size=ref["core_size"])
    dc, dv = _host(D_col, D_val)
    assert "".join(map(str, st["branch"])) == ref["branch"]
    assert st["iters"] == ref["iters"] and st["converged"] == ref["converged"]
    assert ell_sha256(dc) == ref["D_col_sha256"]
    errs = [abs(dv[r, s] - float.fromhex(v)) for r, s, v in ref["samples"]]
    assert max(errs) <= FP64_TOL
    assert abs(st["trace"] - ref["trace_D"]) < 1e-9
    assert abs(np.linalg.norm(dv) - ref["D_frobenius"]) < 1e-9


def test_non_convergence_is_reported(gb, model_cache):
    m = model_cache("small256")
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                  core_size=16, max_iter=3)
    assert st["iters"] == 3 and not st["converged"]


def test_ragged_last_core(gb):
    """N not a multiple of the core size and of the tile size."""
    from synth import ModelSpec, make_model
    m = make_model(ModelSpec(n_sites=181, density=0.08, seed=21, name="r362"))
    assert m["N"] % 16 != 0
    _compare_density(gb, m, 1e-4, 16)


def test_diagonal_hamiltonian(gb):
    import torch
    from oracle.sp2 import density_partitioned
    rng = np.random.default_rng(3)
    N = 70
    d = rng.permutation(np.linspace(-3, 3, N))
    col = np.arange(N, dtype=np.int32)[:, None].copy()
    val = d[:, None].copy()
    D_col, D_val, st = gb.density(_dev(col), _dev(val), 20, 1e-5, core_size=8, idem_tol=1e-14)
    dc, dv = _host(D_col, D_val)
    want = (d <= np.sort(d)[19]).astype(float)
    assert st["converged"]
    # no edges besides self-loops: each subgraph is its core, and column i of D holds the
    # core rows of i with the occupation on the diagonal and zeros elsewhere
    for i in range(N):
        c0 = (i // 8) * 8
        rows = np.arange(c0, min(c0 + 8, N))
        assert np.array_equal(dc[i, :len(rows)], rows)
        assert abs(dv[i, i - c0] - want[i]) < 1e-14
        assert np.abs(np.delete(dv[i, :len(rows)], i - c0)).max() < 1e-14


LAUNCH_MODES = ("device", "per_subgraph", "graph", "host")


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x6", "fp16x3"])
def test_launch_modes_agree(gb, model_cache, precision):
    """The device-driven loop (default), one launch per subgraph, the hipGraph replay and the
    host-driven loop run the same kernels on the same data: results agree bit for bit."""
    m = model_cache("small256")
    outs = {}
    for mode in LAUNCH_MODES:
        D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                      core_size=16, precision=precision, launch_mode=mode)
        outs[mode] = (D_col.cpu().numpy(), D_val.cpu().numpy(), st["branch"], st["iters"])
    ref = outs["device"]
    for mode in LAUNCH_MODES[1:]:
        o = outs[mode]
        assert o[2] == ref[2] and o[3] == ref[3], mode
        assert np.array_equal(o[0], ref[0]) and np.array_equal(o[1], ref[1]), mode


@pytest.mark.parametrize("precision", ["fp64", "bf16x6", "fp16x3"])
def test_launch_modes_agree_n1024(gb, model_cache, precision):
    """The same at N = 1024 (blocks of up to 1024 rows, several tiles per edge and a ragged
    last tile), where the device-driven loops run past their first batch only if the
    expansion is long."""
    m = model_cache("n1024")
    outs = {}
    for mode in LAUNCH_MODES:
        D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                      core_size=16, precision=precision, launch_mode=mode)
        outs[mode] = (D_col.cpu().numpy(), D_val.cpu().numpy(), st["branch"], st["n_square"],
                      st["n_square_lo"])
        print(mode, st["iters"], st["ms"]["sp2"], st["ms"]["total"])
    ref = outs["device"]
    for mode in LAUNCH_MODES[1:]:
        o = outs[mode]
        assert o[2] == ref[2] and o[3:] == ref[3:], mode
        assert np.array_equal(o[0], ref[0]) and np.array_equal(o[1], ref[1]), mode


@pytest.mark.parametrize("name,core", [("small256", 16), ("n1024", 16)])
@pytest.mark.parametrize("precision", ["bf16x6", "fp16x3"])
def test_split_tile_edges_agree(gb, model_cache, name, core, precision):
    """Split squares on 128- and 64-edge tiles (and the tuner's per-bucket choice) accumulate
    every entry over k in the same order, but which of the mirrored pair (r, c) / (c, r) a tile
    computes depends on the tile edge, and the plane products pair the two differently: the
    results agree to the rounding of the low-precision loop (about 1e-8 here, far inside the
    1e-6 bar each of them meets against the oracle)."""
    m = model_cache(name)
    outs = {}
    for pol in ("128", "64", "auto"):
        D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                      core_size=core, precision=precision, tile_policy=pol)
        outs[pol] = (D_col.cpu().numpy(), D_val.cpu().numpy(), st["branch"], st["n_tile64"])
    assert outs["128"][3] == 0 and outs["64"][3] > 0
    for pol in ("64", "auto"):
        assert outs[pol][2] == outs["128"][2]
        assert np.array_equal(outs[pol][0], outs["128"][0])
        assert np.abs(outs[pol][1] - outs["128"][1]).max() < 2e-7, pol


@pytest.mark.parametrize("name,core", [("small256", 16), ("n1024", 16), ("n18000", 32)])
def test_fp16_interleaved_split_is_bit_identical(gb, model_cache, name, core):
    """The fp16 split square with the split under the products (two LDS buffers, tile policies
    "128i" / "64i") runs the same products in the same order as the one that splits between
    barriers: bit-identical D, branches and step counts, for either tile edge."""
    m = model_cache(name)
    Hc, Hv = _dev(m["H_col"]), _dev(m["H_val"])
    p = gb.partition(gb.build_graph(Hc, Hv, 1e-5), core,
                     method="multilevel" if name == "n18000" else "block")
    for a, b in (("128", "128i"), ("64", "64i")):
        outs = []
        for pol in (a, b):
            D_col, D_val, st = gb.density(Hc, Hv, m["n_occ"], 1e-5, partition=p,
                                          precision="fp16x3", tile_policy=pol)
            outs.append((D_col.cpu().numpy(), D_val.cpu().numpy(), st["branch"], st["iters"],
                         st["n_refine_done"]))
        assert outs[0][2:] == outs[1][2:], (a, b)
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_tune_table_round_trip(gb, model_cache, tmp_path):
    import json
    m = model_cache("n1024")
    for precision in ("bf16x6", "fp16x3"):
        gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5, core_size=16,
                   precision=precision)
    path = tmp_path / "tune.json"
    n = gb.tune_save(path)
    t = json.loads(path.read_text())
    assert n >= 1 and len(t["entries"]) == n and t["format"] == "libgb-tune-1"
    assert any(e["kind"] == 13 for e in t["entries"])  # the split-bf16 squares
    assert any(e["kind"] == 14 for e in t["entries"])  # the fp16 squares (either split kernel)
    assert gb.tune_load(path) == n
    t["device"] = "another device"
    path.write_text(json.dumps(t))
    with pytest.raises(gb.GbError):
        gb.tune_load(path)


@pytest.mark.parametrize("mode", ["device", "graph", "host"])
def test_replay_and_max_iter(gb, model_cache, mode):
    m = model_cache("small256")
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                  core_size=16, launch_mode=mode, max_iter=5)
    assert st["iters"] == 5 and not st["converged"]
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                  core_size=16, launch_mode=mode, branch_in=[1, 0, 1])
    assert st["iters"] == 3 and st["branch"] == [1, 0, 1]


@pytest.mark.parametrize("mode", ["device", "graph", "host"])
def test_replay_of_127_steps(gb, model_cache, mode):
    """The longest replay the records hold (127 updates, 128 trace pairs), past the default
    max_iter: every step is applied and recorded, in every launch mode."""
    m = model_cache("small256")
    seq = [i % 2 for i in range(127)]
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                  core_size=16, launch_mode=mode, branch_in=seq)
    assert st["iters"] == 127 and st["branch"] == seq
    assert len(st["t1"]) == 128 and np.isfinite(st["t1"]).all()


@pytest.mark.parametrize("precision,refine", [("fp64", "sp2"), ("fp32", "sp2")])
def test_tile_edges_agree(gb, model_cache, precision, refine):
    """128- and 64-edge tiles accumulate every entry of X^2 over k in the same order, and X^2
    is symmetric bit for bit, so D is identical.  (A McWeeny step multiplies two different
    matrices, S X, whose transpose rounds differently; which triangle is mirrored then
    depends on the tile edge, so that path agrees only to rounding.)"""
    m = model_cache("small256")
    outs = []
    for pol in ("128", "64", "auto", "64s3", "64r"):
        D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                      core_size=16, precision=precision, tile_policy=pol,
                                      refine=refine)
        outs.append((D_val.cpu().numpy(), st["branch"], st["n_tile64"], st["n_refine_done"]))
        if pol == "64s3":
            assert st["n_stage3"] == st["n_sub"]
        if pol == "64r":
            assert st["n_regstage"] == st["n_sub"]
    assert outs[0][2] == 0 and outs[1][2] > 0
    for q, o in enumerate(outs[1:]):
        diff = np.abs(o[0] - outs[0][0]).max()
        print(f"policy {q + 1}: max diff {diff:.3e}, tile64 {o[2]}, refine {o[3]} vs {outs[0][3]}")
        assert o[1] == outs[0][1]
        assert np.array_equal(o[0], outs[0][0])


def test_xcd_and_plain_tile_order_agree(gb, model_cache):
    m = model_cache("small256")
    outs = []
    for order in ("xcd", "plain"):
        D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                      core_size=16, tile_order=order)
        outs.append((D_val.cpu().numpy(), st["branch"]))
    assert outs[0][1] == outs[1][1] and np.array_equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("name,tau,core", [("small256", 1e-3, 8), ("n1024", 1e-5, 16),
                                           ("tiny48", 1e-2, 5)])
def test_bfs_partition_bit_exact(gb, model_cache, name, tau, core):
    from oracle.graph import graph_x2
    from oracle.partition import partition
    m = model_cache(name)
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), tau)
    p = gb.partition(g, core, method="bfs")
    cp, sp, si = _host(*p.arrays())
    ocp, ocv, osp, osi = partition(*graph_x2(m["H_col"], m["H_val"], tau), core, "bfs")
    assert np.array_equal(cp, ocp) and np.array_equal(sp, osp) and np.array_equal(si, osi)


def test_density_with_bfs_partition(gb, model_cache):
    from oracle.graph import graph_x2
    from oracle.sp2 import density_partitioned
    m = model_cache("small256")
    oc, ov, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-4, 16, method="bfs")
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), 1e-4)
    p = gb.partition(g, 16, method="bfs")
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-4,
                                  partition=p)
    assert st["branch"] == info["branch"]
    assert np.array_equal(D_col.cpu().numpy(), oc)
    assert np.abs(D_val.cpu().numpy() - ov).max() <= FP64_TOL


def test_tile_edges_mcweeny_agree_to_rounding(gb, model_cache):
    m = model_cache("small256")
    vals = []
    for pol in ("128", "64"):
        D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                      core_size=16, precision="fp32", tile_policy=pol)
        vals.append(D_val.cpu().numpy())
    assert np.abs(vals[0] - vals[1]).max() < 1e-12


@pytest.mark.parametrize("name,tau,core", [("small256", 1e-5, 16), ("n1024", 1e-5, 16),
                                           ("tiny48", 1e-2, 5)])
def test_multilevel_partition_bit_exact(gb, model_cache, name, tau, core):
    from oracle.graph import graph_x2
    from oracle.partition import partition
    m = model_cache(name)
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), tau)
    p = gb.partition(g, core, method="multilevel")
    cp, sp, si = _host(*p.arrays())
    ocp, ocv, osp, osi = partition(*graph_x2(m["H_col"], m["H_val"], tau), core, "multilevel")
    assert np.array_equal(cp, ocp) and np.array_equal(sp, osp) and np.array_equal(si, osi)


def test_multilevel_device_levels_match_host_levels(gb):
    """The device path builds every coarse level on the GPU (rows ascending, candidate lists
    from k_top_coarse); the host entry point builds them on host threads (rows in first-met
    order): at N = 18000 (four levels) the cores agree index for index."""
    import torch
    from synth import make_model
    m = make_model("n18000")
    g = gb.build_graph(torch.from_numpy(m["H_col"]).cuda(), torch.from_numpy(m["H_val"]).cuda(),
                       1e-5)
    p = gb.partition(g, 32, method="multilevel")
    cp, sp, si = _host(*p.arrays())
    rp, cl = _host(*g.arrays())
    hcp, hcv, _ = gb.partition_host(rp, cl, 32)
    dev_vtx = np.concatenate([si[sp[c]:sp[c] + (cp[c + 1] - cp[c])] for c in range(len(cp) - 1)])
    assert np.array_equal(cp, hcp) and np.array_equal(dev_vtx, hcv)


def test_density_n1024_multilevel_golden(gb, model_cache):
    """FP64 D on multilevel communities against the oracle's stored run on the same cores."""
    from synth import ell_sha256
    ref = json.load(open(os.path.join(GOLDEN, "n1024_fp64_multilevel.json")))
    m = model_cache("n1024")
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), ref["tau"])
    p = gb.partition(g, ref["core_size"], method="multilevel")
    assert ell_sha256(*_host(*p.arrays())) == ref["partition_sha256"]
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], ref["tau"],
                                  partition=p)
    dc, dv = _host(D_col, D_val)
    assert "".join(map(str, st["branch"])) == ref["branch"]
    assert ell_sha256(dc) == ref["D_col_sha256"]
    assert max(abs(dv[r, s] - float.fromhex(v)) for r, s, v in ref["samples"]) <= FP64_TOL


def test_partition_update_bit_exact(gb, model_cache):
    """On-the-fly update: the previous step's multilevel cores carried to the displaced
    system's graph, with their halos there, against the oracle, index for index."""
    from synth import displace_sites, rebuild_hamiltonian
    from oracle.graph import graph_x2
    from oracle.multilevel import partition_multilevel, partition_update
    from oracle.partition import halo_subgraphs
    m0 = model_cache("n1024")
    g0 = gb.build_graph(_dev(m0["H_col"]), _dev(m0["H_val"]), 1e-5)
    p0 = gb.partition(g0, 16, method="multilevel")
    ocp0, ocv0, _ = partition_multilevel(*graph_x2(m0["H_col"], m0["H_val"], 1e-5), 16)
    rng = np.random.default_rng(52)
    m1 = rebuild_hamiltonian(m0, displace_sites(m0["pos"], m0["L"], 0.02, rng))
    g1 = gb.build_graph(_dev(m1["H_col"]), _dev(m1["H_val"]), 1e-5)
    p1 = gb.partition_update(g1, p0)
    cp, sp, si = _host(*p1.arrays())
    rp1, col1 = graph_x2(m1["H_col"], m1["H_val"], 1e-5)
    ocp, ocv, _ = partition_update(rp1, col1, ocp0, ocv0)
    osp, osi = halo_subgraphs(rp1, col1, [ocv[ocp[i]:ocp[i + 1]] for i in range(len(ocp) - 1)])
    assert np.array_equal(cp, ocp) and np.array_equal(sp, osp) and np.array_equal(si, osi)


@pytest.mark.parametrize("name,tau,core", [("small256", 1e-5, 16), ("n1024", 1e-5, 16),
                                           ("tiny48", 1e-2, 5)])
def test_hash_vertex_sets_bit_exact(gb, model_cache, name, tau, core, monkeypatch):
    """Graph and halos on LDS hash sets (the kernels past 2^17 vertices) against the oracle."""
    from oracle.graph import graph_x2
    from oracle.partition import partition
    m = model_cache(name)
    monkeypatch.setenv("GB_VERTEX_SETS", "hash")
    g = gb.build_graph(_dev(m["H_col"]), _dev(m["H_val"]), tau)
    rp, cl = _host(*g.arrays())
    orp, ocl = graph_x2(m["H_col"], m["H_val"], tau)
    assert np.array_equal(rp, orp) and np.array_equal(cl, ocl)
    p = gb.partition(g, core)
    cp, sp, si = _host(*p.arrays())
    ocp, ocv, osp, osi = partition(orp, ocl, core, "block")
    assert np.array_equal(cp, ocp) and np.array_equal(sp, osp) and np.array_equal(si, osi)
