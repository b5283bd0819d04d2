"""Element-by-element parity of D with the oracle (GPU), for every precision of the squaring
loop.

* N = 1024: the whole D (every column, every entry) against the oracle run live.
* N = 18000 and N = 100000, block and multilevel cores: every entry of the D columns of 32 whole
  subgraphs -- the 8 smallest, the 8 largest and 16 drawn at random -- against the oracle on
  those subgraphs with the whole-system oracle run's stored branch sequence replayed
  (oracle/subgraphs.py; the columns of a core depend on its own subgraph once the sequence is
  fixed, Eq. 6).  The cores are the oracle's own (stored communities, or blocks); the GPU
  partition is first checked against the oracle's by its SHA-256, so the picks by size are the
  oracle's subgraphs.

Bars: FP64 1e-9 max-abs with the oracle's branch sequence and step count; the mixed-precision
loops (FP32, split-bf16 or split-fp16 squares with FP64 traces, branches and refinement) 1e-6
max-abs."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
BAR = {"fp64": 1e-9, "fp32": 1e-6, "bf16x6": 1e-6, "fp16x3": 1e-6}


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available()
    import paper_1603_00937_amd as gb
    return gb


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def whole1024(model_cache):
    from oracle.sp2 import density_partitioned
    m = model_cache("n1024")
    oc, ov, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-5, 16)
    return m, oc, ov, info


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x6", "fp16x3"])
def test_n1024_whole_D(gb, whole1024, precision):
    m, oc, ov, info = whole1024
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                  core_size=16, precision=precision)
    dc, dv = D_col.cpu().numpy(), D_val.cpu().numpy()
    w = oc.shape[1]
    assert np.array_equal(dc[:, :w], oc) and (dc[:, w:] == -1).all()
    diff = dv[:, :w] - ov
    err = float(np.abs(diff).max())
    frob = float(np.linalg.norm(diff))
    print(f"n1024 {precision}: iters={st['iters']}+{st['n_refine_done']} max-abs {err:.3e} "
          f"Frobenius {frob:.3e} ({oc.size} entries)")
    assert st["converged"]
    if precision == "fp64":
        assert st["branch"] == info["branch"] and st["iters"] == info["iters"]
    assert (dv[:, w:] == 0).all()
    assert err <= BAR[precision]


def _pick(sizes, rng):
    order = np.argsort(sizes, kind="stable")
    mid = order[8:-8]
    return np.sort(np.concatenate([order[:8], order[-8:],
                                   rng.choice(mid, size=16, replace=False)]))


_ORACLE = {}


def _case(name, method):
    """Model, stored oracle run, picked cores and the oracle's columns of those cores."""
    key = (name, method)
    if key in _ORACLE:
        return _ORACLE[key]
    from synth import make_model, ell_sha256
    tag = "partitioned" if method == "block" else method
    path = os.path.join(GOLDEN, f"{name}_fp64_{tag}.json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle run for {name} {method}")
    ref = json.load(open(path))
    m = _ORACLE.get(name) or make_model(name)
    _ORACLE[name] = m
    assert ell_sha256(m["H_col"], m["H_val"]) == ref["H_sha256"]
    if "core_ptr" in ref:
        cptr = np.asarray(ref["core_ptr"])
        cvtx = np.asarray(ref["core_vtx"], dtype=np.int32)
    else:
        k, N = ref["core_size"], ref["N"]
        cptr = np.minimum(np.arange(0, N + k, k), N)
        cvtx = np.arange(N, dtype=np.int32)
    _ORACLE[key] = (m, ref, cptr, cvtx, None)
    return _ORACLE[key]


def _oracle_columns(key, picks):
    m, ref, cptr, cvtx, cols = _ORACLE[key]
    if cols is None:
        from oracle.subgraphs import core_columns
        import time
        t0 = time.time()
        cores = [cvtx[cptr[c]:cptr[c + 1]] for c in picks]
        cols = core_columns(m["H_col"], m["H_val"], m["n_occ"], ref["tau"], cores,
                            ref["branch"])
        print(f"oracle: {len(picks)} subgraphs of {key} in {time.time() - t0:.1f} s")
        _ORACLE[key] = (m, ref, cptr, cvtx, cols)
    return cols


CASES = [("n18000", "multilevel", "fp64", "device"),
         ("n18000", "multilevel", "bf16x6", "device"),
         ("n18000", "multilevel", "bf16x6", "graph"),
         ("n18000", "multilevel", "fp32", "device"),
         ("n18000", "multilevel", "fp16x3", "device"),
         ("n18000", "block", "fp64", "device"),
         ("n18000", "block", "bf16x6", "host"),
         ("n18000", "block", "fp32", "device"),
         ("n18000", "block", "fp16x3", "device"),
         ("n100000", "multilevel", "fp64", "device"),
         ("n100000", "multilevel", "bf16x6", "device"),
         ("n100000", "multilevel", "bf16x6", "graph"),
         ("n100000", "multilevel", "fp32", "device"),
         ("n100000", "multilevel", "fp16x3", "device"),
         ("n100000", "block", "bf16x6", "device"),
         ("n100000", "block", "fp32", "device"),
         ("n100000", "block", "fp16x3", "device")]


@pytest.mark.parametrize("name,method,precision,launch_mode", CASES)
def test_whole_subgraphs_fullsize(gb, name, method, precision, launch_mode):
    import torch
    from synth import ell_sha256
    m, ref, cptr, cvtx, _ = _case(name, method)
    Hc, Hv = _dev(m["H_col"]), _dev(m["H_val"])
    g = gb.build_graph(Hc, Hv, ref["tau"])
    p = gb.partition(g, ref["core_size"], method=method)
    cp, sp, si = [t.cpu().numpy() for t in p.arrays()]
    assert ell_sha256(cp, sp, si) == ref["partition_sha256"], "partition differs from the oracle's"
    picks = _pick(np.diff(sp), np.random.default_rng(17))
    cols = _oracle_columns((name, method), picks)
    D_col, D_val, st = gb.density(Hc, Hv, m["n_occ"], ref["tau"], partition=p,
                                  precision=precision, launch_mode=launch_mode)
    torch.cuda.synchronize()
    assert st["converged"]
    if precision == "fp64":
        assert "".join(map(str, st["branch"])) == ref["branch"] and st["iters"] == ref["iters"]
    dc, dv = D_col.cpu().numpy(), D_val.cpu().numpy()
    worst, sq, n_ent = 0.0, 0.0, 0
    for c, (rows, vals) in zip(picks, cols):
        verts = cvtx[cptr[c]:cptr[c + 1]]
        n = len(rows)
        assert np.array_equal(dc[verts, :n], np.broadcast_to(rows, (len(verts), n)))
        assert (dc[verts, n:] == -1).all() and (dv[verts, n:] == 0).all()
        d = dv[verts, :n] - vals
        worst = max(worst, float(np.abs(d).max()))
        sq += float((d * d).sum())
        n_ent += d.size
    sizes = np.diff(sp)[picks]
    print(f"{name} {method} {precision} {launch_mode}: iters={st['iters']}+"
          f"{st['n_refine_done']} subgraphs n={sizes.min()}..{sizes.max()} ({n_ent} entries): "
          f"max-abs {worst:.3e} Frobenius {np.sqrt(sq):.3e}")
    assert worst <= BAR[precision]
