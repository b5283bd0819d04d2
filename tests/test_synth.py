"""The seeded input generator: determinism, structure, physics sanity."""
import json
import os

import numpy as np
import pytest

from synth import CONFIGS, ModelSpec, make_model, ell_sha256, make_operator_v
from synth.model import det_exp, morton_order

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_det_exp_close_to_libm():
    x = np.linspace(-5.0, 0.0, 10001)
    rel = np.abs(det_exp(x) / np.exp(x) - 1.0)
    assert rel.max() < 4e-16


@pytest.mark.parametrize("name", ["tiny48", "small256", "n1024"])
def test_generator_deterministic_and_structured(name):
    a = make_model(name)
    b = make_model(name)
    assert np.array_equal(a["H_col"], b["H_col"]) and np.array_equal(a["H_val"], b["H_val"])
    col, val = a["H_col"], a["H_val"]
    N = a["N"]
    assert N == 2 * CONFIGS[name].n_sites and a["n_occ"] == N // 2
    for i in range(0, N, max(1, N // 64)):
        c = col[i][col[i] >= 0]
        assert np.all(np.diff(c) > 0), "columns ascending and unique"
        assert i in c, "diagonal present"
        assert np.all(col[i][len(c):] == -1) and np.all(val[i][len(c):] == 0.0)
    from oracle.bounds import ell_to_dense
    H = ell_to_dense(col, val)
    assert np.array_equal(H, H.T), "exactly symmetric"


def test_model_hashes_match_golden():
    """Bit-identical inputs on every machine: the hashes were written by
    tests/golden/make_golden.py on another host."""
    path = os.path.join(GOLDEN, "model_hashes.json")
    ref = json.load(open(path))
    for name in ("tiny48", "small256", "n1024"):
        m = make_model(name)
        assert ell_sha256(m["H_col"], m["H_val"]) == ref[name], name


def test_gap_and_onsite(model_cache):
    from oracle.bounds import ell_to_dense
    m = model_cache("n1024")
    w = np.linalg.eigvalsh(ell_to_dense(m["H_col"], m["H_val"]))
    assert w[m["n_occ"]] - w[m["n_occ"] - 1] > 0.5, "gapped system"


def test_morton_order_is_permutation():
    rng = np.random.default_rng(0)
    pos = rng.uniform(0, 10.0, (500, 3))
    o = morton_order(pos, 10.0)
    assert np.array_equal(np.sort(o), np.arange(500))


def test_operator_v_symmetric(model_cache):
    from oracle.bounds import ell_to_dense
    m = model_cache("small256")
    V = make_operator_v(m["H_col"], 51)
    Vd = ell_to_dense(m["H_col"], V)
    assert np.array_equal(Vd, Vd.T)
    assert np.all(np.abs(V) <= 1.0)


def test_clustered_geometry_small():
    spec = ModelSpec(n_sites=3000, density=0.03, seed=9, clusters=(4, 500, 0.15), name="c")
    m = make_model(spec)
    assert m["N"] == 6000
    assert m["pos"].min() >= 0.0 and m["pos"].max() < m["L"]


def test_operator_v_pairs_is_symmetric_and_pattern_independent():
    from synth import make_model, operator_v_pairs, displace_sites, rebuild_hamiltonian
    m = make_model("small256")
    V = operator_v_pairs(m["H_col"], 51)
    N, W = m["H_col"].shape
    val = {}
    for i in range(N):
        for t in range(W):
            j = int(m["H_col"][i, t])
            if j >= 0:
                val[(i, j)] = V[i, t]
                assert -1.0 <= V[i, t] < 1.0
            else:
                assert V[i, t] == 0.0
    for (i, j), v in val.items():
        assert val[(j, i)] == v
    rng = np.random.default_rng(52)
    m2 = rebuild_hamiltonian(m, displace_sites(m["pos"], m["L"], 0.3, rng))
    V2 = operator_v_pairs(m2["H_col"], 51)
    same = 0
    for i in range(N):
        for t in range(m2["H_col"].shape[1]):
            j = int(m2["H_col"][i, t])
            if (i, j) in val:
                assert V2[i, t] == val[(i, j)]
                same += 1
    assert same > 0
