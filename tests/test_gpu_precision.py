"""Low-precision squarings with FP64 traces, branches and refinement (GPU).

Error bar: max-abs 1e-6 against the FP64 oracle.  Plain BF16 is a negative control: its
rounding rotates the occupied subspace, which no purification step can undo."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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
def ref1024():
    return json.load(open(os.path.join(GOLDEN, "n1024_fp64_partitioned.json")))


def _sample_err(D_val, ref):
    dv = D_val.cpu().numpy()
    return max(abs(dv[r, s] - float.fromhex(v)) for r, s, v in ref["samples"])


@pytest.mark.parametrize("precision", ["fp32", "bf16x6", "fp16x3"])
def test_mixed_precision_within_1e6(gb, model_cache, ref1024, precision):
    from synth import ell_sha256
    m = model_cache("n1024")
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                  core_size=16, precision=precision, check_idem=True)
    assert ell_sha256(D_col.cpu().numpy()) == ref1024["D_col_sha256"]
    assert st["converged"]
    err = _sample_err(D_val, ref1024)
    print(f"{precision}: iters={st['iters']} err={err:.3e} trace={st['trace']:.9f}")
    assert err <= 1e-6
    # low-precision rounding shifts the summed core trace slightly (it is not an integer for
    # a partitioned D); McWeeny refinement keeps it rather than chasing it
    assert abs(st["trace"] - m["n_occ"]) < 1e-4
    assert st["idem_max"] < 1e-6


def test_bf16x3_and_plain_bf16_are_less_accurate(gb, model_cache, ref1024):
    m = model_cache("n1024")
    errs = {}
    for p in ("bf16x3", "bf16"):
        D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                      core_size=16, precision=p)
        errs[p] = _sample_err(D_val, ref1024)
    print(errs)
    assert errs["bf16"] > 1e-5, "plain BF16 misses the 1e-6 bar (negative control)"
    assert errs["bf16x3"] < errs["bf16"]


def test_fp32_small_matches_oracle_pattern(gb, model_cache):
    from oracle.sp2 import density_partitioned
    m = model_cache("small256")
    oc, ov, info = density_partitioned(m["H_col"], m["H_val"], m["n_occ"], 1e-5, 16)
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                  core_size=16, precision="fp32")
    assert np.array_equal(D_col.cpu().numpy(), oc)
    assert np.abs(D_val.cpu().numpy() - ov).max() <= 1e-6


@pytest.mark.parametrize("refine,first", [("mcweeny", 0), ("sp2", 0), ("mcweeny", 3),
                                          ("mcweeny_blocks", 0)])
def test_refinement_variants(gb, model_cache, ref1024, refine, first):
    m = model_cache("n1024")
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(m["H_val"]), m["n_occ"], 1e-5,
                                  core_size=16, precision="fp32", refine=refine,
                                  n_fp64_first=first, check_idem=True)
    err = _sample_err(D_val, ref1024)
    print(f"fp32 refine={refine} fp64_first={first}: err={err:.3e} idem={st['idem']:.2e} "
          f"trace={st['trace']:.9f} steps={st['n_refine_done']} iters={st['iters']}")
    assert st["converged"]
    assert st["idem_max"] < 1e-8
    assert err <= 1e-6


@pytest.mark.parametrize("precision,core", [("fp32", 16), ("bf16x6", 16), ("bf16x6", 32),
                                            ("fp16x3", 16), ("fp16x3", 32), ("fp32", 40)])
def test_core_row_refinement_matches_whole_blocks(gb, model_cache, precision, core):
    """McWeeny on the core rows (products of the k core rows with X) against McWeeny on whole
    blocks from the same low-precision X: same pattern, values and check to rounding.  Cores
    of 40 exceed the core-row path's 32 rows and take whole blocks both times."""
    m = model_cache("n1024")
    Hc, Hv = _dev(m["H_col"]), _dev(m["H_val"])
    out = {}
    for refine in ("mcweeny", "mcweeny_blocks"):
        D_col, D_val, st = gb.density(Hc, Hv, m["n_occ"], 1e-5, core_size=core,
                                      precision=precision, refine=refine, check_idem=True)
        out[refine] = (D_col.cpu().numpy(), D_val.cpu().numpy(), st)
    (rc, rv, rs), (bc, bv, bs) = out["mcweeny"], out["mcweeny_blocks"]
    diff = float(np.abs(rv - bv).max())
    print(f"{precision} core={core}: rows {rs['n_refine_done']} steps idem_max "
          f"{rs['idem_max']:.2e} {rs['ms']['refine']:.2f} ms; blocks {bs['n_refine_done']} steps "
          f"idem_max {bs['idem_max']:.2e} {bs['ms']['refine']:.2f} ms; max diff {diff:.2e}")
    assert rs["converged"] and bs["converged"]
    assert rs["iters"] == bs["iters"] and rs["branch"] == bs["branch"]
    assert np.array_equal(rc, bc)
    # the core-row path picks its step count in advance, so it may take one step more
    assert rs["n_refine_done"] >= bs["n_refine_done"]
    assert diff <= (1e-11 if rs["n_refine_done"] == bs["n_refine_done"] else 1e-8)
    assert abs(rs["idem_max"] - bs["idem_max"]) <= 1e-10
    assert abs(rs["trace"] - bs["trace"]) <= 1e-9
