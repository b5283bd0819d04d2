"""The C-ABI boundary on the GPU: non-finite input is rejected, a caller-owned workspace gives
the same D as the library's cached buffers, and the max-norm idempotency check is optional."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gb():
    import torch
    assert torch.cuda.is_available()
    import paper_1603_00937_amd as gb
    return gb


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_non_finite_h_is_rejected(gb, model_cache, bad):
    from paper_1603_00937_amd._lib import GB_EINVAL
    m = model_cache("small256")
    hv = m["H_val"].copy()
    # an off-diagonal entry (slot 1 of row 7) and, separately, a diagonal one
    for r, t in ((7, 1), (11, int(np.nonzero(m["H_col"][11] == 11)[0][0]))):
        h = hv.copy()
        h[r, t] = bad
        Hc, Hv = _dev(m["H_col"]), _dev(h)
        for call in (lambda: gb.spectral_bounds(Hc, Hv),
                     lambda: gb.build_graph(Hc, Hv, 1e-5),
                     lambda: gb.density(Hc, Hv, m["n_occ"], 1e-5, core_size=16),
                     lambda: gb.density(Hc, Hv, m["n_occ"], 1e-5, core_size=16, emin=-5.0,
                                        emax=5.0)):
            with pytest.raises(gb.GbError) as e:
                call()
            assert e.value.status == GB_EINVAL and "NaN or Inf" in str(e.value)
    # the library still works afterwards
    D_col, D_val, st = gb.density(_dev(m["H_col"]), _dev(hv), m["n_occ"], 1e-5, core_size=16)
    assert st["converged"]


@pytest.mark.parametrize("precision", ["fp64", "bf16x6", "fp32"])
def test_caller_workspace_matches_cached_buffers(gb, model_cache, precision):
    import torch
    from paper_1603_00937_amd._lib import GB_ESHAPE
    m = model_cache("n1024")
    Hc, Hv = _dev(m["H_col"]), _dev(m["H_val"])
    p = gb.partition(gb.build_graph(Hc, Hv, 1e-5), 16)
    nb = gb.density_workspace(Hc, p, precision=precision)
    total = sum(npad * npad for npad in
                ((np.diff(p.arrays()[1].cpu().numpy()) + 63) // 64 * 64).tolist())
    assert nb >= 2 * 8 * total and nb % 256 == 0
    ref = gb.density(Hc, Hv, m["n_occ"], 1e-5, partition=p, precision=precision)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for _ in range(2):  # the same workspace twice in a row
        out = gb.density(Hc, Hv, m["n_occ"], 1e-5, partition=p, precision=precision,
                         workspace=ws)
        assert out[2]["branch"] == ref[2]["branch"] and out[2]["iters"] == ref[2]["iters"]
        assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
    with pytest.raises(gb.GbError) as e:
        gb.density(Hc, Hv, m["n_occ"], 1e-5, partition=p, precision=precision,
                   workspace=ws[:nb - 256])
    assert e.value.status == GB_ESHAPE


def test_idempotency_check_is_optional(gb, model_cache):
    m = model_cache("small256")
    Hc, Hv = _dev(m["H_col"]), _dev(m["H_val"])
    for precision in ("fp64", "bf16x6"):
        a = gb.density(Hc, Hv, m["n_occ"], 1e-5, core_size=16, precision=precision)
        b = gb.density(Hc, Hv, m["n_occ"], 1e-5, core_size=16, precision=precision,
                       check_idem=True)
        assert math.isnan(a[2]["idem_max"]) and b[2]["idem_max"] < 1e-8
        assert a[2]["branch"] == b[2]["branch"]
        assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())
        assert a[2]["n_near_tie"] == 0


def test_sustained_rates_are_plausible(gb):
    """The library's own matrix-core and HBM rates: within the datasheet figures, and ordered
    as the units are (bf16/fp16 > FP32 > FP64)."""
    r = {k: gb.peak_rate(k) for k in ("fp64", "fp32", "bf16", "fp16", "hbm")}
    print("sustained:", {k: round(v, 1) for k, v in r.items()})
    assert 10 < r["fp64"] <= 78.6 * 1.1 and 20 < r["fp32"] <= 157.3 * 1.1
    assert 200 < r["bf16"] <= 2500 * 1.1 and 200 < r["fp16"] <= 2500 * 1.1
    assert r["bf16"] > r["fp32"] > r["fp64"]
    assert 1000 < r["hbm"] <= 8000 * 1.1
    rate, mhz = gb.peak_rate("bf16", with_clock=True)
    print(f"bf16 loop: {rate:.0f} TFLOP/s at {mhz:.0f} MHz")
    # the datasheet peak is quoted at 2400 MHz: the rate per MHz bounds it
    assert 300 < mhz <= 2600 and rate / mhz <= 2500 / 2400 * 1.1
    with pytest.raises(gb.GbError):
        gb.peak_rate("int8")
