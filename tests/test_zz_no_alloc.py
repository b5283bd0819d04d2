"""The allocation-free spectral bounds (GPU, through the C ABI): the same e_min / e_max bit for bit
as gb_spectral_bounds (and the oracle's Gershgorin bounds), on two calls in a row, the second
with a smaller input, and the same rejection of a non-finite H."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available()
    from paper_1603_00937_amd import _lib
    return _lib.load()


def _bounds(lib, fn, Hc, Hv):
    import torch
    from paper_1603_00937_amd._lib import GbEll
    H = GbEll(Hc.shape[0], Hc.shape[1], Hc.data_ptr(), Hv.data_ptr())
    lo, hi = ctypes.c_double(), ctypes.c_double()
    st = getattr(lib, fn)(ctypes.byref(H), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                          ctypes.byref(lo), ctypes.byref(hi))
    return st, lo.value, hi.value


def test_noalloc_bounds_match_allocating_call(lib, model_cache):
    import torch
    from oracle.bounds import gershgorin
    for name in ("n1024", "small256"):  # the second call on a smaller input
        m = model_cache(name)
        Hc = torch.from_numpy(m["H_col"]).cuda()
        Hv = torch.from_numpy(m["H_val"]).cuda()
        st0, lo0, hi0 = _bounds(lib, "gb_spectral_bounds", Hc, Hv)
        st1, lo1, hi1 = _bounds(lib, "gb_spectral_bounds_noalloc", Hc, Hv)
        assert st0 == 0 and st1 == 0
        assert (lo1.hex(), hi1.hex()) == (lo0.hex(), hi0.hex())
        elo, ehi = gershgorin(m["H_col"], m["H_val"])
        assert (lo1, hi1) == (elo, ehi), name


def test_noalloc_bounds_reject_non_finite(lib, model_cache):
    import torch
    from paper_1603_00937_amd._lib import GB_EINVAL
    m = model_cache("small256")
    hv = m["H_val"].copy()
    hv[5, 1] = float("nan")
    Hc = torch.from_numpy(m["H_col"]).cuda()
    st, _, _ = _bounds(lib, "gb_spectral_bounds_noalloc", Hc, torch.from_numpy(hv).cuda())
    assert st == GB_EINVAL and b"NaN or Inf" in lib.gb_last_error()
    st, lo, hi = _bounds(lib, "gb_spectral_bounds_noalloc", Hc,
                         torch.from_numpy(m["H_val"]).cuda())
    assert st == 0 and lo < hi
