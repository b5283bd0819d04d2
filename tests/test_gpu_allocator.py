"""The device-memory hook and the device views: with torch's caching allocator registered,
graph, partition and density give bit-identical results, every library buffer comes from
the hook, and all of them are returned once the handles are gone and the cached batch
buffers are trimmed."""
import ctypes
import gc

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _run(gb, Hc, Hv, n_occ):
    g = gb.build_graph(Hc, Hv, 1e-5)
    p = gb.partition(g, 16)
    D_col, D_val, st = gb.density(Hc, Hv, n_occ, 1e-5, partition=p)
    rp, col = g.arrays()
    cp, sp, si = p.arrays()
    torch.cuda.synchronize()
    return g, p, [x.cpu().numpy() for x in (rp, col, cp, sp, si, D_col, D_val)], st


def test_torch_allocator_bit_identical(model_cache):
    import paper_1603_00937_amd as gb
    m = model_cache("n1024")
    Hc = torch.from_numpy(m["H_col"]).cuda()
    Hv = torch.from_numpy(m["H_val"]).cuda()
    g0, p0, ref, st0 = _run(gb, Hc, Hv, m["n_occ"])
    del g0, p0
    gb.trim()  # the cached batch buffers come from the hook from now on
    alloc = gb.TorchAllocator()
    gb.set_allocator(alloc)
    try:
        g1, p1, got, st1 = _run(gb, Hc, Hv, m["n_occ"])
        assert alloc.n_alloc > 0
        held = set(alloc.live)
        # the handles' arrays are among the live blocks
        rp_ptr, col_ptr = g1.views()
        cp_ptr, sp_ptr, si_ptr = p1.views()
        for ptr in (rp_ptr, col_ptr, cp_ptr, sp_ptr, si_ptr):
            assert ptr in held
    finally:
        gb.set_allocator(None)
    assert st1["iters"] == st0["iters"] and st1["branch"] == st0["branch"]
    for a, b in zip(ref, got):
        assert a.dtype == b.dtype and np.array_equal(a, b)
    del g1, p1
    gc.collect()
    assert alloc.live != {}  # the cached batch buffers
    gb.trim()
    torch.cuda.synchronize()
    assert alloc.live == {}


def test_views_match_copies(model_cache):
    import paper_1603_00937_amd as gb
    m = model_cache("tiny48")
    Hc = torch.from_numpy(m["H_col"]).cuda()
    Hv = torch.from_numpy(m["H_val"]).cuda()
    g = gb.build_graph(Hc, Hv, 1e-5)
    p = gb.partition(g, 8)
    rp, col = g.arrays()
    cp, sp, si = p.arrays()
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]

    def fetch(ptr, n):
        t = torch.empty(n, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        assert hip.hipMemcpy(t.data_ptr(), ptr, n * 4, 3) == 0  # device to device
        return t
    v_rp, v_col = g.views()
    assert torch.equal(fetch(v_rp, g.n + 1), rp)
    assert torch.equal(fetch(v_col, g.nnz), col)
    v_cp, v_sp, v_si = p.views()
    assert torch.equal(fetch(v_cp, p.n_sub + 1), cp)
    assert torch.equal(fetch(v_sp, p.n_sub + 1), sp)
    assert torch.equal(fetch(v_si, p.total), si)
