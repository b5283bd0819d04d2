"""The C ABI on the CPU: the library loads, exports every declared symbol, and rejects bad
arguments on the host with the documented codes before any device work."""
import ctypes

import numpy as np
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gb.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gb_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1603_00937_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1603_00937_amd.build import build
        build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "gb_density" in names and "gb_build_graph" in names and "gb_partition" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1603_00937_amd import _lib
    assert set(_declared()) == set(_lib.SIGNATURES)


def test_version(lib):
    assert lib.gb_version().startswith(b"libgb")


def _err(lib):
    return lib.gb_last_error().decode()


def test_density_rejects_bad_arguments(lib):
    from paper_1603_00937_amd._lib import GbEll, GbSp2Opts, GB_EINVAL, GB_ESHAPE
    bogus = 0x1000  # never dereferenced: the checks fail first
    H = GbEll(8, 3, bogus, bogus)
    D = GbEll(8, 3, bogus, bogus)
    assert lib.gb_density(None, 4, 1e-5, None, ctypes.byref(D), None, None) == GB_EINVAL
    assert "H is NULL" in _err(lib)
    assert lib.gb_density(ctypes.byref(H), 9, 1e-5, None, ctypes.byref(D), None, None) == GB_EINVAL
    assert "n_occ" in _err(lib)
    assert lib.gb_density(ctypes.byref(H), -1, 1e-5, None, ctypes.byref(D), None, None) == GB_EINVAL
    assert lib.gb_density(ctypes.byref(H), 4, float("nan"), None, ctypes.byref(D), None,
                          None) == GB_EINVAL
    assert lib.gb_density(ctypes.byref(H), 4, -1.0, None, ctypes.byref(D), None, None) == GB_EINVAL
    D2 = GbEll(7, 3, bogus, bogus)
    assert lib.gb_density(ctypes.byref(H), 4, 1e-5, None, ctypes.byref(D2), None, None) == GB_ESHAPE
    o = GbSp2Opts()
    o.precision = 7
    assert lib.gb_density(ctypes.byref(H), 4, 1e-5, ctypes.byref(o), ctypes.byref(D), None,
                          None) == GB_EINVAL
    o = GbSp2Opts()
    o.max_iter = 500
    assert lib.gb_density(ctypes.byref(H), 4, 1e-5, ctypes.byref(o), ctypes.byref(D), None,
                          None) == GB_EINVAL
    o = GbSp2Opts()
    bad = (ctypes.c_uint8 * 2)(0, 3)
    o.branch_in = ctypes.cast(bad, ctypes.c_void_p)
    o.n_branch_in = 2
    assert lib.gb_density(ctypes.byref(H), 4, 1e-5, ctypes.byref(o), ctypes.byref(D), None,
                          None) == GB_EINVAL
    assert "branch_in" in _err(lib)
    o = GbSp2Opts()
    o.emin, o.emax = 2.0, 1.0
    assert lib.gb_density(ctypes.byref(H), 4, 1e-5, ctypes.byref(o), ctypes.byref(D), None,
                          None) == GB_EINVAL


def test_graph_and_partition_reject_bad_arguments(lib):
    from paper_1603_00937_amd._lib import GbEll, GB_EINVAL
    bogus = 0x1000
    H = GbEll(8, 3, bogus, bogus)
    out = ctypes.c_void_p()
    assert lib.gb_build_graph(ctypes.byref(H), None, -1.0, 0.0, 0, None, ctypes.byref(out)) == GB_EINVAL
    assert lib.gb_build_graph(ctypes.byref(H), None, 1e-5, 0.0, 9, None, ctypes.byref(out)) == GB_EINVAL
    assert lib.gb_build_graph(ctypes.byref(H), None, 1e-5, 0.0, 2, None, ctypes.byref(out)) == GB_EINVAL
    assert lib.gb_build_graph(None, None, 1e-5, 0.0, 0, None, ctypes.byref(out)) == GB_EINVAL
    Hn = GbEll(0, 3, bogus, bogus)
    assert lib.gb_build_graph(ctypes.byref(Hn), None, 1e-5, 0.0, 0, None, ctypes.byref(out)) == GB_EINVAL
    assert lib.gb_partition(None, 16, 0, None, ctypes.byref(out)) == GB_EINVAL
    assert lib.gb_graph_info(None, None, None) == GB_EINVAL
    lib.gb_graph_destroy(None)
    lib.gb_partition_destroy(None)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    assert lib.gb_spectral_bounds(None, None, ctypes.byref(lo), ctypes.byref(hi)) == GB_EINVAL
    assert lib.gb_spectral_bounds(ctypes.byref(H), None, None, None) == GB_EINVAL


def test_trim_without_cached_buffers(lib):
    assert lib.gb_trim() == 0


def test_views_and_allocator_reject_bad_arguments(lib):
    from paper_1603_00937_amd._lib import ALLOC_FN, FREE_FN, GB_EINVAL, GB_OK
    p = ctypes.c_void_p()
    assert lib.gb_graph_view(None, None, None, ctypes.byref(p), None) == GB_EINVAL
    assert lib.gb_partition_view(None, None, None, ctypes.byref(p), None, None) == GB_EINVAL
    keep = ALLOC_FN(lambda n, s, c: None)
    assert lib.gb_set_allocator(keep, FREE_FN(), None) == GB_EINVAL
    assert lib.gb_set_allocator(ALLOC_FN(), FREE_FN(lambda p, s, c: None), None) == GB_EINVAL
    assert b"both" in lib.gb_last_error()
    assert lib.gb_set_allocator(ALLOC_FN(), FREE_FN(), None) == GB_OK


def test_no_cpu_fallback_in_product_path():
    """The package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_1603_00937_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in src, fn


def test_struct_layout_matches_header(tmp_path):
    """The ctypes mirrors of the option and stats structs have the C sizes and offsets."""
    import shutil
    import subprocess
    from paper_1603_00937_amd import _lib as L
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    fields = {"gb_sp2_opts": L.GbSp2Opts, "gb_sp2_stats": L.GbSp2Stats, "gb_ell": L.GbEll,
              "gb_foe_opts": L.GbFoeOpts, "gb_foe_stats": L.GbFoeStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){"]
    for cname, py in fields.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname}.{f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.rsplit(" ", 1) for line in out if line)
    for cname, py in fields.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert int(got[f"{cname}.{f[0]}"]) == getattr(py, f[0]).offset, (cname, f[0])


def test_chebyshev_coefficients_match_oracle(lib):
    """Host entry point (no GPU needed) against the oracle's quadrature."""
    from oracle.foe import fermi_coefficients
    import paper_1603_00937_amd as gb
    for emin, emax, beta, mu, order, nodes in [(-4.4, 4.3, 10.0, 0.1, 150, 0),
                                               (-1.0, 2.0, 3.0, -0.5, 20, 64),
                                               (-9.5, 9.7, 40.0, 0.3, 600, 0)]:
        got = np.array(gb.chebyshev_fermi(emin, emax, beta, mu, order, nodes))
        ref = fermi_coefficients(emin, emax, beta, mu, order, nodes or None)
        assert np.abs(got - ref).max() < 1e-14


def test_solve_mu_matches_oracle(lib):
    from oracle.foe import foe_partitioned, solve_mu
    import paper_1603_00937_amd as gb
    from synth import make_model
    m = make_model("small256")
    beta, order = 6.0, 60
    cols, info = foe_partitioned(m["H_col"], m["H_val"], 1e-5, 16, beta, order, n_occ=m["n_occ"])
    mu = gb.foe_solve_mu(info["traces"], info["emin"], info["emax"], beta, m["n_occ"])
    assert abs(mu - info["mu"]) < 1e-11
    # an occupation no mu in [emin, emax] reaches is rejected
    with pytest.raises(gb.GbError):
        gb.foe_solve_mu(info["traces"], info["emin"], info["emax"], beta, m["N"] + 5)


def test_foe_rejects_bad_arguments(lib):
    from paper_1603_00937_amd._lib import GbEll, GbFoeOpts, GB_EINVAL
    bogus = 0x1000
    H = GbEll(8, 3, bogus, bogus)
    D = GbEll(8, 8, bogus, bogus)
    o = GbFoeOpts()
    o.beta, o.order, o.mu = 5.0, 10, 0.0
    assert lib.gb_foe_density(ctypes.byref(H), 4, 1e-5, None, ctypes.byref(D), None, None) == GB_EINVAL
    o.beta = -1.0
    assert lib.gb_foe_density(ctypes.byref(H), 4, 1e-5, ctypes.byref(o), ctypes.byref(D), None, None) == GB_EINVAL
    o.beta, o.order = 5.0, 0
    assert lib.gb_foe_density(ctypes.byref(H), 4, 1e-5, ctypes.byref(o), ctypes.byref(D), None, None) == GB_EINVAL
    o.order, o.mu = 10, float("nan")
    assert lib.gb_foe_density(ctypes.byref(H), 40, 1e-5, ctypes.byref(o), ctypes.byref(D), None, None) == GB_EINVAL
    c = (ctypes.c_double * 4)()
    assert lib.gb_chebyshev_fermi(1.0, 0.0, 1.0, 0.0, 3, 0, c) == GB_EINVAL
    assert lib.gb_chebyshev_fermi(0.0, 1.0, 1.0, 0.0, 0, 0, c) == GB_EINVAL
    assert lib.gb_chebyshev_fermi(0.0, 1.0, 1.0, 0.0, 3, 0, None) == GB_EINVAL


def test_sp2_sequence_matches_oracle(lib):
    from oracle.sequence import sequence_from_gap
    import paper_1603_00937_amd as gb
    for args in [(-8.6, 8.7, -1.2, 0.48), (-4.4, 4.3, 0.1, 0.2), (0.0, 1.0, 0.30, 0.55)]:
        assert gb.sp2_sequence(*args) == sequence_from_gap(*args)
    with pytest.raises(gb.GbError):
        gb.sp2_sequence(0.0, 1.0, 0.6, 0.4)
    with pytest.raises(gb.GbError):
        gb.sp2_sequence(-8.6, 8.7, -1.2, 0.48, max_len=3)
