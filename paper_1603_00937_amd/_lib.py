"""ctypes view of the libgb C ABI (include/gb.h).  Argument marshalling only."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgb.so")

GB_OK, GB_EINVAL, GB_ENOMEM, GB_EHIP, GB_ESHAPE, GB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "GB_OK", -1: "GB_EINVAL", -2: "GB_ENOMEM", -3: "GB_EHIP", -4: "GB_ESHAPE",
                -5: "GB_EUNSUPPORTED"}
GRAPH_MODES = {"x2": 0, "pattern": 1, "dprev": 2, "dprev_symbolic": 3}
PART_METHODS = {"block": 0, "bfs": 1, "multilevel": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "bf16x6": 4, "fp16x3": 5}
# launch modes of gb_density ("batched" is the device-driven default)
LAUNCH_MODES = {"device": 0, "batched": 0, "per_subgraph": 1, "graph": 2, "host": 3}


class GbEll(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("width", ctypes.c_int32),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class GbSp2Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("n_refine", ctypes.c_int32),
                ("refine_kind", ctypes.c_int32), ("n_fp64_first", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("idem_tol", ctypes.c_double),
                ("partition", ctypes.c_void_p), ("core_size", ctypes.c_int32),
                ("branch_in", ctypes.c_void_p), ("n_branch_in", ctypes.c_int32),
                ("emin", ctypes.c_double), ("emax", ctypes.c_double),
                ("keep_tape", ctypes.c_int32), ("tape_stride", ctypes.c_int32),
                ("launch_mode", ctypes.c_int32), ("tile_policy", ctypes.c_int32),
                ("tile_order", ctypes.c_int32), ("check_idem", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class GbSp2Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("n_sub", ctypes.c_int32), ("max_sub", ctypes.c_int32),
                ("branch", ctypes.c_uint8 * 128),
                ("trace", ctypes.c_double), ("idem", ctypes.c_double),
                ("idem_max", ctypes.c_double), ("emin", ctypes.c_double),
                ("emax", ctypes.c_double), ("min_margin", ctypes.c_double),
                ("t1", ctypes.c_double * 128), ("t2", ctypes.c_double * 128),
                ("ms_bounds", ctypes.c_float), ("ms_graph", ctypes.c_float),
                ("ms_part", ctypes.c_float), ("ms_gather", ctypes.c_float),
                ("ms_sp2", ctypes.c_float), ("ms_refine", ctypes.c_float),
                ("ms_scatter", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("ms_square", ctypes.c_float), ("n_square", ctypes.c_int32),
                ("ms_square_lo", ctypes.c_float), ("n_square_lo", ctypes.c_int32),
                ("n_tile64", ctypes.c_int32), ("n_refine_done", ctypes.c_int32),
                ("planes_db", ctypes.c_int32), ("n_stage3", ctypes.c_int32),
                ("n_regstage", ctypes.c_int32),
                ("square_flops", ctypes.c_double), ("square_flops_exec", ctypes.c_double),
                ("tape", ctypes.c_void_p), ("n_near_tie", ctypes.c_int32),
                ("n_split_il", ctypes.c_int32)]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
class GbFoeOpts(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("mu", ctypes.c_double),
                ("order", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("partition", ctypes.c_void_p), ("core_size", ctypes.c_int32),
                ("emin", ctypes.c_double), ("emax", ctypes.c_double),
                ("tile_policy", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("traces", ctypes.c_void_p)]


class GbFoeStats(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("trace", ctypes.c_double),
                ("coef_tail", ctypes.c_double), ("emin", ctypes.c_double),
                ("emax", ctypes.c_double), ("n_sub", ctypes.c_int32),
                ("max_sub", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("ms_bounds", ctypes.c_float), ("ms_graph", ctypes.c_float),
                ("ms_part", ctypes.c_float), ("ms_gather", ctypes.c_float),
                ("ms_terms", ctypes.c_float), ("ms_scatter", ctypes.c_float),
                ("ms_total", ctypes.c_float), ("ms_product", ctypes.c_float),
                ("n_product", ctypes.c_int32), ("product_flops", ctypes.c_double)]


class GbGapEstimate(ctypes.Structure):
    _fields_ = [("homo_bound", ctypes.c_double), ("lumo_bound", ctypes.c_double),
                ("homo_ratio", ctypes.c_double), ("lumo_ratio", ctypes.c_double),
                ("floor", ctypes.c_double), ("homo_iter", ctypes.c_int32 * 3),
                ("lumo_iter", ctypes.c_int32 * 3)]


# gb_alloc_fn / gb_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

SIGNATURES = {
    "gb_version": (ctypes.c_char_p, []),
    "gb_last_error": (ctypes.c_char_p, []),
    "gb_spectral_bounds": (ctypes.c_int32, [_P(GbEll), _vp, _P(ctypes.c_double),
                                            _P(ctypes.c_double)]),
    "gb_spectral_bounds_noalloc": (ctypes.c_int32, [_P(GbEll), _vp, _P(ctypes.c_double),
                                                    _P(ctypes.c_double)]),
    "gb_build_graph": (ctypes.c_int32, [_P(GbEll), _P(GbEll), ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int32, _vp, _P(_vp)]),
    "gb_build_graph_rcut": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_double, _vp, _P(_vp)]),
    "gb_graph_info": (ctypes.c_int32, [_vp, _P(ctypes.c_int32), _P(ctypes.c_int64)]),
    "gb_graph_copy": (ctypes.c_int32, [_vp, _vp, _vp, _vp]),
    "gb_graph_view": (ctypes.c_int32, [_vp, _P(ctypes.c_int32), _P(ctypes.c_int64), _P(_vp),
                                       _P(_vp)]),
    "gb_graph_destroy": (None, [_vp]),
    "gb_partition": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _P(_vp)]),
    "gb_partition_host": (ctypes.c_int32, [ctypes.c_int32, _P(ctypes.c_int32), _P(ctypes.c_int32),
                                           ctypes.c_int32, _P(ctypes.c_int32),
                                           _P(ctypes.c_int32), _P(ctypes.c_int32),
                                           _P(ctypes.c_int64)]),
    "gb_partition_update": (ctypes.c_int32, [_vp, _vp, _vp, _P(_vp)]),
    "gb_partition_update_host": (ctypes.c_int32, [ctypes.c_int32, _P(ctypes.c_int32),
                                                  _P(ctypes.c_int32),
                                                  ctypes.c_int32, _P(ctypes.c_int32),
                                                  _P(ctypes.c_int32), _P(ctypes.c_int32),
                                                  _P(ctypes.c_int32), _P(ctypes.c_int32),
                                                  _P(ctypes.c_int64)]),
    "gb_partition_info": (ctypes.c_int32, [_vp, _P(ctypes.c_int32), _P(ctypes.c_int32),
                                           _P(ctypes.c_int64)]),
    "gb_partition_copy": (ctypes.c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "gb_partition_view": (ctypes.c_int32, [_vp, _P(ctypes.c_int32), _P(ctypes.c_int32), _P(_vp),
                                           _P(_vp), _P(_vp)]),
    "gb_partition_destroy": (None, [_vp]),
    "gb_set_allocator": (ctypes.c_int32, [ALLOC_FN, FREE_FN, _vp]),
    "gb_trim": (ctypes.c_int32, []),
    "gb_peak_rate": (ctypes.c_int32, [ctypes.c_int32, _vp, _P(ctypes.c_double),
                                      _P(ctypes.c_double)]),
    "gb_tune_save": (ctypes.c_int32, [ctypes.c_char_p, _P(ctypes.c_int32)]),
    "gb_tune_load": (ctypes.c_int32, [ctypes.c_char_p, _P(ctypes.c_int32)]),
    "gb_density": (ctypes.c_int32, [_P(GbEll), ctypes.c_int32, ctypes.c_double, _P(GbSp2Opts),
                                    _P(GbEll), _P(GbSp2Stats), _vp]),
    "gb_density_workspace": (ctypes.c_int32, [_P(GbEll), _P(GbSp2Opts), _P(ctypes.c_size_t)]),
    "gb_density_vjp": (ctypes.c_int32, [_vp, _P(GbEll), _P(GbEll), _vp]),
    "gb_tape_destroy": (None, [_vp]),
    "gb_foe_density": (ctypes.c_int32, [_P(GbEll), ctypes.c_int32, ctypes.c_double,
                                        _P(GbFoeOpts), _P(GbEll), _P(GbFoeStats), _vp]),
    "gb_chebyshev_fermi": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                            _P(ctypes.c_double)]),
    "gb_sp2_sequence": (ctypes.c_int32, [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                         _P(ctypes.c_uint8), _P(ctypes.c_int32)]),
    "gb_sp2_estimate_gap": (ctypes.c_int32, [_P(ctypes.c_double), _P(ctypes.c_double),
                                             _P(ctypes.c_uint8), ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             _P(GbGapEstimate)]),
    "gb_foe_solve_mu": (ctypes.c_int32, [_P(ctypes.c_double), ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int32, _P(ctypes.c_double)]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgb.so (built by paper_1603_00937_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgb.so not found at {path}: run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
