"""Torch-facing wrappers of the libgb C ABI.  Argument marshalling only: no arithmetic of
the method happens here, and a missing library is an error (there is no fallback)."""
import ctypes

import torch

from . import _lib as L


class GbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _lib():
    return L.load()


def _check(status):
    if status != L.GB_OK:
        raise GbError(status, _lib().gb_last_error().decode(errors="replace"))


def version() -> str:
    return _lib().gb_version().decode()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ell(col, val):
    _dev(col, torch.int32, "col")
    if val is not None:
        _dev(val, torch.float64, "val")
        if val.shape != col.shape:
            raise ValueError("col and val shapes differ")
    if col.dim() != 2:
        raise ValueError("ELL arrays are 2-D [n, width]")
    return L.GbEll(col.shape[0], col.shape[1], col.data_ptr(),
                   val.data_ptr() if val is not None else None)


def spectral_bounds(H_col, H_val):
    """Gershgorin (e_min, e_max) of H."""
    H = _ell(H_col, H_val)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(_lib().gb_spectral_bounds(ctypes.byref(H), _stream(), ctypes.byref(lo),
                                     ctypes.byref(hi)))
    return lo.value, hi.value


class Graph:
    """Device CSR graph owned by the library."""

    def __init__(self, handle):
        self._h = handle
        n, nnz = ctypes.c_int32(), ctypes.c_int64()
        _check(_lib().gb_graph_info(handle, ctypes.byref(n), ctypes.byref(nnz)))
        self.n, self.nnz = n.value, nnz.value

    @property
    def handle(self):
        return self._h

    def arrays(self):
        rp = torch.empty(self.n + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device="cuda")
        _check(_lib().gb_graph_copy(self._h, rp.data_ptr(), col.data_ptr(), _stream()))
        return rp, col[:self.nnz]

    def __del__(self):
        if getattr(self, "_h", None):
            _lib().gb_graph_destroy(self._h)
            self._h = None


def build_graph(H_col, H_val, tau, mode="x2", aux=None, tau_aux=0.0) -> Graph:
    H = _ell(H_col, H_val)
    A = _ell(*aux) if aux is not None else None
    out = ctypes.c_void_p()
    _check(_lib().gb_build_graph(ctypes.byref(H), ctypes.byref(A) if A is not None else None,
                                 float(tau), float(tau_aux), L.GRAPH_MODES[mode], _stream(),
                                 ctypes.byref(out)))
    return Graph(out)


class Partition:
    """Cores and core+halo subgraph lists owned by the library."""

    def __init__(self, handle):
        self._h = handle
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(_lib().gb_partition_info(handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        self.n_sub, self.max_sub, self.total = a.value, b.value, c.value

    @property
    def handle(self):
        return self._h

    def arrays(self):
        cp = torch.empty(self.n_sub + 1, dtype=torch.int32, device="cuda")
        sp = torch.empty(self.n_sub + 1, dtype=torch.int32, device="cuda")
        si = torch.empty(max(self.total, 1), dtype=torch.int32, device="cuda")
        _check(_lib().gb_partition_copy(self._h, cp.data_ptr(), sp.data_ptr(), si.data_ptr(),
                                        _stream()))
        return cp, sp, si[:self.total]

    def __del__(self):
        if getattr(self, "_h", None):
            _lib().gb_partition_destroy(self._h)
            self._h = None


def partition(graph: Graph, core_size: int, method="block") -> Partition:
    out = ctypes.c_void_p()
    _check(_lib().gb_partition(graph.handle, int(core_size), L.PART_METHODS[method], _stream(),
                               ctypes.byref(out)))
    return Partition(out)


def _stats_dict(st: L.GbSp2Stats) -> dict:
    k = st.iters
    nt = min(k + 1, 128)
    return {
        "iters": k, "converged": bool(st.converged), "n_sub": st.n_sub, "max_sub": st.max_sub,
        "branch": [int(b) for b in st.branch[:min(k, 128)]],
        "trace": st.trace, "idem": st.idem, "idem_max": st.idem_max,
        "emin": st.emin, "emax": st.emax, "min_margin": st.min_margin,
        "t1": list(st.t1[:nt]), "t2": list(st.t2[:nt]),
        "ms": {n: getattr(st, "ms_" + n) for n in
               ("bounds", "graph", "part", "gather", "sp2", "refine", "scatter", "total",
                "square")},
        "n_square": st.n_square, "square_flops": st.square_flops,
        "square_flops_exec": st.square_flops_exec,
    }


def density(H_col, H_val, n_occ, threshold, partition=None, core_size=32, precision="fp64",
            n_refine=0, max_iter=0, idem_tol=0.0, branch_in=None, emin=None, emax=None,
            D=None):
    """Partitioned SP2 density matrix.  Returns (D_col, D_val, stats); D is column-ELL
    [n, max_sub] (row i of the arrays = column i of D).  With ``partition`` None the X2 graph
    at ``threshold`` and a block partition with ``core_size`` are built first."""
    H = _ell(H_col, H_val)
    part = partition
    if part is None:
        part = globals()["partition"](build_graph(H_col, H_val, threshold), core_size)
    n = H.n
    if D is None:
        D_col = torch.empty((n, part.max_sub), dtype=torch.int32, device="cuda")
        D_val = torch.empty((n, part.max_sub), dtype=torch.float64, device="cuda")
    else:
        D_col, D_val = D
    De = _ell(D_col, D_val)
    o = L.GbSp2Opts()
    o.precision = L.PRECISIONS[precision]
    o.n_refine = int(n_refine)
    o.max_iter = int(max_iter)
    o.idem_tol = float(idem_tol)
    o.partition = part.handle
    o.core_size = int(core_size)
    keep = None
    if branch_in is not None:
        keep = (ctypes.c_uint8 * max(len(branch_in), 1))(*[int(b) for b in branch_in])
        o.branch_in = ctypes.cast(keep, ctypes.c_void_p)
        o.n_branch_in = len(branch_in)
    if emin is not None and emax is not None:
        o.emin, o.emax = float(emin), float(emax)
    st = L.GbSp2Stats()
    _check(_lib().gb_density(ctypes.byref(H), int(n_occ), float(threshold), ctypes.byref(o),
                             ctypes.byref(De), ctypes.byref(st), _stream()))
    return D_col, D_val, _stats_dict(st)
