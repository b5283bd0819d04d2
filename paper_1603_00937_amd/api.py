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


def _release(obj, fn):
    """Destroy obj's library handle once.  At interpreter exit the module's globals may already
    be gone (objects alive then are collected after them); the process is ending and its device
    memory with it, so there is nothing to release."""
    h = getattr(obj, "_h", None)
    if not h or _lib is None or L is None:
        return
    try:
        getattr(_lib(), fn)(h)
    except (TypeError, AttributeError):  # module state already torn down at exit
        return
    obj._h = None


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


class TorchAllocator:
    """Device-memory hook that serves the library's allocations from torch's caching
    allocator (blocks are reused in the order of the stream they were allocated on).
    `live` maps pointer -> bytes of the blocks currently held by the library."""

    def __init__(self):
        self.live = {}
        self.n_alloc = 0
        self._alloc_fn = L.ALLOC_FN(self._alloc)
        self._free_fn = L.FREE_FN(self._free)

    def _alloc(self, nbytes, stream, ctx):
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
        except Exception:  # reported by the library as GB_ENOMEM
            return None
        self.live[p] = int(nbytes)
        self.n_alloc += 1
        return p

    def _free(self, ptr, stream, ctx):
        self.live.pop(ptr, None)
        torch.cuda.caching_allocator_delete(ptr)


_ALLOCATORS = []  # every hook ever registered stays alive: a buffer is freed by its maker


def set_allocator(allocator):
    """Route later library allocations through `allocator` (a TorchAllocator), or back to
    the library's own device pool with None."""
    if allocator is None:
        _check(_lib().gb_set_allocator(L.ALLOC_FN(), L.FREE_FN(), None))
        return
    _ALLOCATORS.append(allocator)
    _check(_lib().gb_set_allocator(allocator._alloc_fn, allocator._free_fn, None))


# kernel variant names of gb_sp2_opts.tile_policy
TILE_POLICIES = {"auto": 0, "128": 1, "64": 2, 128: 1, 64: 2, "64s3": 4, "64r": 5, "128i": 6,
                 "64i": 7}

PEAK_KINDS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "hbm": 4, "bf16_32x32": 5,
              "fp16_32x32": 6}


def peak_rate(kind, with_clock=False):
    """Rate this device sustains by the library's own kernels: matrix-core TFLOP/s for "fp64",
    "fp32", "bf16", "fp16" (16 x 16 instructions), "bf16_32x32", "fp16_32x32"; HBM GB/s (read +
    written) for "hbm".  with_clock: also the mean
    core clock (MHz) during the matrix-core loop, as (rate, clock)."""
    r, c = ctypes.c_double(), ctypes.c_double()
    _check(_lib().gb_peak_rate(PEAK_KINDS.get(kind, -1), _stream(), ctypes.byref(r),
                               ctypes.byref(c)))
    return (r.value, c.value) if with_clock else r.value


def tune_save(path) -> int:
    """Write the autotuner's table (JSON, tagged with the library build and device)."""
    n = ctypes.c_int32()
    _check(_lib().gb_tune_save(str(path).encode(), ctypes.byref(n)))
    return n.value


def tune_load(path) -> int:
    """Merge a table written by tune_save on this device and library build."""
    n = ctypes.c_int32()
    _check(_lib().gb_tune_load(str(path).encode(), ctypes.byref(n)))
    return n.value


def trim():
    """Free the batch buffers the library caches between calls."""
    _check(_lib().gb_trim())


def spectral_bounds(H_col, H_val):
    """Gershgorin (e_min, e_max) of H."""
    H = _ell(H_col, H_val)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(_lib().gb_spectral_bounds(ctypes.byref(H), _stream(), ctypes.byref(lo),
                                     ctypes.byref(hi)))
    return lo.value, hi.value


def spectral_bounds_noalloc(H_col, H_val):
    """Gershgorin (e_min, e_max) of H without any device allocation (the library's fixed
    scratch array holds the partials; calls overlapping on one GPU race)."""
    H = _ell(H_col, H_val)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(_lib().gb_spectral_bounds_noalloc(ctypes.byref(H), _stream(), ctypes.byref(lo),
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

    def views(self):
        """Device pointers (row_ptr, col) owned by the graph (read-only, valid while it lives)."""
        rp, col = ctypes.c_void_p(), ctypes.c_void_p()
        _check(_lib().gb_graph_view(self._h, None, None, ctypes.byref(rp), ctypes.byref(col)))
        return rp.value, col.value

    def arrays(self):
        rp = torch.empty(self.n + 1, dtype=torch.int32, device="cuda")
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device="cuda")
        _check(_lib().gb_graph_copy(self._h, rp.data_ptr(), col.data_ptr(), _stream()))
        return rp, col[:self.nnz]

    def __del__(self):
        _release(self, "gb_graph_destroy")


def build_graph(H_col, H_val, tau, mode="x2", aux=None, tau_aux=0.0) -> Graph:
    H = _ell(H_col, H_val)
    A = _ell(*aux) if aux is not None else None
    out = ctypes.c_void_p()
    _check(_lib().gb_build_graph(ctypes.byref(H), ctypes.byref(A) if A is not None else None,
                                 float(tau), float(tau_aux), L.GRAPH_MODES[mode], _stream(),
                                 ctypes.byref(out)))
    return Graph(out)


def build_graph_rcut(pos, box, r_cut, orbs_per_site=2) -> Graph:
    """Divide-and-conquer comparison graph: orbitals adjacent when their sites are closer than
    r_cut (minimum image in the periodic cube of edge ``box``).  pos: GPU float64 [n_sites, 3]."""
    _dev(pos, torch.float64, "pos")
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be [n_sites, 3]")
    out = ctypes.c_void_p()
    _check(_lib().gb_build_graph_rcut(pos.data_ptr(), pos.shape[0], int(orbs_per_site),
                                      float(box), float(r_cut), _stream(), ctypes.byref(out)))
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

    def views(self):
        """Device pointers (core_ptr, sub_ptr, sub_idx) owned by the partition (read-only)."""
        a, b, c = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(_lib().gb_partition_view(self._h, None, None, ctypes.byref(a), ctypes.byref(b),
                                        ctypes.byref(c)))
        return a.value, b.value, c.value

    def arrays(self):
        cp = torch.empty(self.n_sub + 1, dtype=torch.int32, device="cuda")
        sp = torch.empty(self.n_sub + 1, dtype=torch.int32, device="cuda")
        si = torch.empty(max(self.total, 1), dtype=torch.int32, device="cuda")
        _check(_lib().gb_partition_copy(self._h, cp.data_ptr(), sp.data_ptr(), si.data_ptr(),
                                        _stream()))
        return cp, sp, si[:self.total]

    def __del__(self):
        _release(self, "gb_partition_destroy")


def partition(graph: Graph, core_size: int, method="block") -> Partition:
    out = ctypes.c_void_p()
    _check(_lib().gb_partition(graph.handle, int(core_size), L.PART_METHODS[method], _stream(),
                               ctypes.byref(out)))
    return Partition(out)


def partition_update(graph: Graph, prev: Partition) -> Partition:
    """The cores of ``prev`` carried to ``graph`` (same vertices) with their new halos
    (on-the-fly update between MD steps)."""
    out = ctypes.c_void_p()
    _check(_lib().gb_partition_update(graph.handle, prev.handle, _stream(), ctypes.byref(out)))
    return Partition(out)


def partition_update_host(row_ptr, col, prev_core_ptr, prev_core_vtx):
    """Host form of partition_update on numpy CSR and core arrays."""
    import numpy as np
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    pp = np.ascontiguousarray(prev_core_ptr, dtype=np.int32)
    pv = np.ascontiguousarray(prev_core_vtx, dtype=np.int32)
    n = len(rp) - 1
    cp = np.zeros(n + 1, dtype=np.int32)
    cv = np.zeros(max(n, 1), dtype=np.int32)
    nc = ctypes.c_int32()
    cost = ctypes.c_int64()
    i32 = ctypes.POINTER(ctypes.c_int32)
    _check(_lib().gb_partition_update_host(n, rp.ctypes.data_as(i32), cl.ctypes.data_as(i32),
                                           len(pp) - 1, pp.ctypes.data_as(i32),
                                           pv.ctypes.data_as(i32), ctypes.byref(nc),
                                           cp.ctypes.data_as(i32), cv.ctypes.data_as(i32),
                                           ctypes.byref(cost)))
    return cp[:nc.value + 1].copy(), cv[:n].copy(), int(cost.value)


def partition_host(row_ptr, col, core_size):
    """Host: the multilevel cores of a host CSR graph (numpy int32 arrays).  Returns
    (core_ptr, core_vtx, cost) as numpy arrays and the summed (|core| + |halo|)^3."""
    import numpy as np
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    n = len(rp) - 1
    cp = np.zeros(n + 1, dtype=np.int32)
    cv = np.zeros(max(n, 1), dtype=np.int32)
    nc = ctypes.c_int32()
    cost = ctypes.c_int64()
    i32 = ctypes.POINTER(ctypes.c_int32)
    _check(_lib().gb_partition_host(n, rp.ctypes.data_as(i32), cl.ctypes.data_as(i32),
                                    int(core_size), ctypes.byref(nc), cp.ctypes.data_as(i32),
                                    cv.ctypes.data_as(i32), ctypes.byref(cost)))
    return cp[:nc.value + 1].copy(), cv[:n].copy(), int(cost.value)


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
                "square", "square_lo")},
        "n_square": st.n_square, "n_square_lo": st.n_square_lo, "n_tile64": st.n_tile64,
        "n_refine_done": st.n_refine_done, "planes_db": st.planes_db, "n_stage3": st.n_stage3,
        "n_regstage": st.n_regstage,
        "square_flops": st.square_flops,
        "square_flops_exec": st.square_flops_exec,
        "n_near_tie": st.n_near_tie,
        "n_split_il": st.n_split_il,
    }


class Tape:
    """Recorded SP2 expansion (checkpoints) for the adjoint."""

    def __init__(self, handle, H_col, width):
        self._h = handle
        self.H_col = H_col
        self.width = width

    def vjp(self, G_D_val, G_H_val=None):
        """dL/dH on H's ELL pattern from dL/dD on D's column-ELL pattern."""
        _dev(G_D_val, torch.float64, "G_D_val")
        n = self.H_col.shape[0]
        if G_D_val.dim() != 2 or G_D_val.shape[0] != n:
            raise ValueError("G_D_val must be [n, width]")
        if G_H_val is None:
            G_H_val = torch.empty(self.H_col.shape, dtype=torch.float64, device="cuda")
        Gd = L.GbEll(n, G_D_val.shape[1], None, G_D_val.data_ptr())
        Gh = _ell(self.H_col, G_H_val)
        _check(_lib().gb_density_vjp(self._h, ctypes.byref(Gd), ctypes.byref(Gh), _stream()))
        return G_H_val

    def __del__(self):
        _release(self, "gb_tape_destroy")


def _sp2_opts(precision="fp64", n_refine=0, max_iter=0, idem_tol=0.0, part=None, core_size=32,
              refine="mcweeny", n_fp64_first=0, keep_tape=False, tape_stride=0, launch_mode=0,
              tile_policy="auto", tile_order="xcd", check_idem=False, emin=None, emax=None):
    o = L.GbSp2Opts()
    o.precision = L.PRECISIONS[precision]
    o.n_refine = int(n_refine)
    o.refine_kind = {"mcweeny": 0, "sp2": 1, "mcweeny_blocks": 2}[refine]
    o.n_fp64_first = int(n_fp64_first)
    o.max_iter = int(max_iter)
    o.idem_tol = float(idem_tol)
    o.partition = part.handle if part is not None else None
    o.core_size = int(core_size)
    if emin is not None and emax is not None:
        o.emin, o.emax = float(emin), float(emax)
    o.keep_tape = 1 if keep_tape else 0
    o.tape_stride = int(tape_stride)
    o.launch_mode = L.LAUNCH_MODES.get(launch_mode, launch_mode)
    o.tile_policy = TILE_POLICIES.get(tile_policy, tile_policy)
    o.tile_order = {"xcd": 0, "plain": 1}[tile_order]
    o.check_idem = 1 if check_idem else 0
    return o


def density_workspace(H_col, partition, precision="fp64", **kw) -> int:
    """Bytes of caller-owned workspace :func:`density` needs on ``partition`` (pass a uint8
    GPU tensor of at least this size as ``workspace=``)."""
    _dev(H_col, torch.int32, "H_col")
    H = L.GbEll(H_col.shape[0], H_col.shape[1], H_col.data_ptr(), None)
    o = _sp2_opts(precision=precision, part=partition, **kw)
    nb = ctypes.c_size_t()
    _check(_lib().gb_density_workspace(ctypes.byref(H), ctypes.byref(o), ctypes.byref(nb)))
    return nb.value


def density(H_col, H_val, n_occ, threshold, partition=None, core_size=32, precision="fp64",
            n_refine=0, max_iter=0, idem_tol=0.0, branch_in=None, emin=None, emax=None,
            D=None, refine="mcweeny", n_fp64_first=0, keep_tape=False, tape_stride=0, launch_mode=0,
            tile_policy="auto", tile_order="xcd", check_idem=False, workspace=None):
    """Partitioned SP2 density matrix.  Returns (D_col, D_val, stats); D is column-ELL
    [n, max_sub] (row i of the arrays = column i of D).  With ``partition`` None the X2 graph
    at ``threshold`` and a block partition with ``core_size`` are built first.  ``workspace``:
    a uint8 GPU tensor of at least :func:`density_workspace` bytes for the batch buffers
    (needs ``partition``)."""
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
    o = _sp2_opts(precision, n_refine, max_iter, idem_tol, part, core_size, refine, n_fp64_first,
                  keep_tape, tape_stride, launch_mode, tile_policy, tile_order, check_idem,
                  emin, emax)
    if workspace is not None:
        if partition is None:
            raise ValueError("a caller-owned workspace needs a partition")
        _dev(workspace, torch.uint8, "workspace")
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel()
    keep = None
    if branch_in is not None:
        keep = (ctypes.c_uint8 * max(len(branch_in), 1))(*[int(b) for b in branch_in])
        o.branch_in = ctypes.cast(keep, ctypes.c_void_p)
        o.n_branch_in = len(branch_in)
    st = L.GbSp2Stats()
    _check(_lib().gb_density(ctypes.byref(H), int(n_occ), float(threshold), ctypes.byref(o),
                             ctypes.byref(De), ctypes.byref(st), _stream()))
    out = _stats_dict(st)
    if keep_tape:
        out["tape"] = Tape(ctypes.c_void_p(st.tape), H_col, D_col.shape[1])
    return D_col, D_val, out


def chebyshev_fermi(emin, emax, beta, mu, order, n_nodes=0):
    """Host: Chebyshev coefficients c_0 .. c_order of the Fermi function on [emin, emax]."""
    c = (ctypes.c_double * (int(order) + 1))()
    _check(_lib().gb_chebyshev_fermi(float(emin), float(emax), float(beta), float(mu),
                                     int(order), int(n_nodes), c))
    return list(c)


def sp2_sequence(emin, emax, e_homo, e_lumo, delta=1e-12, max_len=127):
    """Host: the pre-determined SP2 branch sequence for a HOMO/LUMO pair (list of 0/1)."""
    out = (ctypes.c_uint8 * max(int(max_len), 1))()
    n = ctypes.c_int32()
    _check(_lib().gb_sp2_sequence(float(emin), float(emax), float(e_homo), float(e_lumo),
                                  float(delta), int(max_len), out, ctypes.byref(n)))
    return [int(out[i]) for i in range(n.value)]


def sp2_estimate_gap(t1, t2, branch, n_occ, emin, emax, floor=0.0):
    """Host: HOMO/LUMO bracket from an SP2 expansion's core traces (t1, t2: one more entry than
    branch).  From a density() stats dict: ``sp2_estimate_gap(**gap_inputs(st, n_occ))``.  Returns a
    dict: homo_bound >= e_homo, lumo_bound <= e_lumo, homo_ratio <= e_homo, lumo_ratio >= e_lumo,
    floor, homo_iter, lumo_iter."""
    nb = len(branch)
    if len(t1) < nb + 1 or len(t2) < nb + 1:
        raise ValueError("t1 and t2 need len(branch) + 1 entries")
    a1 = (ctypes.c_double * (nb + 1))(*[float(x) for x in t1[:nb + 1]])
    a2 = (ctypes.c_double * (nb + 1))(*[float(x) for x in t2[:nb + 1]])
    b = (ctypes.c_uint8 * max(nb, 1))(*[int(x) for x in branch])
    r = L.GbGapEstimate()
    _check(_lib().gb_sp2_estimate_gap(a1, a2, b, nb, float(n_occ), float(emin), float(emax),
                                      float(floor), ctypes.byref(r)))
    return {"homo_bound": r.homo_bound, "lumo_bound": r.lumo_bound,
            "homo_ratio": r.homo_ratio, "lumo_ratio": r.lumo_ratio, "floor": r.floor,
            "homo_iter": tuple(r.homo_iter), "lumo_iter": tuple(r.lumo_iter)}


def gap_inputs(st, n_occ):
    """The arguments of sp2_estimate_gap from a density() stats dict."""
    k = st["iters"]
    return {"t1": st["t1"][:k + 1], "t2": st["t2"][:k + 1], "branch": st["branch"][:k],
            "n_occ": n_occ, "emin": st["emin"], "emax": st["emax"]}


def foe_solve_mu(traces, emin, emax, beta, n_occ, n_nodes=0):
    """Host: mu with sum_n c_n(mu) traces[n] = n_occ."""
    t = (ctypes.c_double * len(traces))(*[float(x) for x in traces])
    mu = ctypes.c_double()
    _check(_lib().gb_foe_solve_mu(t, len(traces) - 1, float(emin), float(emax), float(beta),
                                  float(n_occ), int(n_nodes), ctypes.byref(mu)))
    return mu.value


def foe_density(H_col, H_val, n_occ, threshold, beta, order, mu=None, partition=None,
                core_size=32, n_nodes=0, emin=None, emax=None, D=None, tile_policy="auto",
                tile_order="xcd"):
    """Finite-temperature density matrix by the partitioned Chebyshev expansion of the Fermi
    function (mu None: solved so that the summed core traces equal n_occ).  Returns
    (D_col, D_val, stats) with D column-ELL as in :func:`density`."""
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
    o = L.GbFoeOpts()
    o.beta = float(beta)
    o.mu = float("nan") if mu is None else float(mu)
    o.order = int(order)
    o.n_nodes = int(n_nodes)
    o.partition = part.handle
    o.core_size = int(core_size)
    if emin is not None and emax is not None:
        o.emin, o.emax = float(emin), float(emax)
    o.tile_policy = TILE_POLICIES.get(tile_policy, tile_policy)
    o.tile_order = {"xcd": 0, "plain": 1}[tile_order]
    tr = (ctypes.c_double * (int(order) + 1))()
    o.traces = ctypes.cast(tr, ctypes.c_void_p)
    st = L.GbFoeStats()
    _check(_lib().gb_foe_density(ctypes.byref(H), int(n_occ), float(threshold), ctypes.byref(o),
                                 ctypes.byref(De), ctypes.byref(st), _stream()))
    out = {f: getattr(st, f) for f, _ in L.GbFoeStats._fields_}
    out["traces"] = list(tr)
    return D_col, D_val, out


class DensityFn(torch.autograd.Function):
    """D_val = DensityFn.apply(H_val, H_col, n_occ, threshold, partition, core_size):
    the partitioned SP2 density matrix (column-ELL values; the row indices are in
    ``ctx``-independent D_col returned by :func:`density_with_grad`).  Backward runs the
    library's adjoint; the graph, partition, bounds and branch sequence are held fixed."""

    @staticmethod
    def forward(ctx, H_val, H_col, n_occ, threshold, part, core_size, D_col_out):
        D_col, D_val, st = density(H_col, H_val.detach(), n_occ, threshold, partition=part,
                                   core_size=core_size, keep_tape=True)
        D_col_out.append(D_col)
        D_col_out.append(st)
        ctx.tape = st.pop("tape")
        ctx.mark_non_differentiable(D_col)
        return D_val

    @staticmethod
    def backward(ctx, g):
        G_H = ctx.tape.vjp(g.contiguous())
        return G_H, None, None, None, None, None, None


def density_with_grad(H_col, H_val, n_occ, threshold, partition=None, core_size=32):
    """(D_col, D_val, stats) with D_val differentiable with respect to H_val."""
    if partition is None:
        partition = globals()["partition"](build_graph(H_col, H_val.detach(), threshold), core_size)
    box = []
    D_val = DensityFn.apply(H_val, H_col, n_occ, threshold, partition, core_size, box)
    return box[0], D_val, box[1]
