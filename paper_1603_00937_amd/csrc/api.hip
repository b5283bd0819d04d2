// C ABI entry points: argument checks on the host, handle management, error strings.
// C++ exceptions raised inside the library are converted to gb_status codes here.
#include "internal.h"

#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>

namespace gbi {

namespace {
thread_local char g_err[1024] = "";
std::once_flag g_pool_once;
}  // namespace

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void fail(gb_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  throw Error{code};
}

Allocator g_alloc;  // the registered hook (all null: the device pool)

void* dmalloc(size_t bytes, hipStream_t s, Allocator* used) {
  *used = g_alloc;
  void* p = nullptr;
  if (used->alloc) {
    p = used->alloc(bytes ? bytes : 1, (void*)s, used->ctx);
    if (!p) fail(GB_ENOMEM, "registered allocator returned NULL for %zu bytes", bytes);
    return p;
  }
  // keep freed pool memory cached instead of returning it at every synchronisation
  std::call_once(g_pool_once, [] {
    int dev = 0;
    hipMemPool_t pool;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  });
  const hipError_t e = hipMallocAsync(&p, bytes ? bytes : 1, s);
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    fail(GB_ENOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  return p;
}

void dfree(void* p, hipStream_t s, const Allocator& a) {
  if (!p) return;
  if (a.free) a.free(p, (void*)s, a.ctx);
  else (void)hipFreeAsync(p, s);
}

size_t workspace_total(const size_t slot[Workspace::kSlots]) {
  size_t t = 0;
  for (int i = 0; i < Workspace::kSlots; ++i) t += (slot[i] + 255) / 256 * 256;
  return t;
}

void workspace_layout(Workspace& w, void* base, size_t bytes, const size_t slot[Workspace::kSlots]) {
  const size_t need = workspace_total(slot);
  if (bytes < need)
    fail(GB_ESHAPE, "workspace of %zu bytes is smaller than the %zu bytes this call needs", bytes,
         need);
  if (reinterpret_cast<uintptr_t>(base) % 256)
    fail(GB_EINVAL, "workspace must be 256-byte aligned");
  w.ext = static_cast<char*>(base);
  size_t off = 0;
  for (int i = 0; i < Workspace::kSlots; ++i) {
    w.ext_off[i] = off;
    w.ext_size[i] = slot[i];
    off += (slot[i] + 255) / 256 * 256;
  }
}

void* Workspace::get_bytes(int slot, size_t bytes, hipStream_t s) {
  if (ext) {
    if (bytes > ext_size[slot])
      fail(GB_ESHAPE, "workspace slot %d needs %zu bytes, its layout holds %zu", slot, bytes,
           ext_size[slot]);
    return ext + ext_off[slot];
  }
  Slab& b = slab[slot];
  if (bytes > b.bytes) {
    if (b.p) dfree(b.p, s, b.a);
    b.p = nullptr;
    b.bytes = 0;
    const size_t want = bytes + bytes / 16;  // headroom: sizes drift between MD steps
    b.p = dmalloc(want, s, &b.a);
    b.bytes = want;
  }
  return b.p;
}

void Workspace::release_all() {
  for (auto& b : slab) {
    if (b.p) dfree(b.p, nullptr, b.a);
    b.p = nullptr;
    b.bytes = 0;
  }
}

std::mutex g_ws_mu;
std::vector<Workspace*> g_ws_idle;

Workspace* ws_acquire() {
  int dev = 0;
  GB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (size_t i = 0; i < g_ws_idle.size(); ++i)
    if (g_ws_idle[i]->device == dev) {
      Workspace* w = g_ws_idle[i];
      g_ws_idle.erase(g_ws_idle.begin() + i);
      return w;
    }
  Workspace* w = new Workspace();
  w->device = dev;
  return w;
}

void ws_release(Workspace* w) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  g_ws_idle.push_back(w);
}

void ws_trim() {
  std::vector<Workspace*> idle;
  {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    idle.swap(g_ws_idle);
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (Workspace* w : idle) {
    (void)hipSetDevice(w->device);
    (void)hipDeviceSynchronize();
    w->release_all();
    delete w;
  }
  (void)hipSetDevice(cur);
}

void density(const gb_ell& H, int32_t n_occ, const gb_sp2_opts& o, const Part& P, double emin,
             double emax, const double* x0, gb_ell& D, gb_sp2_stats& st, hipStream_t s,
             TapeData** tape_out, Workspace* ext);

void detach(Csr& c) {
  c.row_ptr.detach_stream();
  c.col.detach_stream();
}
void detach(Part& p) {
  p.core_ptr.detach_stream();
  p.core_vtx.detach_stream();
  p.sub_ptr.detach_stream();
  p.sub_idx.detach_stream();
  p.sub_pos.detach_stream();
  p.col_sub.detach_stream();
  p.col_loc.detach_stream();
}

}  // namespace gbi

using namespace gbi;

namespace {

template <typename F>
gb_status guarded(F&& f) {
  try {
    f();
    g_err[0] = '\0';
    return GB_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GB_ENOMEM;
  } catch (...) {
    set_error("unexpected internal error");
    return GB_EHIP;
  }
}

void check_ell(const gb_ell* A, const char* name, bool need_val = true) {
  if (!A) fail(GB_EINVAL, "%s is NULL", name);
  if (A->n <= 0) fail(GB_EINVAL, "%s->n = %d must be positive", name, A->n);
  if (A->width <= 0) fail(GB_EINVAL, "%s->width = %d must be positive", name, A->width);
  if (!A->col) fail(GB_EINVAL, "%s->col is NULL", name);
  if (need_val && !A->val) fail(GB_EINVAL, "%s->val is NULL", name);
}

void check_tau(double t, const char* name) {
  if (!(t >= 0.0) || std::isinf(t)) fail(GB_EINVAL, "%s = %g must be finite and >= 0", name, t);
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Bounds given by the caller (both 0: Gershgorin): checked before any device work.
void check_given_bounds(double emin, double emax) {
  const bool given = !(emin == 0.0 && emax == 0.0);
  if (given && !(emax > emin && std::isfinite(emin) && std::isfinite(emax)))
    fail(GB_EINVAL, "need finite emax > emin (given %g, %g)", emin, emax);
}

struct EvPair {
  hipEvent_t a = nullptr, b = nullptr;
  EvPair() {
    GB_HIP(hipEventCreate(&a));
    GB_HIP(hipEventCreate(&b));
  }
  ~EvPair() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  EvPair(const EvPair&) = delete;
  EvPair& operator=(const EvPair&) = delete;
  float ms() const {
    float t = 0.f;
    GB_HIP(hipEventElapsedTime(&t, a, b));
    return t;
  }
};

// The front end shared by the expansions: spectral bounds (given or Gershgorin), the X0 values
// on H's pattern, and (unless a partition is given) the X2 graph at `threshold` cut into block
// cores of core_size.
struct Front {
  double emin = 0, emax = 0;
  DBuf<double> x0;
  double* x0_ext = nullptr;  // X0 in a caller-owned workspace (then x0 stays empty)
  const double* x0p() const { return x0_ext ? x0_ext : x0.get(); }
  EvPair ev_bounds;  // around the bounds and X0 (read after the call's final wait)
  gb_partition_s own;
  const Part* P = nullptr;
  float ms_bounds = 0, ms_graph = 0, ms_part = 0;
};

void prepare_front(const gb_ell& H, double threshold, double emin_in, double emax_in,
                   const gb_partition_t* part, int core_size, hipStream_t s, Front& f) {
  const bool given_bounds = !(emin_in == 0.0 && emax_in == 0.0);
  if (given_bounds && !(emax_in > emin_in && std::isfinite(emin_in) && std::isfinite(emax_in)))
    fail(GB_EINVAL, "need finite emax > emin");
  if (part && part->part.n != H.n)
    fail(GB_ESHAPE, "partition is for n = %d, H has n = %d", part->part.n, H.n);
  EvPair ev;
  GB_HIP(hipEventRecord(f.ev_bounds.a, s));
  // the Gershgorin pass also rejects an H holding NaN or Inf (given bounds included)
  double lo = 0, hi = 0;
  bounds(H, s, &lo, &hi);
  f.emin = given_bounds ? emin_in : lo;
  f.emax = given_bounds ? emax_in : hi;
  if (!(f.emax > f.emin))
    fail(GB_EINVAL, "H has an empty spectral range (e_min = e_max = %g)", f.emin);
  if (!f.x0_ext) f.x0 = DBuf<double>((size_t)H.n * H.width, s);
  x0_ell(H, f.emin, f.emax, const_cast<double*>(f.x0p()), s);
  GB_HIP(hipEventRecord(f.ev_bounds.b, s));
  f.P = part ? &part->part : nullptr;
  if (!f.P) {
    GB_HIP(hipEventRecord(ev.a, s));
    Csr g;
    graph_x2(H, f.x0p(), threshold, g, s);
    GB_HIP(hipEventRecord(ev.b, s));
    GB_HIP(hipStreamSynchronize(s));
    f.ms_graph = ev.ms();
    GB_HIP(hipEventRecord(ev.a, s));
    partition_block(g, core_size, f.own.part, s, GB_PART_BLOCK);
    GB_HIP(hipEventRecord(ev.b, s));
    GB_HIP(hipStreamSynchronize(s));
    f.ms_part = ev.ms();
    f.P = &f.own.part;
  }
}

}  // namespace

extern "C" {

const char* gb_version(void) { return "libgb 0.1.0 (gfx950)"; }

const char* gb_last_error(void) { return g_err; }

gb_status gb_trim(void) {
  return guarded([&] {
    ws_trim();
    ml_trim();
  });
}

gb_status gb_set_allocator(gb_alloc_fn alloc, gb_free_fn free_fn, void* ctx) {
  return guarded([&] {
    if ((alloc == nullptr) != (free_fn == nullptr))
      fail(GB_EINVAL, "alloc and free must both be set or both be NULL");
    g_alloc.alloc = alloc;
    g_alloc.free = free_fn;
    g_alloc.ctx = alloc ? ctx : nullptr;
  });
}

gb_status gb_peak_rate(int32_t kind, void* stream, double* rate, double* clock_mhz) {
  return guarded([&] {
    if (!rate) fail(GB_EINVAL, "rate is NULL");
    if (kind < 0 || kind > 6) fail(GB_EINVAL, "unknown kind %d", kind);
    *rate = peak_rate(kind, as_stream(stream), clock_mhz);
  });
}

gb_status gb_tune_save(const char* path, int32_t* n_entries) {
  return guarded([&] {
    if (!path || !*path) fail(GB_EINVAL, "path is NULL or empty");
    const int n = tune_save(path);
    if (n < 0) fail(GB_EINVAL, "cannot write the tuning table to %s", path);
    if (n_entries) *n_entries = n;
  });
}

gb_status gb_tune_load(const char* path, int32_t* n_entries) {
  return guarded([&] {
    if (!path || !*path) fail(GB_EINVAL, "path is NULL or empty");
    std::string why;
    const int n = tune_load(path, &why);
    if (n < 0) fail(GB_EINVAL, "tuning table %s not used: %s", path, why.c_str());
    if (n_entries) *n_entries = n;
  });
}

gb_status gb_spectral_bounds(const gb_ell* H, void* stream, double* emin, double* emax) {
  return guarded([&] {
    check_ell(H, "H");
    if (!emin || !emax) fail(GB_EINVAL, "emin / emax output pointer is NULL");
    bounds(*H, as_stream(stream), emin, emax);
  });
}

gb_status gb_spectral_bounds_noalloc(const gb_ell* H, void* stream, double* emin, double* emax) {
  return guarded([&] {
    check_ell(H, "H");
    if (!emin || !emax) fail(GB_EINVAL, "emin / emax output pointer is NULL");
    bounds_noalloc(*H, as_stream(stream), emin, emax);
  });
}

gb_status gb_build_graph(const gb_ell* H, const gb_ell* aux, double tau, double tau_aux,
                         int32_t mode, void* stream, gb_graph_t** out) {
  return guarded([&] {
    if (!out) fail(GB_EINVAL, "out is NULL");
    *out = nullptr;
    check_ell(H, "H");
    check_tau(tau, "tau");
    if (mode < GB_GRAPH_X2 || mode > GB_GRAPH_DPREV_SYMBOLIC)
      fail(GB_EINVAL, "unknown graph mode %d", mode);
    if (mode == GB_GRAPH_DPREV || mode == GB_GRAPH_DPREV_SYMBOLIC) {
      check_ell(aux, "aux (previous D)");
      check_tau(tau_aux, "tau_aux");
      if (aux->n != H->n) fail(GB_ESHAPE, "aux->n = %d differs from H->n = %d", aux->n, H->n);
    }
    if (mode == GB_GRAPH_PATTERN && aux) {
      check_ell(aux, "aux");
      if (aux->n != H->n) fail(GB_ESHAPE, "aux->n = %d differs from H->n = %d", aux->n, H->n);
    }
    hipStream_t s = as_stream(stream);
    auto* g = new gb_graph_s();
    try {
      if (mode == GB_GRAPH_PATTERN) {
        graph_pattern(aux ? *aux : *H, tau, g->csr, s);
      } else if (mode == GB_GRAPH_DPREV_SYMBOLIC) {
        graph_dprev_symbolic(*H, *aux, tau_aux, g->csr, s);
      } else {
        double emin, emax;
        bounds(*H, s, &emin, &emax);
        DBuf<double> x0((size_t)H->n * H->width, s);
        x0_ell(*H, emin, emax, x0.get(), s);
        if (mode == GB_GRAPH_X2) {
          graph_x2(*H, x0.get(), tau, g->csr, s);
        } else {
          Csr base;
          graph_x2(*H, x0.get(), tau, base, s);
          graph_union_dprev(base, *aux, tau_aux, g->csr, s);
        }
      }
      GB_HIP(hipStreamSynchronize(s));
      detach(g->csr);
    } catch (...) {
      delete g;
      throw;
    }
    *out = g;
  });
}

gb_status gb_build_graph_rcut(const double* pos, int32_t n_sites, int32_t orbs_per_site,
                              double box, double r_cut, void* stream, gb_graph_t** out) {
  return guarded([&] {
    if (!out) fail(GB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!pos) fail(GB_EINVAL, "pos is NULL");
    if (n_sites < 1 || orbs_per_site < 1) fail(GB_EINVAL, "need n_sites, orbs_per_site >= 1");
    if (!(r_cut > 0.0) || std::isinf(r_cut)) fail(GB_EINVAL, "r_cut = %g must be finite and > 0", r_cut);
    if (!(box >= 2.0 * r_cut) || std::isinf(box))
      fail(GB_EINVAL, "box = %g must be finite and at least 2 r_cut", box);
    if ((int64_t)n_sites * orbs_per_site > INT32_MAX) fail(GB_EINVAL, "too many orbitals");
    hipStream_t s = as_stream(stream);
    auto* g = new gb_graph_s();
    try {
      graph_rcut(pos, n_sites, orbs_per_site, box, r_cut, g->csr, s);
      GB_HIP(hipStreamSynchronize(s));
      detach(g->csr);
    } catch (...) {
      delete g;
      throw;
    }
    *out = g;
  });
}

gb_status gb_graph_info(const gb_graph_t* g, int32_t* n, int64_t* nnz) {
  return guarded([&] {
    if (!g) fail(GB_EINVAL, "graph is NULL");
    if (n) *n = g->csr.n;
    if (nnz) *nnz = g->csr.nnz;
  });
}

gb_status gb_graph_copy(const gb_graph_t* g, int32_t* row_ptr, int32_t* col, void* stream) {
  return guarded([&] {
    if (!g) fail(GB_EINVAL, "graph is NULL");
    hipStream_t s = as_stream(stream);
    if (row_ptr)
      GB_HIP(hipMemcpyAsync(row_ptr, g->csr.row_ptr.get(), (g->csr.n + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToDevice, s));
    if (col && g->csr.nnz)
      GB_HIP(hipMemcpyAsync(col, g->csr.col.get(), g->csr.nnz * sizeof(int32_t),
                            hipMemcpyDeviceToDevice, s));
  });
}

gb_status gb_graph_view(const gb_graph_t* g, int32_t* n, int64_t* nnz, const int32_t** row_ptr,
                        const int32_t** col) {
  return guarded([&] {
    if (!g) fail(GB_EINVAL, "graph is NULL");
    if (n) *n = g->csr.n;
    if (nnz) *nnz = g->csr.nnz;
    if (row_ptr) *row_ptr = g->csr.row_ptr.get();
    if (col) *col = g->csr.col.get();
  });
}

void gb_graph_destroy(gb_graph_t* g) { delete g; }

gb_status gb_partition(const gb_graph_t* g, int32_t core_size, int32_t method, void* stream,
                       gb_partition_t** out) {
  return guarded([&] {
    if (!out) fail(GB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) fail(GB_EINVAL, "graph is NULL");
    if (core_size < 1) fail(GB_EINVAL, "core_size = %d must be >= 1", core_size);
    if (method != GB_PART_BLOCK && method != GB_PART_BFS && method != GB_PART_MULTILEVEL)
      fail(GB_EINVAL, "unknown partition method %d", method);
    hipStream_t s = as_stream(stream);
    auto* p = new gb_partition_s();
    try {
      if (method == GB_PART_MULTILEVEL)
        partition_multilevel_dev(g->csr, core_size, p->part, s, nullptr);
      else
        partition_block(g->csr, core_size, p->part, s, method);
      GB_HIP(hipStreamSynchronize(s));
      detach(p->part);
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  });
}

namespace {

void check_host_csr(int32_t n, const int32_t* row_ptr, const int32_t* col) {
  if (n < 1) fail(GB_EINVAL, "n = %d must be >= 1", n);
  if (row_ptr[0] != 0) fail(GB_EINVAL, "row_ptr[0] must be 0");
  for (int v = 0; v < n; ++v) {
    if (row_ptr[v + 1] < row_ptr[v]) fail(GB_EINVAL, "row_ptr decreases at %d", v);
    for (int e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
      if (col[e] < 0 || col[e] >= n) fail(GB_EINVAL, "col[%d] = %d out of range", e, col[e]);
  }
}

void check_cover(int32_t n, int32_t n_cores, const int32_t* ptr, const int32_t* vtx) {
  if (n_cores < 1) fail(GB_EINVAL, "prev_n_cores = %d must be >= 1", n_cores);
  if (ptr[0] != 0 || ptr[n_cores] != n) fail(GB_EINVAL, "prev_core_ptr must run from 0 to n");
  std::vector<char> seen(n, 0);
  for (int c = 0; c < n_cores; ++c) {
    if (ptr[c + 1] <= ptr[c]) fail(GB_EINVAL, "previous core %d is empty or ptr decreases", c);
    for (int i = ptr[c]; i < ptr[c + 1]; ++i) {
      const int v = vtx[i];
      if (v < 0 || v >= n || seen[v]) fail(GB_EINVAL, "prev_core_vtx[%d] = %d repeats or is out of range", i, v);
      seen[v] = 1;
    }
  }
}

}  // namespace

gb_status gb_partition_host(int32_t n, const int32_t* row_ptr, const int32_t* col,
                            int32_t core_size, int32_t* n_cores, int32_t* core_ptr,
                            int32_t* core_vtx, int64_t* cost) {
  return guarded([&] {
    if (!row_ptr || !col || !n_cores || !core_ptr || !core_vtx)
      fail(GB_EINVAL, "row_ptr / col / n_cores / core_ptr / core_vtx is NULL");
    if (core_size < 1) fail(GB_EINVAL, "core_size = %d must be >= 1", core_size);
    check_host_csr(n, row_ptr, col);
    std::vector<int32_t> cp, cv;
    MlStats st;
    partition_multilevel(n, row_ptr, col, core_size, cp, cv, &st);
    *n_cores = (int32_t)cp.size() - 1;
    std::memcpy(core_ptr, cp.data(), cp.size() * 4);
    std::memcpy(core_vtx, cv.data(), cv.size() * 4);
    if (cost) *cost = st.cost;
  });
}

gb_status gb_partition_update(const gb_graph_t* g, const gb_partition_t* prev, void* stream,
                              gb_partition_t** out) {
  return guarded([&] {
    if (!out) fail(GB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g || !prev) fail(GB_EINVAL, "graph / prev is NULL");
    hipStream_t s = as_stream(stream);
    auto* p = new gb_partition_s();
    try {
      partition_multilevel_dev(g->csr, 0, p->part, s, nullptr, &prev->part);
      GB_HIP(hipStreamSynchronize(s));
      detach(p->part);
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  });
}

gb_status gb_partition_update_host(int32_t n, const int32_t* row_ptr, const int32_t* col,
                                   int32_t prev_n_cores, const int32_t* prev_core_ptr,
                                   const int32_t* prev_core_vtx, int32_t* n_cores,
                                   int32_t* core_ptr, int32_t* core_vtx, int64_t* cost) {
  return guarded([&] {
    if (!row_ptr || !col || !prev_core_ptr || !prev_core_vtx || !n_cores || !core_ptr ||
        !core_vtx)
      fail(GB_EINVAL, "an array argument is NULL");
    check_host_csr(n, row_ptr, col);
    check_cover(n, prev_n_cores, prev_core_ptr, prev_core_vtx);
    std::vector<int32_t> pp(prev_core_ptr, prev_core_ptr + prev_n_cores + 1),
        pv(prev_core_vtx, prev_core_vtx + n), cp, cv;
    MlStats st;
    partition_update(n, row_ptr, col, pp, pv, cp, cv, &st);
    *n_cores = (int32_t)cp.size() - 1;
    std::memcpy(core_ptr, cp.data(), cp.size() * 4);
    std::memcpy(core_vtx, cv.data(), cv.size() * 4);
    if (cost) *cost = st.cost;
  });
}

gb_status gb_partition_info(const gb_partition_t* p, int32_t* n_sub, int32_t* max_sub,
                            int64_t* total) {
  return guarded([&] {
    if (!p) fail(GB_EINVAL, "partition is NULL");
    if (n_sub) *n_sub = p->part.n_sub;
    if (max_sub) *max_sub = p->part.max_sub;
    if (total) *total = p->part.total;
  });
}

gb_status gb_partition_copy(const gb_partition_t* p, int32_t* core_ptr, int32_t* sub_ptr,
                            int32_t* sub_idx, void* stream) {
  return guarded([&] {
    if (!p) fail(GB_EINVAL, "partition is NULL");
    hipStream_t s = as_stream(stream);
    const Part& P = p->part;
    if (core_ptr)
      GB_HIP(hipMemcpyAsync(core_ptr, P.core_ptr.get(), (P.n_sub + 1) * 4, hipMemcpyDeviceToDevice, s));
    if (sub_ptr)
      GB_HIP(hipMemcpyAsync(sub_ptr, P.sub_ptr.get(), (P.n_sub + 1) * 4, hipMemcpyDeviceToDevice, s));
    if (sub_idx && P.total)
      GB_HIP(hipMemcpyAsync(sub_idx, P.sub_idx.get(), P.total * 4, hipMemcpyDeviceToDevice, s));
  });
}

gb_status gb_partition_view(const gb_partition_t* p, int32_t* n_sub, int32_t* max_sub,
                            const int32_t** core_ptr, const int32_t** sub_ptr,
                            const int32_t** sub_idx) {
  return guarded([&] {
    if (!p) fail(GB_EINVAL, "partition is NULL");
    const Part& P = p->part;
    if (n_sub) *n_sub = P.n_sub;
    if (max_sub) *max_sub = P.max_sub;
    if (core_ptr) *core_ptr = P.core_ptr.get();
    if (sub_ptr) *sub_ptr = P.sub_ptr.get();
    if (sub_idx) *sub_idx = P.sub_idx.get();
  });
}

void gb_partition_destroy(gb_partition_t* p) { delete p; }

gb_status gb_density(const gb_ell* H, int32_t n_occ, double threshold, const gb_sp2_opts* opts,
                     gb_ell* D, gb_sp2_stats* stats, void* stream) {
  gb_sp2_stats local{};
  gb_sp2_stats& st = stats ? *stats : local;
  return guarded([&] {
    std::memset(&st, 0, sizeof(st));
    st.min_margin = INFINITY;
    check_ell(H, "H");
    check_ell(D, "D");
    if (D->n != H->n) fail(GB_ESHAPE, "D->n = %d differs from H->n = %d", D->n, H->n);
    if (n_occ < 0 || n_occ > H->n) fail(GB_EINVAL, "n_occ = %d outside [0, %d]", n_occ, H->n);
    check_tau(threshold, "threshold");
    gb_sp2_opts o{};
    if (opts) o = *opts;
    if (o.precision < GB_FP64 || o.precision > GB_FP16X3_REFINE)
      fail(GB_EINVAL, "unknown precision %d", o.precision);
    if (o.max_iter < 0 || o.n_refine < 0) fail(GB_EINVAL, "max_iter / n_refine must be >= 0");
    if (o.refine_kind < 0 || o.refine_kind > 2) fail(GB_EINVAL, "unknown refine_kind %d", o.refine_kind);
    if (!(o.idem_tol >= 0.0)) fail(GB_EINVAL, "idem_tol must be >= 0");
    if (o.branch_in && (o.n_branch_in < 0 || o.n_branch_in > 127))
      fail(GB_EINVAL, "n_branch_in = %d outside [0, 127]", o.n_branch_in);
    if (o.branch_in)
      for (int i = 0; i < o.n_branch_in; ++i)
        if (o.branch_in[i] > 1) fail(GB_EINVAL, "branch_in[%d] = %d is not 0 or 1", i, o.branch_in[i]);
    if ((o.max_iter > 0 ? o.max_iter : 100) > 127) fail(GB_EINVAL, "max_iter must be <= 127");
    if (o.keep_tape && o.precision != GB_FP64)
      fail(GB_EUNSUPPORTED, "keep_tape needs precision GB_FP64");
    if (o.tape_stride < 0) fail(GB_EINVAL, "tape_stride must be >= 0");
    if (o.launch_mode < 0 || o.launch_mode > 3) fail(GB_EINVAL, "unknown launch_mode %d", o.launch_mode);
    if (o.check_idem < 0 || o.check_idem > 1) fail(GB_EINVAL, "check_idem must be 0 or 1");
    if (o.workspace && !o.partition)
      fail(GB_EINVAL, "a caller-owned workspace needs a partition (its size depends on it)");
    if (o.tile_policy < 0 || o.tile_policy > 7) fail(GB_EINVAL, "unknown tile_policy %d", o.tile_policy);
    if (o.tile_order < 0 || o.tile_order > 1) fail(GB_EINVAL, "unknown tile_order %d", o.tile_order);
    check_given_bounds(o.emin, o.emax);
    const int core_size = o.core_size > 0 ? o.core_size : 32;
    hipStream_t s = as_stream(stream);
    Front f;
    Workspace ext;
    if (o.workspace) {
      if (o.partition->part.n != H->n)
        fail(GB_ESHAPE, "partition is for n = %d, H has n = %d", o.partition->part.n, H->n);
      size_t slot[Workspace::kSlots];
      density_slots(o.partition->part, H->n, H->width, o, slot);
      workspace_layout(ext, o.workspace, o.workspace_bytes, slot);
      f.x0_ext = static_cast<double*>(ext.get_bytes(8, slot[8], s));
    }
    prepare_front(*H, threshold, o.emin, o.emax, o.partition, core_size, s, f);
    const double emin = f.emin, emax = f.emax;
    st.emin = emin;
    st.emax = emax;
    st.ms_graph = f.ms_graph;
    st.ms_part = f.ms_part;
    const Part* P = f.P;
    st.n_sub = P->n_sub;
    st.max_sub = P->max_sub;
    if (D->width < P->max_sub)
      fail(GB_ESHAPE, "D->width = %d is smaller than the largest subgraph (%d)", D->width,
           P->max_sub);
    TapeData* tape = nullptr;
    try {
      density(*H, n_occ, o, *P, emin, emax, f.x0p(), *D, st, s, o.keep_tape ? &tape : nullptr,
              o.workspace ? &ext : nullptr);
    } catch (...) {
      tape_destroy(tape);
      throw;
    }
    if (tape) {
      st.tape = new gb_tape_s{tape};
    }
    st.ms_bounds = f.ev_bounds.ms();  // the call has waited for its stream
    st.ms_total += st.ms_bounds + f.ms_graph + f.ms_part;
  });
}

gb_status gb_density_workspace(const gb_ell* H, const gb_sp2_opts* opts, size_t* bytes) {
  return guarded([&] {
    if (!bytes) fail(GB_EINVAL, "bytes is NULL");
    *bytes = 0;
    if (!H) fail(GB_EINVAL, "H is NULL");
    if (H->n <= 0 || H->width <= 0) fail(GB_EINVAL, "H->n and H->width must be positive");
    if (!opts || !opts->partition)
      fail(GB_EINVAL, "the workspace size depends on the partition: opts->partition is NULL");
    if (opts->precision < GB_FP64 || opts->precision > GB_FP16X3_REFINE)
      fail(GB_EINVAL, "unknown precision %d", opts->precision);
    if (opts->partition->part.n != H->n)
      fail(GB_ESHAPE, "partition is for n = %d, H has n = %d", opts->partition->part.n, H->n);
    size_t slot[Workspace::kSlots];
    density_slots(opts->partition->part, H->n, H->width, *opts, slot);
    *bytes = workspace_total(slot);
  });
}

gb_status gb_density_vjp(const gb_tape_t* tape, const gb_ell* G_D, gb_ell* G_H, void* stream) {
  return guarded([&] {
    if (!tape || !tape->data) fail(GB_EINVAL, "tape is NULL");
    int tn = 0, tmax = 0;
    tape_dims(tape->data, &tn, &tmax);
    if (!G_D || !G_D->val) fail(GB_EINVAL, "G_D or G_D->val is NULL");
    if (G_D->n != tn) fail(GB_ESHAPE, "G_D->n = %d, the tape has n = %d", G_D->n, tn);
    if (G_D->width < tmax)
      fail(GB_ESHAPE, "G_D->width = %d is smaller than the largest subgraph (%d)", G_D->width,
           tmax);
    check_ell(G_H, "G_H");
    if (G_H->n != tn) fail(GB_ESHAPE, "G_H->n = %d, the tape has n = %d", G_H->n, tn);
    density_vjp(*tape->data, *G_D, *G_H, G_H->val, as_stream(stream));
  });
}

void gb_tape_destroy(gb_tape_t* tape) {
  if (!tape) return;
  tape_destroy(tape->data);
  delete tape;
}

gb_status gb_chebyshev_fermi(double emin, double emax, double beta, double mu, int32_t order,
                             int32_t n_nodes, double* coef) {
  return guarded([&] {
    if (!coef) fail(GB_EINVAL, "coef is NULL");
    if (!(emax > emin) || std::isinf(emax) || std::isinf(emin)) fail(GB_EINVAL, "need finite emax > emin");
    if (!(beta > 0.0) || std::isinf(beta)) fail(GB_EINVAL, "beta = %g must be finite and > 0", beta);
    if (std::isnan(mu)) fail(GB_EINVAL, "mu is NaN");
    if (order < 1) fail(GB_EINVAL, "order = %d must be >= 1", order);
    if (n_nodes < 0) fail(GB_EINVAL, "n_nodes must be >= 0");
    chebyshev_fermi(emin, emax, beta, mu, order, n_nodes, coef);
  });
}

gb_status gb_sp2_sequence(double emin, double emax, double e_homo, double e_lumo, double delta,
                          int32_t max_len, uint8_t* out, int32_t* len) {
  return guarded([&] {
    if (!out || !len) fail(GB_EINVAL, "out / len is NULL");
    if (!(emin < e_homo && e_homo < e_lumo && e_lumo < emax))
      fail(GB_EINVAL, "need e_min < e_homo < e_lumo < e_max");
    if (!(delta > 0.0)) fail(GB_EINVAL, "delta must be > 0");
    if (max_len < 0) fail(GB_EINVAL, "max_len must be >= 0");
    double u = 1.0 - (emax - e_homo) / (emax - emin);
    double v = (emax - e_lumo) / (emax - emin);
    int n = 0;
    while (u > delta || v > delta) {
      if (n == max_len) fail(GB_ESHAPE, "%d steps do not reach delta = %g", max_len, delta);
      if (v > u) {
        out[n++] = 0;
        u = 2.0 * u - u * u;
        v = v * v;
      } else {
        out[n++] = 1;
        u = u * u;
        v = 2.0 * v - v * v;
      }
    }
    *len = n;
  });
}

namespace {

// Distance of an eigenvalue image from its target (side 0: the unoccupied side, distance from 0;
// side 1: the occupied side, distance from 1) taken through branches b[0..n).  Branch `side`
// squares the distance; the other takes d to 2d - d^2.
double gap_forward(double d, const uint8_t* b, int n, int side) {
  for (int k = 0; k < n; ++k) d = (int)b[k] == side ? d * d : 2.0 * d - d * d;
  return d;
}

// The inverse: a distance at step k mapped back through b[k-1], ..., b[0] to step 0.
double gap_back(double d, const uint8_t* b, int k, int side) {
  for (int q = k - 1; q >= 0; --q)
    d = (int)b[q] == side ? std::sqrt(d) : d / (1.0 + std::sqrt(1.0 - d));
  return d;
}

double gap_g(double x) { return x - 0.5 * x * x; }

// x in (0, 1) with g(F(x)) = rho g(x), F the branch maps b[0..n) (bisection to the last
// representable midpoint; g(F(x))/g(x) rises through (0, 1) on an initial interval of x and
// stays >= 1 beyond it).
double gap_solve_ratio(double rho, const uint8_t* b, int n, int side) {
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (gap_g(gap_forward(mid, b, n, side)) - rho * gap_g(mid) < 0.0) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

gb_status gb_sp2_estimate_gap(const double* t1, const double* t2, const uint8_t* branch,
                              int32_t n_branch, double n_occ, double emin, double emax,
                              double floor, gb_gap_estimate* out) {
  return guarded([&] {
    if (!t1 || !t2 || !branch || !out) fail(GB_EINVAL, "t1 / t2 / branch / out is NULL");
    if (n_branch < 1) fail(GB_EINVAL, "n_branch = %d must be >= 1", n_branch);
    if (!(emax > emin)) fail(GB_EINVAL, "need emax > emin");
    for (int i = 0; i < n_branch; ++i)
      if (branch[i] > 1) fail(GB_EINVAL, "branch[%d] = %d is not 0 or 1", i, (int)branch[i]);
    const int nb = n_branch;
    if (!(floor > 0.0))
      floor = std::max(10.0 * (std::fabs(t1[nb] - n_occ) + std::fabs(t1[nb] - t2[nb])),
                       1e-12 * n_occ);
    // per-iterate sums of the distances: side 0 (unoccupied) L = (A + B)/2, side 1 (occupied)
    // U = (A - B)/2, A = t1 - t2, B = t1 - n_occ
    std::vector<double> S[2];
    for (int i = 0; i <= nb; ++i) {
      const double A = t1[i] - t2[i], B = t1[i] - n_occ;
      S[0].push_back(0.5 * (A + B));
      S[1].push_back(0.5 * (A - B));
    }
    const double w = emax - emin;
    gb_gap_estimate r;
    std::memset(&r, 0, sizeof(r));
    r.floor = floor;
    for (int side = 0; side < 2; ++side) {
      const std::vector<double>& own = S[side];
      const std::vector<double>& oth = S[1 - side];
      // clean iterates of this side: right after a branch that does not square it
      std::vector<int> clean;
      for (int i = 1; i <= nb; ++i)
        if ((int)branch[i - 1] != side) clean.push_back(i);
      int ib = -1;
      for (int i : clean) {
        const double val = own[i] + 0.5 * oth[i] * oth[i];
        if (own[i] > floor && val < 0.5) ib = i;
      }
      if (ib < 0)
        fail(GB_EINVAL, "no clean iterate of the %s side above the noise floor %g",
             side ? "occupied" : "unoccupied", floor);
      const double val = own[ib] + 0.5 * oth[ib] * oth[ib];
      const double d_bound = gap_back(2.0 * val / (1.0 + std::sqrt(1.0 - 2.0 * val)), branch, ib,
                                      side);
      int pi = -1, pj = -1;
      for (size_t a = 0; a < clean.size(); ++a) {
        const int i = clean[a];
        for (size_t c = a + 1; c < clean.size(); ++c) {
          const int j = clean[c];
          bool squares = false;
          for (int q = i; q < j; ++q) squares |= (int)branch[q] == side;
          if (!squares) continue;
          if (own[j] > floor && own[i] > own[j]) {
            pi = i;
            pj = j;
          }
          break;
        }
      }
      if (pi < 0)
        fail(GB_EINVAL, "no pair of clean iterates of the %s side above the noise floor %g",
             side ? "occupied" : "unoccupied", floor);
      const double d_ratio =
          gap_back(gap_solve_ratio(own[pj] / own[pi], branch + pi, pj - pi, side), branch, pi, side);
      int32_t* it = side ? r.homo_iter : r.lumo_iter;
      it[0] = ib;
      it[1] = pi;
      it[2] = pj;
      if (side == 0) {
        r.lumo_bound = emax - d_bound * w;
        r.lumo_ratio = emax - d_ratio * w;
      } else {
        r.homo_bound = emax - (1.0 - d_bound) * w;
        r.homo_ratio = emax - (1.0 - d_ratio) * w;
      }
    }
    *out = r;
  });
}

gb_status gb_foe_solve_mu(const double* traces, int32_t order, double emin, double emax,
                          double beta, double n_occ, int32_t n_nodes, double* mu) {
  return guarded([&] {
    if (!traces || !mu) fail(GB_EINVAL, "traces / mu is NULL");
    if (!(emax > emin)) fail(GB_EINVAL, "need emax > emin");
    if (!(beta > 0.0) || std::isinf(beta)) fail(GB_EINVAL, "beta = %g must be finite and > 0", beta);
    if (order < 1) fail(GB_EINVAL, "order = %d must be >= 1", order);
    if (n_nodes < 0) fail(GB_EINVAL, "n_nodes must be >= 0");
    *mu = foe_solve_mu(traces, order, emin, emax, beta, n_occ, n_nodes);
  });
}

gb_status gb_foe_density(const gb_ell* H, int32_t n_occ, double threshold, const gb_foe_opts* opts,
                         gb_ell* D, gb_foe_stats* stats, void* stream) {
  gb_foe_stats local{};
  gb_foe_stats& st = stats ? *stats : local;
  return guarded([&] {
    std::memset(&st, 0, sizeof(st));
    if (!opts) fail(GB_EINVAL, "opts is NULL (beta and order are required)");
    const gb_foe_opts o = *opts;
    check_ell(H, "H");
    check_ell(D, "D");
    if (D->n != H->n) fail(GB_ESHAPE, "D->n = %d differs from H->n = %d", D->n, H->n);
    check_tau(threshold, "threshold");
    if (!(o.beta > 0.0) || std::isinf(o.beta)) fail(GB_EINVAL, "beta = %g must be finite and > 0", o.beta);
    if (o.order < 1) fail(GB_EINVAL, "order = %d must be >= 1", o.order);
    if (o.n_nodes < 0) fail(GB_EINVAL, "n_nodes must be >= 0");
    if (std::isnan(o.mu) && (n_occ < 0 || n_occ > H->n))
      fail(GB_EINVAL, "n_occ = %d outside [0, %d]", n_occ, H->n);
    if (std::isinf(o.mu)) fail(GB_EINVAL, "mu must be finite (or NaN to solve for it)");
    if (o.tile_policy < 0 || o.tile_policy > 5 || o.tile_policy == 3)
      fail(GB_EINVAL, "unknown tile_policy %d", o.tile_policy);
    if (o.tile_order < 0 || o.tile_order > 1) fail(GB_EINVAL, "unknown tile_order %d", o.tile_order);
    check_given_bounds(o.emin, o.emax);
    const int core_size = o.core_size > 0 ? o.core_size : 32;
    hipStream_t s = as_stream(stream);
    Front f;
    prepare_front(*H, threshold, o.emin, o.emax, o.partition, core_size, s, f);
    st.emin = f.emin;
    st.emax = f.emax;
    st.ms_graph = f.ms_graph;
    st.ms_part = f.ms_part;
    st.n_sub = f.P->n_sub;
    st.max_sub = f.P->max_sub;
    if (D->width < f.P->max_sub)
      fail(GB_ESHAPE, "D->width = %d is smaller than the largest subgraph (%d)", D->width,
           f.P->max_sub);
    foe(*H, n_occ, o, *f.P, f.emin, f.emax, *D, st, s);
    st.ms_bounds = f.ev_bounds.ms();
    st.ms_total += st.ms_bounds + f.ms_graph + f.ms_part;
  });
}

}  // extern "C"
