// Internal declarations shared by the libgb translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/gb.h"

namespace gbi {

// ---- errors: C++ exceptions never cross the C ABI; api.hip converts them to codes ----
struct Error {
  gb_status code;
};
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
[[noreturn]] void fail(gb_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define GB_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      ::gbi::fail(GB_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                \
  } while (0)

#define GB_LAUNCH_CHECK() GB_HIP(hipGetLastError())

// ---- device memory: stream-ordered allocations from the device pool, or from the hook
// registered with gb_set_allocator (each buffer remembers the allocator that made it) ----
struct Allocator {
  gb_alloc_fn alloc = nullptr;  // nullptr: the device pool
  gb_free_fn free = nullptr;
  void* ctx = nullptr;
};
void* dmalloc(size_t bytes, hipStream_t s, Allocator* used);
void dfree(void* p, hipStream_t s, const Allocator& a);

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;
  Allocator a;
  DBuf() = default;
  DBuf(size_t count, hipStream_t st) : n(count), s(st) {
    if (count) p = static_cast<T*>(dmalloc(count * sizeof(T), st, &a));
  }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), s(o.s), a(o.a) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { reset(); p = o.p; n = o.n; s = o.s; a = o.a; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (p) dfree(p, s, a);
    p = nullptr;
    n = 0;
  }
  T* get() const { return p; }
  // handle-owned buffers are freed on the null stream (the creating stream may be gone)
  void detach_stream() { s = nullptr; }
};

// ---- cached batch buffers -------------------------------------------------------------------
// The dense batch buffers (tens of GB at N = 100000) are kept between calls instead of being
// returned to the pool: a call leases a workspace (one per concurrent call and device), takes
// its buffers from numbered slots that grow when a call needs more, and gives it back at the
// end.  Every call synchronises its stream before returning, so the next lease may use the
// memory on any stream.  gb_trim frees the idle workspaces.
struct Workspace {
  int device = 0;
  struct Slab {
    void* p = nullptr;
    size_t bytes = 0;
    Allocator a;
  };
  static constexpr int kSlots = 9;
  Slab slab[kSlots];
  // caller-owned memory (gb_sp2_opts.workspace): every slot at a fixed offset of one buffer,
  // sized by density_slots; a request beyond a slot's size is an error, never an allocation
  char* ext = nullptr;
  size_t ext_off[kSlots] = {}, ext_size[kSlots] = {};
  void* get_bytes(int slot, size_t bytes, hipStream_t s);
  template <typename T>
  T* get(int slot, size_t count, hipStream_t s) {
    return static_cast<T*>(get_bytes(slot, count * sizeof(T), s));
  }
  void release_all();
};
Workspace* ws_acquire();
void ws_release(Workspace* w);
void ws_trim();
struct WsLease {
  Workspace* w;
  bool own;
  // ext: a caller-owned workspace (not leased, not returned); nullptr leases a cached one
  explicit WsLease(Workspace* ext = nullptr) : w(ext ? ext : ws_acquire()), own(ext == nullptr) {}
  ~WsLease() {
    if (own) ws_release(w);
  }
  WsLease(const WsLease&) = delete;
  WsLease& operator=(const WsLease&) = delete;
  Workspace* operator->() const { return w; }
};

// ---- scans (scan.hip) ----
// out[0..n] = exclusive prefix sums of in[0..n-1]; out[n] = total.
void exclusive_scan_i32(const int32_t* in, int32_t* out, int n, hipStream_t s);
void exclusive_scan_i64(const int32_t* in, int64_t* out, int n, hipStream_t s);

// ---- sustained rates (peak.hip): TFLOP/s of MFMA kind 0 FP64, 1 FP32, 2 bf16, 3 fp16; GB/s of
// an HBM copy for kind 4 (read + written bytes); clock_mhz (may be NULL): the core clock during
// the MFMA loop (0 for kind 4) ----
double peak_rate(int kind, hipStream_t s, double* clock_mhz);

// ---- vertex sets in LDS (graph.hip) ----
// The graph and halo kernels keep vertex sets either as n-bit LDS bitmaps (fast while n is
// small; LDS grows with n) or as LDS hash sets sorted afterwards (work and LDS independent of
// n).  Hash sets are used above 2^17 vertices; the environment variable GB_VERTEX_SETS=bitmap
// or =hash forces one kind (both give the same sets, in the same order).
bool use_hash_sets(int n);

// ---- graph (graph.hip) ----
struct Csr {
  int32_t n = 0;
  int64_t nnz = 0;
  DBuf<int32_t> row_ptr, col;
};
void bounds(const gb_ell& H, hipStream_t s, double* emin, double* emax);  // synchronises
// the same without allocated device memory (a fixed device array holds the partials)
void bounds_noalloc(const gb_ell& H, hipStream_t s, double* emin, double* emax);
void x0_ell(const gb_ell& H, double emin, double emax, double* x0, hipStream_t s);
void graph_x2(const gb_ell& H, const double* x0, double tau, Csr& out, hipStream_t s);
void graph_pattern(const gb_ell& A, double tau, Csr& out, hipStream_t s);
void graph_union_dprev(const Csr& base, const gb_ell& Dp, double tau_d, Csr& out,
                       hipStream_t s);
void graph_dprev_symbolic(const gb_ell& H, const gb_ell& Dp, double tau_d, Csr& out,
                          hipStream_t s);
void graph_rcut(const double* pos, int n_sites, int m, double box, double r_cut, Csr& out,
                hipStream_t s);

// ---- partition (partition.hip) ----
struct Part {
  int32_t n = 0, n_sub = 0, max_sub = 0;
  int64_t total = 0;
  DBuf<int32_t> core_ptr, core_vtx, sub_ptr, sub_idx;
  DBuf<int32_t> sub_pos;            // rank of sub_idx[p] in its subgraph's ascending order
  DBuf<int32_t> col_sub, col_loc;   // vertex -> (subgraph, local index) of its core
  std::vector<int32_t> h_core_ptr, h_sub_ptr;  // host copies (sizes for planning)
};
void partition_block(const Csr& g, int32_t core_size, Part& out, hipStream_t s, int method);
void finish_partition(const Csr& g, Part& P, hipStream_t s);
void partition_from_cores(const Csr& g, const std::vector<int32_t>& core_ptr,
                          const std::vector<int32_t>& core_vtx, Part& P, hipStream_t s);
struct MlStats {
  int levels = 0, coarsest = 0;
  int64_t cost = 0;  // sum over subgraphs of (|core| + |halo|)^3
  double ms_weights = 0, ms_coarsen = 0, ms_grow = 0, ms_cost = 0;
};
// Host buffers of the multilevel partitioner, kept between calls (mlpart.hip): on graphs of
// millions of edges, touching fresh pages (a fault per 4 KiB) costs as much as the coarsening
// itself, so a call leases a set whose vectors keep their capacity, plus pinned staging for
// the device graph.  gb_trim releases the idle sets.
struct MlScratch;
struct MlLease {
  MlScratch* p;
  MlLease();
  ~MlLease();
  MlLease(const MlLease&) = delete;
  MlLease& operator=(const MlLease&) = delete;
};
void ml_trim();
// pinned host arrays of the lease for a graph of n vertices and nnz entries (grown on demand):
// row pointers, columns, edge weights
void ml_stage(MlScratch& sc, int n, int64_t nnz, int32_t** rp, int32_t** col, int32_t** w);
// host array of the lease for n vertices' candidate lists (n * kMlTop entries)
int32_t* ml_top_buffer(MlScratch& sc, int n);
// Multilevel cores of at most `cap` vertices (host; mlpart.hip); core_vtx ascending per core.
// ew (optional): per CSR entry, the number of common closed neighbours of its two ends
// (computed here when NULL).  sc: the caller's lease (one is taken here when NULL).  stats
// (optional) receives the level count, timings and the cost sum (|core| + |halo|)^3, which is
// only computed when stats is given.  top0 (optional, with ew): per vertex the kMlTop heaviest
// neighbours by (weight, -index), heaviest first, -1 padded (what the matching would compute).
constexpr int kMlTop = 8;
// Coarse levels built where the graph lives (the device path, partition.hip): given the
// matching of level `level` (n vertices, host row pointers frp) -- coarse vertex c is
// {lead[c], match[lead[c]]}, cmap the fine -> coarse map, cvw the coarse weights -- it builds
// the coarse rows (neighbours ascending, the summed weights of the edges between the two vertex
// sets, no self loops) from its own copy of the fine level (the input graph for level 0, else
// the level it built last) and the coarse level's candidate lists for pair cap `cap` (those
// the host would compute: the kMlTop heaviest by (weight, -vertex weight, -index) of every
// vertex with cvw + min cvw <= cap, else -1).  On success *rp, *adj, *ew (CSR of the nc coarse
// vertices) and *top (nc * kMlTop) point at host arrays valid until the next build or the end
// of the partition call; on false the host builds the level (and every later one).
struct MlCoarseDevice {
  virtual ~MlCoarseDevice() = default;
  virtual bool build(int level, int n, const int32_t* frp, int nc,
                     const std::vector<int32_t>& match, const std::vector<int32_t>& cmap,
                     const std::vector<int32_t>& lead, const std::vector<int32_t>& cvw, int cap,
                     const int32_t** rp, const int32_t** adj, const int32_t** ew,
                     const int32_t** top) = 0;
};
// pinned host arrays of the lease for a coarse level built on the device (nc vertices, nnz
// entries, the candidate lists), grown on demand
void ml_stage1(MlScratch& sc, int nc, int64_t nnz, int32_t** rp, int32_t** adj, int32_t** ew,
               int32_t** top);
void partition_multilevel(int n, const int32_t* row_ptr, const int32_t* col, int cap,
                          std::vector<int32_t>& core_ptr, std::vector<int32_t>& core_vtx,
                          MlStats* stats, const int32_t* ew = nullptr, MlScratch* sc = nullptr,
                          const int32_t* top0 = nullptr, MlCoarseDevice* dev1 = nullptr);
// The previous cores carried to a new graph on the same vertices (on-the-fly update between MD
// steps): the cores renumbered as the partitioner emits them, and (when stats is given) their
// cost on the new graph.
void partition_update(int n, const int32_t* row_ptr, const int32_t* col,
                      const std::vector<int32_t>& prev_ptr, const std::vector<int32_t>& prev_vtx,
                      std::vector<int32_t>& core_ptr, std::vector<int32_t>& core_vtx,
                      MlStats* stats);
void partition_multilevel_dev(const Csr& g, int32_t core_size, Part& P, hipStream_t s,
                              MlStats* stats, const Part* prev = nullptr);
void detach(Csr& c);
void detach(Part& p);

// Bytes of each workspace slot a gb_density call takes on partition P of an n x width H
// (sp2.hip); their 256-byte aligned sum is the caller-owned workspace size.
void density_slots(const Part& P, int n, int width, const gb_sp2_opts& o,
                   size_t bytes[Workspace::kSlots]);
// Lays the slots out in a caller buffer of `bytes` bytes (GB_ESHAPE if it is too small).
void workspace_layout(Workspace& w, void* base, size_t bytes, const size_t slot[Workspace::kSlots]);
size_t workspace_total(const size_t slot[Workspace::kSlots]);

// autotuning table (sp2.hip): write / read a JSON file; read returns the entry count or -1
int tune_save(const char* path);
int tune_load(const char* path, std::string* why);

struct TapeData;  // SP2 checkpoints for the adjoint (sp2.hip)
void tape_destroy(TapeData* t);
void tape_dims(const TapeData* t, int* n, int* max_sub);
void density_vjp(TapeData& t, const gb_ell& G_D, const gb_ell& H_pattern, double* G_H,
                 hipStream_t s);

// ---- finite-temperature expansion (sp2.hip) ----
void chebyshev_fermi(double emin, double emax, double beta, double mu, int order, int n_nodes,
                     double* c);
double foe_solve_mu(const double* traces, int order, double emin, double emax, double beta,
                    double n_occ, int n_nodes);
void foe(const gb_ell& H, int32_t n_occ, const gb_foe_opts& o, const Part& P, double emin,
         double emax, gb_ell& D, gb_foe_stats& st, hipStream_t s);

}  // namespace gbi

// graph / partition handles behind the opaque ABI types
struct gb_graph_s {
  gbi::Csr csr;
};
struct gb_partition_s {
  gbi::Part part;
};
struct gb_tape_s {
  gbi::TapeData* data;
};
