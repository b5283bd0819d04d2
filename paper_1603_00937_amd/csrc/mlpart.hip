// Multilevel core partitioner (host code).
//
// The cost of the method is the sum over subgraphs of n_s^3, n_s = |core| + |halo| (the dense
// products of every subgraph; the paper's cost discussion after Eq. 6), and the paper takes its
// communities from a multilevel graph partitioner.  This one is written for that objective with
// a hard cap on the core size (the batched kernels are sized for it):
//   1. edge weights = common closed neighbours of the two ends, so that strongly tied vertices
//      are the ones whose joint halo is smallest;
//   2. coarsening by heavy-edge matching, pairs limited to a quarter of the cap, until no pair
//      can be matched;
//   3. on the coarsest graph, parts grown one at a time by always adding the unassigned
//      neighbour most strongly tied to the part while it fits under the cap, seeds taken in
//      breadth-first order so that parts follow one another through the graph;
//   4. the parts projected back to the input graph.
// Greedy single-vertex refinement passes were tried on the input graph (edge-cut gain, and the
// exact change of sum (|core| + |halo|)^3): with every part at the cap no vertex has room to
// move, the cost passes moved nothing and the edge-cut passes raised the cost slightly, so they
// are not part of the pipeline.
// Everything is integer and every choice has a fixed tie-break, so the result is a function of
// the graph alone.  The visiting order of the matching is a fixed pseudo-random permutation
// (vertices sorted by SplitMix64 of (level << 32 | v)).

#include "internal.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <cstdint>
#include <vector>

namespace gbi {

namespace {

uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// host threads for the independent parts (at most 16)
int worker_count() {
  const unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(16u, h));
}

// Worker threads kept for the life of the process (starting and joining 16 threads costs a few
// hundred microseconds, and a partition runs a dozen parallel passes).  One job at a time: a
// call that finds the pool busy (another partition on another host thread) starts threads of
// its own instead.  The pool is never destroyed, so no thread is joined at exit.
class WorkerPool {
 public:
  bool try_run(int nt, const std::function<void(int)>& f) {
    std::unique_lock<std::mutex> busy(run_mu_, std::try_to_lock);
    if (!busy.owns_lock()) return false;
    while ((int)threads_.size() < nt - 1) {
      const int idx = (int)threads_.size() + 1;
      threads_.emplace_back([this, idx] { loop(idx); });
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &f;
      nt_ = nt;
      pending_ = nt - 1;
      ++gen_;
    }
    cv_.notify_all();
    std::exception_ptr err;
    try {
      f(0);
    } catch (...) {
      err = std::current_exception();  // the other threads still use the job: wait first
    }
    {
      std::unique_lock<std::mutex> lk(mu_);
      done_.wait(lk, [this] { return pending_ == 0; });
      job_ = nullptr;
    }
    if (err) std::rethrow_exception(err);
    return true;
  }

 private:
  void loop(int idx) {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void(int)>* f;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_ != seen; });
        seen = gen_;
        if (idx >= nt_) continue;  // not part of this job
        f = job_;
      }
      (*f)(idx);
      std::lock_guard<std::mutex> lk(mu_);
      if (--pending_ == 0) done_.notify_one();
    }
  }
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_;
  std::vector<std::thread> threads_;
  const std::function<void(int)>* job_ = nullptr;
  int nt_ = 0, pending_ = 0;
  uint64_t gen_ = 0;
};

WorkerPool& worker_pool() {
  static WorkerPool* pool = new WorkerPool;  // one for the process, never destroyed
  return *pool;
}

template <typename F>
void run_workers(int nt, F&& f) {
  if (nt <= 1) {
    f(0);
    return;
  }
  const std::function<void(int)> job = [&f](int t) { f(t); };
  if (worker_pool().try_run(nt, job)) return;
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back(f, t);
  for (auto& x : th) x.join();
}

// A graph level: CSR with edge and vertex weights.  The input level reads the caller's CSR in
// place (its self loops are skipped where they matter); coarse levels own their arrays.
struct Level {
  int n = 0;
  const int32_t* rp = nullptr;
  const int32_t* adj = nullptr;
  const int32_t* ew = nullptr;
  std::vector<int32_t> rp_v, adj_v, ew_v;  // storage of a coarse level (or of host weights)
  bool sorted = false;                     // rows ascending (a level built on the device)
  std::vector<int32_t> vw;                 // vertex weights
  std::vector<int32_t> cmap;               // vertex -> vertex of the next coarser level
};

}  // namespace

struct MlScratch {
  std::vector<Level> lv;  // lv[0]: the input level; coarse levels after it
  std::vector<std::pair<uint64_t, int32_t>> keys;
  std::vector<int32_t> top, match, lead, deg;
  const int32_t* top1 = nullptr;  // the lists of the level the device built last
  // visiting orders by level (a function of the level and the vertex count only, so they are
  // kept for the next call on a graph of the same size)
  std::vector<std::pair<int, std::vector<int32_t>>> orders;
  std::vector<std::vector<int32_t>> adj_t, ew_t, acc;
  int32_t *h_rp = nullptr, *h_col = nullptr, *h_w = nullptr;  // pinned staging
  size_t cap_rp = 0, cap_col = 0, cap_w = 0;
  // pinned arrays of the coarse level built on the device last
  int32_t *h_rp1 = nullptr, *h_adj1 = nullptr, *h_ew1 = nullptr, *h_top1 = nullptr;
  size_t cap_rp1 = 0, cap_adj1 = 0, cap_ew1 = 0, cap_top1 = 0;
};

namespace {

std::mutex g_ml_mu;
std::vector<MlScratch*> g_ml_free;  // idle sets (never destroyed at exit: no HIP calls then)

void pinned_reserve(int32_t*& p, size_t& cap, size_t count) {
  if (count <= cap) return;
  int32_t* old = p;
  p = nullptr;  // consistent (empty) if a call below fails
  cap = 0;
  if (old) GB_HIP(hipHostFree(old));
  const size_t want = count + count / 8;  // headroom for graphs that grow a little
  GB_HIP(hipHostMalloc((void**)&p, want * sizeof(int32_t), hipHostMallocDefault));
  cap = want;
}

const std::vector<int32_t>& visit_order(int n, int level, MlScratch& sc) {
  if ((int)sc.orders.size() <= level) sc.orders.resize(level + 1);
  auto& slot = sc.orders[level];
  if (slot.first == n && (int)slot.second.size() == n) return slot.second;
  auto& k = sc.keys;
  k.resize(n);
  for (int v = 0; v < n; ++v) k[v] = {splitmix64(((uint64_t)level << 32) | (uint32_t)v), v};
  std::sort(k.begin(), k.end());
  slot.first = n;
  slot.second.resize(n);
  for (int i = 0; i < n; ++i) slot.second[i] = k[i].second;
  return slot.second;
}

// The kTop heaviest candidates of every vertex by (edge weight, -vertex weight, -index),
// heaviest first (-1 pads short lists), found on host threads.  The matching below walks a
// vertex's list and takes the first candidate that is still unmatched and fits: that is the
// maximum over all its neighbours unless every listed candidate is taken, in which case it
// scans the whole row as before.
constexpr int kTop = kMlTop;
bool heavier(const Level& f, int e, int u, int e2, int u2) {
  if (f.ew[e] != f.ew[e2]) return f.ew[e] > f.ew[e2];
  if (f.vw[u] != f.vw[u2]) return f.vw[u] < f.vw[u2];
  return u < u2;
}
// Only vertices that can pair with some vertex (vw[v] + min vw <= cap) get a list: the matching
// never reads the others'.
void top_candidates(const Level& f, int cap, int min_vw, std::vector<int32_t>& top) {
  const int n = f.n;
  top.assign((size_t)n * kTop, -1);
  const int nt = f.rp[n] >= (1 << 16) ? worker_count() : 1;
  run_workers(nt, [&](int t) {
    const int v0 = (int)((int64_t)n * t / nt), v1 = (int)((int64_t)n * (t + 1) / nt);
    int te[kTop];
    for (int v = v0; v < v1; ++v) {
      if (f.vw[v] + min_vw > cap) continue;
      int m = 0;
      for (int e = f.rp[v]; e < f.rp[v + 1]; ++e) {
        const int u = f.adj[e];
        if (u == v) continue;
        if (m == kTop && !heavier(f, e, u, te[m - 1], f.adj[te[m - 1]])) continue;
        int i = m < kTop ? m++ : kTop - 1;
        for (; i > 0 && heavier(f, e, u, te[i - 1], f.adj[te[i - 1]]); --i) te[i] = te[i - 1];
        te[i] = e;
      }
      for (int i = 0; i < m; ++i) top[(size_t)v * kTop + i] = f.adj[te[i]];
    }
  });
}

// Heavy-edge matching of f (pairs of weight <= cap); returns false if no pair was matched.
// given_top: the candidate lists of f computed elsewhere (by the weights kernel for the input
// level, by dev1 for a coarse level it built), else NULL
// dev1: builds the coarse level (and its candidate lists, into sc.top1, for pair cap next_cap)
// on the device instead of the host
bool coarsen(Level& f, int cap, int level, Level& c, MlScratch& sc,
             const int32_t* given_top = nullptr, MlCoarseDevice* dev1 = nullptr,
             int next_cap = 0) {
  const int n = f.n;
  // a vertex whose weight plus the smallest weight exceeds cap has no partner (the search below
  // would find none): it stays single without a look at its row, and when no two vertices fit
  // together no pair can form at all
  int min_vw = INT_MAX;
  for (int v = 0; v < n; ++v) min_vw = std::min(min_vw, f.vw[v]);
  if (n < 2 || 2 * (int64_t)min_vw > cap) return false;
  std::vector<int32_t>& match = sc.match;
  match.assign(n, -1);
  if (!given_top) top_candidates(f, cap, min_vw, sc.top);
  const int32_t* top = given_top ? given_top : sc.top.data();
  const std::vector<int32_t>& order = visit_order(n, level, sc);
  bool any = false;
  for (int v : order) {
    if (match[v] >= 0) continue;
    if (f.vw[v] + min_vw > cap) {
      match[v] = v;
      continue;
    }
    int best = -1;
    bool listed_all = true;  // the list holds every neighbour, so no scan is needed
    for (int i = 0; i < kTop; ++i) {
      const int u = top[(size_t)v * kTop + i];
      if (u < 0) break;
      if (i == kTop - 1) listed_all = false;
      if (match[u] < 0 && f.vw[u] + f.vw[v] <= cap) {
        best = u;
        break;
      }
    }
    if (best < 0 && !listed_all) {
      int bw = -1, bvw = INT_MAX;
      for (int e = f.rp[v]; e < f.rp[v + 1]; ++e) {
        const int u = f.adj[e];
        if (u == v || match[u] >= 0 || f.vw[u] + f.vw[v] > cap) continue;
        const int w = f.ew[e];
        if (w > bw || (w == bw && (f.vw[u] < bvw || (f.vw[u] == bvw && u < best)))) {
          best = u;
          bw = w;
          bvw = f.vw[u];
        }
      }
    }
    if (best >= 0) {
      match[v] = best;
      match[best] = v;
      any = true;
    } else {
      match[v] = v;
    }
  }
  if (!any) return false;
  f.cmap.assign(n, -1);
  int nc = 0;
  for (int v = 0; v < n; ++v)
    if (f.cmap[v] < 0) {
      f.cmap[v] = nc;
      f.cmap[match[v]] = nc;
      ++nc;
    }
  c.n = nc;
  c.vw.assign(nc, 0);
  std::vector<int32_t>& lead = sc.lead;  // the lower member of each pair
  lead.assign(nc, -1);
  for (int v = 0; v < n; ++v) {
    c.vw[f.cmap[v]] += f.vw[v];
    if (lead[f.cmap[v]] < 0) lead[f.cmap[v]] = v;
  }
  if (dev1 && dev1->build(level, n, f.rp, nc, match, f.cmap, lead, c.vw, next_cap, &c.rp,
                          &c.adj, &c.ew, &sc.top1)) {
    c.sorted = true;
    return true;
  }
  sc.top1 = nullptr;
  c.sorted = false;
  // coarse adjacency: summed edge weights, no self loops, neighbours in the order first met
  // (the matching breaks every tie by index, so only the breadth-first order on the coarsest
  // level needs them ascending; sort_rows does that there).  Coarse vertices are independent,
  // so contiguous ranges of them are built on separate threads and concatenated in order (the
  // result does not depend on the thread count).
  const int nt = nc >= 1024 ? worker_count() : 1;
  if ((int)sc.adj_t.size() < nt) {
    sc.adj_t.resize(nt);
    sc.ew_t.resize(nt);
    sc.acc.resize(nt);
  }
  auto& adj_t = sc.adj_t;
  auto& ew_t = sc.ew_t;
  std::vector<int32_t>& deg = sc.deg;
  deg.assign(nc, 0);
  auto build = [&](int t) {
    const int c0 = (int)((int64_t)nc * t / nt), c1 = (int)((int64_t)nc * (t + 1) / nt);
    std::vector<int32_t>& acc = sc.acc[t];
    acc.assign(nc, 0);
    std::vector<int32_t> touched;
    adj_t[t].clear();
    ew_t[t].clear();
    for (int cv = c0; cv < c1; ++cv) {
      const int v = lead[cv];
      const int members[2] = {v, match[v]};
      const int nm = match[v] == v ? 1 : 2;
      // every entry is written to the list and kept only if it is the first of its coarse
      // neighbour (weights are positive, so acc == 0 means not yet met): no data-dependent
      // branch in the loop over the edges; the coarse vertex itself starts marked, so self
      // loops never enter the list
      size_t span = 0;
      for (int q = 0; q < nm; ++q) span += f.rp[members[q] + 1] - f.rp[members[q]];
      if (touched.size() < span) touched.resize(span);
      int32_t* tp = touched.data();
      int m = 0;
      acc[cv] = 1;
      for (int q = 0; q < nm; ++q) {
        const int x = members[q];
        for (int e = f.rp[x]; e < f.rp[x + 1]; ++e) {
          const int cu = f.cmap[f.adj[e]];
          const int32_t a = acc[cu];
          tp[m] = cu;
          m += a == 0;
          acc[cu] = a + f.ew[e];
        }
      }
      acc[cv] = 0;
      const size_t o = adj_t[t].size();
      adj_t[t].resize(o + m);
      ew_t[t].resize(o + m);
      for (int i = 0; i < m; ++i) {
        const int cu = tp[i];
        adj_t[t][o + i] = cu;
        ew_t[t][o + i] = acc[cu];
        acc[cu] = 0;
      }
      deg[cv] = m;
    }
  };
  run_workers(nt, build);
  c.rp_v.assign(nc + 1, 0);
  for (int cv = 0; cv < nc; ++cv) c.rp_v[cv + 1] = c.rp_v[cv] + deg[cv];
  c.adj_v.resize(c.rp_v[nc]);
  c.ew_v.resize(c.rp_v[nc]);
  run_workers(nt, [&](int t) {
    const int c0 = (int)((int64_t)nc * t / nt);
    std::copy(adj_t[t].begin(), adj_t[t].end(), c.adj_v.begin() + c.rp_v[c0]);
    std::copy(ew_t[t].begin(), ew_t[t].end(), c.ew_v.begin() + c.rp_v[c0]);
  });
  c.rp = c.rp_v.data();
  c.adj = c.adj_v.data();
  c.ew = c.ew_v.data();
  return true;
}

// Neighbours of a coarse level in ascending order, with their edge weights.
void sort_rows(Level& g) {
  const int nt = g.rp[g.n] >= (1 << 16) ? worker_count() : 1;
  run_workers(nt, [&](int t) {
    const int v0 = (int)((int64_t)g.n * t / nt), v1 = (int)((int64_t)g.n * (t + 1) / nt);
    std::vector<std::pair<int32_t, int32_t>> row;
    for (int v = v0; v < v1; ++v) {
      row.clear();
      for (int e = g.rp[v]; e < g.rp[v + 1]; ++e) row.emplace_back(g.adj_v[e], g.ew_v[e]);
      std::sort(row.begin(), row.end());
      for (int e = g.rp[v], i = 0; e < g.rp[v + 1]; ++e, ++i) {
        g.adj_v[e] = row[i].first;
        g.ew_v[e] = row[i].second;
      }
    }
  });
}

// Breadth-first order of a graph: components in ascending order of their smallest vertex,
// neighbours in ascending index order.
std::vector<int32_t> bfs_order(const Level& g) {
  std::vector<int32_t> o;
  o.reserve(g.n);
  std::vector<char> seen(g.n, 0);
  for (int s0 = 0; s0 < g.n; ++s0) {
    if (seen[s0]) continue;
    seen[s0] = 1;
    size_t head = o.size();
    o.push_back(s0);
    while (head < o.size()) {
      const int v = o[head++];
      for (int e = g.rp[v]; e < g.rp[v + 1]; ++e) {
        const int u = g.adj[e];
        if (!seen[u]) {
          seen[u] = 1;
          o.push_back(u);
        }
      }
    }
  }
  return o;
}

// Parts grown on g (weights <= cap): seeds in breadth-first order; a part repeatedly takes the
// unassigned neighbour with the largest summed edge weight to it (ties: smaller weight, then
// smaller index) that still fits.
// A part that no vertex fits into any more (its weight plus the smallest weight above cap) is
// closed at once: the search would find nothing.
std::vector<int32_t> grow_parts(const Level& g, int cap) {
  std::vector<int32_t> part(g.n, -1), conn(g.n, 0), touched;
  int min_vw = INT_MAX;
  for (int v = 0; v < g.n; ++v) min_vw = std::min(min_vw, g.vw[v]);
  int np = 0;
  for (int seed : bfs_order(g)) {
    if (part[seed] >= 0) continue;
    const int p = np++;
    int w = 0;
    int v = seed;
    touched.clear();
    for (;;) {
      part[v] = p;
      w += g.vw[v];
      if ((int64_t)w + min_vw > cap) break;
      for (int e = g.rp[v]; e < g.rp[v + 1]; ++e) {
        const int u = g.adj[e];
        if (part[u] >= 0) continue;
        if (conn[u] == 0) touched.push_back(u);
        conn[u] += g.ew[e];
      }
      int best = -1, bc = 0, bvw = INT_MAX;
      for (int u : touched) {
        if (part[u] >= 0 || w + g.vw[u] > cap) continue;
        const int cu = conn[u];
        if (cu > bc || (cu == bc && (g.vw[u] < bvw || (g.vw[u] == bvw && u < best)))) {
          best = u;
          bc = cu;
          bvw = g.vw[u];
        }
      }
      if (best < 0) break;
      v = best;
    }
    for (int u : touched) conn[u] = 0;
  }
  return part;
}

int64_t cube(int64_t x) { return x * x * x; }

// sum over parts of (|core| + |halo|)^3 on g (halo: vertices outside the part adjacent to it)
int64_t subgraph_cost(const Level& g, const std::vector<int32_t>& part, int np) {
  const int nt = g.n >= 1024 ? worker_count() : 1;
  std::vector<std::vector<int64_t>> kt(nt, std::vector<int64_t>(np, 0)),
      ht(nt, std::vector<int64_t>(np, 0));
  run_workers(nt, [&](int t) {
    const int u0 = (int)((int64_t)g.n * t / nt), u1 = (int)((int64_t)g.n * (t + 1) / nt);
    std::vector<int32_t> stamp(np, -1);
    for (int u = u0; u < u1; ++u) {
      ++kt[t][part[u]];
      for (int e = g.rp[u]; e < g.rp[u + 1]; ++e) {
        const int p = part[g.adj[e]];
        if (p != part[u] && stamp[p] != u) {
          stamp[p] = u;
          ++ht[t][p];
        }
      }
    }
  });
  int64_t c = 0;
  for (int p = 0; p < np; ++p) {
    int64_t k = 0, h = 0;
    for (int t = 0; t < nt; ++t) {
      k += kt[t][p];
      h += ht[t][p];
    }
    c += cube(k + h);
  }
  return c;
}

}  // namespace

namespace {

// Level 0: the input graph in place (self loops skipped where they matter), weights = common
// closed neighbours (given per CSR entry, or counted here unless want_weights is false), unit
// vertex weights.
void input_level(int n, const int32_t* row_ptr, const int32_t* col, const int32_t* ew, Level& g0,
                 bool want_weights = true) {
  g0.n = n;
  g0.rp = row_ptr;
  g0.adj = col;
  g0.vw.assign(n, 1);
  g0.ew = ew;
  if (ew || !want_weights) return;
  // the number of common closed neighbours: the pair's joint halo is smallest for the
  // neighbour sharing most of its neighbourhood
  g0.ew_v.assign(row_ptr[n], 0);
  const int nt = n >= 1024 ? worker_count() : 1;
  run_workers(nt, [&](int t) {
    const int u0 = (int)((int64_t)n * t / nt), u1 = (int)((int64_t)n * (t + 1) / nt);
    std::vector<int32_t> mark(n, -1);
    for (int u = u0; u < u1; ++u) {
      mark[u] = u;
      for (int e = row_ptr[u]; e < row_ptr[u + 1]; ++e) mark[col[e]] = u;
      for (int e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        const int v = col[e];
        if (v == u) continue;
        int c = 1;  // v itself (it is a neighbour of u)
        for (int f = row_ptr[v]; f < row_ptr[v + 1]; ++f) c += col[f] != v && mark[col[f]] == u;
        g0.ew_v[e] = c;
      }
    }
  });
  g0.ew = g0.ew_v.data();
}

// Non-empty parts in ascending order of their smallest vertex, vertices ascending.
void emit_cores(int n, const std::vector<int32_t>& part, int np, std::vector<int32_t>& core_ptr,
                std::vector<int32_t>& core_vtx) {
  std::vector<int32_t> first(np, INT_MAX), rank(np, -1), size(np, 0);
  for (int v = 0; v < n; ++v) {
    first[part[v]] = std::min(first[part[v]], v);
    ++size[part[v]];
  }
  std::vector<int32_t> ids;
  for (int p = 0; p < np; ++p)
    if (size[p] > 0) ids.push_back(p);
  std::sort(ids.begin(), ids.end(), [&](int a, int b) { return first[a] < first[b]; });
  core_ptr.assign(ids.size() + 1, 0);
  for (size_t i = 0; i < ids.size(); ++i) {
    rank[ids[i]] = (int32_t)i;
    core_ptr[i + 1] = core_ptr[i] + size[ids[i]];
  }
  core_vtx.assign(n, 0);
  std::vector<int32_t> fill(core_ptr.begin(), core_ptr.end() - 1);
  for (int v = 0; v < n; ++v) core_vtx[fill[rank[part[v]]]++] = v;
}

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t) {
  return std::chrono::duration<double, std::milli>(clk::now() - t).count();
}

}  // namespace

MlLease::MlLease() {
  std::lock_guard<std::mutex> lk(g_ml_mu);
  if (g_ml_free.empty()) {
    p = new MlScratch;
  } else {
    p = g_ml_free.back();
    g_ml_free.pop_back();
  }
}

MlLease::~MlLease() {
  std::lock_guard<std::mutex> lk(g_ml_mu);
  g_ml_free.push_back(p);
}

void ml_trim() {
  std::lock_guard<std::mutex> lk(g_ml_mu);
  for (MlScratch* sc : g_ml_free) {
    for (int32_t* q : {sc->h_rp, sc->h_col, sc->h_w, sc->h_rp1, sc->h_adj1, sc->h_ew1,
                       sc->h_top1})
      if (q) GB_HIP(hipHostFree(q));
    delete sc;
  }
  g_ml_free.clear();
}

void ml_stage(MlScratch& sc, int n, int64_t nnz, int32_t** rp, int32_t** col, int32_t** w) {
  pinned_reserve(sc.h_rp, sc.cap_rp, (size_t)n + 1);
  pinned_reserve(sc.h_col, sc.cap_col, (size_t)std::max<int64_t>(nnz, 1));
  if (w) pinned_reserve(sc.h_w, sc.cap_w, (size_t)std::max<int64_t>(nnz, 1));
  *rp = sc.h_rp;
  *col = sc.h_col;
  if (w) *w = sc.h_w;
}

void ml_stage1(MlScratch& sc, int nc, int64_t nnz, int32_t** rp, int32_t** adj, int32_t** ew,
               int32_t** top) {
  pinned_reserve(sc.h_rp1, sc.cap_rp1, (size_t)nc + 1);
  pinned_reserve(sc.h_adj1, sc.cap_adj1, (size_t)std::max<int64_t>(nnz, 1));
  pinned_reserve(sc.h_ew1, sc.cap_ew1, (size_t)std::max<int64_t>(nnz, 1));
  pinned_reserve(sc.h_top1, sc.cap_top1, (size_t)nc * kMlTop);
  *rp = sc.h_rp1;
  *adj = sc.h_adj1;
  *ew = sc.h_ew1;
  *top = sc.h_top1;
}

int32_t* ml_top_buffer(MlScratch& sc, int n) {
  sc.top.resize((size_t)n * kMlTop);
  return sc.top.data();
}

void partition_multilevel(int n, const int32_t* row_ptr, const int32_t* col, int cap,
                          std::vector<int32_t>& core_ptr, std::vector<int32_t>& core_vtx,
                          MlStats* stats, const int32_t* ew, MlScratch* scr,
                          const int32_t* top0, MlCoarseDevice* dev1) {
  std::unique_ptr<MlLease> own;
  if (!scr) {
    own.reset(new MlLease);
    scr = own->p;
  }
  MlScratch& sc = *scr;
  auto t0 = clk::now();
  sc.top1 = nullptr;  // set by this call's dev1 only
  if (sc.lv.empty()) sc.lv.resize(1);  // levels are addressed by index: lv may grow below
  input_level(n, row_ptr, col, ew, sc.lv[0]);
  const double ms_weights = ms_since(t0);
  t0 = clk::now();
  const int ccap = std::max(1, cap / 4);
  int nl = 1;
  for (int level = 0;; ++level) {
    if ((int)sc.lv.size() == nl) sc.lv.emplace_back();
    // the input level's lists come from top0; a coarse level's from dev1 when it built that
    // level (sc.top1 is reset whenever the host builds one)
    const int32_t* given = level == 0 ? top0 : sc.top1;
    if (!coarsen(sc.lv[nl - 1], ccap, level, sc.lv[nl], sc, given, dev1, ccap)) break;
    ++nl;
  }
  // the input level keeps the caller's row order
  if (nl > 1 && !sc.lv[nl - 1].sorted) sort_rows(sc.lv[nl - 1]);
  const double ms_coarsen = ms_since(t0);
  t0 = clk::now();
  std::vector<int32_t> part = grow_parts(sc.lv[nl - 1], cap);
  const double ms_grow = ms_since(t0);
  t0 = clk::now();
  int np = 0;
  for (int p : part) np = std::max(np, p + 1);
  for (int l = nl - 2; l >= 0; --l) {
    std::vector<int32_t> fine(sc.lv[l].n);
    for (int v = 0; v < sc.lv[l].n; ++v) fine[v] = part[sc.lv[l].cmap[v]];
    part.swap(fine);
  }
  // the cost is a statistic (the device path gets the subgraph sizes from its halos anyway)
  const int64_t cost = stats ? subgraph_cost(sc.lv[0], part, np) : 0;
  const double ms_cost = ms_since(t0);
  emit_cores(n, part, np, core_ptr, core_vtx);
  if (stats) {
    stats->levels = nl;
    stats->coarsest = sc.lv[nl - 1].n;
    stats->cost = cost;
    stats->ms_weights = ms_weights;
    stats->ms_coarsen = ms_coarsen;
    stats->ms_grow = ms_grow;
    stats->ms_cost = ms_cost;
  }
}

void partition_update(int n, const int32_t* row_ptr, const int32_t* col,
                      const std::vector<int32_t>& prev_ptr, const std::vector<int32_t>& prev_vtx,
                      std::vector<int32_t>& core_ptr, std::vector<int32_t>& core_vtx,
                      MlStats* stats) {
  auto t0 = clk::now();
  Level g0;
  input_level(n, row_ptr, col, nullptr, g0, false);
  const int np = (int)prev_ptr.size() - 1;
  std::vector<int32_t> part(n, -1);
  for (int p = 0; p < np; ++p)
    for (int i = prev_ptr[p]; i < prev_ptr[p + 1]; ++i) part[prev_vtx[i]] = p;
  const int64_t cost = stats ? subgraph_cost(g0, part, np) : 0;
  emit_cores(n, part, np, core_ptr, core_vtx);
  if (stats) {
    stats->levels = 1;
    stats->coarsest = n;
    stats->cost = cost;
    stats->ms_cost = ms_since(t0);
  }
}

}  // namespace gbi
