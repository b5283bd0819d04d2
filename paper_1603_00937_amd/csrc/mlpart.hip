// Multilevel core partitioner (host code).
//
// The cost of the method is the sum over subgraphs of n_s^3, n_s = |core| + |halo| (the dense
// products of every subgraph; the paper's cost discussion after Eq. 6), and the paper takes its
// communities from a multilevel graph partitioner.  This one is written for that objective with
// a hard cap on the core size (the batched kernels are sized for it):
//   1. coarsening by heavy-edge matching, pairs limited to a quarter of the cap, until no pair
//      can be matched: each level halves the graph while keeping strongly tied vertices
//      together;
//   2. on the coarsest graph, parts grown one at a time by always adding the unassigned
//      neighbour most strongly tied to the part while it fits under the cap, seeds taken in
//      breadth-first order so that parts follow one another through the graph;
//   3. on the way back to the input graph, at every level, greedy passes moving boundary
//      vertices to the neighbouring part they are most tied to when that cuts edge weight and
//      the part has room;
//   4. on the input graph, passes moving vertices to one of their three most tied neighbouring
//      parts when that lowers sum (|core| + |halo|)^3 exactly (halo sizes kept incrementally).
// Everything is integer and every choice has a fixed tie-break, so the result is a function of
// the graph alone.  The visiting order of the matching is a fixed pseudo-random permutation
// (vertices sorted by SplitMix64 of (level << 32 | v)).

#include "internal.h"

#include <algorithm>
#include <chrono>
#include <climits>
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

struct Level {
  int n = 0;
  std::vector<int32_t> rp, adj, ew, vw;  // CSR without self loops, edge and vertex weights
  std::vector<int32_t> cmap;             // vertex -> vertex of the next coarser level
};

std::vector<int32_t> visit_order(int n, int level) {
  std::vector<std::pair<uint64_t, int32_t>> k(n);
  for (int v = 0; v < n; ++v) k[v] = {splitmix64(((uint64_t)level << 32) | (uint32_t)v), v};
  std::sort(k.begin(), k.end());
  std::vector<int32_t> o(n);
  for (int i = 0; i < n; ++i) o[i] = k[i].second;
  return o;
}

// Heavy-edge matching of f (pairs of weight <= cap); returns false if no pair was matched.
bool coarsen(Level& f, int cap, int level, Level& c) {
  const int n = f.n;
  std::vector<int32_t> match(n, -1);
  bool any = false;
  for (int v : visit_order(n, level)) {
    if (match[v] >= 0) continue;
    int best = -1, bw = -1, bvw = INT_MAX;
    for (int e = f.rp[v]; e < f.rp[v + 1]; ++e) {
      const int u = f.adj[e];
      if (match[u] >= 0 || f.vw[u] + f.vw[v] > cap) continue;
      const int w = f.ew[e];
      if (w > bw || (w == bw && (f.vw[u] < bvw || (f.vw[u] == bvw && u < best)))) {
        best = u;
        bw = w;
        bvw = f.vw[u];
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
  for (int v = 0; v < n; ++v) c.vw[f.cmap[v]] += f.vw[v];
  // coarse adjacency: summed edge weights, neighbours ascending, no self loops
  c.rp.assign(nc + 1, 0);
  c.adj.clear();
  c.ew.clear();
  std::vector<int32_t> acc(nc, 0), touched;
  int cv = 0;
  for (int v = 0; v < n; ++v) {
    if (f.cmap[v] != cv) continue;  // the lower member of each pair opens its coarse vertex
    const int members[2] = {v, match[v]};
    const int nm = match[v] == v ? 1 : 2;
    touched.clear();
    for (int q = 0; q < nm; ++q) {
      const int x = members[q];
      for (int e = f.rp[x]; e < f.rp[x + 1]; ++e) {
        const int cu = f.cmap[f.adj[e]];
        if (cu == cv) continue;
        if (acc[cu] == 0) touched.push_back(cu);
        acc[cu] += f.ew[e];
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int cu : touched) {
      c.adj.push_back(cu);
      c.ew.push_back(acc[cu]);
      acc[cu] = 0;
    }
    c.rp[cv + 1] = (int32_t)c.adj.size();
    ++cv;
  }
  return true;
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
std::vector<int32_t> grow_parts(const Level& g, int cap) {
  std::vector<int32_t> part(g.n, -1), conn(g.n, 0), touched;
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

// Greedy passes on g: each vertex (ascending) moves to the neighbouring part with the largest
// positive gain in internal edge weight (ties: smaller part index) if that part has room.
void refine_cut(const Level& g, std::vector<int32_t>& part, std::vector<int32_t>& pw, int cap,
                int passes) {
  const int np = (int)pw.size();
  std::vector<int32_t> conn(np, 0), touched;
  for (int pass = 0; pass < passes; ++pass) {
    int moved = 0;
    for (int v = 0; v < g.n; ++v) {
      const int a = part[v];
      touched.clear();
      for (int e = g.rp[v]; e < g.rp[v + 1]; ++e) {
        const int b = part[g.adj[e]];
        if (conn[b] == 0) touched.push_back(b);
        conn[b] += g.ew[e];
      }
      const int own = conn[a];
      int best = -1, bg = 0;
      for (int b : touched) {
        if (b == a || pw[b] + g.vw[v] > cap) continue;
        const int gain = conn[b] - own;
        if (gain > bg || (gain == bg && gain > 0 && b < best)) {
          best = b;
          bg = gain;
        }
      }
      for (int b : touched) conn[b] = 0;
      if (best >= 0) {
        part[v] = best;
        pw[a] -= g.vw[v];
        pw[best] += g.vw[v];
        ++moved;
      }
    }
    if (!moved) break;
  }
}

int64_t cube(int64_t x) { return x * x * x; }

// Per-vertex counts of neighbours in each part: a sorted (part, count) list per vertex.
struct PartCounts {
  std::vector<std::vector<std::pair<int32_t, int32_t>>> c;
  int get(int u, int p) const {
    const auto& l = c[u];
    auto it = std::lower_bound(l.begin(), l.end(), std::make_pair(p, INT_MIN));
    return (it != l.end() && it->first == p) ? it->second : 0;
  }
  void add(int u, int p, int d) {
    auto& l = c[u];
    auto it = std::lower_bound(l.begin(), l.end(), std::make_pair(p, INT_MIN));
    if (it != l.end() && it->first == p) {
      it->second += d;
      if (it->second == 0) l.erase(it);
    } else {
      l.insert(it, {p, d});
    }
  }
};

// Passes on the input graph lowering sum_p (k_p + h_p)^3 exactly: each vertex (ascending)
// tries its three most tied neighbouring parts (ties: smaller index) with room, and moves to
// the one with the largest decrease.
int64_t refine_cost(const Level& g, std::vector<int32_t>& part, int np, int cap, int passes) {
  const int n = g.n;
  PartCounts pc;
  pc.c.resize(n);
  std::vector<int64_t> k(np, 0), h(np, 0);
  for (int v = 0; v < n; ++v) ++k[part[v]];
  for (int u = 0; u < n; ++u) {
    for (int e = g.rp[u]; e < g.rp[u + 1]; ++e) pc.add(u, part[g.adj[e]], 1);
    for (const auto& pr : pc.c[u])
      if (pr.first != part[u]) ++h[pr.first];
  }
  int64_t cost = 0;
  for (int p = 0; p < np; ++p) cost += cube(k[p] + h[p]);
  std::vector<int32_t> conn(np, 0), touched;
  for (int pass = 0; pass < passes; ++pass) {
    int moved = 0;
    for (int v = 0; v < n; ++v) {
      const int a = part[v];
      // change of h_a if v leaves a: neighbours outside a whose only tie to a is v leave the
      // halo; v joins it if it keeps a neighbour in a
      int64_t dha = pc.get(v, a) > 0 ? 1 : 0;
      for (int e = g.rp[v]; e < g.rp[v + 1]; ++e) {
        const int u = g.adj[e];
        if (part[u] != a && pc.get(u, a) == 1) --dha;
      }
      touched.clear();
      for (int e = g.rp[v]; e < g.rp[v + 1]; ++e) {
        const int b = part[g.adj[e]];
        if (b == a) continue;
        if (conn[b] == 0) touched.push_back(b);
        conn[b] += g.ew[e];
      }
      // the three most tied candidate parts with room
      int cand[3] = {-1, -1, -1};
      for (int b : touched) {
        if (k[b] + 1 > cap) continue;
        for (int q = 0; q < 3; ++q) {
          const int c = cand[q];
          if (c < 0 || conn[b] > conn[c] || (conn[b] == conn[c] && b < c)) {
            for (int r = 2; r > q; --r) cand[r] = cand[r - 1];
            cand[q] = b;
            break;
          }
        }
      }
      for (int b : touched) conn[b] = 0;
      const int64_t before_a = cube(k[a] + h[a]);
      const int64_t after_a = cube(k[a] - 1 + h[a] + dha);
      int best = -1;
      int64_t best_d = 0, best_dhb = 0;
      for (int q = 0; q < 3; ++q) {
        const int b = cand[q];
        if (b < 0) break;
        // change of h_b if v joins b: v leaves the halo of b; neighbours outside b with no tie
        // to b yet join it
        int64_t dhb = pc.get(v, b) > 0 ? -1 : 0;
        for (int e = g.rp[v]; e < g.rp[v + 1]; ++e) {
          const int u = g.adj[e];
          if (part[u] != b && pc.get(u, b) == 0) ++dhb;
        }
        const int64_t d = after_a - before_a + cube(k[b] + 1 + h[b] + dhb) - cube(k[b] + h[b]);
        if (d < best_d) {
          best_d = d;
          best = b;
          best_dhb = dhb;
        }
      }
      if (best < 0) continue;
      for (int e = g.rp[v]; e < g.rp[v + 1]; ++e) {
        const int u = g.adj[e];
        pc.add(u, a, -1);
        pc.add(u, best, 1);
      }
      h[a] += dha;
      h[best] += best_dhb;
      --k[a];
      ++k[best];
      part[v] = best;
      cost += best_d;
      ++moved;
    }
    if (!moved) break;
  }
  return cost;
}

}  // namespace

namespace {

// Level 0: the input graph without self loops, weights = common closed neighbours (given, or
// counted here), unit vertex weights.
void input_level(int n, const int32_t* row_ptr, const int32_t* col, const int32_t* ew, Level& g0) {
  g0.n = n;
  g0.rp.assign(n + 1, 0);
  g0.adj.clear();
  g0.ew.clear();
  for (int v = 0; v < n; ++v) {
    for (int e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
      if (col[e] != v) {
        g0.adj.push_back(col[e]);
        if (ew) g0.ew.push_back(ew[e]);
      }
    g0.rp[v + 1] = (int32_t)g0.adj.size();
  }
  g0.vw.assign(n, 1);
  if (ew) return;
  // edge weight = number of common neighbours (each vertex counted as its own neighbour): the
  // pair's joint halo is smallest for the neighbour sharing most of its neighbourhood
  g0.ew.assign(g0.adj.size(), 0);
  std::vector<int32_t> mark(n, -1);
  for (int u = 0; u < n; ++u) {
    mark[u] = u;
    for (int e = g0.rp[u]; e < g0.rp[u + 1]; ++e) mark[g0.adj[e]] = u;
    for (int e = g0.rp[u]; e < g0.rp[u + 1]; ++e) {
      const int v = g0.adj[e];
      int c = mark[v] == u ? 1 : 0;  // v itself (it is a neighbour of u)
      for (int f = g0.rp[v]; f < g0.rp[v + 1]; ++f) c += mark[g0.adj[f]] == u;
      g0.ew[e] = c;
    }
  }
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

void partition_multilevel(int n, const int32_t* row_ptr, const int32_t* col, int cap,
                          std::vector<int32_t>& core_ptr, std::vector<int32_t>& core_vtx,
                          MlStats* stats, const int32_t* ew) {
  auto t0 = clk::now();
  std::vector<Level> lv(1);  // lv grows below: levels are addressed by index, not reference
  input_level(n, row_ptr, col, ew, lv[0]);
  const double ms_weights = ms_since(t0);
  t0 = clk::now();
  const int ccap = std::max(1, cap / 4);
  for (int level = 0;; ++level) {
    Level c;
    if (!coarsen(lv.back(), ccap, level, c)) break;
    lv.push_back(std::move(c));
  }
  const double ms_coarsen = ms_since(t0);
  t0 = clk::now();
  std::vector<int32_t> part = grow_parts(lv.back(), cap);
  const double ms_grow = ms_since(t0);
  t0 = clk::now();
  int np = 0;
  for (int p : part) np = std::max(np, p + 1);
  for (int l = (int)lv.size() - 1; l >= 0; --l) {
    if (l < (int)lv.size() - 1) {
      std::vector<int32_t> fine(lv[l].n);
      for (int v = 0; v < lv[l].n; ++v) fine[v] = part[lv[l].cmap[v]];
      part.swap(fine);
    }
    std::vector<int32_t> pw(np, 0);
    for (int v = 0; v < lv[l].n; ++v) pw[part[v]] += lv[l].vw[v];
    refine_cut(lv[l], part, pw, cap, 4);
  }
  const double ms_cut = ms_since(t0);
  t0 = clk::now();
  const int64_t cost = refine_cost(lv[0], part, np, cap, 4);
  const double ms_cost = ms_since(t0);
  emit_cores(n, part, np, core_ptr, core_vtx);
  if (stats) {
    stats->levels = (int)lv.size();
    stats->coarsest = lv.back().n;
    stats->cost = cost;
    stats->ms_weights = ms_weights;
    stats->ms_coarsen = ms_coarsen;
    stats->ms_grow = ms_grow;
    stats->ms_cut = ms_cut;
    stats->ms_cost = ms_cost;
  }
}

void partition_update(int n, const int32_t* row_ptr, const int32_t* col, int cap,
                      const std::vector<int32_t>& prev_ptr, const std::vector<int32_t>& prev_vtx,
                      std::vector<int32_t>& core_ptr, std::vector<int32_t>& core_vtx,
                      MlStats* stats, const int32_t* ew) {
  auto t0 = clk::now();
  Level g0;
  input_level(n, row_ptr, col, ew, g0);
  const double ms_weights = ms_since(t0);
  t0 = clk::now();
  const int np = (int)prev_ptr.size() - 1;
  std::vector<int32_t> part(n, -1);
  for (int p = 0; p < np; ++p)
    for (int i = prev_ptr[p]; i < prev_ptr[p + 1]; ++i) part[prev_vtx[i]] = p;
  const int64_t cost = refine_cost(g0, part, np, cap, 4);
  emit_cores(n, part, np, core_ptr, core_vtx);
  if (stats) {
    stats->levels = 1;
    stats->coarsest = n;
    stats->cost = cost;
    stats->ms_weights = ms_weights;
    stats->ms_cost = ms_since(t0);
  }
}

}  // namespace gbi
