// Host-side planner.  See plan.hpp for the method references.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace qtn {

std::string make_graph(int n, int64_t m, const int32_t *edges, Graph *g) {
  if (n < 2) return "graph needs at least 2 vertices";
  if (m < 1) return "graph needs at least 1 edge";
  if (!edges) return "edge array is NULL";
  if (m > (int64_t)1 << 26) return "too many edges";
  g->n = n;
  g->eu.resize(m);
  g->ev.resize(m);
  g->adj.assign(n, {});
  std::vector<std::vector<int>> seen(n);
  for (int64_t e = 0; e < m; e++) {
    int a = edges[2 * e], b = edges[2 * e + 1];
    if (a < 0 || b < 0 || a >= n || b >= n)
      return "edge " + std::to_string(e) + " has an endpoint out of range";
    if (a == b) return "edge " + std::to_string(e) + " is a self-loop";
    for (int x : seen[a])
      if (x == b) return "edge " + std::to_string(e) + " is repeated";
    seen[a].push_back(b);
    seen[b].push_back(a);
    g->eu[e] = a;
    g->ev[e] = b;
    g->adj[a].push_back((int)e);
    g->adj[b].push_back((int)e);
  }
  return "";
}

// Sec. II-B: the observable Z_j Z_k commutes with every gate outside its
// reverse light cone, so those gates cancel against their conjugates.  Walking
// back from the observable, layer l (1-based) keeps mixers on the vertices
// within distance p-l of {j,k} and cost gates on edges touching them.
LightCone build_lightcone(const Graph &g, int e, int p) {
  LightCone lc;
  lc.edge = e;
  lc.j = g.eu[e];
  lc.k = g.ev[e];
  std::vector<int> dist(g.n, -1), queue;
  queue.reserve(g.n);
  dist[lc.j] = 0;
  dist[lc.k] = 0;
  queue.push_back(lc.j);
  queue.push_back(lc.k);
  for (size_t h = 0; h < queue.size(); h++) {
    int u = queue[h];
    if (dist[u] >= p) continue;
    for (int f : g.adj[u]) {
      int w = g.eu[f] == u ? g.ev[f] : g.eu[f];
      if (dist[w] < 0) {
        dist[w] = dist[u] + 1;
        queue.push_back(w);
      }
    }
  }
  // cone vertices ascending, and the edges touching distance <= p-1 ascending
  std::vector<int> verts;
  for (int v = 0; v < g.n; v++)
    if (dist[v] >= 0) verts.push_back(v);
  std::vector<int> cone_edges;
  for (int v : verts)
    if (dist[v] <= p - 1)
      for (int f : g.adj[v]) cone_edges.push_back(f);
  std::sort(cone_edges.begin(), cone_edges.end());
  cone_edges.erase(std::unique(cone_edges.begin(), cone_edges.end()), cone_edges.end());

  auto within = [&](int v, int r) { return dist[v] >= 0 && dist[v] <= r; };
  std::vector<int> cur(g.n, -1);
  int nv = 0;
  for (int v : verts) {
    cur[v] = nv++;
    lc.gates.push_back({kH, 0, 1, {cur[v], -1}});
  }
  for (int l = 1; l <= p; l++) {
    for (int f : cone_edges)
      if (within(g.eu[f], p - l) || within(g.ev[f], p - l))
        lc.gates.push_back({kP, (int8_t)(l - 1), 2, {cur[g.eu[f]], cur[g.ev[f]]}});
    for (int v : verts)
      if (within(v, p - l)) {
        int x = nv++;
        lc.gates.push_back({kR, (int8_t)(l - 1), 2, {x, cur[v]}});
        cur[v] = x;
      }
  }
  lc.gates.push_back({kZ, 0, 1, {cur[lc.j], -1}});
  lc.gates.push_back({kZ, 0, 1, {cur[lc.k], -1}});
  for (int l = p; l >= 1; l--) {
    for (int v : verts)
      if (within(v, p - l)) {
        int y = nv++;
        lc.gates.push_back({kRc, (int8_t)(l - 1), 2, {cur[v], y}});
        cur[v] = y;
      }
    for (int f : cone_edges)
      if (within(g.eu[f], p - l) || within(g.ev[f], p - l))
        lc.gates.push_back({kPc, (int8_t)(l - 1), 2, {cur[g.eu[f]], cur[g.ev[f]]}});
  }
  for (int v : verts) lc.gates.push_back({kH, 0, 1, {cur[v], -1}});
  lc.n_vars = nv;
  return lc;
}

// Greedy min-fill over the interaction graph (a vertex per variable, a clique
// per tensor), with neighbour sets as bitsets.  Eliminating v joins its
// neighbours into a clique; only the neighbours of v and their neighbours can
// change fill, so only those are re-scored.
std::vector<int> minfill_order(const LightCone &lc, uint64_t seed) {
  const int n = lc.n_vars, W = (n + 63) / 64;
  // seed 0: ties by smallest id; otherwise ties broken by a splitmix64 draw
  uint64_t rs = seed;
  auto draw = [&rs]() {
    rs += 0x9E3779B97F4A7C15ull;
    uint64_t z = rs;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  std::vector<uint64_t> adj((size_t)n * W, 0), alive(W, 0);
  auto row = [&](int v) { return &adj[(size_t)v * W]; };
  auto setb = [](uint64_t *r, int b) { r[b >> 6] |= 1ull << (b & 63); };
  auto getb = [](const uint64_t *r, int b) { return (r[b >> 6] >> (b & 63)) & 1; };
  for (const Gate &gt : lc.gates)
    if (gt.rank == 2 && gt.var[0] != gt.var[1]) {
      setb(row(gt.var[0]), gt.var[1]);
      setb(row(gt.var[1]), gt.var[0]);
    }
  for (int v = 0; v < n; v++) setb(alive.data(), v);
  std::vector<int64_t> fill(n);
  std::vector<int> deg(n), nb, order;
  std::vector<uint64_t> tmp(W);
  auto score = [&](int v) {
    const uint64_t *r = row(v);
    nb.clear();
    for (int w = 0; w < W; w++) {
      uint64_t x = r[w] & alive[w];
      while (x) {
        nb.push_back(w * 64 + __builtin_ctzll(x));
        x &= x - 1;
      }
    }
    int64_t f = 0;
    for (int a : nb) {
      const uint64_t *ra = row(a);
      for (int w = 0; w < W; w++) tmp[w] = r[w] & alive[w] & ~ra[w];
      tmp[a >> 6] &= ~(1ull << (a & 63));
      for (int w = 0; w < W; w++) f += __builtin_popcountll(tmp[w]);
    }
    fill[v] = f / 2;
    deg[v] = (int)nb.size();
  };
  for (int v = 0; v < n; v++) score(v);
  std::vector<char> touched(n);
  std::vector<int> ties;
  for (int step = 0; step < n; step++) {
    int best = -1;
    for (int v = 0; v < n; v++) {
      if (!getb(alive.data(), v)) continue;
      if (best < 0 || fill[v] < fill[best] ||
          (fill[v] == fill[best] && deg[v] < deg[best]))
        best = v;
    }
    if (seed) {
      ties.clear();
      for (int v = 0; v < n; v++)
        if (getb(alive.data(), v) && fill[v] == fill[best] && deg[v] == deg[best]) ties.push_back(v);
      best = ties[draw() % ties.size()];
    }
    order.push_back(best);
    alive[best >> 6] &= ~(1ull << (best & 63));
    std::vector<int> nv;
    const uint64_t *rb = row(best);
    for (int w = 0; w < W; w++) {
      uint64_t x = rb[w] & alive[w];
      while (x) {
        nv.push_back(w * 64 + __builtin_ctzll(x));
        x &= x - 1;
      }
    }
    for (int a : nv) {
      uint64_t *ra = row(a);
      for (int b : nv)
        if (b != a) setb(ra, b);
    }
    std::fill(touched.begin(), touched.end(), 0);
    for (int a : nv) {
      touched[a] = 1;
      const uint64_t *ra = row(a);
      for (int w = 0; w < W; w++) {
        uint64_t x = ra[w] & alive[w];
        while (x) {
          touched[w * 64 + __builtin_ctzll(x)] = 1;
          x &= x - 1;
        }
      }
    }
    for (int v = 0; v < n; v++)
      if (touched[v] && getb(alive.data(), v)) score(v);
  }
  return order;
}

double order_cost(const LightCone &lc, const std::vector<int> &order) {
  // sum over buckets of 2^width, from index sets alone
  const int n = lc.n_vars;
  std::vector<int> pos(n);
  for (int i = 0; i < n; i++) pos[order[i]] = i;
  std::vector<std::vector<int>> bucket(n);
  auto place = [&](std::vector<int> vars) {
    int b = n;
    for (int v : vars) b = std::min(b, pos[v]);
    bucket[b].insert(bucket[b].end(), vars.begin(), vars.end());
    bucket[b].push_back(-1);  // tensor separator
  };
  for (const Gate &g : lc.gates) {
    std::vector<int> v = {g.var[0]};
    if (g.rank == 2) v.push_back(g.var[1]);
    place(v);
  }
  double cost = 0;
  std::vector<char> mark(n, 0);
  for (int i = 0; i < n; i++) {
    if (bucket[i].empty()) continue;
    std::vector<int> u;
    for (int v : bucket[i])
      if (v >= 0 && !mark[v]) {
        mark[v] = 1;
        u.push_back(v);
      }
    for (int v : u) mark[v] = 0;
    cost += std::ldexp(1.0, (int)u.size());
    std::vector<int> rest;
    for (int v : u)
      if (v != order[i]) rest.push_back(v);
    if (!rest.empty()) place(rest);
  }
  return cost;
}

int order_width(const LightCone &lc, const std::vector<int> &order, std::vector<int> *widest) {
  const int n = lc.n_vars;
  std::vector<int> pos(n);
  for (int i = 0; i < n; i++) pos[order[i]] = i;
  std::vector<std::vector<int>> bucket(n);
  auto place = [&](const std::vector<int> &vars) {
    int b = n;
    for (int v : vars) b = std::min(b, pos[v]);
    bucket[b].insert(bucket[b].end(), vars.begin(), vars.end());
  };
  for (const Gate &g : lc.gates) {
    std::vector<int> v = {g.var[0]};
    if (g.rank == 2) v.push_back(g.var[1]);
    place(v);
  }
  int best = 0;
  std::vector<char> mark(n, 0);
  std::vector<int> u;
  for (int i = 0; i < n; i++) {
    if (bucket[i].empty()) continue;
    u.clear();
    for (int v : bucket[i])
      if (!mark[v]) {
        mark[v] = 1;
        u.push_back(v);
      }
    for (int v : u) mark[v] = 0;
    if ((int)u.size() > best) {
      best = (int)u.size();
      if (widest) *widest = u;
    }
    std::vector<int> rest;
    for (int v : u)
      if (v != order[i]) rest.push_back(v);
    if (!rest.empty()) place(rest);
  }
  return best;
}

LightCone slice_cone(const LightCone &lc, int var, int slot) {
  LightCone out = lc;
  for (Gate &g : out.gates) {
    if (g.rank != 2 || (g.var[0] != var && g.var[1] != var)) continue;
    const int axis = g.var[0] == var ? 0 : 1;
    g.cut = (int8_t)axis;
    g.cut_slot = (int8_t)slot;
    g.var[0] = g.var[1 - axis];
    g.var[1] = -1;
    g.rank = 1;
  }
  return out;
}

std::vector<int> choose_slices(const LightCone &lc, int cap, int max_vars, int trials,
                               std::vector<int> *order_out, const PlanOptions *plan,
                               double bytes_weight) {
  std::vector<int> fixed;
  LightCone cur = lc;
  auto order_of = [&](const LightCone &c) {
    return trials > 1 ? search_order(c, std::min(trials, 8), plan, bytes_weight) : minfill_order(c);
  };
  std::vector<int> widest, best_order = order_of(cur);
  int w = order_width(cur, best_order, &widest);
  while (w > cap && (int)fixed.size() < max_vars) {
    // a variable can be fixed when every gate holding it has rank 2
    std::vector<char> ok(cur.n_vars, 1);
    for (const Gate &g : cur.gates)
      if (g.rank == 1) ok[g.var[0]] = 0;
    for (int v : fixed) ok[v] = 0;
    int best = -1, best_w = 0;
    double best_cost = 0;
    std::vector<int> best_widest, cand_order;
    for (int v : widest) {
      if (!ok[v]) continue;
      const LightCone t = slice_cone(cur, v, (int)fixed.size());
      const std::vector<int> o = order_of(t);
      std::vector<int> wv;
      const int tw = order_width(t, o, &wv);
      const double tc = order_cost(t, o);
      if (best < 0 || tw < best_w || (tw == best_w && tc < best_cost)) {
        best = v;
        best_w = tw;
        best_cost = tc;
        best_widest = wv;
        cand_order = o;
      }
    }
    if (best < 0) break;  // nothing in the widest bucket can be fixed
    cur = slice_cone(cur, best, (int)fixed.size());
    fixed.push_back(best);
    w = best_w;
    widest = best_widest;
    best_order = cand_order;
  }
  if (order_out) *order_out = best_order;
  return fixed;
}

std::vector<int> search_order(const LightCone &lc, int trials, const PlanOptions *plan,
                              double bytes_weight) {
  // the merged plan's flops + weighted bytes; an order the plan refuses
  // (over the width cap) costs more than any other
  auto cost = [&](const std::vector<int> &o) {
    if (!plan) return order_cost(lc, o);
    ConePlan pl;
    if (!plan_cone(lc, o, *plan, &pl).empty()) return HUGE_VAL;
    return pl.flops + bytes_weight * pl.bytes;
  };
  std::vector<int> best = minfill_order(lc, 0);
  double best_cost = cost(best);
  for (int t = 1; t < trials; t++) {
    std::vector<int> o = minfill_order(lc, 0x5EEDull * (uint64_t)t + (uint64_t)lc.edge);
    const double c = cost(o);
    if (c < best_cost) {
      best_cost = c;
      best.swap(o);
    }
  }
  return best;
}

void group_features(const Group &G, const ConePlan &pl, int precision, float *f) {
  int n_big = 0, max_rank = 0, n_small = 0, n_inter = 0, lv0 = 0;
  double elems = 0, rank_sum = 0;
  for (const Operand &o : G.ops) {
    const Tensor &t = pl.tensors[o.tensor];
    const int r = (int)t.vars.size();
    max_rank = std::max(max_rank, r);
    n_big += r >= 8;
    n_small += r <= 2;
    n_inter += t.gate < 0;
    lv0 += o.level == 0;
    elems += std::ldexp(1.0, r);
    rank_sum += r;
  }
  (void)precision;
  const int es = G.prec == 1 ? 8 : 16;
  double flops = 0;
  for (int l = 0; l < G.L; l++) {
    int factors = (l > 0 ? 1 : 0);
    for (const Operand &o : G.ops) factors += o.level == l;
    flops += std::ldexp(1.0, G.w - l) * 6.0 * std::max(0, factors - 1) +
             std::ldexp(1.0, G.w - l - 1) * 2.0;
  }
  f[0] = (float)G.w;
  f[1] = (float)G.L;
  f[2] = (float)(G.w - G.L);
  f[3] = (float)G.ops.size();
  f[4] = (float)n_big;
  f[5] = (float)max_rank;
  f[6] = (float)std::log2(elems);
  f[7] = (float)(G.w - max_rank);
  f[8] = (float)lv0;
  f[9] = (float)((int)G.ops.size() - lv0);
  f[10] = (float)std::log2(es * (elems + std::ldexp(1.0, G.w - G.L)));
  f[11] = (float)std::log2(std::max(1.0, flops));
  f[12] = (float)n_small;
  // matrix form: 1 + its n bits (the smaller side), 0 if the group has none
  GemmShape gs;
  f[13] = gemm_shape(G, pl, &gs) ? (float)(1 + gs.nbits.size()) : 0.0f;
  (void)rank_sum;
  f[14] = (float)n_inter;
  f[15] = (float)G.prec;
}

bool gemm_shape(const Group &G, const ConePlan &pl, GemmShape *gs) {
  const int n = (int)G.ops.size();
  if (n < 2 || n > 64 || G.w > 31) return false;
  const uint32_t summed = (1u << G.L) - 1u, all = (1u << G.w) - 1u, kept = all & ~summed;
  auto rank = [&](int k) { return (int)pl.tensors[G.ops[k].tensor].vars.size(); };
  // side A: the largest operand; side B: the operand with the most kept bits
  // side A lacks (ties: the larger one)
  int a = 0;
  for (int k = 1; k < n; k++)
    if (rank(k) > rank(a)) a = k;
  int b = -1, best = -1;
  for (int k = 0; k < n; k++) {
    if (k == a) continue;
    const int priv = __builtin_popcount(G.ops[k].mask & kept & ~G.ops[a].mask);
    if (priv > best || (priv == best && rank(k) > rank(b))) {
      best = priv;
      b = k;
    }
  }
  GemmShape s;
  s.a = a;
  s.b = b;
  s.role.assign(n, 0);
  s.role[b] = 1;
  uint32_t ma = G.ops[a].mask, mb = G.ops[b].mask;
  // the rest, largest first: into a side that holds all their bits (side A
  // first), else into the side that gains the fewest kept bits, so that the
  // kept bits private to each side (the m and n dimensions) stay many
  std::vector<int> rest;
  for (int k = 0; k < n; k++)
    if (k != a && k != b) rest.push_back(k);
  std::stable_sort(rest.begin(), rest.end(), [&](int x, int y) { return rank(x) > rank(y); });
  for (int k : rest) {
    const uint32_t mk = G.ops[k].mask;
    int side;
    if ((mk & ~ma) == 0) side = 0;
    else if ((mk & ~mb) == 0) side = 1;
    else side = __builtin_popcount(mk & kept & ~ma) <= __builtin_popcount(mk & kept & ~mb) ? 0 : 1;
    s.role[k] = (int8_t)side;
    (side == 0 ? ma : mb) |= mk;
  }
  for (int q = G.L; q < G.w; q++) {
    const bool in_a = (ma >> q) & 1u, in_b = (mb >> q) & 1u;
    if (in_a && in_b) s.bbits.push_back(q);
    else if (in_b) s.nbits.push_back(q);
    else s.mbits.push_back(q);
  }
  if (s.nbits.size() > s.mbits.size()) {
    // more private kept bits on side B: swap the sides
    std::swap(s.a, s.b);
    for (auto &r : s.role) r = (int8_t)(1 - r);
    s.mbits.swap(s.nbits);
  }
  // an operand with no m or n bit (only batch and summed bits) fits either
  // side: side B, whose factor has fewer entries (N <= M)
  uint32_t mn = 0;
  for (int q : s.mbits) mn |= 1u << q;
  for (int q : s.nbits) mn |= 1u << q;
  for (int k = 0; k < n; k++)
    if (k != s.a && k != s.b && (G.ops[k].mask & mn) == 0) s.role[k] = 1;
  // at least one full 16-wide block of the matrix cores each way
  if (s.nbits.size() < 4) return false;
  if (gs) *gs = s;
  return true;
}

int mask_runs(uint32_t mask, uint8_t *src, uint8_t *len, uint8_t *dst) {
  int nr = 0, d = 0;
  for (int b = 0; b < 32;) {
    if (!((mask >> b) & 1)) {
      b++;
      continue;
    }
    int s = b;
    while (b < 32 && ((mask >> b) & 1)) b++;
    src[nr] = (uint8_t)s;
    len[nr] = (uint8_t)(b - s);
    dst[nr] = (uint8_t)d;
    d += b - s;
    nr++;
  }
  return nr;
}

namespace {

struct BucketRec {
  int pos;
  std::vector<int> U;    // union, sorted by elimination position
  std::vector<int> ops;  // tensor ids in the order they entered the bucket
  int result = -1;       // tensor id, -1 for a scalar
  int target = -1;       // record index receiving the result
  int next = -1, prev = -1;  // merge chain links
};

// First-fit allocator over byte offsets.
struct Arena {
  std::vector<std::pair<int64_t, int64_t>> used;  // (offset, size), sorted
  int64_t peak = 0;
  int64_t alloc(int64_t size) {
    int64_t at = 0;
    size_t i = 0;
    for (; i < used.size(); i++) {
      if (used[i].first - at >= size) break;
      at = used[i].first + used[i].second;
    }
    used.insert(used.begin() + i, {at, size});
    peak = std::max(peak, at + size);
    return at;
  }
  void release(int64_t off) {
    for (size_t i = 0; i < used.size(); i++)
      if (used[i].first == off) {
        used.erase(used.begin() + i);
        return;
      }
  }
};

}  // namespace

std::string plan_cone(const LightCone &lc, const std::vector<int> &order,
                      const PlanOptions &opt, ConePlan *out) {
  const int n = lc.n_vars;
  if ((int)order.size() != n) return "order length differs from the variable count";
  std::vector<int> pos(n, -1);
  for (int i = 0; i < n; i++) {
    int v = order[i];
    if (v < 0 || v >= n || pos[v] >= 0) return "order is not a permutation of the variables";
    pos[v] = i;
  }
  ConePlan &P = *out;
  P = ConePlan();
  P.order = order;
  P.bucket_width.assign(n, 0);

  // initial tensors, indices sorted by elimination position
  for (size_t g = 0; g < lc.gates.size(); g++) {
    const Gate &gt = lc.gates[g];
    Tensor t;
    t.gate = (int)g;
    if (gt.rank == 1) {
      t.vars = {gt.var[0]};
    } else if (pos[gt.var[0]] < pos[gt.var[1]]) {
      t.vars = {gt.var[0], gt.var[1]};
      t.transposed = true;
    } else {
      t.vars = {gt.var[1], gt.var[0]};
    }
    P.tensors.push_back(t);
  }

  // symbolic bucket elimination (Sec. II-B)
  std::vector<std::vector<int>> bucket(n);
  for (size_t t = 0; t < P.tensors.size(); t++)
    bucket[pos[P.tensors[t].vars[0]]].push_back((int)t);
  std::vector<BucketRec> recs;
  std::vector<int> rec_at(n, -1);
  std::vector<char> mark(n, 0);
  for (int i = 0; i < n; i++) {
    if (bucket[i].empty()) continue;
    BucketRec r;
    r.pos = i;
    r.ops = bucket[i];
    std::vector<int> upos;
    for (int t : r.ops)
      for (int v : P.tensors[t].vars)
        if (!mark[v]) {
          mark[v] = 1;
          upos.push_back(pos[v]);
        }
    std::sort(upos.begin(), upos.end());
    for (int q : upos) {
      r.U.push_back(order[q]);
      mark[order[q]] = 0;
    }
    int w = (int)r.U.size();
    P.bucket_width[i] = w;
    P.max_width = std::max(P.max_width, w);
    P.n_buckets++;
    P.paper_flops += 8.0 * std::ldexp(1.0, w);
    if (w > opt.max_width)
      return "bucket width " + std::to_string(w) + " exceeds the cap " +
             std::to_string(opt.max_width);
    if (w > 1) {
      Tensor res;
      res.vars.assign(r.U.begin() + 1, r.U.end());
      r.result = (int)P.tensors.size();
      P.tensors.push_back(res);
      bucket[pos[res.vars[0]]].push_back(r.result);
    }
    rec_at[i] = (int)recs.size();
    recs.push_back(std::move(r));
  }
  for (auto &r : recs)
    if (r.result >= 0) r.target = rec_at[pos[P.tensors[r.result].vars[0]]];

  // merged indices (Sec. II-C): bucket r joins its target t when U_t is a
  // subset of U_r, i.e. |U_t| = |U_r| - 1; one predecessor per target.
  if (opt.max_levels > 1)
    for (size_t r = 0; r < recs.size(); r++) {
      int t = recs[r].target;
      if (t >= 0 && recs[t].prev < 0 && recs[t].U.size() + 1 == recs[r].U.size()) {
        recs[t].prev = (int)r;
        recs[r].next = t;
      }
    }

  // chains -> groups of at most max_levels summed indices
  for (size_t h = 0; h < recs.size(); h++) {
    if (recs[h].prev >= 0) continue;
    std::vector<int> chain;
    for (int r = (int)h; r >= 0; r = recs[r].next) chain.push_back(r);
    for (size_t s = 0; s < chain.size(); s += opt.max_levels) {
      size_t e = std::min(chain.size(), s + (size_t)opt.max_levels);
      Group G;
      const BucketRec &head = recs[chain[s]];
      G.w = (int)head.U.size();
      G.L = (int)(e - s);
      G.first_pos = head.pos;
      G.last_pos = recs[chain[e - 1]].pos;
      std::vector<int> bit(n, -1);
      for (int q = 0; q < G.w; q++) bit[head.U[q]] = q;
      for (size_t c = s; c < e; c++) {
        const BucketRec &r = recs[chain[c]];
        int internal = (c > s) ? recs[chain[c - 1]].result : -1;
        for (int t : r.ops) {
          if (t == internal) continue;
          uint32_t m = 0;
          for (int v : P.tensors[t].vars) m |= 1u << bit[v];
          G.ops.push_back({t, m, (int)(c - s)});
        }
      }
      G.out_tensor = recs[chain[e - 1]].result;
      G.small = G.w <= opt.small_width;
      P.groups.push_back(std::move(G));
    }
  }
  std::stable_sort(P.groups.begin(), P.groups.end(),
                   [](const Group &a, const Group &b) { return a.last_pos < b.last_pos; });

  // precision per group: in mixed mode wide groups run in complex64, narrow
  // ones and every final scalar sum-out in complex128
  for (Group &G : P.groups) {
    if (opt.precision == 2)
      G.prec = (G.w >= opt.mixed_width && G.out_tensor >= 0) ? 1 : 0;
    else
      G.prec = (int8_t)opt.precision;
    if (G.out_tensor >= 0) P.tensors[G.out_tensor].prec = G.prec;
  }
  auto es = [](int prec) { return prec == 0 ? 16.0 : 8.0; };

  // producers, consumers, scalar slots, cost counts
  for (size_t g = 0; g < P.groups.size(); g++) {
    Group &G = P.groups[g];
    if (G.out_tensor >= 0)
      P.tensors[G.out_tensor].producer = (int)g;
    else
      G.scalar_slot = P.n_scalars++;
    double in_bytes = 0;
    std::vector<int> per_level(G.L, 0);
    for (const Operand &o : G.ops) {
      per_level[o.level]++;
      const Tensor &t = P.tensors[o.tensor];
      if (t.gate < 0) P.tensors[o.tensor].consumer = (int)g;
      in_bytes += std::ldexp(1.0, (int)t.vars.size()) * es(t.gate < 0 ? t.prec : G.prec);
    }
    P.bytes += in_bytes + es(G.prec) * std::ldexp(1.0, G.w - G.L);
    for (int l = 0; l < G.L; l++) {
      int factors = per_level[l] + (l > 0 ? 1 : 0);
      P.flops += std::ldexp(1.0, G.w - l) * 6.0 * std::max(0, factors - 1) +
                 std::ldexp(1.0, G.w - l - 1) * 2.0;
    }
  }

  // memory plan (bytes, 256-aligned): outputs are placed before the group's
  // inputs are released
  Arena A;
  for (size_t g = 0; g < P.groups.size(); g++) {
    Group &G = P.groups[g];
    if (G.out_tensor >= 0) {
      int64_t sz = ((int64_t)1 << (G.w - G.L)) * (int64_t)es(G.prec);
      sz = (sz + 255) / 256 * 256;
      P.tensors[G.out_tensor].offset = A.alloc(sz);
    }
    for (const Operand &o : G.ops)
      if (P.tensors[o.tensor].gate < 0) A.release(P.tensors[o.tensor].offset);
  }
  P.arena_bytes = A.peak;
  return "";
}

}  // namespace qtn
