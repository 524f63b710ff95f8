// CPU oracle for the exact global minimum cut.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  The GPU product path
// never calls it, and it shares no code, header or table with the GPU path.
//
// Three independent routes to the same number, written plainly and slowly:
//   O1  mco_bruteforce       - the definition itself (Preliminaries, "Basic
//                              Concepts": capacity c(A) of a cut and
//                              lambda(G) = min over non-empty proper A).
//   O2  mco_stoer_wagner     - the Stoer-Wagner phases (Related Work; a
//                              simpler variant of the NOI algorithm).
//   O3  mco_noi              - sequential Nagamochi-Ono-Ibaraki: repeated
//                              CAPFOREST (appendix Algorithm 3, section
//                              "Nagamochi, Ono and Ibaraki's Algorithm") with
//                              an uncapped max-heap, the plain contraction rule
//                              q(e) >= lambda-hat, and graph contraction
//                              (Preliminaries, contraction G/(u,v)).
// Helpers: mco_cut_value (c(A) by definition) and mco_pair_connectivity
// (lambda(G,s,t) for all pairs by enumeration).
// Upper bound: mco_viecut (the VieCut-style bound of Algorithm 2's first
// step) and its label-propagation step mco_lp_sweep.
// Local tests: mco_pr_tests - the Padberg-Rinaldi tests of one edge (section
// "Exact Minimum Cut Algorithms", the heuristics of Padberg and Rinaldi; the
// paper names them without restating them, so each is written from the cut
// argument that makes it sound).
// Approximation: mco_matula - Matula's (2+eps)-approximation as the paper
// describes it (section "Nagamochi, Ono and Ibaraki's Algorithm" and
// "Bounded Priority Queues"): NOI whose contraction bound is (1/2 - eps)
// times the minimum degree rather than the best cut found.
//
// All arithmetic is exact 64-bit integer.  Inputs are a symmetric CSR
// (row_ptr int64[n+1], col int32[nnz], w int32[nnz]); self-loops are ignored
// (they never cross a cut) and parallel entries count with their total
// weight.  Every function returns 0 on success, a negative code otherwise.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <queue>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

using i64 = int64_t;

struct Csr {
  int32_t n;
  const i64* rp;
  const int32_t* col;
  const int32_t* w;
};

// c(A) = sum of weights of edges with one end in A and one outside
// (Preliminaries, "Basic Concepts").  Each undirected edge appears twice in
// the symmetric CSR, so the entry sum is halved.
i64 cut_value(const Csr& g, const uint8_t* side) {
  i64 s = 0;
  for (int32_t u = 0; u < g.n; ++u)
    for (i64 e = g.rp[u]; e < g.rp[u + 1]; ++e)
      if ((side[u] != 0) != (side[g.col[e]] != 0)) s += g.w[e];
  return s / 2;
}

bool connected_from0(const Csr& g, std::vector<uint8_t>& reach) {
  reach.assign(g.n, 0);
  std::vector<int32_t> st{0};
  reach[0] = 1;
  int32_t cnt = 1;
  while (!st.empty()) {
    int32_t u = st.back();
    st.pop_back();
    for (i64 e = g.rp[u]; e < g.rp[u + 1]; ++e) {
      int32_t v = g.col[e];
      if (!reach[v]) { reach[v] = 1; ++cnt; st.push_back(v); }
    }
  }
  return cnt == g.n;
}

// --------------------------------------------------------------------------
// O1: enumerate every side A that excludes vertex 0, in Gray-code order, and
// update c(A) by the change of one vertex's side.
int bruteforce(const Csr& g, i64* lambda, uint8_t* side_out, i64* conn) {
  const int32_t n = g.n;
  if (n < 2) return -2;
  if (n > 26) return -1;
  std::vector<uint8_t> in(n, 0), best(n, 0);
  i64 cut = 0, bestv = INT64_MAX;
  const uint64_t total = 1ULL << (n - 1);
  if (conn)
    for (int32_t i = 0; i < n * n; ++i) conn[i] = (i / n == i % n) ? 0 : INT64_MAX;
  for (uint64_t i = 1; i < total; ++i) {
    int32_t v = __builtin_ctzll(i) + 1;  // the vertex whose side flips
    for (i64 e = g.rp[v]; e < g.rp[v + 1]; ++e) {
      int32_t u = g.col[e];
      if (u == v) continue;
      cut += (in[u] == in[v]) ? g.w[e] : -(i64)g.w[e];
    }
    in[v] ^= 1;
    if (cut < bestv) { bestv = cut; best = in; }
    if (conn) {
      for (int32_t s = 0; s < n; ++s) {
        if (!in[s]) continue;
        for (int32_t t = 0; t < n; ++t) {
          if (in[t]) continue;
          i64& a = conn[(i64)s * n + t];
          i64& b = conn[(i64)t * n + s];
          if (cut < a) a = cut;
          if (cut < b) b = cut;
        }
      }
    }
  }
  *lambda = bestv;
  if (side_out) std::memcpy(side_out, best.data(), n);
  return 0;
}

// --------------------------------------------------------------------------
// O2: Stoer-Wagner.  Each phase grows a maximum-adjacency order from one
// vertex; the weight of the last vertex t to all others is the cut of the
// phase (t alone versus the rest); t is then merged into the second-last.
int stoer_wagner(const Csr& g, i64* lambda, uint8_t* side_out) {
  const int32_t n = g.n;
  if (n < 2) return -2;
  std::vector<uint8_t> reach;
  if (!connected_from0(g, reach)) {
    *lambda = 0;
    if (side_out)
      for (int32_t v = 0; v < n; ++v) side_out[v] = reach[v] ? 0 : 1;
    return 0;
  }
  std::vector<std::unordered_map<int32_t, i64>> adj(n);
  for (int32_t u = 0; u < n; ++u)
    for (i64 e = g.rp[u]; e < g.rp[u + 1]; ++e)
      if (g.col[e] != u) adj[u][g.col[e]] += g.w[e];
  std::vector<std::vector<int32_t>> members(n);
  for (int32_t v = 0; v < n; ++v) members[v] = {v};
  std::vector<uint8_t> alive(n, 1);
  std::vector<i64> key(n, 0);
  std::vector<uint8_t> added(n, 0);
  i64 best = INT64_MAX;
  std::vector<int32_t> best_side;
  int32_t alive_cnt = n;
  int32_t first = 0;
  while (alive_cnt > 1) {
    while (!alive[first]) ++first;
    for (int32_t v = 0; v < n; ++v) { key[v] = 0; added[v] = 0; }
    std::priority_queue<std::pair<i64, int32_t>> pq;
    pq.push({0, first});
    int32_t prev = -1, last = -1;
    i64 last_key = 0;
    int32_t cnt = 0;
    while (!pq.empty()) {
      auto [k, v] = pq.top();
      pq.pop();
      if (added[v] || k != key[v]) continue;
      added[v] = 1;
      prev = last;
      last = v;
      last_key = k;
      ++cnt;
      for (auto& [u, c] : adj[v])
        if (!added[u]) { key[u] += c; pq.push({key[u], u}); }
    }
    if (cnt != alive_cnt) return -3;  // cannot happen on a connected graph
    if (last_key < best) { best = last_key; best_side = members[last]; }
    // merge last into prev
    for (auto& [u, c] : adj[last]) {
      if (u == prev) continue;
      adj[prev][u] += c;
      adj[u][prev] += c;
      adj[u].erase(last);
    }
    adj[prev].erase(last);
    adj[last].clear();
    members[prev].insert(members[prev].end(), members[last].begin(), members[last].end());
    members[last].clear();
    alive[last] = 0;
    --alive_cnt;
  }
  *lambda = best;
  if (side_out) {
    std::memset(side_out, 0, n);
    for (int32_t v : best_side) side_out[v] = 1;
  }
  return 0;
}

// --------------------------------------------------------------------------
// O3: sequential NOI.
struct WGraph {  // CSR of the current (contracted) graph, no self-loops
  int32_t n = 0;
  std::vector<i64> rp;
  std::vector<int32_t> col;
  std::vector<i64> w;
  std::vector<i64> deg;  // weighted degree
};

uint64_t splitmix(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

int32_t uf_find(std::vector<int32_t>& p, int32_t x) {
  while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
  return x;
}

void uf_union(std::vector<int32_t>& p, int32_t a, int32_t b) {
  a = uf_find(p, a);
  b = uf_find(p, b);
  if (a != b) p[std::max(a, b)] = std::min(a, b);
}

// Contract every block into one vertex, given each vertex's block id in
// [0, nn): parallel edges summed, internal edges dropped (Preliminaries,
// contraction G/(u,v)).
WGraph contract_blocks(const WGraph& g, const std::vector<int32_t>& lab, int32_t nn) {
  std::vector<std::pair<uint64_t, i64>> kv;
  kv.reserve(g.col.size());
  for (int32_t u = 0; u < g.n; ++u)
    for (i64 e = g.rp[u]; e < g.rp[u + 1]; ++e) {
      int32_t a = lab[u], b = lab[g.col[e]];
      if (a != b) kv.push_back({((uint64_t)a << 32) | (uint32_t)b, g.w[e]});
    }
  std::sort(kv.begin(), kv.end());
  WGraph h;
  h.n = nn;
  h.rp.assign(nn + 1, 0);
  h.deg.assign(nn, 0);
  for (size_t i = 0; i < kv.size();) {
    size_t j = i;
    i64 s = 0;
    while (j < kv.size() && kv[j].first == kv[i].first) { s += kv[j].second; ++j; }
    int32_t a = (int32_t)(kv[i].first >> 32);
    h.col.push_back((int32_t)(uint32_t)kv[i].first);
    h.w.push_back(s);
    h.rp[a + 1]++;
    h.deg[a] += s;
    i = j;
  }
  for (int32_t v = 0; v < nn; ++v) h.rp[v + 1] += h.rp[v];
  return h;
}

// Contract every union-find block: block ids numbered by smallest member
// ("Parallel Graph Contraction" for the block-id scheme).
WGraph contract(const WGraph& g, std::vector<int32_t>& p, std::vector<int32_t>& lab) {
  lab.assign(g.n, -1);
  int32_t nn = 0;
  for (int32_t v = 0; v < g.n; ++v) {
    int32_t r = uf_find(p, v);
    if (lab[r] < 0) lab[r] = nn++;
    lab[v] = lab[r];
  }
  return contract_blocks(g, lab, nn);
}

WGraph from_input(const Csr& in) {  // G without self-loops
  WGraph g;
  g.n = in.n;
  g.rp.assign(in.n + 1, 0);
  g.deg.assign(in.n, 0);
  for (int32_t u = 0; u < in.n; ++u)
    for (i64 e = in.rp[u]; e < in.rp[u + 1]; ++e)
      if (in.col[e] != u) {
        g.col.push_back(in.col[e]);
        g.w.push_back(in.w[e]);
        g.rp[u + 1]++;
        g.deg[u] += in.w[e];
      }
  for (int32_t v = 0; v < in.n; ++v) g.rp[v + 1] += g.rp[v];
  return g;
}

// eps_ppm < 0: the exact algorithm (O3).  eps_ppm >= 0: Matula's
// approximation with eps = eps_ppm / 10^6 < 1/2: a round contracts the edges
// with q(e) >= k = min(lambda-hat, max(1, ceil((1/2 - eps) * delta))), delta
// the current graph's minimum degree; lambda-hat stays the smallest real cut
// seen (degrees, prefix cuts), so the answer is a cut of G.
int noi(const Csr& in, uint64_t seed, i64* lambda, uint8_t* side_out, int32_t* rounds_out,
        i64 eps_ppm = -1) {
  const int32_t n0 = in.n;
  if (n0 < 2) return -2;
  std::vector<uint8_t> reach;
  if (!connected_from0(in, reach)) {
    *lambda = 0;
    if (side_out)
      for (int32_t v = 0; v < n0; ++v) side_out[v] = reach[v] ? 0 : 1;
    if (rounds_out) *rounds_out = 0;
    return 0;
  }
  // G_C = G without self-loops (parallel entries stay separate until the
  // first contraction merges them).
  WGraph g = from_input(in);

  std::vector<int32_t> map(n0);  // original vertex -> current vertex
  for (int32_t v = 0; v < n0; ++v) map[v] = v;
  std::vector<uint8_t> side(n0, 0);

  // trivial cut: lambda-hat = minimum weighted degree delta(G)
  auto take_min_degree = [&](i64& lhat) {
    int32_t arg = 0;
    for (int32_t v = 1; v < g.n; ++v)
      if (g.deg[v] < g.deg[arg]) arg = v;
    if (g.deg[arg] < lhat) {
      lhat = g.deg[arg];
      for (int32_t v = 0; v < n0; ++v) side[v] = (map[v] == arg) ? 1 : 0;
    }
  };
  i64 lhat = INT64_MAX;
  take_min_degree(lhat);

  int32_t rounds = 0;
  while (g.n > 2 && lhat > 0) {
    ++rounds;
    i64 lsnap = lhat;  // bound used by the contraction rule this round
    if (eps_ppm >= 0) {
      i64 delta = g.deg[0];
      for (int32_t v = 1; v < g.n; ++v) delta = std::min(delta, g.deg[v]);
      // q(e) >= (1/2 - eps) delta for an integer q(e) means q(e) >= the
      // ceiling of that product
      const i64 k = (delta * (1000000 - 2 * eps_ppm) + 1999999) / 2000000;
      lsnap = std::min(lhat, std::max<i64>(1, k));
    }
    std::vector<i64> r(g.n, 0);
    std::vector<uint8_t> visited(g.n, 0);
    std::vector<int32_t> order;
    order.reserve(g.n);
    std::vector<int32_t> p(g.n);
    for (int32_t v = 0; v < g.n; ++v) p[v] = v;
    std::priority_queue<std::pair<i64, int32_t>> pq;
    int32_t start = (int32_t)(splitmix(seed + (uint64_t)rounds) % (uint64_t)g.n);
    pq.push({0, start});
    i64 alpha = 0;  // c(S) for S = vertices scanned so far; c(empty) = 0
    while (!pq.empty()) {
      auto [k, x] = pq.top();
      pq.pop();
      if (visited[x] || k != r[x]) continue;
      visited[x] = 1;
      order.push_back(x);
      alpha += g.deg[x] - 2 * r[x];
      if ((int32_t)order.size() < g.n && alpha < lhat) {
        lhat = alpha;
        std::vector<uint8_t> inS(g.n, 0);
        for (int32_t s : order) inS[s] = 1;
        for (int32_t v = 0; v < n0; ++v) side[v] = inS[map[v]];
      }
      for (i64 e = g.rp[x]; e < g.rp[x + 1]; ++e) {
        int32_t y = g.col[e];
        if (visited[y]) continue;
        r[y] += g.w[e];
        if (r[y] >= lsnap) uf_union(p, x, y);  // q(e) = r(y) >= lambda-hat
        pq.push({r[y], y});
      }
    }
    std::vector<int32_t> lab;
    WGraph h = contract(g, p, lab);
    for (int32_t v = 0; v < n0; ++v) map[v] = lab[map[v]];
    g = std::move(h);
    if (g.n >= 2) take_min_degree(lhat);
  }
  *lambda = lhat;
  if (side_out) std::memcpy(side_out, side.data(), n0);
  if (rounds_out) *rounds_out = rounds;
  return 0;
}

// --------------------------------------------------------------------------
// VieCut-style upper bound (section "Inexact Shared-Memory Minimum Cuts" and
// Algorithm 2's first step: an inexact solver clusters the graph by label
// propagation, contracts the clusters and applies the Padberg-Rinaldi tests;
// the paper does not restate the details, so they are read as follows).
//
// One synchronous label-propagation sweep: every vertex takes, among its
// neighbours' current labels, the one with the largest total edge weight,
// ties to the smallest label; a vertex without neighbours keeps its label.
void lp_sweep(const WGraph& g, const std::vector<int32_t>& cur, std::vector<int32_t>& nxt) {
  std::vector<std::pair<int32_t, i64>> acc;
  for (int32_t v = 0; v < g.n; ++v) {
    acc.clear();
    for (i64 e = g.rp[v]; e < g.rp[v + 1]; ++e) acc.push_back({cur[g.col[e]], g.w[e]});
    if (acc.empty()) {
      nxt[v] = cur[v];
      continue;
    }
    std::sort(acc.begin(), acc.end());
    int32_t best = acc[0].first;
    i64 best_sum = -1;
    for (size_t i = 0; i < acc.size();) {
      size_t j = i;
      i64 sum = 0;
      while (j < acc.size() && acc[j].first == acc[i].first) sum += acc[j++].second;
      if (sum > best_sum) {  // labels ascend, so the first maximum is the smallest label
        best_sum = sum;
        best = acc[i].first;
      }
      i = j;
    }
    nxt[v] = best;
  }
}

// Levels: `sweeps` label-propagation sweeps from distinct labels; contract
// the label classes (blocks numbered by label value); bound by the minimum
// degree; PR1 (w >= lambda-hat) and PR2 (2w > c(u) or 2w > c(v), strict) on
// that graph with the current bound, contract their components (blocks
// numbered by smallest member) unless the graph is already down to stop_n
// vertices; bound again.  Repeat while the graph has more than stop_n
// vertices, the bound is above 0, fewer than max_levels levels ran and the
// last level removed at least a tenth of the vertices.  Every vertex of a
// contracted graph is a vertex set of G, so every bound is a real cut value.
// exact_finish: the last level graph is solved exactly (O3), as the
// clustering algorithm finishes in the paper's description of it, and its
// minimum cut (a cut of G) lowers the bound.
int viecut(const Csr& in, int32_t sweeps, int32_t stop_n, int32_t max_levels, i64* lambda,
           uint8_t* side_out, int32_t* levels_out, int32_t exact_finish = 0) {
  const int32_t n0 = in.n;
  if (n0 < 2) return -2;
  WGraph g = from_input(in);
  std::vector<int32_t> map(n0);
  for (int32_t v = 0; v < n0; ++v) map[v] = v;
  std::vector<uint8_t> side(n0, 0);
  i64 lhat = INT64_MAX;
  auto bound = [&]() {  // minimum degree of the current graph, smallest vertex on ties
    if (g.n < 2) return;
    int32_t arg = 0;
    for (int32_t v = 1; v < g.n; ++v)
      if (g.deg[v] < g.deg[arg]) arg = v;
    if (g.deg[arg] < lhat) {
      lhat = g.deg[arg];
      for (int32_t v = 0; v < n0; ++v) side[v] = (map[v] == arg) ? 1 : 0;
    }
  };
  bound();
  int32_t levels = 0;
  while (g.n > stop_n && levels < max_levels && lhat > 0) {
    ++levels;
    const int32_t n_before = g.n;
    std::vector<int32_t> label(g.n), nxt(g.n);
    for (int32_t v = 0; v < g.n; ++v) label[v] = v;
    for (int32_t k = 0; k < sweeps; ++k) {
      lp_sweep(g, label, nxt);
      label.swap(nxt);
    }
    // label classes, numbered by label value
    std::vector<uint8_t> used(g.n, 0);
    for (int32_t v = 0; v < g.n; ++v) used[label[v]] = 1;
    std::vector<int32_t> rank(g.n, -1), lab(g.n);
    int32_t nn = 0;
    for (int32_t l = 0; l < g.n; ++l)
      if (used[l]) rank[l] = nn++;
    for (int32_t v = 0; v < g.n; ++v) lab[v] = rank[label[v]];
    g = contract_blocks(g, lab, nn);
    for (int32_t v = 0; v < n0; ++v) map[v] = lab[map[v]];
    bound();
    if (g.n > stop_n && lhat > 0) {
      std::vector<int32_t> p(g.n);
      for (int32_t v = 0; v < g.n; ++v) p[v] = v;
      for (int32_t u = 0; u < g.n; ++u)
        for (i64 e = g.rp[u]; e < g.rp[u + 1]; ++e) {
          const int32_t v = g.col[e];
          const i64 c = g.w[e];
          if (u < v && (c >= lhat || 2 * c > g.deg[u] || 2 * c > g.deg[v])) uf_union(p, u, v);
        }
      std::vector<int32_t> lab2;
      g = contract(g, p, lab2);
      for (int32_t v = 0; v < n0; ++v) map[v] = lab2[map[v]];
      bound();
    }
    if ((int64_t)g.n * 10 > (int64_t)n_before * 9) break;  // shrank by less than a tenth
  }
  if (exact_finish && g.n > 2 && lhat > 0) {
    std::vector<int32_t> w32(g.w.size());
    for (size_t i = 0; i < g.w.size(); ++i) w32[i] = (int32_t)g.w[i];
    i64 lg = 0;
    std::vector<uint8_t> sg(g.n);
    int rc = noi(Csr{g.n, g.rp.data(), g.col.data(), w32.data()}, 1, &lg, sg.data(), nullptr);
    if (rc) return rc;
    if (lg < lhat) {
      lhat = lg;
      for (int32_t v = 0; v < n0; ++v) side[v] = sg[map[v]];
    }
  }
  *lambda = lhat;
  if (side_out) std::memcpy(side_out, side.data(), n0);
  if (levels_out) *levels_out = levels;
  return 0;
}

// Padberg-Rinaldi tests of every entry e = (u, v) with u < v, as bits of
// flags[e] (0 for every other entry):
//   bit 0  PR1: c(e) >= lhat;
//   bit 1  PR2: 2 c(e) > c(u) or 2 c(e) > c(v)  (c(x): weighted degree
//          without self-loops);
//   bit 2  PR3: a common neighbour w (w != u, v) with c(u) < 2 (c(e) + c(u,w))
//          and c(v) < 2 (c(e) + c(v,w));
//   bit 3  PR4: c(e) + sum over common neighbours w of min(c(u,w), c(v,w))
//          >= lhat.
// Strict PR2 and PR3 hold for every non-trivial minimum cut at once (a cut
// that separates u and v with more than v, say, on v's side becomes strictly
// smaller when v crosses over), and PR1 and PR4 bound lambda(u, v) from below,
// so all passing edges can be contracted together while the trivial cuts
// and lambda-hat are kept.
// c(e) is the entry's weight.  PR3 and PR4 are evaluated only where both rows
// list their neighbours in strictly increasing order (so c(u,w) is one entry)
// and hold at most max_deg entries each; elsewhere their bits are 0.
int pr_tests(const Csr& g, i64 lhat, int32_t max_deg, uint8_t* flags) {
  std::vector<i64> deg(g.n, 0);
  for (int32_t u = 0; u < g.n; ++u)
    for (i64 e = g.rp[u]; e < g.rp[u + 1]; ++e)
      if (g.col[e] != u) deg[u] += g.w[e];
  auto increasing = [&](int32_t x) {
    for (i64 e = g.rp[x] + 1; e < g.rp[x + 1]; ++e)
      if (g.col[e] <= g.col[e - 1]) return false;
    return true;
  };
  for (int32_t u = 0; u < g.n; ++u)
    for (i64 e = g.rp[u]; e < g.rp[u + 1]; ++e) {
      flags[e] = 0;
      const int32_t v = g.col[e];
      if (u >= v) continue;
      const i64 c = g.w[e];
      uint8_t f = 0;
      if (c >= lhat) f |= 1;
      if (2 * c > deg[u] || 2 * c > deg[v]) f |= 2;
      const i64 du = g.rp[u + 1] - g.rp[u], dv = g.rp[v + 1] - g.rp[v];
      if (du <= max_deg && dv <= max_deg && increasing(u) && increasing(v)) {
        // the common neighbours, by looking each of u's up in v's row
        bool pr3 = false;
        i64 paths = c;  // the edge, then one two-edge path per common neighbour
        for (i64 a = g.rp[u]; a < g.rp[u + 1]; ++a) {
          const int32_t x = g.col[a];
          if (x == u || x == v) continue;
          for (i64 b = g.rp[v]; b < g.rp[v + 1]; ++b)
            if (g.col[b] == x) {
              const i64 cu = g.w[a], cv = g.w[b];
              paths += std::min(cu, cv);
              if (deg[u] < 2 * (c + cu) && deg[v] < 2 * (c + cv)) pr3 = true;
            }
        }
        if (pr3) f |= 4;
        if (paths >= lhat) f |= 8;
      }
      flags[e] = f;
    }
  return 0;
}

}  // namespace

extern "C" {

int mco_pr_tests(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w, int64_t lhat,
                 int32_t max_deg, uint8_t* flags) {
  if (n < 0 || !rp || !flags) return -1;
  return pr_tests(Csr{n, rp, col, w}, lhat, max_deg, flags);
}

int mco_cut_value(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                  const uint8_t* side, int64_t* value) {
  if (n < 0 || !rp || !side || !value) return -1;
  *value = cut_value(Csr{n, rp, col, w}, side);
  return 0;
}

int mco_bruteforce(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                   int64_t* lambda, uint8_t* side) {
  return bruteforce(Csr{n, rp, col, w}, lambda, side, nullptr);
}

// conn: n*n row-major; conn[s*n+t] = lambda(G, s, t), 0 on the diagonal.
int mco_pair_connectivity(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                          int64_t* conn) {
  int64_t lam;
  if (n > 20) return -1;
  return bruteforce(Csr{n, rp, col, w}, &lam, nullptr, conn);
}

int mco_stoer_wagner(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                     int64_t* lambda, uint8_t* side) {
  return stoer_wagner(Csr{n, rp, col, w}, lambda, side);
}

int mco_noi(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w, uint64_t seed,
            int64_t* lambda, uint8_t* side, int32_t* rounds) {
  return noi(Csr{n, rp, col, w}, seed, lambda, side, rounds);
}

int mco_matula(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w, uint64_t seed,
               int64_t eps_ppm, int64_t* lambda, uint8_t* side, int32_t* rounds) {
  if (eps_ppm < 0 || eps_ppm >= 500000) return -1;
  return noi(Csr{n, rp, col, w}, seed, lambda, side, rounds, eps_ppm);
}


// One label-propagation sweep over the graph as given (self-loops ignored).
int mco_lp_sweep(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w,
                 const int32_t* labels_in, int32_t* labels_out) {
  if (n < 0) return -1;
  WGraph g = from_input(Csr{n, rp, col, w});
  std::vector<int32_t> cur(labels_in, labels_in + n), nxt(n);
  lp_sweep(g, cur, nxt);
  std::memcpy(labels_out, nxt.data(), sizeof(int32_t) * n);
  return 0;
}

int mco_viecut(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w, int32_t sweeps,
               int32_t stop_n, int32_t max_levels, int32_t exact_finish, int64_t* lambda, uint8_t* side,
               int32_t* levels) {
  return viecut(Csr{n, rp, col, w}, sweeps, stop_n, max_levels, lambda, side, levels, exact_finish);
}

}  // extern "C"
