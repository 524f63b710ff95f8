// Seeded synthetic graph generators for the min-cut workloads.
//
// This module only builds inputs: random graphs, duplicate merging, k-core
// peeling, largest-component extraction, a seeded vertex permutation and
// the symmetric CSR layout.  It contains none of the min-cut method's
// arithmetic and is shared by the CPU oracle tests and the GPU path.
//
// Every random draw comes from a counter-based generator (SplitMix64 applied
// to seed, stream and counter), so results do not depend on thread count or
// scheduling.  Instance preparation follows the paper's appendix (k-core,
// then the largest connected component).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <parallel/algorithm>
#include <vector>

namespace {

inline uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

struct Rng {
  uint64_t base;
  Rng(uint64_t seed, uint64_t stream) : base(mix64(seed ^ mix64(stream + 0x51ULL))) {}
  uint64_t at(uint64_t i) const { return mix64(base + i * 0x9e3779b97f4a7c15ULL); }
  // uniform integer in [0, range)
  uint64_t below(uint64_t i, uint64_t range) const {
    return (uint64_t)(((__uint128_t)at(i) * range) >> 64);
  }
  // uniform double in [0, 1)
  double unit(uint64_t i) const { return (double)(at(i) >> 11) * 0x1.0p-53; }
};

struct EdgeList {
  std::vector<uint64_t> key;  // (u << 32) | v with u < v
  std::vector<int32_t> w;
};

inline uint64_t ekey(uint32_t u, uint32_t v) {
  if (u > v) std::swap(u, v);
  return ((uint64_t)u << 32) | v;
}

// Sort keys and merge duplicates.  mode 0: weights add up; mode 1: keep 1.
void merge_duplicates(EdgeList& e, int mode) {
  const size_t m = e.key.size();
  std::vector<size_t> idx;
  bool have_w = !e.w.empty();
  if (!have_w) {
    __gnu_parallel::sort(e.key.begin(), e.key.end());
    std::vector<uint64_t> k2;
    std::vector<int32_t> w2;
    k2.reserve(m);
    w2.reserve(m);
    for (size_t i = 0; i < m;) {
      size_t j = i;
      while (j < m && e.key[j] == e.key[i]) ++j;
      k2.push_back(e.key[i]);
      w2.push_back(mode == 0 ? (int32_t)(j - i) : 1);
      i = j;
    }
    e.key.swap(k2);
    e.w.swap(w2);
    return;
  }
  std::vector<std::pair<uint64_t, int32_t>> kv(m);
  for (size_t i = 0; i < m; ++i) kv[i] = {e.key[i], e.w[i]};
  __gnu_parallel::sort(kv.begin(), kv.end());
  std::vector<uint64_t> k2;
  std::vector<int32_t> w2;
  for (size_t i = 0; i < m;) {
    size_t j = i;
    int64_t s = 0;
    while (j < m && kv[j].first == kv[i].first) { s += kv[j].second; ++j; }
    k2.push_back(kv[i].first);
    w2.push_back(mode == 0 ? (int32_t)s : 1);
    i = j;
  }
  e.key.swap(k2);
  e.w.swap(w2);
}

void drop_self_loops(EdgeList& e) {
  size_t o = 0;
  bool hw = !e.w.empty();
  for (size_t i = 0; i < e.key.size(); ++i) {
    if ((uint32_t)(e.key[i] >> 32) == (uint32_t)e.key[i]) continue;
    e.key[o] = e.key[i];
    if (hw) e.w[o] = e.w[i];
    ++o;
  }
  e.key.resize(o);
  if (hw) e.w.resize(o);
}

// Keep edges whose endpoints both survive; relabel survivors densely in
// increasing id order.  Returns the new vertex count.
int64_t induce(EdgeList& e, const std::vector<char>& keep, int64_t n) {
  std::vector<int64_t> nid(n, -1);
  int64_t c = 0;
  for (int64_t v = 0; v < n; ++v)
    if (keep[v]) nid[v] = c++;
  size_t o = 0;
  for (size_t i = 0; i < e.key.size(); ++i) {
    uint32_t u = (uint32_t)(e.key[i] >> 32), v = (uint32_t)e.key[i];
    if (!keep[u] || !keep[v]) continue;
    e.key[o] = ekey((uint32_t)nid[u], (uint32_t)nid[v]);
    e.w[o] = e.w[i];
    ++o;
  }
  e.key.resize(o);
  e.w.resize(o);
  return c;
}

// k-core on the count of distinct neighbours (edges are already merged).
int64_t kcore(EdgeList& e, int64_t n, int k) {
  std::vector<int64_t> deg(n, 0);
  for (uint64_t kk : e.key) { deg[kk >> 32]++; deg[(uint32_t)kk]++; }
  std::vector<int64_t> off(n + 1, 0);
  for (int64_t v = 0; v < n; ++v) off[v + 1] = off[v] + deg[v];
  std::vector<uint32_t> adj(off[n]);
  std::vector<int64_t> pos(off.begin(), off.end() - 1);
  for (uint64_t kk : e.key) {
    uint32_t u = kk >> 32, v = (uint32_t)kk;
    adj[pos[u]++] = v;
    adj[pos[v]++] = u;
  }
  std::vector<char> alive(n, 1);
  std::vector<uint32_t> stack;
  for (int64_t v = 0; v < n; ++v)
    if (deg[v] < k) { alive[v] = 0; stack.push_back((uint32_t)v); }
  while (!stack.empty()) {
    uint32_t v = stack.back();
    stack.pop_back();
    for (int64_t i = off[v]; i < off[v + 1]; ++i) {
      uint32_t u = adj[i];
      if (alive[u] && --deg[u] < k) { alive[u] = 0; stack.push_back(u); }
    }
  }
  return induce(e, alive, n);
}

uint32_t uf_find(std::vector<uint32_t>& p, uint32_t x) {
  while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
  return x;
}

// Number of connected components (vertices with no edge count as their own).
int64_t components(const EdgeList& e, int64_t n, std::vector<uint32_t>& root) {
  root.resize(n);
  std::iota(root.begin(), root.end(), 0u);
  for (uint64_t kk : e.key) {
    uint32_t a = uf_find(root, kk >> 32), b = uf_find(root, (uint32_t)kk);
    if (a != b) root[std::max(a, b)] = std::min(a, b);
  }
  int64_t c = 0;
  for (int64_t v = 0; v < n; ++v) {
    root[v] = uf_find(root, (uint32_t)v);
    if (root[v] == (uint32_t)v) ++c;
  }
  return c;
}

int64_t largest_component(EdgeList& e, int64_t n) {
  std::vector<uint32_t> root;
  components(e, n, root);
  std::vector<int64_t> size(n, 0);
  for (int64_t v = 0; v < n; ++v) size[root[v]]++;
  int64_t best = 0;
  for (int64_t v = 1; v < n; ++v)
    if (size[v] > size[best]) best = v;
  std::vector<char> keep(n, 0);
  for (int64_t v = 0; v < n; ++v) keep[v] = (root[v] == (uint32_t)best);
  return induce(e, keep, n);
}

// Seeded random relabelling of the vertices.
void permute(EdgeList& e, int64_t n, uint64_t seed) {
  Rng r(seed, 0x7065726dULL);
  std::vector<std::pair<uint64_t, uint32_t>> kv(n);
  for (int64_t v = 0; v < n; ++v) kv[v] = {r.at((uint64_t)v), (uint32_t)v};
  __gnu_parallel::sort(kv.begin(), kv.end());
  std::vector<uint32_t> nid(n);
  for (int64_t i = 0; i < n; ++i) nid[kv[i].second] = (uint32_t)i;
  for (size_t i = 0; i < e.key.size(); ++i)
    e.key[i] = ekey(nid[e.key[i] >> 32], nid[(uint32_t)e.key[i]]);
}

}  // namespace

extern "C" {

typedef struct gg_csr {
  int32_t n;
  int64_t nnz;       // 2 * undirected edges
  int64_t* row_ptr;  // n + 1
  int32_t* col;      // nnz
  int32_t* w;        // nnz
} gg_csr;

void gg_free(gg_csr* g) {
  if (!g) return;
  free(g->row_ptr);
  free(g->col);
  free(g->w);
  g->row_ptr = nullptr;
  g->col = g->w = nullptr;
}

}  // extern "C"

namespace {

// Symmetric CSR with each row sorted by neighbour id.
int to_csr(const EdgeList& e, int64_t n, gg_csr* out) {
  out->n = (int32_t)n;
  out->nnz = 2 * (int64_t)e.key.size();
  out->row_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  out->col = (int32_t*)malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(out->nnz, 1));
  out->w = (int32_t*)malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(out->nnz, 1));
  if (!out->row_ptr || !out->col || !out->w) return -4;
  for (uint64_t kk : e.key) { out->row_ptr[(kk >> 32) + 1]++; out->row_ptr[(uint32_t)kk + 1]++; }
  for (int64_t v = 0; v < n; ++v) out->row_ptr[v + 1] += out->row_ptr[v];
  std::vector<int64_t> pos(out->row_ptr, out->row_ptr + n);
  for (size_t i = 0; i < e.key.size(); ++i) {
    uint32_t u = e.key[i] >> 32, v = (uint32_t)e.key[i];
    out->col[pos[u]] = (int32_t)v; out->w[pos[u]++] = e.w[i];
    out->col[pos[v]] = (int32_t)u; out->w[pos[v]++] = e.w[i];
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    int64_t a = out->row_ptr[v], b = out->row_ptr[v + 1];
    std::vector<std::pair<int32_t, int32_t>> row(b - a);
    for (int64_t i = a; i < b; ++i) row[i - a] = {out->col[i], out->w[i]};
    std::sort(row.begin(), row.end());
    for (int64_t i = a; i < b; ++i) { out->col[i] = row[i - a].first; out->w[i] = row[i - a].second; }
  }
  return 0;
}

}  // namespace

extern "C" {

// Planted-cluster graph: k near-equal clusters over n vertices, each an
// Erdos-Renyi graph with edge probability p (if p < 0 the probability is
// min(1, avg_deg / (s - 1)) for cluster size s, avg_deg = -p).
// Inter-cluster edges: if inter_total > 0, that many edges, each on a
// uniformly chosen pair of distinct clusters with uniform endpoints
// (duplicates redrawn); otherwise every cluster pair gets a uniform count in
// [inter_min, inter_max].  Weights uniform in [wmin, wmax].  Redrawn with a
// derived seed until connected; vertices are randomly relabelled.
int gg_planted(uint64_t seed, int32_t n, int32_t k, double p, int32_t inter_total,
               int32_t inter_min, int32_t inter_max, int32_t wmin, int32_t wmax,
               gg_csr* out) {
  if (n < 2 || k < 1 || k > n || wmin < 1 || wmax < wmin) return -1;
  for (uint64_t attempt = 0; attempt < 1000; ++attempt) {
    uint64_t s = mix64(seed + attempt * 0x1000193ULL);
    Rng r(s, 1), rw(s, 2), ri(s, 3);
    std::vector<int32_t> start(k + 1);
    for (int32_t c = 0; c <= k; ++c) start[c] = (int32_t)((int64_t)n * c / k);
    EdgeList e;
    uint64_t ctr = 0;
    for (int32_t c = 0; c < k; ++c) {
      int32_t a = start[c], b = start[c + 1], sz = b - a;
      double pc = p >= 0 ? p : std::min(1.0, -p / std::max(1, sz - 1));
      uint64_t thr = pc >= 1.0 ? ~0ULL : (uint64_t)std::ldexp(pc, 64);
      for (int32_t i = a; i < b; ++i)
        for (int32_t j = i + 1; j < b; ++j) {
          uint64_t x = r.at(ctr++);
          if (x < thr || pc >= 1.0) e.key.push_back(ekey(i, j));
        }
    }
    std::vector<uint64_t> inter;
    uint64_t ic = 0;
    if (inter_total > 0 && k > 1) {
      std::vector<uint64_t> seen;
      while ((int32_t)inter.size() < inter_total) {
        int32_t c1 = (int32_t)ri.below(ic++, k), c2 = (int32_t)ri.below(ic++, k - 1);
        if (c2 >= c1) ++c2;
        int32_t u = start[c1] + (int32_t)ri.below(ic++, start[c1 + 1] - start[c1]);
        int32_t v = start[c2] + (int32_t)ri.below(ic++, start[c2 + 1] - start[c2]);
        uint64_t kk = ekey(u, v);
        if (std::find(inter.begin(), inter.end(), kk) != inter.end()) continue;
        inter.push_back(kk);
      }
    } else if (k > 1) {
      for (int32_t c1 = 0; c1 < k; ++c1)
        for (int32_t c2 = c1 + 1; c2 < k; ++c2) {
          int32_t t = inter_min + (int32_t)ri.below(ic++, inter_max - inter_min + 1);
          for (int32_t q = 0; q < t; ++q) {
            int32_t u = start[c1] + (int32_t)ri.below(ic++, start[c1 + 1] - start[c1]);
            int32_t v = start[c2] + (int32_t)ri.below(ic++, start[c2 + 1] - start[c2]);
            inter.push_back(ekey(u, v));
          }
        }
    }
    e.key.insert(e.key.end(), inter.begin(), inter.end());
    merge_duplicates(e, 1);
    for (size_t i = 0; i < e.key.size(); ++i)
      e.w[i] = wmin + (int32_t)Rng(s, 4 + e.key[i]).below(0, (uint64_t)(wmax - wmin + 1));
    (void)rw;
    std::vector<uint32_t> root;
    if (components(e, n, root) != 1) continue;
    permute(e, n, s);
    merge_duplicates(e, 0);  // re-sort after relabelling (no duplicates remain)
    return to_csr(e, n, out);
  }
  return -2;
}

// Chung-Lu power-law graph: expected degrees proportional to
// (i + i0)^(-1/(beta-1)) with i0 chosen so the largest expected degree is
// sqrt(n * avg_deg), scaled to mean avg_deg; n*avg_deg/2 edge draws with
// endpoints proportional to the expected degrees.  Self-loops dropped,
// duplicates collapsed.  Weights uniform in [wmin, wmax] per distinct edge.
// Then the kcore-core (kcore <= 1: none) and, if lcc, the largest component;
// vertices randomly relabelled.
int gg_chung_lu(uint64_t seed, int64_t n, double beta, double avg_deg, int32_t wmin,
                int32_t wmax, int32_t kcore_k, int32_t lcc, gg_csr* out) {
  if (n < 2 || beta <= 2.0 || avg_deg <= 0 || wmin < 1 || wmax < wmin) return -1;
  const double gam = 1.0 / (beta - 1.0);
  const double target = std::sqrt((double)n * avg_deg) / avg_deg;  // max / mean
  // mean of (x + i0)^(-gam) over [0, n] by its integral (i0 only shapes the
  // head of the distribution; the exact scale is fixed below from the sum)
  auto ratio = [&](double i0) {
    double mean = (std::pow((double)n + i0, 1.0 - gam) - std::pow(i0, 1.0 - gam)) /
                  ((1.0 - gam) * (double)n);
    return std::pow(i0, -gam) / mean;
  };
  double lo = 1e-3, hi = (double)n;
  for (int it = 0; it < 60; ++it) {
    double mid = std::sqrt(lo * hi);
    if (ratio(mid) > target) lo = mid; else hi = mid;
  }
  const double i0 = std::sqrt(lo * hi);
  std::vector<double> cdf(n + 1, 0.0);
  for (int64_t i = 0; i < n; ++i) cdf[i + 1] = cdf[i] + std::pow((double)i + i0, -gam);
  const double tot = cdf[n];
  const int64_t draws = (int64_t)std::llround((double)n * avg_deg / 2.0);
  EdgeList e;
  e.key.resize(draws);
  Rng r(seed, 11);
#pragma omp parallel for schedule(static)
  for (int64_t d = 0; d < draws; ++d) {
    double x = r.unit(2 * (uint64_t)d) * tot, y = r.unit(2 * (uint64_t)d + 1) * tot;
    int64_t u = std::upper_bound(cdf.begin(), cdf.end(), x) - cdf.begin() - 1;
    int64_t v = std::upper_bound(cdf.begin(), cdf.end(), y) - cdf.begin() - 1;
    u = std::min<int64_t>(std::max<int64_t>(u, 0), n - 1);
    v = std::min<int64_t>(std::max<int64_t>(v, 0), n - 1);
    e.key[d] = ekey((uint32_t)u, (uint32_t)v);
  }
  merge_duplicates(e, 1);
  drop_self_loops(e);
  int64_t nn = n;
  if (kcore_k > 1) nn = kcore(e, nn, kcore_k);
  if (lcc) nn = largest_component(e, nn);
  if (nn < 2) return -2;
  permute(e, nn, seed);
  merge_duplicates(e, 1);
  Rng rw(seed, 12);
  for (size_t i = 0; i < e.key.size(); ++i)
    e.w[i] = wmin + (int32_t)Rng(seed ^ 0xC0FFEEULL, e.key[i]).below(0, (uint64_t)(wmax - wmin + 1));
  (void)rw;
  return to_csr(e, nn, out);
}

// R-MAT graph with 2^scale vertices and n_draws edge draws using quadrant
// probabilities (a, b, c, 1-a-b-c), no noise.  Undirected; self-loops
// dropped; duplicates merged into weight = multiplicity.  Then the
// kcore-core on distinct-neighbour degree and, if lcc, the largest
// component; vertices randomly relabelled.
int gg_rmat(uint64_t seed, int32_t scale, int64_t n_draws, double a, double b, double c,
            int32_t kcore_k, int32_t lcc, gg_csr* out) {
  if (scale < 1 || scale > 30 || n_draws < 1) return -1;
  const uint32_t ta = (uint32_t)std::llround(a * 65536.0);
  const uint32_t tb = (uint32_t)std::llround((a + b) * 65536.0);
  const uint32_t tc = (uint32_t)std::llround((a + b + c) * 65536.0);
  EdgeList e;
  e.key.resize(n_draws);
  Rng r(seed, 21);
#pragma omp parallel for schedule(static)
  for (int64_t d = 0; d < n_draws; ++d) {
    uint32_t u = 0, v = 0;
    uint64_t bits = 0;
    int have = 0;
    uint64_t ctr = (uint64_t)d * 8;
    for (int l = 0; l < scale; ++l) {
      if (have == 0) { bits = r.at(ctr++); have = 4; }
      uint32_t x = (uint32_t)(bits & 0xFFFF);
      bits >>= 16;
      --have;
      uint32_t ub = 0, vb = 0;
      if (x < ta) { ub = 0; vb = 0; }
      else if (x < tb) { ub = 0; vb = 1; }
      else if (x < tc) { ub = 1; vb = 0; }
      else { ub = 1; vb = 1; }
      u = (u << 1) | ub;
      v = (v << 1) | vb;
    }
    e.key[d] = ekey(u, v);
  }
  merge_duplicates(e, 0);
  drop_self_loops(e);
  int64_t nn = (int64_t)1 << scale;
  if (kcore_k > 1) nn = kcore(e, nn, kcore_k);
  if (lcc) nn = largest_component(e, nn);
  if (nn < 2) return -2;
  permute(e, nn, seed);
  merge_duplicates(e, 0);
  return to_csr(e, nn, out);
}

// Small structured graphs with known minimum cuts (for oracle pins).
// kind 0: complete graph K_n with weight w0.
// kind 1: cycle on n vertices with weights from the seed in [wmin, wmax].
// kind 2: two complete graphs K_a (a = n/2) joined by k unit edges on
//         distinct endpoints (k = wmin).
// Returns the plain edge list form (n, arrays) through the CSR.
int gg_structured(int32_t kind, int32_t n, uint64_t seed, int32_t wmin, int32_t wmax,
                  gg_csr* out) {
  EdgeList e;
  Rng r(seed, 31);
  if (kind == 0) {
    for (int32_t i = 0; i < n; ++i)
      for (int32_t j = i + 1; j < n; ++j) { e.key.push_back(ekey(i, j)); e.w.push_back(wmin); }
  } else if (kind == 1) {
    for (int32_t i = 0; i < n; ++i) {
      e.key.push_back(ekey(i, (i + 1) % n));
      e.w.push_back(wmin + (int32_t)r.below((uint64_t)i, (uint64_t)(wmax - wmin + 1)));
    }
  } else if (kind == 2) {
    int32_t a = n / 2;
    for (int32_t i = 0; i < a; ++i)
      for (int32_t j = i + 1; j < a; ++j) {
        e.key.push_back(ekey(i, j)); e.w.push_back(1);
        e.key.push_back(ekey(a + i, a + j)); e.w.push_back(1);
      }
    for (int32_t q = 0; q < wmin && q < a; ++q) { e.key.push_back(ekey(q, a + q)); e.w.push_back(1); }
    n = 2 * a;
  } else {
    return -1;
  }
  merge_duplicates(e, 0);
  return to_csr(e, n, out);
}

}  // extern "C"
