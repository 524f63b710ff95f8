// Parallel bounded CAPFOREST (Algorithm 1, section "Parallel CAPFOREST";
// bounded keys per Lemma 1, section "Bounded Priority Queues").
//
// One wave64 runs one scan at a time.  A scan keeps, in LDS, an
// open-addressing map from vertex id to r(v) (the weight from the vertices
// this scan already visited) together with the vertex state (frontier,
// visited, blacklisted).  pop_max is a wave-wide argmax of the capped key
// min(r, lambda-hat) over the map, which is an exact maximum for any key
// range, so no bucket array has to be sized to lambda-hat.
//
// Visit claims go through a shared int32 array with compare-and-swap, so
// every vertex is visited by at most one scan per round; a scan that loses
// the claim blacklists the vertex locally and leaves it at once (skips both
// the alpha update and its edges).  An edge (x, y) whose r(y) crosses
// lambda-hat while x is scanned is recorded as a contractible pair; the
// pairs are united after the scans.  Early termination (map full, budget
// reached) is safe by Lemma 2.2.  alpha = c(S) for the visited prefix S is
// tracked exactly and its minimum over proper prefixes is reported.
#pragma once
#include "dev.h"

namespace mc {

constexpr uint32_t SLOT_EMPTY = 0xFFFFFFFFu;
constexpr uint32_t VID_MASK = 0x3FFFFFFFu;
constexpr uint32_t ST_VISITED = 0x40000000u;
constexpr uint32_t ST_BLACK = 0x80000000u;
constexpr int32_t FALLBACK_SID = 0x7FFFFFFF;

struct Ctl {
  int32_t err;
  int32_t n_next;        // vertices after compaction
  int64_t emit;          // keys emitted for contraction
  int64_t unique;        // entries after merging
  int64_t pairs;         // contractible pairs recorded by scans
  int64_t pairs_dropped;
  int64_t unions_pr;
  int64_t unions_scan;
  int32_t work_next;     // scan work counter
  int32_t scan_ids;      // scans started
  int32_t n_whole;       // graphs scanned whole with the small map
  int32_t n_whole2;      // graphs scanned whole with the large map
  int32_t n_region;      // graphs scanned by region scans
  int32_t n_active;
  int32_t n_fallback;
  int32_t improved;
  int64_t pops;          // vertices visited by scans
  int64_t overflows;     // scans ended because the map filled
  int64_t whole_nnz;     // adjacency entries of the graphs scanned whole
  int64_t whole_nv;      // vertices of the graphs scanned whole
  int32_t lp_items;      // workgroup items of label propagation (long rows)
  int32_t n_pr;          // graphs where a Padberg-Rinaldi test can pass in the first contraction round
  int64_t lam_floor;     // the smallest bound of a tested graph (Padberg-Rinaldi prefilter)
  int32_t asym;          // symmetry check: some vertex pair's two directions differ
  int32_t pad_;
  int64_t nonref_nnz;    // contraction: entries in rows outside their graph's reference block
};

struct ScanArgs {
  int32_t n;
  const int64_t* rp;
  const int32_t* col;
  const int32_t* w;
  const int64_t* cdeg;
  const int32_t* gid;
  const int64_t* lhat;   // per graph, fixed for the round
  const int32_t* gn;     // per graph vertex count
  const int32_t* gvoff;  // per graph first vertex
  const uint8_t* gmode;  // 0 idle, 1 whole-graph scan, 2 region scans
  const int32_t* whole;  // graphs to scan whole
  const int32_t* whole_count;  // device count of `whole`
  int32_t* claim;
  int32_t* step;
  uint64_t* pairs;
  int64_t pairs_cap;
  uint64_t* best_alpha;  // per graph (alpha << 32) | scan id
  int32_t* scan_k;       // per scan id: length of the best prefix
  int32_t scan_k_cap;
  int32_t* ucount;       // per graph: pairs recorded
  Ctl* ctl;
  uint64_t perm_a, perm_b;
  int32_t perm_bits;
  int32_t whole_mode;    // this launch serves whole-graph items (1) or region items (0)
  int32_t eager;         // skip neighbours already claimed by another scan
  int32_t max_pops;
  uint64_t seed;
  int32_t order;         // ORD kernels: the order among equal keys (tie_rank)
  int32_t visits;        // a vertex may be visited by up to this many scans
  int32_t* vcount;       // visits > 1: per vertex, the visits after the first
};

// ORD: each slot also keeps the pop count of its vertex's last increase,
// which orders equal keys.
template <int CAP, bool ORD = false>
struct ScanLds {
  uint32_t vid[CAP];
  int32_t r[CAP];
  uint16_t tick[ORD ? CAP : 2];
  int32_t used;
  int32_t pad[3];
};

template <int CAP>
__device__ __forceinline__ uint32_t slot_hash(uint32_t v) {
  constexpr int LOG = __builtin_ctz(CAP);
  return (v * 0x9E3779B1u) >> (32 - LOG);
}

// Find y's slot, inserting it if absent.  -1 when the map is too full.
template <int CAP, bool ORD>
__device__ __forceinline__ int map_find_insert(ScanLds<CAP, ORD>& m, uint32_t y) {
  uint32_t h = slot_hash<CAP>(y);
  for (int probe = 0; probe < 64; ++probe) {
    uint32_t cur = m.vid[h];
    if (cur == SLOT_EMPTY) {
      if (atomicAdd(&m.used, 1) >= (CAP * 3) / 4) {
        atomicSub(&m.used, 1);
        return -1;
      }
      uint32_t prev = atomicCAS(&m.vid[h], SLOT_EMPTY, y);
      if (prev == SLOT_EMPTY) return (int)h;
      atomicSub(&m.used, 1);
      cur = prev;
    }
    if ((cur & VID_MASK) == y) return (int)h;
    h = (h + 1) & (CAP - 1);
  }
  return -1;
}

__device__ __forceinline__ uint32_t perm_at(uint64_t a, uint64_t b, int bits, uint64_t i) {
  uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
  return (uint32_t)((a * i + b) & mask);
}

// One bounded scan from `start` inside graph g.  Returns pairs recorded.
//
// With A.visits > 1 a vertex already visited by another scan may be visited
// again, by at most visits - 1 more scans (the multi-visit variant of section
// "Parallel CAPFOREST"): each scan stays a bounded CAPFOREST of its own, so
// its pairs stay contractible.  claim and step describe only first visits, so
// a scan reports prefix cuts only while every vertex it visited was a first
// visit.
template <int CAP, bool ORD>
__device__ int64_t run_scan(const ScanArgs& A, ScanLds<CAP, ORD>& m, int32_t start, int32_t g) {
  const int lane = lane_id();
  // clear the map
  for (int s = lane; s < CAP; s += 64) {
    m.vid[s] = SLOT_EMPTY;
    m.r[s] = 0;
    if constexpr (ORD) m.tick[s] = 0;
  }
  if (lane == 0) m.used = 0;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (lane == 0) (void)map_find_insert<CAP>(m, (uint32_t)start);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

  const int64_t lam = A.lhat[g];
  const int32_t ng = A.gn[g];
  int32_t sid = 0;
  if (lane == 0) sid = atomicAdd(&A.ctl->scan_ids, 1);
  sid = bcast(sid, 0);

  int64_t alpha = 0, best_a = INT64_MAX;
  int32_t k = 0, best_k = 0;
  int64_t npairs = 0;
  bool stop = false, first_visits = true;
  while (!stop) {
    // pop_max: argmax of capped keys over frontier slots (ORD: then the
    // rank of the chosen order, with the slot taken from the lane holding it)
    int slot;
    if constexpr (ORD) {
      uint64_t best = 0;
      int mine = 0;
      for (int s = lane; s < CAP; s += 64) {
        uint32_t u = m.vid[s];
        if (u != SLOT_EMPTY && !(u & (ST_VISITED | ST_BLACK))) {
          int64_t key = m.r[s];
          if (key > lam) key = lam;
          uint64_t c = ((uint64_t)(key + 1) << 32) | tie_rank(A.order, m.tick[s], u & VID_MASK);
          if (c > best) { best = c; mine = s; }
        }
      }
      const uint64_t top = wave_max_u64(best);
      if (top == 0) break;  // queue empty
      slot = __builtin_amdgcn_readlane(mine, (int)__builtin_ctzll(ballot(best == top)));
    } else {
      uint64_t best = 0;
      for (int s = lane; s < CAP; s += 64) {
        uint32_t u = m.vid[s];
        if (u != SLOT_EMPTY && !(u & (ST_VISITED | ST_BLACK))) {
          int64_t key = m.r[s];
          if (key > lam) key = lam;
          uint64_t c = ((uint64_t)(key + 1) << 32) | (uint32_t)s;
          best = c > best ? c : best;
        }
      }
      best = wave_max_u64(best);
      if (best == 0) break;  // queue empty
      slot = (int)(uint32_t)best;
    }
    const int32_t x = (int32_t)(m.vid[slot] & VID_MASK);
    const int64_t rx = m.r[slot];
    int32_t old = 0;
    if (lane == 0) old = atomicCAS(A.claim + x, -1, sid);
    old = bcast(old, 0);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const bool first = old == -1 || old == sid;
    if (!first) {
      // visited elsewhere: visit it again while visits are left, else
      // blacklist it and leave it at once
      int32_t again = 0;
      if (lane == 0 && A.visits > 1) again = atomicAdd(A.vcount + x, 1) < A.visits - 1;
      again = bcast(again, 0);
      if (!again) {
        if (lane == 0) m.vid[slot] |= ST_BLACK;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        continue;
      }
      first_visits = false;
    }
    if (lane == 0) {
      m.vid[slot] |= ST_VISITED;
      if (first) A.step[x] = k + 1;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    ++k;
    alpha += A.cdeg[x] - 2 * rx;  // alpha = c(S) with S the visited prefix
    if (first_visits && k < ng && alpha < best_a) { best_a = alpha; best_k = k; }
    if (k >= A.max_pops) stop = true;

    const int64_t e0 = A.rp[x], e1 = A.rp[x + 1];
    bool full = false;
    for (int64_t base = e0; base < e1; base += 64) {
      const int64_t e = base + lane;
      bool act = e < e1;
      const int64_t ec = act ? e : base;  // loads outside branches: no wait at a branch end
      int32_t y = A.col[ec];
      int32_t c = A.w[ec];
      keep(c);
      y = act ? y : 0;
      c = act ? c : 0;
      if (y == x) act = false;
      if (act && A.eager) {
        int32_t cl = ld_relaxed(A.claim + y);
        if (cl != -1 && cl != sid && (A.visits <= 1 || ld_relaxed(A.vcount + y) >= A.visits - 1)) act = false;
      }
      int sl = -1;
      if (act) {
        sl = map_find_insert<CAP>(m, (uint32_t)y);
        if (sl < 0) { act = false; full = true; }
      }
      bool cross = false;
      if (act) {
        uint32_t u = m.vid[sl];
        if (u & (ST_VISITED | ST_BLACK)) act = false;
      }
      if (act) {
        if constexpr (ORD) m.tick[sl] = (uint16_t)k;
        int64_t before = atomicAdd(&m.r[sl], c);
        int64_t after = before + c;
        cross = before < lam && lam <= after;  // crossing rule of Algorithm 1
      }
      uint64_t cm = ballot(cross);
      if (cm) {
        int cnt = popc64(cm);
        int64_t pbase = 0;
        if (lane == 0) pbase = atomicAdd((unsigned long long*)&A.ctl->pairs, (unsigned long long)cnt);
        pbase = bcast(pbase, 0);
        if (cross) {
          int64_t at = pbase + popc64(cm & lanemask_lt());
          if (at < A.pairs_cap) A.pairs[at] = ((uint64_t)(uint32_t)x << 32) | (uint32_t)y;
        }
        int64_t kept = pbase >= A.pairs_cap ? 0 : (pbase + cnt > A.pairs_cap ? A.pairs_cap - pbase : cnt);
        npairs += kept;
        if (lane == 0 && kept < cnt)
          atomicAdd((unsigned long long*)&A.ctl->pairs_dropped, (unsigned long long)(cnt - kept));
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    if (ballot(full)) {
      stop = true;
      if (lane == 0) atomicAdd((unsigned long long*)&A.ctl->overflows, 1ull);
    }
  }
  if (lane == 0) {
    if (best_a < lam && sid < A.scan_k_cap) {
      A.scan_k[sid] = best_k;
      __threadfence();
      atomic_min_u64(A.best_alpha + g, ((uint64_t)best_a << 32) | (uint32_t)sid);
    }
    if (npairs) atomicAdd(A.ucount + g, (int32_t)npairs);
    atomicAdd((unsigned long long*)&A.ctl->pops, (unsigned long long)k);
  }
  return npairs;
}

// Persistent scan workers.  whole_mode: one scan per listed graph, started
// at a seeded vertex and covering the whole graph (the map holds it).
// Otherwise: region scans started at unclaimed vertices taken in a seeded
// pseudo-random order, 64 candidates per work item.
template <int CAP, bool ORD = false>
__global__ void __launch_bounds__(256) k_capforest(ScanArgs A) {
  extern __shared__ __align__(16) char lds_raw[];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  ScanLds<CAP, ORD>& m = reinterpret_cast<ScanLds<CAP, ORD>*>(lds_raw)[wave];
  while (true) {
    int32_t item = 0;
    if (lane == 0) item = atomicAdd(&A.ctl->work_next, 1);
    item = bcast(item, 0);
    if (A.whole_mode) {
      if (item >= *A.whole_count) break;
      const int32_t g = A.whole[item];
      const int32_t ng = A.gn[g];
      uint64_t h = A.seed * 0x9E3779B97F4A7C15ull + (uint64_t)g * 0xBF58476D1CE4E5B9ull;
      h ^= h >> 29;
      const int32_t start = A.gvoff[g] + (int32_t)(h % (uint64_t)ng);
      run_scan<CAP, ORD>(A, m, start, g);
      continue;
    }
    const uint64_t span = 1ull << A.perm_bits;
    const uint64_t c0 = (uint64_t)item * 64;
    if (c0 >= span) break;
    uint32_t v = perm_at(A.perm_a, A.perm_b, A.perm_bits, c0 + lane);
    bool cand = v < (uint32_t)A.n;
    if (cand) cand = A.gmode[A.gid[v]] == 2;
    uint64_t todo = ballot(cand);
    while (todo) {
      const int src_lane = __builtin_ctzll(todo);
      todo &= todo - 1;
      const int32_t s = bcast((int32_t)v, src_lane);
      if (ld_relaxed(A.claim + s) != -1) continue;
      run_scan<CAP, ORD>(A, m, s, A.gid[s]);
    }
  }
}

}  // namespace mc
