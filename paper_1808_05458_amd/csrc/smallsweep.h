// Capped CAPFOREST sweep of a whole small graph inside one workgroup
// (appendix Algorithm 3 with the cap of Lemma 1; batches of capped vertices
// as in sweep.h).  The graph's vertices [v0, v0 + ng) index LDS arrays
// directly (16-bit local ids): r (weight to the visited set) and the state,
// so every priority update is an LDS atomic.
//
// A vertex enters the capped queue when its r crosses the cap (exactly one
// relaxation crosses, since r only grows).  A step's batch is the part of
// the queue filled since the last step: every unvisited vertex at the cap,
// and nothing can exceed the cap, so they are all maxima of the capped keys
// and any order among them is a legal maximum-adjacency order.  With the
// queue empty every unvisited vertex is below the cap, and one wave pops
// singles by itself, without workgroup barriers, until some vertex reaches
// the cap.  Its maximum comes from a two-level structure: per chunk of 64
// vertices an upper bound of r over the chunk's unvisited vertices (raised
// by an atomic max on every relaxation), and an exact scan of the best
// chunk, which lowers a stale bound and retries.  A batch is relaxed by the
// whole workgroup with its entries spread evenly over the threads.  The
// crossings are the contractible pairs r(y) < cap <= r(y) + c(e) of
// Algorithm 1; alpha (= c(S) of the visited set) is tracked per step from
// the row sums, r and the batch-internal weight.
#pragma once
#include "capforest.h"
#include "sweep.h"

namespace mc {

struct SmallSweepArgs {
  const int64_t* rp;
  const int32_t* col;
  const int32_t* w;
  const int64_t* cdeg;         // weighted degree without self-loops
  const int64_t* lhat;
  const int32_t* gn;
  const int32_t* gvoff;
  const int32_t* list_a;       // graphs to sweep: list_a then list_b, largest first
  const int32_t* count_a;      // device counts of the lists
  const int32_t* list_b;
  const int32_t* count_b;
  int32_t* work;               // work counter (zeroed by the host)
  uint64_t* fb_rs;             // per vertex: visit stamp in the high 32 bits (side)
  int32_t* capq;               // crossing pairs (capx[i], capq[i]) at v0 + i
  int32_t* capx;
  int32_t* npairs;             // per graph: pairs recorded
  uint64_t* best_alpha;        // per graph (alpha << 32) | SWEEP_SID
  int32_t* fb_k;               // per graph: stamp of the best prefix
  int32_t* ucount;
  uint64_t seed;
  int32_t order;               // ORD kernels: the order among equal keys below
                               // the cap (tie_rank: 1 bucket queue, 2 bucket
                               // stack, 3 heap)
};

constexpr int SS_UNROLL = 4;  // entries in flight per thread in a batch relax

// LDS of one sweep: CAP vertices, THREADS threads per workgroup.  ORD: the
// single pops below the cap follow a chosen order among equal keys (the
// chunk bounds then hold (r, rank) pairs and each vertex the step of its
// last increase).
template <int CAP, int THREADS, bool ORD = false>
struct SmallSweepLds {
  static_assert(CAP <= 65536 && CAP % 64 == 0, "16-bit local vertex ids, whole chunks");
  static_assert(!ORD || 2 * CAP < 65536, "a sweep's steps (at most two per vertex) fit the 16-bit ticks");
  static_assert(THREADS % 64 == 0 && THREADS <= 1024, "whole waves");
  static constexpr int NC = CAP / 64;
  static constexpr int NW = THREADS / 64;
  static constexpr bool ordered = ORD;
  using Bound = typename std::conditional<ORD, unsigned long long, uint32_t>::type;
  int32_t r[CAP];
  uint16_t capped[CAP];  // vertices in the order their r reached the cap
  uint32_t st[CAP / 16];  // 2 bits per vertex: 0 unvisited, 2 visited, 3 in the current batch
  Bound cmax[NC];        // per 64-vertex chunk: >= the key of its unvisited vertices
  uint16_t lt[ORD ? CAP : 2];  // ORD: step of each vertex's last increase
  int32_t boff[THREADS + 1];  // a batch chunk: entry offsets of its rows
  int32_t bbase[THREADS];     //   and each row's first entry (graph-relative)
  int32_t wtot[NW];
  int32_t cap_head, cap_tail, npairs, first;
  int32_t b0, nb, stamp;  // the batch capped[b0, b0 + nb); nb < 0: sweep done
  int64_t wsum[NW], wint[NW];
};

// The 2-bit visit state.  Marking is 0 -> 3 (an OR of both bits) and a
// batch becomes visited by 3 -> 2 (clearing the low bit), so concurrent marks
// of vertices sharing a word are atomic bit operations.
template <class LDS>
__device__ __forceinline__ uint32_t ss_state(const LDS& L, int32_t v) {
  return (L.st[v >> 4] >> (2 * (v & 15))) & 3u;
}
template <class LDS>
__device__ __forceinline__ void ss_mark(LDS& L, int32_t v) {
  atomicOr(&L.st[v >> 4], 3u << (2 * (v & 15)));
}
template <class LDS>
__device__ __forceinline__ void ss_visited(LDS& L, int32_t v) {
  atomicAnd(&L.st[v >> 4], ~(1u << (2 * (v & 15))));
}

__device__ __forceinline__ void ss_wave_sync() {
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <class LDS>
__device__ __forceinline__ unsigned long long ss_key(const LDS& L, int32_t order, int32_t v, uint32_t r) {
  return ((unsigned long long)r << 32) | tie_rank(order, L.lt[v], (uint32_t)v);
}

// Relax one entry x -> y of weight c (local ids): update r(y) and its chunk
// bound, and record the crossing r(y) < cap <= r(y) + c as a pair and a
// capped vertex.  Must be called by all lanes of the wave.  tick: the step
// (ORD kernels: the last increase's step, which orders equal keys).
template <class LDS>
__device__ __forceinline__ bool ss_relax(LDS& L, const SmallSweepArgs& A, int32_t v0, int64_t lam,
                                         bool ok, int32_t xl, int32_t yl, int32_t c, int64_t& rows,
                                         int64_t& internal, uint32_t tick = 0) {
  bool cross = false;
  if (ok && yl != xl) {
    rows += c;
    const uint32_t s = ss_state(L, yl);
    if (s == 3) {
      internal += c;
    } else if (s == 0) {
      const int32_t old = atomicAdd(&L.r[yl], c);
      if constexpr (LDS::ordered) {
        L.lt[yl] = (uint16_t)tick;
        atomicMax(&L.cmax[yl >> 6], ((unsigned long long)(uint32_t)(old + c) << 32) | tie_rank(A.order, tick, (uint32_t)yl));
      } else {
        atomicMax(&L.cmax[yl >> 6], (uint32_t)(old + c));
      }
      cross = (int64_t)old < lam && lam <= (int64_t)old + c;
    }
  }
  const uint64_t cm = ballot(cross);
  if (cm) {
    int32_t at = 0, qa = 0;
    if (lane_id() == 0) {
      at = atomicAdd(&L.npairs, popc64(cm));
      qa = atomicAdd(&L.cap_tail, popc64(cm));
    }
    at = bcast(at, 0);
    qa = bcast(qa, 0);
    if (cross) {
      const int32_t rank = popc64(cm & lanemask_lt());
      A.capq[v0 + at + rank] = v0 + yl;
      A.capx[v0 + at + rank] = v0 + xl;
      L.capped[qa + rank] = (uint16_t)yl;
    }
  }
  return cm != 0;
}

// An unvisited vertex of largest r > 0, and that r (one wave, all lanes, no
// other wave active); -1 when none is left.  Among equal keys the lowest
// chunk and the lowest vertex in it are taken (any maximum is a legal next
// vertex).  The caller visits the vertex, so its chunk's bound drops to the
// largest key left in the chunk.  Once the chunk is known every lane loads
// its vertex's row bounds and degree, so the winner's are in flight while
// the chunk is scanned: (ra, rb, cd) of the returned vertex.
template <class LDS>
__device__ __forceinline__ int32_t ss_select(LDS& L, const SmallSweepArgs& A, int32_t v0, int32_t ng,
                                             uint32_t& rx, int64_t& ra, int64_t& rb, int64_t& cd) {
  constexpr int NC = LDS::NC;
  const int lane = lane_id();
  const int nc = (ng + 63) >> 6;
  if constexpr (LDS::ordered) {
    // the same two-level search over (r, rank) keys: any maximum of r is a
    // legal next vertex, and the rank picks among them
    while (true) {
      unsigned long long mine = 0;
      int32_t mine_c = 0;
      for (int c = lane; c < nc && c < NC; c += 64) {
        const unsigned long long k = L.cmax[c];
        if (k > mine) { mine = k; mine_c = c; }
      }
      const unsigned long long bound = wave_max_u64(mine);
      if ((bound >> 32) == 0) return -1;
      const int holder = (int)__builtin_ctzll(ballot(mine == bound));
      const int c = __builtin_amdgcn_readlane(mine_c, holder);
      const int32_t v = c * 64 + lane;
      const int32_t vq = v < ng ? v : ng - 1;
      const int64_t la = A.rp[v0 + vq], lb = A.rp[v0 + vq + 1], lc = A.cdeg[v0 + vq];
      const uint32_t rv = (v < ng && ss_state(L, v) == 0) ? (uint32_t)L.r[v] : 0u;
      const unsigned long long key = rv > 0 ? ss_key(L, A.order, v, rv) : 0ull;
      const unsigned long long exact = wave_max_u64(key);
      if (exact == bound) {
        const int at = (int)__builtin_ctzll(ballot(key == exact));
        const unsigned long long rest = wave_max_u64(lane == at ? 0ull : key);
        if (lane == 0) L.cmax[c] = rest;
        rx = (uint32_t)(exact >> 32);
        ra = readlane_i64(la, at);
        rb = readlane_i64(lb, at);
        cd = readlane_i64(lc, at);
        return c * 64 + at;
      }
      if (lane == 0) L.cmax[c] = exact;  // the bound was stale: lower it, retry
      ss_wave_sync();
    }
  }
  while (true) {
    uint32_t mine = 0;
    int32_t mine_c = 0;
    for (int c = lane; c < nc && c < NC; c += 64) {
      const uint32_t k = L.cmax[c];
      if (k > mine) { mine = k; mine_c = c; }
    }
    const uint32_t bound = wave_max_u32(mine);
    if (bound == 0) return -1;
    const int holder = (int)__builtin_ctzll(ballot(mine == bound));
    const int c = __builtin_amdgcn_readlane(mine_c, holder);
    const int32_t v = c * 64 + lane;
    const int32_t vq = v < ng ? v : ng - 1;
    const int64_t la = A.rp[v0 + vq], lb = A.rp[v0 + vq + 1], lc = A.cdeg[v0 + vq];
    const uint32_t key = (v < ng && ss_state(L, v) == 0) ? (uint32_t)L.r[v] : 0u;
    const uint32_t exact = wave_max_u32(key);
    if (exact == bound) {
      const int at = (int)__builtin_ctzll(ballot(key == exact));
      const uint32_t rest = wave_max_u32(lane == at ? 0u : key);
      if (lane == 0) L.cmax[c] = rest;
      rx = exact;
      ra = readlane_i64(la, at);
      rb = readlane_i64(lb, at);
      cd = readlane_i64(lc, at);
      return c * 64 + at;
    }
    if (lane == 0) L.cmax[c] = exact;  // the bound was stale: lower it, retry
    ss_wave_sync();
  }
}

template <int CAP, int THREADS, bool ORD = false>
__global__ void __launch_bounds__(THREADS) k_small_sweep(SmallSweepArgs A) {
  using LDS = SmallSweepLds<CAP, THREADS, ORD>;
  constexpr int NW = LDS::NW;
  // 16-byte aligned: the static LDS (sh_item) comes first, and the chunk
  // bounds of the ordered kernels take 64-bit LDS atomics, which need
  // naturally aligned addresses
  extern __shared__ __align__(16) char lds_raw[];
  LDS& L = *reinterpret_cast<LDS*>(lds_raw);
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  __shared__ int32_t sh_item;
  while (true) {
    if (threadIdx.x == 0) sh_item = atomicAdd(A.work, 1);
    __syncthreads();
    const int32_t item = sh_item;
    const int32_t na = *A.count_a;
    if (item >= na + *A.count_b) return;
    const int32_t g = item < na ? A.list_a[item] : A.list_b[item - na];
    const int32_t v0 = A.gvoff[g], ng = A.gn[g];
    const int64_t lam = A.lhat[g];
    const int64_t ebase = A.rp[v0];
    for (int i = threadIdx.x; i < ng; i += THREADS) {
      L.r[i] = 0;
      if constexpr (ORD) L.lt[i] = 0;
      A.fb_rs[v0 + i] = 0;
    }
    for (int i = threadIdx.x; i < (ng + 15) / 16; i += THREADS) L.st[i] = 0;
    for (int c = threadIdx.x; c < LDS::NC; c += THREADS) L.cmax[c] = 0;
    uint64_t h = A.seed * 0x9E3779B97F4A7C15ull + (uint64_t)g * 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
    if (threadIdx.x == 0) {
      L.first = (int32_t)(h % (uint64_t)ng);  // the start
      L.cap_head = L.cap_tail = 0;
      L.npairs = 0;
      L.nb = 0;
      L.stamp = 0;
    }
    // alpha = c(S) of the visited prefix S; kept by wave 0, lane 0
    int64_t alpha = 0, best_alpha = INT64_MAX, pend = 0;
    int32_t visited = 0, best_step = 0;
    __syncthreads();
    while (true) {
      if (wave == 0) {
        // fold the batch step just relaxed by the workgroup
        const int32_t pnb = L.nb;
        if (pnb > 0) {
          if (lane == 0) {
            int64_t sum = 0, in = 0;
            for (int k = 0; k < NW; ++k) { sum += L.wsum[k]; in += L.wint[k]; }
            alpha += sum - pend - in;
            visited += pnb;
            if (visited < ng && alpha < best_alpha) { best_alpha = alpha; best_step = L.stamp; }
          }
          const int32_t pb0 = L.b0;
          for (int k = lane; k < pnb; k += 64) ss_visited(L, L.capped[pb0 + k]);
          ss_wave_sync();
        }
        // single pops, by this wave alone, while no vertex is at the cap
        int32_t stamp = L.stamp;
        bool done = false;
        ss_wave_sync();
        bool crossed = L.cap_head != L.cap_tail;  // the batch relax filled the queue
        while (!crossed) {
          ss_wave_sync();
          int32_t xl = L.first;
          uint32_t rx = 0;  // r of the first vertex is 0: nothing is visited yet
          int64_t e0 = 0, e1 = 0, dx = 0;
          if (xl >= 0) {
            ss_wave_sync();
            if (lane == 0) L.first = -1;
            e0 = A.rp[v0 + xl];
            e1 = A.rp[v0 + xl + 1];
            dx = A.cdeg[v0 + xl];
          } else {
            xl = ss_select(L, A, v0, ng, rx, e0, e1, dx);
          }
          if (xl < 0) { done = true; break; }
          ++stamp;
          if (lane == 0) {
            ss_mark(L, xl);
            reinterpret_cast<int32_t*>(A.fb_rs + v0 + xl)[1] = stamp;
          }
          ss_wave_sync();
          int64_t rows = 0, internal = 0;  // unused here: the degree comes from cdeg
          for (int64_t base = e0; base < e1; base += 64) {
            const int64_t e = base + lane;
            const bool ok = e < e1;
            // loads outside branches (a load inside one is waited for at
            // its end, and the weight's load would wait for the column's)
            const int64_t ec = ok ? e : base;
            int32_t yv = A.col[ec], cv = A.w[ec];
            keep(cv);
            crossed |= ss_relax(L, A, v0, lam, ok, xl, ok ? yv - v0 : 0, ok ? cv : 0, rows, internal,
                                (uint32_t)stamp);
          }
          if (lane == 0) {
            alpha += dx - 2 * (int64_t)rx;
            visited += 1;
            if (visited < ng && alpha < best_alpha) { best_alpha = alpha; best_step = stamp; }
            ss_visited(L, xl);
          }
        }
        // publish the next batch: every vertex that reached the cap; mark it
        if (!done) ++stamp;
        if (lane == 0) {
          if (done) {
            L.nb = -1;
          } else {
            L.b0 = L.cap_head;
            L.nb = L.cap_tail - L.cap_head;
            L.cap_head = L.cap_tail;
          }
          L.stamp = stamp;
        }
        ss_wave_sync();
        if (!done) {
          const int32_t b0 = L.b0, nb = L.nb;
          int64_t r2 = 0;
          for (int k = lane; k < nb; k += 64) {
            const int32_t x = L.capped[b0 + k];
            ss_mark(L, x);
            reinterpret_cast<int32_t*>(A.fb_rs + v0 + x)[1] = stamp;
            r2 += 2 * (int64_t)L.r[x];
          }
          r2 = wave_sum_i64(r2);
          pend = r2;
        }
      }
      __syncthreads();
      const int32_t nb = L.nb;
      if (nb < 0) break;
      // batch relax: the batch's entries spread evenly over the workgroup, in
      // chunks of THREADS rows
      const int32_t b0 = L.b0;
      const uint32_t btick = (uint32_t)L.stamp;  // the batch's step
      int64_t rows = 0, internal = 0;
      for (int32_t c0 = 0; c0 < nb; c0 += THREADS) {
        const int32_t cn = min(THREADS, nb - c0);
        int32_t deg = 0;
        if ((int32_t)threadIdx.x < cn) {
          const int32_t x = v0 + L.capped[b0 + c0 + threadIdx.x];
          const int64_t a = A.rp[x];
          deg = (int32_t)(A.rp[x + 1] - a);
          L.bbase[threadIdx.x] = (int32_t)(a - ebase);
        }
        const int32_t incl = wave_incl_sum<int32_t>(deg);
        if (lane == 63) L.wtot[wave] = incl;
        __syncthreads();
        int32_t before = 0;
        for (int k = 0; k < wave; ++k) before += L.wtot[k];
        if ((int32_t)threadIdx.x < cn) L.boff[threadIdx.x] = before + incl - deg;
        if ((int32_t)threadIdx.x == cn - 1) L.boff[cn] = before + incl;
        __syncthreads();
        const int32_t total = L.boff[cn];
        for (int32_t i0 = 0; i0 < total; i0 += THREADS * SS_UNROLL) {
          // rows from LDS first, then every entry's loads together, outside
          // any branch (an idle slot reads the graph's first entry)
          int32_t ys[SS_UNROLL], cs[SS_UNROLL], xs[SS_UNROLL];
          int64_t es[SS_UNROLL];
#pragma unroll
          for (int u = 0; u < SS_UNROLL; ++u) {
            const int32_t i = i0 + u * THREADS + (int32_t)threadIdx.x;
            xs[u] = -1;
            es[u] = ebase;
            if (i < total) {
              int32_t lo = 0, hi = cn - 1;  // the row: last k with boff[k] <= i
              while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (L.boff[mid] <= i) lo = mid;
                else hi = mid - 1;
              }
              es[u] = ebase + L.bbase[lo] + (i - L.boff[lo]);
              xs[u] = L.capped[b0 + c0 + lo];
            }
          }
#pragma unroll
          for (int u = 0; u < SS_UNROLL; ++u) {
            ys[u] = A.col[es[u]];
            cs[u] = A.w[es[u]];
          }
#pragma unroll
          for (int u = 0; u < SS_UNROLL; ++u) {
            keep(ys[u]);
            keep(cs[u]);
            ys[u] = xs[u] >= 0 ? ys[u] - v0 : 0;
            cs[u] = xs[u] >= 0 ? cs[u] : 0;
          }
#pragma unroll
          for (int u = 0; u < SS_UNROLL; ++u)
            ss_relax(L, A, v0, lam, xs[u] >= 0, xs[u], ys[u], cs[u], rows, internal, btick);
        }
        __syncthreads();  // boff and bbase are reused by the next chunk
      }
      rows = wave_sum_i64(rows);
      internal = wave_sum_i64(internal);
      if (lane == 0) { L.wsum[wave] = rows; L.wint[wave] = internal; }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      A.npairs[g] = L.npairs;
      if (best_alpha < lam) {
        A.fb_k[g] = best_step;
        atomic_min_u64(A.best_alpha + g, ((uint64_t)best_alpha << 32) | (uint32_t)SWEEP_SID);
      }
      atomicAdd(A.ucount + g, L.npairs);
    }
    __syncthreads();
  }
}

// Unite the pairs recorded by the small sweeps: graph g's pairs are
// (capx[v0 + i], capq[v0 + i]) for i < npairs[g].
__global__ void k_small_sweep_unite(const int32_t* list, const int32_t* list_count, const int32_t* gvoff,
                                    const int32_t* npairs, const int32_t* capq, const int32_t* capx,
                                    int32_t* parent) {
  const int32_t cnt = *list_count;
  for (int32_t item = blockIdx.x; item < cnt; item += gridDim.x) {
    const int32_t g = list[item];
    const int32_t v0 = gvoff[g], np = npairs[g];
    for (int32_t i = threadIdx.x; i < np; i += blockDim.x) uf_union(parent, capx[v0 + i], capq[v0 + i]);
  }
}

}  // namespace mc
