// Full-graph CAPFOREST with bounded keys (appendix Algorithm 3 with the cap
// of Lemma 1, section "Bounded Priority Queues"), run in parallel over ties.
//
// With keys capped at lambda-hat, every frontier vertex whose r has reached
// the cap is a maximum of the priority queue, and no relaxation can lift any
// key above the cap.  So all capped frontier vertices can be visited as one
// batch: any order of them is a legal maximum-adjacency order, and every
// value q(e) = r(y) produced while the batch is relaxed (atomic adds give
// each edge the value of some order of the batch) is the q(e) of such a
// legal run.  Vertices below the cap are popped one at a time from a bucket
// queue, exactly as the sequential routine does.  The crossing rule
// r(y) < lambda-hat <= r(y) + c(e) unites x and y; each vertex crosses at most
// once, and crossing vertices form the next batch (a FIFO of batches).
//
// alpha = c(S) of the visited set is tracked at batch boundaries:
//   alpha' = alpha + sum_{x in B} (c(x) - 2 r(x)) - 2 w(edges inside B).
//
// A persistent single-workgroup kernel runs the single pops and the small
// batches; a batch larger than the hand-off size goes back to the host,
// which runs it grid-wide (mark, relax, finish) and then rebuilds the bucket
// queue exactly from the frontier (one counting sort), so that the lazy
// entries made stale by a large batch never have to be walked.
#pragma once
#include "dev.h"
#include "rows.h"

namespace mc {

constexpr int SWEEP_THREADS = 1024;
constexpr int SWEEP_BUCKETS = 4096;  // bucket queue for keys below the cap
constexpr int32_t SWEEP_SID = 0x7FFFFFFF;
constexpr int RB_TILE = 4096;        // vertices per workgroup in the rebuild
constexpr int SWEEP_PHASES = 8;      // per-phase step counters kept
constexpr int TAIL_MAX_FORKS = 1024; // concurrent scans of a sweep's tail

enum : int32_t { SW_RUNNING = 0, SW_DONE = 1, SW_BIG = 2, SW_TAIL = 3 };

struct SweepCtl {
  int32_t cap_head, cap_tail;  // capped FIFO: [head, tail) is the pending batch
  int32_t visited;
  int32_t step;                // batches so far (visit order stamps)
  int64_t alpha;
  int64_t best_alpha;
  int32_t best_step;
  int32_t status;
  int64_t pool_next;
  int64_t batch_sum;           // grid-wide batch: sum c(x) - 2 r(x)
  int64_t batch_internal;      // grid-wide batch: 2 w(inside)
  int64_t batch_deg;           // grid-wide batch: sum of row lengths
  int32_t singles, batches, big_batches, rebuilds;
  // per phase (phase k: the sequential kernel's steps after k grid-wide
  // batches, the last phase holding all later ones): single pops, batches
  // and crossings (one union each) made by those steps
  int32_t ph_singles[SWEEP_PHASES], ph_batches[SWEEP_PHASES], ph_cross[SWEEP_PHASES];
  // the tail's concurrent scans (tail.h): list length and cursor, pops, and
  // the best prefix cut (alpha << 32 | process)
  int32_t tail_total, tail_cursor, tail_pops, free_count;
  uint64_t tail_best;
  int64_t tail_rows;           // entries of the rows the tail relaxed
  int64_t seq_rows;            // ... and the sequential kernel
  int64_t rows_done;           // entries in the rows of every visited vertex
  int64_t pull_alpha;          // pull form of a grid-wide batch: c(S + B), summed
  int32_t seg_unsorted;        // a batch row met by the range-owned form lists
                               // its neighbours out of ascending order
  int32_t count_err;           // a pull batch's free vertices differed from
                               // the count the host derived (never expected)
  uint64_t bitmap[SWEEP_BUCKETS / 64];
  int32_t head[SWEEP_BUCKETS];     // recent pushes (lists through the pool)
  int32_t seg_cur[SWEEP_BUCKETS];  // rebuilt segments of seg[]: unread part
  int32_t seg_end[SWEEP_BUCKETS];
  int32_t fill[SWEEP_BUCKETS];     // rebuild scratch
  int32_t tail_k[TAIL_MAX_FORKS];  // per tail process: pops of its best prefix
};

struct SweepArgs {
  const int64_t* rp;
  const int32_t* col;
  const int32_t* w;
  const int64_t* cdeg;
  int32_t* parent;
  uint64_t* rs;      // per vertex: r in the low 32 bits, the visit stamp (batch
                     // number, 0 = not visited) in the high 32 bits, so one
                     // access reads both; a frontier vertex is an unvisited
                     // one with r > 0 (or the start)
  int32_t* capq;     // capped FIFO (each vertex enters at most once)
  int32_t* capx;     // the vertex whose edge made capq[i] cross (united later)
  int2* pool;        // bucket entries (vertex, next)
  int64_t pool_cap;
  int32_t* seg;      // bucket segments written by the rebuild
  SweepCtl* ctl;
  int32_t v0, ng;    // graph vertex range
  int64_t lam;       // lambda-hat for this round
  int32_t shift;     // bucket = key >> shift
  int32_t nwords;    // bitmap words in use
  int32_t nb;        // buckets in use
  int32_t big;       // batches above this size go grid-wide
  int64_t big_entries;  // ... and so do batches whose rows hold more entries
  int32_t start;     // the first vertex (global id)
  int32_t g;         // the graph
  int32_t tail_min;  // hand the tail to concurrent scans once at most tail_max
  int32_t tail_max;  // and at least tail_min vertices are left (0: never)
};

// The kernels that read their arguments from the per-graph argument array
// work on this view of them, with every array typed as global memory.
struct SweepDev {
  const MC_GLOBAL int64_t* rp;
  const MC_GLOBAL int32_t* col;
  const MC_GLOBAL int32_t* w;
  const MC_GLOBAL int64_t* cdeg;
  MC_GLOBAL int32_t* parent;
  MC_GLOBAL uint64_t* rs;
  MC_GLOBAL int32_t* capq;
  MC_GLOBAL int32_t* capx;
  MC_GLOBAL int2* pool;
  int64_t pool_cap;
  MC_GLOBAL int32_t* seg;
  MC_GLOBAL SweepCtl* ctl;
  int32_t v0, ng;
  int64_t lam;
  int32_t shift, nwords, nb, big;
  int64_t big_entries;
  int32_t start, g;
  int32_t tail_min, tail_max;
};

__device__ __forceinline__ SweepDev dev_view(const SweepArgs& a) {
  return SweepDev{(const MC_GLOBAL int64_t*)a.rp, (const MC_GLOBAL int32_t*)a.col, (const MC_GLOBAL int32_t*)a.w,
                  (const MC_GLOBAL int64_t*)a.cdeg, (MC_GLOBAL int32_t*)a.parent, (MC_GLOBAL uint64_t*)a.rs,
                  (MC_GLOBAL int32_t*)a.capq, (MC_GLOBAL int32_t*)a.capx,
                  (MC_GLOBAL int2*)a.pool, a.pool_cap, (MC_GLOBAL int32_t*)a.seg, (MC_GLOBAL SweepCtl*)a.ctl,
                  a.v0, a.ng, a.lam, a.shift, a.nwords, a.nb, a.big, a.big_entries, a.start, a.g,
                  a.tail_min, a.tail_max};
}

// The packed (r, stamp) word: r never exceeds the vertex's weighted degree
// (each entry adds to it once), which is at most INT32_MAX, so an add to r
// never carries into the stamp.
__device__ __forceinline__ int32_t rs_r(uint64_t u) { return (int32_t)(uint32_t)u; }
__device__ __forceinline__ int32_t rs_stamp(uint64_t u) { return (int32_t)(u >> 32); }
__device__ __forceinline__ int32_t* rs_stamp_ptr(uint64_t* p) { return (int32_t*)p + 1; }
__device__ __forceinline__ MC_GLOBAL int32_t* rs_stamp_ptr(MC_GLOBAL uint64_t* p) { return (MC_GLOBAL int32_t*)p + 1; }

__device__ __forceinline__ uint64_t* pool_word(int2* p) { return (uint64_t*)p; }
__device__ __forceinline__ MC_GLOBAL uint64_t* pool_word(MC_GLOBAL int2* p) { return (MC_GLOBAL uint64_t*)p; }

// The queue and FIFO bookkeeping, addressed through generic pointers: the
// persistent workgroup works on LDS copies, the grid-wide kernels on the
// global SweepCtl.
constexpr int SWEEP_RING = 1024;   // newest capped-FIFO entries mirrored in LDS
constexpr int POOL_RING = 2048;    // newest bucket entries mirrored in LDS

struct SweepQ {
  int32_t* cap_head;
  int32_t* cap_tail;
  int64_t* pool_next;
  uint64_t* bitmap;
  int32_t* head;
  int32_t* seg_cur;
  int32_t* seg_end;
  // persistent kernel only (nullptr elsewhere): LDS mirrors of capq[i] and
  // of its row bounds at i % SWEEP_RING
  int32_t* ring;
  int64_t* ring_a;
  int64_t* ring_b;
  // wave-0 steps of the persistent kernel only: LDS mirror of pool[i] at
  // i % POOL_RING, valid for i >= max(*pring_lo, *pool_next - POOL_RING)
  uint64_t* pring;
  int64_t* pring_lo;
  // wave-0 steps only: the last 64-entry chunk of a rebuilt segment read
  // from global memory (sc_hdr: bucket or -1, first index)
  int32_t* sc_v;
  int32_t* sc_hdr;
};

__device__ __forceinline__ SweepQ global_q(SweepCtl* c) {
  return SweepQ{&c->cap_head, &c->cap_tail, &c->pool_next, c->bitmap, c->head, c->seg_cur, c->seg_end,
                nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
}

__device__ __forceinline__ bool pool_mirrored(const SweepQ& q, int64_t idx) {
  if (!q.pring) return false;
  const int64_t lo = *q.pool_next - POOL_RING;
  return idx >= *q.pring_lo && idx >= lo;
}

template <class SA>
__device__ __forceinline__ int2 pool_at(const SA& A, const SweepQ& q, int32_t idx) {
  const uint64_t u = pool_mirrored(q, idx) ? q.pring[idx & (POOL_RING - 1)] : ld_relaxed(pool_word(A.pool + idx));
  return make_int2((int32_t)(uint32_t)u, (int32_t)(u >> 32));
}

template <class SA>
__device__ __forceinline__ void pool_put(const SA& A, const SweepQ& q, int64_t idx, int32_t v, int32_t next) {
  const uint64_t u = ((uint64_t)(uint32_t)next << 32) | (uint32_t)v;
  st_relaxed(pool_word(A.pool + idx), u);
  if (pool_mirrored(q, idx)) q.pring[idx & (POOL_RING - 1)] = u;
}

// Relax edge (x, y, c) while batch `stamp` is being visited.  Every lane of
// the wave calls this (act = false for idle lanes) so that queue and counter
// updates are aggregated per wave.  Returns the weight to add to the
// batch-internal sum (edge inside the batch).
//
// member: y is known to be in the batch (the caller compared it with the
// batch's vertices), so neither its stamp nor its r is touched.
//
// unvisited: (grid-wide batches) y is known to be unvisited, so its stamp is
// not read.
// rsum (PUSH only) adds the weight of an edge into a vertex visited before
// the batch: summed over the batch's rows it is the batch's weight to the
// visited set, which alpha needs (a capped vertex's own r stops being exact
// once the grid-wide relax skips the adds that reach it after its crossing).
template <bool PUSH = true, class SA>
__device__ __forceinline__ int64_t sweep_relax(const SA& A, const SweepQ& q, int32_t x, int32_t y,
                                               int32_t c, int32_t stamp, bool act, int64_t& rsum,
                                               int32_t* wbuf = nullptr, int32_t* wcnt = nullptr,
                                               bool member = false, bool unvisited = false) {
  const int lane = lane_id();
  int64_t internal = 0;
  bool cross = false, push = false;
  int64_t nw = 0, ya = 0, yb = 0;
  if (act && y == x) act = false;
  if (act && PUSH && member) {
    internal = c;
  } else if (act && PUSH) {
    // the sequential kernel is latency-bound: the visit stamp, the add and
    // the row bounds (kept with the FIFO entry if y crosses) are independent,
    // so all are in flight at once.  A visited vertex's r is never read
    // again (alpha takes r(x) of a batch vertex before its batch's rows add
    // to it, or the caller keeps batch vertices out of the adds), so adding
    // to it is harmless
    const uint64_t prev = atomic_add(A.rs + y, (uint64_t)(uint32_t)c);
    const int32_t vs = rs_stamp(prev), old = rs_r(prev);
    if (q.ring_a) {
      ya = A.rp[y];
      yb = A.rp[y + 1];
    }
    if (vs != 0) {
      if (vs == stamp) internal = c;
      else rsum += c;
    } else {
      nw = (int64_t)old + c;
      cross = old < A.lam && A.lam <= nw;
      push = nw < A.lam;
    }
  } else if (act) {
    // grid-wide batches are bandwidth-bound: no add for visited vertices
    // (the stamps do not change while a grid-wide batch is relaxed)
    const int32_t vs = unvisited ? 0 : rs_stamp(ld_relaxed(A.rs + y));
    if (vs != 0) {
      if (vs == stamp) internal = c;
    } else {
      const int32_t old = rs_r(atomic_add(A.rs + y, (uint64_t)(uint32_t)c));
      nw = (int64_t)old + c;
      cross = old < A.lam && A.lam <= nw;
    }
  }
  // crossings: unite, and append y to the capped FIFO (through a per-wave
  // LDS buffer when one is given)
  const uint64_t cm = ballot(cross);
  if (cm && wbuf) {
    const int32_t at = *wcnt;
    if (cross) {
      const int32_t k = at + popc64(cm & lanemask_lt());
      wbuf[2 * k] = y;
      wbuf[2 * k + 1] = x;
    }
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) *wcnt = at + popc64(cm);
    __builtin_amdgcn_wave_barrier();
  } else if (cm) {
    const int leader = __builtin_ctzll(cm);
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(q.cap_tail, popc64(cm));
    base = bcast(base, leader);
    if (cross) {
      const int32_t at = base + popc64(cm & lanemask_lt());
      A.capq[at] = y;
      A.capx[at] = x;
      if (q.ring) {
        q.ring[at & (SWEEP_RING - 1)] = y;
        q.ring_a[at & (SWEEP_RING - 1)] = ya;
        q.ring_b[at & (SWEEP_RING - 1)] = yb;
      }
    }
  }
  // pushes below the cap: one pool reservation per wave, then one list
  // exchange per pushing lane, all in one instruction: lanes that push to
  // the same bucket are applied one after another, each receiving the entry
  // the previous one left, so every bucket's list stays a chain (no loop
  // over the distinct buckets)
  const uint64_t pm = PUSH ? ballot(push) : 0ull;
  if (pm) {
    const int leader = __builtin_ctzll(pm);
    int64_t pbase = 0;
    if (lane == leader)
      pbase = (int64_t)atomicAdd((unsigned long long*)q.pool_next, (unsigned long long)popc64(pm));
    pbase = bcast(pbase, leader);
    const int64_t idx = pbase + popc64(pm & lanemask_lt());
    if (push && idx < A.pool_cap) {
      const int32_t b = (int32_t)(nw >> A.shift);
      const int32_t old_head = atomicExch(&q.head[b], (int32_t)idx);
      atomicOr((unsigned long long*)&q.bitmap[b >> 6], 1ull << (b & 63));
      pool_put(A, q, idx, y, old_head);
    }
  }
  return internal;
}

// Reset each graph's range and queue: graph blockIdx.y of the argument array.
__global__ void k_sweep_init(const SweepArgs* args) {
  const SweepDev A = dev_view(args[blockIdx.y]);
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < A.ng; i += nth) A.rs[A.v0 + i] = 0;
  for (int64_t i = tid; i < SWEEP_BUCKETS; i += nth) {
    A.ctl->head[i] = -1;
    A.ctl->seg_cur[i] = 0;
    A.ctl->seg_end[i] = 0;
  }
  for (int64_t i = tid; i < SWEEP_BUCKETS / 64; i += nth) A.ctl->bitmap[i] = 0;
  for (int64_t i = tid; i < SWEEP_PHASES; i += nth) {
    A.ctl->ph_singles[i] = 0;
    A.ctl->ph_batches[i] = 0;
    A.ctl->ph_cross[i] = 0;
  }
  if (tid == 0) {
    MC_GLOBAL SweepCtl* c = A.ctl;
    c->cap_head = c->cap_tail = 0;
    c->visited = 0;
    c->step = 0;
    c->alpha = 0;
    c->best_alpha = INT64_MAX;
    c->best_step = 0;
    c->status = SW_RUNNING;
    c->pool_next = 1;
    c->batch_sum = c->batch_internal = 0;
    c->batch_deg = 0;
    c->singles = c->batches = c->big_batches = c->rebuilds = 0;
    c->tail_total = c->tail_cursor = c->tail_pops = c->free_count = 0;
    c->tail_best = ~0ull;
    c->tail_rows = c->seq_rows = c->rows_done = c->pull_alpha = 0;
    c->seg_unsorted = 0;
    c->count_err = 0;
  }
}

// The start of every graph in bucket 0 (thread i: graph i of k).
__global__ void k_sweep_seed(const SweepArgs* args, int32_t k) {
  for (int64_t i = gtid(); i < k; i += gstride()) {
    const SweepDev A = dev_view(args[i]);
    *pool_word(A.pool) = (~0ull << 32) | (uint32_t)A.start;  // (vertex, next = -1)
    A.ctl->head[0] = 0;
    A.ctl->bitmap[0] = 1ull;
  }
}

__device__ __forceinline__ void sweep_close_batch(SweepCtl* c, int32_t ng, int64_t sum, int64_t internal,
                                                  int32_t size, int32_t stamp) {
  c->alpha += sum - internal;
  c->visited += size;
  if (c->visited < ng && c->alpha < c->best_alpha) {
    c->best_alpha = c->alpha;
    c->best_step = stamp;
  }
}

// A bucket entry is live if its vertex is unvisited and its r still maps to
// the bucket (u: the vertex's packed word).
template <class SA>
__device__ __forceinline__ bool live_word(const SA& A, uint64_t u, int32_t v, int32_t b, int32_t& key) {
  key = rs_r(u);
  return v >= 0 && rs_stamp(u) == 0 && (int64_t)key < A.lam && (key >> A.shift) == b;
}
template <class SA>
__device__ __forceinline__ bool live_in_bucket(const SA& A, int32_t v, int32_t b, int32_t& key) {
  // no branch around the load (v < 0, an empty slot, reads the start's word)
  return live_word(A, ld_relaxed(A.rs + (v >= 0 ? v : A.start)), v, b, key);
}

// What the single-pop step needs of the popped vertex besides its id: its
// row bounds, its weighted degree and its r (the key it was popped with).
struct PopRow {
  int64_t ra, rb, cd;
  int32_t key;
};

template <class SA>
__device__ __forceinline__ void pop_row_load(const SA& A, int32_t x, int32_t key, PopRow& pr) {
  pr.ra = A.rp[x];
  pr.rb = A.rp[x + 1];
  pr.cd = A.cdeg[x];
  pr.key = key;
}

// A candidate v of bucket b (v < 0: an empty slot): its liveness word and
// its row loaded together, and all four taken as used at once, so they
// complete in one round trip (left to itself, the compiler sinks the row
// loads into the branch taken for a live candidate, after the liveness
// result).
template <class SA>
__device__ __forceinline__ bool pop_candidate(const SA& A, int32_t v, int32_t b, PopRow& cand) {
  const int32_t vx = v >= 0 ? v : A.start;
  uint64_t u = ld_relaxed(A.rs + vx);
  pop_row_load(A, vx, 0, cand);
  asm volatile("" : "+v"(u), "+v"(cand.ra), "+v"(cand.rb), "+v"(cand.cd));
  return live_word(A, u, v, b, cand.key);
}

// Single pop by wave 0: the highest non-empty bucket (bitmap words read by
// the lanes, one each); in it, the recent-push list (lane 0 walks it,
// dropping stale entries, with the row of each candidate loaded alongside
// its liveness) and then the rebuilt segment (64 entries per read, cursor
// only moves forward).  With one key per bucket the first live entry is a
// maximum; with wider buckets the largest live key of the whole bucket is
// taken (the segment entry is then tombstoned).  -1: queue empty.  On
// success pr describes the vertex (the same in every lane).
template <class SA>
__device__ int32_t sweep_pop_wave0(const SA& A, const SweepQ& q, PopRow& pr) {
  const int lane = lane_id();
  while (true) {
    uint64_t word = lane < A.nwords ? ld_relaxed(&q.bitmap[lane]) : 0ull;
    uint64_t m = ballot(word != 0);
    if (m == 0) return -1;
    const int bw = 63 - __builtin_clzll(m);
    const uint64_t wv = bcast(word, bw);
    const int b = bw * 64 + 63 - __builtin_clzll(wv);
    int32_t x = -1;
    if (A.shift == 0) {
      if (lane == 0) {
        int32_t idx = ld_relaxed(&q.head[b]);
        while (idx >= 0) {
          int2 e = pool_at(A, q, idx);
          idx = e.y;
          PopRow cand;
          if (pop_candidate(A, e.x, b, cand)) { x = e.x; pr = cand; break; }
        }
        st_relaxed(&q.head[b], idx);
      }
      x = bcast(x, 0);
      if (x >= 0) {
        pr.ra = bcast(pr.ra, 0);
        pr.rb = bcast(pr.rb, 0);
        pr.cd = bcast(pr.cd, 0);
        pr.key = bcast(pr.key, 0);
        return x;
      }
      // the segment, from the cursor on, 64 entries per pass (a chunk read
      // from global memory stays in LDS for the next pops); every lane
      // loads its entry's row with the liveness
      int32_t cur = ld_relaxed(&q.seg_cur[b]);
      const int32_t end = ld_relaxed(&q.seg_end[b]);
      while (cur < end) {
        const bool cached = q.sc_v && q.sc_hdr[0] == b && cur >= q.sc_hdr[1] && cur < q.sc_hdr[1] + 64;
        const int32_t base = cached ? q.sc_hdr[1] : cur;
        const int32_t lim = min(base + 64, end);
        const int32_t i = cur + lane;
        int32_t v = -1;
        if (cached) {
          if (i < lim) v = q.sc_v[i - base];
        } else {
          if (i < lim) v = ld_relaxed(A.seg + i);
          if (q.sc_v) {
            q.sc_v[lane] = v;
            if (lane == 0) { q.sc_hdr[0] = b; q.sc_hdr[1] = cur; }
          }
        }
        PopRow cand{0, 0, 0, 0};
        const bool live = pop_candidate(A, v, b, cand);
        const uint64_t ok = ballot(live);
        if (ok) {
          const int first = __builtin_ctzll(ok);
          x = __builtin_amdgcn_readlane(v, first);
          pr.ra = readlane_i64(cand.ra, first);
          pr.rb = readlane_i64(cand.rb, first);
          pr.cd = readlane_i64(cand.cd, first);
          pr.key = __builtin_amdgcn_readlane(cand.key, first);
          cur += first + 1;
          break;
        }
        cur = lim;
      }
      if (lane == 0) st_relaxed(&q.seg_cur[b], cur < end ? cur : end);
      if (x >= 0) return x;
    } else {
      // wide bucket: exact maximum over the list and the segment
      int64_t best_key = -1;
      int32_t best_v = -1, best_idx = -1, best_prev = -1;
      if (lane == 0) {
        int32_t idx = ld_relaxed(&q.head[b]), prev = -1;
        while (idx >= 0) {
          int2 e = pool_at(A, q, idx);
          int32_t k = 0;
          if (!live_in_bucket(A, e.x, b, k)) {
            if (prev < 0) st_relaxed(&q.head[b], e.y);
            else pool_put(A, q, prev, pool_at(A, q, prev).x, e.y);
          } else {
            if (k > best_key) { best_key = k; best_v = e.x; best_idx = idx; best_prev = prev; }
            prev = idx;
          }
          idx = e.y;
        }
      }
      best_key = bcast(best_key, 0);
      best_v = bcast(best_v, 0);
      int64_t seg_best = -1;
      int32_t seg_pos = -1;
      const int32_t cur0 = ld_relaxed(&q.seg_cur[b]);
      const int32_t end = ld_relaxed(&q.seg_end[b]);
      for (int32_t base = cur0; base < end; base += 64) {
        const int32_t i = base + lane;
        const int32_t v = i < end ? ld_relaxed(A.seg + i) : -1;
        int32_t k = 0;
        if (live_in_bucket(A, v, b, k) && k > seg_best) { seg_best = k; seg_pos = i; }
      }
      const uint64_t packed =
          wave_max_u64(seg_best < 0 ? 0ull : (((uint64_t)(seg_best + 1) << 32) | (uint32_t)seg_pos));
      int32_t key = 0;
      if (packed != 0 && (int64_t)(packed >> 32) - 1 > best_key) {
        const int32_t pos = (int32_t)(uint32_t)packed;
        x = ld_relaxed(A.seg + pos);
        key = (int32_t)(packed >> 32) - 1;
        if (lane == 0) st_relaxed(A.seg + pos, -1);
      } else if (best_v >= 0) {
        x = best_v;
        key = (int32_t)best_key;
        if (lane == 0) {
          const int32_t nx = pool_at(A, q, best_idx).y;
          if (best_prev < 0) st_relaxed(&q.head[b], nx);
          else pool_put(A, q, best_prev, pool_at(A, q, best_prev).x, nx);
        }
      }
      if (x >= 0) {
        pop_row_load(A, x, key, pr);
        return x;
      }
      if (lane == 0) {
        st_relaxed(&q.head[b], -1);
        st_relaxed(&q.seg_cur[b], end);
      }
    }
    // the bucket holds no live entry
    if (lane == 0) atomicAnd((unsigned long long*)&q.bitmap[bw], ~(1ull << (b & 63)));
  }
}

constexpr int FAST_BATCH = 32;     // batches up to this size run on wave 0 alone
constexpr int64_t FAST_DEG = 2048;  // single pops with rows up to this run on wave 0 alone

// Relax the rows [ra, rb) of `cnt` batch vertices held by lanes 0..cnt-1 of
// `xs` with one wave; returns the batch-internal weight of this wave's lanes.
// Batch membership is decided by comparing with xs, so the batch's visit
// stamps need not be visible yet.
template <class SA>
__device__ __forceinline__ int64_t wave_relax_known(const SA& A, const SweepQ& q, int32_t xs, int64_t ra,
                                                    int64_t rb, int cnt, int32_t stamp, int64_t& rsum) {
  const int lane = lane_id();
  int64_t internal = 0;
  for (int j = 0; j < cnt; ++j) {
    const int32_t x = __builtin_amdgcn_readlane(xs, j);
    const int64_t e0 = readlane_i64(ra, j), e1 = readlane_i64(rb, j);
    for (int64_t base = e0; base < e1; base += 64) {
      const int64_t e = base + lane;
      const bool act = e < e1;
      // loads outside branches (a load inside one is waited for at its end)
      const int64_t ec = act ? e : base;
      int32_t yv = A.col[ec], cv = A.w[ec];
      keep(cv);
      const int32_t y = act ? yv : 0;
      const int32_t c = act ? cv : 0;
      bool member = false;  // with one vertex, y == x is a self-loop, skipped anyway
      for (int k = 0; k < cnt && cnt > 1; ++k) member |= y == __builtin_amdgcn_readlane(xs, k);
      internal += sweep_relax(A, q, x, y, c, stamp, act, rsum, nullptr, nullptr, member);
    }
  }
  return internal;
}

// The persistent workgroup.  Wave 0 drives: it pops, and runs single pops
// with short rows and small batches by itself.  Wide steps (a long row, a
// larger batch) are shared with the other waves, which wait at a barrier for
// the next command.  Exits with SW_DONE (queue empty) or SW_BIG (a batch
// larger than A.big, or with more than A.big_entries entries in its rows, is
// pending; cap_head..cap_tail untouched).
enum : int32_t { CMD_EXIT_DONE = 0, CMD_BATCH = 1, CMD_EXIT_BIG = 2, CMD_SINGLE = 3, CMD_EXIT_TAIL = 4 };

__global__ void __launch_bounds__(SWEEP_THREADS) k_sweep_seq(const SweepArgs* args, const int32_t* run) {
  // one workgroup per graph still running: graph run[blockIdx.x]
  const SweepDev A = dev_view(args[run[blockIdx.x]]);
  __shared__ int32_t sh_x, sh_cmd, sh_h, sh_t, sh_stamp;
  // a wide batch chunk: its vertices, row starts and entry offsets
  __shared__ int32_t sh_bx[SWEEP_THREADS], sh_boff[SWEEP_THREADS + 1], sh_wtot[SWEEP_THREADS / 64];
  __shared__ int64_t sh_bbase[SWEEP_THREADS];
  __shared__ int64_t sh_sum[SWEEP_THREADS / 64], sh_int[SWEEP_THREADS / 64];
  // queue state, resident in LDS while this workgroup runs
  __shared__ int32_t l_head[SWEEP_BUCKETS], l_cur[SWEEP_BUCKETS], l_end[SWEEP_BUCKETS];
  __shared__ uint64_t l_bitmap[SWEEP_BUCKETS / 64];
  __shared__ int32_t l_cap_head, l_cap_tail;
  __shared__ int64_t l_pool_next;
  __shared__ int32_t l_ring[SWEEP_RING];
  __shared__ int64_t l_ring_a[SWEEP_RING], l_ring_b[SWEEP_RING];
  __shared__ uint64_t l_pring[POOL_RING];
  __shared__ int64_t l_pring_lo;
  __shared__ int32_t l_sc_v[64], l_sc_hdr[2];
  MC_GLOBAL SweepCtl* c = A.ctl;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int nwaves = SWEEP_THREADS / 64;
  for (int i = threadIdx.x; i < A.nb; i += SWEEP_THREADS) {
    l_head[i] = c->head[i];
    l_cur[i] = c->seg_cur[i];
    l_end[i] = c->seg_end[i];
  }
  for (int i = threadIdx.x; i < SWEEP_BUCKETS / 64; i += SWEEP_THREADS) l_bitmap[i] = c->bitmap[i];
  // bookkeeping of thread 0 (the only thread that closes batches)
  int32_t step = 0, visited = 0, best_step = 0, singles = 0, batches = 0;
  int32_t singles0 = 0, batches0 = 0, tail0 = 0;
  int64_t alpha = 0, best_alpha = 0, seq_rows = 0;
  if (threadIdx.x == 0) {
    l_cap_head = c->cap_head;
    l_cap_tail = c->cap_tail;
    l_pool_next = c->pool_next;
    l_pring_lo = c->pool_next;  // entries from before this launch are not mirrored
    l_sc_hdr[0] = -1;           // segments were rebuilt since the last launch
    step = c->step;
    visited = c->visited;
    alpha = c->alpha;
    best_alpha = c->best_alpha;
    best_step = c->best_step;
    singles = c->singles;
    batches = c->batches;
    singles0 = singles;
    batches0 = batches;
    tail0 = c->cap_tail;
  }
  __syncthreads();
  // q: steps shared by all waves; qf: wave-0 steps, which also mirror new
  // bucket entries in LDS (only one wave pushes there)
  const SweepQ q{&l_cap_head, &l_cap_tail, &l_pool_next, l_bitmap, l_head, l_cur, l_end,
                 l_ring, l_ring_a, l_ring_b, nullptr, nullptr, nullptr, nullptr};
  SweepQ qf = q;
  qf.pring = l_pring;
  qf.pring_lo = &l_pring_lo;
  qf.sc_v = l_sc_v;
  qf.sc_hdr = l_sc_hdr;
  // FIFO entries appended before this launch are not in the ring
  const int32_t ring_lo = ld_relaxed(&l_cap_tail);
  const bool tail_ok = A.tail_min > 0 && A.shift == 0 && c->big_batches > 0;
  // FIFO entry i (below tail) and its row bounds
  auto fifo_row = [&](int32_t i, int32_t tail, int64_t& a, int64_t& b) -> int32_t {
    if (i >= ring_lo && i >= tail - SWEEP_RING) {
      a = l_ring_a[i & (SWEEP_RING - 1)];
      b = l_ring_b[i & (SWEEP_RING - 1)];
      return l_ring[i & (SWEEP_RING - 1)];
    }
    const int32_t x = ld_relaxed(A.capq + i);
    a = A.rp[x];
    b = A.rp[x + 1];
    return x;
  };
  auto close = [&](int64_t sum, int64_t internal, int32_t size, int32_t stamp) {
    alpha += sum - internal;
    visited += size;
    if (visited < A.ng && alpha < best_alpha) {
      best_alpha = alpha;
      best_step = stamp;
    }
  };
  int exit_cmd = -1;
  while (true) {
    if (wave == 0) {
      // fast loop: steps that one wave handles without barriers
      int cmd = -1;
      while (cmd < 0) {
        const int32_t h = ld_relaxed(q.cap_head), t = ld_relaxed(q.cap_tail);
        const int32_t stamp = bcast(step, 0) + 1;
        if (t > h) {
          const int32_t size = t - h;
          if (size > A.big) { cmd = CMD_EXIT_BIG; break; }
          // the rows' total length decides too: a few hubs can hold more
          // entries than one workgroup (or one wave) should relax.  The
          // first 64 vertices keep their row bounds for the relax.
          int64_t entries = 0, ra = 0, rb = 0;
          int32_t xs = -1;
          for (int32_t i = lane; i < size; i += 64) {
            int64_t a, b;
            const int32_t x = fifo_row(h + i, t, a, b);
            entries += b - a;
            if (i == lane) { xs = x; ra = a; rb = b; }
          }
          entries = wave_sum_i64_dpp(entries);
          if (entries > A.big_entries) { cmd = CMD_EXIT_BIG; break; }
          if (lane == 0) seq_rows += entries;
          if (size > FAST_BATCH || entries > FAST_DEG) {
            if (lane == 0) { sh_h = h; sh_t = t; sh_stamp = stamp; step = stamp; batches += 1; }
            cmd = CMD_BATCH;
            break;
          }
          // mark; the batch's own edges are found by comparing with xs, and
          // its r values are read while the rows are relaxed (no add reaches
          // a batch vertex in this step)
          // (loads outside any branch: a load inside a branch is waited for
          // at the branch's end)
          const int32_t xq = lane < size ? xs : __builtin_amdgcn_readlane(xs, 0);
          const int64_t cd = A.cdeg[xq];
          if (lane < size) st_relaxed(rs_stamp_ptr(A.rs + xs), stamp);
          // sum of c(x) - 2 r(x) over the batch, r(x) = weight to the visited set
          int64_t rsum = 0;
          int64_t internal = wave_relax_known(A, qf, xs, ra, rb, size, stamp, rsum);
          int64_t sum = (lane < size ? cd : 0) - 2 * rsum;
          sum = wave_sum_i64_dpp(sum);
          internal = wave_sum_i64_dpp(internal);
          if (lane == 0) {
            step = stamp;
            batches += 1;
            *q.cap_head = t;
            close(sum, internal, size, stamp);
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        } else {
          // below the cap after a grid-wide batch with few vertices left:
          // the tail goes to concurrent scans (tail.h)
          if (tail_ok) {
            const int32_t left = A.ng - bcast(visited, 0);
            if (left >= A.tail_min && left <= A.tail_max) { cmd = CMD_EXIT_TAIL; break; }
          }
          PopRow pr;
          const int32_t x = sweep_pop_wave0(A, qf, pr);
          if (x < 0) { cmd = CMD_EXIT_DONE; break; }
          const int64_t ra = pr.ra, rb = pr.rb;
          const int64_t deg = rb - ra;
          if (deg > A.big_entries) {
            // a row longer than one workgroup should relax: relaxed grid-wide,
            // as a batch of this one vertex (the FIFO is empty here); its
            // pair with itself unites nothing
            if (lane == 0) {
              const int32_t t = *q.cap_tail;
              A.capq[t] = x;
              A.capx[t] = x;
              *q.cap_tail = t + 1;
            }
            cmd = CMD_EXIT_BIG;
            break;
          }
          if (lane == 0) seq_rows += deg;
          int64_t sum = 0;
          if (lane == 0) {
            st_relaxed(rs_stamp_ptr(A.rs + x), stamp);
            sum = pr.cd - 2 * (int64_t)pr.key;
          }
          if (deg > FAST_DEG) {
            if (lane == 0) { sh_x = x; sh_stamp = stamp; step = stamp; singles += 1; sh_sum[0] = sum; }
            cmd = CMD_SINGLE;
            break;
          }
          // a single vertex has no edge inside its batch (self-loops skipped);
          // its r (below the cap, every add reached it) is exact
          int64_t unused = 0;
          int64_t internal = wave_relax_known(A, qf, x, ra, rb, 1, stamp, unused);
          internal = wave_sum_i64_dpp(internal);
          if (lane == 0) {
            step = stamp;
            singles += 1;
            close(sum, internal, 1, stamp);
          }
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        }
      }
      if (lane == 0) sh_cmd = cmd;
    }
    __threadfence_block();
    __syncthreads();
    const int cmd = sh_cmd;
    if (cmd == CMD_EXIT_DONE || cmd == CMD_EXIT_BIG || cmd == CMD_EXIT_TAIL) { exit_cmd = cmd; break; }
    // a wide step shared by all waves
    const int32_t stamp = sh_stamp;
    int64_t sum = 0, internal = 0;
    int32_t size = 1;
    if (cmd == CMD_SINGLE) {
      const int32_t x = sh_x;
      const int64_t e0 = A.rp[x], e1 = A.rp[x + 1];
      for (int64_t base = e0 + wave * 64; base < e1; base += SWEEP_THREADS) {
        const int64_t e = base + lane;
        const bool act = e < e1;
        const int64_t ec = act ? e : base;
        int32_t yv = A.col[ec], cv = A.w[ec];
        keep(cv);
        int64_t unused = 0;
        internal += sweep_relax(A, q, x, act ? yv : 0, act ? cv : 0, stamp, act, unused);
      }
    } else {
      // the batch's entries spread evenly over the workgroup (a hub row in
      // the batch no longer holds one wave while the others wait), in chunks
      // of SWEEP_THREADS rows
      const int32_t h = sh_h, t = sh_t;
      size = t - h;
      // every vertex of the batch is marked before any row is relaxed (edges
      // inside the batch are recognised by their stamp)
      for (int32_t i = h + threadIdx.x; i < t; i += SWEEP_THREADS) {
        const int32_t x = ld_relaxed(A.capq + i);
        sum += A.cdeg[x];  // minus twice the batch's weight to the visited set, summed by the relax
        st_relaxed(rs_stamp_ptr(A.rs + x), stamp);
      }
      __threadfence_block();
      __syncthreads();
      for (int32_t c0 = h; c0 < t; c0 += SWEEP_THREADS) {
        const int32_t cn = min(SWEEP_THREADS, t - c0);
        int32_t deg = 0;
        if ((int32_t)threadIdx.x < cn) {
          const int32_t x = ld_relaxed(A.capq + c0 + threadIdx.x);
          const int64_t a = A.rp[x];
          deg = (int32_t)(A.rp[x + 1] - a);
          sh_bx[threadIdx.x] = x;
          sh_bbase[threadIdx.x] = a;
        }
        const int32_t incl = wave_incl_sum<int32_t>(deg);
        if (lane == 63) sh_wtot[wave] = incl;
        __threadfence_block();
        __syncthreads();
        int32_t before = 0;
        for (int k = 0; k < wave; ++k) before += sh_wtot[k];
        if ((int32_t)threadIdx.x < cn) sh_boff[threadIdx.x] = before + incl - deg;
        if ((int32_t)threadIdx.x == cn - 1) sh_boff[cn] = before + incl;
        __threadfence_block();
        __syncthreads();
        const int32_t total = sh_boff[cn];
        for (int32_t i0 = 0; i0 < total; i0 += SWEEP_THREADS) {
          const int32_t i = i0 + (int32_t)threadIdx.x;
          const bool act = i < total;
          int32_t x = 0, y = 0, cw = 0;
          if (act) {
            int32_t lo = 0, hi = cn - 1;  // the row: last k with boff[k] <= i
            while (lo < hi) {
              const int32_t mid = (lo + hi + 1) >> 1;
              if (sh_boff[mid] <= i) lo = mid;
              else hi = mid - 1;
            }
            const int64_t e = sh_bbase[lo] + (i - sh_boff[lo]);
            x = sh_bx[lo];
            y = A.col[e];
            cw = A.w[e];
          }
          int64_t rsum = 0;
          internal += sweep_relax(A, q, x, y, cw, stamp, act, rsum);
          sum -= 2 * rsum;
        }
        __threadfence_block();
        __syncthreads();  // the chunk arrays are reused
      }
    }
    sum = wave_sum_i64(sum);
    internal = wave_sum_i64(internal);
    __syncthreads();
    if (lane == 0) {
      if (cmd == CMD_SINGLE) sh_sum[wave] = wave == 0 ? sh_sum[0] : 0;
      else sh_sum[wave] = sum;
      sh_int[wave] = internal;
    }
    __threadfence_block();
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t s2 = 0, in = 0;
      for (int i = 0; i < nwaves; ++i) { s2 += sh_sum[i]; in += sh_int[i]; }
      if (cmd == CMD_BATCH) *q.cap_head = sh_t;
      close(s2, in, size, stamp);
      l_pring_lo = l_pool_next;  // the bucket entries of a shared step are in global memory only
    }
    __threadfence_block();
    __syncthreads();
  }
  // write the state back for the host and the grid-wide kernels
  for (int i = threadIdx.x; i < A.nb; i += SWEEP_THREADS) {
    c->head[i] = l_head[i];
    c->seg_cur[i] = l_cur[i];
    c->seg_end[i] = l_end[i];
  }
  for (int i = threadIdx.x; i < SWEEP_BUCKETS / 64; i += SWEEP_THREADS) c->bitmap[i] = l_bitmap[i];
  if (threadIdx.x == 0) {
    c->cap_head = l_cap_head;
    c->cap_tail = l_cap_tail;
    c->pool_next = l_pool_next;
    c->step = step;
    c->visited = visited;
    c->alpha = alpha;
    c->best_alpha = best_alpha;
    c->best_step = best_step;
    c->singles = singles;
    c->batches = batches;
    c->seq_rows += seq_rows;
    c->rows_done += seq_rows;
    const int ph = min(c->big_batches, SWEEP_PHASES - 1);
    c->ph_singles[ph] += singles - singles0;
    c->ph_batches[ph] += batches - batches0;
    c->ph_cross[ph] += l_cap_tail - tail0;
    c->status = exit_cmd == CMD_EXIT_DONE ? SW_DONE : exit_cmd == CMD_EXIT_TAIL ? SW_TAIL : SW_BIG;
  }
}

// The crossing edges found by the sweeps, united after them: (capx[i],
// capq[i]) of graph blockIdx.y.  Roots are ordered by visit stamp (then
// id): the stamp of the sweep's batch or tail visit, in the high half of
// the vertex's rs word (0 where never visited).  A crossed vertex q is
// visited after the vertex x that made it cross, so nearly every pair links
// the fresh root q under the root of x's tree, which only grows: one
// uncontended compare-and-swap on q's own word.
__global__ void k_sweep_unite(const SweepArgs* args) {
  const SweepDev A = dev_view(args[blockIdx.y]);
  const int32_t n = min(A.ctl->cap_tail, A.ng);  // the tail may count pairs it had no room for
  const auto key = [&](int32_t v) {
    return ((uint64_t)(uint32_t)rs_stamp(ld_relaxed(A.rs + v)) << 32) | (uint32_t)v;
  };
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    uf_union_by(A.parent, A.capx[i], A.capq[i], key);
}

// Per graph: status, FIFO bounds and row entries of the pending batch, for
// the host (one small copy instead of one per graph).
// What the host reads of each running graph after a sequential launch (and
// the mark of a grid-wide batch it handed back): one copy for all of them.
struct SweepStatus {
  int32_t status, cap_head, cap_tail, visited;
  int64_t batch_deg, rows_done;
  int32_t seg_unsorted, count_err;
};
__global__ void k_sweep_status(const SweepArgs* args, const int32_t* run, int32_t k, SweepStatus* out) {
  for (int64_t i = gtid(); i < k; i += gstride()) {
    const MC_GLOBAL SweepCtl* c = (const MC_GLOBAL SweepCtl*)args[run[i]].ctl;
    out[i] = SweepStatus{c->status, c->cap_head, c->cap_tail, c->visited, c->batch_deg, c->rows_done,
                         c->seg_unsorted, c->count_err};
  }
}

// Grid-wide batch [cap_head, cap_tail) of graph run[blockIdx.y], if its
// sequential kernel handed one back: mark every vertex visited, and sum the
// rows' lengths (the host's push or pull choice) and degrees.  Launched
// before the status is read, so one readback serves both.
__global__ void k_sweep_big_mark(const SweepArgs* args, const int32_t* run) {
  const SweepDev A = dev_view(args[run[blockIdx.y]]);
  MC_GLOBAL SweepCtl* c = A.ctl;
  if (c->status != SW_BIG) return;  // uniform: the graph is done, or its tail follows
  const int32_t h = c->cap_head, t = c->cap_tail;
  const int32_t stamp = c->step + 1;
  int64_t sum = 0, deg = 0;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nth = (int64_t)gridDim.x * blockDim.x;
  constexpr int MU = 4;  // batch vertices per thread and step, their loads in flight together
  for (int64_t i0 = h + tid; i0 - lane_id() < t; i0 += nth * MU) {  // wave-uniform bound
    // loads outside the branch (one round trip for all of them); a slot past
    // the end reads the batch's first vertex
    int32_t x[MU];
#pragma unroll
    for (int u = 0; u < MU; ++u) {
      const int64_t i = i0 + u * nth;
      x[u] = A.capq[i < t ? i : h];
    }
    int64_t cd[MU], d[MU];
#pragma unroll
    for (int u = 0; u < MU; ++u) {
      cd[u] = A.cdeg[x[u]];
      d[u] = A.rp[x[u] + 1] - A.rp[x[u]];
    }
#pragma unroll
    for (int u = 0; u < MU; ++u) {
      if (i0 + u * nth < t) {
        sum += cd[u];  // minus twice the batch's weight to the visited set, summed by the relax
        *rs_stamp_ptr(A.rs + x[u]) = stamp;
        deg += d[u];
      }
    }
  }
  // one add per workgroup and counter (adds on one address serialise)
  __shared__ int64_t part[2][8];
  sum = wave_sum_i64(sum);
  deg = wave_sum_i64(deg);
  const int wave = threadIdx.x >> 6;
  if (lane_id() == 0) {
    part[0][wave] = sum;
    part[1][wave] = deg;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s = 0, d = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      s += part[0][k];
      d += part[1][k];
    }
    if (s) atomicAdd((unsigned long long*)&c->batch_sum, (unsigned long long)s);
    if (d) atomicAdd((unsigned long long*)&c->batch_deg, (unsigned long long)d);
  }
}

// Grid-wide batch [h, t): relax every edge of the batch.
// No queue pushes (the queue is rebuilt exactly after the batch); crossing
// vertices collect in a per-wave LDS buffer and go to the FIFO in blocks.
constexpr int BIG_BUF = 256;
__device__ __forceinline__ void flush_wave_buf(const SweepArgs& A, int32_t* wbuf, int32_t* wcnt) {
  const int lane = lane_id();
  const int32_t cnt = *wcnt;
  if (cnt == 0) return;
  int32_t base = 0;
  if (lane == 0) base = atomicAdd(&A.ctl->cap_tail, cnt);
  base = bcast(base, 0);
  for (int32_t i = lane; i < cnt; i += 64) {
    A.capq[base + i] = wbuf[2 * i];
    A.capx[base + i] = wbuf[2 * i + 1];
  }
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) *wcnt = 0;
  __builtin_amdgcn_wave_barrier();
}

// The batch's entries are cut into tiles of BIG_TILE consecutive entries
// (in batch order, from a prefix sum of the row lengths), one tile per
// workgroup at a time and BIG_UNROLL consecutive entries per thread: the
// work is even whatever the row lengths (a few hubs, or many short rows), and
// every thread has several gathers in flight.
constexpr int BIG_UNROLL = 4;
constexpr int BIG_TILE = 256 * BIG_UNROLL;

// The 2-bit state of each vertex while a grid-wide batch is relaxed (16 per
// word, in L2 instead of an 8-byte word gathered from HBM): free, crossed
// the cap during this relax, in the batch, visited before the batch.
enum : uint32_t { BS_FREE = 0, BS_CROSSED = 1, BS_BATCH = 2, BS_VISITED = 3 };

// Before a grid-wide batch is relaxed: the states of the graph's vertices
// (a crossed vertex is in the FIFO, so at this point none is BS_CROSSED).
__global__ void k_sweep_bits(SweepArgs A, uint32_t* st2) {
  const int32_t stamp = A.ctl->step + 1;
  constexpr int BU = 4;  // 64-vertex groups per wave and step, their words loaded together
  const int64_t stride = gstride();
  for (int64_t b0 = (gtid() >> 6) << 6; b0 < A.ng; b0 += stride * BU) {
    int32_t sts[BU];
#pragma unroll
    for (int u = 0; u < BU; ++u) {
      const int64_t i = b0 + u * stride + lane_id();
      sts[u] = rs_stamp(A.rs[A.v0 + (i < A.ng ? i : 0)]);
    }
#pragma unroll
    for (int u = 0; u < BU; ++u) {
      const int64_t base = b0 + u * stride;  // wave-uniform
      if (base >= A.ng) break;
      const int32_t st = base + lane_id() < A.ng ? sts[u] : 0;
      const uint64_t hi = ballot(st != 0);                 // in the batch or visited
      const uint64_t lo = ballot(st != 0 && st != stamp);  // visited
      // interleave: vertex k of a 16-vertex group at bits 2k (lo) and 2k+1 (hi)
      uint32_t word = 0;
      const int g = lane_id() & 3;  // lanes 0..3 each build one word of 16 vertices
      for (int k = 0; k < 16; ++k) {
        const int b = g * 16 + k;
        word |= (uint32_t)((lo >> b) & 1) << (2 * k);
        word |= (uint32_t)((hi >> b) & 1) << (2 * k + 1);
      }
      if (lane_id() < 4) st2[(base >> 4) + g] = word;
    }
  }
}

// Row length of batch vertex i (the prefix sum's input).
struct BatchDeg {
  const int32_t* capq;  // the batch's FIFO entries
  const int64_t* rp;
  __device__ __forceinline__ int64_t operator()(int64_t i) const {
    const int32_t x = capq[i];
    return rp[x + 1] - rp[x];
  }
};

// tile_row[j]: the batch row holding entry j * BIG_TILE (each tile start
// lies in exactly one row of nonzero length).
__global__ void k_sweep_big_tiles(const int64_t* off, int32_t bsz, int32_t* tile_row) {
  for (int64_t i = gtid(); i < bsz; i += gstride()) {
    const int64_t a = off[i], b = off[i + 1];
    for (int64_t j = (a + BIG_TILE - 1) / BIG_TILE; j * BIG_TILE < b; ++j) tile_row[j] = (int32_t)i;
  }
}

// off: bsz + 1 prefix sums of the batch's row lengths (off[bsz] = entries).
// fallback = 1: the launch after a range-owned attempt, which runs only if
// that attempt found a batch row out of order (and so did nothing).
__global__ void __launch_bounds__(256) k_sweep_big_relax(SweepArgs A, int32_t h, int32_t bsz, const int64_t* off,
                                                         const int32_t* tile_row, uint32_t* st2, int32_t fallback) {
  if (fallback && ld_relaxed(&A.ctl->seg_unsorted) == 0) return;
  __shared__ int32_t buf[4][2 * BIG_BUF];
  __shared__ int32_t cnt[4];
  __shared__ int32_t s_x[BIG_TILE];
  __shared__ int64_t s_off[BIG_TILE + 1], s_base[BIG_TILE];
  SweepCtl* c = A.ctl;
  const int32_t stamp = c->step + 1;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  int32_t* wbuf = buf[wave];
  int32_t* wcnt = &cnt[wave];
  if (lane == 0) *wcnt = 0;
  const SweepQ gq = global_q(c);
  const int64_t total = off[bsz];
  const int64_t ntiles = (total + BIG_TILE - 1) / BIG_TILE;
  const int64_t e_idle = A.rp[A.v0];  // an entry of the graph (it has some: a batch is being relaxed)
  int64_t internal = 0, rsum = 0;  // 2 w(inside the batch); the batch's weight to the visited set
  for (int64_t j = blockIdx.x; j < ntiles; j += gridDim.x) {
    const int64_t t0 = j * BIG_TILE, t1 = min(t0 + BIG_TILE, total);
    const int32_t r0 = tile_row[j], r1 = j + 1 < ntiles ? tile_row[j + 1] : bsz - 1;
    // rows [r0, r1] hold the tile; more than BIG_TILE of them only if some
    // are empty, so they go in slices of BIG_TILE rows
    for (int32_t rb = r0; rb <= r1; rb += BIG_TILE) {
      const int32_t nr = min(BIG_TILE, r1 + 1 - rb);
      for (int32_t k = threadIdx.x; k < nr; k += 256) {
        const int32_t x = A.capq[h + rb + k];
        s_x[k] = x;
        s_base[k] = A.rp[x];
        s_off[k] = off[rb + k];
      }
      if (threadIdx.x == 0) s_off[nr] = off[rb + nr];
      __syncthreads();
      const int64_t lo_e = max(s_off[0], t0), hi_e = min(s_off[nr], t1);
      const int64_t i0 = lo_e + (int64_t)threadIdx.x * BIG_UNROLL;
      int32_t row = 0;
      if (i0 < hi_e) {
        int32_t lo = 0, hi = nr - 1;  // last row with s_off[row] <= i0
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= i0) lo = mid;
          else hi = mid - 1;
        }
        row = lo;
      }
      // Each step below is issued for all BIG_UNROLL entries before any
      // result is used, and no global access sits in a divergent branch:
      // the tile costs three round trips (entries, neighbour state, adds),
      // not three per entry.  An idle slot reads the graph's first entry.
      int32_t xs[BIG_UNROLL];
      int64_t es[BIG_UNROLL];
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) {
        const int64_t i = i0 + u;
        xs[u] = -1;
        es[u] = e_idle;
        if (i < hi_e) {
          while (s_off[row + 1] <= i) ++row;  // LDS only
          es[u] = s_base[row] + (i - s_off[row]);
          xs[u] = s_x[row];
        }
      }
      int32_t ys[BIG_UNROLL], cs[BIG_UNROLL];
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) {
        ys[u] = A.col[es[u]];
        cs[u] = A.w[es[u]];
      }
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) keep(cs[u]);  // weights in with the columns
      // the neighbour's state: in the batch (internal weight), visited
      // before it (weight to the visited set), crossed during this relax (its
      // r no longer matters: the add is skipped, Lemma 1), or free (the add,
      // and maybe a crossing)
      uint32_t sw[BIG_UNROLL];
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) sw[u] = st2[(ys[u] - A.v0) >> 4];
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) keep(sw[u]);  // all states in before any add issues
      bool upd[BIG_UNROLL];
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) {
        const int32_t i = ys[u] - A.v0;
        const bool act = xs[u] >= 0 && ys[u] != xs[u];
        const uint32_t st = (sw[u] >> (2 * (i & 15))) & 3u;
        if (act && st == BS_BATCH) internal += cs[u];
        if (act && st == BS_VISITED) rsum += cs[u];
        upd[u] = act && st == BS_FREE;
      }
      // the adds go to r alone, the low half of the word (r + c stays below
      // 2^31, so it never carries into the stamp): a 32-bit return leaves no
      // dead half whose register the compiler would reuse while the add is
      // in flight, which forces a wait for it
      int32_t old[BIG_UNROLL];
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) old[u] = 0;
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u)
        if (upd[u]) old[u] = atomic_add((int32_t*)(A.rs + ys[u]), cs[u]);
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) keep(old[u]);  // all adds issue before the first is used
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) {
        const int64_t r_old = old[u];
        const bool cross = upd[u] && r_old < A.lam && A.lam <= r_old + cs[u];
        if (cross) {  // later adds to this vertex are skipped
          const int32_t i = ys[u] - A.v0;
          atomicOr(&st2[i >> 4], BS_CROSSED << (2 * (i & 15)));
        }
        const uint64_t cm = ballot(cross);
        if (cm) {
          const int32_t at = *wcnt;
          if (cross) {
            const int32_t k = at + popc64(cm & lanemask_lt());
            wbuf[2 * k] = ys[u];
            wbuf[2 * k + 1] = xs[u];
          }
          __builtin_amdgcn_wave_barrier();
          if (lane == 0) *wcnt = at + popc64(cm);
          __builtin_amdgcn_wave_barrier();
          if (*wcnt > BIG_BUF - 64) flush_wave_buf(A, wbuf, wcnt);
        }
      }
      __syncthreads();  // the slice arrays are reused
    }
  }
  // the waves' last crossings: one FIFO reservation for the workgroup
  __shared__ int32_t blk_base;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int32_t tot = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    blk_base = tot ? atomicAdd(&c->cap_tail, tot) : 0;
  }
  __syncthreads();
  {
    int32_t o = blk_base;
    for (int k = 0; k < wave; ++k) o += cnt[k];
    for (int32_t i = lane; i < *wcnt; i += 64) {
      A.capq[o + i] = wbuf[2 * i];
      A.capx[o + i] = wbuf[2 * i + 1];
    }
  }
  // one add per workgroup and counter (adds on one address serialise)
  __shared__ int64_t part[2][4];
  internal = wave_sum_i64(internal);
  rsum = wave_sum_i64(rsum);
  if (lane == 0) {
    part[0][wave] = internal;
    part[1][wave] = rsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t tot = part[0][0] + part[0][1] + part[0][2] + part[0][3];
    const int64_t rs = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    if (tot) atomicAdd((unsigned long long*)&c->batch_internal, (unsigned long long)tot);
    if (rs) atomicAdd((unsigned long long*)&c->batch_sum, (unsigned long long)(-2 * rs));
  }
}

// ---- range-owned form of a push batch
// When the batch's rows are few and long (the hubs of a skewed graph) and
// list their neighbours in ascending order, the graph's vertices are cut
// into ranges of 2^shift, one workgroup per range.  A batch row's
// entries into one range are then one contiguous segment, found once for
// all rows and ranges (k_sweep_seg_bounds), and the range's workgroup adds
// the segments into its range's r held in LDS: no add goes to global memory.
// The adds into one vertex take the order of the workgroup's LDS atomics, a
// legal order of the batch (its members tie at the cap), so the crossing a
// vertex reports is a contractible pair, as in the global form.
constexpr int SEG_MAX_SHIFT = 12;  // ranges of at most 4096 vertices in LDS
constexpr int SEG_THREADS = 512;
constexpr int SEG_UNROLL = 2;

// bnd[i * (nr + 1) + q] for batch row i and range q in [0, nr]: the offset in
// row i of its first entry whose neighbour lies in range q or above (rows in
// ascending neighbour order), the row's length at q = nr.  One pass over the
// batch's entries in tiles of SEG_BTILE (BIG_TILE multiples, so the global
// relax's tile rows serve): an entry writes the cells of the ranges from the
// one after its predecessor's up to its own, the row's last entry also those
// after its own.  (Rows without entries write none; the relax reads their
// length from off.)  A row out of order (an entry below its predecessor)
// sets ctl->seg_unsorted: the range-owned relax then does nothing and the
// global form, launched after it, relaxes the batch instead.
constexpr int SEG_BUNROLL = 4;
constexpr int SEG_BTILE = 256 * SEG_BUNROLL;
static_assert(SEG_BTILE % BIG_TILE == 0, "bounds tiles are whole relax tiles");
__global__ void __launch_bounds__(256) k_sweep_seg_bounds(SweepArgs A, int32_t h, int32_t bsz, const int64_t* off,
                                                          const int32_t* tile_row, int32_t shift, int32_t nr,
                                                          int32_t* bnd) {
  constexpr int TSTEP = SEG_BTILE / BIG_TILE;
  __shared__ int64_t s_off[SEG_BTILE + 1], s_base[SEG_BTILE];
  const int64_t total = off[bsz];
  const int64_t ntiles = (total + SEG_BTILE - 1) / SEG_BTILE;
  const int64_t nbig = (total + BIG_TILE - 1) / BIG_TILE;  // tiles of tile_row
  const int64_t e_idle = A.rp[A.v0];
  for (int64_t j = blockIdx.x; j < ntiles; j += gridDim.x) {
    const int64_t t0 = j * SEG_BTILE, t1 = min(t0 + SEG_BTILE, total);
    const int32_t r0 = tile_row[j * TSTEP], r1 = (j + 1) * TSTEP < nbig ? tile_row[(j + 1) * TSTEP] : bsz - 1;
    for (int32_t rb = r0; rb <= r1; rb += SEG_BTILE) {
      const int32_t nrow = min(SEG_BTILE, r1 + 1 - rb);
      for (int32_t k = threadIdx.x; k < nrow; k += 256) {
        s_base[k] = A.rp[A.capq[h + rb + k]];
        s_off[k] = off[rb + k];
      }
      if (threadIdx.x == 0) s_off[nrow] = off[rb + nrow];
      __syncthreads();
      const int64_t lo_e = max(s_off[0], t0), hi_e = min(s_off[nrow], t1);
      const int64_t i0 = lo_e + (int64_t)threadIdx.x * SEG_BUNROLL;
      int32_t row = 0;
      if (i0 < hi_e) {
        int32_t lo = 0, hi = nrow - 1;  // last row with s_off[row] <= i0
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= i0) lo = mid;
          else hi = mid - 1;
        }
        row = lo;
      }
      int64_t es[SEG_BUNROLL];
      int32_t ps[SEG_BUNROLL], ls[SEG_BUNROLL], ri[SEG_BUNROLL];
#pragma unroll
      for (int u = 0; u < SEG_BUNROLL; ++u) {
        const int64_t i = i0 + u;
        es[u] = e_idle;
        ps[u] = -1;
        ls[u] = 0;
        ri[u] = 0;
        if (i < hi_e) {
          while (s_off[row + 1] <= i) ++row;  // LDS only
          ps[u] = (int32_t)(i - s_off[row]);
          ls[u] = (int32_t)(s_off[row + 1] - s_off[row]);
          es[u] = s_base[row] + ps[u];
          ri[u] = rb + row;
        }
      }
      // an entry's predecessor in its row is this thread's previous entry,
      // except for the first, whose predecessor is loaded (its line is
      // mostly the entry's own)
      int32_t ys[SEG_BUNROLL], yp[SEG_BUNROLL];
#pragma unroll
      for (int u = 0; u < SEG_BUNROLL; ++u) ys[u] = A.col[es[u]];
      yp[0] = A.col[ps[0] > 0 ? es[0] - 1 : es[0]];
#pragma unroll
      for (int u = 1; u < SEG_BUNROLL; ++u) yp[u] = ys[u - 1];
      bool unsorted = false;
#pragma unroll
      for (int u = 0; u < SEG_BUNROLL; ++u) unsorted = unsorted || (ps[u] > 0 && yp[u] > ys[u]);
      if (ballot(unsorted) != 0 && lane_id() == 0) st_relaxed(&A.ctl->seg_unsorted, 1);
#pragma unroll
      for (int u = 0; u < SEG_BUNROLL; ++u) {
        if (ps[u] < 0) continue;
        const int32_t q = (ys[u] - A.v0) >> shift;
        const int32_t qp = ps[u] > 0 ? ((yp[u] - A.v0) >> shift) : -1;
        int32_t* b = bnd + (int64_t)ri[u] * (nr + 1);
        for (int32_t t = qp + 1; t <= q; ++t) b[t] = ps[u];
        if (ps[u] == ls[u] - 1)
          for (int32_t t = q + 1; t <= nr; ++t) b[t] = ls[u];
      }
      __syncthreads();  // the slice arrays are reused
    }
  }
}

// Range q = blockIdx.x of the graph's local ids [q 2^shift, (q + 1) 2^shift):
// its r and visit states staged in LDS, then for every batch row its segment
// into the range (chunks of SEG_THREADS rows, their entries spread evenly over
// the threads), the adds made in LDS, and the free vertices' r written back.
// The batch's internal weight and weight to the visited set are summed as in
// the global form.
__global__ void __launch_bounds__(SEG_THREADS) k_sweep_seg_relax(SweepArgs A, int32_t h, int32_t bsz,
                                                                 const int64_t* off, int32_t shift, int32_t nr,
                                                                 const int32_t* bnd, const uint32_t* st2) {
  constexpr int NW = SEG_THREADS / 64;
  if (ld_relaxed(&A.ctl->seg_unsorted) != 0) return;  // the global form relaxes the batch
  __shared__ int32_t r_loc[1 << SEG_MAX_SHIFT];
  __shared__ uint32_t s_st[(1 << SEG_MAX_SHIFT) / 16];
  __shared__ int32_t s_x[SEG_THREADS];
  __shared__ int64_t s_base[SEG_THREADS];
  __shared__ int64_t s_off[SEG_THREADS + 1];
  __shared__ int64_t wtot[NW];
  __shared__ int32_t buf[NW][2 * BIG_BUF];
  __shared__ int32_t cnt[NW];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int tid = threadIdx.x;
  // range q, consecutive ranges on one XCD (a run's edge lines are read by
  // the neighbouring range too); the grid is nr rounded up to whole XCDs
  const int32_t q = xcd_major(blockIdx.x, gridDim.x);
  if (q >= nr) return;
  const int32_t lo_v = q << shift;  // a multiple of 64
  const int32_t nv = min(1 << shift, A.ng - lo_v);
  for (int32_t i = tid; i < nv; i += SEG_THREADS) r_loc[i] = rs_r(A.rs[A.v0 + lo_v + i]);
  for (int32_t i = tid; i < (nv + 15) / 16; i += SEG_THREADS) s_st[i] = st2[(lo_v >> 4) + i];
  if (lane == 0) cnt[wave] = 0;
  int32_t* wbuf = buf[wave];
  int32_t* wcnt = &cnt[wave];
  __syncthreads();
  const int64_t e_idle = A.rp[A.v0];
  int64_t internal = 0, rsum = 0;
  for (int32_t c0 = 0; c0 < bsz; c0 += SEG_THREADS) {
    const int32_t cn = min(SEG_THREADS, bsz - c0);
    int64_t len = 0;
    if (tid < cn) {
      const int32_t i = c0 + tid;
      const int32_t x = A.capq[h + i];
      // a segment is clamped into its row (a row out of order could leave
      // cells unwritten; reads stay inside the row)
      const int32_t rl = (int32_t)(off[i + 1] - off[i]);
      const int32_t* bi = bnd + (int64_t)i * (nr + 1);
      int32_t a = 0, b = 0;
      if (rl > 0) {
        a = min(max(bi[q], 0), rl);
        b = min(max(bi[q + 1], a), rl);
      }
      len = b - a;
      s_x[tid] = x;
      s_base[tid] = A.rp[x] + a;
    }
    const int64_t incl = wave_incl_sum<int64_t>(len);
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    int64_t before = 0;
    for (int k = 0; k < wave; ++k) before += wtot[k];
    if (tid < cn) s_off[tid] = before + incl - len;
    if (tid == cn - 1) s_off[cn] = before + incl;
    __syncthreads();
    const int64_t total = s_off[cn];
    // a pass's entries: their batch vertex and their column and weight
    // (loads issued here, awaited where they are used)
    int32_t xs[SEG_UNROLL], ys[SEG_UNROLL], cs[SEG_UNROLL];
    auto fetch = [&](int64_t pass) {
      const int64_t i0 = pass + tid * SEG_UNROLL;
      int32_t row = 0;
      if (i0 < total) {
        int32_t lo = 0, hi = cn - 1;  // last row with s_off[row] <= i0
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= i0) lo = mid;
          else hi = mid - 1;
        }
        row = lo;
      }
      int64_t es[SEG_UNROLL];
#pragma unroll
      for (int u = 0; u < SEG_UNROLL; ++u) {
        const int64_t i = i0 + u;
        es[u] = e_idle;
        xs[u] = -1;
        if (i < total) {
          while (s_off[row + 1] <= i) ++row;  // LDS only
          es[u] = s_base[row] + (i - s_off[row]);
          xs[u] = s_x[row];
        }
      }
#pragma unroll
      for (int u = 0; u < SEG_UNROLL; ++u) {
        ys[u] = A.col[es[u]];
        cs[u] = A.w[es[u]];
      }
    };
    if (total > 0) fetch(0);
    // every thread takes every pass (the crossings' buffer is kept per wave,
    // with all lanes present); a slot past the end is idle
    for (int64_t pass = 0; pass < total; pass += SEG_THREADS * SEG_UNROLL) {
      // this pass's entries; the next pass's loads go out before its adds
      int32_t xc[SEG_UNROLL], yc[SEG_UNROLL], cc[SEG_UNROLL];
#pragma unroll
      for (int u = 0; u < SEG_UNROLL; ++u) {
        xc[u] = xs[u];
        yc[u] = ys[u];
        cc[u] = cs[u];
      }
      if (pass + SEG_THREADS * SEG_UNROLL < total) fetch(pass + SEG_THREADS * SEG_UNROLL);
#pragma unroll
      for (int u = 0; u < SEG_UNROLL; ++u) {
        const int32_t yl = yc[u] - A.v0 - lo_v;
        // (a neighbour outside the range would mean a row out of order:
        // never added, and never an LDS access out of bounds)
        const bool act = xc[u] >= 0 && yc[u] != xc[u] && (uint32_t)yl < (uint32_t)nv;
        bool cross = false;
        if (act) {
          const uint32_t st = (s_st[yl >> 4] >> (2 * (yl & 15))) & 3u;
          if (st == BS_BATCH) internal += cc[u];
          else if (st == BS_VISITED) rsum += cc[u];
          else {
            const int32_t old = atomicAdd(&r_loc[yl], cc[u]);
            cross = (int64_t)old < A.lam && A.lam <= (int64_t)old + cc[u];
          }
        }
        const uint64_t cm = ballot(cross);
        if (cm) {
          const int32_t at = *wcnt;
          if (cross) {
            const int32_t k = at + popc64(cm & lanemask_lt());
            wbuf[2 * k] = yc[u];
            wbuf[2 * k + 1] = xc[u];
          }
          __builtin_amdgcn_wave_barrier();
          if (lane == 0) *wcnt = at + popc64(cm);
          __builtin_amdgcn_wave_barrier();
          if (*wcnt > BIG_BUF - 64) flush_wave_buf(A, wbuf, wcnt);
        }
      }
    }
    __syncthreads();  // the row arrays are reused
  }
  // the free vertices' new r (the low half of the packed word)
  for (int32_t i = tid; i < nv; i += SEG_THREADS) {
    const uint32_t st = (s_st[i >> 4] >> (2 * (i & 15))) & 3u;
    if (st == BS_FREE) reinterpret_cast<int32_t*>(A.rs + A.v0 + lo_v + i)[0] = r_loc[i];
  }
  // the waves' last crossings: one FIFO reservation for the workgroup
  __shared__ int32_t blk_base;
  __syncthreads();
  if (tid == 0) {
    int32_t tot = 0;
    for (int k = 0; k < NW; ++k) tot += cnt[k];
    blk_base = tot ? atomicAdd(&A.ctl->cap_tail, tot) : 0;
  }
  __syncthreads();
  {
    int32_t o = blk_base;
    for (int k = 0; k < wave; ++k) o += cnt[k];
    for (int32_t i = lane; i < *wcnt; i += 64) {
      A.capq[o + i] = wbuf[2 * i];
      A.capx[o + i] = wbuf[2 * i + 1];
    }
  }
  __shared__ int64_t part[2][NW];
  internal = wave_sum_i64(internal);
  rsum = wave_sum_i64(rsum);
  if (lane == 0) {
    part[0][wave] = internal;
    part[1][wave] = rsum;
  }
  __syncthreads();
  if (tid == 0) {
    int64_t tot = 0, rs = 0;
    for (int k = 0; k < NW; ++k) {
      tot += part[0][k];
      rs += part[1][k];
    }
    if (tot) atomicAdd((unsigned long long*)&A.ctl->batch_internal, (unsigned long long)tot);
    if (rs) atomicAdd((unsigned long long*)&A.ctl->batch_sum, (unsigned long long)(-2 * rs));
  }
}

// pull: the batch was relaxed in pull form, whose c(S + B) replaces alpha
// (the sum of the free vertices' new r, each their weight to S + B).
// Also clears the bucket counts for the queue rebuild that follows (the
// work of k_sweep_rb_zero).
__global__ void k_sweep_big_finish(SweepArgs A, int32_t t, int32_t pull) {
  SweepCtl* c = A.ctl;
  for (int64_t i = gtid(); i < SWEEP_BUCKETS; i += gstride()) c->seg_end[i] = 0;
  if (gtid() != 0) return;
  const int32_t h = c->cap_head;
  const int32_t stamp = ++c->step;
  c->batches += 1;
  c->big_batches += 1;
  c->cap_head = t;
  c->rows_done += c->batch_deg;
  if (pull) {
    c->batch_sum = c->pull_alpha - c->alpha;
    c->batch_internal = 0;
  }
  sweep_close_batch(c, A.ng, c->batch_sum, c->batch_internal, t - h, stamp);
  // zero for the next grid-wide batch (k_sweep_init zeroes them first)
  c->batch_sum = 0;
  c->batch_internal = 0;
  c->batch_deg = 0;
  c->pull_alpha = 0;
  c->free_count = 0;
  c->status = SW_RUNNING;
}

// ---- pull form of a grid-wide batch
// When the batch's rows hold more entries than the rows of the vertices
// still free (neither visited nor in the batch), each free vertex y sums the
// weight of its edges into the batch instead: one pass over the free rows,
// no atomic on r unless a row spans tiles.  The batch's members tie at the
// cap, so any order of them is legal; y's edges into the batch are taken in
// row order, and the one at which r(y) reaches lambda-hat is y's crossing
// (united later).  alpha after the batch is c(S + B) = the sum over free
// vertices of their new r (each the weight to S + B).

// Before a pull batch: the visit states (as k_sweep_bits) and the list of
// the free vertices with the sum of their r (pull_alpha: the weight to S,
// exact for a vertex that never crossed the cap), in one pass.  Workgroup b
// takes vertices [b FREE_TILE, (b + 1) FREE_TILE) in groups of 64 (one
// ballot each), reserves its list range with one add on free_count (zeroed
// by k_sweep_init and every batch's finish) and writes its free vertices in
// vertex order.  The list's order across workgroups is that of the
// reservations; nothing in the pull depends on it.
constexpr int FREE_TILE = 4096;
__global__ void __launch_bounds__(256) k_sweep_free_bits(SweepArgs A, uint32_t* st2, int32_t* list) {
  constexpr int NG = FREE_TILE / 64;  // groups per tile
  __shared__ uint64_t s_free[NG];
  __shared__ int32_t s_pos[NG + 1];
  __shared__ int64_t s_r[4];
  __shared__ int32_t s_base;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int32_t stamp = A.ctl->step + 1;
  const int64_t t0 = (int64_t)blockIdx.x * FREE_TILE;
  int64_t rsum = 0;
  for (int gi = wave; gi < NG; gi += 4) {
    const int64_t base = t0 + gi * 64;
    const int64_t i = base + lane;
    const uint64_t u = i < A.ng ? A.rs[A.v0 + i] : 0;
    const int32_t st = i < A.ng ? rs_stamp(u) : 0;
    const uint64_t hi = ballot(st != 0);                 // in the batch or visited
    const uint64_t lo = ballot(st != 0 && st != stamp);  // visited
    const bool fr = i < A.ng && st == 0;
    const uint64_t fm = ballot(fr);
    if (fr) rsum += rs_r(u);
    uint32_t word = 0;
    const int g = lane & 3;  // lanes 0..3 each build one word of 16 vertices
    for (int k = 0; k < 16; ++k) {
      const int b = g * 16 + k;
      word |= (uint32_t)((lo >> b) & 1) << (2 * k);
      word |= (uint32_t)((hi >> b) & 1) << (2 * k + 1);
    }
    if (lane < 4 && base < A.ng) st2[(base >> 4) + g] = word;
    if (lane == 0) s_free[gi] = fm;
  }
  rsum = wave_sum_i64(rsum);
  if (lane == 0) s_r[wave] = rsum;
  __syncthreads();
  if (wave == 0) {
    // group offsets within the tile, and the tile's range in the list
    const int32_t c0 = lane < NG ? popc64(s_free[lane]) : 0;
    const int32_t incl = wave_incl_sum<int32_t>(c0);
    if (lane < NG) s_pos[lane] = incl - c0;
    if (lane == 63) {
      s_pos[NG] = incl;
      s_base = incl ? atomicAdd(&A.ctl->free_count, incl) : 0;
      const int64_t r = s_r[0] + s_r[1] + s_r[2] + s_r[3];
      if (r) atomicAdd((unsigned long long*)&A.ctl->pull_alpha, (unsigned long long)r);
    }
  }
  __syncthreads();
  for (int gi = wave; gi < NG; gi += 4) {
    const uint64_t fm = s_free[gi];
    if ((fm >> lane) & 1)
      list[s_base + s_pos[gi] + popc64(fm & lanemask_lt())] = A.v0 + (int32_t)(t0 + gi * 64 + lane);
  }
}

// The free list's length is taken from the counts the host already holds
// (the graph's vertices less the visited ones and the batch), so no
// readback waits for the scan.  Checked here against the scan's total: a
// difference is recorded (count_err) and the list is padded with a vertex of
// the graph up to the assumed length, so every launch sized by it reads
// valid vertices.
__global__ void k_sweep_free_check(SweepArgs A, int32_t assumed, int32_t* list) {
  const int32_t got = A.ctl->free_count;
  if (got != assumed && threadIdx.x == 0) A.ctl->count_err = 1;
  for (int32_t i = got + (int32_t)threadIdx.x; i < assumed; i += blockDim.x) list[i] = A.v0;
}

// The free rows in tiles of BIG_TILE entries (off: prefix sums of the list's
// row lengths; tile_row: each tile's first row, as for the push form).  A
// workgroup's next tile, when its rows fit one slice, has its rows' vertices
// and offsets loaded before this tile's entries and their row starts with
// this tile's state words, so they wait in registers, not on the latency.
__global__ void __launch_bounds__(256) k_sweep_big_pull(SweepArgs A, const int32_t* list, int32_t nl,
                                                        const int64_t* off, const int32_t* tile_row,
                                                        const uint32_t* st2) {
  constexpr int PR = BIG_TILE / 256;  // prefetched rows per thread
  __shared__ int32_t s_y[BIG_TILE];
  __shared__ int64_t s_off[BIG_TILE + 1], s_base[BIG_TILE];
  __shared__ uint32_t e_w[BIG_TILE];
  __shared__ int32_t e_x[BIG_TILE];
  __shared__ uint32_t s_wt[4];
  static_assert(BIG_TILE == 4 * 64 * BIG_UNROLL, "four waves, BIG_UNROLL positions per lane");
  SweepCtl* c = A.ctl;
  const int lane = lane_id();
  const int64_t total = off[nl];
  const int64_t ntiles = (total + BIG_TILE - 1) / BIG_TILE;
  const int64_t e_idle = A.rp[A.v0];
  int64_t into = 0;  // weight of free rows' edges into the batch
  int32_t py[PR];
  int64_t pb[PR], po[PR], po_end = 0;
  bool have = false;  // py, pb, po hold the rows of this tile
  for (int64_t j = blockIdx.x; j < ntiles; j += gridDim.x) {
    const int64_t t0 = j * BIG_TILE, t1 = min(t0 + BIG_TILE, total);
    const int32_t r0 = tile_row[j], r1 = j + 1 < ntiles ? tile_row[j + 1] : nl - 1;
    // the next tile, prefetched when its rows fit one slice
    const int64_t jn = j + gridDim.x;
    int32_t n0 = 0, nn = 0;
    if (jn < ntiles) {
      n0 = tile_row[jn];
      nn = (jn + 1 < ntiles ? tile_row[jn + 1] : nl - 1) + 1 - n0;
    }
    const bool pre = jn < ntiles && nn <= BIG_TILE && r1 + 1 - r0 <= BIG_TILE;
    for (int32_t rb = r0; rb <= r1; rb += BIG_TILE) {
      const int32_t nr = min(BIG_TILE, r1 + 1 - rb);
      if (have) {
#pragma unroll
        for (int u = 0; u < PR; ++u) {
          const int32_t k = (int32_t)threadIdx.x + u * 256;
          if (k < nr) {
            s_y[k] = py[u];
            s_base[k] = pb[u];
            s_off[k] = po[u];
          }
        }
        if (threadIdx.x == 0) s_off[nr] = po_end;
        have = false;
      } else {
        for (int32_t k = threadIdx.x; k < nr; k += 256) {
          const int32_t y = list[rb + k];
          s_y[k] = y;
          s_base[k] = A.rp[y];
          s_off[k] = off[rb + k];
        }
        if (threadIdx.x == 0) s_off[nr] = off[rb + nr];
      }
      __syncthreads();
      const int64_t lo_e = max(s_off[0], t0), hi_e = min(s_off[nr], t1);
      const int64_t i0 = lo_e + (int64_t)threadIdx.x * BIG_UNROLL;
      int32_t row = 0;
      if (i0 < hi_e) {
        int32_t lo = 0, hi = nr - 1;  // last row with s_off[row] <= i0
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= i0) lo = mid;
          else hi = mid - 1;
        }
        row = lo;
      }
      if (pre) {
#pragma unroll
        for (int u = 0; u < PR; ++u) {
          const int32_t k = (int32_t)threadIdx.x + u * 256;
          py[u] = list[n0 + (k < nn ? k : 0)];
          po[u] = off[n0 + (k < nn ? k : 0)];
        }
        if (threadIdx.x == 0) po_end = off[n0 + nn];
      }
      // every entry's loads issued before any is used; an idle slot reads
      // the graph's first entry
      int64_t es[BIG_UNROLL];
      bool ok[BIG_UNROLL];
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) {
        const int64_t i = i0 + u;
        ok[u] = i < hi_e;
        es[u] = e_idle;
        if (ok[u]) {
          while (s_off[row + 1] <= i) ++row;  // LDS only
          es[u] = s_base[row] + (i - s_off[row]);
        }
      }
      int32_t xs[BIG_UNROLL], cs[BIG_UNROLL];
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) {
        xs[u] = A.col[es[u]];
        cs[u] = A.w[es[u]];
      }
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) keep(cs[u]);
      uint32_t sw[BIG_UNROLL];
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) sw[u] = st2[(xs[u] - A.v0) >> 4];
      if (pre) {
#pragma unroll
        for (int u = 0; u < PR; ++u) pb[u] = A.rp[py[u]];
        have = true;
      }
      // the tile's in-batch weights as prefix sums, so that a row's part is
      // the difference of two (in 32 bits: every weighted degree fits 31):
      // a thread's four entries in order, the wave's by a scan, the waves'
      // totals added where a prefix is read
      uint32_t pre4[BIG_UNROLL];
      uint32_t run4 = 0;
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) {
        const int32_t i = xs[u] - A.v0;
        const bool inb = ok[u] && ((sw[u] >> (2 * (i & 15))) & 3u) == BS_BATCH;
        const uint32_t v = inb ? (uint32_t)cs[u] : 0u;
        run4 += v;
        pre4[u] = run4;
        into += v;
      }
      const uint32_t wincl = wave_incl_sum<uint32_t>(run4);
      if (lane == 63) s_wt[threadIdx.x >> 6] = wincl;
#pragma unroll
      for (int u = 0; u < BIG_UNROLL; ++u) {
        if (!ok[u]) continue;
        const int32_t p = (int32_t)(i0 + u - lo_e);
        e_w[p] = wincl - run4 + pre4[u];
        e_x[p] = xs[u];
      }
      __syncthreads();
      // P(p): the tile's in-batch weight over positions [0, p]
      const uint32_t wb1 = s_wt[0], wb2 = wb1 + s_wt[1], wb3 = wb2 + s_wt[2];
      auto P = [&](int32_t p) -> uint32_t {
        const int32_t wv = p / (BIG_UNROLL * 64);  // the wave that wrote position p
        return e_w[p] + (wv == 0 ? 0u : wv == 1 ? wb1 : wv == 2 ? wb2 : wb3);
      };
      // per row: its part of the tile; the crossing, if any
      for (int32_t k0 = 0; k0 < nr; k0 += 256) {
        const int32_t k = k0 + (int32_t)threadIdx.x;
        int32_t y = -1, partner = -1;
        if (k < nr) {
          const int64_t a = max(s_off[k], lo_e), b = min(s_off[k + 1], hi_e);
          if (a < b) {
            const int32_t qa = (int32_t)(a - lo_e), qb = (int32_t)(b - lo_e);
            const uint32_t before = qa > 0 ? P(qa - 1) : 0u;
            const int64_t sum = (int64_t)(P(qb - 1) - before);
            if (sum > 0) {
              y = s_y[k];
              // a row wholly inside this tile has no other writer
              const bool whole = s_off[k] >= t0 && s_off[k + 1] <= t1;
              int32_t* rp32 = (int32_t*)(A.rs + y);
              const int32_t old = whole ? *rp32 : atomic_add(rp32, (int32_t)sum);
              if (whole) *rp32 = old + (int32_t)sum;
              if ((int64_t)old < A.lam && A.lam <= (int64_t)old + sum) {
                // the entry whose weight takes r to the cap (prefixes ascend)
                int32_t lo = qa, hi = qb - 1;
                while (lo < hi) {
                  const int32_t mid = (lo + hi) >> 1;
                  if ((int64_t)old + (int64_t)(P(mid) - before) >= A.lam) hi = mid;
                  else lo = mid + 1;
                }
                partner = e_x[lo];
              }
            }
          }
        }
        const bool cross = partner >= 0;
        const uint64_t cm = ballot(cross);
        if (cm) {
          int32_t at = 0;
          if (lane == 0) at = atomicAdd(&c->cap_tail, popc64(cm));
          at = bcast(at, 0);
          if (cross) {
            const int32_t q = at + popc64(cm & lanemask_lt());
            A.capq[q] = y;
            A.capx[q] = partner;
          }
        }
      }
      __syncthreads();  // the slice arrays are reused
    }
  }
  __shared__ int64_t part[4];
  into = wave_sum_i64(into);
  if (lane == 0) part[threadIdx.x >> 6] = into;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t t = part[0] + part[1] + part[2] + part[3];
    if (t) atomicAdd((unsigned long long*)&c->pull_alpha, (unsigned long long)t);
  }
}


// ---- exact rebuild of the bucket queue from the frontier (counting sort)
__global__ void k_sweep_rb_zero(SweepArgs A) {
  for (int64_t i = gtid(); i < SWEEP_BUCKETS; i += gstride()) A.ctl->seg_end[i] = 0;
}

__global__ void __launch_bounds__(256) k_sweep_rb_count(SweepArgs A) {
  __shared__ int32_t h[SWEEP_BUCKETS];
  for (int i = threadIdx.x; i < A.nb; i += 256) h[i] = 0;
  __syncthreads();
  constexpr int RU = 4;  // vertices per thread and step, their words loaded together
  for (int64_t i0 = gtid(); i0 < A.ng; i0 += gstride() * RU) {
    uint64_t w[RU];
#pragma unroll
    for (int k = 0; k < RU; ++k) {
      const int64_t i = i0 + k * gstride();
      w[k] = A.rs[A.v0 + (int32_t)(i < A.ng ? i : 0)];
    }
#pragma unroll
    for (int k = 0; k < RU; ++k) {
      const int32_t rv = rs_r(w[k]);
      if (i0 + k * gstride() < A.ng && rs_stamp(w[k]) == 0 && rv > 0 && (int64_t)rv < A.lam)
        atomicAdd(&h[rv >> A.shift], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < A.nb; i += 256)
    if (h[i]) atomicAdd(&A.ctl->seg_end[i], h[i]);
}

// One workgroup: segment bounds from the counts; lists and pool emptied.
__global__ void __launch_bounds__(1024) k_sweep_rb_scan(SweepArgs A) {
  __shared__ int32_t part[1024];
  SweepCtl* c = A.ctl;
  const int per = (A.nb + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  int32_t s = 0;
  for (int k = 0; k < per && b0 + k < A.nb; ++k) s += c->seg_end[b0 + k];
  // exclusive scan of the 1024 thread sums: within each wave, then over
  // the 16 wave totals
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int32_t incl = wave_incl_sum<int32_t>(s);
  if (lane == 63) part[wave] = incl;
  __syncthreads();
  int32_t before = 0;
  for (int k = 0; k < wave; ++k) before += part[k];
  int32_t run = before + incl - s;
  for (int k = 0; k < per && b0 + k < A.nb; ++k) {
    const int b = b0 + k;
    const int32_t cnt = c->seg_end[b];
    c->seg_cur[b] = run;
    c->fill[b] = run;
    c->seg_end[b] = run + cnt;
    c->head[b] = -1;
    run += cnt;
  }
  __syncthreads();
  for (int wd = threadIdx.x; wd < SWEEP_BUCKETS / 64; wd += 1024) {
    uint64_t bits = 0;
    for (int k = 0; k < 64; ++k) {
      const int b = wd * 64 + k;
      if (b < A.nb && c->seg_end[b] > c->seg_cur[b]) bits |= 1ull << k;
    }
    c->bitmap[wd] = bits;
  }
  if (threadIdx.x == 0) {
    c->pool_next = 0;
    c->rebuilds += 1;
  }
}

// Frontier vertices into their bucket segments: per workgroup a local
// histogram, one range reservation per bucket, then the writes.
__global__ void __launch_bounds__(256) k_sweep_rb_fill(SweepArgs A) {
  __shared__ int32_t h[SWEEP_BUCKETS];
  constexpr int PER = RB_TILE / 256;
  for (int i = threadIdx.x; i < A.nb; i += 256) h[i] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * RB_TILE;
  int32_t bk[PER], rk[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int64_t i = t0 + q * 256 + threadIdx.x;
    bk[q] = -1;
    rk[q] = 0;
    if (i < A.ng) {
      const int32_t v = A.v0 + (int32_t)i;
      const uint64_t u = A.rs[v];
      const int32_t rv = rs_r(u);
      if (rs_stamp(u) == 0 && rv > 0 && (int64_t)rv < A.lam) {
        bk[q] = rv >> A.shift;
        rk[q] = atomicAdd(&h[bk[q]], 1);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < A.nb; i += 256)
    if (h[i]) h[i] = atomicAdd(&A.ctl->fill[i], h[i]);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q)
    if (bk[q] >= 0) A.seg[h[bk[q]] + rk[q]] = A.v0 + (int32_t)(t0 + q * 256 + threadIdx.x);
}

}  // namespace mc
