// The tail of a full-graph capped sweep as many concurrent scans
// (section "Parallel CAPFOREST": Algorithm 1, Lemma 2).
//
// After its last grid-wide batch a sweep has visited almost every vertex;
// what is left is a few thousand vertices below the cap, which the
// sequential kernel would pop one at a time (each pop a chain of dependent
// memory round trips).  Here the visited set S is a prefix that every
// process shares, and the rest is scanned by many processes, one wave each,
// as in Algorithm 1: a process keeps its own r for the vertices it has
// touched (their weight to S, the sweep's r, plus their weight to the
// process's own visited vertices), visits a vertex of largest key (capped at
// lambda-hat) by claiming it in the shared visited array (a compare-and-swap
// on the vertex's word), blacklists a vertex it finds visited by another
// process (when it tries to visit it, or when an edge leads to it), and
// unites x and y on the crossing r(y) < lambda-hat <= r(y) + c(e).
//
// An untouched vertex's key is its weight to S.  The free frontier vertices
// sit in the rebuilt bucket segments, one key per bucket; a shared index
// names the highest bucket that may still hold a free vertex (lowered only
// when a scan finds a bucket fully visited).  Vertices of one bucket tie, so
// a process takes any free vertex of that bucket (each starts looking at its
// own offset, so the processes rarely collide) whenever no vertex it has
// touched has a larger key.  Each visit is thus of a largest key among the
// vertices the process has not blacklisted, and Lemma 2's argument holds for
// every process: q(e) is a lower bound of the connectivity in G minus the
// process's blacklist at the time e is scanned.  alpha of each prefix S +
// pops is the exact cut of that set in G (r counts S and the process's own
// visits), so the best prefix of any process is a real cut.
//
// A process ends when it has no candidate left and every bucket is fully
// visited, or when its LDS map fills (early termination, safe by Lemma 2).
// Vertices left unvisited stay single blocks for the next round.
#pragma once
#include "smallsweep.h"
#include "sweep.h"

namespace mc {

constexpr int TAIL_WAVES = 4;        // processes per workgroup (one wave each)
constexpr int TAIL_SLOTS = 1024;     // LDS map slots per process
constexpr int32_t TAIL_SID = 0x7FFFFFFE;  // best-prefix record of a tail process

// Visit stamp of process f (the high half of a vertex's word; the low half
// then holds the visit's step).  Bit 31 keeps these apart from the sweep's
// stamps, which are positive.
__device__ __forceinline__ uint32_t tail_pop(int32_t f) { return 0x80000000u | (uint32_t)f; }

// Relaxed device-scope atomics on global memory.
template <typename T>
__device__ __forceinline__ T tail_fetch_add(MC_GLOBAL T* p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T tail_fetch_max(MC_GLOBAL T* p, T v) {
  return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T tail_fetch_min(MC_GLOBAL T* p, T v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t tail_hash(int32_t v) {
  return (int32_t)(((uint32_t)v * 0x9E3779B1u) >> (32 - 10)) & (TAIL_SLOTS - 1);
}

// Insert v (not yet present) with r0; the slot, or -1 when the probe window
// is exhausted.
// v's slot, inserting v with r0 if it is new (lanes that insert the same v
// at once write the same r0); -1 when the probe window is exhausted.
__device__ __forceinline__ int32_t tail_insert(int32_t* keys, int32_t* rv, int32_t v, int32_t r0) {
  int32_t h = tail_hash(v);
  for (int probe = 0; probe < 64; ++probe) {
    const int32_t prev = atomicCAS(&keys[h], -1, v);
    if (prev == -1) {
      rv[h] = r0;
      return h;
    }
    if (prev == v) return h;
    h = (h + 1) & (TAIL_SLOTS - 1);
  }
  return -1;
}

__device__ __forceinline__ int32_t tail_find(const int32_t* keys, int32_t v) {
  int32_t h = tail_hash(v);
  for (int probe = 0; probe < 64; ++probe) {
    const int32_t k = keys[h];
    if (k == v) return h;
    if (k == -1) return -1;
    h = (h + 1) & (TAIL_SLOTS - 1);
  }
  return -1;
}

// The shared record of graph A (one wave): the highest non-empty bucket of
// the rebuilt segments (one key per bucket: the tail runs only with shift 0).
__global__ void k_sweep_tail_init(SweepArgs A) {
  if (threadIdx.x >= 64 || blockIdx.x != 0) return;
  SweepCtl* c = A.ctl;
  int32_t top = -1;
  for (int32_t b = lane_id(); b < A.nb; b += 64)
    if (c->seg_end[b] > c->seg_cur[b]) top = b;
  top = (int32_t)wave_max_u32((uint32_t)(top + 1)) - 1;
  if (lane_id() == 0) {
    c->tail_total = A.nb > 0 ? c->seg_end[A.nb - 1] : 0;
    c->tail_cursor = top;  // the highest bucket that may hold a free vertex
    c->tail_best = ~0ull;
    c->tail_pops = 0;
    c->tail_rows = 0;
  }
}

__global__ void __launch_bounds__(64 * TAIL_WAVES) k_sweep_tail(SweepArgs Aa, int32_t nforks) {
  const SweepDev A = dev_view(Aa);
  __shared__ int32_t s_key[TAIL_WAVES][TAIL_SLOTS];
  __shared__ int32_t s_r[TAIL_WAVES][TAIL_SLOTS];  // r of a touched vertex; -1 empty slot, -2 visited here,
                                                   // -3 blacklisted (visited elsewhere)
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int32_t f = blockIdx.x * TAIL_WAVES + wave;
  if (f >= nforks) return;  // whole waves: no barrier below spans waves
  int32_t* keys = s_key[wave];
  int32_t* rv = s_r[wave];
  for (int i = lane; i < TAIL_SLOTS; i += 64) {
    keys[i] = -1;
    rv[i] = -1;
  }
  ss_wave_sync();
  MC_GLOBAL SweepCtl* c = A.ctl;
  const int64_t lam = A.lam;
  const uint32_t mark = tail_pop(f);
  int64_t alpha = c->alpha;  // c(S)
  const int32_t vis0 = c->visited;
  int32_t step = 0, best_k = 0, used = 0;
  int64_t best = INT64_MAX, rows = 0;
  bool full = false;
  const uint32_t spread = (uint32_t)f * 0x9E3779B1u;  // where this process looks inside a bucket
  // every iteration visits a vertex, blacklists a touched vertex, or finds a
  // bucket without a free vertex (at most one per bucket and visit)
  const int32_t max_it = 4 * TAIL_SLOTS + 2 * A.nb + 2 * c->tail_total + 64;
  for (int32_t it = 0; it < max_it && !full; ++it) {
    // the largest key among touched vertices still unvisited here
    uint64_t cand = 0;
    for (int i = lane; i < TAIL_SLOTS; i += 64) {
      const int32_t r = rv[i];
      const int64_t k = r < 0 ? -1 : min((int64_t)r, lam);
      const uint64_t p = k < 0 ? 0ull : ((uint64_t)(k + 1) << 32) | (uint32_t)i;
      cand = p > cand ? p : cand;
    }
    cand = wave_max_u64(cand);
    const int64_t lkey = cand ? (int64_t)(cand >> 32) - 1 : -1;
    // the largest key of an untouched free vertex is at most the top bucket's
    const int32_t top = ld_relaxed(&c->tail_cursor);
    if (lkey < 0 && top < 0) break;  // nothing left for this process
    int32_t x = -1, slot = -1;
    if (lkey >= (int64_t)top) {
      slot = (int32_t)(uint32_t)cand;
      x = keys[slot];
    } else {
      // a free vertex of the top bucket, from this process's offset on
      const int32_t b0 = ld_relaxed(&c->seg_cur[top]), b1 = ld_relaxed(&c->seg_end[top]);
      const int32_t size = b1 - b0;
      const int32_t off = (int32_t)(((uint64_t)spread * (uint32_t)size) >> 32);
      int32_t hv = -1;
      for (int32_t k0 = 0; k0 < size; k0 += 64) {
        const int32_t k = k0 + lane;
        const int32_t i = b0 + (off + (k < size ? k : 0)) % size;
        const int32_t v = ld_relaxed(A.seg + i);
        const uint32_t st = (uint32_t)(ld_relaxed(A.rs + v) >> 32);
        const uint64_t fr = ballot(k < size && st == 0);
        if (fr) {
          hv = __builtin_amdgcn_readlane(v, __builtin_ctzll(fr));
          break;
        }
      }
      if (hv < 0) {
        // the bucket is fully visited: the next one down becomes the top
        if (lane == 0) {
          int32_t expected = top;
          __hip_atomic_compare_exchange_strong(&c->tail_cursor, &expected, top - 1, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        continue;
      }
      x = hv;
      slot = tail_find(keys, x);  // touched here before: its r includes this process's part
    }
    // visit x: claim it in the shared visited array
    int ok = 0;
    if (lane == 0) {
      int32_t expected = 0;
      ok = __hip_atomic_compare_exchange_strong(rs_stamp_ptr(A.rs + x), &expected, (int32_t)mark,
                                                __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
               ? 1
               : 0;
    }
    ok = __builtin_amdgcn_readlane(ok, 0);
    if (!ok) {
      // visited by another process: blacklisted here
      if (slot >= 0 && lane == 0) rv[slot] = -3;
      ss_wave_sync();
      continue;
    }
    // r(x): from the map, or (untouched here) its weight to S, still in the
    // low half of its word
    const int32_t rx = slot >= 0 ? rv[slot] : rs_r(ld_relaxed(A.rs + x));
    ss_wave_sync();
    if (lane == 0 && slot >= 0) rv[slot] = -2;
    ++step;
    const int64_t xa = A.rp[x], xb = A.rp[x + 1];
    const int64_t cdx = A.cdeg[x];
    rows += xb - xa;
    // the low half becomes the visit's step (the side of a best prefix)
    if (lane == 0) st_relaxed((MC_GLOBAL int32_t*)(A.rs + x), step);
    alpha += cdx - 2 * (int64_t)rx;
    if (vis0 + step < A.ng && alpha < best) {
      best = alpha;
      best_k = step;
    }
    ss_wave_sync();
    for (int64_t base = xa; base < xb; base += 64) {
      const int64_t e = base + lane;
      const bool in = e < xb;
      const int64_t ec = in ? e : base;
      const int32_t y = A.col[ec];
      const int32_t cw = A.w[ec];
      const bool act = in && y != x;
      const uint64_t wd = ld_relaxed(A.rs + (act ? y : x));
      // visited by the sweep or by some process: skipped (blacklisted)
      const bool live = act && rs_stamp(wd) == 0;
      int32_t sl = -1;
      if (live) sl = tail_insert(keys, rv, y, rs_r(wd));  // new: its weight to S; present: unchanged
      const uint64_t lost = ballot(live && sl < 0);
      ss_wave_sync();
      bool cross = false;
      if (sl >= 0) {
        const int32_t old = atomicAdd(&rv[sl], cw);
        cross = old >= 0 && (int64_t)old < lam && lam <= (int64_t)old + cw;
      }
      const uint64_t cm = ballot(cross);
      if (cm) {
        int32_t at = 0;
        if (lane == 0) at = tail_fetch_add(&c->cap_tail, (int32_t)popc64(cm));
        at = bcast(at, 0);
        if (cross) {
          const int32_t i = at + popc64(cm & lanemask_lt());
          if (i < A.ng) {  // beyond the FIFO's room a pair is dropped (fewer unions are safe)
            A.capq[i] = y;
            A.capx[i] = x;
          }
        }
      }
      if (lost) full = true;
      ss_wave_sync();
    }
  }
  if (lane == 0) {
    tail_fetch_add(&c->tail_pops, step);
    tail_fetch_add(&c->tail_rows, rows);
    if (best < lam) {
      c->tail_k[f] = best_k;
      tail_fetch_min(&c->tail_best, ((uint64_t)best << 32) | (uint32_t)f);
    }
  }
}

}  // namespace mc
