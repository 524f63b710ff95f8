// Label propagation for the VieCut-style upper bound (section "Inexact
// Shared-Memory Minimum Cuts"; Algorithm 2 starts from that bound).
//
// One synchronous sweep: every vertex takes, among its neighbours' labels
// before the sweep, the one with the largest total edge weight, ties to the
// smallest label; a vertex without neighbours keeps its label.  The result
// does not depend on the schedule, so the bound built on it is reproducible.
//
// The per-label sums of a row are gathered in an LDS open-addressing map.
// Rows up to LP_WAVE_MAX entries take one wave and a map of at least twice
// the row length (it cannot fill).  Longer rows become workgroup items: a
// row with more entries than one pass holds is split into passes by a hash
// of the label, each pass an item of its own on any workgroup, so the
// passes see disjoint label sets; a pass whose map would fill splits itself
// further.  The best candidate of every item is folded into the row by a
// 64-bit atomic max.
//
// The weights of one vertex sum to less than 2^31 (the total weight of a
// graph is limited to 2(2^31 - 1) over its entries), so a map slot's sum
// fits 32 bits and (sum << 32) | ~label orders candidates by larger sum,
// then smaller label.
#pragma once
#include "capforest.h"
#include "dev.h"

namespace mc {

constexpr int LP_WAVE_MAX = 256;      // longest row of the one-wave path
constexpr int LP_WAVE_SLOTS = 512;    // its map (>= 2 * LP_WAVE_MAX)
constexpr int LP_WAVES = 4;           // waves per workgroup of the one-wave path
constexpr int LP_BLOCK_SLOTS = 8192;  // map of the workgroup path
constexpr int LP_BLOCK_LOAD = 4096;   // entries per pass of the workgroup path (<= slots / 2)
constexpr int LP_BLOCK_THREADS = 256;
constexpr uint32_t LP_EMPTY = 0xFFFFFFFFu;

struct LpArgs {
  int32_t n;
  const int64_t* rp;
  const int32_t* col;
  const int32_t* w;
  const int32_t* gid;
  const int32_t* active;   // per graph: only these graphs' vertices are swept
  const int32_t* cur;      // labels before the sweep
  int32_t* nxt;            // labels after it
  const int32_t* item_off; // exclusive prefix of the workgroup items per vertex
  const int32_t* nitems;   // device: total workgroup items
  uint64_t* best;          // per vertex: best (sum, label) over its items, 0 = none
};

__device__ __forceinline__ uint32_t lp_hash(uint32_t label) { return label * 0x9E3779B1u; }

// A second hash, a bijection of the label, that splits long rows into passes.
__device__ __forceinline__ uint32_t lp_hash2(uint32_t label) {
  uint32_t h = label * 0x85EBCA6Bu;
  return h ^ (h >> 13);
}

// Add c to the slot of `label`, inserting it if absent.  The caller
// guarantees an empty slot exists.
__device__ __forceinline__ void lp_add(uint32_t* keys, uint32_t* sums, uint32_t mask, int shift, uint32_t label,
                                       uint32_t c) {
  uint32_t h = (lp_hash(label) >> shift) & mask;
  while (true) {
    const uint32_t k = atomicCAS(&keys[h], LP_EMPTY, label);
    if (k == LP_EMPTY || k == label) {
      atomicAdd(&sums[h], c);
      return;
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ uint64_t lp_pack(uint32_t sum, uint32_t label) {
  return ((uint64_t)sum << 32) | (uint32_t)~label;
}

__device__ __forceinline__ bool lp_long(const LpArgs& A, int64_t v) {
  return A.rp[v + 1] - A.rp[v] > LP_WAVE_MAX && A.active[A.gid[v]];
}

// Workgroup items of a vertex: none for rows the wave path takes, else one
// per pass of at most LP_BLOCK_LOAD entries.
struct LpItems {
  LpArgs A;
  __device__ __forceinline__ int32_t operator()(int64_t v) const {
    if (!lp_long(A, v)) return 0;
    const int64_t d = A.rp[v + 1] - A.rp[v];
    return (int32_t)((d + LP_BLOCK_LOAD - 1) / LP_BLOCK_LOAD);
  }
};

// One wave per vertex for rows up to LP_WAVE_MAX entries.
__global__ void __launch_bounds__(64 * LP_WAVES) k_lp_wave(LpArgs A) {
  __shared__ uint32_t keys_s[LP_WAVES][LP_WAVE_SLOTS];
  __shared__ uint32_t sums_s[LP_WAVES][LP_WAVE_SLOTS];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  uint32_t* keys = keys_s[wave];
  uint32_t* sums = sums_s[wave];
  const int64_t nw = (int64_t)gridDim.x * LP_WAVES;
  for (int64_t v = (int64_t)blockIdx.x * LP_WAVES + wave; v < A.n; v += nw) {
    if (!A.active[A.gid[v]]) continue;
    const int64_t e0 = A.rp[v], e1 = A.rp[v + 1];
    const int64_t d = e1 - e0;
    if (d > LP_WAVE_MAX) continue;  // a workgroup item
    // map size: a power of two >= max(64, 2d)
    int logm = 6;
    while ((1ll << logm) < 2 * d) ++logm;
    const uint32_t m = 1u << logm, mask = m - 1;
    const int shift = 32 - logm;
    for (uint32_t i = lane; i < m; i += 64) { keys[i] = LP_EMPTY; sums[i] = 0; }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int64_t e = e0 + lane; e < e1; e += 64) {
      const int32_t y = A.col[e];
      if (y != (int32_t)v) lp_add(keys, sums, mask, shift, (uint32_t)A.cur[y], (uint32_t)A.w[e]);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    uint64_t best = 0;
    for (uint32_t i = lane; i < m; i += 64) {
      const uint32_t k = keys[i];
      if (k != LP_EMPTY) {
        const uint64_t c = lp_pack(sums[i], k);
        best = c > best ? c : best;
      }
    }
    best = wave_max_u64(best);
    if (lane == 0) A.nxt[v] = best ? (int32_t)~(uint32_t)best : A.cur[v];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
}

// Workgroup items: pass p of a long row.  A row of d entries has
// P = ceil(d / LP_BLOCK_LOAD) passes; pass p gathers the labels whose second
// hash is p modulo P, so the passes of one row see disjoint label sets and
// run on different workgroups.  A pass whose map would pass 3/4 full splits
// itself by the next hash digit into twice as many sub-passes and starts
// over.  Every item folds its best (sum, label) into best[v].
__global__ void __launch_bounds__(LP_BLOCK_THREADS) k_lp_items(LpArgs A) {
  __shared__ uint32_t keys[LP_BLOCK_SLOTS];
  __shared__ uint32_t sums[LP_BLOCK_SLOTS];
  __shared__ int32_t used, overflow;
  __shared__ uint64_t wbest[LP_BLOCK_THREADS / 64];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int32_t nitems = *A.nitems;
  for (int32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    // the vertex: the last v with item_off[v] <= item (its range is non-empty)
    int32_t lo = 0, hi = A.n - 1;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo + 1) / 2;
      if (A.item_off[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    const int32_t v = lo;
    const int64_t e0 = A.rp[v], e1 = A.rp[v + 1];
    const int64_t d = e1 - e0;
    const uint32_t P = (uint32_t)((d + LP_BLOCK_LOAD - 1) / LP_BLOCK_LOAD);
    const uint32_t p = (uint32_t)(item - A.item_off[v]);
    // map: a power of two >= 2d for a single pass (it cannot fill), else all slots
    int logm = 6;
    while ((1ll << logm) < 2 * d && (1 << logm) < LP_BLOCK_SLOTS) ++logm;
    const uint32_t m = 1u << logm, mask = m - 1;
    const int shift = 32 - logm;
    uint32_t K = 1;     // sub-passes of this pass
    uint64_t best = 0;  // meaningful in thread 0
    for (uint32_t k = 0; k < K; ++k) {
      for (uint32_t i = threadIdx.x; i < m; i += LP_BLOCK_THREADS) { keys[i] = LP_EMPTY; sums[i] = 0; }
      if (threadIdx.x == 0) { used = 0; overflow = 0; }
      __syncthreads();
      for (int64_t e = e0 + threadIdx.x; e < e1; e += LP_BLOCK_THREADS) {
        const int32_t y = A.col[e];
        if (y == v) continue;
        const uint32_t label = (uint32_t)A.cur[y];
        const uint32_t h2 = lp_hash2(label);
        if (P > 1 && h2 % P != p) continue;
        if (K > 1 && (h2 / P) % K != k) continue;
        uint32_t h = (lp_hash(label) >> shift) & mask;
        const uint32_t c = (uint32_t)A.w[e];
        while (true) {
          uint32_t key = keys[h];
          if (key == LP_EMPTY) {
            // claim a new slot only while the map stays at most 3/4 full
            if (atomicAdd(&used, 1) >= (int32_t)(m * 3 / 4)) {
              atomicSub(&used, 1);
              overflow = 1;
              break;
            }
            key = atomicCAS(&keys[h], LP_EMPTY, label);
            if (key == LP_EMPTY) { atomicAdd(&sums[h], c); break; }
            atomicSub(&used, 1);
          }
          if (key == label) { atomicAdd(&sums[h], c); break; }
          h = (h + 1) & mask;
        }
      }
      __syncthreads();
      if (overflow) {  // workgroup-uniform: split into twice the sub-passes
        K *= 2;
        k = (uint32_t)-1;
        if (threadIdx.x == 0) best = 0;
        __syncthreads();
        continue;
      }
      uint64_t b = 0;
      for (uint32_t i = threadIdx.x; i < m; i += LP_BLOCK_THREADS) {
        const uint32_t key = keys[i];
        if (key != LP_EMPTY) {
          const uint64_t c = lp_pack(sums[i], key);
          b = c > b ? c : b;
        }
      }
      b = wave_max_u64(b);
      if (lane == 0) wbest[wave] = b;
      __syncthreads();
      if (threadIdx.x == 0)
        for (int q = 0; q < LP_BLOCK_THREADS / 64; ++q) best = wbest[q] > best ? wbest[q] : best;
      __syncthreads();
    }
    if (threadIdx.x == 0 && best) atomic_max_u64(A.best + v, best);
  }
}

// Long rows take the best over their items; best is cleared for the next sweep.
__global__ void k_lp_finish(LpArgs A) {
  for (int64_t v = gtid(); v < A.n; v += gstride()) {
    if (!lp_long(A, v)) continue;
    const uint64_t b = A.best[v];
    A.nxt[v] = b ? (int32_t)~(uint32_t)b : A.cur[v];
    A.best[v] = 0;
  }
}

// Label classes -> dense block ids, numbered by label value: flag every label
// in use, prefix-sum the flags, then look each vertex's label up.
// carry: graphs not swept keep every vertex as a class of its own (their
// labels were not written), so the level graph still holds them.
__global__ void k_lp_flag(int32_t n, const int32_t* label, const int32_t* gid, const int32_t* active,
                          int32_t carry, int32_t* flag) {
  for (int64_t v = gtid(); v < n; v += gstride()) {
    if (active[gid[v]]) flag[label[v]] = 1;
    else if (carry) flag[v] = 1;
  }
}

__global__ void k_lp_relabel(int32_t n, const int32_t* label, const int32_t* gid, const int32_t* active,
                             int32_t carry, const int32_t* flag, const int32_t* newid, int32_t* lab,
                             int32_t* ngid, int32_t* nnew) {
  for (int64_t v = gtid(); v - lane_id() < n; v += gstride()) {  // wave-uniform bound
    const bool ok = v < n;
    const int32_t g = ok ? gid[v] : -1;
    const bool swept = ok && active[g];
    const bool kept = swept || (ok && carry);
    const bool head = kept && flag[v];  // v is the label of a class (of its own graph)
    if (ok) lab[v] = kept ? newid[swept ? label[v] : (int32_t)v] : -1;
    if (head) ngid[newid[v]] = g;
    wave_add_by_key(nnew, g, 1, head);
  }
}

}  // namespace mc
