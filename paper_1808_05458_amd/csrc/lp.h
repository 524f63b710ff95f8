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
// the row length (it cannot fill).  Longer rows take a workgroup and a fixed
// map; a row with more entries than one pass holds is split into passes by a
// hash of the label, so each pass sees a disjoint set of labels; a pass whose
// map would fill is redone with twice the passes.
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
constexpr int LP_BLOCK_LOAD = 4096;   // entries per pass of the workgroup path
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
  int32_t* heavy;          // rows longer than LP_WAVE_MAX, for the workgroup path
  int32_t* heavy_count;
  int32_t collect;         // append long rows to `heavy` (first sweep of a level)
};

__device__ __forceinline__ uint32_t lp_hash(uint32_t label) { return label * 0x9E3779B1u; }

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
    if (d > LP_WAVE_MAX) {
      if (A.collect && lane == 0) A.heavy[atomicAdd(A.heavy_count, 1)] = (int32_t)v;
      continue;
    }
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

// One workgroup per long row, over the list the wave path collected.
__global__ void __launch_bounds__(LP_BLOCK_THREADS) k_lp_block(LpArgs A) {
  __shared__ uint32_t keys[LP_BLOCK_SLOTS];
  __shared__ uint32_t sums[LP_BLOCK_SLOTS];
  __shared__ int32_t used, overflow;
  __shared__ uint64_t wbest[LP_BLOCK_THREADS / 64];
  constexpr int LOG = __builtin_ctz(LP_BLOCK_SLOTS);
  constexpr uint32_t MASK = LP_BLOCK_SLOTS - 1;
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int32_t cnt = *A.heavy_count;
  for (int32_t item = blockIdx.x; item < cnt; item += gridDim.x) {
    const int32_t v = A.heavy[item];
    const int64_t e0 = A.rp[v], e1 = A.rp[v + 1];
    uint32_t passes = (uint32_t)((e1 - e0 + LP_BLOCK_LOAD - 1) / LP_BLOCK_LOAD);
    uint64_t best = 0;  // meaningful in thread 0
    for (uint32_t p = 0; p < passes; ++p) {
      for (int i = threadIdx.x; i < LP_BLOCK_SLOTS; i += LP_BLOCK_THREADS) { keys[i] = LP_EMPTY; sums[i] = 0; }
      if (threadIdx.x == 0) { used = 0; overflow = 0; }
      __syncthreads();
      for (int64_t e = e0 + threadIdx.x; e < e1; e += LP_BLOCK_THREADS) {
        const int32_t y = A.col[e];
        if (y == v) continue;
        const uint32_t label = (uint32_t)A.cur[y];
        // the pass of a label: a second hash, independent of the slot hash
        if (passes > 1 && ((label * 0x85EBCA6Bu) ^ (label >> 13)) % passes != p) continue;
        uint32_t h = (lp_hash(label) >> (32 - LOG)) & MASK;
        const uint32_t c = (uint32_t)A.w[e];
        while (true) {
          uint32_t k = keys[h];
          if (k == LP_EMPTY) {
            // claim a new slot only while the map stays at most 3/4 full
            if (atomicAdd(&used, 1) >= (LP_BLOCK_SLOTS * 3) / 4) {
              atomicSub(&used, 1);
              overflow = 1;
              break;
            }
            k = atomicCAS(&keys[h], LP_EMPTY, label);
            if (k == LP_EMPTY) { atomicAdd(&sums[h], c); break; }
            atomicSub(&used, 1);
          }
          if (k == label) { atomicAdd(&sums[h], c); break; }
          h = (h + 1) & MASK;
        }
      }
      __syncthreads();
      if (overflow) {  // block-uniform: redo the row with twice the passes
        passes *= 2;
        p = (uint32_t)-1;
        if (threadIdx.x == 0) best = 0;
        __syncthreads();
        continue;
      }
      uint64_t b = 0;
      for (int i = threadIdx.x; i < LP_BLOCK_SLOTS; i += LP_BLOCK_THREADS) {
        const uint32_t k = keys[i];
        if (k != LP_EMPTY) {
          const uint64_t c = lp_pack(sums[i], k);
          b = c > b ? c : b;
        }
      }
      b = wave_max_u64(b);
      if (lane == 0) wbest[wave] = b;
      __syncthreads();
      if (threadIdx.x == 0)
        for (int k = 0; k < LP_BLOCK_THREADS / 64; ++k) best = wbest[k] > best ? wbest[k] : best;
      __syncthreads();
    }
    if (threadIdx.x == 0) A.nxt[v] = best ? (int32_t)~(uint32_t)best : A.cur[v];
  }
}

// Label classes -> dense block ids, numbered by label value: flag every label
// in use, prefix-sum the flags, then look each vertex's label up.
__global__ void k_lp_flag(int32_t n, const int32_t* label, const int32_t* gid, const int32_t* active,
                          int32_t* flag) {
  for (int64_t v = gtid(); v < n; v += gstride())
    if (active[gid[v]]) flag[label[v]] = 1;
}

__global__ void k_lp_relabel(int32_t n, const int32_t* label, const int32_t* gid, const int32_t* active,
                             const int32_t* flag, const int32_t* newid, int32_t* lab, int32_t* ngid,
                             int32_t* nnew) {
  for (int64_t v = gtid(); v - lane_id() < n; v += gstride()) {  // wave-uniform bound
    const bool ok = v < n;
    const int32_t g = ok ? gid[v] : -1;
    const bool kept = ok && active[g];
    const bool head = kept && flag[v];  // v is the label of a class (of its own graph)
    if (ok) lab[v] = kept ? newid[label[v]] : -1;
    if (head) ngid[newid[v]] = g;
    wave_add_by_key(nnew, g, 1, head);
  }
}

}  // namespace mc
