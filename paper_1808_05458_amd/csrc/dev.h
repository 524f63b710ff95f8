// Device-side helpers shared by the min-cut kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MC_WAVE 64
// Global memory.  Pointers that kernels read from device memory (argument
// arrays) are generic to the compiler, and accesses through generic
// pointers are flat accesses, which also count against the LDS wait
// counter; typing them as global gives global accesses.
#define MC_GLOBAL __attribute__((address_space(1)))

namespace mc {

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// Rank of a vertex among equal priority keys (the larger rank is taken
// first), for the priority-queue orders of section "Priority Queue
// Implementations".  tick is the step of the vertex's last key increase;
// one step's increases share it, and a contracted graph's rows list their
// neighbours by increasing id, so the id's low 16 bits order the increases
// of one step as a bucket would have received them.  Order 1 (bucket
// queue): earliest increase first, then the smaller id.  Order 2 (bucket
// stack): latest increase first, then the larger id.  Order 3 (heap): a
// fixed pseudo-random order of the vertices, favouring neither old nor new
// increases.
__device__ __forceinline__ uint32_t tie_rank(int32_t order, uint32_t tick, uint32_t v) {
  const uint32_t lo = v & 0xFFFFu;
  if (order == 1) return ((0xFFFFu - (tick & 0xFFFFu)) << 16) | (0xFFFFu - lo);
  if (order == 2) return ((tick & 0xFFFFu) << 16) | lo;
  return ((v * 0x9E3779B1u) & 0xFFFF0000u) | (0xFFFFu - lo);
}

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) { return __shfl(v, src, MC_WAVE); }

// The value of lane l, which must be the same for the whole wave (a
// constant, or taken from a ballot): a scalar lane read, where shfl is an
// LDS permute with its round trip.  Lane l must have computed v.
template <typename T>
__device__ __forceinline__ T bcast(T v, int l) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}

// Takes v as used at this point: keeps the compiler from sinking the load
// that produced it into the branch that consumes it, so loads issued
// together are waited for together (a load sunk into a branch issues only
// after the branch's condition, which often waits for another load).
__device__ __forceinline__ void keep(int32_t& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void keep(uint32_t& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void keep(int64_t& v) { asm volatile("" : "+v"(v)); }

// Wave-wide reductions (all lanes receive the result).
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, MC_WAVE);
  return v;
}
__device__ __forceinline__ int32_t wave_sum_i32(int32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, MC_WAVE);
  return v;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t t = __shfl_xor(v, o, MC_WAVE);
    v = t < v ? t : v;
  }
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t t = __shfl_xor(v, o, MC_WAVE);
    v = t > v ? t : v;
  }
  return v;
}

// Wave-wide maximum of a 32-bit value (all lanes receive it; all 64 lanes
// must be active).  DPP moves inside each row of 16 lanes (swap neighbours,
// swap pairs, half-row mirror, row mirror) leave every row holding its
// maximum; four lane reads combine the rows.  No LDS traffic, unlike the
// permute-based shuffles above.
// DPP controls: quad_perm 1,0,3,2 and 2,3,0,1, row_half_mirror, row_mirror.
// Applied in this order, each lane combines with a lane of the other half of
// a group that doubles every time (2, 4, 8, 16 lanes).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ int64_t dpp_i64(int64_t v) {
  const uint32_t lo = dpp_u32<CTRL>((uint32_t)(uint64_t)v);
  const uint32_t hi = dpp_u32<CTRL>((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int64_t readlane_i64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  uint32_t t;
  t = dpp_u32<0xB1>(v);
  v = t > v ? t : v;
  t = dpp_u32<0x4E>(v);
  v = t > v ? t : v;
  t = dpp_u32<0x141>(v);
  v = t > v ? t : v;
  t = dpp_u32<0x140>(v);
  v = t > v ? t : v;
  const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
  const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
  const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32);
  const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
  const uint32_t ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// Wave-wide 64-bit sum by the same DPP steps (all 64 lanes active); the
// result is uniform.
__device__ __forceinline__ int64_t wave_sum_i64_dpp(int64_t v) {
  v += dpp_i64<0xB1>(v);
  v += dpp_i64<0x4E>(v);
  v += dpp_i64<0x141>(v);
  v += dpp_i64<0x140>(v);
  return readlane_i64(v, 0) + readlane_i64(v, 16) + readlane_i64(v, 32) + readlane_i64(v, 48);
}

// Lane-order scans and shifts over the wave's 64 lanes by DPP (all lanes
// active), without LDS traffic: inside each row of 16 lanes by shifts of 1,
// 2, 4 and 8 lanes (Hillis-Steele), then across rows by broadcasting lane
// 15 to rows 1 and 3 and lane 31 to rows 2 and 3.  A lane whose source is
// outside its row, or whose row is masked off, keeps `old` (the identity).
// DPP controls: row_shr:n = 0x110 + n, wave_shl:1 = 0x130, wave_shr:1 =
// 0x138, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int CTRL, int ROWS>
__device__ __forceinline__ int32_t dpp_old_i32(int32_t old, int32_t v) {
  return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}
__device__ __forceinline__ int32_t wave_incl_max_i32(int32_t v) {
  constexpr int32_t LO = INT32_MIN;
  int32_t t;
  t = dpp_old_i32<0x111, 0xF>(LO, v); v = t > v ? t : v;
  t = dpp_old_i32<0x112, 0xF>(LO, v); v = t > v ? t : v;
  t = dpp_old_i32<0x114, 0xF>(LO, v); v = t > v ? t : v;
  t = dpp_old_i32<0x118, 0xF>(LO, v); v = t > v ? t : v;
  t = dpp_old_i32<0x142, 0xA>(LO, v); v = t > v ? t : v;
  t = dpp_old_i32<0x143, 0xC>(LO, v); v = t > v ? t : v;
  return v;
}
template <int CTRL, int ROWS>
__device__ __forceinline__ int64_t dpp_old_i64(int64_t old, int64_t v) {
  const int32_t lo = dpp_old_i32<CTRL, ROWS>((int32_t)(uint32_t)(uint64_t)old, (int32_t)(uint32_t)(uint64_t)v);
  const int32_t hi = dpp_old_i32<CTRL, ROWS>((int32_t)((uint64_t)old >> 32), (int32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ int64_t wave_incl_sum_i64(int64_t v) {
  v += dpp_old_i64<0x111, 0xF>(0, v);
  v += dpp_old_i64<0x112, 0xF>(0, v);
  v += dpp_old_i64<0x114, 0xF>(0, v);
  v += dpp_old_i64<0x118, 0xF>(0, v);
  v += dpp_old_i64<0x142, 0xA>(0, v);
  v += dpp_old_i64<0x143, 0xC>(0, v);
  return v;
}
// lane l receives lane l - 1's value (lane 0: `first`), or lane l + 1's
// (lane 63: `last`)
__device__ __forceinline__ int32_t wave_shr1_i32(int32_t v, int32_t first) { return dpp_old_i32<0x138, 0xF>(first, v); }
__device__ __forceinline__ int64_t wave_shr1_i64(int64_t v, int64_t first) { return dpp_old_i64<0x138, 0xF>(first, v); }
__device__ __forceinline__ int32_t wave_shl1_i32(int32_t v, int32_t last) { return dpp_old_i32<0x130, 0xF>(last, v); }

// The same for any 32- or 64-bit integer type.  Call with every lane of
// the wave active, never inside a lane-dependent branch or short circuit:
// a lane that sits out gives its neighbours the fallback value instead of
// its own.
template <int CTRL, int ROWS, typename T>
__device__ __forceinline__ T dpp_old(T old, T v) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp_old_i32<CTRL, ROWS>(__builtin_bit_cast(int32_t, old),
                                                        __builtin_bit_cast(int32_t, v)));
  } else {
    return __builtin_bit_cast(T, dpp_old_i64<CTRL, ROWS>(__builtin_bit_cast(int64_t, old),
                                                        __builtin_bit_cast(int64_t, v)));
  }
}
template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v) {
  v += dpp_old<0x111, 0xF>((T)0, v);
  v += dpp_old<0x112, 0xF>((T)0, v);
  v += dpp_old<0x114, 0xF>((T)0, v);
  v += dpp_old<0x118, 0xF>((T)0, v);
  v += dpp_old<0x142, 0xA>((T)0, v);
  v += dpp_old<0x143, 0xC>((T)0, v);
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_shr1(T v, T first) { return dpp_old<0x138, 0xF>(first, v); }
template <typename T>
__device__ __forceinline__ T wave_shl1(T v, T last) { return dpp_old<0x130, 0xF>(last, v); }

// Relaxed device-scope loads and stores for data other waves update.
template <typename T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_relaxed(const MC_GLOBAL T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(MC_GLOBAL T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Relaxed device-scope fetch-add, for generic and global pointers.
template <typename P, typename T>
__device__ __forceinline__ T atomic_add(P p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Lock-free union-find over int32 parents.  Invariant: parent[v] <= v, so a
// root is always linked under a smaller root and path halving only ever
// shortens a path to an ancestor; concurrent finds and unions stay safe.
template <typename P>
__device__ __forceinline__ int32_t uf_find(P parent, int32_t x) {
  int32_t p = ld_relaxed(parent + x);
  while (p != x) {
    int32_t gp = ld_relaxed(parent + p);
    if (gp != p) st_relaxed(parent + x, gp);  // halving: point at grandparent
    x = p;
    p = gp;
  }
  return x;
}

// Returns true if this call merged two different sets.
template <typename P>
__device__ __forceinline__ bool uf_union(P parent, int32_t a, int32_t b) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return false;
    if (a > b) { int32_t t = a; a = b; b = t; }
    // link the larger root b under the smaller root a
    int32_t expected = b;
    if (__hip_atomic_compare_exchange_strong(parent + b, &expected, a, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return true;
    b = expected;  // b gained a parent meanwhile; retry from there
  }
}

// The same union with the root of smaller key(root) kept as the root.  Any
// fixed strict total order of the vertices keeps the forest acyclic: a root
// is only ever linked under a root of smaller key, whatever order linked
// the trees before.  The order decides the shape: when most pairs join a
// vertex that was never linked to a tree that grows, keying the roots by
// when they joined (earliest first) links each newcomer under the old root
// with a compare-and-swap on its own word, where an order by vertex id
// would keep moving the big tree's root and make every pair retry on it.
template <typename P, typename Key>
__device__ __forceinline__ bool uf_union_by(P parent, int32_t a, int32_t b, Key key) {
  while (true) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return false;
    if (key(a) > key(b)) { int32_t t = a; a = b; b = t; }
    int32_t expected = b;
    if (__hip_atomic_compare_exchange_strong(parent + b, &expected, a, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return true;
    b = expected;  // b gained a parent meanwhile; retry from there
  }
}

__device__ __forceinline__ void atomic_min_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_max_u64(uint64_t* p, uint64_t v) {
  __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// arr[key] += val for every active lane, with one atomic per distinct key
// in the wave (lanes of a wave usually share the graph id).  Must be called
// by all lanes of the wave.
__device__ __forceinline__ void wave_add_by_key(int32_t* arr, int32_t key, int32_t val, bool active) {
  uint64_t todo = ballot(active);
  while (todo) {
    const int32_t k0 = __shfl(key, __builtin_ctzll(todo), 64);
    const bool mine = active && key == k0;
    const uint64_t grp = ballot(mine);
    todo &= ~grp;
    int32_t sum = mine ? val : 0;
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (lane_id() == __builtin_ctzll(grp)) atomicAdd(arr + k0, sum);
  }
}

// Grid-stride helpers
// The chip deals workgroups to its 8 XCDs round-robin (block b runs on XCD
// b % 8), and each XCD has its own L2.  xcd_major renumbers a grid (a
// multiple of 8 blocks) so that each XCD takes one contiguous run of the
// logical indices: neighbouring work items, which share cache lines at
// their edges, then meet in one L2.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int32_t xcd_major(int32_t b, int32_t grid) {
  return (b % NUM_XCD) * (grid / NUM_XCD) + b / NUM_XCD;
}

__device__ __forceinline__ int64_t gtid() {
  return (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
}
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

}  // namespace mc
