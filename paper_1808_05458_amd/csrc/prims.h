// Device-wide primitives: exclusive prefix sums and an LSD radix sort of
// 64-bit keys with a 32-bit payload.  Written for wave64 / 256-thread
// workgroups; every pass is a coalesced sweep over HBM.
#pragma once
#include "dev.h"

namespace mc {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ROWS = 16;                                  // rows of 256 per tile
constexpr int64_t SCAN_TILE = (int64_t)SCAN_THREADS * SCAN_ROWS;  // 4096 elements

// Block-wide inclusive scan of one value per thread (256 threads).
template <typename T>
__device__ __forceinline__ T block_inclusive_scan(T v, T* lds_wave_tot, T& block_total) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const T x = wave_incl_sum<T>(v);
  if (lane == 63) lds_wave_tot[wave] = x;
  __syncthreads();
  T base = 0, tot = 0;
  for (int i = 0; i < SCAN_THREADS / 64; ++i) {
    T t = lds_wave_tot[i];
    if (i < wave) base += t;
    tot += t;
  }
  __syncthreads();
  block_total = tot;
  return x + base;
}

// Input adaptors for scans: plain array, or a 0/1 predicate computed on the fly.
template <typename T>
struct ArrayIn {
  const T* p;
  __device__ __forceinline__ T operator()(int64_t i) const { return p[i]; }
};

template <typename Tout, typename In>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(In in, int64_t n, Tout* partial) {
  __shared__ Tout wt[SCAN_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  // every row's element read before any is added (an element past the end
  // reads the last one and counts zero), so the loads overlap instead of
  // waiting one by one
  Tout v[SCAN_ROWS];
#pragma unroll
  for (int r = 0; r < SCAN_ROWS; ++r) {
    const int64_t i = base + (int64_t)r * SCAN_THREADS + threadIdx.x;
    v[r] = (Tout)in(i < n ? i : n - 1);
  }
  Tout s = 0;
#pragma unroll
  for (int r = 0; r < SCAN_ROWS; ++r) {
    const int64_t i = base + (int64_t)r * SCAN_THREADS + threadIdx.x;
    s += i < n ? v[r] : (Tout)0;
  }
  Tout tot;
  block_inclusive_scan<Tout>(s, wt, tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// out[i] = offset + sum of in[0..i), carry-in per tile from partial[] (already
// exclusive-scanned).  If total != nullptr the grand total is written there.
template <typename Tout, typename In>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(In in, int64_t n, const Tout* partial,
                                                           Tout* out, Tout* total) {
  __shared__ Tout wt[SCAN_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  Tout carry = partial ? partial[blockIdx.x] : (Tout)0;
  Tout vs[SCAN_ROWS];  // all rows read first (see k_scan_reduce)
#pragma unroll
  for (int r = 0; r < SCAN_ROWS; ++r) {
    const int64_t i = base + (int64_t)r * SCAN_THREADS + threadIdx.x;
    vs[r] = (Tout)in(i < n ? i : n - 1);
  }
#pragma unroll
  for (int r = 0; r < SCAN_ROWS; ++r) {
    int64_t i = base + (int64_t)r * SCAN_THREADS + threadIdx.x;
    Tout v = (i < n) ? vs[r] : (Tout)0;
    Tout rowtot;
    Tout inc = block_inclusive_scan<Tout>(v, wt, rowtot);
    if (i < n) out[i] = carry + inc - v;
    if (total && i == n - 1) *total = carry + inc;
    carry += rowtot;
  }
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

inline int grid_for(int64_t n, int threads = 256, int cap = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

template <typename T>
inline void fill(T* p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
}

// Scratch needed by exclusive_scan for n elements (bytes).
template <typename Tout>
inline size_t scan_tmp_bytes(int64_t n) {
  size_t b = 0;
  while (n > SCAN_TILE) {
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    b += (size_t)nb * sizeof(Tout) + 256;
    n = nb;
  }
  return b + 256;
}

// Exclusive prefix sum out[i] = sum in[0..i); *total (device) = sum of all.
template <typename Tout, typename In>
void exclusive_scan(In in, int64_t n, Tout* out, Tout* total, void* tmp, hipStream_t s) {
  if (n <= 0) {
    if (total) fill<Tout>(total, (Tout)0, 1, s);
    return;
  }
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 1) {
    hipLaunchKernelGGL((k_scan_down<Tout, In>), dim3(1), dim3(SCAN_THREADS), 0, s, in, n,
                       (const Tout*)nullptr, out, total);
    return;
  }
  Tout* partial = (Tout*)tmp;
  char* rest = (char*)tmp + (((size_t)nb * sizeof(Tout) + 255) & ~(size_t)255);
  hipLaunchKernelGGL((k_scan_reduce<Tout, In>), dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, partial);
  exclusive_scan<Tout, ArrayIn<Tout>>(ArrayIn<Tout>{partial}, nb, partial, (Tout*)nullptr, rest, s);
  hipLaunchKernelGGL((k_scan_down<Tout, In>), dim3(nb), dim3(SCAN_THREADS), 0, s, in, n,
                     (const Tout*)partial, out, total);
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits.  Per pass: tile histograms (digit-major),
// one exclusive scan over them, then a stable scatter whose in-tile ranks come
// from wave ballots (8 ballots give each lane the set of lanes holding the
// same digit).  A workgroup sorts a tile of RS_THREADS * ITEMS keys; the
// tile size is a launch-shape choice (8, 16 or 32 keys per thread).
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS_DEFAULT = 16;                  // 4096 keys per workgroup
constexpr int RS_ITEMS_MIN = 8;                       // sizes the histogram buffers
constexpr int RS_WAVES = RS_THREADS / 64;

template <int ITEMS>
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint64_t* __restrict__ keys, int64_t n,
                                                        int shift, uint32_t* __restrict__ hist,
                                                        int64_t ntiles) {
  constexpr int TILE = RS_THREADS * ITEMS;
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * TILE;
  // every key of the thread loaded before the first is counted (no load in
  // a branch: a slot past the end reads the tile's first key)
  uint64_t k[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t i = base + (int64_t)r * RS_THREADS + threadIdx.x;
    k[r] = keys[i < n ? i : base];
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t i = base + (int64_t)r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(k[r] >> shift) & 255], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__device__ __forceinline__ uint64_t match_digit(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    uint64_t bb = ballot((d >> b) & 1);
    m &= ((d >> b) & 1) ? bb : ~bb;
  }
  return m;
}

template <int ITEMS>
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(
    const uint64_t* __restrict__ keys, const int32_t* __restrict__ vals, int64_t n, int shift,
    const uint32_t* __restrict__ offs, int64_t ntiles, uint64_t* __restrict__ okeys,
    int32_t* __restrict__ ovals) {
  constexpr int TILE = RS_THREADS * ITEMS;
  constexpr int WAVE_ITEMS = TILE / RS_WAVES;  // consecutive keys per wave
  __shared__ uint32_t cnt[RS_WAVES][256];
  __shared__ uint32_t tile_off[256];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_THREADS) (&cnt[0][0])[i] = 0;
  tile_off[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  __syncthreads();
  const int64_t wbase = (int64_t)blockIdx.x * TILE + (int64_t)wave * WAVE_ITEMS;
  uint64_t k[ITEMS];
  int32_t v[ITEMS];
  uint32_t pos[ITEMS];
  // all of the thread's keys and values in flight together (no load in a
  // branch: a slot past the end reads the tile's first entry)
  const int64_t first = (int64_t)blockIdx.x * TILE;
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int64_t i = wbase + r * 64 + lane;
    k[r] = keys[i < n ? i : first];
    v[r] = vals[i < n ? i : first];
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    int64_t i = wbase + r * 64 + lane;
    bool ok = i < n;
    uint32_t d = ok ? (uint32_t)((k[r] >> shift) & 255) : 0u;
    uint64_t valid = ballot(ok);
    uint64_t peers = match_digit(d) & valid;  // every lane takes part in the ballots
    uint32_t before = ok ? cnt[wave][d] : 0;
    int rank = popc64(peers & lanemask_lt());
    __builtin_amdgcn_wave_barrier();
    if (ok && rank == 0) cnt[wave][d] = before + (uint32_t)popc64(peers);
    __builtin_amdgcn_wave_barrier();
    pos[r] = ok ? before + rank : 0xFFFFFFFFu;
  }
  __syncthreads();
  // exclusive prefix over waves per digit, plus the tile's global offset
  {
    const int d = threadIdx.x;
    uint32_t run = tile_off[d];
    for (int w = 0; w < RS_WAVES; ++w) {
      uint32_t c = cnt[w][d];
      cnt[w][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    if (pos[r] == 0xFFFFFFFFu) continue;
    uint32_t d = (uint32_t)((k[r] >> shift) & 255);
    uint32_t o = cnt[wave][d] + pos[r];
    okeys[o] = k[r];
    ovals[o] = v[r];
  }
}

inline size_t radix_tmp_bytes(int64_t n) {
  const int64_t tile = RS_THREADS * RS_ITEMS_MIN;  // the most tiles of any shape
  int64_t ntiles = (n + tile - 1) / tile;
  size_t h = (size_t)ntiles * 256 * sizeof(uint32_t);
  return 2 * ((h + 255) & ~(size_t)255) + scan_tmp_bytes<uint32_t>(ntiles * 256) + 1024;
}

// Sorts (keys, vals) by the low `bits` bits of the key.  Ping-pongs between
// the two buffer pairs; returns 0 if the result is in (keys, vals), 1 if in
// (keys_alt, vals_alt).  Positions fit in 32 bits (n < 2^32).  `hook(kind,
// pass)` is called before (kind 0/2) and after (kind 1/3) the histogram and
// scatter launches of each pass (timing).
struct NoHook {
  void operator()(int, int) const {}
};

template <int ITEMS, typename Hook>
inline int radix_sort_pairs_t(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt,
                              int64_t n, int bits, void* tmp, hipStream_t s, Hook hook) {
  if (n <= 1 || bits <= 0) return 0;
  constexpr int TILE = RS_THREADS * ITEMS;
  int64_t ntiles = (n + TILE - 1) / TILE;
  size_t hb = ((size_t)ntiles * 256 * sizeof(uint32_t) + 255) & ~(size_t)255;
  uint32_t* hist = (uint32_t*)tmp;
  uint32_t* offs = (uint32_t*)((char*)tmp + hb);
  void* stmp = (char*)tmp + 2 * hb;
  int which = 0;
  for (int shift = 0, pass = 0; shift < bits; shift += 8, ++pass) {
    const uint64_t* ki = which ? keys_alt : keys;
    const int32_t* vi = which ? vals_alt : vals;
    uint64_t* ko = which ? keys : keys_alt;
    int32_t* vo = which ? vals : vals_alt;
    hook(0, pass);
    hipLaunchKernelGGL(k_rs_hist<ITEMS>, dim3(ntiles), dim3(RS_THREADS), 0, s, ki, n, shift, hist, ntiles);
    hook(1, pass);
    exclusive_scan<uint32_t, ArrayIn<uint32_t>>(ArrayIn<uint32_t>{hist}, ntiles * 256, offs,
                                                (uint32_t*)nullptr, stmp, s);
    hook(2, pass);
    hipLaunchKernelGGL(k_rs_scatter<ITEMS>, dim3(ntiles), dim3(RS_THREADS), 0, s, ki, vi, n, shift, offs,
                       ntiles, ko, vo);
    hook(3, pass);
    which ^= 1;
  }
  return which;
}

// tile: keys per workgroup (2048, 4096 or 8192; anything else = 4096).
template <typename Hook = NoHook>
inline int radix_sort_pairs(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt,
                            int64_t n, int bits, void* tmp, hipStream_t s, Hook hook = Hook(),
                            int tile = RS_THREADS * RS_ITEMS_DEFAULT) {
  if (tile == RS_THREADS * 8)
    return radix_sort_pairs_t<8>(keys, vals, keys_alt, vals_alt, n, bits, tmp, s, hook);
  if (tile == RS_THREADS * 32)
    return radix_sort_pairs_t<32>(keys, vals, keys_alt, vals_alt, n, bits, tmp, s, hook);
  return radix_sort_pairs_t<16>(keys, vals, keys_alt, vals_alt, n, bits, tmp, s, hook);
}

}  // namespace mc
