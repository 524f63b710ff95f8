// Entry rows of a CSR without a per-entry source array: the row of every
// WCH-th entry in a table, and a wave-local mapping of a chunk's entries to
// their rows.  Shared by the streaming kernels and the sweeps' pull form
// (there the "rows" are the still-free vertices, over the prefix sums of
// their row lengths).
#pragma once
#include "dev.h"

namespace mc {

// Entry rows without a source array.  A wave takes WCH consecutive entries
// [e0, e0 + WCH), entry e0 + k * 64 + lane in slot k of each lane (every load
// of a slot is one contiguous 256-byte run).  first[c] holds the row of entry
// c * WCH (k_chunk_rows).  The rows starting inside the chunk are marked in
// the wave's own LDS (pos: WCH ints; the largest id where empty rows share a
// start) from one coalesced read of row_ptr per 64 rows, and a maximum scan
// over the positions carries each row id to its entries.  Wave-local: no
// workgroup barrier.
constexpr int WCH = 512;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// The start of row r0 + 1 + lane (row_ptr[n] = nnz past the last row): the
// first 64 row starts a chunk reads, which a caller may load a chunk ahead.
__device__ __forceinline__ int64_t chunk_start0(const int64_t* __restrict__ rp, int32_t n, int32_t r0) {
  const int64_t r = (int64_t)r0 + 1 + lane_id();
  return rp[r < n ? r : n];
}

// chunk_rows with st0 = chunk_start0(rp, n, r0) already loaded.
__device__ __forceinline__ void chunk_rows_from(const int64_t* __restrict__ rp, int32_t n, int64_t e0, int32_t r0,
                                                int64_t st0, int32_t* pos, int32_t (&row)[8]) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 0; k < 8; ++k) pos[lane * 8 + k] = -1;
  wave_lds_sync();
  if (lane == 0) pos[0] = r0;
  const int64_t end = e0 + WCH;
  int64_t st = st0;
  for (int64_t base = (int64_t)r0 + 1;; base += 64) {
    const int64_t r = base + lane;
    const bool in = r <= n && st < end;  // starts are > e0: row r0 holds e0
    if (in) atomicMax(&pos[st - e0], (int32_t)r);
    if (!((ballot(in) >> 63) & 1)) break;  // starts ascend: lane 63 in means more may follow
    const int64_t r2 = r + 64;
    st = rp[r2 < n ? r2 : n];
  }
  wave_lds_sync();
  int32_t v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = pos[lane * 8 + k];
#pragma unroll
  for (int k = 1; k < 8; ++k) v[k] = v[k] > v[k - 1] ? v[k] : v[k - 1];
  // the largest row started at or before each lane's positions (DPP scan)
  const int32_t inc = wave_incl_max_i32(v[7]);
  const int32_t ex = wave_shr1_i32(inc, -1);
#pragma unroll
  for (int k = 0; k < 8; ++k) pos[lane * 8 + k] = v[k] > ex ? v[k] : ex;
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < 8; ++k) row[k] = pos[k * 64 + lane];
  wave_lds_sync();  // pos is reused by the wave's next chunk
}

__device__ __forceinline__ void chunk_rows(const int64_t* __restrict__ rp, int32_t n, int64_t e0, int32_t r0,
                                           int32_t* pos, int32_t (&row)[8]) {
  chunk_rows_from(rp, n, e0, r0, chunk_start0(rp, n, r0), pos, row);
}

// first[c] = the row holding entry c * WCH (one writer per chunk: the
// non-empty row whose entry range contains it).
__global__ void k_chunk_rows(int32_t n, const int64_t* __restrict__ rp, int32_t* __restrict__ first) {
  for (int64_t r = gtid(); r < n; r += gstride()) {
    const int64_t lo = rp[r], hi = rp[r + 1];
    for (int64_t c = (lo + WCH - 1) / WCH; c * WCH < hi; ++c) first[c] = (int32_t)r;
  }
}

// The row of entry c * WCH from first[], clamped into [0, n).
__device__ __forceinline__ int32_t chunk_first(const int32_t* first, int64_t c, int32_t n) {
  const int32_t r0 = first[c];
  return r0 < 0 ? 0 : (r0 >= n ? n - 1 : r0);
}

// Global wave index and count of a launch.
__device__ __forceinline__ int64_t gwave() { return ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; }
__device__ __forceinline__ int64_t gwaves() { return ((int64_t)gridDim.x * blockDim.x) >> 6; }

}  // namespace mc
