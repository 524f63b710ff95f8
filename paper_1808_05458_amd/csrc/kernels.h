// Per-round kernels of the bound-driven contraction loop (Algorithm 2):
// ingest and trivial bound, Padberg-Rinaldi tests, union-find passes,
// block numbering, contraction by sort + merge, bound updates and side
// materialisation.  Many graphs may be packed into one CSR; every graph
// keeps a contiguous vertex range and its own bound lambda-hat.
#pragma once
#include "capforest.h"
#include "prims.h"
#include "smallsweep.h"
#include "sweep.h"
#include "tail.h"
#include "lp.h"

namespace mc {

enum : int32_t { REC_NONE = 0, REC_ALPHA = 1, REC_DEG = 2, REC_DISCONNECTED = 3 };

struct GraphState {  // per-graph device arrays
  const int64_t* voff;  // original vertex offsets [G+1]
  int64_t* lhat;        // best bound found so far (a real cut)
  int32_t* n;           // current vertex count
  int32_t* cvoff;       // current first vertex
  int32_t* nnew;        // vertex count after this round's compaction
  int32_t* active;
  uint64_t* bdeg;       // (weighted degree << 32) | vertex, min over the graph
  uint64_t* balpha;     // (alpha << 32) | scan id
  int32_t* ucount;      // contractible pairs found this round
  int32_t* rec_type;    // improvement this step
  int32_t* rec_id;
  int32_t* rec_k;
  int32_t* fb_k;
  uint8_t* mode;
  int32_t* whole;       // list of whole-scan graphs
  int32_t* fb_list;
  int64_t* wsum;
  int32_t* root0;       // component root of the graph's first vertex
};

// Segmented sum of `val` over runs of equal `key` within the wave (lanes in
// order), by DPP scans: run heads by a one-lane shift, each lane's run start
// by a maximum scan, its segmented prefix as the difference of two prefix
// sums (one lane read for the prefix before the run).  Returns the run's
// sum up to this lane (the run total in its last lane); tail = last lane.
// Every lane of the wave must call it (no lane-dependent branch around it).
template <typename K, typename V>
__device__ __forceinline__ V wave_segsum(K key, V val, bool valid, bool& tail) {
  const int lane = lane_id();
  const K prev = wave_shr1<K>(key, key), next = wave_shl1<K>(key, key);
  const bool head = lane == 0 || prev != key;
  const int32_t start = wave_incl_max_i32(head ? lane : -1);  // lane 0 heads a run
  const V p = wave_incl_sum<V>(valid ? val : (V)0);
  const V before = __shfl(p, start > 0 ? start - 1 : 0, 64);
  tail = lane == 63 || next != key;
  return start > 0 ? (V)(p - before) : p;
}

// ------------------------------------------------------------------ ingest
__global__ void k_check_rowptr(int32_t n, int64_t nnz, const int64_t* rp, Ctl* ctl) {
  for (int64_t v = gtid(); v < n; v += gstride()) {
    if (rp[v] > rp[v + 1]) atomicExch(&ctl->err, -1);
  }
  if (gtid() == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicExch(&ctl->err, -1);
}

// gid per vertex from the graph offsets; original-vertex map starts as id.
__global__ void k_init_vertices(int32_t n, const int64_t* voff, int32_t G, int32_t* gid,
                                int32_t* ogid, int32_t* map) {
  for (int64_t v = gtid(); v < n; v += gstride()) {
    int32_t lo = 0, hi = G;  // find g with voff[g] <= v < voff[g+1]
    while (hi - lo > 1) {
      int32_t mid = (lo + hi) >> 1;
      if (voff[mid] <= v) lo = mid; else hi = mid;
    }
    gid[v] = lo;
    ogid[v] = lo;
    map[v] = (int32_t)v;
  }
}


// The entry sources as an array (src[e] = the row of entry e), for the
// consumers that index entries one at a time.
__global__ void __launch_bounds__(256) k_fill_src(int32_t n, int64_t nnz, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ first, int32_t* __restrict__ src) {
  __shared__ int32_t pos_all[4][WCH];
  int32_t* pos = pos_all[threadIdx.x >> 6];
  const int lane = lane_id();
  for (int64_t ch = gwave(); ch * WCH < nnz; ch += gwaves()) {
    const int64_t e0 = ch * WCH;
    int32_t row[8];
    chunk_rows(rp, n, e0, chunk_first(first, ch, n), pos, row);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t e = e0 + k * 64 + lane;
      if (e < nnz) src[e] = row[k];
    }
  }
}

// Sum of val over each run of equal row among the wave's 64 lanes (rows
// ascend with the lane), added to out[row] once per run.  A slot held by one
// row throughout is one wave sum (long rows); otherwise a segmented sum.
// All 64 lanes must be active.
__device__ __forceinline__ void wave_row_add(int32_t row, int64_t val, bool ok, int64_t* out) {
  const int32_t r_first = __builtin_amdgcn_readfirstlane(row);
  if (ballot(ok && row != r_first) == 0) {
    const int64_t sum = wave_sum_i64_dpp(ok ? val : 0);
    if (lane_id() == 0 && sum) atomicAdd((unsigned long long*)(out + r_first), (unsigned long long)sum);
    return;
  }
  bool tail;
  const int64_t sum = wave_segsum<int32_t, int64_t>(ok ? row : -1, val, ok, tail);
  if (ok && tail && sum) atomicAdd((unsigned long long*)(out + row), (unsigned long long)sum);
}

// Validation and weighted degrees (self-loops excluded; they never cross a
// cut), one WCH-entry chunk per wave step, rows from chunk_rows.  Software
// pipelined: once a chunk is checked and its weights are in LDS, the next
// chunk's entries, the starts of its first rows and its first row's graph
// go out, and the first row of the chunk after that (each a dependent load
// of the one before), so they are in flight during the chunk's sums.
// G = 1: one graph, whose range is [0, n) (no graph lookups).  chmax[c]: the
// largest weight of chunk c (the tests skip chunks by it).
__global__ void __launch_bounds__(256, 5) k_ingest(int32_t n, int64_t nnz, const int64_t* __restrict__ rp,
                                                const int32_t* __restrict__ col,
                                                const int32_t* __restrict__ w,
                                                const int32_t* __restrict__ gid,
                                                const int64_t* __restrict__ voff,
                                                const int32_t* __restrict__ first, int32_t G, int64_t* cdeg,
                                                int32_t* gmaxw, int32_t* chmax, Ctl* ctl) {
  __shared__ int32_t pos_all[4][WCH];
  __shared__ int32_t val_all[4][WCH];
  int32_t* pos = pos_all[threadIdx.x >> 6];
  int32_t* vals = val_all[threadIdx.x >> 6];
  const int lane = lane_id();
  // largest weight of the chunks in one graph, per lane, folded into gmaxw
  // when the graph changes (same-address atomics serialise)
  int32_t run_g = -1, run_m = 0;
  int64_t ch = gwave();
  const int64_t nch = (nnz + WCH - 1) / WCH;
  int32_t y[8], c[8];
  int32_t f = 0, fn = 0, gq = 0;  // first row of the loaded chunk and of the next; the loaded chunk's graph
  int64_t s0 = 0;                 // the loaded chunk's first row starts (chunk_start0)
  // a chunk's entries through a wave-uniform base and 32-bit offsets (one
  // address add per chunk, not one 64-bit add per entry)
  auto load = [&](int64_t at) {
    const int64_t e0 = at * WCH;
    const int32_t len = (int32_t)min((int64_t)WCH, nnz - e0);
    const int32_t* cb = col + e0;
    const int32_t* wb = w + e0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int32_t o = k * 64 + lane;
      const int32_t oc = o < len ? o : 0;
      // each entry is read once here: streamed past the caches
      y[k] = __builtin_nontemporal_load(cb + oc);
      c[k] = __builtin_nontemporal_load(wb + oc);
    }
    f = fn;  // first[at], loaded a step earlier
    s0 = chunk_start0(rp, n, f);
    gq = G > 1 ? gid[f] : 0;
    const int64_t nx = at + gwaves();
    fn = nx < nch ? chunk_first(first, nx, n) : 0;
  };
  if (ch < nch) {
    fn = chunk_first(first, ch, n);
    load(ch);
  }
  for (; ch < nch; ch += gwaves()) {
    const int64_t e0 = ch * WCH;
    const int32_t r0 = f;
    // the chunk's graph: the first row's, when its last row is in it too
    // (graphs are contiguous vertex ranges)
    const int32_t g0 = gq;
    const int32_t lo0 = G > 1 ? (int32_t)voff[g0] : 0;  // vertex ids fit 31 bits
    const int32_t hi0 = G > 1 ? (int32_t)voff[g0 + 1] : n;
    const int32_t len = (int32_t)min((int64_t)WCH, nnz - e0);
    {
      // Prefix form, taken when fewer than 64 rows start inside the chunk
      // (lane i holds the start of row r0 + 1 + i), the chunk lies in one
      // graph, no neighbour is one of the chunk's rows (so no self-loop)
      // and the chunk's sums fit 31 bits: a row's share of the chunk is the
      // difference of the chunk's prefix sums at its ends, and no entry
      // needs its row.
      const int64_t st = s0;
      const bool starts = r0 + 1 + lane < n && st < e0 + len;
      const uint64_t sm = ballot(starts);
      const int32_t r_end = r0 + popc64(sm);  // the chunk's last row when lane 63 does not start one
      bool near = false;
      int32_t cmx = 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool ok = k * 64 + lane < len;
        const int32_t ck = ok ? c[k] : 0;
        cmx = ck > cmx ? ck : cmx;
        near = near || (ok && y[k] >= r0 && y[k] <= r_end);
      }
      const uint32_t cm = wave_max_u32((uint32_t)cmx);
      if (!(sm >> 63) && r_end < hi0 && ballot(near) == 0 && cm < (1u << 22)) {
        if (g0 != run_g) {
          const uint32_t m = wave_max_u32((uint32_t)run_m);
          if (lane == 0 && m && run_g >= 0) atomicMax(gmaxw + run_g, (int32_t)m);
          run_g = g0;
          run_m = 0;
        }
        run_m = cmx > run_m ? cmx : run_m;
        bool bad = false;
        int32_t base = 0;  // the chunk's sum before slot k
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const bool ok = k * 64 + lane < len;
          bad = bad || (ok && ((uint32_t)(y[k] - lo0) >= (uint32_t)(hi0 - lo0) || c[k] < 1));
          const int32_t v = ok ? c[k] : 0;
          const int32_t inc = wave_incl_sum<int32_t>(v);
          vals[k * 64 + lane] = base + inc - v;  // the chunk's entries before this one
          base += __builtin_amdgcn_readlane(inc, 63);
        }
        if (bad) atomicExch(&ctl->err, -1);
        if (lane == 0) chmax[ch] = (int32_t)cm;
        if (ch + gwaves() < nch) load(ch + gwaves());
        wave_lds_sync();
        const int32_t at = starts ? vals[(int32_t)min(max(st - e0, (int64_t)0), (int64_t)WCH - 1)] : base;
        wave_lds_sync();  // vals is rewritten by the next chunk
        // lane i: row r0 + i, from the previous lane's start (or the chunk's
        // first entry) to its own (or the chunk's end)
        const int32_t share = at - wave_shr1<int32_t>(at, 0);
        if (lane <= r_end - r0 && share)
          atomicAdd((unsigned long long*)(cdeg + r0 + lane), (unsigned long long)(int64_t)share);
        continue;
      }
    }
    int32_t row[8];
    chunk_rows_from(rp, n, e0, r0, s0, pos, row);
    const int32_t last_e = len - 1;  // slot and lane of the chunk's last entry
    int32_t row_last = r0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if ((last_e >> 6) == k) row_last = __builtin_amdgcn_readlane(row[k], (int)(last_e & 63));
    const bool one = row_last < hi0;
    if (one && g0 != run_g) {
      const uint32_t m = wave_max_u32((uint32_t)run_m);
      if (lane == 0 && m && run_g >= 0) atomicMax(gmaxw + run_g, (int32_t)m);
      run_g = g0;
      run_m = 0;
    }
    bool bad = false;
    int32_t cmx = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool ok = k * 64 + lane < len;
      // a chunk across a graph boundary (wave-uniform) reads each entry's
      // graph range; graphs are contiguous vertex ranges
      int32_t gk = g0;
      int32_t lo = lo0, hi = hi0;
      if (!one) {
        gk = gid[ok ? row[k] : r0];
        lo = (int32_t)voff[gk];
        hi = (int32_t)voff[gk + 1];
      }
      bad = bad || (ok && ((uint32_t)(y[k] - lo) >= (uint32_t)(hi - lo) || c[k] < 1));
      vals[k * 64 + lane] = (ok && y[k] != row[k]) ? c[k] : 0;
      const int32_t ck = ok ? c[k] : 0;
      cmx = ck > cmx ? ck : cmx;
      if (one) {
        run_m = ck > run_m ? ck : run_m;
      } else {
        const int32_t gu = __builtin_amdgcn_readfirstlane(gk);
        if (ballot(gk == gu) == ~0ull) {
          const uint32_t m = wave_max_u32((uint32_t)ck);
          if (lane == 0 && m) atomicMax(gmaxw + gu, (int32_t)m);
        } else if (ok) {
          atomicMax(gmaxw + gk, ck);
        }
      }
    }
    if (bad) atomicExch(&ctl->err, -1);
    {
      const uint32_t cm = wave_max_u32((uint32_t)cmx);
      if (lane == 0) chmax[ch] = (int32_t)cm;
    }
    // the chunk's weights are in LDS: the next chunk's loads go out and are
    // in flight during the sums below and the next chunk's row mapping
    if (ch + gwaves() < nch) load(ch + gwaves());
    // weighted degrees: each lane sums its 8 consecutive entries by row
    // (positions lane * 8 ..; rows ascend with the position): a row wholly
    // inside the lane is added at once; its first and last rows continue in
    // the neighbouring lanes, so the last is folded into the next lane's
    // first, and the first rows are summed across the wave
    wave_lds_sync();
    int32_t rq[8], vq[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      rq[k] = pos[lane * 8 + k];
      vq[k] = vals[lane * 8 + k];
    }
    wave_lds_sync();  // vals is rewritten by the next chunk
    int32_t hr = rq[0], cur = rq[0], tr = rq[0];
    int64_t hs = 0, ts = 0, acc = 0;
    bool in_head = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (rq[k] != cur) {
        if (in_head) hs = acc;
        else if (acc) atomicAdd((unsigned long long*)(cdeg + cur), (unsigned long long)acc);
        in_head = false;
        cur = rq[k];
        acc = 0;
      }
      acc += vq[k];
    }
    if (in_head) hs = acc;
    else { tr = cur; ts = acc; }
    const bool has_tail = !in_head;
    const int32_t next_head = wave_shl1_i32(hr, hr);
    const bool tail_on = has_tail && lane < 63 && next_head == tr;
    if (has_tail && !tail_on && ts) atomicAdd((unsigned long long*)(cdeg + tr), (unsigned long long)ts);
    hs += wave_shr1_i64(tail_on ? ts : (int64_t)0, 0);
    wave_row_add(hr, hs, true, cdeg);
  }
  const uint32_t m = wave_max_u32((uint32_t)run_m);
  if (lane == 0 && m && run_g >= 0) atomicMax(gmaxw + run_g, (int32_t)m);
}

// Per-graph minimum weighted degree (the trivial cut, section "Basic
// Concepts") and weight totals.
// Each thread takes a contiguous range of vertices (graphs are contiguous
// ranges too, so a thread meets few graph changes), keeps a running minimum
// and sum for the graph it is in and flushes when the graph changes; the
// last flush is combined per wave when the wave ends in one graph.
__device__ __forceinline__ void thread_range(int64_t n, int64_t& a, int64_t& b) {
  const int64_t t = gstride(), per = (n + t - 1) / t;
  a = min(n, gtid() * per);
  b = min(n, a + per);
}

__global__ void k_min_degree(int32_t n, const int64_t* cdeg, const int32_t* gid,
                             const int32_t* active, uint64_t* bdeg, int64_t* wsum) {
  int32_t cur = -1;
  uint64_t best = ~0ull;
  int64_t sum = 0;
  int64_t va, vb;
  thread_range(n, va, vb);
  for (int64_t v = va; v < vb; ++v) {
    const int32_t g = gid[v];
    if (active && !active[g]) continue;
    if (g != cur) {
      if (cur >= 0) {
        atomic_min_u64(bdeg + cur, best);
        if (wsum) atomicAdd((unsigned long long*)(wsum + cur), (unsigned long long)sum);
      }
      cur = g;
      best = ~0ull;
      sum = 0;
    }
    const uint64_t key = ((uint64_t)cdeg[v] << 32) | (uint32_t)v;
    best = key < best ? key : best;
    sum += cdeg[v];
  }
  const int32_t g0 = bcast(cur, 0);
  const bool uniform = ballot(cur == g0) == ~0ull;
  if (uniform && g0 >= 0) {
    const uint64_t m = wave_min_u64(best);
    const int64_t s = wave_sum_i64(sum);
    if (lane_id() == 0) {
      atomic_min_u64(bdeg + g0, m);
      if (wsum) atomicAdd((unsigned long long*)(wsum + g0), (unsigned long long)s);
    }
  } else if (cur >= 0) {
    atomic_min_u64(bdeg + cur, best);
    if (wsum) atomicAdd((unsigned long long*)(wsum + cur), (unsigned long long)sum);
  }
}

// ------------------------------------------------------------ union-find
__global__ void k_iota(int32_t* p, int32_t n) {
  for (int64_t v = gtid(); v < n; v += gstride()) p[v] = (int32_t)v;
}

__global__ void k_union_all_edges(int64_t nnz, const int32_t* src, const int32_t* col, int32_t* parent) {
  for (int64_t e = gtid(); e < nnz; e += gstride()) {
    int32_t u = src[e], v = col[e];
    if (u < v) uf_union(parent, u, v);
  }
}

// Point every vertex at its root.  The walk up is read-only: a halving store
// from one thread could land after another thread's root store on the same
// entry and leave it at a non-root ancestor.  Each thread writes only its
// own entry, and only with the root, so concurrent walks see either the old
// parent (an ancestor) or the root, and every entry ends at its root.
__global__ void k_flatten(int32_t n, int32_t* parent) {
  for (int64_t v = gtid(); v < n; v += gstride()) {
    int32_t x = (int32_t)v, p = ld_relaxed(parent + x);
    while (p != x) {
      x = p;
      p = ld_relaxed(parent + x);
    }
    st_relaxed(parent + v, x);
  }
}

__global__ void k_union_pairs(const uint64_t* pairs, const Ctl* ctl, int64_t cap, int32_t* parent) {
  int64_t np = ctl->pairs < cap ? ctl->pairs : cap;
  for (int64_t i = gtid(); i < np; i += gstride()) {
    uint64_t p = pairs[i];
    uf_union(parent, (int32_t)(p >> 32), (int32_t)(uint32_t)p);
  }
}

// Components per graph: disconnected graphs get lambda = 0 (section "Parallel
// CAPFOREST": a disconnected graph leaves vertices unvisited).
__global__ void k_count_roots(int32_t n, const int32_t* parent, const int32_t* gid, int32_t* cnt) {
  int32_t cur = -1, acc = 0;
  int64_t va, vb;
  thread_range(n, va, vb);
  for (int64_t v = va; v < vb; ++v) {
    if (parent[v] != v) continue;
    const int32_t g = gid[v];
    if (g != cur) {
      if (acc) atomicAdd(cnt + cur, acc);
      cur = g;
      acc = 0;
    }
    ++acc;
  }
  wave_add_by_key(cnt, cur, acc, acc > 0);
}

// ----------------------------------------------------- per-graph bookkeeping
// prok[g] (and the count ctl->n_pr) marks the graphs where a Padberg-Rinaldi
// test can pass in the first round: PR1 needs an edge of weight >=
// lambda-hat, PR2 one of weight above half the minimum degree (the largest
// weight bounds both).
__global__ void k_graph_init(int32_t G, GraphState S, int32_t* root0, const int32_t* parent,
                             const int32_t* gmaxw, int32_t* prok, Ctl* ctl) {
  for (int64_t g = gtid(); g < G; g += gstride()) {
    int32_t ng = (int32_t)(S.voff[g + 1] - S.voff[g]);
    S.n[g] = ng;
    S.cvoff[g] = (int32_t)S.voff[g];
    uint64_t bd = S.bdeg[g];
    int64_t lam = (int64_t)(bd >> 32);
    S.lhat[g] = lam;
    S.rec_type[g] = REC_DEG;
    S.rec_id[g] = (int32_t)(uint32_t)bd;
    S.rec_k[g] = 0;
    if (S.wsum[g] > 2ll * 2147483647ll) atomicExch(&ctl->err, -3);
    if (S.nnew[g] > 1) {  // more than one component
      S.lhat[g] = 0;
      S.rec_type[g] = REC_DISCONNECTED;
      root0[g] = parent[S.voff[g]];
      S.active[g] = 0;
    } else {
      S.active[g] = ng > 2 ? 1 : 0;
    }
    prok[g] = 0;
    if (S.active[g]) {
      atomicAdd(&ctl->n_active, 1);
      const int64_t mw = gmaxw[g];
      if (mw >= S.lhat[g] || 2 * mw > lam) {
        prok[g] = 1;
        atomicAdd(&ctl->n_pr, 1);
      }
    }
  }
}

// side[v] for graphs whose bound improved at this step.
struct SideArgs {
  int32_t n0;
  const int32_t* ogid;
  const int32_t* map;       // original -> current vertex (before this round's relabel for ALPHA)
  const int32_t* rec_type;
  const int32_t* rec_id;
  const int32_t* rec_k;
  const int32_t* claim;
  const int32_t* step;
  const uint64_t* fb_rs;    // sweeps: visit stamp in the high 32 bits
  const int32_t* parent;    // for REC_DISCONNECTED
  const int32_t* root0;
  uint8_t* side;
  int32_t want;             // record type this pass materialises
};

__global__ void k_side(SideArgs A) {
  for (int64_t v = gtid(); v < A.n0; v += gstride()) {
    int32_t g = A.ogid[v];
    int32_t t = A.rec_type[g];
    if (t != A.want) continue;
    int32_t c = A.map[v];
    uint8_t s = 0;
    if (t == REC_DEG) {
      s = c == A.rec_id[g];
    } else if (t == REC_ALPHA) {
      int32_t sid = A.rec_id[g], k = A.rec_k[g];
      if (sid == SWEEP_SID) {
        const int32_t st = (int32_t)(A.fb_rs[c] >> 32);
        s = st >= 1 && st <= k;
      } else if (sid == TAIL_SID) {
        // the sweep's visited set and the first pops of tail process f
        const uint64_t u = A.fb_rs[c];
        const int32_t st = (int32_t)(u >> 32);
        const int32_t f = (k >> 20) & 1023, kk = k & 0xFFFFF;
        s = st >= 1 || ((uint32_t)st == tail_pop(f) && (int32_t)(uint32_t)u <= kk);
      }
      else s = A.claim[c] == sid && A.step[c] <= k;
    } else if (t == REC_DISCONNECTED) {
      s = A.parent[v] != A.root0[g];
    }
    A.side[v] = s;
  }
}

// Round planning: graphs up to whole_small vertices are scanned whole with
// the small LDS map (mode 1), up to whole_max with the large map (mode 3),
// larger ones by region scans (mode 2).  Inactive graphs idle (mode 0).
// Matula's approximation: the round's contraction bound per graph,
// k = min(lambda-hat, max(1, ceil((1/2 - eps) delta))) with eps = ppm / 10^6
// and delta the graph's minimum degree (bdeg, before the round clears it).
__global__ void k_matula_cap(int32_t G, GraphState S, int64_t ppm, int64_t* kcap) {
  for (int64_t g = gtid(); g < G; g += gstride()) {
    const int64_t lam = S.lhat[g];
    const uint64_t bd = S.bdeg[g];
    int64_t k = lam;
    if (bd != ~0ull) {
      const int64_t delta = (int64_t)(bd >> 32);
      // contract q(e) >= (1/2 - eps) delta: for integer q, the ceiling
      const int64_t m = (delta * (1000000 - 2 * ppm) + 1999999) / 2000000;
      k = min(lam, max((int64_t)1, m));
    }
    kcap[g] = k;
  }
}

__global__ void k_round_reset(int32_t G, GraphState S) {
  for (int64_t g = gtid(); g < G; g += gstride()) {
    S.ucount[g] = 0;
    S.balpha[g] = ~0ull;
    S.bdeg[g] = ~0ull;
    S.rec_type[g] = REC_NONE;
    S.nnew[g] = 0;
  }
}

// Mode 4: the Padberg-Rinaldi unions alone leave at most two blocks, so the
// graph goes straight to contraction.  nnew holds the blocks after the tests.
// One workgroup: graph modes, and the two whole-graph lists ordered largest
// first (by size class, a quarter octave wide), so that the persistent
// sweep workgroups take the longest graphs first and finish together.
constexpr int PLAN_THREADS = 1024;
constexpr int PLAN_CLASSES = 128;

__device__ __forceinline__ int plan_class(int32_t n) {
  const int lz = 31 - __builtin_clz((uint32_t)max(n, 1));
  const int frac = lz >= 2 ? ((n >> (lz - 2)) & 3) : 0;
  return lz * 4 + frac;
}

__global__ void __launch_bounds__(PLAN_THREADS) k_plan_split(int32_t G, GraphState S, const int64_t* rp,
                                                             int32_t whole_small, int32_t whole_max,
                                                             int32_t* whole2, Ctl* ctl) {
  __shared__ int32_t off[2][PLAN_CLASSES];
  for (int i = threadIdx.x; i < 2 * PLAN_CLASSES; i += PLAN_THREADS) off[i / PLAN_CLASSES][i % PLAN_CLASSES] = 0;
  __syncthreads();
  int64_t nnz_acc = 0, nv_acc = 0;
  int32_t region = 0;
  for (int64_t g = threadIdx.x; g < G; g += PLAN_THREADS) {
    uint8_t m = 0;
    if (S.active[g]) {
      if (S.nnew[g] <= 2) m = 4;
      else if (S.n[g] <= whole_small) m = 1;
      else if (S.n[g] <= whole_max) m = 3;
      else m = 2;
    }
    S.mode[g] = m;
    if (m == 1 || m == 3) {
      atomicAdd(&off[m == 3][plan_class(S.n[g])], 1);
      const int32_t v0 = S.cvoff[g];
      nnz_acc += rp[v0 + S.n[g]] - rp[v0];
      nv_acc += S.n[g];
    }
    region += m == 2;
  }
  __syncthreads();
  if (threadIdx.x < 2) {  // exclusive offsets, largest class first
    int32_t run = 0;
    for (int c = PLAN_CLASSES - 1; c >= 0; --c) {
      const int32_t k = off[threadIdx.x][c];
      off[threadIdx.x][c] = run;
      run += k;
    }
    if (threadIdx.x == 0) ctl->n_whole = run;
    else ctl->n_whole2 = run;
  }
  __syncthreads();
  for (int64_t g = threadIdx.x; g < G; g += PLAN_THREADS) {
    const uint8_t m = S.mode[g];
    if (m == 1 || m == 3) {
      const int32_t at = atomicAdd(&off[m == 3][plan_class(S.n[g])], 1);
      (m == 3 ? whole2 : S.whole)[at] = (int32_t)g;
    }
    S.nnew[g] = 0;
  }
  if (nnz_acc) atomicAdd((unsigned long long*)&ctl->whole_nnz, (unsigned long long)nnz_acc);
  if (nv_acc) atomicAdd((unsigned long long*)&ctl->whole_nv, (unsigned long long)nv_acc);
  if (region) atomicAdd(&ctl->n_region, region);
}

// ------------------------------------------------------- Padberg-Rinaldi
// For e = (u, v): PR1 w >= lambda-hat, or PR2 2w > c(u) or 2w > c(v)
// (strict).  Both keep every minimum cut when lambda-hat <= the minimum
// degree (sections "Related Work" and "Inexact Shared-Memory Minimum Cuts"
// name the tests; the conditions are restated here).
//
// With a small bound almost every edge passes PR1 and the unions pile onto
// one giant set; done edge by edge they all contend for its root.  So a
// vertex pass first unites each vertex with the first PR_SAMPLE entries of
// its row that pass, the forest is flattened, and the edge pass then skips
// every passing edge whose ends already share a parent (the union is
// idempotent, so the filter only saves work).  Per graph, ucount is set to
// 1 once any edge passed.
constexpr int PR_SAMPLE = 2;

__device__ __forceinline__ bool pr_passes(int64_t c, int64_t lam, int64_t cu, int64_t cv) {
  return c >= lam || 2 * c > cu || 2 * c > cv;
}

// An edge with 2c <= lambda-hat passes neither test: lambda-hat is at most
// the minimum degree, so 2c <= c(u) and 2c <= c(v), and c < lambda-hat.
// Checked first, it spares the two degree gathers of most edges.
__device__ __forceinline__ bool pr_hopeless(int64_t c, int64_t lam) { return 2 * c <= lam; }

__device__ __forceinline__ void pr_flag(int32_t* ucount, int32_t g, int32_t& last) {
  if (g != last) {
    if (ld_relaxed(ucount + g) == 0) st_relaxed(ucount + g, 1);
    last = g;
  }
}

// Loads are grouped so that each round trip serves every entry the thread
// holds, and no load waits inside a divergent branch: an entry that needs
// nothing reads a shared dummy address instead.  chmax (the chunk maxima of
// this graph, or null): a vertex whose sampled entries lie in chunks whose
// largest weight cannot pass skips their loads.
__global__ void k_pr_sample(int32_t n, int64_t nnz, const int64_t* __restrict__ rp,
                            const int32_t* __restrict__ col, const int32_t* __restrict__ w,
                            const int32_t* __restrict__ chmax,
                            const int64_t* __restrict__ cdeg, const int32_t* __restrict__ gid,
                            const int64_t* __restrict__ lhat, const int32_t* __restrict__ active, int32_t* parent,
                            int32_t* ucount) {
  if (nnz <= 0) return;
  int32_t last = -1;
  for (int64_t v = gtid(); v < n; v += gstride()) {
    const int32_t g = gid[v];
    const int64_t cv = cdeg[v], e0 = rp[v], e1 = rp[v + 1];
    const bool act = active[g] != 0;
    const int64_t lam = lhat[g];
    bool live = e1 > e0;
    if (chmax && live) {
      const int64_t el = min(e0 + PR_SAMPLE, e1) - 1;  // the last sampled entry
      const int32_t m0 = chmax[e0 / WCH], m1 = chmax[el / WCH];
      live = !pr_hopeless(m0 > m1 ? m0 : m1, lam);
    }
    int32_t u[PR_SAMPLE], c[PR_SAMPLE];
#pragma unroll
    for (int k = 0; k < PR_SAMPLE; ++k) {
      const int64_t e = live && e0 + k < e1 ? e0 + k : 0;
      u[k] = col[e];
      c[k] = w[e];
    }
    bool keep[PR_SAMPLE];
    int64_t cu[PR_SAMPLE];
#pragma unroll
    for (int k = 0; k < PR_SAMPLE; ++k) {
      keep[k] = act && live && e0 + k < e1 && u[k] != (int32_t)v && !pr_hopeless(c[k], lam);
      cu[k] = cdeg[keep[k] ? u[k] : (int32_t)v];
    }
#pragma unroll
    for (int k = 0; k < PR_SAMPLE; ++k)
      if (keep[k] && pr_passes(c[k], lam, cv, cu[k])) {
        uf_union(parent, (int32_t)v, u[k]);
        pr_flag(ucount, g, last);
      }
  }
}

// ctl->lam_floor = the smallest bound among the tested graphs (one
// workgroup): with it, k_pr drops an edge from its weight alone.
__global__ void __launch_bounds__(256) k_lam_floor(int32_t G, const int64_t* lhat, const int32_t* active,
                                                   Ctl* ctl) {
  __shared__ int64_t part[4];
  int64_t m = INT64_MAX;
  for (int32_t g = threadIdx.x; g < G; g += 256)
    if (active[g]) m = min(m, lhat[g]);
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t t = __shfl_xor(m, o, 64);
    m = min(m, t);
  }
  if (lane_id() == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) ctl->lam_floor = min(min(part[0], part[1]), min(part[2], part[3]));
}

// One WCH-entry chunk per wave step (slot k of each lane: entry
// e0 + k * 64 + lane), loaded in rounds (weight; rows and ends; graph; its
// bound; both degrees), each round for all slots; an entry already decided
// reads a shared dummy address.  A chunk none of whose weights can pass for
// any graph is dropped before its rows are found.  chmax (the chunk maxima
// of this graph, or null): the wave reads the maxima of its next 64 chunks
// at once and skips the hopeless ones without reading their entries.
__global__ void __launch_bounds__(256) k_pr(int32_t n, int64_t nnz, const int64_t* __restrict__ rp,
                                            const int32_t* __restrict__ first,
                                            const int32_t* __restrict__ col, const int32_t* __restrict__ w,
                                            const int32_t* __restrict__ chmax,
                                            const int64_t* __restrict__ cdeg, const int32_t* __restrict__ gid,
                                            const int64_t* __restrict__ lhat, const int32_t* __restrict__ active,
                                            int32_t* parent, int32_t* ucount, Ctl* ctl) {
  __shared__ int32_t pos_all[4][WCH];
  int32_t* pos = pos_all[threadIdx.x >> 6];
  const int lane = lane_id();
  int64_t local = 0;
  int32_t last = -1;
  const int64_t floor = ctl->lam_floor;  // hopeless for every graph: 2c <= floor
  const int64_t nch = (nnz + WCH - 1) / WCH, W = gwaves();
  // the wave's chunks gwave() + m W, m = 0, 1, ..., in groups of 64
  for (int64_t cb = gwave(); cb < nch; cb += 64 * W) {
    const int64_t cl = cb + lane * W;
    uint64_t todo = ballot(cl < nch && (chmax == nullptr || !pr_hopeless(chmax[cl < nch ? cl : 0], floor)));
    while (todo) {
      const int64_t ch = cb + (int64_t)__builtin_ctzll(todo) * W;
      todo &= todo - 1;
      const int64_t e0 = ch * WCH;
      int32_t c[8], u[8], v[8], g[8];
      bool keep[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int64_t e = e0 + k * 64 + lane;
        c[k] = w[e < nnz ? e : e0];
      }
      bool any = false;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        keep[k] = e0 + k * 64 + lane < nnz && !pr_hopeless(c[k], floor);
        any = any || keep[k];
      }
      if (ballot(any) == 0) continue;  // wave-uniform: nothing left to test
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = col[keep[k] ? e0 + k * 64 + lane : e0];
      chunk_rows(rp, n, e0, chunk_first(first, ch, n), pos, u);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        keep[k] = keep[k] && u[k] < v[k];
        g[k] = gid[keep[k] ? u[k] : 0];
      }
      int64_t lam[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool act = active[g[k]] != 0;
        lam[k] = lhat[g[k]];
        keep[k] = keep[k] && act && !pr_hopeless(c[k], lam[k]);
      }
      int64_t cu[8], cv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        cu[k] = cdeg[keep[k] ? u[k] : 0];
        cv[k] = cdeg[keep[k] ? v[k] : 0];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (keep[k] && pr_passes(c[k], lam[k], cu[k], cv[k])) {
          ++local;
          pr_flag(ucount, g[k], last);
          if (ld_relaxed(parent + u[k]) != ld_relaxed(parent + v[k])) uf_union(parent, u[k], v[k]);
        }
    }
  }
  // one add per wave: per-thread adds on the one counter serialise
  local = wave_sum_i64(local);
  if (lane_id() == 0 && local) atomicAdd((unsigned long long*)&ctl->unions_pr, (unsigned long long)local);
}

// The triangle tests of edge (u, v), c = its entry's weight: PR3 (a common
// neighbour w with c(u) < 2 (c + c(u,w)) and c(v) < 2 (c + c(v,w))) and PR4
// (c + the sum over common neighbours of min(c(u,w), c(v,w)) >= lambda-hat).
// Strict PR3 holds for every non-trivial minimum cut at once, PR4 bounds
// lambda(u, v) from below, so passing edges contract together with the
// round's other unions.  Evaluated only when both rows hold at most max_deg
// entries in strictly increasing neighbour order (then c(u,w) is one entry;
// contracted graphs always are); one merge walks both rows to their ends,
// checking the order as it goes.  Returns bit 4 (PR3) and bit 8 (PR4).
__device__ __forceinline__ uint32_t pr34_eval(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                              const int32_t* __restrict__ w, const int64_t* __restrict__ cdeg,
                                              int32_t u, int32_t v, int64_t c, int64_t lam, int32_t max_deg) {
  const int64_t a1 = rp[u + 1], b1 = rp[v + 1];
  int64_t a = rp[u], b = rp[v];
  if (a1 - a > max_deg || b1 - b > max_deg) return 0;
  const int64_t du = cdeg[u], dv = cdeg[v];
  constexpr int32_t END = INT32_MAX;  // past a row's end (vertex ids are below 2^30)
  int32_t x = a < a1 ? col[a] : END, y = b < b1 ? col[b] : END;
  int64_t paths = c;
  bool pr3 = false;
  while (x != END || y != END) {
    const bool adv_a = x <= y, adv_b = y <= x;
    if (x == y && x != u && x != v) {
      const int64_t cu = w[a], cv = w[b];
      paths += cu < cv ? cu : cv;
      pr3 = pr3 || (du < 2 * (c + cu) && dv < 2 * (c + cv));
    }
    if (adv_a) {
      const int32_t px = x;
      ++a;
      x = a < a1 ? col[a] : END;
      if (x != END && x <= px) return 0;
    }
    if (adv_b) {
      const int32_t py = y;
      ++b;
      y = b < b1 ? col[b] : END;
      if (y != END && y <= py) return 0;
    }
  }
  return (pr3 ? 4u : 0u) | (paths >= lam ? 8u : 0u);
}

// Unions of the edges passing PR3 or PR4 (and not already PR1/PR2 unions).
__global__ void k_pr34(int64_t nnz, const int32_t* __restrict__ src, const int32_t* __restrict__ col,
                       const int32_t* __restrict__ w, const int64_t* __restrict__ rp,
                       const int64_t* __restrict__ cdeg, const int32_t* __restrict__ gid,
                       const int64_t* __restrict__ lhat, const int32_t* __restrict__ active, int32_t max_deg,
                       int32_t* parent, int32_t* ucount, Ctl* ctl) {
  int64_t local = 0;
  int32_t last = -1;
  for (int64_t e = gtid(); e < nnz; e += gstride()) {
    const int32_t u = src[e], v = col[e];
    if (u >= v) continue;
    const int32_t g = gid[u];
    if (!active[g]) continue;
    const int64_t lam = lhat[g];
    if (pr_passes(w[e], lam, cdeg[u], cdeg[v])) continue;  // united by the PR1/PR2 pass
    if (!pr34_eval(rp, col, w, cdeg, u, v, w[e], lam, max_deg)) continue;
    ++local;
    pr_flag(ucount, g, last);
    if (ld_relaxed(parent + u) != ld_relaxed(parent + v)) uf_union(parent, u, v);
  }
  // one add per wave: per-thread adds on the one counter serialise
  local = wave_sum_i64(local);
  if (lane_id() == 0 && local) atomicAdd((unsigned long long*)&ctl->unions_pr, (unsigned long long)local);
}

// Every test's outcome per entry (u, v), u < v (bits PR1 1, PR2 2, PR3 4,
// PR4 8; 0 for the other entries), one thread per vertex row.
__global__ void k_pr_flags(int32_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ w, const int64_t* __restrict__ cdeg, int64_t lam,
                           int32_t max_deg, uint8_t* flags) {
  for (int64_t u = gtid(); u < n; u += gstride()) {
    for (int64_t e = rp[u]; e < rp[u + 1]; ++e) {
      const int32_t v = col[e];
      uint32_t f = 0;
      if ((int32_t)u < v) {
        const int64_t c = w[e];
        if (c >= lam) f |= 1;
        if (2 * c > cdeg[u] || 2 * c > cdeg[v]) f |= 2;
        f |= pr34_eval(rp, col, w, cdeg, (int32_t)u, v, c, lam, max_deg);
      }
      flags[e] = (uint8_t)f;
    }
  }
}

// Graphs that get a full-graph sweep this round: region-mode graphs when the
// sweep is the scan of choice, and any graph whose scans found no pair.
__global__ void k_sweep_list(int32_t G, GraphState S, int32_t sweep_region, Ctl* ctl) {
  for (int64_t g = gtid(); g < G; g += gstride())
    if ((S.mode[g] == 2 && sweep_region) || (S.mode[g] != 0 && S.ucount[g] == 0)) {
      int32_t i = atomicAdd(&ctl->n_fallback, 1);
      S.fb_list[i] = (int32_t)g;
    }
}

// Per swept graph: first vertex, vertex count, bound and entry range.
__global__ void k_sweep_info(const int32_t* list, const Ctl* ctl, const int32_t* cvoff, const int32_t* gn,
                             const int64_t* lhat, const int64_t* rp, int64_t* info) {
  for (int64_t i = gtid(); i < ctl->n_fallback; i += gstride()) {
    const int32_t g = list[i];
    info[5 * i] = cvoff[g];
    info[5 * i + 1] = gn[g];
    info[5 * i + 2] = lhat[g];
    info[5 * i + 3] = rp[cvoff[g]];
    info[5 * i + 4] = rp[cvoff[g] + gn[g]];
  }
}

__global__ void k_sweep_report(const SweepArgs* args, int32_t k, GraphState S) {
  for (int64_t i = gtid(); i < k; i += gstride()) {
    const MC_GLOBAL SweepCtl* c = (const MC_GLOBAL SweepCtl*)args[i].ctl;
    const int32_t g = args[i].g;
    // the best prefix of the sweep, or of a tail process (record k: the
    // process in bits 20..29, its pops in the low 20 bits)
    int64_t a = c->best_alpha;
    uint32_t sid = (uint32_t)SWEEP_SID;
    int32_t k = c->best_step;
    const uint64_t tb = c->tail_best;
    if (tb != ~0ull && (int64_t)(tb >> 32) < a) {
      const int32_t f = (int32_t)(uint32_t)tb;
      a = (int64_t)(tb >> 32);
      sid = (uint32_t)TAIL_SID;
      k = (f << 20) | c->tail_k[f];
    }
    if (a < S.lhat[g]) {
      S.fb_k[g] = k;
      atomic_min_u64(S.balpha + g, ((uint64_t)a << 32) | sid);
    }
    atomicAdd(S.ucount + g, min(c->cap_tail, args[i].ng));  // one union per crossing recorded
  }
}

// ------------------------------------------------------------ compaction
// Block ids: every union-find root of a graph that stays in play gets a new
// id in [0, n'), in vertex order, so each graph's range stays contiguous.
struct RootFlag {
  const int32_t* parent;
  const int32_t* gid;
  const int32_t* keep;  // per graph
  int32_t carry;        // 1: every graph is kept
  __device__ __forceinline__ int32_t operator()(int64_t v) const {
    // every load issued whatever the parent and the mode (no load behind a
    // short circuit or a branch: those wait for it at once)
    const int32_t p = parent[v], g = gid[v];
    const int32_t k = keep[g];
    return (int32_t)(p == v) & (int32_t)((carry | k) != 0);
  }
};

__global__ void k_relabel(int32_t n, const int32_t* parent, const int32_t* gid, const int32_t* keep,
                          int32_t carry, const int32_t* newid, int32_t* lab, int32_t* ngid, int32_t* nnew) {
  for (int64_t v = gtid(); v - lane_id() < n; v += gstride()) {  // wave-uniform bound
    const bool ok = v < n;
    const int32_t g = ok ? gid[v] : -1;
    const bool kept = ok && (carry || keep[g]);
    bool root = false;
    if (ok) {
      const int32_t r = parent[v];
      if (!kept) {
        lab[v] = -1;
      } else {
        lab[v] = newid[r];
        root = r == v;
        if (root) ngid[newid[v]] = g;
      }
    }
    wave_add_by_key(nnew, g, 1, root);
  }
}

// Bound update from the scans' best prefix cut alpha (section "Parallel
// CAPFOREST": lambda-hat <- min(lambda-hat, alpha)).
__global__ void k_update_alpha(int32_t G, GraphState S, const int32_t* scan_k, Ctl* ctl) {
  for (int64_t g = gtid(); g < G; g += gstride()) {
    uint64_t b = S.balpha[g];
    if (b == ~0ull || !S.mode[g]) continue;
    int64_t a = (int64_t)(b >> 32);
    if (a < S.lhat[g]) {
      int32_t sid = (int32_t)(uint32_t)b;
      S.lhat[g] = a;
      S.rec_type[g] = REC_ALPHA;
      S.rec_id[g] = sid;
      S.rec_k[g] = (sid == SWEEP_SID || sid == TAIL_SID) ? S.fb_k[g] : scan_k[sid];
      atomicAdd(&ctl->improved, 1);
    }
  }
}

// ----------------------------------------------------------- contraction
// Emit (lab[u] << bits | lab[v], w) for every entry whose ends lie in
// different blocks (internal edges vanish; section "Basic Concepts",
// contraction G/(u,v)).  Workgroup-aggregated compaction.
// The entries inside one block are dropped by the emit, and after a sweep
// most of a graph's vertices usually share one block.  Per graph a reference
// block (the most common block among 64 evenly spaced vertices: any block is
// correct, a large one saves most) and a bitmap of the vertices in it let the
// emit drop an entry whose two ends are both in it from two bit tests in an
// L2-resident bitmap, without gathering the labels.
__global__ void k_block_ref(int32_t G, int32_t n, const int32_t* cvoff, const int32_t* gn, const int32_t* lab,
                            int32_t* ref) {
  const int lane = lane_id();
  for (int64_t g = gtid() >> 6; g < G; g += gstride() >> 6) {
    const int64_t c0 = cvoff[g], cn = gn[g];
    const int64_t v = c0 + (int64_t)lane * cn / 64;
    int32_t l = (cn > 0 && v >= 0 && v < n) ? lab[v] : -1;
    uint64_t todo = ballot(l >= 0);
    int32_t best = -1, best_cnt = 0;
    while (todo) {
      const int32_t cand = __builtin_amdgcn_readlane(l, __builtin_ctzll(todo));
      const uint64_t same = ballot(l == cand);
      const int32_t cnt = popc64(same);
      if (cnt > best_cnt) { best_cnt = cnt; best = cand; }
      todo &= ~same;
    }
    if (lane == 0) ref[g] = best;
  }
}

// bit v of inref: v's block is its graph's reference block (one wave per 64
// vertices).  With rp: also the entries of the rows outside reference
// blocks into ctl->nonref_nnz (the row-wise emit's work).
__global__ void k_block_bits(int32_t n, const int32_t* lab, const int32_t* gid, const int32_t* ref,
                             uint32_t* inref, const int64_t* rp, Ctl* ctl) {
  int64_t rows = 0;
  for (int64_t base = (gtid() >> 6) << 6; base < n; base += gstride()) {
    const int64_t v = base + lane_id();
    const int32_t l = v < n ? lab[v] : -1;
    const bool in = l >= 0 && l == ref[gid[v]];
    const uint64_t m = ballot(in);
    if (lane_id() == 0) {
      inref[base >> 5] = (uint32_t)m;
      inref[(base >> 5) + 1] = (uint32_t)(m >> 32);
    }
    if (rp && l >= 0 && !in) rows += rp[v + 1] - rp[v];
  }
  if (rp) {
    rows = wave_sum_i64(rows);
    if (lane_id() == 0 && rows) atomicAdd((unsigned long long*)&ctl->nonref_nnz, (unsigned long long)rows);
  }
}

__device__ __forceinline__ bool bit_at(const uint32_t* b, int32_t v) { return (b[v >> 5] >> (v & 31)) & 1u; }

// Contraction keys: per crossing entry (u, x) with blocks a = lab[u] != b =
// lab[x], the key (a << bits) | b and the entry's weight.  One WCH-entry
// chunk per wave step, rows from chunk_rows.  Survivors are staged in the
// wave's LDS and written out in runs of up to WCH: one atomic reservation
// per run instead of one per chunk (reservations on the one counter
// serialise).  inref (optional): bit v set when v's block is its graph's
// reference block; an entry with both ends there cannot cross and is
// dropped from the bits alone, before its labels are read.  The order of
// the emitted entries is free: they are sorted next.
__global__ void __launch_bounds__(256) k_emit(int32_t n, int64_t nnz, const int64_t* __restrict__ rp,
                                              const int32_t* __restrict__ first,
                                              const int32_t* __restrict__ col,
                                              const int32_t* __restrict__ w,
                                              const int32_t* __restrict__ lab, int bits,
                                              const uint32_t* __restrict__ inref,
                                              uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                                              Ctl* ctl) {
  __shared__ int32_t pos_all[4][WCH];
  __shared__ uint64_t stk_all[4][WCH];
  __shared__ int32_t stv_all[4][WCH];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  int32_t* pos = pos_all[wave];
  uint64_t* st_k = stk_all[wave];
  int32_t* st_v = stv_all[wave];
  uint32_t st_n = 0;  // wave-uniform
  auto flush = [&]() {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd((unsigned long long*)&ctl->emit, (unsigned long long)st_n);
    base = (unsigned long long)readlane_i64((int64_t)base, 0);
    wave_lds_sync();
    for (uint32_t i = lane; i < st_n; i += 64) {
      keys[base + i] = st_k[i];
      vals[base + i] = st_v[i];
    }
    wave_lds_sync();
    st_n = 0;
  };
  for (int64_t ch = gwave(); ch * WCH < nnz; ch += gwaves()) {
    const int64_t e0 = ch * WCH;
    // the loads of a step are issued for all eight slots before any result
    // is used, and none sits in a lane-divergent branch: a slot with nothing
    // to fetch reads the chunk's first element (one shared line)
    int32_t x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int64_t e = e0 + k * 64 + lane;
      x[k] = col[e < nnz ? e : e0];
    }
    int32_t u[8];
    chunk_rows(rp, n, e0, chunk_first(first, ch, n), pos, u);
    bool skip[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) skip[k] = e0 + k * 64 + lane >= nnz;
    if (inref) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t bu = inref[u[k] >> 5], bx = inref[x[k] >> 5];
        skip[k] = skip[k] | (((bu >> (u[k] & 31)) & (bx >> (x[k] & 31)) & 1u) != 0);
      }
    }
    // a chunk whose entries all stay inside reference blocks (most of them,
    // once a round has contracted most of the graph) loads nothing more
    // (the test is wave-uniform); otherwise every slot's labels and weight
    // go out together, a skipped entry reading the chunk's first (one
    // shared line)
    bool any = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) any = any || !skip[k];
    if (ballot(any) == 0) continue;
    int32_t la[8], lb[8], cw[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      la[k] = lab[skip[k] ? 0 : u[k]];
      lb[k] = lab[skip[k] ? 0 : x[k]];
      cw[k] = w[skip[k] ? e0 : e0 + k * 64 + lane];
    }
    uint64_t key[8];
    uint64_t msk[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool ok = !skip[k] && la[k] >= 0 && lb[k] >= 0 && la[k] != lb[k];
      key[k] = ((uint64_t)(uint32_t)la[k] << bits) | (uint32_t)lb[k];
      msk[k] = ballot(ok);
    }
    uint32_t tot = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) tot += popc64(msk[k]);
    if (tot == 0) continue;  // wave-uniform
    if (st_n + tot > (uint32_t)WCH) flush();
    uint32_t o = st_n;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((msk[k] >> lane) & 1) {
        const uint32_t at = o + popc64(msk[k] & lanemask_lt());
        st_k[at] = key[k];
        st_v[at] = cw[k];
      }
      o += popc64(msk[k]);
    }
    st_n += tot;
  }
  if (st_n) flush();
}

// The same keys, row by row, for contractions where most vertices lie in
// their graph's reference block: only rows of vertices outside it are read.
// The CSR is symmetric (each edge in both rows, same weight), so an entry
// (u, x) with x in a reference block also yields the key of its mirror
// (x, u), whose row is skipped; an entry with both ends outside is emitted
// from each end's own row.  One wave per 64 vertices; each selected row is
// read by the whole wave, 64 entries a step.  Survivors are staged as in
// k_emit.
__global__ void __launch_bounds__(256) k_emit_rows(int32_t n, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col,
                                                   const int32_t* __restrict__ w,
                                                   const int32_t* __restrict__ lab, int bits,
                                                   const uint32_t* __restrict__ inref,
                                                   uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                                                   Ctl* ctl) {
  __shared__ uint64_t stk_all[4][WCH];
  __shared__ int32_t stv_all[4][WCH];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  uint64_t* st_k = stk_all[wave];
  int32_t* st_v = stv_all[wave];
  uint32_t st_n = 0;  // wave-uniform
  auto flush = [&]() {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd((unsigned long long*)&ctl->emit, (unsigned long long)st_n);
    base = (unsigned long long)readlane_i64((int64_t)base, 0);
    wave_lds_sync();
    for (uint32_t i = lane; i < st_n; i += 64) {
      keys[base + i] = st_k[i];
      vals[base + i] = st_v[i];
    }
    wave_lds_sync();
    st_n = 0;
  };
  for (int64_t base = gwave() << 6; base < n; base += gwaves() << 6) {
    const int64_t v = base + lane;
    const int32_t l = v < n ? lab[v] : -1;
    const bool in = v < n && ((inref[v >> 5] >> (v & 31)) & 1u);
    uint64_t todo = ballot(l >= 0 && !in);
    while (todo) {
      const int src_lane = (int)__builtin_ctzll(todo);
      todo &= todo - 1;
      const int32_t u = (int32_t)base + src_lane;
      const int32_t a = __builtin_amdgcn_readlane(l, src_lane);
      const int64_t e0 = rp[u], e1 = rp[u + 1];
      for (int64_t b0 = e0; b0 < e1; b0 += 64) {
        const int64_t e = b0 + lane;
        const bool ok = e < e1;
        const int64_t ec = ok ? e : b0;
        const int32_t x = col[ec];
        const int32_t c = w[ec];
        const bool xin = ok && ((inref[x >> 5] >> (x & 31)) & 1u);
        const int32_t b = ok ? lab[x] : -1;
        const bool keep = ok && b >= 0 && b != a;
        const bool mirror = keep && xin;
        const uint64_t mk = ballot(keep), mm = ballot(mirror);
        const uint32_t tot = popc64(mk) + popc64(mm);
        if (tot == 0) continue;  // wave-uniform
        if (st_n + tot > (uint32_t)WCH) flush();
        if (keep) {
          const uint32_t at = st_n + popc64(mk & lanemask_lt());
          st_k[at] = ((uint64_t)(uint32_t)a << bits) | (uint32_t)b;
          st_v[at] = c;
        }
        if (mirror) {
          const uint32_t at = st_n + popc64(mk) + popc64(mm & lanemask_lt());
          st_k[at] = ((uint64_t)(uint32_t)b << bits) | (uint32_t)a;
          st_v[at] = c;
        }
        st_n += tot;
      }
    }
  }
  if (st_n) flush();
}

struct HeadFlag {
  const uint64_t* keys;
  __device__ __forceinline__ int64_t operator()(int64_t i) const {
    const uint64_t a = keys[i], b = keys[i > 0 ? i - 1 : 0];  // no load behind a short circuit
    return (i == 0 || a != b) ? 1 : 0;
  }
};

// Merge runs of equal (a, b) keys: new entry index = number of run heads
// up to and including i, minus one; weights summed (wave-segmented, then
// one atomic per run piece).
__global__ void __launch_bounds__(256) k_merge(int64_t m, const uint64_t* __restrict__ keys,
                                               const int32_t* __restrict__ vals,
                                               const int64_t* __restrict__ pos, int bits,
                                               int32_t* nsrc, int32_t* ncol, int32_t* nw) {
  const uint64_t mask = (1ull << bits) - 1;
  for (int64_t base = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); base < m;
       base += (int64_t)gridDim.x * 256) {
    int64_t i = base + lane_id();
    bool ok = i < m;
    uint64_t key = ok ? keys[i] : ~0ull;
    bool head = ok && (i == 0 || keys[i - 1] != key);
    // pos[] counts the run heads strictly before i; a non-head element's own
    // head is among them, so its run index is one less
    int64_t p = ok ? pos[i] - (head ? 0 : 1) : -1;
    if (head) {
      nsrc[p] = (int32_t)(key >> bits);
      ncol[p] = (int32_t)(key & mask);
    }
    bool tail;
    int32_t s = wave_segsum<int64_t, int32_t>(p, ok ? vals[i] : 0, ok, tail);
    if (ok && tail) atomicAdd(nw + p, s);
  }
}

// Opt-in symmetry check of the input.  Every entry (u, v, c) with u != v
// becomes the key of its unordered pair {u, v} with +c when it sits in the
// row of the smaller end and -c otherwise; sorted and summed per key
// (k_merge), a symmetric graph leaves every sum 0.
__global__ void __launch_bounds__(256) k_sym_emit(int64_t nnz, const int32_t* __restrict__ src,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ w, int bits,
                                                  uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                                                  Ctl* ctl) {
  const int lane = lane_id();
  for (int64_t base = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); base < nnz;
       base += (int64_t)gridDim.x * 256) {  // wave-uniform bound
    const int64_t e = base + lane;
    const bool ok = e < nnz;
    const int64_t ec = ok ? e : base;
    const int32_t u = src[ec], v = col[ec], c = w[ec];
    const bool keep = ok && u != v;
    const uint64_t m = ballot(keep);
    if (m == 0) continue;
    unsigned long long at = 0;
    if (lane == 0) at = atomicAdd((unsigned long long*)&ctl->emit, (unsigned long long)popc64(m));
    at = bcast(at, 0);
    if (keep) {
      const int64_t i = (int64_t)at + popc64(m & lanemask_lt());
      const uint32_t lo = (uint32_t)min(u, v), hi = (uint32_t)max(u, v);
      keys[i] = ((uint64_t)lo << bits) | hi;
      vals[i] = u < v ? c : -c;
    }
  }
}

// Any nonzero per-pair sum left by the symmetry check sets ctl->asym.
__global__ void k_sym_nonzero(int64_t m, const int32_t* sums, Ctl* ctl) {
  bool bad = false;
  for (int64_t i = gtid(); i < m; i += gstride()) bad |= sums[i] != 0;
  if (ballot(bad) && lane_id() == 0) atomicOr(&ctl->asym, 1);
}

// row_ptr of the merged graph: rp[a] = first entry with source >= a.
__global__ void k_rowptr(int32_t n, int64_t m, const int32_t* nsrc, int64_t* rp) {
  for (int64_t a = gtid(); a <= n; a += gstride()) {
    int64_t lo = 0, hi = m;  // first index with nsrc >= a
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (nsrc[mid] < a) lo = mid + 1; else hi = mid;
    }
    rp[a] = lo;
  }
}

__global__ void __launch_bounds__(256) k_degrees(int64_t m, const int32_t* __restrict__ nsrc,
                                                 const int32_t* __restrict__ nw, int64_t* cdeg) {
  for (int64_t base = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63); base < m;
       base += (int64_t)gridDim.x * 256) {
    int64_t i = base + lane_id();
    bool ok = i < m;
    int32_t a = ok ? nsrc[i] : -1;
    bool tail;
    int64_t s = wave_segsum<int32_t, int64_t>(a, ok ? (int64_t)nw[i] : 0, ok, tail);
    if (ok && tail) atomicAdd((unsigned long long*)(cdeg + a), (unsigned long long)s);
  }
}

// After contraction: new vertex counts and ranges, minimum degree bound of
// the contracted graph (section "Parallel Graph Contraction"), activity.
__global__ void k_finish_round(int32_t G, GraphState S, const int32_t* nvoff_scan, Ctl* ctl) {
  for (int64_t g = gtid(); g < G; g += gstride()) {
    if (!S.mode[g]) {
      if (S.active[g]) S.active[g] = 0;
      S.n[g] = 0;
      continue;
    }
    S.n[g] = S.nnew[g];
    S.cvoff[g] = nvoff_scan[g];
    if (S.nnew[g] >= 2) {
      uint64_t bd = S.bdeg[g];
      int64_t d = (int64_t)(bd >> 32);
      if (bd != ~0ull && d < S.lhat[g]) {
        S.lhat[g] = d;
        S.rec_type[g] = REC_DEG;
        S.rec_id[g] = (int32_t)(uint32_t)bd;
        S.rec_k[g] = 0;
        atomicAdd(&ctl->improved, 1);
      }
    }
    int32_t act = (S.nnew[g] > 2 && S.lhat[g] > 0) ? 1 : 0;
    S.active[g] = act;
    if (act) atomicAdd(&ctl->n_active, 1);
  }
}

// ------------------------------------------------ VieCut-style levels
// Per graph during the clustering levels: S.n / S.cvoff follow the level
// graph, vc_act marks graphs still being coarsened, vc_n0 holds the vertex
// count at the start of the level.
__global__ void k_vc_init(int32_t G, GraphState S, int32_t stop, int32_t* vc_act, int32_t* vc_n0, Ctl* ctl) {
  for (int64_t g = gtid(); g < G; g += gstride()) {
    const int32_t act = (S.active[g] && S.n[g] > stop && S.lhat[g] > 0) ? 1 : 0;
    vc_act[g] = act;
    vc_n0[g] = S.n[g];
    S.rec_type[g] = REC_NONE;
    if (act) atomicAdd(&ctl->n_active, 1);
  }
}

// After a contraction of the level: the new graph's minimum degree bounds
// lambda-hat (each of its vertices is a vertex set of the input graph).
// end_of_level: also stop graphs that shrank by less than a tenth over the
// level, or reached the level limit.
// carry: graphs that stopped stay in the level graph (as themselves), so
// their counts and offsets follow it.
__global__ void k_vc_level(int32_t G, GraphState S, const int32_t* nvoff_scan, int32_t stop, int32_t end_of_level,
                           int32_t last_level, int32_t carry, int32_t* vc_act, int32_t* vc_n0, Ctl* ctl) {
  for (int64_t g = gtid(); g < G; g += gstride()) {
    S.rec_type[g] = REC_NONE;
    if (!vc_act[g]) {
      if (carry) {
        S.n[g] = S.nnew[g];
        S.cvoff[g] = nvoff_scan[g];
      }
      continue;
    }
    const int32_t nn = S.nnew[g];
    S.n[g] = nn;
    S.cvoff[g] = nvoff_scan[g];
    if (nn >= 2) {
      const uint64_t bd = S.bdeg[g];
      const int64_t d = (int64_t)(bd >> 32);
      if (bd != ~0ull && d < S.lhat[g]) {
        S.lhat[g] = d;
        S.rec_type[g] = REC_DEG;
        S.rec_id[g] = (int32_t)(uint32_t)bd;
        S.rec_k[g] = 0;
        atomicAdd(&ctl->improved, 1);
      }
    }
    bool go = nn > stop && S.lhat[g] > 0;
    if (end_of_level) {
      go = go && !last_level && (int64_t)nn * 10 <= (int64_t)vc_n0[g] * 9;
      vc_n0[g] = nn;
    }
    vc_act[g] = go ? 1 : 0;
    if (go) atomicAdd(&ctl->n_active, 1);
  }
}

// The last level graphs become the exact loop's input (the exact finish):
// their counts and offsets stay; a graph with at most two vertices or a zero
// bound is final.
__global__ void k_vc_exact_start(int32_t G, GraphState S, Ctl* ctl) {
  for (int64_t g = gtid(); g < G; g += gstride()) {
    S.rec_type[g] = REC_NONE;
    const int32_t act = (S.active[g] && S.n[g] > 2 && S.lhat[g] > 0) ? 1 : 0;
    S.active[g] = act;
    if (act) atomicAdd(&ctl->n_active, 1);
  }
}

// Back to the input graphs for the exact loop; a zero bound is final.
__global__ void k_vc_done(int32_t G, GraphState S, Ctl* ctl) {
  for (int64_t g = gtid(); g < G; g += gstride()) {
    S.n[g] = (int32_t)(S.voff[g + 1] - S.voff[g]);
    S.cvoff[g] = (int32_t)S.voff[g];
    S.rec_type[g] = REC_NONE;
    const int32_t act = (S.active[g] && S.lhat[g] > 0) ? 1 : 0;
    S.active[g] = act;
    if (act) atomicAdd(&ctl->n_active, 1);
  }
}

__global__ void k_compose_map(int32_t n0, int32_t* map, const int32_t* lab) {
  for (int64_t v = gtid(); v < n0; v += gstride()) {
    int32_t c = map[v];
    map[v] = c >= 0 ? lab[c] : -1;
  }
}

__global__ void k_normalize_side(int32_t G, const int64_t* voff, uint8_t* side, int32_t* flip) {
  for (int64_t g = gtid(); g < G; g += gstride()) flip[g] = side[voff[g]] ? 1 : 0;
}

__global__ void k_apply_flip(int32_t n0, const int32_t* ogid, const int32_t* flip, uint8_t* side) {
  for (int64_t v = gtid(); v < n0; v += gstride())
    if (flip[ogid[v]]) side[v] ^= 1;
}

}  // namespace mc
