// Capped CAPFOREST sweep of a whole small graph inside one workgroup
// (appendix Algorithm 3 with the cap of Lemma 1; batches of capped vertices
// as in sweep.h).  The graph's vertices [v0, v0 + ng) index LDS arrays
// directly: r (weight to the visited set) and the state, so every priority
// update is an LDS atomic.  Each step makes one pass over the graph's slots:
// all frontier vertices whose key reached the cap form the batch; if there
// are none, the frontier vertex with the largest key (< cap) is the batch.
// Crossing edges r(y) < cap <= r(y) + c(e) are recorded as pairs and united
// after the kernel; alpha (= c(S) of the visited set) is tracked per batch.
#pragma once
#include "capforest.h"
#include "sweep.h"

namespace mc {

struct SmallSweepArgs {
  const int64_t* rp;
  const int32_t* col;
  const int32_t* w;
  const int64_t* cdeg;
  const int64_t* lhat;
  const int32_t* gn;
  const int32_t* gvoff;
  const int32_t* list;         // graphs to sweep
  const int32_t* list_count;   // device count of `list`
  int32_t* work;               // work counter (zeroed by the host)
  int32_t* fb_step;            // visit stamp per vertex (side materialisation)
  int32_t* capq;               // crossing pairs (capx[i], capq[i]) at v0 + i
  int32_t* capx;
  int32_t* npairs;             // per graph: pairs recorded
  uint64_t* best_alpha;        // per graph (alpha << 32) | SWEEP_SID
  int32_t* fb_k;               // per graph: stamp of the best prefix
  int32_t* ucount;
  uint64_t seed;
};

constexpr int SS_THREADS = 256;

template <int CAP>
struct SmallSweepLds {
  int32_t r[CAP];
  int32_t batch[CAP];
  uint8_t st[CAP];  // 0 unseen, 1 frontier, 2 visited, 3 in the current batch
  int32_t nbatch, npairs;
  uint64_t best;
  int64_t wsum[SS_THREADS / 64], wint[SS_THREADS / 64];
  uint64_t wbest[SS_THREADS / 64];
};

template <int CAP>
__global__ void __launch_bounds__(SS_THREADS) k_small_sweep(SmallSweepArgs A) {
  extern __shared__ char lds_raw[];
  SmallSweepLds<CAP>& L = *reinterpret_cast<SmallSweepLds<CAP>*>(lds_raw);
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  constexpr int NW = SS_THREADS / 64;
  __shared__ int32_t sh_item;
  while (true) {
    if (threadIdx.x == 0) sh_item = atomicAdd(A.work, 1);
    __syncthreads();
    const int32_t item = sh_item;
    if (item >= *A.list_count) return;
    const int32_t g = A.list[item];
    const int32_t v0 = A.gvoff[g], ng = A.gn[g];
    const int64_t lam = A.lhat[g];
    for (int i = threadIdx.x; i < ng; i += SS_THREADS) {
      L.r[i] = 0;
      L.st[i] = 0;
      A.fb_step[v0 + i] = 0;
    }
    uint64_t h = A.seed * 0x9E3779B97F4A7C15ull + (uint64_t)g * 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
    const int32_t start = (int32_t)(h % (uint64_t)ng);
    if (threadIdx.x == 0) L.npairs = 0;
    __syncthreads();
    if (threadIdx.x == 0) L.st[start] = 1;
    int64_t alpha = 0, best_alpha = INT64_MAX;  // meaningful in thread 0
    int32_t visited = 0, best_step = 0, stamp = 0;
    __syncthreads();
    while (true) {
      // pass 1: capped frontier vertices form the batch; also the largest
      // key below the cap
      if (threadIdx.x == 0) L.nbatch = 0;
      __syncthreads();
      uint64_t best = 0;
      for (int base = wave * 64; base < ng; base += SS_THREADS) {
        const int i = base + lane;
        bool capped = false;
        if (i < ng && L.st[i] == 1) {
          const int64_t key = L.r[i];
          if (key >= lam) {
            capped = true;
          } else {
            const uint64_t c = ((uint64_t)(key + 1) << 32) | (uint32_t)i;
            best = c > best ? c : best;
          }
        }
        const uint64_t m = ballot(capped);
        if (m) {
          int32_t at = 0;
          if (lane == 0) at = atomicAdd(&L.nbatch, popc64(m));
          at = shfl(at, 0);
          if (capped) L.batch[at + popc64(m & lanemask_lt())] = i;
        }
      }
      best = wave_max_u64(best);
      if (lane == 0) L.wbest[wave] = best;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint64_t b = 0;
        for (int k = 0; k < NW; ++k) b = L.wbest[k] > b ? L.wbest[k] : b;
        if (L.nbatch == 0 && b != 0) {
          L.batch[0] = (int32_t)(uint32_t)b;
          L.nbatch = 1;
        }
      }
      __syncthreads();
      const int32_t nb = L.nbatch;
      if (nb == 0) break;  // frontier empty
      ++stamp;
      // mark the batch
      int64_t sum = 0;
      for (int k = threadIdx.x; k < nb; k += SS_THREADS) {
        const int32_t x = L.batch[k];
        L.st[x] = 3;
        A.fb_step[v0 + x] = stamp;
        sum += A.cdeg[v0 + x] - 2 * (int64_t)L.r[x];
      }
      __syncthreads();
      // relax the batch's rows: a wave per batch vertex, lanes over the row
      int64_t internal = 0;
      for (int k = wave; k < nb; k += NW) {
        const int32_t xl = L.batch[k];
        const int32_t x = v0 + xl;
        const int64_t e0 = A.rp[x], e1 = A.rp[x + 1];
        for (int64_t base = e0; base < e1; base += 64) {
          const int64_t e = base + lane;
          bool cross = false;
          int32_t yl = 0;
          if (e < e1) {
            yl = A.col[e] - v0;
            const int32_t c = A.w[e];
            const uint8_t s = L.st[yl];
            if (yl == xl) {
            } else if (s == 3) {
              internal += c;
            } else if (s != 2) {
              const int32_t old = atomicAdd(&L.r[yl], c);
              if (s == 0) L.st[yl] = 1;
              cross = (int64_t)old < lam && lam <= (int64_t)old + c;
            }
          }
          const uint64_t cm = ballot(cross);
          if (cm) {
            int32_t at = 0;
            if (lane == 0) at = atomicAdd(&L.npairs, popc64(cm));
            at = shfl(at, 0);
            if (cross) {
              const int32_t q = v0 + at + popc64(cm & lanemask_lt());
              A.capq[q] = v0 + yl;
              A.capx[q] = x;
            }
          }
        }
      }
      sum = wave_sum_i64(sum);
      internal = wave_sum_i64(internal);
      if (lane == 0) { L.wsum[wave] = sum; L.wint[wave] = internal; }
      __syncthreads();
      for (int k = threadIdx.x; k < nb; k += SS_THREADS) L.st[L.batch[k]] = 2;
      if (threadIdx.x == 0) {
        int64_t s = 0, in = 0;
        for (int k = 0; k < NW; ++k) { s += L.wsum[k]; in += L.wint[k]; }
        alpha += s - in;
        visited += nb;
        if (visited < ng && alpha < best_alpha) { best_alpha = alpha; best_step = stamp; }
      }
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
