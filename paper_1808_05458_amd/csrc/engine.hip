// Round driver and C ABI of the exact minimum-cut library.
//
// Algorithm 2 (Parallel Minimum Cut) on a packed set of graphs: after
// ingest (trivial bound, connectivity) every round runs Padberg-Rinaldi
// tests, bounded CAPFOREST scans (the sequential fallback where a graph got
// no contractible pair), union-find finish and block numbering, the bound
// update from the scans' prefix cuts, contraction and the minimum-degree
// bound of the contracted graph, until every graph has at most two vertices
// or a zero bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mincut.h"
#include "kernels.h"

namespace mc {

#define MC_HIP(call)                              \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) {                       \
      last_hip_error() = e_;                      \
      return MC_EHIP;                             \
    }                                             \
  } while (0)

inline hipError_t& last_hip_error() {
  static thread_local hipError_t e = hipSuccess;
  return e;
}

constexpr int REGION_CAP = 1024;
constexpr int WHOLE_CAP_S = 2048;
constexpr int WHOLE_CAP_L = 8192;
constexpr int SMALL_CAP_S = 2048;  // LDS-resident sweeps of whole small graphs
constexpr int SMALL_CAP_L = 8192;
// contractions of graphs with at least this many entries count the entries
// of rows outside the reference blocks, to choose the row-wise emit
constexpr int64_t ROWWISE_MIN_NNZ = 1 << 22;
constexpr int LDS_PER_CU = 160 * 1024;
constexpr int64_t SWEEP_HANDOFF_ENTRIES = 1 << 16;  // batches with longer rows run grid-wide
constexpr int32_t MAX_SWEEPS = 256;                 // full-graph sweeps run at once

// ------------------------------------------------------------------ timing
struct TimingClass {
  std::string name;
  int64_t launches = 0;
  double ms = 0;
  double bytes = 0;
};

struct Timer {
  bool on = false;
  hipStream_t s = nullptr;
  std::string focus;  // if set, only this class is timed (mc_timing_focus)
  std::vector<TimingClass> classes;
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;

  int cls(const char* name) {
    for (size_t i = 0; i < classes.size(); ++i)
      if (classes[i].name == name) return (int)i;
    classes.push_back(TimingClass{name});
    return (int)classes.size() - 1;
  }
  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
  }
  bool wants(const char* name) const { return on && (focus.empty() || focus == name); }
  // begin/end bracket a launch (or a short sequence) of one class
  int begin(const char* name, hipEvent_t& a) {
    if (!wants(name)) return -1;
    a = ev();
    hipEventRecord(a, s);
    return cls(name);
  }
  void end(int c, hipEvent_t a, double bytes) {
    if (c < 0) return;
    hipEvent_t b = ev();
    hipEventRecord(b, s);
    pending.push_back({c, a, b, bytes});
    if (pending.size() >= 16384) collect();  // bound the events held between reads
  }
  // bytes known only after a class's launches have run
  void add_bytes(const char* name, double bytes) {
    if (!wants(name)) return;
    pending_bytes.push_back({cls(name), bytes});
  }
  std::vector<std::pair<int, double>> pending_bytes;
  void collect() {
    for (auto& pb : pending_bytes) classes[pb.first].bytes += pb.second;
    pending_bytes.clear();
    for (auto& p : pending) {
      float ms = 0;
      hipEventSynchronize(p.b);
      hipEventElapsedTime(&ms, p.a, p.b);
      classes[p.cls].launches += 1;
      classes[p.cls].ms += ms;
      classes[p.cls].bytes += p.bytes;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
};

// One timer per host thread: concurrent solves (the server's lanes) never
// share one, and mc_timing_get reports the calling thread's.
Timer& timer() {
  static thread_local Timer t;
  return t;
}

struct TimedScope {
  int c;
  hipEvent_t a{};
  double bytes;
  TimedScope(const char* name, double b) : bytes(b) { c = timer().begin(name, a); }
  ~TimedScope() { timer().end(c, a, bytes); }
};

// --------------------------------------------------------------- workspace
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Workspace {
  int device = -1;
  int64_t capN = 0, capE = 0, capG = 0;
  // device arrays, carved from one block: the library's own (block != null)
  // or the caller's (opt->workspace)
  void* block = nullptr;
  // vertex arrays
  int32_t *gid[2], *parent, *lab, *claim, *step, *vcount, *capq, *capx, *sw_seg, *newid,
      *map, *ogid;
  SweepCtl* sweep;                  // sweep_slots queues
  int32_t sweep_slots = 0;          // full-graph sweeps run at once (at most MAX_SWEEPS)
  SweepArgs* sw_args;               // per swept graph
  int32_t* sw_run;                  // graphs still running
  SweepStatus* sw_status;
  int64_t* sw_info;
  int64_t *rp, *cdeg;
  uint64_t* fb_rs;  // sweeps: per vertex (r, visit stamp)
  // entry arrays
  int32_t *src, *col, *w;
  int32_t* first;  // the row of every WCH-th entry of the graph being read (k_chunk_rows)
  int32_t* chmax;  // the largest weight of every WCH-entry chunk of the ingested graph
  uint64_t *keys, *keys_alt;
  int32_t *vals, *vals_alt;
  // graph arrays
  int64_t *voff, *lhat, *wsum, *kcap;
  int32_t *gn, *cvoff, *nnew, *active, *ucount, *rec_type, *rec_id, *rec_k, *fb_k, *whole, *gmaxw, *prok,
      *whole2, *fb_list, *root0, *flip, *nvoff, *npairs, *bref;
  uint32_t *inref, *st2;
  uint64_t *bdeg, *balpha;
  uint8_t* mode;
  int32_t* scan_k;
  int64_t scan_k_cap = 0;
  void* tmp;
  size_t tmp_bytes = 0;
  Ctl* ctl;
  // pinned host staging for small read-backs (owned unless borrowed from
  // the stream's own workspace for a call on the caller's memory)
  bool host_owned = true;
  Ctl* ctl_host = nullptr;
  SweepCtl* sweep_host = nullptr;   // single-field readbacks
  SweepArgs* sw_args_host = nullptr;
  int32_t* sw_run_host = nullptr;
  SweepStatus* sw_status_host = nullptr;
  // clustering levels (on first use; after the core arrays in the caller's
  // block): two level graphs that the contractions alternate between,
  // labels, class flags, the long-row list, the map from input vertices to
  // level vertices, per-graph state
  struct Vc {
    int64_t capN = 0, capE = 0, capG = 0;
    void* block = nullptr;
    int32_t *src[2], *col[2], *w[2], *gid[2], *label[2], *map, *flag, *item_off, *act, *n0;
    int64_t *rp[2], *cdeg[2];
    uint64_t* best;
  } vc;

  void release_vc() {
    if (vc.block) hipFree(vc.block);
    vc = Vc{};
  }

  void release_device() {
    release_vc();
    if (block) hipFree(block);
    block = nullptr;
    capN = capE = capG = 0;
  }

  void release() {
    release_device();
    if (host_owned) {
      if (ctl_host) hipHostFree(ctl_host);
      if (sweep_host) hipHostFree(sweep_host);
      if (sw_args_host) hipHostFree(sw_args_host);
      if (sw_run_host) hipHostFree(sw_run_host);
      if (sw_status_host) hipHostFree(sw_status_host);
    }
    ctl_host = nullptr;
    sweep_host = nullptr;
    sw_args_host = nullptr;
    sw_run_host = nullptr;
    sw_status_host = nullptr;
    device = -1;
  }

  int ensure_host() {
    if (ctl_host) return MC_OK;
    if (hipHostMalloc((void**)&ctl_host, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sweep_host, sizeof(SweepCtl), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sw_args_host, sizeof(SweepArgs) * MAX_SWEEPS, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sw_run_host, sizeof(int32_t) * MAX_SWEEPS, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sw_status_host, sizeof(SweepStatus) * MAX_SWEEPS, hipHostMallocDefault) !=
            hipSuccess) {
      release();
      return MC_ENOMEM;
    }
    host_owned = true;
    return MC_OK;
  }
};

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// The sizes a problem of N vertices, E entries and G graphs is laid out for.
static void clamp_sizes(int64_t& N, int64_t& E, int64_t& G) {
  N = std::max<int64_t>(N, 16);
  E = std::max<int64_t>(E, 64);
  G = std::max<int64_t>(G, 1);
}

// Lay the core arrays out from `base` (or only measure, base == nullptr):
// returns the bytes they take, every array 256-byte aligned.
size_t carve(Workspace& ws, char* base, int64_t N, int64_t E, int64_t G) {
  size_t off = 0;
  auto take = [&](auto& ptr, size_t bytes) {
    using P = std::remove_reference_t<decltype(ptr)>;
    if (base) ptr = reinterpret_cast<P>(base + off);
    off += align_up(bytes);
  };
  take(ws.gid[0], (N + 1) * 4);
  take(ws.gid[1], (N + 1) * 4);
  take(ws.parent, (N + 1) * 4);
  take(ws.lab, (N + 1) * 4);
  take(ws.claim, (N + 1) * 4);
  take(ws.step, (N + 1) * 4);
  take(ws.vcount, (N + 1) * 4);
  take(ws.fb_rs, (N + 1) * 8);
  take(ws.newid, (N + 1) * 4);
  take(ws.map, (N + 1) * 4);
  take(ws.ogid, (N + 1) * 4);
  take(ws.capq, (N + 1) * 4);
  take(ws.capx, (N + 1) * 4);
  take(ws.sw_seg, (N + 1) * 4);
  const int64_t slots = std::min<int64_t>(G, MAX_SWEEPS);  // no more graphs than these are swept at once
  if (base) ws.sweep_slots = (int32_t)slots;
  take(ws.sweep, sizeof(SweepCtl) * slots);
  take(ws.sw_args, sizeof(SweepArgs) * slots);
  take(ws.sw_run, sizeof(int32_t) * slots);
  take(ws.sw_status, sizeof(SweepStatus) * slots);
  take(ws.sw_info, (G + 1) * 5 * 8);
  take(ws.rp, (N + 2) * 8);
  take(ws.cdeg, (N + 2) * 8);
  take(ws.src, E * 4);
  take(ws.first, (E / WCH + 2) * 4);
  take(ws.chmax, (E / WCH + 2) * 4);
  take(ws.col, E * 4);
  take(ws.w, E * 4);
  take(ws.keys, (E + 64) * 8);
  take(ws.keys_alt, (E + G + 64) * 8);  // also the sweeps' bucket pools (one entry per relaxation)
  take(ws.vals, E * 4);
  take(ws.vals_alt, E * 4);
  take(ws.voff, (G + 1) * 8);
  take(ws.lhat, (G + 1) * 8);
  take(ws.kcap, (G + 1) * 8);
  take(ws.wsum, (G + 1) * 8);
  take(ws.gn, (G + 1) * 4);
  take(ws.cvoff, (G + 1) * 4);
  take(ws.nnew, (G + 1) * 4);
  take(ws.active, (G + 1) * 4);
  take(ws.ucount, (G + 1) * 4);
  take(ws.rec_type, (G + 1) * 4);
  take(ws.rec_id, (G + 1) * 4);
  take(ws.rec_k, (G + 1) * 4);
  take(ws.fb_k, (G + 1) * 4);
  take(ws.whole, (G + 1) * 4);
  take(ws.whole2, (G + 1) * 4);
  take(ws.fb_list, (G + 1) * 4);
  take(ws.root0, (G + 1) * 4);
  take(ws.flip, (G + 1) * 4);
  take(ws.nvoff, (G + 1) * 4);
  take(ws.bref, (G + 1) * 4);
  take(ws.inref, ((N + 63) / 64 + 1) * 8);
  take(ws.st2, ((N + 63) / 64 + 1) * 16);  // two bits per vertex, whole 64-vertex groups
  take(ws.npairs, (G + 1) * 4);
  take(ws.gmaxw, (G + 1) * 4);
  take(ws.prok, (G + 1) * 4);
  take(ws.bdeg, (G + 1) * 8);
  take(ws.balpha, (G + 1) * 8);
  take(ws.mode, G + 1);
  if (base) ws.scan_k_cap = 2 * N + G + 64;
  take(ws.scan_k, (2 * N + G + 64) * 4);
  size_t t = std::max(scan_tmp_bytes<int64_t>(E + 1), radix_tmp_bytes(E + 1));
  t = std::max(t, scan_tmp_bytes<int32_t>(N + 1));
  if (base) ws.tmp_bytes = t;
  take(ws.tmp, t);
  take(ws.ctl, sizeof(Ctl));
  return off;
}

size_t carve_vc(Workspace::Vc& v, char* base, int64_t N, int64_t E, int64_t G) {
  size_t off = 0;
  auto take = [&](auto& ptr, size_t bytes) {
    using P = std::remove_reference_t<decltype(ptr)>;
    if (base) ptr = reinterpret_cast<P>(base + off);
    off += align_up(bytes);
  };
  for (int k = 0; k < 2; ++k) {
    take(v.src[k], E * 4);
    take(v.col[k], E * 4);
    take(v.w[k], E * 4);
    take(v.gid[k], (N + 1) * 4);
    take(v.label[k], (N + 1) * 4);
    take(v.rp[k], (N + 2) * 8);
    take(v.cdeg[k], (N + 2) * 8);
  }
  take(v.map, (N + 1) * 4);
  take(v.flag, (N + 1) * 4);
  take(v.item_off, (N + 1) * 4);
  take(v.best, (N + 1) * 8);
  take(v.act, (G + 1) * 4);
  take(v.n0, (G + 1) * 4);
  return off;
}

size_t workspace_bytes(int64_t N, int64_t E, int64_t G) {
  clamp_sizes(N, E, G);
  Workspace dummy;
  return carve(dummy, nullptr, N, E, G);
}

size_t vc_workspace_bytes(int64_t N, int64_t E, int64_t G) {
  clamp_sizes(N, E, G);
  Workspace::Vc dummy;
  return carve_vc(dummy, nullptr, N, E, G);
}

// The core arrays for a problem of this size in the library's own block,
// grown (with a quarter of headroom, so a caller whose sizes vary settles
// after a few reallocations) when the problem no longer fits.
int ensure(Workspace& ws, int64_t N, int64_t E, int64_t G) {
  int dev = 0;
  MC_HIP(hipGetDevice(&dev));
  int rc = ws.ensure_host();
  if (rc) return rc;
  if (ws.device == dev && ws.block && N <= ws.capN && E <= ws.capE && G <= ws.capG) return MC_OK;
  if (ws.device == dev && ws.capN > 0) {
    N = std::max(N, ws.capN + ws.capN / 4);
    E = std::max(E, ws.capE + ws.capE / 4);
    G = std::max(G, ws.capG + ws.capG / 4);
  }
  ws.release_device();
  clamp_sizes(N, E, G);
  const size_t bytes = carve(ws, nullptr, N, E, G);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return MC_ENOMEM;
  ws.block = p;
  ws.device = dev;
  carve(ws, (char*)p, N, E, G);
  ws.capN = N;
  ws.capE = E;
  ws.capG = G;
  return MC_OK;
}

// The core arrays in the caller's block (no allocation; MC_EINVAL if it is
// smaller than workspace_bytes).  The clustering arrays follow them there.
int carve_caller(Workspace& ws, void* base, size_t bytes, int64_t N, int64_t E, int64_t G) {
  int dev = 0;
  MC_HIP(hipGetDevice(&dev));
  clamp_sizes(N, E, G);
  const size_t need = carve(ws, nullptr, N, E, G);
  if (!base || bytes < need) return MC_EINVAL;
  carve(ws, (char*)base, N, E, G);
  ws.device = dev;
  ws.capN = N;
  ws.capE = E;
  ws.capG = G;
  ws.vc = Workspace::Vc{};
  return MC_OK;
}

struct CallerBlock {
  char* base = nullptr;   // the caller's workspace, or nullptr
  size_t bytes = 0;
  size_t core = 0;        // bytes the core arrays took
};

int ensure_vc(Workspace& ws, int64_t N, int64_t E, int64_t G, const CallerBlock& cb) {
  Workspace::Vc& v = ws.vc;
  clamp_sizes(N, E, G);
  if (cb.base) {
    const size_t need = carve_vc(v, nullptr, N, E, G);
    if (cb.bytes < cb.core + need) return MC_EINVAL;
    carve_vc(v, cb.base + cb.core, N, E, G);
    v.capN = N;
    v.capE = E;
    v.capG = G;
    return MC_OK;
  }
  if (v.block && N <= v.capN && E <= v.capE && G <= v.capG) return MC_OK;
  ws.release_vc();
  const size_t bytes = carve_vc(v, nullptr, N, E, G);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return MC_ENOMEM;
  v.block = p;
  carve_vc(v, (char*)p, N, E, G);
  v.capN = N;
  v.capE = E;
  v.capG = G;
  return MC_OK;
}

// One label-propagation sweep (L.cur -> L.nxt): short rows on the wave
// path, the passes of long rows as workgroup items, then their results.
// L.item_off must hold the items' prefix (lp_items_prefix) and L.best must
// be zero; the sweep leaves it zero.
void lp_items_prefix(const LpArgs& L, Workspace& ws, hipStream_t s) {
  exclusive_scan<int32_t, LpItems>(LpItems{L}, L.n, (int32_t*)L.item_off, &ws.ctl->lp_items, ws.tmp, s);
}

void lp_sweep(const LpArgs& L, int num_cu, hipStream_t s) {
  hipLaunchKernelGGL(k_lp_wave, dim3(grid_for((int64_t)L.n * 64, 64 * LP_WAVES, num_cu * 16)), dim3(64 * LP_WAVES),
                     0, s, L);
  hipLaunchKernelGGL(k_lp_items, dim3(num_cu * 4), dim3(LP_BLOCK_THREADS), 0, s, L);
  hipLaunchKernelGGL(k_lp_finish, dim3(grid_for(L.n, 256, num_cu * 16)), dim3(256), 0, s, L);
}

struct Problem {
  int32_t G;
  int32_t n;
  int64_t nnz;
  const int64_t* rp;
  const int32_t* col;
  const int32_t* w;
  const int64_t* voff_host;
};

static int bitlen(uint64_t x) { return x == 0 ? 0 : 64 - __builtin_clzll(x); }

// Range size (2^shift vertices) of the range-owned push relax: about
// 640 ranges, each within the LDS array of one workgroup.
static int seg_shift(int32_t ng) {
  const int64_t want = std::max<int64_t>(1, ((int64_t)ng + 639) / 640);
  return std::min(SEG_MAX_SHIFT, std::max(6, bitlen((uint64_t)want - 1)));
}

// The LDS sweep at a launch shape: threads per workgroup (128, 256, 512)
// and workgroups per compute unit (at most what the CU's 160 KiB of LDS
// holds).  The workgroups take graphs from a shared counter, so any shape
// gives the same sweeps.
template <int T, bool ORD>
static void launch_small_sweep_t(int groups, int num_cu, const SmallSweepArgs& SA, hipStream_t s) {
  constexpr int bytes = (int)sizeof(SmallSweepLds<SMALL_CAP_L, T, ORD>);
  const int fit = std::max(1, LDS_PER_CU / bytes);
  groups = std::max(1, std::min(groups > 0 ? groups : 3, fit));
  hipLaunchKernelGGL((k_small_sweep<SMALL_CAP_L, T, ORD>), dim3(num_cu * groups), dim3(T), bytes, s, SA);
}
// SA.order > 0: the kernels that follow a priority-queue order among equal keys
static void launch_small_sweep(int threads, int groups, int num_cu, const SmallSweepArgs& SA, hipStream_t s) {
  if (SA.order > 0) {
    if (threads == 128) launch_small_sweep_t<128, true>(groups, num_cu, SA, s);
    else if (threads == 512) launch_small_sweep_t<512, true>(groups, num_cu, SA, s);
    else launch_small_sweep_t<256, true>(groups, num_cu, SA, s);
    return;
  }
  if (threads == 128) launch_small_sweep_t<128, false>(groups, num_cu, SA, s);
  else if (threads == 512) launch_small_sweep_t<512, false>(groups, num_cu, SA, s);
  else launch_small_sweep_t<256, false>(groups, num_cu, SA, s);
}

// Opt a kernel into more than 64 KiB of dynamic LDS.
static hipError_t allow_lds(const void* fn, int bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// Workgroups of a kernel (threads per workgroup, no dynamic LDS) resident on
// the device at once.  Grid-stride kernels whose workgroups all get the same
// amount of work launch this many: a larger grid leaves a partial second
// wave of workgroups that starts only after the first has finished.
static int resident_grid(const void* kernel, int threads, int num_cu) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
    per_cu = 4;
  return per_cu * num_cu;
}

static bool debug_on() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("MC_DEBUG");
    v = (e && *e && *e != '0') ? 1 : 0;
  }
  return v == 1;
}

struct Solver {
  Workspace& ws;
  hipStream_t s;
  mc_options opt;
  int num_cu = 256;
  int32_t* debug_labels = nullptr;  // first round only: union-find roots
  int64_t* debug_lhat = nullptr;    // first round only: the bound used (host)
  const int64_t* lhat_in = nullptr; // optional starting bounds (host, per graph)
  bool viecut_only = false;         // stop after the clustering bound
  int32_t vc_levels_run = 0;        // clustering levels run (most over graphs)
  mc_stats* stats_out = nullptr;    // per-phase sweep counters (when wanted)
  CallerBlock cb;                   // the caller's workspace, if any
  int32_t ngraphs = 1;              // graphs in the problem being solved
  // ws.first is valid for the graph (rp, n, nnz) named here; a contraction
  // makes it stale
  const int64_t* first_rp = nullptr;
  int32_t first_n = -1;
  int64_t first_nnz = -1;
  // ws.src holds the sources of the loop's current graph (the ingest leaves
  // them unwritten; only some consumers index entries one at a time)
  bool src_ok = false;
  // ws.chmax holds the chunk maxima of the graph (rp, w, nnz) the ingest read
  const int64_t* chmax_rp = nullptr;
  const int32_t* chmax_w = nullptr;
  int64_t chmax_nnz = -1;

  // The row of every WCH-th entry of graph (n, nnz, rp) in ws.first.
  void need_first(int32_t n, int64_t nnz, const int64_t* rp) {
    if (first_rp == rp && first_n == n && first_nnz == nnz) return;
    if (nnz > 0) {
      // row_ptr read once, one int per WCH entries written
      TimedScope t("k_chunk_rows", (double)n * 8 + (double)(nnz / WCH) * 4);
      hipLaunchKernelGGL(k_chunk_rows, dim3(grid_for(n, 256, num_cu * 16)), dim3(256), 0, s, n, rp, ws.first);
    }
    first_rp = rp;
    first_n = n;
    first_nnz = nnz;
  }
  // Launch grid for one wave per WCH-entry chunk, at most `cap` workgroups.
  static dim3 chunk_grid(int64_t nnz, int cap) {
    return dim3(grid_for((nnz + WCH - 1) / WCH * 64, 256, cap));
  }
  // src[e] = the row of entry e of graph (n, nnz, rp).
  void fill_src(int32_t n, int64_t nnz, const int64_t* rp, int32_t* src) {
    if (nnz <= 0) return;
    need_first(n, nnz, rp);
    TimedScope t("k_fill_src", (double)nnz * 4 + (double)n * 8);
    hipLaunchKernelGGL(k_fill_src, chunk_grid(nnz, num_cu * 8), dim3(256), 0, s, n, nnz, rp, ws.first, src);
  }
  // PR1/PR2 on every entry of graph (n, nnz, rp, col, w).
  // The chunk maxima of graph (rp, w, nnz) if the ingest recorded them, else null.
  const int32_t* chunk_maxima(const int64_t* rp, const int32_t* w, int64_t nnz) const {
    return (chmax_rp == rp && chmax_w == w && chmax_nnz == nnz) ? ws.chmax : nullptr;
  }
  int pr_tests(int32_t n, int64_t nnz, const int64_t* rp, const int32_t* col, const int32_t* w,
               const int64_t* cdeg, const int32_t* gid, const int64_t* lhat, const int32_t* active) {
    if (nnz <= 0) return MC_OK;
    need_first(n, nnz, rp);
    // the ingested graph itself: its chunk maxima let the tests skip chunks
    // without reading them
    const int32_t* cm = chunk_maxima(rp, w, nnz);
    hipLaunchKernelGGL(k_pr, chunk_grid(nnz, num_cu * 16), dim3(256), 0, s, n, nnz, rp, ws.first, col, w, cm,
                       cdeg, gid, lhat, active, ws.parent, ws.ucount, ws.ctl);
    return MC_OK;
  }
  void need_src(int32_t n, int64_t nnz, const int64_t* rp) {
    if (src_ok) return;
    fill_src(n, nnz, rp, ws.src);
    src_ok = true;
  }

  int read_ctl() {
    MC_HIP(hipMemcpyAsync(ws.ctl_host, ws.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    MC_HIP(hipStreamSynchronize(s));
    return MC_OK;
  }

  void dump(const char* where, int32_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
            const int32_t* w) {
    if (!debug_on()) return;
    hipStreamSynchronize(s);
    int64_t lh = 0;
    uint64_t ba = 0, bd = 0;
    int32_t gn = 0;
    static int dg = -1;
    if (dg < 0) {
      const char* e = getenv("MC_DEBUG_G");
      dg = e ? atoi(e) : 0;
    }
    hipMemcpy(&lh, ws.lhat + dg, 8, hipMemcpyDeviceToHost);
    hipMemcpy(&ba, ws.balpha + dg, 8, hipMemcpyDeviceToHost);
    hipMemcpy(&bd, ws.bdeg + dg, 8, hipMemcpyDeviceToHost);
    hipMemcpy(&gn, ws.gn + dg, 4, hipMemcpyDeviceToHost);
    int32_t md = 0, act = 0, np = 0, uc = 0, cv = 0;
    hipMemcpy(&act, ws.active + dg, 4, hipMemcpyDeviceToHost);
    hipMemcpy(&np, ws.npairs + dg, 4, hipMemcpyDeviceToHost);
    hipMemcpy(&uc, ws.ucount + dg, 4, hipMemcpyDeviceToHost);
    hipMemcpy(&cv, ws.cvoff + dg, 4, hipMemcpyDeviceToHost);
    uint8_t mdb = 0;
    hipMemcpy(&mdb, ws.mode + dg, 1, hipMemcpyDeviceToHost);
    md = mdb;
    fprintf(stderr, "[mc] g=%d mode=%d active=%d npairs=%d ucount=%d cvoff=%d\n", dg, md, act, np, uc, cv);
    Ctl c;
    hipMemcpy(&c, ws.ctl, sizeof(Ctl), hipMemcpyDeviceToHost);
    fprintf(stderr, "[mc] %s n=%d nnz=%lld lhat0=%lld gn0=%d balpha=(%lld,%u) bdeg=(%lld,%u) "
            "pairs=%lld pr=%lld scans=%d pops=%lld emit=%lld unique=%lld n_next=%d\n",
            where, n, (long long)nnz, (long long)lh, gn, (long long)(ba >> 32), (unsigned)ba,
            (long long)(bd >> 32), (unsigned)bd, (long long)c.pairs, (long long)c.unions_pr,
            c.scan_ids, (long long)c.pops, (long long)c.emit, (long long)c.unique, c.n_next);
    if (n <= 16 && nnz <= 256) {
      std::vector<int64_t> hr(n + 1), cd(n);
      std::vector<int32_t> hc(nnz), hw(nnz);
      hipMemcpy(hr.data(), rp, (n + 1) * 8, hipMemcpyDeviceToHost);
      hipMemcpy(hc.data(), col, nnz * 4, hipMemcpyDeviceToHost);
      hipMemcpy(hw.data(), w, nnz * 4, hipMemcpyDeviceToHost);
      hipMemcpy(cd.data(), ws.cdeg, n * 8, hipMemcpyDeviceToHost);
      for (int v = 0; v < n; ++v) {
        fprintf(stderr, "   v%d cdeg=%lld:", v, (long long)cd[v]);
        for (int64_t e = hr[v]; e < hr[v + 1]; ++e) fprintf(stderr, " %d/%d", hc[e], hw[e]);
        fprintf(stderr, "\n");
      }
    }
  }

  // Full-graph capped sweeps of the listed graphs, all at once: the
  // sequential kernel runs one workgroup per graph, each with its own queue
  // (SweepCtl), FIFO range [v0, v0 + ng) and pool range (the graph's entry
  // range shifted by the graph id, one slot longer for the seed entry; entry
  // ranges are ordered by graph id, so the pools are disjoint).  Between
  // launches the host runs the pending grid-wide batches
  // of every graph that handed one back.  info: per graph (first vertex,
  // vertex count, bound, first entry, end entry).
  int sweep_graphs(const std::vector<int32_t>& glist, const std::vector<int64_t>& info, int round,
                   const int64_t* rp, const int32_t* col, const int32_t* w, const GraphState& S) {
    const int TB = 256;
    const int32_t total = (int32_t)glist.size();
    std::vector<int32_t> run, next;
    for (int32_t c0 = 0; c0 < total; c0 += ws.sweep_slots) {
      const int32_t kq = std::min<int32_t>(ws.sweep_slots, total - c0);
      int32_t k = 0;
      int64_t max_ng = 0, entries = 0;
      for (int32_t i = 0; i < kq; ++i) {
        const int32_t q = c0 + i;
        const int32_t v0 = (int32_t)info[5 * q], ng = (int32_t)info[5 * q + 1];
        const int64_t lam = info[5 * q + 2], e0 = info[5 * q + 3], e1 = info[5 * q + 4];
        if (lam <= 0 || ng < 2) continue;
        SweepArgs A{rp, col, w, ws.cdeg, ws.parent, ws.fb_rs, ws.capq + v0, ws.capx + v0,
                    (int2*)ws.keys_alt + e0 + glist[q], e1 - e0 + 1, ws.sw_seg + v0, ws.sweep + k, v0, ng, lam,
                    0, 1, 1, 0};
        const int lb = bitlen((uint64_t)(lam - 1));
        A.shift = lb > 12 ? lb - 12 : 0;
        A.nb = (int32_t)(((lam - 1) >> A.shift) + 1);
        A.nwords = (A.nb + 63) / 64;
        A.big = opt.sweep_handoff > 0 ? opt.sweep_handoff : 512;
        A.big_entries = SWEEP_HANDOFF_ENTRIES;
        // the tail: concurrent scans once at most a quarter of the graph (at
        // most 2^18 vertices: the pops of a process fit 20 bits) and at
        // least tail_min vertices are left
        A.tail_min = opt.sweep_tail < 0 ? 0 : opt.sweep_tail > 0 ? opt.sweep_tail : 256;
        A.tail_max = std::min(ng / 4, 1 << 18);
        uint64_t h = (opt.seed ? opt.seed : 0x5EEDull) * 0x9E3779B97F4A7C15ull +
                     (uint64_t)round * 0xBF58476D1CE4E5B9ull + (uint64_t)glist[q];
        h ^= h >> 29;
        A.start = v0 + (int32_t)(h % (uint64_t)ng);
        A.g = glist[q];
        ws.sw_args_host[k++] = A;
        max_ng = std::max<int64_t>(max_ng, ng);
        entries += e1 - e0;
      }
      if (k == 0) continue;
      MC_HIP(hipMemcpyAsync(ws.sw_args, ws.sw_args_host, sizeof(SweepArgs) * k, hipMemcpyHostToDevice, s));
      const int gx = std::max(1, std::min(grid_for(std::max<int64_t>(max_ng, SWEEP_BUCKETS), TB, num_cu * 16),
                                          (num_cu * 16 + k - 1) / k));
      hipLaunchKernelGGL(k_sweep_init, dim3(gx, k), dim3(TB), 0, s, ws.sw_args);
      hipLaunchKernelGGL(k_sweep_seed, dim3(grid_for(k, TB, num_cu)), dim3(TB), 0, s, ws.sw_args, k);
      run.resize(k);
      for (int32_t i = 0; i < k; ++i) run[i] = i;
      double big_deg = 0, big_vtx = 0;
      std::vector<int32_t> run_on_device;  // the run list last copied to ws.sw_run
      while (!run.empty()) {
        const int32_t nrun = (int32_t)run.size();
        if (run != run_on_device) {
          std::memcpy(ws.sw_run_host, run.data(), sizeof(int32_t) * nrun);
          MC_HIP(hipMemcpyAsync(ws.sw_run, ws.sw_run_host, sizeof(int32_t) * nrun, hipMemcpyHostToDevice, s));
          run_on_device = run;
        }
        {
          TimedScope t("k_sweep_seq", 0.0);
          hipLaunchKernelGGL(k_sweep_seq, dim3(nrun), dim3(SWEEP_THREADS), 0, s, ws.sw_args, ws.sw_run);
        }
        {
          // per batch vertex its FIFO slot, degree, r word and stamp (the
          // bytes are added once the batches' sizes are read back).  The
          // batch's size is not known here: four workgroups per CU, each
          // thread with four vertices' loads in flight, cover the largest
          // batches in a few steps without dispatching empty waves for the
          // many small ones
          TimedScope t("k_sweep_big_mark", 0.0);
          hipLaunchKernelGGL(k_sweep_big_mark, dim3(std::max(1, num_cu * 4 / nrun), nrun), dim3(TB), 0, s,
                             ws.sw_args, ws.sw_run);
        }
        hipLaunchKernelGGL(k_sweep_status, dim3(grid_for(nrun, TB, num_cu)), dim3(TB), 0, s, ws.sw_args,
                           ws.sw_run, nrun, ws.sw_status);
        MC_HIP(hipMemcpyAsync(ws.sw_status_host, ws.sw_status, sizeof(SweepStatus) * nrun, hipMemcpyDeviceToHost,
                              s));
        MC_HIP(hipStreamSynchronize(s));
        next.clear();
        for (int32_t j = 0; j < nrun; ++j) {
          const SweepStatus c = ws.sw_status_host[j];
          if (c.count_err) return MC_EINTERNAL;
          if (c.status == SW_DONE) continue;
          if (c.status != SW_BIG && c.status != SW_TAIL) return MC_EINTERNAL;
          const SweepArgs& A = ws.sw_args_host[run[j]];
          if (c.status == SW_TAIL) {
            // the tail as concurrent scans over the exact frontier list
            {
              TimedScope t("sweep_rebuild", (double)A.ng * 16);
              hipLaunchKernelGGL(k_sweep_rb_zero, dim3(16), dim3(256), 0, s, A);
              hipLaunchKernelGGL(k_sweep_rb_count, dim3(grid_for(A.ng, TB, num_cu * 4)), dim3(TB), 0, s, A);
              hipLaunchKernelGGL(k_sweep_rb_scan, dim3(1), dim3(1024), 0, s, A);
              hipLaunchKernelGGL(k_sweep_rb_fill, dim3((A.ng + RB_TILE - 1) / RB_TILE), dim3(TB), 0, s, A);
            }
            const int32_t left = A.ng - c.visited;
            int32_t nf = std::min<int32_t>(TAIL_MAX_FORKS, std::max<int32_t>(64, left / 8));
            nf = (nf + TAIL_WAVES - 1) / TAIL_WAVES * TAIL_WAVES;
            hipLaunchKernelGGL(k_sweep_tail_init, dim3(1), dim3(64), 0, s, A);
            TimedScope t("k_sweep_tail", 0.0);
            hipLaunchKernelGGL(k_sweep_tail, dim3(nf / TAIL_WAVES), dim3(64 * TAIL_WAVES), 0, s, A, nf);
            continue;  // the graph's sweep ends with its tail
          }
          const int32_t bh = c.cap_head, bt = c.cap_tail;
          const int64_t bsz = bt - bh;
          timer().add_bytes("k_sweep_big_mark", (double)bsz * 32);
          big_vtx += (double)bsz;
          // push or pull: the batch's rows (summed by the mark) against the
          // rows of the vertices still free (neither visited nor in the batch)
          const int64_t deg_sum = c.batch_deg;
          const int64_t free_rows = (A.pool_cap - 1) - c.rows_done - deg_sum;
          const bool pull = opt.sweep_pull >= 0 && (opt.sweep_pull > 0 || deg_sum > free_rows + A.ng / 8);
          big_deg += (double)deg_sum;
          if (debug_on())
            fprintf(stderr, "[mc] grid-wide batch g=%d size=%lld rows=%lld free_rows=%lld visited_before=%d ng=%d %s\n",
                    A.g, (long long)bsz, (long long)deg_sum, (long long)free_rows, c.visited, A.ng,
                    pull ? "pull" : "push");
          // prefix sums of row lengths (ws.keys and ws.vals are free until
          // the contraction) and each entry tile's first row
          int64_t* off = (int64_t*)ws.keys;
          int32_t* tile_row = ws.vals;
          if (!pull) {
            {
              // per batch vertex its FIFO slot and row bounds, the prefix sum
              // written; then the graph's visit state read once, two bits written
              TimedScope t("sweep_batch_prep", (double)bsz * 28 + (double)A.ng * 8);
              exclusive_scan<int64_t, BatchDeg>(BatchDeg{A.capq + bh, rp}, bsz, off, off + bsz, ws.tmp, s);
              hipLaunchKernelGGL(k_sweep_big_tiles, dim3(grid_for(bsz, TB, num_cu * 16)), dim3(TB), 0, s, off,
                                 (int32_t)bsz, tile_row);
              // the graph's visit states, two bits per vertex
              hipLaunchKernelGGL(k_sweep_bits, dim3(grid_for(A.ng, TB, num_cu * 4)), dim3(TB), 0, s, A, ws.st2);
            }
            // range by range (segments of at least four entries on average,
            // and no batch row of this sweep found out of order so far): the
            // segment table in ws.vals_alt
            const int shift = seg_shift(A.ng);
            const int64_t nr = ((int64_t)A.ng + (1 << shift) - 1) >> shift;
            const int64_t cells = bsz * (nr + 1);
            const bool seg = opt.sweep_seg >= 0 && c.seg_unsorted == 0 && cells <= ws.capE &&
                             (opt.sweep_seg > 0 || cells * 4 <= deg_sum);
            if (seg) {
              {
                // every batch entry's column (and its predecessor's, cached)
                // read, every cell of the table written once
                TimedScope t("k_sweep_seg_bounds", (double)deg_sum * 4 + (double)cells * 4 + (double)bsz * 16);
                static const int bounds_grid = resident_grid((const void*)&k_sweep_seg_bounds, TB, num_cu);
                hipLaunchKernelGGL(k_sweep_seg_bounds, dim3(bounds_grid), dim3(TB), 0, s, A, bh, (int32_t)bsz, off,
                                   tile_row, shift, (int32_t)nr, ws.vals_alt);
              }
              {
                // every batch entry once (col, w), two cells per row and
                // range, and per vertex its word read and r written
                TimedScope t("k_sweep_seg_relax", (double)deg_sum * 8 + (double)cells * 8 + (double)A.ng * 12);
                hipLaunchKernelGGL(k_sweep_seg_relax, dim3((uint32_t)((nr + NUM_XCD - 1) / NUM_XCD * NUM_XCD)),
                                   dim3(SEG_THREADS), 0, s, A, bh,
                                   (int32_t)bsz, (const int64_t*)off, shift, (int32_t)nr,
                                   (const int32_t*)ws.vals_alt, (const uint32_t*)ws.st2);
              }
              {
                // the global form, which returns at once unless the bounds
                // found a row out of order
                TimedScope t("k_sweep_seg_fallback", 0.0);
                static const int relax_grid = resident_grid((const void*)&k_sweep_big_relax, TB, num_cu);
                hipLaunchKernelGGL(k_sweep_big_relax, dim3(relax_grid), dim3(TB), 0, s, A, bh, (int32_t)bsz, off,
                                   tile_row, ws.st2, 1);
              }
            } else {
              // every row of the batch once (col, w: 8 B per entry) and per
              // batch vertex its row bounds
              TimedScope t("k_sweep_big_relax", (double)deg_sum * 8 + (double)bsz * 8);
              static const int relax_grid = resident_grid((const void*)&k_sweep_big_relax, TB, num_cu);
              hipLaunchKernelGGL(k_sweep_big_relax, dim3(relax_grid), dim3(TB), 0, s, A, bh, (int32_t)bsz, off,
                                 tile_row, ws.st2, 0);
            }
          } else {
            // the free vertices (a list in ws.lab, free until the
            // compaction) and their rows' prefix sums
            int32_t* list = ws.lab;
            // the free vertices: neither visited nor in the batch
            const int32_t nfree = (int32_t)std::max<int64_t>(0, (int64_t)A.ng - c.visited - bsz);
            {
              TimedScope t("sweep_batch_prep", (double)A.ng * 16);
              hipLaunchKernelGGL(k_sweep_free_bits, dim3((A.ng + FREE_TILE - 1) / FREE_TILE), dim3(TB), 0, s, A,
                                 ws.st2, list);
              hipLaunchKernelGGL(k_sweep_free_check, dim3(1), dim3(256), 0, s, A, nfree, list);
              exclusive_scan<int64_t, BatchDeg>(BatchDeg{list, rp}, nfree, off, off + nfree, ws.tmp, s);
              hipLaunchKernelGGL(k_sweep_big_tiles, dim3(grid_for(std::max(nfree, 1), TB, num_cu * 16)), dim3(TB), 0,
                                 s, off, nfree, tile_row);
            }
            // every free row once (col, w: 8 B per entry) and per free vertex
            // its row bounds and r
            TimedScope t("k_sweep_big_pull", (double)free_rows * 8 + (double)nfree * 16);
            if (nfree > 0) {
              static const int pull_grid = resident_grid((const void*)&k_sweep_big_pull, TB, num_cu);
              hipLaunchKernelGGL(k_sweep_big_pull, dim3(pull_grid), dim3(TB), 0, s, A, (const int32_t*)list, nfree,
                                 (const int64_t*)off, (const int32_t*)tile_row, (const uint32_t*)ws.st2);
            }
          }
          hipLaunchKernelGGL(k_sweep_big_finish, dim3(1), dim3(256), 0, s, A, bt, pull ? 1 : 0);
          {
            // exact queue rebuild: two passes over the graph's vertices (the
            // finish kernel cleared the bucket counts)
            TimedScope t("sweep_rebuild", (double)A.ng * 16);
            hipLaunchKernelGGL(k_sweep_rb_count, dim3(grid_for(A.ng, TB, num_cu * 4)), dim3(TB), 0, s, A);
            hipLaunchKernelGGL(k_sweep_rb_scan, dim3(1), dim3(1024), 0, s, A);
            hipLaunchKernelGGL(k_sweep_rb_fill, dim3((A.ng + RB_TILE - 1) / RB_TILE), dim3(TB), 0, s, A);
          }
          next.push_back(run[j]);
        }
        run.swap(next);
      }
      // the sequential kernel relaxed every row the grid-wide batches did
      // not (8 B per entry) and visited every other vertex (row bounds,
      // degree, r and stamp, the claim and its union: 40 B per vertex)
      // (timing mode only, which synchronises anyway: the counters are
      // read back per graph, with the per-phase step counts for the stats)
      double crossings = 0;
      if (timer().wants("k_sweep_seq") || timer().wants("k_sweep_tail") || timer().wants("k_sweep_unite")) {
        double visited = 0, seq_rows = 0, tail_rows = 0, tail_pops = 0;
        for (int32_t i = 0; i < k; ++i) {
          SweepCtl c;
          MC_HIP(hipMemcpyAsync(&c, ws.sw_args_host[i].ctl, offsetof(SweepCtl, bitmap), hipMemcpyDeviceToHost, s));
          MC_HIP(hipStreamSynchronize(s));
          visited += c.visited;
          seq_rows += (double)c.seq_rows;
          tail_rows += (double)c.tail_rows;
          tail_pops += c.tail_pops;
          crossings += std::min(c.cap_tail, ws.sw_args_host[i].ng);
          if (stats_out) {
            stats_out->sweep_phases = std::max(stats_out->sweep_phases, std::min(c.big_batches + 1, SWEEP_PHASES));
            stats_out->sweep_big_batches += c.big_batches;
            for (int p = 0; p < SWEEP_PHASES; ++p) {
              stats_out->sweep_singles[p] += c.ph_singles[p];
              stats_out->sweep_batches[p] += c.ph_batches[p];
              stats_out->sweep_cross[p] += c.ph_cross[p];
            }
          }
        }
        timer().add_bytes("k_sweep_seq", seq_rows * 8 + (visited - big_vtx) * 40);
        timer().add_bytes("k_sweep_tail", tail_rows * 8 + tail_pops * 40);
        if (stats_out) {
          stats_out->sweep_tail_pops += (int64_t)tail_pops;
        }
      }
      {
        // one union (a parent word read and written) per crossing
        TimedScope t("k_sweep_unite", 0.0);
        hipLaunchKernelGGL(k_sweep_unite, dim3(gx, k), dim3(TB), 0, s, ws.sw_args);
      }
      if (timer().on) timer().add_bytes("k_sweep_unite", crossings * 8);
      hipLaunchKernelGGL(k_sweep_report, dim3(grid_for(k, TB, num_cu)), dim3(TB), 0, s, ws.sw_args, k, S);
      if (debug_on()) {
        MC_HIP(hipStreamSynchronize(s));
        for (int32_t i = 0; i < k; ++i) {
          SweepCtl c;
          MC_HIP(hipMemcpy(&c, ws.sw_args_host[i].ctl, offsetof(SweepCtl, bitmap), hipMemcpyDeviceToHost));
          fprintf(stderr, "[mc] sweep g=%d v0=%d ng=%d lam=%lld visited=%d singles=%d batches=%d big=%d "
                  "rebuilds=%d unions=%d best_alpha=%lld step=%d\n", ws.sw_args_host[i].g, ws.sw_args_host[i].v0,
                  ws.sw_args_host[i].ng, (long long)ws.sw_args_host[i].lam, c.visited, c.singles, c.batches,
                  c.big_batches, c.rebuilds, c.cap_tail, (long long)c.best_alpha, c.best_step);
        }
      }
    }
    return MC_OK;
  }

  // Opt-in check that the input is symmetric (the entry sources are in
  // ws.src): one sort of the entries keyed by unordered pair, with the two
  // directions' weights summed with opposite signs.  The contraction's
  // buffers are free until the first round.
  int check_symmetry(int32_t N, int64_t E, const int32_t* col, const int32_t* w) {
    const int TB = 256;
    const int bb = std::max(1, bitlen((uint64_t)N - 1));
    MC_HIP(hipMemsetAsync(&ws.ctl->emit, 0, sizeof(int64_t), s));
    hipLaunchKernelGGL(k_sym_emit, dim3(grid_for(E, TB, num_cu * 16)), dim3(TB), 0, s, E, ws.src, col, w, bb,
                       ws.keys, ws.vals, ws.ctl);
    int rc = read_ctl();
    if (rc) return rc;
    const int64_t m = ws.ctl_host->emit;
    if (m == 0) return MC_OK;
    const int which = radix_sort_pairs(ws.keys, ws.vals, ws.keys_alt, ws.vals_alt, m, 2 * bb, ws.tmp, s);
    uint64_t* sk = which ? ws.keys_alt : ws.keys;
    int32_t* sv = which ? ws.vals_alt : ws.vals;
    int32_t* spare = which ? ws.vals : ws.vals_alt;
    int64_t* pos = (int64_t*)(which ? ws.keys : ws.keys_alt);
    exclusive_scan<int64_t, HeadFlag>(HeadFlag{sk}, m, pos, (int64_t*)&ws.ctl->unique, ws.tmp, s);
    rc = read_ctl();
    if (rc) return rc;
    const int64_t m2 = ws.ctl_host->unique;
    fill<int32_t>(ws.w, 0, m2, s);
    hipLaunchKernelGGL(k_merge, dim3(grid_for((m + 255) / 256 * 256, TB, num_cu * 16)), dim3(TB), 0, s, m, sk, sv,
                       pos, bb, ws.col, spare, ws.w);
    hipLaunchKernelGGL(k_sym_nonzero, dim3(grid_for(m2, TB, num_cu * 4)), dim3(TB), 0, s, m2, ws.w, ws.ctl);
    rc = read_ctl();
    if (rc) return rc;
    return ws.ctl_host->asym ? MC_EINVAL : MC_OK;
  }

  // Timing class names of one contraction's stages.
  struct StageNames {
    const char *block_bits, *emit, *sort_hist, *sort_scatter, *merge_scan, *merge, *csr;
  };
  static constexpr StageNames kExactNames{"block_bits", "k_emit", "k_rs_hist", "k_rs_scatter",
                                          "merge_scan", "k_merge", "csr"};
  static constexpr StageNames kVcNames{"vc_contract", "vc_contract", "vc_contract", "vc_contract",
                                       "vc_contract", "vc_contract", "vc_contract"};
  struct Out {
    int32_t *src, *col, *w;
    int64_t *rp, *cdeg;
  };

  // Contract the graph given as CSR (rp_cur, col, w over nnz entries) by the
  // block of every vertex (lab in [0, n_next), -1 = dropped) into n_next
  // vertices (Preliminaries, contraction G/(u,v); section "Parallel Graph
  // Contraction"): emit a (lab u, lab v) key per crossing entry, radix-sort,
  // merge runs of equal keys, build row_ptr and the weighted degrees, and
  // fold each graph's minimum degree into ws.bdeg (cleared by the caller).
  // The entry inputs are consumed before the outputs are written, so `out`
  // may alias them.
  // n_cur, gid_cur: the graph being contracted (vertex count, graph ids).
  int contract(int64_t nnz, const int64_t* rp_cur, const int32_t* col, const int32_t* w, const int32_t* lab,
               int32_t n_cur, const int32_t* gid_cur, int32_t n_next, const int32_t* gid_next, Out out,
               int64_t* m2_out, const StageNames& nm) {
    const int TB = 256;
    auto grid = [&](int64_t n) { return dim3(grid_for(n, TB, num_cu * 16)); };
    auto gridr = [&](int64_t n) { return dim3(grid_for(n, TB, num_cu * 2)); };
    const int bb = std::max(1, bitlen((uint64_t)std::max(n_next, 1) - 1));
    MC_HIP(hipMemsetAsync(&ws.ctl->emit, 0, sizeof(int64_t), s));
    MC_HIP(hipMemsetAsync(&ws.ctl->nonref_nnz, 0, sizeof(int64_t), s));
    // on a large graph the entries of rows outside the reference blocks are
    // counted: when they are few, only those rows are read (k_emit_rows)
    const bool count_rows = nnz >= ROWWISE_MIN_NNZ;
    {
      // the labels read once, one bit written per vertex
      TimedScope t(nm.block_bits, (double)n_cur * (count_rows ? 24 : 8));
      hipLaunchKernelGGL(k_block_ref, dim3(grid_for((int64_t)ngraphs * 64, TB, num_cu * 8)), dim3(TB), 0, s,
                         ngraphs, n_cur, ws.cvoff, ws.gn, lab, ws.bref);
      hipLaunchKernelGGL(k_block_bits, dim3(grid_for(n_cur, TB, num_cu * 16)), dim3(TB), 0, s, n_cur, lab, gid_cur,
                         ws.bref, ws.inref, count_rows ? rp_cur : (const int64_t*)nullptr, ws.ctl);
    }
    bool rowwise = false;
    int64_t nonref = nnz;
    if (count_rows && opt.emit_rows >= 0) {
      int rc = read_ctl();
      if (rc) return rc;
      nonref = ws.ctl_host->nonref_nnz;
      rowwise = opt.emit_rows > 0 || nonref * 4 < nnz;
    } else if (opt.emit_rows > 0) {
      rowwise = true;
    }
    if (rowwise) {
      // per selected vertex its label, bit and row bounds (16 B), per entry
      // of its row col, w and the neighbour's label and bit (12 B); per
      // emitted entry its key and weight (added once the count is read back)
      TimedScope t(nm.emit, (double)n_cur * 8 + (double)nonref * 12);
      static const int rows_grid = resident_grid((const void*)&k_emit_rows, TB, num_cu);
      hipLaunchKernelGGL(k_emit_rows, dim3(grid_for((int64_t)(n_cur + 63) / 64 * 64, TB, rows_grid)), dim3(TB), 0,
                         s, n_cur, rp_cur, col, w, lab, bb, ws.inref, ws.keys, ws.vals, ws.ctl);
    } else {
      need_first(n_cur, nnz, rp_cur);
      // per entry col and w and the label gather (12 B); per emitted entry
      // its key and weight (12 B, added once the count is read back)
      TimedScope t(nm.emit, (double)nnz * 12);
      static const int emit_grid = resident_grid((const void*)&k_emit, TB, num_cu);
      if (nnz > 0)
        hipLaunchKernelGGL(k_emit, chunk_grid(nnz, emit_grid), dim3(TB), 0, s, n_cur, nnz, rp_cur, ws.first, col,
                           w, lab, bb, ws.inref, ws.keys, ws.vals, ws.ctl);
    }
    int rc = read_ctl();
    if (rc) return rc;
    const int64_t m = ws.ctl_host->emit;
    timer().add_bytes(nm.emit, (double)m * 12);
    int which = 0;
    {
      // per pass: the histogram reads every key (8 B); the scatter reads
      // and writes key and weight (24 B)
      int cur = -1;
      hipEvent_t ev0{};
      auto hook = [&](int kind, int) {
        if (kind == 0) cur = timer().begin(nm.sort_hist, ev0);
        else if (kind == 1) timer().end(cur, ev0, (double)m * 8);
        else if (kind == 2) cur = timer().begin(nm.sort_scatter, ev0);
        else timer().end(cur, ev0, (double)m * 24);
      };
      which = radix_sort_pairs(ws.keys, ws.vals, ws.keys_alt, ws.vals_alt, m, 2 * bb, ws.tmp, s, hook, opt.sort_tile);
    }
    uint64_t* sk = which ? ws.keys_alt : ws.keys;
    int32_t* sv = which ? ws.vals_alt : ws.vals;
    int64_t* pos = (int64_t*)(which ? ws.keys : ws.keys_alt);
    {
      TimedScope t(nm.merge_scan, (double)m * 16 + (double)m * 8);
      exclusive_scan<int64_t, HeadFlag>(HeadFlag{sk}, m, pos, (int64_t*)&ws.ctl->unique, ws.tmp, s);
    }
    rc = read_ctl();
    if (rc) return rc;
    const int64_t m2 = m > 0 ? ws.ctl_host->unique : 0;
    fill<int32_t>(out.w, 0, m2, s);
    {
      // sorted keys and weights in (12 B); the merged entries out (12 B)
      TimedScope t(nm.merge, (double)m * 12 + (double)m2 * 12);
      if (m > 0)
        hipLaunchKernelGGL(k_merge, dim3(grid_for((m + 255) / 256 * 256, TB, num_cu * 16)), dim3(TB), 0, s, m, sk,
                           sv, pos, bb, out.src, out.col, out.w);
    }
    {
      TimedScope t(nm.csr, (double)m2 * 12 + (double)n_next * 16);
      hipLaunchKernelGGL(k_rowptr, grid(n_next + 1), dim3(TB), 0, s, n_next, m2, out.src, out.rp);
      fill<int64_t>(out.cdeg, 0, n_next, s);
      if (m2 > 0)
        hipLaunchKernelGGL(k_degrees, dim3(grid_for((m2 + 255) / 256 * 256, TB, num_cu * 16)), dim3(TB), 0, s, m2,
                           out.src, out.w, out.cdeg);
      hipLaunchKernelGGL(k_min_degree, gridr(n_next), dim3(TB), 0, s, n_next, out.cdeg, gid_next,
                         (const int32_t*)nullptr, ws.bdeg, (int64_t*)nullptr);
    }
    *m2_out = m2;
    first_rp = nullptr;  // the graphs may have been written over
    chmax_rp = nullptr;
    return MC_OK;
  }

  // VieCut-style upper bound (section "Inexact Shared-Memory Minimum Cuts";
  // Algorithm 2 starts from it).  Per level: label-propagation sweeps,
  // contraction of the label classes, the minimum degree as a bound, the
  // Padberg-Rinaldi tests against the current bound, contraction of their
  // components, the minimum degree again.  Every vertex of a level graph is
  // a vertex set of the input, so each bound is a real cut; the side of a
  // new bound is written at once.  The input graph's entries, sources and
  // degrees are left as they are for the exact loop, and no union found
  // here enters it.
  // The last level graph, when the clustering bound is finished exactly.
  struct LevelGraph {
    int32_t n;
    int64_t nnz;
    const int64_t* rp;
    const int32_t *col, *w, *src, *gid;
    const int64_t* cdeg;
  };

  int viecut(const Problem& P, GraphState S, const int32_t* gid_in, uint8_t* side, LevelGraph* last = nullptr) {
    const int32_t G = P.G, N = P.n;
    int rc = ensure_vc(ws, N, P.nnz, G, cb);
    if (rc) return rc;
    Workspace::Vc& V = ws.vc;
    const int TB = 256;
    auto grid = [&](int64_t n) { return dim3(grid_for(n, TB, num_cu * 16)); };
    const int32_t stop = opt.viecut_stop > 0 ? opt.viecut_stop : 2;
    const int32_t max_levels = opt.viecut_levels > 0 ? opt.viecut_levels : 32;
    const int32_t sweeps = std::max(0, opt.lp_sweeps);
    // with the exact finish, graphs that stop keep their last level graph in
    // the level graphs that follow
    const int32_t carry = last != nullptr ? 1 : 0;
    MC_HIP(hipMemsetAsync(ws.ctl, 0, sizeof(Ctl), s));
    hipLaunchKernelGGL(k_vc_init, grid(G), dim3(TB), 0, s, G, S, stop, V.act, V.n0, ws.ctl);
    hipLaunchKernelGGL(k_iota, grid(N), dim3(TB), 0, s, V.map, N);
    rc = read_ctl();
    if (rc) return rc;
    int32_t n_act = ws.ctl_host->n_active;
    // the current level graph; the input first
    int32_t n = N;
    int64_t nnz = P.nnz;
    const int64_t* rp = P.rp;
    const int32_t* col = P.col;
    const int32_t* w = P.w;
    const int32_t* src = ws.src;
    const int64_t* cdeg = ws.cdeg;
    const int32_t* gid = gid_in;
    int next = 0;  // level-graph buffer the next contraction writes
    SideArgs sa{N, ws.ogid, V.map, ws.rec_type, ws.rec_id, ws.rec_k, ws.claim, ws.step,
                ws.fb_rs, ws.parent, ws.root0, side, REC_DEG};
    // contract the current graph by ws.lab (ws.nnew holds the new per-graph
    // counts), update the bounds and sides, and move to the new graph
    auto step = [&](int32_t n_next, int end_of_level, int last_level) -> int {
      fill<uint64_t>(ws.bdeg, ~0ull, G, s);
      int64_t m2 = 0;
      Out o{V.src[next], V.col[next], V.w[next], V.rp[next], V.cdeg[next]};
      int r = contract(nnz, rp, col, w, ws.lab, n, gid, n_next, V.gid[next], o, &m2, kVcNames);
      if (r) return r;
      exclusive_scan<int32_t, ArrayIn<int32_t>>(ArrayIn<int32_t>{ws.nnew}, G, ws.nvoff, (int32_t*)nullptr,
                                                ws.tmp, s);
      MC_HIP(hipMemsetAsync(&ws.ctl->n_active, 0, sizeof(int32_t), s));
      hipLaunchKernelGGL(k_vc_level, grid(G), dim3(TB), 0, s, G, S, ws.nvoff, stop, end_of_level, last_level,
                         carry, V.act, V.n0, ws.ctl);
      hipLaunchKernelGGL(k_compose_map, grid(N), dim3(TB), 0, s, N, V.map, ws.lab);
      if (side) {
        TimedScope t("k_side", (double)N * 13);
        hipLaunchKernelGGL(k_side, grid(N), dim3(TB), 0, s, sa);
      }
      r = read_ctl();
      if (r) return r;
      n_act = ws.ctl_host->n_active;
      n = n_next;
      nnz = m2;
      rp = V.rp[next];
      col = V.col[next];
      w = V.w[next];
      src = V.src[next];
      cdeg = V.cdeg[next];
      gid = V.gid[next];
      next ^= 1;
      return MC_OK;
    };
    int level = 0;
    for (; level < max_levels && n_act > 0; ++level) {
      const int last = level + 1 >= max_levels;
      // label propagation from distinct labels
      int32_t* cur = V.label[0];
      int32_t* nxt = V.label[1];
      {
        TimedScope t("vc_lp", (double)nnz * 12 * std::max(sweeps, 1) + (double)n * 24);
        hipLaunchKernelGGL(k_iota, grid(n), dim3(TB), 0, s, cur, n);
        fill<uint64_t>(V.best, 0, n, s);
        LpArgs L{n, rp, col, w, gid, V.act, cur, nxt, V.item_off, &ws.ctl->lp_items, V.best};
        if (sweeps > 0) lp_items_prefix(L, ws, s);
        for (int k = 0; k < sweeps; ++k) {
          L.cur = cur;
          L.nxt = nxt;
          lp_sweep(L, num_cu, s);
          std::swap(cur, nxt);
        }
        // classes numbered by label value
        fill<int32_t>(V.flag, 0, n, s);
        hipLaunchKernelGGL(k_lp_flag, grid(n), dim3(TB), 0, s, n, cur, gid, V.act, carry, V.flag);
        exclusive_scan<int32_t, ArrayIn<int32_t>>(ArrayIn<int32_t>{V.flag}, n, ws.newid, &ws.ctl->n_next,
                                                  ws.tmp, s);
        fill<int32_t>(ws.nnew, 0, G, s);
        hipLaunchKernelGGL(k_lp_relabel, grid(n), dim3(TB), 0, s, n, cur, gid, V.act, carry, V.flag, ws.newid,
                           ws.lab, V.gid[next], ws.nnew);
      }
      rc = read_ctl();
      if (rc) return rc;
      if (debug_on())
        fprintf(stderr, "[mc] viecut level %d: n=%d nnz=%lld long-row items=%d classes=%d active=%d\n", level, n,
                (long long)nnz, ws.ctl_host->lp_items, ws.ctl_host->n_next, n_act);
      rc = step(ws.ctl_host->n_next, 0, last);
      if (rc) return rc;
      if (n_act > 0) {
        // Padberg-Rinaldi tests on the level graph, components contracted
        {
          TimedScope t("vc_pr", (double)nnz * 20 + (double)n * 16);
          hipLaunchKernelGGL(k_iota, grid(n), dim3(TB), 0, s, ws.parent, n);
          hipLaunchKernelGGL(k_pr_sample, grid(n), dim3(TB), 0, s, n, nnz, rp, col, w, chunk_maxima(rp, w, nnz),
                             cdeg, gid, ws.lhat, V.act,
                             ws.parent, ws.ucount);
          hipLaunchKernelGGL(k_flatten, grid(n), dim3(TB), 0, s, n, ws.parent);
          hipLaunchKernelGGL(k_lam_floor, dim3(1), dim3(256), 0, s, G, ws.lhat, V.act, ws.ctl);
          const int prc = pr_tests(n, nnz, rp, col, w, cdeg, gid, ws.lhat, V.act);
          if (prc) return prc;
          hipLaunchKernelGGL(k_flatten, grid(n), dim3(TB), 0, s, n, ws.parent);
          exclusive_scan<int32_t, RootFlag>(RootFlag{ws.parent, gid, V.act, carry}, n, ws.newid, &ws.ctl->n_next,
                                            ws.tmp, s);
          fill<int32_t>(ws.nnew, 0, G, s);
          hipLaunchKernelGGL(k_relabel, grid(n), dim3(TB), 0, s, n, ws.parent, gid, V.act, carry, ws.newid,
                             ws.lab, V.gid[next], ws.nnew);
        }
        rc = read_ctl();
        if (rc) return rc;
        rc = step(ws.ctl_host->n_next, 1, last);
        if (rc) return rc;
      }
    }
    vc_levels_run = level;
    MC_HIP(hipMemsetAsync(&ws.ctl->n_active, 0, sizeof(int32_t), s));
    if (last) {
      // hand the last level graph to the exact loop: its map becomes the
      // loop's original -> current map
      hipLaunchKernelGGL(k_vc_exact_start, grid(G), dim3(TB), 0, s, G, S, ws.ctl);
      MC_HIP(hipMemcpyAsync(ws.map, V.map, (size_t)N * 4, hipMemcpyDeviceToDevice, s));
      *last = LevelGraph{n, nnz, rp, col, w, src, gid, cdeg};
      return MC_OK;
    }
    hipLaunchKernelGGL(k_vc_done, grid(G), dim3(TB), 0, s, G, S, ws.ctl);
    return MC_OK;
  }

  int solve(const Problem& P, int64_t* lambdas, uint8_t* side, mc_stats* st) {
    const int32_t G = P.G;
    ngraphs = G;
    const int32_t N = P.n;
    const int64_t E = P.nnz;
    const bool want_side = side != nullptr;
    int dev = 0;
    MC_HIP(hipGetDevice(&dev));
    MC_HIP(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    // kernels with more than 64 KiB of dynamic LDS, once per process
    static std::once_flag attrs_once;
    static hipError_t attrs_err = hipSuccess;
    std::call_once(attrs_once, [] {
      const std::pair<const void*, int> big[] = {
          {(const void*)k_capforest<WHOLE_CAP_L, false>, (int)sizeof(ScanLds<WHOLE_CAP_L, false>)},
          {(const void*)k_capforest<WHOLE_CAP_S, false>, (int)sizeof(ScanLds<WHOLE_CAP_S, false>)},
          {(const void*)k_capforest<WHOLE_CAP_L, true>, (int)sizeof(ScanLds<WHOLE_CAP_L, true>)},
          {(const void*)k_capforest<WHOLE_CAP_S, true>, (int)sizeof(ScanLds<WHOLE_CAP_S, true>)},
          {(const void*)k_small_sweep<SMALL_CAP_L, 128, false>, (int)sizeof(SmallSweepLds<SMALL_CAP_L, 128, false>)},
          {(const void*)k_small_sweep<SMALL_CAP_L, 256, false>, (int)sizeof(SmallSweepLds<SMALL_CAP_L, 256, false>)},
          {(const void*)k_small_sweep<SMALL_CAP_L, 512, false>, (int)sizeof(SmallSweepLds<SMALL_CAP_L, 512, false>)},
          {(const void*)k_small_sweep<SMALL_CAP_L, 128, true>, (int)sizeof(SmallSweepLds<SMALL_CAP_L, 128, true>)},
          {(const void*)k_small_sweep<SMALL_CAP_L, 256, true>, (int)sizeof(SmallSweepLds<SMALL_CAP_L, 256, true>)},
          {(const void*)k_small_sweep<SMALL_CAP_L, 512, true>, (int)sizeof(SmallSweepLds<SMALL_CAP_L, 512, true>)}};
      hipError_t e = hipSuccess;
      for (const auto& k : big)
        if (e == hipSuccess) e = allow_lds(k.first, k.second);
      attrs_err = e;
    });
    MC_HIP(attrs_err);

    MC_HIP(hipMemcpyAsync(ws.voff, P.voff_host, (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    MC_HIP(hipMemsetAsync(ws.ctl, 0, sizeof(Ctl), s));
    GraphState S{ws.voff, ws.lhat, ws.gn, ws.cvoff, ws.nnew, ws.active, ws.bdeg, ws.balpha,
                 ws.ucount, ws.rec_type, ws.rec_id, ws.rec_k, ws.fb_k, ws.mode, ws.whole,
                 ws.fb_list, ws.wsum, ws.root0};
    const int TB = 256;
    auto grid = [&](int64_t n) { return dim3(grid_for(n, TB, num_cu * 16)); };
    // reductions into per-graph counters: fewer, longer-running threads
    auto gridr = [&](int64_t n) { return dim3(grid_for(n, TB, num_cu * 2)); };

    // ---- ingest: validation, entry sources, weighted degrees, trivial bound
    {
      // row_ptr read once
      TimedScope t("k_check_rowptr", (double)(N + 1) * 8);
      hipLaunchKernelGGL(k_check_rowptr, grid(N), dim3(TB), 0, s, N, E, P.rp, ws.ctl);
    }
    int rc = read_ctl();
    if (rc) return rc;
    if (ws.ctl_host->err) return MC_EINVAL;
    int32_t* gid = ws.gid[0];
    int32_t* gid_next = ws.gid[1];
    {
      hipLaunchKernelGGL(k_init_vertices, grid(N), dim3(TB), 0, s, N, ws.voff, G, gid, ws.ogid, ws.map);
      fill<int64_t>(ws.cdeg, 0, N, s);
      fill<int32_t>(ws.gmaxw, 0, G, s);
      if (E > 0) {
        need_first(N, E, P.rp);
        // per entry col and w (8 B); per vertex its row bounds and its
        // weighted degree (16 B)
        TimedScope t("k_ingest", (double)E * 8 + (double)N * 16);
        static const int ingest_grid = resident_grid((const void*)&k_ingest, TB, num_cu);
        hipLaunchKernelGGL(k_ingest, chunk_grid(E, ingest_grid), dim3(TB), 0, s, N, E, P.rp, P.col, P.w, gid,
                           ws.voff, ws.first, G, ws.cdeg, ws.gmaxw, ws.chmax, ws.ctl);
        chmax_rp = P.rp;
        chmax_w = P.w;
        chmax_nnz = E;
      }
      src_ok = false;
      fill<uint64_t>(ws.bdeg, ~0ull, G, s);
      fill<int64_t>(ws.wsum, 0, G, s);
      hipLaunchKernelGGL(k_min_degree, gridr(N), dim3(TB), 0, s, N, ws.cdeg, gid, (const int32_t*)nullptr,
                         ws.bdeg, ws.wsum);
    }
    // every col must lie inside its graph before any kernel indexes by it
    rc = read_ctl();
    if (rc) return rc;
    if (ws.ctl_host->err) return MC_EINVAL;
    if (opt.validate && E > 0) {
      need_src(N, E, P.rp);
      rc = check_symmetry(N, E, P.col, P.w);
      if (rc) return rc;
    }
    if (opt.scan_mode == 1) {
      // Region scans may never cover a component, so components are found
      // up front.  Sweeps and whole scans need no such pass: a scan that
      // covers a component reports alpha = 0, and a component contracted to
      // one vertex has degree 0.
      TimedScope t("connectivity", (double)E * 8 + (double)N * 16);
      hipLaunchKernelGGL(k_iota, grid(N), dim3(TB), 0, s, ws.parent, N);
      need_src(N, E, P.rp);
      hipLaunchKernelGGL(k_union_all_edges, grid(E), dim3(TB), 0, s, E, ws.src, P.col, ws.parent);
      hipLaunchKernelGGL(k_flatten, grid(N), dim3(TB), 0, s, N, ws.parent);
      fill<int32_t>(ws.nnew, 0, G, s);
      hipLaunchKernelGGL(k_count_roots, gridr(N), dim3(TB), 0, s, N, ws.parent, gid, ws.nnew);
    } else {
      fill<int32_t>(ws.nnew, 1, G, s);  // one component assumed; see above
    }
    hipLaunchKernelGGL(k_graph_init, grid(G), dim3(TB), 0, s, G, S, ws.root0, ws.parent, ws.gmaxw, ws.prok,
                       ws.ctl);
    if (want_side) {
      TimedScope t("k_side", (double)N * 13);
      SideArgs sa{N, ws.ogid, ws.map, ws.rec_type, ws.rec_id, ws.rec_k, ws.claim, ws.step,
                  ws.fb_rs, ws.parent, ws.root0, side, REC_DEG};
      hipLaunchKernelGGL(k_side, grid(N), dim3(TB), 0, s, sa);
      sa.want = REC_DISCONNECTED;
      hipLaunchKernelGGL(k_side, grid(N), dim3(TB), 0, s, sa);
    }
    if (lhat_in) {
      // a caller-supplied upper bound (a real cut value) lowers lambda-hat
      std::vector<int64_t> l0(G);
      MC_HIP(hipMemcpyAsync(l0.data(), ws.lhat, G * 8, hipMemcpyDeviceToHost, s));
      MC_HIP(hipStreamSynchronize(s));
      for (int32_t g = 0; g < G; ++g) l0[g] = std::min(l0[g], lhat_in[g]);
      MC_HIP(hipMemcpyAsync(ws.lhat, l0.data(), G * 8, hipMemcpyHostToDevice, s));
      MC_HIP(hipStreamSynchronize(s));
    }
    rc = read_ctl();
    if (rc) return rc;
    if (ws.ctl_host->err == -3) return MC_EOVERFLOW;
    if (ws.ctl_host->err) return MC_EINVAL;
    // the first round's tests run only where one can pass (a lower starting
    // bound from the caller or the clustering bound may enable PR1)
    // (Matula's bound lies below the best cut, so its tests always run)
    const bool approx = opt.approx_ppm > 0;
    // the clustering bound finished exactly: the exact loop runs on the last
    // level graph, starting from the clustering bound
    const bool finish = viecut_only && opt.viecut_exact;
    const bool pr_first_round =
        ws.ctl_host->n_pr > 0 || lhat_in != nullptr || opt.use_viecut || approx || finish;
    // in the first round only the graphs marked in prok are tested, unless a
    // lower starting bound may have enabled PR1 elsewhere
    const bool pr_first_all = lhat_in != nullptr || opt.use_viecut || approx || finish;
    // the bound the round's tests and scans contract with: the best cut
    // found (exact), or Matula's (1/2 - eps) delta below it
    const int64_t* cap = approx ? ws.kcap : ws.lhat;
    if (st) {
      std::vector<int64_t> l0(G);
      MC_HIP(hipMemcpy(l0.data(), ws.lhat, G * sizeof(int64_t), hipMemcpyDeviceToHost));
      st->lambda_initial = l0[0];
      st->lambda_viecut = -1;
    }
    LevelGraph last{};
    if (opt.use_viecut || viecut_only) {
      rc = viecut(P, S, gid, side, finish ? &last : nullptr);
      if (rc) return rc;
      rc = read_ctl();
      if (rc) return rc;
      if (st) {
        MC_HIP(hipMemcpyAsync(&st->lambda_viecut, ws.lhat, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
      }
      if (viecut_only && !finish) {
        if (want_side) {
          hipLaunchKernelGGL(k_normalize_side, grid(G), dim3(TB), 0, s, G, ws.voff, side, ws.flip);
          hipLaunchKernelGGL(k_apply_flip, grid(N), dim3(TB), 0, s, N, ws.ogid, ws.flip, side);
        }
        MC_HIP(hipMemcpyAsync(lambdas, ws.lhat, G * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        return MC_OK;
      }
    }

    // ---- the contraction loop
    int32_t n = N;
    int64_t nnz = E;
    const int64_t* rp = P.rp;
    const int32_t* col = P.col;
    const int32_t* w = P.w;
    if (finish) {
      // the last level graph is the input: its entry sources, degrees and
      // graph ids go where the loop reads the input's
      n = last.n;
      nnz = last.nnz;
      rp = last.rp;
      col = last.col;
      w = last.w;
      if (last.src != ws.src && nnz > 0) {
        MC_HIP(hipMemcpyAsync(ws.src, last.src, (size_t)nnz * 4, hipMemcpyDeviceToDevice, s));
        src_ok = true;
      }
      if (last.cdeg != ws.cdeg)
        MC_HIP(hipMemcpyAsync(ws.cdeg, last.cdeg, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
      if (last.gid != gid) MC_HIP(hipMemcpyAsync(gid, last.gid, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    }
    int32_t n_active = ws.ctl_host->n_active;
    int round = 0;
    dump("ingest", n, nnz, rp, col, w);
    // graphs scanned whole by one workgroup (modes 1 and 3): LDS-resident
    // capped sweeps index the graph directly; the hash-map scans of
    // scan_mode 2 keep their map at most 3/4 full
    const bool hashed = opt.scan_mode == 2;
    const int32_t cap_l = hashed ? (WHOLE_CAP_L * 3) / 4 : SMALL_CAP_L;
    const int32_t cap_s = hashed ? (WHOLE_CAP_S * 3) / 4 : SMALL_CAP_S;
    const int32_t whole_max = std::min(opt.whole_max > 0 ? opt.whole_max : cap_l, cap_l);
    const int32_t whole_small = std::min(whole_max, cap_s);
    int region_waves = opt.region_waves > 0 ? opt.region_waves : num_cu * 16;
    uint64_t seed = opt.seed ? opt.seed : 0x5EEDull;
    while (n_active > 0 && (opt.max_rounds <= 0 || round < opt.max_rounds)) {
      if (st && round < 64) { st->n_round[round] = n; st->nnz_round[round] = nnz; }
      ++round;
      // per-round control fields (Matula's bound reads the minimum degree
      // before the reset clears it)
      MC_HIP(hipMemsetAsync(ws.ctl, 0, sizeof(Ctl), s));
      if (approx) hipLaunchKernelGGL(k_matula_cap, grid(G), dim3(TB), 0, s, G, S, (int64_t)opt.approx_ppm, ws.kcap);
      hipLaunchKernelGGL(k_round_reset, grid(G), dim3(TB), 0, s, G, S);
      hipLaunchKernelGGL(k_iota, grid(n), dim3(TB), 0, s, ws.parent, n);
      fill<int32_t>(ws.claim, -1, n, s);
      if (opt.scan_visits > 1) fill<int32_t>(ws.vcount, 0, n, s);
      if (opt.use_pr && (round > 1 || pr_first_round)) {
        const int32_t* tested = (round == 1 && !pr_first_all) ? ws.prok : ws.active;
        {
          // per vertex its row bounds, degree, bound and parent, and its
          // first two entries with their neighbours' degrees
          TimedScope t("k_pr_sample", (double)n * 64);
          hipLaunchKernelGGL(k_pr_sample, grid(n), dim3(TB), 0, s, n, nnz, rp, col, w, chunk_maxima(rp, w, nnz),
                             ws.cdeg, gid, cap,
                             tested, ws.parent, ws.ucount);
          hipLaunchKernelGGL(k_flatten, grid(n), dim3(TB), 0, s, n, ws.parent);
        }
        hipLaunchKernelGGL(k_lam_floor, dim3(1), dim3(256), 0, s, G, cap, tested, ws.ctl);
        {
          // every entry's weight (4 B: an entry that cannot pass for any graph
          // is rejected from it alone), per vertex its row bounds and c(u)
          // (16 B): a lower bound of what the tests must read
          TimedScope t("k_pr", (double)nnz * 4 + (double)n * 16);
          const int prc = pr_tests(n, nnz, rp, col, w, ws.cdeg, gid, cap, tested);
          if (prc) return prc;
        }
      }
      // the triangle tests on contracted graphs (from the second round; a
      // negative limit also tests the input): per tested edge both rows
      const int32_t tri_deg = opt.pr_triangle_deg < 0 ? -opt.pr_triangle_deg : opt.pr_triangle_deg;
      if (opt.use_pr && tri_deg > 0 && (round > 1 || opt.pr_triangle_deg < 0)) {
        need_src(n, nnz, rp);
        TimedScope t("k_pr34", (double)nnz * 20);
        hipLaunchKernelGGL(k_pr34, grid(nnz), dim3(TB), 0, s, nnz, ws.src, col, w, rp, ws.cdeg, gid, cap,
                           ws.active, tri_deg, ws.parent, ws.ucount, ws.ctl);
      }
      // blocks left by the tests; graphs already at two blocks skip the scans
      hipLaunchKernelGGL(k_flatten, grid(n), dim3(TB), 0, s, n, ws.parent);
      hipLaunchKernelGGL(k_count_roots, gridr(n), dim3(TB), 0, s, n, ws.parent, gid, ws.nnew);
      // plan: whole-graph scans for small graphs (two map sizes), sweeps or
      // region scans otherwise
      hipLaunchKernelGGL(k_plan_split, dim3(1), dim3(PLAN_THREADS), 0, s, G, S, rp, whole_small, whole_max,
                         ws.whole2, ws.ctl);
      // scans
      ScanArgs A{};
      A.n = n; A.rp = rp; A.col = col; A.w = w; A.cdeg = ws.cdeg; A.gid = gid;
      A.lhat = cap; A.gn = ws.gn; A.gvoff = ws.cvoff; A.gmode = ws.mode;
      A.claim = ws.claim; A.step = ws.step; A.pairs = ws.keys_alt; A.pairs_cap = ws.capE;
      A.best_alpha = ws.balpha; A.scan_k = ws.scan_k; A.scan_k_cap = (int32_t)std::min<int64_t>(ws.scan_k_cap, INT32_MAX);
      A.ucount = ws.ucount; A.ctl = ws.ctl;
      A.eager = opt.eager_blacklist;
      A.max_pops = opt.max_pops > 0 ? opt.max_pops : INT32_MAX;
      A.order = opt.pq_order;
      A.visits = opt.scan_visits > 1 ? opt.scan_visits : 1;
      A.vcount = ws.vcount;
      uint64_t rs = seed + 0x9E3779B97F4A7C15ull * (uint64_t)round;
      rs ^= rs >> 31;
      rs *= 0xBF58476D1CE4E5B9ull;
      A.seed = rs;
      A.perm_bits = std::max(1, bitlen((uint64_t)n - 1));
      A.perm_a = (rs | 1ull) & ((1ull << A.perm_bits) - 1);
      if (A.perm_a == 0) A.perm_a = 1;
      A.perm_b = (rs >> 17) & ((1ull << A.perm_bits) - 1);
      // algorithmic bytes of one region-scan launch: every adjacency entry
      // once (col, w) plus the claim gather, and per vertex row_ptr, cdeg,
      // claim and step.  Whole-graph scans count the graphs they were given
      // (added once the plan's sizes are read back).
      const double scan_bytes = (double)nnz * (8 + (opt.eager_blacklist ? 4 : 0)) + (double)n * 32;
      if (opt.scan_mode == 1 && !opt.force_fallback) {
        TimedScope t("capforest_region", scan_bytes);
        A.whole_mode = 0;
        A.whole = ws.whole;
        A.whole_count = &ws.ctl->n_region;  // unused in region mode
        const int wpb = 4;
        int blocks = std::max(1, region_waves / wpb);
        if (A.order > 0)
          hipLaunchKernelGGL((k_capforest<REGION_CAP, true>), dim3(blocks), dim3(64 * wpb),
                             sizeof(ScanLds<REGION_CAP, true>) * wpb, s, A);
        else
          hipLaunchKernelGGL((k_capforest<REGION_CAP, false>), dim3(blocks), dim3(64 * wpb),
                             sizeof(ScanLds<REGION_CAP, false>) * wpb, s, A);
      }
      if (hashed) {
        TimedScope t("capforest_whole", 0.0);
        // whole-graph scans, one pop at a time: small map, then large map
        MC_HIP(hipMemsetAsync(&ws.ctl->work_next, 0, sizeof(int32_t), s));
        A.whole_mode = 1;
        A.whole = ws.whole;
        A.whole_count = &ws.ctl->n_whole;
        if (A.order > 0)
          hipLaunchKernelGGL((k_capforest<WHOLE_CAP_S, true>), dim3(num_cu * 4), dim3(64),
                             sizeof(ScanLds<WHOLE_CAP_S, true>), s, A);
        else
          hipLaunchKernelGGL((k_capforest<WHOLE_CAP_S, false>), dim3(num_cu * 4), dim3(64),
                             sizeof(ScanLds<WHOLE_CAP_S, false>), s, A);
        MC_HIP(hipMemsetAsync(&ws.ctl->work_next, 0, sizeof(int32_t), s));
        A.whole = ws.whole2;
        A.whole_count = &ws.ctl->n_whole2;
        if (A.order > 0)
          hipLaunchKernelGGL((k_capforest<WHOLE_CAP_L, true>), dim3(num_cu * 2), dim3(64),
                             sizeof(ScanLds<WHOLE_CAP_L, true>), s, A);
        else
          hipLaunchKernelGGL((k_capforest<WHOLE_CAP_L, false>), dim3(num_cu * 2), dim3(64),
                             sizeof(ScanLds<WHOLE_CAP_L, false>), s, A);
      } else {
        // whole small graphs: LDS-resident capped sweeps, one workgroup each,
        // the large-map list first (both lists are ordered largest first)
        SmallSweepArgs SA{rp, col, w, ws.cdeg, cap, ws.gn, ws.cvoff, ws.whole2, &ws.ctl->n_whole2, ws.whole,
                          &ws.ctl->n_whole, &ws.ctl->work_next, ws.fb_rs, ws.capq, ws.capx, ws.npairs,
                          ws.balpha, ws.fb_k, ws.ucount, A.seed, opt.pq_order};
        {
          TimedScope t("k_small_sweep", 0.0);
          MC_HIP(hipMemsetAsync(&ws.ctl->work_next, 0, sizeof(int32_t), s));
          launch_small_sweep(opt.sweep_threads, opt.sweep_groups, num_cu, SA, s);
        }
        hipLaunchKernelGGL(k_small_sweep_unite, dim3(num_cu * 4), dim3(TB), 0, s, ws.whole, &ws.ctl->n_whole,
                           ws.cvoff, ws.npairs, ws.capq, ws.capx, ws.parent);
        hipLaunchKernelGGL(k_small_sweep_unite, dim3(num_cu * 4), dim3(TB), 0, s, ws.whole2, &ws.ctl->n_whole2,
                           ws.cvoff, ws.npairs, ws.capq, ws.capx, ws.parent);
      }
      {
        TimedScope t("k_union_pairs", (double)n * 8);
        hipLaunchKernelGGL(k_union_pairs, grid(n), dim3(TB), 0, s, ws.keys_alt, ws.ctl, ws.capE, ws.parent);
      }
      const int sweep_region = (opt.scan_mode != 1 || opt.force_fallback) ? 1 : 0;
      hipLaunchKernelGGL(k_sweep_list, grid(G), dim3(TB), 0, s, G, S, sweep_region, ws.ctl);
      hipLaunchKernelGGL(k_sweep_info, grid(G), dim3(TB), 0, s, ws.fb_list, ws.ctl, ws.cvoff, ws.gn,
                         cap, rp, ws.sw_info);
      rc = read_ctl();
      if (rc) return rc;
      // whole scans: col and w per entry; row_ptr, cdeg, claim and step (one-pop
      // scans) or row_ptr, cdeg and two stamp writes (LDS sweeps) per vertex
      if (hashed)
        timer().add_bytes("capforest_whole", (double)ws.ctl_host->whole_nnz * 8 + (double)ws.ctl_host->whole_nv * 32);
      else
        timer().add_bytes("k_small_sweep", (double)ws.ctl_host->whole_nnz * 8 + (double)ws.ctl_host->whole_nv * 40);
      if (st) {
        st->unions_pr += ws.ctl_host->unions_pr;
        st->scans += ws.ctl_host->scan_ids;
        st->pops += ws.ctl_host->pops;
        st->overflows += ws.ctl_host->overflows;
      }
      const int32_t n_sweeps = ws.ctl_host->n_fallback;
      if (n_sweeps > 0) {
        std::vector<int64_t> info((size_t)n_sweeps * 5);
        std::vector<int32_t> glist(n_sweeps);
        MC_HIP(hipMemcpyAsync(info.data(), ws.sw_info, info.size() * 8, hipMemcpyDeviceToHost, s));
        MC_HIP(hipMemcpyAsync(glist.data(), ws.fb_list, n_sweeps * 4, hipMemcpyDeviceToHost, s));
        MC_HIP(hipStreamSynchronize(s));
        rc = sweep_graphs(glist, info, round, rp, col, w, S);
        if (rc) return rc;
        if (st) st->fallbacks += n_sweeps;
      }
      // union-find finish and block numbering
      {
        TimedScope t("compact", (double)n * 16);
        hipLaunchKernelGGL(k_flatten, grid(n), dim3(TB), 0, s, n, ws.parent);
        if (debug_labels) {
          MC_HIP(hipMemcpyAsync(debug_labels, ws.parent, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
          MC_HIP(hipMemcpyAsync(debug_lhat, ws.lhat, (size_t)G * 8, hipMemcpyDeviceToHost, s));
          MC_HIP(hipStreamSynchronize(s));
          return MC_OK;
        }
        exclusive_scan<int32_t, RootFlag>(RootFlag{ws.parent, gid, ws.active, 0}, n, ws.newid,
                                          &ws.ctl->n_next, ws.tmp, s);
        fill<int32_t>(ws.nnew, 0, G, s);
        hipLaunchKernelGGL(k_relabel, grid(n), dim3(TB), 0, s, n, ws.parent, gid, ws.active, 0,
                           ws.newid, ws.lab, gid_next, ws.nnew);
      }
      hipLaunchKernelGGL(k_update_alpha, grid(G), dim3(TB), 0, s, G, S, ws.scan_k, ws.ctl);
      if (want_side) {
        TimedScope t("k_side", (double)N * 21);
        SideArgs sa{N, ws.ogid, ws.map, ws.rec_type, ws.rec_id, ws.rec_k, ws.claim, ws.step,
                    ws.fb_rs, ws.parent, ws.root0, side, REC_ALPHA};
        hipLaunchKernelGGL(k_side, grid(N), dim3(TB), 0, s, sa);
      }
      rc = read_ctl();
      if (rc) return rc;
      dump("after-scans", n, nnz, rp, col, w);
      const int32_t n_next = ws.ctl_host->n_next;
      if (st) st->pairs_scan += ws.ctl_host->pairs;
      // contraction: emit, sort, merge, CSR, degrees
      int64_t m2 = 0;
      rc = contract(nnz, rp, col, w, ws.lab, n, gid, n_next, gid_next,
                    Out{ws.src, ws.col, ws.w, ws.rp, ws.cdeg}, &m2, kExactNames);
      if (rc) return rc;
      src_ok = true;
      exclusive_scan<int32_t, ArrayIn<int32_t>>(ArrayIn<int32_t>{ws.nnew}, G, ws.nvoff,
                                                (int32_t*)nullptr, ws.tmp, s);
      hipLaunchKernelGGL(k_compose_map, grid(N), dim3(TB), 0, s, N, ws.map, ws.lab);
      MC_HIP(hipMemsetAsync(&ws.ctl->n_active, 0, sizeof(int32_t), s));
      hipLaunchKernelGGL(k_finish_round, grid(G), dim3(TB), 0, s, G, S, ws.nvoff, ws.ctl);
      if (want_side) {
        TimedScope t("k_side", (double)N * 9);
        SideArgs sa{N, ws.ogid, ws.map, ws.rec_type, ws.rec_id, ws.rec_k, ws.claim, ws.step,
                    ws.fb_rs, ws.parent, ws.root0, side, REC_DEG};
        hipLaunchKernelGGL(k_side, grid(N), dim3(TB), 0, s, sa);
      }
      rc = read_ctl();
      if (rc) return rc;
      // every active graph contracts at least one edge per round (a whole
      // scan or the fallback guarantees a contractible pair)
      if (n_next >= n && n_active > 0) return MC_EINTERNAL;
      n_active = ws.ctl_host->n_active;
      std::swap(gid, gid_next);
      n = n_next;
      nnz = m2;
      rp = ws.rp;
      col = ws.col;
      w = ws.w;
      dump("contracted", n, nnz, rp, col, w);
      MC_HIP(hipGetLastError());
    }
    if (st) st->rounds = round;
    if (want_side) {
      hipLaunchKernelGGL(k_normalize_side, grid(G), dim3(TB), 0, s, G, ws.voff, side, ws.flip);
      hipLaunchKernelGGL(k_apply_flip, grid(N), dim3(TB), 0, s, N, ws.ogid, ws.flip, side);
    }
    MC_HIP(hipMemcpyAsync(lambdas, ws.lhat, G * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MC_HIP(hipStreamSynchronize(s));
    MC_HIP(hipGetLastError());
    return MC_OK;
  }
};

// One cached workspace per (device, stream): calls on different streams
// run concurrently, each on its own arrays; calls on one stream take turns
// on its slot.
struct Slot {
  std::mutex m;
  Workspace ws;
};

std::mutex& registry_mutex() {
  static std::mutex m;
  return m;
}

std::map<std::pair<int, void*>, std::unique_ptr<Slot>>& registry() {
  static std::map<std::pair<int, void*>, std::unique_ptr<Slot>> r;
  return r;
}

int slot_for(void* stream, Slot** out) {
  int dev = 0;
  MC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(registry_mutex());
  auto& p = registry()[{dev, stream}];
  if (!p) p = std::make_unique<Slot>();
  *out = p.get();
  return MC_OK;
}

// A solve on a given workspace and stream (no lock: the caller owns both).
// With opt->workspace the device arrays are carved from the caller's block
// (ws then only lends its pinned host staging).
// ------------------------------------------------------------ tuned settings
// What mc_tune_batched chose, per device and size class of the problem:
// the bit lengths of its graph count, vertex total and entry total (each
// class spans a factor of two in each).
struct TuneKey {
  int dev, g, n, e;
  bool operator<(const TuneKey& o) const {
    return dev != o.dev ? dev < o.dev : g != o.g ? g < o.g : n != o.n ? n < o.n : e < o.e;
  }
};
struct Tuned {
  int32_t sweep_threads, sweep_groups, sort_tile, pr_triangle_deg, pq_order;
};
static std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
static std::map<TuneKey, Tuned>& tune_cache() {
  static std::map<TuneKey, Tuned> c;
  return c;
}
static TuneKey size_class(int32_t G, int64_t n, int64_t nnz) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return TuneKey{dev, bitlen((uint64_t)G), bitlen((uint64_t)n), bitlen((uint64_t)nnz)};
}
static void apply_tuned(const Tuned& t, mc_options& o) {
  o.sweep_threads = t.sweep_threads;
  o.sweep_groups = t.sweep_groups;
  o.sort_tile = t.sort_tile;
  o.pr_triangle_deg = t.pr_triangle_deg;
  o.pq_order = t.pq_order;
}
// The stored settings of P's size class into o; false if there are none.
static bool lookup_tuned(int32_t G, int64_t n, int64_t nnz, mc_options& o) {
  std::lock_guard<std::mutex> lock(tune_mutex());
  const auto it = tune_cache().find(size_class(G, n, nnz));
  if (it == tune_cache().end()) return false;
  apply_tuned(it->second, o);
  return true;
}

int run_on(Workspace& ws, const Problem& P, void* stream, const mc_options* opt, int64_t* lambdas, uint8_t* side,
           mc_stats* st, int32_t* debug_labels = nullptr, int64_t* debug_lhat = nullptr,
           const int64_t* lhat_in = nullptr, int32_t* viecut_levels = nullptr) {
  if (!lambdas || !P.rp || !P.col || !P.w || P.G < 1 || P.n < 2 || P.nnz < 0) return MC_EINVAL;
  if (P.n > (1 << 30) - 1 || P.nnz >= (int64_t)UINT32_MAX) return MC_EINVAL;
  for (int32_t g = 0; g < P.G; ++g) {
    if (P.voff_host[g + 1] < P.voff_host[g]) return MC_EINVAL;
    if (P.voff_host[g + 1] - P.voff_host[g] < 2) return MC_ENOCUT;
  }
  if (P.voff_host[0] != 0 || P.voff_host[P.G] != P.n) return MC_EINVAL;
  auto t0 = std::chrono::steady_clock::now();
  mc_options o;
  mc_options_default(&o);
  if (opt) o = *opt;
  if (o.use_tuned) lookup_tuned(P.G, P.n, P.nnz, o);
  if (o.approx_ppm < 0 || o.approx_ppm >= 500000) return MC_EINVAL;
  if (o.pq_order < 0 || o.pq_order > 3 || o.scan_visits < 0) return MC_EINVAL;
  if (st) {
    std::memset(st, 0, sizeof(*st));
  }
  Workspace caller_ws;
  Workspace* W = &ws;
  CallerBlock cb;
  int rc = MC_OK;
  if (o.workspace) {
    rc = ws.ensure_host();
    if (rc) return rc;
    caller_ws.host_owned = false;
    caller_ws.ctl_host = ws.ctl_host;
    caller_ws.sweep_host = ws.sweep_host;
    caller_ws.sw_args_host = ws.sw_args_host;
    caller_ws.sw_run_host = ws.sw_run_host;
    caller_ws.sw_status_host = ws.sw_status_host;
    rc = carve_caller(caller_ws, o.workspace, (size_t)o.workspace_bytes, P.n, P.nnz, P.G);
    if (rc) return rc;
    cb.base = (char*)o.workspace;
    cb.bytes = (size_t)o.workspace_bytes;
    cb.core = workspace_bytes(P.n, P.nnz, P.G);
    W = &caller_ws;
  } else {
    rc = ensure(ws, P.n, P.nnz, P.G);
    if (rc) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  Timer& T = timer();
  T.on = o.timing != 0;
  T.s = s;
  Solver sv{*W, s, o};
  sv.cb = cb;
  sv.stats_out = st;
  sv.debug_labels = debug_labels;
  sv.debug_lhat = debug_lhat;
  sv.lhat_in = lhat_in;
  sv.viecut_only = viecut_levels != nullptr;
  rc = sv.solve(P, lambdas, side, st);
  if (viecut_levels) *viecut_levels = sv.vc_levels_run;
  // the events are read when the classes are (mc_timing_get), after the
  // caller's timed region, not at the end of every solve
  T.on = false;
  if (st) st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

// ------------------------------------------------------------ no allocation
// mc_mincut_noalloc's workspace: a fixed array in the code object, one copy
// per device, held until the process ends.  Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device
// (the array's name is a host-side stand-in, not a device address).
constexpr size_t NOALLOC_BYTES = 64ull << 20;
constexpr int NOALLOC_DEVICES = 16;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

// Pageable host staging for the same calls (no pinned allocation).
struct NoAllocHost {
  Ctl ctl;
  SweepCtl sweep;
  SweepArgs args[MAX_SWEEPS];
  int32_t run[MAX_SWEEPS];
  SweepStatus status[MAX_SWEEPS];
};

struct NoAllocDevice {
  std::mutex m;          // calls on one device take turns on its array
  void* ptr = nullptr;   // the device's copy of `scratch`
  bool ready = false;
  NoAllocHost host;
};

NoAllocDevice* noalloc_device(int dev) {
  static NoAllocDevice devices[NOALLOC_DEVICES];
  return dev >= 0 && dev < NOALLOC_DEVICES ? &devices[dev] : nullptr;
}

// The library's own entry points: the stream's cached workspace.
int run(const Problem& P, void* stream, const mc_options* opt, int64_t* lambdas, uint8_t* side,
        mc_stats* st, int32_t* debug_labels = nullptr, int64_t* debug_lhat = nullptr,
        const int64_t* lhat_in = nullptr, int32_t* viecut_levels = nullptr) {
  Slot* sl = nullptr;
  int rc = slot_for(stream, &sl);
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(sl->m);
  return run_on(sl->ws, P, stream, opt, lambdas, side, st, debug_labels, debug_lhat, lhat_in, viecut_levels);
}

}  // namespace mc

extern "C" {

void mc_options_default(mc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->seed = 0x5EED;
  o->use_pr = 1;
  o->use_viecut = 0;
  o->eager_blacklist = 1;
  o->lp_sweeps = 2;
  o->pr_triangle_deg = 64;
  o->sweep_tail = 0;
}

int mc_mincut(const mc_graph* g, void* stream, const mc_options* opt, int64_t* lambda,
              uint8_t* side, mc_stats* stats) {
  if (!g || !lambda) return MC_EINVAL;
  if (g->n < 2) return MC_ENOCUT;
  int64_t voff[2] = {0, g->n};
  mc::Problem P{1, g->n, g->nnz, g->row_ptr, g->col, g->w, voff};
  return mc::run(P, stream, opt, lambda, side, stats);
}

int mc_mincut_batched(const mc_batch* b, void* stream, const mc_options* opt, int64_t* lambdas,
                      uint8_t* sides, mc_stats* stats) {
  if (!b || !lambdas || !b->vtx_off || b->num_graphs < 1) return MC_EINVAL;
  mc::Problem P{b->num_graphs, b->n_total, b->nnz_total, b->row_ptr, b->col, b->w, b->vtx_off};
  return mc::run(P, stream, opt, lambdas, sides, stats);
}

int mc_tune_batched(const mc_batch* b, void* stream, const mc_options* base, int32_t reps,
                    mc_tune_result* out) {
  if (!b || !out || !b->vtx_off || b->num_graphs < 1) return MC_EINVAL;
  mc_options o;
  if (base) o = *base;
  else mc_options_default(&o);
  o.timing = 0;
  reps = std::max(1, reps);
  std::vector<int64_t> ref, lam((size_t)b->num_graphs);
  int count = 0;
  // best wall time of `reps` solves at shape c; every solve's lambdas must
  // equal the first solve's
  auto solve_ms = [&](const mc_options& c, double& ms) -> int {
    ms = 1e300;
    for (int r = 0; r < reps; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      const int rc = mc_mincut_batched(b, stream, &c, lam.data(), nullptr, nullptr);
      const auto t1 = std::chrono::steady_clock::now();
      if (rc) return rc;
      ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
      if (ref.empty()) ref = lam;
      else if (lam != ref) return MC_EMISMATCH;
    }
    ++count;
    return MC_OK;
  };
  // workgroups per CU that one LDS sweep of `threads` threads can have
  auto fit = [](int threads) {
    const int bytes = threads == 128   ? (int)sizeof(mc::SmallSweepLds<mc::SMALL_CAP_L, 128>)
                      : threads == 512 ? (int)sizeof(mc::SmallSweepLds<mc::SMALL_CAP_L, 512>)
                                       : (int)sizeof(mc::SmallSweepLds<mc::SMALL_CAP_L, 256>);
    return std::max(1, mc::LDS_PER_CU / bytes);
  };
  o.use_tuned = 0;
  mc_options best = o;
  best.sweep_threads = 256;
  best.sweep_groups = std::min(3, fit(256));
  best.sort_tile = 4096;
  double best_ms = 0, default_ms = 0;
  int rc = solve_ms(best, default_ms);
  if (rc) return rc;
  best_ms = default_ms;
  // one setting at a time, each kept if it is faster (coordinate descent)
  auto try_opts = [&](const mc_options& c) -> int {
    double ms = 0;
    const int r = solve_ms(c, ms);
    if (r) return r;
    if (ms < best_ms) { best_ms = ms; best = c; }
    return MC_OK;
  };
  // the LDS sweep's shape
  const mc_options shape0 = best;
  for (int threads : {128, 256, 512}) {
    for (int groups : {2, 3}) {
      if (groups > fit(threads)) continue;
      if (threads == shape0.sweep_threads && groups == shape0.sweep_groups) continue;
      mc_options c = shape0;
      c.sweep_threads = threads;
      c.sweep_groups = groups;
      if ((rc = try_opts(c))) return rc;
    }
  }
  // the sort tile
  const mc_options shape1 = best;
  for (int tile : {2048, 8192}) {
    mc_options c = shape1;
    c.sort_tile = tile;
    if ((rc = try_opts(c))) return rc;
  }
  // the triangle tests: off, from the first round, or the base's
  const mc_options shape2 = best;
  for (int tri : {0, -64, 64}) {
    if (tri == shape2.pr_triangle_deg) continue;
    mc_options c = shape2;
    c.pr_triangle_deg = tri;
    if ((rc = try_opts(c))) return rc;
  }
  // the priority-queue order among equal keys (changes the rounds)
  const mc_options shape3 = best;
  for (int order : {1, 2, 3}) {
    if (order == shape3.pq_order) continue;
    mc_options c = shape3;
    c.pq_order = order;
    if ((rc = try_opts(c))) return rc;
  }
  {
    std::lock_guard<std::mutex> lock(mc::tune_mutex());
    mc::tune_cache()[mc::size_class(b->num_graphs, b->n_total, b->nnz_total)] =
        mc::Tuned{best.sweep_threads, best.sweep_groups, best.sort_tile, best.pr_triangle_deg, best.pq_order};
  }
  out->best = best;
  out->candidates = count;
  out->reps = reps;
  out->best_ms = best_ms;
  out->default_ms = default_ms;
  return MC_OK;
}

int mc_tune_lookup(const mc_batch* b, mc_options* opt) {
  if (!b || !opt || b->num_graphs < 1) return MC_EINVAL;
  return mc::lookup_tuned(b->num_graphs, b->n_total, b->nnz_total, *opt) ? 1 : 0;
}

void mc_tune_clear(void) {
  std::lock_guard<std::mutex> lock(mc::tune_mutex());
  mc::tune_cache().clear();
}

int mc_debug_first_round(const mc_batch* b, void* stream, const mc_options* opt, const int64_t* lhat_in,
                          int32_t* labels, int64_t* lhat_used) {
  if (!b || !labels || !lhat_used || !b->vtx_off || b->num_graphs < 1) return MC_EINVAL;
  std::vector<int64_t> lam(b->num_graphs);
  mc::Problem P{b->num_graphs, b->n_total, b->nnz_total, b->row_ptr, b->col, b->w, b->vtx_off};
  return mc::run(P, stream, opt, lam.data(), nullptr, nullptr, labels, lhat_used, lhat_in);
}

int mc_viecut_bound(const mc_batch* b, void* stream, const mc_options* opt, int64_t* bounds,
                    uint8_t* sides, int32_t* levels) {
  if (!b || !bounds || !b->vtx_off || b->num_graphs < 1) return MC_EINVAL;
  mc::Problem P{b->num_graphs, b->n_total, b->nnz_total, b->row_ptr, b->col, b->w, b->vtx_off};
  int32_t lv = 0;
  int rc = mc::run(P, stream, opt, bounds, sides, nullptr, nullptr, nullptr, nullptr, &lv);
  if (levels) *levels = lv;
  return rc;
}

int mc_debug_lp_sweep(const mc_graph* g, const int32_t* labels_in, int32_t* labels_out, void* stream) {
  using namespace mc;
  if (!g || !labels_in || !labels_out || g->n < 1 || !g->row_ptr || !g->col || !g->w) return MC_EINVAL;
  Slot* sl = nullptr;
  int rc = slot_for(stream, &sl);
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(sl->m);
  Workspace& ws = sl->ws;
  rc = ensure(ws, g->n, g->nnz, 1);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 0;
  MC_HIP(hipGetDevice(&dev));
  MC_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  rc = ensure_vc(ws, g->n, g->nnz, 1, CallerBlock{});
  if (rc) return rc;
  MC_HIP(hipMemsetAsync(ws.ctl, 0, sizeof(Ctl), s));
  fill<int32_t>(ws.gid[0], 0, g->n, s);
  fill<int32_t>(ws.active, 1, 1, s);
  fill<uint64_t>(ws.vc.best, 0, g->n, s);
  LpArgs L{g->n, g->row_ptr, g->col, g->w, ws.gid[0], ws.active, labels_in, labels_out, ws.vc.item_off,
           &ws.ctl->lp_items, ws.vc.best};
  lp_items_prefix(L, ws, s);
  lp_sweep(L, ncu, s);
  MC_HIP(hipStreamSynchronize(s));
  MC_HIP(hipGetLastError());
  return MC_OK;
}

// weighted degree of every row without self-loops (test hooks only)
__global__ void k_row_degrees(int32_t n, const int64_t* rp, const int32_t* col, const int32_t* w, int64_t* cdeg) {
  for (int64_t u = mc::gtid(); u < n; u += mc::gstride()) {
    int64_t d = 0;
    for (int64_t e = rp[u]; e < rp[u + 1]; ++e)
      if (col[e] != (int32_t)u) d += w[e];
    cdeg[u] = d;
  }
}

int mc_debug_pr_tests(const mc_graph* g, void* stream, int64_t lhat, int32_t max_deg, uint8_t* flags) {
  using namespace mc;
  if (!g || !flags || g->n < 1 || g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && (!g->col || !g->w))) return MC_EINVAL;
  Slot* sl = nullptr;
  int rc = slot_for(stream, &sl);
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(sl->m);
  Workspace& ws = sl->ws;
  rc = ensure(ws, g->n, g->nnz, 1);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid(grid_for(g->n, 256, 65536));
  hipLaunchKernelGGL(k_row_degrees, grid, dim3(256), 0, s, g->n, g->row_ptr, g->col, g->w, ws.cdeg);
  hipLaunchKernelGGL(k_pr_flags, grid, dim3(256), 0, s, g->n, g->row_ptr, g->col, g->w, ws.cdeg, lhat, max_deg,
                     flags);
  MC_HIP(hipStreamSynchronize(s));
  MC_HIP(hipGetLastError());
  return MC_OK;
}

int mc_debug_contract(const mc_graph* g, const int32_t* labels, int32_t n_new, void* stream,
                      int64_t* row_ptr_out, int32_t* col_out, int32_t* w_out, int64_t* nnz_out) {
  using namespace mc;
  if (!g || !labels || !row_ptr_out || !col_out || !w_out || !nnz_out || n_new < 1) return MC_EINVAL;
  Slot* sl = nullptr;
  int rc = slot_for(stream, &sl);
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(sl->m);
  Workspace& ws = sl->ws;
  rc = ensure(ws, std::max(g->n, n_new), g->nnz, 1);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, ncu = 0;
  MC_HIP(hipGetDevice(&dev));
  MC_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int TB = 256;
  const int64_t nnz = g->nnz;
  MC_HIP(hipMemsetAsync(ws.ctl, 0, sizeof(Ctl), s));
  // entry sources
  fill<int64_t>(ws.cdeg, 0, g->n, s);
  int64_t voff[2] = {0, g->n};
  MC_HIP(hipMemcpyAsync(ws.voff, voff, 16, hipMemcpyHostToDevice, s));
  fill<int32_t>(ws.gid[0], 0, g->n, s);
  fill<int32_t>(ws.gmaxw, 0, 1, s);
  hipLaunchKernelGGL(k_check_rowptr, dim3(grid_for(g->n, TB, ncu * 16)), dim3(TB), 0, s, g->n, nnz, g->row_ptr,
                     ws.ctl);
  MC_HIP(hipMemcpyAsync(ws.ctl_host, ws.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  MC_HIP(hipStreamSynchronize(s));
  if (ws.ctl_host->err) return MC_EINVAL;
  const dim3 chunks(grid_for((nnz + WCH - 1) / WCH * 64, TB, ncu * 8));
  if (nnz > 0) {
    hipLaunchKernelGGL(k_chunk_rows, dim3(grid_for(g->n, TB, ncu * 16)), dim3(TB), 0, s, g->n, g->row_ptr, ws.first);
    hipLaunchKernelGGL(k_ingest, chunks, dim3(TB), 0, s, g->n, nnz, g->row_ptr, g->col, g->w, ws.gid[0], ws.voff,
                       ws.first, 1, ws.cdeg, ws.gmaxw, ws.chmax, ws.ctl);
  }
  // every col inside [0, n) before the emit indexes the labels by it
  MC_HIP(hipMemcpyAsync(ws.ctl_host, ws.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  MC_HIP(hipStreamSynchronize(s));
  if (ws.ctl_host->err) return MC_EINVAL;
  const int bb = std::max(1, bitlen((uint64_t)n_new - 1));
  if (nnz > 0)
    hipLaunchKernelGGL(k_emit, chunks, dim3(TB), 0, s, g->n, nnz, g->row_ptr, ws.first, g->col, g->w, labels, bb,
                       (const uint32_t*)nullptr, ws.keys, ws.vals, ws.ctl);
  MC_HIP(hipMemcpyAsync(ws.ctl_host, ws.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  MC_HIP(hipStreamSynchronize(s));
  if (ws.ctl_host->err) return MC_EINVAL;
  const int64_t m = ws.ctl_host->emit;
  const int which = radix_sort_pairs(ws.keys, ws.vals, ws.keys_alt, ws.vals_alt, m, 2 * bb, ws.tmp, s);
  uint64_t* sk = which ? ws.keys_alt : ws.keys;
  int32_t* sv = which ? ws.vals_alt : ws.vals;
  int64_t* pos = (int64_t*)(which ? ws.keys : ws.keys_alt);
  exclusive_scan<int64_t, HeadFlag>(HeadFlag{sk}, m, pos, (int64_t*)&ws.ctl->unique, ws.tmp, s);
  MC_HIP(hipMemcpyAsync(ws.ctl_host, ws.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
  MC_HIP(hipStreamSynchronize(s));
  const int64_t m2 = m > 0 ? ws.ctl_host->unique : 0;
  fill<int32_t>(w_out, 0, m2, s);
  if (m > 0)
    hipLaunchKernelGGL(k_merge, dim3(grid_for((m + 255) / 256 * 256, TB, ncu * 16)), dim3(TB), 0, s, m, sk, sv,
                       pos, bb, ws.src, col_out, w_out);
  hipLaunchKernelGGL(k_rowptr, dim3(grid_for(n_new + 1, TB, ncu * 16)), dim3(TB), 0, s, n_new, m2, ws.src,
                     row_ptr_out);
  MC_HIP(hipStreamSynchronize(s));
  MC_HIP(hipGetLastError());
  *nnz_out = m2;
  return MC_OK;
}

size_t mc_workspace_bytes(int32_t n_total, int64_t nnz_total, int32_t num_graphs) {
  return mc::workspace_bytes(n_total, nnz_total, num_graphs);
}

size_t mc_viecut_workspace_bytes(int32_t n_total, int64_t nnz_total, int32_t num_graphs) {
  return mc::vc_workspace_bytes(n_total, nnz_total, num_graphs);
}

void mc_release(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> lock(mc::registry_mutex());
  auto& r = mc::registry();
  // the slots stay (another thread may be about to lock one); their memory goes
  for (auto& kv : r) {
    if (kv.first.first != dev) continue;
    std::lock_guard<std::mutex> l2(kv.second->m);  // waits for a call in progress on that stream
    kv.second->ws.release();
  }
}

int mc_mincut_noalloc(const mc_graph* g, void* stream, const mc_options* opt, int64_t* lambda, uint8_t* side) {
  using namespace mc;
  if (!g || !lambda) return MC_EINVAL;
  if (g->n < 2) return MC_ENOCUT;
  if (g->n > (1 << 30) - 1 || g->nnz < 0 || g->nnz >= (int64_t)UINT32_MAX) return MC_EINVAL;
  mc_options o;
  mc_options_default(&o);
  if (opt) o = *opt;
  // the clustering bound's level graphs and event timing would allocate
  if (o.use_viecut || o.workspace) return MC_EINVAL;
  o.timing = 0;
  if (workspace_bytes(g->n, g->nnz, 1) > NOALLOC_BYTES) return MC_ETOOBIG;
  int dev = 0;
  MC_HIP(hipGetDevice(&dev));
  NoAllocDevice* D = noalloc_device(dev);
  if (!D) return MC_EINVAL;
  std::lock_guard<std::mutex> lock(D->m);
  if (!D->ready) {
    // once per device, with that device current
    void* p = nullptr;
    MC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    D->ptr = p;
    D->ready = true;
  }
  Workspace lend;  // pageable staging; run_on carves the device arrays from D->ptr
  lend.host_owned = false;
  lend.ctl_host = &D->host.ctl;
  lend.sweep_host = &D->host.sweep;
  lend.sw_args_host = D->host.args;
  lend.sw_run_host = D->host.run;
  lend.sw_status_host = D->host.status;
  o.workspace = D->ptr;
  o.workspace_bytes = NOALLOC_BYTES;
  int64_t voff[2] = {0, g->n};
  Problem P{1, g->n, g->nnz, g->row_ptr, g->col, g->w, voff};
  return run_on(lend, P, stream, &o, lambda, side, nullptr);
}

const char* mc_strerror(int code) {
  switch (code) {
    case MC_OK: return "ok";
    case MC_EINVAL: return "invalid argument or malformed graph";
    case MC_ENOCUT: return "a graph with fewer than two vertices has no cut";
    case MC_EOVERFLOW: return "total edge weight exceeds 2*(2^31-1)";
    case MC_ENOMEM: return "device memory allocation failed";
    case MC_EHIP: return "HIP runtime error";
    case MC_EBUSY: return "server admission queue full";
    case MC_ESTATE: return "unknown ticket or stopped server";
    case MC_EINTERNAL: return "internal error: a round made no progress";
    case MC_EMISMATCH: return "internal error: launch shapes gave different results";
    case MC_ETOOBIG: return "graph too large for the fixed 64 MiB workspace of mc_mincut_noalloc";
    default: return "unknown error";
  }
}

int mc_timing_get(mc_timing_entry* out, int max) {
  auto& T = mc::timer();
  T.collect();
  int n = (int)T.classes.size();
  for (int i = 0; i < n && i < max; ++i) {
    std::memset(&out[i], 0, sizeof(out[i]));
    std::strncpy(out[i].name, T.classes[i].name.c_str(), sizeof(out[i].name) - 1);
    out[i].launches = T.classes[i].launches;
    out[i].ms = T.classes[i].ms;
    out[i].algo_bytes = T.classes[i].bytes;
  }
  return n;
}

void mc_timing_focus(const char* name) { mc::timer().focus = name ? name : ""; }

void mc_timing_reset(void) {
  auto& T = mc::timer();
  T.collect();
  T.classes.clear();
}

}  // extern "C"

#include "server.h"
