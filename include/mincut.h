/* Exact global minimum cut of undirected graphs with positive integer edge
 * weights, on one AMD Instinct MI355X (gfx950).
 *
 * The method is the bound-driven contraction loop of Henzinger, Noe and
 * Schulz, "Shared-memory Exact Minimum Cuts": an upper bound lambda-hat
 * (minimum weighted degree, optionally lowered by a VieCut-style clustering
 * pass), Padberg-Rinaldi tests, many concurrent bounded CAPFOREST scans that
 * mark contractible edges in a union-find (Algorithm 1, Lemmas 1 and 2), and
 * graph contraction, repeated until every graph is solved (Algorithm 2).
 * The result lambda is exact; one side of a minimum cut is also returned
 * (section "Putting Things Together").
 *
 * Conventions for every entry point:
 *  - Graphs are symmetric CSR arrays in DEVICE memory: row_ptr int64[n+1]
 *    (row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz), col int32[nnz],
 *    w int32[nnz] with w >= 1.  Each undirected edge {u,v} appears in row u
 *    and in row v with the same weight.  Self-loops are accepted and ignored
 *    (they never cross a cut); repeated entries count with their total
 *    weight.  Asymmetric input gives an undefined result.
 *  - The sum of all weights of one graph (over entries) must not exceed
 *    2 * (2^31 - 1), so every cut fits in 31 bits (MC_EOVERFLOW otherwise).
 *  - At most 2^30 - 1 vertices in total and nnz < 2^32 per call.
 *  - Inputs are never modified.  The caller owns all input and output
 *    buffers.  The library owns its workspace: one per (device, stream),
 *    allocated on first use, grown when needed, kept until mc_release();
 *    or the caller lends one (mc_options.workspace).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls return
 *    after the stream work has finished.  Calls on different streams are
 *    independent and may run at the same time from different host threads
 *    (each uses its stream's workspace); calls on the same stream take
 *    turns.
 *  - Every function returns MC_OK (0) or a negative MC_E* code; nothing
 *    throws across the ABI.  On error the outputs are unspecified.
 */
#ifndef MINCUT_H
#define MINCUT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MC_OK = 0,
  MC_EINVAL = -1,    /* null pointer, bad sizes, bad row_ptr, col out of range, w < 1 */
  MC_ENOCUT = -2,    /* a graph with fewer than two vertices has no cut */
  MC_EOVERFLOW = -3, /* total weight of a graph above 2 * (2^31 - 1) */
  MC_ENOMEM = -4,    /* device workspace allocation failed */
  MC_EHIP = -5,      /* a HIP runtime call failed */
  MC_EBUSY = -6,     /* server admission full (non-blocking submit) */
  MC_ESTATE = -7,    /* unknown ticket or server stopped */
  MC_EINTERNAL = -8, /* a round made no progress (never expected; reported, not looped) */
  MC_EMISMATCH = -9, /* the autotuner's launch shapes disagreed on a lambda (never expected) */
  MC_ETOOBIG = -10   /* mc_mincut_noalloc: the graph does not fit its fixed workspace */
};

typedef struct mc_graph {
  int32_t n;              /* vertices, >= 2 */
  int64_t nnz;            /* CSR entries (2 x undirected edges) */
  const int64_t* row_ptr; /* device, n + 1 */
  const int32_t* col;     /* device, nnz, in [0, n) */
  const int32_t* w;       /* device, nnz, >= 1 */
} mc_graph;

/* Many independent graphs packed as one CSR (their disjoint union):
 * graph g owns vertices [vtx_off[g], vtx_off[g+1]) and its entries hold
 * GLOBAL vertex ids inside that range. */
typedef struct mc_batch {
  int32_t num_graphs;
  int32_t n_total;
  int64_t nnz_total;
  const int64_t* row_ptr; /* device, n_total + 1 */
  const int32_t* col;     /* device, nnz_total */
  const int32_t* w;       /* device, nnz_total */
  const int64_t* vtx_off; /* HOST, num_graphs + 1, vtx_off[0] = 0 */
} mc_batch;

typedef struct mc_options {
  uint64_t seed;           /* scan start order */
  int32_t use_pr;          /* 1: Padberg-Rinaldi tests every round (default 1) */
  int32_t use_viecut;      /* 1: lower lambda-hat by clustering first (default 0) */
  int32_t region_waves;    /* concurrent region scans; 0 = one per SIMD slot */
  int32_t eager_blacklist; /* 1: skip neighbours already claimed elsewhere (default 1) */
  int32_t max_pops;        /* per-scan budget (early termination); 0 = unbounded */
  int32_t max_rounds;      /* safety cap on rounds; 0 = none */
  int32_t timing;          /* 1: time kernel classes with HIP events (mc_timing) */
  int32_t force_fallback;  /* debug: region scans find nothing, so the
                              sequential fallback always runs */
  int32_t whole_max;       /* graphs up to this size are scanned whole inside
                              one workgroup; 0 = default (8192) */
  int32_t lp_sweeps;       /* clustering sweeps per level when use_viecut */
  int32_t scan_mode;       /* 0 (default): full-graph capped sweeps (small
                              graphs in LDS, large ones grid-wide);
                              1: graphs above whole_max get many concurrent
                              bounded region scans (Algorithm 1), with the
                              sweep as fallback when they find nothing;
                              2: small graphs get one-pop-at-a-time scans
                              with an LDS hash map (no batching) */
  int32_t sweep_handoff;   /* sweep batches above this many vertices run
                              grid-wide; 0 = default (512) */
  int32_t viecut_stop;     /* clustering levels stop at this many vertices
                              per graph; 0 = default (2) */
  int32_t viecut_levels;   /* at most this many clustering levels; 0 =
                              default (32) */
  /* Launch shapes (results do not depend on them; mc_tune_batched picks
   * them for a batch): */
  int32_t sweep_threads;   /* threads per LDS-sweep workgroup: 128, 256 or
                              512; 0 = default (256) */
  int32_t sweep_groups;    /* LDS-sweep workgroups per compute unit, 1..3,
                              clamped to what LDS holds; 0 = default (3) */
  int32_t sort_tile;       /* keys per radix-sort workgroup: 2048, 4096 or
                              8192; 0 = default (4096) */
  int32_t pr_triangle_deg; /* the triangle tests PR3 and PR4 (see
                              mc_debug_pr_tests) on edges whose two rows hold
                              at most |pr_triangle_deg| entries in
                              increasing neighbour order.  > 0: from the
                              second round on (contracted graphs; default
                              64); < 0: from the first round on; 0: PR1 and
                              PR2 only */
  int32_t viecut_exact;    /* mc_viecut_bound only: 1 = finish the clustering
                              levels by solving the last level graph exactly
                              (its minimum cut, a cut of G, lowers the
                              bound, as the clustering algorithm ends in the
                              paper); 0 (default) = the levels' bound alone */
  int32_t approx_ppm;      /* 0 (default): exact.  1 .. 499999: Matula's
                              (2+eps)-approximation with eps = approx_ppm /
                              10^6 (the paper names it beside NOI: the
                              contraction bound of a round is (1/2 - eps)
                              times the graph's minimum degree, capped by the
                              best cut found; an edge contracts when its
                              q(e) reaches that product, i.e. its ceiling).
                              lambda is then a real cut with lambda(G) <=
                              lambda <= lambda(G) / (1/2 - eps), and the side
                              realises it.
                              Outside 0 .. 499999: MC_EINVAL. */
  int32_t validate;        /* 1: also check that every graph is symmetric
                              (for each pair u != v the weights of u's
                              entries to v add up to those of v's entries
                              to u); MC_EINVAL if not.  Costs one sort of the
                              entries.  0 (default): asymmetric input gives
                              an undefined result. */
  void* workspace;         /* NULL (default): the library's workspace for
                              the call's (device, stream), allocated on
                              first use and grown when needed.  Otherwise a
                              DEVICE buffer of workspace_bytes bytes that the
                              call uses instead (no device allocation);
                              it must hold mc_workspace_bytes(n, nnz, G),
                              plus mc_viecut_workspace_bytes(n, nnz, G)
                              when the clustering bound runs (use_viecut or
                              mc_viecut_bound), else MC_EINVAL.  Its
                              contents need no initialisation and are
                              garbage afterwards; two calls in flight must
                              not share one. */
  uint64_t workspace_bytes;
  int32_t sweep_tail;      /* the end of a full-graph capped sweep: 0
                              (default): once its last grid-wide batch has
                              left at most a quarter of the graph (and at
                              most 2^18 vertices) and at least 256 vertices
                              below the cap, the rest is scanned by many
                              concurrent processes that start from the
                              visited set (Algorithm 1's parallel CAPFOREST
                              with blacklisting); > 0: the same with this
                              lower limit; -1: never (one vertex at a time
                              to the end).  Changes which pairs a round
                              unites, never lambda. */
  int32_t sweep_pull;      /* a full-graph sweep's grid-wide batch: 0
                              (default) pushes the batch's rows into their
                              neighbours, or, when the vertices still free
                              hold fewer entries, pulls (each free vertex
                              sums its edges into the batch); 1: always
                              pull; -1: always push.  Changes which pairs a
                              round unites, never lambda. */
  int32_t pq_order;        /* the priority-queue order among equal keys in
                              the LDS sweeps' single pops and in region and
                              whole-graph scans (section "Priority Queue
                              Implementations"): 0 (default) the fastest
                              (the lowest chunk and lane holding the
                              maximum; in scans the highest map slot);
                              1 bucket queue (BQueue: the vertex whose key
                              last rose earliest); 2 bucket stack (BStack:
                              the one whose key last rose latest); 3 heap
                              (a fixed pseudo-random order).  Among the
                              increases of one step, the row order stands
                              in for push order (rows are sorted by
                              neighbour id after the first contraction).
                              Values outside 0..3: MC_EINVAL.  Changes
                              which pairs a round unites, never lambda. */
  int32_t scan_visits;     /* region and whole-graph scans (scan_mode 1 or
                              2): a vertex may be visited by up to this
                              many scans (the multi-visit variant of
                              section "Parallel CAPFOREST"); 0 or 1
                              (default): once.  A scan reports prefix cuts
                              only up to its first repeated visit.
                              Negative: MC_EINVAL. */
  int32_t use_tuned;       /* 1: take sweep_threads, sweep_groups,
                              sort_tile, pr_triangle_deg and pq_order from
                              what mc_tune_batched chose for this
                              problem's size class on the current device
                              (see mc_tune_batched), when there is one;
                              the caller's values otherwise.  Default 0. */
  int32_t emit_rows;       /* the contraction's key emit: 0 (default) reads
                              every entry, or, on graphs of at least 2^22
                              entries where the rows of vertices outside
                              their graph's reference block (its most
                              common block) hold under a quarter of the
                              entries, only those rows (the symmetric
                              CSR gives each skipped row's crossing
                              entries as mirrors); 1: always row-wise;
                              -1: never.  Changes no result. */
  int32_t sweep_seg;       /* push batches of the full-graph sweep: 0
                              (default) relaxes a batch of few long rows
                              range by range (each workgroup owns a range
                              of vertices, whose keys it adds in LDS) when
                              the batch rows' segments average at least 4
                              entries; 1: range by range always; -1: never
                              (all adds in global memory).  Range by range
                              needs the batch rows' neighbours in ascending
                              order: a row found out of order sends that
                              batch, and the rest of the sweep, to the
                              global form.  Changes which pairs a round
                              unites, never lambda. */
} mc_options;

typedef struct mc_stats {
  int32_t rounds;          /* contraction rounds */
  int32_t fallbacks;       /* sequential CAPFOREST runs */
  int64_t unions_pr;       /* pairs marked by Padberg-Rinaldi tests */
  int64_t pairs_scan;      /* pairs marked by CAPFOREST scans */
  int64_t scans;           /* scans started */
  int64_t pops;            /* vertices visited by scans */
  int64_t overflows;       /* scans ended because their LDS map filled */
  int64_t lambda_initial;  /* single graph: minimum weighted degree */
  int64_t lambda_viecut;   /* single graph: bound after clustering (or -1) */
  double ms;               /* wall time of the call */
  int32_t n_round[64];     /* vertices at the start of each round (first 64) */
  int64_t nnz_round[64];   /* entries at the start of each round */
  /* Filled only with opt->timing = 1.  Full-graph capped sweeps (graphs
   * above whole_max), summed over graphs and rounds, per phase: phase k
   * holds the steps of the sequential sweep kernel after k grid-wide
   * batches of its graph (the last phase also every later one). */
  int32_t sweep_phases;      /* phases in use (1 + most grid-wide batches, at most 8) */
  int32_t sweep_big_batches; /* grid-wide batches */
  int32_t sweep_singles[8];  /* single pops below the cap */
  int32_t sweep_batches[8];  /* batches of capped vertices run by the sweep kernel */
  int32_t sweep_cross[8];    /* crossings (each unites two vertices) made by those steps */
  int64_t sweep_tail_pops;   /* vertices visited by the concurrent tail scans */
} mc_stats;

/* Fill `opt` with the defaults. */
void mc_options_default(mc_options* opt);

/* lambda (HOST int64) receives the minimum cut value.  side (DEVICE uint8[n],
 * may be NULL) receives 1 for the vertices of one side of a minimum cut and
 * 0 for the others, with side[0] = 0.  A disconnected graph gives lambda = 0
 * and the side of every vertex outside vertex 0's component.  stats may be
 * NULL.  MC_ENOCUT if n < 2. */
int mc_mincut(const mc_graph* g, void* stream, const mc_options* opt, int64_t* lambda,
              uint8_t* side, mc_stats* stats);

/* All graphs of the batch in one packed solve.  lambdas: HOST int64[G].
 * sides: DEVICE uint8[n_total] or NULL; for each graph its first vertex is
 * on side 0.  MC_ENOCUT if any graph has fewer than two vertices. */
int mc_mincut_batched(const mc_batch* b, void* stream, const mc_options* opt, int64_t* lambdas,
                      uint8_t* sides, mc_stats* stats);

/* Autotuner for the batched form (not in the paper: the packed form and its
 * launch shapes are this library's).  Solves the batch `b` once per
 * candidate and keeps the fastest, one setting at a time: the LDS sweep's
 * threads per workgroup (128, 256, 512) and workgroups per compute unit
 * (2, 3); the radix sort's keys per workgroup (2048, 4096, 8192); the
 * triangle tests (off, from the first round, from the second); the
 * priority-queue order among equal keys (pq_order 0..3, which changes the
 * rounds).  Each candidate is solved `reps` times (at least 1) and its best
 * wall time counts.  Every solve must give the same lambdas (the settings
 * change the schedule and the rounds, never the result): otherwise
 * MC_EMISMATCH.  base: the other options (NULL = defaults); out->best is
 * base with the chosen settings.  The choice is also stored, for the
 * current device, under the batch's size class: the bit lengths of its
 * graph count, vertex total and entry total (a factor of two in each).
 * Solves with use_tuned = 1 whose problem falls in a stored class take it.
 * The store is process-wide and thread-safe.  The batch's inputs are read
 * only; no output buffer is written but *out. */
typedef struct mc_tune_result {
  mc_options best;        /* base with the chosen settings */
  int32_t candidates;     /* launch shapes solved */
  int32_t reps;           /* solves per shape */
  double best_ms;         /* best wall time of one packed solve with `best` */
  double default_ms;      /* ... with the default shape */
} mc_tune_result;
int mc_tune_batched(const mc_batch* b, void* stream, const mc_options* base, int32_t reps,
                    mc_tune_result* out);
/* The settings stored for b's size class on the current device, written
 * into *opt's tuned fields: 1 if there were some, 0 if not (opt unchanged);
 * MC_EINVAL for a NULL argument.  Reads only b's counts. */
int mc_tune_lookup(const mc_batch* b, mc_options* opt);
/* Forget every stored setting. */
void mc_tune_clear(void);

/* Test hook for per-step parity: runs ingest and the first round's
 * Padberg-Rinaldi tests and CAPFOREST scans (Algorithm 2, first loop
 * iteration up to the contraction), then stops.  lhat_in (HOST int64[G] or
 * NULL) caps each graph's starting bound (it must be the value of a real cut).
 * labels (DEVICE int32[n_total]) receives the union-find root of every
 * vertex, i.e. the blocks the round would contract; lhat_used (HOST
 * int64[G]) the bound each graph's tests and scans used.  Contracting the
 * blocks must keep every cut below that bound. */
int mc_debug_first_round(const mc_batch* b, void* stream, const mc_options* opt, const int64_t* lhat_in,
                          int32_t* labels, int64_t* lhat_used);

/* The VieCut-style upper bound alone (section "Inexact Shared-Memory
 * Minimum Cuts"; the first step of Algorithm 2), for every graph of the
 * batch.  Per level: opt->lp_sweeps synchronous label-propagation sweeps
 * (each vertex takes the neighbour label of largest total weight, ties to
 * the smallest label), contraction of the label classes, the Padberg-
 * Rinaldi tests (PR1 w >= bound, PR2 2w > c(u) or c(v)) on that graph and
 * contraction of their components; after each contraction the minimum
 * weighted degree (a real cut: every vertex is a vertex set of the input)
 * lowers the bound, starting from the input's minimum degree.  Levels stop
 * at opt->viecut_stop vertices, after opt->viecut_levels levels, or when a
 * level removes less than a tenth of a graph's vertices.  The result does
 * not depend on scheduling.
 *   bounds: HOST int64[G], each >= the graph's minimum cut.
 *   sides:  DEVICE uint8[n_total] or NULL: a side whose cut weight equals
 *           the bound, the graph's first vertex on side 0.
 *   levels: HOST int32 or NULL: the most levels any graph ran.
 * Errors as mc_mincut_batched.  mc_mincut and mc_mincut_batched run the
 * same bound first when opt->use_viecut = 1. */
int mc_viecut_bound(const mc_batch* b, void* stream, const mc_options* opt, int64_t* bounds,
                    uint8_t* sides, int32_t* levels);

/* Test hook for one label-propagation sweep of the clustering bound (the
 * rule of mc_viecut_bound) on one graph: labels_in and labels_out are
 * DEVICE int32[n], labels in [0, n).  Self-loops are ignored; a vertex
 * without neighbours keeps its label. */
int mc_debug_lp_sweep(const mc_graph* g, const int32_t* labels_in, int32_t* labels_out, void* stream);

/* Test hook for the Padberg-Rinaldi tests (the heuristics of Padberg and
 * Rinaldi that the paper applies in its clustering bound and names in its
 * related work; their conditions are not restated there).  For every entry
 * e = (u, v) with u < v, flags[e] (DEVICE uint8[nnz]) receives bit 1 if
 * c(e) >= lhat (PR1), bit 2 if 2 c(e) > c(u) or 2 c(e) > c(v) (PR2), bit 4 if
 * some common neighbour w != u, v has c(u) < 2 (c(e) + c(u,w)) and
 * c(v) < 2 (c(e) + c(v,w)) (PR3), bit 8 if c(e) + sum over common
 * neighbours of min(c(u,w), c(v,w)) >= lhat (PR4); every other entry gets 0.
 * c(e) is the entry's weight and c(x) the weighted degree without
 * self-loops; PR3 and PR4 are evaluated only where both rows hold at most
 * max_deg entries in strictly increasing neighbour order (else bits 4 and 8
 * are 0).  These are the tests the solve applies (PR3 and PR4 when
 * opt->pr_triangle_deg > 0).  MC_EINVAL for a null pointer or n < 1; the
 * graph itself is not checked (row_ptr monotone from 0 to nnz, every col in
 * [0, n)). */
int mc_debug_pr_tests(const mc_graph* g, void* stream, int64_t lhat, int32_t max_deg, uint8_t* flags);

/* Test hook for the contraction step alone (section "Parallel Graph
 * Contraction"): labels (DEVICE int32[n], values in [0, n_new)) name each
 * vertex's block; the contracted graph (one vertex per block, parallel
 * edges summed, internal edges dropped, rows sorted by neighbour) is written
 * to row_ptr_out (DEVICE int64[n_new+1]), col_out and w_out (DEVICE int32,
 * at least g->nnz entries); *nnz_out (HOST) receives its entry count.
 * MC_EINVAL for a null pointer, n_new < 1, a row_ptr that does not rise
 * from 0 to nnz, a col outside [0, n) or a weight below 1 (checked before
 * any kernel indexes by col); the labels are not checked. */
int mc_debug_contract(const mc_graph* g, const int32_t* labels, int32_t n_new, void* stream,
                      int64_t* row_ptr_out, int32_t* col_out, int32_t* w_out, int64_t* nnz_out);

/* Device bytes the workspace needs for a packed problem of this size. */
size_t mc_workspace_bytes(int32_t n_total, int64_t nnz_total, int32_t num_graphs);

/* Additional device bytes held once the clustering bound has run
 * (use_viecut or mc_viecut_bound): two level graphs and their labels. */
size_t mc_viecut_workspace_bytes(int32_t n_total, int64_t nnz_total, int32_t num_graphs);

/* For callers that cannot allocate device or pinned host memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): mc_mincut with side, lambda and options as there, but the
 * workspace is a fixed 64 MiB array in the library's code object (one per
 * device, held until the process ends) and the host staging is static, so
 * the call allocates nothing (no hipMalloc, hipHostMalloc, hipFree, no
 * event).  Limits: mc_workspace_bytes(n, nnz, 1) <= 64 MiB (else
 * MC_ETOOBIG, before any device work); opt->use_viecut and opt->workspace
 * must be 0 (else MC_EINVAL); opt->timing is ignored.  Every call on a
 * device uses that device's one array: calls on one device take turns (a
 * lock), and the array keeps the last call's contents, which no call reads
 * before writing.  Other errors as mc_mincut. */
int mc_mincut_noalloc(const mc_graph* g, void* stream, const mc_options* opt, int64_t* lambda,
                      uint8_t* side);

/* Free the cached workspaces of every stream of the current device
 * (waiting for a call in progress on one to finish). */
void mc_release(void);

const char* mc_strerror(int code);

/* ---------------------------------------------------------- served form
 * A request loop with continuous batching (no counterpart in the paper; the
 * solver underneath is the same).  Requests are host CSRs of single graphs
 * (same layout and rules as mc_graph, 0-based ids).  `lanes` host threads,
 * each with its own HIP stream and workspace, take requests from a FIFO
 * queue while their device footprint fits mem_budget: a request with more
 * than small_max_nnz entries runs alone, a run of smaller ones is packed
 * into one mc_mincut_batched-style solve (at most max_batch graphs).  Lanes
 * run concurrently, so newly arrived requests start while earlier ones are
 * still on the GPU.  A request's lambda does not depend on its batch.
 * Timing (mc_options.timing) is per host thread and ignored by the lanes. */
typedef struct mc_server mc_server;

typedef struct mc_server_cfg {
  int32_t lanes;           /* concurrent solves; default 4 */
  int32_t max_batch;       /* graphs per packed solve; default 4096 */
  int64_t small_max_nnz;   /* larger requests run alone; default 2^25 (large
                              graphs packed together are swept at once, one
                              workgroup each) */
  int64_t max_batch_nnz;   /* entries per packed solve (a run of small requests
                              stops before passing it); default 2^26 */
  int64_t mem_budget;      /* device bytes of the requests in flight (input,
                              side and solver workspace share); 0 = half of
                              the free memory at creation */
  int32_t queue_cap;       /* waiting requests before MC_EBUSY; default 65536 */
  int32_t device;          /* HIP device; -1 = the current one */
  int32_t validate;        /* 1 (default): check every request while its lane
                              packs it (row_ptr, columns, weights, total) */
  int32_t reserved;
  mc_options opt;          /* solver options of every solve */
} mc_server_cfg;

typedef struct mc_request {
  int32_t n;
  int32_t borrow;          /* 1: the server reads the caller's arrays, which
                              must stay valid until mc_server_wait returns;
                              0: they are copied on submit */
  int64_t nnz;
  const int64_t* row_ptr;  /* HOST, n + 1 */
  const int32_t* col;      /* HOST, nnz */
  const int32_t* w;        /* HOST, nnz */
} mc_request;

typedef struct mc_latency {
  double queue_ms;         /* submit -> admitted by a lane */
  double solve_ms;         /* admitted -> result on the host (upload, solve, side) */
  double total_ms;         /* submit -> result */
  int32_t batch_graphs;    /* graphs in the packed solve it ran in */
  int32_t lane;
} mc_latency;

void mc_server_cfg_default(mc_server_cfg* cfg);

/* Start the lanes.  *out receives the server.  MC_EINVAL for a bad
 * configuration, MC_EHIP if the device is unusable. */
int mc_server_create(const mc_server_cfg* cfg, mc_server** out);

/* Queue one request; *ticket identifies it.  MC_ENOCUT (n < 2), MC_EINVAL
 * (null array, nnz < 0), MC_ENOMEM (footprint above the budget), MC_EBUSY
 * (queue full), MC_ESTATE (server stopping).  A malformed graph is found
 * while it is packed: its mc_server_wait returns MC_EINVAL or MC_EOVERFLOW
 * and the requests batched with it are unaffected. */
int mc_server_submit(mc_server* srv, const mc_request* req, uint64_t* ticket);

/* Block until the request is done; lambda (HOST), side (HOST uint8[n] or
 * NULL; side[0] = 0) and lat (or NULL) receive its result.  The ticket is
 * released.  MC_ESTATE for an unknown ticket or one another thread is
 * already waiting on; otherwise the solve's code. */
int mc_server_wait(mc_server* srv, uint64_t ticket, int64_t* lambda, uint8_t* side, mc_latency* lat);

/* Finish every queued request, stop the lanes and free the server.
 * Results not collected by mc_server_wait are dropped. */
int mc_server_destroy(mc_server* srv);

/* Kernel-class timing, filled when mc_options.timing = 1: launches, summed
 * device time (HIP events on the launch stream) and algorithmic bytes. */
typedef struct mc_timing_entry {
  char name[24];
  int64_t launches;
  double ms;
  double algo_bytes;
} mc_timing_entry;

/* Copies up to `max` entries; returns how many classes exist.  The events
 * of timed solves are read here (waiting for them), not at the end of each
 * solve, so a timed loop pays only for recording them.  Per host thread. */
int mc_timing_get(mc_timing_entry* out, int max);
/* Reads any pending events, then clears the classes. */
void mc_timing_reset(void);
/* Time only the class `name` (NULL or "" = every class), for the calling
 * thread: a timed loop then records two events per launch of that class
 * and none for the others. */
void mc_timing_focus(const char* name);

#ifdef __cplusplus
}
#endif
#endif /* MINCUT_H */
