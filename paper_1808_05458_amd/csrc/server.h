// Served form: a request loop with continuous batching.
//
// Requests (host CSRs) wait in a FIFO queue.  Each lane is a host thread
// with its own HIP stream and solver workspace.  A free lane admits requests
// from the head of the queue while their device footprint fits the memory
// budget: a large request alone, or a run of small ones coalesced into one
// packed solve (the batched form) of bounded size.  Lanes run at the same
// time, so one lane packs on the host while another solves, and requests
// that arrive while others are on the GPU are admitted as soon as a lane
// and memory are free, and their kernels overlap on the device with the
// running solves.  Every graph's contraction state stays on the device for
// its whole solve; only lambda and the side come back.  A request's result
// does not depend on what it was batched with: every graph of a packed
// solve keeps its own bound, vertex range and scans.
#pragma once
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>

namespace mc {

struct ServerRequest {
  uint64_t ticket = 0;
  int32_t n = 0;
  int64_t nnz = 0;
  const int64_t* rp = nullptr;  // host; the caller's (borrowed) or `own_*`
  const int32_t* col = nullptr;
  const int32_t* w = nullptr;
  std::vector<int64_t> own_rp;
  std::vector<int32_t> own_col, own_w;
  int64_t bytes = 0;  // device footprint while in flight
  // result
  int rc = 1;  // 1 = pending
  int rc_pack = MC_OK;
  int64_t lambda = -1;
  std::vector<uint8_t> side;
  std::chrono::steady_clock::time_point t_submit, t_start, t_done;
  int32_t batch_graphs = 0, lane = -1;
  bool claimed = false;  // a waiter holds the ticket (a second waiter gets MC_ESTATE)
};

// Device and pinned host buffers of one lane, grown to the largest batch.
struct LaneBuffers {
  int64_t capN = 0, capE = 0;
  int64_t* rp = nullptr;
  int32_t *col = nullptr, *w = nullptr;
  uint8_t* side = nullptr;
  int64_t* h_rp = nullptr;  // pinned staging
  int32_t *h_col = nullptr, *h_w = nullptr;
  uint8_t* h_side = nullptr;

  void release() {
    if (rp) hipFree(rp);
    if (col) hipFree(col);
    if (w) hipFree(w);
    if (side) hipFree(side);
    if (h_rp) hipHostFree(h_rp);
    if (h_col) hipHostFree(h_col);
    if (h_w) hipHostFree(h_w);
    if (h_side) hipHostFree(h_side);
    *this = LaneBuffers{};
  }
  int ensure(int64_t N, int64_t E) {
    if (N <= capN && E <= capE) return MC_OK;
    release();
    // geometric growth: pinning and freeing are slow, so a lane settles on
    // its largest batch after a few reallocations
    N = std::max<int64_t>(N + N / 2, 1 << 16);
    E = std::max<int64_t>(E + E / 2, 1 << 20);
    if (hipMalloc(&rp, (N + 1) * 8) != hipSuccess || hipMalloc(&col, E * 4) != hipSuccess ||
        hipMalloc(&w, E * 4) != hipSuccess || hipMalloc(&side, N) != hipSuccess ||
        hipHostMalloc((void**)&h_rp, (N + 1) * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_col, E * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_w, E * 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h_side, N, hipHostMallocDefault) != hipSuccess) {
      release();
      return MC_ENOMEM;
    }
    capN = N;
    capE = E;
    return MC_OK;
  }
};

// Copy one request into the packed staging buffers at vertex offset v0 and
// entry offset e0 (columns shifted by v0, row offsets by e0), checking it on
// the way (the packed solve would reject the whole batch for one malformed
// graph): row_ptr monotone from 0 to nnz, columns in range, weights >= 1,
// total weight within 2 (2^31 - 1).  Returns MC_OK, or the error with the
// staging left to be overwritten by the next request.
inline int pack_request(const ServerRequest& r, int64_t v0, int64_t e0, bool check, int64_t* h_rp, int32_t* h_col,
                        int32_t* h_w) {
  const int32_t n = r.n;
  if (check && (r.rp[0] != 0 || r.rp[n] != r.nnz)) return MC_EINVAL;
  for (int32_t v = 0; v < n; ++v) {
    if (check && r.rp[v + 1] < r.rp[v]) return MC_EINVAL;
    h_rp[v0 + v] = r.rp[v] + e0;
  }
  int64_t total = 0;
  bool bad = false;
  for (int64_t e = 0; e < r.nnz; ++e) {
    const int32_t c = r.col[e], x = r.w[e];
    bad |= (c < 0) | (c >= n) | (x < 1);
    total += x;
    h_col[e0 + e] = c + (int32_t)v0;
    h_w[e0 + e] = x;
  }
  if (check && bad) return MC_EINVAL;
  if (check && total > 2ll * 2147483647ll) return MC_EOVERFLOW;
  return MC_OK;
}

struct Server {
  mc_server_cfg cfg;
  int device = 0;
  int64_t budget = 0;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<ServerRequest*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<ServerRequest>> reqs;
  uint64_t next_ticket = 1;
  int64_t in_flight = 0;
  bool stop = false;
  std::vector<std::thread> lanes;

  // Whether the queue head may start now: memory allows it, or nothing else
  // is in flight (a request larger than the budget is refused at submit).
  bool admissible() const {
    return !queue.empty() && (in_flight == 0 || in_flight + queue.front()->bytes <= budget);
  }

  void lane_main(int lane_id) {
    hipSetDevice(device);
    hipStream_t s = nullptr;
    hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    Workspace ws;
    LaneBuffers buf;
    std::vector<ServerRequest*> batch, kept;
    std::vector<int64_t> voff, lambdas;
    while (true) {
      batch.clear();
      {
        std::unique_lock<std::mutex> lk(m);
        cv_work.wait(lk, [&] { return admissible() || (stop && queue.empty()); });
        if (queue.empty()) break;  // stopping and drained
        ServerRequest* r0 = queue.front();
        queue.pop_front();
        batch.push_back(r0);
        in_flight += r0->bytes;
        if (r0->nnz <= cfg.small_max_nnz) {
          int64_t entries = r0->nnz;
          while (!queue.empty() && (int32_t)batch.size() < cfg.max_batch) {
            ServerRequest* r = queue.front();
            if (r->nnz > cfg.small_max_nnz || in_flight + r->bytes > budget ||
                entries + r->nnz > cfg.max_batch_nnz)
              break;
            entries += r->nnz;
            queue.pop_front();
            batch.push_back(r);
            in_flight += r->bytes;
          }
        }
      }
      const auto t_start = std::chrono::steady_clock::now();
      // pack and check in one pass; a malformed request is left out and
      // completes with its error
      int64_t N = 0, E = 0;
      for (const ServerRequest* r : batch) {
        N += r->n;
        E += r->nnz;
      }
      int rc = (N >= (1ll << 30) || E >= (int64_t)UINT32_MAX) ? MC_EINVAL : buf.ensure(N, E);
      voff.assign(1, 0);
      kept.clear();
      if (rc == MC_OK) {
        int64_t e0 = 0;
        for (ServerRequest* r : batch) {
          r->rc_pack = pack_request(*r, voff.back(), e0, cfg.validate != 0, buf.h_rp, buf.h_col, buf.h_w);
          if (r->rc_pack != MC_OK) continue;
          kept.push_back(r);
          voff.push_back(voff.back() + r->n);
          e0 += r->nnz;
        }
        N = voff.back();
        E = e0;
      }
      const int32_t G = (int32_t)kept.size();
      if (rc == MC_OK && G > 0) {
        buf.h_rp[N] = E;
        hipMemcpyAsync(buf.rp, buf.h_rp, (N + 1) * 8, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(buf.col, buf.h_col, E * 4, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(buf.w, buf.h_w, E * 4, hipMemcpyHostToDevice, s);
        Problem P{G, (int32_t)N, E, buf.rp, buf.col, buf.w, voff.data()};
        lambdas.assign(G, -1);
        rc = run_on(ws, P, s, &cfg.opt, lambdas.data(), buf.side, nullptr);
        if (rc == MC_OK) {
          if (hipMemcpyAsync(buf.h_side, buf.side, N, hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess)
            rc = MC_EHIP;
        }
      }
      const auto t_done = std::chrono::steady_clock::now();
      {
        std::lock_guard<std::mutex> lk(m);
        for (int32_t g = 0; g < G; ++g) {
          ServerRequest* r = kept[g];
          if (rc == MC_OK) {
            r->lambda = lambdas[g];
            r->side.assign(buf.h_side + voff[g], buf.h_side + voff[g + 1]);
          }
        }
        for (ServerRequest* r : batch) {
          r->rc = r->rc_pack != MC_OK ? r->rc_pack : rc;
          r->t_start = t_start;
          r->t_done = t_done;
          r->batch_graphs = G;
          r->lane = lane_id;
          in_flight -= r->bytes;
        }
      }
      cv_done.notify_all();
      cv_work.notify_all();  // memory freed: another lane may admit now
    }
    buf.release();
    ws.release();
    hipStreamDestroy(s);
  }
};

}  // namespace mc

extern "C" {

void mc_server_cfg_default(mc_server_cfg* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->lanes = 4;
  c->max_batch = 4096;
  c->small_max_nnz = 1ll << 25;
  c->max_batch_nnz = 1ll << 26;
  c->mem_budget = 0;
  c->queue_cap = 1 << 16;
  c->device = -1;
  c->validate = 1;
  mc_options_default(&c->opt);
}

int mc_server_create(const mc_server_cfg* cfg, mc_server** out) {
  if (!out) return MC_EINVAL;
  *out = nullptr;
  auto S = std::make_unique<mc::Server>();
  mc_server_cfg_default(&S->cfg);
  if (cfg) S->cfg = *cfg;
  mc_server_cfg& c = S->cfg;
  if (c.lanes < 1 || c.lanes > 64 || c.max_batch < 1 || c.small_max_nnz < 0 || c.max_batch_nnz < 1 ||
      c.queue_cap < 1)
    return MC_EINVAL;
  if (c.device < 0) {
    if (hipGetDevice(&S->device) != hipSuccess) return MC_EHIP;
  } else {
    S->device = c.device;
  }
  if (hipSetDevice(S->device) != hipSuccess) return MC_EHIP;
  S->budget = c.mem_budget;
  if (S->budget <= 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return MC_EHIP;
    S->budget = (int64_t)(free_b / 2);
  }
  for (int i = 0; i < c.lanes; ++i) S->lanes.emplace_back(&mc::Server::lane_main, S.get(), i);
  *out = reinterpret_cast<mc_server*>(S.release());
  return MC_OK;
}

int mc_server_submit(mc_server* srv, const mc_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket || !req->row_ptr || !req->col || !req->w) return MC_EINVAL;
  mc::Server* S = reinterpret_cast<mc::Server*>(srv);
  if (req->n < 2) return MC_ENOCUT;
  if (req->nnz < 0) return MC_EINVAL;
  auto r = std::make_unique<mc::ServerRequest>();
  r->n = req->n;
  r->nnz = req->nnz;
  if (req->borrow) {
    r->rp = req->row_ptr;
    r->col = req->col;
    r->w = req->w;
  } else {
    r->own_rp.assign(req->row_ptr, req->row_ptr + req->n + 1);
    r->own_col.assign(req->col, req->col + req->nnz);
    r->own_w.assign(req->w, req->w + req->nnz);
    r->rp = r->own_rp.data();
    r->col = r->own_col.data();
    r->w = r->own_w.data();
  }
  // input CSR, side, and the solver's share of a workspace (its size-
  // dependent part: the fixed part is held by each lane once)
  r->bytes = (int64_t)(req->n + 1) * 8 + req->nnz * 8 + req->n +
             (int64_t)(mc::workspace_bytes(req->n, req->nnz, 1) - mc::workspace_bytes(0, 0, 0));
  if (r->bytes > S->budget) return MC_ENOMEM;
  r->t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(S->m);
    if (S->stop) return MC_ESTATE;
    if ((int64_t)S->queue.size() >= S->cfg.queue_cap) return MC_EBUSY;
    r->ticket = S->next_ticket++;
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->reqs.emplace(r->ticket, std::move(r));
  }
  S->cv_work.notify_one();
  return MC_OK;
}

int mc_server_wait(mc_server* srv, uint64_t ticket, int64_t* lambda, uint8_t* side, mc_latency* lat) {
  if (!srv) return MC_EINVAL;
  mc::Server* S = reinterpret_cast<mc::Server*>(srv);
  std::unique_ptr<mc::ServerRequest> r;
  {
    std::unique_lock<std::mutex> lk(S->m);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second->claimed) return MC_ESTATE;
    mc::ServerRequest* p = it->second.get();
    p->claimed = true;  // only this waiter erases it, so p stays valid while waiting
    S->cv_done.wait(lk, [&] { return p->rc != 1; });
    // submits may have rehashed the map while this thread waited
    it = S->reqs.find(ticket);
    r = std::move(it->second);
    S->reqs.erase(it);
  }
  if (lat) {
    using ms = std::chrono::duration<double, std::milli>;
    lat->queue_ms = ms(r->t_start - r->t_submit).count();
    lat->solve_ms = ms(r->t_done - r->t_start).count();
    lat->total_ms = ms(r->t_done - r->t_submit).count();
    lat->batch_graphs = r->batch_graphs;
    lat->lane = r->lane;
  }
  if (r->rc != MC_OK) return r->rc;
  if (lambda) *lambda = r->lambda;
  if (side) std::memcpy(side, r->side.data(), r->side.size());
  return MC_OK;
}

int mc_server_destroy(mc_server* srv) {
  if (!srv) return MC_EINVAL;
  mc::Server* S = reinterpret_cast<mc::Server*>(srv);
  {
    std::lock_guard<std::mutex> lk(S->m);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->lanes) t.join();
  delete S;
  return MC_OK;
}

}  // extern "C"
