// Request server: keeps many matrices' factors resident on one GPU and runs
// their update requests with continuous batching.  A scheduler thread admits
// requests in arrival order whenever a slot is free and the slot workspaces
// in use stay within the device budget (the footprint of a request is the
// exact workspace its update carves); requests of one matrix run in
// submission order, one at a time; requests of different matrices run on
// their matrices' own streams and overlap on the device.  Cooperative kernels
// (which need all their blocks resident at once) are chained through one
// event so that two of them never run together.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/svlcov.h"
#include "kernels.hpp"
#include "state.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct HostCsr {   // owned copy of a host CSR input
  svlcov_csr c{};
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<char> v;
};

struct Req {
  int64_t ticket = 0;
  int32_t mid = 0;
  svlcov_state *h = nullptr;
  int32_t op = 0;
  HostCsr A, B;
  size_t bytes = 0;
  Clock::time_point t_submit;
  hipEvent_t done = nullptr;
  int slot = -1;
};

struct Slot {
  svl_state::DevBuf ws, stage;
  bool busy = false;
};

struct Mat {
  svlcov_state *h = nullptr;
  bool inflight = false;
};

struct Result {
  bool done = false;
  svlcov_status st = SVLCOV_OK;
  double lat_ms = 0.0;
};

size_t csr_bytes(const svlcov_csr &c) {
  if (c.on_device) return 0;
  const size_t vb = c.val_dtype == SVLCOV_F64 ? 8 : 4;
  return ((size_t)(c.rows + 1) * 8 + 255) / 256 * 256 + ((size_t)c.nnz * 4 + 255) / 256 * 256 +
         ((size_t)c.nnz * vb + 255) / 256 * 256 + 512;
}

svlcov_status copy_csr(const svlcov_csr *in, HostCsr *out) {
  if (!in || in->rows < 0 || in->cols < 0 || in->nnz < 0) return SVLCOV_E_INVALID;
  if (in->val_dtype != SVLCOV_F32 && in->val_dtype != SVLCOV_F64) return SVLCOV_E_INVALID;
  out->c = *in;
  if (in->on_device) return SVLCOV_OK;   // the caller keeps device inputs alive
  if (!in->row_ptr || (in->nnz > 0 && (!in->col_idx || !in->val))) return SVLCOV_E_INVALID;
  const size_t vb = in->val_dtype == SVLCOV_F64 ? 8 : 4;
  out->rp.assign(in->row_ptr, in->row_ptr + in->rows + 1);
  out->ci.assign(in->col_idx, in->col_idx + in->nnz);
  out->v.resize((size_t)in->nnz * vb);
  if (in->nnz > 0) std::memcpy(out->v.data(), in->val, out->v.size());
  out->c.row_ptr = out->rp.data();
  out->c.col_idx = out->ci.data();
  out->c.val = out->v.data();
  return SVLCOV_OK;
}

}  // namespace

struct svlcov_server {
  int device = 0;
  size_t budget = 0;
  std::vector<Slot> slots;
  std::deque<Mat> mats;   // stable element addresses while matrices are attached
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> pending;
  std::vector<Req *> inflight;
  std::unordered_map<int64_t, Result> results;
  std::vector<hipEvent_t> evpool;
  int64_t next_ticket = 1;
  size_t inflight_bytes = 0;
  bool stop = false;
  std::thread worker;
  // admitted requests are enqueued by a pool of dispatch threads: an update
  // waits on the host where it reads the subspace iteration's control
  // scalars, and one thread would serialise the requests there
  std::vector<std::thread> dispatchers;
  std::deque<Req *> to_dispatch;
  std::condition_variable cv_disp;
  hipEvent_t coop_chain = nullptr;
  bool coop_live = false;
  std::mutex coop_mu;
  svlcov_server_stats stats{};
  // fused projections: the server's stream, the descriptor table (pinned
  // staging and device copy) and the timing events of each fused launch
  hipStream_t stream = nullptr;
  char *desc_host = nullptr;   // packed fused batch (pinned staging), bytes
  size_t desc_host_cap = 0;
  char *desc_dev = nullptr;
  size_t desc_dev_cap = 0;
  hipEvent_t desc_copy_ev = nullptr, proj_ev = nullptr;
  bool desc_copy_live = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> fused_ev;
};

namespace {

void complete(svlcov_server *srv, Req *r, svlcov_status st) {
  const double ms =
      std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
  std::lock_guard<std::mutex> lk(srv->mu);
  if (r->slot >= 0) {
    srv->slots[r->slot].busy = false;
    srv->inflight_bytes -= r->bytes;
  }
  srv->mats[r->mid].inflight = false;
  Result &res = srv->results[r->ticket];
  res.done = true;
  res.st = st;
  res.lat_ms = ms;
  srv->stats.completed += 1;
  if (st != SVLCOV_OK) srv->stats.failed += 1;
  if (r->done) srv->evpool.push_back(r->done);
  delete r;
  srv->cv_done.notify_all();
}

// Fused projection: the first step of every admitted update whose inputs
// are device-resident (and not re-validated on the device) runs as one
// launch over all of them on the server's stream, writing C', its FP32 copy
// and the row norms straight into each request's slot workspace at the
// offsets the update will carve; each matrix's stream then waits for it and
// the update skips its own projection.
void fuse_projections(svlcov_server *srv, const std::vector<Req *> &admit) {
  std::vector<svl::ProjDesc> d;
  std::vector<std::pair<Req *, int>> users;   // request, number of sides
  for (Req *r : admit) {
    svlcov_state *h = r->h;
    if (h->validate || !r->A.c.on_device || (r->op == 2 && !r->B.c.on_device)) continue;
    const int64_t s = r->A.c.rows;
    const bool shape_ok =
        r->op == 0 ? r->A.c.cols == h->n
        : r->op == 1 ? r->A.c.cols == h->m
        : (r->B.c.rows == s && r->A.c.cols == h->m && r->B.c.cols == h->n);
    if (!shape_ok || s <= 0 || h->k + s > svl::eig_max_n() || s > svl::gram_max_rows()) continue;
    Slot &sl = srv->slots[r->slot];
    const size_t need = svl_state::op_workspace_bytes(r->op, h->k, s, r->A.c.nnz,
                                                      r->op == 2 ? r->B.c.nnz : 0);
    if (sl.ws.bytes < need) {   // the same growth rule as the update's own
      if (sl.ws.p) (void)hipFreeAsync(sl.ws.p, srv->stream);
      sl.ws = svl_state::DevBuf{};
      const size_t want = need + need / 4 + 4096;
      if (hipMallocAsync(&sl.ws.p, want, srv->stream) != hipSuccess) {
        (void)hipGetLastError();
        sl.ws.p = nullptr;
        continue;
      }
      sl.ws.bytes = want;
    }
    const int sides = r->op == 2 ? 2 : 1;
    for (int q = 0; q < sides; ++q) {
      // add rows projects on V, add columns on U; weights: D on U, E_m on V
      const bool onU = r->op == 1 || (r->op == 2 && q == 0);
      const svlcov_csr &E = q == 0 ? r->A.c : r->B.c;
      size_t o64, o32, orn;
      svl_state::proj_offsets(r->op, h->k, s, q, &o64, &o32, &orn);
      char *ws = (char *)sl.ws.p;
      svl::ProjDesc x;
      x.row_ptr = E.row_ptr;
      x.col_idx = E.col_idx;
      x.val = E.val;
      x.base = onU ? h->Ubase : h->Vbase;
      x.W = onU ? h->WU : h->WV;
      x.Cp64 = (double *)(ws + o64);
      x.Cp32 = h->prec == SVLCOV_FP64 ? nullptr : (float *)(ws + o32);
      x.rown = (double *)(ws + orn);
      x.info = h->info;
      x.s = s;
      x.row0 = 0;
      x.nnz = E.nnz;
      x.vdtype = E.val_dtype;
      x.K = h->k;
      x.fp64 = h->prec == SVLCOV_FP64 ? 1 : 0;
      x.pad = 0;
      d.push_back(x);
    }
    users.push_back({r, sides});
  }
  if (d.empty()) return;
  const svl::ProjBatch pb = svl::spmm_batch_prepare(std::move(d));
  const size_t bytes = pb.bytes();
  // the pinned staging blob is reused once the previous copy has read it
  if (srv->desc_copy_live) (void)hipEventSynchronize(srv->desc_copy_ev);
  if (srv->desc_host_cap < bytes) {
    if (srv->desc_host) (void)hipHostFree(srv->desc_host);
    srv->desc_host = nullptr;
    srv->desc_host_cap = 0;
    if (hipHostMalloc((void **)&srv->desc_host, bytes * 2) != hipSuccess) {
      srv->desc_host = nullptr;
      return;
    }
    srv->desc_host_cap = bytes * 2;
  }
  if (srv->desc_dev_cap < bytes) {
    if (srv->desc_dev) (void)hipFreeAsync(srv->desc_dev, srv->stream);
    srv->desc_dev = nullptr;
    srv->desc_dev_cap = 0;
    if (hipMallocAsync((void **)&srv->desc_dev, bytes * 2, srv->stream) != hipSuccess) {
      srv->desc_dev = nullptr;
      return;
    }
    srv->desc_dev_cap = bytes * 2;
  }
  pb.pack(srv->desc_host);
  if (hipMemcpyAsync(srv->desc_dev, srv->desc_host, bytes, hipMemcpyHostToDevice,
                     srv->stream) != hipSuccess)
    return;
  (void)hipEventRecord(srv->desc_copy_ev, srv->stream);
  srv->desc_copy_live = true;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  if (t0) (void)hipEventRecord(t0, srv->stream);
  svl::spmm_batch(srv->stream, pb, srv->desc_dev);
  if (hipGetLastError() != hipSuccess) return;   // the updates project on their own
  if (t1) (void)hipEventRecord(t1, srv->stream);
  if (t0 && t1) srv->fused_ev.push_back({t0, t1});
  (void)hipEventRecord(srv->proj_ev, srv->stream);
  for (auto &u : users) {
    svlcov_state *h = u.first->h;
    (void)hipStreamWaitEvent(h->stream, srv->proj_ev, 0);
    for (int q = 0; q < u.second; ++q) h->proj_ready[q] = true;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->stats.fused_launches += 1;
  srv->stats.fused_requests += (int64_t)users.size();
}

// Enqueue one admitted request on its matrix's stream with the slot's
// workspace lent to the state for the call.
void dispatch(svlcov_server *srv, Req *r) {
  svlcov_state *h = r->h;
  Slot &sl = srv->slots[r->slot];
  std::swap(h->ws, sl.ws);
  std::swap(h->stage, sl.stage);
  h->lent = true;
  svlcov_status st;
  if (r->op == 0) st = svlcov_add_rows(h, &r->A.c);
  else if (r->op == 1) st = svlcov_add_cols(h, &r->A.c);
  else st = svlcov_update_weights(h, &r->A.c, &r->B.c);
  h->lent = false;
  std::swap(h->ws, sl.ws);
  std::swap(h->stage, sl.stage);
  if (st == SVLCOV_OK && hipEventRecord(r->done, h->stream) != hipSuccess) st = SVLCOV_E_DEVICE;
  if (st != SVLCOV_OK) {
    complete(srv, r, st);
    return;
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->inflight.push_back(r);
  }
  srv->cv_work.notify_one();
}

void dispatch_loop(svlcov_server *srv) {
  (void)hipSetDevice(srv->device);
  for (;;) {
    Req *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv_disp.wait(lk, [&] { return srv->stop || !srv->to_dispatch.empty(); });
      if (srv->to_dispatch.empty()) break;   // stop, and nothing left
      r = srv->to_dispatch.front();
      srv->to_dispatch.pop_front();
    }
    dispatch(srv, r);
  }
}

void worker_loop(svlcov_server *srv) {
  (void)hipSetDevice(srv->device);
  std::vector<char> blocked;
  for (;;) {
    std::vector<Req *> admit;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      if (srv->pending.empty() && srv->inflight.empty()) {
        if (srv->stop && srv->stats.completed == srv->stats.submitted) break;
        // new requests, or a dispatched one that now awaits completion
        srv->cv_work.wait_for(lk, std::chrono::milliseconds(5), [&] {
          return srv->stop || !srv->pending.empty() || !srv->inflight.empty();
        });
        if (srv->stop && srv->pending.empty() && srv->inflight.empty() &&
            srv->stats.completed == srv->stats.submitted)
          break;
      }
      // admission in arrival order; a matrix whose earlier request waits
      // blocks its later ones
      blocked.assign(srv->mats.size(), 0);
      // admitted and not completed: in flight, or still being dispatched
      size_t nin = 0;
      for (const Slot &sl : srv->slots) nin += sl.busy ? 1 : 0;
      for (auto it = srv->pending.begin(); it != srv->pending.end();) {
        Req *r = *it;
        Mat &m = srv->mats[r->mid];
        if (m.inflight || blocked[r->mid]) {
          blocked[r->mid] = 1;
          ++it;
          continue;
        }
        int free_slot = -1;
        for (size_t q = 0; q < srv->slots.size(); ++q)
          if (!srv->slots[q].busy) { free_slot = (int)q; break; }
        if (free_slot < 0) break;
        if (nin + admit.size() > 0 && srv->inflight_bytes + r->bytes > srv->budget) {
          blocked[r->mid] = 1;
          ++it;
          continue;
        }
        r->slot = free_slot;
        r->h = m.h;
        srv->slots[free_slot].busy = true;
        srv->inflight_bytes += r->bytes;
        m.inflight = true;
        if (!srv->evpool.empty()) {
          r->done = srv->evpool.back();
          srv->evpool.pop_back();
        }
        admit.push_back(r);
        it = srv->pending.erase(it);
      }
      const size_t now_in = nin + admit.size();
      if ((int64_t)now_in > srv->stats.peak_inflight) srv->stats.peak_inflight = (int64_t)now_in;
      if ((int64_t)srv->inflight_bytes > srv->stats.peak_workspace_bytes)
        srv->stats.peak_workspace_bytes = (int64_t)srv->inflight_bytes;
    }
    if (!admit.empty()) fuse_projections(srv, admit);
    {
      std::vector<Req *> ready;
      for (Req *r : admit) {
        if (!r->done && hipEventCreateWithFlags(&r->done, hipEventDisableTiming) != hipSuccess) {
          r->done = nullptr;
          complete(srv, r, SVLCOV_E_DEVICE);
          continue;
        }
        ready.push_back(r);
      }
      if (!ready.empty()) {
        {
          std::lock_guard<std::mutex> lk(srv->mu);
          for (Req *r : ready) srv->to_dispatch.push_back(r);
        }
        srv->cv_disp.notify_all();
      }
    }
    // completions
    std::vector<Req *> finished;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      for (auto it = srv->inflight.begin(); it != srv->inflight.end();) {
        if (hipEventQuery((*it)->done) == hipSuccess) {
          finished.push_back(*it);
          it = srv->inflight.erase(it);
        } else {
          ++it;
        }
      }
    }
    for (Req *r : finished) {
      // the update's device-side status (and roll-back on failure)
      const svlcov_status st = svlcov_sync(r->h);
      complete(srv, r, st);
    }
    if (admit.empty() && finished.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

void svlcov_server_default_options(svlcov_server_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->device = 0;
  o->max_inflight = 8;
  o->workspace_budget = (int64_t)8 << 30;
}

svlcov_status svlcov_server_create(svlcov_server **out, const svlcov_server_options *opt) {
  if (!out) return SVLCOV_E_INVALID;
  *out = nullptr;
  svlcov_server_options o;
  if (opt) o = *opt; else svlcov_server_default_options(&o);
  if (o.max_inflight < 1 || o.max_inflight > 64 || o.workspace_budget < 0)
    return SVLCOV_E_INVALID;
  svlcov_server *srv = new (std::nothrow) svlcov_server();
  if (!srv) return SVLCOV_E_NOMEM;
  srv->device = o.device;
  srv->budget = o.workspace_budget > 0 ? (size_t)o.workspace_budget : (size_t)8 << 30;
  srv->slots.resize((size_t)o.max_inflight);
  if (hipSetDevice(srv->device) != hipSuccess ||
      hipEventCreateWithFlags(&srv->coop_chain, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&srv->desc_copy_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&srv->proj_ev, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess) {
    delete srv;
    return SVLCOV_E_DEVICE;
  }
  srv->worker = std::thread(worker_loop, srv);
  const int nd = o.max_inflight < 16 ? o.max_inflight : 16;
  for (int q = 0; q < nd; ++q) srv->dispatchers.emplace_back(dispatch_loop, srv);
  *out = srv;
  return SVLCOV_OK;
}

svlcov_status svlcov_server_attach(svlcov_server *srv, svlcov_state *h, int32_t *matrix_id) {
  if (!srv || !h || !matrix_id) return SVLCOV_E_INVALID;
  if (h->device != srv->device || h->coop_chain) return SVLCOV_E_INVALID;
  const svlcov_status st = svlcov_sync(h);
  if (st != SVLCOV_OK) return st;
  std::lock_guard<std::mutex> lk(srv->mu);
  // the state's own workspaces are not needed any more: requests borrow a slot's
  svl_state::release(h, h->ws);
  svl_state::release(h, h->stage);
  (void)hipStreamSynchronize(h->stream);
  h->coop_chain = &srv->coop_chain;
  h->coop_chain_live = &srv->coop_live;
  h->coop_mu = &srv->coop_mu;
  *matrix_id = (int32_t)srv->mats.size();
  srv->mats.push_back(Mat{h, false});
  return SVLCOV_OK;
}

svlcov_status svlcov_server_submit(svlcov_server *srv, int32_t matrix_id, int32_t op,
                                   const svlcov_csr *A, const svlcov_csr *B, int64_t *ticket) {
  if (!srv || !ticket || op < 0 || op > 2) return SVLCOV_E_INVALID;
  Req *r = new (std::nothrow) Req();
  if (!r) return SVLCOV_E_NOMEM;
  svlcov_status st = copy_csr(A, &r->A);
  if (st == SVLCOV_OK && op == 2) st = copy_csr(B, &r->B);
  if (st != SVLCOV_OK) {
    delete r;
    return st;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (matrix_id < 0 || (size_t)matrix_id >= srv->mats.size() || srv->stop) {
    delete r;
    return SVLCOV_E_INVALID;
  }
  const svlcov_state *h = srv->mats[matrix_id].h;
  r->mid = matrix_id;
  r->op = op;
  r->bytes = svl_state::op_workspace_bytes(op, h->k, r->A.c.rows, r->A.c.nnz,
                                            op == 2 ? r->B.c.nnz : 0) +
             csr_bytes(r->A.c) + (op == 2 ? csr_bytes(r->B.c) : 0);
  r->t_submit = Clock::now();
  r->ticket = srv->next_ticket++;
  *ticket = r->ticket;
  srv->results[r->ticket] = Result{};
  srv->pending.push_back(r);
  srv->stats.submitted += 1;
  srv->cv_work.notify_one();
  return SVLCOV_OK;
}

svlcov_status svlcov_server_poll(svlcov_server *srv, int64_t ticket, int32_t *done,
                                 svlcov_status *result, double *latency_ms) {
  if (!srv || !done) return SVLCOV_E_INVALID;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->results.find(ticket);
  if (it == srv->results.end()) return SVLCOV_E_INVALID;
  *done = it->second.done ? 1 : 0;
  if (it->second.done) {
    if (result) *result = it->second.st;
    if (latency_ms) *latency_ms = it->second.lat_ms;
    srv->results.erase(it);
  }
  return SVLCOV_OK;
}

svlcov_status svlcov_server_wait(svlcov_server *srv, int64_t ticket, svlcov_status *result,
                                 double *latency_ms) {
  if (!srv) return SVLCOV_E_INVALID;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->results.find(ticket);
  if (it == srv->results.end()) return SVLCOV_E_INVALID;
  srv->cv_done.wait(lk, [&] { return srv->results[ticket].done; });
  it = srv->results.find(ticket);
  if (result) *result = it->second.st;
  if (latency_ms) *latency_ms = it->second.lat_ms;
  srv->results.erase(it);
  return SVLCOV_OK;
}

svlcov_status svlcov_server_drain(svlcov_server *srv) {
  if (!srv) return SVLCOV_E_INVALID;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->pending.empty() && srv->inflight.empty() &&
                                     srv->stats.completed == srv->stats.submitted; });
  return SVLCOV_OK;
}

svlcov_status svlcov_server_get_stats(svlcov_server *srv, svlcov_server_stats *out) {
  if (!srv || !out) return SVLCOV_E_INVALID;
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->stats;
  out->fused_ms = 0.0;
  for (auto &e : srv->fused_ev) {   // completed fused launches only
    float ms = 0.f;
    if (hipEventQuery(e.second) == hipSuccess && hipEventElapsedTime(&ms, e.first, e.second) ==
                                                     hipSuccess)
      out->fused_ms += ms;
  }
  return SVLCOV_OK;
}

void svlcov_server_destroy(svlcov_server *srv) {
  if (!srv) return;
  (void)svlcov_server_drain(srv);
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  srv->cv_disp.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  for (std::thread &t : srv->dispatchers)
    if (t.joinable()) t.join();
  (void)hipSetDevice(srv->device);
  for (Mat &m : srv->mats) {
    if (m.h->stream) (void)hipStreamSynchronize(m.h->stream);
    m.h->coop_chain = nullptr;
    m.h->coop_chain_live = nullptr;
    m.h->coop_mu = nullptr;
  }
  for (Slot &s : srv->slots) {
    if (s.ws.p) (void)hipFree(s.ws.p);
    if (s.stage.p) (void)hipFree(s.stage.p);
  }
  for (hipEvent_t e : srv->evpool) (void)hipEventDestroy(e);
  if (srv->stream) (void)hipStreamSynchronize(srv->stream);
  for (auto &e : srv->fused_ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (srv->desc_dev) (void)hipFree(srv->desc_dev);
  if (srv->desc_host) (void)hipHostFree(srv->desc_host);
  if (srv->coop_chain) (void)hipEventDestroy(srv->coop_chain);
  if (srv->desc_copy_ev) (void)hipEventDestroy(srv->desc_copy_ev);
  if (srv->proj_ev) (void)hipEventDestroy(srv->proj_ev);
  if (srv->stream) (void)hipStreamDestroy(srv->stream);
  delete srv;
}

}  // extern "C"
