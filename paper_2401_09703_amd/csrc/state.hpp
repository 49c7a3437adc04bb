// The factor state of one matrix (internal; shared by the update engine and
// the request server).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/svlcov.h"
#include "common.hpp"

namespace svl_state {

struct Snapshot {
  int seq;
  int64_t m, n;
};

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

struct EvRec {
  int ph;
  hipEvent_t a, b;
};

// Device workspace bytes of one update of the given form (op 0 add_rows,
// 1 add_cols, 2 update_weights) at rank K with s update rows.
size_t op_workspace_bytes(int op, int K, int64_t s, int64_t nnzA, int64_t nnzB);
// Offsets in that workspace of the projection outputs of side q (0: the
// sparse side of add rows / add cols, or D of a weight update; 1: E_m).
void proj_offsets(int op, int K, int64_t s, int q, size_t *cp64, size_t *cp32, size_t *rown);

}  // namespace svl_state

struct svlcov_state {
  // device allocator hooks (both set or both NULL; see svlcov_options)
  void *(*dev_alloc)(size_t, void *, void *) = nullptr;
  void (*dev_free)(void *, size_t, void *, void *) = nullptr;
  void *alloc_ctx = nullptr;
  // set by a request server while it lends its slot workspaces to the state:
  // a lent buffer that has to grow is replaced with the server's allocator
  // (plain stream-ordered HIP), never with the hooks
  bool lent = false;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // second stream of an append update (created on first use): the residual
  // Gram, its Cholesky and K run there while the eigensolver, which needs
  // only M, runs on `stream`; ev_fork / ev_join order the two
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int ncu = 0;   // compute units of the device (set with the side stream)
  int side_ok = 1;   // svlcov_options.side_stream
  int prec = SVLCOV_FP64;
  int k = 0;
  int64_t m = 0, n = 0;
  int64_t capU = 0, capV = 0;
  void *Ubase = nullptr, *Vbase = nullptr;  // double (FP64) or float
  double *WU = nullptr, *WV = nullptr, *sigma = nullptr;
  SvDevInfo *info = nullptr;
  unsigned *flags = nullptr;   // tridiagonalisation barrier flags
  unsigned epoch = 0;
  bool launch_failed = false;   // a cooperative launch was refused
  svl_state::DevBuf ws;        // update workspace
  svl_state::DevBuf stage;     // device copies of host CSR inputs
  svl_state::DevBuf outbuf;    // get_factors staging
  // realised factors for pair scores, U_base (W_U Sigma) and V_base W_V in
  // the storage type, valid while q_seq equals seq
  svl_state::DevBuf qU, qV, qW;
  int64_t q_seq = -1;
  double rank_tol = 0, cond_reset = 0;
  int validate = 1;
  int deterministic = 1;   // sparse row update without floating-point atomics
  int seq = 0;
  std::vector<svl_state::Snapshot> history;
  std::atomic<bool> busy{false};
  bool prof = false;
  uint32_t prof_mask = ~0u;   // phases timed while prof is set
  std::vector<svl_state::EvRec> recs;
  std::vector<hipEvent_t> evpool;
  // Set while a request server drives the state: every cooperative launch
  // first waits for *coop_chain and then re-records it, so that cooperative
  // kernels of different matrices never run at the same time (each needs all
  // of its blocks resident at once).  The server dispatches from several host
  // threads, so the wait, the launch and the re-record hold *coop_mu.
  hipEvent_t *coop_chain = nullptr;
  bool *coop_chain_live = nullptr;
  std::mutex *coop_mu = nullptr;
  // Set by a request server for the next update only: the projection of
  // side q (C', its FP32 copy and the row norms) is already in the lent
  // workspace, written by a fused multi-request launch.
  bool proj_ready[2] = {false, false};
  // pinned control words of the iterative eigensolver (allocated on first
  // use) and its counters: filter steps taken, runs handed to the direct
  // solver
  double *ctl_host = nullptr;
  int64_t iter_steps = 0, iter_fallbacks = 0, iter_runs = 0;
  double iter_flops = 0.0;
  size_t elem() const { return prec == SVLCOV_FP64 ? sizeof(double) : sizeof(float); }
};


namespace svl_state {
// Device memory owned by the state: through its hooks when set (and `hooks`),
// else stream-ordered HIP on the state's stream.
inline hipError_t state_alloc(svlcov_state *h, void **p, size_t bytes, bool hooks = true) {
  if (hooks && h->dev_alloc) {
    *p = h->dev_alloc(bytes, (void *)h->stream, h->alloc_ctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMallocAsync(p, bytes, h->stream);
}
inline void state_free(svlcov_state *h, void *p, size_t bytes, bool hooks = true) {
  if (!p) return;
  if (hooks && h->dev_free) h->dev_free(p, bytes, (void *)h->stream, h->alloc_ctx);
  else (void)hipFreeAsync(p, h->stream);
}
inline void release(svlcov_state *h, DevBuf &b) {
  state_free(h, b.p, b.bytes);
  b = DevBuf{};
}
}  // namespace svl_state

// Cooperative-launch ordering hooks (no-ops unless a server drives the state);
// st: the stream the cooperative kernel goes to (default the state's).
inline void coop_enter(svlcov_state *h, hipStream_t st = nullptr) {
  if (!st) st = h->stream;
  if (h->coop_mu) h->coop_mu->lock();
  if (h->coop_chain && *h->coop_chain_live) (void)hipStreamWaitEvent(st, *h->coop_chain, 0);
}
inline void coop_exit(svlcov_state *h, hipStream_t st = nullptr) {
  if (!st) st = h->stream;
  if (h->coop_chain) {
    (void)hipEventRecord(*h->coop_chain, st);
    *h->coop_chain_live = true;
  }
  if (h->coop_mu) h->coop_mu->unlock();
}
