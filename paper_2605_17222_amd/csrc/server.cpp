// Continuous-batching LT server (see the server section of ckks_lt.h).
//
// One worker thread per server.  Under the server mutex it retires finished
// batches (event query, or the simulated end time), expires queued requests
// past their limit, and forms new batches from the head of the queue while a
// stream slot is free and the batch's workspace fits in the arena (first fit
// over 256-byte granules).  The device work is enqueued with the mutex
// released, so submissions and polls never wait for it.  Only the worker
// launches and retires batches.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "host_util.hpp"
#include "internal.hpp"

namespace {

typedef std::chrono::steady_clock Clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

struct Ring {
  const ckks_params* params = nullptr;
  std::vector<int32_t> rot;
  std::vector<const uint64_t*> key;
  ckks_rotkeys keys{};
};

struct Request {
  uint64_t id = 0;
  int ring = 0;
  ckks_lt_item item{};
  std::vector<const uint64_t*> pts;  // own copy of the plaintext pointer array
  std::vector<const double*> slots;  // or of the slot-vector pointer array
  size_t ws_need = 0;                // simulated backend
  int status = CKKS_PENDING;
  double t_submit = 0, t_start = 0, t_done = 0;
};

struct Batch {
  std::vector<Request*> reqs;
  const ckks_params* params = nullptr;  // the ring's, captured under the mutex
  size_t off = 0, bytes = 0;  // arena range
  int slot = 0;               // stream slot
  hipEvent_t done = nullptr;
  double t_end_sim = 0;
};

// First-fit allocator over [0, size) in 256-byte granules.
struct Arena {
  size_t size = 0, peak = 0;
  std::map<size_t, size_t> used;  // offset -> bytes
  static size_t round(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~(size_t)255; }
  bool find(size_t bytes, size_t* off) const {
    size_t cur = 0;
    for (const auto& u : used) {
      if (u.first >= cur + bytes) break;
      cur = u.first + u.second;
    }
    if (cur + bytes > size) return false;
    *off = cur;
    return true;
  }
  bool fits(size_t bytes) const {
    size_t off;
    return find(round(bytes), &off);
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes);
    if (!find(bytes, off)) return false;
    used[*off] = bytes;
    peak = std::max(peak, in_use());
    return true;
  }
  void release(size_t off) { used.erase(off); }
  size_t in_use() const {
    size_t s = 0;
    for (const auto& u : used) s += u.second;
    return s;
  }
};

}  // namespace

struct ckks_server {
  ckks_server_cfg cfg{};
  int device = 0;
  uint8_t* arena_base = nullptr;
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<bool> slot_busy;
  std::deque<Ring> rings;  // deque: references stay valid as rings are added

  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> all;
  std::vector<Batch*> inflight;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread worker;

  long batches = 0, max_batch_seen = 0, max_inflight_seen = 0, completed = 0, failed = 0, rejected = 0;
  double t_first = 0, t_last = 0;

  bool simulated() const { return cfg.backend == CKKS_SERVER_SIMULATED; }
  int workspace(int ring, const std::vector<ckks_lt_item>& items, size_t sim_total, size_t* bytes) const;
  bool launch(Batch* b);
  void complete(Request* r, int status, double t);
  void retire(Batch* b, int status);
  Batch* form_batch();
  void run();
};

int ckks_server::workspace(int ring, const std::vector<ckks_lt_item>& items, size_t sim_total, size_t* bytes) const {
  if (simulated()) {
    *bytes = sim_total;
    return CKKS_OK;
  }
  return ckks_lt_batch_workspace_size(rings[ring].params, (int)items.size(), items.data(), CKKS_LT_TH_BSGS, bytes);
}

void ckks_server::complete(Request* r, int status, double t) {
  r->status = status;
  r->t_done = t;
  t_last = std::max(t_last, t);
  if (status == CKKS_OK)
    ++completed;
  else
    ++failed;
}

// Enqueues a batch on its stream (mutex released: touches only the batch).
bool ckks_server::launch(Batch* b) {
  if (simulated()) {
    b->t_end_sim = now_s() + cfg.simulated_service_s * (1.0 + 0.25 * (double)(b->reqs.size() - 1));
    return true;
  }
  std::vector<ckks_lt_item> items;
  for (Request* r : b->reqs) {
    items.push_back(r->item);
    items.back().status = CKKS_PENDING;  // not yet written by the call
  }
  const int e = ckks_lt_eval_batch(b->params, (int)items.size(), items.data(), CKKS_LT_TH_BSGS,
                                   arena_base + b->off, b->bytes, streams[b->slot]);
  for (size_t t = 0; t < items.size(); ++t) {
    // Each item carries its own result (an item whose arguments or keys fail
    // does not fail the others); an item the call never reached takes the
    // call's code.
    const int st = items[t].status;
    b->reqs[t]->item.status = st == CKKS_PENDING ? (e != CKKS_OK ? e : CKKS_E_DEVICE) : st;
    b->reqs[t]->item.out = items[t].out;  // level and scale set by the call
  }
  if (hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess) {
    b->done = nullptr;
    return false;
  }
  return hipEventRecord(b->done, streams[b->slot]) == hipSuccess;
}

void ckks_server::retire(Batch* b, int status) {
  const double t = now_s();
  for (Request* r : b->reqs) complete(r, status != CKKS_OK ? status : (simulated() ? CKKS_OK : r->item.status), t);
  if (b->done) (void)hipEventDestroy(b->done);
  arena.release(b->off);
  slot_busy[b->slot] = false;
}

// Forms one batch from the head of the queue: requests of the head's ring,
// in arrival order, while the batch's workspace fits in the arena.  Called
// with the mutex held; returns NULL when no batch can start now.
Batch* ckks_server::form_batch() {
  int slot = -1;
  for (size_t s = 0; s < slot_busy.size(); ++s)
    if (!slot_busy[s]) {
      slot = (int)s;
      break;
    }
  if (slot < 0 || queue.empty()) return nullptr;
  const int ring = queue.front()->ring;
  std::vector<ckks_lt_item> trial;
  std::vector<Request*> take;
  size_t need = 0, sim_total = 0;
  for (Request* r : queue) {
    if ((int)take.size() >= cfg.max_batch) break;
    if (r->ring != ring) continue;
    trial.push_back(r->item);
    size_t bytes = 0;
    if (workspace(ring, trial, sim_total + r->ws_need, &bytes) != CKKS_OK || !arena.fits(bytes)) break;
    need = bytes;
    sim_total += r->ws_need;
    take.push_back(r);
  }
  if (take.empty()) return nullptr;  // the head waits for memory
  Batch* b = new Batch;
  b->slot = slot;
  b->reqs = take;
  b->params = rings[ring].params;
  b->bytes = Arena::round(need);
  arena.alloc(b->bytes, &b->off);
  slot_busy[slot] = true;
  for (Request* r : take) queue.erase(std::find(queue.begin(), queue.end(), r));
  const double t = now_s();
  for (Request* r : take) {
    r->t_start = t;
    r->status = CKKS_RUNNING;
  }
  ++batches;
  max_batch_seen = std::max<long>(max_batch_seen, (long)take.size());
  inflight.push_back(b);
  max_inflight_seen = std::max<long>(max_inflight_seen, (long)inflight.size());
  return b;
}

void ckks_server::run() {
  if (!simulated()) (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    // Retire finished batches.
    for (size_t i = 0; i < inflight.size();) {
      Batch* b = inflight[i];
      bool fin = false;
      int st = CKKS_OK;
      if (simulated()) {
        fin = now_s() >= b->t_end_sim;
      } else {
        const hipError_t q = hipEventQuery(b->done);
        if (q != hipErrorNotReady) fin = true, st = q == hipSuccess ? CKKS_OK : CKKS_E_DEVICE;
      }
      if (fin) {
        retire(b, st);
        delete b;
        inflight.erase(inflight.begin() + i);
      } else {
        ++i;
      }
    }
    // Expire queued requests past the limit.
    if (cfg.queue_timeout_s > 0) {
      const double t = now_s();
      for (auto it = queue.begin(); it != queue.end();) {
        if (t - (*it)->t_submit > cfg.queue_timeout_s) {
          complete(*it, CKKS_E_TIMEOUT, t);
          it = queue.erase(it);
        } else {
          ++it;
        }
      }
    }
    if (stop && queue.empty() && inflight.empty()) break;
    // Admit and launch.
    bool launched = false;
    while (Batch* b = form_batch()) {
      lk.unlock();
      const bool ok = launch(b);
      lk.lock();
      if (!ok) {
        // kernels of the batch may already be on the stream: its arena range
        // is released only once they have finished
        if (!simulated()) (void)hipStreamSynchronize(streams[b->slot]);
        retire(b, CKKS_E_DEVICE);
        inflight.erase(std::find(inflight.begin(), inflight.end(), b));
        delete b;
      }
      launched = true;
    }
    if (launched) continue;
    if (inflight.empty()) {
      if (cfg.queue_timeout_s > 0 && !queue.empty())
        cv.wait_for(lk, std::chrono::duration<double>(cfg.queue_timeout_s / 4));
      else
        cv.wait(lk, [&] { return stop || !queue.empty(); });
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      lk.lock();
    }
  }
}

extern "C" {

int ckks_server_create(const ckks_server_cfg* cfg, ckks_server** out) {
  if (!cfg || !out || cfg->max_batch < 1 || cfg->max_inflight < 1 || cfg->max_inflight > 16 ||
      cfg->hbm_budget_bytes == 0)
    return CKKS_E_INVALID_ARG;
  if (cfg->backend != CKKS_SERVER_DEVICE && cfg->backend != CKKS_SERVER_SIMULATED) return CKKS_E_INVALID_ARG;
  *out = nullptr;
  ckks_server* S = nullptr;
  try {
    S = new ckks_server;
    S->cfg = *cfg;
    S->arena.size = cfg->hbm_budget_bytes;
    S->slot_busy.assign(cfg->max_inflight, false);
    if (!S->simulated()) {
      if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return CKKS_E_DEVICE;
      }
      if (hipMalloc(&S->arena_base, cfg->hbm_budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        S->arena_base = nullptr;
        delete S;
        return CKKS_E_NOMEM;
      }
      for (int i = 0; i < cfg->max_inflight; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
          for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
          (void)hipFree(S->arena_base);
          delete S;
          return CKKS_E_DEVICE;
        }
        S->streams.push_back(s);
      }
    }
    S->worker = std::thread([S] { S->run(); });
    *out = S;
    return CKKS_OK;
  } catch (...) {
    if (S) {
      for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
      if (S->arena_base) (void)hipFree(S->arena_base);
      delete S;
    }
    return CKKS_E_NOMEM;
  }
}

int ckks_server_add_ring(ckks_server* S, const ckks_params* params, const ckks_rotkeys* keys, int* ring_id) {
  if (!S || !ring_id || (!params && !S->simulated()) || !keys || keys->count < 0 ||
      (keys->count > 0 && (!keys->rot || !keys->key)))
    return CKKS_E_INVALID_ARG;
  try {
    std::lock_guard<std::mutex> lk(S->mu);
    S->rings.emplace_back();
    Ring& R = S->rings.back();
    R.params = params;
    R.rot.assign(keys->rot, keys->rot + keys->count);
    R.key.assign(keys->key, keys->key + keys->count);
    R.keys.count = keys->count;
    R.keys.rot = R.rot.data();
    R.keys.key = R.key.data();
    R.keys.packed = keys->packed;
    *ring_id = (int)S->rings.size() - 1;
    return CKKS_OK;
  } catch (...) {
    return CKKS_E_NOMEM;
  }
}

int ckks_server_submit(ckks_server* S, const ckks_request* rq, uint64_t* id) {
  if (!S || !rq || !id || rq->ring < 0 || rq->diags.n_diag < 0 ||
      (rq->diags.n_diag > 0 && !rq->diags.pt && !rq->diags.slots) || (rq->diags.pt && rq->diags.slots))
    return CKKS_E_INVALID_ARG;
  Request* r = nullptr;
  try {
    r = new Request;
    r->ring = rq->ring;
    r->item.in = rq->in;
    r->item.diags = rq->diags;
    r->item.out = rq->out;
    r->item.status = CKKS_OK;
    if (rq->diags.pt) {
      r->pts.assign(rq->diags.pt, rq->diags.pt + rq->diags.n_diag);
      r->item.diags.pt = r->pts.data();
    } else if (rq->diags.slots) {
      r->slots.assign(rq->diags.slots, rq->diags.slots + rq->diags.n_diag);
      r->item.diags.slots = r->slots.data();
    }
    r->ws_need = rq->sim_ws_bytes;
    r->t_submit = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    if (rq->ring >= (int)S->rings.size()) {
      delete r;
      return CKKS_E_INVALID_ARG;
    }
    r->item.keys = &S->rings[rq->ring].keys;
    // Admission: the request's own workspace must fit the budget.
    size_t need = 0;
    const int e = S->workspace(rq->ring, std::vector<ckks_lt_item>{r->item}, r->ws_need, &need);
    if (e != CKKS_OK || Arena::round(need) > S->arena.size) {
      ++S->rejected;
      delete r;
      return e != CKKS_OK ? e : CKKS_E_WORKSPACE;
    }
    r->id = S->next_id++;
    if (S->t_first == 0) S->t_first = r->t_submit;
    S->all[r->id] = r;
    S->queue.push_back(r);
    *id = r->id;
    S->cv.notify_one();
    return CKKS_OK;
  } catch (...) {
    delete r;
    return CKKS_E_NOMEM;
  }
}

int ckks_server_poll(ckks_server* S, uint64_t id, int* status, double* latency_s) {
  if (!S || !status) return CKKS_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) return CKKS_E_INVALID_ARG;
  const Request* r = it->second;
  *status = r->status;
  if (latency_s) *latency_s = r->t_done > 0 ? r->t_done - r->t_submit : -1;
  return CKKS_OK;
}

int ckks_server_result(ckks_server* S, uint64_t id, ckks_ct* out) {
  if (!S || !out) return CKKS_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end() || it->second->t_done <= 0) return CKKS_E_INVALID_ARG;
  if (it->second->status != CKKS_OK) return it->second->status;
  *out = it->second->item.out;
  return CKKS_OK;
}

int ckks_server_cancel(ckks_server* S, uint64_t id) {
  if (!S) return CKKS_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(id);
  if (it == S->all.end()) return CKKS_E_INVALID_ARG;
  auto q = std::find(S->queue.begin(), S->queue.end(), it->second);
  if (q == S->queue.end()) return CKKS_E_INVALID_ARG;
  S->queue.erase(q);
  S->complete(it->second, CKKS_E_CANCELLED, now_s());
  return CKKS_OK;
}

int ckks_server_wait_all(ckks_server* S) {
  if (!S) return CKKS_E_INVALID_ARG;
  while (true) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->queue.empty() && S->inflight.empty()) return CKKS_OK;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
}

int ckks_server_stats(ckks_server* S, ckks_server_stat* st) {
  if (!S || !st) return CKKS_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  memset(st, 0, sizeof(*st));
  st->completed = S->completed;
  st->failed = S->failed;
  st->rejected = S->rejected;
  st->queued = (long)S->queue.size();
  for (const Batch* b : S->inflight) st->inflight += (long)b->reqs.size();
  st->batches = S->batches;
  st->max_batch = S->max_batch_seen;
  st->max_inflight = S->max_inflight_seen;
  st->arena_in_use = S->arena.in_use();
  st->arena_peak = S->arena.peak;
  std::vector<double> lat;
  for (const auto& kv : S->all)
    if (kv.second->t_done > 0 && kv.second->status == CKKS_OK) lat.push_back(kv.second->t_done - kv.second->t_submit);
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    // nearest-rank percentiles
    auto pct = [&](double p) {
      const size_t k = (size_t)ceil(p * (double)lat.size());
      return lat[std::min(lat.size(), std::max<size_t>(k, 1)) - 1];
    };
    st->p50_s = pct(0.50);
    st->p99_s = pct(0.99);
    double s = 0;
    for (double x : lat) s += x;
    st->mean_s = s / (double)lat.size();
  }
  st->span_s = S->t_last > S->t_first ? S->t_last - S->t_first : 0;
  return CKKS_OK;
}

void ckks_server_destroy(ckks_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  if (!S->simulated()) {
    for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
    if (S->arena_base) (void)hipFree(S->arena_base);
  }
  for (auto& kv : S->all) delete kv.second;
  delete S;
}

}  // extern "C"
