// Continuous-batching query server over one reference index.
//
// Requests (host query sets) are queued on submit. Each worker thread owns a
// context and a HIP stream; when idle it admits the queued requests in
// arrival order while their estimated device working memory fits the
// server's budget (counting the batches other workers have in flight), runs
// them as one batched query (one tile: the sets concatenated, one join pass
// over the index, per-set slices of the sorted result) and posts each
// request's result. Requests that arrive while a batch is on the GPU are
// picked up by the next idle worker, so batches overlap on the device. A
// request's result is its own slice of its batch, exactly what a query of
// that set alone returns.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sd_host.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  std::vector<uint8_t> codes;
  std::vector<int64_t> offsets;
  uint64_t est_bytes = 0;
  Clock::time_point t_submit;
  bool cancelled = false;
};

struct Result {
  int status = SD_OK;
  int64_t n = 0;
  uint32_t* i = nullptr;
  uint32_t* j = nullptr;
  uint8_t* d = nullptr;
  double latency_s = 0.0;
  int64_t batch_size = 0;
};

}  // namespace

struct sd_server {
  const sd_index* index = nullptr;
  int device = 0;
  sd_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Request*> running;  // admitted, not finished
  std::unordered_map<uint64_t, Result> done;
  uint64_t next_id = 1;
  uint64_t in_flight_bytes = 0;
  bool stopping = false;
  std::vector<std::thread> workers;
  // counters
  uint64_t n_batches = 0, n_requests_done = 0, max_batch = 0;
};

namespace {

// Working memory of one request on the device, by its variant count (the
// query elements twice, candidates and results with generous margins).
uint64_t estimate_bytes(const std::vector<int64_t>& offs, int k) {
  uint64_t keys = 0, n = offs.size() - 1;
  for (uint64_t x = 0; x < n; ++x) {
    const int64_t L = offs[x + 1] - offs[x];
    uint64_t v = 1;
    if (k >= 1) v += (uint64_t)L;
    if (k >= 2) v += (uint64_t)L * (uint64_t)(L - 1) / 2;
    keys += v;
  }
  return keys * 24 + n * 64 + (1u << 20);
}

void post(sd_server* sv, Request* r, const Result& res) {
  Result out = res;
  out.latency_s = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
  if (r->cancelled) {
    std::free(out.i);
    std::free(out.j);
    std::free(out.d);
    out = Result{};
    out.status = SD_E_CANCELLED;
  }
  sv->done[r->id] = out;
  sv->running.erase(r->id);
  delete r;
}

void worker_main(sd_server* sv) {
  sd_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  int init_rc = sd_create(&ctx, sv->device, 0);
  if (init_rc == SD_OK && hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    init_rc = SD_E_HIP;
  }
  for (;;) {
    std::vector<Request*> batch;
    uint64_t bytes = 0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] { return sv->stopping || !sv->pending.empty(); });
      if (sv->stopping && sv->pending.empty()) break;
      // admit in arrival order while the budget and the batch limit allow;
      // a request alone over the whole budget is rejected
      while (!sv->pending.empty()) {
        Request* r = sv->pending.front();
        if (r->cancelled) {
          sv->pending.pop_front();
          Result res;
          res.status = SD_E_CANCELLED;
          post(sv, r, res);
          continue;
        }
        const uint64_t budget = sv->cfg.hbm_budget;
        if (budget && r->est_bytes > budget) {
          sv->pending.pop_front();
          Result res;
          res.status = SD_E_NOMEM;
          post(sv, r, res);
          continue;
        }
        if (budget && sv->in_flight_bytes + bytes + r->est_bytes > budget) break;
        if (sv->cfg.max_batch_requests > 0 && (int)batch.size() >= sv->cfg.max_batch_requests) break;
        sv->pending.pop_front();
        sv->running[r->id] = r;
        batch.push_back(r);
        bytes += r->est_bytes;
      }
      if (batch.empty()) {  // budget held by other workers: wait for one to finish
        sv->cv_done.wait_for(lk, std::chrono::milliseconds(1));
        continue;
      }
      sv->in_flight_bytes += bytes;
    }
    // run the batch
    std::vector<sd_seqs> sets(batch.size());
    std::vector<sd_pairs> outs(batch.size());
    for (size_t x = 0; x < batch.size(); ++x) {
      Request* r = batch[x];
      sets[x] = sd_seqs{r->codes.data(), r->offsets.data(), (int64_t)r->offsets.size() - 1, 0};
      outs[x] = sd_pairs{};
      outs[x].on_device = 0;
    }
    int rc = init_rc;
    if (rc == SD_OK) {
      ctx->batch_tile_seqs = 0x7FFFFFFF;  // one tile: the whole admitted batch
      ctx->probe = sv->cfg.probe;
      if (sv->cfg.weighted)
        rc = sd_query_batch_weighted(ctx, sv->index, (int)batch.size(), sets.data(),
                                     sv->cfg.subst, sv->cfg.indel, sv->cfg.max_score, outs.data(),
                                     stream);
      else
        rc = sd_query_batch(ctx, sv->index, (int)batch.size(), sets.data(), sv->cfg.k,
                            outs.data(), stream);
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      for (size_t x = 0; x < batch.size(); ++x) {
        Result res;
        res.status = rc;
        res.batch_size = (int64_t)batch.size();
        if (rc == SD_OK) {
          // move the pinned result into malloc'd arrays owned by the caller
          const int64_t n = outs[x].n;
          res.n = n;
          res.i = static_cast<uint32_t*>(std::malloc(n ? n * 4 : 4));
          res.j = static_cast<uint32_t*>(std::malloc(n ? n * 4 : 4));
          res.d = static_cast<uint8_t*>(std::malloc(n ? n : 1));
          if (!res.i || !res.j || !res.d) {
            std::free(res.i);
            std::free(res.j);
            std::free(res.d);
            res = Result{};
            res.status = SD_E_NOMEM;
          } else if (n) {
            std::memcpy(res.i, outs[x].i, n * 4);
            std::memcpy(res.j, outs[x].j, n * 4);
            std::memcpy(res.d, outs[x].d, n);
          }
          sd_pairs_free(ctx, &outs[x]);
        }
        post(sv, batch[x], res);
      }
      sv->in_flight_bytes -= bytes;
      sv->n_batches += 1;
      sv->n_requests_done += batch.size();
      if (batch.size() > sv->max_batch) sv->max_batch = batch.size();
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
  if (stream) (void)hipStreamDestroy(stream);
  sd_destroy(ctx);
}

}  // namespace

extern "C" {

int sd_server_create(const sd_index* index, int device, const sd_server_config* cfg,
                     sd_server** out) {
  if (!index || !cfg || !out) return SD_E_INVAL;
  *out = nullptr;
  if (cfg->k < 0 || cfg->k > index->k || cfg->workers < 0 || cfg->workers > 16 ||
      cfg->probe < 0 || cfg->probe > 1)
    return SD_E_INVAL;
  if (device != index->device) return SD_E_INVAL;
  sd_server* sv = new (std::nothrow) sd_server();
  if (!sv) return SD_E_NOMEM;
  sv->index = index;
  sv->device = device;
  sv->cfg = *cfg;
  const int nw = cfg->workers ? cfg->workers : 2;
  try {
    for (int w = 0; w < nw; ++w) sv->workers.emplace_back(worker_main, sv);
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stopping = true;
    }
    sv->cv_work.notify_all();
    for (auto& t : sv->workers) t.join();
    delete sv;
    return SD_E_NOMEM;
  }
  *out = sv;
  return SD_OK;
}

int sd_server_submit(sd_server* sv, const sd_seqs* q, uint64_t* request_id) {
  if (!sv || !q || !request_id) return SD_E_INVAL;
  if (q->on_device) return SD_E_INVAL;
  if (q->n < 0 || (q->n > 0 && (!q->codes || !q->offsets))) return SD_E_INVAL;
  Request* r = new (std::nothrow) Request();
  if (!r) return SD_E_NOMEM;
  try {
    r->offsets.assign(q->offsets, q->offsets + q->n + 1);
    if (q->n == 0 && !q->offsets) r->offsets.assign(1, 0);
    const int64_t total = r->offsets.back();
    if (r->offsets[0] != 0 || total < 0) {
      delete r;
      return SD_E_INVAL;
    }
    for (int64_t x = 0; x < q->n; ++x)
      if (r->offsets[x + 1] < r->offsets[x]) {
        delete r;
        return SD_E_INVAL;
      }
    r->codes.assign(q->codes, q->codes + total);
    r->est_bytes = estimate_bytes(r->offsets, sv->cfg.k);
  } catch (...) {
    delete r;
    return SD_E_NOMEM;
  }
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) {
      delete r;
      return SD_E_STATE;
    }
    r->id = sv->next_id++;
    *request_id = r->id;
    sv->pending.push_back(r);
  }
  sv->cv_work.notify_one();
  return SD_OK;
}

int sd_server_poll(sd_server* sv, uint64_t request_id, int timeout_ms, sd_pairs* out,
                   double* latency_s) {
  if (!sv || !out) return SD_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  std::unique_lock<std::mutex> lk(sv->mu);
  auto ready = [&] { return sv->done.count(request_id) > 0; };
  if (!ready()) {
    bool known = request_id > 0 && request_id < sv->next_id;
    if (!known) return SD_E_INVAL;
    if (timeout_ms == 0) return SD_E_STATE;  // not finished yet
    if (timeout_ms < 0)
      sv->cv_done.wait(lk, ready);
    else if (!sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
      return SD_E_STATE;
  }
  Result res = sv->done[request_id];
  sv->done.erase(request_id);
  if (latency_s) *latency_s = res.latency_s;
  if (res.status != SD_OK) return res.status;
  out->n = res.n;
  out->i = res.i;
  out->j = res.j;
  out->d = res.d;
  out->on_device = 0;
  return SD_OK;
}

int sd_server_cancel(sd_server* sv, uint64_t request_id) {
  if (!sv) return SD_E_INVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  for (Request* r : sv->pending)
    if (r->id == request_id) {
      r->cancelled = true;
      return SD_OK;
    }
  auto it = sv->running.find(request_id);
  if (it != sv->running.end()) {
    it->second->cancelled = true;
    return SD_OK;
  }
  return sv->done.count(request_id) ? SD_E_STATE : SD_E_INVAL;
}

int sd_server_stats(sd_server* sv, int64_t* batches, int64_t* requests, int64_t* max_batch) {
  if (!sv) return SD_E_INVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (batches) *batches = (int64_t)sv->n_batches;
  if (requests) *requests = (int64_t)sv->n_requests_done;
  if (max_batch) *max_batch = (int64_t)sv->max_batch;
  return SD_OK;
}

void sd_server_free_pairs(sd_pairs* p) {
  if (!p) return;
  std::free(p->i);
  std::free(p->j);
  std::free(p->d);
  p->i = nullptr;
  p->j = nullptr;
  p->d = nullptr;
  p->n = 0;
}

void sd_server_destroy(sd_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
    for (Request* r : sv->pending) r->cancelled = true;
  }
  sv->cv_work.notify_all();
  for (auto& t : sv->workers) t.join();
  for (auto& kv : sv->done) {
    std::free(kv.second.i);
    std::free(kv.second.j);
    std::free(kv.second.d);
  }
  delete sv;
}

}  // extern "C"
