// C entry points of the symdel library, the context and its device memory
// pool. Every entry point converts exceptions into SD_E_* codes, so no call
// aborts the process and the context stays usable after an error.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <thread>
#include <unordered_set>
#include <vector>

#include "sd_host.h"
#include "sd_internal.h"

namespace sd {

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error{SD_E_HIP, std::string(what) + ": " + hipGetErrorString(e)};
  }
}

static size_t size_class(size_t bytes) {
  if (bytes < 256) bytes = 256;
  if (bytes <= (1u << 20)) {
    size_t p = 256;
    while (p < bytes) p <<= 1;
    return p;
  }
  const size_t g = 2u << 20;
  return (bytes + g - 1) / g * g;
}

void release_cache(sd_ctx* c) {
  for (auto& kv : c->cache) {
    (void)hipFree(kv.second);
    c->held -= kv.first;
  }
  c->cache.clear();
}

// A block from the allocator hook: counted against the budget, returned to
// the hook by dfree.
static void* hook_alloc(sd_ctx* c, size_t sz) {
  if (c->budget && c->held + sz > c->budget) release_cache(c);
  if (c->budget && c->held + sz > c->budget)
    throw Error{SD_E_NOMEM, "device memory budget exceeded: need " + std::to_string(sz) +
                                " more bytes, holding " + std::to_string(c->held) + " of " +
                                std::to_string(c->budget)};
  void* p = c->ualloc(sz, c->uarg);
  if (!p) throw Error{SD_E_NOMEM, "the allocator hook returned NULL for " + std::to_string(sz) + " bytes"};
  c->held += sz;
  c->live[p] = sz;
  return p;
}

// A block carved from the fixed area of a no-allocation call: 256-byte
// aligned, in order; exhausting the area fails the call.
static void* arena_alloc(sd_ctx* c, size_t bytes) {
  const size_t at = (c->arena_used + 255) / 256 * 256;
  const size_t sz = bytes ? bytes : 1;
  if (at > c->arena_size || sz > c->arena_size - at)
    throw Error{SD_E_NOMEM, "the fixed scratch area (" + std::to_string(c->arena_size) +
                                " bytes) is too small for this input: " + std::to_string(at) +
                                " bytes in use, " + std::to_string(sz) + " more needed"};
  c->arena_used = at + sz;
  return c->arena + at;
}

static bool in_arena(const sd_ctx* c, const void* p) {
  const unsigned char* q = static_cast<const unsigned char*>(p);
  return c->arena && q >= c->arena && q < c->arena + c->arena_size;
}

void* dalloc(sd_ctx* c, size_t bytes) {
  if (c->arena) return arena_alloc(c, bytes);
  const size_t sz = size_class(bytes);
  if (c->ualloc) return hook_alloc(c, sz);
  // a cached block up to twice the size serves the request; under a budget
  // only up to an eighth more, so that a reused block does not hold much
  // memory the budget could give to another request
  auto it = c->cache.lower_bound(sz);
  if (it != c->cache.end() && it->first <= (c->budget ? sz + sz / 8 : 2 * sz)) {
    void* p = it->second;
    c->live[p] = it->first;
    c->cache.erase(it);
    return p;
  }
  if (c->budget && c->held + sz > c->budget) release_cache(c);
  if (c->budget && c->held + sz > c->budget)
    throw Error{SD_E_NOMEM, "device memory budget exceeded: need " + std::to_string(sz) +
                                " more bytes, holding " + std::to_string(c->held) + " of " +
                                std::to_string(c->budget)};
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_cache(c);
    e = hipMalloc(&p, sz);
  }
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error{SD_E_NOMEM, "hipMalloc of " + std::to_string(sz) + " bytes failed"};
  }
  c->held += sz;
  c->live[p] = sz;
  return p;
}

void dfree(sd_ctx* c, void* p) {
  if (!p || in_arena(c, p)) return;
  auto it = c->live.find(p);
  if (it == c->live.end()) return;
  if (c->ualloc) {
    c->held -= it->second;
    c->live.erase(it);
    c->ufree(p, c->uarg);
    return;
  }
  c->cache.insert({it->second, p});
  c->live.erase(it);
}

void* index_alloc(sd_ctx* c, sd_index* idx, size_t bytes) {
  if (!bytes) bytes = 16;
  void* p = nullptr;
  if (c->ualloc) {
    idx->ufree = c->ufree;
    idx->uarg = c->uarg;
    p = c->ualloc(bytes, c->uarg);
    if (!p) throw Error{SD_E_NOMEM, "the allocator hook returned NULL for an index array"};
    return p;
  }
  if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error{SD_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes for an index failed"};
  }
  return p;
}

void index_release(sd_index* idx, void* p) {
  if (!p) return;
  if (idx->ufree)
    idx->ufree(p, idx->uarg);
  else
    (void)hipFree(p);
}

uint32_t next_epoch(sd_ctx* c, uint64_t words, hipStream_t s) {
  if (words > c->status_words) {
    if (c->status) dfree(c, c->status);
    uint64_t w = words + words / 4 + 4096;
    c->status = dalloc_t<uint64_t>(c, w);
    c->status_words = w;
    launch_fill_u64(c->status, 0, w, s);
    c->epoch = 0;
  }
  if (++c->epoch >= 0xFFFFu) {
    launch_fill_u64(c->status, 0, c->status_words, s);
    c->epoch = 1;
  }
  return c->epoch;
}

uint32_t* fresh_counters(sd_ctx* c, size_t n, hipStream_t s) {
  if (n > c->counters_n) {
    if (c->counters) dfree(c, c->counters);
    c->counters = dalloc_t<uint32_t>(c, n);
    c->counters_n = n;
  }
  launch_fill_u32(c->counters, 0, n, s);
  c->tile_slot = 0;  // every slot is zero again
  return c->counters;
}

void* readback(sd_ctx* c, const void* dptr, size_t bytes, hipStream_t s) {
  if (bytes > c->pinned_bytes) {
    if (c->arena)
      throw Error{SD_E_NOMEM, "a read-back of " + std::to_string(bytes) +
                                  " bytes exceeds the staging area allocated at set-up"};
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    size_t want = bytes < 65536 ? 65536 : bytes;
    hip_check(hipHostMalloc(&c->pinned, want, hipHostMallocDefault), "hipHostMalloc");
    c->pinned_bytes = want;
  }
  hip_check(hipMemcpyAsync(c->pinned, dptr, bytes, hipMemcpyDeviceToHost, s), "read-back copy");
  hip_check(hipStreamSynchronize(s), "read-back synchronise");
  return c->pinned;
}

constexpr size_t kHostCacheBytes = 512ull << 20;  // released result blocks kept per context

void* host_block(sd_ctx* c, size_t bytes) {
  auto it = c->host_cache.lower_bound(bytes);
  if (it != c->host_cache.end() && it->first <= 2 * bytes + 65536) {
    void* p = it->second;
    c->host_live[p] = it->first;
    c->host_cache_bytes -= it->first;
    c->host_cache.erase(it);
    return p;
  }
  void* p = nullptr;
  hip_check(hipHostMalloc(&p, bytes, hipHostMallocDefault), "hipHostMalloc");
  c->host_live[p] = bytes;
  return p;
}

void host_release(sd_ctx* c, void* p) {
  auto h = c->host_live.find(p);
  if (h == c->host_live.end()) return;
  const size_t bytes = h->second;
  c->host_live.erase(h);
  // make room by dropping the largest kept blocks; a block larger than the
  // whole budget is freed at once
  while (!c->host_cache.empty() && c->host_cache_bytes + bytes > kHostCacheBytes) {
    auto last = std::prev(c->host_cache.end());
    (void)hipHostFree(last->second);
    c->host_cache_bytes -= last->first;
    c->host_cache.erase(last);
  }
  if (bytes > kHostCacheBytes) {
    (void)hipHostFree(p);
    return;
  }
  c->host_cache.emplace(bytes, p);
  c->host_cache_bytes += bytes;
}

StageTimer::StageTimer(sd_ctx* ctx, hipStream_t st) : c(ctx), s(st), on(ctx->timing != 0) {
  if (!on) return;
  if (c->events.empty()) c->events.resize(SD_MAX_STAGES + 1, nullptr);
  for (auto& e : c->events)
    if (!e) hip_check(hipEventCreate(&e), "hipEventCreate");
  hip_check(hipEventRecord(c->events[0], s), "hipEventRecord");
}

void StageTimer::mark(const char* name, double bytes, int nl) {
  // a launch that the runtime rejected surfaces here, named by its stage
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    throw Error{SD_E_HIP, std::string("a kernel launch of stage ") + name + " failed: " +
                              hipGetErrorString(e)};
  if (!on || names.size() >= SD_MAX_STAGES) return;
  names.push_back({name, bytes});
  launches.push_back(nl);
  hip_check(hipEventRecord(c->events[names.size()], s), "hipEventRecord");
}

void StageTimer::finish() {
  c->stats.n_stages = 0;
  if (!on) return;
  hip_check(hipEventSynchronize(c->events[names.size()]), "hipEventSynchronize");
  for (size_t x = 0; x < names.size(); ++x) {
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, c->events[x], c->events[x + 1]), "hipEventElapsedTime");
    std::snprintf(c->stats.stage_name[x], sizeof(c->stats.stage_name[x]), "%s",
                  names[x].first.c_str());
    c->stats.stage_ms[x] = ms;
    c->stats.stage_bytes[x] = names[x].second;
    c->stats.stage_launches[x] = launches[x];
  }
  c->stats.n_stages = (int32_t)names.size();
}

}  // namespace sd

using sd::Error;

// After a failed call: wait for the device (kernels of the call may still be
// queued), then give back every device block the call took that is still
// live, except the context's own areas. A failed call returns no result, so
// nothing it allocated is owned by the caller.
static void reclaim_failed_call(sd_ctx* c, const std::unordered_set<void*>& before) {
  (void)hipDeviceSynchronize();
  (void)hipGetLastError();
  std::vector<void*> stray;
  for (auto& kv : c->live)
    if (!before.count(kv.first) && kv.first != c->status && kv.first != c->counters)
      stray.push_back(kv.first);
  for (void* p : stray) sd::dfree(c, p);
}

template <typename F>
static int guarded(sd_ctx* c, F&& f) {
  std::unordered_set<void*> before;
  if (c) {
    c->last_error.clear();
    for (auto& kv : c->live) before.insert(kv.first);
  }
  int code = SD_OK;
  try {
    f();
    const hipError_t e = hipGetLastError();  // a rejected launch is never left behind
    if (e != hipSuccess)
      throw Error{SD_E_HIP, std::string("a kernel launch failed: ") + hipGetErrorString(e)};
    return SD_OK;
  } catch (const Error& e) {
    if (c) c->last_error = e.msg;
    code = e.code;
  } catch (const std::bad_alloc&) {
    if (c) c->last_error = "host allocation failed";
    code = SD_E_NOMEM;
  } catch (const std::exception& e) {
    if (c) c->last_error = e.what();
    code = SD_E_INVAL;
  }
  if (c) reclaim_failed_call(c, before);
  return code;
}

// Run f with the context's metric set to `metric`, restoring it afterwards.
template <typename F>
static void with_metric(sd_ctx* c, int metric, F&& f) {
  const int saved = c->metric;
  c->metric = metric;
  try {
    f();
  } catch (...) {
    c->metric = saved;
    throw;
  }
  c->metric = saved;
}

// pinned host staging for read-backs: the largest one (the full-key sort's
// digit histograms, 16 KiB) fits, so it never grows after sd_create
constexpr size_t kPinnedStaging = 65536;

extern "C" {

int sd_create(sd_ctx** out, int device, uint64_t hbm_budget_bytes) {
  if (!out) return SD_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return SD_E_HIP;
  }
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    return SD_E_HIP;
  }
  sd_ctx* c = new (std::nothrow) sd_ctx();
  if (!c) return SD_E_NOMEM;
  c->device = device;
  c->budget = hbm_budget_bytes;
  // set-up of the no-allocation entry point: the per-device address of its
  // fixed scratch area, and the pinned staging area for small read-backs
  // (allocated here so that no later call has to)
  if (sd::noalloc_setup(device) != SD_OK ||
      hipHostMalloc(&c->pinned, kPinnedStaging, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    return SD_E_HIP;
  }
  c->pinned_bytes = kPinnedStaging;
  *out = c;
  return SD_OK;
}

void sd_destroy(sd_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  sd::graph_plans_release(c);  // synchronises the device first
  (void)hipDeviceSynchronize();
  for (auto& kv : c->live) {
    if (c->ualloc)
      c->ufree(kv.first, c->uarg);
    else
      (void)hipFree(kv.first);
  }
  c->live.clear();
  sd::release_cache(c);
  for (auto& kv : c->host_live) (void)hipHostFree(kv.first);
  for (auto& kv : c->host_cache) (void)hipHostFree(kv.second);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->stage_host) (void)hipHostFree(c->stage_host);
  if (c->stage_event) (void)hipEventDestroy(c->stage_event);
  for (auto& e : c->events)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

int sd_set_option(sd_ctx* c, int option, int64_t value) {
  if (!c) return SD_E_INVAL;
  switch (option) {
    case SD_OPT_TIMING:
      c->timing = value ? 1 : 0;
      return SD_OK;
    case SD_OPT_PATH:
      if (value < 0 || value > 2) return SD_E_INVAL;
      c->path = (int)value;
      return SD_OK;
    case SD_OPT_GROUP_CAP:
      if (value != 0 && !sd::group_cap_supported((int)value)) return SD_E_INVAL;
      c->group_cap = (int)value;
      return SD_OK;
    case SD_OPT_GROUP_BITS:
      if (value < 0 || value > 23) return SD_E_INVAL;
      c->group_bits = (int)value;
      return SD_OK;
    case SD_OPT_SORT_ITEMS:
      if (value != 0 && value != 16 && value != 32) return SD_E_INVAL;
      c->sort_items = (int)value;
      return SD_OK;
    case SD_OPT_BATCH_TILE:
      if (value < 0) return SD_E_INVAL;
      c->batch_tile_seqs = value;
      return SD_OK;
    case SD_OPT_GROUP_BATCHES:
      if (value < 0 || value > 64) return SD_E_INVAL;
      c->group_batches = (int)value;
      return SD_OK;
    case SD_OPT_PROBE:
      if (value < 0 || value > 1) return SD_E_INVAL;
      c->probe = (int)value;
      return SD_OK;
    case SD_OPT_PAIR_SORT:
      if (value < 0 || value > 2) return SD_E_INVAL;
      c->pair_sort = (int)value;
      return SD_OK;
    case SD_OPT_JOIN_ELEMS:
      if (value < 0 || value > (1 << 20)) return SD_E_INVAL;
      c->join_elems = (int)value;
      return SD_OK;
    case SD_OPT_BATCH_GRAPH:
      if (value < 0 || value > 1) return SD_E_INVAL;
      c->batch_graph = (int)value;
      if (!value) sd::graph_plans_release(c);
      return SD_OK;
    case SD_OPT_GROUP_SHAPE:
      if (value < 0 || value > 2) return SD_E_INVAL;
      c->group_shape = (int)value;
      return SD_OK;
    case SD_OPT_STREAM:
      if (value < 0 || value > 2) return SD_E_INVAL;
      c->stream = (int)value;
      return SD_OK;
    case SD_OPT_STREAM_ELEMS:
      if (value < 0) return SD_E_INVAL;
      c->stream_elems = (uint64_t)value;
      return SD_OK;
    case SD_OPT_METRIC:
      if (value != SD_METRIC_LEVENSHTEIN && value != SD_METRIC_HAMMING) return SD_E_INVAL;
      c->metric = (int)value;
      return SD_OK;
    default:
      c->last_error = "unknown option";
      return SD_E_INVAL;
  }
}

int sd_set_allocator(sd_ctx* c, sd_alloc_fn alloc, sd_free_fn free_fn, void* user) {
  if (!c) return SD_E_INVAL;
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    c->last_error = "give both the allocation and the release function, or neither";
    return SD_E_INVAL;
  }
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::hip_check(hipDeviceSynchronize(), "synchronise");
    // the context's own areas move to the new provider; anything else still
    // live is a result the caller has not released
    if (c->status) sd::dfree(c, c->status);
    if (c->counters) sd::dfree(c, c->counters);
    c->status = nullptr;
    c->status_words = 0;
    c->counters = nullptr;
    c->counters_n = 0;
    if (!c->live.empty())
      throw Error{SD_E_STATE, "results of this context are still live (release them with sd_pairs_free first)"};
    sd::release_cache(c);
    c->ualloc = alloc;
    c->ufree = free_fn;
    c->uarg = user;
  });
}

int sd_self_search(sd_ctx* c, const sd_seqs* seqs, int k, sd_pairs* out, void* stream) {
  if (!c || !seqs || !out) return SD_E_INVAL;
  const int32_t want_device = out->on_device;
  std::memset(out, 0, sizeof(*out));
  out->on_device = want_device;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::self_search(c, seqs, k, out, static_cast<hipStream_t>(stream));
  });
}

int sd_self_search_hamming(sd_ctx* c, const sd_seqs* seqs, int k, sd_pairs* out, void* stream) {
  if (!c || !seqs || !out) return SD_E_INVAL;
  const int32_t want_device = out->on_device;
  std::memset(out, 0, sizeof(*out));
  out->on_device = want_device;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    with_metric(c, SD_METRIC_HAMMING, [&] {
      sd::self_search(c, seqs, k, out, static_cast<hipStream_t>(stream));
    });
  });
}

int sd_paired_self_search(sd_ctx* c, const sd_seqs* a, const sd_seqs* b, int k, sd_pairs* out,
                          void* stream) {
  if (!c || !a || !b || !out) return SD_E_INVAL;
  const int32_t want_device = out->on_device;
  std::memset(out, 0, sizeof(*out));
  out->on_device = want_device;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::paired_self_search(c, a, b, k, out, static_cast<hipStream_t>(stream));
  });
}

int sd_self_search_noalloc(sd_ctx* c, const sd_seqs* seqs, int k, uint32_t* out_i,
                           uint32_t* out_j, uint8_t* out_d, int64_t capacity, int64_t* n_out,
                           void* stream) {
  if (!c || !seqs || !n_out) return SD_E_INVAL;
  *n_out = 0;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::self_search_noalloc(c, seqs, k, out_i, out_j, out_d, capacity, n_out,
                            static_cast<hipStream_t>(stream));
  });
}

int sd_pair_distance(sd_ctx* c, const sd_seqs* a, const sd_seqs* b, const uint32_t* ia,
                     const uint32_t* ib, int64_t n, uint8_t* d_out, void* stream) {
  if (!c) return SD_E_INVAL;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::pair_distance(c, a, b, ia, ib, n, d_out, static_cast<hipStream_t>(stream));
  });
}

int sd_index_build(sd_ctx* c, const sd_seqs* ref, int k, sd_index** out, void* stream) {
  if (!c || !ref || !out) return SD_E_INVAL;
  *out = nullptr;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    *out = sd::index_build(c, ref, k, static_cast<hipStream_t>(stream));
  });
}

void sd_index_free(sd_index* idx) { sd::index_free(idx); }

int sd_index_info(const sd_index* idx, int64_t* n_ref, int64_t* n_keys, int32_t* k,
                  int64_t* bytes) {
  if (!idx) return SD_E_INVAL;
  if (n_ref) *n_ref = (int64_t)idx->n_ref;
  if (n_keys) *n_keys = (int64_t)idx->n_keys;
  if (k) *k = idx->k;
  if (bytes) *bytes = (int64_t)idx->bytes;
  return SD_OK;
}

int sd_index_build_learned(sd_ctx* c, const sd_seqs* ref, int k, const sd_learned_config* cfg,
                           sd_index** out, void* stream) {
  if (!c || !ref || !out) return SD_E_INVAL;
  *out = nullptr;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    *out = sd::learned_build(c, ref, k, cfg, static_cast<hipStream_t>(stream));
  });
}

int sd_index_learned_info(const sd_index* idx, sd_learned_info* out, float* loss_curve,
                          int32_t cap) {
  if (!idx || !out || !idx->learned || cap < 0) return SD_E_INVAL;
  *out = idx->info;
  if (loss_curve) {
    const size_t n = std::min<size_t>((size_t)cap, idx->loss_curve.size());
    if (n) std::memcpy(loss_curve, idx->loss_curve.data(), n * sizeof(float));
  }
  return SD_OK;
}

int sd_autotune(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k, int reps,
                sd_tune_result* out, void* stream) {
  if (!c) return SD_E_INVAL;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::autotune(c, idx, nsets, sets, k, reps, out, static_cast<hipStream_t>(stream));
  });
}

int sd_autotune_cache(sd_ctx* c, const char* path) {
  if (!c) return SD_E_INVAL;
  if (path && std::strlen(path) > 4095) return SD_E_INVAL;
  c->tune_cache = path ? path : "";
  return SD_OK;
}

int sd_mlp_gradients(sd_ctx* c, const float* params, const float* x, const float* y, uint32_t n,
                     float* grad, float* loss, void* stream) {
  if (!c) return SD_E_INVAL;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::mlp_gradients(c, params, x, y, n, grad, loss, static_cast<hipStream_t>(stream));
  });
}

static void reset_pairs(sd_pairs* p) {
  const int32_t want_device = p->on_device;
  std::memset(p, 0, sizeof(*p));
  p->on_device = want_device;
}

int sd_query(sd_ctx* c, const sd_index* idx, const sd_seqs* q, int k, sd_pairs* out,
             void* stream) {
  if (!c || !q || !out) return SD_E_INVAL;
  reset_pairs(out);
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::query_sets(c, idx, 1, q, k, nullptr, out, static_cast<hipStream_t>(stream));
  });
}

int sd_query_hamming(sd_ctx* c, const sd_index* idx, const sd_seqs* q, int k, sd_pairs* out,
                     void* stream) {
  if (!c || !q || !out) return SD_E_INVAL;
  reset_pairs(out);
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    with_metric(c, SD_METRIC_HAMMING, [&] {
      sd::query_sets(c, idx, 1, q, k, nullptr, out, static_cast<hipStream_t>(stream));
    });
  });
}

int sd_query_batch(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k,
                   sd_pairs* outs, void* stream) {
  if (!c || nsets < 0 || (nsets > 0 && (!sets || !outs))) return SD_E_INVAL;
  for (int x = 0; x < nsets; ++x) reset_pairs(&outs[x]);
  const int rc = guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::query_sets(c, idx, nsets, sets, k, nullptr, outs, static_cast<hipStream_t>(stream));
  });
  if (rc != SD_OK)  // all or nothing: release whatever was produced before the error
    for (int x = 0; x < nsets; ++x) sd_pairs_free(c, &outs[x]);
  return rc;
}

int sd_query_weighted(sd_ctx* c, const sd_index* idx, const sd_seqs* q, const uint8_t* subst,
                      int indel, int max_score, sd_pairs* out, void* stream) {
  if (!c || !q || !out) return SD_E_INVAL;
  reset_pairs(out);
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::query_weighted(c, idx, 1, q, subst, indel, max_score, out,
                       static_cast<hipStream_t>(stream));
  });
}

int sd_query_batch_weighted(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets,
                            const uint8_t* subst, int indel, int max_score, sd_pairs* outs,
                            void* stream) {
  if (!c || nsets < 0 || (nsets > 0 && (!sets || !outs))) return SD_E_INVAL;
  for (int x = 0; x < nsets; ++x) reset_pairs(&outs[x]);
  const int rc = guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    sd::query_weighted(c, idx, nsets, sets, subst, indel, max_score, outs,
                       static_cast<hipStream_t>(stream));
  });
  if (rc != SD_OK)
    for (int x = 0; x < nsets; ++x) sd_pairs_free(c, &outs[x]);
  return rc;
}

int sd_get_stats(const sd_ctx* c, sd_stats* out) {
  if (!c || !out) return SD_E_INVAL;
  *out = c->stats;
  return SD_OK;
}

int sd_pairs_copy(sd_ctx* c, const sd_pairs* p, uint32_t* i, uint32_t* j, uint8_t* d,
                  int dst_on_device, void* stream) {
  if (!c || !p) return SD_E_INVAL;
  if (p->n == 0) return SD_OK;
  if (!i || !j || !d || !p->i || !p->j || !p->d) return SD_E_INVAL;
  return guarded(c, [&] {
    sd::hip_check(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipMemcpyKind kind;
    if (p->on_device)
      kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    else
      kind = dst_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
    const size_t n = (size_t)p->n;
    if (kind == hipMemcpyHostToHost) {
      // a host result is complete when the search returns: plain copies, the
      // i array on a second thread when the result is large
      std::thread ti;
      if (n >= (1u << 18))
        ti = std::thread([&] { std::memcpy(i, p->i, n * 4); });
      else
        std::memcpy(i, p->i, n * 4);
      std::memcpy(j, p->j, n * 4);
      std::memcpy(d, p->d, n);
      if (ti.joinable()) ti.join();
      return;
    }
    sd::hip_check(hipMemcpyAsync(i, p->i, n * 4, kind, s), "copy i");
    sd::hip_check(hipMemcpyAsync(j, p->j, n * 4, kind, s), "copy j");
    sd::hip_check(hipMemcpyAsync(d, p->d, n, kind, s), "copy d");
    sd::hip_check(hipStreamSynchronize(s), "copy synchronise");
  });
}

void sd_pairs_free(sd_ctx* c, sd_pairs* p) {
  if (!c || !p) return;
  if (p->i && c->host_live.count(p->i)) {
    // a host result: i, j and d share the block that starts at i
    sd::host_release(c, p->i);
  } else {
    for (void* a : {(void*)p->i, (void*)p->j, (void*)p->d})
      if (a) sd::dfree(c, a);
  }
  p->i = nullptr;
  p->j = nullptr;
  p->d = nullptr;
  p->n = 0;
}

const char* sd_strerror(int code) {
  switch (code) {
    case SD_OK: return "ok";
    case SD_E_INVAL: return "invalid argument";
    case SD_E_ALPHABET: return "residue code outside 0..19";
    case SD_E_LENGTH: return "sequence length outside [1, 24]";
    case SD_E_TOO_MANY: return "too many sequences or variants for 32-bit ids";
    case SD_E_NOMEM: return "out of device memory or over the HBM budget";
    case SD_E_HIP: return "HIP runtime error";
    case SD_E_CANCELLED: return "cancelled";
    case SD_E_STATE: return "wrong state for this call";
    default: return "unknown error";
  }
}

const char* sd_last_error(const sd_ctx* c) { return c ? c->last_error.c_str() : ""; }

}  // extern "C"
