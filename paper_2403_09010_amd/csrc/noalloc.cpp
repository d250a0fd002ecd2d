// Self search with no device allocation, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc). Every scratch block of the call -- packed sequences, variant
// elements, sort buffers, candidates, the look-back status and counter
// areas, the unpacked result -- is carved in order from one fixed device
// array, `scratch`, of SD_NOALLOC_SCRATCH_BYTES; the result is copied into
// the caller's arrays. The kernels are the ones sd_self_search runs; they
// take addresses inside the area as arguments like any other buffer.
//
// Each device the library runs on holds its own copy of the array for the
// life of the process. Its device address is resolved once per device, by
// sd_create with that device current (noalloc_setup). The array's name is
// only a host-side stand-in for the symbol: host code never passes it to a
// kernel or a copy, only the resolved address.
//
// Calls share the area of their device and each overwrites what the last
// one left, so calls that overlap on one device (two host threads, or two
// streams without ordering between them) race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <utility>

#include "sd_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[SD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_area[kMaxDevices] = {};

unsigned char* area_of(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return device >= 0 && device < kMaxDevices ? g_area[device] : nullptr;
}

// The context's own per-call areas and size hints are set aside while a
// no-allocation call runs (its status and counter areas come from the fixed
// area, and hints left by large ordinary calls must not size its buffers),
// and put back afterwards, also when the call fails.
struct FixedAreaScope {
  sd_ctx* c;
  uint64_t* status;
  size_t status_words;
  uint32_t epoch;
  uint32_t* counters;
  size_t counters_n;
  int timing;
  FixedAreaScope(sd_ctx* ctx, unsigned char* base)
      : c(ctx),
        status(ctx->status),
        status_words(ctx->status_words),
        epoch(ctx->epoch),
        counters(ctx->counters),
        counters_n(ctx->counters_n),
        timing(ctx->timing) {
    c->status = nullptr;
    c->status_words = 0;
    c->epoch = 0;
    c->counters = nullptr;
    c->counters_n = 0;
    c->timing = 0;  // stage events are created lazily; none are needed here
    std::swap(c->out_hint, c->noalloc_hint);
    c->arena = base;
    c->arena_size = SD_NOALLOC_SCRATCH_BYTES;
    c->arena_used = 0;
  }
  ~FixedAreaScope() {
    c->arena = nullptr;
    c->arena_size = 0;
    c->arena_used = 0;
    std::swap(c->out_hint, c->noalloc_hint);
    c->status = status;
    c->status_words = status_words;
    c->epoch = epoch;
    c->counters = counters;
    c->counters_n = counters_n;
    c->timing = timing;
  }
};

}  // namespace

namespace sd {

int noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= kMaxDevices) return SD_E_HIP;
  if (g_area[device]) return SD_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return SD_E_HIP;
  }
  g_area[device] = static_cast<unsigned char*>(p);
  return SD_OK;
}

void self_search_noalloc(sd_ctx* c, const sd_seqs* seqs, int k, uint32_t* out_i, uint32_t* out_j,
                         uint8_t* out_d, int64_t capacity, int64_t* n_out, hipStream_t s) {
  if (!seqs || !n_out) throw Error{SD_E_INVAL, "null sequence set or result count"};
  *n_out = 0;
  if (seqs->n > SD_NOALLOC_MAX_SEQS)
    throw Error{SD_E_TOO_MANY, "the no-allocation self search takes at most " +
                                   std::to_string(SD_NOALLOC_MAX_SEQS) + " sequences, got " +
                                   std::to_string(seqs->n)};
  if (capacity < 0 || (capacity > 0 && (!out_i || !out_j || !out_d)))
    throw Error{SD_E_INVAL, "bad output arrays"};
  unsigned char* base = area_of(c->device);
  if (!base) throw Error{SD_E_HIP, "the fixed scratch area of this device was not set up"};
  sd_pairs r{};
  r.on_device = 1;
  {
    FixedAreaScope scope(c, base);
    self_search(c, seqs, k, &r, s);
    *n_out = r.n;
    if (r.n > capacity)
      throw Error{SD_E_NOMEM, "the result has " + std::to_string(r.n) +
                                  " pairs; the output arrays hold " + std::to_string(capacity)};
    if (r.n) {
      hip_check(hipMemcpyAsync(out_i, r.i, (size_t)r.n * 4, hipMemcpyDeviceToDevice, s), "copy i");
      hip_check(hipMemcpyAsync(out_j, r.j, (size_t)r.n * 4, hipMemcpyDeviceToDevice, s), "copy j");
      hip_check(hipMemcpyAsync(out_d, r.d, (size_t)r.n, hipMemcpyDeviceToDevice, s), "copy d");
    }
    // the area is reused by the next call: wait until this one is done with it
    hip_check(hipStreamSynchronize(s), "synchronise");
  }
}

}  // namespace sd
