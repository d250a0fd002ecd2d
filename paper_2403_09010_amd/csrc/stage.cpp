// Host staging of sequence sets. A batch of query sets becomes tile CSR
// arrays: the offsets of every device set come to pinned host memory with
// one synchronisation, the checks and the rebasing onto the tile's
// concatenated codes run on host threads into pinned memory, and each tile's
// offsets go back with one copy. A single host set goes to the device as it
// is, after the same checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "sd_host.h"

namespace sd {

namespace {

constexpr int64_t kGrain = 1 << 18;  // sequences per work item
constexpr unsigned kMaxThreads = 16;

// a piece of one span: its sequences [lo, hi) (set-local)
struct Item {
  size_t span;
  int64_t lo, hi;
};

std::vector<Item> items_of(const std::vector<SetSpan>& spans) {
  std::vector<Item> it;
  for (size_t x = 0; x < spans.size(); ++x)
    for (int64_t y = spans[x].first; y < spans[x].first + spans[x].count; y += kGrain)
      it.push_back(Item{x, y, std::min(y + kGrain, spans[x].first + spans[x].count)});
  return it;
}

// fn(item index) for every item, on up to kMaxThreads threads taking items
// in turn (inline for one or two items)
template <class F>
void for_items(size_t n, F&& fn) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned nt = (unsigned)std::min<size_t>({n, (size_t)hw, (size_t)kMaxThreads});
  if (nt <= 2) {
    for (size_t x = 0; x < n; ++x) fn(x);
    return;
  }
  std::atomic<size_t> next{0};
  auto work = [&] {
    for (size_t x = next.fetch_add(1); x < n; x = next.fetch_add(1)) fn(x);
  };
  std::vector<std::thread> th;
  th.reserve(nt - 1);
  try {
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(work);
  } catch (...) {
    // no more threads: the items are shared by the ones that started
  }
  work();
  for (auto& t : th) t.join();
}

}  // namespace

DevSeqs stage_seqs(sd_ctx* c, Scratch& sc, const sd_seqs* s, hipStream_t st) {
  DevSeqs d{s->codes, s->offsets, (uint64_t)s->n};
  if (s->on_device || s->n == 0) return d;
  const int64_t n = s->n;
  const int64_t* so = s->offsets;
  if (so[0] != 0) throw Error{SD_E_INVAL, "offsets must start at 0"};
  const int64_t total = so[n];
  if (total < 0) throw Error{SD_E_INVAL, "offsets must not decrease"};
  uint8_t* codes = sc.get<uint8_t>((uint64_t)total + 1);
  int64_t* offs = sc.get<int64_t>((uint64_t)n + 1);
  if (c->arena) {
    // no-allocation calls: no pinned area, direct copies from the caller's memory
    check_spans({so}, {SetSpan{0, 0, n}}, false, nullptr, nullptr);
    if (total)
      hip_check(hipMemcpyAsync(codes, s->codes, (size_t)total, hipMemcpyHostToDevice, st),
                "H2D codes");
    hip_check(hipMemcpyAsync(offs, so, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, st),
              "H2D offsets");
    d.codes = codes;
    d.offs = offs;
    return d;
  }
  // pieces of the codes (bytes) and of the offsets (words), copied into the
  // pinned area by host threads, the offsets checked on the way (every
  // sequence inside codes[0, total)); this thread sends each finished piece
  // to the device in order, so the copies to the device overlap the copies
  // into pinned memory
  const size_t cpad = ((size_t)total + 255) & ~(size_t)255;
  uint8_t* area = reinterpret_cast<uint8_t*>(stage_area(c, cpad + (size_t)(n + 1) * 8));
  int64_t* aoff = reinterpret_cast<int64_t*>(area + cpad);
  struct Part {
    bool words;      // offsets (words) or codes (bytes)
    int64_t lo, hi;  // [lo, hi) in its unit
  };
  std::vector<Part> parts;
  constexpr int64_t kBytes = 2 << 20;
  for (int64_t x = 0; x < total; x += kBytes) parts.push_back(Part{false, x, std::min(x + kBytes, total)});
  for (int64_t x = 0; x <= n; x += kBytes / 8) parts.push_back(Part{true, x, std::min(x + kBytes / 8, n + 1)});
  const size_t np = parts.size();
  std::unique_ptr<std::atomic<int>[]> state(new std::atomic<int>[np]);  // 0 pending, 1 ready, 2 bad offsets
  for (size_t x = 0; x < np; ++x) state[x].store(0);
  auto fill = [&](size_t x) {
    const Part& p = parts[x];
    bool ok = true;
    if (p.words) {
      std::memcpy(aoff + p.lo, so + p.lo, (size_t)(p.hi - p.lo) * 8);
      for (int64_t y = p.lo; y < p.hi && y < n; ++y) ok = ok && so[y + 1] >= so[y];
    } else {
      std::memcpy(area + p.lo, s->codes + p.lo, (size_t)(p.hi - p.lo));
    }
    state[x].store(ok ? 1 : 2, std::memory_order_release);
  };
  std::atomic<size_t> next{0};
  std::vector<std::thread> th;
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const unsigned nt = (unsigned)std::min<size_t>({np / 2, (size_t)hw, (size_t)8});
  bool bad = false;
  try {
    try {
      for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&] {
          for (size_t x = next.fetch_add(1); x < np; x = next.fetch_add(1)) fill(x);
        });
    } catch (...) {
      // no more threads: the ones that started (or this one) fill the pieces
    }
    for (size_t x = 0; x < np; ++x) {
      if (th.empty()) fill(x);
      int v;
      while ((v = state[x].load(std::memory_order_acquire)) == 0) std::this_thread::yield();
      if (v == 2) bad = true;
      if (bad) continue;  // nothing more goes to the device; the threads finish their pieces
      const Part& p = parts[x];
      if (p.words)
        hip_check(hipMemcpyAsync(offs + p.lo, aoff + p.lo, (size_t)(p.hi - p.lo) * 8,
                                 hipMemcpyHostToDevice, st),
                  "H2D offsets");
      else
        hip_check(hipMemcpyAsync(codes + p.lo, area + p.lo, (size_t)(p.hi - p.lo),
                                 hipMemcpyHostToDevice, st),
                  "H2D codes");
    }
  } catch (...) {
    for (auto& t : th) t.join();
    (void)hipStreamSynchronize(st);  // the area may be in use by copies already enqueued
    throw;
  }
  for (auto& t : th) t.join();
  stage_done(c, st);
  if (bad) throw Error{SD_E_INVAL, "offsets must not decrease"};
  d.codes = codes;
  d.offs = offs;
  return d;
}

int64_t* stage_area(sd_ctx* c, size_t bytes) {
  if (c->stage_pending) {
    hip_check(hipEventSynchronize(c->stage_event), "wait for staging copies");
    c->stage_pending = false;
  }
  if (bytes > c->stage_bytes) {
    if (c->stage_host) (void)hipHostFree(c->stage_host);
    c->stage_host = nullptr;
    c->stage_bytes = 0;
    const size_t want = std::max<size_t>(bytes + bytes / 4, 1 << 20);
    hip_check(hipHostMalloc(reinterpret_cast<void**>(&c->stage_host), want, hipHostMallocDefault),
              "hipHostMalloc");
    c->stage_bytes = want;
  }
  return c->stage_host;
}

void stage_done(sd_ctx* c, hipStream_t s) {
  if (!c->stage_event)
    hip_check(hipEventCreateWithFlags(&c->stage_event, hipEventDisableTiming), "event");
  hip_check(hipEventRecord(c->stage_event, s), "record");
  c->stage_pending = true;
}

std::vector<const int64_t*> set_offsets(const sd_seqs* sets, int first, int last, int64_t* area,
                                        hipStream_t s) {
  std::vector<const int64_t*> of(last, nullptr);
  bool copied = false;
  for (int x = first; x < last; ++x) {
    const sd_seqs& st = sets[x];
    if (!st.n) continue;
    if (!st.on_device) {
      of[x] = st.offsets;
      continue;
    }
    hip_check(hipMemcpyAsync(area, st.offsets, (size_t)(st.n + 1) * 8, hipMemcpyDeviceToHost, s),
              "read offsets");
    of[x] = area;
    area += st.n + 1;
    copied = true;
  }
  if (copied) hip_check(hipStreamSynchronize(s), "synchronise");
  for (int x = first; x < last; ++x)
    if (of[x] && of[x][0] != 0) throw Error{SD_E_INVAL, "offsets must start at 0"};
  return of;
}

void check_spans(const std::vector<const int64_t*>& offs, const std::vector<SetSpan>& spans,
                 bool check_len, const uint64_t* vlen, uint64_t* sums) {
  const std::vector<Item> it = items_of(spans);
  std::vector<int> err(it.size(), SD_OK);
  std::vector<uint64_t> part(it.size(), 0);
  for_items(it.size(), [&](size_t x) {
    const int64_t* so = offs[spans[it[x].span].set];
    uint64_t sum = 0;
    for (int64_t y = it[x].lo; y < it[x].hi; ++y) {
      const int64_t L = so[y + 1] - so[y];
      if (L < 0) {
        err[x] = SD_E_INVAL;
        return;
      }
      if ((check_len || vlen) && (L < 1 || L > KEY_MAX_LEN_HOST)) {
        err[x] = SD_E_LENGTH;
        return;
      }
      if (vlen) sum += vlen[L];
    }
    part[x] = sum;
  });
  for (size_t x = 0; x < it.size(); ++x) {
    if (err[x] == SD_E_INVAL) throw Error{SD_E_INVAL, "offsets must not decrease"};
    if (err[x] == SD_E_LENGTH) throw Error{SD_E_LENGTH, "a sequence length is outside [1, 24]"};
  }
  if (!sums) return;
  for (size_t x = 0; x < spans.size(); ++x) sums[x] = 0;
  for (size_t x = 0; x < it.size(); ++x) sums[it[x].span] += part[x];
}

int64_t rebase_spans(const std::vector<const int64_t*>& offs, const std::vector<SetSpan>& spans,
                     int64_t* dst) {
  // where each span starts in dst, and its code base
  std::vector<int64_t> q0(spans.size()), c0(spans.size());
  int64_t q = 0, cpos = 0;
  for (size_t x = 0; x < spans.size(); ++x) {
    q0[x] = q;
    c0[x] = cpos;
    if (!spans[x].count) continue;
    const int64_t* so = offs[spans[x].set];
    q += spans[x].count;
    cpos += so[spans[x].first + spans[x].count] - so[spans[x].first];
  }
  dst[q] = cpos;
  const std::vector<Item> it = items_of(spans);
  for_items(it.size(), [&](size_t x) {
    const SetSpan& sp = spans[it[x].span];
    const int64_t* so = offs[sp.set];
    const int64_t shift = c0[it[x].span] - so[sp.first];
    int64_t* d = dst + q0[it[x].span] - sp.first;
    for (int64_t y = it[x].lo; y < it[x].hi; ++y) d[y] = so[y] + shift;
  });
  return cpos;
}

uint64_t host_code_bytes(const sd_seqs* sets, const std::vector<SetSpan>& spans) {
  uint64_t b = 0;
  for (const SetSpan& sp : spans)
    if (sp.count && !sets[sp.set].on_device)
      b += (uint64_t)(sets[sp.set].offsets[sp.first + sp.count] - sets[sp.set].offsets[sp.first]);
  return b;
}

void stage_codes(const sd_seqs* sets, const std::vector<const int64_t*>& offs,
                 const std::vector<SetSpan>& spans, const int64_t* dst, uint8_t* codes,
                 uint8_t* pin, hipStream_t s) {
  // per span: its first tile sequence, its codes and, for host spans, its
  // place in the pinned room
  struct Part {
    const uint8_t* src;
    uint64_t bytes, pin_at;
    int64_t tile_at;
  };
  std::vector<Part> parts(spans.size());
  int64_t q = 0;
  uint64_t pat = 0;
  for (size_t x = 0; x < spans.size(); ++x) {
    const SetSpan& sp = spans[x];
    const int64_t a = sp.count ? offs[sp.set][sp.first] : 0;
    const int64_t b = sp.count ? offs[sp.set][sp.first + sp.count] : 0;
    parts[x] = Part{sets[sp.set].codes + a, (uint64_t)(b - a), pat, dst[q]};
    if (!sets[sp.set].on_device) pat += (uint64_t)(b - a);
    q += sp.count;
  }
  // host spans into pinned memory, in pieces of at most kGrain * 8 bytes
  struct Cut {
    size_t part;
    uint64_t lo, hi;
  };
  std::vector<Cut> cuts;
  constexpr uint64_t kBytes = (uint64_t)kGrain * 8;
  for (size_t x = 0; x < spans.size(); ++x)
    if (!sets[spans[x].set].on_device)
      for (uint64_t y = 0; y < parts[x].bytes; y += kBytes)
        cuts.push_back(Cut{x, y, std::min(y + kBytes, parts[x].bytes)});
  for_items(cuts.size(), [&](size_t x) {
    const Part& p = parts[cuts[x].part];
    std::memcpy(pin + p.pin_at + cuts[x].lo, p.src + cuts[x].lo, cuts[x].hi - cuts[x].lo);
  });
  // one copy per run of consecutive host spans (contiguous on both sides),
  // one per device span
  for (size_t x = 0; x < spans.size();) {
    if (sets[spans[x].set].on_device) {
      if (parts[x].bytes)
        hip_check(hipMemcpyAsync(codes + parts[x].tile_at, parts[x].src, parts[x].bytes,
                                 hipMemcpyDeviceToDevice, s),
                  "copy codes");
      ++x;
      continue;
    }
    size_t y = x;
    uint64_t run = 0;
    while (y < spans.size() && !sets[spans[y].set].on_device) run += parts[y++].bytes;
    if (run)
      hip_check(hipMemcpyAsync(codes + parts[x].tile_at, pin + parts[x].pin_at, run,
                               hipMemcpyHostToDevice, s),
                "copy codes");
    x = y;
  }
}

void host_result(sd_ctx* c, uint64_t n, sd_pairs* out) {
  const uint64_t m = n ? n : 1;
  uint8_t* h = static_cast<uint8_t*>(host_block(c, m * 9));
  out->n = (int64_t)n;
  out->i = reinterpret_cast<uint32_t*>(h);
  out->j = reinterpret_cast<uint32_t*>(h + m * 4);
  out->d = h + m * 8;
}

void fill_host_slices(sd_ctx* c, const uint32_t* di, const uint32_t* dj, const uint8_t* dd,
                      uint64_t n, const std::vector<HostSlice>& slices, sd_pairs* outs,
                      hipStream_t s) {
  if (!n) return;
  uint8_t* h = reinterpret_cast<uint8_t*>(stage_area(c, n * 9));
  uint32_t* hi = reinterpret_cast<uint32_t*>(h);
  uint32_t* hj = hi + n;
  uint8_t* hd = h + n * 8;
  hip_check(hipMemcpyAsync(hi, di, n * 4, hipMemcpyDeviceToHost, s), "D2H");
  hip_check(hipMemcpyAsync(hj, dj, n * 4, hipMemcpyDeviceToHost, s), "D2H");
  hip_check(hipMemcpyAsync(hd, dd, n, hipMemcpyDeviceToHost, s), "D2H");
  hip_check(hipStreamSynchronize(s), "D2H synchronise");
  // pieces of at most kGrain pairs of one slice
  struct Cut {
    size_t slice;
    uint64_t lo, hi;  // within the slice
  };
  std::vector<Cut> cuts;
  for (size_t x = 0; x < slices.size(); ++x)
    for (uint64_t y = 0; y < slices[x].n; y += kGrain)
      cuts.push_back(Cut{x, y, std::min<uint64_t>(y + kGrain, slices[x].n)});
  for_items(cuts.size(), [&](size_t x) {
    const HostSlice& sl = slices[cuts[x].slice];
    const sd_pairs& o = outs[sl.set];
    const uint64_t a = cuts[x].lo, b = cuts[x].hi;
    for (uint64_t t = a; t < b; ++t) o.i[sl.at + t] = (uint32_t)((int64_t)hi[sl.lo + t] + sl.shift);
    std::memcpy(o.j + sl.at + a, hj + sl.lo + a, (b - a) * 4);
    std::memcpy(o.d + sl.at + a, hd + sl.lo + a, b - a);
  });
}

}  // namespace sd
