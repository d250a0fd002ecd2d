// The library's host staging (csrc/stage.cpp) on the CPU under
// AddressSanitizer and UBSan, built by tests/test_sanitizers.py. Host memory
// stands in for device and pinned memory: the few HIP calls the staging
// makes are defined below as plain copies, and device blocks come from
// malloc. Checks the pieces of a large host set, the offset checks and their
// order, the sums of a length table, the rebased offsets and codes of split
// spans and host results cut from one device result against plain loops. Exits 0 and
// prints "ok" when every check holds.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "sd_host.h"

namespace sd {
void* dalloc(sd_ctx*, size_t bytes) { return std::malloc(bytes ? bytes : 1); }
void dfree(sd_ctx*, void* p) { std::free(p); }
void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error{SD_E_HIP, what};
}
void* host_block(sd_ctx*, size_t bytes) { return std::malloc(bytes); }
}  // namespace sd

namespace {
int events_live = 0;
char event_token;
}  // namespace

extern "C" {
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) {
  *p = std::malloc(n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = reinterpret_cast<hipEvent_t>(&event_token);
  ++events_live;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
}

namespace {

int failures = 0;
void check(bool ok, const char* what) {
  std::printf("%-58s %s\n", what, ok ? "ok" : "FAILED");
  failures += !ok;
}

uint64_t state = 0x9E3779B97F4A7C15ull;
uint32_t draw(uint32_t m) {
  state ^= state << 13;
  state ^= state >> 7;
  state ^= state << 17;
  return (uint32_t)(state % m);
}

struct HostSet {
  std::vector<uint8_t> codes;
  std::vector<int64_t> offs{0};
  sd_seqs view(int on_device = 0) const {
    return sd_seqs{codes.data(), offs.data(), (int64_t)offs.size() - 1, on_device};
  }
};

HostSet make(int64_t n) {
  HostSet s;
  for (int64_t x = 0; x < n; ++x) {
    const int L = 1 + (int)draw(24);
    for (int t = 0; t < L; ++t) s.codes.push_back((uint8_t)draw(20));
    s.offs.push_back((int64_t)s.codes.size());
  }
  return s;
}

// the error code staging raises for set s, or SD_OK
template <class F>
int code_of(F&& f) {
  try {
    f();
  } catch (const sd::Error& e) {
    return e.code;
  }
  return SD_OK;
}

}  // namespace

int main() {
  sd_ctx* c = new sd_ctx();
  // a large host set: many 2 MiB pieces of codes and of offsets
  const HostSet big = make(600000);
  {
    const sd_seqs v = big.view();
    sd::Scratch sc(c);
    const sd::DevSeqs d = sd::stage_seqs(c, sc, &v, nullptr);
    check(d.n == 600000 && std::memcmp(d.codes, big.codes.data(), big.codes.size()) == 0 &&
              std::memcmp(d.offs, big.offs.data(), big.offs.size() * 8) == 0,
          "stage_seqs: codes and offsets arrive whole");
    check(c->stage_pending, "stage_seqs: the pinned area is marked in use");
  }
  {
    HostSet bad = big;
    bad.offs[450001] = bad.offs[450000] - 1;
    const sd_seqs v = bad.view();
    sd::Scratch sc(c);
    check(code_of([&] { sd::stage_seqs(c, sc, &v, nullptr); }) == SD_E_INVAL,
          "stage_seqs: a decreasing offset deep in the set");
    bad = big;
    bad.offs[0] = 2;
    const sd_seqs w = bad.view();
    check(code_of([&] { sd::stage_seqs(c, sc, &w, nullptr); }) == SD_E_INVAL,
          "stage_seqs: a first offset other than 0");
  }
  // batches: "device" sets (their offsets read into the area) and host sets
  std::vector<HostSet> sets;
  for (int64_t n : {0, 7, 300000, 1, 450000, 25}) sets.push_back(make(n));
  std::vector<sd_seqs> views;
  for (size_t x = 0; x < sets.size(); ++x) views.push_back(sets[x].view((int)(x % 2)));
  size_t words = 0;
  for (const auto& s : sets) words += s.offs.size();
  int64_t* area = sd::stage_area(c, words * 8 + (1u << 22));
  check(!c->stage_pending, "stage_area: waits for the last copies");
  const std::vector<const int64_t*> so = sd::set_offsets(views.data(), 1, 6, area, nullptr);
  bool views_ok = so[0] == nullptr;
  for (int x = 1; x < 6; ++x)
    views_ok = views_ok && std::memcmp(so[x], sets[x].offs.data(), sets[x].offs.size() * 8) == 0;
  check(views_ok, "set_offsets: host views of device and host sets");
  // spans that split sets, and empty ones
  std::vector<sd::SetSpan> spans = {{1, 0, 7},       {2, 0, 123456}, {2, 123456, 0},
                                    {2, 123456, 176544}, {3, 0, 1}, {4, 1000, 449000},
                                    {5, 0, 25}};
  uint64_t vlen[25];
  for (int L = 0; L <= 24; ++L) vlen[L] = (uint64_t)(L * L + 1);
  std::vector<uint64_t> sums(spans.size());
  sd::check_spans(so, spans, true, vlen, sums.data());
  bool sums_ok = true;
  for (size_t x = 0; x < spans.size(); ++x) {
    uint64_t want = 0;
    for (int64_t y = spans[x].first; y < spans[x].first + spans[x].count; ++y)
      want += vlen[so[spans[x].set][y + 1] - so[spans[x].set][y]];
    sums_ok = sums_ok && sums[x] == want;
  }
  check(sums_ok, "check_spans: length-table sums per span");
  std::vector<int64_t> dst(2000000, -7);
  const int64_t ctot = sd::rebase_spans(so, spans, dst.data());
  std::vector<int64_t> want{0};
  for (const auto& sp : spans)
    for (int64_t y = sp.first; y < sp.first + sp.count; ++y)
      want.push_back(want.back() + so[sp.set][y + 1] - so[sp.set][y]);
  check(ctot == want.back() && std::equal(want.begin(), want.end(), dst.begin()) &&
            dst[want.size()] == -7,
        "rebase_spans: offsets laid end to end, nothing written past");
  // the spans' codes into one tile: device spans copied directly, host
  // spans through the pinned room, runs of host spans in one copy
  {
    std::vector<uint8_t> tile((size_t)ctot + 1, 0xEE), pin(sd::host_code_bytes(views.data(), spans));
    sd::stage_codes(views.data(), so, spans, dst.data(), tile.data(), pin.data(), nullptr);
    std::vector<uint8_t> want_codes;
    for (const auto& sp : spans)
      if (sp.count)
        want_codes.insert(want_codes.end(), sets[sp.set].codes.begin() + so[sp.set][sp.first],
                          sets[sp.set].codes.begin() + so[sp.set][sp.first + sp.count]);
    check(want_codes.size() == (size_t)ctot &&
              std::equal(want_codes.begin(), want_codes.end(), tile.begin()) && tile[ctot] == 0xEE,
          "stage_codes: the tile's codes in span order, nothing past");
  }
  // the first failing sequence in span order decides the error
  {
    std::vector<int64_t> o = sets[4].offs;
    o[300001] = o[300000];      // a length 0 (SD_E_LENGTH) ...
    o[400001] = o[400000] - 1;  // ... before a decreasing offset (SD_E_INVAL)
    std::vector<const int64_t*> v = so;
    v[4] = o.data();
    check(code_of([&] { sd::check_spans(v, spans, true, nullptr, nullptr); }) == SD_E_LENGTH,
          "check_spans: an earlier length error wins");
    check(code_of([&] { sd::check_spans(v, spans, false, nullptr, nullptr); }) == SD_E_INVAL,
          "check_spans: without length checks the offset error remains");
    check(code_of([&] { sd::check_spans(v, spans, false, vlen, sums.data()); }) == SD_E_LENGTH,
          "check_spans: a length table checks lengths too");
    o[300001] = o[300000] + 30;  // a length above 24
    o[300002] = o[300001] + 1;
    o[400001] = o[400000] + 1;
    check(code_of([&] { sd::check_spans(v, spans, true, nullptr, nullptr); }) == SD_E_LENGTH,
          "check_spans: a length above 24");
  }
  {
    std::vector<sd_seqs> bad = views;
    std::vector<int64_t> o = sets[2].offs;
    o[0] = 1;
    bad[2].offsets = o.data();
    check(code_of([&] { sd::set_offsets(bad.data(), 0, 6, area, nullptr); }) == SD_E_INVAL,
          "set_offsets: a device set whose first offset is not 0");
  }
  // host results cut from one (q, r)-sorted "device" result: three sets,
  // one split over two slices and one empty
  {
    const uint64_t n = 700000;
    std::vector<uint32_t> di(n), dj(n);
    std::vector<uint8_t> dd(n);
    for (uint64_t t = 0; t < n; ++t) {
      di[t] = (uint32_t)(1000 + t / 3);
      dj[t] = draw(1u << 30);
      dd[t] = (uint8_t)draw(3);
    }
    const std::vector<sd::HostSlice> sl = {
        {0, 0, 300000, 0, -1000}, {2, 300000, 100000, 0, 5}, {0, 400000, 300000, 300000, -7}};
    sd_pairs outs[3] = {};
    sd::host_result(c, 600000, &outs[0]);
    sd::host_result(c, 0, &outs[1]);
    sd::host_result(c, 100000, &outs[2]);
    sd::fill_host_slices(c, di.data(), dj.data(), dd.data(), n, sl, outs, nullptr);
    bool ok = outs[0].n == 600000 && outs[1].n == 0 && outs[2].n == 100000;
    for (const auto& x : sl)
      for (uint64_t t = 0; ok && t < x.n; ++t) {
        const sd_pairs& o = outs[x.set];
        ok = o.i[x.at + t] == (uint32_t)((int64_t)di[x.lo + t] + x.shift) &&
             o.j[x.at + t] == dj[x.lo + t] && o.d[x.at + t] == dd[x.lo + t];
      }
    check(ok, "fill_host_slices: every slice at its place, ids shifted");
    for (auto& o : outs) std::free(o.i);
  }
  sd::stage_done(c, nullptr);
  (void)sd::stage_area(c, 16);
  check(!c->stage_pending && events_live == 1, "stage_done / stage_area: one event, waited on");
  std::free(c->stage_host);
  delete c;
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
