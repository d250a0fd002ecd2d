// Host orchestration of the self-search pipeline (paper, Appendix A,
// XTNeighbor steps 1-7), all device work on the caller's stream:
//   1 pack            codes -> 128-bit keys, per-sequence variant counts
//   2 scan            variant offsets (decoupled look-back)
//   3 vargen          (key, id) for every <= k-deletion variant
//   4 group           stable LSD radix sort of (key, id) by the 128-bit key
//   5 emit            id pairs inside every run of equal keys
//   6 pair sort       LSD radix sort of the 64-bit pairs
//   7 verify          drop repeats, keep Levenshtein <= k, compact in order
// The host synchronises only to read sizes that decide allocations: the key
// total (with the validation flags), the non-trivial digits of the key sort,
// the candidate count and the result count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "sd_internal.h"

namespace sd {

namespace {

struct DevSeqs {
  const uint8_t* codes;
  const int64_t* offs;
  uint64_t n;
};

void check_seqs(const sd_seqs* s) {
  if (!s) throw Error{SD_E_INVAL, "null sequence set"};
  if (s->n < 0) throw Error{SD_E_INVAL, "negative sequence count"};
  if (s->n > 0 && (!s->codes || !s->offsets)) throw Error{SD_E_INVAL, "null codes or offsets"};
  if ((uint64_t)s->n >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "at most 2^32 - 2 sequences"};
}

DevSeqs stage_seqs(sd_ctx* c, Scratch& sc, const sd_seqs* s, hipStream_t st) {
  DevSeqs d{s->codes, s->offsets, (uint64_t)s->n};
  if (s->on_device || s->n == 0) return d;
  const int64_t total = s->offsets[s->n];
  if (s->offsets[0] != 0) throw Error{SD_E_INVAL, "offsets must start at 0"};
  for (int64_t x = 0; x < s->n; ++x)  // every sequence must lie inside codes[0, total)
    if (s->offsets[x + 1] < s->offsets[x]) throw Error{SD_E_INVAL, "offsets must not decrease"};
  uint8_t* codes = sc.get<uint8_t>((uint64_t)total + 1);
  int64_t* offs = sc.get<int64_t>((uint64_t)s->n + 1);
  if (total)
    hip_check(hipMemcpyAsync(codes, s->codes, (size_t)total, hipMemcpyHostToDevice, st), "H2D codes");
  hip_check(hipMemcpyAsync(offs, s->offsets, (size_t)(s->n + 1) * 8, hipMemcpyHostToDevice, st),
            "H2D offsets");
  d.codes = codes;
  d.offs = offs;
  return d;
}

void raise_validation(uint32_t err) {
  if (err & SD_ERRBIT_LENGTH) throw Error{SD_E_LENGTH, "a sequence length is outside [1, 24]"};
  if (err & SD_ERRBIT_ALPHABET) throw Error{SD_E_ALPHABET, "a residue code is >= 20"};
  if (err & SD_ERRBIT_INDEX) throw Error{SD_E_INVAL, "an index is out of range"};
}

int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b)) ++b;
  return b;
}

// Sort records by the given digit positions in LSD order; returns true if
// the result sits in the second buffer set.
bool radix_sort(sd_ctx* c, Scratch& sc, uint64_t* a0, uint64_t* a1, uint32_t* av, uint64_t* b0,
                uint64_t* b1, uint32_t* bv, int nwords, bool has_val, uint32_t n,
                const std::vector<int>& digits, const uint32_t* hist, uint32_t* counters,
                int& counter_slot, uint32_t* err, hipStream_t s) {
  bool flip = false;
  const uint64_t tiles = (n + onesweep_tile(nwords, has_val) - 1) / onesweep_tile(nwords, has_val);
  for (int q : digits) {
    const uint32_t epoch = next_epoch(c, tiles * 256, s);
    const uint64_t* i0 = flip ? b0 : a0;
    const uint64_t* i1 = flip ? b1 : a1;
    const uint32_t* iv = flip ? bv : av;
    uint64_t* o0 = flip ? a0 : b0;
    uint64_t* o1 = flip ? a1 : b1;
    uint32_t* ov = flip ? av : bv;
    launch_onesweep(i0, i1, iv, o0, o1, ov, nwords, has_val, n, q, hist + q * 256, c->status,
                    counters + counter_slot++, epoch, err, s);
    flip = !flip;
  }
  (void)sc;
  return flip;
}

}  // namespace

void self_search(sd_ctx* c, const sd_seqs* seqs, int k, sd_pairs* out, hipStream_t s) {
  check_seqs(seqs);
  if (k < 0 || k > 2) throw Error{SD_E_INVAL, "k must be 0, 1 or 2"};
  c->stats = sd_stats{};
  c->stats.n_seqs = seqs->n;
  if (seqs->n == 0) return;
  Scratch sc(c);
  StageTimer tm(c, s);
  const DevSeqs in = stage_seqs(c, sc, seqs, s);
  const uint64_t n = in.n;
  uint32_t* counters = fresh_counters(c, 128, s);
  int slot = 0;
  uint32_t* lb_err = counters + 100;  // look-back bound hits (checked at the end)

  // 1-2: pack and variant offsets
  u128* seq = sc.get<u128>(n);
  uint32_t* vcnt = sc.get<uint32_t>(n);
  uint64_t* voff = sc.get<uint64_t>(n + 1);
  uint32_t* err = counters + slot++;
  launch_pack(in.codes, in.offs, n, k, seq, vcnt, err, s);
  {
    const uint64_t tiles = (n + scan_tile() - 1) / scan_tile();
    const uint32_t epoch = next_epoch(c, tiles, s);
    launch_scan_excl(vcnt, voff, n, c->status, counters + slot++, epoch, lb_err, s);
  }
  tm.mark("pack_scan", (double)n * (16 + 16 + 8 + 4 + 4 + 8), 2);
  uint64_t nkeys;
  {
    // one read-back: validation flags (counter 0) and the key total
    hip_check(hipMemcpyAsync(counters + 64, voff + n, 8, hipMemcpyDeviceToDevice, s), "copy");
    const uint32_t* h = static_cast<const uint32_t*>(readback(c, counters, 66 * 4, s));
    raise_validation(h[0]);
    uint64_t tot;
    std::memcpy(&tot, h + 64, 8);
    nkeys = tot;
  }
  if (nkeys >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "more than 2^32 - 2 deletion variants"};
  c->stats.n_keys = (int64_t)nkeys;
  const uint32_t nk = (uint32_t)nkeys;

  // 3: variants
  uint64_t* klo = sc.get<uint64_t>(nk);
  uint64_t* khi = sc.get<uint64_t>(nk);
  uint32_t* kid = sc.get<uint32_t>(nk);
  uint64_t* klo2 = sc.get<uint64_t>(nk);
  uint64_t* khi2 = sc.get<uint64_t>(nk);
  uint32_t* kid2 = sc.get<uint32_t>(nk);
  launch_vargen(seq, voff, n, k, klo, khi, kid, s);
  tm.mark("vargen", (double)nk * 20 + (double)n * 24, 1);

  // 4: group equal keys (stable LSD radix sort over the non-trivial digits)
  uint32_t* hist = sc.get<uint32_t>(16 * 256);
  launch_fill_u32(hist, 0, 16 * 256, s);
  launch_radix_hist(klo, khi, 2, nk, hist, s);
  std::vector<int> digits;
  {
    const uint32_t* h = static_cast<const uint32_t*>(readback(c, hist, 16 * 256 * 4, s));
    for (int q = 0; q < 16; ++q) {
      bool trivial = false;
      for (int b = 0; b < 256; ++b)
        if (h[q * 256 + b] == nk) trivial = true;
      if (!trivial) digits.push_back(q);
    }
  }
  tm.mark("sort_hist", (double)nk * 16, 2);
  const bool kflip = radix_sort(c, sc, klo, khi, kid, klo2, khi2, kid2, 2, true, nk, digits, hist,
                                counters, slot, lb_err, s);
  c->stats.n_sort_passes = (int32_t)digits.size();
  tm.mark("sort_passes", (double)nk * 40 * digits.size(), (int)digits.size());
  const uint64_t* slo = kflip ? klo2 : klo;
  const uint64_t* shi = kflip ? khi2 : khi;
  const uint32_t* sid = kflip ? kid2 : kid;

  // 5: pairs inside groups of equal keys
  uint64_t cap = nk / 16 + 65536;
  uint64_t* cand = dalloc_t<uint64_t>(c, cap);
  unsigned long long* ccount = reinterpret_cast<unsigned long long*>(counters + 96);
  launch_emit_runs(slo, shi, sid, nk, cand, cap, ccount, s);
  uint64_t nc;
  {
    const uint64_t* h = static_cast<const uint64_t*>(readback(c, ccount, 8, s));
    nc = *h;
  }
  if (nc > cap) {  // capacity guess too small: grow and emit again
    dfree(c, cand);
    cap = nc;
    cand = dalloc_t<uint64_t>(c, cap);
    launch_fill_u64(reinterpret_cast<uint64_t*>(ccount), 0, 1, s);
    launch_emit_runs(slo, shi, sid, nk, cand, cap, ccount, s);
  }
  sc.blocks.push_back(cand);
  c->stats.n_cand_raw = (int64_t)nc;
  tm.mark("emit", (double)nk * 20 + (double)nc * 8, 1);
  if (nc >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "more than 2^32 - 2 candidate pairs"};

  // 6: sort candidate pairs (only the digits that can differ)
  uint64_t* cand2 = sc.get<uint64_t>(nc);
  const uint64_t* sorted = cand;
  if (nc > 1) {
    const int nb = bits_for(n - 1);
    std::vector<int> pd;
    for (int q = 0; q < (nb + 7) / 8; ++q) pd.push_back(q);
    for (int q = 0; q < (nb + 7) / 8; ++q) pd.push_back(4 + q);
    uint32_t* phist = sc.get<uint32_t>(8 * 256);
    launch_fill_u32(phist, 0, 8 * 256, s);
    launch_radix_hist(cand, nullptr, 1, nc, phist, s);
    const bool pflip = radix_sort(c, sc, cand, nullptr, nullptr, cand2, nullptr, nullptr, 1, false,
                                  (uint32_t)nc, pd, phist, counters, slot, lb_err, s);
    sorted = pflip ? cand2 : cand;
    tm.mark("pair_sort", (double)nc * 8 + (double)nc * 16 * pd.size(), 2 + (int)pd.size());
  } else {
    tm.mark("pair_sort", 0, 0);
  }

  // 7: verify and compact
  uint32_t* oi = dalloc_t<uint32_t>(c, nc);
  uint32_t* oj = dalloc_t<uint32_t>(c, nc);
  uint8_t* od = dalloc_t<uint8_t>(c, nc);
  uint64_t npairs = 0;
  try {
    unsigned long long* pcount = reinterpret_cast<unsigned long long*>(counters + 98);
    if (nc) {
      const uint64_t tiles = (nc + compact_tile() - 1) / compact_tile();
      const uint32_t epoch = next_epoch(c, tiles, s);
      launch_verify_compact(sorted, nc, seq, seq, k, oi, oj, od, c->status, counters + slot++,
                            epoch, pcount, lb_err, s);
      tm.mark("verify", (double)nc * (8 + 32) + (double)nc * 9, 1);
    } else {
      tm.mark("verify", 0, 0);
    }
    // counters 98-99: result count, 100: look-back errors
    const uint32_t* h = static_cast<const uint32_t*>(readback(c, counters + 98, 12, s));
    uint64_t cnt;
    std::memcpy(&cnt, h, 8);
    if (h[2] & SD_ERRBIT_LOOKBACK) throw Error{SD_E_HIP, "internal error: a look-back wait timed out"};
    npairs = nc ? cnt : 0;
    tm.finish();
  } catch (...) {
    dfree(c, oi);
    dfree(c, oj);
    dfree(c, od);
    throw;
  }
  c->stats.n_pairs = (int64_t)npairs;
  out->n = (int64_t)npairs;
  if (out->on_device) {
    out->i = oi;
    out->j = oj;
    out->d = od;
    return;
  }
  // host result: pinned arrays owned by the context until sd_pairs_free
  void *hi = nullptr, *hj = nullptr, *hd = nullptr;
  try {
    const size_t m = npairs ? npairs : 1;
    hip_check(hipHostMalloc(&hi, m * 4, hipHostMallocDefault), "hipHostMalloc");
    c->host_live[hi] = 1;
    hip_check(hipHostMalloc(&hj, m * 4, hipHostMallocDefault), "hipHostMalloc");
    c->host_live[hj] = 1;
    hip_check(hipHostMalloc(&hd, m, hipHostMallocDefault), "hipHostMalloc");
    c->host_live[hd] = 1;
    if (npairs) {
      hip_check(hipMemcpyAsync(hi, oi, npairs * 4, hipMemcpyDeviceToHost, s), "D2H");
      hip_check(hipMemcpyAsync(hj, oj, npairs * 4, hipMemcpyDeviceToHost, s), "D2H");
      hip_check(hipMemcpyAsync(hd, od, npairs, hipMemcpyDeviceToHost, s), "D2H");
    }
    hip_check(hipStreamSynchronize(s), "D2H synchronise");
  } catch (...) {
    for (void* p : {hi, hj, hd})
      if (p) {
        (void)hipHostFree(p);
        c->host_live.erase(p);
      }
    dfree(c, oi);
    dfree(c, oj);
    dfree(c, od);
    throw;
  }
  dfree(c, oi);
  dfree(c, oj);
  dfree(c, od);
  out->i = static_cast<uint32_t*>(hi);
  out->j = static_cast<uint32_t*>(hj);
  out->d = static_cast<uint8_t*>(hd);
}

void pair_distance(sd_ctx* c, const sd_seqs* a, const sd_seqs* b, const uint32_t* ia,
                   const uint32_t* ib, int64_t n, uint8_t* d_out, hipStream_t s) {
  check_seqs(a);
  check_seqs(b);
  if (n < 0 || (n > 0 && (!ia || !ib || !d_out))) throw Error{SD_E_INVAL, "bad pair arrays"};
  if (n == 0) return;
  Scratch sc(c);
  const DevSeqs da = stage_seqs(c, sc, a, s);
  const DevSeqs db = stage_seqs(c, sc, b, s);
  uint32_t* counters = fresh_counters(c, 128, s);
  u128* sa = sc.get<u128>(da.n);
  u128* sb = sc.get<u128>(db.n);
  launch_pack(da.codes, da.offs, da.n, 0, sa, nullptr, counters, s);
  launch_pack(db.codes, db.offs, db.n, 0, sb, nullptr, counters, s);
  const uint32_t* h = static_cast<const uint32_t*>(readback(c, counters, 4, s));
  raise_validation(h[0]);
  launch_pair_distance(sa, da.n, sb, db.n, ia, ib, (uint64_t)n, d_out, counters + 1, s);
  const uint32_t* e = static_cast<const uint32_t*>(readback(c, counters + 1, 4, s));
  if (e[0] & SD_ERRBIT_INDEX) throw Error{SD_E_INVAL, "a pair index is out of range"};
}

}  // namespace sd
