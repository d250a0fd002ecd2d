// Host orchestration of the self-search pipeline (paper, Appendix A,
// XTNeighbor steps 1-7). All device work runs on the caller's stream:
//   1 pack            codes -> 128-bit keys, per-sequence variant counts
//   2 scan            variant offsets (decoupled look-back)
//   3-5 grouping      equal deletion variants brought together and the id
//                     pairs inside every group emitted, by one of two paths:
//        full-key     (key, id) records, stable LSD radix sort over every
//                     non-trivial digit of the 128-bit key, run emission
//        hashed       64-bit elements [hash of the key | id], LSD passes over
//                     the top hash bits, grouping of each hash segment by the
//                     full stored hash in LDS (segments too large for LDS are
//                     sorted by the full hash); a hash collision only adds a
//                     candidate that step 7 rejects
//   6 pair sort       LSD radix sort of the 64-bit candidate pairs
//   7 verify          drop repeats, keep Levenshtein <= k, compact in order
// The host synchronises only to read sizes that decide allocations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sd_host.h"

namespace sd {

// Stable LSD sort of nk (key, id) records over the non-trivial digits of the
// 128-bit key.
SortedKeys full_key_sort(Call& cl, uint64_t* klo, uint64_t* khi, uint32_t* kid, uint32_t nk) {
  sd_ctx* c = cl.c;
  uint64_t* klo2 = cl.sc.get<uint64_t>(nk);
  uint64_t* khi2 = cl.sc.get<uint64_t>(nk);
  uint32_t* kid2 = cl.sc.get<uint32_t>(nk);
  uint32_t* hist = cl.sc.get<uint32_t>(16 * 256);
  launch_fill_u32(hist, 0, 16 * 256, cl.s);
  launch_radix_hist(klo, khi, 2, nk, hist, cl.s);
  std::vector<Digit> digits;
  std::vector<const uint32_t*> hists;
  {
    const uint32_t* h = static_cast<const uint32_t*>(readback(c, hist, 16 * 256 * 4, cl.s));
    for (int q = 0; q < 16; ++q) {
      bool trivial = false;  // every key has the same digit: the pass would not move anything
      for (int b = 0; b < 256; ++b)
        if (h[q * 256 + b] == nk) trivial = true;
      if (!trivial) {
        digits.push_back(Digit{q / 8, (q % 8) * 8, 255u});
        hists.push_back(hist + q * 256);
      }
    }
  }
  cl.tm.mark("sort_hist", (double)nk * 16, 2);
  const bool flip = radix_sort(cl, klo, khi, kid, klo2, khi2, kid2, 2, true, nk, digits, hists);
  cl.tm.mark("sort_passes", (double)nk * 40 * digits.size(), (int)digits.size());
  return SortedKeys{flip ? klo2 : klo, flip ? khi2 : khi, flip ? kid2 : kid, (int)digits.size()};
}

namespace {

// Full-key grouping: the key sort, then emission of the pairs in each run of
// equal keys.
Cands fullkey_group(Call& cl, uint64_t* klo, uint64_t* khi, uint32_t* kid, uint32_t nk,
                    int& passes_out) {
  sd_ctx* c = cl.c;
  const SortedKeys sk = full_key_sort(cl, klo, khi, kid, nk);
  passes_out = sk.passes;
  const uint64_t* slo = sk.lo;
  const uint64_t* shi = sk.hi;
  const uint32_t* sid = sk.id;

  uint64_t cap = nk / 16 + 65536;
  Cands out;
  out.p = dalloc_t<uint64_t>(c, cap);
  unsigned long long* ccount = reinterpret_cast<unsigned long long*>(cl.counters + CNT_CAND2);
  launch_fill_u64(reinterpret_cast<uint64_t*>(ccount), 0, 1, cl.s);
  launch_emit_runs(slo, shi, sid, nk, out.p, cap, ccount, cl.s);
  const uint64_t nc = *static_cast<const uint64_t*>(readback(c, ccount, 8, cl.s));
  if (nc > cap) {  // the capacity guess was too small: grow and emit again
    dfree(c, out.p);
    out.p = nullptr;
    out.p = dalloc_t<uint64_t>(c, nc);
    launch_fill_u64(reinterpret_cast<uint64_t*>(ccount), 0, 1, cl.s);
    launch_emit_runs(slo, shi, sid, nk, out.p, nc, ccount, cl.s);
  }
  out.n = nc;
  cl.tm.mark("emit", (double)nk * 20 + (double)nc * 8, 1);
  return out;
}

// Elements of hash segments too large for LDS: sort them by the full hash
// and emit pairs by runs of equal hash.
Cands oversized_group(Call& cl, const uint64_t* E, const uint64_t* big, uint64_t nb,
                      uint32_t idbits) {
  sd_ctx* c = cl.c;
  hipStream_t s = cl.s;
  std::vector<uint64_t> hb(2 * nb), off(nb);
  hip_check(hipMemcpyAsync(hb.data(), big, nb * 16, hipMemcpyDeviceToHost, s), "D2H big");
  hip_check(hipStreamSynchronize(s), "synchronise");
  uint64_t tot = 0;
  for (uint64_t x = 0; x < nb; ++x) {
    off[x] = tot;
    tot += hb[2 * x + 1] - hb[2 * x];
  }
  uint64_t* doff = cl.sc.get<uint64_t>(nb);
  hip_check(hipMemcpyAsync(doff, off.data(), nb * 8, hipMemcpyHostToDevice, s), "H2D offsets");
  uint64_t* g1 = cl.sc.get<uint64_t>(tot);
  uint64_t* g2 = cl.sc.get<uint64_t>(tot);
  launch_gather_big(E, big, doff, (uint32_t)nb, g1, s);
  uint32_t* hist = cl.sc.get<uint32_t>(8 * 256);
  launch_fill_u32(hist, 0, 8 * 256, s);
  launch_radix_hist(g1, nullptr, 1, tot, hist, s);
  const std::vector<Digit> digits = top_digits((int)idbits);
  std::vector<const uint32_t*> hists;
  for (const Digit& d : digits) hists.push_back(hist + (d.shift / 8) * 256);
  const bool flip =
      radix_sort(cl, g1, nullptr, nullptr, g2, nullptr, nullptr, 1, false, (uint32_t)tot, digits, hists);
  const uint64_t* sorted = flip ? g2 : g1;
  uint64_t cap = tot / 8 + 65536;
  Cands out;
  out.p = dalloc_t<uint64_t>(c, cap);
  unsigned long long* ccount = reinterpret_cast<unsigned long long*>(cl.counters + CNT_CAND2);
  launch_fill_u64(reinterpret_cast<uint64_t*>(ccount), 0, 1, s);
  launch_emit_hash_runs(sorted, tot, idbits, out.p, cap, ccount, s);
  const uint64_t nc = *static_cast<const uint64_t*>(readback(c, ccount, 8, s));
  if (nc > cap) {
    dfree(c, out.p);
    out.p = nullptr;
    out.p = dalloc_t<uint64_t>(c, nc);
    launch_fill_u64(reinterpret_cast<uint64_t*>(ccount), 0, 1, s);
    launch_emit_hash_runs(sorted, tot, idbits, out.p, nc, ccount, s);
  }
  out.n = nc;
  return out;
}

Cands group_segments(Call& cl, const uint64_t* E, uint32_t nk, int cap, int bits,
                     uint32_t idbits);

// Hashed grouping: elements [hash | id], LSD passes over the top `bits` hash
// bits, grouping of each segment by its full hash in LDS.
Cands hashed_group(Call& cl, const u128* seq, const uint64_t* voff, uint64_t n, int k, uint32_t nk,
                   int& passes_out) {
  sd_ctx* c = cl.c;
  hipStream_t s = cl.s;
  int cap, bits;
  hashed_plan(c, nk, &cap, &bits);
  const uint32_t idbits = n <= (1ull << 24) ? 24u : 32u;
  const std::vector<Digit> digits = bits ? top_digits(64 - bits) : std::vector<Digit>();
  uint64_t* e1 = cl.sc.get<uint64_t>(nk);
  uint64_t* e2 = cl.sc.get<uint64_t>(nk);
  uint32_t* hist = cl.sc.get<uint32_t>(3 * 256);
  launch_fill_u32(hist, 0, 3 * 256, s);
  uint32_t shifts[3] = {0, 0, 0}, masks[3] = {0, 0, 0};
  for (size_t x = 0; x < digits.size(); ++x) {
    shifts[x] = (uint32_t)digits[x].shift;
    masks[x] = digits[x].mask;
  }
  // the first pass's digits are counted during generation, per fixed tile of
  // the generator's output (the tiles every counted pass uses)
  const uint32_t spt = vargen_seqs_per_tile(n, nk);
  const uint64_t ftiles = fixed_tiles(nk);
  uint32_t* tcounts = nullptr;
  if (!digits.empty()) {
    tcounts = cl.sc.get<uint32_t>(ftiles * 256);
    launch_fill_u32(tcounts, 0, ftiles * 256, s);
  }
  // only the first pass's digits are counted by the generator (every later
  // pass is counted over fixed tiles of its own input)
  launch_vargen_hash(seq, voff, n, k, true, e1, idbits, digits.empty() ? 0 : 1, shifts, masks, hist,
                     tcounts, spt, s, fixed_tile_elems());
  cl.tm.mark("vargen_hash", (double)nk * 8 + (double)n * 24, 2);
  // pass 1 from the generator's counts (the count scans, then the scatter),
  // then the later passes
  bool flip = false;
  if (!digits.empty()) {
    uint32_t* local = cl.sc.get<uint32_t>(ftiles * 256);
    uint32_t* bsum = cl.sc.get<uint32_t>((uint64_t)counted_scan_rows(ftiles) * 256);
    launch_counted_scan(tcounts, ftiles, 1, local, bsum, s);
    cl.tm.mark("counted_scan", (double)ftiles * 256 * 12, 2);
    launch_counted_scatter(e1, e2, nk, digits[0].shift, digits[0].mask, ftiles, local, bsum,
                           nullptr, 0, 0, cl.lb_err(), s);
    cl.tm.mark("hash_counted_pass", (double)nk * 16, 1);
    flip = true;
  }
  // later passes: counted too, from a count of fixed tiles (a read of the
  // data instead of a look-back chain between tiles)
  for (size_t x = 1; x < digits.size(); ++x) {
    uint64_t* in = flip ? e2 : e1;
    uint64_t* other = flip ? e1 : e2;
    const uint64_t tiles = fixed_tiles(nk);
    uint32_t* counts = cl.sc.get<uint32_t>(tiles * 256);
    uint32_t* local = cl.sc.get<uint32_t>(tiles * 256);
    uint32_t* bsum = cl.sc.get<uint32_t>((uint64_t)counted_scan_rows(tiles) * 256);
    launch_tile_counts(in, nk, digits[x].shift, digits[x].mask, counts, s);
    launch_counted_scan(counts, tiles, 1, local, bsum, s);
    cl.tm.mark("tile_counts", (double)nk * 8 + (double)tiles * 256 * 12, 3);
    launch_counted_scatter(in, other, nk, digits[x].shift, digits[x].mask, tiles, local, bsum,
                           nullptr, 0, 0, cl.lb_err(), s);
    cl.tm.mark("hash_passes", (double)nk * 16, 1);
    flip = !flip;
  }
  passes_out = (int)digits.size();
  const uint64_t* E = flip ? e2 : e1;
  return group_segments(cl, E, nk, cap, bits, idbits);
}

// Grouping of elements sorted by their top `bits` bits: the segment table,
// then one workgroup per run of segments groups each by the full stored hash
// in LDS and emits the id pairs of every group; ranges too large for LDS are
// sorted by the full hash and emitted by runs.
Cands group_segments(Call& cl, const uint64_t* E, uint32_t nk, int cap, int bits,
                     uint32_t idbits) {
  sd_ctx* c = cl.c;
  hipStream_t s = cl.s;
  // segment table, then one workgroup per `spw` segment values
  const uint32_t nseg = 1u << bits;
  const uint32_t segshift = 64u - (uint32_t)bits;
  uint32_t* seg_start = cl.sc.get<uint32_t>(nseg);
  uint32_t* seg_end = cl.sc.get<uint32_t>(nseg);
  launch_seg_bounds(E, nk, segshift, seg_start, seg_end, s);
  cl.tm.mark("seg_bounds", (double)nseg * 8, 1);
  const double mean_seg = (double)nk / nseg;
  // segments per workgroup: about one LDS batch's worth, times the batches a
  // workgroup runs in sequence (the next batch's loads overlap the current
  // batch's grouping)
  const uint32_t per_batch =
      (uint32_t)std::max(1.0, std::floor(0.8 * cap / std::max(mean_seg, 1.0) + 0.5));
  const uint32_t spw = per_batch * (uint32_t)(c->group_batches ? c->group_batches : 4);
  // listed ranges: segments over 2 cap elements, split segments with a half
  // over cap / 2 candidates, and batches with over cap / 2 prefilter
  // candidates; each is listed once and holds more than cap / 2 elements of
  // its own, so 2 nk / cap entries suffice (twice that are allocated)
  const uint64_t nbig_cap = 4 * (uint64_t)nk / cap + 2;
  uint64_t* big = cl.sc.get<uint64_t>(2 * nbig_cap);
  uint64_t* big2 = cl.sc.get<uint64_t>(2 * nbig_cap);
  unsigned long long* nbig = reinterpret_cast<unsigned long long*>(cl.counters + CNT_NBIG);
  unsigned long long* nbig2 = reinterpret_cast<unsigned long long*>(cl.counters + CNT_NBIG2);
  static_assert(CNT_NBIG2 == CNT_NBIG + 2, "both counts are cleared by one fill");
  Cands cand = sharded_output(
      cl, nk / 24, "group_local",
      [&](const ShardArgs& out) {
        launch_fill_u64(reinterpret_cast<uint64_t*>(nbig), 0, 2, s);
        const uint32_t splitbit = segshift >= 1 ? segshift - 1 : 64u;
        launch_group_seg(cap, c->group_shape, E, seg_start, seg_end, nseg, spw, idbits, splitbit, out, big,
                         nbig, s);
        // the ranges listed above, with a table for a whole batch of
        // candidates; what still does not fit goes to big2
        launch_group_listed(cap, E, big, nbig, nbig_cap, idbits, splitbit, out, big2, nbig2, s);
      },
      [&](uint64_t n) { return (double)nk * 8 + (double)n * 8; });
  uint64_t nb[2];
  std::memcpy(nb, readback(c, nbig, 16, s), 16);
  if (nb[0] > nbig_cap) throw Error{SD_E_HIP, "internal error: listed ranges exceed their bound"};
  const uint64_t nb2 = nb[1];
  c->stats.n_big_segments = (int64_t)nb2;
  if (nb2) {
    Cands extra = oversized_group(cl, E, big2, nb2, idbits);
    if (extra.n) {
      uint64_t* merged = dalloc_t<uint64_t>(c, cand.n + extra.n);
      if (cand.n)
        hip_check(hipMemcpyAsync(merged, cand.p, cand.n * 8, hipMemcpyDeviceToDevice, s), "merge");
      hip_check(hipMemcpyAsync(merged + cand.n, extra.p, extra.n * 8, hipMemcpyDeviceToDevice, s),
                "merge");
      dfree(c, cand.p);
      cand.p = merged;
      cand.n += extra.n;
    }
    dfree(c, extra.p);
    cl.tm.mark("oversized", 0, 0);
  }
  return cand;
}

}  // namespace

uint64_t bucket_sort_verify(Call& cl, const BucketPlan& p, uint64_t* cand, uint64_t nc,
                            uint64_t* cand2, uint64_t na, uint64_t nbseq, const u128* a,
                            const u128* sb, int k, int self_pairs,
                            uint32_t* oi, uint32_t* oj, uint8_t* od, bool* over,
                            const char* sort_stage, const char* verify_stage, const u128* a2,
                            const u128* sb2) {
  sd_ctx* c = cl.c;
  hipStream_t s = cl.s;
  unsigned long long* pcount = reinterpret_cast<unsigned long long*>(cl.counters + CNT_PAIRS);
  launch_fill_u64(reinterpret_cast<uint64_t*>(pcount), 0, 1, s);
  BucketBufs b{cl.sc.get<uint32_t>(p.counts), cl.sc.get<uint64_t>(p.counts + 1),
               cl.sc.get<uint64_t>(nc),       cl.sc.get<uint32_t>(p.nb),
               cl.sc.get<uint64_t>(p.nb + 1),
               nullptr,                       cl.tile_counter(),
               0,                             cl.tile_counter(),
               0,                             cl.lb_err()};
  // two epochs of one status array (each scan sees only its own words)
  b.scan_epoch = next_epoch(c, bucket_status_words(p), s);
  b.scan2_epoch = next_epoch(c, bucket_status_words(p), s);
  b.status = c->status;
  launch_bucket_count(cand, nc, p.shift, p.nb, b.cnt, s);
  launch_scan_excl(b.cnt, b.off, p.counts, b.status, b.scan_ctr, b.scan_epoch, b.err, s);
  launch_bucket_scatter(cand, nc, p.shift, p.nb, b.off, cand2, s);
  cl.tm.mark(sort_stage, (double)nc * 24 + (double)p.counts * 24, 3);
  launch_bucket_verify(cand2, cand, b.packed, b.off, nc, p.nb, p.jb, p.low, na, nbseq, a, sb, k,
                       c->metric, self_pairs, b.bcount, b.err, s, a2, sb2);
  launch_scan_excl(b.bcount, b.bpos, p.nb, b.status, b.scan2_ctr, b.scan2_epoch, b.err, s);
  launch_bucket_place(b.packed, b.off, nc, p.nb, p.jb, p.low, b.bcount, b.bpos, oi, oj, od,
                      pcount, s);
  cl.tm.mark(verify_stage, (double)nc * 8, 3);
  const uint32_t* h = static_cast<const uint32_t*>(readback(c, cl.counters + CNT_PAIRS, 12, s));
  uint64_t cntp;
  std::memcpy(&cntp, h, 8);
  if (h[2] & SD_ERRBIT_LOOKBACK) throw Error{SD_E_HIP, "internal error: a look-back wait timed out"};
  if (h[2] & SD_ERRBIT_PLACEMENT) throw Error{SD_E_HIP, "internal error: a counted pass misplaced"};
  if (h[2] & SD_ERRBIT_INDEX) throw Error{SD_E_HIP, "internal error: a candidate id out of range"};
  *over = (h[2] & SD_ERRBIT_BUCKET) != 0;
  if (*over) launch_fill_u32(cl.lb_err(), 0, 1, s);
  return cntp;
}

// Tunables of the hashed path for a key count: the LDS capacity of a batch
// and the number of hash bits the LSD passes sort by. Segment sizes are close
// to Poisson(mean), so the bits are the fewest for which mean + 3.5 sqrt(mean)
// fits the capacity (the rare larger segment takes the sort-and-runs path).
// Context options override either.
void hashed_plan(const sd_ctx* c, uint64_t nk, int* cap, int* bits) {
  const int cp = c->group_cap ? c->group_cap : 2048;
  int b = c->group_bits;
  if (b <= 0) {
    b = 0;
    while (b < 23) {
      const double mean = (double)nk / (double)(1ull << b);
      if (mean + 3.5 * std::sqrt(mean) <= cp) break;
      ++b;
    }
  }
  *cap = cp;
  *bits = b;
}

namespace {

// Steps 6-7 on a candidate array: sort the (i << 32 | j) candidates over the
// digits that can differ, then drop repeats, keep the pairs within k and
// compact them in order. n is the number of sequences (ids are below n).
struct Verified {
  uint32_t* i = nullptr;
  uint32_t* j = nullptr;
  uint8_t* d = nullptr;
  uint64_t n = 0;
};

Verified sort_and_verify(Call& cl, uint64_t* cand, uint64_t nc, uint64_t n, int k, const u128* seq,
                         const u128* planes, const u128* seq2 = nullptr,
                         const u128* planes2 = nullptr) {
  sd_ctx* c = cl.c;
  hipStream_t s = cl.s;
  if (nc >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "more than 2^32 - 2 candidate pairs"};
  uint64_t* cand2 = cl.sc.get<uint64_t>(nc);
  const int jb = std::max(1, bits_for(n - 1));
  const BucketPlan bp = bucket_plan(c, nc, jb, jb);
  if (bp.bits >= 0) {
    // 6-7 bucketed: one scatter by the top bits of i, then per bucket a sort,
    // the repeats dropped and the verification, all in LDS
    c->stats.n_pair_buckets += bp.nb;
    Verified v;
    v.i = dalloc_t<uint32_t>(c, nc);
    v.j = dalloc_t<uint32_t>(c, nc);
    v.d = dalloc_t<uint8_t>(c, nc);
    bool over = false;
    try {
      v.n = bucket_sort_verify(cl, bp, cand, nc, cand2, n, n,
                               c->metric == SD_METRIC_HAMMING ? seq : planes, seq, k, 1, v.i, v.j,
                               v.d, &over, "pair_sort", "verify", planes2, seq2);
    } catch (...) {
      dfree(c, v.i);
      dfree(c, v.j);
      dfree(c, v.d);
      throw;
    }
    if (!over) return v;
    // a bucket too large even for one workgroup's sort in global memory
    // (very many candidates of a few sequences): sort and verify the whole
    // bucketed copy with global passes instead (the first array was
    // overwritten)
    dfree(c, v.i);
    dfree(c, v.j);
    dfree(c, v.d);
    c->stats.n_pair_fallbacks += 1;
    std::swap(cand, cand2);
  }
  // 6: sort candidate pairs (only the digits that can differ)
  const uint64_t* sorted = cand;
  if (nc > 1) {
    const int nb = bits_for(n - 1);
    std::vector<Digit> pd;
    for (int q = 0; q < (nb + 7) / 8; ++q) pd.push_back(Digit{0, 8 * q, 255u});
    for (int q = 0; q < (nb + 7) / 8; ++q) pd.push_back(Digit{0, 32 + 8 * q, 255u});
    bool pflip;
    if (pair_sort_counted(c, nc)) {
      // large: counted passes over fixed tiles
      pflip = counted_sort(cl, cand, cand2, (uint32_t)nc, pd);
      cl.tm.mark("pair_sort", (double)nc * 24 * pd.size(), 4 * (int)pd.size());
    } else {
      // small: one histogram, then onesweep passes (fewer launches)
      std::vector<const uint32_t*> ph;
      uint32_t* phist = cl.sc.get<uint32_t>(8 * 256);
      launch_fill_u32(phist, 0, 8 * 256, s);
      launch_radix_hist(cand, nullptr, 1, nc, phist, s);
      for (const Digit& d : pd) ph.push_back(phist + (d.shift / 8) * 256);
      pflip = radix_sort(cl, cand, nullptr, nullptr, cand2, nullptr, nullptr, 1, false,
                         (uint32_t)nc, pd, ph);
      cl.tm.mark("pair_sort", (double)nc * 8 + (double)nc * 16 * pd.size(), 2 + (int)pd.size());
    }
    sorted = pflip ? cand2 : cand;
  } else {
    cl.tm.mark("pair_sort", 0, 0);
  }

  // 7: verify and compact
  Verified v;
  v.i = dalloc_t<uint32_t>(c, nc);
  v.j = dalloc_t<uint32_t>(c, nc);
  v.d = dalloc_t<uint8_t>(c, nc);
  try {
    unsigned long long* pcount = reinterpret_cast<unsigned long long*>(cl.counters + CNT_PAIRS);
    launch_fill_u64(reinterpret_cast<uint64_t*>(pcount), 0, 1, s);
    if (nc) {
      const uint64_t tiles = (nc + compact_tile() - 1) / compact_tile();
      const uint32_t epoch = next_epoch(c, tiles, s);
      launch_verify_compact(sorted, nc, n, n, c->metric == SD_METRIC_HAMMING ? seq : planes, seq, k,
                            c->metric, 1, v.i, v.j, v.d, c->status, cl.tile_counter(), epoch,
                            pcount, cl.lb_err(), s, planes2, seq2);
      cl.tm.mark("verify", (double)nc * (8 + 32) + (double)nc * 9, 1);
    } else {
      cl.tm.mark("verify", 0, 0);
    }
    const uint32_t* h = static_cast<const uint32_t*>(readback(c, cl.counters + CNT_PAIRS, 12, s));
    uint64_t cnt;
    std::memcpy(&cnt, h, 8);
    if (h[2] & SD_ERRBIT_LOOKBACK) throw Error{SD_E_HIP, "internal error: a look-back wait timed out"};
    if (h[2] & SD_ERRBIT_PLACEMENT) throw Error{SD_E_HIP, "internal error: a counted pass misplaced"};
    if (h[2] & SD_ERRBIT_INDEX) throw Error{SD_E_HIP, "internal error: a candidate id out of range"};
    v.n = nc ? cnt : 0;
  } catch (...) {
    dfree(c, v.i);
    dfree(c, v.j);
    dfree(c, v.d);
    throw;
  }
  return v;
}

// Device bytes per element of a column group at its peak (the sharded
// generation output and the gathered elements; later, the two sort buffers,
// tile counts and candidates), and per sequence for what the streamed search
// keeps throughout (packed keys, bit planes, counts, offsets, pairs found).
constexpr uint64_t kStreamBytesPerElem = 24;
constexpr uint64_t kStreamBytesPerSeq = 64;

// Elements per column group of a streamed search, or 0 to search in memory:
// SD_OPT_STREAM 1 never streams, 2 always does; automatically, a search
// streams when its variants exceed what 32-bit element counts address or what
// the in-memory path (two 8-byte element buffers, tile counts and candidates:
// about 18 bytes per variant) would need beyond the context's budget.
uint64_t stream_group_elems(const sd_ctx* c, uint64_t n, uint64_t nkeys) {
  if (c->stream == 1 || c->path == 1) {
    if (nkeys >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "more than 2^32 - 2 deletion variants"};
    return 0;
  }
  const uint64_t fixed = kStreamBytesPerSeq * n + (1ull << 20);
  const bool too_many = nkeys >= 0xFFFFFFFFull;
  const bool over_budget = c->budget && fixed + 18 * nkeys > c->budget;
  if (c->stream != 2 && !too_many && !over_budget) return 0;
  uint64_t cap = c->stream_elems;
  if (!cap) {
    uint64_t avail = 0;
    if (c->budget) {
      avail = c->budget > fixed ? c->budget - fixed : 0;
    } else {
      size_t fr = 0, tot = 0;
      hip_check(hipMemGetInfo(&fr, &tot), "hipMemGetInfo");
      avail = (uint64_t)fr / 10 * 8;
    }
    cap = avail / kStreamBytesPerElem;
  }
  cap = std::min<uint64_t>(cap, 0xFFFFFFFEull);
  if (cap < 4096) throw Error{SD_E_NOMEM, "the device memory budget leaves no room for a column group"};
  return cap;
}

// Streamed self search (Section II C, "Overcoming memory bottlenecks", and
// the XTNeighbor-Streaming steps of Appendix A), for variant sets larger than
// device memory or the budget allows. The variant space is cut into
// 2^STREAM_BIN_BITS bins by the top bits of the variant hash; equal variants
// share a bin, so every group of equal variants lies in one bin. A first
// generator pass only counts each bin's variants; Next-Fit packing then
// forms column groups of consecutive bins that fit the per-group capacity
// (order-preserving, as in the paper). Each column group is one pass: the
// generator runs over every sequence again and keeps the group's variants
// (the paper's 2-D buffer read column-wise: rows are the generator
// workgroups' sequence ranges, columns the bins), and the in-memory path's
// grouping, pair sort and verification run on them alone. A pair can share
// variants in several groups, so the pairs of all groups are sorted, made
// unique and verified once more at the end (the paper's cross-chunk
// duplicate removal, bounded by the pairs instead of the candidates).
Verified streamed_search(Call& cl, const u128* seq, const u128* planes, const uint64_t* voff,
                         uint64_t n, int k, uint64_t nkeys, uint64_t cap) {
  sd_ctx* c = cl.c;
  hipStream_t s = cl.s;
  const uint32_t idbits = n <= (1ull << 24) ? 24u : 32u;
  const uint32_t spb = vargen_seqs_per_tile(n, nkeys);
  constexpr uint32_t NBINS = 1u << STREAM_BIN_BITS;
  uint32_t* bins = cl.sc.get<uint32_t>(NBINS);
  launch_fill_u32(bins, 0, NBINS, s);
  launch_vargen_bins(seq, voff, n, k, idbits, bins, spb, s);
  cl.tm.mark("stream_bins", (double)n * 24, 1);
  std::vector<uint64_t> cnt(NBINS);
  {
    const uint32_t* h = static_cast<const uint32_t*>(readback(c, bins, NBINS * 4, s));
    for (uint32_t b = 0; b < NBINS; ++b) cnt[b] = h[b];
  }
  // Next-Fit: consecutive bins while they fit the capacity
  struct Group {
    uint32_t lo, hi;
    uint64_t n;
  };
  std::vector<Group> groups;
  for (uint32_t b = 0; b < NBINS; ++b) {
    if (cnt[b] > cap)
      throw Error{SD_E_NOMEM, "a hash bin of " + std::to_string(cnt[b]) +
                                  " variants exceeds the column-group capacity of " +
                                  std::to_string(cap) + " (raise the device memory budget)"};
    if (!cnt[b]) continue;
    if (groups.empty() || groups.back().n + cnt[b] > cap)
      groups.push_back(Group{b, b + 1, cnt[b]});
    else {
      groups.back().hi = b + 1;
      groups.back().n += cnt[b];
    }
  }
  c->stats.n_stream_groups = (int64_t)groups.size();
  // the verified pairs of every group, as (i << 32 | j), appended in turn
  std::vector<std::pair<uint64_t*, uint64_t>> found;
  uint64_t nfound = 0;
  int passes = 0;
  uint64_t raw = 0;
  try {
    for (const Group& g : groups) {
      Scratch gsc(c);
      Call gcl{c, s, gsc, cl.tm, cl.counters};
      // the column group's elements, gathered into one array
      Cands E;
      {
        Scratch shard_sc(c);  // the shard regions are given back after the gather
        Call scl{c, s, shard_sc, cl.tm, cl.counters};
        E = sharded_output(
            scl, g.n, "stream_gen",
            [&](const ShardArgs& a) {
              launch_vargen_stream(seq, voff, n, k, idbits, g.lo, g.hi, a, spb, s);
            },
            [&](uint64_t m) { return (double)n * 24 + (double)m * 8; }, true);
      }
      gsc.blocks.push_back(E.p);
      if (E.n != g.n) throw Error{SD_E_HIP, "internal error: a column group lost variants"};
      const uint32_t ng = (uint32_t)E.n;
      int gcap, bits;
      hashed_plan(c, ng, &gcap, &bits);
      const std::vector<Digit> digits = bits ? top_digits(64 - bits) : std::vector<Digit>();
      uint64_t* e2 = gsc.get<uint64_t>(ng);
      // counted LSD passes over fixed tiles (a count of each pass's input,
      // the count scans, the XCD-contiguous scatter), timed as the in-memory
      // path's later passes are
      bool flip = false;
      if (!digits.empty()) {
        const uint64_t tiles = fixed_tiles(ng);
        uint32_t* counts = gsc.get<uint32_t>(tiles * 256);
        uint32_t* local = gsc.get<uint32_t>(tiles * 256);
        uint32_t* bsum = gsc.get<uint32_t>((uint64_t)counted_scan_rows(tiles) * 256);
        for (const Digit& d : digits) {
          const uint64_t* in = flip ? e2 : E.p;
          uint64_t* outp = flip ? E.p : e2;
          launch_tile_counts(in, ng, d.shift, d.mask, counts, s);
          launch_counted_scan(counts, tiles, 1, local, bsum, s);
          cl.tm.mark("tile_counts", (double)ng * 8 + (double)tiles * 256 * 12, 3);
          launch_counted_scatter(in, outp, ng, d.shift, d.mask, tiles, local, bsum, nullptr, 0, 0,
                                 cl.lb_err(), s);
          cl.tm.mark("hash_passes", (double)ng * 16, 1);
          flip = !flip;
        }
      }
      passes += (int)digits.size();
      Cands cand = group_segments(gcl, flip ? e2 : E.p, ng, gcap, bits, idbits);
      gsc.blocks.push_back(cand.p);
      raw += cand.n;
      const Verified v = sort_and_verify(gcl, cand.p, cand.n, n, k, seq, planes);
      gsc.blocks.push_back(v.i);
      gsc.blocks.push_back(v.j);
      gsc.blocks.push_back(v.d);
      uint64_t* ij = dalloc_t<uint64_t>(c, v.n);
      found.push_back({ij, v.n});
      launch_join_pairs(v.i, v.j, v.n, ij, s);
      nfound += v.n;
    }
    c->stats.n_sort_passes = passes;
    c->stats.n_cand_raw = (int64_t)raw;
    // all groups' pairs: one array, then the cross-group duplicates go
    uint64_t* all = cl.sc.get<uint64_t>(nfound);
    uint64_t at = 0;
    for (auto& f : found) {
      if (f.second)
        hip_check(hipMemcpyAsync(all + at, f.first, f.second * 8, hipMemcpyDeviceToDevice, s),
                  "merge pairs");
      at += f.second;
      dfree(c, f.first);
      f.first = nullptr;
    }
    return sort_and_verify(cl, all, nfound, n, k, seq, planes);
  } catch (...) {
    for (auto& f : found) dfree(c, f.first);
    throw;
  }
}

}  // namespace

// Paired-chain self search (Discussion: the two chains of a receptor joined
// by a token that is never deleted): every pair of records i < j with
// Lev(a_i, a_j) + Lev(b_i, b_j) <= k. Both chains are packed and validated
// as single chains; the variants of the joined strings go through the hashed
// grouping, the pair sort and a verification that sums both chains'
// distances.
void paired_self_search(sd_ctx* c, const sd_seqs* a, const sd_seqs* b, int k, sd_pairs* out,
                        hipStream_t s) {
  check_seqs(a);
  check_seqs(b);
  if (a->n != b->n) throw Error{SD_E_INVAL, "both chains must hold the same number of records"};
  if (k < 0 || k > 3) throw Error{SD_E_INVAL, "k must be 0, 1, 2 or 3"};
  c->stats = sd_stats{};
  c->stats.n_seqs = a->n;
  if (a->n == 0) return;
  Scratch sc(c);
  StageTimer tm(c, s);
  const DevSeqs ia = stage_seqs(c, sc, a, s);
  const DevSeqs ib = stage_seqs(c, sc, b, s);
  const uint64_t n = ia.n;
  Call cl{c, s, sc, tm, fresh_counters(c, CNT_TOTAL, s)};
  uint32_t* counters = cl.counters;
  u128* sa = sc.get<u128>(n);
  u128* pa = sc.get<u128>(n);
  u128* sb = sc.get<u128>(n);
  u128* pb = sc.get<u128>(n);
  uint32_t* vcnt = sc.get<uint32_t>(n);
  uint64_t* voff = sc.get<uint64_t>(n + 1);
  launch_pack(ia.codes, ia.offs, n, 0, false, sa, pa, nullptr, counters + CNT_ERR, s);
  launch_pack(ib.codes, ib.offs, n, 0, false, sb, pb, nullptr, counters + CNT_ERR, s);
  launch_paired_count(sa, sb, n, k, vcnt, s);
  {
    const uint64_t tiles = (n + scan_tile() - 1) / scan_tile();
    const uint32_t epoch = next_epoch(c, tiles, s);
    launch_scan_excl(vcnt, voff, n, c->status, cl.tile_counter(), epoch, cl.lb_err(), s);
  }
  tm.mark("pack_scan", (double)n * 2 * (16 + 16 + 16 + 8) + (double)n * 12, 4);
  uint64_t nkeys;
  {
    hip_check(hipMemcpyAsync(counters + CNT_NKEYS, voff + n, 8, hipMemcpyDeviceToDevice, s), "copy");
    const uint32_t* h = static_cast<const uint32_t*>(readback(c, counters, (CNT_NKEYS + 2) * 4, s));
    raise_validation(h[CNT_ERR]);
    std::memcpy(&nkeys, h + CNT_NKEYS, 8);
  }
  if (nkeys >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "more than 2^32 - 2 deletion variants"};
  c->stats.n_keys = (int64_t)nkeys;
  const uint32_t nk = (uint32_t)nkeys;
  const uint32_t idbits = n <= (1ull << 24) ? 24u : 32u;
  uint64_t* e1 = sc.get<uint64_t>(nk);
  uint64_t* e2 = sc.get<uint64_t>(nk);
  launch_vargen_paired(sa, sb, voff, n, k, idbits, e1, s);
  tm.mark("vargen_paired", (double)nk * 8 + (double)n * 40, 1);
  int cap, bits;
  hashed_plan(c, nk, &cap, &bits);
  const std::vector<Digit> digits = bits ? top_digits(64 - bits) : std::vector<Digit>();
  const bool flip = digits.empty() ? false : counted_sort(cl, e1, e2, nk, digits);
  tm.mark("hash_passes", (double)nk * 24 * digits.size(), 4 * (int)digits.size());
  c->stats.n_sort_passes = (int)digits.size();
  Cands cand = group_segments(cl, flip ? e2 : e1, nk, cap, bits, idbits);
  sc.blocks.push_back(cand.p);
  c->stats.n_cand_raw = (int64_t)cand.n;
  const Verified v = sort_and_verify(cl, cand.p, cand.n, n, k, sa, pa, sb, pb);
  try {
    tm.finish();
  } catch (...) {
    dfree(c, v.i);
    dfree(c, v.j);
    dfree(c, v.d);
    throw;
  }
  c->stats.n_pairs = (int64_t)v.n;
  finish_output(c, v.i, v.j, v.d, v.n, out, s);
}

void self_search(sd_ctx* c, const sd_seqs* seqs, int k, sd_pairs* out, hipStream_t s) {
  check_seqs(seqs);
  if (k < 0 || k > 3) throw Error{SD_E_INVAL, "k must be 0, 1, 2 or 3"};
  if (k == 3 && c->path == 1)
    throw Error{SD_E_INVAL, "k = 3 runs on the hashed grouping path only (SD_OPT_PATH 0 or 2)"};
  c->stats = sd_stats{};
  c->stats.n_seqs = seqs->n;
  if (seqs->n == 0) return;
  Scratch sc(c);
  StageTimer tm(c, s);
  const DevSeqs in = stage_seqs(c, sc, seqs, s);
  const uint64_t n = in.n;
  Call cl{c, s, sc, tm, fresh_counters(c, CNT_TOTAL, s)};
  uint32_t* counters = cl.counters;

  // 1-2: pack and variant offsets
  u128* seq = sc.get<u128>(n);
  u128* planes = sc.get<u128>(n);
  uint32_t* vcnt = sc.get<uint32_t>(n);
  uint64_t* voff = sc.get<uint64_t>(n + 1);
  // the hashed path generates each distinct variant string of a sequence once
  launch_pack(in.codes, in.offs, n, k, c->path != 1, seq, planes, vcnt, counters + CNT_ERR, s);
  {
    const uint64_t tiles = (n + scan_tile() - 1) / scan_tile();
    const uint32_t epoch = next_epoch(c, tiles, s);
    launch_scan_excl(vcnt, voff, n, c->status, cl.tile_counter(), epoch, cl.lb_err(), s);
  }
  tm.mark("pack_scan", (double)n * (16 + 16 + 16 + 8 + 4 + 4 + 8), 2);
  uint64_t nkeys;
  {
    // one read-back: validation flags and the key total
    hip_check(hipMemcpyAsync(counters + CNT_NKEYS, voff + n, 8, hipMemcpyDeviceToDevice, s), "copy");
    const uint32_t* h = static_cast<const uint32_t*>(readback(c, counters, (CNT_NKEYS + 2) * 4, s));
    raise_validation(h[CNT_ERR]);
    std::memcpy(&nkeys, h + CNT_NKEYS, 8);
  }
  c->stats.n_keys = (int64_t)nkeys;

  Verified v;
  const uint64_t group_elems = stream_group_elems(c, n, nkeys);
  if (group_elems) {
    v = streamed_search(cl, seq, planes, voff, n, k, nkeys, group_elems);
  } else {
    // 3-5: grouping and in-group emission
    const uint32_t nk = (uint32_t)nkeys;
    Cands cand;
    int passes = 0;
    if (c->path == 1) {
      uint64_t* klo = sc.get<uint64_t>(nk);
      uint64_t* khi = sc.get<uint64_t>(nk);
      uint32_t* kid = sc.get<uint32_t>(nk);
      launch_vargen(seq, voff, n, k, klo, khi, kid, s);
      tm.mark("vargen", (double)nk * 20 + (double)n * 24, 1);
      cand = fullkey_group(cl, klo, khi, kid, nk, passes);
    } else {
      cand = hashed_group(cl, seq, voff, n, k, nk, passes);
    }
    sc.blocks.push_back(cand.p);
    c->stats.n_sort_passes = passes;
    c->stats.n_cand_raw = (int64_t)cand.n;
    // 6-7: pair sort, verification
    v = sort_and_verify(cl, cand.p, cand.n, n, k, seq, planes);
  }
  try {
    tm.finish();
  } catch (...) {
    dfree(c, v.i);
    dfree(c, v.j);
    dfree(c, v.d);
    throw;
  }
  c->stats.n_pairs = (int64_t)v.n;
  finish_output(c, v.i, v.j, v.d, v.n, out, s);
}

void finish_output(sd_ctx* c, uint32_t* oi, uint32_t* oj, uint8_t* od, uint64_t npairs,
                   sd_pairs* out, hipStream_t s) {
  out->n = (int64_t)npairs;
  if (out->on_device) {
    out->i = oi;
    out->j = oj;
    out->d = od;
    return;
  }
  // host result: one pinned block (i, j, then d) owned by the context until
  // sd_pairs_free
  void* blk = nullptr;
  const size_t m = npairs ? npairs : 1;
  try {
    blk = host_block(c, m * 9);
    if (npairs) {
      uint8_t* h = static_cast<uint8_t*>(blk);
      hip_check(hipMemcpyAsync(h, oi, npairs * 4, hipMemcpyDeviceToHost, s), "D2H");
      hip_check(hipMemcpyAsync(h + m * 4, oj, npairs * 4, hipMemcpyDeviceToHost, s), "D2H");
      hip_check(hipMemcpyAsync(h + m * 8, od, npairs, hipMemcpyDeviceToHost, s), "D2H");
    }
    hip_check(hipStreamSynchronize(s), "D2H synchronise");
  } catch (...) {
    if (blk) host_release(c, blk);
    dfree(c, oi);
    dfree(c, oj);
    dfree(c, od);
    out->n = 0;
    throw;
  }
  dfree(c, oi);
  dfree(c, oj);
  dfree(c, od);
  uint8_t* h = static_cast<uint8_t*>(blk);
  out->i = reinterpret_cast<uint32_t*>(h);
  out->j = reinterpret_cast<uint32_t*>(h + m * 4);
  out->d = h + m * 8;
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
  uint32_t* counters = fresh_counters(c, CNT_TOTAL, s);
  u128* sa = sc.get<u128>(da.n);
  u128* sb = sc.get<u128>(db.n);
  launch_pack(da.codes, da.offs, da.n, 0, false, sa, nullptr, nullptr, counters, s);
  launch_pack(db.codes, db.offs, db.n, 0, false, sb, nullptr, nullptr, counters, s);
  const uint32_t* h = static_cast<const uint32_t*>(readback(c, counters, 4, s));
  raise_validation(h[0]);
  launch_pair_distance(sa, da.n, sb, db.n, ia, ib, (uint64_t)n, d_out, counters + 1, s);
  const uint32_t* e = static_cast<const uint32_t*>(readback(c, counters + 1, 4, s));
  if (e[0] & SD_ERRBIT_INDEX) throw Error{SD_E_INVAL, "a pair index is out of range"};
}

}  // namespace sd
