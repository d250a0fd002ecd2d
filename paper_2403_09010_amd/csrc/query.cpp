// Query-versus-reference search (paper Section II A lookup with the variant
// map built once for the reference; Section IV database lookups; Section
// III D weighted rescoring after the Levenshtein prefilter).
//
// Index build (once per reference set R and radius k):
//   pack, scan, every <= k-deletion variant of R as [hash | ref id], sorted by
//   the full hash, repeated elements removed, and a directory of 2^B hash
//   segments. The index owns its device memory and is shared read-only.
// Query (per tile of query sequences, one or many sets concatenated):
//   pack, scan, query variants as [hash | query id], LSD passes over the same
//   top B hash bits, query segment table, a segment-wise join against the
//   index, pair sort, exact verification (or weighted rescoring), and for a
//   batch of sets a split of the sorted result into per-set slices.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sd_host.h"

namespace sd {

Packed pack_and_count(Call& cl, const DevSeqs& in, int k, bool distinct) {
  Packed p;
  p.seq = cl.sc.get<u128>(in.n);
  p.planes = cl.sc.get<u128>(in.n);
  uint32_t* vcnt = cl.sc.get<uint32_t>(in.n);
  p.voff = cl.sc.get<uint64_t>(in.n + 1);
  launch_fill_u32(cl.counters + CNT_ERR, 0, 1, cl.s);
  launch_pack(in.codes, in.offs, in.n, k, distinct, p.seq, p.planes, vcnt, cl.counters + CNT_ERR,
              cl.s);
  const uint64_t tiles = (in.n + scan_tile() - 1) / scan_tile();
  const uint32_t epoch = next_epoch(cl.c, tiles, cl.s);
  launch_scan_excl(vcnt, p.voff, in.n, cl.c->status, cl.tile_counter(), epoch, cl.lb_err(), cl.s);
  hip_check(hipMemcpyAsync(cl.counters + CNT_NKEYS, p.voff + in.n, 8, hipMemcpyDeviceToDevice, cl.s),
            "copy");
  const uint32_t* h =
      static_cast<const uint32_t*>(readback(cl.c, cl.counters, (CNT_NKEYS + 2) * 4, cl.s));
  raise_validation(h[CNT_ERR]);
  std::memcpy(&p.nkeys, h + CNT_NKEYS, 8);
  if (p.nkeys >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "more than 2^32 - 2 deletion variants"};
  return p;
}

void check_lookback(Call& cl) {
  const uint32_t* h = static_cast<const uint32_t*>(readback(cl.c, cl.counters + CNT_LBERR, 4, cl.s));
  if (h[0] & SD_ERRBIT_LOOKBACK) throw Error{SD_E_HIP, "internal error: a look-back wait timed out"};
  if (h[0] & SD_ERRBIT_PLACEMENT) throw Error{SD_E_HIP, "internal error: a counted pass misplaced"};
}

namespace {

constexpr uint32_t JOIN_LDS_MIN_Q = 8;  // segments with fewer query elements search global memory

int index_bits(uint64_t nkeys) {
  // segments of about 1/2 to 1/4 of the join kernel's LDS capacity
  int b = 0;
  while (b < 24 && (double)nkeys / (double)(1ull << b) > 0.4 * join_cap()) ++b;
  return b;
}

// Hash bits of a query tile's join segments: the index's own B, or fewer
// for a small tile (about `per` query elements a segment, at least 2^4
// segments; `per` is the cube root of the tile's element count, at least
// 64, unless SD_OPT_JOIN_ELEMS sets it; 1 keeps the index's own). The join runs one workgroup per segment, so with the
// index's 2^B segments a small query would launch mostly workgroups that
// find no query element, and each would stage its index segment in LDS for
// a few lookups; a coarser segment is the union of 2^(B - bits) index
// segments, searched in global memory.
int join_bits(const sd_ctx* c, const sd_index* idx, uint64_t nk) {
  if (c->join_elems == 1) return idx->bits;  // the index's own segments
  const uint64_t per =
      c->join_elems ? (uint64_t)c->join_elems : std::max<uint64_t>(64, (uint64_t)std::cbrt((double)nk));
  int b = 4;
  while (b < 24 && (nk >> (b + 1)) >= per) ++b;
  return std::min(b, idx->bits);
}

// One tile of queries: returns pool blocks (i = tile-local query id, j = ref
// id, d) sorted by (i, j) and their count.
TileOut query_tile(Call& cl, const sd_index* idx, const DevSeqs& q, int k, const WeightedSpec* w) {
  sd_ctx* c = cl.c;
  hipStream_t s = cl.s;
  TileOut out;
  if (q.n == 0) return out;
  if (idx->learned) return learned_tile(cl, idx, q, k, w);
  if (q.n >= (1ull << idx->idbits)) throw Error{SD_E_TOO_MANY, "query tile exceeds the index id width"};
  const Packed p = pack_and_count(cl, q, k, true);
  out.nkeys = p.nkeys;
  const uint32_t nk = (uint32_t)p.nkeys;
  cl.tm.mark("q_pack_scan", (double)q.n * 56, 2);

  // query elements, grouped by the top hash bits of the join segments
  const int bits = join_bits(c, idx, nk);
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
  const uint32_t spt = vargen_seqs_per_tile(q.n, nk);
  uint32_t* tcounts = nullptr;
  if (!digits.empty()) {
    tcounts = cl.sc.get<uint32_t>(((q.n + spt - 1) / spt) * 256);
  }
  launch_vargen_hash(p.seq, p.voff, q.n, k, true, e1, idx->idbits, digits.empty() ? 0 : 1, shifts,
                     masks, hist, tcounts, spt, s);
  std::vector<const uint32_t*> hists;
  for (size_t x = 0; x < digits.size(); ++x) hists.push_back(hist + 256 * x);
  // the first pass from the generator's counts, the later ones counted over
  // fixed tiles
  const CountedFirst first{tcounts, (q.n + spt - 1) / spt, p.voff, spt, q.n};
  bool flip = false;
  if (!digits.empty()) {
    flip = radix_sort(cl, e1, nullptr, nullptr, e2, nullptr, nullptr, 1, false, nk,
                      std::vector<Digit>(digits.begin(), digits.begin() + 1),
                      std::vector<const uint32_t*>(hists.begin(), hists.begin() + 1), &first);
    if (digits.size() > 1) {
      const bool f2 = counted_sort(cl, flip ? e2 : e1, flip ? e1 : e2, nk,
                                   std::vector<Digit>(digits.begin() + 1, digits.end()));
      if (f2) flip = !flip;
    }
  }
  const uint64_t* Eq = flip ? e2 : e1;
  const uint32_t nseg = 1u << bits;
  uint32_t* qs = cl.sc.get<uint32_t>(nseg);
  uint32_t* qe = cl.sc.get<uint32_t>(nseg);
  launch_seg_bounds(Eq, nk, 64u - (uint32_t)bits, qs, qe, s);
  // the index's segments at the same bits (its own directory, or coarser
  // bounds found in its sorted array)
  const uint32_t* rs = idx->seg_start;
  const uint32_t* re = idx->seg_end;
  if (bits < idx->bits) {
    uint32_t* crs = cl.sc.get<uint32_t>(nseg);
    uint32_t* cre = cl.sc.get<uint32_t>(nseg);
    launch_seg_bounds(idx->E, idx->n_keys, 64u - (uint32_t)bits, crs, cre, s);
    rs = crs;
    re = cre;
  }
  cl.tm.mark("q_vargen_passes", (double)nk * (8 + 16 * digits.size()),
             (bits < idx->bits ? 3 : 2) + (int)digits.size());

  // join against the index
  Cands cj = sharded_output(
      cl, nk / 4, "join",
      [&](const ShardArgs& out) {
        launch_join_seg(idx->E, rs, re, Eq, qs, qe, nseg, idx->idbits, JOIN_LDS_MIN_Q, out, s);
      },
      [&](uint64_t n) { return (double)nk * 8 + (double)n * 8; });
  cl.sc.blocks.push_back(cj.p);
  uint64_t* cand = cj.p;
  const uint64_t nc = cj.n;
  out.ncand = nc;
  TileOut v = verify_candidates(cl, p.seq, p.planes, q.n, idx->ref_seq, idx->n_ref, cand, nc, k, w);
  v.nkeys = out.nkeys;
  v.ncand = nc;
  return v;
}

}  // namespace

TileOut query_tile_eager(Call& cl, const sd_index* idx, const DevSeqs& q, int k) {
  return query_tile(cl, idx, q, k, nullptr);
}

namespace {

void check_index(const sd_ctx* c, const sd_index* idx, int k) {
  if (!idx) throw Error{SD_E_INVAL, "null index"};
  if (idx->device != c->device) throw Error{SD_E_INVAL, "index lives on another device"};
  if (k < 0 || k > idx->k) throw Error{SD_E_INVAL, "k must lie in [0, the index's k]"};
}

}  // namespace

// Sort (q, r) candidate pairs over the digits that can differ, then verify
// (or rescore) and compact them in order.
TileOut verify_candidates(Call& cl, const u128* qseq, const u128* qplanes, uint64_t nq,
                          const u128* rseq, uint64_t nr,
                          uint64_t* cand, uint64_t nc, int k, const WeightedSpec* w) {
  sd_ctx* c = cl.c;
  hipStream_t s = cl.s;
  TileOut out;
  if (nc >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "more than 2^32 - 2 candidate pairs"};

  // unweighted: buckets by the top bits of q, each sorted and verified in LDS
  const int rbits = bits_for(nr ? nr - 1 : 0), qbits = bits_for(nq ? nq - 1 : 0);
  const BucketPlan bp = w ? BucketPlan() : bucket_plan(c, nc, qbits, rbits);
  if (bp.bits >= 0) {
    c->stats.n_pair_buckets += bp.nb;
    uint64_t* cand2 = cl.sc.get<uint64_t>(nc);
    out.i = dalloc_t<uint32_t>(c, nc);
    out.j = dalloc_t<uint32_t>(c, nc);
    out.d = dalloc_t<uint8_t>(c, nc);
    bool over = false;
    try {
      out.n = bucket_sort_verify(cl, bp, cand, nc, cand2, nq, nr,
                                 c->metric == SD_METRIC_HAMMING ? qseq : qplanes, rseq, k, 0,
                                 out.i, out.j, out.d, &over, "q_pair_sort", "q_verify");
    } catch (...) {
      dfree(c, out.i);
      dfree(c, out.j);
      dfree(c, out.d);
      throw;
    }
    if (!over) return out;
    dfree(c, out.i);
    dfree(c, out.j);
    dfree(c, out.d);
    out = TileOut();
    c->stats.n_pair_fallbacks += 1;
    cand = cand2;  // every candidate, bucketed (the first array was overwritten)
  }

  // sort (q, r) pairs over the digits that can differ
  const uint64_t* sorted = cand;
  if (nc > 1) {
    uint64_t* cand2 = cl.sc.get<uint64_t>(nc);
    std::vector<Digit> pd;
    const int rb = bits_for(nr ? nr - 1 : 0), qb = bits_for(nq ? nq - 1 : 0);
    for (int x = 0; x < (rb + 7) / 8; ++x) pd.push_back(Digit{0, 8 * x, 255u});
    for (int x = 0; x < (qb + 7) / 8; ++x) pd.push_back(Digit{0, 32 + 8 * x, 255u});
    bool pf;
    if (pair_sort_counted(c, nc)) {
      // large: counted passes over fixed tiles
      pf = counted_sort(cl, cand, cand2, (uint32_t)nc, pd);
    } else {
      // small: one histogram, then onesweep passes (fewer launches)
      uint32_t* phist = cl.sc.get<uint32_t>(8 * 256);
      launch_fill_u32(phist, 0, 8 * 256, s);
      launch_radix_hist(cand, nullptr, 1, nc, phist, s);
      std::vector<const uint32_t*> ph;
      for (const Digit& d : pd) ph.push_back(phist + (d.shift / 8) * 256);
      pf = radix_sort(cl, cand, nullptr, nullptr, cand2, nullptr, nullptr, 1, false, (uint32_t)nc,
                      pd, ph);
    }
    sorted = pf ? cand2 : cand;
  }
  cl.tm.mark("q_pair_sort", (double)nc * 16, 1);

  // verify (or rescore) and compact
  out.i = dalloc_t<uint32_t>(c, nc);
  out.j = dalloc_t<uint32_t>(c, nc);
  out.d = dalloc_t<uint8_t>(c, nc);
  try {
    unsigned long long* pcount = reinterpret_cast<unsigned long long*>(cl.counters + CNT_PAIRS);
    launch_fill_u64(reinterpret_cast<uint64_t*>(pcount), 0, 1, s);
    if (nc) {
      if (w) {
        const uint64_t tiles = (nc + weighted_tile() - 1) / weighted_tile();
        const uint32_t epoch = next_epoch(c, tiles, s);
        launch_verify_weighted(sorted, nc, qseq, rseq, k, w->subst, w->indel,
                               w->max_score, out.i, out.j, out.d, c->status, cl.tile_counter(),
                               epoch, pcount, cl.lb_err(), s);
      } else {
        const uint64_t tiles = (nc + compact_tile() - 1) / compact_tile();
        const uint32_t epoch = next_epoch(c, tiles, s);
        launch_verify_compact(sorted, nc, nq, nr, c->metric == SD_METRIC_HAMMING ? qseq : qplanes, rseq, k,
                              c->metric, 0, out.i, out.j, out.d, c->status,
                              cl.tile_counter(), epoch, pcount, cl.lb_err(), s);
      }
    }
    const uint32_t* h = static_cast<const uint32_t*>(readback(c, cl.counters + CNT_PAIRS, 12, s));
    uint64_t cnt;
    std::memcpy(&cnt, h, 8);
    if (h[2] & SD_ERRBIT_LOOKBACK) throw Error{SD_E_HIP, "internal error: a look-back wait timed out"};
    if (h[2] & SD_ERRBIT_PLACEMENT) throw Error{SD_E_HIP, "internal error: a counted pass misplaced"};
    if (h[2] & SD_ERRBIT_INDEX) throw Error{SD_E_HIP, "internal error: a candidate id out of range"};
    out.n = nc ? cnt : 0;
    cl.tm.mark("q_verify", (double)nc * 49, 1);
  } catch (...) {
    dfree(c, out.i);
    dfree(c, out.j);
    dfree(c, out.d);
    throw;
  }
  return out;
}

void index_free(sd_index* idx) {
  if (!idx) return;
  (void)hipSetDevice(idx->device);
  for (void* p : {(void*)idx->ref_seq, (void*)idx->E, (void*)idx->seg_start, (void*)idx->seg_end,
                  (void*)idx->keys, (void*)idx->kid, (void*)idx->params, idx->coord, idx->leaves})
    index_release(idx, p);
  delete idx;
}

sd_index* index_build(sd_ctx* c, const sd_seqs* ref, int k, hipStream_t s) {
  check_seqs(ref);
  if (k < 0 || k > 3) throw Error{SD_E_INVAL, "k must be 0, 1, 2 or 3"};
  sd_index* idx = new sd_index();
  idx->device = c->device;
  idx->k = k;
  idx->n_ref = (uint64_t)ref->n;
  idx->idbits = ref->n <= (1ll << 24) ? 24u : 32u;
  try {
    Scratch sc(c);
    StageTimer tm(c, s);
    Call cl{c, s, sc, tm, fresh_counters(c, CNT_TOTAL, s)};
    const DevSeqs in = stage_seqs(c, sc, ref, s);
    idx->ref_seq = static_cast<u128*>(index_alloc(c, idx, std::max<uint64_t>(in.n, 1) * 16));
    uint64_t nk = 0;
    const uint64_t* E = nullptr;
    if (in.n) {
      const Packed p = pack_and_count(cl, in, k, true);
      hip_check(hipMemcpyAsync(idx->ref_seq, p.seq, in.n * 16, hipMemcpyDeviceToDevice, s), "copy");
      nk = p.nkeys;
      uint64_t* e1 = sc.get<uint64_t>(nk);
      uint64_t* e2 = sc.get<uint64_t>(nk);
      uint32_t* unused = sc.get<uint32_t>(3 * 256);
      const uint32_t z[3] = {0, 0, 0};
      launch_vargen_hash(p.seq, p.voff, in.n, k, true, e1, idx->idbits, 0, z, z, unused, nullptr,
                         VG_MAX_SEQS_PER_BLOCK, s);
      uint32_t* hist = sc.get<uint32_t>(8 * 256);
      launch_fill_u32(hist, 0, 8 * 256, s);
      launch_radix_hist(e1, nullptr, 1, nk, hist, s);
      const std::vector<Digit> digits = top_digits((int)idx->idbits);
      std::vector<const uint32_t*> hists;
      for (const Digit& d : digits) hists.push_back(hist + (d.shift / 8) * 256);
      const bool flip = radix_sort(cl, e1, nullptr, nullptr, e2, nullptr, nullptr, 1, false,
                                   (uint32_t)nk, digits, hists);
      uint64_t* sorted = flip ? e2 : e1;
      uint64_t* uniq = flip ? e1 : e2;
      unsigned long long* ucount = reinterpret_cast<unsigned long long*>(cl.counters + CNT_CAND);
      const uint64_t tiles = (nk + unique_tile() - 1) / unique_tile();
      const uint32_t epoch = next_epoch(c, tiles, s);
      launch_unique_compact(sorted, nk, uniq, c->status, cl.tile_counter(), epoch, ucount,
                            cl.lb_err(), s);
      nk = *static_cast<const uint64_t*>(readback(c, ucount, 8, s));
      check_lookback(cl);
      E = uniq;
    }
    idx->n_keys = nk;
    idx->bits = index_bits(nk);
    const uint32_t nseg = 1u << idx->bits;
    idx->E = static_cast<uint64_t*>(index_alloc(c, idx, std::max<uint64_t>(nk, 1) * 8));
    idx->seg_start = static_cast<uint32_t*>(index_alloc(c, idx, (size_t)nseg * 4));
    idx->seg_end = static_cast<uint32_t*>(index_alloc(c, idx, (size_t)nseg * 4));
    if (nk)
      hip_check(hipMemcpyAsync(idx->E, E, nk * 8, hipMemcpyDeviceToDevice, s), "copy index");
    launch_seg_bounds(idx->E, nk, 64u - (uint32_t)idx->bits, idx->seg_start, idx->seg_end, s);
    hip_check(hipStreamSynchronize(s), "synchronise");
    idx->bytes = idx->n_ref * 16 + nk * 8 + (uint64_t)nseg * 8;
  } catch (...) {
    index_free(idx);
    throw;
  }
  return idx;
}

// Queries of one or more sets. Sets are packed into tiles of at most
// tile_seqs sequences (a set is never split); each tile runs the query
// pipeline and its sorted result is cut into per-set slices.
void query_sets(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k,
                const WeightedSpec* w, sd_pairs* outs, hipStream_t s) {
  check_index(c, idx, k);
  if (nsets < 0 || (nsets > 0 && (!sets || !outs))) throw Error{SD_E_INVAL, "bad set arrays"};
  for (int x = 0; x < nsets; ++x) check_seqs(&sets[x]);
  // the captured-graph batch takes unweighted queries on a hashed index
  if (c->batch_graph && !w && !idx->learned && nsets > 0) {
    query_sets_graph(c, idx, nsets, sets, k, outs, s);
    return;
  }
  c->stats = sd_stats{};
  // host-side phases, printed to stderr when SD_DEBUG_BATCH is set
  const bool dbg = std::getenv("SD_DEBUG_BATCH") != nullptr;
  auto t_last = std::chrono::steady_clock::now();
  auto lap = [&](const char* what) {
    if (!dbg) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "batch: %-22s %8.3f ms\n", what,
                 std::chrono::duration<double, std::milli>(now - t_last).count());
    t_last = now;
  };
  const uint64_t id_limit = (1ull << idx->idbits) - 2;
  const uint64_t tile_limit =
      std::min<uint64_t>(id_limit, c->batch_tile_seqs ? (uint64_t)c->batch_tile_seqs : (4ull << 20));
  int first = 0;
  while (first < nsets) {
    // the tile: sets [first, last), whole sets while they fit
    uint64_t tot = 0;
    int last = first;
    while (last < nsets) {
      const sd_seqs& st = sets[last];
      if ((uint64_t)st.n > id_limit) throw Error{SD_E_TOO_MANY, "a query set exceeds the index id width"};
      if (last > first && tot + (uint64_t)st.n > tile_limit) break;
      tot += (uint64_t)st.n;
      ++last;
    }
    Scratch sc(c);
    StageTimer tm(c, s);
    Call cl{c, s, sc, tm, fresh_counters(c, CNT_TOTAL, s)};
    // concatenate the tile's sets into one device CSR
    DevSeqs q{nullptr, nullptr, tot};
    std::vector<uint32_t> base(last - first + 1, 0);
    {
      uint64_t qpos = 0;
      for (int x = first; x < last; ++x) {
        base[x - first] = (uint32_t)qpos;
        qpos += (uint64_t)sets[x].n;
      }
      base[last - first] = (uint32_t)qpos;
    }
    if (last - first == 1 && sets[first].on_device) {
      q = DevSeqs{sets[first].codes, sets[first].offsets, (uint64_t)sets[first].n};
    } else {
      // the sets' offsets on the host (device sets read into pinned memory
      // with one wait), checked and rebased on host threads into pinned
      // memory, one copy of the tile's offsets; codes one copy per device
      // set and one per run of host sets (through pinned memory)
      size_t dev_words = 0;
      std::vector<SetSpan> spans;
      for (int x = first; x < last; ++x)
        if (sets[x].n) {
          if (sets[x].on_device) dev_words += (size_t)sets[x].n + 1;
          spans.push_back(SetSpan{x, 0, sets[x].n});
        }
      const uint64_t pin_bytes = host_code_bytes(sets, spans);
      int64_t* area = stage_area(c, (dev_words + tot + 1) * 8 + pin_bytes);
      const std::vector<const int64_t*> so = set_offsets(sets, first, last, area, s);
      check_spans(so, spans, false, nullptr, nullptr);
      int64_t* hoffs = area + dev_words;
      const int64_t codes_tot = rebase_spans(so, spans, hoffs);
      uint8_t* codes = sc.get<uint8_t>((uint64_t)codes_tot + 1);
      int64_t* offs = sc.get<int64_t>(tot + 1);
      stage_codes(sets, so, spans, hoffs, codes, reinterpret_cast<uint8_t*>(hoffs + tot + 1), s);
      hip_check(hipMemcpyAsync(offs, hoffs, (tot + 1) * 8, hipMemcpyHostToDevice, s),
                "copy offsets");
      stage_done(c, s);
      q = DevSeqs{codes, offs, tot};
    }
    lap("tile inputs");
    TileOut r = query_tile(cl, idx, q, k, w);
    lap("tile pipeline");
    c->stats.n_seqs += (int64_t)tot;
    c->stats.n_keys += (int64_t)r.nkeys;
    c->stats.n_cand_raw += (int64_t)r.ncand;
    c->stats.n_pairs += (int64_t)r.n;
    const int ns = last - first;
    if (ns == 1) {
      finish_output(c, r.i, r.j, r.d, r.n, &outs[first], s);
    } else {
      // per-set slices of the (q, r)-sorted tile result
      uint32_t* dbase = sc.get<uint32_t>(ns + 1);
      uint64_t* bounds = sc.get<uint64_t>(ns + 1);
      hip_check(hipMemcpyAsync(dbase, base.data(), (ns + 1) * 4, hipMemcpyHostToDevice, s), "copy");
      launch_set_ranges(r.i, r.n, dbase, (uint32_t)(ns + 1), bounds, s);
      std::vector<uint64_t> hb(ns + 1);
      hip_check(hipMemcpyAsync(hb.data(), bounds, (ns + 1) * 8, hipMemcpyDeviceToHost, s), "bounds");
      hip_check(hipStreamSynchronize(s), "synchronise");
      bool host_out = true;
      for (int x = first; x < last; ++x) host_out = host_out && !outs[x].on_device;
      try {
        if (host_out) {
          // host results: the tile's result comes over once and is cut on the
          // host (ids made set-local on the way)
          std::vector<HostSlice> sl;
          for (int x = 0; x < ns; ++x) {
            host_result(c, hb[x + 1] - hb[x], &outs[first + x]);
            sl.push_back(HostSlice{first + x, hb[x], hb[x + 1] - hb[x], 0, -(int64_t)base[x]});
          }
          fill_host_slices(c, r.i, r.j, r.d, r.n, sl, outs, s);
        }
        for (int x = 0; x < ns && !host_out; ++x) {
          const uint64_t lo = hb[x], n = hb[x + 1] - hb[x];
          uint32_t* oi = dalloc_t<uint32_t>(c, n);
          uint32_t* oj = dalloc_t<uint32_t>(c, n);
          uint8_t* od = dalloc_t<uint8_t>(c, n);
          launch_slice_rebase(r.i, r.j, r.d, lo, n, -(int64_t)base[x], oi, oj, od, s);
          finish_output(c, oi, oj, od, n, &outs[first + x], s);
        }
      } catch (...) {
        dfree(c, r.i);
        dfree(c, r.j);
        dfree(c, r.d);
        throw;
      }
      hip_check(hipStreamSynchronize(s), "synchronise");
      dfree(c, r.i);
      dfree(c, r.j);
      dfree(c, r.d);
    }
    tm.finish();
    lap("tile results");
    first = last;
  }
}

void query_weighted(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets,
                    const uint8_t* subst, int indel, int max_score, sd_pairs* outs,
                    hipStream_t s) {
  if (!subst) throw Error{SD_E_INVAL, "null substitution table"};
  if (indel < 0 || indel > 255 || max_score < 0) throw Error{SD_E_INVAL, "bad costs"};
  Scratch sc(c);
  uint8_t* dsub = sc.get<uint8_t>(400);
  hip_check(hipMemcpyAsync(dsub, subst, 400, hipMemcpyHostToDevice, s), "copy costs");
  const WeightedSpec w{dsub, (uint32_t)indel, (uint32_t)max_score};
  query_sets(c, idx, nsets, sets, idx ? idx->k : 0, &w, outs, s);
}

}  // namespace sd
