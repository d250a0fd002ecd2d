// Batched query search as one captured HIP graph: many query sets against
// one device-resident reference index (the database lookup of the paper's
// Section IV, run for a whole batch of repertoires at once).
//
// The batch is cut into tiles of at most T sequences; a set larger than T is
// split into consecutive chunks, so a tile is a list of (set, first sequence,
// count) pieces. Everything whose size the host can know is sized before
// the capture from the sequence lengths alone:
//   * the query variants are generated with multiplicity (all V(L, k)
//     deletion sets; a repeated variant only repeats a candidate, which the
//     pair sort drops), so each tile's variant count is exact on the host;
//   * the candidate array of a tile has a fixed capacity (from the
//     candidates per variant seen last time on the context), filled with
//     ~0 before the join's output is gathered into it, so the pair sort and
//     the verification run over the whole capacity (~0 sorts last and the
//     verification skips it) and need no count from the device.
// No host read of a device size happens inside the capture. After the graph
// has run, one read-back per tile gives its pair count, the join's output
// size and the per-piece result bounds; a tile whose candidates overflowed
// its capacity is run again eagerly (query_tile), and the capacity hint
// grows. The instantiated graph and its buffers are kept by the context and
// replayed for the next batch of the same shape (same tiles, same variant
// counts): only the input copies run before the replay.
//
// Look-back kernels of the graph use a status area and tile counters of the
// plan's own, cleared by fill kernels inside the graph at the start of every
// tile (no memset nodes), with fixed epochs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "sd_host.h"

namespace sd {

namespace {
// Host-side phases of a batch, printed to stderr when SD_DEBUG_BATCH is set.
struct PhaseClock {
  bool on = std::getenv("SD_DEBUG_BATCH") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void lap(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "graph batch: %-22s %8.3f ms\n", what,
                 std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};
}  // namespace

namespace {

constexpr uint32_t kJoinLdsMinQ = 8;  // as the eager join: smaller query segments search global memory
constexpr uint32_t kEpochScan = 1, kEpochVerify = 2, kEpochBucketScan = 3, kEpochBucketCounts = 4;
constexpr double kMinCandRatio = 1.0 / 1024;  // candidates per variant the capacity assumes at least

struct Piece {
  int set;          // index of the query set
  int64_t first;    // first sequence of the set in this piece
  int64_t count;    // sequences
};

struct TileBufs {
  std::vector<Piece> pieces;
  uint64_t n = 0, ncodes = 0, nk = 0, cap = 0;
  uint8_t* codes = nullptr;       // the tile's concatenated CSR
  int64_t* offs = nullptr;
  uint32_t* counters = nullptr;   // CNT_TOTAL u32: validation, tile counters, pair count
  unsigned long long* ctr = nullptr;  // join shard counters (OUT_SHARDS + 1)
  uint64_t* off = nullptr;            // join shard offsets (OUT_SHARDS + 1)
  uint32_t* pbase = nullptr;      // tile-local first id of every piece, and the tile size
  uint64_t* bounds = nullptr;     // result position of every piece start, and of the end
  uint32_t* oi = nullptr;         // verified (tile-local q, r, d), capacity cap
  uint32_t* oj = nullptr;
  uint8_t* od = nullptr;
};

}  // namespace

// A captured batch: its shape, the graph and every buffer the graph uses.
struct GraphPlan {
  std::string key;
  sd_ctx* c = nullptr;
  std::vector<void*> blocks;  // pool blocks held by the plan
  std::vector<TileBufs> tiles;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  uint64_t over_cap = 0;  // the join's spill capacity
  uint64_t* status = nullptr;
  uint64_t status_words = 0;
  template <typename T>
  T* get(uint64_t count) {
    T* p = dalloc_t<T>(c, count);
    blocks.push_back(p);
    return p;
  }
  ~GraphPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : blocks) dfree(c, p);
  }
};

void graph_plans_release(sd_ctx* c) {
  (void)hipDeviceSynchronize();
  c->graph_plans.clear();
}

namespace {

uint64_t variants_of_length(int64_t L, int k) {
  uint64_t v = 1;
  for (int m = 1; m <= k && m <= L; ++m) {
    uint64_t c = 1;
    for (int t = 0; t < m; ++t) c = c * (uint64_t)(L - t) / (uint64_t)(t + 1);
    v += c;
  }
  return v;
}

// Enqueue one tile's pipeline on stream s (capturing). Shared work buffers
// are sized for the largest tile.
struct Shared {
  u128* seq;
  u128* planes;
  uint32_t* vcnt;
  uint64_t* voff;
  uint64_t* e1;
  uint64_t* e2;
  uint32_t* tcounts;
  uint32_t* local;
  uint32_t* bsum;
  uint32_t* qs;
  uint32_t* qe;
  uint64_t* shard_base;
  uint64_t shard_region;
  uint64_t* shard_over;
  uint64_t shard_over_cap;
  uint64_t* cand;
  uint64_t* cand2;
  uint32_t* pcounts;
  uint32_t* plocal;
  uint32_t* pbsum;
  uint32_t* bcnt;  // bucketed pair sort: count table and its scan,
  uint64_t* boff;
  uint32_t* bcount;  // bucket pair counts and their scan
  uint64_t* bpos;
  uint64_t* packed;  // every bucket's kept pairs
};

// The pair sort of a tile: bucketed (as the eager path) over the whole
// candidate capacity, whose unused ~0 slots fall in no bucket.
BucketPlan tile_bucket_plan(const sd_ctx* c, const sd_index* idx, const TileBufs& t) {
  return bucket_plan(c, t.cap, bits_for(t.n ? t.n - 1 : 0), bits_for(idx->n_ref ? idx->n_ref - 1 : 0));
}

void enqueue_tile(const sd_ctx* c, const sd_index* idx, int k, GraphPlan& plan, TileBufs& t,
                  const Shared& w, hipStream_t s) {
  uint32_t* ctrs = t.counters;
  uint32_t* err = ctrs + CNT_LBERR;
  int slot = CNT_TILE0;
  launch_fill_u32(ctrs, 0, CNT_TOTAL, s);
  launch_fill_u64(plan.status, 0, plan.status_words, s);
  // pack (all V(L, k) deletion sets) and the variant offsets
  launch_pack(t.codes, t.offs, t.n, k, false, w.seq, w.planes, w.vcnt, ctrs + CNT_ERR, s);
  launch_scan_excl(w.vcnt, w.voff, t.n, plan.status, ctrs + slot++, kEpochScan, err, s);
  // query elements, the first pass's digits counted per fixed tile
  const int bits = idx->bits;
  const std::vector<Digit> digits = bits ? top_digits(64 - bits) : std::vector<Digit>();
  const uint32_t nk = (uint32_t)t.nk;
  const uint32_t spt = vargen_seqs_per_tile(t.n, t.nk);
  const uint64_t ftiles = fixed_tiles(nk);
  uint32_t shifts[3] = {0, 0, 0}, masks[3] = {0, 0, 0};
  for (size_t x = 0; x < digits.size() && x < 3; ++x) {
    shifts[x] = (uint32_t)digits[x].shift;
    masks[x] = digits[x].mask;
  }
  if (!digits.empty()) launch_fill_u32(w.tcounts, 0, ftiles * 256, s);
  launch_vargen_hash(w.seq, w.voff, t.n, k, false, w.e1, idx->idbits, digits.empty() ? 0 : 1,
                     shifts, masks, nullptr, digits.empty() ? nullptr : w.tcounts, spt, s,
                     fixed_tile_elems());
  bool flip = false;
  for (size_t x = 0; x < digits.size(); ++x) {
    const uint64_t* in = flip ? w.e2 : w.e1;
    uint64_t* out = flip ? w.e1 : w.e2;
    if (x > 0) launch_tile_counts(in, nk, digits[x].shift, digits[x].mask, w.tcounts, s);
    launch_counted_scan(w.tcounts, ftiles, 1, w.local, w.bsum, s);
    launch_counted_scatter(in, out, nk, digits[x].shift, digits[x].mask, ftiles, w.local, w.bsum,
                           nullptr, 0, 0, err, s);
    flip = !flip;
  }
  const uint64_t* Eq = flip ? w.e2 : w.e1;
  const uint32_t nseg = 1u << bits;
  launch_seg_bounds(Eq, nk, 64u - (uint32_t)bits, w.qs, w.qe, s);
  // join into the shards, then gather into the fixed-capacity candidate
  // array (unused slots keep ~0)
  launch_fill_u64(reinterpret_cast<uint64_t*>(t.ctr), 0, out_shards() + 1, s);
  const ShardArgs sa{w.shard_base, w.shard_region, w.shard_over, w.shard_over_cap, t.ctr};
  launch_join_seg(idx->E, idx->seg_start, idx->seg_end, Eq, w.qs, w.qe, nseg, idx->idbits,
                  kJoinLdsMinQ, sa, s);
  launch_fill_u64(w.cand, ~0ull, t.cap, s);
  launch_gather_shards(w.shard_base, w.shard_region, w.shard_over, w.shard_over_cap, t.ctr, t.off,
                       w.cand, s, t.cap);
  unsigned long long* pcount = reinterpret_cast<unsigned long long*>(ctrs + CNT_PAIRS);
  const BucketPlan bp = tile_bucket_plan(c, idx, t);
  if (bp.bits >= 0) {
    // sort and verify per bucket in LDS; a bucket over LDS size flags the
    // tile (SD_ERRBIT_BUCKET), which then runs again eagerly
    const BucketBufs b{w.bcnt,      w.boff,      w.packed,         w.bcount,
                       w.bpos,      plan.status, ctrs + slot,      kEpochBucketScan,
                       ctrs + slot + 1, kEpochBucketCounts, err};
    slot += 2;
    bucket_enqueue(bp, b, w.cand, t.cap, w.cand2, t.n, idx->n_ref,
                   c->metric == SD_METRIC_HAMMING ? w.seq : w.planes, idx->ref_seq, k, c->metric,
                   0, t.oi, t.oj, t.od, pcount, s);
    launch_set_ranges(t.oi, t.cap, t.pbase, (uint32_t)t.pieces.size() + 1, t.bounds, s, pcount);
    return;
  }
  // pair sort over the whole capacity (counted passes)
  std::vector<Digit> pd;
  const int rb = bits_for(idx->n_ref ? idx->n_ref - 1 : 0), qb = bits_for(t.n ? t.n - 1 : 0);
  for (int x = 0; x < (rb + 7) / 8; ++x) pd.push_back(Digit{0, 8 * x, 255u});
  for (int x = 0; x < (qb + 7) / 8; ++x) pd.push_back(Digit{0, 32 + 8 * x, 255u});
  const uint64_t ptiles = fixed_tiles(t.cap);
  bool pf = false;
  for (const Digit& d : pd) {
    const uint64_t* in = pf ? w.cand2 : w.cand;
    uint64_t* out = pf ? w.cand : w.cand2;
    launch_tile_counts(in, (uint32_t)t.cap, d.shift, d.mask, w.pcounts, s);
    launch_counted_scan(w.pcounts, ptiles, 1, w.plocal, w.pbsum, s);
    launch_counted_scatter(in, out, (uint32_t)t.cap, d.shift, d.mask, ptiles, w.plocal, w.pbsum,
                           nullptr, 0, 0, err, s);
    pf = !pf;
  }
  const uint64_t* sorted = pf ? w.cand2 : w.cand;
  // verification and ordered compaction, then the piece bounds
  launch_verify_compact(sorted, t.cap, t.n, idx->n_ref, c->metric == SD_METRIC_HAMMING ? w.seq : w.planes,
                        idx->ref_seq, k, c->metric, 0, t.oi, t.oj, t.od, plan.status, ctrs + slot++,
                        kEpochVerify, pcount, err, s);
  launch_set_ranges(t.oi, t.cap, t.pbase, (uint32_t)t.pieces.size() + 1, t.bounds, s, pcount);
}

// The shape a cached plan serves: the index's arrays and sizes (the graph
// holds their addresses), k, the metric and every tile's pieces and sizes.
std::string plan_key(const sd_ctx* c, const sd_index* idx, int k, uint64_t T,
                     const std::vector<TileBufs>& tiles) {
  std::string key = std::to_string((uintptr_t)idx->E) + "," +
                    std::to_string((uintptr_t)idx->seg_start) + "," +
                    std::to_string((uintptr_t)idx->seg_end) + "," +
                    std::to_string((uintptr_t)idx->ref_seq) + "," + std::to_string(idx->n_keys) +
                    "," + std::to_string(idx->n_ref) + "," + std::to_string(idx->bits) + "," +
                    std::to_string(idx->idbits) + "/" + std::to_string(k) + "/" +
                    std::to_string(T) + "/" + std::to_string(c->metric) + "/" +
                    std::to_string(c->pair_sort);
  for (const TileBufs& t : tiles) {
    key += "|" + std::to_string(t.n) + "," + std::to_string(t.ncodes) + "," + std::to_string(t.nk) +
           "," + std::to_string(t.cap);
    for (const Piece& p : t.pieces)
      key += ":" + std::to_string(p.set) + "," + std::to_string(p.first) + "," +
             std::to_string(p.count);
  }
  return key;
}

}  // namespace

void query_sets_graph(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k,
                      sd_pairs* outs, hipStream_t s) {
  PhaseClock clk;
  const uint64_t id_limit = (1ull << idx->idbits) - 2;
  const uint64_t T = std::min<uint64_t>(
      id_limit, c->batch_tile_seqs ? (uint64_t)c->batch_tile_seqs : (4ull << 20));
  // tiles of at most T sequences from the set sizes alone; a set larger than
  // the room left is split
  std::vector<TileBufs> tiles(1);
  for (int x = 0; x < nsets; ++x) {
    int64_t done = 0;
    while (done < sets[x].n) {
      if (tiles.back().n >= T) tiles.emplace_back();
      TileBufs& t = tiles.back();
      const int64_t take = std::min<int64_t>(sets[x].n - done, (int64_t)(T - t.n));
      t.pieces.push_back(Piece{x, done, take});
      t.n += (uint64_t)take;
      done += take;
    }
  }
  // the variant counts and code sizes need every length: every set's offsets
  // on the host (device sets read into pinned memory with one wait), checked
  // and summed on host threads
  size_t dev_words = 0, tile_words = 0;
  for (int x = 0; x < nsets; ++x)
    if (sets[x].n && sets[x].on_device) dev_words += (size_t)sets[x].n + 1;
  for (const TileBufs& t : tiles) tile_words += t.n + 1;
  std::vector<SetSpan> spans;
  for (const TileBufs& t : tiles)
    for (const Piece& pc : t.pieces) spans.push_back(SetSpan{pc.set, pc.first, pc.count});
  const uint64_t pin_bytes = host_code_bytes(sets, spans);
  int64_t* area = stage_area(c, (dev_words + tile_words) * 8 + pin_bytes);
  const std::vector<const int64_t*> so = set_offsets(sets, 0, nsets, area, s);
  {
    uint64_t vlen[KEY_MAX_LEN_HOST + 1];  // V(L, k) by length
    for (int L = 0; L <= KEY_MAX_LEN_HOST; ++L) vlen[L] = variants_of_length(L, k);
    std::vector<uint64_t> sums(spans.size());
    check_spans(so, spans, true, vlen, sums.data());
    size_t at = 0;
    for (TileBufs& t : tiles)
      for (const Piece& pc : t.pieces) {
        t.nk += sums[at++];
        t.ncodes += (uint64_t)(so[pc.set][pc.first + pc.count] - so[pc.set][pc.first]);
      }
  }
  if (tiles.back().pieces.empty()) tiles.pop_back();
  clk.lap("lengths and sizes");
  c->stats = sd_stats{};
  for (int x = 0; x < nsets; ++x) {
    outs[x].n = 0;
    outs[x].i = outs[x].j = nullptr;
    outs[x].d = nullptr;
    c->stats.n_seqs += sets[x].n;
  }
  if (tiles.empty()) {  // only empty sets
    for (int x = 0; x < nsets; ++x)
      finish_output(c, dalloc_t<uint32_t>(c, 0), dalloc_t<uint32_t>(c, 0), dalloc_t<uint8_t>(c, 0),
                    0, &outs[x], s);
    return;
  }
  for (const TileBufs& t : tiles)
    if (t.nk >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "more than 2^32 - 2 deletion variants in a tile"};
  // candidate capacity from the candidates per variant seen before
  const double ratio = std::max(c->graph_cand_ratio, kMinCandRatio);
  for (TileBufs& t : tiles)
    t.cap = std::min<uint64_t>(0xFFFFFFF0ull, (uint64_t)((double)t.nk * ratio * 1.1) + 65536);
  const std::string key = plan_key(c, idx, k, T, tiles);
  clk.lap("plan key");

  GraphPlan* plan = nullptr;
  for (auto& p : c->graph_plans)
    if (p->key == key) plan = p.get();
  if (!plan) {
    graph_plans_release(c);  // one cached shape per context
    auto up = std::make_shared<GraphPlan>();
    up->c = c;
    up->key = key;
    GraphPlan& P = *up;
    uint64_t max_n = 1, max_nk = 1, max_cap = 1, max_counts = 1, max_nb = 1, max_bwords = 1;
    for (const TileBufs& t : tiles) {
      max_n = std::max(max_n, t.n);
      max_nk = std::max(max_nk, t.nk);
      max_cap = std::max(max_cap, t.cap);
      const BucketPlan bp = tile_bucket_plan(c, idx, t);
      if (bp.bits >= 0) {
        max_counts = std::max(max_counts, bp.counts);
        max_nb = std::max<uint64_t>(max_nb, bp.nb);
        max_bwords = std::max(max_bwords, bucket_status_words(bp));
      }
    }
    const uint32_t NS = out_shards();
    Shared w{};
    w.seq = P.get<u128>(max_n);
    w.planes = P.get<u128>(max_n);
    w.vcnt = P.get<uint32_t>(max_n);
    w.voff = P.get<uint64_t>(max_n + 1);
    w.e1 = P.get<uint64_t>(max_nk);
    w.e2 = P.get<uint64_t>(max_nk);
    const uint64_t ft = fixed_tiles(max_nk);
    w.tcounts = P.get<uint32_t>(ft * 256);
    w.local = P.get<uint32_t>(ft * 256);
    // (scan rows are not monotone in the tile count: room for any tile's)
    w.bsum = P.get<uint32_t>(((uint64_t)counted_scan_rows(ft) + 512) * 256);
    w.qs = P.get<uint32_t>(1ull << idx->bits);
    w.qe = P.get<uint32_t>(1ull << idx->bits);
    w.shard_region = max_cap / NS + max_cap / (2 * NS) + 16;
    w.shard_base = P.get<uint64_t>(w.shard_region * NS);
    w.shard_over_cap = max_cap / 4 + 4096;
    P.over_cap = w.shard_over_cap;
    w.shard_over = P.get<uint64_t>(w.shard_over_cap);
    w.cand = P.get<uint64_t>(max_cap);
    w.cand2 = P.get<uint64_t>(max_cap);
    const uint64_t pt = fixed_tiles(max_cap);
    w.pcounts = P.get<uint32_t>(pt * 256);
    w.plocal = P.get<uint32_t>(pt * 256);
    w.pbsum = P.get<uint32_t>(((uint64_t)counted_scan_rows(pt) + 512) * 256);
    w.bcnt = P.get<uint32_t>(max_counts);
    w.boff = P.get<uint64_t>(max_counts + 1);
    w.bcount = P.get<uint32_t>(max_nb);
    w.packed = P.get<uint64_t>(max_cap);
    w.bpos = P.get<uint64_t>(max_nb + 1);
    P.status_words = std::max<uint64_t>(
                         std::max<uint64_t>(max_n / scan_tile() + 2, max_cap / compact_tile() + 2),
                         std::max<uint64_t>(max_bwords, max_nb + 2)) +
                     64;
    P.status = P.get<uint64_t>(P.status_words);
    for (TileBufs& t : tiles) {
      t.codes = P.get<uint8_t>(t.ncodes + 1);
      t.offs = P.get<int64_t>(t.n + 1);
      t.counters = P.get<uint32_t>(CNT_TOTAL);
      t.ctr = P.get<unsigned long long>(NS + 1);
      t.off = P.get<uint64_t>(NS + 1);
      t.pbase = P.get<uint32_t>(t.pieces.size() + 1);
      t.bounds = P.get<uint64_t>(t.pieces.size() + 1);
      t.oi = P.get<uint32_t>(t.cap);
      t.oj = P.get<uint32_t>(t.cap);
      t.od = P.get<uint8_t>(t.cap);
      // tile-local first id of every piece, and the tile size
      std::vector<uint32_t> pb(t.pieces.size() + 1);
      uint64_t q = 0;
      for (size_t x = 0; x < t.pieces.size(); ++x) {
        pb[x] = (uint32_t)q;
        q += (uint64_t)t.pieces[x].count;
      }
      pb[t.pieces.size()] = (uint32_t)q;
      hip_check(hipMemcpyAsync(t.pbase, pb.data(), pb.size() * 4, hipMemcpyHostToDevice, s),
                "piece bases");
      hip_check(hipStreamSynchronize(s), "synchronise");
    }
    P.tiles = std::move(tiles);
    // capture on a stream of the plan's own (the caller's may be the legacy
    // stream, which cannot capture)
    hip_check(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking), "capture stream");
    hip_check(hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      for (TileBufs& t : P.tiles) enqueue_tile(c, idx, k, P, t, w, P.cap_stream);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(P.cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      throw;
    }
    hip_check(hipStreamEndCapture(P.cap_stream, &P.graph), "end capture");
    hip_check(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0), "instantiate graph");
    c->graph_plans.push_back(std::move(up));
    plan = c->graph_plans.back().get();
    c->stats.n_graph_captures += 1;
  }
  clk.lap("plan");

  // inputs of this batch into the plan's tile buffers (offsets rebased into
  // pinned memory, one copy per tile; codes one copy per device piece and
  // one per run of host pieces), then the replay
  {
    int64_t* dst = area + dev_words;
    uint8_t* pin = reinterpret_cast<uint8_t*>(area + dev_words + tile_words);
    size_t at = 0;
    for (TileBufs& t : plan->tiles) {
      const std::vector<SetSpan> ts(spans.begin() + at, spans.begin() + at + t.pieces.size());
      at += t.pieces.size();
      rebase_spans(so, ts, dst);
      stage_codes(sets, so, ts, dst, t.codes, pin, s);
      pin += host_code_bytes(sets, ts);
      hip_check(hipMemcpyAsync(t.offs, dst, (t.n + 1) * 8, hipMemcpyHostToDevice, s),
                "copy offsets");
      dst += t.n + 1;
    }
    stage_done(c, s);
  }
  hipEvent_t ready = nullptr, done = nullptr;
  clk.lap("inputs");
  hip_check(hipEventCreateWithFlags(&ready, hipEventDisableTiming), "event");
  hip_check(hipEventCreateWithFlags(&done, hipEventDisableTiming), "event");
  hip_check(hipEventRecord(ready, s), "record");
  hip_check(hipStreamWaitEvent(plan->cap_stream, ready, 0), "wait");
  hip_check(hipGraphLaunch(plan->exec, plan->cap_stream), "launch graph");
  hip_check(hipEventRecord(done, plan->cap_stream), "record");
  hip_check(hipStreamWaitEvent(s, done, 0), "wait");
  hip_check(hipStreamSynchronize(s), "synchronise");
  (void)hipEventDestroy(ready);
  (void)hipEventDestroy(done);
  c->stats.n_graph_launches += 1;
  clk.lap("replay");

  // results: per tile its counters, join size and piece bounds; a tile that
  // overflowed its candidate capacity runs again eagerly
  const uint32_t NS = out_shards();
  struct TileResult {
    uint32_t* i;
    uint32_t* j;
    uint8_t* d;
    std::vector<uint64_t> bounds;
    bool own = false;  // pool blocks of an eager rerun, freed below
  };
  std::vector<TileResult> res(plan->tiles.size());
  double cand_per_key = 0.0;
  Scratch sc(c);
  StageTimer tm(c, s);
  try {
    for (size_t x = 0; x < plan->tiles.size(); ++x) {
      TileBufs& t = plan->tiles[x];
      std::vector<uint32_t> h(CNT_TOTAL);
      uint64_t tail[2];
      hip_check(hipMemcpyAsync(h.data(), t.counters, CNT_TOTAL * 4, hipMemcpyDeviceToHost, s), "rb");
      hip_check(hipMemcpyAsync(&tail[0], t.off + NS, 8, hipMemcpyDeviceToHost, s), "rb");
      hip_check(hipMemcpyAsync(&tail[1], t.ctr + NS, 8, hipMemcpyDeviceToHost, s), "rb");
      res[x].bounds.assign(t.pieces.size() + 1, 0);
      hip_check(hipMemcpyAsync(res[x].bounds.data(), t.bounds, res[x].bounds.size() * 8,
                               hipMemcpyDeviceToHost, s), "rb");
      hip_check(hipStreamSynchronize(s), "synchronise");
      raise_validation(h[CNT_ERR]);
      if (h[CNT_LBERR] & SD_ERRBIT_LOOKBACK)
        throw Error{SD_E_HIP, "internal error: a look-back wait timed out"};
      if (h[CNT_LBERR] & SD_ERRBIT_PLACEMENT)
        throw Error{SD_E_HIP, "internal error: a counted pass misplaced"};
      if (h[CNT_LBERR] & SD_ERRBIT_INDEX)
        throw Error{SD_E_HIP, "internal error: a candidate id out of range"};
      const uint64_t joined = tail[0] + tail[1];  // regions (clamped) plus the spill
      const bool spilled = tail[1] > plan->over_cap;
      cand_per_key = std::max(cand_per_key, (double)joined / (double)std::max<uint64_t>(t.nk, 1));
      // a bucket too large for LDS also runs the tile again eagerly (where
      // the global passes take over)
      const bool bucket_over = (h[CNT_LBERR] & SD_ERRBIT_BUCKET) != 0;
      if (joined <= t.cap && !spilled && !bucket_over) {
        res[x].i = t.oi;
        res[x].j = t.oj;
        res[x].d = t.od;
        continue;
      }
      // overflow: this tile again, eagerly, with room sized from the count
      c->stats.n_graph_retries += 1;
      if (std::getenv("SD_DEBUG_BATCH"))
        std::fprintf(stderr,
                     "graph batch: tile %zu runs again (candidates %llu, capacity %llu, spill %llu "
                     "of %llu, bucket over %d)\n",
                     x, (unsigned long long)joined, (unsigned long long)t.cap,
                     (unsigned long long)tail[1], (unsigned long long)plan->over_cap,
                     (int)bucket_over);
      Call cl{c, s, sc, tm, fresh_counters(c, CNT_TOTAL, s)};
      const TileOut r = query_tile_eager(cl, idx, DevSeqs{t.codes, t.offs, t.n}, k);
      res[x].i = r.i;
      res[x].j = r.j;
      res[x].d = r.d;
      res[x].own = true;
      std::vector<uint32_t> pb(t.pieces.size() + 1);
      hip_check(hipMemcpy(pb.data(), t.pbase, pb.size() * 4, hipMemcpyDeviceToHost), "rb");
      uint64_t* db = sc.get<uint64_t>(pb.size());
      launch_set_ranges(r.i, r.n, t.pbase, (uint32_t)pb.size(), db, s);
      hip_check(hipMemcpyAsync(res[x].bounds.data(), db, pb.size() * 8, hipMemcpyDeviceToHost, s),
                "rb");
      hip_check(hipStreamSynchronize(s), "synchronise");
    }
    // the capacity follows the candidates per variant: up at once after an
    // overflow, down (to 1.2 times what was seen) once it is twice too
    // large, so that a steady workload keeps its captured graph
    if (cand_per_key > c->graph_cand_ratio)
      c->graph_cand_ratio = cand_per_key;
    else if (2.0 * cand_per_key < c->graph_cand_ratio)
      c->graph_cand_ratio = std::max(1.2 * cand_per_key, kMinCandRatio);
    clk.lap("read-backs");
    // per set: its pieces' slices in order, query ids made set-local
    std::vector<uint64_t> total(nsets, 0);
    for (size_t x = 0; x < plan->tiles.size(); ++x)
      for (size_t p = 0; p < plan->tiles[x].pieces.size(); ++p)
        total[plan->tiles[x].pieces[p].set] += res[x].bounds[p + 1] - res[x].bounds[p];
    std::vector<uint64_t> at(nsets, 0);
    bool host_out = true;
    for (int x = 0; x < nsets; ++x) host_out = host_out && !outs[x].on_device;
    uint64_t npairs = 0;
    if (host_out) {
      // host results: each tile's result comes over once and is cut on the
      // host into the sets' pinned blocks
      for (int x = 0; x < nsets; ++x) host_result(c, total[x], &outs[x]);
      for (size_t x = 0; x < plan->tiles.size(); ++x) {
        const TileBufs& t = plan->tiles[x];
        std::vector<HostSlice> sl;
        uint32_t q = 0;
        for (size_t p = 0; p < t.pieces.size(); ++p) {
          const Piece& pc = t.pieces[p];
          const uint64_t lo = res[x].bounds[p], n = res[x].bounds[p + 1] - lo;
          // tile-local id q + y is set-local id pc.first + y
          sl.push_back(HostSlice{pc.set, lo, n, at[pc.set], pc.first - (int64_t)q});
          at[pc.set] += n;
          npairs += n;
          q += (uint32_t)pc.count;
        }
        fill_host_slices(c, res[x].i, res[x].j, res[x].d, res[x].bounds.back(), sl, outs, s);
      }
    } else {
      std::vector<uint32_t*> si(nsets), sj(nsets);
      std::vector<uint8_t*> sd(nsets);
      for (int x = 0; x < nsets; ++x) {
        si[x] = dalloc_t<uint32_t>(c, total[x]);
        sj[x] = dalloc_t<uint32_t>(c, total[x]);
        sd[x] = dalloc_t<uint8_t>(c, total[x]);
      }
      for (size_t x = 0; x < plan->tiles.size(); ++x) {
        const TileBufs& t = plan->tiles[x];
        uint32_t q = 0;
        for (size_t p = 0; p < t.pieces.size(); ++p) {
          const Piece& pc = t.pieces[p];
          const uint64_t lo = res[x].bounds[p], n = res[x].bounds[p + 1] - lo;
          launch_slice_rebase(res[x].i, res[x].j, res[x].d, lo, n, pc.first - (int64_t)q,
                              si[pc.set] + at[pc.set], sj[pc.set] + at[pc.set],
                              sd[pc.set] + at[pc.set], s);
          at[pc.set] += n;
          npairs += n;
          q += (uint32_t)pc.count;
        }
      }
      for (int x = 0; x < nsets; ++x) finish_output(c, si[x], sj[x], sd[x], total[x], &outs[x], s);
      hip_check(hipStreamSynchronize(s), "synchronise");
    }
    clk.lap("per-set results");
    c->stats.n_pairs = (int64_t)npairs;
  } catch (...) {
    for (auto& r : res)
      if (r.own) {
        dfree(c, r.i);
        dfree(c, r.j);
        dfree(c, r.d);
      }
    throw;
  }
  for (auto& r : res)
    if (r.own) {
      dfree(c, r.i);
      dfree(c, r.j);
      dfree(c, r.d);
    }
}

}  // namespace sd
