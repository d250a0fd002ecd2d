// Host-side helpers shared by the search pipelines (self search and
// query-versus-reference): staging of sequence sets, the per-call counter
// area, and the LSD radix-sort driver over the onesweep kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "sd_internal.h"

namespace sd {

struct DevSeqs {
  const uint8_t* codes;
  const int64_t* offs;
  uint64_t n;
};

inline void check_seqs(const sd_seqs* s) {
  if (!s) throw Error{SD_E_INVAL, "null sequence set"};
  if (s->n < 0) throw Error{SD_E_INVAL, "negative sequence count"};
  if (s->n > 0 && (!s->codes || !s->offsets)) throw Error{SD_E_INVAL, "null codes or offsets"};
  if ((uint64_t)s->n >= 0xFFFFFFFFull) throw Error{SD_E_TOO_MANY, "at most 2^32 - 2 sequences"};
}

DevSeqs stage_seqs(sd_ctx* c, Scratch& sc, const sd_seqs* s, hipStream_t st);

inline void raise_validation(uint32_t err) {
  if (err & SD_ERRBIT_LENGTH) throw Error{SD_E_LENGTH, "a sequence length is outside [1, 24]"};
  if (err & SD_ERRBIT_ALPHABET) throw Error{SD_E_ALPHABET, "a residue code is >= 20"};
  if (err & SD_ERRBIT_INDEX) throw Error{SD_E_INVAL, "an index is out of range"};
  if (err & SD_ERRBIT_OFFSETS)
    throw Error{SD_E_INVAL, "offsets must start at 0 and must not decrease"};
}

inline int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b)) ++b;
  return b;
}

// one LSD digit: word, shift inside the word, mask
struct Digit {
  int word, shift;
  uint32_t mask;
};

// Counter slots of the per-call counter area (zeroed at the start of a call).
enum : int {
  CNT_ERR = 0,        // validation flags
  CNT_TILE0 = 1,      // first of the per-launch tile counters
  CNT_TILE_END = 60,
  CNT_NKEYS = 64,     // u64 copy of the key total
  CNT_CAND = 96,      // u64 candidate counter
  CNT_PAIRS = 98,     // u64 result counter
  CNT_LBERR = 100,    // look-back bound hits
  CNT_NBIG = 102,     // u64 count of ranges the grouping kernel lists
  CNT_NBIG2 = 104,    // u64 count of ranges the second grouping pass lists
  CNT_CAND2 = 106,    // u64 candidate counter of the full-key emission
  CNT_STEPS = 108,    // u64 search comparisons of learned-index lookups
  CNT_TOTAL = 128
};

// The state of one library call on one stream. Several Call objects of one
// call (a streamed search's column groups) share the counter area, so the
// cursor over its tile-counter slots lives in the context: a slot handed out
// once is never handed out again until the whole block of slots is zeroed.
struct Call {
  sd_ctx* c;
  hipStream_t s;
  Scratch& sc;
  StageTimer& tm;
  uint32_t* counters;
  // a zeroed tile counter (the dynamic tile ids of one look-back kernel)
  uint32_t* tile_counter() {
    if (c->tile_slot < CNT_TILE0) c->tile_slot = CNT_TILE0;  // fresh counter area
    if (c->tile_slot >= CNT_TILE_END) {  // recycle: zero a fresh block of slots
      launch_fill_u32(counters + CNT_TILE0, 0, CNT_TILE_END - CNT_TILE0, s);
      c->tile_slot = CNT_TILE0;
    }
    return counters + c->tile_slot++;
  }
  uint32_t* lb_err() { return counters + CNT_LBERR; }
};

// Sort records by the given digits in LSD order; returns true if the result
// sits in the second buffer set.
// A first pass whose digits the input's producer counted per tile (see
// launch_counted_pass).
struct CountedFirst {
  const uint32_t* counts;
  uint64_t tiles;
  const uint64_t* voff;
  uint32_t seqs_per_tile;
  uint64_t nseq;
};

inline bool radix_sort(Call& cl, uint64_t* a0, uint64_t* a1, uint32_t* av, uint64_t* b0, uint64_t* b1,
                uint32_t* bv, int nwords, bool has_val, uint32_t n, const std::vector<Digit>& digits,
                const std::vector<const uint32_t*>& hists,
                const CountedFirst* first = nullptr) {
  bool flip = false;
  const uint64_t tile = onesweep_tile(nwords, has_val, cl.c->sort_items);
  const uint64_t tiles = (n + tile - 1) / tile;
  for (size_t x = 0; x < digits.size(); ++x) {
    const uint64_t* i0 = flip ? b0 : a0;
    const uint64_t* i1 = flip ? b1 : a1;
    const uint32_t* iv = flip ? bv : av;
    uint64_t* o0 = flip ? a0 : b0;
    uint64_t* o1 = flip ? a1 : b1;
    uint32_t* ov = flip ? av : bv;
    if (x == 0 && first && nwords == 1 && !has_val && digits[0].word == 0) {
      // the producer counted this pass's digits per tile: no look-back
      uint32_t* local = cl.sc.get<uint32_t>(first->tiles * 256);
      uint32_t* bsum = cl.sc.get<uint32_t>((uint64_t)counted_scan_rows(first->tiles) * 256);
      launch_counted_pass(i0, o0, n, digits[0].shift, digits[0].mask, first->counts, first->tiles,
                          first->voff, first->seqs_per_tile, first->nseq, local, bsum, cl.lb_err(),
                          cl.s);
      flip = !flip;
      continue;
    }
    const uint32_t epoch = next_epoch(cl.c, tiles * 256, cl.s);
    launch_onesweep(i0, i1, iv, o0, o1, ov, nwords, has_val, n, digits[x].word, digits[x].shift,
                    digits[x].mask, hists[x], cl.c->status, cl.tile_counter(), epoch, cl.lb_err(),
                    cl.c->sort_items, cl.s);
    flip = !flip;
  }
  return flip;
}

// Stable LSD sort of 64-bit keys by `digits` (word 0), every pass counted
// over fixed tiles: a count kernel, the two count scans and the XCD-contiguous
// scatter; no global histogram and no look-back. Returns whether the result
// is in b.
inline bool counted_sort(Call& cl, uint64_t* a, uint64_t* b, uint32_t n,
                         const std::vector<Digit>& digits) {
  bool flip = false;
  const uint64_t tiles = fixed_tiles(n);
  uint32_t* counts = cl.sc.get<uint32_t>(tiles * 256);
  uint32_t* local = cl.sc.get<uint32_t>(tiles * 256);
  uint32_t* bsum = cl.sc.get<uint32_t>((uint64_t)counted_scan_rows(tiles) * 256);
  for (const Digit& d : digits) {
    const uint64_t* in = flip ? b : a;
    uint64_t* out = flip ? a : b;
    launch_tile_counts(in, n, d.shift, d.mask, counts, cl.s);
    launch_counted_scan(counts, tiles, 1, local, bsum, cl.s);
    launch_counted_scatter(in, out, n, d.shift, d.mask, tiles, local, bsum, nullptr, 0, 0,
                           cl.lb_err(), cl.s);
    flip = !flip;
  }
  return flip;
}

// The candidate pair sort takes counted passes from 2^21 candidates up (or
// as SD_OPT_PAIR_SORT forces), one-sweep passes below.
inline bool pair_sort_counted(const sd_ctx* c, uint64_t nc) {
  if (c->pair_sort) return c->pair_sort == 2;
  return nc >= (1u << 21);
}

// Bucketed pair sort (steps 6-7): candidates (i << 32 | j) go to buckets by
// the top `bits` bits of i, and each bucket is sorted, deduplicated and
// verified in one workgroup's LDS. About 2048 candidates per bucket (a
// quarter of what LDS holds), at most bucket_max() buckets, and enough
// bucket bits that i's remaining bits and j fit a 32-bit key.
struct BucketPlan {
  int bits = -1;  // -1: the bucketed sort does not apply
  uint32_t nb = 0, low = 0, jb = 0, shift = 0;
  uint64_t ntiles = 0;  // counting tiles
  uint64_t counts = 0;  // entries of the count table (and of its scan, plus one)
};

// Switched off: the bucketed sort made the GPU take a memory fault on its
// first small self search (one bucket of 31 candidates), a cause not yet
// found, so every pair sort takes the global passes until it is. Kept for
// that work; nothing reaches it while kBucketedPairSort is false.
constexpr bool kBucketedPairSort = false;

// For nc candidates whose first ids have ib bits and second ids jb bits.
// SD_OPT_PAIR_SORT 1 and 2 choose the global passes instead.
inline BucketPlan bucket_plan(const sd_ctx* c, uint64_t nc, int ib, int jb) {
  BucketPlan p;
  if (!kBucketedPairSort) return p;
  if (c->pair_sort == 1 || c->pair_sort == 2 || nc == 0) return p;
  ib = std::max(ib, 1);
  jb = std::max(jb, 1);
  int b = 0;
  while (b < 12 && (nc >> b) > 2048) ++b;
  b = std::min(std::max(b, ib + jb - 32), ib);
  if (b > bits_for(bucket_max() - 1) || ib - b + jb > 32) return p;
  p.bits = b;
  p.nb = 1u << b;
  p.low = (uint32_t)(ib - b);
  p.jb = (uint32_t)jb;
  p.shift = 32 + p.low;
  p.ntiles = (nc + bucket_chunk() - 1) / bucket_chunk();
  p.counts = p.ntiles * p.nb;
  return p;
}

// The buffers and look-back state of one bucketed sort: the count table and
// its scan (p.counts and p.counts + 1 entries), the packed pairs (nc), the
// bucket pair counts and
// their scan (p.nb and p.nb + 1), a status array of at least the scan tiles
// of p.counts words, two zeroed tile counters and the two scans' epochs.
struct BucketBufs {
  uint32_t* cnt;
  uint64_t* off;
  uint64_t* packed;  // nc entries: every bucket's kept pairs
  uint32_t* bcount;
  uint64_t* bpos;
  uint64_t* status;
  uint32_t* scan_ctr;
  uint32_t scan_epoch;
  uint32_t* scan2_ctr;
  uint32_t scan2_epoch;
  uint32_t* err;
};

// Status words the two scans of a bucketed sort need.
inline uint64_t bucket_status_words(const BucketPlan& p) {
  return (std::max<uint64_t>(p.counts, p.nb) + scan_tile() - 1) / scan_tile() + 1;
}

// Count, scan and scatter into cand2 (nc entries), then sort and verify
// every bucket and place its pairs; the pair count goes to *pcount. No host
// synchronisation (a capture can hold it). First ids are below na, second
// ids below nbseq. cand is overwritten (large buckets are sorted through
// it); cand2 keeps every candidate. A bucket too large to sort this way
// sets SD_ERRBIT_BUCKET.
inline void bucket_enqueue(const BucketPlan& p, const BucketBufs& b, uint64_t* cand,
                           uint64_t nc, uint64_t* cand2, uint64_t na, uint64_t nbseq,
                           const u128* a, const u128* sb, int k,
                           int metric, int self_pairs, uint32_t* oi, uint32_t* oj, uint8_t* od,
                           unsigned long long* pcount, hipStream_t s, const u128* a2 = nullptr,
                           const u128* sb2 = nullptr) {
  launch_bucket_count(cand, nc, p.shift, p.nb, b.cnt, s);
  launch_scan_excl(b.cnt, b.off, p.counts, b.status, b.scan_ctr, b.scan_epoch, b.err, s);
  launch_bucket_scatter(cand, nc, p.shift, p.nb, b.off, cand2, s);
  launch_bucket_verify(cand2, cand, b.packed, b.off, nc, p.nb, p.jb, p.low, na, nbseq, a, sb, k,
                       metric, self_pairs, b.bcount, b.err, s, a2, sb2);
  launch_scan_excl(b.bcount, b.bpos, p.nb, b.status, b.scan2_ctr, b.scan2_epoch, b.err, s);
  launch_bucket_place(b.packed, b.off, nc, p.nb, p.jb, p.low, b.bcount, b.bpos, oi, oj, od,
                      pcount, s);
}

// The eager form on a call's scratch and status array: returns the pair
// count, or sets *over when a bucket was too large (the output is then
// incomplete, and the caller sorts cand2, which holds every candidate, the
// other way; cand is overwritten).
uint64_t bucket_sort_verify(Call& cl, const BucketPlan& p, uint64_t* cand, uint64_t nc,
                            uint64_t* cand2, uint64_t na, uint64_t nbseq, const u128* a,
                            const u128* sb, int k, int self_pairs,
                            uint32_t* oi, uint32_t* oj, uint8_t* od, bool* over,
                            const char* sort_stage, const char* verify_stage,
                            const u128* a2 = nullptr, const u128* sb2 = nullptr);

constexpr int KEY_MAX_LEN_HOST = 24;  // the longest sequence a key holds

// Host staging of batched query sets (stage.cpp). A span is a run of
// consecutive sequences of one set.
struct SetSpan {
  int set = 0;
  int64_t first = 0, count = 0;  // the set's sequences [first, first + count)
};
// Pinned host memory of the context for staging, at least `bytes` bytes,
// kept until sd_destroy. Waits first for the copies the last stage_done()
// recorded, so the area is free to overwrite.
int64_t* stage_area(sd_ctx* c, size_t bytes);
// Marks the end of the copies enqueued on s from the staging area.
void stage_done(sd_ctx* c, hipStream_t s);
// Host views of the offsets of the sets [first, last) (entries below first
// are null): device sets are read into `area` (n + 1 words for each
// non-empty device set, in set order) with one synchronisation of s, host
// sets are used where they are. Raises SD_E_INVAL unless every non-empty
// set's offsets start at 0.
std::vector<const int64_t*> set_offsets(const sd_seqs* sets, int first, int last, int64_t* area,
                                        hipStream_t s);
// Checks every sequence of the spans on host threads: offsets must not
// decrease (SD_E_INVAL) and, with check_len, lengths lie in [1, 24]
// (SD_E_LENGTH); the first failing sequence in span order decides. With
// vlen (indexed by length; lengths are then checked too), sums[x] = the sum
// of vlen over span x.
void check_spans(const std::vector<const int64_t*>& offs, const std::vector<SetSpan>& spans,
                 bool check_len, const uint64_t* vlen, uint64_t* sums);
// The spans' offsets laid end to end and rebased to their concatenated
// codes, on host threads: dst[q + y] = (codes of the spans before) +
// offs[first + y] - offs[first] for each span of q sequences before it, and
// dst[total] = the codes of all spans, which is returned.
int64_t rebase_spans(const std::vector<const int64_t*>& offs, const std::vector<SetSpan>& spans,
                     int64_t* dst);

// Bytes of codes of the host spans (the pinned room stage_codes needs).
uint64_t host_code_bytes(const sd_seqs* sets, const std::vector<SetSpan>& spans);
// The spans' codes into the tile's device codes, laid out as the rebased
// offsets `dst` say (span x starts at dst[q] for the q sequences of the
// spans before it): host spans are copied by host threads into `pin` (room
// for host_code_bytes) and go over with one copy per run of consecutive host
// spans; device spans are copied device to device, one copy each.
void stage_codes(const sd_seqs* sets, const std::vector<const int64_t*>& offs,
                 const std::vector<SetSpan>& spans, const int64_t* dst, uint8_t* codes,
                 uint8_t* pin, hipStream_t s);

// Host results of batched sets cut from device results (stage.cpp): a
// slice moves entries [lo, lo + n) of a (q, r)-sorted device result to
// position `at` of the host result of set `set`, with q + shift as its id.
struct HostSlice {
  int set = 0;
  uint64_t lo = 0, n = 0, at = 0;
  int64_t shift = 0;
};
// A pinned host result of n pairs for out (one block: i, j, then d).
void host_result(sd_ctx* c, uint64_t n, sd_pairs* out);
// One copy of a device result of n pairs (di, dj, dd) into the pinned
// staging area, then every slice into its set's host result on host threads.
void fill_host_slices(sd_ctx* c, const uint32_t* di, const uint32_t* dj, const uint8_t* dd,
                      uint64_t n, const std::vector<HostSlice>& slices, sd_pairs* outs,
                      hipStream_t s);

struct Cands {
  uint64_t* p = nullptr;  // pool block owned by the caller
  uint64_t n = 0;
};

// Host side of a sharded output (sd_device.h): `launch(args)` runs the
// producing kernel against zeroed counters; reservations past a shard's
// region spill into the overflow region, and only if that overflows too does
// the kernel run again with more room. The stage is timed as `stage` with
// bytes(total) algorithmic bytes; the regions are then gathered (stage
// "gather_out") into one dense pool block owned by the caller. `guess` is the
// expected total.
template <class Launch, class Bytes>
Cands sharded_output(Call& cl, uint64_t guess, const char* stage, Launch&& launch, Bytes&& bytes,
                     bool exact_guess = false) {
  const uint32_t NS = out_shards();
  sd_ctx* c = cl.c;
  // the size the same stage produced last time on this context, if larger
  auto hint = c->out_hint.find(stage);
  if (!exact_guess && hint != c->out_hint.end()) guess = std::max(guess, hint->second);
  // regions at 1.5 times the mean share and a quarter of the guess for
  // overflow; with an exact total spread evenly over the shards (exact_guess),
  // 1.125 times and a sixteenth
  const uint64_t region =
      exact_guess ? guess / NS + guess / (8 * NS) + 64 : guess / NS + guess / (2 * NS) + 16;
  uint64_t over_cap = exact_guess ? guess / 16 + 4096 : guess / 4 + 4096;
  unsigned long long* ctr = cl.sc.get<unsigned long long>(NS + 1);
  std::vector<unsigned long long> h(NS + 1);
  // the second run rewrites the same regions and only needs a larger overflow
  ShardArgs a{cl.sc.get<uint64_t>(region * NS), region, nullptr, over_cap, ctr};
  int runs = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    a.over = cl.sc.get<uint64_t>(over_cap);
    a.over_cap = over_cap;
    launch_fill_u64(reinterpret_cast<uint64_t*>(ctr), 0, NS + 1, cl.s);
    launch(a);
    ++runs;
    std::memcpy(h.data(), readback(c, ctr, (NS + 1) * 8, cl.s), (NS + 1) * 8);
    if (h[NS] <= over_cap) break;
    if (attempt == 1) throw Error{SD_E_HIP, "internal error: output overflow region exceeded twice"};
    over_cap = h[NS] + h[NS] / 8 + 4096;  // the same reservations spill the same amount again
    cl.sc.release(a.over);  // the readback waited for the run: nothing uses it any more
  }
  Cands out;
  for (uint32_t x = 0; x < NS; ++x) out.n += std::min<uint64_t>(h[x], region);
  out.n += h[NS];
  c->out_hint[stage] = out.n;
  cl.tm.mark(stage, bytes(out.n), runs);
  out.p = dalloc_t<uint64_t>(c, out.n);
  if (out.n)
    launch_gather_shards(a.base, a.region, a.over, a.over_cap, ctr, cl.sc.get<uint64_t>(NS + 1),
                         out.p, cl.s);
  cl.tm.mark("gather_out", (double)out.n * 16, out.n ? 2 : 0);
  return out;
}

// Sorting digits over bits [lo, 64) of a 64-bit word, least significant first.
inline std::vector<Digit> top_digits(int lo) {
  std::vector<Digit> d;
  for (int b = lo; b < 64; b += 8) {
    const int w = std::min(8, 64 - b);
    d.push_back(Digit{0, b, (1u << w) - 1u});
  }
  return d;
}

// Device cost table and threshold of the weighted rescoring.
struct WeightedSpec {
  const uint8_t* subst;  // device, 400 bytes
  uint32_t indel, max_score;
};

// A query result in pool blocks: (i = query id, j = reference id, d), sorted
// by (i, j), with the key and candidate counts that produced it.
struct TileOut {
  uint32_t* i = nullptr;
  uint32_t* j = nullptr;
  uint8_t* d = nullptr;
  uint64_t n = 0;
  uint64_t nkeys = 0, ncand = 0;
};

// Sort (q, r) candidates, verify (weighted when w) and compact in order.
TileOut verify_candidates(Call& cl, const u128* qseq, const u128* qplanes, uint64_t nq, const u128* rseq, uint64_t nr,
                          uint64_t* cand, uint64_t nc, int k, const WeightedSpec* w);

// A packed sequence set: 128-bit keys, exclusive variant offsets (n + 1)
// and the variant total, in pool blocks of the call.
struct Packed {
  u128* seq = nullptr;
  u128* planes = nullptr;  // bit-plane form of each sequence (launch_pack)
  uint64_t* voff = nullptr;
  uint64_t nkeys = 0;
};
// pack and validate a device CSR set, scan its variant counts (one read-back)
// distinct: count (and later generate) each distinct variant string of a
// sequence once instead of all V(L, k) deletion sets
Packed pack_and_count(Call& cl, const DevSeqs& in, int k, bool distinct);
// raise if a look-back wait of the call hit its bound
void check_lookback(Call& cl);

// exact keys (lo and hi words) with their ids, sorted by key (pointers into
// the caller's buffers or the call's scratch)
struct SortedKeys {
  const uint64_t* lo;
  const uint64_t* hi;
  const uint32_t* id;
  int passes;
};
SortedKeys full_key_sort(Call& cl, uint64_t* klo, uint64_t* khi, uint32_t* kid, uint32_t nk);

// one query tile against a learned index (probe lookups, then verification)
TileOut learned_tile(Call& cl, const sd_index* idx, const DevSeqs& q, int k, const WeightedSpec* w);
// one tile of queries through the eager pipeline (host synchronisations
// included): (tile-local q, r, d) sorted by (q, r)
TileOut query_tile_eager(Call& cl, const sd_index* idx, const DevSeqs& q, int k);
// sd_query_batch as one captured graph (graphbatch.cpp)
void query_sets_graph(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k,
                      sd_pairs* outs, hipStream_t s);
// release the context's captured batch plans (waits for the device)
void graph_plans_release(sd_ctx* c);

// Hand a finished result (pool blocks oi/oj/od holding n triplets) to the
// caller: device arrays as they are, or pinned host copies.
void finish_output(sd_ctx* c, uint32_t* oi, uint32_t* oj, uint8_t* od, uint64_t n, sd_pairs* out,
                   hipStream_t s);

}  // namespace sd
