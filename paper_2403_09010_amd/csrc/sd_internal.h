// Host-side internals of the symdel library: the context, its device memory
// pool and the kernel launchers each translation unit provides.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/symdel.h"

typedef unsigned __int128 u128;

// device-side validation flags
#define SD_ERRBIT_LENGTH 1u
#define SD_ERRBIT_ALPHABET 2u
#define SD_ERRBIT_INDEX 4u
#define SD_ERRBIT_LOOKBACK 8u  // a look-back wait hit its bound (internal error)
#define SD_ERRBIT_PLACEMENT 16u  // a counted pass computed a position past the end (internal error)
#define SD_ERRBIT_BUCKET 32u  // a pair bucket exceeded what one workgroup sorts (the host takes another path)
#define SD_ERRBIT_OFFSETS 64u  // a set's offsets do not start at 0 or decrease

namespace sd {

// ------------------------------------------------------------------ launchers
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s);
uint32_t out_shards();
// (writes stop at cap elements of out; off[] receives the shard offsets and,
// at [OUT_SHARDS], the overflow's offset, so the total is off[OUT_SHARDS] +
// min(counter[OUT_SHARDS], over_cap))
void launch_gather_shards(const uint64_t* base, uint64_t region, const uint64_t* over,
                          uint64_t over_cap, const unsigned long long* counter, uint64_t* off,
                          uint64_t* out, hipStream_t s,
                          uint64_t cap = ~0ull);
// a sharded output as passed to the producing kernels (sd_device.h ShardOut)
struct ShardArgs {
  uint64_t* base;
  uint64_t region;
  uint64_t* over;
  uint64_t over_cap;
  unsigned long long* counter;
};
void launch_radix_hist(const uint64_t* w0, const uint64_t* w1, int nwords, uint64_t n,
                       uint32_t* hist, hipStream_t s);
uint64_t onesweep_tile(int nwords, bool has_val, int items);
// one stable pass by the digit (word[word] >> shift) & mask, mask <= 255
void launch_onesweep(const uint64_t* in0, const uint64_t* in1, const uint32_t* vin,
                     uint64_t* out0, uint64_t* out1, uint32_t* vout, int nwords, bool has_val,
                     uint32_t n, int word, int shift, uint32_t mask, const uint32_t* hist256,
                     uint64_t* status, uint32_t* tile_counter, uint32_t epoch, uint32_t* err,
                     int items, hipStream_t s);
// A keys-only pass over input that its producer wrote in consecutive ranges
// ("tiles") and counted: tile t holds the elements [voff[t * seqs_per_tile],
// voff[min((t + 1) * seqs_per_tile, nseq)]) and counts[t][d] of them have
// digit d. local needs tiles * 256 and bsum counted_scan_rows(tiles) * 256
// entries of scratch. A position past n (counts that disagree with the
// input) sets SD_ERRBIT_PLACEMENT in *err and is not written.
uint32_t counted_scan_rows(uint64_t tiles);
void launch_counted_pass(const uint64_t* in, uint64_t* out, uint32_t n, int shift, uint32_t mask,
                         const uint32_t* counts, uint64_t tiles, const uint64_t* voff,
                         uint32_t seqs_per_tile, uint64_t nseq, uint32_t* local, uint32_t* bsum,
                         uint32_t* err, hipStream_t s);
// Fixed tiles for a counted pass over data nobody counted: fixed_tiles(n)
// rows of digit counts by launch_tile_counts; the scatter then takes voff =
// nullptr (tile t is elements [t * 4096, t * 4096 + 4096)).
uint64_t fixed_tiles(uint64_t n);
void launch_tile_counts(const uint64_t* in, uint32_t n, int shift, uint32_t mask, uint32_t* counts,
                        hipStream_t s);
// the two halves of launch_counted_pass: the count scans, then the scatter.
// Here a tile's counts may be the sum of rows_per_tile consecutive rows of
// counts (nrows rows); the scatter's tiles are then rows_per_tile times as
// many sequences.
void launch_counted_scan(const uint32_t* counts, uint64_t nrows, uint32_t rows_per_tile,
                         uint32_t* local, uint32_t* bsum, hipStream_t s);
void launch_counted_scatter(const uint64_t* in, uint64_t* out, uint32_t n, int shift, uint32_t mask,
                            uint64_t tiles, const uint32_t* local, const uint32_t* bsum,
                            const uint64_t* voff, uint32_t seqs_per_tile, uint64_t nseq,
                            uint32_t* err, hipStream_t s);
uint64_t scan_tile();
// Bucketed pair sort (steps 6-7): candidates per counting tile, the largest
// bucket sorted in LDS, the most buckets.
uint32_t bucket_chunk();
uint32_t bucket_cap();
uint32_t bucket_max();
// cnt[b * ntiles + t] = candidates of tile t (bucket_chunk() each) whose
// value >> shift is b, for b < nb <= bucket_max().
void launch_bucket_count(const uint64_t* cand, uint64_t nc, uint32_t shift, uint32_t nb,
                         uint32_t* cnt, hipStream_t s);
// Scatter by bucket from the exclusive scan `off` of that table (bucket-major).
void launch_bucket_scatter(const uint64_t* cand, uint64_t nc, uint32_t shift, uint32_t nb,
                           const uint64_t* off, uint64_t* out, hipStream_t s);
// Per bucket (the range off[b * ntiles] .. of cand, which is only read):
// sort, drop repeats (and i >= j if self_pairs), verify as
// launch_verify_compact does, and write the kept pairs in order, packed as
// key << 8 | distance (key = i's `low` bits below the bucket bits above j's
// jb bits, low + jb <= 32), at the start of the bucket's range of packed;
// bcount[b] = their number. A bucket over bucket_cap() candidates is sorted
// through its range of scratch (overwritten). A bucket over 2^18
// candidates, or one that cannot be cut into pieces of bucket_cap(), sets
// SD_ERRBIT_BUCKET in *err and counts 0. Ids at or above na (first) or
// nbseq (second) set SD_ERRBIT_INDEX and are never read. Values >> shift >=
// nb (the ~0 of an unused candidate slot) are in no bucket.
void launch_bucket_verify(const uint64_t* cand, uint64_t* scratch, uint64_t* packed,
                          const uint64_t* off, uint64_t nc, uint32_t nb, uint32_t jb, uint32_t low,
                          uint64_t na, uint64_t nbseq, const u128* a, const u128* seq_b, int k,
                          int metric, int self_pairs, uint32_t* bcount, uint32_t* err,
                          hipStream_t s, const u128* a2 = nullptr, const u128* seq_b2 = nullptr);
// Every bucket's packed pairs to out_*[bpos[b] ..) (bpos = exclusive scan of
// bcount, nb + 1 entries); *out_count = bpos[nb].
void launch_bucket_place(const uint64_t* packed, const uint64_t* off, uint64_t nc, uint32_t nb,
                         uint32_t jb, uint32_t low, const uint32_t* bcount, const uint64_t* bpos,
                         uint32_t* out_i, uint32_t* out_j, uint8_t* out_d,
                         unsigned long long* out_count, hipStream_t s);
void launch_scan_excl(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* status,
                      uint32_t* tile_counter, uint32_t epoch, uint32_t* err, hipStream_t s);

// vcnt[i]: the variants of sequence i, all V(L, k) of them or, with
// distinct, only the distinct strings among them (variant_canonical)
// planes (optional): per sequence its residues' five bit planes (plane b in
// bits [24 b, 24 b + 24)) and its length in bits 127..120, the pattern form
// of the verification's distance
void launch_pack(const uint8_t* codes, const int64_t* offs, uint64_t n, int k, bool distinct,
                 u128* seq, u128* planes, uint32_t* vcnt, uint32_t* err, hipStream_t s);
void launch_vargen(const u128* seq, const uint64_t* voff, uint64_t nseq, int k,
                   uint64_t* key_lo, uint64_t* key_hi, uint32_t* id, hipStream_t s);
void launch_emit_runs(const uint64_t* key_lo, const uint64_t* key_hi, const uint32_t* id,
                      uint64_t n, uint64_t* cand, uint64_t cap,
                      unsigned long long* counter, hipStream_t s);
uint64_t compact_tile();
// out[t] = (uint64_t)i[t] << 32 | j[t]
void launch_join_pairs(const uint32_t* i, const uint32_t* j, uint64_t n, uint64_t* out,
                       hipStream_t s);
// metric SD_METRIC_LEVENSHTEIN: a = bit planes of the first sequences (pack);
// SD_METRIC_HAMMING: a = their packed keys
// self_pairs: drop candidates with i >= j (self search). With a2 and seq_b2
// (paired-chain records: the second chains' planes and keys), the distance
// is the sum over both chains and metric is not used.
// (first ids at or above na, second ids at or above nbseq set
// SD_ERRBIT_INDEX in *err and are never read)
void launch_verify_compact(const uint64_t* cand, uint64_t c, uint64_t na, uint64_t nbseq,
                           const u128* a, const u128* seq_b, int k, int metric, int self_pairs,
                           uint32_t* out_i, uint32_t* out_j, uint8_t* out_d, uint64_t* status,
                           uint32_t* tile_counter, uint32_t epoch, unsigned long long* out_count,
                           uint32_t* err, hipStream_t s, const u128* a2 = nullptr,
                           const u128* seq_b2 = nullptr);
// hashed grouping (element = hash of the key in the top 64 - idbits bits, id below)
// Every variant as [hash | id] in voff order; block b generates sequences
// [b * seqs_per_block, ...) (1 <= seqs_per_block <= VG_MAX_SEQS_PER_BLOCK).
// hist[q * 256 + d] receives the digit counts of pass q, unless tcounts is
// non-null: then tcounts holds npass * G rows of 256 (G = ceil(nseq /
// seqs_per_block) blocks, every entry written), pass q's block counts at rows
// q * G .. q * G + G - 1; the first G rows are the tiles of a counted first
// pass and launch_hist_rows sums the others into hist.
constexpr uint32_t VG_MAX_SEQS_PER_BLOCK = 64;
// Sequences per generator block for a counted first pass: tiles of about
// 3584 elements, which with at most 301 variants per sequence fit the pass's
// 4096-element chunk in one piece.
inline uint32_t vargen_seqs_per_tile(uint64_t nseq, uint64_t nkeys) {
  if (!nseq || !nkeys) return VG_MAX_SEQS_PER_BLOCK;
  const uint64_t per = 3584 * nseq / nkeys;
  return (uint32_t)std::min<uint64_t>(VG_MAX_SEQS_PER_BLOCK, std::max<uint64_t>(1, per));
}
// Generator blocks per counted tile: when a block's sequences yield well
// under 3584 variants (few variants per sequence), several blocks form one
// tile so that the tile still fills most of a chunk.
inline uint32_t vargen_blocks_per_tile(uint64_t nseq, uint64_t nkeys, uint32_t spb) {
  if (!nseq || !nkeys) return 1;
  const double per_block = (double)nkeys / (double)nseq * spb;
  return (uint32_t)std::max(1.0, std::floor(3584.0 / per_block));
}
// distinct: voff counts distinct variants (launch_pack with distinct) and
// only the canonical deletion sets are written
// ftile != 0 (one pass, with tcounts zeroed by the caller): tcounts holds the
// first digit's counts per fixed output tile of ftile elements (the tiles of
// launch_counted_scatter without voff) instead of one row per block.
void launch_vargen_hash(const u128* seq, const uint64_t* voff, uint64_t nseq, int k, bool distinct,
                        uint64_t* elem, uint32_t idbits, int npass, const uint32_t* shifts,
                        const uint32_t* masks, uint32_t* hist, uint32_t* tcounts,
                        uint32_t seqs_per_block, hipStream_t s, uint32_t ftile = 0);
// elements per fixed tile of the counted passes
uint32_t fixed_tile_elems();
// Streamed search (column groups of hash bins): STREAM_BIN_BITS top hash
// bits name a variant's bin. launch_vargen_bins adds every distinct
// variant's bin to hist[1 << STREAM_BIN_BITS] (zeroed by the caller);
// launch_vargen_stream appends the elements of the variants whose bin lies
// in [blo, bhi) to the sharded output, hash rotated left by the bin bits.
constexpr int STREAM_BIN_BITS = 8;
void launch_vargen_bins(const u128* seq, const uint64_t* voff, uint64_t nseq, int k,
                        uint32_t idbits, uint32_t* hist, uint32_t seqs_per_block, hipStream_t s);
void launch_vargen_stream(const u128* seq, const uint64_t* voff, uint64_t nseq, int k,
                          uint32_t idbits, uint32_t blo, uint32_t bhi, const ShardArgs& a,
                          uint32_t seqs_per_block, hipStream_t s);
// Paired-chain records (a_i, b_i): vcnt[i] = deletion sets of up to k of the
// La + Lb residue positions; the generator writes every such variant of the
// joined string a T b as [hash | id] at voff[i] (with multiplicity).
void launch_paired_count(const u128* sa, const u128* sb, uint64_t n, int k, uint32_t* vcnt,
                         hipStream_t s);
void launch_vargen_paired(const u128* sa, const u128* sb, const uint64_t* voff, uint64_t n, int k,
                          uint32_t idbits, uint64_t* elem, hipStream_t s);
// after launch_vargen_hash with tcounts: hist[q * 256 + d] for q >= 1 from the
// stored block rows
void launch_hist_rows(const uint32_t* tcounts, uint64_t nseq, uint32_t seqs_per_block, int npass,
                      uint32_t* hist, hipStream_t s);
bool group_cap_supported(int cap);
void launch_seg_bounds(const uint64_t* E, uint64_t n, uint32_t segshift, uint32_t* seg_start,
                       uint32_t* seg_end, hipStream_t s);
// splitbit: the hash bit below the segment bits (segments of up to 2 cap
// elements are grouped in two halves by it); 64 disables splitting
// shape (capacity 2048 only): 0 = 256 threads at five waves per SIMD, 1 = 256
// threads at four, 2 = 512 threads at four
void launch_group_seg(int cap, int shape, const uint64_t* E, const uint32_t* seg_start,
                      const uint32_t* seg_end, uint32_t nseg, uint32_t spw, uint32_t idbits,
                      uint32_t splitbit, const ShardArgs& out, uint64_t* big,
                      unsigned long long* nbig, hipStream_t s);
// second pass over the *nlisted (device count, at most max_listed) ranges
// launch_group_seg listed in big[], with a table for cap candidates; ranges
// that still do not fit go to big2[]
void launch_group_listed(int cap, const uint64_t* E, const uint64_t* big,
                         const unsigned long long* nlisted, uint64_t max_listed, uint32_t idbits,
                         uint32_t splitbit, const ShardArgs& out, uint64_t* big2,
                         unsigned long long* nbig2, hipStream_t s);
void launch_gather_big(const uint64_t* E, const uint64_t* big, const uint64_t* out_off,
                       uint32_t nseg, uint64_t* out, hipStream_t s);
void launch_emit_hash_runs(const uint64_t* E, uint64_t n, uint32_t idbits, uint64_t* cand,
                           uint64_t cap, unsigned long long* counter, hipStream_t s);
void launch_pair_distance(const u128* seq_a, uint64_t na, const u128* seq_b, uint64_t nb,
                          const uint32_t* ia, const uint32_t* ib, uint64_t n, uint8_t* d,
                          uint32_t* err, hipStream_t s);
// query-versus-reference
uint64_t unique_tile();
void launch_unique_compact(const uint64_t* in, uint64_t n, uint64_t* out, uint64_t* status,
                           uint32_t* tile_counter, uint32_t epoch, unsigned long long* out_count,
                           uint32_t* err, hipStream_t s);
int join_cap();
void launch_join_seg(const uint64_t* Er, const uint32_t* rseg_start, const uint32_t* rseg_end,
                     const uint64_t* Eq, const uint32_t* qseg_start, const uint32_t* qseg_end,
                     uint32_t nseg, uint32_t idbits, uint32_t lds_min_q, const ShardArgs& out,
                     hipStream_t s);
uint64_t weighted_tile();
void launch_verify_weighted(const uint64_t* cand, uint64_t c, const u128* sa, const u128* sb,
                            int k, const uint8_t* subst, uint32_t indel, uint32_t max_score,
                            uint32_t* oi, uint32_t* oj, uint8_t* od, uint64_t* status,
                            uint32_t* tile_counter, uint32_t epoch, unsigned long long* out_count,
                            uint32_t* err, hipStream_t s);
// bounds[s] = first position of qi[0, n) (n = min(n, *n_dev) with n_dev) whose
// value is >= set_base[s]
void launch_set_ranges(const uint32_t* qi, uint64_t n, const uint32_t* set_base, uint32_t nb,
                       uint64_t* bounds, hipStream_t s, const unsigned long long* n_dev = nullptr);
// oi[t] = qi[lo + t] + shift, oj[t] = rj[lo + t], od[t] = d[lo + t] for t < n
void launch_slice_rebase(const uint32_t* qi, const uint32_t* rj, const uint8_t* d, uint64_t lo,
                         uint64_t n, int64_t shift, uint32_t* oi, uint32_t* oj, uint8_t* od,
                         hipStream_t s);
// learned index
size_t leaf_bytes();
size_t coord_bytes();
int coord_lengths();
int coord_res();
void coord_offsets(size_t* lmin_off, size_t* rows_off);
void launch_interleave(const uint64_t* hi, const uint64_t* lo, uint64_t n, u128* out, hipStream_t s);
void launch_coord_counts(const u128* keys, uint64_t n, uint32_t S, uint32_t* counts, hipStream_t s);
void launch_train_sample(const u128* keys, uint64_t n, uint32_t S, const void* coord, float* x,
                         float* y, hipStream_t s);
uint32_t mlp_grad_blocks(uint32_t n);
void launch_mlp_grad(const float* p, const float* x, const float* y, uint32_t n, float* partial,
                     hipStream_t s);
void launch_grad_reduce(const float* partial, uint32_t nblocks, float* out, hipStream_t s);
int adam_state_floats();
void launch_adam_step(float* p, float* state, const float* partial, uint32_t nblocks, float lr,
                      int update, float* loss_out, uint32_t loss_cap, hipStream_t s);
void launch_adam_best(float* p, const float* state, hipStream_t s);
void launch_leaf_fit_all(const u128* keys, uint64_t n, const void* coord, const float* p,
                         uint32_t nleaves, void* leaves, hipStream_t s);
// coord_lengths_used: table rows of the model (lmax - lmin + 1, or 0)
void launch_probe(const u128* qseq, const uint64_t* qvoff, uint64_t nq, const u128* keys,
                  const uint32_t* kid, uint64_t n, int learned, const void* coord,
                  uint32_t coord_lengths_used, const float* p, uint32_t nleaves,
                  const void* leaves, const ShardArgs& out, unsigned long long* steps,
                  hipStream_t s);

// ------------------------------------------------------------------ errors

struct GraphPlan;  // a captured batched query (graphbatch.cpp)

struct Error {
  int code;
  std::string msg;
};

}  // namespace sd

// ------------------------------------------------------------------ context

struct sd_ctx {
  int device = 0;
  uint64_t budget = 0;  // 0 = unbounded
  uint64_t held = 0;    // bytes of device memory held (live + cached)
  std::string last_error;
  std::multimap<size_t, void*> cache;      // free device blocks by size (own hipMalloc blocks)
  std::unordered_map<void*, size_t> live;  // device blocks in use
  // allocator hook (sd_set_allocator): when set, device blocks come from
  // ualloc and go back to ufree at once (no cache of our own)
  sd_alloc_fn ualloc = nullptr;
  sd_free_fn ufree = nullptr;
  void* uarg = nullptr;
  // fixed-area mode (sd_self_search_noalloc): while arena is set, device
  // blocks are carved from [arena, arena + arena_size) in order and never
  // released one by one; the whole area is reused by the next such call
  unsigned char* arena = nullptr;
  size_t arena_size = 0, arena_used = 0;
  // pinned host result blocks (i, j and d of one result in one block) by
  // size, and released blocks kept for the next results
  std::unordered_map<void*, size_t> host_live;
  std::multimap<size_t, void*> host_cache;
  size_t host_cache_bytes = 0;
  // look-back state
  uint64_t* status = nullptr;
  size_t status_words = 0;
  uint32_t epoch = 0;
  uint32_t* counters = nullptr;  // small device counter area
  size_t counters_n = 0;
  int tile_slot = 0;  // next tile-counter slot of the current call (0: none handed out yet)
  void* pinned = nullptr;  // pinned host staging for small read-backs
  size_t pinned_bytes = 0;
  // pinned host staging of batched query sets (their offsets, the tiles'
  // rebased offsets), and the event after the last copies out of it
  int64_t* stage_host = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t stage_event = nullptr;
  bool stage_pending = false;
  sd_stats stats{};
  int timing = 0;
  int path = 0;        // 0 automatic, 1 full-key sort, 2 hashed
  int group_cap = 0;   // hashed path: LDS batch capacity (0 = automatic)
  int group_bits = 0;  // hashed path: hash bits sorted by the LSD passes (0 = automatic)
  int group_batches = 0;  // hashed path: LDS batches per workgroup (0 = automatic)
  int sort_items = 0;  // keys-only radix passes: items per thread, 16 or 32 (0 = automatic)
  int pair_sort = 0;   // candidate pair sort: 0 automatic, 1 one-sweep passes, 2 counted passes
  int group_shape = 0; // hashed path grouping kernel shape at capacity 2048 (SD_OPT_GROUP_SHAPE)
  int metric = SD_METRIC_LEVENSHTEIN;  // distance of the final filter (SD_OPT_METRIC)
  int stream = 0;              // streamed self search: 0 automatic, 1 never, 2 always
  uint64_t stream_elems = 0;   // elements per column group (0: from the budget)
  int64_t batch_tile_seqs = 0;  // query batches: sequences per tile (0 = automatic)
  int join_elems = 0;           // query tiles: query elements a join segment aims at (0 = automatic)
  std::string tune_cache;       // autotuner cache file (empty: none)
  int probe = 0;                // learned indexes: 0 model window, 1 whole-array binary search
  std::map<std::string, uint64_t> out_hint;  // last output size of each sharded stage
  std::map<std::string, uint64_t> noalloc_hint;  // the same, for no-allocation calls
  std::vector<hipEvent_t> events;
  // graph-captured batches (SD_OPT_BATCH_GRAPH): the cached plan of the last
  // batch shape, and the candidates per query variant seen so far (sizes the
  // candidate capacity of the next plan)
  int batch_graph = 0;
  std::vector<std::shared_ptr<sd::GraphPlan>> graph_plans;
  double graph_cand_ratio = 1.0 / 8.0;
};

// A reference deletion index. Hashed kind: every <= k-deletion variant of
// the reference set as [hash | ref id], sorted by the full hash without
// repeats, plus a directory of 2^bits hash segments. Learned kind: the exact
// keys sorted, their reference ids, and the two-stage position model. Owns
// its device memory (index_alloc), read-only after the build.
struct sd_index {
  int device = 0;
  // the allocator hook of the building context (null: hipMalloc / hipFree)
  sd_free_fn ufree = nullptr;
  void* uarg = nullptr;
  int k = 0;
  int learned = 0;  // 0 hashed, 1 learned
  uint32_t idbits = 24;
  int bits = 0;
  uint64_t n_ref = 0, n_keys = 0, bytes = 0;
  u128* ref_seq = nullptr;
  uint64_t* E = nullptr;
  uint32_t* seg_start = nullptr;
  uint32_t* seg_end = nullptr;
  // learned kind
  u128* keys = nullptr;
  uint32_t* kid = nullptr;
  float* params = nullptr;  // device, SD_MLP_PARAMS floats
  void* coord = nullptr;    // device coordinate model (residue frequency tables)
  uint32_t coord_rows = 0;  // key lengths with a table row (lmax - lmin + 1)
  void* leaves = nullptr;   // device leaf records
  uint32_t nleaves = 0;
  sd_learned_info info{};
  std::vector<float> loss_curve;
};

namespace sd {

// device memory pool (throws Error on failure)
void* dalloc(sd_ctx* c, size_t bytes);
void dfree(sd_ctx* c, void* p);
// a device array owned by an index (from the context's allocator hook if it
// has one, else hipMalloc); released by index_free
void* index_alloc(sd_ctx* c, sd_index* idx, size_t bytes);
void index_release(sd_index* idx, void* p);
template <typename T>
T* dalloc_t(sd_ctx* c, uint64_t count) {
  return static_cast<T*>(dalloc(c, (size_t)(count ? count : 1) * sizeof(T)));
}
// RAII list of scratch blocks released at scope exit
struct Scratch {
  sd_ctx* c;
  std::vector<void*> blocks;
  explicit Scratch(sd_ctx* ctx) : c(ctx) {}
  template <typename T>
  T* get(uint64_t count) {
    T* p = dalloc_t<T>(c, count);
    blocks.push_back(p);
    return p;
  }
  // give one block back before the scope ends (it leaves the list, so the
  // destructor does not free whatever later reuses its address)
  void release(void* p) {
    for (size_t x = 0; x < blocks.size(); ++x)
      if (blocks[x] == p) {
        blocks.erase(blocks.begin() + (long)x);
        dfree(c, p);
        return;
      }
  }
  ~Scratch() {
    for (void* p : blocks) dfree(c, p);
  }
};

void hip_check(hipError_t e, const char* what);
// once per device, with that device current: resolve the device address of
// the no-allocation entry point's fixed scratch area (SD_OK or SD_E_HIP)
int noalloc_setup(int device);
// sd_self_search_noalloc: the self search with every device block carved
// from the device's fixed scratch area, the result copied to the caller's
// arrays (*n_out = the result size, also when it exceeds capacity)
void self_search_noalloc(sd_ctx* c, const sd_seqs* seqs, int k, uint32_t* out_i, uint32_t* out_j,
                         uint8_t* out_d, int64_t capacity, int64_t* n_out, hipStream_t s);
// look-back status area with at least `words` words; returns a fresh epoch
uint32_t next_epoch(sd_ctx* c, uint64_t words, hipStream_t s);
// zeroed device counters (at least n), on stream s
uint32_t* fresh_counters(sd_ctx* c, size_t n, hipStream_t s);
// copy `bytes` from device to the pinned staging area and wait for stream s
void* readback(sd_ctx* c, const void* dptr, size_t bytes, hipStream_t s);
// Pinned host memory for a host result (a released block of bytes to twice
// that, else a new one); host_release keeps a block for reuse (up to a
// bounded total per context) or frees it.
void* host_block(sd_ctx* c, size_t bytes);
void host_release(sd_ctx* c, void* p);

// stage timing (HIP events on the call's stream; no host synchronisation
// until the end of the call)
struct StageTimer {
  sd_ctx* c;
  hipStream_t s;
  bool on;
  std::vector<std::pair<std::string, double>> names;  // name, algorithmic bytes
  std::vector<int> launches;
  StageTimer(sd_ctx* ctx, hipStream_t st);
  void mark(const char* name, double bytes, int launches = 1);  // ends the stage begun by the previous mark
  void finish();  // waits for the stream and fills ctx->stats
};

// the search pipelines
void hashed_plan(const sd_ctx* c, uint64_t nk, int* cap, int* bits);
void self_search(sd_ctx* c, const sd_seqs* seqs, int k, sd_pairs* out, hipStream_t s);
void paired_self_search(sd_ctx* c, const sd_seqs* a, const sd_seqs* b, int k, sd_pairs* out,
                        hipStream_t s);
void pair_distance(sd_ctx* c, const sd_seqs* a, const sd_seqs* b, const uint32_t* ia,
                   const uint32_t* ib, int64_t n, uint8_t* d_out, hipStream_t s);
struct WeightedSpec;
sd_index* index_build(sd_ctx* c, const sd_seqs* ref, int k, hipStream_t s);
void index_free(sd_index* idx);
void query_sets(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k,
                const WeightedSpec* w, sd_pairs* outs, hipStream_t s);
void query_weighted(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets,
                    const uint8_t* subst, int indel, int max_score, sd_pairs* outs,
                    hipStream_t s);
sd_index* learned_build(sd_ctx* c, const sd_seqs* ref, int k, const sd_learned_config* cfg,
                        hipStream_t s);
void autotune(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k, int reps,
              sd_tune_result* out, hipStream_t s);
void mlp_gradients(sd_ctx* c, const float* params, const float* x, const float* y, uint32_t n,
                   float* grad, float* loss, hipStream_t s);

}  // namespace sd
