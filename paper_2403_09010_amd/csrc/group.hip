// Hashed grouping path for gfx950: equal deletion variants are brought
// together without sorting the 128-bit keys themselves.
//
//   k_vargen_hash   every <= k-deletion variant of every sequence as one
//                   64-bit element [hash of the variant | sequence id],
//                   with 24 id bits (40 hash bits) up to 2^24 sequences and
//                   32 id bits (32 hash bits) above; also the digit
//                   histograms of the hash passes
//   (LSD passes)    k_onesweep_keys over the top B hash bits (radix.hip):
//                   equal keys have equal hashes, so every group of equal
//                   keys lies inside one "segment" of equal top-B bits
//   k_seg_bounds    the [start, end) range of every segment
//   k_group_seg     one workgroup per run of whole segments: an LDS hash
//                   table groups the elements by their full stored hash and
//                   emits the id pairs of every group (the paper's
//                   uniqueCount + expand, Appendix A steps 4-5)
//   k_gather_big    segments larger than the LDS capacity are copied out,
//   k_emit_hash_runs  sorted by their full hash and emitted by runs
//
// Grouping by a hash instead of the exact key cannot lose a pair (equal keys
// hash alike); a collision only adds a candidate whose exact distance the
// verification step then rejects, so the result is the same set.
#include "sd_device.h"
#include "sd_internal.h"

namespace sdk {

// 64-bit hash of a string y of length m: h(y) = C[m] xor the XOR over
// positions j of rotr(B[y_j], j), with B (per residue) and C (per length)
// fixed pseudo-random words. Rotation commutes with XOR, so a residue that
// moves one or two places left after a deletion changes its term by a left
// rotation of 1 or 2: with the prefix XORs P[i] of the undeleted string, the
// variant without positions p1 < p2 hashes to
//   C[m] ^ P[p1] ^ rotl(P[p2] ^ P[p1 + 1], 1) ^ rotl(P[L] ^ P[p2 + 1], 2),
// five LDS reads instead of rebuilding the 128-bit key. One deletion is the
// case p2 = L, none the case p1 = L, p2 = L + 1 (P is constant past L). Only
// the load balance and the rate of extra candidates depend on the hash.
struct HashTab {
  uint64_t b[32];  // per residue code (code 20 is the paired-chain join token)
  uint64_t c[64];  // per string length (paired-chain variants reach 49)
};

// splitmix64 (Steele, Lea and Flood, 2014) as a compile-time generator
constexpr uint64_t splitmix_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

constexpr HashTab make_hash_tab() {
  HashTab t{};
  uint64_t state = 0x5D3E1B7A2C4F9081ull;
  for (int x = 0; x < 32; ++x) t.b[x] = splitmix_next(state);
  for (int x = 0; x < 64; ++x) t.c[x] = splitmix_next(state);
  return t;
}

__constant__ HashTab kHashTab = make_hash_tab();

// a mix of a stored hash for LDS table slots
__device__ __forceinline__ uint32_t slot_mix(uint64_t h) {
  uint32_t x = (uint32_t)h ^ (uint32_t)(h >> 32) * 0x9E3779B1u;
  x ^= x >> 15;
  x *= 0x2C1B3C6Du;
  x ^= x >> 12;
  x *= 0x297A2D39u;
  x ^= x >> 15;
  return x;
}

// ------------------------------------------------------------------ vargen + hash

constexpr int VG_NT = 256;
constexpr int VG_SEQS = sd::VG_MAX_SEQS_PER_BLOCK;

// Digit q of the hash passes is (e >> shift[q]) & mask[q].
struct PassDigits {
  uint32_t shift[3];
  uint32_t mask[3];
};

// prefix XORs per sequence: indices 0..L + 2 <= 26 are read (0..L + 3 with
// three deletions); an odd row length starts consecutive rows in different
// LDS banks
constexpr int VG_PRE = 27;
constexpr int VG_PRE3 = 29;

// Deletion pairs in colexicographic order (p2 major): pair u is (p1, p2)
// with u = p2 (p2 - 1) / 2 + p1, the same for every length L (a string of
// length L uses the first C(L, 2) of them). Entry: p1 | p2 << 8.
constexpr int VG_PAIRS = KEY_MAX_LEN * (KEY_MAX_LEN - 1) / 2;
static_assert(VG_PAIRS % 2 == 0, "the pair table is copied as 32-bit words");

struct PairTab {
  uint32_t w[VG_PAIRS / 2];  // entries 2 i and 2 i + 1, low half first
};

constexpr PairTab make_pair_tab() {
  PairTab t{};
  int u = 0;
  for (int p2 = 1; p2 < KEY_MAX_LEN; ++p2)
    for (int p1 = 0; p1 < p2; ++p1, ++u) {
      const uint32_t e = (uint32_t)p1 | ((uint32_t)p2 << 8);
      t.w[u / 2] |= (u % 2) ? e << 16 : e;
    }
  return t;
}

__constant__ PairTab kPairTab = make_pair_tab();

// C(p, 3) for p = 0..KEY_MAX_LEN: the colexicographic rank of the first
// triple with largest position p (triples with largest position p3 are the
// pairs below p3 in their own colexicographic order).
struct TriTab {
  uint16_t c3[KEY_MAX_LEN + 1];
};

constexpr TriTab make_tri_tab() {
  TriTab t{};
  for (int p = 0; p <= KEY_MAX_LEN; ++p) t.c3[p] = (uint16_t)(p * (p - 1) * (p - 2) / 6);
  return t;
}

__constant__ TriTab kTriTab = make_tri_tab();

// Deletion positions of variant v of a string of length L, with up to three
// deletions, as a padded triple (see variant_canonical3): v = 0 none, 1..L
// one, then the C(L, 2) pairs, then the triples, each in colexicographic
// order. The largest position of a triple is found by binary search of c3.
__device__ __forceinline__ void variant_positions3(const uint16_t* s_pairs, const uint16_t* s_c3,
                                                   uint32_t L, uint32_t v, uint32_t& p1,
                                                   uint32_t& p2, uint32_t& p3) {
  const uint32_t np = L * (L - 1) / 2;
  if (v == 0) {
    p1 = L;
    p2 = L + 1;
    p3 = L + 2;
  } else if (v <= L) {
    p1 = v - 1;
    p2 = L;
    p3 = L + 1;
  } else if (v <= L + np) {
    const uint32_t pr = s_pairs[v - 1 - L];
    p1 = pr & 0xFFu;
    p2 = pr >> 8;
    p3 = L;
  } else {
    const uint32_t u = v - 1 - L - np;
    uint32_t lo = 2, hi = L - 1;  // the largest p3 with c3[p3] <= u
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (s_c3[mid] <= u)
        lo = mid;
      else
        hi = mid - 1;
    }
    p3 = lo;
    const uint32_t pr = s_pairs[u - s_c3[lo]];
    p1 = pr & 0xFFu;
    p2 = pr >> 8;
  }
}

// Deletion positions of variant v of a string of length L in the enumeration
// order (v = 0 the string itself, v = 1..L one deletion at v - 1, then the
// pairs in colexicographic order), in the form the prefix-XOR hash takes:
// p2 = L for one deletion, p1 = L and p2 = L + 1 for none.
__device__ __forceinline__ void variant_positions(const uint16_t* s_pairs, uint32_t L, uint32_t v,
                                                  uint32_t& p1, uint32_t& p2) {
  const uint32_t u = v > L ? v - 1 - L : 0u;
  const uint32_t pr = s_pairs[u < (uint32_t)VG_PAIRS ? u : 0u];
  const bool none = v == 0, one = v != 0 && v <= L;
  p1 = none ? L : one ? v - 1 : (pr & 0xFFu);
  p2 = none ? L + 1 : one ? L : (pr >> 8);
}

// One block per spb sequences; every V(L, k) deletion set of each is
// enumerated (see the loop below for how waves share them out). DISTINCT: the
// variant offsets count distinct strings only
// (num_distinct_variants), and a wave writes the canonical deletion sets of
// the sequence compactly, in enumeration order, at its offset. K3: up to
// three deletions (padded triples, variant_positions3 and
// variant_canonical3); the hash of a variant with at most two deletions is
// the same either way.
// MODE 0 writes every variant at its offset (and counts digits); MODE 1
// writes nothing and only counts the first digit (the bin histogram of the
// streamed search); MODE 2 keeps the variants whose bin (top STREAM_BIN_BITS
// hash bits) lies in [blo, bhi) and appends them to the sharded output sout,
// one reservation per wave, with the hash rotated left by the bin bits (the
// bits that still tell variants of one column group apart move to the top).
template <bool DISTINCT, bool K3, int MODE>
__global__ __launch_bounds__(VG_NT) void k_vargen_hash(const u128* __restrict__ seq,
                                                       const uint64_t* __restrict__ voff,
                                                       uint64_t nseq, int k,
                                                       uint64_t* __restrict__ elem,
                                                       uint32_t idbits, int npass, PassDigits pd,
                                                       uint32_t* __restrict__ hist,
                                                       uint32_t* __restrict__ tcounts,
                                                       uint32_t spb, ShardOut sout, uint32_t blo,
                                                       uint32_t bhi, uint32_t ftile) {
  constexpr int NWV = VG_NT / 64;
  constexpr int PRE = K3 ? VG_PRE3 : VG_PRE;
  __shared__ uint64_t s_off[VG_SEQS + 1];
  __shared__ uint64_t s_pre[VG_SEQS * PRE];
  __shared__ uint64_t s_c[32];
  __shared__ uint32_t s_len[VG_SEQS];
  __shared__ uint32_t s_n1[VG_SEQS], s_n2[VG_SEQS];  // canonical-test masks
  __shared__ uint32_t s_n3[K3 ? VG_SEQS : 1];
  __shared__ uint16_t s_c3[K3 ? KEY_MAX_LEN + 1 : 1];
  __shared__ uint32_t s_roff[VG_SEQS + 1];            // block-local deletion-set prefix
  // the digit counts; until the prefix XORs are done, the same LDS holds
  // the hash's per-residue words
  __shared__ __align__(16) uint32_t s_h[3 * 256];
  uint64_t* s_b = reinterpret_cast<uint64_t*>(s_h);  // [32]
  __shared__ __align__(4) uint16_t s_pairs[VG_PAIRS];
  // spb <= VG_SEQS sequences per block
  const uint64_t s0 = (uint64_t)blockIdx.x * spb;
  const uint32_t ns = (uint32_t)min<uint64_t>(spb, nseq - s0);
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  // every global load of the set-up is issued at once (one thread loads at
  // most one offset, one key, one hash word and one pair-table word;
  // ns <= 64 < VG_NT), so the block waits for one memory round trip
  const uint32_t tx = threadIdx.x;
  const uint64_t ld_off = tx <= ns ? voff[s0 + tx] : 0;
  const u128 key = tx < ns ? seq[s0 + tx] : (u128)0;
  const uint64_t ld_tab = tx < 32 ? kHashTab.b[tx] : tx < 64 ? kHashTab.c[tx - 32] : 0;
  const uint32_t ld_pair = tx < (uint32_t)VG_PAIRS / 2 ? kPairTab.w[tx] : 0u;
  if (tx <= ns) s_off[tx] = ld_off;
  if (tx < 32) s_b[tx] = ld_tab;
  else if (tx < 64) s_c[tx - 32] = ld_tab;
  if (tx < (uint32_t)VG_PAIRS / 2) reinterpret_cast<uint32_t*>(s_pairs)[tx] = ld_pair;
  if (K3 && tx <= (uint32_t)KEY_MAX_LEN) s_c3[tx] = kTriTab.c3[tx];
  __syncthreads();
  // one thread per sequence: the prefix XORs P[t] of the position terms
  // rotr(B[s[i]], i), i < t, for t = 0 .. L + 2 (P[L + 1] = P[L + 2] = P[L],
  // which the hash reads for "no second deletion"), and the canonical-test
  // masks: n1 bit t = (t = L - 1 or s[t] != s[t + 1]), n2 bit t =
  // (t = L - 2 or s[t] != s[t + 2])
  if (tx < ns) {
    const uint32_t L = key_len(key);
    uint64_t* P = s_pre + tx * PRE;
    uint64_t acc = 0;
    uint32_t n1 = 0, n2 = 0, r1 = 0, r2 = 0;  // r1 = s[t - 1], r2 = s[t - 2]
    uint32_t n3 = 0, r3 = 0;                  // r3 = s[t - 3]
    u128 kk = key << 8;                        // residue t at the top 5 bits
    P[0] = 0;
    for (uint32_t t = 0; t < L; ++t) {
      const uint32_t r = (uint32_t)(kk >> 123);
      kk <<= 5;
      acc ^= __builtin_rotateright64(s_b[r], t);
      P[t + 1] = acc;
      if (DISTINCT) {
        if (t >= 1) n1 |= (uint32_t)(r1 != r) << (t - 1);
        if (t >= 2) n2 |= (uint32_t)(r2 != r) << (t - 2);
        if (K3 && t >= 3) n3 |= (uint32_t)(r3 != r) << (t - 3);
        r3 = r2;
        r2 = r1;
        r1 = r;
      }
    }
    P[L + 1] = acc;
    P[L + 2] = acc;
    if (K3) P[L + 3] = acc;
    if (DISTINCT) {
      if (L >= 1) n1 |= 1u << (L - 1);
      if (L >= 2) n2 |= 1u << (L - 2);
      s_n1[tx] = n1;
      s_n2[tx] = n2;
      if (K3) {  // bits p >= L - 3 hold no residue three places on
        const uint32_t all = (1u << L) - 1u;
        s_n3[tx] = n3 | (L >= 3 ? all & ~((1u << (L - 3)) - 1u) : all);
      }
    }
    s_len[tx] = L;
  }
  __syncthreads();
  // the keys and table words are dead: the area becomes the digit counts
  for (uint32_t x = threadIdx.x; x < 3 * 256; x += VG_NT) s_h[x] = 0;
  // block-local first deletion set of each sequence: V(L, k) each
  if (w == 0) {
    const uint32_t c = lane < ns ? (DISTINCT ? num_variants(s_len[lane], k)
                                             : (uint32_t)(s_off[lane + 1] - s_off[lane]))
                                 : 0u;
    const uint32_t incl = wave_incl_scan(c);
    if (lane < ns) s_roff[lane + 1] = incl;
    if (lane == 0) s_roff[0] = 0;
  }
  __syncthreads();
  const uint64_t g0 = s_off[0];
  const uint64_t idmask = (1ull << idbits) - 1;
  const uint32_t sh[3] = {pd.shift[0], pd.shift[1], pd.shift[2]};
  const uint32_t mk[3] = {pd.mask[0], pd.mask[1], pd.mask[2]};
  uint64_t* __restrict__ out = elem + g0;
  const bool tiled = tcounts != nullptr;
  // ftile != 0 (with tcounts, one pass): the first pass's digits are counted
  // per fixed output tile of ftile elements instead of per block, so that the
  // first LSD pass runs over aligned tiles like the later ones. The block's
  // elements [g0, g0 + its count) meet at most three tiles in LDS (slots 0-2
  // of s_h, from tile0 on; local offsets b1 and b2 start slots 1 and 2);
  // anything further goes to global memory directly.
  const uint64_t tile0 = ftile ? g0 / ftile : 0;
  const uint32_t b1 = ftile ? (uint32_t)((tile0 + 1) * ftile - g0) : 0u;
  const uint32_t b2 = b1 + ftile, b3 = b2 + ftile;
  // Each wave takes a contiguous quarter of the sequences. A sequence with
  // more than 64 deletion sets is enumerated alone, 128 at a time; runs of
  // consecutive smaller ones share one 64-lane chunk (lane -> sequence by a
  // binary search of the block-local prefix s_roff).
  auto emit = [&](uint64_t e, bool keep, uint32_t at, uint32_t rank, uint32_t end) {
    // (the pack kernel's count and the canonical test agree, so the bound
    // never drops a variant; it keeps any disagreement in range)
    if (keep && at + rank < end) {
      if constexpr (MODE == 0) out[at + rank] = e;
      if (ftile) {
        const uint32_t lo = at + rank;
        const uint32_t d = (uint32_t)(e >> sh[0]) & mk[0];
        if (lo < b3)
          atomicAdd(&s_h[((lo >= b1) + (lo >= b2)) * 256u + d], 1u);
        else
          atomicAdd(&tcounts[(tile0 + 3 + (lo - b3) / ftile) * 256 + d], 1u);
      } else {
#pragma unroll
        for (int q = 0; q < 3; ++q)
          if (q < npass) atomicAdd(&s_h[q * 256 + ((uint32_t)(e >> sh[q]) & mk[q])], 1u);
      }
    }
  };
  // MODE 2: one shard reservation for the wave's kept lanes (bal is the
  // wave's ballot of keep, so every lane takes the same branch). A wave's
  // reservations go to consecutive shards from a start that is odd multiple
  // of its wave index, so every shard is equally likely to be any wave's
  // first, second, ... (the shards fill evenly, also with few workgroups).
  uint32_t nres = 0;
  auto put_sharded = [&](uint64_t e, bool keep, uint64_t bal) {
    if (!bal) return;
    const uint32_t sel = (blockIdx.x * NWV + w) * 17u + nres++;
    uint64_t pos = 0, ob = 0;
    if (lane == 0) {
      const ShardResv r = shard_reserve(sout, sel, (uint64_t)__popcll(bal));
      pos = r.pos;
      ob = r.obase;
    }
    pos = __shfl(pos, 0, 64);
    ob = __shfl(ob, 0, 64);
    if (keep) shard_put(sout, sel, ShardResv{pos, ob}, mask_rank(bal), e);
  };
  // the element of a variant's hash h (MODE 2: rotated, and only inside the
  // column group's bins)
  auto element = [&](uint64_t h, uint64_t id, bool& valid) -> uint64_t {
    if constexpr (MODE == 2) {
      const uint32_t bin = (uint32_t)(h >> (64 - sd::STREAM_BIN_BITS));
      valid = valid && bin >= blo && bin < bhi;
      return (__builtin_rotateleft64(h, sd::STREAM_BIN_BITS) & ~idmask) | id;
    }
    return (h & ~idmask) | id;
  };
  // what every variant of sequence x reads, loaded once per sequence: the
  // length, the extended canonical-test masks, the prefix-XOR row with its
  // entry P[L], and the length words C[L - d] for d = 0, 1, 2 deletions
  struct SeqVals {
    uint32_t L, n1x, n2x, n3;
    const uint64_t* P;
    uint64_t pl, c0, c1, c2, c3, id;
  };
  auto seq_vals = [&](uint32_t x) {
    SeqVals q;
    q.L = s_len[x];
    q.P = s_pre + x * PRE;
    q.pl = q.P[q.L];
    q.c0 = s_c[q.L];
    q.c1 = s_c[q.L >= 1 ? q.L - 1 : 0u];
    q.c2 = s_c[q.L >= 2 ? q.L - 2 : 0u];
    q.c3 = K3 ? s_c[q.L >= 3 ? q.L - 3 : 0u] : 0;
    q.n1x = q.n2x = q.n3 = 0;
    if (DISTINCT) canonical_ext_masks(s_n1[x], s_n2[x], q.L, q.n1x, q.n2x);
    if (DISTINCT && K3) q.n3 = s_n3[x];
    q.id = s0 + x;
    return q;
  };
  auto variant = [&](SeqVals q, uint32_t v, bool valid, uint64_t& e) -> bool {
    if constexpr (K3) {
      uint32_t p1, p2, p3;
      variant_positions3(s_pairs, s_c3, q.L, valid ? v : 0u, p1, p2, p3);
      const uint64_t cm = p3 < q.L ? q.c3 : p2 < q.L ? q.c2 : p1 < q.L ? q.c1 : q.c0;
      const uint64_t* P = q.P;
      const uint64_t h = cm ^ P[p1] ^ __builtin_rotateleft64(P[p2] ^ P[p1 + 1], 1) ^
                         __builtin_rotateleft64(P[p3] ^ P[p2 + 1], 2) ^
                         __builtin_rotateleft64(q.pl ^ P[p3 + 1], 3);
      e = element(h, q.id, valid);
      return valid && (!DISTINCT || variant_canonical3(q.n1x, q.n2x, q.n3, q.L, p1, p2, p3));
    }
    uint32_t p1, p2;
    variant_positions(s_pairs, q.L, valid ? v : 0u, p1, p2);
    const uint64_t cm = p2 < q.L ? q.c2 : p1 < q.L ? q.c1 : q.c0;
    const uint64_t* P = q.P;
    const uint64_t h = cm ^ P[p1] ^ __builtin_rotateleft64(P[p2] ^ P[p1 + 1], 1) ^
                       __builtin_rotateleft64(q.pl ^ P[p2 + 1], 2);
    e = element(h, q.id, valid);
    return valid && (!DISTINCT || variant_canonical_ext(q.n1x, q.n2x, p1, p2));
  };
  const uint32_t xa = w * ns / NWV, xb = (w + 1) * ns / NWV;
  for (uint32_t x = xa; x < xb;) {
    const uint32_t nraw = s_roff[x + 1] - s_roff[x];
    const uint32_t end_x = (uint32_t)(s_off[x + 1] - g0);
    if (nraw > 64) {
      uint32_t at = (uint32_t)(s_off[x] - g0);  // next output slot of this sequence
      const SeqVals q = seq_vals(x);
      for (uint32_t c0 = 0; c0 < nraw; c0 += 128) {
        uint64_t e[2];
        bool keep[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint32_t v = c0 + 64 * u + lane;
          keep[u] = variant(q, v, v < nraw, e[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint64_t bal = __ballot(keep[u]);
          if constexpr (MODE == 2)
            put_sharded(e[u], keep[u], bal);
          else
            emit(e[u], keep[u], at, mask_rank(bal), end_x);
          at += (uint32_t)__popcll(bal);
        }
      }
      ++x;
      continue;
    }
    // sequences x .. y - 1 fill at most 64 lanes
    uint32_t y = x + 1;
    while (y < xb && s_roff[y + 1] - s_roff[x] <= 64) ++y;
    const uint32_t slot = s_roff[x] + lane;
    const bool valid = slot < s_roff[y];
    uint32_t lo = x, hi = y - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (s_roff[mid] <= slot)
        lo = mid;
      else
        hi = mid - 1;
    }
    uint64_t e;
    const bool keep = variant(seq_vals(lo), slot - s_roff[lo], valid, e);
    const uint64_t bal = __ballot(keep);
    if constexpr (MODE == 2) {
      put_sharded(e, keep, bal);
    } else {
      // rank among the kept lanes of the same sequence (a contiguous lane range)
      const uint32_t zl = s_roff[lo] - s_roff[x];
      const uint64_t mine = bal & ~((1ull << zl) - 1ull);
      emit(e, keep, (uint32_t)(s_off[lo] - g0), mask_rank(mine), (uint32_t)(s_off[lo + 1] - g0));
    }
    x = y;
  }
  __syncthreads();
  // With tcounts, every pass's counts are stored as this block's rows (pass
  // q's rows start at q * gridDim.x): pass 0's are the tiles of the counted
  // first pass, the others are summed by k_hist_rows (plain stores instead
  // of thousands of blocks adding into the same 256 counters).
  if (tiled && ftile) {
    // neighbouring blocks share the tiles at their edges: add
    for (uint32_t x = threadIdx.x; x < 3u * 256; x += VG_NT)
      if (s_h[x]) atomicAdd(&tcounts[(tile0 + (x >> 8)) * 256 + (x & 255u)], s_h[x]);
  } else if (tiled) {
    for (uint32_t x = threadIdx.x; x < (uint32_t)npass * 256; x += VG_NT)
      tcounts[((uint64_t)(x >> 8) * gridDim.x + blockIdx.x) * 256 + (x & 255u)] = s_h[x];
  } else {
    for (uint32_t x = threadIdx.x; x < (uint32_t)npass * 256; x += VG_NT)
      if (s_h[x]) atomicAdd(&hist[x], s_h[x]);
  }
}

// hist[q * 256 + d] += the sum over rows r of rows[(q * nrows + r) * 256 + d]
// for passes q = 1 .. npass - 1; block (x, q - 1) sums a slice of the rows.
constexpr int HR_LOADS = 16;
__global__ __launch_bounds__(256) void k_hist_rows(const uint32_t* __restrict__ rows,
                                                   uint32_t nrows, uint32_t* __restrict__ hist) {
  const uint32_t q = blockIdx.y + 1, d = threadIdx.x;
  const uint32_t per = (nrows + gridDim.x - 1) / gridDim.x;
  const uint32_t r0 = min(blockIdx.x * per, nrows), r1 = min(r0 + per, nrows);
  const uint32_t* __restrict__ base = rows + (uint64_t)q * nrows * 256 + d;
  uint32_t sum = 0;
  for (uint32_t r = r0; r < r1; r += HR_LOADS) {
    uint32_t c[HR_LOADS];
#pragma unroll
    for (int u = 0; u < HR_LOADS; ++u) c[u] = r + u < r1 ? base[(uint64_t)(r + u) * 256] : 0u;
#pragma unroll
    for (int u = 0; u < HR_LOADS; ++u) sum += c[u];
  }
  if (sum) atomicAdd(&hist[q * 256 + d], sum);
}

// ------------------------------------------------------------------ segment bounds

// After the LSD passes E is sorted by its top B bits (segshift = 64 - B; a
// shift of 64 means one segment), so segment v is [seg_start[v], seg_end[v])
// with seg_start[v] the first position whose top bits are >= v. One thread
// per boundary v in [0, nseg] finds it by binary search (the upper levels of
// all searches share cache lines), which touches a few MB instead of reading
// the whole array; an absent segment gets an empty range.
__device__ __forceinline__ uint32_t seg_of(uint64_t e, uint32_t segshift) {
  return segshift >= 64 ? 0u : (uint32_t)(e >> segshift);
}

__global__ __launch_bounds__(256) void k_seg_bounds(const uint64_t* __restrict__ E, uint32_t n,
                                                    uint32_t segshift, uint32_t nseg,
                                                    uint32_t* __restrict__ seg_start,
                                                    uint32_t* __restrict__ seg_end) {
  const uint32_t v = blockIdx.x * 256 + threadIdx.x;
  if (v > nseg) return;
  uint32_t lo = 0, hi = n;
  if (v == nseg) {
    lo = n;
  } else {
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (seg_of(E[mid], segshift) < v)
        lo = mid + 1;
      else
        hi = mid;
    }
  }
  if (v < nseg) seg_start[v] = lo;
  if (v > 0) seg_end[v - 1] = lo;
}

// ------------------------------------------------------------------ local grouping

// LDS layout for a batch of at most CAP elements, which arrive in registers;
// only the prefilter's candidates (at most MC of them: CAP / 2 in the main
// grouping kernel, CAP in the second pass over listed ranges) are grouped in
// LDS, 22 bytes each:
//   [0, 8 MC)        the compacted candidates (hash | id)
//   [8 MC, 16 MC)    the prefilter's two bitmaps (32 MC bits each), then
//                    the open-addressing table, 2 MC slots of candidate + 1
//   [16 MC, 20 MC)   per representative: the last member pushed (or NONE)
//   [20 MC, 22 MC)   per member: the member pushed before it (or NONE); a
//                    repeated (hash, id) is marked REPEAT and never pushed
// A batch with more than MC candidates is listed instead (for the second
// pass, whose table holds CAP). A split half (<= CAP elements) is staged in
// [0, 8 CAP), which for MC = CAP / 2 covers the table area.
constexpr uint32_t NONE16 = 0xFFFFu;
constexpr uint16_t REPEAT16 = 0xFFFEu;
constexpr int GROUP_LDS_PER_CAND = 22;

// One batch of m_in <= CAP elements whose values arrive in registers
// (element x = threadIdx.x + r * NTH is in e_in[r]); the caller has already
// issued the loads of the next batch, so their latency overlaps this batch's
// LDS work. On entry and on return the table area (2 MC words) is zero.
//
// Most elements have a hash no other element of the batch shares. A
// prefilter finds the rest first: every element sets the bit of its low hash
// bits in a bitmap of 32 MC bits (atomicOr returns whether the bit was
// already set; if so the bit is also set in a second bitmap), and only the
// elements whose bit ends up in the second bitmap (every element of a group
// of equal hashes, plus about m / (32 MC) of the others) are compacted, in
// order, and grouped in the table. No pair is lost: equal hashes have equal
// bits.
// Pairs collect in an LDS buffer of GROUP_PBUF entries (pbuf_n of them used,
// a block-uniform count) and go out with one reservation when it fills or
// the workgroup ends, instead of one global atomic per batch.
constexpr uint32_t GROUP_PBUF = 896;

template <int NTH>
__device__ void flush_pairs(const ShardOut& out, const uint64_t* s_pbuf, uint32_t n,
                            uint64_t* s_base) {
  if (threadIdx.x == 0) {
    const ShardResv r = shard_reserve(out, blockIdx.x, n);
    s_base[0] = r.pos;
    s_base[1] = r.obase;
  }
  __syncthreads();
  const ShardResv r{s_base[0], s_base[1]};
  for (uint32_t i = threadIdx.x; i < n; i += NTH) shard_put(out, blockIdx.x, r, i, s_pbuf[i]);
  __syncthreads();
}

template <int CAP, int NTH, int MCAND = CAP / 2>
__device__ bool group_batch(const uint64_t (&e_in)[CAP / NTH], uint32_t m_in, uint32_t idbits,
                            const ShardOut& out, unsigned char* lds, uint64_t* s_tmp64,
                            uint64_t* s_base, uint64_t* s_pbuf, uint32_t& pbuf_n, uint64_t ga,
                            uint64_t gb, uint64_t* __restrict__ big,
                            unsigned long long* __restrict__ nbig) {
  constexpr int PER = CAP / NTH;
  constexpr uint32_t MC = MCAND;
  static_assert(MC <= (uint32_t)CAP && MC <= 0xFFF0u, "members are 16-bit indices");
  constexpr int NW = NTH / 64;
  constexpr int NC = PER * NW;
  static_assert(NC % 4 == 0, "compaction counts are read four at a time");
  __shared__ __align__(16) uint32_t s_cnt[NC];
  uint64_t* s_e = reinterpret_cast<uint64_t*>(lds);
  uint32_t* s_tab = reinterpret_cast<uint32_t*>(lds + MC * 8);
  uint32_t* s_chead = reinterpret_cast<uint32_t*>(lds + MC * 16);
  uint16_t* s_next = reinterpret_cast<uint16_t*>(lds + MC * 20);
  const uint64_t idmask = (1ull << idbits) - 1;
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;

  // prefilter: the two bitmaps occupy the (zero) table area
  uint32_t* s_seen = s_tab;
  uint32_t* s_twice = s_tab + MC;
  uint32_t bitx[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const uint32_t x = threadIdx.x + r * NTH;
    bitx[r] = (uint32_t)(e_in[r] >> idbits) & (32u * MC - 1);
    if (x < m_in) {
      const uint32_t bit = 1u << (bitx[r] & 31u);
      if (atomicOr(&s_seen[bitx[r] >> 5], bit) & bit) atomicOr(&s_twice[bitx[r] >> 5], bit);
    }
  }
  __syncthreads();
  uint64_t keep[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const uint32_t x = threadIdx.x + r * NTH;
    keep[r] = __ballot(x < m_in && ((s_twice[bitx[r] >> 5] >> (bitx[r] & 31u)) & 1u));
    if (lane == 0) s_cnt[r * NW + w] = (uint32_t)__popcll(keep[r]);
  }
  __syncthreads();
  // every thread sums the counts before each of its (row, wave) pieces; the
  // bitmaps are dead now and are cleared for the next batch
  uint32_t before[PER];
  uint32_t m = 0;
#pragma unroll
  for (int i = 0; i < NC; i += 4) {
    const uint4 c4 = *reinterpret_cast<const uint4*>(&s_cnt[i]);
    const uint32_t c[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if ((i + j) % NW == (int)w) before[(i + j) / NW] = m;
      m += c[j];
    }
  }
  for (uint32_t x = threadIdx.x; x < 2 * MC; x += NTH) s_tab[x] = 0;
  if (m > MC) {
    // too many candidates for the table: the batch's whole range is listed
    // for the second pass (a pair found twice is dropped at verification)
    if (threadIdx.x == 0) {
      const unsigned long long x = atomicAdd(nbig, 1ull);
      big[2 * x] = ga;
      big[2 * x + 1] = gb;
    }
    __syncthreads();
    return true;
  }
#pragma unroll
  for (int r = 0; r < PER; ++r)
    if ((keep[r] >> lane) & 1u) s_e[before[r] + mask_rank(keep[r])] = e_in[r];
  for (uint32_t x = threadIdx.x; x < m; x += NTH) s_chead[x] = NONE16;
  __syncthreads();
  if (m == 0) return false;
  uint32_t ts = 64;  // table slots: a power of two >= 2m
  while (ts < 2 * m) ts <<= 1;

  // Repeated (hash, id) come from one sequence yielding one variant twice
  // (deleting either of two equal neighbours); inside a segment the stable
  // passes keep generation order, so equal ids are adjacent. Everything else
  // goes into the table and onto its representative's member chain.
  for (uint32_t x = threadIdx.x; x < m; x += NTH) {
    const uint64_t ex = s_e[x];
    const uint64_t h = ex >> idbits;
    const uint64_t id = ex & idmask;
    bool repeat = false;
    for (int y = (int)x - 1; y >= 0 && (s_e[y] & idmask) == id; --y) {
      if ((s_e[y] >> idbits) == h) {
        repeat = true;
        break;
      }
    }
    if (repeat) {
      s_next[x] = REPEAT16;
    } else {
      uint32_t slot = slot_mix(h) & (ts - 1);
      uint32_t rep;
      while (true) {
        uint32_t t = s_tab[slot];
        if (t == 0) {
          t = atomicCAS(&s_tab[slot], 0u, x + 1);
          if (t == 0) {
            rep = x;
            break;
          }
        }
        if ((s_e[t - 1] >> idbits) == h) {
          rep = t - 1;
          break;
        }
        slot = (slot + 1) & (ts - 1);
      }
      s_next[x] = (uint16_t)atomicExch(&s_chead[rep], x);
    }
  }
  __syncthreads();
  // each member pairs with the members pushed before it (distinct ids)
  uint32_t mycnt = 0;
  for (uint32_t x = threadIdx.x; x < m; x += NTH) {
    uint32_t y = s_next[x];
    if (y != REPEAT16)
      for (; y != NONE16; y = s_next[y]) ++mycnt;
  }
  // output slots in the pair buffer (or, for a batch with more pairs than
  // the buffer holds, one reservation of its own in the block's shard). The
  // batch total is a property of its groups (per-thread counts depend on the
  // order members were pushed), so every shard's count is reproducible.
  const uint32_t incl = wave_incl_scan(mycnt);
  if (lane == 63) s_tmp64[w] = incl;
  __syncthreads();
  uint64_t excl = incl - mycnt, total = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const uint64_t t = s_tmp64[q];
    if (q < (int)w) excl += t;
    total += t;
  }
  if (total) {
    if (pbuf_n + total > GROUP_PBUF) {
      flush_pairs<NTH>(out, s_pbuf, pbuf_n, s_base);
      pbuf_n = 0;
    }
    const bool direct = total > GROUP_PBUF;
    if (direct) {
      if (threadIdx.x == 0) {
        const ShardResv r = shard_reserve(out, blockIdx.x, total);
        s_base[0] = r.pos;
        s_base[1] = r.obase;
      }
      __syncthreads();
    }
    if (mycnt) {
      const ShardResv r{s_base[0], s_base[1]};
      uint64_t j = excl;
      for (uint32_t x = threadIdx.x; x < m; x += NTH) {
        uint32_t y = s_next[x];
        if (y == REPEAT16) continue;
        const uint32_t id = (uint32_t)(s_e[x] & idmask);
        for (; y != NONE16; y = s_next[y]) {
          const uint32_t other = (uint32_t)(s_e[y] & idmask);
          const uint32_t lo = id < other ? id : other, hi = id < other ? other : id;
          const uint64_t pair = ((uint64_t)lo << 32) | hi;
          if (direct)
            shard_put(out, blockIdx.x, r, j++, pair);
          else
            s_pbuf[pbuf_n + j++] = pair;
        }
      }
    }
    if (!direct) pbuf_n += (uint32_t)total;
  }
  // the table is not read by the emission: clear it for the next batch
  for (uint32_t x = threadIdx.x; x < ts; x += NTH) s_tab[x] = 0;
  __syncthreads();  // the next batch rewrites the LDS
  return false;
}

// The next batch of a workgroup's segment range starting at segment v:
// consecutive non-empty segments while they fit in CAP elements (returns 1).
// A segment of CAP < size <= 2 CAP is returned alone (returns 2) to be
// grouped in two halves by one more hash bit; a larger one is listed in
// big[] (the second pass hands it on to the sort-and-runs path) and skipped.
// Returns 0 when the range
// is exhausted.
template <int CAP>
__device__ __forceinline__ int next_batch(const uint32_t* __restrict__ seg_start,
                                          const uint32_t* __restrict__ seg_end, uint32_t& v,
                                          uint32_t v1, uint32_t& a, uint32_t& b, bool can_split,
                                          uint64_t* __restrict__ big,
                                          unsigned long long* __restrict__ nbig) {
  while (v < v1) {
    a = seg_start[v];
    b = seg_end[v];
    if (a == b) {
      ++v;
      continue;
    }
    if (b - a > (uint32_t)CAP) {
      ++v;
      if (can_split && b - a <= 2u * CAP) return 2;
      if (threadIdx.x == 0) {
        const unsigned long long x = atomicAdd(nbig, 1ull);
        big[2 * x] = a;
        big[2 * x + 1] = b;
      }
      continue;
    }
    uint32_t w = v + 1;
    while (w < v1) {
      const uint32_t a2 = seg_start[w], b2 = seg_end[w];
      if (a2 != b2) {
        if (b2 - a > (uint32_t)CAP) break;
        b = b2;
      }
      ++w;
    }
    v = w;
    return 1;
  }
  return 0;
}

// Count (part < 0) or stably compact into s_e (part 0 or 1) the elements of
// [a, b), b - a <= 2 CAP, whose hash bit `bit` equals part; thread t takes a
// contiguous chunk so the compaction keeps the segment's order. Returns the
// number of elements with the bit set (count) or compacted (part).
template <int CAP, int NTH>
__device__ uint32_t split_part(const uint64_t* __restrict__ E, uint32_t a, uint32_t b,
                               uint32_t bit, int part, uint64_t* s_e, uint64_t* s_tmp64) {
  const uint32_t n = b - a;
  const uint32_t chunk = (n + NTH - 1) / NTH;
  const uint32_t c0 = min(threadIdx.x * chunk, n), c1 = min(c0 + chunk, n);
  const uint32_t want = part < 0 ? 1u : (uint32_t)part;
  uint64_t mine = 0;
  for (uint32_t x = c0; x < c1; ++x) mine += ((E[a + x] >> bit) & 1u) == want;
  uint64_t total;
  uint64_t pos = block_excl_scan<NTH>(mine, s_tmp64, &total);
  if (part >= 0) {
    for (uint32_t x = c0; x < c1; ++x) {
      const uint64_t e = E[a + x];
      if (((e >> bit) & 1u) == want) s_e[pos++] = e;
    }
  }
  __syncthreads();
  return (uint32_t)total;
}

// One workgroup per `spw` consecutive segment values, processed as batches;
// the elements of batch t + 1 are loaded into registers while batch t is
// grouped. WPE is the occupancy the register allocation aims at (waves per
// SIMD; 1 leaves it to the compiler).
template <int CAP, int NTH, int WPE>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(WPE))) void k_group_seg(
    const uint64_t* __restrict__ E, const uint32_t* __restrict__ seg_start,
    const uint32_t* __restrict__ seg_end, uint32_t nseg, uint32_t spw, uint32_t idbits,
    uint32_t splitbit, ShardOut out, uint64_t* __restrict__ big,
    unsigned long long* __restrict__ nbig) {
  constexpr int PER = CAP / NTH;
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ uint64_t s_tmp64[NTH / 64];
  __shared__ uint64_t s_base[2];
  __shared__ uint64_t s_pbuf[GROUP_PBUF];
  uint32_t pbuf_n = 0;
  constexpr uint32_t MC = CAP / 2;
  uint64_t* s_e = reinterpret_cast<uint64_t*>(lds);
  uint32_t* s_tab = reinterpret_cast<uint32_t*>(lds + MC * 8);
  // group_batch expects a zero table area
  for (uint32_t x = threadIdx.x; x < 2 * MC; x += NTH) s_tab[x] = 0;
  __syncthreads();
  const bool can_split = splitbit >= idbits && splitbit < 64;
  const uint32_t v0 = blockIdx.x * spw;
  const uint32_t v1 = min(v0 + spw, nseg);
  uint32_t v = v0, a = 0, b = 0;
  int kind = next_batch<CAP>(seg_start, seg_end, v, v1, a, b, can_split, big, nbig);
  uint64_t cur[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const uint32_t x = threadIdx.x + r * NTH;
    cur[r] = (kind == 1 && x < b - a) ? E[a + x] : 0;
  }
  while (kind) {
    if (kind == 2) {
      // a segment of up to 2 CAP elements: equal hashes share every bit, so
      // the halves by the next hash bit are grouped one after the other
      const uint32_t ones = split_part<CAP, NTH>(E, a, b, splitbit, -1, s_e, s_tmp64);
      const uint32_t zeros = (b - a) - ones;
      if (ones > (uint32_t)CAP || zeros > (uint32_t)CAP) {
        if (threadIdx.x == 0) {
          const unsigned long long x = atomicAdd(nbig, 1ull);
          big[2 * x] = a;
          big[2 * x + 1] = b;
        }
      } else {
        for (int part = 0; part < 2; ++part) {
          const uint32_t m = split_part<CAP, NTH>(E, a, b, splitbit, part, s_e, s_tmp64);
          uint64_t e[PER];
#pragma unroll
          for (int r = 0; r < PER; ++r) {
            const uint32_t x = threadIdx.x + r * NTH;
            e[r] = x < m ? s_e[x] : 0;
          }
          __syncthreads();
          // the staging overwrote the table area
          for (uint32_t x = threadIdx.x; x < 2 * MC; x += NTH) s_tab[x] = 0;
          __syncthreads();
          // a listed half lists the whole segment: the other half must not
          // list it again
          if (group_batch<CAP, NTH>(e, m, idbits, out, lds, s_tmp64, s_base, s_pbuf, pbuf_n, a, b,
                                    big, nbig))
            break;
        }
      }
      kind = next_batch<CAP>(seg_start, seg_end, v, v1, a, b, can_split, big, nbig);
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const uint32_t x = threadIdx.x + r * NTH;
        cur[r] = (kind == 1 && x < b - a) ? E[a + x] : 0;
      }
      continue;
    }
    const uint32_t m = b - a;
    uint32_t na = 0, nb = 0;
    const int nkind = next_batch<CAP>(seg_start, seg_end, v, v1, na, nb, can_split, big, nbig);
    uint64_t nxt[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const uint32_t x = threadIdx.x + r * NTH;
      nxt[r] = (nkind == 1 && x < nb - na) ? E[na + x] : 0;
    }
    group_batch<CAP, NTH>(cur, m, idbits, out, lds, s_tmp64, s_base, s_pbuf, pbuf_n, a, b, big,
                          nbig);
#pragma unroll
    for (int r = 0; r < PER; ++r) cur[r] = nxt[r];
    a = na;
    b = nb;
    kind = nkind;
  }
  if (pbuf_n) flush_pairs<NTH>(out, s_pbuf, pbuf_n, s_base);
}

// Second pass over the ranges k_group_seg listed, big[0, 2 *nlisted): batches
// with more than CAP / 2 prefilter candidates, segments with such a split
// half, and segments over 2 CAP elements. Each workgroup takes ranges in turn
// with a table for a whole batch of candidates (MC = CAP, twice the LDS of
// the main kernel, so fewer workgroups fit on a CU; few ranges come here).
// The count is read from device memory, so the launch follows k_group_seg's
// with no host round trip and writes into the same sharded output; a count
// over max_listed (which the listing cannot reach) is clamped to it.
// A range over CAP elements is split by one more hash bit, as in k_group_seg;
// a range that still does not fit is listed in big2[] for the sort-and-runs
// path.
template <int CAP, int NTH>
__global__ __launch_bounds__(NTH) void k_group_listed(
    const uint64_t* __restrict__ E, const uint64_t* __restrict__ big,
    const unsigned long long* __restrict__ nlisted_p, uint64_t max_listed, uint32_t idbits,
    uint32_t splitbit, ShardOut out, uint64_t* __restrict__ big2,
    unsigned long long* __restrict__ nbig2) {
  constexpr int PER = CAP / NTH;
  const uint64_t nlisted = min((uint64_t)*nlisted_p, max_listed);
  if (blockIdx.x >= nlisted) return;
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ uint64_t s_tmp64[NTH / 64];
  __shared__ uint64_t s_base[2];
  __shared__ uint64_t s_pbuf[GROUP_PBUF];
  uint32_t pbuf_n = 0;
  uint64_t* s_e = reinterpret_cast<uint64_t*>(lds);
  uint32_t* s_tab = reinterpret_cast<uint32_t*>(lds + CAP * 8);
  // group_batch expects a zero table area; it leaves it zero, and the
  // staging of a split half ([0, 8 CAP)) does not reach it
  for (uint32_t x = threadIdx.x; x < 2u * CAP; x += NTH) s_tab[x] = 0;
  __syncthreads();
  const bool can_split = splitbit >= idbits && splitbit < 64;
  for (uint64_t g = blockIdx.x; g < nlisted; g += gridDim.x) {
    const uint32_t a = (uint32_t)big[2 * g], b = (uint32_t)big[2 * g + 1];
    const uint32_t n = b - a;
    if (n <= (uint32_t)CAP) {
      uint64_t e[PER];
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const uint32_t x = threadIdx.x + r * NTH;
        e[r] = x < n ? E[a + x] : 0;
      }
      group_batch<CAP, NTH, CAP>(e, n, idbits, out, lds, s_tmp64, s_base, s_pbuf, pbuf_n, a, b,
                                 big2, nbig2);
      continue;
    }
    bool whole = !can_split || n > 2u * CAP;
    if (!whole) {
      const uint32_t ones = split_part<CAP, NTH>(E, a, b, splitbit, -1, s_e, s_tmp64);
      whole = ones > (uint32_t)CAP || n - ones > (uint32_t)CAP;
    }
    if (whole) {
      if (threadIdx.x == 0) {
        const unsigned long long x = atomicAdd(nbig2, 1ull);
        big2[2 * x] = a;
        big2[2 * x + 1] = b;
      }
      continue;
    }
    for (int part = 0; part < 2; ++part) {
      const uint32_t m = split_part<CAP, NTH>(E, a, b, splitbit, part, s_e, s_tmp64);
      uint64_t e[PER];
#pragma unroll
      for (int r = 0; r < PER; ++r) {
        const uint32_t x = threadIdx.x + r * NTH;
        e[r] = x < m ? s_e[x] : 0;
      }
      __syncthreads();  // group_batch rewrites s_e
      group_batch<CAP, NTH, CAP>(e, m, idbits, out, lds, s_tmp64, s_base, s_pbuf, pbuf_n, a, b,
                                 big2, nbig2);
    }
  }
  if (pbuf_n) flush_pairs<NTH>(out, s_pbuf, pbuf_n, s_base);
}

// ------------------------------------------------------------------ oversized segments

// Listed segments [big[2s], big[2s+1]) are copied contiguously from
// out_off[s].
__global__ __launch_bounds__(256) void k_gather_big(const uint64_t* __restrict__ E,
                                                    const uint64_t* __restrict__ big,
                                                    const uint64_t* __restrict__ out_off,
                                                    uint32_t nseg, uint64_t* __restrict__ out) {
  for (uint32_t s = blockIdx.y; s < nseg; s += gridDim.y) {
    const uint64_t a = big[2 * s], b = big[2 * s + 1], o = out_off[s];
    for (uint64_t p = a + (uint64_t)blockIdx.x * 256 + threadIdx.x; p < b;
         p += (uint64_t)gridDim.x * 256)
      out[o + (p - a)] = E[p];
  }
}

// In an array sorted stably by the full hash (ids ascend inside a run of
// equal hashes), the first occurrence of each id pairs with every later
// distinct id of its run. Appends after a per-block reservation on *counter;
// writes past cap are dropped but still counted.
__global__ __launch_bounds__(256) void k_emit_hash_runs(const uint64_t* __restrict__ E,
                                                        uint64_t n, uint32_t idbits,
                                                        uint64_t* __restrict__ cand, uint64_t cap,
                                                        unsigned long long* __restrict__ counter) {
  __shared__ uint64_t s_tmp[4];
  __shared__ uint64_t s_base;
  const uint64_t idmask = (1ull << idbits) - 1;
  const uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  bool first = p < n;
  if (first && p > 0) first = E[p] != E[p - 1];
  uint64_t cnt = 0;
  if (first) {
    const uint64_t h = E[p] >> idbits;
    for (uint64_t q = p + 1; q < n && (E[q] >> idbits) == h; ++q) cnt += E[q] != E[q - 1];
  }
  uint64_t total;
  const uint64_t excl = block_excl_scan<256>(cnt, s_tmp, &total);
  if (threadIdx.x == 0) s_base = total ? atomicAdd(counter, (unsigned long long)total) : 0;
  __syncthreads();
  if (cnt) {
    uint64_t pos = s_base + excl;
    const uint64_t h = E[p] >> idbits;
    const uint64_t ip = E[p] & idmask;
    for (uint64_t q = p + 1; q < n && (E[q] >> idbits) == h; ++q) {
      if (E[q] != E[q - 1]) {
        // (lo, hi): ids ascend inside a run when every listed range is a
        // contiguous piece of the sorted array listed once (the grouping
        // kernel never lists a range twice); the order is kept explicitly
        const uint64_t iq = E[q] & idmask;
        if (pos < cap) cand[pos] = ip < iq ? (ip << 32) | iq : (iq << 32) | ip;
        ++pos;
      }
    }
  }
}

// ------------------------------------------------------------------ paired chains
//
// Paired-chain records (Discussion: the CDR3s of both chains of a receptor
// joined by a token that is never deleted). A record (a, b) is the joined
// string a T b of length La + 1 + Lb <= 49; its variants delete at most k of
// the La + Lb residue positions and keep T, so two records within
// Lev(a) + Lev(b) <= k share a variant (delete per chain as in the
// single-chain argument). Variants are hashed like single chains (the same
// rotation hash over the joined string, T as residue code 20) and written
// with multiplicity at the record's offsets: a repeated variant of one record
// only repeats a candidate, which the pair sort drops.
constexpr uint32_t PAIR_TOKEN_CODE = 20;
constexpr int PV_RECORDS = 64;  // records per generator workgroup

__device__ __forceinline__ uint64_t choose2(uint64_t x) { return x * (x - 1) / 2; }
__device__ __forceinline__ uint64_t choose3(uint64_t x) { return x * (x - 1) * (x - 2) / 6; }

// Deletion sets of up to k of the D deletable positions, with multiplicity:
// sum_{m <= k} C(D, m).
__device__ __forceinline__ uint32_t paired_num_variants(uint32_t D, int k) {
  uint32_t v = 1;
  if (k >= 1) v += D;
  if (k >= 2 && D >= 2) v += (uint32_t)choose2(D);
  if (k >= 3 && D >= 3) v += (uint32_t)choose3(D);
  return v;
}

__global__ __launch_bounds__(256) void k_paired_count(const u128* __restrict__ sa,
                                                      const u128* __restrict__ sb, uint64_t n,
                                                      int k, uint32_t* __restrict__ vcnt) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) vcnt[i] = paired_num_variants(key_len(sa[i]) + key_len(sb[i]), k);
}

// The largest x with choose2(x) <= u (colexicographic unranking of a pair).
__device__ __forceinline__ uint32_t colex2_top(uint64_t u) {
  uint32_t x = (uint32_t)((1.0 + sqrt(1.0 + 8.0 * (double)u)) * 0.5);
  while (x > 1 && choose2(x) > u) --x;
  while (choose2(x + 1) <= u) ++x;
  return x;
}

__device__ __forceinline__ uint32_t colex3_top(uint64_t u) {
  uint32_t x = (uint32_t)cbrt(6.0 * (double)u) + 1;
  while (x > 2 && choose3(x) > u) --x;
  while (choose3(x + 1) <= u) ++x;
  return x;
}

// One thread per variant slot of the workgroup's records: unrank the
// deletion set (none, one, pairs, then triples, each in colexicographic
// order over the deletable positions), map deletable index x to joined
// position x (< La) or x + 1, and hash the remaining joined string.
__global__ __launch_bounds__(256) void k_vargen_paired(const u128* __restrict__ sa,
                                                       const u128* __restrict__ sb,
                                                       const uint64_t* __restrict__ voff,
                                                       uint64_t n, int k, uint32_t idbits,
                                                       uint64_t* __restrict__ elem) {
  __shared__ uint64_t s_off[PV_RECORDS + 1];
  __shared__ u128 s_a[PV_RECORDS], s_b[PV_RECORDS];
  __shared__ uint64_t s_hb[32], s_hc[64];
  const uint64_t r0 = (uint64_t)blockIdx.x * PV_RECORDS;
  const uint32_t nr = (uint32_t)min<uint64_t>(PV_RECORDS, n - r0);
  for (uint32_t x = threadIdx.x; x <= nr; x += 256) s_off[x] = voff[r0 + x];
  for (uint32_t x = threadIdx.x; x < nr; x += 256) {
    s_a[x] = sa[r0 + x];
    s_b[x] = sb[r0 + x];
  }
  if (threadIdx.x < 32) s_hb[threadIdx.x] = kHashTab.b[threadIdx.x];
  if (threadIdx.x < 64) s_hc[threadIdx.x] = kHashTab.c[threadIdx.x];
  __syncthreads();
  const uint64_t idmask = (1ull << idbits) - 1;
  const uint64_t g0 = s_off[0], g1 = s_off[nr];
  for (uint64_t g = g0 + threadIdx.x; g < g1; g += 256) {
    uint32_t lo = 0, hi = nr - 1;  // the last record with s_off[x] <= g
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= g)
        lo = mid;
      else
        hi = mid - 1;
    }
    const u128 a = s_a[lo], b = s_b[lo];
    const uint32_t la = key_len(a), lb = key_len(b), D = la + lb;
    uint64_t v = g - s_off[lo];
    uint32_t del[3] = {64, 64, 64};  // deletable indices, ascending
    uint32_t m = 0;
    if (v == 0) {
      m = 0;
    } else if (v <= D) {
      m = 1;
      del[0] = (uint32_t)(v - 1);
    } else if (v <= D + choose2(D)) {
      m = 2;
      const uint64_t u = v - 1 - D;
      del[1] = colex2_top(u);
      del[0] = (uint32_t)(u - choose2(del[1]));
    } else {
      m = 3;
      const uint64_t u = v - 1 - D - choose2(D);
      del[2] = colex3_top(u);
      const uint64_t r = u - choose3(del[2]);
      del[1] = colex2_top(r);
      del[0] = (uint32_t)(r - choose2(del[1]));
    }
    uint64_t gone = 0;  // joined positions deleted
    for (uint32_t q = 0; q < m; ++q) gone |= 1ull << (del[q] < la ? del[q] : del[q] + 1);
    uint64_t h = s_hc[la + lb + 1 - m];
    uint32_t j = 0;
    for (uint32_t t = 0; t <= D; ++t) {
      if ((gone >> t) & 1u) continue;
      const uint32_t r = t < la ? key_residue(a, (int)t)
                                : t == la ? PAIR_TOKEN_CODE : key_residue(b, (int)(t - la - 1));
      h ^= __builtin_rotateright64(s_hb[r], j);
      ++j;
    }
    elem[g] = (h & ~idmask) | (r0 + lo);
  }
}

}  // namespace sdk

namespace sd {

void launch_vargen_hash(const u128* seq, const uint64_t* voff, uint64_t nseq, int k, bool distinct,
                        uint64_t* elem, uint32_t idbits, int npass, const uint32_t* shifts,
                        const uint32_t* masks, uint32_t* hist, uint32_t* tcounts,
                        uint32_t seqs_per_block, hipStream_t s, uint32_t ftile) {
  if (!nseq) return;
  if (seqs_per_block < 1 || seqs_per_block > (uint32_t)sdk::VG_SEQS)
    throw Error{SD_E_INVAL, "internal error: sequences per generator block out of range"};
  sdk::PassDigits pd;
  for (int q = 0; q < 3; ++q) {
    pd.shift[q] = q < npass ? shifts[q] : 0;
    pd.mask[q] = q < npass ? masks[q] : 0;
  }
  const unsigned g = (unsigned)((nseq + seqs_per_block - 1) / seqs_per_block);
  if (k > 3) throw Error{SD_E_INVAL, "internal error: at most three deletions"};
  uint32_t* tc = npass ? tcounts : nullptr;
  const ShardOut none{nullptr, 0, nullptr, 0, nullptr};
  if (distinct && k == 3)
    hipLaunchKernelGGL((sdk::k_vargen_hash<true, true, 0>), dim3(g), dim3(sdk::VG_NT), 0, s, seq,
                       voff, nseq, k, elem, idbits, npass, pd, hist, tc, seqs_per_block, none, 0u,
                       0u, ftile);
  else if (distinct)
    hipLaunchKernelGGL((sdk::k_vargen_hash<true, false, 0>), dim3(g), dim3(sdk::VG_NT), 0, s, seq,
                       voff, nseq, k, elem, idbits, npass, pd, hist, tc, seqs_per_block, none, 0u,
                       0u, ftile);
  else if (k == 3)
    hipLaunchKernelGGL((sdk::k_vargen_hash<false, true, 0>), dim3(g), dim3(sdk::VG_NT), 0, s, seq,
                       voff, nseq, k, elem, idbits, npass, pd, hist, tc, seqs_per_block, none, 0u,
                       0u, ftile);
  else
    hipLaunchKernelGGL((sdk::k_vargen_hash<false, false, 0>), dim3(g), dim3(sdk::VG_NT), 0, s,
                       seq, voff, nseq, k, elem, idbits, npass, pd, hist, tc, seqs_per_block, none,
                       0u, 0u, ftile);
}

void launch_vargen_bins(const u128* seq, const uint64_t* voff, uint64_t nseq, int k,
                        uint32_t idbits, uint32_t* hist, uint32_t seqs_per_block, hipStream_t s) {
  if (!nseq) return;
  if (seqs_per_block < 1 || seqs_per_block > (uint32_t)sdk::VG_SEQS || k > 3)
    throw Error{SD_E_INVAL, "internal error: generator shape out of range"};
  sdk::PassDigits pd{};
  pd.shift[0] = 64 - STREAM_BIN_BITS;
  pd.mask[0] = (1u << STREAM_BIN_BITS) - 1u;
  const unsigned g = (unsigned)((nseq + seqs_per_block - 1) / seqs_per_block);
  const ShardOut none{nullptr, 0, nullptr, 0, nullptr};
  if (k == 3)
    hipLaunchKernelGGL((sdk::k_vargen_hash<true, true, 1>), dim3(g), dim3(sdk::VG_NT), 0, s, seq,
                       voff, nseq, k, nullptr, idbits, 1, pd, hist, nullptr, seqs_per_block, none,
                       0u, 0u, 0u);
  else
    hipLaunchKernelGGL((sdk::k_vargen_hash<true, false, 1>), dim3(g), dim3(sdk::VG_NT), 0, s, seq,
                       voff, nseq, k, nullptr, idbits, 1, pd, hist, nullptr, seqs_per_block, none,
                       0u, 0u, 0u);
}

void launch_paired_count(const u128* sa, const u128* sb, uint64_t n, int k, uint32_t* vcnt,
                         hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_paired_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sa,
                     sb, n, k, vcnt);
}

void launch_vargen_paired(const u128* sa, const u128* sb, const uint64_t* voff, uint64_t n, int k,
                          uint32_t idbits, uint64_t* elem, hipStream_t s) {
  if (!n) return;
  if (k > 3) throw Error{SD_E_INVAL, "internal error: at most three deletions"};
  const unsigned g = (unsigned)((n + sdk::PV_RECORDS - 1) / sdk::PV_RECORDS);
  hipLaunchKernelGGL(sdk::k_vargen_paired, dim3(g), dim3(256), 0, s, sa, sb, voff, n, k, idbits,
                     elem);
}

void launch_vargen_stream(const u128* seq, const uint64_t* voff, uint64_t nseq, int k,
                          uint32_t idbits, uint32_t blo, uint32_t bhi, const ShardArgs& a,
                          uint32_t seqs_per_block, hipStream_t s) {
  if (!nseq) return;
  if (seqs_per_block < 1 || seqs_per_block > (uint32_t)sdk::VG_SEQS || k > 3)
    throw Error{SD_E_INVAL, "internal error: generator shape out of range"};
  const sdk::PassDigits pd{};
  const unsigned g = (unsigned)((nseq + seqs_per_block - 1) / seqs_per_block);
  const ShardOut out{a.base, a.region, a.over, a.over_cap, a.counter};
  if (k == 3)
    hipLaunchKernelGGL((sdk::k_vargen_hash<true, true, 2>), dim3(g), dim3(sdk::VG_NT), 0, s, seq,
                       voff, nseq, k, nullptr, idbits, 0, pd, nullptr, nullptr, seqs_per_block, out,
                       blo, bhi, 0u);
  else
    hipLaunchKernelGGL((sdk::k_vargen_hash<true, false, 2>), dim3(g), dim3(sdk::VG_NT), 0, s, seq,
                       voff, nseq, k, nullptr, idbits, 0, pd, nullptr, nullptr, seqs_per_block, out,
                       blo, bhi, 0u);
}

void launch_hist_rows(const uint32_t* tcounts, uint64_t nseq, uint32_t seqs_per_block, int npass,
                      uint32_t* hist, hipStream_t s) {
  if (!nseq || !tcounts || npass < 2) return;
  const unsigned g = (unsigned)((nseq + seqs_per_block - 1) / seqs_per_block);
  hipLaunchKernelGGL(sdk::k_hist_rows, dim3(std::min(128u, g), npass - 1), dim3(256), 0, s, tcounts,
                     g, hist);
}

void launch_seg_bounds(const uint64_t* E, uint64_t n, uint32_t segshift, uint32_t* seg_start,
                       uint32_t* seg_end, hipStream_t s) {
  const uint32_t nseg = segshift >= 64 ? 1u : (1u << (64u - segshift));
  const uint32_t g = (nseg + 1 + 255) / 256;
  hipLaunchKernelGGL(sdk::k_seg_bounds, dim3(g), dim3(256), 0, s, E, (uint32_t)n, segshift, nseg,
                     seg_start, seg_end);
}

static size_t group_lds(int cap) { return (size_t)(cap / 2) * sdk::GROUP_LDS_PER_CAND; }

template <int CAP, int NTH, int WPE>
static void launch_group_t(const uint64_t* E, const uint32_t* ss, const uint32_t* se,
                           uint32_t nseg, uint32_t spw, uint32_t idbits, uint32_t splitbit,
                           const ShardArgs& a, uint64_t* big, unsigned long long* nbig,
                           hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    attr = true;
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&sdk::k_group_seg<CAP, NTH, WPE>),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)group_lds(CAP)) != hipSuccess)
      (void)hipGetLastError();  // the launch reports any real problem
  }
  const unsigned g = (nseg + spw - 1) / spw;
  const ShardOut out{a.base, a.region, a.over, a.over_cap, a.counter};
  hipLaunchKernelGGL((sdk::k_group_seg<CAP, NTH, WPE>), dim3(g), dim3(NTH), group_lds(CAP), s, E, ss,
                     se, nseg, spw, idbits, splitbit, out, big, nbig);
}

static size_t listed_lds(int cap) { return (size_t)cap * sdk::GROUP_LDS_PER_CAND; }

template <int CAP, int NTH>
static void launch_listed_t(const uint64_t* E, const uint64_t* big,
                            const unsigned long long* nlisted, uint64_t max_listed,
                            uint32_t idbits, uint32_t splitbit, const ShardArgs& a, uint64_t* big2,
                            unsigned long long* nbig2, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    attr = true;
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&sdk::k_group_listed<CAP, NTH>),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)listed_lds(CAP)) != hipSuccess)
      (void)hipGetLastError();  // the launch reports any real problem
  }
  // a few workgroups per CU; each takes listed ranges in turn
  const unsigned g = (unsigned)std::min<uint64_t>(max_listed, 1024u);
  const ShardOut out{a.base, a.region, a.over, a.over_cap, a.counter};
  hipLaunchKernelGGL((sdk::k_group_listed<CAP, NTH>), dim3(g), dim3(NTH), listed_lds(CAP), s, E,
                     big, nlisted, max_listed, idbits, splitbit, out, big2, nbig2);
}

void launch_group_listed(int cap, const uint64_t* E, const uint64_t* big,
                         const unsigned long long* nlisted, uint64_t max_listed, uint32_t idbits,
                         uint32_t splitbit, const ShardArgs& out, uint64_t* big2,
                         unsigned long long* nbig2, hipStream_t s) {
  if (!max_listed) return;
  switch (cap) {
    case 4096:
      launch_listed_t<4096, 512>(E, big, nlisted, max_listed, idbits, splitbit, out, big2, nbig2, s);
      break;
    case 2048:
      launch_listed_t<2048, 256>(E, big, nlisted, max_listed, idbits, splitbit, out, big2, nbig2, s);
      break;
    case 1024:
      launch_listed_t<1024, 128>(E, big, nlisted, max_listed, idbits, splitbit, out, big2, nbig2, s);
      break;
    default:
      launch_listed_t<256, 64>(E, big, nlisted, max_listed, idbits, splitbit, out, big2, nbig2, s);
      break;
  }
}

bool group_cap_supported(int cap) { return cap == 4096 || cap == 2048 || cap == 1024 || cap == 256; }

void launch_group_seg(int cap, int shape, const uint64_t* E, const uint32_t* seg_start,
                      const uint32_t* seg_end, uint32_t nseg, uint32_t spw, uint32_t idbits,
                      uint32_t splitbit, const ShardArgs& out, uint64_t* big,
                      unsigned long long* nbig, hipStream_t s) {
  if (!nseg) return;
  switch (cap) {
    case 4096:
      launch_group_t<4096, 512, 1>(E, seg_start, seg_end, nseg, spw, idbits, splitbit, out, big,
                                   nbig, s);
      break;
    case 2048:
      if (shape == 1)  // 256 threads, registers for four waves per SIMD (no spills)
        launch_group_t<2048, 256, 4>(E, seg_start, seg_end, nseg, spw, idbits, splitbit, out, big,
                                     nbig, s);
      else if (shape == 2)  // 512 threads, four elements per thread
        launch_group_t<2048, 512, 4>(E, seg_start, seg_end, nseg, spw, idbits, splitbit, out, big,
                                     nbig, s);
      else  // 256 threads, registers for five waves per SIMD
        launch_group_t<2048, 256, 5>(E, seg_start, seg_end, nseg, spw, idbits, splitbit, out, big,
                                     nbig, s);
      break;
    case 1024:
      launch_group_t<1024, 128, 1>(E, seg_start, seg_end, nseg, spw, idbits, splitbit, out, big,
                                   nbig, s);
      break;
    default:
      launch_group_t<256, 64, 1>(E, seg_start, seg_end, nseg, spw, idbits, splitbit, out, big,
                                 nbig, s);
      break;
  }
}

void launch_gather_big(const uint64_t* E, const uint64_t* big, const uint64_t* out_off,
                       uint32_t nseg, uint64_t* out, hipStream_t s) {
  if (!nseg) return;
  hipLaunchKernelGGL(sdk::k_gather_big, dim3(64, nseg < 4096 ? nseg : 4096), dim3(256), 0, s, E,
                     big, out_off, nseg, out);
}

void launch_emit_hash_runs(const uint64_t* E, uint64_t n, uint32_t idbits, uint64_t* cand,
                           uint64_t cap, unsigned long long* counter, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_emit_hash_runs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, E,
                     n, idbits, cand, cap, counter);
}

}  // namespace sd
