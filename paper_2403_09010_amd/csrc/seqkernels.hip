// Sequence-side kernels of the symdel library for gfx950:
//   k_pack            compress CSR residue codes into exact 128-bit keys
//                     (Appendix A XTNeighbor step 1, "compress")
//   k_vargen          every deletion variant with <= k deletions as a key and
//                     its source id (steps 2-3, the one-to-many "expand")
//   k_emit_runs       groups of equal keys in a sorted key array -> id pairs
//                     (steps 4-5, "uniqueCount" + "expand")
//   k_verify_compact  drop repeated candidates, keep pairs with Levenshtein
//                     distance <= k (or, in Hamming mode, equal lengths and
//                     Hamming distance <= k), compact in order (steps 6-7)
//   k_pair_distance   Levenshtein distance of given pairs
#include "sd_device.h"
#include "sd_internal.h"

namespace sdk {

constexpr int NT = 256;

// ------------------------------------------------------------------ Levenshtein
//
// Bit-parallel edit distance (Myers 1999, in the global-distance form of
// Hyyro 2001): the pattern a (m <= 24 residues) lives in one 32-bit word, the
// text b is consumed one residue per step, and the score tracks the last row
// of the dynamic programme. Bits above m-1 carry junk that never reaches the
// low m bits (only shifts left and carries move bits, and they move upward).
__device__ __forceinline__ uint32_t lev_keys(u128 a, u128 b) {
  const uint32_t m = key_len(a), n = key_len(b);
  if (m == 0) return n;
  if (n == 0) return m;
  uint32_t ares[KEY_MAX_LEN];
#pragma unroll
  for (int t = 0; t < KEY_MAX_LEN; ++t) ares[t] = (uint32_t)t < m ? key_residue(a, t) : 31u;
  uint32_t pv = (1u << m) - 1u, mv = 0u, score = m;
  const uint32_t top = 1u << (m - 1);
  u128 text = b;
  for (uint32_t j = 0; j < n; ++j) {
    const uint32_t c = (uint32_t)(text >> 115) & 31u;
    text <<= 5;
    uint32_t eq = 0;
#pragma unroll
    for (int t = 0; t < KEY_MAX_LEN; ++t) eq |= (ares[t] == c ? 1u : 0u) << t;
    const uint32_t xv = eq | mv;
    const uint32_t xh = (((eq & pv) + pv) ^ pv) | eq;
    uint32_t ph = mv | ~(xh | pv);
    uint32_t mh = pv & xh;
    if (ph & top)
      ++score;
    else if (mh & top)
      --score;
    ph = (ph << 1) | 1u;
    mh = mh << 1;
    pv = mh | ~(xv | ph);
    mv = ph & xv;
  }
  return score;
}

// The same distance with the pattern as bit planes: plane b (bits [24 b,
// 24 b + 24) of pa) holds bit b of every residue of a, the length is in bits
// 127..120. The positions of a that match the text residue c are then
// ~OR_b (plane_b ^ (bit b of c ? all ones : 0)), a few bit operations per
// text residue instead of one comparison per pattern position.
__device__ __forceinline__ uint32_t lev_planes(u128 pa, u128 b) {
  const uint32_t m = (uint32_t)(pa >> 120), n = key_len(b);
  if (m == 0) return n;
  if (n == 0) return m;
  const uint64_t lo = (uint64_t)pa, hi = (uint64_t)(pa >> 64);
  const uint32_t P0 = (uint32_t)lo & 0xFFFFFFu, P1 = (uint32_t)(lo >> 24) & 0xFFFFFFu;
  const uint32_t P2 = (uint32_t)((lo >> 48) | (hi << 16)) & 0xFFFFFFu;
  const uint32_t P3 = (uint32_t)(hi >> 8) & 0xFFFFFFu, P4 = (uint32_t)(hi >> 32) & 0xFFFFFFu;
  const uint32_t mmask = (1u << m) - 1u;
  uint32_t pv = mmask, mv = 0u, score = m;
  const uint32_t top = 1u << (m - 1);
  uint64_t th = (uint64_t)(b >> 64), tl = (uint64_t)b;  // residue j at bits 115 - 5j .. 119 - 5j
  for (uint32_t j = 0; j < n; ++j) {
    const uint32_t c = (uint32_t)(th >> 51) & 31u;
    th = (th << 5) | (tl >> 59);
    tl <<= 5;
    const uint32_t x = (P0 ^ (0u - (c & 1u))) | (P1 ^ (0u - ((c >> 1) & 1u))) |
                       (P2 ^ (0u - ((c >> 2) & 1u))) | (P3 ^ (0u - ((c >> 3) & 1u))) |
                       (P4 ^ (0u - ((c >> 4) & 1u)));
    const uint32_t eq = ~x & mmask;
    const uint32_t xv = eq | mv;
    const uint32_t xh = (((eq & pv) + pv) ^ pv) | eq;
    uint32_t ph = mv | ~(xh | pv);
    uint32_t mh = pv & xh;
    if (ph & top)
      ++score;
    else if (mh & top)
      --score;
    ph = (ph << 1) | 1u;
    mh = mh << 1;
    pv = mh | ~(xv | ph);
    mv = ph & xv;
  }
  return score;
}

// Hamming distance of two packed keys of equal length (Section III C's
// filter): residues sit in 5-bit fields at bits [5 g, 5 g + 5), so a field of
// a XOR b is non-zero exactly where the residues differ; OR-ing each field's
// five bits into its lowest bit and counting those bits gives the distance.
// Fields past the length are zero in both keys.
__device__ __forceinline__ uint32_t hamming_keys(u128 a, u128 b) {
  constexpr uint64_t LOW = 0x0084210842108421ull;  // bits 0, 5, 10, ..., 55
  const u128 x = a ^ b;
  const uint64_t lo = (uint64_t)x & ((1ull << 60) - 1ull);         // fields 0..11
  const uint64_t hi = (uint64_t)(x >> 60) & ((1ull << 60) - 1ull);  // fields 12..23
  const uint64_t flo = (lo | (lo >> 1) | (lo >> 2) | (lo >> 3) | (lo >> 4)) & LOW;
  const uint64_t fhi = (hi | (hi >> 1) | (hi >> 2) | (hi >> 3) | (hi >> 4)) & LOW;
  return (uint32_t)(__popcll(flo) + __popcll(fhi));
}

// ------------------------------------------------------------------ pack

__global__ __launch_bounds__(NT) void k_pack(const uint8_t* __restrict__ codes,
                                             const int64_t* __restrict__ offs, uint64_t n, int k,
                                             int distinct, u128* __restrict__ seq,
                                             u128* __restrict__ planes,
                                             uint32_t* __restrict__ vcnt,
                                             uint32_t* __restrict__ err) {
  const uint64_t i = (uint64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const int64_t a = offs[i], b = offs[i + 1];
  const int64_t L = b - a;
  if (L < 1 || L > KEY_MAX_LEN) {
    atomicOr(err, SD_ERRBIT_LENGTH);
    seq[i] = 0;
    if (planes) planes[i] = 0;
    if (vcnt) vcnt[i] = 0;
    return;
  }
  u128 key = (u128)L << 120;
  uint32_t pl[5] = {0, 0, 0, 0, 0};
  bool bad = false;
  for (int t = 0; t < (int)L; ++t) {
    const uint32_t c = codes[a + t];
    bad |= c >= 20u;
    key |= (u128)(c & 31u) << (115 - 5 * t);
#pragma unroll
    for (int q = 0; q < 5; ++q) pl[q] |= ((c >> q) & 1u) << t;
  }
  if (bad) atomicOr(err, SD_ERRBIT_ALPHABET);
  seq[i] = key;
  if (planes) {
    const uint64_t lo = (uint64_t)pl[0] | ((uint64_t)pl[1] << 24) | ((uint64_t)pl[2] << 48);
    const uint64_t hi = ((uint64_t)pl[2] >> 16) | ((uint64_t)pl[3] << 8) | ((uint64_t)pl[4] << 32) |
                        ((uint64_t)L << 56);
    planes[i] = ((u128)hi << 64) | lo;
  }
  if (vcnt) {
    uint32_t c = num_variants((uint32_t)L, k);
    if (distinct) {
      uint32_t n1, n2;
      canonical_masks(pl, (uint32_t)L, n1, n2);
      c = num_distinct_variants(n1, n2, (uint32_t)L, k);
      if (k >= 3) c += num_distinct_triples(n1, n2, canonical_mask3(pl, (uint32_t)L), (uint32_t)L);
    }
    vcnt[i] = c;
  }
}

// ------------------------------------------------------------------ vargen

constexpr int VG_SEQS = 64;  // sequences per block

__global__ __launch_bounds__(NT) void k_vargen(const u128* __restrict__ seq,
                                               const uint64_t* __restrict__ voff, uint64_t nseq,
                                               uint64_t* __restrict__ key_lo,
                                               uint64_t* __restrict__ key_hi,
                                               uint32_t* __restrict__ id) {
  __shared__ uint64_t s_off[VG_SEQS + 1];
  __shared__ u128 s_seq[VG_SEQS];
  const uint64_t s0 = (uint64_t)blockIdx.x * VG_SEQS;
  const uint32_t ns = (uint32_t)min<uint64_t>(VG_SEQS, nseq - s0);
  for (uint32_t x = threadIdx.x; x <= ns; x += NT) s_off[x] = voff[s0 + x];
  for (uint32_t x = threadIdx.x; x < ns; x += NT) s_seq[x] = seq[s0 + x];
  __syncthreads();
  const uint64_t g0 = s_off[0], g1 = s_off[ns];
  for (uint64_t g = g0 + threadIdx.x; g < g1; g += NT) {
    uint32_t lo = 0, hi = ns - 1;  // last x with s_off[x] <= g
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= g)
        lo = mid;
      else
        hi = mid - 1;
    }
    const u128 key = key_variant(s_seq[lo], (uint32_t)(g - s_off[lo]));
    key_lo[g] = (uint64_t)key;
    key_hi[g] = (uint64_t)(key >> 64);
    id[g] = (uint32_t)(s0 + lo);
  }
}

// ------------------------------------------------------------------ group emission

__device__ __forceinline__ bool same_key(const uint64_t* lo, const uint64_t* hi, uint64_t x,
                                         uint64_t y) {
  return lo[x] == lo[y] && hi[x] == hi[y];
}

// In a key-sorted array (stable, so ids ascend inside a group), the first
// occurrence of each id pairs with every later distinct id of its group.
// Candidates (i << 32 | j), i < j, are appended after a per-block reservation
// on *counter; writes past cap are dropped but still counted.
__global__ __launch_bounds__(NT) void k_emit_runs(const uint64_t* __restrict__ klo,
                                                  const uint64_t* __restrict__ khi,
                                                  const uint32_t* __restrict__ id, uint64_t n,
                                                  uint64_t* __restrict__ cand, uint64_t cap,
                                                  unsigned long long* __restrict__ counter) {
  __shared__ uint64_t s_tmp[NT / 64];
  __shared__ uint64_t s_base;
  const uint64_t p = (uint64_t)blockIdx.x * NT + threadIdx.x;
  bool first = p < n;
  if (first && p > 0) first = !(same_key(klo, khi, p, p - 1) && id[p] == id[p - 1]);
  uint64_t cnt = 0;
  if (first) {
    for (uint64_t q = p + 1; q < n && same_key(klo, khi, q, p); ++q) cnt += id[q] != id[q - 1];
  }
  uint64_t total;
  const uint64_t excl = block_excl_scan<NT>(cnt, s_tmp, &total);
  if (threadIdx.x == 0) s_base = total ? atomicAdd(counter, (unsigned long long)total) : 0;
  __syncthreads();
  if (cnt) {
    uint64_t pos = s_base + excl;
    const uint64_t ip = (uint64_t)id[p] << 32;
    for (uint64_t q = p + 1; q < n && same_key(klo, khi, q, p); ++q) {
      if (id[q] != id[q - 1]) {
        if (pos < cap) cand[pos] = ip | id[q];
        ++pos;
      }
    }
  }
}

// ------------------------------------------------------------------ verify

constexpr int CITEMS = 8;
constexpr uint8_t DROP = 0xFFu;  // verdict of a pair over k

// The final filter of one candidate pair (i, j): its distance, or DROP.
// MODE 0: pa holds the bit-plane form of the first sequences (pack's planes)
// and the distance is Levenshtein; MODE 1: pa holds their packed keys and the
// distance is Hamming over equal lengths; MODE 2 (paired-chain records): pa
// and sb are the first chains (planes, keys), pa2 and sb2 the second, and the
// distance is the sum of the two chains' Levenshtein distances. The length
// difference bounds each distance from below and skips most far pairs.
template <int MODE>
__device__ __forceinline__ uint8_t pair_verdict(const u128* __restrict__ pa,
                                                const u128* __restrict__ sb,
                                                const u128* __restrict__ pa2,
                                                const u128* __restrict__ sb2, uint32_t i,
                                                uint32_t j, int k) {
  const u128 a = pa[i], b = sb[j];
  const int la = (int)(a >> 120), lb = (int)key_len(b);
  if (MODE == 1) {
    if (la == lb) {
      const uint32_t dd = hamming_keys(a, b);
      if (dd <= (uint32_t)k) return (uint8_t)dd;
    }
  } else if (MODE == 2) {
    const u128 a2 = pa2[i], b2 = sb2[j];
    const int la2 = (int)(a2 >> 120), lb2 = (int)key_len(b2);
    if (abs(la - lb) + abs(la2 - lb2) <= k) {
      const uint32_t d1 = lev_planes(a, b);
      if (d1 <= (uint32_t)k) {
        const uint32_t dd = d1 + lev_planes(a2, b2);
        if (dd <= (uint32_t)k) return (uint8_t)dd;
      }
    }
  } else if (abs(la - lb) <= k) {
    const uint32_t dd = lev_planes(a, b);
    if (dd <= (uint32_t)k) return (uint8_t)dd;
  }
  return DROP;
}

// A tile of NT * CITEMS sorted candidates per workgroup. Repeats (a candidate
// equal to its predecessor) are dropped first and the distinct candidates
// listed in LDS in order; the distances then run over that dense list, each
// thread taking a contiguous piece, so a wave does not run the distance once
// per candidate slot while most of its lanes hold repeats. Kept pairs are
// written in candidate order after a look-back over the tiles. MODE and the
// sequence arrays are those of pair_verdict.
template <int MODE>
__global__ __launch_bounds__(NT) void k_verify_compact(
    const uint64_t* __restrict__ cand, uint64_t c, uint32_t na, uint32_t nbseq,
    const u128* __restrict__ pa, const u128* __restrict__ sb, const u128* __restrict__ pa2,
    const u128* __restrict__ sb2, int k, int self_pairs, uint32_t* __restrict__ oi,
    uint32_t* __restrict__ oj, uint8_t* __restrict__ od, uint64_t* __restrict__ status,
    uint32_t* __restrict__ tile_counter, uint32_t epoch, unsigned long long* __restrict__ out_count,
    uint32_t* __restrict__ err) {
  constexpr int TILE = NT * CITEMS;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_tmp[NT / 64];
  __shared__ uint64_t s_excl;
  __shared__ uint64_t s_list[TILE];  // the tile's distinct candidates, in order
  __shared__ uint8_t s_dist[TILE];   // their distances, DROP if over k
  if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  if (tile >= gridDim.x) return;
  const uint64_t first = tile * TILE + (uint64_t)threadIdx.x * CITEMS;
  uint64_t vals[CITEMS];
  uint32_t umask = 0;
  uint64_t prev = first > 0 && first - 1 < c ? cand[first - 1] : ~0ull;
#pragma unroll
  for (int x = 0; x < CITEMS; ++x) {
    const uint64_t e = first + x;
    vals[x] = e < c ? cand[e] : 0;
    // a self search pairs i < j only (a candidate of one sequence with itself
    // can come from two of its variants that share a hash)
    const bool ordered = !self_pairs || (uint32_t)(vals[x] >> 32) < (uint32_t)vals[x];
    // ~0 marks an unused slot of a fixed-capacity candidate array (it sorts last)
    if (e < c && (e == 0 || vals[x] != prev) && ordered && vals[x] != ~0ull) umask |= 1u << x;
    prev = vals[x];
  }
  uint32_t ntot;
  uint32_t at = block_excl_scan<NT>((uint32_t)__popc(umask), s_tmp, &ntot);
#pragma unroll
  for (int x = 0; x < CITEMS; ++x)
    if ((umask >> x) & 1u) s_list[at++] = vals[x];
  __syncthreads();
  const uint32_t per = (ntot + NT - 1) / NT;
  const uint32_t l0 = min(threadIdx.x * per, ntot), l1 = min(l0 + per, ntot);
  uint32_t cnt = 0;
  for (uint32_t l = l0; l < l1; ++l) {
    const uint64_t v = s_list[l];
    const uint32_t i = (uint32_t)(v >> 32), j = (uint32_t)v;
    uint8_t d = DROP;
    if (i < na && j < nbseq)
      d = pair_verdict<MODE>(pa, sb, pa2, sb2, i, j, k);
    else  // an id out of range is an internal error: flagged, never read
      atomicOr(err, SD_ERRBIT_INDEX);
    s_dist[l] = d;  // read back below by this thread only
    cnt += d != DROP;
  }
  uint32_t total;
  const uint32_t texcl = block_excl_scan<NT>(cnt, s_tmp, &total);
  if (threadIdx.x == 0) s_excl = lb_exclusive(status, tile, 1, epoch, total, err);
  __syncthreads();
  uint64_t pos = s_excl + texcl;
  for (uint32_t l = l0; l < l1; ++l) {
    const uint8_t d = s_dist[l];
    if (d != DROP) {
      const uint64_t v = s_list[l];
      oi[pos] = (uint32_t)(v >> 32);
      oj[pos] = (uint32_t)v;
      od[pos] = d;
      ++pos;
    }
  }
  if (threadIdx.x == 0 && tile == gridDim.x - 1) *out_count = s_excl + total;
}

// ------------------------------------------------------------------ bucketed pair sort
//
// Steps 6-7 in one sort pass over HBM: candidates (i << 32 | j) are first
// scattered into buckets by the top B bits of i (counted per tile, one
// exclusive scan over the bucket-major count table, a scatter with LDS
// cursors); every bucket then fits one workgroup's LDS, where it is sorted,
// deduplicated and verified, and its kept pairs are written in order after a
// look-back over the buckets. Within a bucket the key (i's low bits, j)
// fits 32 bits. Buckets hold candidates of disjoint i ranges in increasing
// order, so the concatenation of the sorted buckets is the sorted array.

constexpr int PB_NT = 512;             // threads of the bucket kernels
constexpr int PB_NW = PB_NT / 64;
constexpr uint32_t PB_CHUNK = 16384;   // candidates per counting tile
constexpr uint32_t PB_MAX_BUCKETS = 4096;
constexpr uint32_t PB_CAP = 8192;      // largest bucket sorted in LDS

// cnt[b * ntiles + t] = candidates of tile t in bucket b (v >> shift)
__global__ __launch_bounds__(PB_NT) void k_bucket_count(const uint64_t* __restrict__ cand,
                                                        uint64_t nc, uint32_t shift, uint32_t nb,
                                                        uint32_t ntiles,
                                                        uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_h[PB_MAX_BUCKETS];
  for (uint32_t b = threadIdx.x; b < nb; b += PB_NT) s_h[b] = 0;
  __syncthreads();
  const uint64_t t = blockIdx.x;
  const uint64_t e0 = t * PB_CHUNK, e1 = min<uint64_t>(nc, e0 + PB_CHUNK);
  for (uint64_t e = e0 + threadIdx.x; e < e1; e += PB_NT) {
    const uint32_t b = (uint32_t)(cand[e] >> shift);
    if (b < nb) atomicAdd(&s_h[b], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += PB_NT) cnt[(uint64_t)b * ntiles + t] = s_h[b];
}

// out[off[b * ntiles + t] + rank] = the tile's candidates of bucket b (the
// order inside a bucket is not kept: the bucket is sorted afterwards)
__global__ __launch_bounds__(PB_NT) void k_bucket_scatter(const uint64_t* __restrict__ cand,
                                                          uint64_t nc, uint32_t shift, uint32_t nb,
                                                          uint32_t ntiles,
                                                          const uint64_t* __restrict__ off,
                                                          uint64_t* __restrict__ out) {
  __shared__ uint32_t s_at[PB_MAX_BUCKETS];
  const uint64_t t = blockIdx.x;
  for (uint32_t b = threadIdx.x; b < nb; b += PB_NT) s_at[b] = (uint32_t)off[(uint64_t)b * ntiles + t];
  __syncthreads();
  const uint64_t e0 = t * PB_CHUNK, e1 = min<uint64_t>(nc, e0 + PB_CHUNK);
  for (uint64_t e = e0 + threadIdx.x; e < e1; e += PB_NT) {
    const uint64_t v = cand[e];
    const uint32_t b = (uint32_t)(v >> shift);
    if (b < nb) out[atomicAdd(&s_at[b], 1u)] = v;
  }
}

// One stable LSD pass over 8 bits of n <= PB_CAP keys in LDS, src -> dst.
// Wave w ranks the 64-key chunks [w * cpw, (w + 1) * cpw) in order: lanes
// with equal digits find each other by ballots (match_digit8), the lowest of
// them adds the group to the wave's count of that digit, and the rank of a
// lane is the number of equal lanes below it. Counts are scanned digit-major,
// wave-minor, so the pass keeps the order of equal digits.
__device__ __forceinline__ void lds_radix_pass(const uint32_t* src, uint32_t* dst, uint32_t n,
                                               uint32_t shift, uint32_t* s_cnt, uint32_t* s_tmp) {
  const uint32_t lane = lane_id(), w = threadIdx.x / 64;
  const uint32_t chunks = (n + 63) / 64, cpw = (chunks + PB_NW - 1) / PB_NW;
  const uint32_t c0 = min(chunks, w * cpw), c1 = min(chunks, c0 + cpw);
  for (uint32_t x = threadIdx.x; x < PB_NW * 256; x += PB_NT) s_cnt[x] = 0;
  __syncthreads();
  uint32_t* mine = s_cnt + w * 256;
  for (uint32_t c = c0; c < c1; ++c) {
    const uint32_t x = c * 64 + lane;
    const bool valid = x < n;
    const uint32_t d = valid ? (src[x] >> shift) & 255u : 0u;
    const uint64_t peers = match_digit8(d, __ballot(valid));
    if (valid && mask_rank(peers) == 0) mine[d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: exclusive over the waves, then over the digits
  uint32_t tot = 0;
  if (threadIdx.x < 256) {
    for (int v = 0; v < PB_NW; ++v) {
      const uint32_t cv = s_cnt[v * 256 + threadIdx.x];
      s_cnt[v * 256 + threadIdx.x] = tot;
      tot += cv;
    }
  }
  uint32_t all;
  const uint32_t base = block_excl_scan<PB_NT>(tot, s_tmp, &all);
  if (threadIdx.x < 256)
    for (int v = 0; v < PB_NW; ++v) s_cnt[v * 256 + threadIdx.x] += base;
  __syncthreads();
  for (uint32_t c = c0; c < c1; ++c) {
    const uint32_t x = c * 64 + lane;
    const bool valid = x < n;
    const uint32_t key = valid ? src[x] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    const uint64_t peers = match_digit8(d, __ballot(valid));
    const uint32_t rank = mask_rank(peers);
    const uint32_t at = mine[d];
    if (valid) dst[at + rank] = key;
    if (valid && rank == 0) mine[d] = at + (uint32_t)__popcll(peers);
  }
  __syncthreads();
}

// Bucket by bucket, independently: load the bucket's candidates as 32-bit
// keys (i's low `low` bits above j's `jb` bits), sort them, drop repeats
// (and, for a self search, pairs with i >= j), verify the rest
// (pair_verdict) and write the kept pairs, packed as key << 8 | distance, in
// order at the start of the bucket's range of `packed`; bcount[b] = their
// number. The bucketed candidates are only read, so the host can still sort
// them the other way if a bucket is left out. k_bucket_place then moves every bucket's pairs to its place in the
// output. No bucket waits for another, so a large one costs only its own
// time.
// A bucket of up to PB_CAP candidates is sorted in LDS. A larger one (the
// candidates of a cluster of near-equal sequences, which repeat once per
// shared variant) is split by the next 12 key bits into sub-buckets: one
// count, a scan and a scatter into the bucket's range of `scratch`, then
// consecutive sub-buckets are grouped into runs of at most PB_CAP and each
// run is sorted and verified in LDS like a small bucket; its sorted keys go
// back in place and its verdicts to the second half of that range until the
// bucket's pairs are written. A
// bucket over PB_BIG candidates, or with a sub-bucket over PB_CAP / 2, is
// left out: it sets SD_ERRBIT_BUCKET in *err and counts as empty, and the
// host sorts and verifies the whole array the other way.
constexpr uint32_t PB_BIG = 1u << 18;
constexpr uint32_t PB_SUB_BITS = 12;
constexpr uint32_t PB_GROUP = PB_CAP / 2;  // group starts are PB_GROUP apart
constexpr uint32_t PB_MAXG = PB_BIG / PB_GROUP;
constexpr uint32_t PB_WCHUNK = PB_NT * 8;  // positions per write round of a large bucket

// Sort n <= PB_CAP keys in LDS (LSD passes over `bits` bits); returns the
// buffer that holds them.
__device__ __forceinline__ uint32_t* lds_sort(uint32_t* a, uint32_t* b, uint32_t n, uint32_t bits,
                                              uint32_t* s_cnt, uint32_t* s_tmp) {
  for (uint32_t sh = 0; sh < bits; sh += 8) {
    lds_radix_pass(a, b, n, sh, s_cnt, s_tmp);
    uint32_t* q = a;
    a = b;
    b = q;
  }
  return a;
}

template <int MODE>
__global__ __launch_bounds__(PB_NT) void k_bucket_verify(
    const uint64_t* __restrict__ cand, uint64_t* __restrict__ scratch,
    uint64_t* __restrict__ packed, const uint64_t* __restrict__ off, uint32_t ntiles, uint32_t nb,
    uint32_t jb, uint32_t low, uint32_t na, uint32_t nbseq, const u128* __restrict__ pa,
    const u128* __restrict__ sb, const u128* __restrict__ pa2, const u128* __restrict__ sb2, int k,
    int self_pairs, uint32_t* __restrict__ bcount, uint32_t* __restrict__ err) {
  __shared__ uint32_t s_a[PB_CAP];
  __shared__ uint32_t s_b[PB_CAP];
  __shared__ uint32_t s_cnt[PB_NW * 256];
  __shared__ uint32_t s_tmp[PB_NW];
  __shared__ uint32_t s_grp[PB_MAXG + 1];
  __shared__ uint32_t s_bad;
  const uint32_t t = blockIdx.x;
  const uint64_t b0 = off[(uint64_t)t * ntiles], b1 = off[(uint64_t)(t + 1) * ntiles];
  const uint32_t m = (uint32_t)min<uint64_t>(b1 - b0, (uint64_t)PB_BIG + 1);
  const uint32_t jmask = jb >= 32 ? ~0u : (1u << jb) - 1u;
  const uint32_t lmask = (1u << low) - 1u;
  const uint32_t ibase = t << low;
  const uint32_t kbits = low + jb;
  auto first_of = [&](uint32_t key) { return ibase | (key >> jb); };
  auto key_of = [&](uint64_t v) {
    return ((((uint32_t)(v >> 32)) & lmask) << jb) | ((uint32_t)v & jmask);
  };
  auto keep_of = [&](const uint32_t* keys, uint32_t x) {
    const uint32_t key = keys[x];
    return (x == 0 || keys[x - 1] != key) && (!self_pairs || first_of(key) < (key & jmask));
  };
  uint64_t* __restrict__ outp = packed + b0;  // packed pairs, in order
  // the verdict of a listed pair (an id out of range is an internal error:
  // flagged, never read)
  auto verdict_of = [&](uint32_t key) -> uint8_t {
    const uint32_t i = first_of(key), j = key & jmask;
    if (i >= na || j >= nbseq) {
      atomicOr(err, SD_ERRBIT_INDEX);
      return DROP;
    }
    return pair_verdict<MODE>(pa, sb, pa2, sb2, i, j, k);
  };
  if (m > PB_BIG) {
    if (threadIdx.x == 0) {
      atomicOr(err, SD_ERRBIT_BUCKET);
      bcount[t] = 0;
    }
    return;
  }
  if (m <= PB_CAP) {
    // (a separate code path, so that it addresses LDS directly)
    for (uint32_t x = threadIdx.x; x < m; x += PB_NT) s_a[x] = key_of(cand[b0 + x]);
    __syncthreads();
    uint32_t* src = lds_sort(s_a, s_b, m, kbits, s_cnt, s_tmp);
    uint32_t* dst = src == s_a ? s_b : s_a;
    // distinct ordered pairs, listed in order in the other buffer
    const uint32_t per = (m + PB_NT - 1) / PB_NT;
    const uint32_t x0 = min(threadIdx.x * per, m), x1 = min(x0 + per, m);
    uint32_t keep = 0;
    for (uint32_t x = x0; x < x1; ++x) keep += keep_of(src, x);
    uint32_t ntot;
    uint32_t at = block_excl_scan<PB_NT>(keep, s_tmp, &ntot);
    for (uint32_t x = x0; x < x1; ++x)
      if (keep_of(src, x)) dst[at++] = src[x];
    __syncthreads();
    uint8_t* s_dist = reinterpret_cast<uint8_t*>(src);  // (where the sorted keys were)
    const uint32_t per2 = (ntot + PB_NT - 1) / PB_NT;
    const uint32_t l0 = min(threadIdx.x * per2, ntot), l1 = min(l0 + per2, ntot);
    uint32_t cnt = 0;
    for (uint32_t l = l0; l < l1; ++l) {
      const uint8_t d = verdict_of(dst[l]);
      s_dist[l] = d;  // read back below by this thread only
      cnt += d != DROP;
    }
    uint32_t total;
    uint32_t pos = block_excl_scan<PB_NT>(cnt, s_tmp, &total);
    for (uint32_t l = l0; l < l1; ++l)
      if (s_dist[l] != DROP) outp[pos++] = ((uint64_t)dst[l] << 8) | s_dist[l];
    if (threadIdx.x == 0) bcount[t] = total;
    return;
  }
  // large bucket: sub-bucket counts (kept in s_b while grouping and scattering)
  const uint32_t sbits = min(PB_SUB_BITS, kbits), ssh = kbits - sbits, nsub = 1u << sbits;
  uint32_t* starts = s_b;
  for (uint32_t x = threadIdx.x; x < nsub; x += PB_NT) starts[x] = 0;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  for (uint32_t x = threadIdx.x; x < m; x += PB_NT) atomicAdd(&starts[key_of(cand[b0 + x]) >> ssh], 1u);
  __syncthreads();
  {
    // exclusive scan, eight entries a thread; a sub-bucket over PB_CAP -
    // PB_GROUP cannot be grouped
    constexpr uint32_t PER = (1u << PB_SUB_BITS) / PB_NT;
    const uint32_t e0 = threadIdx.x * PER;
    uint32_t v[PER], sum = 0, big = 0;
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q) {
      v[q] = e0 + q < nsub ? starts[e0 + q] : 0u;
      big |= v[q] > PB_CAP - PB_GROUP;
      sum += v[q];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan<PB_NT>(sum, s_tmp, &tot);
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q)
      if (e0 + q < nsub) {
        starts[e0 + q] = run;
        run += v[q];
      }
    if (big) s_bad = 1;
  }
  __syncthreads();
  if (s_bad) {
    if (threadIdx.x == 0) {
      atomicOr(err, SD_ERRBIT_BUCKET);
      bcount[t] = 0;
    }
    return;
  }
  // group g: the sub-buckets that start in [g PB_GROUP, (g + 1) PB_GROUP),
  // at most PB_GROUP + (PB_CAP - PB_GROUP) candidates
  const uint32_t ng = (m + PB_GROUP - 1) / PB_GROUP;
  for (uint32_t g = threadIdx.x; g <= ng; g += PB_NT) {
    uint32_t lo = 0, hi = nsub;  // first sub-bucket starting at or after g PB_GROUP
    while (lo < hi) {
      const uint32_t mid = (lo + hi) / 2;
      if (starts[mid] < g * PB_GROUP)
        lo = mid + 1;
      else
        hi = mid;
    }
    s_grp[g] = g == ng || lo == nsub ? m : starts[lo];
  }
  __syncthreads();
  // scatter by sub-bucket into scratch (the order inside a sub-bucket is not kept)
  uint32_t* A = reinterpret_cast<uint32_t*>(scratch + b0);
  for (uint32_t x = threadIdx.x; x < m; x += PB_NT) {
    const uint32_t key = key_of(cand[b0 + x]);
    A[atomicAdd(&starts[key >> ssh], 1u)] = key;
  }
  __syncthreads();
  // per group: sort and verify in LDS; the sorted keys go back in place in
  // A (after the whole group is in LDS), the verdicts after A
  uint32_t* S = A;
  uint8_t* V = reinterpret_cast<uint8_t*>(A + m);
  uint32_t total = 0;
  for (uint32_t g = 0; g < ng; ++g) {
    const uint32_t lo = s_grp[g], n = s_grp[g + 1] - lo;
    if (n == 0) continue;
    for (uint32_t x = threadIdx.x; x < n; x += PB_NT) s_a[x] = A[lo + x];
    __syncthreads();
    const uint32_t* src = lds_sort(s_a, s_b, n, kbits, s_cnt, s_tmp);
    uint32_t cnt = 0;
    for (uint32_t x = threadIdx.x; x < n; x += PB_NT) {
      const uint32_t key = src[x];
      uint8_t d = DROP;
      if (keep_of(src, x)) d = verdict_of(key);
      S[lo + x] = key;
      V[lo + x] = d;
      cnt += d != DROP;
    }
    uint32_t gt;
    (void)block_excl_scan<PB_NT>(cnt, s_tmp, &gt);
    total += gt;
  }
  __syncthreads();
  // the kept pairs in order, PB_WCHUNK positions a round, 8 a thread
  uint32_t base = 0;
  for (uint32_t c0 = 0; c0 < m; c0 += PB_WCHUNK) {
    const uint32_t x0 = min(c0 + threadIdx.x * 8u, m), x1 = min(x0 + 8u, m);
    uint32_t cnt = 0;
    for (uint32_t x = x0; x < x1; ++x) cnt += V[x] != DROP;
    uint32_t round;
    uint32_t pos = base + block_excl_scan<PB_NT>(cnt, s_tmp, &round);
    for (uint32_t x = x0; x < x1; ++x)
      if (V[x] != DROP) outp[pos++] = ((uint64_t)S[x] << 8) | V[x];
    base += round;
  }
  if (threadIdx.x == 0) bcount[t] = total;
}

// Every bucket's packed pairs to their place (bpos, the exclusive scan of
// the bucket counts) in the output arrays; *out_count = the total.
__global__ __launch_bounds__(PB_NT) void k_bucket_place(
    const uint64_t* __restrict__ packed, const uint64_t* __restrict__ off, uint32_t ntiles,
    uint32_t nb, uint32_t jb, uint32_t low, const uint32_t* __restrict__ bcount,
    const uint64_t* __restrict__ bpos, uint32_t* __restrict__ oi, uint32_t* __restrict__ oj,
    uint8_t* __restrict__ od, unsigned long long* __restrict__ out_count) {
  const uint32_t jmask = jb >= 32 ? ~0u : (1u << jb) - 1u;
  for (uint32_t t = blockIdx.x; t < nb; t += gridDim.x) {
    const uint64_t* src = packed + off[(uint64_t)t * ntiles];
    const uint32_t cnt = bcount[t];
    const uint64_t pos = bpos[t];
    const uint32_t ibase = t << low;
    for (uint32_t r = threadIdx.x; r < cnt; r += PB_NT) {
      const uint64_t v = src[r];
      const uint32_t key = (uint32_t)(v >> 8);
      oi[pos + r] = ibase | (key >> jb);
      oj[pos + r] = key & jmask;
      od[pos + r] = (uint8_t)v;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *out_count = bpos[nb];
}

__global__ __launch_bounds__(NT) void k_join_pairs(const uint32_t* __restrict__ i,
                                                   const uint32_t* __restrict__ j, uint64_t n,
                                                   uint64_t* __restrict__ out) {
  const uint64_t t = (uint64_t)blockIdx.x * NT + threadIdx.x;
  if (t < n) out[t] = ((uint64_t)i[t] << 32) | j[t];
}

__global__ __launch_bounds__(NT) void k_pair_distance(const u128* __restrict__ sa, uint64_t na,
                                                      const u128* __restrict__ sb, uint64_t nb,
                                                      const uint32_t* __restrict__ ia,
                                                      const uint32_t* __restrict__ ib, uint64_t n,
                                                      uint8_t* __restrict__ d,
                                                      uint32_t* __restrict__ err) {
  const uint64_t t = (uint64_t)blockIdx.x * NT + threadIdx.x;
  if (t >= n) return;
  const uint32_t x = ia[t], y = ib[t];
  if (x >= na || y >= nb) {  // out-of-range pair: flag it, read nothing
    atomicOr(err, SD_ERRBIT_INDEX);
    d[t] = 255;
    return;
  }
  const uint32_t v = lev_keys(sa[x], sb[y]);
  d[t] = (uint8_t)(v > 255u ? 255u : v);
}

}  // namespace sdk

namespace sd {

static unsigned blocks_for(uint64_t n, uint64_t per) { return (unsigned)((n + per - 1) / per); }

void launch_pack(const uint8_t* codes, const int64_t* offs, uint64_t n, int k, bool distinct,
                 u128* seq, u128* planes, uint32_t* vcnt, uint32_t* err, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_pack, dim3(blocks_for(n, sdk::NT)), dim3(sdk::NT), 0, s, codes, offs,
                     n, k, distinct ? 1 : 0, seq, planes, vcnt, err);
}

void launch_vargen(const u128* seq, const uint64_t* voff, uint64_t nseq, int k, uint64_t* key_lo,
                   uint64_t* key_hi, uint32_t* id, hipStream_t s) {
  (void)k;
  if (!nseq) return;
  hipLaunchKernelGGL(sdk::k_vargen, dim3(blocks_for(nseq, sdk::VG_SEQS)), dim3(sdk::NT), 0, s,
                     seq, voff, nseq, key_lo, key_hi, id);
}

void launch_emit_runs(const uint64_t* key_lo, const uint64_t* key_hi, const uint32_t* id,
                      uint64_t n, uint64_t* cand, uint64_t cap, unsigned long long* counter,
                      hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_emit_runs, dim3(blocks_for(n, sdk::NT)), dim3(sdk::NT), 0, s, key_lo,
                     key_hi, id, n, cand, cap, counter);
}

uint64_t compact_tile() { return (uint64_t)sdk::NT * sdk::CITEMS; }

uint32_t bucket_chunk() { return sdk::PB_CHUNK; }
uint32_t bucket_cap() { return sdk::PB_CAP; }
uint32_t bucket_max() { return sdk::PB_MAX_BUCKETS; }

void launch_bucket_count(const uint64_t* cand, uint64_t nc, uint32_t shift, uint32_t nb,
                         uint32_t* cnt, hipStream_t s) {
  if (!nc) return;
  const uint32_t nt = blocks_for(nc, sdk::PB_CHUNK);
  hipLaunchKernelGGL(sdk::k_bucket_count, dim3(nt), dim3(sdk::PB_NT), 0, s, cand, nc, shift, nb,
                     nt, cnt);
}

void launch_bucket_scatter(const uint64_t* cand, uint64_t nc, uint32_t shift, uint32_t nb,
                           const uint64_t* off, uint64_t* out, hipStream_t s) {
  if (!nc) return;
  const uint32_t nt = blocks_for(nc, sdk::PB_CHUNK);
  hipLaunchKernelGGL(sdk::k_bucket_scatter, dim3(nt), dim3(sdk::PB_NT), 0, s, cand, nc, shift, nb,
                     nt, off, out);
}

void launch_bucket_verify(const uint64_t* cand, uint64_t* scratch, uint64_t* packed,
                          const uint64_t* off, uint64_t nc, uint32_t nb, uint32_t jb, uint32_t low,
                          uint64_t na, uint64_t nbseq, const u128* a, const u128* seq_b, int k,
                          int metric, int self_pairs, uint32_t* bcount, uint32_t* err,
                          hipStream_t s, const u128* a2, const u128* seq_b2) {
  if (!nc) return;
  const uint32_t nt = blocks_for(nc, sdk::PB_CHUNK);
  const uint32_t na32 = (uint32_t)std::min<uint64_t>(na, 0xFFFFFFFFull);
  const uint32_t nb32 = (uint32_t)std::min<uint64_t>(nbseq, 0xFFFFFFFFull);
  if (a2)
    hipLaunchKernelGGL(sdk::k_bucket_verify<2>, dim3(nb), dim3(sdk::PB_NT), 0, s, cand, scratch,
                       packed, off, nt, nb, jb, low, na32, nb32, a, seq_b, a2, seq_b2, k,
                       self_pairs, bcount, err);
  else if (metric == SD_METRIC_HAMMING)
    hipLaunchKernelGGL(sdk::k_bucket_verify<1>, dim3(nb), dim3(sdk::PB_NT), 0, s, cand, scratch,
                       packed, off, nt, nb, jb, low, na32, nb32, a, seq_b, nullptr, nullptr, k,
                       self_pairs, bcount, err);
  else
    hipLaunchKernelGGL(sdk::k_bucket_verify<0>, dim3(nb), dim3(sdk::PB_NT), 0, s, cand, scratch,
                       packed, off, nt, nb, jb, low, na32, nb32, a, seq_b, nullptr, nullptr, k,
                       self_pairs, bcount, err);
}

void launch_bucket_place(const uint64_t* packed, const uint64_t* off, uint64_t nc, uint32_t nb,
                         uint32_t jb, uint32_t low, const uint32_t* bcount, const uint64_t* bpos,
                         uint32_t* out_i, uint32_t* out_j, uint8_t* out_d,
                         unsigned long long* out_count, hipStream_t s) {
  if (!nc) return;
  const uint32_t nt = blocks_for(nc, sdk::PB_CHUNK);
  hipLaunchKernelGGL(sdk::k_bucket_place, dim3(std::min<uint32_t>(nb, 2048)), dim3(sdk::PB_NT), 0,
                     s, packed, off, nt, nb, jb, low, bcount, bpos, out_i, out_j, out_d, out_count);
}

void launch_join_pairs(const uint32_t* i, const uint32_t* j, uint64_t n, uint64_t* out,
                       hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_join_pairs, dim3(blocks_for(n, sdk::NT)), dim3(sdk::NT), 0, s, i, j, n,
                     out);
}

void launch_verify_compact(const uint64_t* cand, uint64_t c, uint64_t na, uint64_t nbseq,
                           const u128* a, const u128* seq_b, int k, int metric, int self_pairs,
                           uint32_t* out_i, uint32_t* out_j, uint8_t* out_d, uint64_t* status,
                           uint32_t* tile_counter, uint32_t epoch, unsigned long long* out_count,
                           uint32_t* err, hipStream_t s, const u128* a2, const u128* seq_b2) {
  if (!c) return;
  const dim3 g(blocks_for(c, compact_tile()));
  const uint32_t na32 = (uint32_t)std::min<uint64_t>(na, 0xFFFFFFFFull);
  const uint32_t nb32 = (uint32_t)std::min<uint64_t>(nbseq, 0xFFFFFFFFull);
  if (a2)
    hipLaunchKernelGGL(sdk::k_verify_compact<2>, g, dim3(sdk::NT), 0, s, cand, c, na32, nb32, a,
                       seq_b, a2, seq_b2, k, self_pairs, out_i, out_j, out_d, status, tile_counter,
                       epoch, out_count, err);
  else if (metric == SD_METRIC_HAMMING)
    hipLaunchKernelGGL(sdk::k_verify_compact<1>, g, dim3(sdk::NT), 0, s, cand, c, na32, nb32, a,
                       seq_b, nullptr, nullptr, k, self_pairs, out_i, out_j, out_d, status,
                       tile_counter, epoch, out_count, err);
  else
    hipLaunchKernelGGL(sdk::k_verify_compact<0>, g, dim3(sdk::NT), 0, s, cand, c, na32, nb32, a,
                       seq_b, nullptr, nullptr, k, self_pairs, out_i, out_j, out_d, status,
                       tile_counter, epoch, out_count, err);
}

void launch_pair_distance(const u128* seq_a, uint64_t na, const u128* seq_b, uint64_t nb,
                          const uint32_t* ia, const uint32_t* ib, uint64_t n, uint8_t* d,
                          uint32_t* err, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_pair_distance, dim3(blocks_for(n, sdk::NT)), dim3(sdk::NT), 0, s,
                     seq_a, na, seq_b, nb, ia, ib, n, d, err);
}

}  // namespace sd
