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

// A tile of NT * CITEMS sorted candidates per workgroup. Repeats (a candidate
// equal to its predecessor) are dropped first and the distinct candidates
// listed in LDS in order; the distances then run over that dense list, each
// thread taking a contiguous piece, so a wave does not run the distance once
// per candidate slot while most of its lanes hold repeats. Kept pairs are
// written in candidate order after a look-back over the tiles.
// MODE 0: pa holds the bit-plane form of the first sequences (pack's planes)
// and the distance is Levenshtein; MODE 1: pa holds their packed keys and the
// distance is Hamming over equal lengths; MODE 2 (paired-chain records): pa
// and sb are the first chains (planes, keys), pa2 and sb2 the second, and the
// distance is the sum of the two chains' Levenshtein distances.
template <int MODE>
__global__ __launch_bounds__(NT) void k_verify_compact(
    const uint64_t* __restrict__ cand, uint64_t c, const u128* __restrict__ pa,
    const u128* __restrict__ sb, const u128* __restrict__ pa2, const u128* __restrict__ sb2,
    int k, int self_pairs, uint32_t* __restrict__ oi,
    uint32_t* __restrict__ oj, uint8_t* __restrict__ od, uint64_t* __restrict__ status,
    uint32_t* __restrict__ tile_counter, uint32_t epoch, unsigned long long* __restrict__ out_count,
    uint32_t* __restrict__ err) {
  constexpr int TILE = NT * CITEMS;
  constexpr uint8_t DROP = 0xFFu;
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
    if (e < c && (e == 0 || vals[x] != prev) && ordered) umask |= 1u << x;
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
    const u128 a = pa[v >> 32], b = sb[(uint32_t)v];
    const int la = (int)(a >> 120), lb = (int)key_len(b);
    uint8_t d = DROP;
    if (MODE == 1) {
      if (la == lb) {
        const uint32_t dd = hamming_keys(a, b);
        if (dd <= (uint32_t)k) d = (uint8_t)dd;
      }
    } else if (MODE == 2) {
      const u128 a2 = pa2[v >> 32], b2 = sb2[(uint32_t)v];
      const int la2 = (int)(a2 >> 120), lb2 = (int)key_len(b2);
      if (abs(la - lb) + abs(la2 - lb2) <= k) {
        const uint32_t d1 = lev_planes(a, b);
        if (d1 <= (uint32_t)k) {
          const uint32_t dd = d1 + lev_planes(a2, b2);
          if (dd <= (uint32_t)k) d = (uint8_t)dd;
        }
      }
    } else if (abs(la - lb) <= k) {
      const uint32_t dd = lev_planes(a, b);
      if (dd <= (uint32_t)k) d = (uint8_t)dd;
    }
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

void launch_join_pairs(const uint32_t* i, const uint32_t* j, uint64_t n, uint64_t* out,
                       hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_join_pairs, dim3(blocks_for(n, sdk::NT)), dim3(sdk::NT), 0, s, i, j, n,
                     out);
}

void launch_verify_compact(const uint64_t* cand, uint64_t c, const u128* a, const u128* seq_b,
                           int k, int metric, int self_pairs, uint32_t* out_i, uint32_t* out_j,
                           uint8_t* out_d, uint64_t* status, uint32_t* tile_counter, uint32_t epoch,
                           unsigned long long* out_count, uint32_t* err, hipStream_t s,
                           const u128* a2, const u128* seq_b2) {
  if (!c) return;
  const dim3 g(blocks_for(c, compact_tile()));
  if (a2)
    hipLaunchKernelGGL(sdk::k_verify_compact<2>, g, dim3(sdk::NT), 0, s, cand, c, a, seq_b, a2,
                       seq_b2, k, self_pairs, out_i, out_j, out_d, status, tile_counter, epoch,
                       out_count, err);
  else if (metric == SD_METRIC_HAMMING)
    hipLaunchKernelGGL(sdk::k_verify_compact<1>, g, dim3(sdk::NT), 0, s, cand, c, a, seq_b,
                       nullptr, nullptr, k, self_pairs, out_i, out_j, out_d, status, tile_counter,
                       epoch, out_count, err);
  else
    hipLaunchKernelGGL(sdk::k_verify_compact<0>, g, dim3(sdk::NT), 0, s, cand, c, a, seq_b,
                       nullptr, nullptr, k, self_pairs, out_i, out_j, out_d, status, tile_counter,
                       epoch, out_count, err);
}

void launch_pair_distance(const u128* seq_a, uint64_t na, const u128* seq_b, uint64_t nb,
                          const uint32_t* ia, const uint32_t* ib, uint64_t n, uint8_t* d,
                          uint32_t* err, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_pair_distance, dim3(blocks_for(n, sdk::NT)), dim3(sdk::NT), 0, s,
                     seq_a, na, seq_b, nb, ia, ib, n, d, err);
}

}  // namespace sd
