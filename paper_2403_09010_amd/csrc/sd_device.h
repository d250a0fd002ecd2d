// Device-side helpers shared by the HIP kernels of the symdel library:
// the exact 128-bit variant key, wave64 primitives and the decoupled
// look-back status words.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned __int128 u128;

// ------------------------------------------------------------------ keys
//
// A sequence or deletion variant of length L <= 24 is one 128-bit integer:
// bits 127..120 hold L, residue t occupies bits [115 - 5t, 119 - 5t]
// (residues most significant first), unused low bits are zero. The packing
// is injective, so equal keys are equal strings (the paper's compression of
// a CDR3 into 12 bytes at 5 bits per residue, Appendix A, widened to 24
// residues and a length field so that no two strings share a key).
constexpr int KEY_FIELD_BITS = 120;
constexpr int KEY_MAX_LEN = 24;

__device__ __forceinline__ u128 u128_one() { return (u128)1; }

__device__ __forceinline__ uint32_t key_len(u128 key) { return (uint32_t)(key >> 120); }

__device__ __forceinline__ uint32_t key_residue(u128 key, int t) {
  return (uint32_t)(key >> (115 - 5 * t)) & 31u;
}

// The key of the string with position p removed (0 <= p < L).
__device__ __forceinline__ u128 key_delete(u128 key, int p) {
  const uint32_t L = key_len(key);
  const u128 field = key & ((u128_one() << KEY_FIELD_BITS) - 1);
  const u128 above = field & ~((u128_one() << (120 - 5 * p)) - 1);
  const u128 below = field & ((u128_one() << (115 - 5 * p)) - 1);
  return ((u128)(L - 1) << 120) | above | (below << 5);
}

// Number of deletion variants with at most k deleted positions, counted
// with multiplicity: sum_{m <= min(k, L)} C(L, m) (Section II A).
__host__ __device__ __forceinline__ uint32_t num_variants(uint32_t L, int k) {
  uint32_t v = 1;
  if (k >= 1 && L >= 1) v += L;
  if (k >= 2 && L >= 2) v += L * (L - 1) / 2;
  if (k >= 3 && L >= 3) v += L * (L - 1) * (L - 2) / 6;
  return v;
}

// Equal strings from different deletion sets. Deleting D from s gives t;
// the greedy leftmost embedding of t in s (match each position of s to the
// next character of t whenever they agree) deletes a unique set D*(t), so
// keeping only the variants with D = D* keeps each distinct string once. For
// |D| <= 2 the test is local: with t_j the j-th character of t,
//   {p}       is D*  iff p = L - 1 or s[p] != s[p + 1]
//   {p1 < p2} is D*  iff s[p1] != t[p1] (t[p1] = s[p1 + 1], or s[p1 + 2]
//             when p2 = p1 + 1; vacuous when p1 = L - 2 = |t|) and
//             (p2 = L - 1 or s[p2] != s[p2 + 1])
// (greedy reaches p1 with every earlier position matched, and reaches p2
// with every position between matched). Deletion variants of one string are
// counted once each this way (Section II A defines the variant set; the
// multiplicity only changes how often a pair is found, not which pairs).
// With n1 bit p = (p = L - 1 or s[p] != s[p + 1]) and n2 bit p = (p = L - 2
// or s[p] != s[p + 2]), in the position forms of variant_positions (p2 = L:
// one deletion at p1; p1 = L: none).
__device__ __forceinline__ bool variant_canonical(uint32_t n1, uint32_t n2, uint32_t L,
                                                  uint32_t p1, uint32_t p2) {
  if (p1 >= L) return true;
  if (p2 >= L) return (n1 >> p1) & 1u;
  const uint32_t a = p1 + 1 < p2 ? (n1 >> p1) : (n2 >> p1);
  return (a & (n1 >> p2) & 1u) != 0;
}

// The same test with no case split: n1 gains bits L and L + 1 and n2 bits
// L - 1 and L, which only the "one deletion" (p2 = L) and "none" (p1 = L,
// p2 = L + 1) forms read, so those forms pass exactly when variant_canonical
// passes them (one deletion at p < L - 1 reads n1 bit p; at L - 1, and none,
// read forced bits) and a pair p1 < p2 < L reads the original bits.
__device__ __forceinline__ void canonical_ext_masks(uint32_t n1, uint32_t n2, uint32_t L,
                                                    uint32_t& n1x, uint32_t& n2x) {
  n1x = n1 | (3u << L);
  n2x = n2 | (1u << L) | (L >= 1 ? 1u << (L - 1) : 0u);
}

__device__ __forceinline__ bool variant_canonical_ext(uint32_t n1x, uint32_t n2x, uint32_t p1,
                                                      uint32_t p2) {
  const uint32_t sel = p2 > p1 + 1 ? n1x : n2x;
  return ((sel >> p1) & (n1x >> p2) & 1u) != 0;
}

// Number of distinct strings among the deletion variants with at most k
// deletions: the canonical sets above, counted in O(L) from the same masks
// (the run count is the number of canonical first deletions p1 <= p2 - 2).
__device__ __forceinline__ uint32_t num_distinct_variants(uint32_t n1, uint32_t n2, uint32_t L,
                                                          int k) {
  uint32_t c = 1;
  if (k >= 1) c += (uint32_t)__popc(n1);
  if (k >= 2)
    for (uint32_t p2 = 1; p2 < L; ++p2)
      if ((n1 >> p2) & 1u)
        c += (uint32_t)__popc(n1 & ((1u << (p2 - 1)) - 1u)) + ((n2 >> (p2 - 1)) & 1u);
  return c;
}

// The masks of variant_canonical from a string's five residue bit planes
// (bit t of plane q is bit q of residue t).
__device__ __forceinline__ void canonical_masks(const uint32_t (&pl)[5], uint32_t L, uint32_t& n1,
                                                uint32_t& n2) {
  uint32_t d1 = 0, d2 = 0;
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    d1 |= pl[q] ^ (pl[q] >> 1);
    d2 |= pl[q] ^ (pl[q] >> 2);
  }
  n1 = (d1 & ((1u << (L - 1)) - 1u)) | (1u << (L - 1));
  n2 = L >= 2 ? (d2 & ((1u << (L - 2)) - 1u)) | (1u << (L - 2)) : 0u;
}

// Three deletions (k = 3). In general D is D* iff every deleted position p
// whose next kept position q(p) exists holds a different residue than q(p)
// (greedy reaches p with everything before matched and would match s[p]
// where t continues with s[q(p)]). For |D| <= 3, q(p) - p is 1, 2 or 3, so a
// third mask n3 bit p = (p >= L - 3 or s[p] != s[p + 3]) completes the test.
// Sets are taken as padded triples p1 < p2 < p3 (a pair is (p1, p2, L), one
// deletion (p1, L, L + 1), none (L, L + 1, L + 2)); n1x and n2x are the
// extended masks of canonical_ext_masks.
__device__ __forceinline__ bool variant_canonical3(uint32_t n1x, uint32_t n2x, uint32_t n3,
                                                   uint32_t L, uint32_t p1, uint32_t p2,
                                                   uint32_t p3) {
  const bool run3 = p3 < L && p3 == p2 + 1;  // p2 and p3 both deleted, adjacent
  const bool c3 = p3 >= L || ((n1x >> p3) & 1u);
  const bool c2 = p2 >= L || (((run3 ? n2x : n1x) >> p2) & 1u);
  const uint32_t m1 = p2 > p1 + 1 ? n1x : (p2 < L && run3) ? n3 : n2x;
  const bool c1 = p1 >= L || ((m1 >> p1) & 1u);
  return c1 && c2 && c3;
}

// Canonical sets of exactly three deletions, in O(L^2) from the masks: for
// every canonical last two deletions (p2, p3), first deletions p1 <= p2 - 2
// need n1, and p1 = p2 - 1 needs n2 (p3 > p2 + 1) or n3 (p3 = p2 + 1).
__device__ __forceinline__ uint32_t num_distinct_triples(uint32_t n1, uint32_t n2, uint32_t n3,
                                                         uint32_t L) {
  uint32_t c = 0;
  for (uint32_t p3 = 2; p3 < L; ++p3) {
    if (!((n1 >> p3) & 1u)) continue;
    for (uint32_t p2 = 1; p2 < p3; ++p2) {
      const bool adj = p3 == p2 + 1;
      if (!(((adj ? n2 : n1) >> p2) & 1u)) continue;
      c += (uint32_t)__popc(n1 & ((1u << (p2 - 1)) - 1u)) + (((adj ? n3 : n2) >> (p2 - 1)) & 1u);
    }
  }
  return c;
}

// n3 of variant_canonical3 from the residue bit planes.
__device__ __forceinline__ uint32_t canonical_mask3(const uint32_t (&pl)[5], uint32_t L) {
  uint32_t d3 = 0;
#pragma unroll
  for (int q = 0; q < 5; ++q) d3 |= pl[q] ^ (pl[q] >> 3);
  const uint32_t hi = L >= 3 ? ~((1u << (L - 3)) - 1u) : ~0u;  // bits p >= L - 3
  return (d3 | hi) & ((1u << L) - 1u);
}

// Variant number v of a key in the enumeration order: v = 0 keeps the
// string, v = 1..L deletes position v-1, larger v delete a position pair
// (p1 < p2) in lexicographic order. The pair index u = v - 1 - L is unranked
// in closed form: T(p) = p (2L - 1 - p) / 2 pairs start before p, so p1 is
// the largest p with T(p) <= u, a root of a quadratic (one correction step
// each way absorbs the rounding of sqrtf).
__device__ __forceinline__ u128 key_variant(u128 key, uint32_t v) {
  const uint32_t L = key_len(key);
  if (v == 0) return key;
  if (v <= L) return key_delete(key, (int)v - 1);
  const int u = (int)(v - 1 - L);
  const int a = 2 * (int)L - 1;
  int p1 = (int)((a - sqrtf((float)(a * a - 8 * u))) * 0.5f);
  p1 = p1 < 0 ? 0 : p1;
  if ((p1 + 1) * (a - p1 - 1) / 2 <= u) ++p1;
  if (p1 * (a - p1) / 2 > u) --p1;
  const int p2 = p1 + 1 + (u - p1 * (a - p1) / 2);
  return key_delete(key_delete(key, p2), p1);
}

// ------------------------------------------------------------------ wave64

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of mask in lanes below this lane
__device__ __forceinline__ uint32_t mask_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Lanes of `live` whose 8-bit digit equals this lane's: for each bit, keep
// the lanes that agree with this lane on it. m is 0 or all ones (this lane's
// bit, a signed one-bit field extract), so the agreeing lanes are
// ~(ballot ^ m); v_bitop3 applies peers & ~(ballot ^ m) to each 32-bit half
// in one instruction. Its table 0x84 is symmetric in the first and third
// operands, so it does not depend on which of them indexes the high bit.
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, uint64_t live) {
  uint32_t lo = (uint32_t)live, hi = (uint32_t)(live >> 32);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    uint32_t m;  // the compiler would expand a constant-offset field extract into two shifts
    asm volatile("v_bfe_i32 %0, %1, %2, 1" : "=v"(m) : "v"(d), "s"(b));
    const uint64_t bb = __ballot(m != 0);
    lo = __builtin_amdgcn_bitop3_b32((uint32_t)bb, lo, m, 0x84);
    hi = __builtin_amdgcn_bitop3_b32((uint32_t)(bb >> 32), hi, m, 0x84);
  }
  return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T t = __shfl_up(v, o, 64);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

// Exclusive scan of one value per thread over a block of NT threads (NT a
// multiple of 64, at most 1024). s_tmp holds NT/64 entries. Returns the
// exclusive prefix; *total receives the block sum. Contains barriers.
template <int NT, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* s_tmp, T* total) {
  constexpr int NW = NT / 64;
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x / 64;
  T incl = wave_incl_scan(v);
  if (lane == 63) s_tmp[w] = incl;
  __syncthreads();
  T before = 0, sum = 0;
#pragma unroll
  for (int x = 0; x < NW; ++x) {
    T t = s_tmp[x];
    if ((uint32_t)x < w) before += t;
    sum += t;
  }
  __syncthreads();
  *total = sum;
  return before + incl - v;
}

// ------------------------------------------------------------------ sharded output
//
// Variable-length output of many writers (candidate pairs, matches). One
// global counter would serialise every reservation on one address, so the
// output is split into OUT_SHARDS regions of `region` slots, each with its
// own counter; a writer reserves in shard (sel % OUT_SHARDS). The part of a
// reservation that runs past its region's end goes to a shared overflow
// region (counter[OUT_SHARDS]); only if that overflows too are slots dropped,
// which the host sees in the counters and answers by running the kernel
// again with more room. The host then gathers everything into one array.
constexpr uint32_t OUT_SHARDS = 1024;

struct ShardOut {
  uint64_t* base;               // OUT_SHARDS * region slots
  uint64_t region;              // slots per shard
  uint64_t* over;               // overflow slots
  uint64_t over_cap;
  unsigned long long* counter;  // OUT_SHARDS + 1 counters, zeroed before the kernel
};

// A reservation of cnt slots: slot j (0 <= j < cnt) is shard[pos + j] while
// pos + j < region, else over[obase + (pos + j - max(pos, region))].
struct ShardResv {
  uint64_t pos, obase;
};

// Taken by one lane for its wave or block.
__device__ __forceinline__ ShardResv shard_reserve(const ShardOut& o, uint32_t sel, uint64_t cnt) {
  ShardResv r;
  r.pos = atomicAdd(&o.counter[sel % OUT_SHARDS], (unsigned long long)cnt);
  const uint64_t end = r.pos + cnt;
  const uint64_t spill = end > o.region ? end - (r.pos > o.region ? r.pos : o.region) : 0;
  r.obase = spill ? atomicAdd(&o.counter[OUT_SHARDS], (unsigned long long)spill) : 0;
  return r;
}

__device__ __forceinline__ void shard_put(const ShardOut& o, uint32_t sel, const ShardResv& r,
                                          uint64_t j, uint64_t v) {
  const uint64_t gi = r.pos + j;
  if (gi < o.region) {
    o.base[(uint64_t)(sel % OUT_SHARDS) * o.region + gi] = v;
  } else {
    const uint64_t oi = r.obase + (gi - (r.pos > o.region ? r.pos : o.region));
    if (oi < o.over_cap) o.over[oi] = v;
  }
}

// ------------------------------------------------------------------ look-back
//
// Decoupled look-back (Merrill & Garland, "Single-pass parallel prefix scan
// with decoupled look-back", 2016). One 64-bit status word per (tile, lane of
// the scan): bits 63..48 an epoch that tags the pass, bits 47..46 a flag
// (1 = tile aggregate only, 2 = inclusive prefix), bits 45..0 the value.
// Words from an older epoch read as "not ready", so the status array never
// needs clearing between passes.
constexpr uint64_t LB_AGG = 1, LB_PREFIX = 2;
constexpr uint64_t LB_VALUE_MASK = (1ull << 46) - 1;

__device__ __forceinline__ uint64_t lb_pack(uint64_t epoch, uint64_t flag, uint64_t value) {
  return (epoch << 48) | (flag << 46) | (value & LB_VALUE_MASK);
}

__device__ __forceinline__ void lb_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lb_load(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish this tile's aggregate, walk back over earlier tiles until an
// inclusive prefix is found, publish this tile's inclusive prefix and return
// the exclusive prefix. `stride` is the distance between consecutive tiles'
// words for this lane. Tiles must be numbered in the order they started
// (dynamic tile ids), so every earlier tile is resident or finished.
// The wait is bounded: after LB_SPIN_LIMIT polls of one word the tile sets
// SD_ERRBIT_LOOKBACK in *err and stops waiting (the host then reports an
// error), so every wave exits even if an earlier tile never publishes.
constexpr uint32_t LB_SPIN_LIMIT = 1u << 16;
__device__ __forceinline__ uint64_t lb_exclusive(uint64_t* status, uint64_t tile, uint64_t stride,
                                                 uint64_t epoch, uint64_t aggregate,
                                                 uint32_t* err) {
  uint64_t* mine = status + tile * stride;
  if (tile == 0) {
    lb_store(mine, lb_pack(epoch, LB_PREFIX, aggregate));
    return 0;
  }
  lb_store(mine, lb_pack(epoch, LB_AGG, aggregate));
  uint64_t excl = 0;
  int64_t j = (int64_t)tile - 1;
  uint32_t spins = 0;
  while (true) {
    const uint64_t s = lb_load(status + (uint64_t)j * stride);
    const uint64_t flag = (s >> 46) & 3u;
    if ((s >> 48) != epoch || flag == 0) {
      if (++spins >= LB_SPIN_LIMIT) {
        atomicOr(err, 8u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    spins = 0;
    excl += s & LB_VALUE_MASK;
    if (flag == LB_PREFIX) break;
    --j;
  }
  lb_store(mine, lb_pack(epoch, LB_PREFIX, excl + aggregate));
  return excl;
}
