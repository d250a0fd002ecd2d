// LSD radix sort primitives for gfx950 (wave64, 160 KB LDS per CU).
//
// Records are one or two 64-bit key words (structure of arrays: word 0 is
// the least significant) with an optional 32-bit payload. A pass sorts
// stably by one 8-bit digit:
//   * the digit histograms of every pass come from one read of the keys
//     (k_radix_hist), so each pass knows its global bucket bases;
//   * each pass is a single kernel (k_onesweep): a tile ranks its elements
//     with wave64 ballots (match-any over the 8 digit bits, mbcnt for the
//     rank below the lane), keeps per-wave digit counters in LDS, publishes
//     its per-digit counts and finds its global offsets by decoupled
//     look-back, then writes through LDS so that each digit's elements leave
//     the tile as one contiguous run.
// This is the paper's sortKeyValues / sort primitive (Section II B; Appendix A
// steps 4 and 6) written for CDNA4 instead of taken from a library.
#include <algorithm>

#include "sd_device.h"
#include "sd_internal.h"

namespace sdk {

constexpr int RADIX = 256;
constexpr int NT = 256;  // threads per block: four wave64s
constexpr int NWAVE = NT / 64;

// ------------------------------------------------------------------ histogram

template <int NW>
__global__ __launch_bounds__(NT) void k_radix_hist(const uint64_t* __restrict__ w0,
                                                   const uint64_t* __restrict__ w1, uint64_t n,
                                                   uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[NW * 8 * RADIX];
  for (int x = threadIdx.x; x < NW * 8 * RADIX; x += NT) s_h[x] = 0;
  __syncthreads();
  for (uint64_t e = (uint64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (uint64_t)gridDim.x * NT) {
    const uint64_t a = w0[e];
#pragma unroll
    for (int q = 0; q < 8; ++q) atomicAdd(&s_h[q * RADIX + ((a >> (8 * q)) & 255u)], 1u);
    if (NW == 2) {
      const uint64_t b = w1[e];
#pragma unroll
      for (int q = 0; q < 8; ++q) atomicAdd(&s_h[(8 + q) * RADIX + ((b >> (8 * q)) & 255u)], 1u);
    }
  }
  __syncthreads();
  for (int x = threadIdx.x; x < NW * 8 * RADIX; x += NT)
    if (s_h[x]) atomicAdd(&hist[x], s_h[x]);
}

// ------------------------------------------------------------------ one pass

template <int NW, bool HAS_VAL, int ITEMS>
__global__ __launch_bounds__(NT) void k_onesweep(
    const uint64_t* __restrict__ in0, const uint64_t* __restrict__ in1,
    const uint32_t* __restrict__ vin, uint64_t* __restrict__ out0, uint64_t* __restrict__ out1,
    uint32_t* __restrict__ vout, uint32_t n, int word, int shift, uint32_t mask,
    const uint32_t* __restrict__ hist256, uint64_t* __restrict__ status,
    uint32_t* __restrict__ tile_counter, uint32_t epoch, uint32_t* __restrict__ err) {
  constexpr int TILE = NT * ITEMS;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_wh[NWAVE][RADIX];  // per-wave digit counts, then per-wave offsets
  __shared__ uint32_t s_lstart[RADIX];     // digit start inside the tile
  __shared__ uint32_t s_gstart[RADIX];     // digit start in the output for this tile
  __shared__ uint32_t s_tmp[NWAVE];
  __shared__ uint32_t s_gidx[TILE];        // output index of each staged slot
  __shared__ uint64_t s_stage[TILE];

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint32_t w = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  for (int x = tid; x < NWAVE * RADIX; x += NT) (&s_wh[0][0])[x] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  if (tile >= gridDim.x) return;  // counters are zeroed per pass; never taken
  const uint64_t base = (uint64_t)tile * TILE;
  const uint32_t nvalid = (uint32_t)min<uint64_t>((uint64_t)TILE, (uint64_t)n - base);

  uint64_t k0[ITEMS], k1[ITEMS];
  uint32_t val[ITEMS], dig[ITEMS], rnk[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint64_t e = base + (uint64_t)w * 64 * ITEMS + (uint64_t)r * 64 + lane;
    const bool valid = e < n;
    k0[r] = valid ? in0[e] : 0;
    if (NW == 2) k1[r] = valid ? in1[e] : 0;
    if (HAS_VAL) val[r] = valid ? vin[e] : 0;
  }
  // rank: elements are ordered (wave, item, lane), which is memory order
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint64_t e = base + (uint64_t)w * 64 * ITEMS + (uint64_t)r * 64 + lane;
    const bool valid = e < n;
    const uint64_t kw = (NW == 2 && word == 1) ? k1[r] : k0[r];
    const uint32_t d = (uint32_t)(kw >> shift) & mask;
    const uint64_t peers = match_digit8(d, __ballot(valid));
    const uint32_t below = mask_rank(peers);
    uint32_t prev = 0;
    if (valid) prev = s_wh[w][d];
    if (valid && below == 0) s_wh[w][d] = prev + (uint32_t)__popcll(peers);
    dig[r] = valid ? d : RADIX;
    rnk[r] = prev + below;
  }
  __syncthreads();

  // per-digit tile counts, per-wave offsets, bucket bases, look-back
  {
    const uint32_t t = tid;
    const uint32_t c0 = s_wh[0][t], c1 = s_wh[1][t], c2 = s_wh[2][t], c3 = s_wh[3][t];
    const uint32_t tot = c0 + c1 + c2 + c3;
    uint32_t sum;
    const uint32_t bbase = block_excl_scan<NT>(hist256[t], s_tmp, &sum);
    const uint32_t lstart = block_excl_scan<NT>(tot, s_tmp, &sum);
    const uint64_t excl = lb_exclusive(status + t, tile, RADIX, epoch, tot, err);
    s_wh[0][t] = 0;
    s_wh[1][t] = c0;
    s_wh[2][t] = c0 + c1;
    s_wh[3][t] = c0 + c1 + c2;
    s_lstart[t] = lstart;
    s_gstart[t] = bbase + (uint32_t)excl;
  }
  __syncthreads();

  uint32_t lpos[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint32_t d = dig[r];
    if (d < RADIX) {
      const uint32_t off = s_wh[w][d] + rnk[r];
      lpos[r] = s_lstart[d] + off;
      s_gidx[lpos[r]] = s_gstart[d] + off;
    }
  }
  // word 0
#pragma unroll
  for (int r = 0; r < ITEMS; ++r)
    if (dig[r] < RADIX) s_stage[lpos[r]] = k0[r];
  __syncthreads();
  for (uint32_t s = tid; s < nvalid; s += NT) out0[s_gidx[s]] = s_stage[s];
  if (NW == 2) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
      if (dig[r] < RADIX) s_stage[lpos[r]] = k1[r];
    __syncthreads();
    for (uint32_t s = tid; s < nvalid; s += NT) out1[s_gidx[s]] = s_stage[s];
  }
  if (HAS_VAL) {
    uint32_t* s_v = reinterpret_cast<uint32_t*>(s_stage);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
      if (dig[r] < RADIX) s_v[lpos[r]] = val[r];
    __syncthreads();
    for (uint32_t s = tid; s < nvalid; s += NT) vout[s_gidx[s]] = s_v[s];
  }
}

// Keys-only pass over one 64-bit word with larger tiles: the staged key
// itself gives its digit, so no per-slot output index is kept in LDS and the
// tile can hold twice as many elements in the same LDS footprint (fewer tiles
// means fewer look-back chains, which bound the pass at small element sizes).
template <int ITEMS>
__global__ __launch_bounds__(NT) void k_onesweep_keys(const uint64_t* __restrict__ in,
                                                      uint64_t* __restrict__ out, uint32_t n,
                                                      int shift, uint32_t mask,
                                                      const uint32_t* __restrict__ hist256,
                                                      uint64_t* __restrict__ status,
                                                      uint32_t* __restrict__ tile_counter,
                                                      uint32_t epoch, uint32_t* __restrict__ err) {
  constexpr int TILE = NT * ITEMS;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_wh[NWAVE][RADIX];
  __shared__ uint32_t s_lstart[RADIX];
  __shared__ uint32_t s_gstart[RADIX];
  __shared__ uint32_t s_tmp[NWAVE];
  __shared__ uint64_t s_stage[TILE];

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint32_t w = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(tile_counter, 1u);
  for (int x = tid; x < NWAVE * RADIX; x += NT) (&s_wh[0][0])[x] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  if (tile >= gridDim.x) return;  // counters are zeroed per pass; never taken
  const uint64_t base = (uint64_t)tile * TILE;
  const uint32_t nvalid = (uint32_t)min<uint64_t>((uint64_t)TILE, (uint64_t)n - base);

  const uint64_t* __restrict__ tin = in + base;
  const uint32_t lbase = w * 64 * ITEMS + lane;
  uint64_t k0[ITEMS];
  uint32_t dr[ITEMS];  // digit << 16 | rank inside the wave (digit 256: no element)
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint32_t le = lbase + r * 64;
    k0[r] = le < nvalid ? tin[le] : 0;
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const bool valid = lbase + r * 64 < nvalid;
    const uint32_t d = (uint32_t)(k0[r] >> shift) & mask;
    const uint64_t peers = match_digit8(d, __ballot(valid));
    const uint32_t below = mask_rank(peers);
    uint32_t prev = 0;
    if (valid) prev = s_wh[w][d];
    if (valid && below == 0) s_wh[w][d] = prev + (uint32_t)__popcll(peers);
    dr[r] = ((valid ? d : (uint32_t)RADIX) << 16) | (prev + below);
  }
  __syncthreads();
  {
    const uint32_t t = tid;
    const uint32_t c0 = s_wh[0][t], c1 = s_wh[1][t], c2 = s_wh[2][t], c3 = s_wh[3][t];
    const uint32_t tot = c0 + c1 + c2 + c3;
    uint32_t sum;
    const uint32_t bbase = block_excl_scan<NT>(hist256[t], s_tmp, &sum);
    const uint32_t lstart = block_excl_scan<NT>(tot, s_tmp, &sum);
    const uint64_t excl = lb_exclusive(status + t, tile, RADIX, epoch, tot, err);
    s_wh[0][t] = 0;
    s_wh[1][t] = c0;
    s_wh[2][t] = c0 + c1;
    s_wh[3][t] = c0 + c1 + c2;
    s_lstart[t] = lstart;
    s_gstart[t] = bbase + (uint32_t)excl;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const uint32_t d = dr[r] >> 16;
    if (d < RADIX) s_stage[s_lstart[d] + s_wh[w][d] + (dr[r] & 0xFFFFu)] = k0[r];
  }
  __syncthreads();
  // counts that disagree with the input would place past the end: such a
  // write is dropped and reported
  for (uint32_t s = tid; s < nvalid; s += NT) {
    const uint64_t v = s_stage[s];
    const uint32_t d = (uint32_t)(v >> shift) & mask;
    const uint32_t pos = s_gstart[d] + (s - s_lstart[d]);
    if (pos < n)
      out[pos] = v;
    else
      atomicOr(err, SD_ERRBIT_PLACEMENT);
  }
}

// ------------------------------------------------------------------ counted pass

// A keys-only pass over input written by a producer in consecutive ranges
// ("tiles") whose digits it also counted: tile t holds the elements
// [voff[t spt], voff[min((t + 1) spt, nseq)]) and counts[t][d] of them have
// digit d. After a scan of the counts every tile knows where its digit runs
// go, so the pass needs no look-back chain between tiles; a tile is placed in
// chunks of CT_CHUNK elements, each advancing per-digit cursors.
constexpr int CT_ITEMS = 16;
constexpr uint32_t CT_CHUNK = NT * CT_ITEMS;
constexpr int CT_LOADS = 16;  // loads in flight per thread in the count scans

// Per block of R consecutive tiles and per digit: the exclusive running sum
// inside the block (into local) and the block total (into bsum). A tile's
// counts are the sum of G consecutive rows of counts (nrows rows in all).
__global__ __launch_bounds__(RADIX) void k_tile_scan_local(const uint32_t* __restrict__ counts,
                                                           uint32_t nrows, uint32_t G,
                                                           uint32_t tiles, uint32_t R,
                                                           uint32_t* __restrict__ local,
                                                           uint32_t* __restrict__ bsum) {
  const uint32_t d = threadIdx.x;
  const uint32_t t0 = blockIdx.x * R, t1 = min(t0 + R, tiles);
  uint32_t run = 0;
  for (uint32_t t = t0; t < t1; t += CT_LOADS) {
    uint32_t c[CT_LOADS];
#pragma unroll
    for (int u = 0; u < CT_LOADS; ++u) {
      c[u] = 0;
      if (t + u < t1) {
        const uint32_t r0 = (t + u) * G, r1 = min(r0 + G, nrows);
        for (uint32_t r = r0; r < r1; ++r) c[u] += counts[(uint64_t)r * RADIX + d];
      }
    }
#pragma unroll
    for (int u = 0; u < CT_LOADS; ++u) {
      if (t + u < t1) local[(uint64_t)(t + u) * RADIX + d] = run;
      run += c[u];
    }
  }
  bsum[(uint64_t)blockIdx.x * RADIX + d] = run;
}

// One block: bsum[b][d] becomes the start of block b's digit-d elements in
// the sorted output (digit base plus the totals of earlier blocks). Thread
// (g, d) runs digit d over a quarter g of the rows.
constexpr int CT_SCAN_GROUPS = 4;
__global__ __launch_bounds__(CT_SCAN_GROUPS * RADIX) void k_tile_scan_blocks(
    uint32_t* __restrict__ bsum, uint32_t nb) {
  constexpr int NTH = CT_SCAN_GROUPS * RADIX;
  __shared__ uint32_t s_part[CT_SCAN_GROUPS][RADIX];
  __shared__ uint32_t s_base[RADIX];
  __shared__ uint32_t s_tmp[NTH / 64];
  const uint32_t d = threadIdx.x % RADIX, g = threadIdx.x / RADIX;
  const uint32_t per = (nb + CT_SCAN_GROUPS - 1) / CT_SCAN_GROUPS;
  const uint32_t b0 = min(g * per, nb), b1 = min(b0 + per, nb);
  uint32_t run = 0;
  for (uint32_t b = b0; b < b1; b += CT_LOADS) {
    uint32_t c[CT_LOADS];
#pragma unroll
    for (int u = 0; u < CT_LOADS; ++u) c[u] = b + u < b1 ? bsum[(uint64_t)(b + u) * RADIX + d] : 0u;
#pragma unroll
    for (int u = 0; u < CT_LOADS; ++u) {
      if (b + u < b1) bsum[(uint64_t)(b + u) * RADIX + d] = run;
      run += c[u];
    }
  }
  s_part[g][d] = run;
  __syncthreads();
  uint32_t total = 0;
  if (g == 0) {
    for (int q = 0; q < CT_SCAN_GROUPS; ++q) {
      const uint32_t c = s_part[q][d];
      s_part[q][d] = total;
      total += c;
    }
  }
  // digit bases: threads 0..255 (group 0) are the digits in order
  uint32_t all;
  const uint32_t base = block_excl_scan<NTH>(total, s_tmp, &all);
  if (g == 0) s_base[d] = base;
  __syncthreads();
  const uint32_t add = s_part[g][d] + s_base[d];
  for (uint32_t b = b0; b < b1; ++b) bsum[(uint64_t)b * RADIX + d] += add;
}

// Digit counts of fixed tiles of CT_CHUNK elements (one row of 256 per tile),
// for a counted pass over data whose producer did not count it.
__global__ __launch_bounds__(NT) void k_tile_counts(const uint64_t* __restrict__ in, uint32_t n,
                                                    int shift, uint32_t mask,
                                                    uint32_t* __restrict__ counts) {
  __shared__ uint32_t s_h[RADIX];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * CT_CHUNK;
  const uint32_t nvalid = (uint32_t)min<uint64_t>((uint64_t)CT_CHUNK, (uint64_t)n - base);
  const uint64_t* __restrict__ tin = in + base;
  uint64_t v[CT_ITEMS];
#pragma unroll
  for (int r = 0; r < CT_ITEMS; ++r) {
    const uint32_t e = r * NT + threadIdx.x;
    v[r] = e < nvalid ? tin[e] : 0;
  }
#pragma unroll
  for (int r = 0; r < CT_ITEMS; ++r)
    if (r * NT + threadIdx.x < nvalid) atomicAdd(&s_h[(uint32_t)(v[r] >> shift) & mask], 1u);
  __syncthreads();
  counts[(uint64_t)blockIdx.x * RADIX + threadIdx.x] = s_h[threadIdx.x];
}

// Workgroups are dispatched to the eight XCDs in turn; this maps them so that
// each XCD takes one contiguous range of tiles in order. Consecutive tiles
// write adjacent pieces of every digit's run, so the cache lines they share
// are completed in one XCD's L2 instead of being written back partially by
// two (a bijection of [0, G)).
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t G) {
  const uint32_t x = b & 7u;
  uint32_t start = 0;
  for (uint32_t q = 0; q < x; ++q) start += (G - q + 7) / 8;
  return start + (b >> 3);
}

template <int ITEMS>
__global__ __launch_bounds__(NT) void k_scatter_counted(
    const uint64_t* __restrict__ in, uint64_t* __restrict__ out, uint32_t n, int shift,
    uint32_t mask, const uint32_t* __restrict__ local, const uint32_t* __restrict__ off1,
    const uint32_t* __restrict__ boff, uint32_t R1, uint32_t R2,
    const uint64_t* __restrict__ voff, uint32_t spt, uint64_t nseq, uint32_t* __restrict__ err) {
  constexpr int CHUNK = NT * ITEMS;
  __shared__ uint32_t s_wh[NWAVE][RADIX];
  __shared__ uint32_t s_lstart[RADIX];
  __shared__ uint32_t s_gstart[RADIX];
  __shared__ uint32_t s_tmp[NWAVE];
  __shared__ uint64_t s_stage[CHUNK];

  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u;
  const uint32_t w = tid >> 6;
  const uint32_t tile = xcd_contiguous(blockIdx.x, gridDim.x);
  // tiles by sequence ranges (voff), or fixed CHUNK-element tiles (no voff)
  uint64_t a, b;
  if (voff) {
    const uint64_t q0 = (uint64_t)tile * spt;
    a = voff[q0];
    b = voff[min<uint64_t>(q0 + spt, nseq)];
  } else {
    a = (uint64_t)tile * CHUNK;
    b = min<uint64_t>(a + CHUNK, n);
  }
  // this thread's digit (tid) cursor in the output
  uint32_t cur = boff[(uint64_t)(tile / R1 / R2) * RADIX + tid] +
                 off1[(uint64_t)(tile / R1) * RADIX + tid] + local[(uint64_t)tile * RADIX + tid];
  for (uint64_t c0 = a; c0 < b; c0 += CHUNK) {
    for (int x = tid; x < NWAVE * RADIX; x += NT) (&s_wh[0][0])[x] = 0;
    __syncthreads();
    const uint32_t nvalid = (uint32_t)min<uint64_t>((uint64_t)CHUNK, b - c0);
    const uint64_t* __restrict__ tin = in + c0;
    const uint32_t lbase = w * 64 * ITEMS + lane;
    uint64_t k0[ITEMS];
    uint32_t dr[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const uint32_t le = lbase + r * 64;
      k0[r] = le < nvalid ? tin[le] : 0;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const bool valid = lbase + r * 64 < nvalid;
      const uint32_t d = (uint32_t)(k0[r] >> shift) & mask;
      const uint64_t peers = match_digit8(d, __ballot(valid));
      const uint32_t below = mask_rank(peers);
      uint32_t prev = 0;
      if (valid) prev = s_wh[w][d];
      if (valid && below == 0) s_wh[w][d] = prev + (uint32_t)__popcll(peers);
      dr[r] = ((valid ? d : (uint32_t)RADIX) << 16) | (prev + below);
    }
    __syncthreads();
    {
      const uint32_t t = tid;
      const uint32_t n0 = s_wh[0][t], n1 = s_wh[1][t], n2 = s_wh[2][t], n3 = s_wh[3][t];
      uint32_t sum;
      const uint32_t lstart = block_excl_scan<NT>(n0 + n1 + n2 + n3, s_tmp, &sum);
      s_wh[0][t] = 0;
      s_wh[1][t] = n0;
      s_wh[2][t] = n0 + n1;
      s_wh[3][t] = n0 + n1 + n2;
      s_lstart[t] = lstart;
      s_gstart[t] = cur;
      cur += n0 + n1 + n2 + n3;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const uint32_t d = dr[r] >> 16;
      if (d < RADIX) s_stage[s_lstart[d] + s_wh[w][d] + (dr[r] & 0xFFFFu)] = k0[r];
    }
    __syncthreads();
    // counts that disagree with the input would place past the end: such a
    // write is dropped and reported
    for (uint32_t s = tid; s < nvalid; s += NT) {
      const uint64_t v = s_stage[s];
      const uint32_t d = (uint32_t)(v >> shift) & mask;
      const uint32_t pos = s_gstart[d] + (s - s_lstart[d]);
      if (pos < n)
        out[pos] = v;
      else
        atomicOr(err, SD_ERRBIT_PLACEMENT);
    }
    __syncthreads();  // the next chunk rewrites the LDS
  }
}

// ------------------------------------------------------------------ scan

// Exclusive scan of n 32-bit counts into n + 1 64-bit offsets (out[n] is the
// total) in one pass with decoupled look-back.
constexpr int SCAN_ITEMS = 16;
__global__ __launch_bounds__(NT) void k_scan_excl(const uint32_t* __restrict__ in,
                                                  uint64_t* __restrict__ out, uint64_t n,
                                                  uint64_t* __restrict__ status,
                                                  uint32_t* __restrict__ tile_counter,
                                                  uint32_t epoch, uint32_t* __restrict__ err) {
  constexpr int TILE = NT * SCAN_ITEMS;
  __shared__ uint32_t s_tile;
  __shared__ uint64_t s_tmp[NWAVE];
  __shared__ uint64_t s_excl;
  if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  if (tile >= gridDim.x) return;
  const uint64_t first = tile * TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint64_t tsum = 0;
#pragma unroll
  for (int x = 0; x < SCAN_ITEMS; ++x) {
    v[x] = (first + x < n) ? in[first + x] : 0u;
    tsum += v[x];
  }
  uint64_t total;
  const uint64_t texcl = block_excl_scan<NT>(tsum, s_tmp, &total);
  if (threadIdx.x == 0) s_excl = lb_exclusive(status, tile, 1, epoch, total, err);
  __syncthreads();
  uint64_t run = s_excl + texcl;
#pragma unroll
  for (int x = 0; x < SCAN_ITEMS; ++x) {
    if (first + x < n) out[first + x] = run;
    run += v[x];
    if (first + x + 1 == n) out[n] = run;
  }
}

// Exclusive prefix of the shards' written counts min(counter[s], region);
// one block of OUT_SHARDS threads. off[OUT_SHARDS] = the overflow's start.
__global__ __launch_bounds__(OUT_SHARDS) void k_shard_offsets(
    const unsigned long long* __restrict__ counter, uint64_t region, uint64_t* __restrict__ off) {
  __shared__ uint64_t s_tmp[OUT_SHARDS / 64];
  const uint64_t c = min((uint64_t)counter[threadIdx.x], region);
  uint64_t total;
  off[threadIdx.x] = block_excl_scan<OUT_SHARDS>(c, s_tmp, &total);
  if (threadIdx.x == 0) off[OUT_SHARDS] = total;
}

// Shard s's written slots go to out at off[s] (block s); blocks OUT_SHARDS
// and up copy the overflow after them, grid-stride.
__global__ __launch_bounds__(256) void k_gather_shards(const uint64_t* __restrict__ base,
                                                       uint64_t region,
                                                       const uint64_t* __restrict__ over,
                                                       uint64_t over_cap,
                                                       const unsigned long long* __restrict__ counter,
                                                       const uint64_t* __restrict__ off,
                                                       uint64_t* __restrict__ out, uint64_t cap) {
  const uint32_t sh = blockIdx.x;
  if (sh < OUT_SHARDS) {
    const uint64_t o = off[sh];
    const uint64_t cnt = min(min((uint64_t)counter[sh], region), o < cap ? cap - o : 0);
    const uint64_t* src = base + (uint64_t)sh * region;
    uint64_t* dst = out + o;
    for (uint64_t x = threadIdx.x; x < cnt; x += 256) dst[x] = src[x];
  } else {
    const uint64_t o = off[OUT_SHARDS];
    const uint64_t cnt = min(min((uint64_t)counter[OUT_SHARDS], over_cap), o < cap ? cap - o : 0);
    uint64_t* dst = out + o;
    const uint64_t nb = gridDim.x - OUT_SHARDS;
    for (uint64_t x = (uint64_t)(sh - OUT_SHARDS) * 256 + threadIdx.x; x < cnt; x += nb * 256)
      dst[x] = over[x];
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, uint64_t n) {
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

}  // namespace sdk

// ------------------------------------------------------------------ launchers

namespace sd {

static unsigned grid_for(uint64_t n, unsigned per_block, unsigned cap) {
  uint64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
}

uint32_t out_shards() { return OUT_SHARDS; }

// off: OUT_SHARDS + 1 scratch words
void launch_gather_shards(const uint64_t* base, uint64_t region, const uint64_t* over,
                          uint64_t over_cap, const unsigned long long* counter, uint64_t* off,
                          uint64_t* out, hipStream_t s, uint64_t cap) {
  hipLaunchKernelGGL(sdk::k_shard_offsets, dim3(1), dim3(OUT_SHARDS), 0, s, counter, region, off);
  hipLaunchKernelGGL(sdk::k_gather_shards, dim3(OUT_SHARDS + 256), dim3(256), 0, s, base, region,
                     over, over_cap, counter, off, out, cap);
}

void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_fill_u64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
}

void launch_radix_hist(const uint64_t* w0, const uint64_t* w1, int nwords, uint64_t n,
                       uint32_t* hist, hipStream_t s) {
  if (!n) return;
  const unsigned g = grid_for(n, sdk::NT * 16, 2048);
  if (nwords == 2)
    hipLaunchKernelGGL(sdk::k_radix_hist<2>, dim3(g), dim3(sdk::NT), 0, s, w0, w1, n, hist);
  else
    hipLaunchKernelGGL(sdk::k_radix_hist<1>, dim3(g), dim3(sdk::NT), 0, s, w0, w1, n, hist);
}

// keys-only passes take 16 or 32 items per thread (the autotuner picks)
static int keys_items(int items) { return items == 16 ? 16 : 32; }

uint64_t onesweep_tile(int nwords, bool has_val, int items) {
  if (nwords == 1 && !has_val) return (uint64_t)sdk::NT * keys_items(items);
  return (uint64_t)sdk::NT * 16;
}

void launch_onesweep(const uint64_t* in0, const uint64_t* in1, const uint32_t* vin,
                     uint64_t* out0, uint64_t* out1, uint32_t* vout, int nwords, bool has_val,
                     uint32_t n, int word, int shift, uint32_t mask, const uint32_t* hist256,
                     uint64_t* status, uint32_t* tile_counter, uint32_t epoch, uint32_t* err,
                     int items, hipStream_t s) {
  if (!n) return;
  const uint64_t tile = onesweep_tile(nwords, has_val, items);
  const uint64_t tiles = (n + tile - 1) / tile;
  dim3 g((unsigned)tiles), b(sdk::NT);
  if (nwords == 2 && has_val)
    hipLaunchKernelGGL((sdk::k_onesweep<2, true, 16>), g, b, 0, s, in0, in1, vin, out0, out1,
                       vout, n, word, shift, mask, hist256, status, tile_counter, epoch, err);
  else if (nwords == 2)
    hipLaunchKernelGGL((sdk::k_onesweep<2, false, 16>), g, b, 0, s, in0, in1, vin, out0, out1,
                       vout, n, word, shift, mask, hist256, status, tile_counter, epoch, err);
  else if (has_val)
    hipLaunchKernelGGL((sdk::k_onesweep<1, true, 16>), g, b, 0, s, in0, in1, vin, out0, out1,
                       vout, n, word, shift, mask, hist256, status, tile_counter, epoch, err);
  else if (keys_items(items) == 16)
    hipLaunchKernelGGL((sdk::k_onesweep_keys<16>), g, b, 0, s, word == 1 ? in1 : in0, out0, n,
                       shift, mask, hist256, status, tile_counter, epoch, err);
  else
    hipLaunchKernelGGL((sdk::k_onesweep_keys<32>), g, b, 0, s, word == 1 ? in1 : in0, out0, n,
                       shift, mask, hist256, status, tile_counter, epoch, err);
}

// The count scan in three levels, each a single round of loads per thread:
// tiles in blocks of R1 = 16 (exclusive sums into local, block sums into
// sums1), those block sums in blocks of R2 (exclusive sums into off1, block
// sums into sums2), and sums2 in one block with the digit bases. bsum holds
// off1 (nb1 rows), sums1 (nb1 rows) and sums2 (nb2 rows).
struct ScanShape {
  uint32_t R1, nb1, R2, nb2;
};
static ScanShape scan_shape(uint64_t tiles) {
  ScanShape g;
  g.R1 = 16;
  g.nb1 = (uint32_t)((tiles + g.R1 - 1) / g.R1);
  g.R2 = std::max<uint32_t>(16, (g.nb1 + 255) / 256);
  g.nb2 = (g.nb1 + g.R2 - 1) / g.R2;
  return g;
}

uint32_t counted_scan_rows(uint64_t tiles) {
  const ScanShape g = scan_shape(tiles);
  return 2 * g.nb1 + g.nb2;
}

void launch_counted_scan(const uint32_t* counts, uint64_t nrows, uint32_t rows_per_tile,
                         uint32_t* local, uint32_t* bsum, hipStream_t s) {
  if (!nrows) return;
  const uint64_t tiles = (nrows + rows_per_tile - 1) / rows_per_tile;
  const ScanShape g = scan_shape(tiles);
  uint32_t* off1 = bsum;
  uint32_t* sums1 = bsum + (uint64_t)g.nb1 * sdk::RADIX;
  uint32_t* sums2 = bsum + (uint64_t)2 * g.nb1 * sdk::RADIX;
  hipLaunchKernelGGL(sdk::k_tile_scan_local, dim3(g.nb1), dim3(sdk::RADIX), 0, s, counts,
                     (uint32_t)nrows, rows_per_tile, (uint32_t)tiles, g.R1, local, sums1);
  hipLaunchKernelGGL(sdk::k_tile_scan_local, dim3(g.nb2), dim3(sdk::RADIX), 0, s, sums1, g.nb1, 1u,
                     g.nb1, g.R2, off1, sums2);
  hipLaunchKernelGGL(sdk::k_tile_scan_blocks, dim3(1), dim3(sdk::CT_SCAN_GROUPS * sdk::RADIX), 0, s,
                     sums2, g.nb2);
}

void launch_counted_scatter(const uint64_t* in, uint64_t* out, uint32_t n, int shift, uint32_t mask,
                            uint64_t tiles, const uint32_t* local, const uint32_t* bsum,
                            const uint64_t* voff, uint32_t seqs_per_tile, uint64_t nseq,
                            uint32_t* err, hipStream_t s) {
  if (!n || !tiles) return;
  const ScanShape g = scan_shape(tiles);
  hipLaunchKernelGGL((sdk::k_scatter_counted<sdk::CT_ITEMS>), dim3((unsigned)tiles), dim3(sdk::NT),
                     0, s, in, out, n, shift, mask, local, bsum,
                     bsum + (uint64_t)2 * g.nb1 * sdk::RADIX, g.R1, g.R2, voff, seqs_per_tile, nseq,
                     err);
}

uint64_t fixed_tiles(uint64_t n) { return (n + sdk::CT_CHUNK - 1) / sdk::CT_CHUNK; }

uint32_t fixed_tile_elems() { return sdk::CT_CHUNK; }

void launch_tile_counts(const uint64_t* in, uint32_t n, int shift, uint32_t mask, uint32_t* counts,
                        hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_tile_counts, dim3((unsigned)fixed_tiles(n)), dim3(sdk::NT), 0, s, in, n,
                     shift, mask, counts);
}

void launch_counted_pass(const uint64_t* in, uint64_t* out, uint32_t n, int shift, uint32_t mask,
                         const uint32_t* counts, uint64_t tiles, const uint64_t* voff,
                         uint32_t seqs_per_tile, uint64_t nseq, uint32_t* local, uint32_t* bsum,
                         uint32_t* err, hipStream_t s) {
  if (!n || !tiles) return;
  launch_counted_scan(counts, tiles, 1, local, bsum, s);
  launch_counted_scatter(in, out, n, shift, mask, tiles, local, bsum, voff, seqs_per_tile, nseq,
                         err, s);
}

uint64_t scan_tile() { return (uint64_t)sdk::NT * sdk::SCAN_ITEMS; }

void launch_scan_excl(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* status,
                      uint32_t* tile_counter, uint32_t epoch, uint32_t* err, hipStream_t s) {
  const uint64_t tiles = n ? (n + scan_tile() - 1) / scan_tile() : 0;
  if (!tiles) {
    launch_fill_u64(out, 0, 1, s);
    return;
  }
  hipLaunchKernelGGL(sdk::k_scan_excl, dim3((unsigned)tiles), dim3(sdk::NT), 0, s, in, out, n,
                     status, tile_counter, epoch, err);
}

}  // namespace sd
