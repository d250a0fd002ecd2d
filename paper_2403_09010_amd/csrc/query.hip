// Query-versus-reference kernels for gfx950 (the database-lookup use of the
// method: queries from a patient repertoire against a reference set, paper
// Section IV; the symmetric-deletion lookup of Section II A with the variant
// map built once for the reference).
//
//   k_unique_compact  drop adjacent repeats from a sorted 64-bit array
//                     (ordered compaction with decoupled look-back)
//   k_join_seg        one workgroup per hash segment: query elements of the
//                     segment look their full hash up in the reference
//                     index segment (sorted by hash) and emit (q, r) pairs.
//                     Busy segments stage the index segment in LDS; sparse
//                     ones search global memory, so a small query does not
//                     read the whole index.
//   k_verify_weighted candidate pairs rescored by a substitution-weighted
//                     alignment cost (Section III D: a Levenshtein prefilter
//                     followed by a finer metric), kept when both the unit
//                     distance is <= k and the score is <= max_score
//   k_set_ranges      per-set slices of a (q, r)-sorted result
//   k_slice_rebase    copy one set's slice with query ids made set-local
#include "sd_device.h"
#include "sd_internal.h"

namespace sdk {

constexpr int QNT = 256;

// ------------------------------------------------------------------ unique

constexpr int UITEMS = 16;

__global__ __launch_bounds__(QNT) void k_unique_compact(
    const uint64_t* __restrict__ in, uint64_t n, uint64_t* __restrict__ out,
    uint64_t* __restrict__ status, uint32_t* __restrict__ tile_counter, uint32_t epoch,
    unsigned long long* __restrict__ out_count, uint32_t* __restrict__ err) {
  constexpr int TILE = QNT * UITEMS;
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_tmp[QNT / 64];
  __shared__ uint64_t s_excl;
  if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  if (tile >= gridDim.x) return;
  const uint64_t first = tile * TILE + (uint64_t)threadIdx.x * UITEMS;
  uint32_t keep = 0, cnt = 0;
#pragma unroll
  for (int x = 0; x < UITEMS; ++x) {
    const uint64_t e = first + x;
    if (e < n && (e == 0 || in[e] != in[e - 1])) {
      keep |= 1u << x;
      ++cnt;
    }
  }
  uint32_t total;
  const uint32_t texcl = block_excl_scan<QNT>(cnt, s_tmp, &total);
  if (threadIdx.x == 0) s_excl = lb_exclusive(status, tile, 1, epoch, total, err);
  __syncthreads();
  uint64_t pos = s_excl + texcl;
#pragma unroll
  for (int x = 0; x < UITEMS; ++x)
    if (keep & (1u << x)) out[pos++] = in[first + x];
  if (threadIdx.x == 0 && tile == gridDim.x - 1) *out_count = s_excl + total;
}

// ------------------------------------------------------------------ join

// lower bound of hash h in a[lo, hi) (elements compared by e >> idbits)
__device__ __forceinline__ uint32_t lower_bound_hash(const uint64_t* a, uint32_t lo, uint32_t hi,
                                                     uint64_t h, uint32_t idbits) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((a[mid] >> idbits) < h)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// First index in (lb, m] whose hash differs from a[lb]'s (== h), by galloping
// then a binary search of the last step.
__device__ __forceinline__ uint32_t run_end_hash(const uint64_t* a, uint32_t lb, uint32_t m,
                                                 uint64_t h, uint32_t idbits) {
  uint32_t eq = lb, step = 1, hi;
  while (true) {
    const uint32_t pr = eq + step;
    if (pr >= m || pr < eq) {
      hi = m;
      break;
    }
    if ((a[pr] >> idbits) != h) {
      hi = pr;
      break;
    }
    eq = pr;
    step <<= 1;
  }
  uint32_t lo = eq + 1;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if ((a[mid] >> idbits) == h)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <int CAP>
__global__ __launch_bounds__(QNT) void k_join_seg(
    const uint64_t* __restrict__ Er, const uint32_t* __restrict__ rseg_start,
    const uint32_t* __restrict__ rseg_end, const uint64_t* __restrict__ Eq,
    const uint32_t* __restrict__ qseg_start, const uint32_t* __restrict__ qseg_end,
    uint32_t idbits, uint32_t lds_min_q, ShardOut out) {
  __shared__ uint64_t s_r[CAP];
  const uint32_t v = blockIdx.x;
  const uint32_t qs = qseg_start[v], qe = qseg_end[v];
  if (qs == qe) return;
  const uint32_t rs = rseg_start[v], re = rseg_end[v];
  if (rs == re) return;
  const uint32_t m = re - rs;
  const bool use_lds = (qe - qs) >= lds_min_q && m <= (uint32_t)CAP;
  if (use_lds) {
    for (uint32_t x = threadIdx.x; x < m; x += QNT) s_r[x] = Er[rs + x];
    __syncthreads();
  }
  const uint64_t idmask = (1ull << idbits) - 1;
  const uint32_t lane = threadIdx.x & 63u;
  for (uint32_t c0 = qs; c0 < qe; c0 += QNT) {
    const uint32_t p = c0 + threadIdx.x;
    uint32_t lb = 0, cnt = 0;
    uint64_t eq = 0;
    if (p < qe) {
      eq = Eq[p];
      const uint64_t h = eq >> idbits;
      const uint64_t* a = use_lds ? s_r : Er + rs;
      lb = lower_bound_hash(a, 0, m, h, idbits);
      if (lb < m && (a[lb] >> idbits) == h) cnt = run_end_hash(a, lb, m, h, idbits) - lb;
    }
    // one reservation per wave with matches, in the wave's own shard; the
    // wave writes its matches together (slot t belongs to the lane whose
    // inclusive count first exceeds t)
    const uint64_t incl = wave_incl_scan((uint64_t)cnt);
    const uint64_t wtot = __shfl(incl, 63, 64);
    if (wtot) {
      const uint32_t sel = blockIdx.x * (QNT / 64) + (threadIdx.x >> 6);
      ShardResv r{0, 0};
      if (lane == 63u) r = shard_reserve(out, sel, wtot);
      r.pos = __shfl(r.pos, 63, 64);
      r.obase = __shfl(r.obase, 63, 64);
      for (uint64_t t0 = 0; t0 < wtot; t0 += 64) {
        const uint64_t t = t0 + lane;
        uint32_t lo = 0, hi = 63;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (__shfl(incl, (int)mid, 64) <= t)
            lo = mid + 1;
          else
            hi = mid;
        }
        const uint32_t olb = __shfl(lb, (int)lo, 64);
        const uint64_t oex = __shfl(incl, (int)lo, 64) - __shfl((uint64_t)cnt, (int)lo, 64);
        const uint64_t oq = __shfl(eq, (int)lo, 64);
        if (t < wtot) {
          const uint32_t x = olb + (uint32_t)(t - oex);
          const uint64_t er = use_lds ? s_r[x] : Er[rs + x];
          shard_put(out, sel, r, t, ((oq & idmask) << 32) | (er & idmask));
        }
      }
    }
  }
}

// ------------------------------------------------------------------ weighted verify

// Minimum-cost global alignment of a and b with substitution costs sub[20][20]
// and a fixed indel cost, by the full dynamic programme (rows kept in
// registers: both strings have at most 24 residues).
__device__ __forceinline__ uint32_t weighted_keys(u128 a, u128 b, const uint8_t* sub,
                                                  uint32_t indel) {
  const uint32_t la = key_len(a), lb = key_len(b);
  uint32_t row[KEY_MAX_LEN + 1];
#pragma unroll
  for (int y = 0; y <= KEY_MAX_LEN; ++y) row[y] = (uint32_t)y * indel;
  for (uint32_t x = 1; x <= la; ++x) {
    const uint32_t ca = key_residue(a, (int)x - 1);
    uint32_t diag = row[0];
    row[0] = x * indel;
#pragma unroll
    for (int y = 1; y <= KEY_MAX_LEN; ++y) {
      if ((uint32_t)y <= lb) {
        const uint32_t cb = key_residue(b, y - 1);
        const uint32_t up = row[y];
        uint32_t best = diag + sub[ca * 20 + cb];
        const uint32_t del = up + indel, ins = row[y - 1] + indel;
        best = del < best ? del : best;
        best = ins < best ? ins : best;
        diag = up;
        row[y] = best;
      }
    }
  }
  uint32_t res = 0;
#pragma unroll
  for (int y = 0; y <= KEY_MAX_LEN; ++y)
    if ((uint32_t)y == lb) res = row[y];
  return res;
}

__device__ __forceinline__ uint32_t lev_small(u128 a, u128 b) {
  // unit-cost distance by the same programme (used only for the k filter)
  const uint32_t la = key_len(a), lb = key_len(b);
  uint32_t row[KEY_MAX_LEN + 1];
#pragma unroll
  for (int y = 0; y <= KEY_MAX_LEN; ++y) row[y] = (uint32_t)y;
  for (uint32_t x = 1; x <= la; ++x) {
    const uint32_t ca = key_residue(a, (int)x - 1);
    uint32_t diag = row[0];
    row[0] = x;
#pragma unroll
    for (int y = 1; y <= KEY_MAX_LEN; ++y) {
      if ((uint32_t)y <= lb) {
        const uint32_t cb = key_residue(b, y - 1);
        const uint32_t up = row[y];
        uint32_t best = diag + (ca == cb ? 0u : 1u);
        const uint32_t del = up + 1, ins = row[y - 1] + 1;
        best = del < best ? del : best;
        best = ins < best ? ins : best;
        diag = up;
        row[y] = best;
      }
    }
  }
  uint32_t res = 0;
#pragma unroll
  for (int y = 0; y <= KEY_MAX_LEN; ++y)
    if ((uint32_t)y == lb) res = row[y];
  return res;
}

constexpr int WITEMS = 4;

__global__ __launch_bounds__(QNT) void k_verify_weighted(
    const uint64_t* __restrict__ cand, uint64_t c, const u128* __restrict__ sa,
    const u128* __restrict__ sb, int k, const uint8_t* __restrict__ subst, uint32_t indel,
    uint32_t max_score, uint32_t* __restrict__ oi, uint32_t* __restrict__ oj,
    uint8_t* __restrict__ od, uint64_t* __restrict__ status, uint32_t* __restrict__ tile_counter,
    uint32_t epoch, unsigned long long* __restrict__ out_count, uint32_t* __restrict__ err) {
  constexpr int TILE = QNT * WITEMS;
  __shared__ uint8_t s_sub[400];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_tmp[QNT / 64];
  __shared__ uint64_t s_excl;
  for (int x = threadIdx.x; x < 400; x += QNT) s_sub[x] = subst[x];
  if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
  __syncthreads();
  const uint64_t tile = s_tile;
  if (tile >= gridDim.x) return;
  const uint64_t first = tile * TILE + (uint64_t)threadIdx.x * WITEMS;
  uint32_t keepmask = 0, cnt = 0;
  uint8_t score[WITEMS];
#pragma unroll
  for (int x = 0; x < WITEMS; ++x) {
    const uint64_t e = first + x;
    score[x] = 0;
    if (e < c) {
      const uint64_t v = cand[e];
      if (e == 0 || cand[e - 1] != v) {
        const u128 a = sa[v >> 32], b = sb[(uint32_t)v];
        const int la = (int)key_len(a), lb = (int)key_len(b);
        if (abs(la - lb) <= k && lev_small(a, b) <= (uint32_t)k) {
          const uint32_t s = weighted_keys(a, b, s_sub, indel);
          if (s <= max_score) {
            keepmask |= 1u << x;
            score[x] = (uint8_t)(s > 255u ? 255u : s);
            ++cnt;
          }
        }
      }
    }
  }
  uint32_t total;
  const uint32_t texcl = block_excl_scan<QNT>(cnt, s_tmp, &total);
  if (threadIdx.x == 0) s_excl = lb_exclusive(status, tile, 1, epoch, total, err);
  __syncthreads();
  uint64_t pos = s_excl + texcl;
#pragma unroll
  for (int x = 0; x < WITEMS; ++x) {
    if (keepmask & (1u << x)) {
      const uint64_t v = cand[first + x];
      oi[pos] = (uint32_t)(v >> 32);
      oj[pos] = (uint32_t)v;
      od[pos] = score[x];
      ++pos;
    }
  }
  if (threadIdx.x == 0 && tile == gridDim.x - 1) *out_count = s_excl + total;
}

// ------------------------------------------------------------------ per-set slices

// bounds[s] = first result index whose query id is >= set_base[s] (s <= nsets,
// set_base[nsets] = total queries); the result's query ids are ascending.
__global__ void k_set_ranges(const uint32_t* __restrict__ qi, uint64_t n,
                             const unsigned long long* __restrict__ n_dev,
                             const uint32_t* __restrict__ set_base, uint32_t nb,
                             uint64_t* __restrict__ bounds) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nb) return;
  const uint32_t key = set_base[s];
  uint64_t lo = 0, hi = n_dev ? min(n, (uint64_t)*n_dev) : n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (qi[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  bounds[s] = lo;
}

__global__ void k_slice_rebase(const uint32_t* __restrict__ qi, const uint32_t* __restrict__ rj,
                               const uint8_t* __restrict__ d, uint64_t lo, uint64_t n,
                               int64_t shift, uint32_t* __restrict__ oi,
                               uint32_t* __restrict__ oj, uint8_t* __restrict__ od) {
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (uint64_t)gridDim.x * blockDim.x) {
    oi[t] = (uint32_t)((int64_t)qi[lo + t] + shift);
    oj[t] = rj[lo + t];
    od[t] = d[lo + t];
  }
}

}  // namespace sdk

namespace sd {

uint64_t unique_tile() { return (uint64_t)sdk::QNT * sdk::UITEMS; }

void launch_unique_compact(const uint64_t* in, uint64_t n, uint64_t* out, uint64_t* status,
                           uint32_t* tile_counter, uint32_t epoch, unsigned long long* out_count,
                           uint32_t* err, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_unique_compact, dim3((unsigned)((n + unique_tile() - 1) / unique_tile())),
                     dim3(sdk::QNT), 0, s, in, n, out, status, tile_counter, epoch, out_count, err);
}

constexpr int JOIN_CAP = 4096;
int join_cap() { return JOIN_CAP; }

void launch_join_seg(const uint64_t* Er, const uint32_t* rseg_start, const uint32_t* rseg_end,
                     const uint64_t* Eq, const uint32_t* qseg_start, const uint32_t* qseg_end,
                     uint32_t nseg, uint32_t idbits, uint32_t lds_min_q, const ShardArgs& a,
                     hipStream_t s) {
  if (!nseg) return;
  const ShardOut out{a.base, a.region, a.over, a.over_cap, a.counter};
  hipLaunchKernelGGL(sdk::k_join_seg<JOIN_CAP>, dim3(nseg), dim3(sdk::QNT), 0, s, Er, rseg_start,
                     rseg_end, Eq, qseg_start, qseg_end, idbits, lds_min_q, out);
}

uint64_t weighted_tile() { return (uint64_t)sdk::QNT * sdk::WITEMS; }

void launch_verify_weighted(const uint64_t* cand, uint64_t c, const u128* sa, const u128* sb,
                            int k, const uint8_t* subst, uint32_t indel, uint32_t max_score,
                            uint32_t* oi, uint32_t* oj, uint8_t* od, uint64_t* status,
                            uint32_t* tile_counter, uint32_t epoch, unsigned long long* out_count,
                            uint32_t* err, hipStream_t s) {
  if (!c) return;
  hipLaunchKernelGGL(sdk::k_verify_weighted,
                     dim3((unsigned)((c + weighted_tile() - 1) / weighted_tile())), dim3(sdk::QNT),
                     0, s, cand, c, sa, sb, k, subst, indel, max_score, oi, oj, od, status,
                     tile_counter, epoch, out_count, err);
}

void launch_set_ranges(const uint32_t* qi, uint64_t n, const uint32_t* set_base, uint32_t nb,
                       uint64_t* bounds, hipStream_t s, const unsigned long long* n_dev) {
  if (!nb) return;
  hipLaunchKernelGGL(sdk::k_set_ranges, dim3((nb + 255) / 256), dim3(256), 0, s, qi, n, n_dev,
                     set_base, nb, bounds);
}

void launch_slice_rebase(const uint32_t* qi, const uint32_t* rj, const uint8_t* d, uint64_t lo,
                         uint64_t n, int64_t shift, uint32_t* oi, uint32_t* oj, uint8_t* od,
                         hipStream_t s) {
  if (!n) return;
  uint64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(sdk::k_slice_rebase, dim3((unsigned)g), dim3(256), 0, s, qi, rj, d, lo, n,
                     shift, oi, oj, od);
}

}  // namespace sd
