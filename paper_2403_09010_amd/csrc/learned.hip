// Learned index over a reference deletion index sorted by the exact 128-bit
// key: a model that can change the speed of a lookup and never its result.
//
// The model predicts a key's position in the sorted keys in three steps:
//   coordinate  a factorised residue model (per length L and position t, the
//               frequency of each residue, fitted by counting a sample of the
//               keys) maps the key to its arithmetic-coding coordinate in
//               [0, 1): the length's cumulative share, then for each of the
//               first 12 residues the cumulative frequency of the smaller
//               residues scaled by the probability of the prefix before it.
//               The coordinate is monotone in key order and would be the
//               rank fraction if residues were independent given (L, t).
//   stage 1     an FP32 MLP 1 -> H (tanh) -> 1 maps the coordinate to the
//               rank fraction (trained by gradient descent on the device);
//               its output selects one of F leaves
//   stage 2     per leaf, the line through the leaf's first and last key
//               over the FP64 coordinate predicts the position
// Each leaf stores its exact worst error eps over every indexed key that the
// model sends to it, computed after training by the same device functions
// the lookups call, so an equality lookup that searches [p - eps, p + eps]
// finds exactly what a binary search over the whole array finds.
//
// Kernels
//   k_interleave       (hi, lo) word arrays -> one 16-byte key per entry
//   k_coord_counts     residue counts per (L, t) and length counts of a sample
//   k_train_sample     (coordinate, rank / n) samples at evenly spaced ranks
//   k_mlp_grad         forward and backward of the mean squared error over
//                      the samples, one hidden unit per lane; one partial
//                      gradient per block
//   k_grad_reduce      partial gradients summed in block order
//   k_adam_step        the same sum, then one Adam update (device step count,
//                      so a captured graph of training steps can be replayed);
//                      the parameters with the lowest loss seen are kept
//   k_adam_best        those parameters become the model
//   k_leaf_range       first and last position of the keys of each leaf
//   k_leaf_fit         the leaf lines
//   k_leaf_eps         exact per-leaf worst error
//   k_probe            query variants generated on the fly and looked up in
//                      the sorted keys (learned window or whole array),
//                      (query, reference) candidates emitted
#include "sd_device.h"
#include "sd_internal.h"

namespace sdk {

constexpr int H = SD_MLP_HIDDEN;
constexpr int NP = SD_MLP_PARAMS;  // w1[H] b1[H] w2[H] b2
constexpr int LNT = 256;
constexpr int NL = KEY_MAX_LEN + 1;  // key lengths 0 .. 24
constexpr int NR = 20;               // residue codes

struct Leaf {  // 32 bytes: one load per probe
  double slope, cmin;
  uint32_t lo, hi, eps, count;  // first and last position, error bound, keys sent here
};
static_assert(sizeof(Leaf) == 32, "leaf record size");

// Residues that enter the coordinate: later ones refine it below the
// resolution that separates the indexed keys (about 3.6 bits of entropy per
// residue), and a fixed count lets every table load issue at once.
constexpr int COORD_RES = 12;
constexpr int ROW = COORD_RES * NR;  // table entries per key length

// The coordinate model: lencum[L] = share of keys shorter than L
// (lencum[25] = 1); for lengths lmin..lmax that occur in the index,
// rows[(L - lmin) * ROW + t * 20 + c] = (cumulative frequency of residues
// below c, frequency of c) at position t < 12 of length-L keys. FP32 table
// entries keep the rows of every length within 48 KB, so a lookup kernel
// holds them in LDS; the coordinate itself is accumulated in FP64.
struct Coord {
  double lencum[NL + 1];
  uint32_t lmin, lmax;
  float2 rows[NL * ROW];
};

// Not inlined: the build and the lookups must run the same instructions
// (the build reads the tables from global memory, a lookup from LDS).
__device__ __noinline__ double key_coord(const double* __restrict__ lencum,
                                         const float2* __restrict__ rows, uint32_t lmin,
                                         uint32_t lmax, u128 key) {
  const uint32_t L = key_len(key);
  double x = 0.0;
  if (L >= lmin && L <= lmax) {
    const float2* row = rows + (size_t)(L - lmin) * ROW;
    float2 e[COORD_RES];
#pragma unroll
    for (int t = 0; t < COORD_RES; ++t)
      e[t] = (uint32_t)t < L ? row[t * NR + key_residue(key, t)] : make_float2(0.0f, 1.0f);
    double w = 1.0;
#pragma unroll
    for (int t = 0; t < COORD_RES; ++t) {
      x = fma(w, (double)e[t].x, x);
      w = w * (double)e[t].y;
    }
  }
  return fma(lencum[L + 1] - lencum[L], x, lencum[L]);
}

__device__ __forceinline__ double key_coord(const Coord* __restrict__ cm, u128 key) {
  return key_coord(cm->lencum, cm->rows, cm->lmin, cm->lmax, key);
}

__device__ __noinline__ float mlp_forward(const float* __restrict__ p, float x) {
  float y = p[3 * H];
#pragma unroll 4
  for (int j = 0; j < H; ++j) y += p[2 * H + j] * tanhf(p[j] * x + p[H + j]);
  return y;
}

__device__ __noinline__ uint32_t leaf_of(const float* __restrict__ p, uint32_t nleaves, double c) {
  const float f = mlp_forward(p, (float)c) * (float)nleaves;
  if (!(f > 0.0f)) return 0;  // NaN included
  if (f >= (float)nleaves) return nleaves - 1;
  return (uint32_t)f;
}

// For an indexed key the prediction lies in [lo, hi] of its leaf; keys that
// are not indexed may land anywhere, so the value is clamped before the
// integer conversion.
__device__ __noinline__ int64_t leaf_predict(const Leaf& f, double c) {
  const double p = floor((double)f.lo + f.slope * (c - f.cmin));
  return (int64_t)fmin(fmax(p, -1.0e18), 1.0e18);
}

// ------------------------------------------------------------------ layout

__global__ __launch_bounds__(LNT) void k_interleave(const uint64_t* __restrict__ hi,
                                                    const uint64_t* __restrict__ lo, uint64_t n,
                                                    u128* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * LNT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * LNT)
    out[i] = ((u128)hi[i] << 64) | lo[i];
}

// ------------------------------------------------------------------ model fit

// counts[(L * 24 + t) * 20 + c] and counts[NL * 24 * 20 + L] over the S keys
// at ranks s * n / S
__global__ __launch_bounds__(LNT) void k_coord_counts(const u128* __restrict__ keys, uint64_t n,
                                                      uint32_t S, uint32_t* __restrict__ counts) {
  constexpr int NT = NL * KEY_MAX_LEN * NR;
  __shared__ uint32_t s_c[NT + NL];
  for (int x = threadIdx.x; x < NT + NL; x += LNT) s_c[x] = 0;
  __syncthreads();
  for (uint32_t s = blockIdx.x * LNT + threadIdx.x; s < S; s += gridDim.x * LNT) {
    const u128 key = keys[(uint64_t)s * n / S];
    const uint32_t L = key_len(key);
    atomicAdd(&s_c[NT + L], 1u);
    for (uint32_t t = 0; t < L; ++t)
      atomicAdd(&s_c[(L * KEY_MAX_LEN + t) * NR + key_residue(key, (int)t)], 1u);
  }
  __syncthreads();
  for (int x = threadIdx.x; x < NT + NL; x += LNT)
    if (s_c[x]) atomicAdd(&counts[x], s_c[x]);
}

__global__ __launch_bounds__(LNT) void k_train_sample(const u128* __restrict__ keys, uint64_t n,
                                                      uint32_t S, const Coord* __restrict__ cm,
                                                      float* __restrict__ x, float* __restrict__ y) {
  const uint32_t s = blockIdx.x * LNT + threadIdx.x;
  if (s >= S) return;
  const uint64_t i = (uint64_t)s * n / S;
  x[s] = (float)key_coord(cm, keys[i]);
  y[s] = (float)((double)i / (double)n);
}

// partial[b * (NP + 1) + t]: block b's sum of d(loss)/d(param t) for t < NP
// and of the loss for t = NP, loss = mean over n of (f(x) - y)^2.
// One hidden unit per lane: a group of H = 32 lanes takes one sample at a
// time, the output is a butterfly sum over the group, and each lane
// accumulates the gradient of its own unit's three parameters.
static_assert(H == 32, "one hidden unit per lane of a half wave");
constexpr int GROUPS = LNT / H;

__global__ __launch_bounds__(LNT) void k_mlp_grad(const float* __restrict__ p,
                                                  const float* __restrict__ x,
                                                  const float* __restrict__ y, uint32_t n,
                                                  float* __restrict__ partial) {
  __shared__ float s_red[GROUPS][3 * H + 2];
  const uint32_t j = threadIdx.x % H, grp = threadIdx.x / H;
  const float w1 = p[j], b1 = p[H + j], w2 = p[2 * H + j], b2 = p[3 * H];
  const float inv_n = 1.0f / (float)n;
  float gw1 = 0.0f, gb1 = 0.0f, gw2 = 0.0f, gb2 = 0.0f, loss = 0.0f;
  for (uint32_t s = blockIdx.x * GROUPS + grp; s < n; s += gridDim.x * GROUPS) {
    const float xs = x[s];
    const float h = tanhf(w1 * xs + b1);
    float out = w2 * h;
#pragma unroll
    for (int o = H / 2; o > 0; o >>= 1) out += __shfl_xor(out, o, H);
    const float err = out + b2 - y[s];
    const float go = 2.0f * err * inv_n;  // d(loss)/d(out)
    const float dz = go * w2 * (1.0f - h * h);
    gw1 += dz * xs;
    gb1 += dz;
    gw2 += go * h;
    gb2 += go;
    loss += err * err * inv_n;
  }
  s_red[grp][j] = gw1;
  s_red[grp][H + j] = gb1;
  s_red[grp][2 * H + j] = gw2;
  if (j == 0) {
    s_red[grp][3 * H] = gb2;
    s_red[grp][3 * H + 1] = loss;
  }
  __syncthreads();
  for (int t = threadIdx.x; t <= NP; t += LNT) {
    float v = 0.0f;
#pragma unroll
    for (int q = 0; q < GROUPS; ++q) v += s_red[q][t];
    partial[(uint64_t)blockIdx.x * (NP + 1) + t] = v;
  }
}

// Sum of the block partials of entry t in block order; the loads are issued
// eight at a time so the serial chain is of additions, not of memory latency.
__device__ __forceinline__ float sum_partials(const float* __restrict__ partial, uint32_t nblocks,
                                              int t) {
  float v = 0.0f;
  uint32_t b = 0;
  for (; b + 8 <= nblocks; b += 8) {
    float q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] = partial[(uint64_t)(b + u) * (NP + 1) + t];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += q[u];
  }
  for (; b < nblocks; ++b) v += partial[(uint64_t)b * (NP + 1) + t];
  return v;
}

__global__ void k_grad_reduce(const float* __restrict__ partial, uint32_t nblocks,
                              float* __restrict__ out) {
  const int t = threadIdx.x;
  if (t <= NP) out[t] = sum_partials(partial, nblocks, t);
}

// Adam state: state[0] = steps taken, [1, 1 + NP) first moments,
// [1 + NP, 1 + 2 NP) second moments, [1 + 2 NP] the lowest loss seen,
// [2 + 2 NP, 2 + 3 NP) the parameters that had it.
constexpr int ADAM_STATE = 3 * NP + 2;

// One Adam step from the block partials. The partials hold the gradient and
// loss of the current parameters: if that loss is the lowest so far, the
// parameters are kept before they are updated. With update == 0 only that
// bookkeeping runs (the evaluation after the last step). loss_out[step]
// receives the loss of each step's gradient pass.
__global__ void k_adam_step(float* __restrict__ p, float* __restrict__ state,
                            const float* __restrict__ partial, uint32_t nblocks, float lr,
                            int update, float* __restrict__ loss_out, uint32_t loss_cap) {
  __shared__ float s_g[NP + 1];
  __shared__ int s_better;
  const int t = threadIdx.x;
  const float step = state[0] + 1.0f;
  if (t <= NP) s_g[t] = sum_partials(partial, nblocks, t);
  __syncthreads();
  if (t == 0) {
    const float loss = s_g[NP];
    const uint32_t si = (uint32_t)step - 1u;
    if (update && si < loss_cap) loss_out[si] = loss;
    const float best = state[1 + 2 * NP];
    s_better = (state[0] == 0.0f || loss < best) ? 1 : 0;  // NaN never counts as better
    if (s_better) state[1 + 2 * NP] = loss;
  }
  __syncthreads();
  if (t < NP) {
    if (s_better) state[2 + 2 * NP + t] = p[t];
    if (update) {
      const float b1 = 0.9f, b2 = 0.999f, gsum = s_g[t];
      const float m = b1 * state[1 + t] + (1.0f - b1) * gsum;
      const float v = b2 * state[1 + NP + t] + (1.0f - b2) * gsum * gsum;
      state[1 + t] = m;
      state[1 + NP + t] = v;
      const float mh = m / (1.0f - powf(b1, step)), vh = v / (1.0f - powf(b2, step));
      p[t] -= lr * mh / (sqrtf(vh) + 1e-8f);
    }
  }
  __syncthreads();  // every thread has read state[0]
  if (t == 0 && update) state[0] = step;
}

// The parameters with the lowest loss seen become the model.
__global__ void k_adam_best(float* __restrict__ p, const float* __restrict__ state) {
  const int t = threadIdx.x;
  if (t < NP) p[t] = state[2 + 2 * NP + t];
}

// ------------------------------------------------------------------ leaves

__global__ void k_leaf_init(Leaf* __restrict__ leaves, uint32_t nleaves) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nleaves) leaves[l] = Leaf{0.0, 0.0, 0xFFFFFFFFu, 0u, 0u, 0u};
}

__global__ __launch_bounds__(LNT) void k_leaf_range(const u128* __restrict__ keys, uint64_t n,
                                                    const Coord* __restrict__ cm,
                                                    const float* __restrict__ p, uint32_t nleaves,
                                                    Leaf* __restrict__ leaves) {
  for (uint64_t i = (uint64_t)blockIdx.x * LNT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * LNT) {
    const uint32_t l = leaf_of(p, nleaves, key_coord(cm, keys[i]));
    // The active lanes of a wave are a prefix holding consecutive positions,
    // and sorted keys usually share a leaf: then the first active lane
    // records the whole run with one update of each field.
    const uint64_t active = __ballot(true);
    const uint32_t leader = (uint32_t)__ffsll((long long)active) - 1u;
    const uint32_t l0 = __shfl(l, (int)leader, 64);
    if (__ballot(l == l0) == active) {
      if (lane_id() == leader) {
        const uint32_t run = (uint32_t)__popcll(active);
        atomicMin(&leaves[l].lo, (uint32_t)i);
        atomicMax(&leaves[l].hi, (uint32_t)i + run - 1u);
        atomicAdd(&leaves[l].count, run);
      }
    } else {
      atomicMin(&leaves[l].lo, (uint32_t)i);
      atomicMax(&leaves[l].hi, (uint32_t)i);
      atomicAdd(&leaves[l].count, 1u);
    }
  }
}

__global__ void k_leaf_fit(const u128* __restrict__ keys, const Coord* __restrict__ cm,
                           uint32_t nleaves, Leaf* __restrict__ leaves) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nleaves) return;
  Leaf f = leaves[l];
  if (f.lo > f.hi) {  // empty leaf
    f.slope = 0.0;
    f.cmin = 0.0;
  } else {
    const double a = key_coord(cm, keys[f.lo]), b = key_coord(cm, keys[f.hi]);
    f.cmin = a;
    f.slope = b > a ? (double)(f.hi - f.lo) / (b - a) : 0.0;
  }
  f.eps = 0;
  leaves[l] = f;
}

__global__ __launch_bounds__(LNT) void k_leaf_eps(const u128* __restrict__ keys, uint64_t n,
                                                  const Coord* __restrict__ cm,
                                                  const float* __restrict__ p, uint32_t nleaves,
                                                  Leaf* __restrict__ leaves) {
  for (uint64_t i = (uint64_t)blockIdx.x * LNT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * LNT) {
    const double c = key_coord(cm, keys[i]);
    const uint32_t l = leaf_of(p, nleaves, c);
    const int64_t d = leaf_predict(leaves[l], c) - (int64_t)i;
    const uint64_t e64 = (uint64_t)(d < 0 ? -d : d);
    uint32_t e = (uint32_t)(e64 > 0xFFFFFFFFull ? 0xFFFFFFFFull : e64);
    // The active lanes are a prefix of the wave and usually share a leaf:
    // then a shift-down maximum leaves the wave's maximum in the first lane,
    // which makes the only atomic.
    const uint64_t active = __ballot(true);
    const uint32_t leader = (uint32_t)__ffsll((long long)active) - 1u;
    const uint32_t l0 = __shfl(l, (int)leader, 64);
    if (__ballot(l == l0) == active) {
      const uint32_t lane = lane_id();
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t other = __shfl_down(e, o, 64);
        if (lane + (uint32_t)o < 64u && ((active >> (lane + (uint32_t)o)) & 1ull))
          e = other > e ? other : e;
      }
      if (lane == leader) atomicMax(&leaves[l].eps, e);
    } else {
      atomicMax(&leaves[l].eps, e);
    }
  }
}

// ------------------------------------------------------------------ probe

// First index in (lb, b] whose key differs from keys[lb] == key (or b):
// galloping from lb, then a binary search of the last step, so a run of c
// equal keys costs O(log c) reads instead of c.
__device__ __forceinline__ uint64_t run_end(const u128* __restrict__ keys, uint64_t lb,
                                            uint64_t b, u128 key) {
  uint64_t eq = lb, step = 1, hi;
  while (true) {
    const uint64_t pr = eq + step;
    if (pr >= b) {
      hi = b;
      break;
    }
    if (keys[pr] != key) {
      hi = pr;
      break;
    }
    eq = pr;
    step <<= 1;
  }
  uint64_t lo = eq + 1;  // keys[eq] == key; the first difference is in [lo, hi]
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (keys[mid] == key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

constexpr int PB_SEQS = 64;

// One workgroup per 64 query sequences; each wave walks the variants of its
// own 16 of them, 64 at a time, with no block-wide barrier after the start:
// a lane generates its variant, predicts its position (coordinate tables in
// LDS) and binary-searches the model's window (or the whole array); the
// wave reserves output slots for its matches with one atomic and writes them
// together. Dynamic LDS: lencum (26 doubles) then the used table rows.
__global__ __launch_bounds__(LNT) void k_probe(
    const u128* __restrict__ qseq, const uint64_t* __restrict__ qvoff, uint64_t nq,
    const u128* __restrict__ keys, const uint32_t* __restrict__ kid, uint64_t n, int learned,
    const Coord* __restrict__ cm, const float* __restrict__ p, uint32_t nleaves,
    const Leaf* __restrict__ leaves, ShardOut out, unsigned long long* __restrict__ steps_total) {
  extern __shared__ __align__(16) unsigned char s_dyn[];
  __shared__ uint64_t s_off[PB_SEQS + 1];
  __shared__ u128 s_seq[PB_SEQS];
  double* s_lencum = reinterpret_cast<double*>(s_dyn);
  float2* s_rows = reinterpret_cast<float2*>(s_dyn + (NL + 1) * sizeof(double));
  const uint64_t s0 = (uint64_t)blockIdx.x * PB_SEQS;
  const uint32_t ns = (uint32_t)min<uint64_t>(PB_SEQS, nq - s0);
  for (uint32_t x = threadIdx.x; x <= ns; x += LNT) s_off[x] = qvoff[s0 + x];
  for (uint32_t x = threadIdx.x; x < ns; x += LNT) s_seq[x] = qseq[s0 + x];
  const uint32_t lmin = cm->lmin, lmax = cm->lmax;
  if (learned) {
    for (uint32_t x = threadIdx.x; x <= (uint32_t)NL; x += LNT) s_lencum[x] = cm->lencum[x];
    const uint32_t nrow = lmax >= lmin ? (lmax - lmin + 1) * ROW : 0;
    for (uint32_t x = threadIdx.x; x < nrow; x += LNT) s_rows[x] = cm->rows[x];
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  constexpr uint32_t PER_WAVE = PB_SEQS / (LNT / 64);
  const uint32_t xa = min(w * PER_WAVE, ns), xb = min(xa + PER_WAVE, ns);
  const uint64_t wa = s_off[xa], wb = s_off[xb];
  uint32_t steps = 0;
  for (uint64_t r0 = wa; r0 < wb; r0 += 64) {
    const uint64_t g = r0 + lane;
    uint64_t lb = 0;
    uint32_t cnt = 0, q = 0;
    if (g < wb) {
      uint32_t lo = xa, hi = xb - 1;  // the sequence whose variants hold g
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= g)
          lo = mid;
        else
          hi = mid - 1;
      }
      q = (uint32_t)(s0 + lo);
      const u128 key = key_variant(s_seq[lo], (uint32_t)(g - s_off[lo]));
      uint64_t a = 0, b = n;    // the window; b also bounds the run of equal keys
      uint64_t sa = 0, sb = n;  // the lower bound lies in [sa, sb]
      if (learned) {
        const double c = key_coord(s_lencum, s_rows, lmin, lmax, key);
        const Leaf f = leaves[leaf_of(p, nleaves, c)];
        int64_t pr = 0;
        if (f.lo > f.hi) {
          b = 0;  // no indexed key is sent to this leaf, so the key is absent
        } else {
          pr = leaf_predict(f, c);
          const int64_t ua = pr - (int64_t)f.eps, ub = pr + (int64_t)f.eps + 1;
          a = ua < 0 ? 0 : (uint64_t)ua;
          b = ub < 0 ? 0 : ((uint64_t)ub > n ? n : (uint64_t)ub);
          if (a > b) a = b;
        }
        sa = a;
        sb = b;
      }
      while (sa < sb) {  // lower bound of key in [sa, sb]
        const uint64_t mid = (sa + sb) >> 1;
        ++steps;
        if (keys[mid] < key)
          sa = mid + 1;
        else
          sb = mid;
      }
      lb = sa;
      if (lb < b && keys[lb] == key) cnt = (uint32_t)(run_end(keys, lb, b, key) - lb);
    }
    // the wave's matches, written together: output slot t belongs to the
    // lane whose inclusive count first exceeds t
    const uint64_t incl = wave_incl_scan((uint64_t)cnt);
    const uint64_t wtot = __shfl(incl, 63, 64);
    if (wtot) {  // one reservation per wave with matches, in the wave's own shard
      const uint32_t sel = blockIdx.x * (LNT / 64) + w;
      ShardResv r{0, 0};
      if (lane == 63) r = shard_reserve(out, sel, wtot);
      r.pos = __shfl(r.pos, 63, 64);
      r.obase = __shfl(r.obase, 63, 64);
      for (uint64_t t0 = 0; t0 < wtot; t0 += 64) {
        const uint64_t t = t0 + lane;
        uint32_t lo = 0, hi = 63;
        while (lo < hi) {  // the same number of steps in every lane
          const uint32_t mid = (lo + hi) >> 1;
          if (__shfl(incl, (int)mid, 64) <= t)
            lo = mid + 1;
          else
            hi = mid;
        }
        const uint64_t olb = __shfl(lb, (int)lo, 64);
        const uint64_t oex = __shfl(incl, (int)lo, 64) - __shfl((uint64_t)cnt, (int)lo, 64);
        const uint32_t oq = __shfl(q, (int)lo, 64);
        if (t < wtot) shard_put(out, sel, r, t, ((uint64_t)oq << 32) | kid[olb + (t - oex)]);
      }
    }
  }
  const uint32_t wsteps = __shfl(wave_incl_scan(steps), 63, 64);
  if (lane == 0 && wsteps) atomicAdd(steps_total, (unsigned long long)wsteps);
}

}  // namespace sdk

namespace sd {

static unsigned grid_for(uint64_t n) {
  uint64_t g = (n + sdk::LNT - 1) / sdk::LNT;
  return (unsigned)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

size_t leaf_bytes() { return sizeof(sdk::Leaf); }
size_t coord_bytes() { return sizeof(sdk::Coord); }
int coord_lengths() { return sdk::NL; }
int coord_res() { return sdk::COORD_RES; }
void coord_offsets(size_t* lmin_off, size_t* rows_off) {
  *lmin_off = offsetof(sdk::Coord, lmin);
  *rows_off = offsetof(sdk::Coord, rows);
}

void launch_interleave(const uint64_t* hi, const uint64_t* lo, uint64_t n, u128* out, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(sdk::k_interleave, dim3(grid_for(n)), dim3(sdk::LNT), 0, s, hi, lo, n, out);
}

void launch_coord_counts(const u128* keys, uint64_t n, uint32_t S, uint32_t* counts,
                         hipStream_t s) {
  if (!S) return;
  uint32_t g = (S + sdk::LNT * 32 - 1) / (sdk::LNT * 32);
  g = g > 512 ? 512 : g;
  hipLaunchKernelGGL(sdk::k_coord_counts, dim3(g), dim3(sdk::LNT), 0, s, keys, n, S, counts);
}

void launch_train_sample(const u128* keys, uint64_t n, uint32_t S, const void* coord, float* x,
                         float* y, hipStream_t s) {
  if (!S) return;
  hipLaunchKernelGGL(sdk::k_train_sample, dim3((S + sdk::LNT - 1) / sdk::LNT), dim3(sdk::LNT), 0, s,
                     keys, n, S, static_cast<const sdk::Coord*>(coord), x, y);
}

uint32_t mlp_grad_blocks(uint32_t n) {
  const uint32_t b = (n + sdk::GROUPS * 64 - 1) / (sdk::GROUPS * 64);
  return b < 1 ? 1 : (b > 128 ? 128 : b);
}

void launch_mlp_grad(const float* p, const float* x, const float* y, uint32_t n, float* partial,
                     hipStream_t s) {
  hipLaunchKernelGGL(sdk::k_mlp_grad, dim3(mlp_grad_blocks(n)), dim3(sdk::LNT), 0, s, p, x, y, n,
                     partial);
}

void launch_grad_reduce(const float* partial, uint32_t nblocks, float* out, hipStream_t s) {
  hipLaunchKernelGGL(sdk::k_grad_reduce, dim3(1), dim3(128), 0, s, partial, nblocks, out);
}

int adam_state_floats() { return sdk::ADAM_STATE; }

void launch_adam_step(float* p, float* state, const float* partial, uint32_t nblocks, float lr,
                      int update, float* loss_out, uint32_t loss_cap, hipStream_t s) {
  hipLaunchKernelGGL(sdk::k_adam_step, dim3(1), dim3(128), 0, s, p, state, partial, nblocks, lr,
                     update, loss_out, loss_cap);
}

void launch_adam_best(float* p, const float* state, hipStream_t s) {
  hipLaunchKernelGGL(sdk::k_adam_best, dim3(1), dim3(128), 0, s, p, state);
}

void launch_leaf_fit_all(const u128* keys, uint64_t n, const void* coord, const float* p,
                         uint32_t nleaves, void* leaves, hipStream_t s) {
  sdk::Leaf* lv = static_cast<sdk::Leaf*>(leaves);
  const sdk::Coord* cm = static_cast<const sdk::Coord*>(coord);
  hipLaunchKernelGGL(sdk::k_leaf_init, dim3((nleaves + 255) / 256), dim3(256), 0, s, lv, nleaves);
  hipLaunchKernelGGL(sdk::k_leaf_range, dim3(grid_for(n)), dim3(sdk::LNT), 0, s, keys, n, cm, p,
                     nleaves, lv);
  hipLaunchKernelGGL(sdk::k_leaf_fit, dim3((nleaves + 255) / 256), dim3(256), 0, s, keys, cm,
                     nleaves, lv);
  hipLaunchKernelGGL(sdk::k_leaf_eps, dim3(grid_for(n)), dim3(sdk::LNT), 0, s, keys, n, cm, p,
                     nleaves, lv);
}

void launch_probe(const u128* qseq, const uint64_t* qvoff, uint64_t nq, const u128* keys,
                  const uint32_t* kid, uint64_t n, int learned, const void* coord,
                  uint32_t coord_lengths_used, const float* p, uint32_t nleaves,
                  const void* leaves, const ShardArgs& a, unsigned long long* steps,
                  hipStream_t s) {
  if (!nq) return;
  const ShardOut out{a.base, a.region, a.over, a.over_cap, a.counter};
  // the learned lookups stage the coordinate rows of lengths lmin..lmax in LDS
  const size_t lds = (sdk::NL + 1) * sizeof(double) +
                     (size_t)coord_lengths_used * sdk::ROW * sizeof(float2);
  hipLaunchKernelGGL(sdk::k_probe, dim3((unsigned)((nq + sdk::PB_SEQS - 1) / sdk::PB_SEQS)),
                     dim3(sdk::LNT), learned ? lds : 0, s, qseq, qvoff, nq, keys, kid, n, learned,
                     static_cast<const sdk::Coord*>(coord), p, nleaves,
                     static_cast<const sdk::Leaf*>(leaves), out, steps);
}

}  // namespace sd
