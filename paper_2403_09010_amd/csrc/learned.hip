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
//                      so a captured graph of training steps can be replayed)
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

// The coordinate model: tab[(L * 24 + t) * 20 + c] = (cumulative frequency of
// residues below c, frequency of c) at position t of length-L keys, and
// lencum[L] = share of keys shorter than L (lencum[25] = 1).
struct Coord {
  double2 tab[NL * KEY_MAX_LEN * NR];
  double lencum[NL + 1];
};

// Residues that enter the coordinate: later ones refine it below the
// resolution that separates the indexed keys (about 3.6 bits of entropy per
// residue), and a fixed count lets every table load issue at once.
constexpr int COORD_RES = 12;

// Not inlined: the build and the lookups must run the same instructions.
__device__ __noinline__ double key_coord(const Coord* __restrict__ cm, u128 key) {
  const uint32_t L = key_len(key);
  const double2* row = cm->tab + (size_t)L * KEY_MAX_LEN * NR;
  double2 e[COORD_RES];
#pragma unroll
  for (int t = 0; t < COORD_RES; ++t)
    e[t] = (uint32_t)t < L ? row[t * NR + key_residue(key, t)] : make_double2(0.0, 1.0);
  double x = 0.0, w = 1.0;
#pragma unroll
  for (int t = 0; t < COORD_RES; ++t) {
    x = fma(w, e[t].x, x);
    w = w * e[t].y;
  }
  return fma(cm->lencum[L + 1] - cm->lencum[L], x, cm->lencum[L]);
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

// state[0] = steps taken, state[1 .. NP] = first moments, state[NP+1 .. 2NP]
// = second moments; loss_out[step] = the loss of the step's gradient pass
__global__ void k_adam_step(float* __restrict__ p, float* __restrict__ state,
                            const float* __restrict__ partial, uint32_t nblocks, float lr,
                            float* __restrict__ loss_out, uint32_t loss_cap) {
  const int t = threadIdx.x;
  const float step = state[0] + 1.0f;
  if (t <= NP) {
    const float gsum = sum_partials(partial, nblocks, t);
    if (t == NP) {
      const uint32_t si = (uint32_t)step - 1u;
      if (si < loss_cap) loss_out[si] = gsum;
    } else {
      const float b1 = 0.9f, b2 = 0.999f;
      const float m = b1 * state[1 + t] + (1.0f - b1) * gsum;
      const float v = b2 * state[1 + NP + t] + (1.0f - b2) * gsum * gsum;
      state[1 + t] = m;
      state[1 + NP + t] = v;
      const float mh = m / (1.0f - powf(b1, step)), vh = v / (1.0f - powf(b2, step));
      p[t] -= lr * mh / (sqrtf(vh) + 1e-8f);
    }
  }
  __syncthreads();  // every thread has read state[0]
  if (t == 0) state[0] = step;
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

constexpr int PB_SEQS = 64;

__global__ __launch_bounds__(LNT) void k_probe(
    const u128* __restrict__ qseq, const uint64_t* __restrict__ qvoff, uint64_t nq,
    const u128* __restrict__ keys, const uint32_t* __restrict__ kid, uint64_t n, int learned,
    const Coord* __restrict__ cm, const float* __restrict__ p, uint32_t nleaves,
    const Leaf* __restrict__ leaves, uint64_t* __restrict__ cand, uint64_t cap,
    unsigned long long* __restrict__ ccount, unsigned long long* __restrict__ steps_total) {
  __shared__ uint64_t s_off[PB_SEQS + 1];
  __shared__ u128 s_seq[PB_SEQS];
  __shared__ uint32_t s_tmp[LNT / 64];
  __shared__ unsigned long long s_base;
  const uint64_t s0 = (uint64_t)blockIdx.x * PB_SEQS;
  const uint32_t ns = (uint32_t)min<uint64_t>(PB_SEQS, nq - s0);
  for (uint32_t x = threadIdx.x; x <= ns; x += LNT) s_off[x] = qvoff[s0 + x];
  for (uint32_t x = threadIdx.x; x < ns; x += LNT) s_seq[x] = qseq[s0 + x];
  __syncthreads();
  const uint64_t g0 = s_off[0], g1 = s_off[ns];
  uint32_t steps = 0;
  for (uint64_t r0 = g0; r0 < g1; r0 += LNT) {
    const uint64_t g = r0 + threadIdx.x;
    uint64_t lb = 0;
    uint32_t cnt = 0, q = 0;
    if (g < g1) {
      uint32_t lo = 0, hi = ns - 1;  // the sequence whose variants hold g
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= g)
          lo = mid;
        else
          hi = mid - 1;
      }
      q = (uint32_t)(s0 + lo);
      const u128 key = key_variant(s_seq[lo], (uint32_t)(g - s_off[lo]));
      uint64_t a = 0, b = n;
      if (learned) {
        const double c = key_coord(cm, key);
        const Leaf f = leaves[leaf_of(p, nleaves, c)];
        if (f.lo > f.hi) {
          b = 0;  // no indexed key is sent to this leaf, so the key is absent
        } else {
          const int64_t pr = leaf_predict(f, c);
          const int64_t wa = pr - (int64_t)f.eps, wb = pr + (int64_t)f.eps + 1;
          a = wa < 0 ? 0 : (uint64_t)wa;
          b = wb < 0 ? 0 : ((uint64_t)wb > n ? n : (uint64_t)wb);
          if (a > b) a = b;
        }
      }
      uint64_t hi_b = b;
      while (a < hi_b) {  // lower bound of key in [a, b)
        const uint64_t mid = (a + hi_b) >> 1;
        ++steps;
        if (keys[mid] < key)
          a = mid + 1;
        else
          hi_b = mid;
      }
      lb = a;
      while (lb + cnt < b && keys[lb + cnt] == key) ++cnt;
    }
    uint32_t total;
    const uint32_t excl = block_excl_scan<LNT>(cnt, s_tmp, &total);
    if (threadIdx.x == 0) s_base = total ? atomicAdd(ccount, (unsigned long long)total) : 0ull;
    __syncthreads();
    uint64_t pos = s_base + excl;
    for (uint32_t x = 0; x < cnt; ++x, ++pos)
      if (pos < cap) cand[pos] = ((uint64_t)q << 32) | kid[lb + x];
    __syncthreads();  // s_base is rewritten by the next round
  }
  uint32_t tot;
  (void)block_excl_scan<LNT>(steps, s_tmp, &tot);
  if (threadIdx.x == 0 && tot) atomicAdd(steps_total, (unsigned long long)tot);
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

void launch_adam_step(float* p, float* state, const float* partial, uint32_t nblocks, float lr,
                      float* loss_out, uint32_t loss_cap, hipStream_t s) {
  hipLaunchKernelGGL(sdk::k_adam_step, dim3(1), dim3(128), 0, s, p, state, partial, nblocks, lr,
                     loss_out, loss_cap);
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
                  const uint32_t* kid, uint64_t n, int learned, const void* coord, const float* p,
                  uint32_t nleaves, const void* leaves, uint64_t* cand, uint64_t cap,
                  unsigned long long* ccount, unsigned long long* steps, hipStream_t s) {
  if (!nq) return;
  hipLaunchKernelGGL(sdk::k_probe, dim3((unsigned)((nq + sdk::PB_SEQS - 1) / sdk::PB_SEQS)),
                     dim3(sdk::LNT), 0, s, qseq, qvoff, nq, keys, kid, n, learned,
                     static_cast<const sdk::Coord*>(coord), p, nleaves,
                     static_cast<const sdk::Leaf*>(leaves), cand, cap, ccount, steps);
}

}  // namespace sd
