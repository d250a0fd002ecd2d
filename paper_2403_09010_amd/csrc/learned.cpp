// Learned reference index: build (exact-key sort, the counted coordinate
// model, device training of the stage-1 MLP, leaf fit with exact error
// bounds) and lookups of query tiles.
//
// The model only narrows where a lookup searches. Every leaf's bound eps is
// the exact worst distance between predicted and true position over all
// indexed keys the model sends to that leaf, computed after training by the
// same device functions the lookups call, so a lookup inside
// [p - eps, p + eps] returns the same reference ids as a binary search over
// all keys. Candidates then go through the same pair sort and verification as
// the hashed index.
//
// Training: full-batch Adam on the mean squared error between the MLP output
// and the rank fraction at evenly spaced ranks. One step is a gradient pass
// (block partials) and an update kernel that sums the partials in a fixed
// order; a chunk of steps is captured once as a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sd_host.h"

namespace sd {

namespace {

constexpr int NP = SD_MLP_PARAMS;
constexpr int H = SD_MLP_HIDDEN;
constexpr int GRAPH_STEPS = 25;  // training steps per captured graph

// Initial parameters: unit j is a tanh step centred at the sample quantile
// (j + 1/2) / H, as steep as the local spacing of the quantiles, with output
// weight 1 / (2H) and bias 1/2, so the untrained network already rises from
// 0 to 1 across the data.
void quantile_init(const std::vector<float>& xs, float* p) {
  const size_t S = xs.size();
  auto q = [&](double f) {
    double r = f * (double)S;
    size_t i = r <= 0 ? 0 : (size_t)r;
    return xs[std::min(i, S - 1)];
  };
  for (int j = 0; j < H; ++j) {
    const float c = q((j + 0.5) / H);
    const float a = q((double)j / H), b = q((j + 1.0) / H);
    const float width = std::max(b - a, 1e-4f);
    const float steep = 2.0f / width;
    p[j] = steep;
    p[H + j] = -steep * c;
    p[2 * H + j] = 0.5f / (float)H;
  }
  p[3 * H] = 0.5f;
}

uint32_t default_leaves_log2(uint64_t nk) {
  int l = 4;
  while (l < 22 && ((uint64_t)1 << l) * 256 < nk) ++l;
  return (uint32_t)l;
}

}  // namespace

sd_index* learned_build(sd_ctx* c, const sd_seqs* ref, int k, const sd_learned_config* cfg,
                        hipStream_t s) {
  check_seqs(ref);
  if (k < 0 || k > 2) throw Error{SD_E_INVAL, "k must be 0, 1 or 2"};
  sd_learned_config conf{};
  if (cfg) conf = *cfg;
  if (conf.leaves_log2 != 0 && (conf.leaves_log2 < 4 || conf.leaves_log2 > 24))
    throw Error{SD_E_INVAL, "leaves_log2 must be 0 or lie in [4, 24]"};
  if (conf.steps < -1 || conf.steps > 1000000) throw Error{SD_E_INVAL, "bad step count"};
  if (!(conf.lr >= 0.0f) || conf.lr > 1.0f) throw Error{SD_E_INVAL, "bad learning rate"};
  if (conf.samples > (1u << 24)) throw Error{SD_E_INVAL, "at most 2^24 training samples"};
  const int steps = conf.steps < 0 ? 400 : conf.steps;
  const float lr = conf.lr > 0.0f ? conf.lr : 2e-4f;

  sd_index* idx = new sd_index();
  idx->device = c->device;
  idx->k = k;
  idx->learned = 1;
  idx->idbits = 32;
  idx->n_ref = (uint64_t)ref->n;
  hipStream_t ts = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  try {
    Scratch sc(c);
    StageTimer tm(c, s);
    Call cl{c, s, sc, tm, fresh_counters(c, CNT_TOTAL, s)};
    const DevSeqs in = stage_seqs(c, sc, ref, s);
    idx->ref_seq = static_cast<u128*>(index_alloc(c, idx, std::max<uint64_t>(in.n, 1) * 16));
    idx->params = static_cast<float*>(index_alloc(c, idx, NP * sizeof(float)));
    uint64_t nk = 0;
    if (in.n) {
      const Packed p = pack_and_count(cl, in, k, false);
      hip_check(hipMemcpyAsync(idx->ref_seq, p.seq, in.n * 16, hipMemcpyDeviceToDevice, s), "copy");
      nk = p.nkeys;
      uint64_t* klo = sc.get<uint64_t>(nk);
      uint64_t* khi = sc.get<uint64_t>(nk);
      uint32_t* kid = sc.get<uint32_t>(nk);
      launch_vargen(p.seq, p.voff, in.n, k, klo, khi, kid, s);
      const SortedKeys sk = full_key_sort(cl, klo, khi, kid, (uint32_t)nk);
      check_lookback(cl);
      idx->keys = static_cast<u128*>(index_alloc(c, idx, nk * 16));
      idx->kid = static_cast<uint32_t*>(index_alloc(c, idx, nk * 4));
      launch_interleave(sk.hi, sk.lo, nk, idx->keys, s);
      hip_check(hipMemcpyAsync(idx->kid, sk.id, nk * 4, hipMemcpyDeviceToDevice, s), "copy ids");
    }
    idx->n_keys = nk;
    sd_learned_info& info = idx->info;
    const uint32_t lg = conf.leaves_log2 ? (uint32_t)conf.leaves_log2 : default_leaves_log2(nk);
    idx->nleaves = 1u << lg;
    info.leaves = (int32_t)idx->nleaves;
    idx->leaves = index_alloc(c, idx, (size_t)idx->nleaves * leaf_bytes());

    // coordinate model: residue frequencies per (length, position) and
    // length shares, counted over keys at evenly spaced ranks
    idx->coord = index_alloc(c, idx, coord_bytes());
    {
      const int NLn = coord_lengths();
      const size_t ntab = (size_t)NLn * 24 * 20;
      const uint32_t SC = (uint32_t)std::min<uint64_t>(nk, 1u << 22);
      uint32_t* cnt = sc.get<uint32_t>(ntab + NLn);
      launch_fill_u32(cnt, 0, ntab + NLn, s);
      launch_coord_counts(idx->keys, nk, SC, cnt, s);
      std::vector<uint32_t> hc(ntab + NLn);
      hip_check(hipMemcpyAsync(hc.data(), cnt, hc.size() * 4, hipMemcpyDeviceToHost, s), "D2H counts");
      hip_check(hipStreamSynchronize(s), "synchronise");
      // layout: lencum[25 + 1] (double), lmin, lmax (u32), then FP32
      // (cumulative, frequency) pairs for t < 12 of lengths lmin..lmax
      const int R = coord_res();
      size_t off_lmin = 0, off_rows = 0;
      coord_offsets(&off_lmin, &off_rows);
      std::vector<unsigned char> model(coord_bytes(), 0);
      uint32_t lmin = 1, lmax = 0;
      for (int L = NLn - 1; L >= 0; --L)
        if (hc[ntab + L]) lmin = (uint32_t)L;
      for (int L = 0; L < NLn; ++L)
        if (hc[ntab + L]) lmax = (uint32_t)L;
      const double alpha = 0.5;  // additive smoothing: every residue and length keeps a share
      float* rows = reinterpret_cast<float*>(model.data() + off_rows);
      for (uint32_t L = lmin; L <= lmax && L < (uint32_t)NLn; ++L)
        for (int t = 0; t < R && t < (int)L; ++t) {
          const uint32_t* row = &hc[((size_t)L * 24 + t) * 20];
          double tot = 0.0;
          for (int c = 0; c < 20; ++c) tot += row[c];
          double cum = 0.0;
          for (int c = 0; c < 20; ++c) {
            const double pr = (row[c] + alpha) / (tot + 20 * alpha);
            const size_t e = ((size_t)(L - lmin) * R + t) * 20 + c;
            rows[2 * e] = (float)cum;
            rows[2 * e + 1] = (float)pr;
            cum += pr;
          }
        }
      double* lencum = reinterpret_cast<double*>(model.data());
      double tot = 0.0;
      for (int L = 0; L < NLn; ++L) tot += hc[ntab + L] + alpha;
      lencum[0] = 0.0;
      for (int L = 0; L < NLn; ++L) lencum[L + 1] = lencum[L] + (hc[ntab + L] + alpha) / tot;
      std::memcpy(model.data() + off_lmin, &lmin, 4);
      std::memcpy(model.data() + off_lmin + 4, &lmax, 4);
      idx->coord_rows = lmax >= lmin ? lmax - lmin + 1 : 0;
      hip_check(hipMemcpyAsync(idx->coord, model.data(), coord_bytes(), hipMemcpyHostToDevice, s),
                "H2D coordinate model");
      hip_check(hipStreamSynchronize(s), "synchronise");
    }

    // training samples and initial parameters
    const uint32_t S = nk ? (uint32_t)std::min<uint64_t>(conf.samples ? conf.samples : 65536u, nk) : 0;
    float hp[NP];
    float* sx = sc.get<float>(std::max<uint32_t>(S, 1));
    float* sy = sc.get<float>(std::max<uint32_t>(S, 1));
    if (conf.use_init) {
      std::memcpy(hp, conf.init, sizeof(hp));
    } else if (S) {
      launch_train_sample(idx->keys, nk, S, idx->coord, sx, sy, s);
      std::vector<float> xs(S);
      hip_check(hipMemcpyAsync(xs.data(), sx, (size_t)S * 4, hipMemcpyDeviceToHost, s), "D2H");
      hip_check(hipStreamSynchronize(s), "synchronise");
      quantile_init(xs, hp);
    } else {
      quantile_init(std::vector<float>(1, 0.0f), hp);
    }
    hip_check(hipMemcpyAsync(idx->params, hp, sizeof(hp), hipMemcpyHostToDevice, s), "H2D params");
    if (conf.use_init && S) launch_train_sample(idx->keys, nk, S, idx->coord, sx, sy, s);

    for (int e = 0; e < 4; ++e) hip_check(hipEventCreate(&ev[e]), "event");
    hip_check(hipEventRecord(ev[0], s), "event");
    const int nsteps = S ? steps : 0;
    float best_loss = 0.0f;
    idx->loss_curve.assign((size_t)nsteps, 0.0f);
    if (nsteps) {
      const uint32_t nb = mlp_grad_blocks(S);
      float* partial = sc.get<float>((uint64_t)nb * (NP + 1));
      float* state = sc.get<float>((uint64_t)adam_state_floats());
      float* losses = sc.get<float>((uint64_t)nsteps);
      launch_fill_u32(reinterpret_cast<uint32_t*>(state), 0, (uint64_t)adam_state_floats(), s);
      // one captured chunk of steps, replayed on a private stream
      hip_check(hipStreamCreateWithFlags(&ts, hipStreamNonBlocking), "stream");
      hip_check(hipEventRecord(ev[1], s), "event");
      hip_check(hipStreamWaitEvent(ts, ev[1], 0), "wait");
      const int chunk = std::min(nsteps, GRAPH_STEPS);
      hip_check(hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal), "capture");
      for (int x = 0; x < chunk; ++x) {
        launch_mlp_grad(idx->params, sx, sy, S, partial, ts);
        launch_adam_step(idx->params, state, partial, nb, lr, 1, losses, (uint32_t)nsteps, ts);
      }
      hip_check(hipStreamEndCapture(ts, &graph), "capture");
      hip_check(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0), "instantiate");
      int done = 0;
      for (; done + chunk <= nsteps; done += chunk) hip_check(hipGraphLaunch(gexec, ts), "graph launch");
      for (; done < nsteps; ++done) {
        launch_mlp_grad(idx->params, sx, sy, S, partial, ts);
        launch_adam_step(idx->params, state, partial, nb, lr, 1, losses, (uint32_t)nsteps, ts);
      }
      // evaluate the last update, then keep the best parameters seen
      launch_mlp_grad(idx->params, sx, sy, S, partial, ts);
      launch_adam_step(idx->params, state, partial, nb, lr, 0, losses, (uint32_t)nsteps, ts);
      launch_adam_best(idx->params, state, ts);
      hip_check(hipMemcpyAsync(&best_loss, state + 1 + 2 * NP, 4, hipMemcpyDeviceToHost, ts),
                "D2H best loss");
      hip_check(hipEventRecord(ev[2], ts), "event");
      hip_check(hipStreamWaitEvent(s, ev[2], 0), "wait");
      hip_check(hipMemcpyAsync(idx->loss_curve.data(), losses, (size_t)nsteps * 4,
                               hipMemcpyDeviceToHost, s),
                "D2H losses");
    }
    hip_check(hipEventRecord(ev[1], s), "event");
    launch_leaf_fit_all(idx->keys, nk, idx->coord, idx->params, idx->nleaves, idx->leaves, s);
    hip_check(hipEventRecord(ev[3], s), "event");

    // leaf statistics
    std::vector<unsigned char> lv((size_t)idx->nleaves * leaf_bytes());
    hip_check(hipMemcpyAsync(lv.data(), idx->leaves, lv.size(), hipMemcpyDeviceToHost, s), "D2H leaves");
    hip_check(hipMemcpyAsync(info.params, idx->params, sizeof(info.params), hipMemcpyDeviceToHost, s),
              "D2H params");
    hip_check(hipStreamSynchronize(s), "synchronise");
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, ev[0], ev[1]), "elapsed");
    info.train_ms = ms;
    hip_check(hipEventElapsedTime(&ms, ev[1], ev[3]), "elapsed");
    info.fit_ms = ms;
    info.steps = nsteps;
    info.loss_first = nsteps ? idx->loss_curve.front() : 0.0f;
    info.loss_last = nsteps ? best_loss : 0.0f;
    double sum_eps = 0.0, sum_win = 0.0;
    uint64_t counted = 0;
    for (uint32_t l = 0; l < idx->nleaves; ++l) {
      uint32_t f[4];  // lo, hi, eps, count after the two doubles
      std::memcpy(f, lv.data() + (size_t)l * leaf_bytes() + 16, 16);
      if (f[0] > f[1]) {
        ++info.empty_leaves;
        continue;
      }
      info.max_eps = std::max(info.max_eps, f[2]);
      sum_eps += (double)f[2] * f[3];
      sum_win += std::log2(2.0 * f[2] + 1.0) * f[3];
      counted += f[3];
    }
    if (counted != nk) throw Error{SD_E_HIP, "internal error: leaf counts do not cover the keys"};
    info.mean_eps = nk ? sum_eps / (double)nk : 0.0;
    info.mean_window_log2 = nk ? sum_win / (double)nk : 0.0;
    idx->bytes = idx->n_ref * 16 + nk * 20 + (uint64_t)idx->nleaves * leaf_bytes() + NP * 4 +
                 coord_bytes();
  } catch (...) {
    if (ts) (void)hipStreamSynchronize(ts);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ts) (void)hipStreamDestroy(ts);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    index_free(idx);
    throw;
  }
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  if (ts) (void)hipStreamDestroy(ts);
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  return idx;
}

TileOut learned_tile(Call& cl, const sd_index* idx, const DevSeqs& q, int k, const WeightedSpec* w) {
  sd_ctx* c = cl.c;
  hipStream_t s = cl.s;
  const Packed p = pack_and_count(cl, q, k, false);
  const uint64_t nk = p.nkeys;
  cl.tm.mark("q_pack_scan", (double)q.n * 56, 2);
  const int learned = c->probe == 0 ? 1 : 0;
  unsigned long long* steps = reinterpret_cast<unsigned long long*>(cl.counters + CNT_STEPS);
  Cands cp = sharded_output(
      cl, nk / 4, "probe",
      [&](const ShardArgs& out) {
        launch_fill_u64(reinterpret_cast<uint64_t*>(steps), 0, 1, s);
        launch_probe(p.seq, p.voff, q.n, idx->keys, idx->kid, idx->n_keys, learned, idx->coord,
                     idx->coord_rows, idx->params, idx->nleaves, idx->leaves, out, steps, s);
      },
      [&](uint64_t n) { return (double)nk * 16 + (double)n * 12; });
  cl.sc.blocks.push_back(cp.p);
  uint64_t* cand = cp.p;
  const uint64_t nc = cp.n;
  uint64_t nsteps;
  std::memcpy(&nsteps, readback(c, steps, 8, s), 8);
  c->stats.n_probe_steps += (int64_t)nsteps;
  TileOut v = verify_candidates(cl, p.seq, p.planes, q.n, idx->ref_seq, idx->n_ref, cand, nc, k, w);
  v.nkeys = nk;
  v.ncand = nc;
  return v;
}

void mlp_gradients(sd_ctx* c, const float* params, const float* x, const float* y, uint32_t n,
                   float* grad, float* loss, hipStream_t s) {
  if (!params || !x || !y || !grad || !loss) throw Error{SD_E_INVAL, "null pointer"};
  if (n == 0 || n > (1u << 24)) throw Error{SD_E_INVAL, "n must lie in [1, 2^24]"};
  Scratch sc(c);
  float* dp = sc.get<float>(NP);
  float* dx = sc.get<float>(n);
  float* dy = sc.get<float>(n);
  const uint32_t nb = mlp_grad_blocks(n);
  float* partial = sc.get<float>((uint64_t)nb * (NP + 1));
  float* out = sc.get<float>(NP + 1);
  hip_check(hipMemcpyAsync(dp, params, NP * 4, hipMemcpyHostToDevice, s), "H2D");
  hip_check(hipMemcpyAsync(dx, x, (size_t)n * 4, hipMemcpyHostToDevice, s), "H2D");
  hip_check(hipMemcpyAsync(dy, y, (size_t)n * 4, hipMemcpyHostToDevice, s), "H2D");
  launch_mlp_grad(dp, dx, dy, n, partial, s);
  launch_grad_reduce(partial, nb, out, s);
  const float* h = static_cast<const float*>(readback(c, out, (NP + 1) * 4, s));
  std::memcpy(grad, h, NP * 4);
  *loss = h[NP];
}

}  // namespace sd
