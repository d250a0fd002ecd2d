// Autotuner: runs a caller's sample through candidate configurations of the
// context's tunables and keeps the fastest in the context.
//
// Self search (index == NULL): grouping path, LDS batch capacity of the
// hashed path (its hash-bit count follows from the capacity) and items per
// thread of the keys-only radix passes. Query batches (index given): query
// tile size and radix items per thread. Every candidate runs once to warm
// the memory pool, then `reps` times; the score is the mean host wall time of
// the synchronous call, so allocation and read-back costs count too. Results
// are identical for every configuration; only speed changes.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <functional>
#include <vector>

#include "sd_host.h"

namespace sd {

namespace {

struct Knobs {
  int path, group_cap, sort_items;
  int64_t tile;
};

Knobs read_knobs(const sd_ctx* c) { return Knobs{c->path, c->group_cap, c->sort_items, c->batch_tile_seqs}; }

void set_knobs(sd_ctx* c, const Knobs& k) {
  c->path = k.path;
  c->group_cap = k.group_cap;
  c->sort_items = k.sort_items;
  c->batch_tile_seqs = k.tile;
}

double seconds_of(const std::function<void()>& fn, int reps) {
  fn();  // warm-up: fills the pool's size classes
  const auto t0 = std::chrono::steady_clock::now();
  for (int r = 0; r < reps; ++r) fn();
  const auto t1 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(t1 - t0).count() / reps;
}

}  // namespace

void autotune(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k, int reps,
              sd_tune_result* out, hipStream_t s) {
  if (!out || nsets < 1 || !sets) throw Error{SD_E_INVAL, "bad tuning sample"};
  if (reps < 1 || reps > 100) throw Error{SD_E_INVAL, "reps must lie in [1, 100]"};
  const Knobs start = read_knobs(c);
  std::vector<Knobs> cand;
  if (!idx) {
    if (nsets != 1) throw Error{SD_E_INVAL, "self-search tuning takes one sample set"};
    for (int items : {16, 32})
      for (int cap : {1024, 2048, 4096}) cand.push_back(Knobs{2, cap, items, start.tile});
    cand.push_back(Knobs{1, start.group_cap, 16, start.tile});
  } else {
    for (int items : {16, 32})
      for (int64_t tile : {1ll << 20, 1ll << 21, 1ll << 22, 1ll << 23})
        cand.push_back(Knobs{start.path, start.group_cap, items, tile});
  }
  std::vector<sd_pairs> outs((size_t)nsets);
  auto run = [&]() {
    for (auto& o : outs) {
      std::memset(&o, 0, sizeof(o));
      o.on_device = 1;
    }
    try {
      if (!idx)
        self_search(c, &sets[0], k, &outs[0], s);
      else
        query_sets(c, idx, nsets, sets, k, nullptr, outs.data(), s);
    } catch (...) {
      for (auto& o : outs) sd_pairs_free(c, &o);
      throw;
    }
    for (auto& o : outs) sd_pairs_free(c, &o);
  };
  std::memset(out, 0, sizeof(*out));
  double best = 0.0;
  int best_i = -1;
  try {
    for (size_t x = 0; x < cand.size(); ++x) {
      set_knobs(c, cand[x]);
      const double t = seconds_of(run, reps);
      if (best_i < 0 || t < best) {
        best = t;
        best_i = (int)x;
      }
      ++out->trials;
    }
    set_knobs(c, start);
    out->default_s = seconds_of(run, reps);
  } catch (...) {
    set_knobs(c, start);
    throw;
  }
  set_knobs(c, cand[best_i]);
  out->path = c->path;
  out->group_cap = c->group_cap;
  out->sort_items = c->sort_items;
  out->batch_tile = c->batch_tile_seqs;
  out->best_s = best;
}

}  // namespace sd
