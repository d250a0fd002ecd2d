// Autotuner: runs a caller's sample through candidate configurations of the
// context's tunables and keeps the fastest in the context.
//
// Self search (index == NULL), in two stages: a grid over the LDS batch
// capacity of the hashed path and the items per thread of the keys-only
// radix passes (plus the full-key path), then, from the best of the grid,
// one knob at a time: the hash bits the LSD passes sort by (the radix
// width of the grouping sort: the automatic choice, one bit more, two bits
// more, which can add an 8-bit pass), the candidate pair sort (one-sweep or
// counted passes) and the grouping kernel's shape. Query batches (index
// given): a grid over the query tile size and the radix items per thread,
// then the captured-graph batch on or off. Every candidate runs once to warm
// the memory pool, then `reps` times; the score is the mean host wall time
// of the synchronous call, so allocation and read-back costs count too.
// Results are identical for every configuration; only speed changes.
//
// With a cache file (sd_autotune_cache), the choice is stored under a key of
// the device architecture, the kind of call, a shape bucket (log2 of the
// sequences and of the sets) and k; a later sd_autotune with the same key
// applies the stored choice without running the sample. The file is a flat
// JSON object: key -> {knob: integer}.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "sd_host.h"

namespace sd {

namespace {

struct Knobs {
  int path, group_cap, sort_items, group_bits, pair_sort, group_shape, batch_graph;
  int64_t tile;
};

Knobs read_knobs(const sd_ctx* c) {
  return Knobs{c->path,      c->group_cap,   c->sort_items,  c->group_bits,
               c->pair_sort, c->group_shape, c->batch_graph, c->batch_tile_seqs};
}

void set_knobs(sd_ctx* c, const Knobs& k) {
  c->path = k.path;
  c->group_cap = k.group_cap;
  c->sort_items = k.sort_items;
  c->group_bits = k.group_bits;
  c->pair_sort = k.pair_sort;
  c->group_shape = k.group_shape;
  c->batch_graph = k.batch_graph;
  c->batch_tile_seqs = k.tile;
}

double seconds_of(const std::function<void()>& fn, int reps) {
  fn();  // warm-up: fills the pool's size classes (and captures a batch graph)
  const auto t0 = std::chrono::steady_clock::now();
  for (int r = 0; r < reps; ++r) fn();
  const auto t1 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(t1 - t0).count() / reps;
}

// ---- the cache file: {"key": {"knob": int, ...}, ...}

using Entry = std::map<std::string, int64_t>;

void skip_ws(const std::string& s, size_t& p) {
  while (p < s.size() && (s[p] == ' ' || s[p] == '\n' || s[p] == '\r' || s[p] == '\t')) ++p;
}

bool parse_string(const std::string& s, size_t& p, std::string& out) {
  skip_ws(s, p);
  if (p >= s.size() || s[p] != '"') return false;
  const size_t e = s.find('"', p + 1);
  if (e == std::string::npos) return false;
  out = s.substr(p + 1, e - p - 1);
  p = e + 1;
  return true;
}

bool expect(const std::string& s, size_t& p, char ch) {
  skip_ws(s, p);
  if (p >= s.size() || s[p] != ch) return false;
  ++p;
  return true;
}

// A cache that does not parse is treated as empty (it is rewritten whole).
std::map<std::string, Entry> read_cache(const std::string& path) {
  std::map<std::string, Entry> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t p = 0;
  if (!expect(s, p, '{')) return {};
  skip_ws(s, p);
  if (p < s.size() && s[p] == '}') return m;
  while (true) {
    std::string key;
    if (!parse_string(s, p, key) || !expect(s, p, ':') || !expect(s, p, '{')) return {};
    Entry e;
    skip_ws(s, p);
    if (p < s.size() && s[p] == '}') {
      ++p;
    } else {
      while (true) {
        std::string name;
        if (!parse_string(s, p, name) || !expect(s, p, ':')) return {};
        skip_ws(s, p);
        size_t used = 0;
        long long v = 0;
        try {
          v = std::stoll(s.substr(p, 32), &used);
        } catch (...) {
          return {};
        }
        p += used;
        e[name] = v;
        skip_ws(s, p);
        if (p < s.size() && s[p] == ',') {
          ++p;
          continue;
        }
        if (!expect(s, p, '}')) return {};
        break;
      }
    }
    m[key] = e;
    skip_ws(s, p);
    if (p < s.size() && s[p] == ',') {
      ++p;
      continue;
    }
    if (!expect(s, p, '}')) return {};
    break;
  }
  return m;
}

void write_cache(const std::string& path, const std::map<std::string, Entry>& m) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) throw Error{SD_E_INVAL, "cannot write the tuning cache " + path};
    f << "{\n";
    size_t x = 0;
    for (const auto& kv : m) {
      f << "  \"" << kv.first << "\": {";
      size_t y = 0;
      for (const auto& nv : kv.second) f << (y++ ? ", " : "") << "\"" << nv.first << "\": " << nv.second;
      f << "}" << (++x < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0)
    throw Error{SD_E_INVAL, "cannot replace the tuning cache " + path};
}

Entry to_entry(const Knobs& k) {
  return Entry{{"path", k.path},           {"group_cap", k.group_cap},
               {"sort_items", k.sort_items}, {"group_bits", k.group_bits},
               {"pair_sort", k.pair_sort}, {"group_shape", k.group_shape},
               {"batch_graph", k.batch_graph}, {"batch_tile", k.tile}};
}

bool from_entry(const Entry& e, Knobs& k) {
  auto get = [&](const char* n, int64_t& v) {
    auto it = e.find(n);
    if (it == e.end()) return false;
    v = it->second;
    return true;
  };
  int64_t v[8];
  const char* names[8] = {"path", "group_cap", "sort_items", "group_bits",
                          "pair_sort", "group_shape", "batch_graph", "batch_tile"};
  for (int x = 0; x < 8; ++x)
    if (!get(names[x], v[x])) return false;
  k = Knobs{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5], (int)v[6], v[7]};
  return true;
}

std::string tune_key(const sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  } else {
    (void)hipGetLastError();
  }
  auto bucket = [](double v) { return std::to_string(v >= 1.0 ? (int)std::floor(std::log2(v)) : 0); };
  int64_t total = 0;
  for (int x = 0; x < nsets; ++x) total += sets[x].n;
  const std::string kind = idx ? "query/r" + bucket((double)idx->n_ref) : std::string("self");
  return arch + "/" + kind + "/s" + bucket((double)total) + "/n" + bucket((double)nsets) + "/k" +
         std::to_string(k);
}

}  // namespace

void autotune(sd_ctx* c, const sd_index* idx, int nsets, const sd_seqs* sets, int k, int reps,
              sd_tune_result* out, hipStream_t s) {
  if (!out || nsets < 1 || !sets) throw Error{SD_E_INVAL, "bad tuning sample"};
  if (reps < 1 || reps > 100) throw Error{SD_E_INVAL, "reps must lie in [1, 100]"};
  if (!idx && nsets != 1) throw Error{SD_E_INVAL, "self-search tuning takes one sample set"};
  std::memset(out, 0, sizeof(*out));
  const Knobs start = read_knobs(c);
  // a stored choice for this key needs no trials
  std::string key;
  std::map<std::string, Entry> cache;
  if (!c->tune_cache.empty()) {
    key = tune_key(c, idx, nsets, sets, k);
    cache = read_cache(c->tune_cache);
    auto it = cache.find(key);
    Knobs kb;
    if (it != cache.end() && from_entry(it->second, kb)) {
      set_knobs(c, kb);
      out->path = kb.path;
      out->group_cap = kb.group_cap;
      out->sort_items = kb.sort_items;
      out->batch_tile = kb.tile;
      out->group_bits = kb.group_bits;
      out->pair_sort = kb.pair_sort;
      out->group_shape = kb.group_shape;
      out->batch_graph = kb.batch_graph;
      out->from_cache = 1;
      return;
    }
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
  double best = 0.0;
  Knobs best_k = start;
  bool have = false;
  auto trial = [&](const Knobs& kb) {
    set_knobs(c, kb);
    const double t = seconds_of(run, reps);
    ++out->trials;
    if (!have || t < best) {
      best = t;
      best_k = kb;
      have = true;
    }
  };
  try {
    // stage 1: a grid
    if (!idx) {
      for (int items : {16, 32})
        for (int cap : {1024, 2048, 4096}) {
          Knobs kb = start;
          kb.path = 2;
          kb.group_cap = cap;
          kb.sort_items = items;
          trial(kb);
        }
      if (k <= 2) {
        Knobs kb = start;
        kb.path = 1;
        kb.sort_items = 16;
        trial(kb);
      }
    } else {
      for (int items : {16, 32})
        for (int64_t tile : {1ll << 20, 1ll << 21, 1ll << 22, 1ll << 23}) {
          Knobs kb = start;
          kb.sort_items = items;
          kb.tile = tile;
          kb.batch_graph = 0;
          trial(kb);
        }
    }
    // stage 2: one knob at a time from the best of the grid
    const Knobs base = best_k;
    std::vector<Knobs> more;
    if (!idx) {
      if (base.path != 1) {
        // the automatic hash-bit count for the sample's key count (the
        // last trial's)
        int auto_bits = -1;
        if (c->stats.n_keys > 0) {
          const int save_cap = c->group_cap, save_bits = c->group_bits;
          c->group_cap = base.group_cap;
          c->group_bits = 0;
          int cp = 0;
          hashed_plan(c, (uint64_t)c->stats.n_keys, &cp, &auto_bits);
          c->group_cap = save_cap;
          c->group_bits = save_bits;
        }
        for (int db : {1, 2}) {
          if (auto_bits < 0) break;
          Knobs kb = base;
          kb.group_bits = std::min(23, auto_bits + db);
          more.push_back(kb);
        }
        if (base.group_cap == 2048 || base.group_cap == 0) {
          Knobs kb = base;
          kb.group_shape = 1;
          more.push_back(kb);
        }
      }
      for (int ps : {1, 2}) {
        Knobs kb = base;
        kb.pair_sort = ps;
        more.push_back(kb);
      }
    } else {
      Knobs kb = base;
      kb.batch_graph = 1;
      more.push_back(kb);
    }
    for (const Knobs& kb : more) trial(kb);
    set_knobs(c, start);
    out->default_s = seconds_of(run, reps);
  } catch (...) {
    set_knobs(c, start);
    throw;
  }
  set_knobs(c, best_k);
  out->path = c->path;
  out->group_cap = c->group_cap;
  out->sort_items = c->sort_items;
  out->batch_tile = c->batch_tile_seqs;
  out->group_bits = c->group_bits;
  out->pair_sort = c->pair_sort;
  out->group_shape = c->group_shape;
  out->batch_graph = c->batch_graph;
  out->best_s = best;
  if (!c->tune_cache.empty()) {
    cache[key] = to_entry(best_k);
    write_cache(c->tune_cache, cache);
  }
}

}  // namespace sd
