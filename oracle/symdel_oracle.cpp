// CPU ORACLE for symmetric-deletion (SymDel) neighbour search.
//
// TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the
// benchmark's CPU-baseline leg load this library. It shares no code, header,
// table or helper with the GPU library and does not know its key packing:
// sequences are plain byte strings and deletion variants are std::string.
//
// What it computes (paper, Section II A and the SymDel step list of
// Appendix A; Fig. 1):
//   Self(S, k)  = { (i, j, d) : i < j, d = Lev(S_i, S_j) <= k }, sorted by (i, j)
//   Query(R, Q, k) = { (q, r, d) : d = Lev(Q_q, R_r) <= k }, sorted by (q, r)
// where Lev is the unit-cost insertion/deletion/substitution edit distance.
// The SymDel route to that set: (1) generate every deletion variant with up
// to k deleted positions, (2) store variant -> source ids in a multi-value
// hash map, (3) look the variants up again to collect candidate pairs, (4)
// drop duplicate pairs and pairs above the threshold (Fig. 1C/1D).
//
// Hamming mode (Section III C, where the comparison with a Hamming-only tool
// changes only the final filter of the method): the same SymDel candidates,
// kept when the two sequences have equal length and differ in at most k
// positions. Hamming(a, b) <= k implies Lev(a, b) <= k, so the deletion
// candidates contain every such pair.
//
// Paired-chain mode (Discussion: the CDR3s of both chains joined by a
// joining token that is never deleted): a record is (a, b); its variants
// are a' TOKEN b' with a' and b' deletion variants of a and b, at most k
// positions deleted in total and the token kept. The token must align with
// itself, so the distance of two records is Lev(a1, a2) + Lev(b1, b2); if
// that is <= k, deleting per chain as in the single-chain proof gives a
// shared variant with at most k deletions on each side.
//
// Weighted mode (Section III D: a Levenshtein prefilter followed by a
// finer, substitution-weighted score): score = minimum-cost global alignment
// with a 20x20 substitution cost table and a fixed indel cost.
//
// Everything is unoptimised on purpose. The plain entry points run on one
// thread. or_self_search_sharded runs the same steps on all host cores with
// bounded memory (the CPU-baseline plan for the large workloads): the
// variant space is split into P shards by a hash of the variant string, each
// shard regenerates every variant and keeps only its own, so a shard's map
// holds about 1/P of the variants; equal variants always fall into the same
// shard, so the union of the shards' bucket pairs is exactly the candidate
// set of the single map.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

// Wagner-Fischer dynamic programme over the full (la+1) x (lb+1) table.
// D(x, y) is the distance between the first x residues of a and the first y
// residues of b; the table lives in one reused buffer.
int lev_full(const uint8_t* a, int la, const uint8_t* b, int lb) {
  static thread_local std::vector<int> buf;
  const int w = lb + 1;
  buf.assign((size_t)(la + 1) * w, 0);
  auto D = [&](int x, int y) -> int& { return buf[(size_t)x * w + y]; };
  for (int x = 0; x <= la; ++x) D(x, 0) = x;
  for (int y = 0; y <= lb; ++y) D(0, y) = y;
  for (int x = 1; x <= la; ++x)
    for (int y = 1; y <= lb; ++y) {
      int sub = D(x - 1, y - 1) + (a[x - 1] == b[y - 1] ? 0 : 1);
      int del = D(x - 1, y) + 1;
      int ins = D(x, y - 1) + 1;
      D(x, y) = std::min(sub, std::min(del, ins));
    }
  return D(la, lb);
}

// Hamming distance: the number of positions at which equal-length strings
// differ; -1 for strings of different lengths (no Hamming distance).
int hamming(const uint8_t* a, int la, const uint8_t* b, int lb) {
  if (la != lb) return -1;
  int d = 0;
  for (int x = 0; x < la; ++x) d += a[x] != b[x];
  return d;
}

// Minimum-cost global alignment: substitution a->b costs subst[a*20+b],
// an insertion or deletion costs indel.
int weighted_full(const uint8_t* a, int la, const uint8_t* b, int lb, const uint8_t* subst,
                  int indel) {
  static thread_local std::vector<int> buf;
  const int w = lb + 1;
  buf.assign((size_t)(la + 1) * w, 0);
  auto D = [&](int x, int y) -> int& { return buf[(size_t)x * w + y]; };
  for (int x = 0; x <= la; ++x) D(x, 0) = x * indel;
  for (int y = 0; y <= lb; ++y) D(0, y) = y * indel;
  for (int x = 1; x <= la; ++x)
    for (int y = 1; y <= lb; ++y) {
      int sub = D(x - 1, y - 1) + subst[a[x - 1] * 20 + b[y - 1]];
      int del = D(x - 1, y) + indel;
      int ins = D(x, y - 1) + indel;
      D(x, y) = std::min(sub, std::min(del, ins));
    }
  return D(la, lb);
}

// Every set of m <= k positions of a string of length L, for m = 0, 1, ...,
// min(k, L), each m-subset in lexicographic order: fn(pos, m) is called
// once per set with pos[0] < ... < pos[m-1].
template <class F>
void for_each_deletion_set(int L, int k, F&& fn) {
  const int kk = std::min(k, L);
  std::vector<int> pos;
  for (int m = 0; m <= kk; ++m) {
    pos.resize(m);
    for (int t = 0; t < m; ++t) pos[t] = t;
    while (true) {
      fn(pos, m);
      // advance to the next m-subset in lexicographic order
      int t = m - 1;
      while (t >= 0 && pos[t] == L - m + t) --t;
      if (t < 0) break;
      ++pos[t];
      for (int u = t + 1; u < m; ++u) pos[u] = pos[u - 1] + 1;
    }
  }
}

// s without the positions pos[0..m-1]
std::string delete_positions(const std::string& s, const std::vector<int>& pos, int m) {
  std::string v;
  int next = 0;
  for (int x = 0; x < (int)s.size(); ++x) {
    if (next < m && pos[next] == x) {
      ++next;
      continue;
    }
    v.push_back(s[x]);
  }
  return v;
}

// Every string obtained from s by deleting a set of m <= k positions, in the
// order of for_each_deletion_set. A string of length L yields
// sum_{m<=k} C(L, m) variants counted with multiplicity (56 for L = 10,
// k = 2, Section II A).
void deletion_variants(const std::string& s, int k, std::vector<std::string>& out) {
  out.clear();
  for_each_deletion_set((int)s.size(), k, [&](const std::vector<int>& pos, int m) {
    out.push_back(delete_positions(s, pos, m));
  });
}

// Paired variants a' TOKEN b' of a record (a, b) with at most k deletions in
// total; TOKEN is a byte no residue takes.
constexpr char PAIR_TOKEN = (char)0xFF;
void paired_variants(const std::string& a, const std::string& b, int k, std::vector<std::string>& out) {
  out.clear();
  std::vector<std::string> va, vb;
  for (int m1 = 0; m1 <= k; ++m1) {
    va.clear();
    for_each_deletion_set((int)a.size(), m1, [&](const std::vector<int>& pos, int m) {
      if (m == m1) va.push_back(delete_positions(a, pos, m));
    });
    vb.clear();
    for_each_deletion_set((int)b.size(), k - m1, [&](const std::vector<int>& pos, int m) {
      vb.push_back(delete_positions(b, pos, m));
    });
    for (const std::string& x : va)
      for (const std::string& y : vb) out.push_back(x + PAIR_TOKEN + y);
  }
}

std::string seq_at(const uint8_t* codes, const int64_t* offs, int64_t i) {
  return std::string(reinterpret_cast<const char*>(codes + offs[i]),
                     (size_t)(offs[i + 1] - offs[i]));
}

struct Result {
  std::vector<uint32_t> a, b;
  std::vector<int32_t> d;
  int64_t raw = 0;  // candidate count with multiplicity (before de-duplication)
};

typedef std::unordered_map<std::string, std::vector<uint32_t>> MultiMap;

// SymDel steps 1-2: variants of every sequence into the multi-value map.
void build_map(const uint8_t* codes, const int64_t* offs, int64_t n, int k, MultiMap& map) {
  std::vector<std::string> vars;
  for (int64_t i = 0; i < n; ++i) {
    deletion_variants(seq_at(codes, offs, i), k, vars);
    for (const std::string& v : vars) {
      std::vector<uint32_t>& ids = map[v];
      if (ids.empty() || ids.back() != (uint32_t)i) ids.push_back((uint32_t)i);
    }
  }
}

// SymDel step 3 for a self search: every bucket yields all its id pairs.
void self_candidates(const MultiMap& map, std::vector<uint64_t>& cand, int64_t& raw) {
  raw = 0;
  for (const auto& kv : map) {
    const std::vector<uint32_t>& ids = kv.second;
    for (size_t x = 0; x < ids.size(); ++x)
      for (size_t y = x + 1; y < ids.size(); ++y) {
        uint32_t lo = std::min(ids[x], ids[y]), hi = std::max(ids[x], ids[y]);
        cand.push_back(((uint64_t)lo << 32) | hi);
        ++raw;
      }
  }
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
}

// SymDel step 3 for a query search: look each query variant up in the
// reference map.
void query_candidates(const MultiMap& refmap, const uint8_t* qc, const int64_t* qo, int64_t nq,
                      int k, std::vector<uint64_t>& cand, int64_t& raw) {
  raw = 0;
  std::vector<std::string> vars;
  for (int64_t q = 0; q < nq; ++q) {
    deletion_variants(seq_at(qc, qo, q), k, vars);
    for (const std::string& v : vars) {
      auto it = refmap.find(v);
      if (it == refmap.end()) continue;
      for (uint32_t r : it->second) {
        cand.push_back(((uint64_t)q << 32) | r);
        ++raw;
      }
    }
  }
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
}

// FNV-1a (64-bit) over the bytes of a variant; it only decides which shard
// owns the variant, so any fixed function of the string would do.
uint64_t fnv1a(const std::string& v) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char ch : v) {
    h ^= ch;
    h *= 1099511628211ull;
  }
  return h;
}

// fnv1a(delete_positions(s, pos, m)) without building the string
uint64_t fnv1a_deleted(const std::string& s, const std::vector<int>& pos, int m) {
  uint64_t h = 1469598103934665603ull;
  int next = 0;
  for (int x = 0; x < (int)s.size(); ++x) {
    if (next < m && pos[next] == x) {
      ++next;
      continue;
    }
    h ^= (unsigned char)s[x];
    h *= 1099511628211ull;
  }
  return h;
}

int pick_threads(int nthreads) {
  if (nthreads > 0) return nthreads;
  const unsigned hc = std::thread::hardware_concurrency();
  return hc ? (int)hc : 1;
}

// Run body(t) for t = 0 .. nthreads-1 on their own threads and join them.
template <class F>
void run_threads(int nthreads, F&& body) {
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t) pool.emplace_back(body, t);
  for (std::thread& th : pool) th.join();
}

}  // namespace

extern "C" {

int or_lev(const uint8_t* a, int la, const uint8_t* b, int lb) { return lev_full(a, la, b, lb); }

int or_hamming(const uint8_t* a, int la, const uint8_t* b, int lb) { return hamming(a, la, b, lb); }

int or_weighted(const uint8_t* a, int la, const uint8_t* b, int lb, const uint8_t* subst,
                int indel) {
  return weighted_full(a, la, b, lb, subst, indel);
}

// Distances from one string to each of n strings (CSR).
void or_lev_one_to_many(const uint8_t* a, int la, const uint8_t* codes, const int64_t* offs,
                        int64_t n, int32_t* out) {
  for (int64_t i = 0; i < n; ++i)
    out[i] = lev_full(a, la, codes + offs[i], (int)(offs[i + 1] - offs[i]));
}

// Deletion variants of one string: writes up to cap variants, each padded to
// 32 bytes in out (cap * 32 bytes), their lengths in out_len; returns the count.
int64_t or_variants(const uint8_t* s, int L, int k, uint8_t* out, int32_t* out_len, int64_t cap) {
  std::vector<std::string> vars;
  deletion_variants(std::string(reinterpret_cast<const char*>(s), (size_t)L), k, vars);
  for (size_t v = 0; v < vars.size() && (int64_t)v < cap; ++v) {
    std::memset(out + v * 32, 0, 32);
    std::memcpy(out + v * 32, vars[v].data(), std::min<size_t>(vars[v].size(), 32));
    out_len[v] = (int32_t)vars[v].size();
  }
  return (int64_t)vars.size();
}

// Self search by SymDel; returns a result handle (free with or_free).
void* or_self_search(const uint8_t* codes, const int64_t* offs, int64_t n, int k) {
  Result* res = new Result();
  MultiMap map;
  build_map(codes, offs, n, k, map);
  std::vector<uint64_t> cand;
  self_candidates(map, cand, res->raw);
  for (uint64_t c : cand) {  // SymDel step 4: verify and keep d <= k
    uint32_t i = (uint32_t)(c >> 32), j = (uint32_t)c;
    int d = lev_full(codes + offs[i], (int)(offs[i + 1] - offs[i]), codes + offs[j],
                     (int)(offs[j + 1] - offs[j]));
    if (d <= k) {
      res->a.push_back(i);
      res->b.push_back(j);
      res->d.push_back(d);
    }
  }
  return res;
}

// Self search by SymDel on several threads with bounded memory: SymDel steps
// 1-3 per shard of the variant space (shard s keeps the variants whose hash
// is s modulo nshards), the shards' candidates merged, sorted and
// de-duplicated, then step 4 on contiguous slices of the sorted candidates
// (one slice per thread, concatenated in order). Returns the same triplets
// as or_self_search. At most min(nthreads, nshards) threads run at once
// (nthreads <= 0: one per hardware thread; nshards <= 0: one per thread).
void* or_self_search_sharded(const uint8_t* codes, const int64_t* offs, int64_t n, int k,
                             int nshards, int nthreads) {
  Result* res = new Result();
  const int T0 = pick_threads(nthreads);
  const int P = nshards > 0 ? nshards : T0;
  const int T = std::min(T0, P);
  std::vector<std::vector<uint64_t>> shard_cand(P);
  std::vector<int64_t> shard_raw(P, 0);
  std::atomic<int> next{0};
  run_threads(T, [&](int) {
    for (;;) {
      const int sh = next.fetch_add(1);
      if (sh >= P) break;
      MultiMap map;
      for (int64_t i = 0; i < n; ++i) {
        const std::string si = seq_at(codes, offs, i);
        // the variants of si this shard owns (the hash decides before the
        // string is built)
        for_each_deletion_set((int)si.size(), k, [&](const std::vector<int>& pos, int m) {
          if ((int)(fnv1a_deleted(si, pos, m) % (uint64_t)P) != sh) return;
          std::vector<uint32_t>& ids = map[delete_positions(si, pos, m)];
          if (ids.empty() || ids.back() != (uint32_t)i) ids.push_back((uint32_t)i);
        });
      }
      self_candidates(map, shard_cand[sh], shard_raw[sh]);
    }
  });
  std::vector<uint64_t> cand;
  size_t tot = 0;
  for (const auto& v : shard_cand) tot += v.size();
  cand.reserve(tot);
  for (auto& v : shard_cand) {
    cand.insert(cand.end(), v.begin(), v.end());
    std::vector<uint64_t>().swap(v);
  }
  for (int64_t r : shard_raw) res->raw += r;
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  // SymDel step 4 on T contiguous slices, kept in order
  std::vector<Result> part(T);
  const size_t nc = cand.size();
  run_threads(T, [&](int t) {
    const size_t lo = nc * (size_t)t / (size_t)T, hi = nc * (size_t)(t + 1) / (size_t)T;
    for (size_t x = lo; x < hi; ++x) {
      const uint32_t i = (uint32_t)(cand[x] >> 32), j = (uint32_t)cand[x];
      const int d = lev_full(codes + offs[i], (int)(offs[i + 1] - offs[i]), codes + offs[j],
                             (int)(offs[j + 1] - offs[j]));
      if (d <= k) {
        part[t].a.push_back(i);
        part[t].b.push_back(j);
        part[t].d.push_back(d);
      }
    }
  });
  for (const Result& r : part) {
    res->a.insert(res->a.end(), r.a.begin(), r.a.end());
    res->b.insert(res->b.end(), r.b.begin(), r.b.end());
    res->d.insert(res->d.end(), r.d.begin(), r.d.end());
  }
  return res;
}

// Self search in Hamming mode: SymDel steps 1-3 as in or_self_search, step 4
// keeps the candidates with equal lengths and Hamming distance <= k.
void* or_self_search_hamming(const uint8_t* codes, const int64_t* offs, int64_t n, int k) {
  Result* res = new Result();
  MultiMap map;
  build_map(codes, offs, n, k, map);
  std::vector<uint64_t> cand;
  self_candidates(map, cand, res->raw);
  for (uint64_t c : cand) {
    uint32_t i = (uint32_t)(c >> 32), j = (uint32_t)c;
    int d = hamming(codes + offs[i], (int)(offs[i + 1] - offs[i]), codes + offs[j],
                    (int)(offs[j + 1] - offs[j]));
    if (d >= 0 && d <= k) {
      res->a.push_back(i);
      res->b.push_back(j);
      res->d.push_back(d);
    }
  }
  return res;
}

// Paired-chain self search: SymDel steps 1-3 over the paired variants, step
// 4 keeps Lev(a_i, a_j) + Lev(b_i, b_j) <= k. Records are (a_i, b_i) for
// i < n, two CSR sets with the same n.
void* or_paired_self_search(const uint8_t* ac, const int64_t* ao, const uint8_t* bc,
                            const int64_t* bo, int64_t n, int k) {
  Result* res = new Result();
  MultiMap map;
  std::vector<std::string> vars;
  for (int64_t i = 0; i < n; ++i) {
    paired_variants(seq_at(ac, ao, i), seq_at(bc, bo, i), k, vars);
    for (const std::string& v : vars) {
      std::vector<uint32_t>& ids = map[v];
      if (ids.empty() || ids.back() != (uint32_t)i) ids.push_back((uint32_t)i);
    }
  }
  std::vector<uint64_t> cand;
  self_candidates(map, cand, res->raw);
  for (uint64_t c : cand) {
    uint32_t i = (uint32_t)(c >> 32), j = (uint32_t)c;
    int d = lev_full(ac + ao[i], (int)(ao[i + 1] - ao[i]), ac + ao[j], (int)(ao[j + 1] - ao[j])) +
            lev_full(bc + bo[i], (int)(bo[i + 1] - bo[i]), bc + bo[j], (int)(bo[j + 1] - bo[j]));
    if (d <= k) {
      res->a.push_back(i);
      res->b.push_back(j);
      res->d.push_back(d);
    }
  }
  return res;
}

// Number of paired variants of one record, with multiplicity.
int64_t or_paired_variant_count(const uint8_t* a, int la, const uint8_t* b, int lb, int k) {
  std::vector<std::string> vars;
  paired_variants(std::string(reinterpret_cast<const char*>(a), (size_t)la),
                  std::string(reinterpret_cast<const char*>(b), (size_t)lb), k, vars);
  return (int64_t)vars.size();
}

// The candidate pairs of a self search before verification (unique, sorted),
// with d = -1; raw multiplicity in or_raw.
void* or_self_candidates(const uint8_t* codes, const int64_t* offs, int64_t n, int k) {
  Result* res = new Result();
  MultiMap map;
  build_map(codes, offs, n, k, map);
  std::vector<uint64_t> cand;
  self_candidates(map, cand, res->raw);
  for (uint64_t c : cand) {
    res->a.push_back((uint32_t)(c >> 32));
    res->b.push_back((uint32_t)c);
    res->d.push_back(-1);
  }
  return res;
}

// Query search by SymDel: (q, r, d) with Lev(Q_q, R_r) <= k.
void* or_query_search(const uint8_t* rc, const int64_t* ro, int64_t nr, const uint8_t* qc,
                      const int64_t* qo, int64_t nq, int k) {
  Result* res = new Result();
  MultiMap map;
  build_map(rc, ro, nr, k, map);
  std::vector<uint64_t> cand;
  query_candidates(map, qc, qo, nq, k, cand, res->raw);
  for (uint64_t c : cand) {
    uint32_t q = (uint32_t)(c >> 32), r = (uint32_t)c;
    int d = lev_full(qc + qo[q], (int)(qo[q + 1] - qo[q]), rc + ro[r], (int)(ro[r + 1] - ro[r]));
    if (d <= k) {
      res->a.push_back(q);
      res->b.push_back(r);
      res->d.push_back(d);
    }
  }
  return res;
}

// Query search in Hamming mode: (q, r, d) with equal lengths and d =
// Hamming(Q_q, R_r) <= k, from the SymDel candidates.
void* or_query_search_hamming(const uint8_t* rc, const int64_t* ro, int64_t nr, const uint8_t* qc,
                              const int64_t* qo, int64_t nq, int k) {
  Result* res = new Result();
  MultiMap map;
  build_map(rc, ro, nr, k, map);
  std::vector<uint64_t> cand;
  query_candidates(map, qc, qo, nq, k, cand, res->raw);
  for (uint64_t c : cand) {
    uint32_t q = (uint32_t)(c >> 32), r = (uint32_t)c;
    int d = hamming(qc + qo[q], (int)(qo[q + 1] - qo[q]), rc + ro[r], (int)(ro[r + 1] - ro[r]));
    if (d >= 0 && d <= k) {
      res->a.push_back(q);
      res->b.push_back(r);
      res->d.push_back(d);
    }
  }
  return res;
}

// Weighted query: SymDel candidates at Levenshtein radius k, rescored with the
// weighted alignment cost, kept when the score is <= max_score.
void* or_query_weighted(const uint8_t* rc, const int64_t* ro, int64_t nr, const uint8_t* qc,
                        const int64_t* qo, int64_t nq, int k, const uint8_t* subst, int indel,
                        int max_score) {
  Result* res = new Result();
  MultiMap map;
  build_map(rc, ro, nr, k, map);
  std::vector<uint64_t> cand;
  query_candidates(map, qc, qo, nq, k, cand, res->raw);
  for (uint64_t c : cand) {
    uint32_t q = (uint32_t)(c >> 32), r = (uint32_t)c;
    const uint8_t* a = qc + qo[q];
    int la = (int)(qo[q + 1] - qo[q]);
    const uint8_t* b = rc + ro[r];
    int lb = (int)(ro[r + 1] - ro[r]);
    if (lev_full(a, la, b, lb) > k) continue;
    int s = weighted_full(a, la, b, lb, subst, indel);
    if (s <= max_score) {
      res->a.push_back(q);
      res->b.push_back(r);
      res->d.push_back(s);
    }
  }
  return res;
}

// Definitions written out directly: every pair, full DP.
void* or_brute_self(const uint8_t* codes, const int64_t* offs, int64_t n, int k) {
  Result* res = new Result();
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      int li = (int)(offs[i + 1] - offs[i]), lj = (int)(offs[j + 1] - offs[j]);
      if (std::abs(li - lj) > k) continue;  // Lev >= |length difference|
      int d = lev_full(codes + offs[i], li, codes + offs[j], lj);
      if (d <= k) {
        res->a.push_back((uint32_t)i);
        res->b.push_back((uint32_t)j);
        res->d.push_back(d);
      }
    }
  return res;
}

// Hamming definitions over every pair: equal lengths, mismatches <= k.
void* or_brute_self_hamming(const uint8_t* codes, const int64_t* offs, int64_t n, int k) {
  Result* res = new Result();
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      int d = hamming(codes + offs[i], (int)(offs[i + 1] - offs[i]), codes + offs[j],
                      (int)(offs[j + 1] - offs[j]));
      if (d >= 0 && d <= k) {
        res->a.push_back((uint32_t)i);
        res->b.push_back((uint32_t)j);
        res->d.push_back(d);
      }
    }
  return res;
}

void* or_brute_query_hamming(const uint8_t* rc, const int64_t* ro, int64_t nr, const uint8_t* qc,
                             const int64_t* qo, int64_t nq, int k) {
  Result* res = new Result();
  for (int64_t q = 0; q < nq; ++q)
    for (int64_t r = 0; r < nr; ++r) {
      int d = hamming(qc + qo[q], (int)(qo[q + 1] - qo[q]), rc + ro[r], (int)(ro[r + 1] - ro[r]));
      if (d >= 0 && d <= k) {
        res->a.push_back((uint32_t)q);
        res->b.push_back((uint32_t)r);
        res->d.push_back(d);
      }
    }
  return res;
}

// Paired definition over every pair: Lev(a_i, a_j) + Lev(b_i, b_j) <= k.
void* or_brute_paired(const uint8_t* ac, const int64_t* ao, const uint8_t* bc, const int64_t* bo,
                      int64_t n, int k) {
  Result* res = new Result();
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      int d = lev_full(ac + ao[i], (int)(ao[i + 1] - ao[i]), ac + ao[j], (int)(ao[j + 1] - ao[j])) +
              lev_full(bc + bo[i], (int)(bo[i + 1] - bo[i]), bc + bo[j], (int)(bo[j + 1] - bo[j]));
      if (d <= k) {
        res->a.push_back((uint32_t)i);
        res->b.push_back((uint32_t)j);
        res->d.push_back(d);
      }
    }
  return res;
}

void* or_brute_query(const uint8_t* rc, const int64_t* ro, int64_t nr, const uint8_t* qc,
                     const int64_t* qo, int64_t nq, int k) {
  Result* res = new Result();
  for (int64_t q = 0; q < nq; ++q)
    for (int64_t r = 0; r < nr; ++r) {
      int lq = (int)(qo[q + 1] - qo[q]), lr = (int)(ro[r + 1] - ro[r]);
      if (std::abs(lq - lr) > k) continue;
      int d = lev_full(qc + qo[q], lq, rc + ro[r], lr);
      if (d <= k) {
        res->a.push_back((uint32_t)q);
        res->b.push_back((uint32_t)r);
        res->d.push_back(d);
      }
    }
  return res;
}

void* or_brute_weighted(const uint8_t* rc, const int64_t* ro, int64_t nr, const uint8_t* qc,
                        const int64_t* qo, int64_t nq, const uint8_t* subst, int indel,
                        int max_score) {
  Result* res = new Result();
  for (int64_t q = 0; q < nq; ++q)
    for (int64_t r = 0; r < nr; ++r) {
      int s = weighted_full(qc + qo[q], (int)(qo[q + 1] - qo[q]), rc + ro[r],
                            (int)(ro[r + 1] - ro[r]), subst, indel);
      if (s <= max_score) {
        res->a.push_back((uint32_t)q);
        res->b.push_back((uint32_t)r);
        res->d.push_back(s);
      }
    }
  return res;
}

int64_t or_size(void* h) { return (int64_t)static_cast<Result*>(h)->a.size(); }
int64_t or_raw(void* h) { return static_cast<Result*>(h)->raw; }

void or_copy(void* h, uint32_t* a, uint32_t* b, int32_t* d) {
  Result* r = static_cast<Result*>(h);
  std::memcpy(a, r->a.data(), r->a.size() * sizeof(uint32_t));
  std::memcpy(b, r->b.data(), r->b.size() * sizeof(uint32_t));
  std::memcpy(d, r->d.data(), r->d.size() * sizeof(int32_t));
}

void or_free(void* h) { delete static_cast<Result*>(h); }

}  // extern "C"
