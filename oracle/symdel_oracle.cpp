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
// Weighted mode (Section III D: a Levenshtein prefilter followed by a
// finer, substitution-weighted score): score = minimum-cost global alignment
// with a 20x20 substitution cost table and a fixed indel cost.
//
// Everything is single threaded and unoptimised on purpose.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
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

// Every string obtained from s by deleting a set of m <= k positions, for
// m = 0, 1, ..., min(k, |s|), position sets in lexicographic order. A string
// of length L yields sum_{m<=k} C(L, m) variants counted with multiplicity
// (56 for L = 10, k = 2, Section II A).
void deletion_variants(const std::string& s, int k, std::vector<std::string>& out) {
  out.clear();
  const int L = (int)s.size();
  const int kk = std::min(k, L);
  std::vector<int> pos;
  for (int m = 0; m <= kk; ++m) {
    pos.resize(m);
    for (int t = 0; t < m; ++t) pos[t] = t;
    while (true) {
      std::string v;
      int next = 0;
      for (int x = 0; x < L; ++x) {
        if (next < m && pos[next] == x) {
          ++next;
          continue;
        }
        v.push_back(s[x]);
      }
      out.push_back(v);
      // advance to the next m-subset in lexicographic order
      int t = m - 1;
      while (t >= 0 && pos[t] == L - m + t) --t;
      if (t < 0) break;
      ++pos[t];
      for (int u = t + 1; u < m; ++u) pos[u] = pos[u - 1] + 1;
    }
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

}  // namespace

extern "C" {

int or_lev(const uint8_t* a, int la, const uint8_t* b, int lb) { return lev_full(a, la, b, lb); }

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
