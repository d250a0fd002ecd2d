// The oracle's SymDel routes against its brute-force all-pairs routes on
// small random sets over a 3-letter alphabet (many neighbours, many repeated
// deletion variants), built with AddressSanitizer and UBSan by
// tests/test_sanitizers.py. Exits 0 and prints "ok" when every pair of
// results is identical.
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
void* or_self_search(const uint8_t*, const int64_t*, int64_t, int);
void* or_self_search_sharded(const uint8_t*, const int64_t*, int64_t, int, int, int);
void* or_self_search_hamming(const uint8_t*, const int64_t*, int64_t, int);
void* or_paired_self_search(const uint8_t*, const int64_t*, const uint8_t*, const int64_t*, int64_t,
                            int);
void* or_query_search(const uint8_t*, const int64_t*, int64_t, const uint8_t*, const int64_t*,
                      int64_t, int);
void* or_query_search_hamming(const uint8_t*, const int64_t*, int64_t, const uint8_t*,
                              const int64_t*, int64_t, int);
void* or_query_weighted(const uint8_t*, const int64_t*, int64_t, const uint8_t*, const int64_t*,
                        int64_t, int, const uint8_t*, int, int);
void* or_brute_self(const uint8_t*, const int64_t*, int64_t, int);
void* or_brute_self_hamming(const uint8_t*, const int64_t*, int64_t, int);
void* or_brute_query_hamming(const uint8_t*, const int64_t*, int64_t, const uint8_t*,
                             const int64_t*, int64_t, int);
void* or_brute_paired(const uint8_t*, const int64_t*, const uint8_t*, const int64_t*, int64_t, int);
void* or_brute_query(const uint8_t*, const int64_t*, int64_t, const uint8_t*, const int64_t*,
                     int64_t, int);
void* or_brute_weighted(const uint8_t*, const int64_t*, int64_t, const uint8_t*, const int64_t*,
                        int64_t, const uint8_t*, int, int);
int64_t or_size(void*);
void or_copy(void*, uint32_t*, uint32_t*, int32_t*);
void or_free(void*);
}

namespace {

uint64_t state = 88172645463325252ull;
uint32_t draw(uint32_t m) {  // xorshift64, uniform enough for test data
  state ^= state << 13;
  state ^= state >> 7;
  state ^= state << 17;
  return (uint32_t)(state % m);
}

struct Set {
  std::vector<uint8_t> codes;
  std::vector<int64_t> offs{0};
  int64_t n() const { return (int64_t)offs.size() - 1; }
};

// n strings of length 1..maxlen over codes 0..alpha-1; every fourth one a
// copy of an earlier string with one edit, so pairs within k are common
Set make(int n, int maxlen, int alpha) {
  Set s;
  for (int x = 0; x < n; ++x) {
    std::vector<uint8_t> w;
    if (x >= 4 && x % 4 == 0) {
      const int y = (int)draw((uint32_t)x);
      w.assign(s.codes.begin() + s.offs[y], s.codes.begin() + s.offs[y + 1]);
      const uint32_t op = draw(3), at = draw((uint32_t)w.size());
      if (op == 0) w[at] = (uint8_t)draw(alpha);
      else if (op == 1 && w.size() > 1) w.erase(w.begin() + at);
      else if ((int)w.size() < maxlen) w.insert(w.begin() + at, (uint8_t)draw(alpha));
    } else {
      const int L = 1 + (int)draw((uint32_t)maxlen);
      for (int t = 0; t < L; ++t) w.push_back((uint8_t)draw(alpha));
    }
    s.codes.insert(s.codes.end(), w.begin(), w.end());
    s.offs.push_back((int64_t)s.codes.size());
  }
  return s;
}

struct Triples {
  std::vector<uint32_t> a, b;
  std::vector<int32_t> d;
};

Triples take(void* h) {
  Triples t;
  const int64_t n = or_size(h);
  t.a.resize(n);
  t.b.resize(n);
  t.d.resize(n);
  if (n) or_copy(h, t.a.data(), t.b.data(), t.d.data());
  or_free(h);
  return t;
}

int failures = 0;
void same(const char* what, int k, void* x, void* y) {
  const Triples p = take(x), q = take(y);
  const bool ok = p.a == q.a && p.b == q.b && p.d == q.d;
  std::printf("%-22s k=%d: %zu and %zu triples%s\n", what, k, p.a.size(), q.a.size(),
              ok ? "" : "  DIFFER");
  failures += !ok;
}

}  // namespace

int main() {
  const Set s = make(400, 9, 3);
  const Set r = make(300, 9, 3);
  const Set q = make(200, 9, 3);
  const Set pa = make(250, 7, 3), pb = make(250, 7, 3);
  std::vector<uint8_t> subst(400);
  for (int x = 0; x < 20; ++x)
    for (int y = 0; y < 20; ++y) subst[x * 20 + y] = x == y ? 0 : (uint8_t)(3 + (x + y) % 2);
  for (int k = 0; k <= 3; ++k) {
    same("self", k, or_self_search(s.codes.data(), s.offs.data(), s.n(), k),
         or_brute_self(s.codes.data(), s.offs.data(), s.n(), k));
    same("self sharded", k, or_self_search_sharded(s.codes.data(), s.offs.data(), s.n(), k, 5, 3),
         or_self_search(s.codes.data(), s.offs.data(), s.n(), k));
    same("self hamming", k, or_self_search_hamming(s.codes.data(), s.offs.data(), s.n(), k),
         or_brute_self_hamming(s.codes.data(), s.offs.data(), s.n(), k));
    same("query", k,
         or_query_search(r.codes.data(), r.offs.data(), r.n(), q.codes.data(), q.offs.data(),
                         q.n(), k),
         or_brute_query(r.codes.data(), r.offs.data(), r.n(), q.codes.data(), q.offs.data(),
                        q.n(), k));
    same("query hamming", k,
         or_query_search_hamming(r.codes.data(), r.offs.data(), r.n(), q.codes.data(),
                                 q.offs.data(), q.n(), k),
         or_brute_query_hamming(r.codes.data(), r.offs.data(), r.n(), q.codes.data(),
                                q.offs.data(), q.n(), k));
    same("paired", k,
         or_paired_self_search(pa.codes.data(), pa.offs.data(), pb.codes.data(), pb.offs.data(),
                               pa.n(), k),
         or_brute_paired(pa.codes.data(), pa.offs.data(), pb.codes.data(), pb.offs.data(), pa.n(),
                         k));
  }
  // weighted: score <= 8 with costs 3, 4 and indel 8 needs Lev <= 2
  same("query weighted", 2,
       or_query_weighted(r.codes.data(), r.offs.data(), r.n(), q.codes.data(), q.offs.data(),
                         q.n(), 2, subst.data(), 8, 8),
       or_brute_weighted(r.codes.data(), r.offs.data(), r.n(), q.codes.data(), q.offs.data(),
                         q.n(), subst.data(), 8, 8));
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
