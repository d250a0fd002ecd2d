/*
 * Seeded synthetic CDR3-like sequence generator.
 *
 * This module produces test and benchmark INPUTS only. It holds none of the
 * search method's arithmetic (no deletion variants, no distances, no key
 * packing); both the CPU oracle and the GPU library consume its output.
 *
 * Residue codes are 0..19 in the order "ACDEFGHIKLMNPQRSTVWY" ('C' = 1,
 * 'F' = 4). Sequences are returned in CSR form: sequence i occupies
 * codes[offsets[i] .. offsets[i+1]).
 *
 * Random numbers: SplitMix64 (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), uniform doubles from the top
 * 53 bits, normals by the Box-Muller transform. No library distribution is
 * used, so the byte stream is fixed by the seed on every platform.
 *
 * Recipe (one sequence at a time, i = 0, 1, ...):
 *   - with probability fresh_frac (always for i = 0) a fresh sequence:
 *     L = round-half-away(Normal(15, 2)) clipped to [8, 24], first residue C,
 *     last residue F, interior residues i.i.d. from a Zipf(s=1) distribution
 *     over a permutation of the 20 codes fixed by PERM_SEED;
 *   - otherwise a mutant: copy sequence u (u uniform in [0, i)) and apply 1 or
 *     2 edits (equally likely), each a substitution, insertion or deletion
 *     (equally likely) at a uniform interior position. A substituted residue
 *     is redrawn until it differs. An insertion at L = 24 or a deletion at
 *     L = 8 becomes a substitution at a freshly drawn position, so every
 *     length stays in [8, 24].
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define CDR3_MIN_LEN 8
#define CDR3_MAX_LEN 24
#define CODE_C 1
#define CODE_F 4
#define PERM_SEED 12345ULL
#define TWO_PI 6.283185307179586476925286766559

static inline uint64_t sm64_next(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* uniform in [0, 1) with 53 random bits */
static inline double u01(uint64_t* s) { return (double)(sm64_next(s) >> 11) * 0x1.0p-53; }

/* uniform integer in [0, n) */
static inline int64_t below(uint64_t* s, int64_t n) {
  int64_t r = (int64_t)(u01(s) * (double)n);
  return r < n ? r : n - 1;
}

static double normal(uint64_t* s, double mu, double sigma) {
  double u1 = 1.0 - u01(s); /* (0, 1] */
  double u2 = u01(s);
  return mu + sigma * sqrt(-2.0 * log(u1)) * cos(TWO_PI * u2);
}

typedef struct {
  uint8_t code_of_rank[20];
  double cdf[20];
} residue_table;

static void make_table(residue_table* t) {
  uint64_t s = PERM_SEED;
  for (int r = 0; r < 20; ++r) t->code_of_rank[r] = (uint8_t)r;
  for (int r = 19; r > 0; --r) { /* Fisher-Yates */
    int j = (int)below(&s, r + 1);
    uint8_t tmp = t->code_of_rank[r];
    t->code_of_rank[r] = t->code_of_rank[j];
    t->code_of_rank[j] = tmp;
  }
  double h = 0.0;
  for (int r = 1; r <= 20; ++r) h += 1.0 / r;
  double acc = 0.0;
  for (int r = 1; r <= 20; ++r) {
    acc += (1.0 / r) / h;
    t->cdf[r - 1] = acc;
  }
  t->cdf[19] = 1.0;
}

static inline uint8_t draw_residue(const residue_table* t, uint64_t* s) {
  double u = u01(s);
  int r = 0;
  while (r < 19 && u >= t->cdf[r]) ++r;
  return t->code_of_rank[r];
}

static int fresh(const residue_table* t, uint64_t* s, uint8_t* out) {
  double x = normal(s, 15.0, 2.0);
  long L = lround(x);
  if (L < CDR3_MIN_LEN) L = CDR3_MIN_LEN;
  if (L > CDR3_MAX_LEN) L = CDR3_MAX_LEN;
  out[0] = CODE_C;
  for (long p = 1; p < L - 1; ++p) out[p] = draw_residue(t, s);
  out[L - 1] = CODE_F;
  return (int)L;
}

/* Apply 1 or 2 random interior edits to buf[0..L); returns the new length. */
static int mutate(const residue_table* t, uint64_t* s, uint8_t* buf, int L) {
  int nedits = 1 + (int)below(s, 2);
  for (int e = 0; e < nedits; ++e) {
    int kind = (int)below(s, 3); /* 0 substitution, 1 insertion, 2 deletion */
    if (kind == 1 && L >= CDR3_MAX_LEN) kind = 0;
    if (kind == 2 && L <= CDR3_MIN_LEN) kind = 0;
    if (kind == 0) {
      int p = 1 + (int)below(s, L - 2);
      uint8_t c;
      do { c = draw_residue(t, s); } while (c == buf[p]);
      buf[p] = c;
    } else if (kind == 1) {
      int slot = 1 + (int)below(s, L - 1); /* new residue lands at index slot */
      uint8_t c = draw_residue(t, s);
      memmove(buf + slot + 1, buf + slot, (size_t)(L - slot));
      buf[slot] = c;
      ++L;
    } else {
      int p = 1 + (int)below(s, L - 2);
      memmove(buf + p, buf + p + 1, (size_t)(L - p - 1));
      --L;
    }
  }
  return L;
}

/*
 * Generate n sequences into codes (capacity >= 24 * n) and offsets (n + 1).
 * Returns the total number of residues written.
 */
int64_t cdr3_generate(uint64_t seed, int64_t n, double fresh_frac, uint8_t* codes, int64_t* offsets) {
  residue_table t;
  make_table(&t);
  uint64_t s = seed;
  int64_t pos = 0;
  uint8_t buf[CDR3_MAX_LEN + 4];
  offsets[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    int L;
    if (i == 0 || u01(&s) < fresh_frac) {
      L = fresh(&t, &s, buf);
    } else {
      int64_t u = below(&s, i);
      L = (int)(offsets[u + 1] - offsets[u]);
      memcpy(buf, codes + offsets[u], (size_t)L);
      L = mutate(&t, &s, buf, L);
    }
    memcpy(codes + pos, buf, (size_t)L);
    pos += L;
    offsets[i + 1] = pos;
  }
  return pos;
}

/*
 * Query-set generator for query-versus-reference search. Each sequence is,
 * with probability ref_mut_frac, a 1-2-edit mutant of a uniformly chosen
 * reference sequence; otherwise it follows cdr3_generate's recipe within the
 * set (fresh with probability fresh_frac, else a mutant of an earlier query).
 */
int64_t cdr3_generate_query(uint64_t seed, int64_t n, double fresh_frac, double ref_mut_frac,
                            const uint8_t* ref_codes, const int64_t* ref_offsets, int64_t nref,
                            uint8_t* codes, int64_t* offsets) {
  residue_table t;
  make_table(&t);
  uint64_t s = seed;
  int64_t pos = 0;
  uint8_t buf[CDR3_MAX_LEN + 4];
  offsets[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    int L;
    if (nref > 0 && u01(&s) < ref_mut_frac) {
      int64_t u = below(&s, nref);
      L = (int)(ref_offsets[u + 1] - ref_offsets[u]);
      memcpy(buf, ref_codes + ref_offsets[u], (size_t)L);
      L = mutate(&t, &s, buf, L);
    } else if (i == 0 || u01(&s) < fresh_frac) {
      L = fresh(&t, &s, buf);
    } else {
      int64_t u = below(&s, i);
      L = (int)(offsets[u + 1] - offsets[u]);
      memcpy(buf, codes + offsets[u], (size_t)L);
      L = mutate(&t, &s, buf, L);
    }
    memcpy(codes + pos, buf, (size_t)L);
    pos += L;
    offsets[i + 1] = pos;
  }
  return pos;
}

/*
 * Paired-chain records (two CDR3-like chains per record, for the paired
 * search of the paper's Discussion). Record i is fresh with probability
 * fresh_frac (i = 0 always): both chains follow the fresh recipe. Otherwise
 * it copies a uniformly chosen earlier record and applies one mutate() call
 * (1-2 interior edits) to one of its two chains, chosen uniformly.
 * Capacities: 24 * n residues per chain.
 */
void cdr3_generate_paired(uint64_t seed, int64_t n, double fresh_frac, uint8_t* codes_a,
                          int64_t* offs_a, uint8_t* codes_b, int64_t* offs_b) {
  residue_table t;
  make_table(&t);
  uint64_t s = seed;
  uint8_t ba[CDR3_MAX_LEN + 4], bb[CDR3_MAX_LEN + 4];
  offs_a[0] = 0;
  offs_b[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    int La, Lb;
    if (i == 0 || u01(&s) < fresh_frac) {
      La = fresh(&t, &s, ba);
      Lb = fresh(&t, &s, bb);
    } else {
      int64_t u = below(&s, i);
      La = (int)(offs_a[u + 1] - offs_a[u]);
      Lb = (int)(offs_b[u + 1] - offs_b[u]);
      memcpy(ba, codes_a + offs_a[u], (size_t)La);
      memcpy(bb, codes_b + offs_b[u], (size_t)Lb);
      if (below(&s, 2) == 0)
        La = mutate(&t, &s, ba, La);
      else
        Lb = mutate(&t, &s, bb, Lb);
    }
    memcpy(codes_a + offs_a[i], ba, (size_t)La);
    offs_a[i + 1] = offs_a[i] + La;
    memcpy(codes_b + offs_b[i], bb, (size_t)Lb);
    offs_b[i + 1] = offs_b[i] + Lb;
  }
}

/* count integers, each round(exp(U(ln lo, ln hi))) */
void cdr3_loguniform_sizes(uint64_t seed, int64_t count, double lo, double hi, int64_t* out) {
  uint64_t s = seed;
  double a = log(lo), b = log(hi);
  for (int64_t q = 0; q < count; ++q) {
    double v = exp(a + (b - a) * u01(&s));
    int64_t r = (int64_t)llround(v);
    if (r < (int64_t)lo) r = (int64_t)lo;
    if (r > (int64_t)hi) r = (int64_t)hi;
    out[q] = r;
  }
}

/* Poisson process: count arrival times (seconds) at the given rate (1/s). */
void cdr3_poisson_arrivals(uint64_t seed, int64_t count, double rate, double* out) {
  uint64_t s = seed;
  double t = 0.0;
  for (int64_t q = 0; q < count; ++q) {
    t += -log(1.0 - u01(&s)) / rate;
    out[q] = t;
  }
}

/* Symmetric 20x20 substitution costs: 0 on the diagonal, each off-diagonal
 * pair uniform in {lo, hi} (integers). */
void cdr3_cost_matrix(uint64_t seed, int lo, int hi, uint8_t* out) {
  uint64_t s = seed;
  for (int a = 0; a < 20; ++a) {
    out[a * 20 + a] = 0;
    for (int b = a + 1; b < 20; ++b) {
      uint8_t c = (uint8_t)(lo + below(&s, hi - lo + 1));
      out[a * 20 + b] = c;
      out[b * 20 + a] = c;
    }
  }
}

/* Residue probabilities by code (for tests of the recipe). */
void cdr3_residue_probs(double* out20) {
  residue_table t;
  make_table(&t);
  double prev = 0.0;
  for (int r = 0; r < 20; ++r) {
    out20[t.code_of_rank[r]] = t.cdf[r] - prev;
    prev = t.cdf[r];
  }
}
