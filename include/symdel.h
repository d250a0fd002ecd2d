/*
 * symdel.h -- C ABI of the MI355X symmetric-deletion neighbour search.
 *
 * Problem (paper, Section II and the XTNeighbor step list of Appendix A):
 * given a list of amino-acid sequences and a distance threshold k, return
 * every pair within Levenshtein distance k as (i, j, d) triplets. The method
 * generates every deletion variant with at most k deleted positions, groups
 * equal variants, emits the id pairs inside each group, removes duplicate
 * pairs and keeps the pairs whose exact distance is <= k.
 *
 * Conventions shared by every entry point
 *   - Sequences are CSR: sequence i is codes[offsets[i] .. offsets[i+1]),
 *     residue codes 0..19 in the order "ACDEFGHIKLMNPQRSTVWY". Lengths must
 *     lie in [1, 24] (a variant is packed exactly into 128 bits: 8 bits of
 *     length and 24 residues of 5 bits). At most 2^32 - 2 sequences.
 *   - Input pointers are host or device memory as the sd_seqs.on_device flag
 *     says. The caller keeps them alive until the call returns (every call
 *     below is synchronous with respect to the host: it returns after the
 *     work it enqueued on `stream` has finished).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). All
 *     device work of a call is enqueued on that stream.
 *   - Every function returns SD_OK (0) or a negative SD_E_* code and never
 *     aborts the process. After an error the context stays usable and
 *     sd_last_error() describes the failure.
 *   - Results are bit-deterministic: the same input gives the same bytes.
 */
#ifndef SYMDEL_H
#define SYMDEL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SD_OK 0
#define SD_E_INVAL (-1)     /* null pointer, bad size or k outside {0, 1, 2} */
#define SD_E_ALPHABET (-2)  /* a residue code >= 20 */
#define SD_E_LENGTH (-3)    /* a sequence length outside [1, 24] */
#define SD_E_TOO_MANY (-4)  /* more sequences or variants than 32-bit ids allow */
#define SD_E_NOMEM (-5)     /* device allocation failed or the HBM budget is exceeded */
#define SD_E_HIP (-6)       /* a HIP runtime error */
#define SD_E_CANCELLED (-7) /* the request was cancelled */
#define SD_E_STATE (-8)     /* the object is in the wrong state for the call */

typedef struct sd_ctx sd_ctx;

/* A sequence set in CSR form (see conventions above). */
typedef struct {
  const uint8_t* codes;   /* residue codes, offsets[n] bytes */
  const int64_t* offsets; /* n + 1 non-decreasing offsets, offsets[0] == 0 */
  int64_t n;              /* number of sequences */
  int32_t on_device;      /* 1: both pointers are device memory; 0: host memory */
} sd_seqs;

/*
 * A result: n triplets (i[t], j[t], d[t]) in structure-of-arrays form.
 * The caller sets on_device before the call (1: leave the arrays in device
 * memory; 0: host memory). The library owns the arrays; release them with
 * sd_pairs_free() before sd_destroy().
 */
typedef struct {
  int64_t n;
  uint32_t* i;
  uint32_t* j;
  uint8_t* d;
  int32_t on_device;
  int32_t reserved;
} sd_pairs;

/* Per-call counters and stage timings of the last search on a context. */
#define SD_MAX_STAGES 16
typedef struct {
  int64_t n_seqs;         /* sequences searched */
  int64_t n_keys;         /* deletion variants generated (with multiplicity) */
  int64_t n_cand_raw;     /* candidate pairs emitted inside groups (with multiplicity) */
  int64_t n_cand_unique;  /* distinct candidate pairs */
  int64_t n_pairs;        /* pairs returned */
  int32_t n_stages;       /* valid entries below (0 unless SD_OPT_TIMING is on) */
  int32_t n_sort_passes;  /* radix passes run by the grouping sort */
  int64_t n_big_segments; /* hashed path: hash segments too large for LDS (full-key path) */
  char stage_name[SD_MAX_STAGES][24];
  double stage_ms[SD_MAX_STAGES];      /* device time between HIP events on `stream` */
  double stage_bytes[SD_MAX_STAGES];   /* algorithmic HBM bytes of the stage */
  int32_t stage_launches[SD_MAX_STAGES];
} sd_stats;

/* Options for sd_set_option. */
#define SD_OPT_TIMING 1  /* 1: record per-stage HIP events (adds no host synchronisation) */
#define SD_OPT_PATH 2       /* grouping path: 0 = automatic, 1 = full-key LSD sort, 2 = hashed segments */
#define SD_OPT_GROUP_CAP 3  /* hashed path: LDS batch capacity, 0 (automatic), 256, 1024, 2048 or 4096 */
#define SD_OPT_GROUP_BITS 4 /* hashed path: hash bits sorted by LSD passes, 0 (automatic) .. 23 */
#define SD_OPT_SORT_ITEMS 5 /* keys-only radix passes: items per thread, 0 (automatic), 16 or 32 */

/*
 * Create a context on HIP device `device`. hbm_budget_bytes bounds the
 * device memory the context may hold at once (0: no bound).
 * Errors: SD_E_INVAL (out == NULL), SD_E_HIP (bad device).
 */
int sd_create(sd_ctx** out, int device, uint64_t hbm_budget_bytes);

/* Release a context and all device memory it holds. NULL is ignored. */
void sd_destroy(sd_ctx* ctx);

/* Set an SD_OPT_* option. Errors: SD_E_INVAL for an unknown option or value. */
int sd_set_option(sd_ctx* ctx, int option, int64_t value);

/*
 * Self search (paper, Appendix A XTNeighbor steps 1-7): every pair i < j of
 * `seqs` with Levenshtein distance d <= k, sorted by (i, j) ascending, with
 * d the exact unit-cost edit distance. Duplicate input sequences give d = 0
 * pairs. k must be 0, 1 or 2.
 * Errors: SD_E_INVAL, SD_E_ALPHABET, SD_E_LENGTH, SD_E_TOO_MANY, SD_E_NOMEM,
 * SD_E_HIP. On error out->n == 0 and nothing needs freeing.
 */
int sd_self_search(sd_ctx* ctx, const sd_seqs* seqs, int k, sd_pairs* out, void* stream);

/*
 * Exact Levenshtein distance of n given pairs (the verification step, paper
 * Appendix A step 7): d_out[t] = Lev(a[ia[t]], b[ib[t]]) capped at 255.
 * ia, ib and d_out are device pointers; a and b follow their on_device flags.
 * Errors: SD_E_INVAL, SD_E_ALPHABET, SD_E_LENGTH, SD_E_NOMEM, SD_E_HIP.
 */
int sd_pair_distance(sd_ctx* ctx, const sd_seqs* a, const sd_seqs* b, const uint32_t* ia,
                     const uint32_t* ib, int64_t n, uint8_t* d_out, void* stream);

/* Counters and stage timings of the last successful search on ctx. */
int sd_get_stats(const sd_ctx* ctx, sd_stats* out);

/*
 * Copy a result into caller-owned arrays of at least pairs->n entries
 * (device memory if dst_on_device, else host memory). The copy is enqueued on
 * `stream` and finished before the call returns.
 * Errors: SD_E_INVAL (null pointers with n > 0), SD_E_HIP.
 */
int sd_pairs_copy(sd_ctx* ctx, const sd_pairs* pairs, uint32_t* i, uint32_t* j, uint8_t* d,
                  int dst_on_device, void* stream);

/* Release the arrays of a result (safe on a zeroed or already freed result). */
void sd_pairs_free(sd_ctx* ctx, sd_pairs* pairs);

/* Static text for an SD_* code. */
const char* sd_strerror(int code);

/* Text of the last error on ctx ("" if none). Valid until the next call on ctx. */
const char* sd_last_error(const sd_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SYMDEL_H */
