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
 *   - A context serves one call at a time (calls on one context must not
 *     overlap); separate contexts may run calls concurrently, also on one
 *     device. Inside a call, host-side staging of inputs and results may use
 *     up to 16 short-lived host threads.
 */
#ifndef SYMDEL_H
#define SYMDEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SD_OK 0
#define SD_E_INVAL (-1)     /* null pointer, bad size or k outside {0, 1, 2, 3} */
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
 * sd_pairs_free() before sd_destroy(). Host arrays are pinned memory, the
 * three of one result in one block, which the context keeps after
 * sd_pairs_free() for later results (up to 512 MiB of such blocks).
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
  int64_t n_big_segments; /* hashed path: ranges neither grouping kernel could hold in LDS,
                             grouped by a sort on the full hash instead */
  int64_t n_probe_steps;  /* learned indexes: comparisons made by the lookups' searches */
  int64_t n_stream_groups; /* streamed self search: column groups processed (0: in memory) */
  int64_t n_graph_captures; /* batched queries: graphs captured (SD_OPT_BATCH_GRAPH) */
  int64_t n_graph_launches; /* batched queries: graph launches (a replay reuses a capture) */
  int64_t n_graph_retries;  /* batched queries: tiles run again eagerly after a candidate overflow */
  int64_t n_pair_buckets;   /* self search: buckets of the LDS pair sort (0: global passes) */
  int64_t n_pair_fallbacks; /* self search: bucketed pair sorts redone with global passes because
                               a bucket outgrew LDS */
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
#define SD_OPT_BATCH_TILE 6 /* query batches: at most this many query sequences per tile (0: 4Mi) */
#define SD_OPT_PROBE 7      /* learned indexes: 0 = search the model's window, 1 = binary search over the whole index */
#define SD_OPT_GROUP_BATCHES 8 /* hashed path: LDS batches each workgroup groups in sequence, 0 (automatic: 4) .. 64 */
#define SD_OPT_PAIR_SORT 9  /* candidate pair sort of self searches: 0 automatic (buckets by the
                               top bits of i, each sorted and verified in LDS, up to 2^22
                               sequences; else global passes), 1 one-sweep LSD passes,
                               2 counted LSD passes */
#define SD_OPT_METRIC 10    /* distance of the final filter of every search on the context:
                               SD_METRIC_LEVENSHTEIN (default) or SD_METRIC_HAMMING */
#define SD_OPT_STREAM 11    /* self search in column groups of hash bins (bounded memory):
                               0 automatic (when the variants exceed 2^32 - 2 or the
                               in-memory path would exceed the budget), 1 never, 2 always */
#define SD_OPT_JOIN_ELEMS 15 /* query tiles (eager): query elements a join segment aims at; a
                                tile with fewer than that per index segment joins over coarser
                                segments (unions of index segments); 0 = automatic (the cube
                                root of the tile's element count, at least 64), 1 keeps the
                                index's own segments for any tile */
#define SD_OPT_BATCH_GRAPH 14 /* sd_query_batch as one captured HIP graph: 0 off (tiles with host
                                 synchronisations), 1 on (capture once per batch shape, then replay) */
#define SD_OPT_GROUP_SHAPE 13 /* hashed path grouping kernel at LDS capacity 2048: 0 (256 threads,
                                 five waves per SIMD), 1 (256 threads, four), 2 (512 threads, four) */
#define SD_OPT_STREAM_ELEMS 12 /* streamed self search: variants per column group at most
                                  (0: from the budget, or 80% of free device memory) */

/* Distances of the final filter (paper, Appendix A step 7; Section III C). */
#define SD_METRIC_LEVENSHTEIN 0 /* unit-cost insertions, deletions and substitutions */
#define SD_METRIC_HAMMING 1     /* equal lengths only; the number of differing positions */

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
 * Device-memory provider of a context (not a step of the method: the host
 * framework that owns device memory, e.g. PyTorch's caching allocator, lends
 * it to the search). With alloc and free_fn set, every device allocation the
 * context makes -- a call's scratch, device result arrays, the context's
 * look-back and counter areas, and the arrays of an index built on it -- is
 * taken from alloc(bytes, user) and given back with free_fn(ptr, user); the
 * context then keeps no cache of its own (the provider is expected to cache).
 * alloc must return device memory of the context's device aligned to at
 * least 256 bytes, usable on the stream of the call that asked for it, or
 * NULL: the call in progress then fails with SD_E_NOMEM, gives back what it
 * took and leaves the context usable. free_fn may be handed a block while
 * work on the call's stream that used it is still queued, so the provider
 * must only reuse it in that stream's order (PyTorch's allocator does). An
 * index keeps the free function and user pointer it was built with and
 * calls them from sd_index_free, so `user` must outlive such an index.
 * alloc == free_fn == NULL returns to the context's own hipMalloc pool. The
 * hbm budget of sd_create applies either way. Server workers use contexts of
 * their own and are not affected.
 * Errors: SD_E_INVAL (only one of alloc and free_fn given), SD_E_STATE (the
 * context still holds device results not released with sd_pairs_free).
 */
typedef void* (*sd_alloc_fn)(size_t bytes, void* user);
typedef void (*sd_free_fn)(void* ptr, void* user);
int sd_set_allocator(sd_ctx* ctx, sd_alloc_fn alloc, sd_free_fn free_fn, void* user);

/*
 * Self search (paper, Appendix A XTNeighbor steps 1-7): every pair i < j of
 * `seqs` with Levenshtein distance d <= k, sorted by (i, j) ascending, with
 * d the exact unit-cost edit distance. Duplicate input sequences give d = 0
 * pairs. k must be 0, 1, 2 or 3 (three deletions, the paper's Fig. 2C and
 * Section III D distance 3, run on the hashed grouping path only).
 *
 * Bounded memory (Section II C, "Overcoming memory bottlenecks"; the
 * XTNeighbor-Streaming steps of Appendix A): when the variants exceed
 * 2^32 - 2 or the in-memory path would exceed the context's HBM budget
 * (SD_OPT_STREAM 0), the search runs in column groups of hash bins: one
 * generator pass counts every bin, Next-Fit packs consecutive bins into
 * groups that fit the budget (or SD_OPT_STREAM_ELEMS), and each group is
 * generated, grouped, sorted and verified alone before the pairs of all
 * groups are merged. The result is the same set either way.
 * Errors: SD_E_INVAL, SD_E_ALPHABET, SD_E_LENGTH, SD_E_TOO_MANY, SD_E_NOMEM,
 * SD_E_HIP. On error out->n == 0 and nothing needs freeing.
 */
int sd_self_search(sd_ctx* ctx, const sd_seqs* seqs, int k, sd_pairs* out, void* stream);

/*
 * Self search in Hamming mode (paper, Section III C: for the comparison with
 * a Hamming-only tool the method keeps its candidate generation and changes
 * only the final filter): every pair i < j of equal length whose sequences
 * differ in at most k positions, sorted by (i, j), with d the Hamming
 * distance. Sequences of different lengths never pair. The deletion-variant
 * candidates contain every such pair, since Hamming(a, b) <= k implies
 * Levenshtein(a, b) <= k. Same as sd_self_search with SD_OPT_METRIC =
 * SD_METRIC_HAMMING (the context's option is left as it was).
 * Errors: as sd_self_search.
 */
int sd_self_search_hamming(sd_ctx* ctx, const sd_seqs* seqs, int k, sd_pairs* out, void* stream);

/*
 * Paired-chain self search (paper, Discussion: the CDR3s of both chains of a
 * receptor joined by a token that is never deleted). Record i is the pair
 * (a_i, b_i) of sequences a->codes.. and b->codes.. (both sets hold the same
 * number of records, each chain 1..24 residues). Returns every pair of
 * records i < j with d = Lev(a_i, a_j) + Lev(b_i, b_j) <= k, sorted by (i, j).
 * The deletion variants are those of the joined string a T b with at most k
 * residues deleted and T kept: two records within d <= k share one (delete
 * per chain as in the single-chain argument), so the candidates are
 * complete. k must be 0..3. Errors: as sd_self_search, and SD_E_INVAL when
 * the two sets differ in size.
 */
int sd_paired_self_search(sd_ctx* ctx, const sd_seqs* a, const sd_seqs* b, int k, sd_pairs* out,
                          void* stream);

/*
 * Self search that allocates nothing: for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The result equals sd_self_search's on
 * the same context options (every pair i < j with distance <= k, sorted by
 * (i, j)), written to the caller's device arrays out_i, out_j, out_d of
 * `capacity` entries each; *n_out is the number of pairs.
 *
 * No device memory and no pinned host memory is allocated: every scratch
 * buffer of the call is carved from a fixed device array of
 * SD_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends (its address is resolved by sd_create), and the
 * read-back staging area is the one sd_create allocated. The allocator hook
 * and the HBM budget do not apply. Inputs should be device memory (host
 * inputs are copied into the fixed array). The call returns after its work
 * on `stream` has finished.
 *
 * All calls on one device share that array and each overwrites what the
 * previous one left: calls that overlap on one device (two host threads, or
 * streams without ordering between them) race and must not be made.
 *
 * Errors: as sd_self_search; SD_E_TOO_MANY for more than
 * SD_NOALLOC_MAX_SEQS sequences; SD_E_NOMEM when the call's scratch does
 * not fit the fixed array (heavily repeated inputs make many candidates) or
 * when the result exceeds `capacity` (then *n_out holds the size needed and
 * the arrays are untouched); SD_E_INVAL for a negative capacity or missing
 * output arrays.
 */
#define SD_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
#define SD_NOALLOC_MAX_SEQS 16384
int sd_self_search_noalloc(sd_ctx* ctx, const sd_seqs* seqs, int k, uint32_t* out_i,
                           uint32_t* out_j, uint8_t* out_d, int64_t capacity, int64_t* n_out,
                           void* stream);

/*
 * Exact Levenshtein distance of n given pairs (the verification step, paper
 * Appendix A step 7): d_out[t] = Lev(a[ia[t]], b[ib[t]]) capped at 255.
 * ia, ib and d_out are device pointers; a and b follow their on_device flags.
 * Errors: SD_E_INVAL, SD_E_ALPHABET, SD_E_LENGTH, SD_E_NOMEM, SD_E_HIP.
 */
int sd_pair_distance(sd_ctx* ctx, const sd_seqs* a, const sd_seqs* b, const uint32_t* ia,
                     const uint32_t* ib, int64_t n, uint8_t* d_out, void* stream);

/*
 * Reference index for query-versus-reference search (the database lookup of
 * the paper's Section IV, with the symmetric-deletion variant map of Section
 * II A built once for the reference): every <= k-deletion variant of `ref`,
 * stored on the context's device and owned by the index, read-only after the
 * build (several contexts on the same device may query it concurrently).
 * Release with sd_index_free (no context needed). k must be 0, 1, 2 or 3.
 * Errors: as sd_self_search.
 */
typedef struct sd_index sd_index;
int sd_index_build(sd_ctx* ctx, const sd_seqs* ref, int k, sd_index** out, void* stream);
void sd_index_free(sd_index* index);
/* Size of an index; any output pointer may be NULL. */
int sd_index_info(const sd_index* index, int64_t* n_ref, int64_t* n_keys, int32_t* k,
                  int64_t* bytes);

/*
 * Learned reference index. The paper has no learned component; this one can
 * change the speed of a lookup and never its result. The index holds every
 * <= k-deletion variant of `ref` as its exact 128-bit key (the compressed
 * form of Appendix A widened to 24 residues plus a length field), sorted by
 * key with the reference id beside it, and a model of a key's position:
 *   coordinate  per (length, position) residue frequencies and length shares,
 *               counted over a sample of the keys, give each key its
 *               arithmetic-coding coordinate in [0, 1) (monotone in key order)
 *   stage 1     an FP32 MLP 1 -> SD_MLP_HIDDEN (tanh) -> 1 maps the
 *               coordinate to the rank fraction; it is trained on the device
 *               by full-batch Adam on the mean squared error at cfg.samples
 *               evenly spaced ranks (the parameters with the lowest loss
 *               seen are kept), and its output picks a leaf
 *   stage 2     per leaf, the line through the leaf's first and last key
 *               over the FP64 coordinate
 * After training every leaf stores its exact worst position error eps over
 * all indexed keys, and a lookup searches only [p - eps, p + eps]. Queries
 * (sd_query, sd_query_batch, the weighted forms and the server) accept the
 * index like a hashed one and return identical results; SD_OPT_PROBE = 1
 * switches a context's lookups to a binary search over the whole key array
 * (the same lookup without the model) and sd_stats.n_probe_steps counts the
 * comparisons either way. Release with sd_index_free.
 */
#define SD_MLP_HIDDEN 32
#define SD_MLP_PARAMS (3 * SD_MLP_HIDDEN + 1) /* w1[H], b1[H], w2[H], b2 */
typedef struct {
  int32_t leaves_log2; /* stage-2 leaves = 2^leaves_log2 in [4, 24] (0: about 256 keys per leaf) */
  int32_t steps;       /* Adam steps (0 trains nothing; -1: 400) */
  float lr;            /* Adam learning rate (0: 2e-4) */
  uint32_t samples;    /* training samples, at most 2^24 (0: 65536) */
  int32_t use_init;    /* 1: start from init[]; 0: tanh units placed at sample quantiles */
  float init[SD_MLP_PARAMS];
} sd_learned_config;
int sd_index_build_learned(sd_ctx* ctx, const sd_seqs* ref, int k, const sd_learned_config* cfg,
                           sd_index** out, void* stream);

/* Model of a learned index (SD_E_INVAL for a hashed index). */
typedef struct {
  int32_t leaves;
  int32_t steps;            /* Adam steps taken */
  uint32_t max_eps;         /* largest leaf error bound */
  uint32_t empty_leaves;
  double mean_eps;          /* leaf error bound averaged over the indexed keys */
  double mean_window_log2;  /* log2(2 eps + 1) averaged over the indexed keys */
  float loss_first;         /* training loss of the initial parameters */
  float loss_last;          /* training loss of the returned parameters (the lowest seen) */
  double train_ms, fit_ms;  /* device time of training and of the leaf fit */
  float params[SD_MLP_PARAMS];
} sd_learned_info;
/* loss_curve (host, may be NULL) receives the first min(cap, steps) losses. */
int sd_index_learned_info(const sd_index* index, sd_learned_info* out, float* loss_curve,
                          int32_t cap);

/*
 * Gradient of the stage-1 training loss, computed by the same device kernels
 * the training runs: loss = (1/n) sum_s (f(x_s) - y_s)^2 with
 * f(x) = b2 + sum_j w2[j] tanh(w1[j] x + b1[j]). params (SD_MLP_PARAMS
 * floats), x and y (n floats) are host arrays; grad (SD_MLP_PARAMS floats)
 * and *loss are written on the host. Partial sums are reduced in a fixed
 * order, so the result is deterministic. Errors: SD_E_INVAL (null pointer,
 * n == 0 or n > 2^24), SD_E_NOMEM, SD_E_HIP.
 */
int sd_mlp_gradients(sd_ctx* ctx, const float* params, const float* x, const float* y, uint32_t n,
                     float* grad, float* loss, void* stream);

/*
 * Query search: every (q, r) with Levenshtein(query q, reference r) <= k,
 * returned as (i = q, j = r, d), sorted by (q, r). k must not exceed the
 * index's k. Errors: as sd_self_search, and SD_E_INVAL for an index on
 * another device.
 */
int sd_query(sd_ctx* ctx, const sd_index* index, const sd_seqs* q, int k, sd_pairs* out,
             void* stream);

/*
 * Query search in Hamming mode (Section III C's filter, as in
 * sd_self_search_hamming): every (q, r) of equal length with Hamming
 * distance <= k, returned as (i = q, j = r, d), sorted by (q, r). k must not
 * exceed the index's k. Same as sd_query with SD_OPT_METRIC =
 * SD_METRIC_HAMMING. Errors: as sd_query.
 */
int sd_query_hamming(sd_ctx* ctx, const sd_index* index, const sd_seqs* q, int k, sd_pairs* out,
                     void* stream);

/*
 * Batched query search: nsets query sets against one index in as few
 * pipeline runs as the tile limit allows (SD_OPT_BATCH_TILE); outs[s] is the
 * result of set s exactly as sd_query would return it (query ids local to
 * the set). The caller sets outs[s].on_device for every set. On error no
 * result is returned.
 */
int sd_query_batch(sd_ctx* ctx, const sd_index* index, int nsets, const sd_seqs* sets, int k,
                   sd_pairs* outs, void* stream);

/*
 * Weighted query (Section III D: a Levenshtein prefilter followed by a finer
 * substitution-weighted metric): candidates within Levenshtein distance
 * index.k, rescored by the minimum-cost global alignment with substitution
 * costs subst[a * 20 + b] (host array of 400 bytes) and indel cost `indel`;
 * pairs with score <= max_score are returned with d = score (capped at 255),
 * sorted by (q, r).
 */
int sd_query_weighted(sd_ctx* ctx, const sd_index* index, const sd_seqs* q, const uint8_t* subst,
                      int indel, int max_score, sd_pairs* out, void* stream);

/* sd_query_weighted for nsets query sets at once (as sd_query_batch). */
int sd_query_batch_weighted(sd_ctx* ctx, const sd_index* index, int nsets, const sd_seqs* sets,
                            const uint8_t* subst, int indel, int max_score, sd_pairs* outs,
                            void* stream);

/*
 * Continuous-batching query server over one index (serving query sets as
 * they arrive). Worker threads each hold a context and a HIP stream; an idle
 * worker admits the queued requests in arrival order while their estimated
 * device working memory, together with the batches other workers have in
 * flight, fits hbm_budget, and runs them as one batched query. Requests that
 * arrive while batches run join the next batch, and batches of different
 * workers overlap on the GPU. A request's result is identical to a query of
 * that set alone (sd_query, or sd_query_weighted when `weighted`).
 * The index must outlive the server.
 */
typedef struct sd_server sd_server;
typedef struct {
  int32_t k;                  /* lookup radius, at most the index's k */
  int32_t workers;            /* batches in flight at once, 1..16 (0: 2) */
  int32_t max_batch_requests; /* requests admitted into one batch (0: no limit) */
  int32_t weighted;           /* 1: rescore as sd_query_weighted with the fields below */
  uint64_t hbm_budget;        /* device working memory of all batches in flight (0: no bound) */
  uint8_t subst[400];
  int32_t indel;
  int32_t max_score;
  int32_t probe; /* SD_OPT_PROBE of the workers' contexts (learned indexes) */
} sd_server_config;

/* Errors: SD_E_INVAL (bad config, index on another device), SD_E_NOMEM. */
int sd_server_create(const sd_index* index, int device, const sd_server_config* cfg,
                     sd_server** out);
/* Queue a query set (host memory, copied before return); returns its id. */
int sd_server_submit(sd_server* server, const sd_seqs* q, uint64_t* request_id);
/*
 * Wait up to timeout_ms (-1: forever, 0: do not wait) for a request's result.
 * On SD_OK `out` holds host arrays owned by the caller (release with
 * sd_server_free_pairs) and *latency_s the seconds from submit to completion.
 * SD_E_STATE: not finished within the timeout. SD_E_CANCELLED: cancelled.
 * SD_E_NOMEM: the request alone exceeds hbm_budget. Other codes: the batch's
 * error. A result is returned once.
 */
int sd_server_poll(sd_server* server, uint64_t request_id, int timeout_ms, sd_pairs* out,
                   double* latency_s);
/* Cancel a queued or running request (its poll then returns SD_E_CANCELLED). */
int sd_server_cancel(sd_server* server, uint64_t request_id);
/* Batches run, requests finished and the largest batch so far. */
int sd_server_stats(sd_server* server, int64_t* batches, int64_t* requests, int64_t* max_batch);
void sd_server_free_pairs(sd_pairs* pairs);
/* Stop the workers (queued requests are cancelled) and free the server. */
void sd_server_destroy(sd_server* server);

/*
 * Autotuner: run a sample through candidate values of the context's tunables
 * and keep the fastest in the context (results never depend on them).
 * index == NULL tunes the self search on sets[0] (nsets must be 1) in two
 * stages: a grid over the grouping path, SD_OPT_GROUP_CAP and
 * SD_OPT_SORT_ITEMS, then, one at a time from the best of the grid,
 * SD_OPT_GROUP_BITS (the radix width of the grouping sort: the automatic
 * count plus one or two bits), SD_OPT_PAIR_SORT and SD_OPT_GROUP_SHAPE. With
 * an index it tunes sd_query_batch over the nsets sets: a grid over
 * SD_OPT_BATCH_TILE and SD_OPT_SORT_ITEMS, then SD_OPT_BATCH_GRAPH. Each
 * candidate runs once to warm up and then `reps` times (1..100); the score
 * is the mean wall time of the call. On error the context keeps its
 * previous options.
 * With a cache file set by sd_autotune_cache, a choice stored under the same
 * key (device architecture; self, or query with floor(log2) of the
 * reference count; floor(log2) of the sequence count and of the set count;
 * k) is applied without trials (from_cache = 1,
 * trials = 0, best_s = default_s = 0); otherwise the new choice is added to
 * the file.
 */
typedef struct {
  int32_t trials;
  int32_t path, group_cap, sort_items; /* the chosen SD_OPT_PATH, SD_OPT_GROUP_CAP, SD_OPT_SORT_ITEMS */
  int64_t batch_tile;                  /* the chosen SD_OPT_BATCH_TILE */
  double best_s;                       /* mean seconds per call with the chosen options */
  double default_s;                    /* the same with the options the context had before */
  int32_t group_bits, pair_sort;       /* the chosen SD_OPT_GROUP_BITS, SD_OPT_PAIR_SORT */
  int32_t group_shape, batch_graph;    /* the chosen SD_OPT_GROUP_SHAPE, SD_OPT_BATCH_GRAPH */
  int32_t from_cache;                  /* 1: applied from the cache file without trials */
  int32_t reserved;
} sd_tune_result;
int sd_autotune(sd_ctx* ctx, const sd_index* index, int nsets, const sd_seqs* sets, int k,
                int reps, sd_tune_result* out, void* stream);
/*
 * Set (path != NULL) or clear (path == NULL) the JSON file sd_autotune reads
 * and writes: an object of keys "<arch>/self/s<log2 seqs>/n<log2 sets>/k<k>"
 * or "<arch>/query/r<log2 refs>/s<log2 seqs>/n<log2 sets>/k<k>", each an object of option name -> integer. A file that does
 * not exist or does not parse counts as empty and is rewritten whole (via a
 * temporary file beside it) when a new choice is stored. Nothing is read
 * until sd_autotune runs. SD_E_INVAL if path is longer than 4095 bytes.
 */
int sd_autotune_cache(sd_ctx* ctx, const char* path);

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
