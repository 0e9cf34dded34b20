/*
 * fr.h -- exhaustive filtered top-K retrieval on AMD MI355X (gfx950).
 *
 * The operation is the paper's on-GPU hybrid retrieval (Sec. 5.3, "System
 * Implementation", and the appendix "Optimizing System on GPU"): every query
 * is checked against every document by a term predicate in conjunctive
 * normal form (F-TBR), every matching document is scored by the inner
 * product of its embedding with the query embedding (F-EBR), and the K best
 * scores are returned (appendix, "Fast Top K Selection").  Queries are
 * processed in batches that share one pass over the corpus (appendix,
 * "Batch Inference"), and every byte of device memory is reserved when the
 * index is created (appendix, "Memory Pre-Allocation").
 *
 * Conventions for every entry point:
 *  - Return value: FR_OK (0) or a negative fr_status.  On error a
 *    thread-local message is available from fr_last_error(); outputs are
 *    unspecified and the index is unchanged, except FR_EDEVICE, which marks
 *    the index as failed so that later calls return FR_EDEVICE at once.
 *  - The caller owns every pointer it passes; the library never frees or
 *    keeps them.  The library owns the corpus and its workspaces.
 *  - Pointers are host memory unless FR_DEVICE_PTRS is set in `flags`; then
 *    embeddings, ids, queries and outputs are device pointers on the
 *    index's device.  Term lists, CNF batches and K values are always host
 *    memory, because the host validates and compiles them.
 *  - One call at a time per index, except fr_search calls that run on
 *    different streams (at most `n_workspaces` in flight).
 */
#ifndef FR_H
#define FR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr_index fr_index;  /* opaque; owns all device memory */

typedef enum {
  FR_OK = 0,
  FR_EINVAL = -1,        /* bad argument (sizes, term id >= vocab, K > k_max...) */
  FR_ENOMEM = -2,        /* device or pinned allocation failed in fr_create */
  FR_ECAPACITY = -3,     /* more live documents than `capacity` */
  FR_EDUPID = -4,        /* inserting an id that is already live */
  FR_ENOTFOUND = -5,     /* deleting an id that is not live */
  FR_EUNSUPPORTED = -6,  /* configuration or input this library does not handle */
  FR_EDEVICE = -7,       /* a HIP call failed; the index is no longer usable */
  FR_EBUSY = -8          /* no free workspace and FR_NOWAIT was given */
} fr_status;

typedef enum {
  FR_F32 = 0,            /* corpus scored in FP32 on the matrix cores */
  FR_BF16 = 1,           /* BF16 corpus + BF16 query, FP32 accumulate, FP32 rescore */
  FR_FP8_E4M3 = 2        /* OCP E4M3FN corpus with one FP32 scale per row and
                            per query, FP32 accumulate, FP32 rescore */
} fr_dtype;

/* flags */
#define FR_DEVICE_PTRS 1u  /* data pointers are device pointers (see above) */
#define FR_NOWAIT      2u  /* fr_search: return FR_EBUSY instead of waiting for a workspace */
#define FR_GRAPH       4u  /* fr_search: replay the workspace's captured HIP graph of the
                              device sequence (captured on first use and again whenever
                              the tiling, corpus extent or output pointers change); the
                              call's fr_timings entry then has scan_ms == total_ms */
#define FR_ASYNC       8u  /* fr_search: enqueue on `stream` and return even when `stream`
                              is NULL (then the null stream); needs FR_DEVICE_PTRS */
#define FR_PRESELECT  16u  /* fr_search: sign-code coarse pre-selection before exact
                              scoring (see fr_set_quantizer); not with FR_GRAPH */

typedef struct {
  uint64_t capacity;       /* maximum live documents (slots); rounded up to 1024 */
  uint32_t dim;            /* embedding dimension, 1..256 (padded to 64 inside) */
  uint32_t vocab;          /* term ids are in [0, vocab); vocab <= 1<<20 with per-term
                              bitmaps, <= 1<<31 with list_terms */
  uint32_t k_max;          /* largest K a query may ask for, 1..4096 */
  uint32_t rescore_r;      /* BF16/FP8: most approximate candidates rescored in
                              FP32 per query (R), k_max..4096; 0 -> 4096.
                              Ignored for FR_F32 */
  uint32_t rescore_min;    /* BF16/FP8: query q rescores
                              R_q = min(rescore_r, max(rescore_min, 4*k[q]))
                              candidates; 0 -> rescore_r (the same R for all) */
  fr_dtype dtype;
  uint32_t max_batch;      /* most queries per fr_search call (0 -> 1024) */
  uint32_t max_clauses;    /* most clauses per batch (0 -> 8 per query) */
  uint32_t max_literals;   /* most literals per batch (0 -> 32 per query) */
  uint32_t n_workspaces;   /* fr_search calls that may be in flight (0 -> 1) */
  uint32_t cand_cap;       /* candidate slots per query per pass (0 -> default) */
  int device;              /* HIP device ordinal */
  uint32_t quant_bits;     /* sign-code bits per document for FR_PRESELECT searches:
                              0 (none), 64, 128, 256 or 512 (the paper's choice) */
  uint32_t quant_factor;   /* FR_PRESELECT keeps quantK = min(quant_factor * k[q], 65536)
                              documents per query (0 -> 200, the paper's choice) */
  uint32_t list_terms;     /* 0: per-term document bitmaps (vocab / 8 bytes per document).
                              L > 0: each document's terms as a list of at most L ids
                              (4 L bytes per document; appendix "TBR": attribute values
                              padded to maxNumAttr), for large vocabularies.  A search
                              then builds bitmaps of its batch's distinct terms only
                              (at most batch_terms) from the lists, before the mask pass.
                              At most 4096 */
  uint32_t batch_terms;    /* list_terms only: most distinct terms in one search batch,
                              1..1024 (0 -> 1024); a larger batch fails with FR_EINVAL */
} fr_config;

/* A batch of CNF predicates in CSR-of-CSR form (host memory):
 * query q has clauses [clause_off[q], clause_off[q+1]); clause c has
 * literals terms[literal_off[c] .. literal_off[c+1]).  A document matches
 * query q iff for every clause it holds at least one literal term.  A query
 * with no clause matches every live document; an empty clause matches none.
 * Duplicate literals are allowed.  (Sec. 5.3: each TBR query becomes a CNF;
 * appendix "TBR": a clause is met when the document's values overlap it.) */
typedef struct {
  uint32_t n_queries;
  const uint32_t* clause_off;   /* [n_queries + 1], clause_off[0] = 0 */
  const uint32_t* literal_off;  /* [n_clauses + 1], literal_off[0] = 0 */
  const uint32_t* terms;        /* [n_literals] */
} fr_cnf_batch;

/* Per-call statistics of the last completed fr_search (host memory). */
typedef struct {
  uint32_t n_queries;
  uint32_t n_passes;        /* scan passes (1 unless a candidate buffer overflowed) */
  uint64_t candidates;      /* candidates appended over all queries and passes */
  uint64_t n_live;          /* live documents scanned */
  uint64_t n_terms_batch;   /* distinct terms referenced by the batch */
  double   alg_bytes;       /* algorithmic HBM bytes of the scan */
  double   alg_flops;       /* 2 * dim * n_queries * n_slots_scanned */
  float    ms_scan;         /* device time of the first scan pass */
  float    ms_total;        /* device time from the first scan pass to the end of the call's
                              device work (with host buffers, the result copies included) */
  uint32_t n_sparse;        /* queries the sparse routing took out of the scan */
  float    ms_call;         /* device time of the whole call, from its input upload to the end
                              of its device work */
} fr_search_stats;

/* Create an index on `cfg->device` and reserve all its device memory:
 * corpus storage for `capacity` documents (embeddings in the chosen dtype,
 * an FP32 master copy for the rescoring dtypes, per-term document bitmaps
 * of vocab bits per document, ids, live bits) and `n_workspaces` search
 * workspaces sized by max_batch / k_max / rescore_r (appendix, "Memory
 * Pre-Allocation").  `out` receives the handle.  Errors: FR_EINVAL,
 * FR_EUNSUPPORTED, FR_ENOMEM, FR_EDEVICE. */
fr_status fr_create(const fr_config* cfg, fr_index** out);

/* Release everything the index owns (the counterpart of the pre-allocation
 * of fr_create: the appendix, "Memory Pre-Allocation", reserves all memory
 * when the retriever is constructed, so it is returned only here).  NULL is
 * allowed.  Waits for work in flight on the index's streams; pointers the
 * caller passed to earlier calls are never touched.  Always FR_OK. */
fr_status fr_destroy(fr_index* ix);

/* Replace the whole corpus by `n` documents: the dense matrices the search
 * scans are built on the device from them (appendix, "Storing Dense
 * Matrix": embeddings, their quantised copy and the term data are kept as
 * separate dense device arrays; here the embeddings as 32-row matrix-core
 * tiles and the terms as per-term document bitmaps), inside the memory
 * reserved by fr_create (appendix, "Memory Pre-Allocation").
 * emb:      n x dim FP32, row-major (host, or device with FR_DEVICE_PTRS);
 *           values must be finite.
 * ids:      n external ids, unique, each < 0xFFFFFFFF.
 * term_off: n + 1 offsets (host) into `terms` (host); the term list of doc
 *           i is terms[term_off[i] .. term_off[i+1]), ids < vocab,
 *           duplicates allowed.
 * Documents occupy slots 0..n-1 in input order.  Synchronous.
 * Errors: FR_EINVAL (shape, non-finite value, duplicate id, term >= vocab),
 * FR_ECAPACITY (n > capacity), FR_EDEVICE. */
fr_status fr_load_corpus(fr_index* ix, uint64_t n, const float* emb, const uint32_t* ids,
                         const uint64_t* term_off, const uint32_t* terms, uint32_t flags);

/* Keep the corpus current as jobs are created and closed (Sec. 2: the job
 * pool changes daily, new postings appear and old ones close).
 * Delete `n_del` live ids, then insert `n_ins` new documents (same layout
 * as fr_load_corpus, host memory), as one all-or-nothing update: the whole call is
 * validated before any device work (unknown or repeated delete id ->
 * FR_ENOTFOUND; inserting an id that stays live -> FR_EDUPID; too many
 * live docs -> FR_ECAPACITY).  Freed slots are reused.  The update is
 * ordered after every search already issued on the index and before every
 * later one, on the device: it is enqueued on the index's stream behind the
 * searches in flight, later searches on other streams wait for it there, and
 * the call returns without waiting for either (a later search captured into
 * a caller's graph waits on the host instead; searches that a caller
 * replays from its own graph are ordered by the caller).  The inputs are
 * copied into the library's pinned staging before the call returns, so the
 * caller may reuse them at once.  Only an update larger than one staging
 * chunk (16,384 documents) waits on the host, for the previous chunk's
 * copies.  A delete clears exactly the deleted document's term bits, from
 * the term lists the library keeps on the host (a copy of every live
 * document's list, compacted once half of it is stale).
 * `out_epoch` (may be NULL) receives the new corpus epoch (incremented once
 * per successful load or update).  A device error while enqueueing marks
 * the index failed (FR_EDEVICE). */
fr_status fr_update_docs(fr_index* ix, uint64_t n_del, const uint32_t* del_ids,
                         uint64_t n_ins, const uint32_t* ins_ids, const float* ins_emb,
                         const uint64_t* ins_term_off, const uint32_t* ins_terms,
                         uint64_t* out_epoch);

/* Filtered top-K for a batch of n_q queries in one pass over the corpus:
 * the hybrid retrieval of Sec. 5.3 ("System Implementation": a term
 * predicate in conjunctive normal form, then the inner product with the
 * query embedding, then the K best), with the appendix's "EBR" (inner
 * product against every matching document), "Fast Top K Selection"
 * (a score histogram bounds which documents can still reach the top K;
 * the result is exact) and "Batch Inference" (the queries of one call
 * share one scan of the corpus).
 * queries:   n_q x dim FP32 row-major.
 * cnf:       predicates (host, see fr_cnf_batch), cnf->n_queries == n_q.
 * k:         n_q values (host), each 0..k_max.
 * out_ids:   n_q x k_max; row q holds the ids of the best min(k[q],
 *            n_match[q]) matches ordered by (score desc, id asc), then
 *            0xFFFFFFFF.
 * out_scores:n_q x k_max FP32 scores (the FP32 inner product; for BF16/FP8
 *            the FP32 rescored value), then -INFINITY.
 * out_count: n_q entries, min(k[q], n_match[q]).
 * out_nmatch:n_q entries, live documents satisfying the predicate.
 * stream:    NULL without FR_ASYNC -> synchronous on the index's stream.
 *            Otherwise a hipStream_t (NULL with FR_ASYNC: the null
 *            stream); the call is enqueued and returns, and requires
 *            FR_DEVICE_PTRS (inputs and outputs stay valid until the
 *            stream passes the call).  FR_GRAPH needs a non-null stream.
 * For BF16/FP8 indexes the approximate scores select the best min(R_q,
 * n_match) candidates by (approximate score desc, id asc), which are
 * rescored in FP32 and ordered by (FP32 score desc, id asc).
 * Failure marker: a query whose candidates cannot be held even by the
 * second pass (more documents tie within one score bucket than `cand_cap`)
 * gets out_count[q] = 0xFFFFFFFF and a padding row; n_match is still
 * exact.  A synchronous call with host buffers then returns
 * FR_EUNSUPPORTED; an asynchronous or device-pointer call returns FR_OK
 * when it was enqueued, so the caller must check out_count for the marker
 * once the stream has passed the call.
 * Errors: FR_EINVAL, FR_EBUSY (FR_NOWAIT and no free workspace),
 * FR_EUNSUPPORTED, FR_EDEVICE. */
fr_status fr_search(fr_index* ix, uint32_t n_q, const float* queries, const fr_cnf_batch* cnf,
                    const uint32_t* k, uint32_t* out_ids, float* out_scores,
                    uint32_t* out_count, uint64_t* out_nmatch, void* stream, uint32_t flags);

/* fr_search for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * same search as fr_search with FR_DEVICE_PTRS (same arguments, results and
 * failure marker; `flags` must hold FR_DEVICE_PTRS and may add FR_ASYNC),
 * but the per-search device memory (query tiles, thresholds, histograms,
 * candidate buffers, predicate masks, selection buffers) is laid out in a
 * fixed 128 MiB scratch array that each device holds in the library's code
 * object until the process ends; the call makes no allocation of any kind.
 * The caller passes device queries and device outputs as for fr_search.
 * Limit: the call's workspace (about n_q x (cand_cap x 8 + 128 KiB FP32 or
 * 256 KiB BF16/FP8 + rescore_r x 12) bytes plus 32 KiB per 1024 documents
 * for every started block of 256 queries) must fit in the 128 MiB; a larger
 * request fails with FR_EINVAL and a message, before any device work.  For
 * example 256 FP32 queries over 1M documents with the default cand_cap fit.
 * Every call on one device shares that device's scratch, which keeps the
 * last call's contents (each call initialises what it reads): calls that
 * overlap in time on one device, from any index or stream, race and must be
 * ordered by the caller (the same stream, or events).
 * Errors: FR_EINVAL, FR_EUNSUPPORTED, FR_EDEVICE. */
fr_status fr_search_noalloc(fr_index* ix, uint32_t n_q, const float* queries,
                            const fr_cnf_batch* cnf, const uint32_t* k, uint32_t* out_ids,
                            float* out_scores, uint32_t* out_count, uint64_t* out_nmatch,
                            void* stream, uint32_t flags);

/* Sign-code coarse pre-selection (Sec. 5.3, last paragraph; appendix
 * "Optimizing System on GPU", Quantization): an OP+ORP-like code per
 * document, of quant_bits bits.  Bit j of a code is set when the sum over
 * bin j of sign * coordinate is positive, bin j being the table entries
 * bin_off[j] .. bin_off[j+1] of (bin_dim, bin_sign); the paper builds the
 * bins from a random permutation of the coordinates cut into equal parts,
 * with a random sign per coordinate, and the caller draws them (the
 * library's tests use several permutations with bins of two coordinates
 * when quant_bits exceeds half the dimension).  Sums are taken in FP32 in
 * table order from +0.
 * An FR_PRESELECT search scores every predicate match by the number of code
 * bits it shares with the query's code (the popcount of the complemented
 * XOR of the words), keeps the quantK = min(quant_factor * k[q], 65536)
 * best by (that score desc, id asc), scores only those in FP32 against the
 * FP32 copy of the embeddings, and returns their top k[q] by (FP32 score
 * desc, id asc), in the layout of fr_search.  out_nmatch still counts every
 * match.  A query with more matches tied at its cut-off score than
 * max(min(quant_factor * k_max, 65536), 16384) gets the failure marker of
 * fr_search.
 * bin_off: quant_bits + 1 entries (host), bin_off[0] = 0, non-decreasing,
 * at most quant_bits x (dim rounded up to 64) entries in all; bin_dim: each
 * < dim; bin_sign: each +1.0f or -1.0f.  Replaces the table and re-encodes
 * every stored document from its FP32 copy; later loads and inserts are
 * encoded as they are written.  Synchronous (waits for searches in flight).
 * Errors: FR_EINVAL (index without quant_bits, malformed table), FR_EDEVICE. */
fr_status fr_set_quantizer(fr_index* ix, const uint32_t* bin_off, const uint32_t* bin_dim,
                           const float* bin_sign);

/* Message of the last failed call on this thread ("" if none). */
const char* fr_last_error(void);

/* Statistics of the last synchronous fr_search (or of the last one whose
 * stream has completed when fr_stats is called).  */
fr_status fr_stats(fr_index* ix, fr_search_stats* out);

/* Device times of the most recent fr_search calls (at most `max`, oldest
 * first, at most 64 remembered): scan_ms[i] is the first scan pass,
 * total_ms[i] from the first scan pass to the end of the call's device work
 * (both measured with HIP events on the call's stream).  `n` receives how many
 * were written; waits for those calls to finish.  Either array may be
 * NULL. */
fr_status fr_timings(fr_index* ix, uint32_t max, float* scan_ms, float* total_ms, uint32_t* n);

/* Current number of live documents, corpus epoch and slots in use (the
 * highest occupied slot + 1).  Any output may be NULL. */
fr_status fr_info(fr_index* ix, uint64_t* n_live, uint64_t* epoch, uint64_t* n_slots);

/* ---- serving ----------------------------------------------------------- */

/* A request loop over one index (appendix, "Batch Inference": requests are
 * bundled so that one scan of the corpus answers a whole batch; the batch
 * size trades latency for throughput).  Requests are queued by
 * fr_server_submit from any thread; a dispatcher thread forms a batch of
 * everything pending (in submission order, up to max_batch queries and the
 * index's clause and literal limits) whenever fewer than max_inflight
 * batches are on the device, so the batch size follows the arrival rate,
 * and enqueues it on the server's own stream (fr_search with device
 * buffers the server owns); a completion thread copies each finished
 * batch's rows to the caller's buffers.  Batches run and complete in
 * submission order.  Updates go to the index directly (fr_update_docs);
 * they are ordered between batches by the index. */
typedef struct fr_server fr_server;

typedef struct {
  uint32_t max_batch;     /* queries per batch, 1..the index's max_batch (0 -> max_batch) */
  uint32_t max_inflight;  /* batches on the device at once, 1..the index's n_workspaces
                             (0 -> min(2, n_workspaces)); 2 keeps the device busy
                             while the host forms the next batch */
  uint32_t max_wait_us;   /* while no batch is on the device, wait up to this long after
                             the oldest request's arrival for a fuller batch (0 -> never) */
} fr_server_config;

typedef struct {
  uint64_t batches;         /* batches dispatched */
  uint64_t queries;         /* requests dispatched */
  uint64_t failed;          /* requests completed with a status other than FR_OK */
  uint32_t max_batch_seen;  /* largest batch dispatched */
  uint32_t pending;         /* requests waiting for a batch now */
} fr_server_stats;

/* Start a server on `ix` (which must outlive it).  Allocates its stream,
 * events and max_inflight sets of device and pinned batch buffers, and
 * starts its two threads.  Errors: FR_EINVAL, FR_ENOMEM, FR_EDEVICE. */
fr_status fr_server_create(fr_index* ix, const fr_server_config* cfg, fr_server** out);

/* Queue n requests: queries n x dim FP32 (host), their predicates (host,
 * see fr_cnf_batch; cnf->n_queries == n), k (host, each 0..k_max), and
 * t_arrival_ns (host, fr_clock_ns() times; NULL -> now), the times the
 * requests count as arrived for max_wait_us.  All inputs are copied before
 * the call returns.  The results go to caller memory that must stay valid
 * until the requests complete: out_ids / out_scores n x k_max (rows as
 * fr_search writes them), out_count and out_nmatch n entries, and, when not
 * NULL, out_done_ns (n completion times, fr_clock_ns) and out_status (n
 * fr_status values: FR_OK; FR_EUNSUPPORTED for a query marked failed,
 * whose out_count is then 0xFFFFFFFF; or the error of a batch that could
 * not be enqueued, whose rows are padding with count 0xFFFFFFFF).  Requests
 * get consecutive tickets; `out_first_ticket` receives the first.  The whole
 * call is validated first (K > k_max, a term >= vocab, a request with more
 * clauses or literals than one search takes -> FR_EINVAL, nothing queued).
 * Errors: FR_EINVAL (also after fr_server_destroy began). */
fr_status fr_server_submit(fr_server* sv, uint32_t n, const float* queries,
                           const fr_cnf_batch* cnf, const uint32_t* k,
                           const uint64_t* t_arrival_ns, uint32_t* out_ids, float* out_scores,
                           uint32_t* out_count, uint64_t* out_nmatch, uint64_t* out_done_ns,
                           int32_t* out_status, uint64_t* out_first_ticket);

/* Wait until every request with a ticket <= `ticket` has completed (its
 * outputs written).  timeout_ms: 0 polls, 0xFFFFFFFF waits without limit.
 * Errors: FR_EINVAL (ticket never issued), FR_EBUSY (timed out). */
fr_status fr_server_wait(fr_server* sv, uint64_t ticket, uint32_t timeout_ms);

/* Counters since fr_server_create. */
fr_status fr_server_get_stats(fr_server* sv, fr_server_stats* out);

/* Serve every request already queued, stop both threads and release the
 * server's memory.  NULL is allowed. */
fr_status fr_server_destroy(fr_server* sv);

/* The clock of t_arrival_ns and out_done_ns: a monotonic clock in ns. */
uint64_t fr_clock_ns(void);

/* ---- testing and tuning entry points ---------------------------------- */

/* Predicate masks only (step 2 of the hot path, Sec. 5.3): out_bits (host)
 * receives n_q rows of ceil(n_slots/64) 64-bit words; bit s of row q is set
 * iff slot s is live and satisfies query q.  Slot s of fr_load_corpus is
 * input row s; fr_debug_slots maps slots to ids after updates.
 * Synchronous. */
fr_status fr_debug_masks(fr_index* ix, const fr_cnf_batch* cnf, uint64_t* out_bits,
                         uint64_t n_words_per_query);

/* Stored element codes of slots [slot0, slot0+n): out_codes receives
 * n x dpad elements row-major in the index dtype (FP32 values, BF16 bits as
 * uint16, or E4M3FN codes as uint8; dpad = dim rounded up to 64, padding is
 * zero) and, if not NULL, out_scales the n FP8 row scales (1.0 for other
 * dtypes).  Pins the device quantizers.  Synchronous. */
fr_status fr_debug_rows(fr_index* ix, uint64_t slot0, uint64_t n, void* out_codes,
                        float* out_scales);

/* Slot -> id table (host, n entries; 0xFFFFFFFF for a free slot). */
fr_status fr_debug_slots(fr_index* ix, uint32_t* out_ids, uint64_t n);

/* First-pass candidates of the last synchronous fr_search (BF16/FP8): for
 * each query up to rescore_r ids and their approximate scores, ordered by
 * (approximate score desc, id asc); `count` receives how many.  Host
 * outputs of n_q x rescore_r. */
fr_status fr_debug_candidates(fr_index* ix, uint32_t n_q, uint32_t* out_ids,
                              float* out_scores, uint32_t* out_count);

/* Scan tiling: `query_blocks` blocks of 32 queries per wavefront (1, 2 or
 * 4) and `waves` wavefronts per workgroup (4 or 8), so one pass over a
 * 1024-document group serves 32*query_blocks*waves queries; and
 * `groups_per_item` groups per work item, used when a batch has more than
 * 32 query tiles (below that the scan cuts the corpus into equal tile
 * ranges, one item per workgroup).  Zeros restore the per-batch
 * defaults.  FR_EUNSUPPORTED if this library has no such scan kernel for the
 * index's dtype and dimension.  Used by the autotuner and by tests. */
fr_status fr_set_tiling(fr_index* ix, uint32_t query_blocks, uint32_t waves,
                        uint32_t groups_per_item);

/* Search strategies (bits of fr_set_strategy and of the autotuner's
 * choice; 0 = both features on; an index starts with FR_STRAT_NO_REFRESH).  FR_STRAT_NO_SPECULATION: start every
 * query from the safe threshold (the K'-th best of the sample) instead of the
 * tighter speculative one (see fr_search).  FR_STRAT_NO_REFRESH: the scan
 * does not raise thresholds from the candidates it has found (the bucket
 * histogram of the appendix's "Fast Top K Selection"); they stay at their
 * start.  Results are identical under every strategy, except that a query
 * taken out of the scan by sparse routing gets its FP32 scores from another
 * summation order (equal within the FP32 dot-product error bound; its ids
 * differ only where such scores tie within it). */
#define FR_STRAT_NO_SPECULATION 1u
#define FR_STRAT_NO_REFRESH     2u
/* Sparse routing, levels 1..7 (appendix "Message Passing between Layers"
 * and "EBR": only the rows that passed the predicate are scored, which pays
 * when few pass): a query with at most n_live * 2^(level-11) matches (0.1%
 * at level 1, 6.25% at level 7), and, for BF16/FP8 indexes, at most its
 * selection size R_q, skips the scan; its matching rows are listed from the
 * predicate masks and scored one by one in FP32, then selected exactly.  The
 * results are the same as without routing (for BF16/FP8 all of such a
 * query's matches are within its R_q, so its FP32 top K is what the
 * rescoring of the scan's candidates gives).  Not used by
 * fr_search_noalloc. */
#define FR_STRAT_SPARSE(level)  ((uint32_t)(level) << 4)
#define FR_STRAT_SPARSE_MASK    0xF0u

/* Set the search strategy: with `pinned` nonzero it is used for every search;
 * otherwise it is the default that tuned choices override.  FR_EINVAL for
 * unknown bits. */
fr_status fr_set_strategy(fr_index* ix, uint32_t strategy, int pinned);

/* The autotuner of the batch form (appendix, "Batch Inference": the batch
 * size trades latency for throughput; here the tile shape, the items and the
 * selection strategy are tuned per batch shape).  On the given batch (host
 * pointers; outputs are scratch) it first searches untimed for half a second
 * (the GPU's clocks settle to their sustained level), then, a trial being
 * one unmeasured search and the median device time of the next ones, it
 * times every scan tiling this library
 * has for the index's dtype and dimension with the default strategy, then
 * the other strategies with the three fastest tilings (3 searches per
 * trial), and the three fastest trials again (9 searches each).  The winner is recorded
 * in the index's tuning table under (device arch, dtype, dimension, vocabulary,
 * ceil(log2 n_q), ceil(log2 of the largest K'), floor(-log2 of the median
 * selectivity)); searches without a pinned tiling use the table entry of
 * their Q and K' buckets (of several selectivity buckets, the one nearest the
 * last measured).  Pinned tilings and strategies are left as they were.  The
 * out_* pointers (may be NULL) receive the choice (groups 0 = per-batch
 * default). */
fr_status fr_autotune(fr_index* ix, uint32_t n_q, const float* queries, const fr_cnf_batch* cnf,
                      const uint32_t* k, uint32_t flags, uint32_t* out_query_blocks,
                      uint32_t* out_waves, uint32_t* out_groups, uint32_t* out_strategy);

/* The configuration a search of n_q queries with these K values (host)
 * would use now: tiling, groups per item (resolved, never 0), strategy, and
 * where it comes from (`out_source`: 0 the per-batch defaults, 1 a pinned
 * tiling, 2 the tuning table).  Any output may be NULL. */
fr_status fr_tuning_choice(fr_index* ix, uint32_t n_q, const uint32_t* k,
                           uint32_t* out_query_blocks, uint32_t* out_waves,
                           uint32_t* out_groups, uint32_t* out_strategy, uint32_t* out_source);

/* Sign codes of slots [slot0, slot0 + n) (host out, n x quant_bits / 64
 * words, bit b of word w = code bit 64 w + b).  Waits for work in flight. */
fr_status fr_debug_codes(fr_index* ix, uint64_t slot0, uint64_t n, uint64_t* out);

/* Write the tuning table as JSON lines (one object per entry: arch, dtype,
 * dim, vocab, q_bucket, k_bucket, sel_bucket, query_blocks, waves,
 * groups_per_item, strategy, ms) to `path`, replacing the file. */
fr_status fr_tuning_save(fr_index* ix, const char* path);

/* Add the entries of a file written by fr_tuning_save that match this
 * index (same arch, dtype, dim and vocab, and a tiling this library has) to its
 * tuning table; other lines are skipped.  `out_loaded` (may be NULL)
 * receives how many were added. */
fr_status fr_tuning_load(fr_index* ix, const char* path, uint32_t* out_loaded);

#ifdef __cplusplus
}
#endif
#endif /* FR_H */
