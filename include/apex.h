/*
 * apex.h - C ABI of the MI355X (gfx950) exhaustive search engine for
 * combinatorial synthesis libraries (CSLs) scored by a structure-factorised
 * surrogate: "APEX: Approximate-but-Exhaustive Search for Ultra-Large
 * Combinatorial Synthesis Libraries" (arXiv 2510.24380).
 *
 * The operation (Section 4, eqs. "factorizer", "surrogate", "apex_topk"):
 *   For every compound chi = (t, {(r, s)}) of the library - one synthon per
 *   R-group ("slot") of reaction t - the engine forms the compound embedding as
 *   the sum of its per-slot synthon rows, evaluates the decoder on it (one linear
 *   layer is the paper's linear probe; deeper decoders are Linear -> act -> ...
 *   -> Linear), and returns the k compounds with the largest objective w . heads
 *   among those whose heads satisfy every inclusive bound lo <= head <= hi.
 *   Equal objectives rank the lower compound id first. No compound is ever
 *   written to memory; only the running candidate set is.
 *
 * Compound ids: reactions in order; inside reaction t with slot sizes
 * (n0, n1[, n2]) the id of assignment (i0, i1[, i2]) is
 *   offset_t + (i0 * n1 + i1) * n2 + i2,      n2 = 1 and i2 = 0 for two slots,
 * where offset_t is the number of compounds of reactions 0..t-1 (a 64-bit
 * integer; libraries may exceed 2^32 compounds).
 *
 * Conventions for every call:
 *   - Every function returns an apex_status; APEX_OK is 0, errors are negative.
 *     No C++ exception crosses this boundary. apex_last_error() gives the text of
 *     the calling thread's most recent error.
 *   - Arguments are validated on the host before anything is launched; an
 *     invalid argument leaves every handle usable.
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary host memory. The library never frees caller memory
 *     and never allocates device memory: all device scratch comes from
 *     caller-provided workspaces whose size the *_workspace_size calls report.
 *     An engine keeps a small pool of pinned host buffers for reading results
 *     back (page-locked host memory, freed by apex_engine_destroy).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls
 *     that launch work return after it has completed on that stream unless stated
 *     otherwise.
 */
#ifndef APEX_H
#define APEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  APEX_OK = 0,
  APEX_E_INVALID = -1,     /* bad argument, shape or state */
  APEX_E_NOMEM = -2,       /* a caller workspace or memory budget is too small */
  APEX_E_DEVICE = -3,      /* a HIP call failed; the text names the hipError_t */
  APEX_E_UNSUPPORTED = -4, /* valid request outside what this library implements */
  APEX_E_PENDING = -5,     /* server: the query has not finished yet */
  APEX_E_CANCELLED = -6    /* server: the query was cancelled */
} apex_status;

enum { APEX_ACT_NONE = 0, APEX_ACT_RELU = 1, APEX_ACT_SILU = 2 };
enum { APEX_PREC_FP32 = 0, APEX_PREC_BF16 = 1, APEX_PREC_FP8 = 2 };
#define APEX_PREC_MASK(p) (1u << (p))

/* Limits of this library. */
#define APEX_MAX_HEADS 32        /* decoder output width H of a one-layer (linear-probe) decoder */
#define APEX_MAX_MLP_HEADS 16    /* decoder output width H with hidden layers */
#define APEX_MAX_CONSTRAINTS 16  /* bounds per query */
#define APEX_MAX_FUSED_QUERIES 32

typedef struct apex_library apex_library;
typedef struct apex_decoder apex_decoder;
typedef struct apex_engine apex_engine;
typedef struct apex_server apex_server;

/* ------------------------------------------------------------------------ */
/* Library (Section 4.2: the hierarchy D = (T, R, S, psi, phi); Appendix A.1) */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t n_reactions;         /* T >= 1 */
  const uint32_t* n_slots;      /* host [T]; each 2 or 3 (R-groups per reaction) */
  const uint32_t* slot_sizes;   /* host [sum n_slots]; synthons per slot, each >= 1 */
  uint32_t d;                   /* embedding width, >= 1 */
  const float* tables;          /* device [rows x d] row-major FP32, rows in
                                   (reaction, slot, synthon) order; these are the
                                   associative embeddings u_{r,s} (eq. "assoc_embeds"). */
} apex_library_desc;

/* Keeps a non-owning reference to desc->tables: the caller keeps that memory
 * alive and unchanged until every engine built on the library is destroyed.
 * Errors: APEX_E_INVALID for a NULL pointer, zero sizes, n_slots not in {2,3},
 * a reaction with more than 2^32-1 compounds in its first slot(s), or a total
 * compound count that overflows 64 bits. */
apex_status apex_library_create(const apex_library_desc* desc, apex_library** out);
apex_status apex_library_destroy(apex_library* lib);
/* Total compounds (sum over reactions of the product of slot sizes). Host only. */
apex_status apex_library_num_compounds(const apex_library* lib, uint64_t* out);
/* Host-side id -> (reaction, synthon index per slot) map; synthon is [n x 3],
 * unused third entries are 0. APEX_E_INVALID if an id is out of range (entries
 * before it are written). */
apex_status apex_decode_ids(const apex_library* lib, const uint64_t* ids, size_t n, uint32_t* reaction,
                            uint32_t* synthon);

/* Associative embeddings (Section 4.2, eq. "assoc_embeds"), the step that
 * produces the library tables: for R-group r (slot s of reaction t, in
 * (reaction, slot) order) with key matrix K_r (d x dU) and each of its synthons
 * with value vector v (dU), the table row is u = K_r v. Run per R-group as one
 * grouped GEMM on the FP32 matrix cores (FP32 accumulation). The library gives
 * the shape (slot sizes, d); its own tables are not read, so `out` may be the
 * very buffer the library was created over (then create engines after this).
 * keys: device [n_slots_total x d x dU] FP32 row-major; values: device
 * [rows x dU] FP32, rows in (reaction, slot, synthon) order; out: device
 * [rows x d] FP32. workspace: device, >= apex_assoc_workspace_size bytes,
 * 256-byte aligned. Synchronous on `stream`. Errors: APEX_E_INVALID (null
 * pointers, misaligned workspace), APEX_E_NOMEM (workspace too small),
 * APEX_E_UNSUPPORTED (dU outside 1..APEX_MAX_ASSOC_DU), APEX_E_DEVICE. */
#define APEX_MAX_ASSOC_DU 256
apex_status apex_assoc_workspace_size(const apex_library* lib, size_t* bytes);
apex_status apex_assoc_embeddings(const apex_library* lib, uint32_t dU, const float* keys, const float* values,
                                  float* out, void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Decoder (eq. "surrogate" and its MLP generalisation)                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t n_layers;      /* 1, 2 or 3 */
  const uint32_t* dims;   /* host [n_layers + 1]; dims[0] = library d, dims[n_layers] = H */
  uint32_t act;           /* APEX_ACT_*, applied after every layer except the last */
  const float* const* W;  /* host array of n_layers device pointers; W[l] is
                             dims[l+1] x dims[l] row-major FP32 */
  const float* const* b;  /* host array of n_layers device pointers; b[l] has dims[l+1] */
} apex_decoder_desc;

/* Keeps non-owning references to the weights until every engine using the
 * decoder has been created (engines copy what they need). Supported shapes
 * (else APEX_E_UNSUPPORTED): H = dims[n_layers] <= APEX_MAX_HEADS with one
 * layer and <= APEX_MAX_MLP_HEADS with two or three; with two or three layers
 * the first hidden width dims[1] is 128, 256 or 512, and with three layers the
 * second hidden width dims[2] is a multiple of 32 up to 512. One layer is the
 * paper's linear probe (the 28-head LinearProbe of Appendix A.8 fits): every
 * head is a sum of per-synthon scalar contributions plus its bias (eq. "apex"),
 * and the search runs the paper's scalar-contribution enumeration (Appendix
 * A.5): per query, every synthon row's objective contribution and constrained
 * head values are formed once, then each compound costs one add and one
 * compare on its objective. Such engines run in FP32 only (no matrix layer is
 * left after the first layer is applied per synthon). Errors:
 * APEX_E_INVALID for NULL pointers, n_layers outside 1..3, a zero width or an
 * unknown activation. */
apex_status apex_decoder_create(const apex_decoder_desc* desc, apex_decoder** out);
apex_status apex_decoder_destroy(apex_decoder* dec);

/* ------------------------------------------------------------------------ */
/* Engine: resident tables and weights for one (library, decoder)            */
/* ------------------------------------------------------------------------ */
/* precisions: OR of APEX_PREC_MASK(p) for the precisions searches may use.
 * Creation runs the one-time precompute of Section 4.3 (eq. "apex"): the first
 * decoder layer is distributed over the slot sum, P = U W1^T (+ b1 on slot 0),
 * once per synthon row, and the later layers are converted to the MFMA operand
 * layouts of each precision (BF16; FP8-E4M3 with per-tensor scales). The
 * workspace (device, >= the size reported, 256-byte aligned) holds all of it
 * and must stay allocated and untouched until apex_engine_destroy. */
apex_status apex_engine_workspace_size(const apex_library* lib, const apex_decoder* dec, uint32_t precisions,
                                       size_t* bytes);
apex_status apex_engine_create(apex_library* lib, apex_decoder* dec, uint32_t precisions, void* workspace,
                               size_t workspace_bytes, void* stream, apex_engine** out);
apex_status apex_engine_destroy(apex_engine* eng);

/* ------------------------------------------------------------------------ */
/* Queries (eq. "apex_topk")                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t head; /* < H */
  float lo;      /* inclusive lower bound; -INFINITY for none */
  float hi;      /* inclusive upper bound; +INFINITY for none */
} apex_constraint;

typedef struct {
  const float* objective_w;            /* host [H]: maximise w . heads (negate to minimise) */
  uint32_t n_constraints;              /* <= APEX_MAX_CONSTRAINTS */
  const apex_constraint* constraints;  /* host */
  uint64_t k;                          /* >= 1 */
  uint32_t precision;                  /* APEX_PREC_*; must be enabled in the engine */
  uint32_t pool_factor;                /* BF16/FP8: the pool_factor * k best low-precision
                                          candidates are rescored in FP32; 0 means 4 */
  uint32_t n_subset;                   /* 0 = whole library */
  const uint32_t* subset;              /* host [n_subset] distinct reaction indices */
  uint32_t flags;                      /* APEX_QUERY_* */
} apex_query;

/* Query flag: the violation-ranked fallback (Section 4.3, the violation c(x)
 * and the lexicographic queue over (c, objective) without its final removal of
 * violators). When fewer than k compounds satisfy every bound, the remaining
 * places go to the least-violating compounds, c(x) = -sum over constraints of
 * max(0, lo - f) + max(0, f - hi), best (largest) c first; violators with equal
 * c rank by lower id. Feasible compounds (c = 0) come first, by objective as
 * without the flag. apex_search and apex_search_noalloc on one-layer
 * (linear-probe) engines only; APEX_E_UNSUPPORTED elsewhere. */
#define APEX_QUERY_KEEP_VIOLATORS 1u

/* Result arrays are the caller's host memory. Short answers are copied in from
 * the library's readback buffer; answers whose arrays exceed 4 MB are copied
 * from the device straight into them (n_found entries each), which is a DMA
 * when they are pinned host memory (hipHostMalloc): a caller that reuses
 * pinned result arrays across searches pays no host copy for them. */
typedef struct {
  uint64_t capacity;    /* entries each array below can hold (>= k) */
  uint64_t* ids;        /* host [capacity] compound ids, best first */
  float* objective;     /* host [capacity] FP32 objective */
  float* heads;         /* host [capacity x H] FP32 heads, or NULL */
  uint32_t* reaction;   /* host [capacity] or NULL */
  uint32_t* synthon;    /* host [capacity x 3] or NULL */
  uint64_t n_found;     /* out: min(k, feasible compounds) */
  uint64_t n_scored;    /* out: compounds the search evaluated */
  uint64_t n_candidates;/* out: candidate entries appended while streaming */
  uint32_t n_reruns;    /* out: chunks re-run after a candidate-buffer overflow */
  float* violation;     /* host [capacity] or NULL: c(x) of each entry (0 when feasible);
                           written for APEX_QUERY_KEEP_VIOLATORS queries */
} apex_result;

/* Device workspace a search of this query needs: candidate buffers, the pool,
 * selection and rescoring scratch. Depends on k, precision and subset only. */
apex_status apex_query_workspace_size(const apex_engine* eng, const apex_query* q, size_t* bytes);

/* One query, synchronous on `stream`. Writes min(k, feasible) entries ordered by
 * (objective desc, id asc). FP32 precision returns the exact top-k of the FP32
 * surrogate; BF16/FP8 enumerate in low precision with bounds relaxed by a
 * per-head margin, keep the pool_factor * k best, rescore those in FP32 with the
 * exact bounds and return the best k of the pool.
 * Errors: APEX_E_INVALID (bad query, head index, NaN bound, lo > hi, k = 0,
 * precision not enabled, result capacity < k), APEX_E_NOMEM (workspace smaller
 * than apex_query_workspace_size), APEX_E_DEVICE. */
apex_status apex_search(apex_engine* eng, const apex_query* q, void* workspace, size_t workspace_bytes,
                        void* stream, apex_result* result);

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): apex_search without a workspace
 * argument. Its device scratch is a static array of APEX_STATIC_SCRATCH_BYTES
 * inside the library, one per GPU, resident from the first call on that GPU
 * until the process ends; the results are read back through ordinary
 * (pageable) host memory. It calls no hipMalloc, hipFree, hipHostMalloc or
 * other device or pinned allocator. The engine's device must be current.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (from several threads or streams) race and must be serialised by the caller.
 * Each call initialises everything it reads, so the contents left by the
 * previous call do not matter. Results equal apex_search's for the same query.
 * Errors: as apex_search, plus APEX_E_NOMEM when the query's workspace
 * (apex_query_workspace_size) exceeds APEX_STATIC_SCRATCH_BYTES (roughly
 * k <= 2e4 in FP32, k <= 3e3 in BF16/FP8 with the default pool) and
 * APEX_E_INVALID when the current device is not the engine's. */
#define APEX_STATIC_SCRATCH_BYTES (64u << 20)
apex_status apex_search_noalloc(apex_engine* eng, const apex_query* q, void* stream, apex_result* result);

/* Several queries fused into one pass over the library: the combine and the
 * decoder run once per compound, the objective, bounds and selection once per
 * query. All queries must use the same precision; n <= APEX_MAX_FUSED_QUERIES.
 * The workspace is the sum of the queries' sizes (apex_batch_workspace_size).
 * Each result equals what apex_search returns for that query alone. */
apex_status apex_batch_workspace_size(const apex_engine* eng, const apex_query* qs, uint32_t n, size_t* bytes);
apex_status apex_search_batch(apex_engine* eng, const apex_query* qs, uint32_t n, void* workspace,
                              size_t workspace_bytes, void* stream, apex_result* results);

/* ------------------------------------------------------------------------ */
/* Serving loop: continuous batching of queries over one engine              */
/* ------------------------------------------------------------------------ */
typedef struct {
  void* pool;               /* device memory for per-query workspaces */
  size_t pool_bytes;        /* admission budget: queries wait until their workspace fits */
  uint32_t max_active;      /* queries enumerating at once, <= APEX_MAX_FUSED_QUERIES */
  void* stream;             /* hipStream_t the server launches on (one: each pass already fuses
                               every active query, and passes depend on each other's thresholds) */
  uint64_t chunk_compounds; /* scheduling granularity; 0 = engine default */
} apex_server_config;

typedef struct {
  uint64_t submitted, completed, cancelled, failed;
  uint64_t active, waiting;
  double p50_latency_ms, p99_latency_ms, max_latency_ms;
  double compounds_per_s;   /* compounds evaluated per second of device-busy time */
  uint64_t compounds_scored;
} apex_server_stats;

/* The server owns a host thread. submit copies the query (and its arrays) and
 * returns a ticket at once; a query is admitted when its workspace fits in the
 * pool and fewer than max_active queries run. Admitted queries join the next
 * chunk pass: every pass evaluates one chunk of reactions once for all active
 * queries that still need it (continuous batching at chunk granularity).
 * poll copies the result into `result` and returns APEX_OK when done,
 * APEX_E_PENDING before (waiting up to timeout_ms), APEX_E_CANCELLED, or the
 * query's own error. A result can be polled once; its ticket is then released. */
apex_status apex_server_create(apex_engine* eng, const apex_server_config* cfg, apex_server** out);
apex_status apex_server_submit(apex_server* srv, const apex_query* q, uint64_t* ticket);
apex_status apex_server_poll(apex_server* srv, uint64_t ticket, apex_result* result, int timeout_ms);
apex_status apex_server_cancel(apex_server* srv, uint64_t ticket);
/* Statistics so far (the _get suffix: in C a function cannot take the name of
 * the struct type apex_server_stats). */
apex_status apex_server_stats_get(apex_server* srv, apex_server_stats* out);
apex_status apex_server_destroy(apex_server* srv);

/* Heads of listed compounds, evaluated with the enumeration arithmetic of one
 * precision (FP32, or BF16/FP8 before rescoring): the per-slot rows are
 * combined in FP32 and the decoder runs on MFMA (a one-layer decoder: the
 * synthons' contributions are summed in slot order). ids: device [n] compound
 * ids; heads: device [n x S] FP32 with S = 16 when H <= 16 and 32 otherwise,
 * columns >= H are 0; an id >= the library size yields a row of NaN. Asynchronous on `stream`. Errors: APEX_E_INVALID (NULL
 * pointers, precision not enabled), APEX_E_DEVICE. */
apex_status apex_engine_heads(apex_engine* eng, const uint64_t* ids, uint32_t n, uint32_t precision, float* heads,
                              void* stream);

/* Quantiles of the FP32 heads over compounds of the library: the percentile
 * thresholds of counter-screening queries (Appendix A.11: e.g. every off-target
 * docking score above its 50th percentile). ids: device [n] compound ids, or
 * NULL for n compounds the engine draws itself (a seeded stratified sample of
 * the whole library, distinct when n is at most the library size);
 * 1 <= n <= APEX_MAX_QUANTILE_COMPOUNDS. levels: host [n_levels] in [0, 1],
 * n_levels <= APEX_MAX_QUANTILE_LEVELS. out: host [n_levels x H]:
 * out[l * H + h] is the levels[l] quantile of head h over the compounds whose
 * head h is finite (linear interpolation between closest ranks, position
 * levels[l] * (n_finite - 1); NaN if none is finite). Uses scratch inside the
 * engine workspace: not safe concurrently with another quantile call on the
 * same engine. Synchronous on `stream`. Errors: APEX_E_INVALID, APEX_E_DEVICE. */
#define APEX_MAX_QUANTILE_COMPOUNDS 8192
#define APEX_MAX_QUANTILE_LEVELS 256
apex_status apex_engine_head_quantiles(apex_engine* eng, const uint64_t* ids, uint32_t n, const float* levels,
                                       uint32_t n_levels, float* out, void* stream);

/* ------------------------------------------------------------------------ */
/* Kernel timing                                                             */
/* ------------------------------------------------------------------------ */
/* Reads and resets the engine's timing of the fused enumeration kernel, then
 * turns timing on (enable != 0) or off. While on, every launch of that kernel
 * during apex_search / apex_search_batch is bracketed by HIP events on the
 * search stream; *ms is the summed event time, *launches the launch count and
 * *compounds the library compounds those launches evaluated. Any output
 * pointer may be NULL. Host only; not safe to call during a concurrent search
 * on the same engine. */
apex_status apex_engine_profile(apex_engine* eng, int enable, double* ms, uint64_t* launches, uint64_t* compounds);

/* ------------------------------------------------------------------------ */
const char* apex_status_string(apex_status s);
const char* apex_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* APEX_H */
