/*
 * burr.h - C ABI of the MI355X Bumped Ribbon Retrieval (BuRR) library.
 *
 * A retrieval structure stores a static function f: S -> {0,1}^r for a set S
 * of distinct 64-bit keys; a query of x in S returns f(x), a query of any
 * other key returns an arbitrary r-bit value (Becht, Lehmann, Sanders,
 * arXiv 2411.12365, Sec. 1). Construction solves a banded GF(2) system in
 * layers: keys that cannot be placed, or whose row would cross the end of an
 * independently solved slot range, are bumped to the next layer (Sec. 2
 * "bumping", Sec. 3 "Bumping"); the last layer is a plain ribbon scaled up
 * until it solves (Sec. 3).
 *
 * Conventions for every entry point:
 *   - pointers named keys/values/out are DEVICE pointers (HIP global memory)
 *     unless the name says host_; they stay owned by the caller and must
 *     remain valid until the call returns (or, for the *_async calls, until
 *     the given stream has passed the call);
 *   - keys are u64; values and query outputs are u8 for r <= 8, u16 for
 *     r <= 16, u32 for r <= 32 (only the low r bits are used);
 *   - return codes: BURR_OK (0) or a negative BURR_E_* code; functions that
 *     return a handle return NULL on error. burr_last_error() gives the code
 *     of the calling thread's last failed call.
 *   - the library never calls PyTorch; it allocates device memory through
 *     the allocator callbacks in burr_params, or through HIP's stream-ordered
 *     allocator when they are NULL.
 */
#ifndef BURR_H
#define BURR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BURR_ABI_VERSION 2u

enum {
  BURR_OK = 0,
  BURR_E_INVALID = -1,    /* bad argument or parameter */
  BURR_E_NOMEM = -2,      /* device or host allocation failed */
  BURR_E_UNSOLVABLE = -3, /* final layer failed every scale-up attempt
                             (in practice: one key given two values) */
  BURR_E_DEVICE = -4,     /* a HIP call failed */
  BURR_E_BUDGET = -5,     /* request larger than a server's memory budget */
  BURR_E_EVICTED = -6     /* a server evicted or dropped the target structure */
};

/* Keep the device copy of every layer's input keys (debugging, parity tests);
 * read them with burr_debug_layer_keys. */
#define BURR_FLAG_KEEP_LAYER_KEYS 1u
/* Allocate the build's temporary buffers for this build only instead of
 * reusing the library's per-device workspace (kept between builds up to
 * BURR_WORKSPACE_CACHE_BYTES bytes per device, default a quarter of the
 * device's memory; see burr_release_workspaces). */
#define BURR_FLAG_NO_WORKSPACE_CACHE 2u

typedef void* (*burr_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*burr_free_fn)(void* ptr, void* stream, void* ctx);

/* Construction parameters. Every field that changes the structure is stored
 * in the handle and in its export. */
typedef struct burr_params {
  uint32_t abi_version;    /* BURR_ABI_VERSION */
  uint32_t bucket;         /* b, slots per bucket; the HIP path supports 64 */
  uint32_t load_num;       /* BuRR layer: m = b*ceil(n*load_num/(load_den*b)) */
  uint32_t load_den;       /*   (overloaded table, Sec. 2; default 97/100) */
  uint32_t final_num;      /* final plain ribbon slots per key, >= 1 */
  uint32_t final_den;      /*   (default 110/100; +1/10 per failed attempt) */
  uint32_t layers;         /* BuRR layers before the final one (default 3) */
  uint32_t t_lo;           /* middle 2-bit threshold values, 0<t_lo<t_hi<b */
  uint32_t t_hi;           /*   (Sec. 2 "2-bit" thresholds; default 16, 32) */
  uint32_t ranges;         /* max independent ranges per layer (Sec. 3) */
  uint32_t minbpt;         /* min buckets per range (Sec. 3 "minbpt") */
  uint32_t final_attempts; /* scale-up attempts of the final layer */
  uint32_t filter_mode;    /* 1: values ignored, store an r-bit fingerprint */
  uint32_t flags;          /* BURR_FLAG_* */
  uint64_t seed;           /* hash seed */
  void* stream;            /* hipStream_t all work is ordered on (a build's
                              back-substitution runs on an internal stream that
                              waits for and is waited on by this one through
                              events); NULL = null stream */
  burr_alloc_fn alloc;     /* device workspace allocator; NULL = HIP pool */
  burr_free_fn free;
  void* alloc_ctx;
  uint32_t threshold_mode; /* BURR_THRESH_*: how bump thresholds are stored (Sec. 2) */
  uint32_t cut_strategy;   /* BURR_CUT_*: where ranges end (Sec. 3 "Selecting Cut
                              Points"); with a strategy other than EQUAL, each range
                              end is chosen among the cut_search buckets around the
                              equal split's (at most half a range away on either
                              side), by the bucket headers of the sorted keys */
  uint32_t cut_search;     /* buckets searched per cut (the paper uses 50) */
  uint32_t reserved;       /* 0 */
} burr_params;

/* threshold_mode: 2-bit thresholds (four values {0, t_lo, t_hi, b} per
 * bucket), or 1+-bit thresholds (one bit per bucket; the exact threshold,
 * any offset, stored only for buckets that bump, found through a rank
 * directory of the bits) (Sec. 2). */
#define BURR_THRESH_2BIT 0u
#define BURR_THRESH_1PLUS 1u
/* cut_strategy (Sec. 3): EQUAL splits the buckets evenly; MINBUMP ends a
 * range at the bucket whose forced bumping bumps the fewest keys; MAXPREV at
 * the bucket with the most keys starting in the w-1 slots before it (keys
 * that can fill the gap); DIFF at the smallest difference of the two. */
#define BURR_CUT_EQUAL 0u
#define BURR_CUT_MINBUMP 1u
#define BURR_CUT_MAXPREV 2u
#define BURR_CUT_DIFF 3u

typedef struct burr_handle burr_handle;
typedef struct burr_batch burr_batch;

typedef struct burr_layer_stats {
  uint64_t n;        /* keys entering the layer */
  uint64_t m;        /* slots */
  uint64_t nbuckets; /* m / b */
  uint64_t nranges;  /* independently solved ranges */
  uint64_t bumped;   /* keys passed to the next layer */
  uint64_t steps;    /* XOR-and-shift elimination steps; counted only by a library
                        built with -DBURR_SOLVE_STATS, else 0 */
  double ms_sort;    /* device time of the sort kernels (hipEvents) */
  double ms_solve;   /* device time of the insertion kernel */
  double ms_backsub; /* device time of back-substitution (on an internal stream,
                        beside the next layer's work) */
  double ms_gather;  /* device time of code packing, bump counts and bumped-key
                        compaction */
} burr_layer_stats;

typedef struct burr_stats {
  uint64_t n;                     /* keys stored */
  uint32_t r;                     /* value bits */
  uint32_t layers_built;          /* BuRR layers with keys */
  burr_layer_stats layer[32];
  uint64_t final_n, final_m, final_attempt;
  uint64_t table_bytes;           /* device bytes of codes + solution words */
  double ms_sort, ms_solve, ms_final, ms_total; /* device time of the build */
} burr_stats;

/* Fills *p with the defaults above (one range, seed 0, no callbacks). */
void burr_default_params(burr_params* p);

/* Builds a structure for n keys (device u64[n]) with r-bit values (device
 * array, see conventions; may be NULL in filter mode). Keys must be
 * distinct; a key repeated with the same value is harmless; n < 0xF0000000
 * (item indices are 32-bit; the same bound holds for a batch's total). The build runs on
 * p->stream and returns when it is complete (it reads one counter per layer
 * back to the host). Returns NULL on error (see burr_last_error). The handle
 * owns one device allocation per layer; free it with burr_free.
 * Method: Sec. 2 (ribbon insertion, 2-bit thresholds, overloading) and
 * Sec. 3 (ranges made independent by bumping keys at range ends, minimum
 * buckets per range, sequential final layer). */
burr_handle* burr_build(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
                        const burr_params* p);

/* burr_build for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same structure, export bytes and query results as burr_build with the same
 * keys, values, r and *p, but the call makes no device allocation (no
 * hipMalloc, hipFree, stream-ordered pool or allocator callback; p->alloc and
 * p->free are ignored) and creates no stream. Its temporary buffers live in a
 * fixed device array of 128 MiB that the library holds on every GPU it runs
 * on until the process ends (enough for about 1.3M keys; more keys:
 * BURR_E_INVALID, with a message on stderr). The structure's tables are
 * written to table_mem (device, 256-byte aligned, caller-owned, table_cap
 * bytes; burr_estimate_build_bytes's table_bytes is enough); it must outlive
 * the handle. BURR_E_NOMEM if table_cap turns out too small. The array is
 * shared by every call on a GPU and keeps the last call's contents: calls
 * that overlap on one GPU would race for it, so the library serializes them
 * (a second call waits until the first has returned). Runs on p->stream and
 * returns when the build is complete; BURR_FLAG_KEEP_LAYER_KEYS is rejected.
 * burr_free releases the handle (not table_mem). Host bookkeeping of the
 * handle is ordinary host memory. */
burr_handle* burr_build_noalloc(const uint64_t* keys, const void* values, uint64_t n,
                                uint32_t r, const burr_params* p, void* table_mem,
                                size_t table_cap);

/* Queries n keys (device u64[n]) into out (device, value width of r): for
 * each layer, skip it if the key's offset is below its bucket's threshold,
 * else return the parity of the key's row AND the table window, per column
 * (Sec. 2, Fig. 1a). Enqueued on `stream` (a hipStream_t; NULL: the null
 * stream) and returns without waiting. */
int burr_query(const burr_handle* h, const uint64_t* keys, uint64_t n, void* out, void* stream);

/* Filter mode only: out[i] = 1 if the stored value of keys[i] equals its
 * fingerprint (always 1 for stored keys; 2^-r false positive rate): a
 * retrieval structure that stores key fingerprints is an approximate
 * membership filter (Sec. 1; the paper's experiments use BuRR as an 8-bit
 * filter, Sec. 4). Same layer walk as burr_query; out is a device u8[n]. */
int burr_contains(const burr_handle* h, const uint64_t* keys, uint64_t n, uint8_t* out,
                  void* stream);

/* Frees a handle returned by burr_build or burr_import. A batch member's
 * handle is not freed this way (BURR_E_INVALID): free its batch. */
void burr_free(burr_handle* h);

/* Sizes and device times of h's build. For a batch member the per-layer and
 * total times are those of the whole batch (its layers were built together). */
int burr_get_stats(const burr_handle* h, burr_stats* s);

/* Builds `count` independent structures at once (many small sets, e.g. one per
 * shard or per document). Structure i stores keys[host_offsets[i],
 * host_offsets[i+1]) (device keys, host offsets, host_offsets[0] = 0, non-
 * decreasing; an empty range gives an empty structure) with host_r[i] value
 * bits (1..32); values (device) are laid out like keys, in elements of the
 * value width of the LARGEST host_r[i]. Each structure is the one burr_build
 * would make from its own keys and p: same layers, tables, export bytes and
 * query results (Sec. 2 and 3 per structure; keys of different structures
 * never meet). The layers of all structures are built together, one launch
 * per kernel and layer, so a batch of small structures fills the GPU like
 * one large build. Runs on p->stream and returns when done; NULL on error. */
burr_batch* burr_build_batch(const uint64_t* keys, const void* values,
                             const uint64_t* host_offsets, const uint32_t* host_r,
                             uint32_t count, const burr_params* p);

/* One size class of a tuning table: structures with up to n_max keys (in the
 * last class also any larger ones) keep at least minbpt buckets per range.
 * ns_per_key and bits_per_key are what burr_autotune measured for this
 * choice (informational). */
typedef struct burr_tune_entry {
  uint64_t n_max;
  uint32_t minbpt;
  uint32_t reserved;
  double ns_per_key;
  double bits_per_key;
} burr_tune_entry;

/* burr_build_batch with each structure's minimum buckets per range (Sec. 3
 * "Minimum Buckets per Thread": it fixes how many ranges, hence boundary
 * bumps, a layer has) taken from the size class of `table` (entries
 * ascending in n_max) that holds its key count, instead of p->minbpt. Each
 * member's export records its own value, so burr_build with that minbpt
 * gives the same structure. BURR_E_INVALID if the table is empty, not
 * strictly ascending or holds a zero minbpt. */
burr_batch* burr_build_batch_tuned(const uint64_t* keys, const void* values,
                                   const uint64_t* host_offsets, const uint32_t* host_r,
                                   uint32_t count, const burr_params* p,
                                   const burr_tune_entry* table, uint32_t entries);

/* Autotuner of the range split per size class (classes: n_max[] ascending,
 * nclasses of them; candidates[]: minimum buckets per range to try, each
 * >= 1), run with p's other settings on the current device and p->stream on
 * synthetic inputs (uniform random keys and r-bit values made on the
 * device). Each timing is the best of reps builds after one warm-up.
 *  - With a size sample (sizes[], nsizes structure sizes, e.g. a sample of
 *    the batches to be built): coordinate descent on whole batches of that
 *    mix. Every class starts at p->minbpt; class by class, a candidate
 *    replaces it if the mixed batch builds more than 3 % faster, or if it
 *    gives smaller tables (fewer bits per key) at no more than 3 % above the
 *    fastest time so far and above the untuned batch's time.
 *  - Without (sizes NULL): each class is timed alone, as batches of about
 *    keys_per_trial keys of structures of the geometric middle of the class
 *    (from n_max[c-1], or n_max[0]/4, to n_max[c]); out[c] keeps the fastest
 *    candidate, among those within 3 % of it p->minbpt if it is one, else
 *    the one with the smallest tables.
 * out receives nclasses entries (with the mix: the mixed batch's ns and bits
 * per key in every entry). Allocates and frees device memory for the
 * synthetic inputs. BURR_OK, or BURR_E_INVALID / NOMEM / DEVICE. */
int burr_autotune(const burr_params* p, uint32_t r, const uint64_t* sizes, uint64_t nsizes,
                  const uint64_t* n_max, uint32_t nclasses, const uint32_t* candidates,
                  uint32_t ncandidates, uint64_t keys_per_trial, uint32_t reps,
                  burr_tune_entry* out);

/* Number of structures in a batch (0 for NULL). */
uint32_t burr_batch_size(const burr_batch* b);

/* Handle of structure i (NULL if out of range). It is valid until the batch
 * is freed and works with burr_query, burr_contains, burr_get_stats,
 * burr_export and burr_debug_layer_keys. */
const burr_handle* burr_batch_member(const burr_batch* b, uint32_t i);

/* Frees a batch and every member's tables. */
void burr_batch_free(burr_batch* b);

/* Canonical little-endian serialisation, version 2 (layout in the library's
 * export code): header (parameters, r, layers built, threshold mode, cut
 * strategy), then per BuRR layer n, m, ranges, the thresholds (packed 2-bit
 * codes, or 1+-bit bit words, count and threshold bytes), the
 * column-interleaved solution words and, with a cut strategy, the last
 * bucket of every range but the last; then the final layer. Copies to host
 * memory; *needed receives the size (pass host_buf = NULL to query it). */
int burr_export(const burr_handle* h, void* host_buf, size_t cap, size_t* needed);

/* Rebuilds a handle from export bytes (host memory); p supplies only the
 * stream and allocator (may be NULL). */
burr_handle* burr_import(const void* host_buf, size_t len, const burr_params* p);

/* With BURR_FLAG_KEEP_LAYER_KEYS: copies up to cap keys that entered layer
 * `layer` (layers_built = the final layer) to host memory, in an unspecified
 * order; returns their number (or a negative code). */
int64_t burr_debug_layer_keys(const burr_handle* h, uint32_t layer, uint64_t* host_out,
                              uint64_t cap);

/* Device bytes a build of n keys with r-bit values is expected to hold:
 * *table_bytes for the finished structure (layer 0 exact, deeper layers and
 * the final one at a bound on the bump rate) and *workspace_bytes for the
 * build's temporary buffers. Host computation only. */
int burr_estimate_build_bytes(uint64_t n, uint32_t r, const burr_params* p,
                              uint64_t* table_bytes, uint64_t* workspace_bytes);

/* ---------------------------------------------------------------------------
 * Serving: a request loop that keeps built structures resident on the device
 * and runs build and query requests concurrently under a device-memory
 * budget (continuous batching). Worker threads inside the library each own
 * one HIP stream; a request runs as soon as its memory fits and a worker is
 * free, while earlier requests are still running. Build requests that are
 * waiting together are packed into one batched build (burr_build_batch), so
 * small builds share launches; every structure is still the one burr_build
 * makes from its own keys, and every query result the one burr_query gives.
 * ------------------------------------------------------------------------- */
typedef struct burr_server burr_server;

#define BURR_SERVER_EVICT_LRU 1u /* evict least recently used idle structures
                                    when a build does not fit the budget */
#define BURR_SERVER_NO_DEVICE 2u /* scheduling only: requests complete without
                                    device work (tests of the admission
                                    policy); results are not computed */

typedef struct burr_server_config {
  uint32_t abi_version;    /* BURR_ABI_VERSION */
  uint32_t workers;        /* worker threads = HIP streams (default 4, >= 1) */
  uint64_t budget_bytes;   /* resident tables + in-flight build workspace */
  uint32_t max_batch;      /* most build requests packed together (default 1024) */
  uint32_t flags;          /* BURR_SERVER_* */
  uint64_t max_batch_keys; /* most keys in one packed build (default 2^28) */
} burr_server_config;

enum { BURR_REQ_BUILD = 1, BURR_REQ_QUERY = 2 };

typedef struct burr_completion {
  uint64_t req_id;
  uint64_t struct_id;  /* build: id of the new structure (= its req_id); query: target */
  uint32_t kind;       /* BURR_REQ_* */
  int32_t status;      /* BURR_OK or a negative code */
  uint64_t n;          /* keys of the request */
  uint64_t batch_id;   /* builds packed into one batched build share it */
  double t_submit_ms;  /* host steady clock, ms since the server was created */
  double t_start_ms;   /* dispatched to a worker */
  double t_end_ms;     /* device work finished */
} burr_completion;

typedef struct burr_server_info {
  uint64_t resident_bytes;  /* tables of resident structures */
  uint64_t inflight_bytes;  /* reserved by running builds */
  uint64_t peak_bytes;      /* largest resident + inflight seen */
  uint64_t resident;        /* resident structures */
  uint64_t pending;         /* submitted, not dispatched */
  uint64_t running;         /* dispatched, not complete */
  uint64_t completed;       /* completions produced */
  uint64_t evictions;       /* structures evicted under pressure */
  uint64_t batches;         /* batched builds run */
} burr_server_info;

/* Fills *c with defaults (budget 0 = unlimited). */
void burr_server_default_config(burr_server_config* c);

/* Creates a server; p gives the construction parameters of every structure
 * (its stream and allocator fields are ignored: workers use their own
 * streams and HIP's pool). NULL on error. */
burr_server* burr_server_create(const burr_server_config* c, const burr_params* p);

/* Enqueues a build of n keys (device) with r-bit values (device, width of r;
 * NULL in filter mode). The arrays must hold their data when the call is
 * made and stay valid until the request's completion. *req_id receives the
 * request id, which is also the structure's id. Returns BURR_E_BUDGET if the
 * build alone exceeds the budget. Builds are admitted in arrival order. */
int burr_server_submit_build(burr_server* s, const uint64_t* keys, const void* values,
                             uint64_t n, uint32_t r, uint64_t* req_id);

/* Enqueues a query of n keys (device) against structure struct_id into out
 * (device, value width of its r). A query of a structure still being built
 * waits for it; one of an unknown, dropped or evicted structure completes
 * with BURR_E_EVICTED. Same lifetime rules as builds. */
int burr_server_submit_query(burr_server* s, uint64_t struct_id, const uint64_t* keys,
                             uint64_t n, void* out, uint64_t* req_id);

/* Moves up to max finished requests into out (host); *got receives their
 * number. With timeout_ms > 0 waits that long for at least one, unless
 * nothing is outstanding. */
int burr_server_poll(burr_server* s, burr_completion* out, uint32_t max, uint32_t* got,
                     int64_t timeout_ms);

/* Waits until every submitted request has finished (completions stay
 * available to burr_server_poll). */
int burr_server_drain(burr_server* s);

/* Releases a resident structure (its memory is returned once no query of it
 * runs). Queries submitted later complete with BURR_E_EVICTED. */
int burr_server_drop(burr_server* s, uint64_t struct_id);

/* Handle of a resident structure (NULL otherwise); valid until it is
 * dropped or evicted. Not for use while a drop may race with it. */
const burr_handle* burr_server_handle(burr_server* s, uint64_t struct_id);

int burr_server_get_info(burr_server* s, burr_server_info* info);

/* Waits for running and pending requests, then frees every structure. */
void burr_server_destroy(burr_server* s);

/* Frees the workspaces the library keeps between builds (device memory
 * allocated with hipMalloc) and the host tables of freed batches it keeps for
 * reuse. Call when no build is running. */
void burr_release_workspaces(void);

int burr_last_error(void);
const char* burr_error_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* BURR_H */
