/*
 * burr_oracle.h - plain sequential CPU oracle for Bumped Ribbon Retrieval
 * (BuRR) with the parallel scheme of bumping keys at range boundaries.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this code: only tests/, the smoke check and the benchmark's CPU
 * baseline leg may use it. It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * Source: Becht, Lehmann, Sanders, "Brief Announcement: Parallel Construction
 * of Bumped Ribbon Retrieval" (arXiv 2411.12365). The paper defines the method
 * at concept level (Sec. 2 "Preliminaries", Sec. 3 "Parallelization"); every
 * detail it leaves open is fixed by the readings listed in each function's
 * comment in burr_oracle.c.
 *
 * A range-parallel driver (ref_build_mt) builds the same bytes on many
 * threads; it is pinned to the sequential builder by equality of exports.
 *
 * Parity pins: thresholds, solution words and bump sets are pinned by dense
 * GF(2) brute force on tiny inputs, the query invariant, range independence
 * and closed-form bounds (tests/test_oracle_*.py). The hash is a reading of
 * ours (the paper does not define one): parity unpinned against the paper;
 * its structure is pinned against the published MurmurHash3 finalizer and
 * Lemire's multiply-shift range reduction by independent computations.
 */
#ifndef BURR_ORACLE_H
#define BURR_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  REF_OK = 0,
  REF_E_INVALID = -1,
  REF_E_NOMEM = -2,
  REF_E_UNSOLVABLE = -3,
};

typedef struct ref_params {
  uint32_t bucket;          /* b: slots per bucket, a multiple of 64 */
  uint32_t load_num;        /* BuRR layer slots per key = load_num/load_den */
  uint32_t load_den;
  uint32_t final_num;       /* final plain ribbon slots per key */
  uint32_t final_den;
  uint32_t layers;          /* BuRR layers before the final plain layer */
  uint32_t t_lo;            /* middle 2-bit threshold values, 0<t_lo<t_hi<b */
  uint32_t t_hi;
  uint32_t ranges;          /* maximum number of independent ranges per layer */
  uint32_t minbpt;          /* minimum buckets per range */
  uint32_t final_attempts;  /* scale-up attempts of the final layer */
  uint32_t filter_mode;     /* 1: stored value is an r-bit key fingerprint */
  uint64_t seed;
  uint32_t threshold_mode;  /* 0: 2-bit thresholds, 1: 1+-bit thresholds (Sec. 2) */
  uint32_t cut_strategy;    /* range ends (Sec. 3 "Selecting Cut Points"): 0 equal
                               split, 1 minbump, 2 maxprev, 3 diff */
  uint32_t cut_search;      /* buckets searched around each equal-split cut */
  uint32_t pad;
} ref_params;

/* per-layer statistics, index 0..layers_built-1; the final layer is
 * reported by ref_final_info */
typedef struct ref_layer_info {
  uint64_t n;          /* keys entering the layer */
  uint64_t m;          /* slots */
  uint64_t nbuckets;   /* m / b */
  uint64_t nranges;    /* independent ranges */
  uint64_t bumped;     /* keys sent to the next layer */
  uint64_t forced;     /* keys bumped because they cross a range boundary */
  uint64_t pivots;     /* rows placed */
  uint64_t redundant;  /* equations that reduced to 0 = 0 */
  uint64_t steps;      /* XOR-and-shift elimination steps (statistics) */
} ref_layer_info;

typedef struct ref_final_info {
  uint64_t n;
  uint64_t m;
  uint64_t attempt;    /* index of the successful scale-up attempt */
  uint64_t steps;
} ref_final_info;

typedef struct ref_burr ref_burr;

/* hash primitives, exported so tests can check them against independent
 * computations */
uint64_t ref_fmix64(uint64_t k);
uint64_t ref_fastrange(uint64_t h, uint64_t n);
void ref_hash(uint64_t key, uint32_t layer, uint64_t m, uint64_t seed,
              uint64_t* start, uint64_t* coeff);
uint32_t ref_fingerprint(uint64_t key, uint32_t r, uint64_t seed);

/* Build. keys: n host u64; values: host u8 (r<=8) / u16 (r<=16) / u32
 * (r<=32), ignored in filter mode. On success *out owns everything. */
int ref_build(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
              const ref_params* p, ref_burr** out);
void ref_free(ref_burr* h);

/* The same structure built by the range-parallel driver (Sec. 3: every
 * thread solves its own ranges) on `threads` threads (0: all online CPUs).
 * Byte-identical export to ref_build. */
int ref_build_mt(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
                 const ref_params* p, uint32_t threads, ref_burr** out);

/* Layers first_layer..layers-1 and the final layer, built from keys that
 * enter layer first_layer (values as for ref_build); threads as for
 * ref_build_mt (1: sequential). Its export starts at that layer (the header
 * records it). Used to check the deeper layers of a structure whose first
 * layers are too large for the oracle, fed with the GPU's own bumped keys. */
int ref_build_from(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
                   const ref_params* p, uint32_t first_layer, uint32_t threads,
                   ref_burr** out);

/* Layer geometry of a BuRR layer entered by nkeys keys: slots, buckets and
 * ranges (Sec. 3: equal bucket-aligned ranges of at least minbpt buckets). */
void ref_layer_geometry(const ref_params* p, uint64_t nkeys, uint64_t* m, uint64_t* nbuckets,
                        uint64_t* nranges);
/* Buckets [first, last) of range rho. */
void ref_range_buckets(uint64_t nbuckets, uint64_t nranges, uint64_t rho, uint64_t* first,
                       uint64_t* last);
/* Start bucket s / bucket of each key in layer `layer` of m slots. */
void ref_start_buckets(const uint64_t* keys, uint64_t n, uint32_t layer, uint64_t m,
                       uint64_t seed, uint32_t bucket, uint32_t* out);
/* Range rho of layer `layer` (< p->layers) entered by n_layer keys, solved on
 * its own from the n keys whose start slot lies in it (values as for
 * ref_build; ignored in filter mode). Writes the range's threshold codes (one
 * byte per bucket), its column-interleaved solution words ((last - first) *
 * bucket / 64 * r words) and its bumped keys in input order (cap n).
 * REF_E_INVALID if a key starts outside the range. */
int ref_layer_range(const ref_params* p, uint32_t r, uint32_t layer, uint64_t n_layer,
                    uint64_t rho, const uint64_t* keys, const void* values, uint64_t n,
                    uint8_t* codes, uint64_t* W, uint64_t* bumped, uint64_t* nbumped);

/* Query n keys; out has the value width of r (u8/u16/u32). */
int ref_query(const ref_burr* h, const uint64_t* keys, uint64_t n, void* out);

/* Canonical little-endian serialisation; *needed receives the size. */
int ref_export(const ref_burr* h, uint8_t* buf, uint64_t cap, uint64_t* needed);

uint32_t ref_layers_built(const ref_burr* h);
int ref_get_layer_info(const ref_burr* h, uint32_t layer, ref_layer_info* out);
int ref_get_final_info(const ref_burr* h, ref_final_info* out);
/* Keys entering layer `layer` (layer == layers_built: the final layer), in
 * the oracle's own order; copy at most cap keys, return the count. */
uint64_t ref_layer_keys(const ref_burr* h, uint32_t layer, uint64_t* out, uint64_t cap);
/* Thresholds of layer `layer`, one byte per bucket: the 2-bit code index,
 * or with 1+-bit thresholds the threshold itself. */
uint64_t ref_layer_codes(const ref_burr* h, uint32_t layer, uint8_t* out, uint64_t cap);
/* Last bucket of every range of layer `layer` (cut points). */
uint64_t ref_layer_cuts(const ref_burr* h, uint32_t layer, uint64_t* out, uint64_t cap);
/* Solution Z of layer `layer` (layer == layers_built: final), one u32 per slot. */
uint64_t ref_layer_solution(const ref_burr* h, uint32_t layer, uint32_t* out, uint64_t cap);

#ifdef __cplusplus
}
#endif
#endif
