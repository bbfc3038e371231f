/*
 * burr_oracle.c - plain sequential CPU oracle for Bumped Ribbon Retrieval
 * (BuRR) with boundary bumping (arXiv 2411.12365).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline leg of the benchmark. It is deliberately simple and slow: one
 * thread, qsort, bit-by-bit back-substitution and bit-by-bit queries. It shares
 * no code with the HIP library.
 *
 * What it computes, step by step (the paper names the steps; the details are
 * readings, stated at each function):
 *   1. hash every key of a layer to a start slot s, a 64-bit coefficient row c
 *      and an r-bit value v                                 (Sec. 2, ribbon)
 *   2. order the keys by start slot                (Sec. 4, sorting step)
 *   3. cut the slot array into ranges, bump keys whose row would cross a range
 *      end, and insert the remaining keys bucket by bucket with 2-bit bump
 *      thresholds                    (Sec. 2 bumping, Sec. 3 "Bumping")
 *   4. back-substitute the solution and store it column-interleaved
 *   5. recurse on bumped keys; the last layer is a plain ribbon that is
 *      scaled up until it solves                 (Sec. 3 last layer, Sec. 4)
 *   6. query: walk the layers, check the bucket threshold, AND the window of
 *      the table with c and take the parity per column   (Sec. 2, Fig. 1a)
 *
 * Hash: parity unpinned against the paper (the paper does not define one).
 */
#include "burr_oracle.h"

#include <stdlib.h>
#include <string.h>

#define REF_W 64u

/* ------------------------------------------------------------------------ */
/* Hashing (Sec. 2: a key's hash row selects the slots whose XOR is its     */
/* value; spatial coupling confines the row to a window of width w).         */
/* Reading: MurmurHash3's 64-bit finalizer as the mixer, Lemire's            */
/* multiply-shift reduction for the start slot.                              */
/* ------------------------------------------------------------------------ */

/* MurmurHash3 fmix64 (Appleby, public domain): xor-shift 33, multiply,
 * xor-shift 33, multiply, xor-shift 33. A bijection on 64-bit words. */
uint64_t ref_fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

/* floor(h * n / 2^64): maps a uniform 64-bit word to [0, n). */
uint64_t ref_fastrange(uint64_t h, uint64_t n) {
  unsigned __int128 prod = (unsigned __int128)h * (unsigned __int128)n;
  return (uint64_t)(prod >> 64);
}

/* Start slot s in [0, m - w] and coefficient row c (bit j <-> slot s+j,
 * bit 0 forced to 1 so the row starts exactly at s) of `key` in `layer`.
 * Layer salts: fmix64(seed ^ (2*layer+1)) for s, fmix64(seed ^ (2*layer+2))
 * for c. */
void ref_hash(uint64_t key, uint32_t layer, uint64_t m, uint64_t seed,
              uint64_t* start, uint64_t* coeff) {
  uint64_t salt_s = ref_fmix64(seed ^ (2ull * layer + 1ull));
  uint64_t salt_c = ref_fmix64(seed ^ (2ull * layer + 2ull));
  *start = ref_fastrange(ref_fmix64(key ^ salt_s), m - REF_W + 1);
  *coeff = ref_fmix64(key ^ salt_c) | 1ull;
}

/* Filter mode fingerprint (Sec. 1: a retrieval structure storing key
 * fingerprints is an approximate membership filter): the top r bits of
 * fmix64(key ^ fmix64(~seed)). */
uint32_t ref_fingerprint(uint64_t key, uint32_t r, uint64_t seed) {
  uint64_t h = ref_fmix64(key ^ ref_fmix64(~seed));
  return (uint32_t)(h >> (64 - r));
}

/* ------------------------------------------------------------------------ */
/* Data                                                                      */
/* ------------------------------------------------------------------------ */

typedef struct ref_layer {
  ref_layer_info info;
  uint64_t* keys;      /* input keys of this layer */
  uint32_t* vals;      /* their r-bit values */
  uint8_t* code;       /* 2-bit threshold code per bucket */
  uint32_t* Z;         /* solution, one r-bit word per slot */
  uint64_t* W;         /* column-interleaved solution words, m/64 * r */
} ref_layer;

struct ref_burr {
  ref_params p;
  uint32_t r;
  uint64_t n;
  uint32_t built;          /* BuRR layers built */
  ref_layer layer[64];
  ref_layer fin;           /* final plain ribbon layer (code unused) */
  ref_final_info fin_info;
};

static uint32_t ref_mask(uint32_t r) {
  return r >= 32 ? 0xffffffffu : ((1u << r) - 1u);
}

static uint32_t ref_value_at(const void* values, uint32_t r, uint64_t i) {
  if (r <= 8) return ((const uint8_t*)values)[i];
  if (r <= 16) return ((const uint16_t*)values)[i];
  return ((const uint32_t*)values)[i];
}

static void ref_store_value(void* out, uint32_t r, uint64_t i, uint32_t v) {
  if (r <= 8) ((uint8_t*)out)[i] = (uint8_t)v;
  else if (r <= 16) ((uint16_t*)out)[i] = (uint16_t)v;
  else ((uint32_t*)out)[i] = v;
}

/* ------------------------------------------------------------------------ */
/* Layer geometry                                                            */
/* ------------------------------------------------------------------------ */

/* Slots of a BuRR layer with nkeys keys: the overloaded table of Sec. 2
 * (fewer slots than keys), m = b * max(1, ceil(load * n / b)). */
static uint64_t ref_layer_slots(const ref_params* p, uint64_t nkeys) {
  uint64_t b = p->bucket;
  unsigned __int128 num = (unsigned __int128)nkeys * p->load_num;
  unsigned __int128 den = (unsigned __int128)p->load_den * b;
  uint64_t nb = (uint64_t)((num + den - 1) / den);
  if (nb < 1) nb = 1;
  return nb * b;
}

/* Number of independent ranges (one per "thread" in Sec. 3): at most
 * p->ranges, and every range keeps at least minbpt buckets (Sec. 3 "Minimum
 * Buckets per Thread"), and never fewer than 2 buckets. */
static uint64_t ref_layer_ranges(const ref_params* p, uint64_t nbuckets) {
  uint64_t per = p->minbpt < 2 ? 2 : p->minbpt;
  uint64_t R = nbuckets / per;
  if (R > p->ranges) R = p->ranges;
  if (R < 1) R = 1;
  return R;
}

/* First bucket of range rho: floor(rho * B / R) (equal integer split). */
static uint64_t ref_range_first_bucket(uint64_t rho, uint64_t B, uint64_t R) {
  return (uint64_t)(((unsigned __int128)rho * B) / R);
}

/* Final layer slots for attempt a: 64 * max(1, ceil(n * (final + a/10))),
 * i.e. each failed attempt scales the table up by a tenth of n
 * (Sec. 3 and 4: a last layer that does not solve is made larger). */
static uint64_t ref_final_slots(const ref_params* p, uint64_t nkeys, uint32_t a) {
  unsigned __int128 num =
      (unsigned __int128)nkeys * ((uint64_t)p->final_num * 10u + (uint64_t)a * p->final_den);
  unsigned __int128 den = (unsigned __int128)p->final_den * 10u * REF_W;
  uint64_t nb = (uint64_t)((num + den - 1) / den);
  if (nb < 1) nb = 1;
  return nb * REF_W;
}

/* ------------------------------------------------------------------------ */
/* Gaussian elimination on the banded system (Sec. 2, Fig. 1b)               */
/* ------------------------------------------------------------------------ */

enum { INS_PLACED = 0, INS_REDUNDANT = 1, INS_CONFLICT = 2 };

/* Insert the equation (row c starting at slot s, right-hand side v) into the
 * echelon rows C/V: XOR with the row stored at the current leading slot and
 * shift to the next 1-bit until an empty slot is found. Rows are only ever
 * written into empty slots, so undoing an insertion is clearing that slot. */
static int ref_insert(uint64_t* C, uint32_t* V, uint64_t m, uint64_t s,
                      uint64_t c, uint32_t v, uint64_t* placed, uint64_t* steps) {
  uint64_t i = s;
  for (;;) {
    if (i >= m) abort(); /* unreachable: rows stay inside [s, s+63] */
    if (C[i] == 0) {
      C[i] = c;
      V[i] = v;
      *placed = i;
      return INS_PLACED;
    }
    c ^= C[i];
    v ^= V[i];
    (*steps)++;
    if (c == 0) return v == 0 ? INS_REDUNDANT : INS_CONFLICT;
    unsigned j = (unsigned)__builtin_ctzll(c);
    c >>= j;
    i += j;
  }
}

/* Back-substitution from the last slot down: Z[i] = V[i] xor the Z values
 * selected by the higher bits of C[i]; free slots get 0 (any value would be
 * correct, Sec. 1; zero makes the solution unique). */
static void ref_back_substitute(const uint64_t* C, const uint32_t* V, uint32_t* Z,
                                uint64_t m) {
  for (uint64_t i = m; i-- > 0;) {
    if (C[i] == 0) {
      Z[i] = 0;
      continue;
    }
    uint32_t z = V[i];
    for (unsigned j = 1; j < 64; j++) {
      if ((C[i] >> j) & 1ull) {
        if (i + j >= m) abort();
        z ^= Z[i + j];
      }
    }
    Z[i] = z;
  }
}

/* Column-interleaved storage: word W[k*r + col], bit t = bit col of Z[64k+t]. */
static void ref_interleave(const uint32_t* Z, uint64_t m, uint32_t r, uint64_t* W) {
  uint64_t blocks = m / 64;
  memset(W, 0, blocks * r * sizeof(uint64_t));
  for (uint64_t i = 0; i < m; i++)
    for (uint32_t col = 0; col < r; col++)
      if ((Z[i] >> col) & 1u) W[(i / 64) * r + col] |= 1ull << (i % 64);
}

/* ------------------------------------------------------------------------ */
/* Sorting by start slot (Sec. 4 names this sorting step). Plain qsort of   */
/* (start, input index).                                                     */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t s; uint64_t idx; } ref_pos;

static int ref_pos_cmp(const void* a, const void* b) {
  const ref_pos* x = (const ref_pos*)a;
  const ref_pos* y = (const ref_pos*)b;
  if (x->s != y->s) return x->s < y->s ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One BuRR layer with boundary bumping                                      */
/* ------------------------------------------------------------------------ */

/*
 * Range rho of a layer with B buckets cut into R ranges: its buckets
 * [first, last) are processed in order (thresholds, chunks and forced bumps
 * as described at ref_build_layer). The rows live in C/V, which cover the
 * slot window [base, base + mwin): slot s is C[s - base]. order lists the
 * keys of these buckets sorted by start slot; bstart[beta - bbase] is the
 * first position of bucket beta in order and codes[beta - bbase] receives its
 * threshold code. bump[idx] is set for every bumped key (idx = the key's
 * order[].idx); placed is scratch of one entry per key.
 */
static void ref_solve_range(const ref_params* p, uint64_t B, uint64_t R, uint64_t rho,
                            const ref_pos* order, const uint64_t* bstart, uint64_t bbase,
                            const uint64_t* coef, const uint32_t* vals, uint64_t* C,
                            uint32_t* V, uint64_t mwin, uint64_t base, uint8_t* codes,
                            uint8_t* bump, uint64_t* placed, ref_layer_info* info) {
  const uint64_t b = p->bucket;
  const uint64_t theta[4] = {0, p->t_lo, p->t_hi, b};
  uint64_t first = ref_range_first_bucket(rho, B, R);
  uint64_t last = ref_range_first_bucket(rho + 1, B, R); /* exclusive */
  uint64_t range_end = last * b;                         /* slot */
  for (uint64_t beta = first; beta < last; beta++) {
    uint64_t lo = bstart[beta - bbase], hi = bstart[beta - bbase + 1];
    /* forced bumps: only in a range's last bucket, never in the last range */
    unsigned kf = 0;
    if (rho + 1 < R && beta + 1 == last) {
      int any = 0;
      uint64_t omax = 0;
      for (uint64_t t = lo; t < hi; t++) {
        uint64_t s = order[t].s;
        if (s + REF_W > range_end) { /* s > range_end - w */
          any = 1;
          if (s - beta * b > omax) omax = s - beta * b;
        }
      }
      if (any) {
        kf = 4; /* smallest theta above omax; theta[3] = b > omax always */
        for (unsigned k = 0; k < 4; k++)
          if (theta[k] > omax) { kf = k; break; }
      }
    }
    unsigned code = kf;
    for (unsigned k = 3; k > kf; k--) {
      uint64_t nplaced = 0;
      int conflict = 0;
      for (uint64_t t = lo; t < hi && !conflict; t++) {
        uint64_t s = order[t].s;
        uint64_t o = s - beta * b;
        if (o < theta[k - 1] || o >= theta[k]) continue;
        uint64_t id = order[t].idx;
        uint64_t at = 0;
        int res = ref_insert(C, V, mwin, s - base, coef[id], vals[id], &at, &info->steps);
        if (res == INS_PLACED) placed[nplaced++] = at;
        else if (res == INS_REDUNDANT) info->redundant++;
        else conflict = 1;
      }
      if (conflict) {
        for (uint64_t u = 0; u < nplaced; u++) {
          C[placed[u]] = 0;
          V[placed[u]] = 0;
        }
        code = k;
        break;
      }
    }
    codes[beta - bbase] = (uint8_t)code;
    for (uint64_t t = lo; t < hi; t++) {
      uint64_t o = order[t].s - beta * b;
      if (o < theta[code]) {
        bump[order[t].idx] = 1;
        info->bumped++;
        if (beta + 1 == last && rho + 1 < R && order[t].s + REF_W > range_end) info->forced++;
      }
    }
  }
}

/*
 * Builds layer `li` from keys/vals (n of them). Returns the bumped keys in
 * *next_keys / *next_vals (malloc'd) and their count in *next_n.
 *
 * Thresholds (Sec. 2): every bucket of b consecutive slots stores a 2-bit
 * code selecting theta in {0, t_lo, t_hi, b}; keys of the bucket whose offset
 * o = s mod b is below theta are bumped, the others are kept. A bucket is
 * processed in chunks of decreasing offset ([t_hi,b), [t_lo,t_hi), [0,t_lo));
 * the first chunk whose insertion meets an inconsistent equation is undone
 * and theta becomes that chunk's upper end. This yields the smallest theta
 * for which the kept keys stay solvable.
 *
 * Ranges (Sec. 3 "Bumping"): the slot array is cut into equal bucket-aligned
 * ranges. A key of range rho whose row could cross the range end
 * (s > end - w) must be bumped, so its bucket's theta is at least the
 * smallest threshold value above the largest such offset. With b = w = 64
 * this bumps the last bucket of a range completely as soon as one of its
 * keys lies past its first slot - the paper's "bucket B1 needs to be bumped
 * completely because its last key needs to be bumped". Rows of kept keys
 * therefore never leave their range and ranges solve independently; the
 * loop below still runs them one after another.
 */
static int ref_build_layer(ref_burr* h, uint32_t li, const uint64_t* keys,
                           const uint32_t* vals, uint64_t n, uint64_t** next_keys,
                           uint32_t** next_vals, uint64_t* next_n) {
  const ref_params* p = &h->p;
  ref_layer* L = &h->layer[li];
  const uint64_t b = p->bucket;
  const uint64_t m = ref_layer_slots(p, n);
  const uint64_t B = m / b;
  const uint64_t R = ref_layer_ranges(p, B);

  memset(&L->info, 0, sizeof(L->info));
  L->info.n = n;
  L->info.m = m;
  L->info.nbuckets = B;
  L->info.nranges = R;

  L->code = (uint8_t*)calloc(B, 1);
  L->Z = (uint32_t*)calloc(m, sizeof(uint32_t));
  L->W = (uint64_t*)calloc((m / 64) * h->r + 1, sizeof(uint64_t));
  uint64_t* C = (uint64_t*)calloc(m, sizeof(uint64_t));
  uint32_t* V = (uint32_t*)calloc(m, sizeof(uint32_t));
  ref_pos* order = (ref_pos*)malloc((n + 1) * sizeof(ref_pos));
  uint64_t* coef = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  uint64_t* bstart = (uint64_t*)calloc(B + 1, sizeof(uint64_t));
  uint8_t* bump = (uint8_t*)calloc(n + 1, 1);
  uint64_t* placed = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  if (!L->code || !L->Z || !L->W || !C || !V || !order || !coef || !bstart || !bump ||
      !placed) {
    free(C); free(V); free(order); free(coef); free(bstart); free(bump); free(placed);
    return REF_E_NOMEM;
  }

  /* 1. hash */
  for (uint64_t i = 0; i < n; i++) {
    uint64_t s, c;
    ref_hash(keys[i], li, m, p->seed, &s, &c);
    order[i].s = s;
    order[i].idx = i;
    coef[i] = c;
  }
  /* 2. sort by start slot; bstart[beta] = first sorted position in bucket */
  qsort(order, n, sizeof(ref_pos), ref_pos_cmp);
  for (uint64_t i = 0, beta = 0; beta <= B; beta++) {
    while (i < n && order[i].s / b < beta) i++;
    bstart[beta] = i;
  }

  /* 3. ranges, buckets, chunks */
  for (uint64_t rho = 0; rho < R; rho++)
    ref_solve_range(p, B, R, rho, order, bstart, 0, coef, vals, C, V, m, 0, L->code, bump,
                    placed, &L->info);
  for (uint64_t i = 0; i < m; i++) L->info.pivots += (C[i] != 0);
  /* redundant count above includes equations later undone with their chunk;
   * recount them exactly: kept = n - bumped = pivots + redundant */
  L->info.redundant = n - L->info.bumped - L->info.pivots;

  /* 4. back-substitution and interleaved storage */
  ref_back_substitute(C, V, L->Z, m);
  ref_interleave(L->Z, m, h->r, L->W);

  /* 5. bumped keys, in input order */
  uint64_t nb = L->info.bumped;
  uint64_t* nk = (uint64_t*)malloc((nb + 1) * sizeof(uint64_t));
  uint32_t* nv = (uint32_t*)malloc((nb + 1) * sizeof(uint32_t));
  if (!nk || !nv) {
    free(nk); free(nv);
    free(C); free(V); free(order); free(coef); free(bstart); free(bump); free(placed);
    return REF_E_NOMEM;
  }
  for (uint64_t i = 0, j = 0; i < n; i++)
    if (bump[i]) { nk[j] = keys[i]; nv[j] = vals[i]; j++; }
  *next_keys = nk;
  *next_vals = nv;
  *next_n = nb;

  free(C); free(V); free(order); free(coef); free(bstart); free(bump); free(placed);
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Final layer: plain ribbon, no bumping, scaled up until it solves          */
/* (Sec. 3: no bumping is possible in the last layer; Sec. 4: when its      */
/* system has no solution, the layer is made larger and built again).       */
/* ------------------------------------------------------------------------ */
static int ref_build_final(ref_burr* h, const uint64_t* keys, const uint32_t* vals,
                           uint64_t n) {
  const ref_params* p = &h->p;
  ref_layer* F = &h->fin;
  memset(&h->fin_info, 0, sizeof(h->fin_info));
  h->fin_info.n = n;
  F->info.n = n;
  if (n == 0) {
    h->fin_info.m = 0;
    F->info.m = 0;
    F->W = (uint64_t*)calloc(1, sizeof(uint64_t));
    F->Z = (uint32_t*)calloc(1, sizeof(uint32_t));
    return F->W && F->Z ? REF_OK : REF_E_NOMEM;
  }
  const uint32_t li = p->layers; /* the final layer hashes as layer index L */
  for (uint32_t a = 0; a < p->final_attempts; a++) {
    uint64_t m = ref_final_slots(p, n, a);
    uint64_t* C = (uint64_t*)calloc(m, sizeof(uint64_t));
    uint32_t* V = (uint32_t*)calloc(m, sizeof(uint32_t));
    ref_pos* order = (ref_pos*)malloc(n * sizeof(ref_pos));
    uint64_t* coef = (uint64_t*)malloc(n * sizeof(uint64_t));
    if (!C || !V || !order || !coef) {
      free(C); free(V); free(order); free(coef);
      return REF_E_NOMEM;
    }
    for (uint64_t i = 0; i < n; i++) {
      uint64_t s, c;
      ref_hash(keys[i], li, m, p->seed, &s, &c);
      order[i].s = s;
      order[i].idx = i;
      coef[i] = c;
    }
    qsort(order, n, sizeof(ref_pos), ref_pos_cmp);
    int ok = 1;
    uint64_t steps = 0;
    for (uint64_t t = 0; t < n && ok; t++) {
      uint64_t at;
      int res = ref_insert(C, V, m, order[t].s, coef[order[t].idx], vals[order[t].idx],
                           &at, &steps);
      if (res == INS_CONFLICT) ok = 0;
    }
    h->fin_info.steps += steps;
    if (ok) {
      F->info.m = m;
      h->fin_info.m = m;
      h->fin_info.attempt = a;
      F->Z = (uint32_t*)calloc(m, sizeof(uint32_t));
      F->W = (uint64_t*)calloc((m / 64) * h->r + 1, sizeof(uint64_t));
      if (!F->Z || !F->W) {
        free(C); free(V); free(order); free(coef);
        return REF_E_NOMEM;
      }
      ref_back_substitute(C, V, F->Z, m);
      ref_interleave(F->Z, m, h->r, F->W);
      free(C); free(V); free(order); free(coef);
      return REF_OK;
    }
    free(C); free(V); free(order); free(coef);
  }
  return REF_E_UNSOLVABLE;
}

/* ------------------------------------------------------------------------ */
/* Build / free                                                              */
/* ------------------------------------------------------------------------ */

static int ref_params_valid(const ref_params* p, uint32_t r, const void* values) {
  if (!p) return 0;
  if (r < 1 || r > 32) return 0;
  if (p->bucket == 0 || p->bucket % 64 != 0) return 0;
  if (!(p->t_lo > 0 && p->t_lo < p->t_hi && p->t_hi < p->bucket)) return 0;
  if (p->load_num == 0 || p->load_den == 0) return 0;
  if (p->final_num == 0 || p->final_den == 0) return 0;
  if (p->final_num < p->final_den) return 0;
  if (p->layers > 32) return 0;
  if (p->ranges == 0 || p->final_attempts == 0) return 0;
  if (!p->filter_mode && values == NULL) return 0;
  return 1;
}

static void ref_free_layer(ref_layer* L) {
  free(L->keys); free(L->vals); free(L->code); free(L->Z); free(L->W);
  memset(L, 0, sizeof(*L));
}

void ref_free(ref_burr* h) {
  if (!h) return;
  for (uint32_t i = 0; i < 64; i++) ref_free_layer(&h->layer[i]);
  ref_free_layer(&h->fin);
  free(h);
}

int ref_build(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
              const ref_params* p, ref_burr** out) {
  *out = NULL;
  if (!ref_params_valid(p, r, values)) return REF_E_INVALID;
  if (n > 0 && keys == NULL) return REF_E_INVALID;
  ref_burr* h = (ref_burr*)calloc(1, sizeof(ref_burr));
  if (!h) return REF_E_NOMEM;
  h->p = *p;
  h->r = r;
  h->n = n;

  /* O1: values masked to r bits, or fingerprints in filter mode */
  uint64_t* cur_k = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  uint32_t* cur_v = (uint32_t*)malloc((n + 1) * sizeof(uint32_t));
  if (!cur_k || !cur_v) { free(cur_k); free(cur_v); ref_free(h); return REF_E_NOMEM; }
  for (uint64_t i = 0; i < n; i++) {
    cur_k[i] = keys[i];
    cur_v[i] = p->filter_mode ? ref_fingerprint(keys[i], r, p->seed)
                              : (ref_value_at(values, r, i) & ref_mask(r));
  }
  uint64_t cur_n = n;

  uint32_t li = 0;
  while (li < p->layers && cur_n > 0) {
    ref_layer* L = &h->layer[li];
    L->keys = cur_k;
    L->vals = cur_v;
    uint64_t* nk = NULL;
    uint32_t* nv = NULL;
    uint64_t nn = 0;
    int rc = ref_build_layer(h, li, cur_k, cur_v, cur_n, &nk, &nv, &nn);
    if (rc != REF_OK) { h->built = li + 1; ref_free(h); return rc; }
    cur_k = nk;
    cur_v = nv;
    cur_n = nn;
    li++;
  }
  h->built = li;
  h->fin.keys = cur_k;
  h->fin.vals = cur_v;
  int rc = ref_build_final(h, cur_k, cur_v, cur_n);
  if (rc != REF_OK) { ref_free(h); return rc; }
  *out = h;
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* One range of a layer on its own (Sec. 3: once the keys whose rows could   */
/* cross a range end are bumped, the ranges solve independently). Used for  */
/* sampled checks of structures too large for a whole oracle build.          */
/* ------------------------------------------------------------------------ */

void ref_layer_geometry(const ref_params* p, uint64_t nkeys, uint64_t* m, uint64_t* nbuckets,
                        uint64_t* nranges) {
  *m = ref_layer_slots(p, nkeys);
  *nbuckets = *m / p->bucket;
  *nranges = ref_layer_ranges(p, *nbuckets);
}

void ref_range_buckets(uint64_t nbuckets, uint64_t nranges, uint64_t rho, uint64_t* first,
                       uint64_t* last) {
  *first = ref_range_first_bucket(rho, nbuckets, nranges);
  *last = ref_range_first_bucket(rho + 1, nbuckets, nranges);
}

void ref_start_buckets(const uint64_t* keys, uint64_t n, uint32_t layer, uint64_t m,
                       uint64_t seed, uint32_t bucket, uint32_t* out) {
  for (uint64_t i = 0; i < n; i++) {
    uint64_t s, c;
    ref_hash(keys[i], layer, m, seed, &s, &c);
    out[i] = (uint32_t)(s / bucket);
  }
}

int ref_layer_range(const ref_params* p, uint32_t r, uint32_t layer, uint64_t n_layer,
                    uint64_t rho, const uint64_t* keys, const void* values, uint64_t n,
                    uint8_t* codes, uint64_t* W, uint64_t* bumped, uint64_t* nbumped) {
  if (!ref_params_valid(p, r, values) || layer >= p->layers || n > n_layer) return REF_E_INVALID;
  if (n > 0 && keys == NULL) return REF_E_INVALID;
  const uint64_t b = p->bucket;
  uint64_t m, B, R, first, last;
  ref_layer_geometry(p, n_layer, &m, &B, &R);
  if (rho >= R) return REF_E_INVALID;
  ref_range_buckets(B, R, rho, &first, &last);
  /* rows of kept keys stay inside the range: forced bumps keep them off its
   * end, and in the last range s <= m - w */
  const uint64_t base = first * b, mwin = (last - first) * b;
  uint64_t* C = (uint64_t*)calloc(mwin, sizeof(uint64_t));
  uint32_t* V = (uint32_t*)calloc(mwin, sizeof(uint32_t));
  uint32_t* Z = (uint32_t*)calloc(mwin, sizeof(uint32_t));
  ref_pos* order = (ref_pos*)malloc((n + 1) * sizeof(ref_pos));
  uint64_t* coef = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  uint32_t* vals = (uint32_t*)malloc((n + 1) * sizeof(uint32_t));
  uint64_t* bstart = (uint64_t*)calloc(last - first + 1, sizeof(uint64_t));
  uint8_t* bump = (uint8_t*)calloc(n + 1, 1);
  uint64_t* placed = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  int rc = REF_OK;
  if (!C || !V || !Z || !order || !coef || !vals || !bstart || !bump || !placed) {
    rc = REF_E_NOMEM;
    goto done;
  }
  for (uint64_t i = 0; i < n; i++) {
    uint64_t s, c;
    ref_hash(keys[i], layer, m, p->seed, &s, &c);
    if (s < base || s >= base + mwin) {
      rc = REF_E_INVALID; /* the key belongs to another range */
      goto done;
    }
    order[i].s = s;
    order[i].idx = i;
    coef[i] = c;
    vals[i] = p->filter_mode ? ref_fingerprint(keys[i], r, p->seed)
                             : (ref_value_at(values, r, i) & ref_mask(r));
  }
  qsort(order, n, sizeof(ref_pos), ref_pos_cmp);
  for (uint64_t i = 0, beta = first; beta <= last; beta++) {
    while (i < n && order[i].s / b < beta) i++;
    bstart[beta - first] = i;
  }
  ref_layer_info info;
  memset(&info, 0, sizeof(info));
  ref_solve_range(p, B, R, rho, order, bstart, first, coef, vals, C, V, mwin, base, codes, bump,
                  placed, &info);
  ref_back_substitute(C, V, Z, mwin);
  ref_interleave(Z, mwin, r, W);
  *nbumped = 0;
  for (uint64_t i = 0; i < n; i++)
    if (bump[i]) bumped[(*nbumped)++] = keys[i];
done:
  free(C); free(V); free(Z); free(order); free(coef); free(vals); free(bstart); free(bump);
  free(placed);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Query (Sec. 2, Fig. 1a: multiply the key's hash row with the table)       */
/* ------------------------------------------------------------------------ */

/* bit col of Z[slot], read back from the interleaved words */
static uint32_t ref_table_bit(const uint64_t* W, uint32_t r, uint64_t slot, uint32_t col) {
  return (uint32_t)((W[(slot / 64) * r + col] >> (slot % 64)) & 1ull);
}

static uint32_t ref_query_one(const ref_burr* h, uint64_t key) {
  const ref_params* p = &h->p;
  const uint64_t theta[4] = {0, p->t_lo, p->t_hi, p->bucket};
  for (uint32_t li = 0; li <= h->built; li++) {
    const ref_layer* L = li < h->built ? &h->layer[li] : &h->fin;
    uint64_t m = L->info.m;
    if (m == 0) return 0; /* empty final layer */
    uint64_t s, c;
    ref_hash(key, li < h->built ? li : p->layers, m, p->seed, &s, &c);
    if (li < h->built) {
      uint64_t beta = s / p->bucket;
      uint64_t o = s % p->bucket;
      if (o < theta[L->code[beta]]) continue; /* bumped: look one layer down */
    }
    uint32_t out = 0;
    for (uint32_t col = 0; col < h->r; col++) {
      uint32_t par = 0;
      for (unsigned j = 0; j < 64; j++)
        if ((c >> j) & 1ull) par ^= ref_table_bit(L->W, h->r, s + j, col);
      out |= par << col;
    }
    return out;
  }
  return 0;
}

int ref_query(const ref_burr* h, const uint64_t* keys, uint64_t n, void* out) {
  if (!h || (n > 0 && (!keys || !out))) return REF_E_INVALID;
  for (uint64_t i = 0; i < n; i++) ref_store_value(out, h->r, i, ref_query_one(h, keys[i]));
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Export: canonical little-endian bytes                                     */
/*   header: u64 magic "BuRRexp1", u32 x 16 (version, w, b, r, load_num,     */
/*   load_den, final_num, final_den, layers, t_lo, t_hi, ranges, minbpt,     */
/*   final_attempts, filter_mode, layers_built), u64 seed, u64 n             */
/*   per BuRR layer: u64 n, m, ranges; u64 code words ceil(B/32) (bucket     */
/*   beta at bits 2*(beta%32)); u64 solution words m/64*r                    */
/*   final: u64 n, m, attempt; u64 solution words m/64*r                     */
/* ------------------------------------------------------------------------ */

typedef struct { uint8_t* buf; uint64_t cap; uint64_t len; } ref_out;

static void ref_put(ref_out* o, uint64_t v, unsigned bytes) {
  for (unsigned i = 0; i < bytes; i++) {
    if (o->len < o->cap) o->buf[o->len] = (uint8_t)(v >> (8 * i));
    o->len++;
  }
}

int ref_export(const ref_burr* h, uint8_t* buf, uint64_t cap, uint64_t* needed) {
  if (!h) return REF_E_INVALID;
  ref_out o = {buf, buf ? cap : 0, 0};
  const ref_params* p = &h->p;
  ref_put(&o, 0x3170786552527542ull, 8); /* "BuRRexp1" */
  const uint32_t hdr[16] = {1u, REF_W, p->bucket, h->r, p->load_num, p->load_den,
                            p->final_num, p->final_den, p->layers, p->t_lo, p->t_hi,
                            p->ranges, p->minbpt, p->final_attempts, p->filter_mode,
                            h->built};
  for (int i = 0; i < 16; i++) ref_put(&o, hdr[i], 4);
  ref_put(&o, p->seed, 8);
  ref_put(&o, h->n, 8);
  for (uint32_t li = 0; li < h->built; li++) {
    const ref_layer* L = &h->layer[li];
    ref_put(&o, L->info.n, 8);
    ref_put(&o, L->info.m, 8);
    ref_put(&o, L->info.nranges, 8);
    uint64_t B = L->info.nbuckets;
    for (uint64_t wd = 0; wd < (B + 31) / 32; wd++) {
      uint64_t word = 0;
      for (uint64_t beta = wd * 32; beta < B && beta < wd * 32 + 32; beta++)
        word |= (uint64_t)L->code[beta] << (2 * (beta % 32));
      ref_put(&o, word, 8);
    }
    for (uint64_t wd = 0; wd < (L->info.m / 64) * h->r; wd++) ref_put(&o, L->W[wd], 8);
  }
  ref_put(&o, h->fin_info.n, 8);
  ref_put(&o, h->fin_info.m, 8);
  ref_put(&o, h->fin_info.attempt, 8);
  for (uint64_t wd = 0; wd < (h->fin_info.m / 64) * h->r; wd++) ref_put(&o, h->fin.W[wd], 8);
  if (needed) *needed = o.len;
  return (buf && o.len > cap) ? REF_E_INVALID : REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Introspection for tests                                                   */
/* ------------------------------------------------------------------------ */

uint32_t ref_layers_built(const ref_burr* h) { return h ? h->built : 0; }

int ref_get_layer_info(const ref_burr* h, uint32_t layer, ref_layer_info* out) {
  if (!h || layer >= h->built || !out) return REF_E_INVALID;
  *out = h->layer[layer].info;
  return REF_OK;
}

int ref_get_final_info(const ref_burr* h, ref_final_info* out) {
  if (!h || !out) return REF_E_INVALID;
  *out = h->fin_info;
  return REF_OK;
}

uint64_t ref_layer_keys(const ref_burr* h, uint32_t layer, uint64_t* out, uint64_t cap) {
  if (!h || layer > h->built) return 0;
  const ref_layer* L = layer < h->built ? &h->layer[layer] : &h->fin;
  uint64_t n = L->info.n;
  if (out)
    for (uint64_t i = 0; i < n && i < cap; i++) out[i] = L->keys[i];
  return n;
}

uint64_t ref_layer_codes(const ref_burr* h, uint32_t layer, uint8_t* out, uint64_t cap) {
  if (!h || layer >= h->built) return 0;
  const ref_layer* L = &h->layer[layer];
  uint64_t B = L->info.nbuckets;
  if (out)
    for (uint64_t i = 0; i < B && i < cap; i++) out[i] = L->code[i];
  return B;
}

uint64_t ref_layer_solution(const ref_burr* h, uint32_t layer, uint32_t* out, uint64_t cap) {
  if (!h || layer > h->built) return 0;
  const ref_layer* L = layer < h->built ? &h->layer[layer] : &h->fin;
  uint64_t m = L->info.m;
  if (out)
    for (uint64_t i = 0; i < m && i < cap; i++) out[i] = L->Z[i];
  return m;
}
