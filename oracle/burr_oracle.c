/*
 * burr_oracle.c - plain sequential CPU oracle for Bumped Ribbon Retrieval
 * (BuRR) with boundary bumping (arXiv 2411.12365).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline leg of the benchmark. It is deliberately simple and slow: one
 * thread, qsort, bit-by-bit back-substitution and bit-by-bit queries. It shares
 * no code with the HIP library. A range-parallel driver (ref_build_mt, the
 * paper's own scheme of one partition per thread) runs the same per-range
 * steps on many threads for large inputs and timing; its output is checked
 * against the sequential builder byte for byte.
 *
 * What it computes, step by step (the paper names the steps; the details are
 * readings, stated at each function):
 *   1. hash every key of a layer to a start slot s, a 64-bit coefficient row c
 *      and an r-bit value v                                 (Sec. 2, ribbon)
 *   2. order the keys by start slot                (Sec. 4, sorting step)
 *   3. cut the slot array into ranges (equal split, or cut points chosen by
 *      the minbump / maxprev / diff search), bump keys whose row would cross
 *      a range end, and insert the remaining keys bucket by bucket with 2-bit
 *      or 1+-bit bump thresholds     (Sec. 2 bumping, Sec. 3 "Bumping",
 *                                     "Selecting Cut Points")
 *   4. back-substitute the solution and store it column-interleaved
 *   5. recurse on bumped keys; the last layer is a plain ribbon that is
 *      scaled up until it solves                 (Sec. 3 last layer, Sec. 4)
 *   6. query: walk the layers, check the bucket threshold, AND the window of
 *      the table with c and take the parity per column   (Sec. 2, Fig. 1a)
 *
 * Hash: parity unpinned against the paper (the paper does not define one).
 */
#include "burr_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

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
  uint8_t* code;       /* per bucket: 2-bit code index, or the 1+-bit threshold */
  uint32_t* Z;         /* solution, one r-bit word per slot */
  uint64_t* W;         /* column-interleaved solution words, m/64 * r */
  uint64_t* cut_last;  /* last bucket of every range (nranges entries) */
} ref_layer;

struct ref_burr {
  ref_params p;
  uint32_t r;
  uint64_t n;
  uint32_t first;          /* index of the first layer built (0 for ref_build) */
  uint32_t built;          /* BuRR layers built, counted from layer 0 */
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
/* Thresholds (Sec. 2: 2-bit and 1+-bit)                                     */
/* ------------------------------------------------------------------------ */

/* The stored threshold value of a bucket: with 2-bit thresholds the code
 * indexes the four values {0, t_lo, t_hi, b}; with 1+-bit thresholds the
 * byte is the threshold itself (0: the bucket's bit is clear, nothing
 * bumped; else the exact value kept for the bumped bucket). Keys with
 * offset below it are bumped. */
static uint64_t ref_theta(const ref_params* p, uint8_t code) {
  if (p->threshold_mode == 1) return code;
  const uint64_t theta[4] = {0, p->t_lo, p->t_hi, p->bucket};
  return theta[code & 3u];
}

/* Threshold forced on the last bucket beta of a range that is not the
 * layer's last one (Sec. 3 "Bumping"): a key whose row could cross the range
 * end (s > end - w) must be bumped, so the threshold is the smallest
 * allowed value above the largest offset of such a key; 0 if there is none.
 * Keys lie in order[lo, hi). With 2-bit thresholds the result is a code
 * index, with 1+-bit thresholds a threshold value. */
static unsigned ref_forced(const ref_params* p, uint64_t beta, uint64_t range_end,
                           const ref_pos* order, uint64_t lo, uint64_t hi) {
  const uint64_t b = p->bucket;
  int any = 0;
  uint64_t omax = 0;
  for (uint64_t t = lo; t < hi; t++) {
    uint64_t s = order[t].s;
    if (s + REF_W > range_end) { /* s > range_end - w */
      any = 1;
      if (s - beta * b > omax) omax = s - beta * b;
    }
  }
  if (!any) return 0;
  if (p->threshold_mode == 1) return (unsigned)(omax + 1);
  for (unsigned k = 0; k < 4; k++)
    if (ref_theta(p, (uint8_t)k) > omax) return k;
  return 3; /* unreachable: theta[3] = b > omax */
}

/* ------------------------------------------------------------------------ */
/* Cut points (Sec. 3 "Selecting Cut Points")                                */
/* ------------------------------------------------------------------------ */

/*
 * Last bucket of every range of a layer with B buckets and R ranges, keys
 * sorted in order[] with bucket starts bstart[]. Without a search
 * (cut_strategy 0, or cut_search < 2) the ranges are the equal integer split,
 * range rho = buckets [floor(rho B / R), floor((rho+1) B / R)).
 *
 * With a search, the last bucket of range rho < R-1 is chosen among the
 * buckets within h of the equal split's, h = min(cut_search / 2,
 * (floor(B/R) - 2) / 2), so that every range keeps at least two buckets and
 * each cut can be chosen on its own. For a candidate bucket beta (it would be
 * the range's last bucket, whose forced threshold bumps keys):
 *   bumped(beta) = keys of beta below the threshold forced on it,
 *   prev(beta)   = keys whose start lies in the w-1 slots before beta,
 * and the strategies pick the candidate with
 *   1 minbump: the fewest bumped(beta),
 *   2 maxprev: the most prev(beta) (keys that can fill the gap),
 *   3 diff:    the smallest bumped(beta) - prev(beta);
 * ties go to the candidate nearest to the equal split, then the lower one.
 */
static void ref_choose_cuts(const ref_params* p, uint64_t B, uint64_t R, const ref_pos* order,
                            const uint64_t* bstart, uint64_t* cut_last) {
  const uint64_t b = p->bucket;
  for (uint64_t rho = 0; rho < R; rho++)
    cut_last[rho] = ref_range_first_bucket(rho + 1, B, R) - 1;
  if (p->cut_strategy == 0 || p->cut_search < 2 || R < 2) return;
  const uint64_t L = B / R;
  uint64_t h = p->cut_search / 2;
  const uint64_t hmax = L >= 2 ? (L - 2) / 2 : 0;
  if (h > hmax) h = hmax;
  if (h == 0) return;
  for (uint64_t rho = 0; rho + 1 < R; rho++) {
    const uint64_t b0 = cut_last[rho];
    int have = 0;
    int64_t best = 0;
    uint64_t best_beta = b0, best_dist = 0;
    for (uint64_t beta = b0 - h; beta <= b0 + h; beta++) {
      const uint64_t lo = bstart[beta], hi = bstart[beta + 1];
      const uint64_t end = (beta + 1) * b;
      const uint64_t T = ref_theta(p, (uint8_t)ref_forced(p, beta, end, order, lo, hi));
      int64_t bumped = 0, prev = 0;
      for (uint64_t t = lo; t < hi; t++)
        if (order[t].s - beta * b < T) bumped++;
      /* keys starting in slots [beta*b - (w-1), beta*b) */
      for (uint64_t t = bstart[beta]; t-- > 0;) {
        if (order[t].s + (REF_W - 1) < beta * b) break;
        prev++;
      }
      int64_t score = p->cut_strategy == 1 ? bumped
                    : p->cut_strategy == 2 ? -prev
                                           : bumped - prev;
      const uint64_t dist = beta > b0 ? beta - b0 : b0 - beta;
      if (!have || score < best || (score == best && dist < best_dist)) {
        have = 1;
        best = score;
        best_beta = beta;
        best_dist = dist;
      }
    }
    cut_last[rho] = best_beta;
  }
}

/* ------------------------------------------------------------------------ */
/* One range of a BuRR layer (Sec. 2 bumping, Sec. 3 "Bumping")             */
/* ------------------------------------------------------------------------ */

/*
 * Range of buckets [first, last] (last_range: the layer's last range, which
 * bumps nothing for the range end). The rows live in C/V, which cover the
 * slot window [base, base + mwin): slot s is C[s - base]. order lists the
 * keys of these buckets sorted by start slot; bstart[beta - bbase] is the
 * first position of bucket beta in order and codes[beta - bbase] receives its
 * threshold (ref_theta). bump[idx] is set for every bumped key (idx = the
 * key's order[].idx); placed is scratch of one entry per key of a bucket.
 *
 * 2-bit thresholds: a bucket is inserted in chunks of decreasing offset,
 * [t_hi, b), [t_lo, t_hi), [0, t_lo); the first chunk whose insertion meets
 * an inconsistent equation is undone and the threshold becomes that chunk's
 * upper end.
 * 1+-bit thresholds: the keys are inserted one by one in decreasing offset
 * order; at the first inconsistent key, with offset o, the keys of offset o
 * inserted before it are undone and the threshold is o + 1 (keys with equal
 * offsets share their fate, since a threshold is an offset).
 * Either way the threshold is the smallest allowed value (at least the
 * forced one) for which the kept equations stay consistent.
 */
static void ref_solve_range(const ref_params* p, uint64_t first, uint64_t last, int last_range,
                            const ref_pos* order, const uint64_t* bstart, uint64_t bbase,
                            const uint64_t* coef, const uint32_t* vals, uint64_t* C,
                            uint32_t* V, uint64_t mwin, uint64_t base, uint8_t* codes,
                            uint8_t* bump, uint64_t* placed, ref_layer_info* info) {
  const uint64_t b = p->bucket;
  const uint64_t range_end = (last + 1) * b; /* slot */
  for (uint64_t beta = first; beta <= last; beta++) {
    uint64_t lo = bstart[beta - bbase], hi = bstart[beta - bbase + 1];
    const int at_end = !last_range && beta == last;
    const unsigned kf = at_end ? ref_forced(p, beta, range_end, order, lo, hi) : 0;
    unsigned code = kf;
    if (p->threshold_mode == 1) {
      /* keys with offset >= kf, highest offset first (order is ascending) */
      uint64_t nplaced = 0, group = b; /* offset of the current group */
      for (uint64_t t = hi; t-- > lo;) {
        uint64_t s = order[t].s;
        uint64_t o = s - beta * b;
        if (o < kf) break;
        if (o != group) {
          group = o;
          nplaced = 0; /* earlier groups are final */
        }
        uint64_t id = order[t].idx;
        uint64_t at = 0;
        int res = ref_insert(C, V, mwin, s - base, coef[id], vals[id], &at, &info->steps);
        if (res == INS_PLACED) {
          placed[nplaced++] = at;
        } else if (res == INS_REDUNDANT) {
          info->redundant++;
        } else {
          for (uint64_t u = 0; u < nplaced; u++) {
            C[placed[u]] = 0;
            V[placed[u]] = 0;
          }
          code = (unsigned)(o + 1);
          break;
        }
      }
    } else {
      const uint64_t theta[4] = {0, p->t_lo, p->t_hi, b};
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
    }
    codes[beta - bbase] = (uint8_t)code;
    const uint64_t T = ref_theta(p, (uint8_t)code);
    for (uint64_t t = lo; t < hi; t++) {
      uint64_t o = order[t].s - beta * b;
      if (o < T) {
        bump[order[t].idx] = 1;
        info->bumped++;
        if (at_end && order[t].s + REF_W > range_end) info->forced++;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* One BuRR layer                                                            */
/* ------------------------------------------------------------------------ */

/* Largest number of keys in one bucket (scratch size of ref_solve_range). */
static uint64_t ref_max_bucket(const uint64_t* bstart, uint64_t B) {
  uint64_t mx = 0;
  for (uint64_t beta = 0; beta < B; beta++)
    if (bstart[beta + 1] - bstart[beta] > mx) mx = bstart[beta + 1] - bstart[beta];
  return mx;
}

/*
 * Builds layer `li` from keys/vals (n of them). Returns the bumped keys in
 * *next_keys / *next_vals (malloc'd) and their count in *next_n.
 *
 * Steps: hash every key (start slot, row), sort by start slot, cut the
 * buckets into ranges (ref_choose_cuts), solve every range on its own
 * (ref_solve_range: forced bumps at the range end make the ranges
 * independent, Sec. 3; the loop below still runs them one after another),
 * back-substitute the whole layer and store it column-interleaved, and pass
 * the bumped keys, in input order, to the next layer.
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
  L->cut_last = (uint64_t*)calloc(R, sizeof(uint64_t));
  uint64_t* C = (uint64_t*)calloc(m, sizeof(uint64_t));
  uint32_t* V = (uint32_t*)calloc(m, sizeof(uint32_t));
  ref_pos* order = (ref_pos*)malloc((n + 1) * sizeof(ref_pos));
  uint64_t* coef = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  uint64_t* bstart = (uint64_t*)calloc(B + 1, sizeof(uint64_t));
  uint8_t* bump = (uint8_t*)calloc(n + 1, 1);
  uint64_t* placed = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  if (!L->code || !L->Z || !L->W || !L->cut_last || !C || !V || !order || !coef || !bstart ||
      !bump || !placed) {
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

  /* 3. ranges, buckets, thresholds */
  ref_choose_cuts(p, B, R, order, bstart, L->cut_last);
  for (uint64_t rho = 0, first = 0; rho < R; rho++) {
    ref_solve_range(p, first, L->cut_last[rho], rho + 1 == R, order, bstart, 0, coef, vals, C,
                    V, m, 0, L->code, bump, placed, &L->info);
    first = L->cut_last[rho] + 1;
  }
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
  if (p->threshold_mode > 1 || (p->threshold_mode == 1 && p->bucket > 192)) return 0;
  if (p->cut_strategy > 3) return 0;
  return 1;
}

static void ref_free_layer(ref_layer* L) {
  free(L->keys); free(L->vals); free(L->code); free(L->Z); free(L->W); free(L->cut_last);
  memset(L, 0, sizeof(*L));
}

void ref_free(ref_burr* h) {
  if (!h) return;
  for (uint32_t i = 0; i < 64; i++) ref_free_layer(&h->layer[i]);
  ref_free_layer(&h->fin);
  free(h);
}

static int ref_build_layer_mt(ref_burr* h, uint32_t li, const uint64_t* keys,
                              const uint32_t* vals, uint64_t n, uint32_t threads,
                              uint64_t** next_keys, uint32_t** next_vals, uint64_t* next_n);

/* Layers first..layers-1, then the final layer, from keys that enter layer
 * `first`. threads <= 1: the plain sequential layer builder; more: the
 * range-parallel one (same result). */
static int ref_build_impl(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
                          const ref_params* p, uint32_t first, uint32_t threads,
                          ref_burr** out) {
  *out = NULL;
  if (!ref_params_valid(p, r, values) || first > p->layers) return REF_E_INVALID;
  if (n > 0 && keys == NULL) return REF_E_INVALID;
  ref_burr* h = (ref_burr*)calloc(1, sizeof(ref_burr));
  if (!h) return REF_E_NOMEM;
  h->p = *p;
  h->r = r;
  h->n = n;
  h->first = first;

  /* values masked to r bits, or fingerprints in filter mode */
  uint64_t* cur_k = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  uint32_t* cur_v = (uint32_t*)malloc((n + 1) * sizeof(uint32_t));
  if (!cur_k || !cur_v) { free(cur_k); free(cur_v); ref_free(h); return REF_E_NOMEM; }
  for (uint64_t i = 0; i < n; i++) {
    cur_k[i] = keys[i];
    cur_v[i] = p->filter_mode ? ref_fingerprint(keys[i], r, p->seed)
                              : (ref_value_at(values, r, i) & ref_mask(r));
  }
  uint64_t cur_n = n;

  uint32_t li = first;
  while (li < p->layers && cur_n > 0) {
    ref_layer* L = &h->layer[li];
    L->keys = cur_k;
    L->vals = cur_v;
    uint64_t* nk = NULL;
    uint32_t* nv = NULL;
    uint64_t nn = 0;
    int rc = threads > 1
                 ? ref_build_layer_mt(h, li, cur_k, cur_v, cur_n, threads, &nk, &nv, &nn)
                 : ref_build_layer(h, li, cur_k, cur_v, cur_n, &nk, &nv, &nn);
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

int ref_build(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
              const ref_params* p, ref_burr** out) {
  return ref_build_impl(keys, values, n, r, p, 0, 1, out);
}

int ref_build_from(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
                   const ref_params* p, uint32_t first_layer, uint32_t threads,
                   ref_burr** out) {
  return ref_build_impl(keys, values, n, r, p, first_layer, threads, out);
}

/* ------------------------------------------------------------------------ */
/* Range-parallel layer builder (Sec. 3: one partition of the equation      */
/* system per thread). The same steps as ref_build_layer, split over         */
/* threads: hashing by key index, the sort by bucket-aligned parts of the    */
/* slot array (each part sorted on its own; concatenated they give qsort's   */
/* order), the ranges by range index, and back-substitution and storage per  */
/* range (kept rows never cross a range end). Its output equals the         */
/* sequential builder's byte for byte (tests/test_oracle_parallel.py).       */
/* ------------------------------------------------------------------------ */

typedef struct {
  const ref_params* p;
  uint32_t li, r, T;
  const uint64_t* keys;
  const uint32_t* vals;
  uint64_t n, m, B, R;
  ref_pos* order;     /* hashed, then sorted */
  ref_pos* tmp;
  uint64_t* coef;
  uint64_t* cnt;      /* T x T: keys of thread t's input chunk in part q */
  uint64_t* bstart;
  uint64_t* cut_last;
  uint8_t* code;
  uint8_t* bump;
  uint64_t* C;
  uint32_t* V;
  uint32_t* Z;
  uint64_t* W;
  uint64_t max_bucket;
  ref_layer_info* info; /* per thread */
  int* err;             /* per thread */
} ref_mt;

typedef struct { ref_mt* M; uint32_t t; int phase; } ref_mt_arg;

static uint64_t ref_mt_part(const ref_mt* M, uint64_t s) {
  return (uint64_t)(((unsigned __int128)(s / M->p->bucket) * M->T) / M->B);
}

static void* ref_mt_run(void* arg) {
  ref_mt_arg* a = (ref_mt_arg*)arg;
  ref_mt* M = a->M;
  const uint32_t t = a->t, T = M->T;
  const uint64_t lo = M->n * t / T, hi = M->n * (t + 1) / T;
  if (a->phase == 0) { /* hash a chunk of keys, count per part */
    for (uint64_t i = lo; i < hi; i++) {
      uint64_t s, c;
      ref_hash(M->keys[i], M->li, M->m, M->p->seed, &s, &c);
      M->order[i].s = s;
      M->order[i].idx = i;
      M->coef[i] = c;
      M->cnt[(uint64_t)t * T + ref_mt_part(M, s)]++;
    }
  } else if (a->phase == 1) { /* scatter the chunk to its parts */
    uint64_t* pos = (uint64_t*)malloc(T * sizeof(uint64_t));
    if (!pos) { M->err[t] = 1; return NULL; }
    for (uint32_t q = 0; q < T; q++) pos[q] = M->cnt[(uint64_t)t * T + q];
    for (uint64_t i = lo; i < hi; i++) M->tmp[pos[ref_mt_part(M, M->order[i].s)]++] = M->order[i];
    free(pos);
  } else if (a->phase == 2) { /* sort part t */
    const uint64_t plo = M->cnt[t], phi = t + 1 < T ? M->cnt[t + 1] : M->n;
    qsort(M->tmp + plo, phi - plo, sizeof(ref_pos), ref_pos_cmp);
  } else { /* ranges [t R / T, (t+1) R / T): solve, back-substitute, store */
    const uint64_t b = M->p->bucket;
    const uint64_t r0 = M->R * t / T, r1 = M->R * (t + 1) / T;
    uint64_t* placed = (uint64_t*)malloc((M->max_bucket + 1) * sizeof(uint64_t));
    if (!placed) { M->err[t] = 1; return NULL; }
    for (uint64_t rho = r0; rho < r1; rho++) {
      const uint64_t first = rho ? M->cut_last[rho - 1] + 1 : 0, last = M->cut_last[rho];
      ref_solve_range(M->p, first, last, rho + 1 == M->R, M->order, M->bstart, 0, M->coef,
                      M->vals, M->C, M->V, M->m, 0, M->code, M->bump, placed, &M->info[t]);
      const uint64_t base = first * b, len = (last - first + 1) * b;
      ref_back_substitute(M->C + base, M->V + base, M->Z + base, len);
      ref_interleave(M->Z + base, len, M->r, M->W + (base / 64) * M->r);
    }
    free(placed);
  }
  return NULL;
}

static int ref_mt_phase(ref_mt* M, int phase) {
  pthread_t th[256];
  ref_mt_arg args[256];
  for (uint32_t t = 0; t < M->T; t++) {
    args[t].M = M;
    args[t].t = t;
    args[t].phase = phase;
    if (pthread_create(&th[t], NULL, ref_mt_run, &args[t]) != 0) return REF_E_NOMEM;
  }
  for (uint32_t t = 0; t < M->T; t++) pthread_join(th[t], NULL);
  for (uint32_t t = 0; t < M->T; t++)
    if (M->err[t]) return REF_E_NOMEM;
  return REF_OK;
}

static int ref_build_layer_mt(ref_burr* h, uint32_t li, const uint64_t* keys,
                              const uint32_t* vals, uint64_t n, uint32_t threads,
                              uint64_t** next_keys, uint32_t** next_vals, uint64_t* next_n) {
  const ref_params* p = &h->p;
  ref_layer* L = &h->layer[li];
  ref_mt M;
  memset(&M, 0, sizeof(M));
  M.p = p;
  M.li = li;
  M.r = h->r;
  M.T = threads > 256 ? 256 : threads;
  M.keys = keys;
  M.vals = vals;
  M.n = n;
  M.m = ref_layer_slots(p, n);
  M.B = M.m / p->bucket;
  M.R = ref_layer_ranges(p, M.B);
  if (M.T > M.B) M.T = (uint32_t)M.B;
  const uint32_t T = M.T;

  memset(&L->info, 0, sizeof(L->info));
  L->info.n = n;
  L->info.m = M.m;
  L->info.nbuckets = M.B;
  L->info.nranges = M.R;
  L->code = (uint8_t*)calloc(M.B, 1);
  L->Z = (uint32_t*)calloc(M.m, sizeof(uint32_t));
  L->W = (uint64_t*)calloc((M.m / 64) * h->r + 1, sizeof(uint64_t));
  L->cut_last = (uint64_t*)calloc(M.R, sizeof(uint64_t));
  M.code = L->code;
  M.Z = L->Z;
  M.W = L->W;
  M.cut_last = L->cut_last;
  M.C = (uint64_t*)calloc(M.m, sizeof(uint64_t));
  M.V = (uint32_t*)calloc(M.m, sizeof(uint32_t));
  M.order = (ref_pos*)malloc((n + 1) * sizeof(ref_pos));
  M.tmp = (ref_pos*)malloc((n + 1) * sizeof(ref_pos));
  M.coef = (uint64_t*)malloc((n + 1) * sizeof(uint64_t));
  M.cnt = (uint64_t*)calloc((uint64_t)T * T, sizeof(uint64_t));
  M.bstart = (uint64_t*)calloc(M.B + 1, sizeof(uint64_t));
  M.bump = (uint8_t*)calloc(n + 1, 1);
  M.info = (ref_layer_info*)calloc(T, sizeof(ref_layer_info));
  M.err = (int*)calloc(T, sizeof(int));
  int rc = REF_OK;
  if (!L->code || !L->Z || !L->W || !L->cut_last || !M.C || !M.V || !M.order || !M.tmp ||
      !M.coef || !M.cnt || !M.bstart || !M.bump || !M.info || !M.err) {
    rc = REF_E_NOMEM;
    goto done;
  }
  /* 1. hash; 2. sort by bucket-aligned parts */
  if ((rc = ref_mt_phase(&M, 0)) != REF_OK) goto done;
  {
    uint64_t run = 0; /* cnt[t][q] -> first position of chunk t's keys in part q */
    uint64_t* part_first = (uint64_t*)malloc(T * sizeof(uint64_t));
    if (!part_first) { rc = REF_E_NOMEM; goto done; }
    for (uint32_t q = 0; q < T; q++) {
      part_first[q] = run;
      for (uint32_t t = 0; t < T; t++) {
        const uint64_t c = M.cnt[(uint64_t)t * T + q];
        M.cnt[(uint64_t)t * T + q] = run;
        run += c;
      }
    }
    if ((rc = ref_mt_phase(&M, 1)) != REF_OK) { free(part_first); goto done; }
    for (uint32_t q = 0; q < T; q++) M.cnt[q] = part_first[q]; /* part starts */
    free(part_first);
  }
  if ((rc = ref_mt_phase(&M, 2)) != REF_OK) goto done;
  {
    ref_pos* x = M.order;
    M.order = M.tmp;
    M.tmp = x;
  }
  for (uint64_t i = 0, beta = 0; beta <= M.B; beta++) {
    while (i < n && M.order[i].s / p->bucket < beta) i++;
    M.bstart[beta] = i;
  }
  M.max_bucket = ref_max_bucket(M.bstart, M.B);
  /* 3. ranges (cut points chosen in order), 4. solve and store per range */
  ref_choose_cuts(p, M.B, M.R, M.order, M.bstart, M.cut_last);
  if ((rc = ref_mt_phase(&M, 3)) != REF_OK) goto done;
  for (uint32_t t = 0; t < T; t++) {
    L->info.bumped += M.info[t].bumped;
    L->info.forced += M.info[t].forced;
    L->info.steps += M.info[t].steps;
  }
  for (uint64_t i = 0; i < M.m; i++) L->info.pivots += (M.C[i] != 0);
  L->info.redundant = n - L->info.bumped - L->info.pivots;
  /* 5. bumped keys, in input order */
  {
    uint64_t nb = L->info.bumped;
    uint64_t* nk = (uint64_t*)malloc((nb + 1) * sizeof(uint64_t));
    uint32_t* nv = (uint32_t*)malloc((nb + 1) * sizeof(uint32_t));
    if (!nk || !nv) { free(nk); free(nv); rc = REF_E_NOMEM; goto done; }
    for (uint64_t i = 0, j = 0; i < n; i++)
      if (M.bump[i]) { nk[j] = keys[i]; nv[j] = vals[i]; j++; }
    *next_keys = nk;
    *next_vals = nv;
    *next_n = nb;
  }
done:
  free(M.C); free(M.V); free(M.order); free(M.tmp); free(M.coef); free(M.cnt);
  free(M.bstart); free(M.bump); free(M.info); free(M.err);
  return rc;
}

int ref_build_mt(const uint64_t* keys, const void* values, uint64_t n, uint32_t r,
                 const ref_params* p, uint32_t threads, ref_burr** out) {
  if (threads == 0) {
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    threads = c > 0 ? (uint32_t)c : 1;
  }
  return ref_build_impl(keys, values, n, r, p, 0, threads, out);
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
  if (p->cut_strategy != 0 && p->cut_search >= 2) return REF_E_INVALID; /* cuts need neighbours */
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
  ref_solve_range(p, first, last - 1, rho + 1 == R, order, bstart, first, coef, vals, C, V,
                  mwin, base, codes, bump, placed, &info);
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
  for (uint32_t li = h->first; li <= h->built; li++) {
    const ref_layer* L = li < h->built ? &h->layer[li] : &h->fin;
    uint64_t m = L->info.m;
    if (m == 0) return 0; /* empty final layer */
    uint64_t s, c;
    ref_hash(key, li < h->built ? li : p->layers, m, p->seed, &s, &c);
    if (li < h->built) {
      uint64_t beta = s / p->bucket;
      uint64_t o = s % p->bucket;
      if (o < ref_theta(p, L->code[beta])) continue; /* bumped: look one layer down */
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
/*   header: u64 magic "BuRRexp1", u32 x 20 (version 2, w, b, r, load_num,   */
/*   load_den, final_num, final_den, layers, t_lo, t_hi, ranges, minbpt,     */
/*   final_attempts, filter_mode, layers_built, threshold_mode,              */
/*   cut_strategy, cut_search, first layer), u64 seed, u64 n                 */
/*   per BuRR layer (first .. layers_built-1): u64 n, m, ranges; then        */
/*     2-bit: u64 code words ceil(B/32) (bucket beta at bits 2*(beta%32)),   */
/*     1+-bit: u64 bit words ceil(B/64) (bit beta%64 of word beta/64 set if  */
/*       the bucket bumps), u64 K = set bits, ceil(K/8) u64 words holding    */
/*       the thresholds minus 1 of those buckets as bytes, in bucket order;  */
/*     u64 solution words m/64*r;                                            */
/*     with a cut strategy: ceil((R-1)/2) u64 words holding the last bucket  */
/*       of ranges 0..R-2 as u32                                             */
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
  const uint32_t hdr[20] = {2u, REF_W, p->bucket, h->r, p->load_num, p->load_den,
                            p->final_num, p->final_den, p->layers, p->t_lo, p->t_hi,
                            p->ranges, p->minbpt, p->final_attempts, p->filter_mode,
                            h->built, p->threshold_mode, p->cut_strategy, p->cut_search,
                            h->first};
  for (int i = 0; i < 20; i++) ref_put(&o, hdr[i], 4);
  ref_put(&o, p->seed, 8);
  ref_put(&o, h->n, 8);
  for (uint32_t li = h->first; li < h->built; li++) {
    const ref_layer* L = &h->layer[li];
    ref_put(&o, L->info.n, 8);
    ref_put(&o, L->info.m, 8);
    ref_put(&o, L->info.nranges, 8);
    uint64_t B = L->info.nbuckets;
    if (p->threshold_mode == 1) {
      uint64_t K = 0;
      for (uint64_t wd = 0; wd < (B + 63) / 64; wd++) {
        uint64_t word = 0;
        for (uint64_t beta = wd * 64; beta < B && beta < wd * 64 + 64; beta++)
          if (L->code[beta]) { word |= 1ull << (beta % 64); K++; }
        ref_put(&o, word, 8);
      }
      ref_put(&o, K, 8);
      uint64_t k = 0;
      for (uint64_t beta = 0; beta < B; beta++)
        if (L->code[beta]) { ref_put(&o, (uint64_t)(L->code[beta] - 1), 1); k++; }
      for (; k % 8; k++) ref_put(&o, 0, 1);
    } else {
      for (uint64_t wd = 0; wd < (B + 31) / 32; wd++) {
        uint64_t word = 0;
        for (uint64_t beta = wd * 32; beta < B && beta < wd * 32 + 32; beta++)
          word |= (uint64_t)L->code[beta] << (2 * (beta % 32));
        ref_put(&o, word, 8);
      }
    }
    for (uint64_t wd = 0; wd < (L->info.m / 64) * h->r; wd++) ref_put(&o, L->W[wd], 8);
    if (p->cut_strategy != 0) {
      uint64_t R = L->info.nranges, k = 0;
      for (; k + 1 < R; k++) ref_put(&o, L->cut_last[k], 4);
      for (; k % 2; k++) ref_put(&o, 0, 4);
    }
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
  if (!h || layer < h->first || layer >= h->built || !out) return REF_E_INVALID;
  *out = h->layer[layer].info;
  return REF_OK;
}

int ref_get_final_info(const ref_burr* h, ref_final_info* out) {
  if (!h || !out) return REF_E_INVALID;
  *out = h->fin_info;
  return REF_OK;
}

uint64_t ref_layer_keys(const ref_burr* h, uint32_t layer, uint64_t* out, uint64_t cap) {
  if (!h || layer < h->first || layer > h->built) return 0;
  const ref_layer* L = layer < h->built ? &h->layer[layer] : &h->fin;
  uint64_t n = L->info.n;
  if (out)
    for (uint64_t i = 0; i < n && i < cap; i++) out[i] = L->keys[i];
  return n;
}

uint64_t ref_layer_codes(const ref_burr* h, uint32_t layer, uint8_t* out, uint64_t cap) {
  if (!h || layer < h->first || layer >= h->built) return 0;
  const ref_layer* L = &h->layer[layer];
  uint64_t B = L->info.nbuckets;
  if (out)
    for (uint64_t i = 0; i < B && i < cap; i++) out[i] = L->code[i];
  return B;
}

uint64_t ref_layer_cuts(const ref_burr* h, uint32_t layer, uint64_t* out, uint64_t cap) {
  if (!h || layer < h->first || layer >= h->built) return 0;
  const ref_layer* L = &h->layer[layer];
  uint64_t R = L->info.nranges;
  if (out)
    for (uint64_t i = 0; i < R && i < cap; i++) out[i] = L->cut_last[i];
  return R;
}

uint64_t ref_layer_solution(const ref_burr* h, uint32_t layer, uint32_t* out, uint64_t cap) {
  if (!h || layer < h->first || layer > h->built) return 0;
  const ref_layer* L = layer < h->built ? &h->layer[layer] : &h->fin;
  uint64_t m = L->info.m;
  if (out)
    for (uint64_t i = 0; i < m && i < cap; i++) out[i] = L->Z[i];
  return m;
}
