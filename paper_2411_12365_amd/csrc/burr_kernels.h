// burr_kernels.h - host-side launchers of the HIP kernels (internal to the
// library; the public interface is include/burr.h). Every launcher works on
// one layer of one or more structures described by a LayerGeom.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "burr_dev.h"

namespace burr {

// Exclusive prefix sum of n u32 values in place; `tmp` needs scan_tmp_words(n) u32.
size_t scan_tmp_words(size_t n);
hipError_t scan_exclusive(uint32_t* data, size_t n, uint32_t* tmp, hipStream_t s);

// Sorting of one layer's keys by (bucket, chunk) - three levels:
//   level 1: hash every key, partition into nb1 bins of S sub-bins
//   level 2: per bin, partition into its sub-bins of kSubBuckets buckets
//   level 3: per sub-bin, order by (bucket, chunk) in LDS and write the
//            item stream (bucket headers + records) and the bucket starts
// Every level writes contiguous runs (tiles are ordered in LDS first). When
// a workgroup's (bin, sub-bin) counters fit in LDS, one counting pass over
// the keys serves both partition levels (plan.H > 0).
struct SortPlan {
  uint32_t nsub;       // sub-bins (level-3 workgroups)
  uint32_t nb1;        // level-1 bins
  uint32_t S;          // sub-bins per bin
  uint32_t G1;         // level-1 workgroups
  uint64_t per_group;  // keys per level-1 workgroup
  uint32_t U2;         // level-2 workgroups launched (bound on the chunks)
  uint32_t H;          // fused counting: level-2 chunks per bin (0: a counting pass per level)
  float invS;          // 1/S rounded to nearest (on the host)
  uint32_t cs;         // fused counting: level-1 workgroups per level-2 chunk
  uint32_t cc;         // fused counting: level-1 workgroups per counting workgroup (divides cs)
  uint32_t Hc;         // fused counting: counting workgroups
  bool big1, big2;     // tiles of twice the records at level 1 / level 2
};
// nstructs: structures in the layer (a batch's tiles are sized for them)
SortPlan plan_sort(uint64_t nkeys, uint64_t nbuckets, uint32_t nstructs);
// u32 words of counts2 a plan needs
uint64_t sort_counts2_words(const SortPlan& sp);

// Words that the launches after a sort need zeroed (the insertion's step
// counter and failure flags, the bump-count scan's last entry, the final
// layer's spill occupancy): the sort's level-3 kernel, which every sort ends
// with, clears them, so no memset launch of their own sits on the build's
// critical path. Unused entries have n = 0.
struct SortClear {
  uint32_t* p[2];
  uint64_t n[2];
};

struct SortArgs {
  const uint64_t* keys;   // input keys (g.nkeys), structure j at g.key_off[j]
  const void* vals;       // input values or nullptr (filter fingerprints)
  uint32_t vbytes;        // 1, 2 or 4
  uint32_t mask_values;   // first layer: mask to r bits / compute fingerprints
  uint64_t fp_salt;       // fingerprint salt (filter mode)
  uint32_t filter;        // values are fingerprints
  LayerGeom g;
  SortPlan plan;
  uint32_t* counts1;      // nb1 * G1 (+1), scanned in place
  uint32_t* counts2;      // sort_counts2_words(plan), scanned in place
  uint32_t* scan_tmp;     // for the larger of the two scans
  uint32_t* binlo;        // nb1 + 1
  uint32_t* nch;          // nb1 + 1
  uint32_t* cbase;        // nb1 + 1
  uint32_t* sstart;       // nsub + 1
  void* r1;               // nkeys intermediate records of 12 or 16 bytes (level 1 output)
  void* r2;               // the same, level 2 output
  Rec* out_rec;           // item stream (nkeys + nbuckets)
  uint32_t* bstart;       // B + 1 bucket start offsets
  SortClear clear;        // zeroed by the last sort kernel
};
hipError_t sort_layer(const SortArgs& a, hipStream_t s);

// Cut points of a BuRR layer (g.cut_strategy != 0): rfirst[rho] = first
// global bucket of global range rho (nranges + 1 entries), from the bucket
// headers of the sorted item stream.
hipError_t choose_cuts(const Rec* rec, const uint32_t* bstart, const LayerGeom& g, uint32_t* rfirst,
                       hipStream_t s);

// Per-range insertion with 2-bit thresholds and boundary bumping: one wave
// per range, its 64 lanes insert a bucket's records together against a ring
// of 128 rows in LDS.
struct SolveArgs {
  const Rec* rec;
  const uint32_t* bstart;
  LayerGeom g;
  uint64_t* rowsC;     // m rows, written through at placement
  uint32_t* rowsV;     // m values
  uint64_t* occ;       // m/64 occupancy words
  uint8_t* code8;      // B codes (not in plain mode)
  uint32_t* bump;      // B bumped-key counts (not in plain mode)
  uint32_t* fail;      // per structure: 1 inconsistent final layer, >= 2 internal error
  uint64_t* steps;     // optional: total elimination steps (statistics)
  uint32_t nrec;       // number of items (prefetch bound)
  // final-layer segments: rows that land past a segment's end go to its
  // spill buffer (64 rows + occupancy word per segment) instead of failing
  uint64_t* spillC;
  uint32_t* spillV;
  uint64_t* spill_occ;
  // optional, 16 u64 zeroed by the caller: the first wave that stops with an
  // internal error records [1, code, range, structure, header item, records,
  // bucket, buckets, candidates, 0, kept, threshold, forced, 0, 0, first bucket]
  uint64_t* diag;
};
hipError_t solve_layer(const SolveArgs& a, hipStream_t s);

// Back-substitution per range into column-interleaved words
// W[word_base[j] + k*r_j + col]. Free slots hold row 0 and value 0 (as every
// released block does). bnd (optional, 64 u32 per range): solution values of
// the 63 slots after each range's end (final-layer segments, whose rows
// cross segment ends). max_waves (0: one wave per NG ranges): the grid's
// width, but at least a quarter of the full grid (a long back-substitution
// held to a few waves would outlast the work it overlaps); its waves then
// take the ranges in turn.
hipError_t back_substitute(const uint64_t* rowsC, const uint32_t* rowsV, const LayerGeom& g,
                           uint64_t* W, hipStream_t s, const uint32_t* bnd = nullptr,
                           uint32_t max_waves = 0);

// code8[B] -> packed 2-bit code words of every structure
hipError_t pack_codes(const uint8_t* code8, const LayerGeom& g, uint64_t ncode_words,
                      uint64_t* words, hipStream_t s);

// 1+-bit thresholds: code8[B] (threshold per bucket, 0 = none) -> bit words
// (nwords = code_base of the layer), thresholds - 1 as bytes at thr_base[j],
// rank directory at rank_base[j] (u32 per 8 bit words), thresholds per
// structure in kcount[J]. pc: nwords + 1 u32 of workspace.
hipError_t pack_thresholds(const uint8_t* code8, const LayerGeom& g, uint64_t nwords,
                           uint64_t* bits, uint32_t* pc, uint32_t* scan_tmp, uint8_t* thr,
                           uint32_t* rank, uint32_t* kcount, hipStream_t s);

// Copy the bumped suffix of every bucket into the next layer's input.
hipError_t gather_bumped(const Rec* rec, const uint32_t* bstart,
                         const uint32_t* off /* scanned bump counts, B+1 */, uint64_t B,
                         uint64_t* next_keys, uint32_t* next_vals, hipStream_t s);

// out[j] = off[bucket_base[j]] for j <= J (bumped keys before structure j)
hipError_t struct_offsets(const uint32_t* off, const LayerGeom& g, uint32_t* out, hipStream_t s);

// Final plain layer, after the per-segment solve (g.nranges = segments):
// merge each structure's segments' spill rows pairwise over log2 levels,
// then compute each segment's boundary values.
struct FinalArgs {
  LayerGeom g;
  uint64_t* rowsC;
  uint32_t* rowsV;
  uint64_t* occ;
  uint64_t* spillC;
  uint32_t* spillV;
  uint64_t* spill_occ;
  uint32_t* fail;     // per structure
  uint32_t* z0first;  // segments x 64: a segment's first 63 values with a zero boundary
  uint64_t* xfirst;   // segments x 64: their dependence on the 63 boundary values
  uint32_t* bnd;      // segments x 64: true values of the 63 slots after each segment
};
hipError_t final_merge(const FinalArgs& a, uint64_t max_segments, hipStream_t s);
hipError_t final_boundaries(const FinalArgs& a, hipStream_t s);

// Copies the inputs of J structures, each in its own device arrays, into
// one key array and one value array of out_vb-byte elements (structure j at
// off[j]). tab (device): J key pointers, J value pointers (0 in filter mode),
// J+1 offsets, J input value widths - one u64 each.
hipError_t concat_inputs(const uint64_t* tab, uint32_t J, uint64_t n, uint64_t* out_keys,
                         void* out_vals, uint32_t out_vb, hipStream_t s);

// n synthetic keys (SplitMix64 stream of `seed`) and, if vals, n values
// (stream of vseed AND vmask) in elements of vb bytes.
hipError_t fill_stream(uint64_t* keys, void* vals, uint32_t vb, uint64_t n, uint64_t seed,
                       uint64_t vseed, uint64_t vmask, hipStream_t s);

hipError_t query(const QueryPlan& plan, const uint64_t* keys, uint64_t n, void* out,
                 uint32_t out_bytes, uint32_t contains, uint64_t fp_salt, hipStream_t s);

}  // namespace burr
