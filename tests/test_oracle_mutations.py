"""The pins are strong enough: plausible mistakes planted in copies of the
oracle (on the CPU, in a temporary directory) must each fail at least one pin.

Every mutant is compiled and checked in a child process, so a mutant that
aborts counts as caught without taking the test runner down.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "chunks_low_to_high": ("for (unsigned k = 3; k > kf; k--) {",
                           "for (unsigned k = kf + 1; k <= 3; k++) {"),
    "bump_high_offsets": ("if (o < T) {", "if (o >= T && T) {"),
    "forced_off_by_one": ("if (s + REF_W > range_end) {", "if (s + REF_W > range_end + 1) {"),
    "backsub_index": ("z ^= Z[i + j];", "z ^= Z[i + j - 1];"),
    "mixer_constant": ("k *= 0xc4ceb9fe1a85ec53ULL;", "k *= 0xc4ceb9fe1a85ec55ULL;"),
    "mixer_shift": ("  k ^= k >> 33;\n  return k;", "  k ^= k >> 31;\n  return k;"),
    "fastrange_low_word": ("return (uint64_t)(prod >> 64);", "return (uint64_t)(prod >> 63) % n;"),
    "interleave_block": ("W[(i / 64) * r + col] |= 1ull << (i % 64);",
                         "W[(i / 64) * r + (r - 1 - col)] |= 1ull << (i % 64);"),
    "final_scale": ("(uint64_t)a * p->final_den", "(uint64_t)a * p->final_den * 0"),
    "row_not_anchored": ("*coeff = ref_fmix64(key ^ salt_c) | 1ull;",
                         "*coeff = ref_fmix64(key ^ salt_c) | 2ull;"),
    "code_shifted": ("code = k;\n          break;", "code = k - 1;\n          break;"),
    "redundant_is_conflict": ("return v == 0 ? INS_REDUNDANT : INS_CONFLICT;",
                              "return INS_CONFLICT;"),
    "query_threshold": ("if (o < ref_theta(p, L->code[beta])) continue;",
                        "if (o <= ref_theta(p, L->code[beta])) continue;"),
    "layer_salt": ("uint64_t salt_s = ref_fmix64(seed ^ (2ull * layer + 1ull));",
                   "uint64_t salt_s = ref_fmix64(seed ^ (2ull * layer + 2ull));"),
    "range_split": ("return (uint64_t)(((unsigned __int128)rho * B) / R);",
                    "return (uint64_t)(((unsigned __int128)rho * B + R - 1) / R);"),
    "start_span_short": ("*start = ref_fastrange(ref_fmix64(key ^ salt_s), m - REF_W + 1);",
                         "*start = ref_fastrange(ref_fmix64(key ^ salt_s), m - REF_W);"),
    "salt_plus_not_xor": ("uint64_t salt_s = ref_fmix64(seed ^ (2ull * layer + 1ull));",
                          "uint64_t salt_s = ref_fmix64(seed + (2ull * layer + 1ull));"),
    "salts_swapped": ("uint64_t salt_s = ref_fmix64(seed ^ (2ull * layer + 1ull));\n"
                      "  uint64_t salt_c = ref_fmix64(seed ^ (2ull * layer + 2ull));",
                      "uint64_t salt_s = ref_fmix64(seed ^ (2ull * layer + 2ull));\n"
                      "  uint64_t salt_c = ref_fmix64(seed ^ (2ull * layer + 1ull));"),
    "fingerprint_salt": ("uint64_t h = ref_fmix64(key ^ ref_fmix64(~seed));",
                         "uint64_t h = ref_fmix64(key ^ ref_fmix64(seed));"),
    "one_plus_threshold_low": ("code = (unsigned)(o + 1);", "code = (unsigned)o;"),
    "one_plus_undo_earlier_groups": ("          nplaced = 0; /* earlier groups are final */\n", ""),
    "one_plus_forced": ("if (p->threshold_mode == 1) return (unsigned)(omax + 1);",
                        "if (p->threshold_mode == 1) return (unsigned)(omax + 2);"),
    "cut_prev_window": ("if (order[t].s + (REF_W - 1) < beta * b) break;",
                        "if (order[t].s + REF_W < beta * b) break;"),
    "cut_tie_break": ("(score == best && dist < best_dist)", "(score == best && dist <= best_dist)"),
    "cut_window": ("const uint64_t hmax = L >= 2 ? (L - 2) / 2 : 0;",
                   "const uint64_t hmax = L >= 2 ? (L - 1) / 2 : 0;"),
    "cut_maxprev_sign": ("p->cut_strategy == 2 ? -prev", "p->cut_strategy == 2 ? prev"),
    "parallel_backsub_short": ("ref_back_substitute(M->C + base, M->V + base, M->Z + base, len);",
                               "ref_back_substitute(M->C + base, M->V + base, M->Z + base, len - 64);"),
    "parallel_part_of_slot": ("return (uint64_t)(((unsigned __int128)(s / M->p->bucket) * M->T) / M->B);",
                              "return (uint64_t)(((unsigned __int128)(s / M->p->bucket) * M->T) / M->B) % 2;"),
    "load_rounding": ("uint64_t nb = (uint64_t)((num + den - 1) / den);\n  if (nb < 1) nb = 1;\n  return nb * b;",
                      "uint64_t nb = (uint64_t)(num / den);\n  if (nb < 1) nb = 1;\n  return nb * b;"),
}

CHECK = r"""
import sys
sys.path.insert(0, {root!r})
import oracle
oracle._LIB_PATH = {lib!r}
oracle._lib = None
from tests import test_oracle_bruteforce as bf, test_oracle_hash as th
from tests import test_oracle_hash_composition as hc
from paper_2411_12365_amd import workload as W
import numpy as np
failed = []
def run(name, fn, *a):
    try:
        fn(*a)
    except Exception as e:
        failed.append(name)
for case in bf.CASES[:5] + bf.CASES[7:8] + bf.CASES[12:]:
    run("brute%r" % (case[:2],), bf.test_layers_match_dense_definition, *case)
for case in bf.CUT_CASES[1:2] + bf.CUT_CASES[3:4]:
    run("cuts%r" % (case[0],), bf.test_cut_points_match_definition, *case)
from tests import test_oracle_parallel as tp
for case in (tp.CASES[0], tp.CASES[3], tp.CASES[4]):
    run("parallel%r" % (case[:2],), tp.test_parallel_driver_equals_sequential, *case, 3)
run("edge", bf.test_boundary_edge_case)
run("dups", bf.test_equal_duplicates_are_redundant_equations)
run("indep", th.test_start_and_row_are_independent)
run("final", bf.test_final_layer_scale_up_attempts)
run("fmix", th.test_fmix64_is_inverted_by_the_published_steps)
run("fastrange", th.test_fastrange_is_exact_floor)
run("hashshape", th.test_hash_ranges_and_row_shape)
run("layers", th.test_layers_hash_independently)
for layer in (0, 3):
    run("start_salt%d" % layer, hc.test_start_salt_zero_reduces_to_the_finalizer, layer)
    run("row_salt%d" % layer, hc.test_row_salt_zero_reduces_to_the_finalizer, layer)
run("fp_salt", hc.test_fingerprint_salt_zero_reduces_to_the_finalizer)
run("largest_start", hc.test_largest_start_at_any_seed)
run("golden", hc.test_golden_vectors)
def query_inv():
    k = W.keys(20000, 3); v = W.values(20000, 8, 4)
    b = oracle.build(k, v, 8, oracle.Params(ranges=16))
    assert (b.query(k) == v).all()
run("query", query_inv)
print("FAILED:" + ",".join(failed))
"""


def _mutated_check(name, old, new, tmp):
    src = open(os.path.join(ROOT, "oracle", "burr_oracle.c")).read()
    assert old in src, f"mutation {name} no longer applies"
    d = os.path.join(tmp, name)
    os.makedirs(d)
    with open(os.path.join(d, "burr_oracle.c"), "w") as f:
        f.write(src.replace(old, new, 1))
    with open(os.path.join(d, "burr_oracle.h"), "w") as f:
        f.write(open(os.path.join(ROOT, "oracle", "burr_oracle.h")).read())
    lib = os.path.join(d, "libmut.so")
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", os.path.join(d, "burr_oracle.c"),
                           "-o", lib])
    try:
        proc = subprocess.run([sys.executable, "-c", CHECK.format(root=ROOT, lib=lib)],
                              capture_output=True, text=True, timeout=30)
    except subprocess.TimeoutExpired:
        return "hung"  # e.g. an elimination that never advances
    if proc.returncode != 0:
        return "crashed"
    line = [ln for ln in proc.stdout.splitlines() if ln.startswith("FAILED:")]
    return line[-1][len("FAILED:"):] if line else "no-output"


def test_unmutated_oracle_passes_the_mutation_checks(tmp_path):
    assert _mutated_check("identity", "#define REF_W 64u", "#define REF_W 64u", str(tmp_path)) == ""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    caught = _mutated_check(name, old, new, str(tmp_path))
    assert caught != "", f"mutant {name} passed every pin"
