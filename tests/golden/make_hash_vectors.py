"""Writes hash_vectors.txt: start slot, coefficient row and fingerprints of
sampled (key, layer, m, seed) tuples as the oracle computes them.

Calls only the oracle. The file is a regression fixture of the oracle's hash
(the hash is a reading: the paper defines none); the test that reads it also
checks every line against an independent recomputation of the reading and
against special cases that reduce it to the published finalizer alone.

Usage: python tests/golden/make_hash_vectors.py
"""
import os
import random
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

MS = [64, 65, 127, 128, 129, 4096, 970_048, 97_000_000, 970_000_000,
      (1 << 40) - 1, (1 << 40) + 64]


def main():
    rng = random.Random(20241112)
    lines = ["# key layer m seed start row fp1 fp8 fp16 fp32 (hex u64 / decimal)",
             "# reading 1 of the oracle's hash; written by make_hash_vectors.py from the oracle"]
    for i in range(400):
        key = rng.getrandbits(64) if i % 7 else rng.choice([0, 1, (1 << 64) - 1, 1 << 63])
        layer = rng.randrange(0, 6)
        m = MS[i % len(MS)] if i % 3 else rng.randrange(64, 1 << 41)
        seed = rng.getrandbits(64) if i % 5 else rng.randrange(0, 16)
        s, c = oracle.hash_key(key, layer, m, seed)
        fps = [oracle.fingerprint(key, r, seed) for r in (1, 8, 16, 32)]
        lines.append(f"{key:016x} {layer} {m} {seed:016x} {s} {c:016x} "
                     + " ".join(str(f) for f in fps))
    with open(os.path.join(HERE, "hash_vectors.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
