"""Search a hash-predicate seed whose marked set has an exact size, using the CPU oracle only.

The single-large-instance workload marks index i when the low `bits` bits of SplitMix64_i(seed) are
zero.  Over 2^n indices the expected hit count is 2^(n - bits); this script takes the first seed at or
above `--start` whose hit count is exactly `--m`, and prints it with its marked indices.

    python oracle/find_hash_seed.py --n 28 --bits 25 --m 8 --start 0x6A09E667F3BCC908
"""
from __future__ import annotations

import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--bits", type=int, default=25)
    ap.add_argument("--m", type=int, default=8)
    ap.add_argument("--start", type=lambda s: int(s, 0), default=0x6A09E667F3BCC908)
    ap.add_argument("--tries", type=int, default=200)
    a = ap.parse_args()
    o = oracle.default()
    for t in range(a.tries):
        seed = (a.start + t) & (2**64 - 1)
        marks, count = o.hash_marks(a.n, seed, a.bits, cap=4 * a.m + 16)
        print(f"seed {seed:#018x}: {count} hits", flush=True)
        if count == a.m:
            print(f"FOUND seed={seed:#018x} marks={[int(x) for x in marks]}")
            return
    sys.exit("no seed found")


if __name__ == "__main__":
    main()
