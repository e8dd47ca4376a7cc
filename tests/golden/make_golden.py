"""Write the stored expected values under tests/golden/ that come from the CPU oracle.

Only the oracle (the `oracle` package) is called here; nothing from the HIP library.

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(_HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def write_hash_marks() -> None:
    w = workloads.HASH_N28
    marks, count = oracle.default().hash_marks(w.n, w.hash_seed, w.hash_bits, cap=64)
    path = os.path.join(_HERE, "hash_marks_n28.txt")
    with open(path, "w") as f:
        f.write("# Marked set of the single-large-instance workload: n = 28, hash seed "
                f"{w.hash_seed:#018x}, predicate (SplitMix64_i(seed) mod 2^{w.hash_bits}) == 0.\n")
        f.write("# Enumerated over all 2^28 indices by the CPU oracle (tests/golden/make_golden.py).\n")
        f.write(f"# count {count}\n")
        for x in marks.tolist():
            f.write(f"{x}\n")


if __name__ == "__main__":
    write_hash_marks()
