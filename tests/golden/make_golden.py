"""Writes tests/golden/hash_vectors.txt from the oracle alone.

The hash is this project's definition (a seeded mixer built on the
SplitMix64 finalizer), so these vectors pin the GPU library to the oracle,
not to an external source; the oracle itself is pinned by the published
SplitMix64 outputs in splitmix64_state0.txt.

Run from the repository root:  python tests/golden/make_golden.py
"""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_1712_09624_amd import workload as W  # noqa: E402


def main():
    keys = [np.zeros(16, np.uint8), np.full(16, 0xFF, np.uint8),
            np.arange(16, dtype=np.uint8)]
    keys += list(W.five_tuples(29, 1))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hash_vectors.txt")
    with open(out, "w") as f:
        f.write("# Hash test vectors written by tests/golden/make_golden.py from the oracle.\n")
        f.write(f"# seed {W.HASH_SEED:016x}\n")
        f.write("# key(hex, 16 bytes)  h(hex)  p14 a14 tag  p24 a24\n")
        for k in keys:
            h = int(O.hash_keys(k.reshape(1, 16), W.HASH_SEED)[0])
            s14 = O.split(h, 14)
            s24 = O.split(h, 24)
            f.write(f"{bytes(k).hex()} {h:016x} {s14['p']} {s14['a']} {s14['tag']} "
                    f"{s24['p']} {s24['a']}\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
