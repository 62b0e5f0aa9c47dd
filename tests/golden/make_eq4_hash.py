"""Write eq4_hash.txt: Eq. 4 (Sec. 3.2) evaluated by the oracle for a fixed set of block keys.

Run from the repository root: python tests/golden/make_eq4_hash.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

KEYS = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (-1, 0, 0), (1, 2, 3), (-5, 7, -11),
        (1000, -2000, 300), (-1048574, 1048574, -1), (123456, -654321, 777777)]
SIZES = [1 << 16, 1 << 20, 1 << 22, 1000003]


def main():
    oracle.build(force=False)
    lines = ["# Eq. 4 (Sec. 3.2): H = (x p1 xor y p2 xor z p3) mod n_hash, p1 = 73856093, p2 = 19349669,",
             "# p3 = 83492791; products and xor in 32-bit unsigned arithmetic (the paper prints no",
             "# vectors; these are the oracle's evaluation of the equation).",
             "# x y z n_hash H"]
    for (x, y, z) in KEYS:
        for n in SIZES:
            lines.append(f"{x} {y} {z} {n} {oracle.eq4_hash(x, y, z, n)}")
    with open(os.path.join(HERE, "eq4_hash.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
