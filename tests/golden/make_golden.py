"""Writes the stored expected values under tests/golden/ from the oracle only.

pcg_kat.txt -- known answers of the jitter hash (Section 3.2's per-pixel random
offset, drawn as a PCG hash chain of Jarzynski and Olano 2020): pcg(v) for
a set of inputs, and the chained offset bits (h >> 8) for a grid of pixels,
frames and seeds. The HIP library must reproduce them bit for bit.

Run: python tests/golden/make_golden.py
"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.cloud import pcg_hash, jitter_offset  # noqa: E402

PCG_INPUTS = [0, 1, 2, 3, 7, 255, 256, 1609, 5344, 65535, 65536, 123456789,
              0x7FFFFFFF, 0x80000000, 0xDEADBEEF, 0xFFFFFFFE, 0xFFFFFFFF]
GRID = [(px, py, frame, seed)
        for seed in (0, 1609)
        for frame in (0, 1, 15)
        for py in (0, 1, 719, 1079)
        for px in (0, 1, 2, 1279, 1919, 3839)]


def main():
    path = os.path.join(HERE, "pcg_kat.txt")
    with open(path, "w") as f:
        f.write("# pcg v -> pcg(v); written by tests/golden/make_golden.py from the oracle\n")
        for v in PCG_INPUTS:
            f.write(f"pcg {v} {pcg_hash(v)}\n")
        f.write("# jit px py frame seed -> (h >> 8), where j = (h >> 8) * 2^-24\n")
        for px, py, fr, sd in GRID:
            bits = int(round(jitter_offset(px, py, fr, sd) * 2 ** 24))
            f.write(f"jit {px} {py} {fr} {sd} {bits}\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
