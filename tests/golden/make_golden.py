#!/usr/bin/env python3
"""Writes tests/golden/edt_7x6x5.txt from the CPU oracle only.

The paper prints no numeric worked example of the transform (Sec. III-C),
so this fixture holds the oracle's own result on a small hand-built map --
five sites, two of them equidistant from many voxels -- as a regression
fixture for the oracle and the device path.  Its values are pinned by the
definition: the fixture test recomputes each one by exhaustive search.
Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

SHAPE = (5, 6, 7)   # (nz, ny, nx)
SITES = [(0, 0, 0), (6, 5, 4), (3, 2, 2), (1, 4, 0), (5, 0, 3)]   # (x, y, z)


def build():
    occ = np.zeros(SHAPE, np.uint8)
    for x, y, z in SITES:
        occ[z, y, x] = 1
    return occ


def main():
    occ = build()
    d2, site = oracle.edt(occ)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "edt_7x6x5.txt")
    with open(path, "w") as f:
        f.write("# exact squared EDT of a 7 x 6 x 5 map (x fastest), sites (x,y,z): "
                + " ".join(f"{s}" for s in SITES) + "\n")
        f.write("# definition: Sec. III-C (closest occupied voxel); ties -> smallest linear index\n")
        f.write("# columns: linear_index d2 site\n")
        for i, (a, b) in enumerate(zip(d2.ravel(), site.ravel())):
            f.write(f"{i} {a} {b}\n")
    print(path)


if __name__ == "__main__":
    main()
