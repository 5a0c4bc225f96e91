"""Writes the oracle regression snapshots in this folder.

Calls only the oracle and the seeded input generator.  Each snapshot freezes
the oracle's output for one small seeded case so that an unintended change to
the oracle's arithmetic shows up as a test failure; what makes the values
right is pinned separately (closed forms, library routines, identities).

    python tests/golden/make_golden.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import inverse  # noqa: E402
from paper_1908_06096_amd.inputs import spectral_coefficients  # noqa: E402

CASES = [
    # (file, truncation, grid, seed)
    ("oracle_T7_full_seed3.txt", 7, "full", 3),
    ("oracle_T7_octahedral_seed3.txt", 7, "octahedral", 3),
]


def main():
    for fname, N, grid, seed in CASES:
        s = spectral_coefficients(N, 1, seed=seed)
        spec = s[..., 0] + 1j * s[..., 1]
        _four, g = inverse(spec, N, grid)
        with open(os.path.join(HERE, fname), "w") as fh:
            fh.write("# oracle synthesis of seeded coefficients (inputs.spectral_coefficients)\n")
            fh.write(f"# truncation {N} grid {grid} seed {seed} fields 1; grid values ring-major, north to south\n")
            for v in g[0]:
                fh.write(f"{v:.17e}\n")


if __name__ == "__main__":
    main()
