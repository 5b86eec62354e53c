"""Write p128_reference.txt: the 8 smallest eigenvalues of the clamped-plate
workload (Lap^2 u = lambda u on the unit square, u = du/dn = 0 on the edges,
Bogner-Fox-Schmit elements on 128 x 128 cells, 64,516 dofs), computed by the
FP64 oracle's reference eigensolver (shift-invert Lanczos about 0, tolerance
1e-14).  Calls only the oracle and the input generator.

Usage:  python tests/golden/make_p128_reference.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bpjd_oracle as o            # noqa: E402
from paper_2203_06327_amd import workloads as w  # noqa: E402


def main():
    plate, cfg = w.config_plate("p128")
    lam, _ = o.reference_eigs(plate.K, plate.M, 8)
    with open(os.path.join(HERE, "p128_reference.txt"), "w") as fh:
        fh.write("# 8 smallest eigenvalues of (K, M) for Lap^2 u = lambda u on the unit square with\n"
                 "# clamped edges, Bogner-Fox-Schmit elements on 128 x 128 cells (64,516 dofs);\n"
                 "# written by tests/golden/make_p128_reference.py from the oracle's reference\n"
                 "# eigensolver (shift-invert Lanczos, tolerance 1e-14).\n")
        for i, v in enumerate(lam, 1):
            fh.write(f"{i:2d} {v:.15e}\n")


if __name__ == "__main__":
    main()
