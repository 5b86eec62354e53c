"""Write c4_reference.txt: the 8 smallest eigenvalues of the clamped-plate
workload (Lap^2 u = lambda u on the unit square, u = du/dn = 0 on the edges,
Bogner-Fox-Schmit elements on 256 x 256 cells, 260,100 dofs), computed by the
FP64 oracle's reference eigensolver (shift-invert Lanczos about 0, tolerance
1e-14, then Rayleigh-Ritz on its vectors), each with the relative accuracy the
FP64 data allow: u (x^T |K| x / x^T K x + x^T |M| x / x^T M x) with u = 2^-53,
the first-order change of the eigenvalue when every entry of K and M moves by one
rounding.  At this mesh size the fourth-order operator cancels terms 10^8 times
larger than lambda x in K x, so that floor exceeds 1e-10.  The header also
records the pencil's largest eigenvalue and u lambda_max / lambda_1, the relative
residual that FP64 vectors can be held to (entries with relative errors of order
u reach up to that residual).  Calls only the oracle and the input generator.

Usage:  python tests/golden/make_c4_reference.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bpjd_oracle as o            # noqa: E402
from paper_2203_06327_amd import workloads as w  # noqa: E402


def main():
    plate, cfg = w.config_plate("c4")
    lam, X = o.reference_eigs(plate.K, plate.M, 8)
    aK, aM = abs(plate.K), abs(plate.M)
    floor = [2.0 ** -53 * (X[:, i] @ (aK @ X[:, i]) / (X[:, i] @ (plate.K @ X[:, i]))
                           + X[:, i] @ (aM @ X[:, i]) / (X[:, i] @ (plate.M @ X[:, i]))) for i in range(8)]
    lmax = o.largest_eigenvalue(plate.K, plate.M)
    with open(os.path.join(HERE, "c4_reference.txt"), "w") as fh:
        fh.write("# 8 smallest eigenvalues of (K, M) for Lap^2 u = lambda u on the unit square with\n"
                 "# clamped edges, Bogner-Fox-Schmit elements on 256 x 256 cells (260,100 dofs);\n"
                 "# written by tests/golden/make_c4_reference.py from the oracle's reference\n"
                 "# eigensolver (shift-invert Lanczos, tolerance 1e-14, Rayleigh-Ritz on its vectors).\n"
                 f"# lambda_max = {lmax:.6e}\n"
                 f"# residual_floor = {2.0 ** -53 * lmax / lam[0]:.3e}   (u lambda_max / lambda_1)\n"
                 "# columns: index, eigenvalue, relative accuracy the FP64 data allow\n")
        for i, (v, f) in enumerate(zip(lam, floor), 1):
            fh.write(f"{i:2d} {v:.15e} {f:.3e}\n")
    print(np.asarray(lam), np.asarray(floor))


if __name__ == "__main__":
    main()
