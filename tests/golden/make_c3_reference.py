"""Write c3_reference.txt: the 13 smallest eigenvalues of the 1,056,759-dof
rectangle workload ([0,1] x [0,1.01], P1 on the uniform "/" mesh with 1024 x 1034
cells), computed by the FP64 oracle's reference eigensolver (shift-invert Lanczos
about 0, tolerance 1e-14).  Calls only the oracle and the input generator.

Usage:  python tests/golden/make_c3_reference.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bpjd_oracle as o            # noqa: E402
from paper_2203_06327_amd import workloads as w  # noqa: E402


def main():
    mesh, cfg = w.config_mesh("c3")
    lam, _ = o.reference_eigs(mesh.K, mesh.M, 13)
    with open(os.path.join(HERE, "c3_reference.txt"), "w") as fh:
        fh.write("# 13 smallest eigenvalues of (K, M) for -Laplace u = lambda u on [0,1] x [0,1.01],\n"
                 "# P1 on the uniform '/' mesh with 1024 x 1034 cells (1,056,759 dofs), homogeneous\n"
                 "# Dirichlet data; written by tests/golden/make_c3_reference.py from the oracle's\n"
                 "# reference eigensolver (shift-invert Lanczos, tolerance 1e-14).\n")
        for i, v in enumerate(lam, 1):
            fh.write(f"{i:2d} {v:.15e}\n")


if __name__ == "__main__":
    main()
