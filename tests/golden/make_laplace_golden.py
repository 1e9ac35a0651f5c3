"""Writes laplace_sh_sphere_2m_first16.txt: the 16 lowest eigenvalues of the
cotangent Laplacian (lumped mass) of the SH-displaced sphere of about 2.0M
faces (the mesh of workloads.sh_sphere_2m, FP32 vertex positions), computed
by the CPU oracle (oracle/laplace.py, shift-invert ARPACK). Takes a few
minutes; run from the repository root:

    python tests/golden/make_laplace_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import laplace as LP  # noqa: E402
from paper_2606_05581_amd import workloads as W  # noqa: E402


def mesh():
    rng = np.random.default_rng(1002)
    V, F = W.sh_displaced_sphere(316, 16, 0.05, rng)
    V = W.normalise_unit_ball(V)
    return V.astype(np.float32), F.astype(np.int32)


if __name__ == "__main__":
    V, F = mesh()
    lam, _, _ = LP.laplacian_basis(V.astype(np.float64), F, 16)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "laplace_sh_sphere_2m_first16.txt")
    with open(out, "w") as f:
        f.write("# 16 lowest eigenvalues of L phi = lambda M phi (cotangent stiffness, lumped mass) on the\n")
        f.write("# SH-displaced sphere of workloads.sh_sphere_2m; written by make_laplace_golden.py (oracle)\n")
        for v in lam:
            f.write(f"{v:.17e}\n")
    print(out)
