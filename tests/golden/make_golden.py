"""Write the small golden fixtures in this folder.

Calls only the oracle's exact rational arithmetic (``oracle.exact``); the
inputs come from the seeded generators.  Each file stores its inputs as
hexadecimal floats so that it does not depend on the generator staying
unchanged.  Run:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import exact  # noqa: E402
from paper_1612_01855_amd import inputs as gen  # noqa: E402


def _write(name, header, mats):
    with open(os.path.join(HERE, name), "w") as f:
        for line in header:
            f.write("# " + line + "\n")
        for key, m in mats:
            m = np.asarray(m, dtype=np.float64)
            f.write(f"{key} {m.shape[0]} {m.shape[1]}\n")
            for row in m:
                f.write(" ".join(float(v).hex() for v in row) + "\n")


def main():
    # 1. Integer unit-lower matrix: det = 1, so the exact inverse is integral.
    L = gen.int_unit_lower(10, 4)
    Linv = exact.inverse(exact.to_q(L))
    assert exact.is_integer_matrix(Linv)
    _write("int_unit_lower_n10.txt",
           ["Unit lower-triangular L with strict-lower entries in {-1,0,1}.",
            "Linv = exact inverse by Gauss-Jordan over the rationals (oracle.exact).",
            "Problem statement: Sec. I; block inverse postcondition: Alg. Diagonal-Inverter."],
           [("L", L), ("Linv", exact.to_float(Linv))])
    # 2. A small system of the easy family and its exact solution, rounded
    #    once to binary64 (round-to-nearest of the exact rational).
    L, B = gen.easy_system(6, 3, 0)
    X = exact.solve(L, B)
    _write("easy_n6_k3.txt",
           ["L: diagonal U[1,2], strict lower U[-1,1]/n; B ~ N(0,1); seed 0.",
            "X = exact rational solution of L X = B (Gauss-Jordan on Q), rounded once.",
            "Problem statement: Sec. I."],
           [("L", L), ("B", B), ("X", exact.to_float(X))])
    # 3. Ill-conditioned Cholesky factor of the rank-deficient Gram family.
    L = gen.hard_lower(8, 1)
    B = gen.rhs(8, 2, 1)
    X = exact.solve(L, B)
    _write("hard_n8_k2.txt",
           ["L = chol(G G^T/m + eps I), G 8x4, eps = 1e-12 lambda_max; B ~ N(0,1); seed 1.",
            "X = exact rational solution of L X = B (Gauss-Jordan on Q), rounded once.",
            "Problem statement: Sec. I."],
           [("L", L), ("B", B), ("X", exact.to_float(X))])


if __name__ == "__main__":
    main()
