"""Writes c3_tuxv_oracle_error.txt: the relative Frobenius truncation error
||A - U S V^T||_F / ||A||_F of the oracle's TUXV (Alg. 7, j_max = 1, plus the
SVD of X) at rank k = 256 on the 20000 x 10000 matrix with singular values
0.9^(i/10) (Haar factors, seed 3), b = 64, p = 8.  Calls only the oracle and
the input generator.

    python tests/golden/make_c3_tuxv_error.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1509_06820_amd import inputs  # noqa: E402


def main():
    A, prm = inputs.config_matrix("c3")
    ref = oracle.tuxv(A, prm["k"], prm["b"], prm["p"], seed=prm["seed"])
    e = np.linalg.norm(A - (ref["U"] * ref["s"]) @ ref["VT"]) / np.linalg.norm(A)
    opt = inputs.optimal_truncation_error(inputs.sigma_power(10000, 0.9, 10.0), prm["k"])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_tuxv_oracle_error.txt")
    with open(out, "w") as f:
        f.write("# TUXV (oracle) truncation error, 20000 x 10000, sigma_i = 0.9^(i/10), k = 256, b = 64, p = 8,\n")
        f.write("# seed 3; written by tests/golden/make_c3_tuxv_error.py\n")
        f.write(f"oracle_error: {e:.12e}\n")
        f.write(f"optimal_error: {opt:.12e}\n")
    print(out, e, opt)


if __name__ == "__main__":
    main()
