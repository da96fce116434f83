"""Writes the stored expected values under tests/golden/ by calling only the
oracle (the paper prints no worked numeric example, so every stored value here
is an oracle output on a seeded input, kept as a regression fixture)."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1902_10078_amd import inputs  # noqa: E402


def main():
    n, k = 12, 3
    L0, y = inputs.config0(seed=0, n=n, k=k)
    Q = oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0)
    rng = np.random.default_rng(99)
    S = inputs.random_sym_band_dd(n, k, rng)
    out = oracle.gauss_loss(Q, k, y, S)
    path = os.path.join(HERE, "gauss_loss_n12_k3.txt")
    with open(path, "w") as f:
        f.write("# oracle outputs, config-0 recipe at n=12 k=3 (seed 0), S seed 99\n")
        f.write("# loss = logdet Q - y^T Q^{-1} y + tr(Q^{-1} S)\n")
        f.write("parts " + " ".join(repr(float(v)) for v in out["parts"]) + "\n")
        for name in ("L", "Sig", "Qbar"):
            for j in range(n):
                f.write(name + " " + str(j) + " " + " ".join(repr(float(v)) for v in out[name][j]) + "\n")
        f.write("z " + " ".join(repr(float(v)) for v in out["z"]) + "\n")
        f.write("ybar " + " ".join(repr(float(v)) for v in out["ybar"]) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
