"""Regression of the oracle against its stored fixture (written by
tests/golden/make_golden.py, which calls only the oracle)."""
import os

import numpy as np

import oracle
from paper_1902_10078_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def load_golden():
    d = {"L": {}, "Sig": {}, "Qbar": {}}
    with open(os.path.join(HERE, "golden", "gauss_loss_n12_k3.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            t = line.split()
            if t[0] in d:
                d[t[0]][int(t[1])] = [float(v) for v in t[2:]]
            else:
                d[t[0]] = np.array([float(v) for v in t[1:]])
    for name in ("L", "Sig", "Qbar"):
        d[name] = np.array([d[name][j] for j in range(len(d[name]))])
    return d


def test_oracle_matches_golden():
    g = load_golden()
    n, k = 12, 3
    L0, y = inputs.config0(seed=0, n=n, k=k)
    Q = oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0)
    S = inputs.random_sym_band_dd(n, k, np.random.default_rng(99))
    out = oracle.gauss_loss(Q, k, y, S)
    for name in ("parts", "L", "Sig", "Qbar", "z", "ybar"):
        np.testing.assert_allclose(out[name], g[name], rtol=1e-14, atol=1e-14)
