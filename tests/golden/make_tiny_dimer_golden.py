"""Write tests/golden/tiny_dimer_seeds.json: the 16 lowest positive-band
eigenvalues of the tiny dimer (cubic 10 bohr, Gamma, Ecut 5 Ha, 24^3 grid,
N = 515) for seeds 0, 1 and 2 (the seed draws the potential noise and the
projector couplings).  Computed only with the FP64 oracle: the dense 4N x 4N
operator diagonalised by LAPACK, eigenvalues above the mid-gap -c^2.

Run from the repository root:  python tests/golden/make_tiny_dimer_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import sysgen  # noqa: E402
from oracle import dks, lobpcgf  # noqa: E402


def main():
    out = {"workload": "tiny_dimer: cubic 10 bohr, Gamma, Ecut 5 Ha, 24^3, c=137.036",
           "method": "dense eigh of the FP64 oracle operator, eigenvalues above -c^2",
           "seeds": {}}
    for seed in (0, 1, 2):
        s = sysgen.tiny_dimer(seed)
        op = dks.DKSOperator(s)
        w, _ = lobpcgf.lowest_positive(op.dense(), 16, s.c)
        out["seeds"][str(seed)] = {"N": int(op.N), "eigenvalues": [float(v) for v in w]}
        print(seed, op.N, w[:8])
    path = os.path.join(ROOT, "tests", "golden", "tiny_dimer_seeds.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
