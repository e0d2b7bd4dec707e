"""Write tests/golden/uneven_batch_seed0_sys<i>.json: the 48 lowest positive-band
eigenvalues of systems of the 16-system uneven batch (seed 0):
  15  a four-atom cubic cell whose spectrum has a 2e-3 Ha gap right above the
      wanted 40 bands;
  13  eight eigenvalues (four Kramers pairs) within 1.2e-3 Ha straddling the
      wanted 32 bands, with the next pair 2.3e-4 Ha above a 40-column block.
Computed only with the FP64 oracle: the dense 4N x 4N operator diagonalised by
LAPACK, eigenvalues above -c^2 in ascending order.

Run from the repository root:  python tests/golden/make_uneven_batch_golden.py [index ...]
(default: 15 13)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import sysgen  # noqa: E402
from oracle import dks  # noqa: E402


def main(index):
    s = sysgen.uneven_batch(seed=0, count=16)[index]
    op = dks.DKSOperator(s)
    t = time.time()
    w = np.linalg.eigvalsh(op.dense())
    pos = w[w > -s.c ** 2][:48]
    out = {"system": f"sysgen.uneven_batch(seed=0, count=16)[{index}]", "N": int(op.N),
           "n_bands": int(s.n_bands), "eigenvalues": [float(v) for v in pos],
           "method": "dense eigh of the FP64 oracle operator (numpy.linalg.eigvalsh)",
           "seconds": round(time.time() - t, 1)}
    path = os.path.join(ROOT, "tests", "golden", f"uneven_batch_seed0_sys{index}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["N"], pos[38:42])


if __name__ == "__main__":
    for i in (sys.argv[1:] or ["15", "13"]):
        main(int(i))
