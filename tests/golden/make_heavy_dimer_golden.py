"""Write tests/golden/heavy_dimer_seed0.json: the 40 lowest positive-band
eigenvalues of the heavy-dimer workload (cubic 20 bohr, Ecut 30 Ha, 96^3 grid,
seed 0), computed only with the FP64 oracle (matrix-free Algorithm 1 from two
independent start blocks, which must agree).

Run from the repository root:  python tests/golden/make_heavy_dimer_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import sysgen  # noqa: E402
from oracle import dks, lobpcgf  # noqa: E402


def main():
    s = sysgen.heavy_dimer(0)
    op = dks.DKSOperator(s)
    n = s.n_bands
    runs = []
    for seed in (0, 1):
        phi = sysgen.start_block(op.miller, s.lattice, s.kpts[0], n, seed)
        t = time.time()
        r = lobpcgf.solve(op, n, phi0=phi, tol=1e-8, n_iter=400)
        print(f"seed {seed}: {r.iterations} iterations, converged={r.converged}, "
              f"max|r|={r.resnorms.max():.2e}, {time.time() - t:.0f}s", flush=True)
        runs.append(r)
    lam0, lam1 = runs[0].eigvals, runs[1].eigvals
    assert runs[0].converged and runs[1].converged
    assert np.max(np.abs(lam0 - lam1)) < 1e-8, np.max(np.abs(lam0 - lam1))
    out = {
        "workload": "heavy_dimer seed 0: cubic 20 bohr, Gamma, Ecut 30 Ha, 96^3, c=137.036, 40 bands",
        "source": "oracle/lobpcgf.py Algorithm 1 (FP64, matrix-free), two start blocks",
        "npw": int(op.N),
        "eigenvalues": [float(x) for x in lam0],
        "residual_norms": [float(x) for x in runs[0].resnorms],
        "max_seed_disagreement": float(np.max(np.abs(lam0 - lam1))),
        "min_ritz_seen": float(min(min(r.min_ritz_history) for r in runs)),
    }
    path = os.path.join(ROOT, "tests", "golden", "heavy_dimer_seed0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
