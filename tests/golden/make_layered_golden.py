"""Write tests/golden/layered_crystal_seed0_k0.json: the 40 lowest positive-band
eigenvalues of k-point 0 of the layered crystal (hexagonal a = 7.8, c = 54 bohr,
five atoms in quintuple-layer stacking, Ecut 25 Ha, 48 x 48 x 320 grid, seed 0;
k-point 0 of the shifted 4 x 4 x 1 Monkhorst-Pack grid, N ~ 17.0k planewaves).

Computed only with the FP64 oracle: the matrix-free Algorithm 1 of
oracle/lobpcgf.py with 16 buffer columns (a 56-column block of which the first
40 must converge), from two independent start blocks that must agree.  4N is
about 68 000, out of reach of a dense diagonalisation, so that the 40 values
are the lowest ones is backed by the two starts, not by a dense solve.  (The
full 120-band block of the library is compared on these 40; the oracle's
numpy FFTs make 120 bands a matter of many hours.)

Run from the repository root:  python tests/golden/make_layered_golden.py
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

N_WANT = 40
N_BUFFER = 16


def main():
    s = sysgen.layered_crystal(0)
    op = dks.DKSOperator(s, 0)
    n = N_WANT + N_BUFFER
    runs = []
    for seed in (0, 1):
        phi = sysgen.start_block(op.miller, s.lattice, s.kpts[0], n, 500 + seed)
        t = time.time()
        r = lobpcgf.solve(op, n, phi0=phi, tol=1e-8, n_iter=400, n_want=N_WANT)
        print(f"seed {seed}: {r.iterations} iterations, converged={r.converged}, "
              f"max|r| (wanted)={r.resnorms[:N_WANT].max():.2e}, {time.time() - t:.0f}s",
              flush=True)
        runs.append(r)
    lam0, lam1 = runs[0].eigvals[:N_WANT], runs[1].eigvals[:N_WANT]
    assert runs[0].converged and runs[1].converged
    assert np.max(np.abs(lam0 - lam1)) < 1e-8, np.max(np.abs(lam0 - lam1))
    out = {
        "workload": "layered_crystal seed 0, k-point 0: hexagonal a=7.8 c=54 bohr, 5 atoms, "
                    "Ecut 25 Ha, 48x48x320, c=137.036",
        "kpoint": [float(v) for v in s.kpts[0]],
        "source": "oracle/lobpcgf.py Algorithm 1 (FP64, matrix-free), two start blocks",
        "npw": int(op.N),
        "n_bands": N_WANT,
        "buffer_columns": N_BUFFER,
        "eigenvalues": [float(x) for x in lam0],
        "residual_norms": [float(x) for x in runs[0].resnorms[:N_WANT]],
        "max_seed_disagreement": float(np.max(np.abs(lam0 - lam1))),
        "min_ritz_seen": float(min(min(r.min_ritz_history) for r in runs)),
    }
    path = os.path.join(ROOT, "tests", "golden", "layered_crystal_seed0_k0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
