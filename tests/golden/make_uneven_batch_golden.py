"""Write the dense-oracle spectra of the uneven batch (seed 0).

* ``uneven_batch_seed0_sys<i>.json`` for the systems named on the command line
  (default 15 13 27), the historical per-system files:
    15  a four-atom cubic cell whose spectrum has a 2e-3 Ha gap right above the
        wanted 40 bands;
    13  eight eigenvalues (four Kramers pairs) within 1.2e-3 Ha straddling the
        wanted 32 bands, with the next pair 2.3e-4 Ha above a 40-column block;
    27  N = 1743, 24 wanted bands whose last pair lies 1.1e-3 Ha below the
        next state inside a 16-state cluster.
* ``uneven_batch_seed0_dense.json`` (``--all``): every system of the 64-system
  batch whose basis has N <= 2500 planewaves (4N <= 10000, a dense
  diagonalisation of minutes), keyed by system index.

Each entry holds the lowest max(48, n_bands + 24) eigenvalues above the
mid-gap -c^2, ascending.  Computed only with the FP64 oracle: the dense
4N x 4N operator diagonalised by LAPACK (numpy.linalg.eigvalsh).

Run from the repository root:
    python tests/golden/make_uneven_batch_golden.py [index ...]
    python tests/golden/make_uneven_batch_golden.py --all
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

NPW_DENSE_MAX = 2500


def spectrum(s):
    op = dks.DKSOperator(s)
    t = time.time()
    w = np.linalg.eigvalsh(op.dense())
    keep = max(48, s.n_bands + 24)
    pos = w[w > -s.c ** 2][:keep]
    return op.N, pos, time.time() - t


def write_one(systems, index):
    s = systems[index]
    N, pos, dt = spectrum(s)
    out = {"system": f"sysgen.uneven_batch(seed=0, count=64)[{index}]", "N": int(N),
           "n_bands": int(s.n_bands), "eigenvalues": [float(v) for v in pos],
           "method": "dense eigh of the FP64 oracle operator (numpy.linalg.eigvalsh)",
           "seconds": round(dt, 1)}
    path = os.path.join(ROOT, "tests", "golden", f"uneven_batch_seed0_sys{index}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    nb = s.n_bands
    print(path, N, pos[nb - 2:nb + 2], flush=True)


def write_all(systems):
    path = os.path.join(ROOT, "tests", "golden", "uneven_batch_seed0_dense.json")
    out = {"source": "sysgen.uneven_batch(seed=0, count=64)",
           "method": "dense eigh of the FP64 oracle operator (numpy.linalg.eigvalsh); "
                     f"systems with N <= {NPW_DENSE_MAX}",
           "systems": {}}
    if os.path.exists(path):
        out = json.load(open(path))
    for i, s in enumerate(systems):
        if str(i) in out["systems"]:
            continue
        N = int(dks.planewave_basis(s.lattice, s.kpts[0], s.ecut)[0].shape[0])
        if N > NPW_DENSE_MAX:
            continue
        N, pos, dt = spectrum(s)
        out["systems"][str(i)] = {"N": int(N), "n_bands": int(s.n_bands),
                                  "eigenvalues": [float(v) for v in pos],
                                  "seconds": round(dt, 1)}
        with open(path, "w") as f:   # written after every system: the run is long
            json.dump(out, f, indent=1)
        print(f"system {i}: N={N} n={s.n_bands} {dt:.0f}s", flush=True)
    print("wrote", path)


if __name__ == "__main__":
    systems = sysgen.uneven_batch(seed=0, count=64)
    args = sys.argv[1:]
    if args == ["--all"]:
        write_all(systems)
    else:
        for i in (args or ["15", "13", "27"]):
            write_one(systems, int(i))
