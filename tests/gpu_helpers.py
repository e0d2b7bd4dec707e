"""Shared helpers of the GPU parity tests (no arithmetic of the method here)."""
import numpy as np


def perm_to_oracle(lib_miller, orc_miller):
    """Index array p with lib order g -> oracle index p[g] (same planewave)."""
    pos = {tuple(int(v) for v in m): i for i, m in enumerate(orc_miller)}
    return np.array([pos[tuple(int(v) for v in m)] for m in lib_miller], dtype=np.int64)


def to_lib(X_orc, p):
    """(n, 4, N) block in oracle order -> library order."""
    return np.ascontiguousarray(X_orc[..., p])


def to_orc(X_lib, p):
    out = np.empty_like(X_lib)
    out[..., p] = X_lib
    return out


def random_block(rng, n, N, dtype=np.complex128):
    x = rng.standard_normal((n, 4, N)) + 1j * rng.standard_normal((n, 4, N))
    return x.astype(dtype)


def cluster_projectors_match(lam_ref, V_ref, V_test, tol=1e-6, gap=1e-6):
    """Spectral projectors of every complete cluster of lam_ref agree."""
    n = len(lam_ref)
    start = 0
    worst = 0.0
    for i in range(1, n + 1):
        if i == n or lam_ref[i] - lam_ref[i - 1] > gap:
            a, b = start, i
            Pr = V_ref[:, a:b] @ V_ref[:, a:b].conj().T
            Q, _ = np.linalg.qr(V_test[:, a:b])
            Pl = Q @ Q.conj().T
            worst = max(worst, float(np.linalg.norm(Pr - Pl)))
            start = i
    return worst
