"""Pins of the oracle's filter and Algorithm 1 (LOBPCG-F) against the dense
definition of the answer, spectral identities and the paper's claims.  CPU only.
"""
import math

import numpy as np
import pytest

import sysgen
from oracle import dks, lobpcgf

C = sysgen.C_LIGHT


@pytest.fixture(scope="module")
def tiny():
    s = sysgen.tiny_dimer(0)
    op = dks.DKSOperator(s)
    H = op.dense()
    w, v = np.linalg.eigh(H)
    return s, op, H, w, v


def _clusters(lam, tol=1e-6):
    out, start = [], 0
    for i in range(1, len(lam) + 1):
        if i == len(lam) or lam[i] - lam[i - 1] > tol:
            out.append((start, i))
            start = i
    return out


def test_filter_acts_spectrally(tiny):
    """f(H) v_i = (eps_i - C)^2 / Omega^2 v_i on exact eigenvectors (Eq. filter)."""
    s, op, H, w, v = tiny
    C_, Om = lobpcgf.filter_constants(op.spectrum_bounds(), s.c)
    idx = [0, 5, len(w) // 2 - 1, len(w) // 2, len(w) // 2 + 7, len(w) - 1]
    V = v[:, idx]
    FV = lobpcgf.apply_filter(lobpcgf.block_apply(op), V, C_, Om)
    f = (w[idx] - C_) ** 2 / Om ** 2
    assert np.max(np.abs(FV - V * f[None, :])) < 1e-9
    pos = w[w > -s.c ** 2]
    fpos = (pos - C_) ** 2 / Om ** 2
    assert fpos.max() <= 1.0 + 1e-12 and fpos.max() > 0.99


@pytest.mark.parametrize("c", [12.25, 38.73, C])
def test_filter_damping_factor(c):
    """Sec. 3.1: gamma_LOBPCG ~ Delta/w, gamma_F ~ w/Delta.  With the dense
    spectrum, the amplification of the negative-band error relative to the
    positive-band error is computed for the lowest Ritz value and compared with
    w/Delta; the filtered factor must be below 1 and shrink as c grows."""
    s = sysgen.tiny_dimer(0, c=c, ecut=2.5, grid=(16, 16, 16))
    op = dks.DKSOperator(s)
    w = np.linalg.eigvalsh(op.dense())
    pos, neg = w[w > -c * c], w[w <= -c * c]
    lam = pos[0]
    width = max(pos.max() - pos.min(), neg.max() - neg.min())
    delta = pos.min() - neg.max()
    C_, Om = lobpcgf.filter_constants(op.spectrum_bounds(), c)
    f = lambda e: (e - C_) ** 2 / Om ** 2
    g_plain = np.max(np.abs(neg - lam)) / np.max(np.abs(pos - lam))
    g_filt = np.max(np.abs(f(neg) * (neg - lam))) / np.max(np.abs(f(pos) * (pos - lam)))
    assert g_plain > 0.5 * delta / width
    assert g_filt < 4.0 * width / delta
    assert g_filt < 1.0


def test_lobpcgf_matches_dense_definition(tiny):
    """Algorithm 1 returns the 8 lowest positive-band eigenpairs of the dense
    matrix: eigenvalues to 1e-8 Ha, spectral projectors of each cluster."""
    s, op, H, w, v = tiny
    lam_ref, vec_ref = lobpcgf.lowest_positive(H, 8, s.c)
    phi = sysgen.start_block(op.miller, s.lattice, s.kpts[0], 8, 0)
    r = lobpcgf.solve(op, 8, phi0=phi, tol=1e-9, n_iter=200)
    assert r.converged
    assert np.max(np.abs(r.eigvals - lam_ref)) < 1e-8
    # |lambda - exact| <= ||r|| (Hermitian residual bound)
    assert np.all(np.abs(r.eigvals - lam_ref) <= r.resnorms + 1e-12)
    X = r.X / np.linalg.norm(r.X, axis=0)
    for a, b in _clusters(lam_ref):
        Pr = vec_ref[:, a:b] @ vec_ref[:, a:b].conj().T
        Q, _ = np.linalg.qr(X[:, a:b])
        Pl = Q @ Q.conj().T
        assert np.linalg.norm(Pr - Pl) < 1e-6
    # never a Ritz value in or below the gap
    assert min(r.min_ritz_history) > -s.c ** 2
    # the small component stays small: ||chi|| / ||phi|| <= q_max / (2c) per band
    N = op.N
    qmax = math.sqrt(np.max(np.einsum("ij,ij->i", op.q, op.q)))
    for j in range(8):
        phi_n = np.linalg.norm(X[:2 * N, j])
        chi_n = np.linalg.norm(X[2 * N:, j])
        assert chi_n / phi_n <= qmax / (2 * s.c)


def test_lobpcgf_at_k_point_with_ragged_block():
    """A k != 0 system with a block size that does not divide the pairs (n = 5).

    The tolerance is the 1e-8 Ha target: with ||H|| ~ 4e4 the FP64 residual floor
    of the implicit HX/HP products is ~1e-10, and a tolerance at that floor makes
    the last active column stagnate on rounding noise."""
    s = sysgen.tiny_dimer(2, ecut=3.0, grid=(18, 18, 18))
    s.kpts = np.array([[0.11, -0.07, 0.05]])
    op = dks.DKSOperator(s)
    lam_ref, _ = lobpcgf.lowest_positive(op.dense(), 5, s.c)
    phi = sysgen.start_block(op.miller, s.lattice, s.kpts[0], 5, 3)
    r = lobpcgf.solve(op, 5, phi0=phi, tol=1e-8, n_iter=300)
    assert r.converged
    assert np.max(np.abs(r.eigvals - lam_ref)) < 1e-8
    assert min(r.min_ritz_history) > -s.c ** 2


def test_standard_lobpcg_collapses_without_the_filter(tiny):
    """Sec. 3.1: without F the negative-band error grows by ~Delta/w per
    iteration and LOBPCG falls into the negative band (variational collapse);
    LOBPCG-F from the same start never does."""
    s, op, H, w, v = tiny
    phi = sysgen.start_block(op.miller, s.lattice, s.kpts[0], 8, 0)
    X0 = lobpcgf.kinetic_balance(op, phi)
    # contaminate with 1e-15 of the lowest negative-band eigenvector
    X0 = X0.reshape(8, -1).T
    X0 = X0 / np.linalg.norm(X0, axis=0)
    X0 = X0 + 1e-15 * v[:, [0]]
    C_, Om = lobpcgf.filter_constants(op.spectrum_bounds(), s.c)
    plain = lobpcgf.lobpcgf(lobpcgf.block_apply(op), X0, 8, C_, Om, n_iter=12, tol=1e-9,
                            use_filter=False)
    assert min(plain.min_ritz_history) < -s.c ** 2
    filt = lobpcgf.lobpcgf(lobpcgf.block_apply(op), X0, 8, C_, Om, n_iter=12, tol=1e-9,
                           use_filter=True)
    assert min(filt.min_ritz_history) > -s.c ** 2


def test_kinetic_balance_gives_free_eigenvectors():
    """With V = 0 the kinetic-balance spinor of a single planewave is an exact
    positive-energy eigenvector with E = sqrt(c^2 q^2 + c^4) - c^2."""
    s = sysgen.tiny_dimer(0, noise=0.0, with_nonlocal=False, ecut=2.0, grid=(12, 12, 12))
    s.v_loc = np.zeros_like(s.v_loc)
    op = dks.DKSOperator(s)
    rng = np.random.default_rng(0)
    phi = np.zeros((3, 2, op.N), dtype=complex)
    picks = [0, 4, op.N - 1]
    for b, g in enumerate(picks):
        phi[b, :, g] = rng.standard_normal(2) + 1j * rng.standard_normal(2)
    X = lobpcgf.kinetic_balance(op, phi)
    HX = op.apply(X)
    for b, g in enumerate(picks):
        q2 = float(op.q[g] @ op.q[g])
        E = math.sqrt(s.c ** 2 * q2 + s.c ** 4) - s.c ** 2
        assert np.max(np.abs(HX[b] - E * X[b])) < 1e-9


@pytest.mark.parametrize("max_dim", [16, 32])
def test_davidson_f_matches_dense_definition(tiny, max_dim):
    """The filter inside a block Davidson iteration (Sec. 3 opening, Sec. 5)
    reaches the same answer as Algorithm 1: the 8 lowest positive-band
    eigenvalues of the dense matrix to 1e-8 Ha, within each residual norm, and
    no Ritz value in or below the gap.  max_dim = 16 restarts the space every
    step or two, 32 lets it grow to four blocks."""
    s, op, H, w, v = tiny
    lam_ref, _ = lobpcgf.lowest_positive(H, 8, s.c)
    phi = sysgen.start_block(op.miller, s.lattice, s.kpts[0], 8, 0)
    r = lobpcgf.solve(op, 8, phi0=phi, tol=1e-9, n_iter=200, method="davidson", max_dim=max_dim)
    assert r.converged
    assert np.max(np.abs(r.eigvals - lam_ref)) < 1e-8
    # |lambda - exact| <= ||r||, up to the dense solver's backward error eps ||H||
    slack = 16 * np.finfo(float).eps * np.linalg.norm(H, 2)
    assert np.all(np.abs(r.eigvals - lam_ref) <= r.resnorms + slack)
    assert min(r.min_ritz_history) > -s.c ** 2


def test_davidson_collapses_without_the_filter(tiny):
    """Without F the Davidson space, like LOBPCG's, takes in the negative band
    from a start block contaminated at 1e-15 (Sec. 3.1's argument holds for any
    solver whose new directions are the residuals); with F it never does."""
    s, op, H, w, v = tiny
    phi = sysgen.start_block(op.miller, s.lattice, s.kpts[0], 8, 0)
    X0 = lobpcgf.kinetic_balance(op, phi).reshape(8, -1).T
    X0 = X0 / np.linalg.norm(X0, axis=0) + 1e-15 * v[:, [0]]
    C_, Om = lobpcgf.filter_constants(op.spectrum_bounds(), s.c)
    plain = lobpcgf.davidson_f(lobpcgf.block_apply(op), X0, 8, C_, Om, n_iter=12, tol=1e-9,
                               use_filter=False)
    assert min(plain.min_ritz_history) < -s.c ** 2
    filt = lobpcgf.davidson_f(lobpcgf.block_apply(op), X0, 8, C_, Om, n_iter=12, tol=1e-9,
                              use_filter=True)
    assert min(filt.min_ritz_history) > -s.c ** 2


@pytest.mark.parametrize("c", [137.036, 3.0])
def test_dirac_teter_scales_every_free_eigenvector(c):
    """The preconditioner's spectral form: every eigenvector of the free Dirac
    block (LAPACK on the oracle's dense kinetic operator, positive and
    negative band, small cell) is scaled by the Teter factor of its |energy|
    over E.  At c = 3 the small components are a third of the large ones, so a
    wrong projector, sign or component order fails."""
    import dataclasses
    s = dataclasses.replace(sysgen.tiny_dimer(0), ecut=2.0, c=c)
    op = dks.DKSOperator(s)
    w, V = np.linalg.eigh(op.kinetic_dense())
    E = 0.7
    got = lobpcgf.dirac_teter(V, op.q, c, E=np.full(V.shape[1], E))
    want = V * lobpcgf.teter_factor(np.abs(w) / E)[None, :]
    # LAPACK's eigenvectors carry ~eps ||H|| / (shell gap) ~ 2e-10 of rounding
    assert np.abs(got - want).max() < 1e-9


def test_dirac_teter_is_hermitian_positive_and_teter_in_the_nonrelativistic_limit():
    """T at fixed E is Hermitian positive definite; for c -> infinity a
    large-component residual gets the scalar Teter factor of |k+G|^2 / 2E; the
    per-column energy of a single free positive state is its own energy, so T
    scales it by the Teter factor at x = 1 (65/81); the two-component form is
    the plain factor."""
    import dataclasses
    s = dataclasses.replace(sysgen.tiny_dimer(0), ecut=2.0)
    op = dks.DKSOperator(s)
    N, c = op.N, s.c
    rng = np.random.default_rng(5)
    R = rng.standard_normal((4 * N, 3)) + 1j * rng.standard_normal((4 * N, 3))
    E = np.array([0.4, 1.3, 2.0])
    TR = lobpcgf.dirac_teter(R, op.q, c, E=E)
    M = np.stack([lobpcgf.dirac_teter(np.eye(4 * N)[:, j:j + 1], op.q, c, E=E[:1]).ravel()
                  for j in range(4 * N)], axis=1)
    assert np.abs(M - M.conj().T).max() < 1e-14
    assert np.linalg.eigvalsh(0.5 * (M + M.conj().T)).min() > 0
    assert np.abs(TR[:, 0] - M @ R[:, 0]).max() < 1e-12
    # nonrelativistic limit on the large component
    phi = np.zeros((4 * N, 1), dtype=complex)
    phi[:2 * N, 0] = R[:2 * N, 0]
    out = lobpcgf.dirac_teter(phi, op.q, 1e5, E=np.array([0.9]))
    q2 = np.einsum("ij,ij->i", op.q, op.q)
    k = lobpcgf.teter_factor(0.5 * q2 / 0.9)
    want = (R[:2 * N, 0].reshape(2, N) * k[None, :]).ravel()
    assert np.abs(out[:2 * N, 0] - want).max() < 1e-8 * np.abs(want).max()
    # one free positive state of one planewave (LAPACK on its 4 x 4 block of
    # the dense kinetic operator): E is its energy, T scales it by 65/81
    g = int(np.argmax(q2))
    sel = np.arange(4) * N + g
    w4, V4 = np.linalg.eigh(op.kinetic_dense()[np.ix_(sel, sel)])
    v = np.zeros((4 * N, 1), dtype=complex)
    v[sel, 0] = V4[:, 3]   # the upper (positive) pair
    assert w4[3] > 0
    assert np.abs(lobpcgf.dirac_teter(v, op.q, c) - v * 65.0 / 81.0).max() < 1e-12
    # two components: the scalar factor of |k+G|^2 / 2
    R2 = R[:2 * N, :1]
    out2 = lobpcgf.dirac_teter(R2, op.q, c, ncomp=2, E=np.array([0.9]))
    assert np.abs(out2[:, 0] - (R2[:, 0].reshape(2, N) * k[None, :]).ravel()).max() < 1e-14
