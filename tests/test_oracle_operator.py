"""Pins of the oracle's discretised DKS operator against closed forms, brute
force and symmetries.  CPU only.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a wrong normalisation) fails at
least one of them.
"""
import math

import numpy as np
import pytest
import scipy.special as sps
from scipy.spatial.transform import Rotation

import sysgen
from oracle import dks, lobpcgf

C = sysgen.C_LIGHT


def make_system(L=8.0, ecut=2.5, grid=(16, 16, 16), v=None, tau=((0.0, 0.0, 0.0),),
                proj=(), c=C, kpt=(0.0, 0.0, 0.0), lattice=None, n_bands=4):
    A = sysgen.cubic(L) if lattice is None else np.asarray(lattice, dtype=float)
    if v is None:
        v = np.zeros(grid)
    return sysgen.System("t", A, np.array([kpt], dtype=float), ecut, tuple(grid), c,
                         np.asarray(v, dtype=float), np.array(tau, dtype=float), list(proj),
                         n_bands)


def group(atom=0, l=0, n_rad=1, r=0.7, dp=None, dm=None, rng=None):
    rng = rng or np.random.default_rng(0)
    if dp is None:
        dp = rng.uniform(-2, 2, (n_rad, n_rad)); dp = dp + dp.T
    if dm is None:
        dm = rng.uniform(-2, 2, (n_rad, n_rad)); dm = dm + dm.T
    return sysgen.ProjGroup(atom, l, n_rad, r, np.atleast_2d(dp), np.atleast_2d(dm))


# ---------------------------------------------------------------------------
# basis
# ---------------------------------------------------------------------------

def test_basis_matches_bruteforce_enumeration():
    """Sphere |k+G|^2/2 <= Ecut against a brute-force scan of a much larger box."""
    for A, k, ecut in [(sysgen.cubic(10.0), (0, 0, 0), 5.0),
                       (sysgen.hexagonal(7.8, 14.0), (0.05, -0.11, 0.02), 6.0)]:
        mil, q = dks.planewave_basis(A, np.array(k, float), ecut)
        b = 2 * math.pi * np.linalg.inv(A).T
        r = np.arange(-15, 16)
        box = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
        qq = box @ b + np.array(k)
        inside = box[0.5 * (qq * qq).sum(1) <= ecut]
        assert sorted(map(tuple, inside)) == sorted(map(tuple, mil))
        assert np.allclose(q, mil @ b + np.array(k))
    # sphere size of the 10 bohr / 5 Ha dimer workload
    mil, _ = dks.planewave_basis(sysgen.cubic(10.0), np.zeros(3), 5.0)
    assert mil.shape[0] == 515


# ---------------------------------------------------------------------------
# free Dirac operator (V = 0): closed form +-sqrt(c^2 q^2 + c^4) - c^2
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("c", [C, 11.7])
def test_free_dirac_closed_form(c):
    s = make_system(L=10.0, ecut=5.0, grid=(24, 24, 24), c=c)
    op = dks.DKSOperator(s)
    w = np.linalg.eigvalsh(op.dense())
    # closed form written from the Miller indices of a cubic cell: q = 2 pi n / L
    q2 = ((2 * math.pi / 10.0) ** 2) * (op.miller ** 2).sum(1)
    e = np.sqrt(c * c * q2 + c ** 4)
    ref = np.sort(np.concatenate([e - c * c, e - c * c, -e - c * c, -e - c * c]))
    assert np.max(np.abs(w - ref)) < 1e-9 * c * c
    if c == C:
        # degeneracy shells of the positive band: 2, 12, 24, 16, 12 (x2 spin of 1, 6, 12, 8, 6 PWs)
        pos = w[w > -c * c]
        levels, counts = [], []
        for x in pos:
            if levels and abs(x - levels[-1]) < 1e-8:
                counts[-1] += 1
            else:
                levels.append(x); counts.append(1)
        assert counts[:5] == [2, 12, 24, 16, 12]
        # first shell |G| = 2 pi / 10: E = c^2 q^2 / (sqrt(c^4 + c^2 q^2) + c^2)
        qa = 2 * math.pi / 10.0
        assert abs(levels[1] - (math.sqrt(c ** 4 + c * c * qa * qa) - c * c)) < 1e-9


def test_free_dirac_helper_matches_dense():
    s = make_system(L=9.0, ecut=3.0, grid=(18, 18, 18), kpt=(0.1, 0.05, -0.2))
    op = dks.DKSOperator(s)
    w = np.linalg.eigvalsh(op.dense())
    assert np.max(np.abs(w - dks.free_dirac_levels(op.q, op.c))) < 1e-8


# ---------------------------------------------------------------------------
# local potential on the grid
# ---------------------------------------------------------------------------

def test_constant_potential_shifts_every_eigenvalue():
    v0 = -3.25
    s0 = make_system(L=8.0, ecut=2.5, grid=(16, 16, 16))
    s1 = make_system(L=8.0, ecut=2.5, grid=(16, 16, 16), v=np.full((16, 16, 16), v0))
    w0 = np.linalg.eigvalsh(dks.DKSOperator(s0).dense())
    w1 = np.linalg.eigvalsh(dks.DKSOperator(s1).dense())
    assert np.max(np.abs(w1 - (w0 + v0))) < 1e-8


def test_single_cosine_couples_only_g_plus_minus_g0():
    """V(r) = 2a cos(G0.r + p) has Vhat(+G0) = a e^{ip}, Vhat(-G0) = a e^{-ip}, zero elsewhere."""
    a, p = 0.37, 0.61
    n0 = np.array([1, 2, 0])
    grid = (12, 12, 12)
    L = 7.0
    A = sysgen.cubic(L)
    r = sysgen.grid_points(A, grid)
    g0 = 2 * math.pi / L * n0
    v = 2 * a * np.cos(r @ g0 + p)
    op = dks.DKSOperator(make_system(L=L, ecut=2.0, grid=grid, v=v))
    vl = op.local_dense()
    d = op.miller[:, None, :] - op.miller[None, :, :]
    plus = np.all(d == n0, axis=-1)
    minus = np.all(d == -n0, axis=-1)
    assert plus.any() and minus.any()
    assert np.allclose(vl[plus], a * np.exp(1j * p), atol=1e-13)
    assert np.allclose(vl[minus], a * np.exp(-1j * p), atol=1e-13)
    assert np.max(np.abs(vl[~(plus | minus)])) < 1e-13


def test_local_matrix_elements_bruteforce_sum():
    """<G|V|G'> against the direct grid sum N_g^-1 sum_j e^{-iG.r_j} V(r_j) e^{iG'.r_j}."""
    rng = np.random.default_rng(3)
    grid = (6, 8, 10)
    A = np.array([[6.0, 0.3, 0.0], [0.0, 7.0, 0.4], [0.2, 0.0, 8.0]])
    v = rng.standard_normal(grid)
    op = dks.DKSOperator(make_system(lattice=A, ecut=1.2, grid=grid, v=v))
    vl = op.local_dense()
    r = sysgen.grid_points(A, grid).reshape(-1, 3)
    G = op.miller @ (2 * math.pi * np.linalg.inv(A).T)
    E = np.exp(1j * (G @ r.T))                     # N x Ng
    brute = (E.conj() * v.reshape(-1)[None, :]) @ E.T / v.size
    assert np.max(np.abs(vl - brute)) < 1e-12


# ---------------------------------------------------------------------------
# angular algebra of the spin-orbit projectors
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_spin_orbit_projectors(l):
    lz, lp, lm = dks.angular_momentum(l)
    lx = 0.5 * (lp + lm)
    ly = -0.5j * (lp - lm)
    assert np.allclose(lx @ ly - ly @ lx, 1j * lz)
    assert np.allclose(lx @ lx + ly @ ly + lz @ lz, l * (l + 1) * np.eye(2 * l + 1))
    ls, pp, pm = dks.spin_orbit(l)
    d = 2 * (2 * l + 1)
    assert np.allclose(pp + pm, np.eye(d))
    assert np.allclose(pp @ pp, pp) and np.allclose(pm @ pm, pm)
    assert np.allclose(pp @ pm, 0)
    assert round(np.trace(pp).real) == 2 * l + 2
    assert round(np.trace(pm).real) == 2 * l
    ev = np.sort(np.linalg.eigvalsh(ls))
    expect = np.sort([-(l + 1) / 2.0] * (2 * l) + [l / 2.0] * (2 * l + 2))
    assert np.allclose(ev, expect)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_solid_harmonics_match_scipy(l):
    rng = np.random.default_rng(l)
    q = rng.standard_normal((50, 3))
    rq = np.linalg.norm(q, axis=1)
    theta = np.arccos(q[:, 2] / rq)
    phi = np.arctan2(q[:, 1], q[:, 0])
    for m in range(-l, l + 1):
        ref = rq ** l * sps.sph_harm_y(l, m, theta, phi)
        assert np.allclose(dks.solid_harmonic(l, m, q), ref, atol=1e-12)


def _kernel(groups, q, qp):
    """2x2 spin kernel sum beta(q) W beta(q')^* of unnormalised projectors at tau = 0."""
    out = np.zeros((2, 2), dtype=complex)
    for g in groups:
        w = dks.coupling_matrix(g)
        b = dks.projector_values(g, q[None, :], np.zeros(3), normalise=False)[0]
        bp = dks.projector_values(g, qp[None, :], np.zeros(3), normalise=False)[0]
        npj = b.size
        for s in range(2):
            for t in range(2):
                rows = [2 * p + s for p in range(npj)]
                cols = [2 * p + t for p in range(npj)]
                out[s, t] += b @ w[np.ix_(rows, cols)] @ bp.conj()
    return out


def test_nonlocal_kernel_is_rotation_covariant():
    """K(Rq, Rq') = U K(q, q') U^+ with U = exp(-i theta n.sigma/2): the spin-orbit
    coupling is a scalar under joint orbital + spin rotation."""
    rng = np.random.default_rng(11)
    groups = [group(0, l, 2, 0.6, rng=rng) for l in range(3)]
    sig = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
           np.array([[1, 0], [0, -1]], complex)]
    for trial in range(5):
        rot = Rotation.random(random_state=trial)
        rv = rot.as_rotvec()
        th = np.linalg.norm(rv)
        n = rv / th
        ns = sum(n[i] * sig[i] for i in range(3))
        U = math.cos(th / 2) * np.eye(2) - 1j * math.sin(th / 2) * ns
        R = rot.as_matrix()
        q, qp = rng.standard_normal(3), rng.standard_normal(3)
        k0 = _kernel(groups, q, qp)
        k1 = _kernel(groups, R @ q, R @ qp)
        assert np.allclose(k1, U @ k0 @ U.conj().T, atol=1e-12)
        assert np.abs(k0).max() > 1e-3


def test_nonlocal_multiplicities_single_atom():
    """One atom at the origin of a cubic cell, l = 1, one radial function: the
    three projectors are orthonormal over the cubic-symmetric sphere, so V_2 has
    eigenvalue D+ four times (j = 3/2), D- twice (j = 1/2) and zero otherwise."""
    dp, dm = 1.7, -0.9
    g = group(0, 1, 1, 0.8, dp=[[dp]], dm=[[dm]])
    op = dks.DKSOperator(make_system(L=8.0, ecut=3.0, grid=(16, 16, 16), proj=[g]))
    w = np.linalg.eigvalsh(op.nonlocal_dense_2c())
    nz = np.sort(w[np.abs(w) > 1e-9])
    assert np.allclose(nz, [dm, dm, dp, dp, dp, dp], atol=1e-10)
    # two radial functions and l = 0..2: rank n_rad * 2(2l+1) summed
    gs = [group(0, l, 2, 0.8, rng=np.random.default_rng(l)) for l in range(3)]
    op = dks.DKSOperator(make_system(L=8.0, ecut=3.0, grid=(16, 16, 16), proj=gs))
    w = np.linalg.eigvalsh(op.nonlocal_dense_2c())
    assert np.count_nonzero(np.abs(w) > 1e-8) == 2 * (2 + 6 + 10)


# ---------------------------------------------------------------------------
# the whole operator
# ---------------------------------------------------------------------------

def _tiny_with_everything(seed=0, c=C, kpt=(0.0, 0.0, 0.0)):
    s = sysgen.tiny_dimer(seed, c=c, ecut=2.5, grid=(16, 16, 16))
    s.kpts = np.array([kpt], dtype=float)
    return s


def test_dense_is_hermitian_and_matrix_free_agrees():
    s = _tiny_with_everything(kpt=(0.07, -0.03, 0.11))
    op = dks.DKSOperator(s)
    H = op.dense()
    assert np.max(np.abs(H - H.conj().T)) < 1e-12
    rng = np.random.default_rng(5)
    X = rng.standard_normal((3, 4, op.N)) + 1j * rng.standard_normal((3, 4, op.N))
    Y = rng.standard_normal((3, 4, op.N)) + 1j * rng.standard_normal((3, 4, op.N))
    HX, HY = op.apply(X), op.apply(Y)
    ref = (H @ X.reshape(3, -1).T).T.reshape(X.shape)
    assert np.max(np.abs(HX - ref)) < 1e-10 * np.abs(ref).max()
    lhs = np.vdot(X.reshape(-1), HY.reshape(-1))
    rhs = np.conj(np.vdot(Y.reshape(-1), HX.reshape(-1)))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_kramers_degeneracy_at_gamma_and_k_minus_k():
    op = dks.DKSOperator(_tiny_with_everything())
    w = np.linalg.eigvalsh(op.dense())
    # eigvalsh is accurate to ~eps ||H|| with ||H|| ~ 2c^2
    assert np.max(np.abs(w[0::2] - w[1::2])) < 1e-12 * C * C
    pos = w[w > -C * C]
    assert np.max(np.abs(pos[0::2] - pos[1::2])) < 1e-9
    k = (0.13, -0.05, 0.21)
    wk = np.linalg.eigvalsh(dks.DKSOperator(_tiny_with_everything(kpt=k)).dense())
    wmk = np.linalg.eigvalsh(dks.DKSOperator(_tiny_with_everything(kpt=tuple(-x for x in k))).dense())
    assert np.max(np.abs(wk - wmk)) < 1e-12 * C * C
    # a k != 0 breaks the pairs (so the check above is not vacuous)
    assert np.max(np.abs(wk[0::2] - wk[1::2])) > 1e-6


def _rotation_unitary(op, perm_fn, U2):
    """4N x 4N operator psi(G) -> U2 psi(R^-1 G) on both two-spinors."""
    N = op.N
    index = {tuple(m): i for i, m in enumerate(op.miller)}
    P = np.zeros((N, N))
    for i, m in enumerate(op.miller):
        P[index[perm_fn(tuple(m))], i] = 1.0
    D = np.kron(np.eye(2), U2)
    return np.kron(D, P)


def test_operator_commutes_with_cubic_rotations():
    """Single atom at the origin of a cubic cell (spherical Gaussian, SOC
    projectors l <= 2): H commutes with C4 rotations about z and x taken jointly on
    the planewave index and on the spin of both two-spinors."""
    L, grid = 8.0, (16, 16, 16)
    A = sysgen.cubic(L)
    v = sysgen.gaussian_potential(A, grid, np.zeros((1, 3)), [-5.0], [0.9])
    rng = np.random.default_rng(2)
    gs = [group(0, l, 2, 0.7, rng=rng) for l in range(3)]
    op = dks.DKSOperator(make_system(L=L, ecut=2.2, grid=grid, v=v, proj=gs))
    H = op.dense()
    s = 1 / math.sqrt(2)
    # C4 about z: (x, y, z) -> (-y, x, z); spin rotation exp(-i pi/4 sigma_z)
    Uz = np.diag([np.exp(-1j * math.pi / 4), np.exp(1j * math.pi / 4)])
    Mz = _rotation_unitary(op, lambda m: (-m[1], m[0], m[2]), Uz)
    # C4 about x: (x, y, z) -> (x, -z, y); spin rotation exp(-i pi/4 sigma_x)
    Ux = s * np.array([[1, -1j], [-1j, 1]])
    Mx = _rotation_unitary(op, lambda m: (m[0], -m[2], m[1]), Ux)
    for M in (Mz, Mx):
        assert np.max(np.abs(M @ H @ M.conj().T - H)) < 1e-9
    # the wrong spin sense must fail (the check is sensitive to sigma conventions)
    Mbad = _rotation_unitary(op, lambda m: (-m[1], m[0], m[2]), Uz.conj())
    assert np.max(np.abs(Mbad @ H @ Mbad.conj().T - H)) > 1e-3


def test_translation_invariance_of_spectrum():
    """Moving every atom and the sampled potential by one grid vector leaves the
    spectrum unchanged (pins the structure-factor sign against V_loc placement)."""
    s = _tiny_with_everything()
    w0 = np.linalg.eigvalsh(dks.DKSOperator(s).dense())
    shift = np.array([3, -2, 5])
    s.v_loc = np.roll(s.v_loc, shift, axis=(0, 1, 2))
    s.tau = s.tau + (shift / np.array(s.grid)) @ s.lattice
    w1 = np.linalg.eigvalsh(dks.DKSOperator(s).dense())
    assert np.max(np.abs(w1 - w0)) < 1e-8


def test_nonrelativistic_limit():
    """As c grows, the positive-band DKS eigenvalues approach those of
    |q|^2/2 + V_loc + V_2 with an error that falls as 1/c^2."""
    errs = []
    for c in (1e3, 1e4):
        s = _tiny_with_everything(c=c)
        op = dks.DKSOperator(s)
        lam, _ = lobpcgf.lowest_positive(op.dense(), 8, c)
        ref = np.linalg.eigvalsh(op.pauli_dense())[:8]
        errs.append(np.max(np.abs(lam - ref)))
    assert errs[1] < 1e-5
    assert 50.0 < errs[0] / errs[1] < 200.0


def test_spectrum_bounds_enclose_the_bands():
    s = _tiny_with_everything()
    op = dks.DKSOperator(s)
    w = np.linalg.eigvalsh(op.dense())
    ekin, vmin, vmax, vmean, nl = op.spectrum_bounds()
    C_, Om = lobpcgf.filter_constants(op.spectrum_bounds(), s.c)
    pos = w[w > -s.c ** 2]
    neg = w[w <= -s.c ** 2]
    assert pos.max() <= C_ + Om + 1e-9
    assert neg.min() < C_ < neg.max() or abs(C_ - 0.5 * (neg.min() + neg.max())) < 50


def test_ksso_apply_matches_its_dense_form():
    """The two-component KSSO operator (Table 1), matrix-free, equals its dense
    form |q|^2/2 + V_loc + V_2 (pauli_dense, itself pinned by the
    nonrelativistic limit of the DKS operator) on random blocks, and is
    Hermitian."""
    s = _tiny_with_everything(c=sysgen.C_LIGHT)
    op = dks.DKSOperator(s)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((3, 2, op.N)) + 1j * rng.standard_normal((3, 2, op.N))
    H2 = op.pauli_dense()
    ref = (H2 @ X.reshape(3, -1).T).T.reshape(3, 2, op.N)
    got = op.apply_ksso(X)
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))
    assert np.max(np.abs(H2 - H2.conj().T)) < 1e-12
