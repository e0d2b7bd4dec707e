"""Pins of the oracle's SCF pieces (Eq. density, the Hartree and LDA parts of
V_hxc, Fermi occupations, Kerker and Anderson mixing) against closed forms,
brute force, finite differences and a case whose self-consistent answer is
known exactly.  CPU only."""
import dataclasses
import math

import numpy as np
import pytest

import sysgen
from oracle import dks, lobpcgf, scf


def _small_dimer(seed=0):
    return sysgen.tiny_dimer(seed, ecut=3.0, grid=(18, 18, 18), n_bands=10)


def test_density_normalisation_brute_force_and_kramers():
    """rho integrates to sum f over the cell; at three grid points it equals
    the direct planewave sum |sum_G c_G exp(i (k+G).r)|^2 / Omega (no FFT);
    Kramers pairs with equal occupations leave no spin density (Gamma)."""
    s = _small_dimer(1)
    op = dks.DKSOperator(s)
    n = 10
    eps, vec = lobpcgf.lowest_positive(op.dense(), n, s.c)
    X = vec.T.reshape(n, 4, op.N)
    f, _ = scf.fermi(eps, 6.0, scf.K_BOLTZMANN * 5000.0)
    rho, m = scf.density(op, X, f)
    omega = scf.cell_volume(s.lattice)
    assert abs(rho.sum() * omega / rho.size - f.sum()) < 1e-11
    assert np.abs(m).max() < 1e-8 * rho.max()
    # brute force at a few points
    pts = [(0, 0, 0), (3, 7, 11), (17, 1, 9)]
    b = dks.reciprocal_lattice(s.lattice)
    for j in pts:
        r = (np.array(j) / np.array(s.grid)) @ s.lattice
        ph = np.exp(1j * (op.q @ r))
        val = 0.0
        for i in range(n):
            psi = X[i] @ ph / math.sqrt(omega)
            val += f[i] * float(np.sum(np.abs(psi) ** 2))
        assert abs(val - rho[j]) < 1e-12 * max(1.0, rho.max())
    del b


def test_spin_density_of_a_single_spinor():
    """One occupied spinor (phi_up, phi_dn, chi_up, chi_dn) = (a, b, 0, 0) u(r):
    m = |u|^2 (2 Re(a* b), 2 Im(a* b), |a|^2 - |b|^2); the small component
    enters with the opposite sign (Eq. density)."""
    s = _small_dimer(0)
    op = dks.DKSOperator(s)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(op.N) + 1j * rng.standard_normal(op.N)
    u /= np.linalg.norm(u)
    a, bb = 0.6, 0.8j
    X = np.zeros((1, 4, op.N), dtype=np.complex128)
    X[0, 0], X[0, 1] = a * u, bb * u
    rho, m = scf.density(op, X, np.array([1.0]))
    want = np.array([2 * (np.conj(a) * bb).real, 2 * (np.conj(a) * bb).imag, abs(a) ** 2 - abs(bb) ** 2])
    for k in range(3):
        assert np.allclose(m[k], want[k] * rho, atol=1e-13)
    Y = np.zeros_like(X)
    Y[0, 2], Y[0, 3] = a * u, bb * u
    rho2, m2 = scf.density(op, Y, np.array([1.0]))
    assert np.allclose(rho2, rho, atol=1e-14) and np.allclose(m2, -m, atol=1e-13)


@pytest.mark.parametrize("lat", ["cubic", "hexagonal"])
def test_hartree_of_a_cosine(lat):
    """rho = cos(G0.r) gives V_H = 4 pi / |G0|^2 cos(G0.r) exactly (Poisson's
    equation); on a hexagonal cell |G0|^2 carries the cross term b1.b2."""
    A = sysgen.cubic(9.0) if lat == "cubic" else sysgen.hexagonal(6.0, 9.0)
    grid = (12, 12, 15)
    b = dks.reciprocal_lattice(A)
    mvec = np.array([1, 2, -1])
    G0 = mvec @ b
    r = sysgen.grid_points(A, grid)
    rho = np.cos(r @ G0).reshape(grid)
    vh = scf.hartree(rho, A)
    assert np.allclose(vh, 4 * math.pi / float(G0 @ G0) * rho, atol=1e-12)
    # a constant density has no Hartree potential (neutralising background)
    assert np.abs(scf.hartree(np.full(grid, 0.3), A)).max() < 1e-14


def test_kerker_factor_on_a_cosine():
    A = sysgen.cubic(8.0)
    grid = (10, 10, 10)
    G0 = np.array([2, 0, 1]) @ dks.reciprocal_lattice(A)
    r = sysgen.grid_points(A, grid)
    x = np.cos(r @ G0).reshape(grid) + 0.25
    g2 = float(G0 @ G0)
    out = scf.kerker(x, A, 0.7)
    assert np.allclose(out, g2 / (g2 + 0.49) * (x - 0.25) + 0.25, atol=1e-13)


def test_lda_exchange_closed_form_and_polarised_ratio():
    """Without correlation the exchange energy per electron is
    -(3/4)(3 rho / pi)^(1/3) (unpolarised) and 2^(1/3) times that when fully
    polarised (Slater)."""
    rho = np.array([1e-3, 0.02, 0.7, 5.0])
    rs = (3 / (4 * np.pi * rho)) ** (1 / 3)
    eps0, _, _ = scf.lda_eps(rho, np.zeros_like(rho))
    ecu, _ = scf._pz_corr(rs, scf._PZ["U"])
    assert np.allclose(eps0 - ecu, -0.75 * (3 * rho / np.pi) ** (1 / 3), rtol=1e-13)
    eps1, _, _ = scf.lda_eps(rho, np.ones_like(rho))
    ecp, _ = scf._pz_corr(rs, scf._PZ["P"])
    assert np.allclose(eps1 - ecp, 2 ** (1 / 3) * (eps0 - ecu), rtol=1e-13)


def test_pz_correlation_is_continuous_at_rs_1():
    """The Perdew-Zunger low- and high-density forms meet at rs = 1 (value to
    the rounding of the published coefficients, slope to 2 %)."""
    for key in ("U", "P"):
        p = scf._PZ[key]
        lo_e = p["B"] + p["D"]
        hi_e = p["g"] / (1 + p["b1"] + p["b2"])
        assert abs(lo_e - hi_e) < 1e-4, key
        lo_d = p["A"] + p["C"] + p["D"]
        hi_d = -p["g"] * (0.5 * p["b1"] + p["b2"]) / (1 + p["b1"] + p["b2"]) ** 2
        assert abs(lo_d - hi_d) < 0.02 * abs(hi_d), key


@pytest.mark.parametrize("rho,zeta", [(0.002, 0.0), (0.03, 0.3), (0.6, -0.5), (4.0, 0.9),
                                      (0.25, 0.0), (1.5, 0.2)])
def test_lda_potentials_are_derivatives_of_the_energy(rho, zeta):
    """v_up and v_dn against central differences of rho eps_xc(rho_up, rho_dn)
    (densities on both sides of rs = 1)."""
    def e_of(ru, rd):
        r = ru + rd
        eps, _, _ = scf.lda_eps(np.array([r]), np.array([(ru - rd) / r]))
        return r * eps[0]
    ru, rd = rho * (1 + zeta) / 2, rho * (1 - zeta) / 2
    _, vu, vd = scf.lda_eps(np.array([rho]), np.array([zeta]))
    h = 1e-6 * rho
    fu = (e_of(ru + h, rd) - e_of(ru - h, rd)) / (2 * h)
    fd = (e_of(ru, rd + h) - e_of(ru, rd - h)) / (2 * h)
    assert abs(vu[0] - fu) < 1e-7 * max(1, abs(fu))
    assert abs(vd[0] - fd) < 1e-7 * max(1, abs(fd))


def test_lda_b_field_follows_the_magnetisation():
    """B_xc = (v_up - v_dn)/2 along m/|m|: parallel to m, zero where m = 0."""
    rho = np.full((2, 2, 2), 0.05)
    m = np.zeros((3, 2, 2, 2))
    m[:, 0, 0, 0] = [0.01, -0.02, 0.005]
    vxc, bxc, _ = scf.lda_xc(rho, m)
    u = m[:, 0, 0, 0] / np.linalg.norm(m[:, 0, 0, 0])
    bb = bxc[:, 0, 0, 0]
    assert np.allclose(np.cross(bb, u), 0, atol=1e-15) and bb @ u < 0   # favours alignment
    assert np.all(bxc[:, 1, 1, 1] == 0)


def test_fermi_occupations():
    eps = np.array([-3.0, -2.0, -2.0, -1.0, -1.0, 0.5, 0.6, 2.0])
    for n_el in (1.0, 3.0, 4.5, 7.0):
        for kT in (1e-3, 0.05, 0.5):
            f, mu = scf.fermi(eps, n_el, kT)
            assert abs(f.sum() - n_el) < 1e-10
            assert np.all(np.diff(f) <= 1e-15) and np.all((f >= 0) & (f <= 1))
    f, _ = scf.fermi(eps, 3.0, 1e-4)   # cold: the three lowest full
    assert np.allclose(f, [1, 1, 1, 0, 0, 0, 0, 0], atol=1e-12)


def test_anderson_solves_a_linear_fixed_point():
    """On x = A x + b with a contraction A, Anderson's combination of the full
    history is a Krylov method: the exact solution after at most dim + 1
    steps (np.linalg.solve as the reference)."""
    rng = np.random.default_rng(0)
    d = 6
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    A = Q @ np.diag(rng.uniform(-0.8, 0.8, d)) @ Q.T
    b = rng.standard_normal(d)
    x_star = np.linalg.solve(np.eye(d) - A, b)
    mix = scf.Anderson(depth=d + 2, alpha=0.5)
    x = np.zeros(d)
    for _ in range(d + 2):
        x = mix.step(x, A @ x + b - x)
    assert np.linalg.norm(x - x_star) < 1e-9 * np.linalg.norm(x_star)


def test_scf_of_the_uniform_gas_is_known_exactly():
    """No ions (V_ext = a constant V0, no projectors): every eigenstate is a
    free Dirac planewave spinor, degenerate shells are occupied equally, so the
    density is uniform rho0 = n_el / Omega, V_H = 0, m = 0 and the
    self-consistent potential is V0 + v_xc(rho0): the eigenvalues are the free
    Dirac levels shifted by v_xc(rho0)."""
    s = sysgen.tiny_dimer(0, ecut=2.0, grid=(12, 12, 12), n_bands=14, with_nonlocal=False)
    v0 = -0.3
    s = dataclasses.replace(s, v_loc=np.full(s.grid, v0))
    n, n_el = 14, 10.0   # the two lowest shells (2 + 12 states) complete
    out = scf.scf(s, n, n_el, temperature=5000.0, tol=1e-11, max_iter=10)
    assert out.converged, out.residuals
    omega = scf.cell_volume(s.lattice)
    rho0 = n_el / omega
    vxc0 = scf.lda_xc(np.full((1, 1, 1), rho0))[0][0, 0, 0]
    assert np.allclose(out.rho, rho0, rtol=1e-10)
    assert np.abs(out.m).max() < 1e-9 * rho0
    assert np.allclose(out.v, v0 + vxc0, atol=1e-10)
    q = dks.planewave_basis(s.lattice, s.kpts[0], s.ecut)[1]
    lev = dks.free_dirac_levels(q, s.c)
    lev = lev[lev > -s.c ** 2][:n]
    assert np.allclose(out.eigvals, lev + v0 + vxc0, atol=1e-9)


def test_scf_of_the_uniform_gas_ksso():
    """The same gas with the two-component operator (model "ksso"): the
    self-consistent eigenvalues are |q|^2 / 2 + V0 + v_xc(rho0), each twice."""
    s = sysgen.tiny_dimer(0, ecut=2.0, grid=(12, 12, 12), n_bands=14, with_nonlocal=False)
    v0 = 0.2
    s = dataclasses.replace(s, v_loc=np.full(s.grid, v0))
    n, n_el = 14, 9.0
    out = scf.scf(s, n, n_el, tol=1e-11, max_iter=10, model="ksso")
    assert out.converged, out.residuals
    rho0 = n_el / scf.cell_volume(s.lattice)
    vxc0 = scf.lda_xc(np.full((1, 1, 1), rho0))[0][0, 0, 0]
    q = dks.planewave_basis(s.lattice, s.kpts[0], s.ecut)[1]
    lev = np.sort(np.repeat(0.5 * np.einsum("ij,ij->i", q, q), 2))[:n]
    assert np.allclose(out.eigvals, lev + v0 + vxc0, atol=1e-10)
    assert np.abs(out.m).max() < 1e-9 * rho0


def test_scf_dimer_fixed_point_is_independent_of_the_mixing():
    """The tiny dimer's SCF reaches the same self-consistent potential and
    eigenvalues with two different mixing settings, and that potential
    reproduces itself (V_out = V_in) to the tolerance."""
    s = _small_dimer(0)
    n, n_el = 10, 6.0
    a = scf.scf(s, n, n_el, tol=1e-9, depth=6, alpha=0.5)
    b = scf.scf(s, n, n_el, tol=1e-9, depth=4, alpha=0.4, q0=1.2, max_iter=100)
    assert a.converged and b.converged, (a.residuals, b.residuals)
    assert np.abs(a.v - b.v).max() < 1e-7 * np.abs(a.v).max()
    assert np.abs(a.eigvals - b.eigvals).max() < 1e-7
    assert abs(a.free_energy - b.free_energy) < 1e-7
    # the Hartree energy is positive and the occupations hold n_el electrons
    assert abs(a.occ.sum() - n_el) < 1e-10
