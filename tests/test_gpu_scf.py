"""The self-consistent field pieces (dks_density, dks_hartree, dks_kerker,
dks_lda_xc, dks_set/get_local_potential) and the loop (dks_scf) on the GPU
against the FP64 oracle of oracle/scf.py on the same inputs.

Tolerances: the fields are FP64 FFT results, compared element by element
within 1e-12 of their largest value (rounding of O(log N_g) eps on values of
order one); the LDA within 1e-12 relative plus 1e-13 of the field's largest
value (pointwise formulas; B_xc is a difference of nearly equal potentials at
small polarisation); the SCF fixed
points within 1e-6 of the potential's scale and 1e-7 Ha for eigenvalues and
the free energy (both loops stop at a residual of 1e-9 and reach the fixed
point from different iterates)."""
import dataclasses
import math

import numpy as np
import pytest

import sysgen
from oracle import dks, lobpcgf, scf
from tests.gpu_helpers import perm_to_oracle, random_block, to_lib, to_orc
from tests.test_gpu_parity import _dk, _hexagonal_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _small_dimer(seed=0):
    return sysgen.tiny_dimer(seed, ecut=3.0, grid=(18, 18, 18), n_bands=10)


def _dense_states(s, n):
    op = dks.DKSOperator(s)
    eps, vec = lobpcgf.lowest_positive(op.dense(), n, s.c)
    return op, eps, vec.T.reshape(n, 4, op.N)


@pytest.mark.parametrize("which", ["dimer", "hexagonal"])
def test_density_matches_oracle(dev, which):
    """rho and m of the same occupied spinors: the dense eigenvectors of the
    small dimer (Kramers pairs) and a random block on the hexagonal k-point
    cell (a nonzero spin density)."""
    dk = _dk()
    if which == "dimer":
        s = _small_dimer(2)
        op, eps, Xo = _dense_states(s, 10)
        occ, _ = scf.fermi(eps, 6.0, scf.K_BOLTZMANN * 5000.0)
    else:
        s = _hexagonal_system()
        op = dks.DKSOperator(s)
        Xo = random_block(np.random.default_rng(3), 5, op.N)
        Xo /= np.linalg.norm(Xo.reshape(5, -1), axis=1)[:, None, None]
        occ = np.array([1.0, 0.7, 0.0, 0.4, 1.0])
    rho_ref, m_ref = scf.density(op, Xo, occ)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    Xd = torch.from_numpy(to_lib(Xo, p)).to(dev)
    print(f"[density] {which} grid={s.grid}", flush=True)
    rho, m = dk.density(b, 0, Xd, occ)
    torch.cuda.synchronize()
    b.close()
    rho, m = rho.cpu().numpy(), m.cpu().numpy()
    scale = np.abs(rho_ref).max()
    assert np.abs(rho - rho_ref).max() < 1e-12 * scale
    assert np.abs(m - m_ref).max() < 1e-12 * scale


def test_density_ksso_components(dev):
    """Two-component blocks (model KSSO): rho and m = phi^+ sigma phi equal the
    four-component densities of the same spinors with zero small components."""
    dk = _dk()
    s = _small_dimer(0)
    op = dks.DKSOperator(s)
    X2 = random_block(np.random.default_rng(4), 3, op.N)[:, :2]
    X2 /= np.linalg.norm(X2.reshape(3, -1), axis=1)[:, None, None]
    X4 = np.zeros((3, 4, op.N), dtype=np.complex128)
    X4[:, :2] = X2
    occ = np.array([1.0, 0.5, 0.25])
    rho_ref, m_ref = scf.density(op, X4, occ)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    Xd = torch.from_numpy(np.ascontiguousarray(X2[..., p])).to(dev)
    rho, m = dk.density(b, 0, Xd, occ, model=dk.MODEL_KSSO)
    torch.cuda.synchronize()
    b.close()
    scale = np.abs(rho_ref).max()
    assert np.abs(rho.cpu().numpy() - rho_ref).max() < 1e-12 * scale
    assert np.abs(m.cpu().numpy() - m_ref).max() < 1e-12 * scale


def test_density_heavy_dimer_sampled(dev):
    """The 40 bands of the 96^3 heavy dimer: rho integrates to sum f and equals
    the direct planewave sum at sampled grid points (no FFT on the oracle side)."""
    dk = _dk()
    s = sysgen.heavy_dimer(0)
    b = dk.init_basis([s])
    N, grid, mil = dk.basis_info(b, 0)
    nb = 40
    X = random_block(np.random.default_rng(11), nb, N)
    X /= np.linalg.norm(X.reshape(nb, -1), axis=1)[:, None, None]
    occ = np.linspace(1.0, 0.0, nb)
    print("[density heavy dimer] 40 bands", flush=True)
    rho, _ = dk.density(b, 0, torch.from_numpy(X).to(dev), occ, with_mag=False)
    torch.cuda.synchronize()
    b.close()
    rho = rho.cpu().numpy()
    omega = scf.cell_volume(s.lattice)
    assert abs(rho.sum() * omega / rho.size - occ.sum()) < 1e-11 * occ.sum()
    B = dks.reciprocal_lattice(s.lattice)
    G = mil @ B
    for j in [(0, 0, 0), (48, 48, 48), (5, 77, 31)]:
        r = (np.array(j) / np.array(grid)) @ s.lattice
        ph = np.exp(1j * (G @ r))
        psi = np.einsum("bcg,g->bc", X, ph) / math.sqrt(omega)
        want = float(np.sum(occ[:, None] * np.abs(psi) ** 2))
        assert abs(rho[j] - want) < 1e-11 * np.abs(rho).max(), j


@pytest.mark.parametrize("which", ["cubic", "hexagonal", "unsplit"])
def test_hartree_and_kerker_match_oracle(dev, which):
    """A random density on a cubic grid, the hexagonal cell (non-orthogonal
    reciprocal vectors) and a grid with an 81-point axis (radix transforms)."""
    dk = _dk()
    s = {"cubic": _small_dimer(0), "hexagonal": _hexagonal_system(),
         "unsplit": sysgen.tiny_dimer(0, grid=(16, 81, 16))}[which]
    rng = np.random.default_rng(7)
    f = rng.uniform(0.0, 1.0, s.grid)
    vh_ref = scf.hartree(f, s.lattice)
    kk_ref = scf.kerker(f, s.lattice, 0.9)
    b = dk.init_basis([s])
    fd = torch.from_numpy(f).to(dev)
    print(f"[hartree/kerker] {which} grid={s.grid}", flush=True)
    vh = dk.hartree(b, 0, fd).cpu().numpy()
    kk = dk.kerker(b, 0, fd, 0.9).cpu().numpy()
    b.close()
    assert np.abs(vh - vh_ref).max() < 1e-12 * np.abs(vh_ref).max()
    assert np.abs(kk - kk_ref).max() < 1e-12 * np.abs(kk_ref).max()


def test_lda_matches_oracle(dev):
    """Densities spanning rs < 1 and rs > 1 (and below the cut-off) with
    random spin densities |m| < rho."""
    dk = _dk()
    s = _small_dimer(0)
    rng = np.random.default_rng(8)
    rho = 10.0 ** rng.uniform(-16, 1, s.grid)
    m = rng.standard_normal((3,) + s.grid)
    m *= (rho * rng.uniform(0, 1, s.grid) / np.sqrt(np.sum(m * m, axis=0)))[None]
    vxc_ref, bxc_ref, exc_ref = scf.lda_xc(rho, m)
    b = dk.init_basis([s])
    vxc, bxc, exc = dk.lda_xc(b, 0, torch.from_numpy(rho).to(dev), torch.from_numpy(m).to(dev))
    b.close()
    # B_xc = (v_up - v_dn) / 2 cancels to ~zeta of the potentials: its rounding
    # is eps |v| / |B|, so it is compared on the scale of the field
    for got, ref in ((vxc, vxc_ref), (bxc, bxc_ref), (exc, exc_ref)):
        got = got.cpu().numpy()
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max()), np.abs(got - ref).max()


def test_local_potential_round_trip_and_operator(dev):
    """A new potential set on the basis comes back unchanged, H X follows it
    (the oracle operator with the same potential) and the filter constants
    follow its mean and maximum."""
    dk = _dk()
    s = _small_dimer(1)
    rng = np.random.default_rng(12)
    v = s.v_loc + rng.uniform(-0.5, 0.5, s.grid)
    b = dk.init_basis([s])
    C0, _ = dk.filter_constants(b, 0)
    dk.set_local_potential(b, 0, torch.from_numpy(v).to(dev))
    back = dk.get_local_potential(b, 0).cpu().numpy()
    assert np.array_equal(back, v)
    C1, O1 = dk.filter_constants(b, 0)
    assert abs((C1 - C0) - (v.mean() - s.v_loc.mean())) < 1e-9
    op = dks.DKSOperator(dataclasses.replace(s, v_loc=v))
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    X = random_block(rng, 3, N)
    Xd = torch.from_numpy(X).to(dev)
    HXd = torch.empty_like(Xd)
    dk.apply_H(b, 0, Xd, HXd)
    got = HXd.cpu().numpy()
    b.close()
    ref = to_lib(op.apply(to_orc(X, p)), p)
    assert np.abs(got - ref).max() < 2e-13 * np.abs(ref).max()


def _uniform_gas(v0, model):
    s = sysgen.tiny_dimer(0, ecut=2.0, grid=(12, 12, 12), n_bands=14, with_nonlocal=False)
    return dataclasses.replace(s, v_loc=np.full(s.grid, v0))


@pytest.mark.parametrize("model", ["dks", "ksso"])
def test_scf_uniform_gas_closed_form(dev, model):
    """The ion-free gas: the self-consistent potential is V0 + v_xc(n/Omega) and
    the eigenvalues the free levels shifted by v_xc (closed form)."""
    dk = _dk()
    v0, n, n_el = -0.3, 14, 10.0
    s = _uniform_gas(v0, model)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    nc = 4 if model == "dks" else 2
    X0 = np.zeros((n, nc, N), dtype=np.complex128)
    X0[:, :2] = sysgen.start_block(mil, s.lattice, s.kpts[0], n, 1)
    Xd = torch.from_numpy(X0).to(dev)
    so = dk.scf_default_opts(n_electrons=n_el, tol=1e-10, max_scf=30)
    eo = dk.default_opts(kinetic_balance=1 if model == "dks" else 0, tol=1e-9,
                         model=dk.MODEL_DKS if model == "dks" else dk.MODEL_KSSO,
                         use_filter=1 if model == "dks" else 0)
    print(f"[scf uniform gas] {model}", flush=True)
    lam, occ, info, rc = dk.scf(b, 0, n, Xd, so, eo)
    v = dk.get_local_potential(b, 0).cpu().numpy()
    b.close()
    print(f"  scf steps {info['iterations']}, eigensolver iterations {info['eig_iterations']}", flush=True)
    assert rc == 0 and info["converged"] == 1, info
    rho0 = n_el / scf.cell_volume(s.lattice)
    vxc0 = scf.lda_xc(np.full((1, 1, 1), rho0))[0][0, 0, 0]
    assert np.abs(v - (v0 + vxc0)).max() < 1e-9
    q = dks.planewave_basis(s.lattice, s.kpts[0], s.ecut)[1]
    if model == "dks":
        lev = dks.free_dirac_levels(q, s.c)
        lev = lev[lev > -s.c ** 2][:n]
    else:
        lev = np.sort(np.repeat(0.5 * np.einsum("ij,ij->i", q, q), 2))[:n]
    assert np.abs(lam - (lev + v0 + vxc0)).max() < 1e-8
    assert abs(occ.sum() - n_el) < 1e-10


def test_scf_dimer_matches_oracle(dev):
    """The small dimer's SCF (6 electrons in the 10 lowest positive-band states
    at 5000 K, Anderson + Kerker mixing, 3 LOBPCG-F iterations per step):
    self-consistent potential, eigenvalues and free energy against the
    oracle's loop with exact eigenpairs."""
    dk = _dk()
    s = _small_dimer(0)
    n, n_el = 10, 6.0
    ref = scf.scf(s, n, n_el, tol=1e-10, max_iter=80)
    assert ref.converged
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    X0 = np.zeros((n, 4, N), dtype=np.complex128)
    X0[:, :2] = sysgen.start_block(mil, s.lattice, s.kpts[0], n, 2)
    Xd = torch.from_numpy(X0).to(dev)
    so = dk.scf_default_opts(n_electrons=n_el, tol=1e-10, max_scf=80)
    eo = dk.default_opts(kinetic_balance=1, tol=1e-9)
    print("[scf small dimer]", flush=True)
    lam, occ, info, rc = dk.scf(b, 0, n, Xd, so, eo)
    v = dk.get_local_potential(b, 0).cpu().numpy()
    b.close()
    print(f"  scf steps {info['iterations']} (oracle {len(ref.residuals)}), "
          f"residual {info['residual']:.2e}, free energy {info['free_energy']:.10f} "
          f"(oracle {ref.free_energy:.10f})", flush=True)
    assert rc == 0 and info["converged"] == 1, info
    assert np.abs(v - ref.v).max() < 1e-6 * np.abs(ref.v).max()
    assert np.abs(lam - ref.eigvals).max() < 1e-7
    assert abs(info["free_energy"] - ref.free_energy) < 1e-7
    assert abs(info["fermi"] - ref.mu) < 1e-7
    assert info["max_bxc"] < 1e-8


def test_scf_argument_errors(dev):
    """Electron counts outside (0, wanted bands) and descriptions with several
    k-points are EINVAL; nothing is changed."""
    dk = _dk()
    s = _small_dimer(0)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    X = torch.zeros((8, 4, N), dtype=torch.complex128, device=dev)
    for n_el in (0.0, 8.0, 12.0):
        with pytest.raises(dk.DksError) as e:
            dk.scf(b, 0, 8, X, dk.scf_default_opts(n_electrons=n_el))
        assert e.value.code == -1
    b.close()
    s2 = dataclasses.replace(s, kpts=np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0]]))
    b = dk.init_basis([s2])
    with pytest.raises(dk.DksError) as e:
        dk.scf(b, 0, 8, X, dk.scf_default_opts(n_electrons=4.0))
    assert e.value.code == -1 and "k-point" in str(e.value)
    b.close()
