"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Tolerances (derived from the arithmetic, see the design notes).  apply_H is
compared per (band, component) row, each row's error divided by that row's
own largest reference value, so that the large-component rows (kinetic terms
~c|q||chi|) are not judged on the scale of the small-component rows (~2c^2|chi|):
* apply_H FP64: every row within 2e-13 of its max|HX| (FFT and GEMM rounding
  of O(log N_g) eps);
* apply_H FP32: every row within 2e-5 of its max|HX|;
* the potential terms at their own scale: with chi = 0 the large rows of H X
  hold only the local and nonlocal potentials (no kinetic term enters them),
  within 1e-12 (FP64) or 2e-5 (FP32) of the row; with phi = 0 the small rows
  hold -2c^2 chi plus the potentials, and after the oracle's -2c^2 chi is taken
  off both sides the rest must agree within 4 u max|2c^2 chi| (the library's
  rounding of that term, u the unit roundoff) plus 1e-12 / 2e-5 of the row's
  potential terms;
* eigenvalues: within 1e-8 Ha of the dense oracle (FP64 and after the FP64
  polish of the mixed modes), every residual below 1e-8, cluster projectors
  within 1e-6.
"""
import dataclasses
import math

import numpy as np
import pytest

import sysgen
from oracle import dks, lobpcgf
from tests.gpu_helpers import cluster_projectors_match, perm_to_oracle, random_block, to_lib, to_orc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dk():
    import paper_1211_1446_amd as dk
    return dk


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _hexagonal_system():
    rng = np.random.default_rng(42)
    A = sysgen.hexagonal(6.0, 9.0)
    grid = (18, 18, 25)
    tau = np.array([[0.3, 0.2, 2.0], [1.5, 2.1, 6.1]])
    v = sysgen.gaussian_potential(A, grid, tau, [-6.0, -9.0], [0.7, 0.6])
    v = v + rng.uniform(-0.01, 0.01, size=grid)
    proj = []
    for a in range(2):
        for l in range(4):
            nr = 3 if l < 2 else 1
            dp = rng.uniform(-2, 2, (nr, nr)); dp = dp + dp.T
            dm = rng.uniform(-2, 2, (nr, nr)); dm = dm + dm.T
            proj.append(sysgen.ProjGroup(a, l, nr, 0.65, dp, dm))
    k = np.array([[0.11, -0.05, 0.17]])
    return sysgen.System("hex", A, k, 3.0, grid, sysgen.C_LIGHT, v, tau, proj, 5)


def row_errors(got, ref):
    """Per (band, component) row: max|got - ref| / max|ref| of that row (the
    largest over all rows is returned)."""
    num = np.abs(got - ref).max(axis=-1)
    den = np.abs(ref).max(axis=-1)
    return float(np.max(num / np.where(den > 0, den, 1.0)))


def free_dirac_part(s, X_orc, k_index=0):
    """The oracle's H X with the local and nonlocal potentials switched off:
    the free-Dirac (kinetic + mass) term alone."""
    free = dataclasses.replace(s, v_loc=np.zeros_like(s.v_loc), proj=[])
    return dks.DKSOperator(free, k_index).apply(X_orc)


UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24}
TOL = {"fp64": 2e-13, "fp32": 2e-5}
TOL_POT = {"fp64": 1e-12, "fp32": 2e-5}


def component_errors(s, got, ref, Xo, prec, part):
    """Error of the potential terms at their own scale (see the module notes).

    part = "large": X has chi = 0, the large rows of H X are potential only.
    part = "small": X has phi = 0, the small rows minus the oracle's free-Dirac
    term are potential only, up to the library's rounding of -2c^2 chi.
    Returns the largest ratio error / bound over the rows (<= 1 passes)."""
    worst = 0.0
    if part == "large":
        num = np.abs(got[:, :2] - ref[:, :2]).max(axis=-1)
        den = TOL_POT[prec] * np.abs(ref[:, :2]).max(axis=-1)
    else:
        kin = free_dirac_part(s, Xo)
        pot_ref = ref[:, 2:] - kin[:, 2:]
        num = np.abs((got[:, 2:] - kin[:, 2:]) - pot_ref).max(axis=-1)
        big = np.abs(kin[:, 2:]).max(axis=-1)
        den = 4 * UNIT_ROUNDOFF[prec] * big + TOL_POT[prec] * np.abs(pot_ref).max(axis=-1)
    worst = max(worst, float(np.max(num / den)))
    return worst


def _apply_parity(dev, s, nb, seed, prec, X=None, k_index=0):
    """Row error of the library's H X against the oracle on the block X
    (random when not given); also returns (got, ref, X in oracle order)."""
    dk = _dk()
    op = dks.DKSOperator(s, k_index)
    b = dk.init_basis([s])
    N, grid, mil = dk.basis_info(b, k_index)
    assert N == op.N and tuple(grid) == tuple(s.grid)
    p = perm_to_oracle(mil, op.miller)
    if X is None:
        X = random_block(np.random.default_rng(seed), nb, N)
    ctype = torch.complex128 if prec == "fp64" else torch.complex64
    Xd = torch.from_numpy(X).to(dev, ctype)
    HXd = torch.empty_like(Xd)
    print(f"[apply_H parity] {s.name} nb={nb} N={N} grid={grid} {prec}", flush=True)
    dk.apply_H(b, k_index, Xd, HXd)
    torch.cuda.synchronize()
    got = to_orc(HXd.cpu().numpy().astype(np.complex128), p)
    Xo = to_orc(Xd.cpu().numpy().astype(np.complex128), p)   # the block as the library saw it
    b.close()
    ref = op.apply(Xo)
    return row_errors(got, ref), got, ref, Xo


def one_component_blocks(rng, nb, N):
    """(chi = 0 block, phi = 0 block), random otherwise."""
    Xl = random_block(rng, nb, N)
    Xl[:, 2:] = 0
    Xs = random_block(rng, nb, N)
    Xs[:, :2] = 0
    return Xl, Xs


def check_apply(dev, s, nb, seed, prec):
    err, _, _, _ = _apply_parity(dev, s, nb, seed, prec)
    assert err < TOL[prec], err
    Xl, Xs = one_component_blocks(np.random.default_rng(seed + 100), nb, s_npw(s))
    for part, X in (("large", Xl), ("small", Xs)):
        err, got, ref, Xo = _apply_parity(dev, s, nb, seed, prec, X=X)
        assert err < TOL[prec], (part, err)
        ratio = component_errors(s, got, ref, Xo, prec, part)
        print(f"  {part}-component block: error / bound = {ratio:.2e}", flush=True)
        assert ratio < 1.0, (part, ratio)


def s_npw(s, k_index=0):
    return dks.DKSOperator(s, k_index).N


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_h_tiny_dimer(dev, prec):
    check_apply(dev, sysgen.tiny_dimer(0), 8, 1, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_h_hexagonal_kpoint_ragged(dev, prec):
    """General lattice, k != 0, odd grid (18, 18, 25), l up to 3, three radial
    functions, 5 bands (a ragged band tile)."""
    check_apply(dev, _hexagonal_system(), 5, 2, prec)


def test_apply_h_edge_sizes(dev):
    dk = _dk()
    s = sysgen.tiny_dimer(0)
    op = dks.DKSOperator(s)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    # nb = 0 is a no-op
    Xd = torch.zeros((1, 4, N), dtype=torch.complex128, device=dev)
    HXd = torch.full_like(Xd, 7.0)
    dk.apply_H(b, 0, Xd, HXd, nb=0)
    torch.cuda.synchronize()
    assert torch.all(HXd == 7.0)
    # a single planewave in one component
    X = np.zeros((1, 4, N), dtype=np.complex128)
    X[0, 2, N // 3] = 1.0 - 0.5j
    ref = op.apply(to_orc(X, p))
    Xd = torch.from_numpy(X).to(dev)
    dk.apply_H(b, 0, Xd, HXd)
    got = to_orc(HXd.cpu().numpy(), p)
    assert np.abs(got - ref).max() < 2e-13 * np.abs(ref).max()
    b.close()


@pytest.mark.parametrize("grid", [(16, 81, 16), (81, 16, 18)])
def test_apply_h_plane_axis_without_two_step_split(dev, grid):
    """A plane axis of 81 points has no compiled two-step split: both plane
    axes then take the radix transforms in natural order, and the potential
    table must follow that order (tiny dimer on the stretched grid)."""
    dk = _dk()
    s = sysgen.tiny_dimer(0, grid=grid)
    op = dks.DKSOperator(s)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    X = random_block(np.random.default_rng(9), 3, N)
    Xd = torch.from_numpy(X).to(dev)
    HXd = torch.empty_like(Xd)
    print(f"[apply_H grid {grid}]", flush=True)
    dk.apply_H(b, 0, Xd, HXd)
    got = to_orc(HXd.cpu().numpy(), p)
    ref = op.apply(to_orc(X, p))
    b.close()
    assert np.abs(got - ref).max() < 2e-13 * np.abs(ref).max()


def test_apply_filter_matches_oracle(dev):
    dk = _dk()
    s = sysgen.tiny_dimer(3)
    op = dks.DKSOperator(s)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    C, Om = dk.filter_constants(b, 0)
    rng = np.random.default_rng(4)
    Y = random_block(rng, 3, N)
    ref = lobpcgf.apply_filter(lambda Z: op.apply(Z), to_orc(Y, p), C, Om)
    Yd = torch.from_numpy(Y).to(dev)
    FYd = torch.empty_like(Yd)
    dk.apply_filter(b, 0, Yd, FYd, C, Om)
    got = to_orc(FYd.cpu().numpy(), p)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    b.close()


def test_apply_h_heavy_dimer_full_block_sampled(dev):
    """The full 40-band heavy-dimer block (96^3 grid, 62 669 planewaves) in one
    call, as the benchmark launches it; sampled bands against the oracle."""
    dk = _dk()
    s = sysgen.heavy_dimer(0)
    op = dks.DKSOperator(s)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    rng = np.random.default_rng(9)
    phi = sysgen.start_block(mil, s.lattice, s.kpts[0], 40, 0)
    X = np.zeros((40, 4, N), dtype=np.complex128)
    X[:, :2] = phi
    X[:, 2:] = 0.02 * (rng.standard_normal((40, 2, N)) + 1j * rng.standard_normal((40, 2, N)))
    Xd = torch.from_numpy(X).to(dev)
    HXd = torch.empty_like(Xd)
    print("[apply_H heavy dimer] nb=40", flush=True)
    dk.apply_H(b, 0, Xd, HXd)
    torch.cuda.synchronize()
    got = HXd.cpu().numpy()
    for band in (0, 17, 39):
        ref = op.apply(to_orc(X[band:band + 1], p))
        g = to_orc(got[band:band + 1], p)
        assert np.abs(g - ref).max() < 2e-13 * np.abs(ref).max(), band
    b.close()


def _solve_tiny(dev, mode, seed=0, n=8, **kw):
    dk = _dk()
    s = sysgen.tiny_dimer(seed)
    op = dks.DKSOperator(s)
    lam_ref, vec_ref = lobpcgf.lowest_positive(op.dense(), n, s.c)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    X0 = np.zeros((n, 4, N), dtype=np.complex128)
    X0[:, :2] = sysgen.start_block(mil, s.lattice, s.kpts[0], n, seed)
    Xd = torch.from_numpy(X0).to(dev)
    opts = dk.default_opts(mode=mode, kinetic_balance=1, **kw)
    print(f"[lobpcgf_solve tiny] mode={mode} n={n} seed={seed}", flush=True)
    lam, res, info, rc = dk.lobpcgf_solve(b, 0, n, Xd, opts)
    Xo = to_orc(Xd.cpu().numpy(), p).reshape(n, -1).T
    b.close()
    return lam, res, info, rc, lam_ref, vec_ref, Xo, s


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_lobpcgf_tiny_dimer_matches_dense(dev, mode):
    lam, res, info, rc, lam_ref, vec_ref, Xo, s = _solve_tiny(dev, mode)
    assert rc == 0, info
    assert np.max(np.abs(lam - lam_ref)) < 1e-8, (lam - lam_ref)
    assert np.all(res < 1e-8)
    assert info["min_ritz"] > -s.c ** 2
    assert np.allclose(np.linalg.norm(Xo, axis=0), 1.0, atol=1e-10)
    assert cluster_projectors_match(lam_ref, vec_ref, Xo) < 1e-6
    if mode >= 1:
        assert info["iters_reduced"] > 0


@pytest.mark.parametrize("mode", [0, 1])
def test_lobpcgf_buffer_columns(dev, mode):
    """A block of 10 with n_buffer = 2: the 8 wanted pairs converge to the dense
    ones; convergence and the info fields cover only them."""
    lam, res, info, rc, lam_ref, vec_ref, Xo, s = _solve_tiny(dev, mode, n=10, n_buffer=2)
    assert rc == 0, info
    assert info["converged"] == 1 and info["n_converged"] == 8, info
    assert np.max(np.abs(lam[:8] - lam_ref[:8])) < 1e-8, (lam[:8] - lam_ref[:8])
    assert np.all(res[:8] < 1e-8)
    assert info["max_resnorm"] == pytest.approx(float(np.max(res[:8])))
    assert cluster_projectors_match(lam_ref[:8], vec_ref[:, :8], Xo[:, :8]) < 1e-6


def test_lobpcgf_buffer_out_of_range(dev):
    dk = _dk()
    s = sysgen.tiny_dimer(0)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    X0 = np.zeros((4, 4, N), dtype=np.complex128)
    X0[:, :2] = sysgen.start_block(mil, s.lattice, s.kpts[0], 4, 0)
    Xd = torch.from_numpy(X0).to(dev)
    with pytest.raises(Exception):
        dk.lobpcgf_solve(b, 0, 4, Xd, dk.default_opts(n_buffer=4))
    b.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_reduced_precision_stage_alone(dev, mode):
    """The FP32 (mode 1) or BF16-Gram (mode 2) stage by itself, 40 iterations
    with T = I, followed only by the FP64 polish's first Rayleigh-Ritz (n_iter = 0): its
    eigenvalues already sit near the dense ones, far below the start block's
    error, so the reduced-precision Gram products carry the right numbers."""
    lam, res, info, rc, lam_ref, vec_ref, Xo, s = _solve_tiny(
        dev, mode, n_iter=0, mixed_iter=40, mixed_tol=-1.0, preconditioner=0)
    err = np.max(np.abs(lam - lam_ref))
    print(f"mode {mode}: reduced stage max |lambda - dense| = {err:.3e}", flush=True)
    assert info["iters_reduced"] == 40
    assert err < 1e-3, err


def test_lobpcgf_ragged_block_and_kpoint(dev):
    """n = 5 at a k-point (pairs split), hexagonal cell with l <= 3 projectors."""
    dk = _dk()
    s = _hexagonal_system()
    op = dks.DKSOperator(s)
    n = 5
    lam_ref, _ = lobpcgf.lowest_positive(op.dense(), n, s.c)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    X0 = np.zeros((n, 4, N), dtype=np.complex128)
    X0[:, :2] = sysgen.start_block(mil, s.lattice, s.kpts[0], n, 5)
    Xd = torch.from_numpy(X0).to(dev)
    lam, res, info, rc = dk.lobpcgf_solve(b, 0, n, Xd, dk.default_opts(kinetic_balance=1, n_iter=400))
    b.close()
    assert rc == 0, info
    assert np.max(np.abs(lam - lam_ref)) < 1e-8


def test_lobpcgf_error_paths(dev):
    dk = _dk()
    s = sysgen.tiny_dimer(0)
    b = dk.init_basis([s])
    N, _, _ = dk.basis_info(b, 0)
    X = torch.zeros((171, 4, N), dtype=torch.complex128, device=dev)
    with pytest.raises(dk.DksError) as e:
        dk.lobpcgf_solve(b, 0, 171, X)
    assert e.value.code == -1
    # a rank-deficient start block (two identical columns) -> DKS_ECHOL
    X = torch.zeros((2, 4, N), dtype=torch.complex128, device=dev)
    X[:, 0, 0] = 1.0
    with pytest.raises(dk.DksError) as e:
        dk.lobpcgf_solve(b, 0, 2, X, dk.default_opts(n_init=0))
    assert e.value.code == -4
    # iteration cap -> warning status with valid outputs
    X0 = np.zeros((4, 4, N), dtype=np.complex128)
    _, _, mil = dk.basis_info(b, 0)
    X0[:, :2] = sysgen.start_block(mil, s.lattice, s.kpts[0], 4, 0)
    Xd = torch.from_numpy(X0).to(dev)
    lam, res, info, rc = dk.lobpcgf_solve(b, 0, 4, Xd, dk.default_opts(n_iter=1, kinetic_balance=1))
    assert rc == 1 and np.all(np.isfinite(lam)) and info["iterations"] == 1
    b.close()


def test_filter_damping_across_c(dev):
    """The filter of Sec. 3.1 (f(E) = (E - C)^2 / Omega^2) on exact eigenvectors
    of the small dimer (dense oracle) at c/2, c and 2c, the c-scan of the
    filter's efficiency: in FP64 f(H)u = f(lambda)u for the lowest positive state
    and the top of the negative band (to 1e-12 of |u| = 1), and the damping of
    the negative band relative to the positive one, |F u_-| / |F u_+|, shrinks
    as c grows (it goes as (w / 4c^2)^2).  FP32 reaches the same damping up to
    its rounding floor (1e-6: rounding of terms ~2c^2 |u|, divided by Omega)."""
    dk = _dk()
    c0 = sysgen.C_LIGHT
    ratios = []
    for c in (0.5 * c0, c0, 2.0 * c0):
        s = sysgen.tiny_dimer(0, c=c, ecut=2.5, grid=(16, 16, 16))
        op = dks.DKSOperator(s)
        w, V = np.linalg.eigh(op.dense())
        ipos = int(np.argmax(w > -c * c))   # lowest positive-band state
        ineg = ipos - 1                     # top of the negative band
        b = dk.init_basis([s])
        N, _, mil = dk.basis_info(b, 0)
        p = perm_to_oracle(mil, op.miller)
        C, Om = dk.filter_constants(b, 0)
        U = np.stack([V[:, ipos].reshape(4, N), V[:, ineg].reshape(4, N)])
        Ud = torch.from_numpy(to_lib(U, p)).to(dev)
        print(f"[filter c-scan] c={c:.3f} N={N} lambda+={w[ipos]:.6f} lambda-={w[ineg]:.3f}", flush=True)
        FUd = torch.empty_like(Ud)
        dk.apply_filter(b, 0, Ud, FUd, C, Om)
        got = to_orc(FUd.cpu().numpy(), p)
        f = (w[[ipos, ineg]] - C) ** 2 / Om ** 2
        for j in range(2):
            assert np.linalg.norm(got[j] - f[j] * U[j]) < 1e-12, (c, j)
        ratios.append(np.linalg.norm(got[1]) / np.linalg.norm(got[0]))
        U32 = Ud.to(torch.complex64)
        FU32 = torch.empty_like(U32)
        dk.apply_filter(b, 0, U32, FU32, C, Om)
        g32 = FU32.cpu().numpy()
        r32 = np.linalg.norm(g32[1]) / np.linalg.norm(g32[0])
        assert abs(r32 - ratios[-1]) < 1e-6, (c, r32, ratios[-1])
        b.close()
    assert ratios[0] > ratios[1] > ratios[2], ratios


def test_standard_lobpcg_collapses_and_lobpcgf_does_not(dev):
    """Sec. 3.1 on the GPU: from a start block carrying 1e-15 of the lowest
    negative-band eigenvector (dense oracle), plain LOBPCG (use_filter = 0,
    T = I as in the analysis) falls into the negative continuum and the call
    returns DKS_ECOLLAPSE,
    while LOBPCG-F from the same block converges to the dense eigenvalues."""
    dk = _dk()
    s = sysgen.tiny_dimer(0)
    op = dks.DKSOperator(s)
    H = op.dense()
    w, V = np.linalg.eigh(H)
    lam_ref = w[w > -s.c ** 2][:8]
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    phi = sysgen.start_block(op.miller, s.lattice, s.kpts[0], 8, 0)
    X0 = lobpcgf.kinetic_balance(op, phi)
    X0 = X0 / np.linalg.norm(X0.reshape(8, -1), axis=1)[:, None, None]
    X0 = X0 + 1e-15 * V[:, 0].reshape(1, 4, N)
    X0 = to_lib(X0, p)
    print("[collapse] use_filter=0, 1e-15 negative-band content", flush=True)
    Xd = torch.from_numpy(X0).to(dev)
    with pytest.raises(dk.DksError) as e:
        dk.lobpcgf_solve(b, 0, 8, Xd, dk.default_opts(use_filter=0, n_iter=40, tol=1e-9,
                                                      preconditioner=dk.PRECOND_NONE))
    assert e.value.code == -5, str(e.value)
    print("[collapse] LOBPCG-F from the same block", flush=True)
    Xd = torch.from_numpy(X0).to(dev)
    lam, res, info, rc = dk.lobpcgf_solve(b, 0, 8, Xd, dk.default_opts(n_iter=200))
    b.close()
    assert rc == 0, info
    assert info["min_ritz"] > -s.c ** 2, info
    assert np.max(np.abs(lam - lam_ref)) < 1e-8


@pytest.mark.parametrize("form", [0, 1, 2, 3, 4, 5])
def test_apply_h_every_plane_form(dev, form):
    """Every plane kernel form the autotuner may pick (task split or whole lines
    per wave, large or 256-thread workgroups, column loads and stores folded
    into the a2 steps) and odd z tiles give the same H X, in FP64 and FP32:
    tiny dimer (24^3, all forms), the 96^3 heavy dimer (sampled bands; its
    plane exceeds the small forms' budget, which then fall back) and the
    hexagonal cell at k != 0 (rows of uneven length)."""
    dk = _dk()
    cases = ((sysgen.tiny_dimer(0), 6, None), (sysgen.heavy_dimer(0), 6, (0, 5)),
             (_hexagonal_system(), 4, None))
    for s, nb, bands in cases:
        op = dks.DKSOperator(s)
        b = dk.init_basis([s])
        N, _, mil = dk.basis_info(b, 0)
        p = perm_to_oracle(mil, op.miller)
        dk.set_tuning(b, 0, 3 if s.grid[0] < 50 else 5, form, 512)
        X = random_block(np.random.default_rng(form + 30), nb, N)
        for prec, ctype in (("fp64", torch.complex128), ("fp32", torch.complex64)):
            Xd = torch.from_numpy(X).to(dev).to(ctype)
            HXd = torch.empty_like(Xd)
            print(f"[plane form {form}] {s.name} nb={nb} {prec}", flush=True)
            dk.apply_H(b, 0, Xd, HXd)
            torch.cuda.synchronize()
            got = HXd.to(torch.complex128).cpu().numpy()
            for band in (bands or range(nb)):
                ref = op.apply(to_orc(X[band:band + 1], p))
                err = row_errors(to_orc(got[band:band + 1], p), ref)
                assert err < TOL[prec], (s.name, prec, band, err)
        b.close()
