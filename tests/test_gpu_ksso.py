"""The two-component KSSO operator (the paper's Table 1 comparison module) on the
GPU: dks_apply_H_ksso against the oracle's matrix-free apply, the standard
LOBPCG solve (model = KSSO) against the oracle's dense two-component
spectrum, and the nonrelativistic limit seen from the GPU: the DKS
eigenvalues at c = 1e3 and 3e3 approach the KSSO ones with an error that
falls as 1/c^2 (Sec. 2)."""
import numpy as np
import pytest

import sysgen
from oracle import dks
from tests.gpu_helpers import perm_to_oracle, to_orc
from tests.test_gpu_parity import TOL, _dk, _hexagonal_system, row_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _ksso_parity(dev, s, nb, seed, prec):
    dk = _dk()
    op = dks.DKSOperator(s)
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((nb, 2, N)) + 1j * rng.standard_normal((nb, 2, N))
    ctype = torch.complex128 if prec == "fp64" else torch.complex64
    Xd = torch.from_numpy(X).to(dev, ctype)
    HXd = torch.empty_like(Xd)
    print(f"[apply_H_ksso] {s.name} nb={nb} N={N} {prec}", flush=True)
    dk.apply_H_ksso(b, 0, Xd, HXd)
    torch.cuda.synchronize()
    got = to_orc(HXd.cpu().numpy().astype(np.complex128), p)
    Xo = to_orc(Xd.cpu().numpy().astype(np.complex128), p)
    b.close()
    return row_errors(got, op.apply_ksso(Xo))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_ksso_tiny_dimer(dev, prec):
    err = _ksso_parity(dev, sysgen.tiny_dimer(0), 7, 3, prec)
    assert err < TOL[prec], err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_ksso_hexagonal_kpoint(dev, prec):
    err = _ksso_parity(dev, _hexagonal_system(), 5, 4, prec)
    assert err < TOL[prec], err


def _ksso_solve(dk, dev, s, n, mode, seed=0):
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    X0 = sysgen.start_block(mil, s.lattice, s.kpts[0], n, seed)     # (n, 2, N)
    Xd = torch.from_numpy(np.ascontiguousarray(X0)).to(dev)
    o = dk.default_opts(model=dk.MODEL_KSSO, mode=mode, n_iter=400)
    lam, res, info, rc = dk.lobpcgf_solve(b, 0, n, Xd, o)
    b.close()
    return np.asarray(lam), np.asarray(res), info, rc


@pytest.mark.parametrize("mode", [0, 1])
def test_ksso_lobpcg_matches_dense(dev, mode):
    """Standard LOBPCG on the KSSO operator (no filter): the 8 lowest
    eigenvalues of the dense two-component oracle to 1e-8 Ha."""
    dk = _dk()
    s = sysgen.tiny_dimer(1)
    ref = np.linalg.eigvalsh(dks.DKSOperator(s).pauli_dense())[:8]
    print(f"[KSSO LOBPCG] mode={mode}", flush=True)
    lam, res, info, rc = _ksso_solve(dk, dev, s, 8, mode)
    assert rc == 0, info
    assert np.all(res < 1e-8)
    assert np.max(np.abs(lam - ref)) < 1e-8, lam - ref


def test_nonrelativistic_limit_on_the_gpu(dev):
    """DKS (LOBPCG-F) minus KSSO (LOBPCG) eigenvalues, both from the library,
    shrink as 1/c^2 between c = 1e3 and 3e3 (ratio 9 up to higher orders)."""
    dk = _dk()
    errs = []
    for c in (1e3, 3e3):
        s = sysgen.tiny_dimer(0, c=c, ecut=2.5, grid=(16, 16, 16))
        lam_k, _, info_k, rc_k = _ksso_solve(dk, dev, s, 8, 0)
        b = dk.init_basis([s])
        N, _, mil = dk.basis_info(b, 0)
        X0 = np.zeros((8, 4, N), dtype=np.complex128)
        X0[:, :2] = sysgen.start_block(mil, s.lattice, s.kpts[0], 8, 0)
        Xd = torch.from_numpy(X0).to(dev)
        print(f"[NR limit] c={c:g}", flush=True)
        lam_d, _, info_d, rc_d = dk.lobpcgf_solve(b, 0, 8, Xd,
                                                 dk.default_opts(kinetic_balance=1, n_iter=400))
        b.close()
        assert rc_k == 0 and rc_d == 0, (info_k, info_d)
        errs.append(float(np.max(np.abs(np.asarray(lam_d) - lam_k))))
    print(f"  |DKS - KSSO| at c = 1e3, 3e3: {errs}", flush=True)
    assert 6.0 < errs[0] / errs[1] < 12.0, errs
