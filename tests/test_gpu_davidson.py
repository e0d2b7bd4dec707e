"""The filter inside a block Davidson iteration (method = DKS_METHOD_DAVIDSON;
the paper names Davidson-type solvers as another home for F, Sec. 3 opening and
Sec. 5) on the GPU, against the dense FP64 oracle and its goldens: eigenvalues
within 1e-8 Ha, every wanted residual below 1e-8, no Ritz value in the gap, and
collapse without the filter as for LOBPCG."""
import json
import os

import numpy as np
import pytest

import sysgen
from oracle import dks, lobpcgf
from tests.gpu_helpers import cluster_projectors_match, perm_to_oracle, to_lib, to_orc
from tests.test_gpu_parity import _dk, _hexagonal_system

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _start(dk, b, s, n, seed):
    N, _, mil = dk.basis_info(b, 0)
    X0 = np.zeros((n, 4, N), dtype=np.complex128)
    X0[:, :2] = sysgen.start_block(mil, s.lattice, s.kpts[0], n, seed)
    return X0, mil


@pytest.mark.parametrize("ddim", [2, 4])
def test_davidson_tiny_dimer_matches_dense(dev, ddim):
    """Tiny dimer, 8 bands, the space restarted at 2n (every step) or 4n
    vectors: dense eigenvalues and cluster projectors."""
    dk = _dk()
    s = sysgen.tiny_dimer(0)
    op = dks.DKSOperator(s)
    n = 8
    lam_ref, vec_ref = lobpcgf.lowest_positive(op.dense(), n, s.c)
    b = dk.init_basis([s])
    X0, mil = _start(dk, b, s, n, 0)
    p = perm_to_oracle(mil, op.miller)
    Xd = torch.from_numpy(X0).to(dev)
    print(f"[davidson tiny] davidson_dim={ddim}", flush=True)
    lam, res, info, rc = dk.lobpcgf_solve(
        b, 0, n, Xd, dk.default_opts(method=dk.METHOD_DAVIDSON, davidson_dim=ddim,
                                     kinetic_balance=1, n_iter=400))
    Xo = to_orc(Xd.cpu().numpy(), p).reshape(n, -1).T
    b.close()
    print(f"  iterations {info['iterations']}, H applies {info['h_applies']}", flush=True)
    assert rc == 0 and info["converged"] == 1, info
    assert np.max(np.abs(lam - lam_ref)) < 1e-8, lam - lam_ref
    assert np.all(res < 1e-8)
    assert info["min_ritz"] > -s.c ** 2
    assert cluster_projectors_match(lam_ref, vec_ref, Xo) < 1e-6


def test_davidson_ragged_block_and_kpoint(dev):
    """n = 5 at a k-point of the hexagonal cell (pairs split by the block)."""
    dk = _dk()
    s = _hexagonal_system()
    op = dks.DKSOperator(s)
    n = 5
    lam_ref, _ = lobpcgf.lowest_positive(op.dense(), n, s.c)
    b = dk.init_basis([s])
    X0, _ = _start(dk, b, s, n, 5)
    Xd = torch.from_numpy(X0).to(dev)
    print("[davidson hexagonal k-point] n=5", flush=True)
    lam, res, info, rc = dk.lobpcgf_solve(
        b, 0, n, Xd, dk.default_opts(method=dk.METHOD_DAVIDSON, kinetic_balance=1, n_iter=400))
    b.close()
    assert rc == 0, info
    assert np.max(np.abs(lam - lam_ref)) < 1e-8, lam - lam_ref


@pytest.mark.parametrize("sysno,buf", [(50, 8), (22, 8)])
def test_davidson_generator_systems(dev, sysno, buf):
    """Systems of the 64-system uneven batch with their generator band counts
    plus buffer columns: 50 (N = 1045, 24 bands) and 22 (N = 1743, 64 bands,
    a 288-vector space); the wanted eigenvalues against the dense-oracle golden."""
    dk = _dk()
    ref = np.array(json.load(open(os.path.join(GOLDEN, "uneven_batch_seed0_dense.json")))
                   ["systems"][str(sysno)]["eigenvalues"])
    s = sysgen.uneven_batch(seed=0, count=64)[sysno]
    nw = s.n_bands
    n = nw + buf
    b = dk.init_basis([s])
    X0, _ = _start(dk, b, s, n, 200 + sysno)
    Xd = torch.from_numpy(X0).to(dev)
    print(f"[davidson system {sysno}] n={n} buffer={buf}", flush=True)
    lam, res, info, rc = dk.lobpcgf_solve(
        b, 0, n, Xd, dk.default_opts(method=dk.METHOD_DAVIDSON, kinetic_balance=1, n_iter=400,
                                     n_buffer=buf))
    b.close()
    print(f"  iterations {info['iterations']}, H applies {info['h_applies']}, "
          f"max|r| {info['max_resnorm']:.2e}", flush=True)
    assert rc == 0 and info["converged"] == 1, info
    assert np.all(np.asarray(res)[:nw] < 1e-8)
    assert np.max(np.abs(np.asarray(lam)[:nw] - ref[:nw])) < 1e-8


def test_davidson_collapses_without_the_filter(dev):
    """Sec. 3.1's argument for a Davidson space: from a block carrying 1e-15 of
    the lowest negative-band eigenvector, the unfiltered iteration falls into
    the negative continuum (DKS_ECOLLAPSE); with F it converges."""
    dk = _dk()
    s = sysgen.tiny_dimer(0)
    op = dks.DKSOperator(s)
    w, V = np.linalg.eigh(op.dense())
    lam_ref = w[w > -s.c ** 2][:8]
    b = dk.init_basis([s])
    N, _, mil = dk.basis_info(b, 0)
    p = perm_to_oracle(mil, op.miller)
    phi = sysgen.start_block(op.miller, s.lattice, s.kpts[0], 8, 0)
    X0 = lobpcgf.kinetic_balance(op, phi)
    X0 = X0 / np.linalg.norm(X0.reshape(8, -1), axis=1)[:, None, None]
    X0 = to_lib(X0 + 1e-15 * V[:, 0].reshape(1, 4, N), p)
    print("[davidson collapse] use_filter=0", flush=True)
    with pytest.raises(dk.DksError) as e:
        dk.lobpcgf_solve(b, 0, 8, torch.from_numpy(X0).to(dev),
                         dk.default_opts(method=dk.METHOD_DAVIDSON, use_filter=0, n_iter=40,
                                         tol=1e-9, preconditioner=dk.PRECOND_NONE))
    assert e.value.code == -5, str(e.value)
    print("[davidson collapse] with the filter", flush=True)
    lam, res, info, rc = dk.lobpcgf_solve(b, 0, 8, torch.from_numpy(X0).to(dev),
                                          dk.default_opts(method=dk.METHOD_DAVIDSON, n_iter=200))
    b.close()
    assert rc == 0, info
    assert np.max(np.abs(lam - lam_ref)) < 1e-8


def test_davidson_invalid_options(dev):
    """The Davidson form runs in FP64 only; an unknown method is EINVAL."""
    dk = _dk()
    s = sysgen.tiny_dimer(0)
    b = dk.init_basis([s])
    X0, _ = _start(dk, b, s, 8, 0)
    for kw in (dict(method=dk.METHOD_DAVIDSON, mode=dk.MODE_MIXED_FP32), dict(method=7)):
        with pytest.raises(dk.DksError) as e:
            dk.lobpcgf_solve(b, 0, 8, torch.from_numpy(X0).to(dev), dk.default_opts(**kw))
        assert e.value.code == -1, (kw, str(e.value))
    b.close()


def test_davidson_batch_lanes(dev):
    """A k, -k pair of the hexagonal cell through dks_lobpcgf_solve_batch on the
    lanes with the Davidson method: both spectra equal the dense one; the graph
    form refuses the method."""
    import dataclasses
    dk = _dk()
    s1 = _hexagonal_system()
    k = s1.kpts[0]
    s = dataclasses.replace(s1, kpts=np.array([k, -k]))
    n = 6
    ref = lobpcgf.lowest_positive(dks.DKSOperator(s, 0).dense(), n, s.c)[0]
    b = dk.init_basis([s])
    Xs = []
    for i in range(2):
        N, _, mil = dk.basis_info(b, i)
        X0 = np.zeros((n, 4, N), dtype=np.complex128)
        X0[:, :2] = sysgen.start_block(mil, s.lattice, s.kpts[i], n, 4 + i)
        Xs.append(torch.from_numpy(X0).to(dev))
    print("[davidson batch] k, -k", flush=True)
    o = dk.default_opts(method=dk.METHOD_DAVIDSON, kinetic_balance=1, n_iter=400)
    lams, ress, infos, rc = dk.lobpcgf_solve_batch(b, [0, 1], [n, n], Xs, o)
    assert rc == 0, infos
    for lam in lams:
        assert np.max(np.abs(np.asarray(lam) - ref)) < 1e-8
    o.batch_graph = 1
    with pytest.raises(dk.DksError) as e:
        dk.lobpcgf_solve_batch(b, [0, 1], [n, n], Xs, o)
    assert e.value.code == -1
    b.close()
