"""The self-consistent field loop around the DKS eigenproblem, in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``density``        -- rho(r) and the spin density m(r) of Eq. (density) on
                        the FFT grid from the occupied spinors;
* ``hartree``        -- the electrostatic (Hartree) part of V_hxc (Sec. 2.1) of
                        a periodic density: V_H(G) = 4 pi rho(G) / |G|^2, G != 0;
* ``lda_xc``         -- the local (spin) density approximation the paper uses
                        (Sec. 2.1: Ceperley-Alder correlation as parametrised by
                        Perdew and Zunger, with Slater exchange and the von
                        Barth-Hedin spin interpolation), giving V_xc = dE/drho
                        and B_xc = dE/dm;
* ``fermi``          -- occupations at the electronic temperature of Sec. 4.2
                        (Fermi-Dirac, Mermin's finite-temperature functional);
* ``kerker``         -- the Kerker preconditioner of the density residual
                        (Sec. 4), G^2 / (G^2 + q0^2) in reciprocal space;
* ``Anderson``       -- Anderson mixing (Sec. 4) of the local effective
                        potential, with the Kerker step as its preconditioner;
* ``scf``            -- the outer loop: eigenpairs of H[V_in], occupations,
                        densities, V_out = V_ext + V_H + V_xc, stop when
                        ||V_out - V_in|| / ||V_in|| < tol (the measure of
                        Sec. 4.4), else mix.

Readings where the paper is silent (listed in the design notes):
* one electron per spinor band (a Kramers pair holds two), occupations
  f_i = 1 / (1 + exp((eps_i - mu) / kT)) with mu set so that sum f_i = n_el;
* psi(r) = Omega^-1/2 sum_G c_G exp(i (k + G).r), so that rho integrates to
  sum f_i over the cell; m(r) = sum_i f_i (phi^+ sigma phi - chi^+ sigma chi)
  (Eq. density);
* the FFT frequency of index m along an axis of N points is m for m < N/2 and
  m - N otherwise (so the Nyquist index of an even N is -N/2), and V_H is the
  real part of the inverse transform;
* E_xc depends on m through |m| only (the local spin polarisation zeta =
  |m| / rho), so B_xc = (v_up - v_dn) / 2 along m / |m|;
* densities below 1e-14 bohr^-3 carry no exchange-correlation energy;
* potential mixing (V_in is mixed, not rho): with x the input potential and
  r = V_out - V_in its residual, Anderson's combination of the last `depth`
  pairs (least squares on the residual differences) is followed by the step
  x + alpha K[r], K the Kerker factor G^2 / (G^2 + q0^2) for G != 0 and 1 at
  G = 0 (the damping is for long-wavelength charge sloshing; a constant
  shift of V moves no charge, and the residual measure includes it);
* the total free energy F = sum f eps - int (V_in - V_ext) rho + E_H + E_xc - T S
  with S = -k_B sum [f ln f + (1 - f) ln(1 - f)] (energies shifted by -c^2
  per electron like the eigenvalues; no ion-ion term in these synthetic cells).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import dks, lobpcgf

K_BOLTZMANN = 3.166811563e-6   # Ha / K

# Perdew-Zunger parametrisation of the Ceperley-Alder correlation energy per
# electron (Ha), unpolarised (U) and fully polarised (P): gamma, beta1, beta2
# for rs >= 1; A, B, C, D for rs < 1
_PZ = {
    "U": dict(g=-0.1423, b1=1.0529, b2=0.3334, A=0.0311, B=-0.048, C=0.0020, D=-0.0116),
    "P": dict(g=-0.0843, b1=1.3981, b2=0.2611, A=0.01555, B=-0.0269, C=0.0007, D=-0.0048),
}
# Slater exchange per electron of the unpolarised gas: -(3/4) (3/pi)^(1/3) rho^(1/3)
# = -(3/(4 pi)) (9 pi / 4)^(1/3) / rs
_CX = 0.75 * (9.0 * math.pi / 4.0) ** (1.0 / 3.0) / math.pi
_RHO_MIN = 1e-14


def cell_volume(lattice) -> float:
    return float(abs(np.linalg.det(np.asarray(lattice, dtype=np.float64))))


def _slots(op):
    return tuple(np.mod(op.miller[:, d], op.grid[d]) for d in range(3))


def spinors_on_grid(op, X: np.ndarray) -> np.ndarray:
    """psi_i(r_j) (n, 4, N1, N2, N3) of the blocks X (n, 4, N): the sum over the
    basis of c_G exp(2 pi i n.j / N) divided by sqrt(Omega).  The common phase
    exp(i k.r) is dropped: no density below depends on it."""
    n = X.shape[0]
    omega = cell_volume(op.system.lattice)
    sl = _slots(op)
    out = np.empty((n, 4) + op.grid, dtype=np.complex128)
    for i in range(n):
        for c in range(4):
            g = np.zeros(op.grid, dtype=np.complex128)
            g[sl] = X[i, c]
            out[i, c] = np.fft.ifftn(g) * (op.ng / math.sqrt(omega))
    return out


def density(op, X: np.ndarray, occ: np.ndarray):
    """Eq. (density): rho = sum_i f_i psi_i^+ psi_i and
    m = sum_i f_i psi_i^+ diag(sigma, -sigma) psi_i, on the grid (natural
    order).  Returns rho (N1, N2, N3) and m (3, N1, N2, N3)."""
    psi = spinors_on_grid(op, X)
    rho = np.zeros(op.grid)
    m = np.zeros((3,) + op.grid)
    for i, f in enumerate(occ):
        if f == 0.0:
            continue
        p = psi[i]
        rho += f * np.sum(np.abs(p) ** 2, axis=0)
        for sgn, (u, d) in ((1.0, (p[0], p[1])), (-1.0, (p[2], p[3]))):
            ud = np.conj(u) * d
            m[0] += sgn * f * 2.0 * ud.real
            m[1] += sgn * f * 2.0 * ud.imag
            m[2] += sgn * f * (np.abs(u) ** 2 - np.abs(d) ** 2)
    return rho, m


def fft_g2(lattice, grid) -> np.ndarray:
    """|G|^2 on the FFT grid, frequency m for m < N/2 and m - N otherwise."""
    b = dks.reciprocal_lattice(np.asarray(lattice, dtype=np.float64))
    f = [np.where(np.arange(n) < (n + 1) // 2, np.arange(n), np.arange(n) - n) for n in grid]
    m1, m2, m3 = np.meshgrid(*f, indexing="ij")
    G = m1[..., None] * b[0] + m2[..., None] * b[1] + m3[..., None] * b[2]
    return np.einsum("...i,...i->...", G, G)


def _filter_g(field: np.ndarray, kernel: np.ndarray) -> np.ndarray:
    """Real part of IFFT[kernel(G) FFT[field]] (FFT normalised by 1/N_g)."""
    return np.real(np.fft.ifftn(np.fft.fftn(field) * kernel))


def hartree(rho: np.ndarray, lattice) -> np.ndarray:
    """V_H with V_H(G) = 4 pi rho(G) / |G|^2 for G != 0 and 0 at G = 0 (the
    neutralising background), rho(G) = N_g^-1 sum_j rho_j exp(-2 pi i G.j/N)."""
    g2 = fft_g2(lattice, rho.shape)
    k = np.zeros_like(g2)
    nz = g2 > 0
    k[nz] = 4.0 * math.pi / g2[nz]
    return _filter_g(rho, k)


def kerker(r: np.ndarray, lattice, q0: float) -> np.ndarray:
    """Kerker preconditioner G^2 / (G^2 + q0^2) of a potential residual; the
    G = 0 part (a constant shift) passes unchanged."""
    g2 = fft_g2(lattice, r.shape)
    k = g2 / (g2 + q0 * q0)
    k[0, 0, 0] = 1.0
    return _filter_g(r, k)


def _pz_corr(rs: np.ndarray, p: dict):
    """Correlation energy per electron and its rs derivative (Perdew-Zunger)."""
    rs = np.asarray(rs, dtype=np.float64)
    e = np.empty_like(rs)
    de = np.empty_like(rs)
    hi = rs >= 1.0
    s = np.sqrt(rs[hi])
    den = 1.0 + p["b1"] * s + p["b2"] * rs[hi]
    e[hi] = p["g"] / den
    de[hi] = -p["g"] * (0.5 * p["b1"] / s + p["b2"]) / den ** 2
    lo = ~hi
    r = rs[lo]
    lr = np.log(r)
    e[lo] = p["A"] * lr + p["B"] + p["C"] * r * lr + p["D"] * r
    de[lo] = p["A"] / r + p["C"] * (lr + 1.0) + p["D"]
    return e, de


def _fz(z):
    return ((1.0 + z) ** (4.0 / 3.0) + (1.0 - z) ** (4.0 / 3.0) - 2.0) / (2.0 ** (4.0 / 3.0) - 2.0)


def _dfz(z):
    return (4.0 / 3.0) * ((1.0 + z) ** (1.0 / 3.0) - (1.0 - z) ** (1.0 / 3.0)) / (2.0 ** (4.0 / 3.0) - 2.0)


def lda_eps(rho: np.ndarray, zeta: np.ndarray):
    """Exchange-correlation energy per electron eps_xc(rho, zeta) and the
    potentials v_up, v_dn = d(rho eps_xc)/d rho_up,dn (local spin density
    approximation with the Perdew-Zunger correlation).  Densities below
    1e-14 give zeros."""
    rho = np.asarray(rho, dtype=np.float64)
    z = np.clip(np.asarray(zeta, dtype=np.float64), -1.0, 1.0)
    eps = np.zeros_like(rho)
    vu = np.zeros_like(rho)
    vd = np.zeros_like(rho)
    ok = rho > _RHO_MIN
    r = rho[ok]
    zz = z[ok]
    rs = (3.0 / (4.0 * math.pi * r)) ** (1.0 / 3.0)
    # exchange: unpolarised value times the spin factor
    exu = -_CX / rs
    sx = 0.5 * ((1.0 + zz) ** (4.0 / 3.0) + (1.0 - zz) ** (4.0 / 3.0))
    dsx = (2.0 / 3.0) * ((1.0 + zz) ** (1.0 / 3.0) - (1.0 - zz) ** (1.0 / 3.0))
    ex = exu * sx
    dex_drs = (_CX / rs ** 2) * sx
    dex_dz = exu * dsx
    # correlation: interpolation between the unpolarised and polarised fits
    ecu, decu = _pz_corr(rs, _PZ["U"])
    ecp, decp = _pz_corr(rs, _PZ["P"])
    f = _fz(zz)
    ec = ecu + f * (ecp - ecu)
    dec_drs = decu + f * (decp - decu)
    dec_dz = _dfz(zz) * (ecp - ecu)
    e = ex + ec
    de_drs = dex_drs + dec_drs
    de_dz = dex_dz + dec_dz
    common = e - rs / 3.0 * de_drs
    eps[ok] = e
    vu[ok] = common + (1.0 - zz) * de_dz
    vd[ok] = common - (1.0 + zz) * de_dz
    return eps, vu, vd


def lda_xc(rho: np.ndarray, m: Optional[np.ndarray] = None):
    """V_xc = dE_xc/drho, B_xc = dE_xc/dm (3, ...) and E_xc per unit volume
    (rho eps_xc) of the local spin density approximation; zeta = |m| / rho."""
    if m is None:
        m = np.zeros((3,) + rho.shape)
    mn = np.sqrt(np.sum(m * m, axis=0))
    zeta = np.where(rho > _RHO_MIN, mn / np.maximum(rho, _RHO_MIN), 0.0)
    eps, vu, vd = lda_eps(rho, zeta)
    vxc = 0.5 * (vu + vd)
    bm = 0.5 * (vu - vd)
    unit = np.where(mn > 0, m / np.where(mn > 0, mn, 1.0), 0.0)
    return vxc, bm * unit, rho * eps


def fermi(eps: np.ndarray, n_el: float, kT: float):
    """Occupations f_i in [0, 1] with sum f_i = n_el (bisection on mu)."""
    eps = np.asarray(eps, dtype=np.float64)
    if not (0 < n_el < len(eps)):
        raise ValueError("n_el must lie strictly between 0 and the number of bands")

    def occ(mu):
        x = np.clip((eps - mu) / kT, -700.0, 700.0)
        return 1.0 / (1.0 + np.exp(x))
    lo, hi = eps.min() - 50 * kT - 1.0, eps.max() + 50 * kT + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if occ(mid).sum() < n_el:
            lo = mid
        else:
            hi = mid
    mu = 0.5 * (lo + hi)
    return occ(mu), mu


def entropy(f: np.ndarray) -> float:
    """S / k_B = -sum [f ln f + (1 - f) ln(1 - f)]."""
    f = np.clip(np.asarray(f, dtype=np.float64), 1e-300, 1.0)
    g = np.clip(1.0 - f, 1e-300, 1.0)
    return float(-np.sum(f * np.log(f) + g * np.log(g)))


class Anderson:
    """Anderson mixing of a vector fixed point x = g(x) with a preconditioned
    step: keeps the last ``depth`` pairs (x_j, r_j = g(x_j) - x_j); the next
    input is  x_bar + alpha P[r_bar]  with  x_bar = x - dX gamma,
    r_bar = r - dR gamma,  gamma = argmin |r - dR gamma|_2  (dX, dR the
    differences of successive stored pairs)."""

    def __init__(self, depth: int = 6, alpha: float = 0.5, precond=None):
        self.depth, self.alpha = depth, alpha
        self.precond = precond if precond is not None else (lambda r: r)
        self.xs: List[np.ndarray] = []
        self.rs: List[np.ndarray] = []

    def step(self, x: np.ndarray, r: np.ndarray) -> np.ndarray:
        self.xs.append(x.ravel().copy())
        self.rs.append(r.ravel().copy())
        if len(self.xs) > self.depth + 1:
            self.xs.pop(0)
            self.rs.pop(0)
        xb, rb = self.xs[-1].copy(), self.rs[-1].copy()
        k = len(self.xs) - 1
        if k > 0:
            dX = np.stack([self.xs[j + 1] - self.xs[j] for j in range(k)], axis=1)
            dR = np.stack([self.rs[j + 1] - self.rs[j] for j in range(k)], axis=1)
            gamma = _small_lsq(dR, rb)
            xb = xb - dX @ gamma
            rb = rb - dR @ gamma
        return (xb + self.alpha * self.precond(rb.reshape(x.shape)).ravel()).reshape(x.shape)


def _small_lsq(dR: np.ndarray, r: np.ndarray) -> np.ndarray:
    """argmin |r - dR g|_2 through the normal equations with a relative
    Tikhonov term of 1e-12 of the trace (the history can be nearly dependent)."""
    A = dR.T @ dR
    b = dR.T @ r
    A = A + 1e-12 * max(np.trace(A), 1e-300) * np.eye(A.shape[0])
    return np.linalg.solve(A, b)


@dataclasses.dataclass
class ScfResult:
    v: np.ndarray            # self-consistent V_in (natural grid)
    eigvals: np.ndarray      # lowest n positive-band eigenvalues of H[v]
    occ: np.ndarray
    mu: float
    rho: np.ndarray
    m: np.ndarray
    residuals: List[float]   # ||V_out - V_in|| / ||V_in|| per step
    free_energy: float
    converged: bool


def _operator_with(system, v, k_index=0):
    return dks.DKSOperator(dataclasses.replace(system, v_loc=np.asarray(v, dtype=np.float64)), k_index)


def free_energy(eps, f, v_in, v_ext, rho, vh, exc_density, omega, kT) -> float:
    ng = rho.size
    dv = omega / ng
    e_band = float(np.dot(f, eps))
    dc = float(np.sum((v_in - v_ext) * rho)) * dv
    e_h = 0.5 * float(np.sum(vh * rho)) * dv
    e_xc = float(np.sum(exc_density)) * dv
    return e_band - dc + e_h + e_xc - kT * entropy(f)


def lowest_states(system, v, n: int, model: str = "dks"):
    """The n lowest eigenpairs of the operator with local potential v: the
    positive band of the DKS operator (model "dks"), or the two-component
    Kohn-Sham operator with spin-orbit coupling (model "ksso", Table 1),
    whose spinors are returned with zero small components."""
    op = _operator_with(system, v)
    if model == "dks":
        eps, vec = lobpcgf.lowest_positive(op.dense(), n, system.c)
        return op, eps, vec.T.reshape(n, 4, op.N)
    w, vec = np.linalg.eigh(op.pauli_dense())
    X = np.zeros((n, 4, op.N), dtype=np.complex128)
    X[:, :2] = vec[:, :n].T.reshape(n, 2, op.N)
    return op, w[:n], X


def scf(system, n: int, n_el: float, temperature: float = 5000.0, tol: float = 1e-8,
        max_iter: int = 60, depth: int = 6, alpha: float = 0.5, q0: float = 0.8,
        model: str = "dks") -> ScfResult:
    """The SCF loop with exact eigenpairs of each H[V_in] (the dense definition
    of Algorithm 1's answer), the n lowest states (of the positive band for
    DKS) occupied by n_el electrons at `temperature` (K).  The sigma.B_xc term
    of Eq. (DKS) is left out of H: the densities here are Kramers-paired and
    carry no spin density (B_xc = 0), which the tests check."""
    v_ext = np.asarray(system.v_loc, dtype=np.float64)
    omega = cell_volume(system.lattice)
    kT = K_BOLTZMANN * temperature
    mix = Anderson(depth, alpha, lambda r: kerker(r, system.lattice, q0))
    v_in = v_ext.copy()
    res: List[float] = []
    for it in range(max_iter):
        op, eps, X = lowest_states(system, v_in, n, model)
        f, mu = fermi(eps, n_el, kT)
        rho, m = density(op, X, f)
        vh = hartree(rho, system.lattice)
        vxc, bxc, exc = lda_xc(rho, m)
        v_out = v_ext + vh + vxc
        r = v_out - v_in
        res.append(float(np.linalg.norm(r) / np.linalg.norm(v_in)))
        F = free_energy(eps, f, v_in, v_ext, rho, vh, exc, omega, kT)
        if res[-1] < tol:
            return ScfResult(v_in, eps, f, mu, rho, m, res, F, True)
        if it + 1 == max_iter:
            break
        v_in = mix.step(v_in, r)
    return ScfResult(v_in, eps, f, mu, rho, m, res, F, False)
