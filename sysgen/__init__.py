"""Seeded synthetic inputs for the four-component planewave Dirac-Kohn-Sham
eigenproblem.

This module produces *physical inputs only*: lattice, k-points, cutoff, FFT
grid, speed of light, atom positions, the local potential sampled on the grid,
projector radii and the real symmetric coupling matrices of the separable
spin-orbit projectors, and the large-component start block of the iteration.
It holds none of the method's arithmetic (no Hamiltonian, no basis tables
beyond counting planewaves to size a workload, no filter, no eigen-solver), so
that the test oracle and the GPU library can both consume it while sharing no
code with each other.

The workloads stand in for the paper's Pt2/Au2/TlF dimers and the layered
Bi2Se3 crystal (Sec. 4.1, Table 2); the paper's HGH pseudopotential data are
replaced by atom-centred Gaussians and Gaussian-radial projectors.

Random draws use ``numpy.random.default_rng(seed)`` in a fixed order:
atom positions (when random) -> potential noise (C order) -> coupling matrices
(atom, l, then D+ before D-, upper triangle row-major).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

C_LIGHT = 137.036


@dataclasses.dataclass
class ProjGroup:
    """One (atom, l) block of separable projectors.

    ``d_plus``/``d_minus`` are real symmetric ``n_rad x n_rad`` couplings (Ha)
    of the j = l + 1/2 and j = l - 1/2 channels; ``r_l`` is the radial scale
    (bohr) of the Gaussian radial functions.
    """
    atom: int
    l: int
    n_rad: int
    r_l: float
    d_plus: np.ndarray
    d_minus: np.ndarray


@dataclasses.dataclass
class System:
    """A fully specified synthetic DKS eigenproblem (all FP64, Hartree a.u.)."""
    name: str
    lattice: np.ndarray          # 3x3, rows a1, a2, a3 (bohr)
    kpts: np.ndarray             # nk x 3 Cartesian (bohr^-1)
    ecut: float                  # Ha; basis is |k+G|^2/2 <= ecut
    grid: tuple                  # (N1, N2, N3)
    c: float                     # speed of light
    v_loc: np.ndarray            # (N1, N2, N3) real, on r_j = (j/N) . A, j3 fastest
    tau: np.ndarray              # natom x 3 Cartesian positions (bohr)
    proj: List[ProjGroup]
    n_bands: int
    seed: int = 0

    @property
    def natom(self) -> int:
        return int(self.tau.shape[0])


# --------------------------------------------------------------------------
# helpers (geometry only)
# --------------------------------------------------------------------------

def grid_points(lattice: np.ndarray, grid) -> np.ndarray:
    """Cartesian r_j = (j1/N1, j2/N2, j3/N3) . A, shape (N1, N2, N3, 3)."""
    n1, n2, n3 = grid
    f1 = np.arange(n1) / n1
    f2 = np.arange(n2) / n2
    f3 = np.arange(n3) / n3
    frac = np.stack(np.meshgrid(f1, f2, f3, indexing="ij"), axis=-1)
    return frac @ lattice


def gaussian_potential(lattice, grid, tau, depths, widths) -> np.ndarray:
    """Sum over atoms and periodic images of depth * exp(-|r - tau - R|^2 / (2 w^2)).

    Each image contributes on the window of grid points within
    w * sqrt(2 ln 1e16) of its centre, beyond which every term is below 1e-16
    of the depth.
    """
    lattice = np.asarray(lattice, dtype=np.float64)
    n = np.array(grid)
    v = np.zeros(grid, dtype=np.float64)
    ainv = np.linalg.inv(lattice)                # r . ainv = fractional coords
    hfrac = np.linalg.norm(ainv, axis=0)          # fractional extent per unit length
    for a in range(tau.shape[0]):
        w = float(widths[a])
        rc = w * math.sqrt(2.0 * math.log(1e16))
        f0 = np.asarray(tau[a], dtype=np.float64) @ ainv
        ext = rc * hfrac
        ranges = [range(int(math.floor(-f0[d] - ext[d])) - 1,
                        int(math.ceil(1.0 - f0[d] + ext[d])) + 1) for d in range(3)]
        for i in ranges[0]:
            for j in ranges[1]:
                for k in ranges[2]:
                    fc = f0 + np.array([i, j, k], dtype=np.float64)
                    lo = np.maximum(np.ceil((fc - ext) * n).astype(int), 0)
                    hi = np.minimum(np.floor((fc + ext) * n).astype(int), n - 1)
                    if np.any(hi < lo):
                        continue
                    idx = [np.arange(lo[d], hi[d] + 1) for d in range(3)]
                    fr = np.stack(np.meshgrid(idx[0] / n[0], idx[1] / n[1], idx[2] / n[2],
                                              indexing="ij"), axis=-1)
                    d = (fr - fc) @ lattice
                    r2 = np.einsum("...i,...i->...", d, d)
                    v[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] += \
                        depths[a] * np.exp(-r2 / (2.0 * w * w))
    return v


def _sym_matrix(rng, n, lo=-2.0, hi=2.0) -> np.ndarray:
    m = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            m[i, j] = m[j, i] = rng.uniform(lo, hi)
    return m


def _draw_projectors(rng, natom, lmax_per_atom, n_rad, radii) -> List[ProjGroup]:
    groups = []
    for a in range(natom):
        for l in range(lmax_per_atom[a] + 1):
            dp = _sym_matrix(rng, n_rad)
            dm = _sym_matrix(rng, n_rad)
            groups.append(ProjGroup(atom=a, l=l, n_rad=n_rad, r_l=float(radii[a]),
                                    d_plus=dp, d_minus=dm))
    return groups


def smooth_size(nmin: int) -> int:
    """Smallest 2^a 3^b 5^c >= nmin."""
    n = max(1, nmin)
    while True:
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return n
        n += 1


def cubic(L: float) -> np.ndarray:
    return np.diag([L, L, L]).astype(np.float64)


def hexagonal(a: float, c: float) -> np.ndarray:
    return np.array([[a, 0.0, 0.0],
                     [-0.5 * a, 0.5 * math.sqrt(3.0) * a, 0.0],
                     [0.0, 0.0, c]], dtype=np.float64)


def reciprocal(lattice: np.ndarray) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij (geometry of the cell)."""
    return 2.0 * math.pi * np.linalg.inv(lattice).T


def monkhorst_pack(lattice, n1, n2, n3) -> np.ndarray:
    """Shifted Monkhorst-Pack grid in Cartesian coordinates."""
    b = reciprocal(lattice)
    ks = []
    for i in range(n1):
        for j in range(n2):
            for k in range(n3):
                f = np.array([(2 * i - n1 + 1) / (2.0 * n1),
                              (2 * j - n2 + 1) / (2.0 * n2),
                              (2 * k - n3 + 1) / (2.0 * n3)])
                ks.append(f @ b)
    return np.array(ks)


def miller_box(lattice: np.ndarray, kpt, ecut: float) -> np.ndarray:
    """All integer triples whose |k + n.B| could be <= sqrt(2 ecut) (a superset)."""
    qmax = math.sqrt(2.0 * ecut) + float(np.linalg.norm(kpt))
    lens = np.linalg.norm(lattice, axis=1)
    nb = [int(math.floor(qmax * l / (2.0 * math.pi))) + 1 for l in lens]
    r = [np.arange(-m, m + 1) for m in nb]
    g = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    return g


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def tiny_dimer(seed: int = 0, c: float = C_LIGHT, noise: float = 0.01,
               with_nonlocal: bool = True, ecut: float = 5.0,
               grid=(24, 24, 24), n_bands: int = 8) -> System:
    """Cubic 10 bohr cell, Gamma, Ecut 5 Ha, 24^3 grid, dimer 2.5 bohr along z.

    Gaussians of depth -20 Ha and width 0.8 bohr, U(-0.01, 0.01) noise,
    l = 0, 1 projectors with one radial function, couplings U(-2, 2) Ha.
    """
    rng = np.random.default_rng(seed)
    A = cubic(10.0)
    tau = np.array([[5.0, 5.0, 3.75], [5.0, 5.0, 6.25]])
    v = gaussian_potential(A, grid, tau, [-20.0, -20.0], [0.8, 0.8])
    v = v + rng.uniform(-noise, noise, size=grid) if noise > 0 else v
    proj = _draw_projectors(rng, 2, [1, 1], 1, [0.8, 0.8]) if with_nonlocal else []
    return System("tiny_dimer", A, np.zeros((1, 3)), ecut, tuple(grid), c, v, tau,
                  proj, n_bands, seed)


def heavy_dimer(seed: int = 0, c: float = C_LIGHT) -> System:
    """Cubic 20 bohr cell, Gamma, Ecut 30 Ha, 96^3 grid, 40 bands.

    Gaussians of depth -80 Ha and width 0.4 bohr (2.5 bohr bond along z, centred),
    U(-0.01, 0.01) noise, l = 0..2 projectors with two radial functions each.
    """
    rng = np.random.default_rng(seed)
    A = cubic(20.0)
    tau = np.array([[10.0, 10.0, 8.75], [10.0, 10.0, 11.25]])
    grid = (96, 96, 96)
    v = gaussian_potential(A, grid, tau, [-80.0, -80.0], [0.4, 0.4])
    v = v + rng.uniform(-0.01, 0.01, size=grid)
    proj = _draw_projectors(rng, 2, [2, 2], 2, [0.4, 0.4])
    return System("heavy_dimer", A, np.zeros((1, 3)), 30.0, grid, c, v, tau, proj, 40, seed)


def layered_crystal(seed: int = 0, c: float = C_LIGHT, nk=(4, 4, 1)) -> System:
    """Hexagonal a = 7.8, c = 54 bohr, 5 atoms in quintuple-layer positions,
    Ecut 25 Ha, 48x48x320 grid, 120 bands, shifted Monkhorst-Pack k grid.
    """
    rng = np.random.default_rng(seed)
    A = hexagonal(7.8, 54.0)
    d1 = rng.uniform(3.6, 4.0)
    d2 = d1 + rng.uniform(3.6, 4.0)
    zc = 27.0
    zs = [zc - d2, zc - d1, zc, zc + d1, zc + d2]
    inplane = [(0, 0), (1 / 3, 2 / 3), (2 / 3, 1 / 3), (0, 0), (1 / 3, 2 / 3)]
    tau = np.array([[f1, f2, z / 54.0] for (f1, f2), z in zip(inplane, zs)]) @ A
    depths = [-30.0, -45.0, -30.0, -45.0, -30.0]
    widths = [0.7, 0.6, 0.7, 0.6, 0.7]
    grid = (48, 48, 320)
    v = gaussian_potential(A, grid, tau, depths, widths)
    v = v + rng.uniform(-0.01, 0.01, size=grid)
    proj = _draw_projectors(rng, 5, [2] * 5, 2, widths)
    kp = monkhorst_pack(A, *nk)
    return System("layered_crystal", A, kp, 25.0, grid, c, v, tau, proj, 120, seed)


def _sphere_count(A, ecut) -> int:
    b = reciprocal(A)
    g = miller_box(A, np.zeros(3), ecut)
    q = g @ b
    return int(np.count_nonzero(0.5 * np.einsum("ij,ij->i", q, q) <= ecut))


def _sphere_nmax(A, ecut) -> np.ndarray:
    b = reciprocal(A)
    g = miller_box(A, np.zeros(3), ecut)
    q = g @ b
    inside = 0.5 * np.einsum("ij,ij->i", q, q) <= ecut
    return np.abs(g[inside]).max(axis=0)


def uneven_batch(seed: int = 0, count: int = 64, c: float = C_LIGHT,
                 npw_range=(500, 8000)) -> List[System]:
    """Independent cubic systems of uneven size: L in [8, 16] bohr, Ecut in
    [5, 20] Ha (rejection-sampled so that the sphere holds npw_range planewaves),
    1-4 atoms, 8-64 bands; grid per axis = smallest 2^a3^b5^c >= 4 n_max + 1.
    """
    rng = np.random.default_rng(seed)
    systems = []
    for s in range(count):
        while True:
            L = rng.uniform(8.0, 16.0)
            ecut = rng.uniform(5.0, 20.0)
            A = cubic(L)
            npw = _sphere_count(A, ecut)
            if npw_range[0] <= npw <= npw_range[1]:
                break
        nmax = _sphere_nmax(A, ecut)
        grid = tuple(smooth_size(4 * int(m) + 1) for m in nmax)
        natom = int(rng.integers(1, 5))
        tau = rng.uniform(0.0, L, size=(natom, 3))
        depths = rng.uniform(-40.0, -10.0, size=natom)
        widths = rng.uniform(0.5, 1.0, size=natom)
        lmax = [int(rng.integers(0, 3)) for _ in range(natom)]
        n_rad = int(rng.integers(1, 3))
        n_bands = int(rng.integers(1, 9)) * 8
        v = gaussian_potential(A, grid, tau, depths, widths)
        v = v + rng.uniform(-0.01, 0.01, size=grid)
        proj = _draw_projectors(rng, natom, lmax, n_rad, widths)
        systems.append(System(f"uneven_{s}", A, np.zeros((1, 3)), float(ecut), grid, c, v,
                              tau, proj, n_bands, seed))
    return systems


# --------------------------------------------------------------------------
# start block
# --------------------------------------------------------------------------

def start_block(miller: np.ndarray, lattice: np.ndarray, kpt, n: int, seed: int,
                noise: float = 1e-2) -> np.ndarray:
    """Large-component start block phi, shape (n, 2, N), in the order of ``miller``.

    Band b is a unit-weight planewave at the b-th lowest |k+G| (ties broken by
    the lexicographic Miller triple) with a seeded random spin direction, plus
    seeded complex noise of relative size ``noise`` on every coefficient.  All
    draws are made in lexicographic Miller order, so the block is the same
    function of the planewave set whatever order a caller lists it in.
    """
    miller = np.asarray(miller, dtype=np.int64)
    N = miller.shape[0]
    if n > N:
        raise ValueError("more bands than planewaves")
    lex = np.lexsort((miller[:, 2], miller[:, 1], miller[:, 0]))
    b = reciprocal(lattice)
    q = (miller[lex] @ b) + np.asarray(kpt)[None, :]
    q2 = np.round(np.einsum("ij,ij->i", q, q), 9)
    order = np.lexsort((np.arange(N), q2))       # stable: |q| then lexicographic
    rng = np.random.default_rng(seed + 7919)
    canon = np.zeros((n, 2, N), dtype=np.complex128)
    canon += noise * (rng.standard_normal((n, 2, N)) + 1j * rng.standard_normal((n, 2, N)))
    for band in range(n):
        theta = math.acos(rng.uniform(-1.0, 1.0))
        phi = rng.uniform(0.0, 2.0 * math.pi)
        canon[band, 0, order[band]] += math.cos(theta / 2.0)
        canon[band, 1, order[band]] += math.sin(theta / 2.0) * complex(math.cos(phi), math.sin(phi))
    out = np.empty_like(canon)
    out[:, :, lex] = canon
    return out
