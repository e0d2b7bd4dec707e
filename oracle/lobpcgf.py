"""LOBPCG-F (Algorithm 1) and the dense definition of its answer, in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``lowest_positive``   -- the answer Algorithm 1 returns, by definition: the n
                           lowest eigenpairs of the positive energy band of the
                           discretised operator (Alg. 1 'Output'; the band split
                           of Sec. 1: positive and negative bands separated by a
                           gap of width Delta ~ 2c^2).
* ``apply_filter``      -- f(H) Y = (H - C)^2 Y / Omega^2, Eq. (filter).
* ``filter_constants``  -- C in the negative continuum, Omega so that f = 1 at the
                           top of the positive band (Sec. 3.1 text after Eq. filter).
* ``block_rayleigh_ritz`` -- a locally optimal block iteration: Rayleigh-Ritz
                           on the current block, new directions from the
                           unconverged residuals, and a momentum block;
* ``lobpcgf``           -- Algorithm 1 as that iteration with the filter on
                           the start block and on every residual direction.
                           With ``use_filter=False`` it is the standard LOBPCG
                           the paper compares against.
* ``davidson_f``        -- the same filter inside a block Davidson iteration,
                           the other preconditioned solver the paper names for
                           it (Sec. 3 opening, Sec. 5).
* ``dirac_teter``       -- the preconditioner T of Alg. 1 ("solve T Y = R"):
                           the Teter-Payne-Allan factor that Sec. 4 employs in
                           both LOBPCG and LOBPCG-F, applied to a spinor
                           through the spectral projectors of the free Dirac
                           block of each planewave (a reading: the paper does
                           not say how the factor treats the small component).

Readings where the paper is silent (each listed in the design notes):
* complex data: the transposes of Alg. 1 are conjugate transposes;
* the residual test uses the absolute 2-norm of each column with ||x_i|| = 1;
* the columns of Y and P are scaled to unit norm before the Gram matrices are
  formed (this leaves the spanned subspace, hence the Ritz pairs, unchanged);
* optional buffer columns (``n_want`` < n): iterated with the block, not
  required to converge;
* HX and HP are carried by the same linear combinations as X and P
  (HX <- (HZ) V, HP <- [0, HY, HP] V), so each iteration applies H three times
  (twice inside the filter, once to Y), the count given in Sec. 3.2;
* the n Ritz pairs kept are the n lowest above the mid-gap -c^2 (Alg. 1's
  output is the lowest part of the positive band; in exact arithmetic every
  Ritz value of the filtered subspace lies there, and the selection keeps a
  rounding-level negative-band direction from entering X);
* if the Gram matrix of [X, Y, P] is not numerically positive definite, the
  iteration retries the Rayleigh-Ritz step without P.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla


def lowest_positive(H: np.ndarray, n: int, c: float):
    """Eigenvalues (ascending) and eigenvectors of the n lowest positive-band states.

    The positive band is everything above the middle of the gap, -c^2 in
    shifted units (the gap runs from about -2c^2 to 0).
    """
    w, v = np.linalg.eigh(H)
    pos = np.nonzero(w > -c * c)[0]
    if pos.size < n:
        raise ValueError("fewer positive-band states than requested")
    sel = pos[:n]
    return w[sel], v[:, sel]


def apply_filter(apply_h: Callable, Y: np.ndarray, C: float, Omega: float) -> np.ndarray:
    """f(H) Y with f(E) = (E - C)^2 / Omega^2 (Eq. filter): two applications of H."""
    W = apply_h(Y) - C * Y
    return (apply_h(W) - C * W) / (Omega * Omega)


def filter_constants(bounds, c: float):
    """(C, Omega) from analytic spectrum bounds (the paper gives no values).

    ``bounds`` = (e_kin_max, v_min, v_max, v_mean, nl_bound).  The free negative
    band spans [-2c^2 - e_kin_max, -2c^2]; C is put at its middle, moved by the
    mean local potential.  Omega = (upper bound of the positive band) - C, so
    f <= 1 on the positive band and f = 1 at (or just above) its top.
    """
    ekin, vmin, vmax, vmean, nl = bounds
    C = -2.0 * c * c - 0.5 * ekin + vmean
    top = ekin + vmax + nl
    return C, top - C


# ----------------------------------------------------------------------------
# Algorithm 1 as an instance of a generic block Rayleigh-Ritz iteration
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class LobpcgResult:
    eigvals: np.ndarray
    X: np.ndarray                  # K x n, columns are the eigenvectors
    resnorms: np.ndarray
    iterations: int
    converged: bool
    min_ritz_history: List[float]
    ritz_history: List[np.ndarray]
    dropped_p: int


def _unit_columns(M: np.ndarray):
    nrm = np.linalg.norm(M, axis=0)
    nrm[nrm == 0.0] = 1.0
    return M / nrm[None, :], nrm


def project(Z: np.ndarray, HZ: np.ndarray, n: int, floor: float = -math.inf):
    """Rayleigh-Ritz on span Z: the n lowest pairs above ``floor`` of the
    projected pencil (Z^H H Z) v = theta (Z^H Z) v, ascending.  Returns
    (theta_all, theta_n, V_n); raises LinAlgError when Z^H Z is not numerically
    positive definite or fewer than n Ritz values lie above the floor."""
    A = Z.conj().T @ HZ
    S = Z.conj().T @ Z
    A = 0.5 * (A + A.conj().T)
    S = 0.5 * (S + S.conj().T)
    theta, V = sla.eigh(A, S)
    keep = np.nonzero(theta > floor)[0][:n]
    if keep.size < n:
        raise np.linalg.LinAlgError("fewer than n Ritz values above the floor")
    return theta, theta[keep], V[:, keep]


def residuals(X: np.ndarray, HX: np.ndarray, lam: np.ndarray):
    """R = H X - X diag(lam) and the 2-norm of each column."""
    R = HX - X * lam[None, :]
    return R, np.linalg.norm(R, axis=0)


def block_rayleigh_ritz(apply_h: Callable, X0: np.ndarray, n: int, directions: Callable,
                        prepare: Optional[Callable] = None, n_iter: int = 100,
                        tol: float = 1e-8, n_want: Optional[int] = None,
                        max_history: int = 0, floor: float = -math.inf) -> LobpcgResult:
    """Locally optimal block iteration with Rayleigh-Ritz on three blocks.

    The subspace of each step is spanned by the current Ritz block X, new
    directions W = directions(R_a) built from the residual columns R_a that are
    not yet below tol (soft locking), and the momentum block P, the part of the
    previous step's update that came from outside X.  The n lowest Ritz pairs
    of that subspace form the next X.  ``prepare`` maps the start block before
    the first projection.  Convergence: the first ``n_want`` (default n)
    residual norms below tol; the remaining columns are buffer columns that are
    iterated but need not converge.  When the subspace's Gram matrix is not
    numerically positive definite the step is taken without P.  Only Ritz
    values above ``floor`` are kept.
    """
    n_want = n if n_want is None else n_want
    X = np.array(X0, dtype=np.complex128, copy=True)
    if prepare is not None:
        X = prepare(X)
    HX = apply_h(X)
    theta, lam, V = project(X, HX, n, floor)
    X, HX = X @ V, HX @ V
    R, norms = residuals(X, HX, lam)
    P = HP = None
    hist_min: List[float] = [float(theta.min())]
    hist: List[np.ndarray] = []
    dropped = 0
    it = 0
    converged = bool(np.all(norms[:n_want] < tol))
    while not converged and it < n_iter:
        it += 1
        active = np.nonzero(norms >= tol)[0]
        W, _ = _unit_columns(directions(R[:, active]))
        HW = apply_h(W)
        extra = [W] if P is None else [W, P]
        hextra = [HW] if P is None else [HW, HP]
        try:
            Z = np.concatenate([X] + extra, axis=1)
            HZ = np.concatenate([HX] + hextra, axis=1)
            theta, lam, V = project(Z, HZ, n, floor)
        except np.linalg.LinAlgError:
            if P is None:
                raise
            dropped += 1
            Z = np.concatenate([X, W], axis=1)
            HZ = np.concatenate([HX, HW], axis=1)
            theta, lam, V = project(Z, HZ, n, floor)
        hist_min.append(float(theta.min()))
        if max_history:
            hist.append(theta.copy())
        X, HX = Z @ V, HZ @ V
        R, norms = residuals(X, HX, lam)
        converged = bool(np.all(norms[:n_want] < tol))
        if converged:
            break
        # momentum: the new combination of the non-X blocks, for the columns
        # still active
        nx = X.shape[1]
        keep = V[nx:, :][:, np.nonzero(norms >= tol)[0]]
        P, pn = _unit_columns(Z[:, nx:] @ keep)
        HP = (HZ[:, nx:] @ keep) / pn[None, :]
    return LobpcgResult(lam, X, norms, it, converged, hist_min, hist, dropped)


def lobpcgf(apply_h: Callable, X0: np.ndarray, n: int, C: float, Omega: float,
            n_init: int = 3, n_iter: int = 100, tol: float = 1e-8,
            use_filter: bool = True, precond: Optional[Callable] = None,
            max_history: int = 0, n_want: Optional[int] = None,
            half_gap: Optional[float] = None) -> LobpcgResult:
    """Algorithm 1 (LOBPCG-F) on the K x n start block X0 (columns = spinors,
    K = 4N): the block iteration above with the filter f(H) applied n_init
    times to the start block and to every preconditioned residual.  With
    ``use_filter=False`` it is the standard LOBPCG of the paper's comparison.

    ``apply_h`` maps a K x m block to H times it.  ``precond`` solves T Y = R
    (identity when None, as in the analysis of Sec. 3.1).  ``half_gap`` (c^2 in
    the shifted units) places the mid-gap below which LOBPCG-F keeps no Ritz
    value; None keeps the n lowest.
    """
    def f_of_h(Y):
        return apply_filter(apply_h, Y, C, Omega)

    def prepare(X):
        if use_filter:
            for _ in range(n_init):
                X, _ = _unit_columns(f_of_h(X))
        return X

    def directions(R):
        Y = R if precond is None else precond(R)
        return f_of_h(Y) if use_filter else Y

    # LOBPCG-F keeps the n lowest Ritz pairs of the positive band, above the
    # mid-gap -c^2 (in exact arithmetic every Ritz value of the filtered
    # subspace is there); plain LOBPCG keeps the n lowest of all
    floor = -half_gap if use_filter and half_gap is not None else -math.inf
    return block_rayleigh_ritz(apply_h, X0, n, directions, prepare=prepare, n_iter=n_iter,
                               tol=tol, n_want=n_want, max_history=max_history, floor=floor)


def teter_factor(x: np.ndarray) -> np.ndarray:
    """The Teter-Payne-Allan factor p / (p + 16 x^4), p = 27 + 18x + 12x^2 +
    8x^3, of the kinetic energy ratio x (1 at x = 0, ~1/(2x) for large x)."""
    p = 27.0 + 18.0 * x + 12.0 * x * x + 8.0 * x ** 3
    return p / (p + 16.0 * x ** 4)


def dirac_teter(R: np.ndarray, q: np.ndarray, c: float, ncomp: int = 4,
                E: Optional[np.ndarray] = None, e_min: float = 1e-3) -> np.ndarray:
    """T R for the K x m residual block R (columns = spinors, components
    phi_up, phi_dn, chi_up, chi_dn of N planewaves each; K = ncomp N), q the
    N x 3 wave vectors k+G (Sec. 4: the Teter preconditioner in both solvers;
    Alg. 1: T Y = R).

    At each planewave the free Dirac block (shifted by -c^2, as the operator)
    [[0, c s.q], [c s.q, -2c^2]] has the eigenvalues e+ = sqrt(c^4 + c^2 q^2)
    - c^2 and e- = -sqrt(c^4 + c^2 q^2) - c^2, each twice, with the spectral
    projectors P+- = (1 +- (M + c^2)/sqrt(c^4 + c^2 q^2)) / 2.  T multiplies
    P+ R by the Teter factor of e+ / E and P- R by that of |e-| / E, with E per
    column the mean e+ of the residual's positive part (at least e_min).  T is
    Hermitian positive definite (for fixed E) and keeps the spinor structure
    of the free positive and negative states.  For ncomp = 2 (the
    two-component operator, no small component) it is the plain Teter factor
    of |k+G|^2 / 2.  ``E`` (optional, length m) fixes the energies.
    """
    N = q.shape[0]
    m = R.shape[1]
    Rr = R.T.reshape(m, ncomp, N)
    q2 = np.einsum("ij,ij->i", q, q)
    if ncomp == 2:
        ep = 0.5 * q2
        Pp = Rr
        Pm = np.zeros_like(Rr)
        em_abs = ep
    else:
        root = np.sqrt(c ** 4 + c * c * q2)
        ep = c * c * q2 / (root + c * c)          # e+ without cancellation
        em_abs = root + c * c                      # |e-|
        qx, qy, qz = q[:, 0], q[:, 1], q[:, 2]

        def sdot(u):                               # (sigma . q) u on a two-spinor
            a, b = u[:, 0], u[:, 1]
            return np.stack([qz * a + (qx - 1j * qy) * b, (qx + 1j * qy) * a - qz * b], axis=1)

        phi, chi = Rr[:, :2], Rr[:, 2:]
        shifted = np.concatenate([c * c * phi + c * sdot(chi), c * sdot(phi) - c * c * chi], axis=1)
        Pp = 0.5 * (Rr + shifted / root[None, None, :])
        Pm = Rr - Pp
    if E is None:
        w = np.sum(np.abs(Pp) ** 2, axis=1)        # m x N
        den = w.sum(axis=1)
        num = w @ ep
        E = np.where(den > 0, num / np.where(den > 0, den, 1.0), e_min)
        E = np.maximum(E, e_min)
    E = np.asarray(E, dtype=float)
    out = (Pp * teter_factor(ep[None, :] / E[:, None])[:, None, :] +
           Pm * teter_factor(em_abs[None, :] / E[:, None])[:, None, :])
    return out.reshape(m, ncomp * N).T


def davidson_f(apply_h: Callable, X0: np.ndarray, n: int, C: float, Omega: float,
               n_init: int = 3, n_iter: int = 200, tol: float = 1e-8,
               use_filter: bool = True, max_dim: Optional[int] = None,
               n_want: Optional[int] = None, half_gap: Optional[float] = None) -> LobpcgResult:
    """Block Davidson with the filter as its preconditioner (Sec. 3 opening,
    Sec. 5: the filter serves any preconditioned iterative solver).

    The search space V starts as the start block after n_init filter
    applications.  Each step: Rayleigh-Ritz on span V (the n lowest pairs above
    the mid-gap, as in Algorithm 1), the Ritz block X and its residuals R, and,
    for the columns whose residual norm is not below tol, the new directions
    f(H) R appended to V.  When V would exceed ``max_dim`` columns (default
    4n) it restarts from X.  Nothing is discarded between restarts, so the
    space keeps every direction the filter produced.  If the Gram matrix of V
    is not numerically positive definite the step restarts from the last X
    and its new directions.
    """
    n_want = n if n_want is None else n_want
    max_dim = 4 * n if max_dim is None else max_dim

    def f_of_h(Y):
        return apply_filter(apply_h, Y, C, Omega)

    floor = -half_gap if use_filter and half_gap is not None else -math.inf
    V = np.array(X0, dtype=np.complex128, copy=True)
    if use_filter:
        for _ in range(n_init):
            V, _ = _unit_columns(f_of_h(V))
    HV = apply_h(V)
    hist_min: List[float] = []
    dropped = 0
    it = 0
    X = HX = W = HW = None
    while True:
        try:
            theta, lam, Vz = project(V, HV, n, floor)
        except np.linalg.LinAlgError:
            if X is None or V.shape[1] <= n + W.shape[1]:
                raise
            dropped += 1
            V = np.concatenate([X, W], axis=1)
            HV = np.concatenate([HX, HW], axis=1)
            theta, lam, Vz = project(V, HV, n, floor)
        hist_min.append(float(theta.min()))
        X, HX = V @ Vz, HV @ Vz
        R, norms = residuals(X, HX, lam)
        converged = bool(np.all(norms[:n_want] < tol))
        if converged or it >= n_iter:
            break
        it += 1
        active = np.nonzero(norms >= tol)[0]
        Y = R[:, active]
        W, _ = _unit_columns(f_of_h(Y) if use_filter else Y)
        HW = apply_h(W)
        if V.shape[1] + W.shape[1] > max_dim:
            V, HV = X, HX
        V = np.concatenate([V, W], axis=1)
        HV = np.concatenate([HV, HW], axis=1)
    return LobpcgResult(lam, X, norms, it, converged, hist_min, [], dropped)


# ----------------------------------------------------------------------------
# helpers to run Algorithm 1 on a DKSOperator
# ----------------------------------------------------------------------------

def block_apply(op) -> Callable:
    """Wrap DKSOperator.apply for K x m column blocks (component-major columns)."""
    N = op.N

    def apply_h(M):
        m = M.shape[1]
        X = M.T.reshape(m, 4, N)
        return op.apply(X).reshape(m, 4 * N).T
    return apply_h


def kinetic_balance(op, phi: np.ndarray) -> np.ndarray:
    """Start block from large components phi (n, 2, N) via kinetic balance.

    Eq. (RKB) builds the small component from the large one with sigma.p / (2mc);
    the exact free positive-energy spinor uses c sigma.q / (E_q + c^2) with
    E_q = sqrt(c^2 q^2 + c^4), which equals sigma.q/(2c) as q -> 0.  Returns a
    (n, 4, N) block.
    """
    c = op.c
    qx, qy, qz = op.q[:, 0], op.q[:, 1], op.q[:, 2]
    eq = np.sqrt(c * c * np.einsum("ij,ij->i", op.q, op.q) + c ** 4)
    fac = c / (eq + c * c)
    out = np.zeros((phi.shape[0], 4, op.N), dtype=np.complex128)
    out[:, 0:2] = phi
    out[:, 2] = fac * (qz * phi[:, 0] + (qx - 1j * qy) * phi[:, 1])
    out[:, 3] = fac * ((qx + 1j * qy) * phi[:, 0] - qz * phi[:, 1])
    return out


def solve(op, n: int, X0: Optional[np.ndarray] = None, phi0: Optional[np.ndarray] = None,
          C: Optional[float] = None, Omega: Optional[float] = None, method: str = "lobpcg",
          **kw) -> LobpcgResult:
    """Run Algorithm 1 (method "lobpcg") or the filtered block Davidson
    (method "davidson") on ``op`` for the n lowest positive-band states."""
    if X0 is None:
        X0 = kinetic_balance(op, phi0)
    X0 = np.asarray(X0).reshape(X0.shape[0], -1).T
    if C is None or Omega is None:
        C, Omega = filter_constants(op.spectrum_bounds(), op.c)
    kw.setdefault("half_gap", op.c * op.c)
    run = {"lobpcg": lobpcgf, "davidson": davidson_f}[method]
    return run(block_apply(op), X0, n, C, Omega, **kw)
