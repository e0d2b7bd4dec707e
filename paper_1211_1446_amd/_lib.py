"""ctypes binding of libdks (include/dks.h).  Argument marshalling only.

Device blocks are torch tensors on the GPU ([n][4][N] complex128 or complex64,
contiguous); the stream is torch's current stream unless one is passed.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libdks.so")

DKS_FP64, DKS_FP32 = 0, 1
MODE_FP64, MODE_MIXED_FP32, MODE_MIXED_BF16GRAM = 0, 1, 2
MODEL_DKS, MODEL_KSSO = 0, 1
METHOD_LOBPCG, METHOD_DAVIDSON = 0, 1
PRECOND_DEFAULT, PRECOND_NONE, PRECOND_TETER = -1, 0, 1

_STATUS = {0: "DKS_OK", -1: "DKS_EINVAL", -2: "DKS_ENOMEM", -3: "DKS_EHIP", -4: "DKS_ECHOL",
           -5: "DKS_ECOLLAPSE", -6: "DKS_EINTERNAL", 1: "DKS_WNOTCONV"}


class DksError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class _ProjGroup(ct.Structure):
    _fields_ = [("atom", ct.c_int), ("l", ct.c_int), ("n_rad", ct.c_int), ("r_l", ct.c_double),
                ("d_plus", ct.POINTER(ct.c_double)), ("d_minus", ct.POINTER(ct.c_double))]


class _SystemDesc(ct.Structure):
    _fields_ = [("lattice", ct.c_double * 9), ("nk", ct.c_int), ("kpts", ct.POINTER(ct.c_double)),
                ("ecut", ct.c_double), ("grid", ct.c_int * 3), ("c", ct.c_double),
                ("v_loc", ct.POINTER(ct.c_double)), ("natom", ct.c_int),
                ("tau", ct.POINTER(ct.c_double)), ("nproj_groups", ct.c_int),
                ("proj", ct.POINTER(_ProjGroup))]


class SolveOpts(ct.Structure):
    _fields_ = [("C", ct.c_double), ("Omega", ct.c_double), ("n_init", ct.c_int),
                ("n_iter", ct.c_int), ("tol", ct.c_double), ("mode", ct.c_int),
                ("mixed_tol", ct.c_double), ("mixed_iter", ct.c_int),
                ("kinetic_balance", ct.c_int), ("use_filter", ct.c_int),
                ("iter_ms", ct.POINTER(ct.c_double)), ("n_buffer", ct.c_int), ("model", ct.c_int),
                ("batch_graph", ct.c_int), ("graph_chunk", ct.c_int),
                ("item_buffer", ct.POINTER(ct.c_int)), ("method", ct.c_int),
                ("davidson_dim", ct.c_int), ("preconditioner", ct.c_int)]


class SolveInfo(ct.Structure):
    _fields_ = [("iterations", ct.c_int), ("iters_reduced", ct.c_int), ("converged", ct.c_int),
                ("n_converged", ct.c_int), ("h_applies", ct.c_int), ("basis_drops", ct.c_int),
                ("p_restarts", ct.c_int), ("neg_ritz_discarded", ct.c_int),
                ("min_ritz", ct.c_double), ("max_resnorm", ct.c_double),
                ("C", ct.c_double), ("Omega", ct.c_double),
                ("graph_iterations", ct.c_int), ("graph_exit", ct.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ScfOpts(ct.Structure):
    _fields_ = [("n_electrons", ct.c_double), ("temperature", ct.c_double), ("max_scf", ct.c_int),
                ("tol", ct.c_double), ("eig_iters", ct.c_int), ("n_init_first", ct.c_int),
                ("n_init_next", ct.c_int), ("anderson_depth", ct.c_int), ("alpha", ct.c_double),
                ("kerker_q0", ct.c_double), ("max_bxc", ct.c_double),
                ("history", ct.POINTER(ct.c_double)), ("eig_history", ct.POINTER(ct.c_double))]


class ScfInfo(ct.Structure):
    _fields_ = [("iterations", ct.c_int), ("eig_iterations", ct.c_int), ("converged", ct.c_int),
                ("eig_converged", ct.c_int), ("residual", ct.c_double), ("fermi", ct.c_double),
                ("free_energy", ct.c_double), ("e_hartree", ct.c_double), ("e_xc", ct.c_double),
                ("max_mag", ct.c_double), ("max_bxc", ct.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def library_path() -> str:
    return _LIBPATH


def _load():
    if not os.path.exists(_LIBPATH):
        raise ImportError(f"libdks.so not built at {_LIBPATH}; run __graft_entry__.build()")
    lib = ct.CDLL(_LIBPATH)
    vp, i, d = ct.c_void_p, ct.c_int, ct.c_double
    lib.dks_init_basis.argtypes = [ct.POINTER(_SystemDesc), i, i, ct.POINTER(vp)]
    lib.dks_num_systems.argtypes = [vp]
    lib.dks_basis_info.argtypes = [vp, i, ct.POINTER(i), ct.POINTER(i), ct.POINTER(i)]
    lib.dks_apply_H.argtypes = [vp, i, vp, vp, i, i, vp]
    lib.dks_apply_H_noalloc.argtypes = [vp, i, vp, vp, i, i, vp]
    lib.dks_apply_H_ksso.argtypes = [vp, i, vp, vp, i, i, vp]
    lib.dks_autotune.argtypes = [vp, i, ct.POINTER(i), ct.POINTER(i), i, vp]
    lib.dks_get_tuning.argtypes = [vp, i, ct.POINTER(i), ct.POINTER(i), ct.POINTER(i)]
    lib.dks_set_tuning.argtypes = [vp, i, i, i, i]
    lib.dks_apply_filter.argtypes = [vp, i, vp, vp, i, d, d, i, vp]
    lib.dks_precondition.argtypes = [vp, i, vp, i, i, i, vp]
    lib.dks_filter_constants.argtypes = [vp, i, ct.POINTER(d), ct.POINTER(d)]
    lib.dks_default_opts.argtypes = [ct.POINTER(SolveOpts)]
    lib.dks_default_opts.restype = None
    lib.dks_lobpcgf_solve.argtypes = [vp, i, i, vp, ct.POINTER(d), ct.POINTER(d),
                                      ct.POINTER(SolveOpts), ct.POINTER(SolveInfo), vp]
    lib.dks_lobpcgf_solve_batch.argtypes = [vp, i, ct.POINTER(i), ct.POINTER(i), ct.POINTER(vp),
                                            ct.POINTER(ct.POINTER(d)), ct.POINTER(ct.POINTER(d)),
                                            ct.POINTER(SolveOpts), ct.POINTER(SolveInfo), vp]
    lib.dks_density.argtypes = [vp, i, i, vp, i, ct.POINTER(d), vp, vp, vp]
    lib.dks_hartree.argtypes = [vp, i, vp, vp, vp]
    lib.dks_kerker.argtypes = [vp, i, vp, vp, d, vp]
    lib.dks_lda_xc.argtypes = [vp, i, vp, vp, vp, vp, vp, vp]
    lib.dks_get_local_potential.argtypes = [vp, i, vp, vp]
    lib.dks_set_local_potential.argtypes = [vp, i, vp, vp]
    lib.dks_scf_default_opts.argtypes = [ct.POINTER(ScfOpts)]
    lib.dks_scf_default_opts.restype = None
    lib.dks_scf.argtypes = [vp, i, i, vp, ct.POINTER(d), ct.POINTER(d), ct.POINTER(ScfOpts),
                            ct.POINTER(SolveOpts), ct.POINTER(ScfInfo), vp]
    lib.dks_free_basis.argtypes = [vp]
    lib.dks_free_basis.restype = None
    lib.dks_last_error.restype = ct.c_char_p
    lib.dks_profile_enable.argtypes = [i]
    lib.dks_profile_enable.restype = None
    lib.dks_profile_report.argtypes = [ct.c_char_p, ct.c_size_t]
    return lib


_lib = _load()


def _check(rc: int, allow_warning: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_warning):
        raise DksError(rc, _lib.dks_last_error().decode(errors="replace"))
    return rc


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


class Basis:
    """Owns a dks_basis handle and the host arrays it was built from."""

    def __init__(self, handle: int, keep):
        self.handle = ct.c_void_p(handle)
        self._keep = keep

    def close(self):
        if self.handle:
            _lib.dks_free_basis(self.handle)
            self.handle = ct.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def init_basis(systems: Sequence, device: int = 0) -> Basis:
    """dks_init_basis over objects with the fields of dks_system_desc
    (lattice, kpts, ecut, grid, c, v_loc, tau, proj[atom, l, n_rad, r_l, d_plus, d_minus])."""
    keep = []
    descs = (_SystemDesc * len(systems))()
    for di, s in enumerate(systems):
        D = descs[di]
        lat = np.ascontiguousarray(s.lattice, dtype=np.float64).reshape(9)
        for j in range(9):
            D.lattice[j] = float(lat[j])
        k = np.ascontiguousarray(s.kpts, dtype=np.float64).reshape(-1, 3)
        v = np.ascontiguousarray(s.v_loc, dtype=np.float64)
        tau = np.ascontiguousarray(s.tau, dtype=np.float64).reshape(-1, 3)
        keep += [k, v, tau]
        D.nk = k.shape[0]
        D.kpts = _dptr(k)
        D.ecut = float(s.ecut)
        for j in range(3):
            D.grid[j] = int(s.grid[j])
        D.c = float(s.c)
        D.v_loc = _dptr(v)
        D.natom = tau.shape[0]
        D.tau = _dptr(tau)
        groups = (_ProjGroup * max(1, len(s.proj)))()
        for gi, g in enumerate(s.proj):
            dp = np.ascontiguousarray(g.d_plus, dtype=np.float64)
            dm = np.ascontiguousarray(g.d_minus, dtype=np.float64)
            keep += [dp, dm]
            groups[gi].atom, groups[gi].l, groups[gi].n_rad = int(g.atom), int(g.l), int(g.n_rad)
            groups[gi].r_l = float(g.r_l)
            groups[gi].d_plus, groups[gi].d_minus = _dptr(dp), _dptr(dm)
        keep.append(groups)
        D.nproj_groups = len(s.proj)
        D.proj = ct.cast(groups, ct.POINTER(_ProjGroup))
    keep.append(descs)
    h = ct.c_void_p()
    _check(_lib.dks_init_basis(descs, len(systems), device, ct.byref(h)))
    return Basis(h.value, keep)


def free_basis(b: Basis) -> None:
    b.close()


def num_systems(b: Basis) -> int:
    return int(_lib.dks_num_systems(b.handle))


def basis_info(b: Basis, sys: int = 0, miller: bool = True):
    """(N, grid, miller (N x 3) or None)."""
    n = ct.c_int()
    grid = (ct.c_int * 3)()
    _check(_lib.dks_basis_info(b.handle, sys, ct.byref(n), grid, None))
    mil = None
    if miller:
        mil = np.zeros((n.value, 3), dtype=np.int32)
        _check(_lib.dks_basis_info(b.handle, sys, ct.byref(n), grid,
                                   mil.ctypes.data_as(ct.POINTER(ct.c_int))))
    return n.value, tuple(grid), mil


def _stream(stream):
    if stream is None:
        import torch
        return ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ct.c_void_p(stream.cuda_stream)
    return ct.c_void_p(stream)


def _prec_of(t) -> int:
    import torch
    if t.dtype == torch.complex128:
        return DKS_FP64
    if t.dtype == torch.complex64:
        return DKS_FP32
    raise TypeError("blocks must be complex128 or complex64")


def _check_block(t, nb, N, ncomp=4):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("blocks must be contiguous device tensors")
    if t.numel() < nb * ncomp * N:
        raise ValueError(f"block smaller than nb x {ncomp} x N")


def apply_H(b: Basis, sys: int, X, HX, nb: Optional[int] = None, stream=None) -> None:
    """HX = H X (dks_apply_H); X, HX torch tensors [nb][4][N]."""
    N, _, _ = basis_info(b, sys, miller=False)
    nb = X.shape[0] if nb is None else nb
    _check_block(X, nb, N)
    _check_block(HX, nb, N)
    if HX.dtype != X.dtype:
        raise TypeError("X and HX precision differ")
    _check(_lib.dks_apply_H(b.handle, sys, ct.c_void_p(X.data_ptr()), ct.c_void_p(HX.data_ptr()),
                            nb, _prec_of(X), _stream(stream)))


def apply_H_noalloc(b: Basis, sys: int, X, HX, nb: Optional[int] = None, stream=None) -> None:
    """HX = H X without any device allocation (dks_apply_H_noalloc)."""
    N, _, _ = basis_info(b, sys, miller=False)
    nb = X.shape[0] if nb is None else nb
    _check_block(X, nb, N)
    _check_block(HX, nb, N)
    if HX.dtype != X.dtype:
        raise TypeError("X and HX precision differ")
    _check(_lib.dks_apply_H_noalloc(b.handle, sys, ct.c_void_p(X.data_ptr()),
                                    ct.c_void_p(HX.data_ptr()), nb, _prec_of(X), _stream(stream)))


def apply_H_ksso(b: Basis, sys: int, X, HX, nb: Optional[int] = None, stream=None) -> None:
    """HX = H_KSSO X, the two-component operator (dks_apply_H_ksso); [nb][2][N]."""
    N, _, _ = basis_info(b, sys, miller=False)
    nb = X.shape[0] if nb is None else nb
    _check_block(X, nb, N, 2)
    _check_block(HX, nb, N, 2)
    if HX.dtype != X.dtype:
        raise TypeError("X and HX precision differ")
    _check(_lib.dks_apply_H_ksso(b.handle, sys, ct.c_void_p(X.data_ptr()),
                                 ct.c_void_p(HX.data_ptr()), nb, _prec_of(X), _stream(stream)))


def apply_filter(b: Basis, sys: int, Y, FY, C: float, Omega: float, nb: Optional[int] = None,
                 stream=None) -> None:
    """FY = (H - C)^2 Y / Omega^2 (dks_apply_filter)."""
    N, _, _ = basis_info(b, sys, miller=False)
    nb = Y.shape[0] if nb is None else nb
    _check_block(Y, nb, N)
    _check_block(FY, nb, N)
    _check(_lib.dks_apply_filter(b.handle, sys, ct.c_void_p(Y.data_ptr()),
                                 ct.c_void_p(FY.data_ptr()), nb, float(C), float(Omega),
                                 _prec_of(Y), _stream(stream)))


def precondition(b: Basis, sys: int, Y, model: int = 0, nb: Optional[int] = None,
                 stream=None) -> None:
    """Y <- T Y in place, the Teter preconditioner (dks_precondition); Y is
    [nb][4][N] for model 0 (DKS), [nb][2][N] for model 1 (KSSO)."""
    N, _, _ = basis_info(b, sys, miller=False)
    nb = Y.shape[0] if nb is None else nb
    _check_block(Y, nb, N, 4 if model == 0 else 2)
    _check(_lib.dks_precondition(b.handle, sys, ct.c_void_p(Y.data_ptr()), nb, int(model),
                                 _prec_of(Y), _stream(stream)))


def filter_constants(b: Basis, sys: int = 0):
    C, Om = ct.c_double(), ct.c_double()
    _check(_lib.dks_filter_constants(b.handle, sys, ct.byref(C), ct.byref(Om)))
    return C.value, Om.value


def autotune(b: Basis, systems: Sequence[int], nbs: Sequence[int], prec: int = DKS_FP64,
             stream=None) -> None:
    """Time and pick the launch shapes of H X for each system (dks_autotune)."""
    n = len(systems)
    if len(nbs) != n:
        raise ValueError("one band count per system")
    sa = (ct.c_int * max(n, 1))(*[int(v) for v in systems])
    na = (ct.c_int * max(n, 1))(*[int(v) for v in nbs])
    _check(_lib.dks_autotune(b.handle, n, sa, na, int(prec), _stream(stream)))


def get_tuning(b: Basis, sys: int) -> dict:
    """The launch shapes in use for system `sys` (dks_get_tuning)."""
    t, p, k = ct.c_int(), ct.c_int(), ct.c_int()
    _check(_lib.dks_get_tuning(b.handle, sys, ct.byref(t), ct.byref(p), ct.byref(k)))
    return {"tile_z": t.value, "plane_form": p.value, "ip_blocks": k.value}


def set_tuning(b: Basis, sys: int, tile_z: int, plane_form: int, ip_blocks: int) -> None:
    """Apply stored launch shapes to system `sys` (dks_set_tuning)."""
    _check(_lib.dks_set_tuning(b.handle, sys, int(tile_z), int(plane_form), int(ip_blocks)))


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    _lib.dks_default_opts(ct.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def profile_enable(on: bool = True) -> None:
    """Bracket every library kernel launch of this thread with HIP events."""
    _lib.dks_profile_enable(1 if on else 0)


def profile_report() -> dict:
    """{kernel: {"count", "total_ms"}} since the last report (synchronises the device)."""
    import json
    buf = ct.create_string_buffer(1 << 16)
    _check(_lib.dks_profile_report(buf, len(buf)))
    return json.loads(buf.value.decode())


def lobpcgf_solve(b: Basis, sys: int, n: int, X, opts: Optional[SolveOpts] = None, stream=None,
                  allow_notconv: bool = True, iter_ms: Optional[np.ndarray] = None):
    """Algorithm 1 on the complex128 device block X (in: X0, out: eigenvectors).

    ``iter_ms``: optional float64 array receiving the wall time of each
    main-loop iteration.  Returns (eigenvalues (n,), residual norms (n,), info
    dict, status)."""
    import torch
    if X.dtype != torch.complex128:
        raise TypeError("X must be complex128")
    N, _, _ = basis_info(b, sys, miller=False)
    o = opts if opts is not None else default_opts()
    _check_block(X, n, N, 2 if o.model == MODEL_KSSO else 4)
    lam = np.zeros(n)
    res = np.zeros(n)
    info = SolveInfo()
    if iter_ms is not None:
        need = o.n_iter + (o.mixed_iter if o.mode != MODE_FP64 else 0)
        if iter_ms.dtype != np.float64 or iter_ms.size < need or not iter_ms.flags.c_contiguous:
            raise ValueError(f"iter_ms must be a contiguous float64 array of >= {need} entries")
        o.iter_ms = _dptr(iter_ms)
    rc = _lib.dks_lobpcgf_solve(b.handle, sys, n, ct.c_void_p(X.data_ptr()), _dptr(lam), _dptr(res),
                                ct.byref(o), ct.byref(info), _stream(stream))
    _check(rc, allow_warning=allow_notconv)
    return lam, res, info.as_dict(), rc


def lobpcgf_solve_batch(b: Basis, systems: Sequence[int], ns: Sequence[int], Xs: Sequence,
                        opts: Optional[SolveOpts] = None, stream=None, allow_notconv: bool = True,
                        item_buffer: Optional[Sequence[int]] = None):
    """Algorithm 1 on several systems of one basis (dks_lobpcgf_solve_batch).
    ``item_buffer``: optional buffer-column count per item (overrides n_buffer).

    ``Xs[i]``: complex128 device block [ns[i]][4][N_i] (in: start block, out:
    eigenvectors).  Returns (list of eigenvalue arrays, list of residual arrays,
    list of info dicts, status)."""
    import torch
    nsys = len(systems)
    if not (len(ns) == nsys and len(Xs) == nsys):
        raise ValueError("systems, ns and Xs must have the same length")
    ncomp = 2 if (opts is not None and opts.model == MODEL_KSSO) else 4
    for s_, n_, X in zip(systems, ns, Xs):
        if X.dtype != torch.complex128:
            raise TypeError("every block must be complex128")
        N, _, _ = basis_info(b, int(s_), miller=False)
        _check_block(X, int(n_), N, ncomp)
    lams = [np.zeros(int(n_)) for n_ in ns]
    ress = [np.zeros(int(n_)) for n_ in ns]
    infos = (SolveInfo * max(nsys, 1))()
    sys_a = (ct.c_int * max(nsys, 1))(*[int(v) for v in systems])
    n_a = (ct.c_int * max(nsys, 1))(*[int(v) for v in ns])
    x_a = (ct.c_void_p * max(nsys, 1))(*[X.data_ptr() for X in Xs])
    dp = ct.POINTER(ct.c_double)
    l_a = (dp * max(nsys, 1))(*[a.ctypes.data_as(dp) for a in lams])
    r_a = (dp * max(nsys, 1))(*[a.ctypes.data_as(dp) for a in ress])
    o = opts if opts is not None else default_opts()
    if item_buffer is not None:
        if len(item_buffer) != nsys:
            raise ValueError("item_buffer needs one entry per item")
        buf_a = (ct.c_int * max(nsys, 1))(*[int(v) for v in item_buffer])
        o.item_buffer = ct.cast(buf_a, ct.POINTER(ct.c_int))
    rc = _lib.dks_lobpcgf_solve_batch(b.handle, nsys, sys_a, n_a, x_a, l_a, r_a, ct.byref(o),
                                      infos, _stream(stream))
    o.item_buffer = ct.POINTER(ct.c_int)()
    _check(rc, allow_warning=allow_notconv)
    return lams, ress, [infos[i].as_dict() for i in range(nsys)], rc


# ---- the self-consistent field loop ---------------------------------------

def _grid_shape(b: Basis, sys: int):
    _, grid, _ = basis_info(b, sys, miller=False)
    return tuple(int(g) for g in grid)


def _field(t, count, name):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() < count:
        raise ValueError(f"{name} must be a contiguous float64 device tensor of >= {count} values")
    return ct.c_void_p(t.data_ptr())


def density(b: Basis, sys: int, X, occ, model: int = MODEL_DKS, stream=None, with_mag: bool = True):
    """rho (N1, N2, N3) and m (3, N1, N2, N3) device tensors of the bands X with
    occupations occ (dks_density)."""
    import torch
    if X.dtype != torch.complex128:
        raise TypeError("X must be complex128")
    N, _, _ = basis_info(b, sys, miller=False)
    occ = np.ascontiguousarray(occ, dtype=np.float64)
    nb = occ.size
    _check_block(X, nb, N, 2 if model == MODEL_KSSO else 4)
    g = _grid_shape(b, sys)
    rho = torch.empty(g, dtype=torch.float64, device=X.device)
    mag = torch.empty((3,) + g, dtype=torch.float64, device=X.device) if with_mag else None
    _check(_lib.dks_density(b.handle, sys, model, ct.c_void_p(X.data_ptr()), nb, _dptr(occ),
                            ct.c_void_p(rho.data_ptr()),
                            ct.c_void_p(mag.data_ptr()) if mag is not None else None, _stream(stream)))
    return rho, mag


def hartree(b: Basis, sys: int, rho, out=None, stream=None):
    """V_H of the density rho (dks_hartree)."""
    import torch
    g = _grid_shape(b, sys)
    ng = int(np.prod(g))
    out = torch.empty(g, dtype=torch.float64, device=rho.device) if out is None else out
    _check(_lib.dks_hartree(b.handle, sys, _field(rho, ng, "rho"), _field(out, ng, "out"), _stream(stream)))
    return out


def kerker(b: Basis, sys: int, x, q0: float, out=None, stream=None):
    """The Kerker preconditioner G^2 / (G^2 + q0^2) of a grid field (dks_kerker)."""
    import torch
    g = _grid_shape(b, sys)
    ng = int(np.prod(g))
    out = torch.empty(g, dtype=torch.float64, device=x.device) if out is None else out
    _check(_lib.dks_kerker(b.handle, sys, _field(x, ng, "x"), _field(out, ng, "out"), float(q0),
                           _stream(stream)))
    return out


def lda_xc(b: Basis, sys: int, rho, mag=None, stream=None):
    """(v_xc, B_xc, rho eps_xc) of the local spin density approximation (dks_lda_xc)."""
    import torch
    g = _grid_shape(b, sys)
    ng = int(np.prod(g))
    vxc = torch.empty(g, dtype=torch.float64, device=rho.device)
    bxc = torch.empty((3,) + g, dtype=torch.float64, device=rho.device)
    exc = torch.empty(g, dtype=torch.float64, device=rho.device)
    _check(_lib.dks_lda_xc(b.handle, sys, _field(rho, ng, "rho"),
                           _field(mag, 3 * ng, "mag") if mag is not None else None,
                           ct.c_void_p(vxc.data_ptr()), ct.c_void_p(bxc.data_ptr()),
                           ct.c_void_p(exc.data_ptr()), _stream(stream)))
    return vxc, bxc, exc


def get_local_potential(b: Basis, sys: int, stream=None):
    import torch
    g = _grid_shape(b, sys)
    v = torch.empty(g, dtype=torch.float64, device="cuda")
    _check(_lib.dks_get_local_potential(b.handle, sys, ct.c_void_p(v.data_ptr()), _stream(stream)))
    return v


def set_local_potential(b: Basis, sys: int, v, stream=None) -> None:
    g = _grid_shape(b, sys)
    _check(_lib.dks_set_local_potential(b.handle, sys, _field(v, int(np.prod(g)), "v"), _stream(stream)))


def scf_default_opts(**kw) -> ScfOpts:
    o = ScfOpts()
    _lib.dks_scf_default_opts(ct.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def scf(b: Basis, sys: int, n: int, X, sopts: ScfOpts, eopts: Optional[SolveOpts] = None,
        stream=None, allow_notconv: bool = True, history: Optional[np.ndarray] = None,
        eig_history: Optional[np.ndarray] = None):
    """The SCF loop (dks_scf) on the complex128 block X (in: start block, out:
    last eigenvectors).  ``history``: optional float64 array of >= max_scf
    entries receiving each step's ||V_out - V_in|| / ||V_in||.  Returns
    (eigenvalues, occupations, info dict, status)."""
    import torch
    if X.dtype != torch.complex128:
        raise TypeError("X must be complex128")
    N, _, _ = basis_info(b, sys, miller=False)
    eo = eopts if eopts is not None else default_opts()
    _check_block(X, n, N, 2 if eo.model == MODEL_KSSO else 4)
    lam = np.zeros(n)
    occ = np.zeros(n)
    info = ScfInfo()
    if history is not None:
        if history.dtype != np.float64 or history.size < sopts.max_scf or not history.flags.c_contiguous:
            raise ValueError(f"history must be a contiguous float64 array of >= {sopts.max_scf} entries")
        sopts.history = _dptr(history)
    if eig_history is not None:
        if (eig_history.dtype != np.float64 or eig_history.size < sopts.max_scf
                or not eig_history.flags.c_contiguous):
            raise ValueError(f"eig_history must be a contiguous float64 array of >= {sopts.max_scf} entries")
        sopts.eig_history = _dptr(eig_history)
    rc = _lib.dks_scf(b.handle, sys, n, ct.c_void_p(X.data_ptr()), _dptr(lam), _dptr(occ),
                      ct.byref(sopts), ct.byref(eo), ct.byref(info), _stream(stream))
    _check(rc, allow_warning=allow_notconv)
    return lam, occ, info.as_dict(), rc
