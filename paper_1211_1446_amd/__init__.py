"""MI355X (gfx950) hot path of LOBPCG-F for the four-component planewave
Dirac-Kohn-Sham eigenproblem.

The work runs in ``libdks.so`` (hand-written HIP kernels behind the C ABI of
``include/dks.h``); this package only marshals arguments.  Importing it loads
the library and raises if it has not been built: there is no fallback.
"""
from ._lib import (  # noqa: F401
    DKS_FP32, DKS_FP64, MODE_FP64, MODE_MIXED_BF16GRAM, MODE_MIXED_FP32, MODEL_DKS, MODEL_KSSO,
    METHOD_DAVIDSON, METHOD_LOBPCG, PRECOND_DEFAULT, PRECOND_NONE, PRECOND_TETER, precondition,
    Basis, DksError,
    apply_filter, apply_H, apply_H_ksso, apply_H_noalloc, autotune, basis_info, get_tuning, set_tuning, default_opts, filter_constants, free_basis, init_basis,
    library_path, lobpcgf_solve, lobpcgf_solve_batch, num_systems, profile_enable,
    profile_report,
    ScfInfo, ScfOpts, density, get_local_potential, hartree, kerker, lda_xc, scf,
    scf_default_opts, set_local_potential,
)
