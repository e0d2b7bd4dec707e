/*
 * dks.h -- C ABI of libdks, the MI355X (gfx950) hot path of LOBPCG-F for the
 * four-component planewave Dirac-Kohn-Sham eigenproblem (Lin, Shao, E,
 * "Efficient iterative method for solving the Dirac-Kohn-Sham density
 * functional theory").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units are Hartree atomic units (m = 1, e = hbar = 1); every energy passed in
 * or out is shifted by -c^2, the convention of the paper's Sec. 4, so the
 * positive continuum starts at 0 and the negative band sits near -2c^2.
 *
 * A spinor block X holding nb bands is device memory laid out [nb][4][N]:
 * band-major, then the four components (phi_up, phi_dn, chi_up, chi_dn) --
 * the large and small two-spinors of Sec. 2.1 -- then the N planewaves of the
 * system's sphere in the library's order (exported by dks_basis_info).  Complex
 * numbers are interleaved (re, im): complex128 for DKS_FP64, complex64 for
 * DKS_FP32.  Rows of one band are contiguous, so band j starts at
 * X + j * 4 * N complex elements.
 *
 * Every call returns a dks_status: 0 on success, < 0 on error (outputs are then
 * unspecified), > 0 for a warning with valid outputs.  dks_last_error() returns
 * a message for the calling thread's last failure.  Device pointers must be
 * allocated on the device the basis was created on; `stream` is a hipStream_t
 * (NULL = the default stream) and every call is asynchronous on it unless
 * stated otherwise.  Calls on one basis must not overlap on different streams.
 */
#ifndef DKS_H
#define DKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int dks_status;
#define DKS_OK          0
#define DKS_EINVAL     (-1)   /* bad argument (null, size, grid smaller than the sphere...) */
#define DKS_ENOMEM     (-2)   /* device or host allocation failed */
#define DKS_EHIP       (-3)   /* a HIP runtime call failed */
#define DKS_ECHOL      (-4)   /* Gram matrix of the start block not positive definite */
#define DKS_ECOLLAPSE  (-5)   /* a Ritz value fell below -c^2 (variational collapse) */
#define DKS_EINTERNAL  (-6)   /* unexpected host-side failure (e.g. a thread could not start) */
#define DKS_WNOTCONV    1     /* iteration limit reached; outputs valid, residuals reported */

typedef enum { DKS_FP64 = 0, DKS_FP32 = 1 } dks_prec;

typedef enum {
  DKS_MODE_FP64 = 0,          /* every step in FP64 */
  DKS_MODE_MIXED_FP32 = 1,    /* FP32 operator, filter, Gram and updates; FP64 Rayleigh-Ritz;
                                 then FP64 polish iterations to the requested tolerance */
  DKS_MODE_MIXED_BF16GRAM = 2 /* as MIXED_FP32 but, while the median residual of the FP32
                                 stage exceeds 10 * mixed_tol, the Gram products split each
                                 FP32 input into two BF16 numbers (x ~ hi + lo, each rounded
                                 to nearest even) and accumulate hi*hi + hi*lo + lo*hi in FP32
                                 on the BF16 matrix cores (plain BF16 inputs are too coarse
                                 for the Dirac Rayleigh-Ritz).  Three BF16 products per FP32
                                 product on the K = 32 BF16 instruction: the Gram launch is
                                 about 1.3x faster than MIXED_FP32's, the time to solution
                                 about the same (the Gram is a small share of it) */
} dks_mode;

/* Which operator a solve works on (the modules of the paper's Table 1). */
typedef enum {
  DKS_MODEL_DKS = 0,   /* four-component Dirac-Kohn-Sham, blocks [n][4][N] (LOBPCG-F) */
  DKS_MODEL_KSSO = 1   /* two-component Kohn-Sham with spin-orbit coupling, |k+G|^2/2 +
                          V_loc + V_2, blocks [n][2][N] (phi_up, phi_dn); solved by
                          standard LOBPCG, the paper's comparison: use_filter and
                          kinetic_balance are ignored */
} dks_model;

/* The preconditioner T of Algorithm 1 (solve T Y = R for the residual block R). */
typedef enum {
  DKS_PRECOND_DEFAULT = -1, /* the method's own: DKS_PRECOND_TETER for Algorithm 1 (Sec. 4
                               employs it in both LOBPCG and LOBPCG-F), DKS_PRECOND_NONE for
                               DKS_METHOD_DAVIDSON (its filtered space stalled with the
                               factor on systems of the uneven batch) */
  DKS_PRECOND_NONE = 0,   /* T = I (the analysis of Sec. 3.1) */
  DKS_PRECOND_TETER = 1   /* the Teter-Payne-Allan factor K(x) = p / (p + 16 x^4),
                             p = 27 + 18x + 12x^2 + 8x^3 (Sec. 4: used in both LOBPCG and
                             LOBPCG-F), applied per planewave through the spectral
                             projectors P+- of the free Dirac block [[0, c s.q],
                             [c s.q, -2c^2]]: P+ R scaled by K(e+ / E), P- R by K(|e-| / E),
                             e+- = +-sqrt(c^4 + c^2 q^2) - c^2, E per column the mean e+ of
                             the residual's positive part (>= 1e-3 Ha).  The two-component
                             model: K(|k+G|^2 / 2E) */
} dks_precond;

/* The iterative method a solve uses. */
typedef enum {
  DKS_METHOD_LOBPCG = 0,    /* Algorithm 1: LOBPCG-F (or standard LOBPCG, use_filter = 0) */
  DKS_METHOD_DAVIDSON = 1   /* the filter inside a block Davidson iteration (the paper's remark
                               that F can precondition other iterative solvers): the subspace
                               keeps every filtered residual block f(H) R of the unconverged
                               columns up to davidson_dim * n vectors, then restarts from the
                               Ritz vectors; FP64 only */
} dks_method;

/* One (atom, l) block of separable projectors of Eq. (HGH): couplings of the
 * j = l + 1/2 channel (d_plus) and of the j = l - 1/2 channel (d_minus), each a
 * real symmetric n_rad x n_rad matrix (row-major, Ha).  Radial functions are
 * (q r_l)^(2(i-1)) exp(-q^2 r_l^2 / 2), i = 1..n_rad, times the complex solid
 * harmonic |q|^l Y_lm, times exp(-i q.tau_atom); each (atom, l, i) set of 2l+1
 * functions is scaled by one common factor so that the mean over m of their
 * squared 2-norms over the planewave sphere is 1.  0 <= l <= 3, 1 <= n_rad <= 3. */
typedef struct {
  int atom;
  int l;
  int n_rad;
  double r_l;
  const double *d_plus;
  const double *d_minus;
} dks_proj_group;

/* Physical description of one system (Sec. 2: Eq. (vDKS) at fixed potential).
 * All pointers are host memory owned by the caller and only read during
 * dks_init_basis.  One description with nk k-points yields nk consecutive
 * system indices that share the sampled local potential. */
typedef struct {
  double lattice[9];          /* rows a1, a2, a3 (bohr), any non-singular cell */
  int nk;                     /* number of k-points (>= 1) */
  const double *kpts;         /* nk x 3 Cartesian (bohr^-1); {0,0,0} is Gamma */
  double ecut;                /* Ha: basis is { G : |k + G|^2 / 2 <= ecut } (Sec. 2.3) */
  int grid[3];                /* FFT grid N1, N2, N3; each a product of 2, 3, 5; <= 512 */
  double c;                   /* speed of light (137.036 in a.u.) */
  const double *v_loc;        /* N1*N2*N3 real values of the local potential at
                                 r_j = (j1/N1) a1 + (j2/N2) a2 + (j3/N3) a3, j3 fastest */
  int natom;
  const double *tau;          /* natom x 3 Cartesian positions (bohr) */
  int nproj_groups;
  const dks_proj_group *proj; /* may be NULL when nproj_groups == 0 */
} dks_system_desc;

typedef struct dks_basis dks_basis;   /* opaque; owned by the library */

/* Build the planewave basis, the projector tables, FFT plans and device copies
 * of the potential for every (description, k-point) pair, on device `device`.
 * The sphere is ordered by xy-column (n1, n2) lexicographically, then n3
 * ascending.  Errors: DKS_EINVAL for a null pointer, an empty sphere, a grid that
 * is not 2-3-5 smooth or too small to hold the sphere (N_d <= 2 max|n_d|), l or
 * n_rad out of range; DKS_ENOMEM / DKS_EHIP from the device.  On success *out
 * owns everything it allocated until dks_free_basis. */
dks_status dks_init_basis(const dks_system_desc *descs, int ndesc, int device, dks_basis **out);

/* Number of systems (sum of nk over the descriptions). */
int dks_num_systems(const dks_basis *b);

/* Sphere size N of system `sys`; optionally its FFT grid (3 ints) and the
 * Miller index triple of every planewave in the library's order (N x 3 ints,
 * caller-owned host buffer).  Synchronous, host only. */
dks_status dks_basis_info(const dks_basis *b, int sys, int *npw, int *grid3, int *miller);

/* HX = H X for a block of nb bands (Eq. (vDKS) with V_hxc folded into the local
 * potential, shifted by -c^2): the per-planewave 4x4 free-Dirac block, the local
 * potential through zero-padded 3D FFTs on the system grid, and the separable
 * spin-orbit projectors applied identically to the large and the small
 * two-spinor.  X and HX are device blocks [nb][4][N] of precision `prec`; they
 * must not overlap.  The library owns its FFT scratch (grown on demand). */
dks_status dks_apply_H(dks_basis *b, int sys, const void *X, void *HX, int nb,
                       dks_prec prec, void *stream);

/* HX = H X exactly as dks_apply_H, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  This call allocates nothing (no hipMalloc, no host heap,
 * no events, also with dks_profile_enable on).  Its scratch (FFT intermediate,
 * projector coefficients, partial sums) is one library-owned device array of
 * DKS_NOALLOC_SCRATCH_BYTES per GPU, held from the first dks_init_basis on that
 * GPU until the process ends; the block is processed in chunks of bands sized
 * to fit it (heavy dimer, 96^3 grid, FP64: 5 bands per chunk).  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (different streams
 * or threads, or with dks_apply_H_noalloc work still queued on another stream)
 * race and give wrong results.  X and HX as for dks_apply_H.  Errors: those of
 * dks_apply_H, and DKS_EINVAL when a single band needs more scratch than the
 * array holds (4 N_3 n_xycolumns complex values plus the projector terms). */
#define DKS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
dks_status dks_apply_H_noalloc(dks_basis *b, int sys, const void *X, void *HX, int nb,
                               dks_prec prec, void *stream);

/* HX = H_KSSO X for the two-component operator of the KSSO module (Table 1):
 * |k+G|^2/2 per planewave, the local potential through the same zero-padded
 * FFTs, and the same separable spin-orbit projectors V_2 that act on each
 * two-spinor of the Dirac operator (Eq. (HGH)).  No energy shift (the
 * nonrelativistic operator has no rest mass).  X and HX are device blocks
 * [nb][2][N] of precision `prec` that must not overlap. */
dks_status dks_apply_H_ksso(dks_basis *b, int sys, const void *X, void *HX, int nb,
                            dks_prec prec, void *stream);

/* FY = f(H) Y with f(E) = (E - C)^2 / Omega^2, the filter of Eq. (filter)
 * (two applications of H).  Y and FY must not overlap. */
dks_status dks_apply_filter(dks_basis *b, int sys, const void *Y, void *FY, int nb,
                            double C, double Omega, dks_prec prec, void *stream);

/* Y <- T Y in place: the preconditioner DKS_PRECOND_TETER of Algorithm 1 (the
 * Teter factor of Sec. 4 through each planewave's free Dirac projectors; see
 * dks_precond) on nb device blocks [nb][4][N] (model DKS_MODEL_DKS) or
 * [nb][2][N] (DKS_MODEL_KSSO, the plain factor of |k+G|^2 / 2), complex
 * double or float by prec.  The per-column energies are computed from Y
 * itself.  Uses a library-owned scratch of nb doubles. */
dks_status dks_precondition(dks_basis *b, int sys, void *Y, int nb, int model, dks_prec prec,
                            void *stream);

/* The library's default filter constants for system `sys`: C at the middle of
 * the free negative band moved by the mean local potential, Omega = (an upper
 * bound of the positive band) - C, so that f <= 1 on the positive band (the
 * paper asks for C in the negative continuum and f = 1 at the top of the
 * positive band, Sec. 3.1, without giving values).  Host only. */
dks_status dks_filter_constants(const dks_basis *b, int sys, double *C, double *Omega);

typedef struct {
  double C, Omega;      /* filter constants; NaN selects dks_filter_constants */
  int n_init;           /* filter applications on X0 before the first Rayleigh-Ritz (the
                           initial filtering of Algorithm 1; the paper uses 3, then 1 for a
                           warm start) */
  int n_iter;           /* maximum iterations of the main loop */
  double tol;           /* convergence: 2-norm of every residual column < tol (Ha) */
  int mode;             /* dks_mode */
  double mixed_tol;     /* mixed modes: residual at which the reduced-precision stage stops
                           (it also stops when its residual stagnates); <= 0 runs exactly
                           mixed_iter reduced-precision iterations.  Default 3e-4 */
  int mixed_iter;       /* mixed modes: cap on reduced-precision iterations */
  int kinetic_balance;  /* 1: rebuild the small components of X0 from the large ones,
                           chi = c sigma.q phi / (E_q + c^2) (Eq. (RKB)) */
  int use_filter;       /* 1: LOBPCG-F; 0: standard LOBPCG (the paper's comparison) */
  double *iter_ms;      /* optional caller-owned host array of n_iter (+ mixed_iter in the
                           mixed modes) entries: wall time of each main-loop iteration in
                           ms, in execution order (each iteration ends with a stream sync) */
  int n_buffer;         /* 0 <= n_buffer < n: the last n_buffer columns of the block are
                           iterated with the rest but need not converge; convergence, the
                           stagnation test and info.n_converged / max_resnorm cover the
                           first n - n_buffer.  A block larger than the wanted count speeds
                           up the wanted columns when a near-degenerate group straddles
                           the wanted count (the rate of column i is set by the gap to
                           eigenvalue n + 1, not i + 1).  Default 0 */
  int model;            /* dks_model: the operator solved; blocks are [n][4][N] for
                           DKS_MODEL_DKS, [n][2][N] for DKS_MODEL_KSSO.  Default DKS */
  int batch_graph;      /* dks_lobpcgf_solve_batch only.  0: every item on its own lane
                           (a stream and a host thread deciding each iteration).  1: all
                           items in lockstep, in groups, each group's items captured into
                           one HIP graph of graph_chunk iterations on a stream of its own
                           (the groups run concurrently): convergence, stagnation and the
                           iteration cap are decided on the device, finished items become
                           empty launches, the host waits once per chunk; the graph form
                           keeps every iteration's shape (converged columns are locked by
                           clearing their search directions) and keeps P orthogonal to X;
                           items that leave it unconverged (stall, a failed
                           Rayleigh-Ritz, a broken-down step) are finished on the lanes
                           from their last good block.  Algorithm 1 only (method =
                           DKS_METHOD_LOBPCG; else DKS_EINVAL).  Default 0 */
  int graph_chunk;      /* iterations per graph launch (even, >= 2).  Default 8 */
  const int *item_buffer; /* dks_lobpcgf_solve_batch only: optional caller-owned host array
                           of nsys buffer-column counts, item i taking item_buffer[i] in
                           place of n_buffer (each in [0, n[i])).  Default NULL */
  int method;           /* dks_method.  Default DKS_METHOD_LOBPCG */
  int davidson_dim;     /* DKS_METHOD_DAVIDSON: largest subspace, in multiples of n (>= 2;
                           capped at 510 vectors).  Default 4 */
  int preconditioner;   /* dks_precond: T of Algorithm 1 ("solve T Y = R"), applied to the
                           residual block before the filter (Sec. 4 places the filter after
                           the standard preconditioner).  Default DKS_PRECOND_DEFAULT */
} dks_solve_opts;

typedef struct {
  int iterations;       /* main-loop iterations, all stages */
  int iters_reduced;    /* of which in the reduced-precision stage */
  int converged;        /* 1 if every residual < tol */
  int n_converged;
  int h_applies;        /* band-applications of H (one per band per apply) */
  int basis_drops;      /* Y/P directions removed as numerically dependent */
  int p_restarts;       /* iterations whose P block was dropped */
  int neg_ritz_discarded; /* Ritz values below -c^2 left out of X (LOBPCG-F only) */
  double min_ritz;      /* smallest Ritz value seen (collapse monitor) */
  double max_resnorm;   /* largest final residual norm */
  double C, Omega;      /* filter constants used */
  int graph_iterations; /* batch_graph: iterations taken inside the captured graphs */
  int graph_exit;       /* batch_graph: how the item left the last graph stage: 1 converged,
                           2 Rayleigh-Ritz failed, 3 a Ritz value below the spectrum (broken-
                           down step), 4 stalled, 5 iteration cap, 6 wanted residuals jumped
                           a thousandfold (broken-down step); 0: no graph stage ran */
} dks_solve_info;

void dks_default_opts(dks_solve_opts *o);

/* Algorithm 1 (LOBPCG-F) for the n lowest positive-band eigenpairs of system
 * `sys`.  X: device complex128 block [n][4][N]; in: the start block X0, out: the
 * eigenvectors (unit 2-norm).  lambda: host array of n eigenvalues (ascending,
 * shifted by -c^2).  resnorms: optional host array of n final residual norms.
 * info: optional.  Synchronous on `stream`.  Inside the call the Gram product
 * S = Z^H Z and its Cholesky run on a second stream of the library, ordered
 * with `stream` by events, beside the application of H to the filtered block;
 * every such operation has finished when the call returns.  The library
 * allocates its workspace (about 13 blocks of n bands) on first use and keeps
 * it for reuse.  Calls that overlap on one basis race.
 * Returns DKS_WNOTCONV if n_iter was reached, DKS_ECOLLAPSE if a Ritz value fell
 * below -c^2, DKS_ECHOL if the start block is numerically rank deficient. */
dks_status dks_lobpcgf_solve(dks_basis *b, int sys, int n, void *X, double *lambda,
                             double *resnorms, const dks_solve_opts *opts,
                             dks_solve_info *info, void *stream);

/* Algorithm 1 on several systems of one basis at once: the k-points of a
 * description, or independent systems of uneven size and band count (each k
 * and each system is a separate eigenproblem, Sec. 2).  Item i solves system
 * sys[i] for n[i] bands with block X[i] ([n[i]][4][N] complex128, device; in:
 * start block, out: eigenvectors), eigenvalues into the host array lambda[i]
 * (n[i] doubles) and, when resnorms is not NULL, residual norms into
 * resnorms[i]; info, when not NULL, is an array of nsys records.  The same
 * options apply to every item; opts->iter_ms is ignored.  Items run on up to 8
 * library-owned streams (one host thread each; a free lane takes the next item,
 * largest 4N n^2 first), each lane with its own workspace, kept with the basis
 * for reuse;
 * they start after the work queued on `stream` and `stream` waits for all of
 * them.  Returns the most severe item status (errors before DKS_WNOTCONV), with
 * dks_last_error naming the item; every item is attempted. */
dks_status dks_lobpcgf_solve_batch(dks_basis *b, int nsys, const int *sys, const int *n,
                                   void *const *X, double *const *lambda,
                                   double *const *resnorms, const dks_solve_opts *opts,
                                   dks_solve_info *info, void *stream);

/* Launch-shape autotuner.  For each listed system, H X on nb[i] bands (precision
 * `prec`) is timed with HIP events for each candidate of one launch shape at a
 * time, the others held, and the fastest is kept in the basis for every later
 * call on that system: the z-transform tile (xy-columns per workgroup, 2-64
 * within the LDS), the plane kernel form (see dks_get_tuning), and the split-K
 * target of the projector product (256-2048 workgroups).  Results do not change (only
 * rounding order).  Synchronous; allocates two blocks of nb bands while it runs.
 * Calls on the basis must not overlap it. */
dks_status dks_autotune(dks_basis *b, int nsys, const int *sys, const int *nb, dks_prec prec,
                        void *stream);

/* The launch shapes in use for system `sys` (NULL pointers are skipped): z tile,
 * plane kernel form (0: FP64 768 / FP32 512 threads, 1: 256 threads for planes
 * within its LDS budget, 2 and 3: the same with each wave owning whole lines of
 * every line pass, 4 and 5: forms 0 and 1 with the column loads and stores
 * folded into the first and last transform steps), projector split-K target.
 * An unset plane form is reported as the one FP64 applies use (FP32 applies
 * take form 0 or 1 then).  Host only. */
dks_status dks_get_tuning(const dks_basis *b, int sys, int *tile_z, int *plane_form,
                          int *ip_blocks);

/* Set the launch shapes of system `sys` (a stored autotuner table):
 * 1 <= tile_z <= 64 within the LDS for the grid's third axis, plane_form in
 * [-1, 5] (-1: by size and precision; a small form on a plane above its budget
 * falls back to the large one), ip_blocks in [0, 65536] (0: default).  Host
 * only; calls on the basis must not overlap it. */
dks_status dks_set_tuning(dks_basis *b, int sys, int tile_z, int plane_form, int ip_blocks);

/* Kernel timing (a diagnostic for roofline accounting).  When enabled, every
 * kernel the library launches on the calling thread is bracketed by a pair of
 * HIP events on its stream.  dks_profile_report synchronises the device, writes
 * a JSON object {"kernel": {"count": c, "total_ms": t}, ...} into buf (always
 * NUL-terminated, truncated to len) and clears the records.  Disabled by
 * default; enabling costs two event records per launch. */
void dks_profile_enable(int on);
dks_status dks_profile_report(char *buf, size_t len);

/* ---- the self-consistent field loop (Sec. 2.1: Eq. density, V_hxc; Sec. 4) ----
 * Real-space fields are FP64 device arrays on the FFT grid of the description
 * of `sys`, natural order (index j3 fastest), ng = N1 N2 N3 values each. */

/* Eq. (density): rho(r) = sum_i occ[i] psi_i^+ psi_i and the spin density
 * m(r) = sum_i occ[i] psi_i^+ diag(sigma, -sigma) psi_i of the nb FP64 bands X
 * of system `sys` ([nb][4][N] complex128 for DKS_MODEL_DKS; [nb][2][N] for
 * DKS_MODEL_KSSO, where m = sum occ phi^+ sigma phi), with
 * psi(r) = Omega^-1/2 sum_G c_G exp(i (k+G).r): rho in electrons / bohr^3
 * integrates to sum occ over the cell.  rho: ng values; mag: 3 ng values
 * (m_x | m_y | m_z) or NULL.  occ: host, nb values >= 0 (bands with 0 are
 * skipped).  Allocates real-space scratch of up to 512 MB on first use (kept
 * by the basis); calls on one basis must not overlap.  Asynchronous on
 * `stream`. */
dks_status dks_density(dks_basis *b, int sys, int model, const void *X, int nb, const double *occ,
                       double *rho, double *mag, void *stream);

/* The Hartree part of V_hxc (Sec. 2.1) of a periodic density:
 * V_H(G) = 4 pi rho(G) / |G|^2 for G != 0, 0 at G = 0 (neutralising
 * background), rho(G) = N_g^-1 sum_j rho_j exp(-2 pi i G.r_j); the frequency of
 * FFT index m along an axis of N points is m for m < N/2, else m - N; vh is the
 * real part of the inverse transform.  rho and vh: ng values (may alias). */
dks_status dks_hartree(dks_basis *b, int sys, const double *rho, double *vh, void *stream);

/* The Kerker preconditioner of Sec. 4 applied to a potential residual:
 * out(G) = G^2 / (G^2 + q0^2) in(G), the G = 0 part passed unchanged.  q0 > 0
 * (bohr^-1).  in and out: ng values (may alias). */
dks_status dks_kerker(dks_basis *b, int sys, const double *in, double *out, double q0, void *stream);

/* The exchange-correlation part of V_hxc in the local spin density
 * approximation of Sec. 2.1: Slater exchange and the Perdew-Zunger
 * parametrisation of the Ceperley-Alder correlation, spin-interpolated in the
 * local polarisation zeta = |m| / rho.  vxc = dE_xc/drho (ng), bxc = dE_xc/dm
 * (3 ng, along m, or NULL), exc = rho eps_xc (ng, or NULL).  mag NULL means
 * m = 0.  Densities below 1e-14 bohr^-3 give zeros. */
dks_status dks_lda_xc(dks_basis *b, int sys, const double *rho, const double *mag, double *vxc,
                      double *bxc, double *exc, void *stream);

/* Read or replace the local potential V_loc(r) of the description of `sys`
 * (ng values, natural order).  Replacing it changes the operator of every
 * k-point of that description (H, the filter constants' bounds) for all later
 * calls; it synchronises `stream` (the bounds are read on the host) and fails
 * with DKS_EINVAL on a non-finite value. */
dks_status dks_get_local_potential(const dks_basis *b, int sys, double *v, void *stream);
dks_status dks_set_local_potential(dks_basis *b, int sys, const double *v, void *stream);

typedef struct {
  double n_electrons;   /* electrons (one per spinor band), 0 < n_electrons < wanted bands */
  double temperature;   /* electronic temperature (K) of the Fermi-Dirac occupations.  Default 5000 */
  int max_scf;          /* SCF steps.  Default 60 */
  double tol;           /* stop when ||V_out - V_in|| / ||V_in|| < tol and the last solve
                           converged (Sec. 4.4's measure).  Default 1e-8 */
  int eig_iters;        /* eigensolver iterations per SCF step (Table 6: 3).  Default 3 */
  int n_init_first;     /* filter applications on the start block, first step.  Default 3 */
  int n_init_next;      /* the same on later steps (Sec. 3.2).  Default 1 */
  int anderson_depth;   /* stored differences of successive inputs and residuals (<= 15).
                           Default 6 */
  double alpha;         /* step on the preconditioned residual.  Default 0.5 */
  double kerker_q0;     /* Kerker wavevector (bohr^-1).  Default 0.8 */
  double max_bxc;       /* largest |B_xc| (Ha) accepted at the fixed point: the operator applies
                           V_xc but not the sigma.B_xc term, so a spin-polarised
                           self-consistent density fails with DKS_EINVAL (iterates on the way
                           may carry one).  Default 1e-6 */
  double *history;      /* optional caller-owned host array of max_scf entries: the measure
                           ||V_out - V_in|| / ||V_in|| of each step.  Default NULL */
  double *eig_history;  /* optional caller-owned host array of max_scf entries: the largest
                           wanted residual norm of each step's solve.  Default NULL */
} dks_scf_opts;

typedef struct {
  int iterations;       /* SCF steps taken */
  int eig_iterations;   /* eigensolver iterations over all steps */
  int converged;        /* 1 if tol was met */
  int eig_converged;    /* the last solve's convergence flag */
  double residual;      /* last ||V_out - V_in|| / ||V_in|| */
  double fermi;         /* Fermi level (Ha, shifted by -c^2 like the eigenvalues) */
  double free_energy;   /* sum f eps - int (V_in - V_ext) rho + E_H + E_xc - T S (Ha) */
  double e_hartree, e_xc;
  double max_mag;       /* largest |m_x|, |m_y| or |m_z| (bohr^-3) */
  double max_bxc;       /* largest component of B_xc (Ha) */
} dks_scf_info;

void dks_scf_default_opts(dks_scf_opts *o);

/* The SCF loop of Sec. 4 on system `sys` (a description with one k-point):
 * each step takes eig_iters iterations of the solver configured by `eopts`
 * (LOBPCG-F by default; n_iter and n_init are set per step, kinetic balance is
 * applied on the first step only) from the block X ([n][4][N] or [n][2][N],
 * in: start block, out: last eigenvectors), occupies the n - n_buffer wanted
 * bands with Fermi-Dirac occupations holding n_electrons, builds rho and m
 * (dks_density), V_out = V_ext + V_H + V_xc (V_ext: the potential the basis
 * held when the call began), and stops when the measure falls below tol with
 * the solve converged, else mixes: Anderson's combination over the stored
 * differences of successive (V_in, residual) pairs followed by a
 * Kerker-preconditioned step of size alpha.  When the measure falls below tol
 * before the solve has converged, the next step keeps V_in and runs the solver
 * for up to eopts->n_iter iterations to its tolerance.  On return the basis holds the
 * last V_in, lambda (host, n) the eigenvalues of the last solve, occ (host, n,
 * or NULL) the occupations (0 for buffer columns).  DKS_WNOTCONV (> 0) when
 * max_scf steps pass without convergence; eigensolver errors are returned as
 * they are.  Synchronous. */
dks_status dks_scf(dks_basis *b, int sys, int n, void *X, double *lambda, double *occ,
                   const dks_scf_opts *sopts, const dks_solve_opts *eopts, dks_scf_info *info,
                   void *stream);

/* Release everything owned by the basis (after synchronising its device). */
void dks_free_basis(dks_basis *b);

/* Message describing the calling thread's last error ("" if none). */
const char *dks_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DKS_H */
