// Internal declarations of libdks: device-side tables of one system, scratch
// management and the kernel launchers shared by the operator, the dense
// linear algebra and the LOBPCG-F driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dks.h"

namespace dks {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
const char *get_error();

struct Error {
  dks_status code;
  std::string msg;
};

#define DKS_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::dks::Error{DKS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define DKS_REQUIRE(cond, code, msg)                          \
  do {                                                        \
    if (!(cond)) throw ::dks::Error{(code), std::string(msg)}; \
  } while (0)

// Status and message of the exception being handled (call inside a catch
// block): dks::Error keeps its code, a failed host allocation is DKS_ENOMEM,
// anything else DKS_EINTERNAL.
dks_status status_of_current_exception(std::string &msg);

// Runs f() (returning dks_status) and turns any exception into a status, with
// the message recorded for dks_last_error: no exception leaves an entry point.
template <typename F> dks_status guarded(F &&f) {
  try {
    return f();
  } catch (...) {
    std::string msg;
    const dks_status rc = status_of_current_exception(msg);
    set_error(msg);
    return rc;
  }
}

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using cplx = typename cvec<T>::type;

// ---------------------------------------------------------------------------
// FFT plan of one axis
// ---------------------------------------------------------------------------
constexpr int kMaxPass = 8;
struct FftPlan {
  int n;
  int npass;
  int radix[kMaxPass];
};
FftPlan make_plan(int n);   // radices from {8, 6, 5, 4, 3, 2}; n must be 2-3-5 smooth

// ---------------------------------------------------------------------------
// device buffer (owned)
// ---------------------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t nbytes) {  // grow-only
    if (nbytes <= bytes) return;
    release();
    if (nbytes == 0) return;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{DKS_ENOMEM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed"};
    }
    bytes = nbytes;
  }
  template <typename T> T *as() const { return static_cast<T *>(p); }
};

void upload(DevBuf &b, const void *host, size_t bytes);

// Launch a kernel, bracketed by profiling events when profiling is enabled.
#define DKS_LAUNCH(name, kern, grid, block, smem, st, ...)        \
  do {                                                            \
    ::dks::ProfScope ps_((name), (st));                           \
    hipLaunchKernelGGL(kern, grid, block, smem, st, __VA_ARGS__); \
  } while (0)

// Suspends the optional kernel timing of the calling thread for its lifetime
// (the timing creates HIP events, which an allocation-free call must not).
struct ProfPause {
  ProfPause();
  ~ProfPause();
  ProfPause(const ProfPause &) = delete;
  ProfPause &operator=(const ProfPause &) = delete;

 private:
  bool was_on_;
};

// Takes the device address of the allocation-free entry point's scratch array
// on `device` (which must be current); once per device, at dks_init_basis.
void noalloc_scratch_setup(int device);

// Brackets one kernel launch with HIP events when profiling is enabled.
struct ProfScope {
  ProfScope(const char *name, hipStream_t st);
  ~ProfScope();
  ProfScope(const ProfScope &) = delete;
  ProfScope &operator=(const ProfScope &) = delete;

 private:
  hipStream_t st_;
  int idx_ = -1;
};

// ---------------------------------------------------------------------------
// one system (one description at one k-point)
// ---------------------------------------------------------------------------
struct ProjGroupHost {
  int atom, l, n_rad, p0, dim;   // dim = n_rad (2l+1) scalar projectors starting at p0
  int woff;                      // offset (complex elements) of W (2 dim x 2 dim, row-major)
};

struct System {
  // geometry
  double lattice[9];
  double kpt[3];
  double ecut, c;
  int grid[3];
  int ng;
  int N;              // planewaves
  int ncol;           // xy-columns (n1, n2) of the sphere
  int nrows;          // distinct n1 values among the columns
  int vsrc;           // index of the shared local potential
  // host copies
  std::vector<int> miller;        // N x 3, library order
  std::vector<double> q;          // N x 3
  std::vector<int> col_off;       // ncol + 1
  std::vector<int4> col_info;     // {n1 slot, n2 slot, n3 start, len}
  std::vector<int> rows;          // the nrows distinct n1 slots
  std::vector<ProjGroupHost> groups;
  int nproj = 0;                  // scalar projectors
  int wtotal = 0;                 // complex elements of all W blocks
  double qmax2 = 0;
  double nl_bound = 0;
  // device tables
  DevBuf d_col_off, d_col_info, d_rows, d_gmap;   // gmap: per G {local column, z slot}
  DevBuf d_ctab;                                  // [nrows][n2]: column at (row, n2 slot) or -1
  DevBuf d_rowflag;                               // [n1]: 1 where the n1 slot is a sphere row
  DevBuf d_q64, d_q32;                            // SoA qx | qy | qz
  DevBuf d_B64, d_B32;                            // [nproj][N] complex
  DevBuf d_W64;                                   // all W blocks, complex double
  DevBuf d_Winfo;                                 // per (group): int4 {p0, dim, woff, 0}
  FftPlan plan[3];
  DevBuf d_plan;                                  // the three plans, for the kernels
  // launch shapes (defaults from the sizes; dks_autotune measures and sets them)
  int tile_z;                                     // xy-columns per z-FFT workgroup
  int plane_form = -1;                            // plane kernel: 0 FP64 768 / FP32 512
                                                  // threads, 1 256 threads (small planes),
                                                  // 2 and 3 the same with the line passes
                                                  // split by whole lines per wave; -1: 1 if
                                                  // the plane fits the small LDS budget, else 0
  int ip_blocks = 0;                              // projector product: split-K target
                                                  // (workgroups per launch; 0: the default)
};

struct Potential {
  int grid[3];
  double vmin, vmax, vmean;
  DevBuf d_v64, d_v32;            // plane layout [N3][N1][N2]
  DevBuf d_tw64[3], d_tw32[3];    // exp(-2 pi i t / n_d), t < n_d
  DevBuf d_nat[3];                // natural index of real-space position p along axis d
};

}  // namespace dks

namespace dks {
// Device scratch of one H.X pipeline: column-pruned FFT intermediate, projector
// coefficients and GEMM partial sums.  Concurrent applies need separate ones.
struct Workspace {
  DevBuf t1, nlc, nlc2, part;
};
}  // namespace dks

struct dks_basis {
  int device = 0;
  std::vector<dks::System *> sys;
  std::vector<dks::Potential *> pot;
  // apply_H / apply_filter scratch of the unbatched entry points
  dks::Workspace ws;
  dks::DevBuf ftmp64, ftmp32;
  dks::DevBuf pE;   // partial sums of the per-column energies of dks_precondition
  // solver workspace (created on first solve)
  void *solver = nullptr;
  // self-consistent field workspace (created on first use)
  void *scf = nullptr;
  ~dks_basis();
};

namespace dks {

// Workgroups are handed to the eight XCDs of the chip in turn (workgroup L to
// XCD L mod 8), and each XCD has its own L2.  xcd_order maps L to a work index
// so that each XCD gets one contiguous range of work indices, issued in order:
// work items that share data (neighbouring indices) then meet in one L2.
// A bijection of [0, total).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_order(int L, int total) {
  const int per = total / kXcds, rem = total % kXcds;
  const int x = L % kXcds, q = L / kXcds;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + q;
}

// ---------------------------------------------------------------------------
// launchers (all asynchronous on `st`)
// ---------------------------------------------------------------------------
// HX = scale * ((H - shift) X) for nb bands, precision T.  ncomp = 4: the
// four-component Dirac operator on blocks [nb][4][N]; ncomp = 2: the
// two-component Kohn-Sham operator with spin-orbit coupling (|q|^2/2 + V_loc +
// V_2) on blocks [nb][2][N].
// `skip` (optional, device): every kernel of the call returns at once when
// *skip != 0 (a finished system inside a graph-captured batch).  `band_skip`
// (optional, device, one int per band): the grid transforms skip the flagged
// bands, whose rows of X must be zero (their H X rows are then the zero that
// the kinetic and nonlocal kernel writes).
template <typename T>
void apply_h(dks_basis *b, int sys, const cplx<T> *X, cplx<T> *HX, int nb, double shift,
             double scale, hipStream_t st, Workspace &ws, int ncomp = 4,
             const int *skip = nullptr, const int *band_skip = nullptr);
// The same on caller-provided scratch (nothing is allocated): the column-pruned
// FFT intermediate, the projector coefficients before and after the couplings W,
// and the split-K partial sums of the projector product, of the sizes
// apply_scratch_bytes gives for nb bands.
struct ApplyScratch {
  void *t1 = nullptr;
  double2 *nlc = nullptr, *nlc2 = nullptr, *part = nullptr;
};
template <typename T>
void apply_scratch_bytes(const dks_basis *b, int sys, int nb, size_t bytes[4], int ncomp = 4);
template <typename T>
void apply_h_on(dks_basis *b, int sys, const cplx<T> *X, cplx<T> *HX, int nb, double shift,
                double scale, hipStream_t st, const ApplyScratch &scr, int ncomp = 4,
                const int *skip = nullptr, const int *band_skip = nullptr);

// Y <- T Y in place for m spinors (the Teter preconditioner of Algorithm 1 on
// the spectral projectors of each planewave's free Dirac block; two
// components: the plain factor).  part: device scratch of
// m * kTpaMaxBlocks double2 (partial sums of the per-column energies).  With
// `src` (and `idx`, device, m rows): Y row j <- T src row idx[j], the gather
// of the active residuals folded in (src must not overlap Y).
constexpr int kTpaMaxBlocks = 64;
int tpa_blocks(int N);
template <typename T>
void precondition(dks_basis *b, int sys, cplx<T> *Y, int m, hipStream_t st, int ncomp,
                  double2 *part, const int *skip = nullptr, const cplx<T> *src = nullptr,
                  const int *idx = nullptr);

// out[i][j] = sum_k conj(A_i[k]) B_j[k] (+ the same with B2 into out2), FP64 result,
// rows addressed by element offsets.  M, Nn <= 512.  `hermitian` (A and B the same
// rows, both products Hermitian): only the tiles on and above the diagonal are
// multiplied, the rest are mirrored.
template <typename T>
void gemm_ip(const cplx<T> *A, const int64_t *aoff, int M, const cplx<T> *B, const int64_t *boff,
             int Nn, const cplx<T> *B2, int64_t K, double2 *out, double2 *out2, int ldo,
             DevBuf &part, hipStream_t st, bool hermitian = false, const int *skip = nullptr);
// The same product with caller-provided split-K partial sums: `part` holds at
// least gemm_ip_part_elems(M, Nn, K, B2 != null, hermitian) double2.
// `blocks`: split-K target (about this many workgroups per launch; 0: the default).
size_t gemm_ip_part_elems(int M, int Nn, int64_t K, bool two, bool hermitian, int blocks = 0);
template <typename T>
void gemm_ip_raw(const cplx<T> *A, const int64_t *aoff, int M, const cplx<T> *B, const int64_t *boff,
                 int Nn, const cplx<T> *B2, int64_t K, double2 *out, double2 *out2, int ldo,
                 double2 *part, hipStream_t st, bool hermitian = false,
                 const int *skip = nullptr, int blocks = 0);
// The same product with the FP32 inputs rounded to BF16 and FP32 accumulation.
void gemm_ip_bf16(const float2 *A, const int64_t *aoff, int M, const float2 *B, const int64_t *boff,
                  int Nn, const float2 *B2, int64_t K, double2 *out, double2 *out2, int ldo,
                  DevBuf &part, hipStream_t st, bool hermitian = false);

// out_j[k] = alpha * sum_i V[i][j] A_i[k] (+ beta out_j[k]); V FP64 m x n (ld ldv).
template <typename T>
void gemm_up(const cplx<T> *A, const int64_t *aoff, int m, const double2 *V, int ldv, int n,
             int64_t K, cplx<T> *out, int64_t ldo, double beta, hipStream_t st, double alpha = 1.0);
// The same V applied to two row sets in one launch: out1 from A1 and out2 from
// A2 (X and H X, P and H P); A2 = null is gemm_up.  `tag`: profiling name of the
// launch (default k_gemm_up.f64 / .f32).
template <typename T>
void gemm_up2(const cplx<T> *A1, const cplx<T> *A2, const int64_t *aoff, int m, const double2 *V,
              int ldv, int n, int64_t K, cplx<T> *out1, cplx<T> *out2, int64_t ldo, double beta,
              hipStream_t st, double alpha = 1.0, const char *tag = nullptr,
              const int *skip = nullptr);

// R_j = HX_j - lambda_j X_j and ||R_j||^2 (FP64) for n columns of length K.
template <typename T>
void residual(const cplx<T> *X, const cplx<T> *HX, const double *lam, int n, int64_t K,
              cplx<T> *R, double *norm2, DevBuf &part, hipStream_t st, const int *skip = nullptr);

// column squared norms of n rows of length K
template <typename T>
void col_norm2(const cplx<T> *X, int n, int64_t K, double *norm2, DevBuf &part, hipStream_t st);

// dst row i = src row idx[i] (scaled by s[i] if s != null)
template <typename T>
void gather_rows(const cplx<T> *src, const int *idx, int m, int64_t K, cplx<T> *dst,
                 hipStream_t st);

template <typename Ts, typename Td>
void convert(const cplx<Ts> *src, cplx<Td> *dst, int64_t count, hipStream_t st);

template <typename T>
void scale_rows(cplx<T> *X, const double *s, int n, int64_t K, hipStream_t st);

// Every band-component of the ncols FP64 rows X ([ncols][N]) on the real-space
// grid: R[cc][p3][p1][p2] (the real-space order of the potential table), no
// 1/sqrt(volume) factor.  t1: real_space_t1_bytes of scratch.
size_t real_space_t1_bytes(const dks_basis *b, int sys, int ncols);
void real_space_planes(dks_basis *b, int sys, const double2 *X, int ncols, void *t1, double2 *R,
                       hipStream_t st);
// LDS limits of the self-consistent field kernels (once, with the others)
void init_scf_kernel_attributes();

// small component from the large one by kinetic balance, in place on [n][4][N]
void kinetic_balance(dks_basis *b, int sys, double2 *X, int n, hipStream_t st);

// Rayleigh-Ritz on (A, S) of size nz: V (nz x nkeep, row-major ld nkeep), theta (nkeep) are
// the nkeep lowest Ritz pairs above floor_val.  info[0] = kept basis columns, info[1] =
// status (0 ok, 1 too few independent columns, 2 too few Ritz values above floor_val),
// info[2] = dropped columns, info[3] = Ritz values below floor_val; dinfo[0] = smallest
// Ritz value, dinfo[1] = smallest Cholesky pivot kept (S scaled to unit diagonal: the
// squared sine of the angle between a basis column and the span of the columns before it).
// `forced_drop` (nz ints or null): 1 marks a column to skip.  `tstamp` (optional,
// device, kRRStamps entries): wall-clock stamps of the phases, for tuning.
constexpr int kRRStamps = 24;
// device scratch bytes rayleigh_ritz needs for an nz x nz problem keeping nkeep
size_t rr_scratch_bytes(int nz, int nkeep);
void rayleigh_ritz(const double2 *A, const double2 *S, int nz, int nkeep, double drop_tol,
                   double floor_val, const int *forced_drop, double2 *V, double *theta, int *info, double *dinfo,
                   DevBuf &scratch, hipStream_t st, long long *tstamp = nullptr,
                   const int *skip = nullptr);
// The same in two parts, for a caller that has S before A: rayleigh_ritz_s
// (scaling, Cholesky with dropping, L^-1: S only) and, on the same scratch,
// rayleigh_ritz_a (the scaled A and everything after); the second must be
// ordered after the first.
void rayleigh_ritz_s(const double2 *S, int nz, int nkeep, double drop_tol, const int *forced_drop,
                     int *info, double *dinfo, DevBuf &scratch, hipStream_t st);
void rayleigh_ritz_a(const double2 *A, int nz, int nkeep, double floor_val, const int *forced_drop,
                     double2 *V, double *theta, int *info, double *dinfo, DevBuf &scratch,
                     hipStream_t st);

}  // namespace dks
