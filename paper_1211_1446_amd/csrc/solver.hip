// Algorithm 1 (LOBPCG-F) driven from the host: every step on the block runs in
// the library's kernels on one stream; the host reads back only the small
// Rayleigh-Ritz results and the residual norms once per iteration to decide
// convergence and the active (unlocked) columns of Algorithm 1.
//
// Workspace per precision: two copies of the subspace Z = [X | Y | P] and of
// HZ = [HX | HY | HP] (3n rows each, K = 4N complex per row), a residual block
// and a filter temporary.  Iteration k reads Z_cur and writes the new X and P
// into Z_nxt, then the two swap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>

#include <type_traits>
#include <vector>
#include <thread>
#include <atomic>
#include <string>

#include "dks_internal.h"

namespace dks {

template <typename T> struct Blocks {
  int n = 0;
  int64_t K = 0;
  DevBuf Z[2], HZ[2], R, W;
  DevBuf snap;   // best X of a stage that met an ill-conditioned basis (lazily allocated)
  void ensure(int n_, int64_t K_) {
    size_t rowb = sizeof(cplx<T>) * (size_t)K_;
    for (int i = 0; i < 2; ++i) {
      Z[i].ensure(rowb * 3 * n_);
      HZ[i].ensure(rowb * 3 * n_);
    }
    R.ensure(rowb * n_);
    W.ensure(rowb * n_);
    n = n_;
    K = K_;
  }
  cplx<T> *z(int i, int row) { return Z[i].as<cplx<T>>() + (size_t)row * K; }
  cplx<T> *hz(int i, int row) { return HZ[i].as<cplx<T>>() + (size_t)row * K; }
};

// Pinned host staging of the per-iteration transfers.  A copy between the
// device and pageable memory holds the host until the stream reaches it, which
// drains the GPU before the next launches; pinned ones stay asynchronous.
// Grow-only, one buffer per use: each is rewritten by the host only after a
// stream synchronisation has retired the copy that read it.
struct HostBuf {
  void *p = nullptr;
  size_t bytes = 0;
  HostBuf() = default;
  HostBuf(const HostBuf &) = delete;
  HostBuf &operator=(const HostBuf &) = delete;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  template <typename U> U *as(size_t count) {
    const size_t need = sizeof(U) * count;
    if (need > bytes) {
      if (p) {
        DKS_HIP(hipDeviceSynchronize());   // no copy may still read the old buffer
        (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
      }
      DKS_HIP(hipHostMalloc(&p, need, hipHostMallocDefault));
      bytes = need;
    }
    return static_cast<U *>(p);
  }
};

struct Solver {
  Blocks<double> b64;
  Blocks<float> b32;
  DevBuf dv, dhv;   // Davidson subspace V and H V (up to davidson_dim x n rows)
  DevBuf gS, gA, Vz, Vp, Wxp, theta, lam, norms, lockmask, pE, rinfo, rdinfo, off, idx, forced, rrs,
      part, part2, tst;
  DevBuf rrout;   // Rayleigh-Ritz result laid out as its host copy h_rr
  DevBuf part_s;  // split-K partial sums of S formed on the second stream
  HostBuf h_rr, h_lam, h_res, h_act, h_vp;
  Workspace ws;   // H.X scratch of this solver's applies
  hipEvent_t rr_ev = nullptr;   // the Rayleigh-Ritz result has reached the host
  // second stream (default priority) for the S phase of the Rayleigh-Ritz,
  // which runs beside the application of H to Y; its two events
  hipStream_t st2 = nullptr;
  hipEvent_t ev_s = nullptr, ev_p0 = nullptr;
  Solver() = default;
  Solver(const Solver &) = delete;
  Solver &operator=(const Solver &) = delete;
  ~Solver() {
    if (rr_ev) (void)hipEventDestroy(rr_ev);
    if (ev_s) (void)hipEventDestroy(ev_s);
    if (ev_p0) (void)hipEventDestroy(ev_p0);
    if (st2) (void)hipStreamDestroy(st2);
  }
};

// Lanes of dks_lobpcgf_solve_batch: a solver workspace and a stream each,
// kept with the basis so that repeated batches reuse their allocations.
// Two lanes per hardware queue the process has (GPU_MAX_HW_QUEUES, 4 unless
// set): each lane waits on the host a few times per iteration, and a second
// lane on the same queue keeps it fed meanwhile (64-system batch on 4 queues:
// 4.1 s with 4 lanes, 3.3 s with 8).
constexpr int kMaxBatchLanes = 32;
static int batch_lanes() {
  static int v = 0;
  if (!v) {
    const char *e = std::getenv("GPU_MAX_HW_QUEUES");
    const int q = (e && std::atoi(e) > 0) ? std::atoi(e) : 4;
    v = std::max(1, std::min(kMaxBatchLanes, 2 * q));
  }
  return v;
}
struct Lane {
  Solver sv;
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
};
struct BatchLanes {
  Lane lane[kMaxBatchLanes];
  ~BatchLanes() {
    for (auto &l : lane) {
      if (l.done) (void)hipEventDestroy(l.done);
      if (l.st) (void)hipStreamDestroy(l.st);
    }
  }
};

// The basis keeps one Solver for the unbatched entry point and, once a batch
// has run, its lanes.
struct GraphPool;
struct SolverSet {
  Solver main;
  BatchLanes *lanes = nullptr;
  GraphPool *graph = nullptr;
  ~SolverSet();
};
static SolverSet *solvers_of(dks_basis *b) {
  if (!b->solver) b->solver = new SolverSet();
  return static_cast<SolverSet *>(b->solver);
}

// DKS_LOG=1 in the environment prints one JSON line per Rayleigh-Ritz step to stderr.
static bool log_enabled() {
  static int v = -1;
  if (v < 0) {
    const char *e = std::getenv("DKS_LOG");
    v = (e && *e && *e != '0') ? 1 : 0;
  }
  return v == 1;
}

struct Ctx {
  dks_basis *b;
  int sys;
  hipStream_t st;
  Solver *sv;
  const dks_solve_opts *o;
  dks_solve_info *info;
  double C, Om, c2;
  int64_t K;
  int N;
  int ncomp = 4;                      // 4: Dirac spinors (DKS); 2: two-component (KSSO)
  bool filt = true;                   // the filter of LOBPCG-F is applied
  bool guard = true;                  // breakdown guard (Ritz values may not fall below predecessors)
  int iter_slot = 0, iter_cap = 0;   // entries written to / capacity of opts.iter_ms
  double floor = -1e300;              // Ritz values below are discarded (mid-gap -c^2 with F)
  bool bf16_gram = false;             // reduced-precision stage: Gram products from BF16 inputs
  bool split_rr = false;              // S half of the Rayleigh-Ritz beside H Y (unbatched solves)
};

// Row offsets of Z = [rows 0..n) U [n, n+m) U [2n, 2n+mp) of a 3n-row block.
__global__ void k_offsets(int64_t *off, int n, int m, int mp, int64_t K) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int nz = n + m + mp;
  if (i >= nz) return;
  int row = (i < n + m) ? i : (2 * n + (i - n - m));
  off[i] = (int64_t)row * K;
}

// The preconditioner in effect: an explicit choice, else the method's own
// (the Teter factor for Algorithm 1, Sec. 4; T = I for the Davidson method,
// whose space stalled with it on systems of the uneven batch).
static bool use_teter(const dks_solve_opts &o) {
  if (o.preconditioner >= 0) return o.preconditioner == DKS_PRECOND_TETER;
  return o.method != DKS_METHOD_DAVIDSON;
}

template <typename T>
static void filter_inplace(Ctx &x, cplx<T> *Y, cplx<T> *W, int m) {
  // W = (H - C) Y ; Y = (H - C) W / Omega^2   (Eq. filter)
  apply_h<T>(x.b, x.sys, Y, W, m, x.C, 1.0, x.st, x.sv->ws, x.ncomp);
  apply_h<T>(x.b, x.sys, W, Y, m, x.C, 1.0 / (x.Om * x.Om), x.st, x.sv->ws, x.ncomp);
  if (x.info) x.info->h_applies += 2 * m;
}

static double residual_level(std::vector<double> r) {
  std::nth_element(r.begin(), r.begin() + r.size() / 2, r.end());
  return r[r.size() / 2];
}

// Median residual of the columns not yet below tol (0 when all are), and their count.
static double active_level(const std::vector<double> &r, double tol, int &nact) {
  std::vector<double> a;
  for (double v : r)
    if (!(v < tol)) a.push_back(v);
  nact = (int)a.size();
  return a.empty() ? 0.0 : residual_level(a);
}

constexpr int kStallFp64 = 20;     // iterations without a new best residual before stopping
// FP64: iterations without a new best residual before a filtered restart, and
// how many such restarts a stage makes before the stall test above may stop it
constexpr int kStallRestartFp64 = 8;
constexpr int kStallRestarts = 3;
// the same when converged columns come back, at least kRegressSpacing
// iterations after the previous restart and at most kRegressRestarts times
constexpr int kRegressRestarts = 16;
constexpr int kRegressSpacing = 10;
// P is made orthogonal to X after an FP64 Rayleigh-Ritz step whose basis had a
// Cholesky pivot (unit-diagonal scaling) below this, and after every FP32 one
// (where rounding, 2^-24 of each column, swamps P's part outside span X long
// before such a pivot shows)
constexpr double kOrthoPivot = 1e-4;
constexpr int kMaxRollbacks = 8;   // discarded broken-down steps before a stage gives up
constexpr int kStallFp32 = 4;
constexpr int kPolishFilters = 2;  // filter applications on the block entering the FP64 polish
// MIXED_BF16GRAM: BF16-input Gram products while the median residual exceeds
// this multiple of mixed_tol (their rounding, ~2^-9 per element and averaged
// over K terms, stops mattering only once the residuals are that small), FP32
// Gram products after.
constexpr double kBf16GramExit = 10.0;
constexpr double kBf16DropTol = 1e-3;

template <typename T> struct LoopState {
  int cur = 0;
  int m = 0;       // active columns (rows of Y)
  int mp = 0;      // rows of P
  std::vector<int> act;
  std::vector<double> lam, res;
  bool converged = false;
  int iters = 0;
  double min_piv = 1.0;   // smallest Cholesky pivot of the last Rayleigh-Ritz basis
  int dropped = 0;   // directions the last Rayleigh-Ritz removed as dependent
  bool xhx_queued = false;   // the last Rayleigh-Ritz queued X, H X of the next step
  int s_nz = 0;              // subspace size of an S half queued ahead of H Y (0: none)
};

// X_new = Z V[:, :n], HX_new = HZ V into the other half of the double buffer.
template <typename T>
static void queue_xhx(Ctx &x, Blocks<T> &bk, int cur, int nz, int n, const double2 *Vz) {
  Solver &sv = *x.sv;
  const int nxt = 1 - cur;
  gemm_up2<T>(bk.Z[cur].template as<cplx<T>>(), bk.HZ[cur].template as<cplx<T>>(),
              sv.off.as<int64_t>(), nz, Vz, n, n, bk.K, bk.z(nxt, 0), bk.hz(nxt, 0), bk.K, 0.0,
              x.st);
}

// The Rayleigh-Ritz result in one device buffer laid out as its host copy:
// [info 4 x int | dinfo 2 x double | theta n | V nz x n] in double2 units, so
// that one copy brings it over.
struct RRView {
  int *info;
  double *dinfo, *theta;
  double2 *V;
};
static size_t rr_count(int nz, int n) { return 2 + (size_t)(n + 1) / 2 + (size_t)nz * n; }
static RRView rr_view(double2 *base, int n) {
  RRView v;
  v.info = reinterpret_cast<int *>(base);
  v.dinfo = reinterpret_cast<double *>(base + 1);
  v.theta = reinterpret_cast<double *>(base + 2);
  v.V = base + 2 + (n + 1) / 2;
  return v;
}

// The S half of the next Rayleigh-Ritz, queued before H Y: Z = [X, Y, P] is
// complete once Y is filtered, and S = Z^H Z with its scaling, Cholesky and
// L^-1 needs nothing else.  The S product (with partial sums of its own) and
// the one-workgroup S phase run on the second stream, beside the application
// of H to Y, and ritz() waits for them before the A half.
template <typename T>
static void queue_s_half(Ctx &x, Blocks<T> &bk, LoopState<T> &s, int n, double drop_tol) {
  Solver &sv = *x.sv;
  const int nz = n + s.m + s.mp;
  sv.off.ensure(sizeof(int64_t) * 3 * n);
  DKS_LAUNCH("k_offsets", k_offsets, dim3((nz + 255) / 256), dim3(256), 0, x.st, sv.off.as<int64_t>(),
             n, s.m, s.mp, bk.K);
  DKS_HIP(hipGetLastError());
  sv.gS.ensure(sizeof(double2) * nz * nz);
  sv.gA.ensure(sizeof(double2) * nz * nz);
  sv.part_s.ensure(sizeof(double2) * gemm_ip_part_elems(nz, nz, bk.K, false, true));
  if (!sv.st2) DKS_HIP(hipStreamCreateWithFlags(&sv.st2, hipStreamNonBlocking));
  if (!sv.ev_s) DKS_HIP(hipEventCreateWithFlags(&sv.ev_s, hipEventDisableTiming));
  if (!sv.ev_p0) DKS_HIP(hipEventCreateWithFlags(&sv.ev_p0, hipEventDisableTiming));
  const size_t nrr = rr_count(nz, n);
  sv.rrout.ensure(sizeof(double2) * nrr);
  const RRView d = rr_view(sv.rrout.as<double2>(), n);
  DKS_HIP(hipEventRecord(sv.ev_s, x.st));
  DKS_HIP(hipStreamWaitEvent(sv.st2, sv.ev_s, 0));
  double dtol = drop_tol;
  bool bf16 = false;
  if constexpr (std::is_same<T, float>::value) {
    if (x.bf16_gram) {
      // the BF16-split product, and its wider drop tolerance (see ritz)
      gemm_ip_bf16(bk.Z[s.cur].template as<float2>(), sv.off.as<int64_t>(), nz,
                   bk.Z[s.cur].template as<float2>(), sv.off.as<int64_t>(), nz, nullptr, bk.K,
                   sv.gS.as<double2>(), nullptr, nz, sv.part_s, sv.st2, /*hermitian=*/true);
      dtol = std::max(drop_tol, kBf16DropTol);
      bf16 = true;
    }
  }
  if (!bf16)
    gemm_ip<T>(bk.Z[s.cur].template as<cplx<T>>(), sv.off.as<int64_t>(), nz,
               bk.Z[s.cur].template as<cplx<T>>(), sv.off.as<int64_t>(), nz, nullptr, bk.K,
               sv.gS.as<double2>(), nullptr, nz, sv.part_s, sv.st2, /*hermitian=*/true);
  rayleigh_ritz_s(sv.gS.as<double2>(), nz, n, dtol, nullptr, d.info, d.dinfo, sv.rrs, sv.st2);
  DKS_HIP(hipEventRecord(sv.ev_p0, sv.st2));
  s.s_nz = nz;
}

// Rayleigh-Ritz on Z_cur rows described by (n, m, mp); returns false when
// fewer than n directions survive even without P.
template <typename T>
static bool ritz(Ctx &x, Blocks<T> &bk, LoopState<T> &s, int n, double drop_tol,
                 std::vector<double2> &hV) {
  Solver &sv = *x.sv;
  int mp = s.mp;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const int nz = n + s.m + mp;
    // S = Z^H Z and the S phase were queued ahead of H Y (queue_s_half)
    const bool s_ready = attempt == 0 && s.s_nz == nz;
    s.s_nz = 0;
    if (s_ready) {
      bool bf16 = false;
      if constexpr (std::is_same<T, float>::value) {
        if (x.bf16_gram) {
          gemm_ip_bf16(bk.Z[s.cur].template as<float2>(), sv.off.as<int64_t>(), nz,
                       bk.HZ[s.cur].template as<float2>(), sv.off.as<int64_t>(), nz, nullptr,
                       bk.K, sv.gA.as<double2>(), nullptr, nz, sv.part, x.st, /*hermitian=*/true);
          bf16 = true;
        }
      }
      if (!bf16)
        gemm_ip<T>(bk.Z[s.cur].template as<cplx<T>>(), sv.off.as<int64_t>(), nz,
                   bk.HZ[s.cur].template as<cplx<T>>(), sv.off.as<int64_t>(), nz, nullptr, bk.K,
                   sv.gA.as<double2>(), nullptr, nz, sv.part, x.st, /*hermitian=*/true);
    } else {
      sv.off.ensure(sizeof(int64_t) * 3 * n);
      DKS_LAUNCH("k_offsets", k_offsets, dim3((nz + 255) / 256), dim3(256), 0, x.st, sv.off.as<int64_t>(),
                         n, s.m, mp, bk.K);
      DKS_HIP(hipGetLastError());
      sv.gS.ensure(sizeof(double2) * nz * nz);
      sv.gA.ensure(sizeof(double2) * nz * nz);
      if constexpr (std::is_same<T, float>::value) {
        if (x.bf16_gram) {
          gemm_ip_bf16(bk.Z[s.cur].template as<float2>(), sv.off.as<int64_t>(), nz,
                       bk.Z[s.cur].template as<float2>(), sv.off.as<int64_t>(), nz,
                       bk.HZ[s.cur].template as<float2>(), bk.K, sv.gS.as<double2>(),
                       sv.gA.as<double2>(), nz, sv.part, x.st, /*hermitian=*/true);
        } else {
          gemm_ip<T>(bk.Z[s.cur].template as<cplx<T>>(), sv.off.as<int64_t>(), nz,
                     bk.Z[s.cur].template as<cplx<T>>(), sv.off.as<int64_t>(), nz,
                     bk.HZ[s.cur].template as<cplx<T>>(), bk.K, sv.gS.as<double2>(),
                     sv.gA.as<double2>(), nz, sv.part, x.st, /*hermitian=*/true);
        }
      } else {
        gemm_ip<T>(bk.Z[s.cur].template as<cplx<T>>(), sv.off.as<int64_t>(), nz,
                   bk.Z[s.cur].template as<cplx<T>>(), sv.off.as<int64_t>(), nz,
                   bk.HZ[s.cur].template as<cplx<T>>(), bk.K, sv.gS.as<double2>(),
                   sv.gA.as<double2>(), nz, sv.part, x.st, /*hermitian=*/true);
      }
    }
    const size_t nrr = rr_count(nz, n);
    sv.rrout.ensure(sizeof(double2) * nrr);
    const RRView d = rr_view(sv.rrout.as<double2>(), n);
    const bool stamps = log_enabled() && !s_ready;
    if (stamps) sv.tst.ensure(sizeof(long long) * kRRStamps);
    // BF16-split Gram products carry relative errors of a few 1e-6: directions
    // whose scaled overlap pivot is not well above that are dropped
    const double dtol = (sizeof(T) == 4 && x.bf16_gram) ? std::max(drop_tol, kBf16DropTol) : drop_tol;
    if (s_ready) {
      DKS_HIP(hipStreamWaitEvent(x.st, sv.ev_p0, 0));
      rayleigh_ritz_a(sv.gA.as<double2>(), nz, n, x.floor, nullptr, d.V, d.theta, d.info, d.dinfo,
                      sv.rrs, x.st);
    } else {
      rayleigh_ritz(sv.gA.as<double2>(), sv.gS.as<double2>(), nz, n, dtol, x.floor, nullptr, d.V,
                    d.theta, d.info, d.dinfo, sv.rrs, x.st,
                    stamps ? sv.tst.as<long long>() : nullptr);
    }
    if (stamps) {
      // reduction phases: scaling, Cholesky, L^-1, products + Hermitian part,
      // tridiagonal reduction (stamps 0-5 of k_rr_reduce)
      long long ts[6];
      DKS_HIP(hipMemcpyAsync(ts, sv.tst.p, sizeof(ts), hipMemcpyDeviceToHost, x.st));
      DKS_HIP(hipStreamSynchronize(x.st));
      std::fprintf(stderr, "{\"rr_phase_us\": [");
      for (int k = 1; k < 6; ++k) std::fprintf(stderr, "%s%.1f", k > 1 ? ", " : "", (ts[k] - ts[k - 1]) / 100.0);
      std::fprintf(stderr, "]}\n");
    }
    // status, Ritz values and vectors in one copy
    double2 *hr = sv.h_rr.as<double2>(nrr);
    const RRView h = rr_view(hr, n);
    int *info = h.info;
    double *dinfo = h.dinfo;
    double *hth = h.theta;
    double2 *hvz = h.V;
    DKS_HIP(hipMemcpyAsync(hr, sv.rrout.p, sizeof(double2) * nrr, hipMemcpyDeviceToHost, x.st));
    // X and H X of the next step (Z V[:, :n], HZ V) are queued before the host
    // waits for the copies, so that the device works while the host reads the
    // result.  They go to the half of the double buffer that the step does not
    // read; after a failed Rayleigh-Ritz the retry queues them again.
    if (!sv.rr_ev) DKS_HIP(hipEventCreateWithFlags(&sv.rr_ev, hipEventDisableTiming));
    DKS_HIP(hipEventRecord(sv.rr_ev, x.st));
    queue_xhx<T>(x, bk, s.cur, nz, n, d.V);
    s.xhx_queued = true;
    DKS_HIP(hipEventSynchronize(sv.rr_ev));
    if (log_enabled())
      std::fprintf(stderr,
                   "{\"prec\": %d, \"nz\": %d, \"n\": %d, \"m\": %d, \"mp\": %d, \"kept\": %d, "
                   "\"status\": %d, \"min_ritz\": %.12g}\n",
                   (int)sizeof(T), nz, n, s.m, mp, info[0], info[1], dinfo[0]);
    if (info[1] == 0) {
      s.dropped = info[2];
      s.min_piv = dinfo[1];
      if (x.info) {
        x.info->basis_drops += info[2];
        x.info->neg_ritz_discarded += info[3];
        x.info->min_ritz = std::min(x.info->min_ritz, dinfo[0]);
      }
      s.mp = mp;
      hV.assign(hvz, hvz + (size_t)nz * n);
      s.lam.assign(hth, hth + n);
      return true;
    }
    if (mp == 0) return false;
    mp = 0;   // retry without P
    if (x.info) x.info->p_restarts += 1;
  }
  return false;
}

// X_new = Z V[:, :n], HX_new = HZ V; residual and norms; active set; P, HP.
template <typename T>
static void update(Ctx &x, Blocks<T> &bk, LoopState<T> &s, int n, const std::vector<double2> &hV,
                   double tol) {
  Solver &sv = *x.sv;
  const int nz = n + s.m + s.mp;
  const int nxt = 1 - s.cur;
  if (!s.xhx_queued)
    queue_xhx<T>(x, bk, s.cur, nz, n, rr_view(sv.rrout.as<double2>(), n).V);
  s.xhx_queued = false;
  sv.lam.ensure(sizeof(double) * n);
  double *hl = sv.h_lam.as<double>(n);
  std::copy(s.lam.begin(), s.lam.end(), hl);
  DKS_HIP(hipMemcpyAsync(sv.lam.p, hl, sizeof(double) * n, hipMemcpyHostToDevice, x.st));
  sv.norms.ensure(sizeof(double) * n);
  residual<T>(bk.z(nxt, 0), bk.hz(nxt, 0), sv.lam.as<double>(), n, bk.K, bk.R.template as<cplx<T>>(),
              sv.norms.as<double>(), sv.part2, x.st);
  double *hres = sv.h_res.as<double>(n);
  DKS_HIP(hipMemcpyAsync(hres, sv.norms.p, sizeof(double) * n, hipMemcpyDeviceToHost, x.st));
  // wait on an event of the copy (a spinning wait) rather than the stream
  if (!sv.rr_ev) DKS_HIP(hipEventCreateWithFlags(&sv.rr_ev, hipEventDisableTiming));
  DKS_HIP(hipEventRecord(sv.rr_ev, x.st));
  DKS_HIP(hipEventSynchronize(sv.rr_ev));
  s.res.assign(hres, hres + n);
  for (auto &r : s.res) r = std::sqrt(std::max(r, 0.0));
  if (log_enabled()) {
    std::fprintf(stderr, "{\"prec\": %d, \"lam\": [", (int)sizeof(T));
    for (int j = 0; j < n; ++j) std::fprintf(stderr, "%s%.12g", j ? ", " : "", s.lam[j]);
    std::fprintf(stderr, "], \"res\": [");
    for (int j = 0; j < n; ++j) std::fprintf(stderr, "%s%.3e", j ? ", " : "", s.res[j]);
    std::fprintf(stderr, "]}\n");
  }
  std::vector<int> act;
  for (int j = 0; j < n; ++j)
    if (!(s.res[j] < tol)) act.push_back(j);
  const int mnew = (int)act.size();
  // converged once the wanted columns are (the buffer columns stay active)
  const int nwant = n - x.o->n_buffer;
  s.converged = true;
  for (int j = 0; j < nwant; ++j)
    if (!(s.res[j] < tol)) s.converged = false;
  if (mnew > 0 && s.m + s.mp > 0) {
    // conjugate directions P = [0, Y, P] V[:, act] (Algorithm 1), HP alike
    const int nyp = s.m + s.mp;
    const size_t nvp = (size_t)nyp * mnew;
    double2 *vp = sv.h_vp.as<double2>(nvp);
    for (int i = 0; i < nyp; ++i)
      for (int a = 0; a < mnew; ++a) vp[(size_t)i * mnew + a] = hV[(size_t)(n + i) * n + act[a]];
    sv.Vp.ensure(sizeof(double2) * nvp);
    DKS_HIP(hipMemcpyAsync(sv.Vp.p, vp, sizeof(double2) * nvp, hipMemcpyHostToDevice, x.st));
    const int64_t *offyp = sv.off.as<int64_t>() + n;
    gemm_up2<T>(bk.Z[s.cur].template as<cplx<T>>(), bk.HZ[s.cur].template as<cplx<T>>(), offyp,
                nyp, sv.Vp.as<double2>(), mnew, mnew, bk.K, bk.z(nxt, 2 * n), bk.hz(nxt, 2 * n),
                bk.K, 0.0, x.st);
    // P against the new X: P -= X (X^H P), HP -= HX (X^H P), in FP32 and, in
    // FP64, once the last basis was ill-conditioned.  The directions of P
    // formed above can lie mostly inside span X (the Rayleigh-Ritz rotates
    // near-degenerate Ritz vectors into each other from one step to the next,
    // and P carries those rotations along), so that its useful part, the part
    // outside span X, is a small fraction of each column: the Cholesky pivots
    // of P's columns are then small.  Left in, the overlaps of that part are resolved only to
    // rounding relative to the whole column, and close clusters stop
    // converging at ~1e-7 in FP64.  Removing the span-X part keeps P, in the
    // Rayleigh-Ritz basis, the new direction that it stands for.
    if (sizeof(T) == 4 || s.min_piv < kOrthoPivot) {
      sv.Wxp.ensure(sizeof(double2) * (size_t)n * mnew);
      gemm_ip<T>(bk.z(nxt, 0), nullptr, n, bk.z(nxt, 2 * n), nullptr, mnew, nullptr, bk.K,
                 sv.Wxp.as<double2>(), nullptr, mnew, sv.part, x.st);
      gemm_up2<T>(bk.z(nxt, 0), bk.hz(nxt, 0), nullptr, n, sv.Wxp.as<double2>(), mnew, mnew, bk.K,
                  bk.z(nxt, 2 * n), bk.hz(nxt, 2 * n), bk.K, 1.0, x.st, -1.0,
                  sizeof(T) == 8 ? "k_gemm_up.portho.f64" : "k_gemm_up.portho.f32");
    }
  }
  s.mp = (mnew > 0 && s.m + s.mp > 0) ? mnew : 0;
  s.m = mnew;
  s.act = act;
  s.cur = nxt;
}

// One precision stage of Algorithm 1 on the block already in Z[cur] rows [0, n).
// n_init: filter applications on the start block before the first Rayleigh-Ritz.
template <typename T>
static dks_status run_stage(Ctx &x, Blocks<T> &bk, LoopState<T> &s, int n, int n_init,
                            double tol, int max_iter, double drop_tol, int stall_window,
                            int restart_window) {
  Solver &sv = *x.sv;
  const bool filt = x.filt;
  s.cur = 0;
  s.m = 0;
  s.mp = 0;
  s.converged = false;
  s.xhx_queued = false;
  s.s_nz = 0;
  // initial filtering of the start block
  if (filt)
    for (int k = 0; k < n_init; ++k) filter_inplace<T>(x, bk.z(0, 0), bk.W.template as<cplx<T>>(), n);
  // Rayleigh-Ritz on the start block, first residual
  apply_h<T>(x.b, x.sys, bk.z(0, 0), bk.hz(0, 0), n, 0.0, 1.0, x.st, x.sv->ws, x.ncomp);
  if (x.info) x.info->h_applies += n;
  std::vector<double2> hV;
  if (!ritz<T>(x, bk, s, n, drop_tol, hV))
    throw Error{DKS_ECHOL, "the start block is numerically rank deficient"};
  update<T>(x, bk, s, n, hV, tol);
  int best_nact = 0;
  double best =
      active_level(std::vector<double>(s.res.begin(), s.res.begin() + (n - x.o->n_buffer)), tol, best_nact);
  int stall = 0;
  int rollbacks = 0;
  int stall_restarts = 0, regress_restarts = 0, last_restart = -kRegressSpacing;
  // Restart from the current X after a discarded step: the filter, applied
  // twice, removes the negative-band content the broken-down step let in (each
  // pass damps it by ~(w/2c^2)^2, as for the block entering the FP64 polish);
  // then H X is formed anew and the Rayleigh-Ritz runs on X alone (no Y, P).
  auto restart = [&]() {
    if (filt)
      for (int k = 0; k < kPolishFilters; ++k)
        filter_inplace<T>(x, bk.z(s.cur, 0), bk.W.template as<cplx<T>>(), n);
    apply_h<T>(x.b, x.sys, bk.z(s.cur, 0), bk.hz(s.cur, 0), n, 0.0, 1.0, x.st, x.sv->ws, x.ncomp);
    if (x.info) {
      x.info->h_applies += n;
      x.info->p_restarts += 1;
    }
    s.m = 0;
    s.mp = 0;
    if (!ritz<T>(x, bk, s, n, drop_tol, hV))
      throw Error{DKS_ECHOL, "the restarted block is numerically rank deficient"};
    update<T>(x, bk, s, n, hV, tol);
  };
  // Once the basis has turned ill-conditioned (a dropped direction or a
  // discarded step) the iteration can degrade gradually; from then on the best
  // X so far (largest wanted residual) is kept and returned if the last is worse.
  // A filtered restart marks the same trouble.
  const int nwant = n - x.o->n_buffer;
  auto wanted_max = [&]() {
    double mx = 0;
    for (int j = 0; j < nwant; ++j) mx = std::max(mx, s.res[j]);
    return mx;
  };
  bool risky = false, snap_ok = false;
  double snap_mx = std::numeric_limits<double>::infinity();
  std::vector<double> snap_lam, snap_res;
  auto keep_best = [&]() {
    risky = risky || s.dropped > 0 || rollbacks > 0 || stall_restarts > 0 || regress_restarts > 0;
    const double mx = wanted_max();
    if (!risky || !(mx < snap_mx)) return;
    bk.snap.ensure(sizeof(cplx<T>) * (size_t)bk.K * n);
    DKS_HIP(hipMemcpyAsync(bk.snap.p, bk.z(s.cur, 0), sizeof(cplx<T>) * (size_t)bk.K * n,
                           hipMemcpyDeviceToDevice, x.st));
    snap_ok = true;
    snap_mx = mx;
    snap_lam = s.lam;
    snap_res = s.res;
  };
  // main loop
  while (!s.converged && s.iters < max_iter) {
    const auto t0 = std::chrono::steady_clock::now();
    s.iters++;
    if (x.info) x.info->iterations++;
    const int m = s.m;
    // preconditioned residual: Y = T R[:, active] (T = I unless opts.preconditioner)
    sv.idx.ensure(sizeof(int) * n);
    int *ha = sv.h_act.as<int>(n);
    std::copy(s.act.begin(), s.act.end(), ha);
    DKS_HIP(hipMemcpyAsync(sv.idx.p, ha, sizeof(int) * m, hipMemcpyHostToDevice, x.st));
    if (use_teter(*x.o)) {
      // T reads the active rows of R itself (no separate gather)
      sv.pE.ensure(sizeof(double2) * n * kTpaMaxBlocks);
      precondition<T>(x.b, x.sys, bk.z(s.cur, n), m, x.st, x.ncomp, sv.pE.as<double2>(), nullptr,
                      bk.R.template as<cplx<T>>(), sv.idx.as<int>());
    } else {
      gather_rows<T>(bk.R.template as<cplx<T>>(), sv.idx.as<int>(), m, bk.K, bk.z(s.cur, n), x.st);
    }
    // the filtering step: Y = f(H) Y
    if (filt) filter_inplace<T>(x, bk.z(s.cur, n), bk.W.template as<cplx<T>>(), m);
    if (x.split_rr && !log_enabled())
      queue_s_half<T>(x, bk, s, n, drop_tol);
    apply_h<T>(x.b, x.sys, bk.z(s.cur, n), bk.hz(s.cur, n), m, 0.0, 1.0, x.st, x.sv->ws, x.ncomp);
    if (x.info) x.info->h_applies += m;
    // Rayleigh-Ritz on Z = [X, Y, P]
    const std::vector<double> lam_prev = s.lam;
    if (!ritz<T>(x, bk, s, n, drop_tol, hV))
      throw Error{DKS_ECHOL, "Rayleigh-Ritz lost the X block"};
    // Breakdown guard.  span Z contains span X, so no Ritz value can lie
    // below its predecessor by more than the block residual allows (Weyl:
    // the i-th eigenvalue of H is within |R|_2 <= |R|_F of the i-th Ritz
    // value of X).  A larger fall means the projected pencil is no longer a
    // compression of H: the recurrences for HX and HP have drifted in an
    // ill-conditioned basis.  The step is then discarded (X is still that of
    // the previous step) and the iteration restarts from X.  The argument holds
    // for the positive band only (the Ritz values must stay above the negative
    // band to be compared with its eigenvalues), so it guards LOBPCG-F; plain
    // LOBPCG on the Dirac operator is left unguarded, and its fall into the
    // negative band, the variational collapse of Sec. 3.1, is reported as such.
    // The two-component operator has no negative band and is guarded.
    if (x.guard) {
      double rf = 0;
      for (double r : s.res) rf += r * r;
      rf = std::sqrt(rf);
      bool broke = false;
      for (int j = 0; j < n; ++j)
        if (s.lam[j] < lam_prev[j] - (10.0 * rf + 1e-9 * std::fabs(lam_prev[j]))) broke = true;
      if (broke) {
        s.lam = lam_prev;
        if (++rollbacks > kMaxRollbacks) break;   // keep the last good state
        restart();
        continue;
      }
    }
    // new X, residuals, soft locking, new P
    keep_best();   // the state this step starts from (its X survives in Z[cur])
    const std::vector<double> res_prev = s.res;
    const std::vector<int> act_prev = s.act;
    const int m_prev = s.m, cur_prev = s.cur;
    update<T>(x, bk, s, n, hV, tol);
    {
      // the same guard on the residuals: a jump by three orders of magnitude
      // in one step is the same breakdown seen from the vectors.  The previous
      // X is still in Z[cur_prev].
      double mx_prev = 0, mx = 0;
      for (double r : res_prev) mx_prev = std::max(mx_prev, r);
      for (double r : s.res) mx = std::max(mx, r);
      if (x.guard && !(mx <= 1e3 * mx_prev)) {
        s.cur = cur_prev;
        s.lam = lam_prev;
        s.res = res_prev;
        s.act = act_prev;
        s.m = m_prev;
        s.mp = 0;
        s.converged = false;
        if (++rollbacks > kMaxRollbacks) break;
        restart();
        continue;
      }
    }
    if (x.o->iter_ms && x.iter_slot < x.iter_cap)
      x.o->iter_ms[x.iter_slot++] =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (x.bf16_gram && !(residual_level(s.res) > kBf16GramExit * x.o->mixed_tol))
      x.bf16_gram = false;
    // stagnation: neither a column newly below tol nor a new low of the median
    // residual of the remaining columns for `restart_window` iterations starts
    // a filtered restart (FP64, a few times); after those, `stall_window` such
    // iterations mean the iteration sits on its rounding floor: stop instead
    // of iterating on noise.  (The worst residual is gap-limited and not
    // monotone in the first iterations; columns already converged no longer
    // move the level.)
    int nact = 0;
    const double level =
        active_level(std::vector<double>(s.res.begin(), s.res.begin() + (n - x.o->n_buffer)), tol, nact);
    // Wanted columns that had converged coming back above tol, more than a
    // Kramers pair at once, is the same negative-band content showing in the
    // columns no longer iterated on; left alone it ends in a broken-down step.
    if (restart_window > 0 && regress_restarts < kRegressRestarts && nact > best_nact + 2 &&
        s.iters - last_restart >= kRegressSpacing) {
      ++regress_restarts;
      last_restart = s.iters;
      restart();
      stall = 0;
      best = active_level(std::vector<double>(s.res.begin(), s.res.begin() + nwant), tol, best_nact);
      continue;
    }
    if (nact < best_nact) {
      best_nact = nact;
      best = level;
      stall = 0;
    } else if (level < 0.95 * best) {
      best = level;
      stall = 0;
    } else {
      ++stall;
      const bool can_restart = restart_window > 0 && stall_restarts < kStallRestarts;
      if (can_restart && stall >= restart_window) {
        // A stall well above the rounding floor of the operator is, in FP64,
        // negative-band content that X has gathered from the rounding of its
        // updates: Y and P are filtered, so that no Rayleigh-Ritz over
        // [X, Y, P] can take it out again, and the residual carries it times
        // ~2c^2.  A restart filters X itself (and drops P).
        ++stall_restarts;
        restart();
        stall = 0;
        best = active_level(std::vector<double>(s.res.begin(), s.res.begin() + nwant), tol, best_nact);
      } else if (!can_restart && stall_window > 0 && stall >= stall_window) {
        break;
      }
    }
  }
  keep_best();
  if (snap_ok && !s.converged && wanted_max() > snap_mx) {
    DKS_HIP(hipMemcpyAsync(bk.z(s.cur, 0), bk.snap.p, sizeof(cplx<T>) * (size_t)bk.K * n,
                           hipMemcpyDeviceToDevice, x.st));
    s.lam = snap_lam;
    s.res = snap_res;
  }
  return s.converged ? DKS_OK : DKS_WNOTCONV;
}

// The filter inside a Davidson-type solver (the paper's closing remark that F
// can precondition other iterative methods): a block Davidson iteration in
// FP64 whose subspace V keeps every filtered residual block f(H) R of the
// unconverged columns until it would exceed max_dim rows, then restarts
// from the current Ritz vectors.  Each step is a Rayleigh-Ritz on span V (the
// same Gram products and FP64 reduction as Algorithm 1, n lowest Ritz pairs
// above the floor), X = V Vz and H X = (H V) Vz, the residuals, and one
// filter + H application to the new block.  The result goes to Z[0] rows
// [0, n) of `bk` with s.lam and s.res.
static dks_status run_davidson(Ctx &x, Blocks<double> &bk, LoopState<double> &s, int n, int n_init,
                               double tol, int max_iter, int max_dim) {
  Solver &sv = *x.sv;
  const int64_t K = x.K;
  const size_t rowb = sizeof(double2) * (size_t)K;
  sv.dv.ensure(rowb * max_dim);
  sv.dhv.ensure(rowb * max_dim);
  double2 *V = sv.dv.as<double2>(), *HV = sv.dhv.as<double2>();
  auto row = [&](double2 *base, int r) { return base + (size_t)r * K; };
  // start block: already in Z[0] rows [0, n)
  DKS_HIP(hipMemcpyAsync(V, bk.z(0, 0), rowb * n, hipMemcpyDeviceToDevice, x.st));
  if (x.filt)
    for (int k = 0; k < n_init; ++k) filter_inplace<double>(x, V, bk.W.as<double2>(), n);
  apply_h<double>(x.b, x.sys, V, HV, n, 0.0, 1.0, x.st, sv.ws, x.ncomp);
  if (x.info) x.info->h_applies += n;
  int dim = n;
  s.cur = 0;
  s.converged = false;
  s.iters = 0;
  const int nwant = n - x.o->n_buffer;
  std::vector<double2> hV;
  double2 *Xb = bk.z(0, 0), *HXb = bk.hz(0, 0);
  for (;;) {
    // Rayleigh-Ritz on span V (retried from the Ritz vectors alone if the
    // subspace turned numerically dependent)
    bool ok = false;
    for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
      sv.gS.ensure(sizeof(double2) * dim * dim);
      sv.gA.ensure(sizeof(double2) * dim * dim);
      gemm_ip<double>(V, nullptr, dim, V, nullptr, dim, HV, K, sv.gS.as<double2>(),
                      sv.gA.as<double2>(), dim, sv.part, x.st, true);
      sv.Vz.ensure(sizeof(double2) * dim * n);
      sv.theta.ensure(sizeof(double) * n);
      sv.rinfo.ensure(sizeof(int) * 4);
      sv.rdinfo.ensure(sizeof(double) * 2);
      rayleigh_ritz(sv.gA.as<double2>(), sv.gS.as<double2>(), dim, n, 1e-10, x.floor, nullptr,
                    sv.Vz.as<double2>(), sv.theta.as<double>(), sv.rinfo.as<int>(),
                    sv.rdinfo.as<double>(), sv.rrs, x.st);
      double2 *hr = sv.h_rr.as<double2>(2 + (size_t)n);
      int *inf4 = reinterpret_cast<int *>(hr);
      double *dinfo = reinterpret_cast<double *>(hr + 1);
      double *hth = reinterpret_cast<double *>(hr + 2);
      DKS_HIP(hipMemcpyAsync(inf4, sv.rinfo.p, sizeof(int) * 4, hipMemcpyDeviceToHost, x.st));
      DKS_HIP(hipMemcpyAsync(dinfo, sv.rdinfo.p, sizeof(double) * 2, hipMemcpyDeviceToHost, x.st));
      DKS_HIP(hipMemcpyAsync(hth, sv.theta.p, sizeof(double) * n, hipMemcpyDeviceToHost, x.st));
      DKS_HIP(hipStreamSynchronize(x.st));
      if (inf4[1] == 0) {
        ok = true;
        s.lam.assign(hth, hth + n);
        if (x.info) {
          x.info->basis_drops += inf4[2];
          x.info->neg_ritz_discarded += inf4[3];
          x.info->min_ritz = std::min(x.info->min_ritz, dinfo[0]);
        }
      } else if (dim > n && s.iters > 0) {
        // restart from the last Ritz vectors (still in Xb, HXb)
        DKS_HIP(hipMemcpyAsync(V, Xb, rowb * n, hipMemcpyDeviceToDevice, x.st));
        DKS_HIP(hipMemcpyAsync(HV, HXb, rowb * n, hipMemcpyDeviceToDevice, x.st));
        dim = n;
        if (x.info) x.info->p_restarts += 1;
      } else {
        break;
      }
    }
    if (!ok) throw Error{DKS_ECHOL, "the Davidson subspace is numerically rank deficient"};
    // Ritz vectors, residuals
    gemm_up2<double>(V, HV, nullptr, dim, sv.Vz.as<double2>(), n, n, K, Xb, HXb, K, 0.0, x.st);
    sv.lam.ensure(sizeof(double) * n);
    sv.norms.ensure(sizeof(double) * n);
    residual<double>(Xb, HXb, sv.theta.as<double>(), n, K, bk.R.as<double2>(), sv.norms.as<double>(),
                     sv.part2, x.st);
    double *hres = sv.h_res.as<double>(n);
    DKS_HIP(hipMemcpyAsync(hres, sv.norms.p, sizeof(double) * n, hipMemcpyDeviceToHost, x.st));
    DKS_HIP(hipStreamSynchronize(x.st));
    s.res.assign(hres, hres + n);
    for (auto &r : s.res) r = std::sqrt(std::max(r, 0.0));
    s.converged = true;
    for (int j = 0; j < nwant; ++j)
      if (!(s.res[j] < tol)) s.converged = false;
    if (s.converged || s.iters >= max_iter) break;
    s.iters++;
    if (x.info) x.info->iterations++;
    // new block: the filtered residuals of the columns not yet below tol
    std::vector<int> act;
    for (int j = 0; j < n; ++j)
      if (!(s.res[j] < tol)) act.push_back(j);
    const int m = (int)act.size();
    if (dim + m > max_dim) {
      DKS_HIP(hipMemcpyAsync(V, Xb, rowb * n, hipMemcpyDeviceToDevice, x.st));
      DKS_HIP(hipMemcpyAsync(HV, HXb, rowb * n, hipMemcpyDeviceToDevice, x.st));
      dim = n;
    }
    sv.idx.ensure(sizeof(int) * n);
    int *ha = sv.h_act.as<int>(n);
    std::copy(act.begin(), act.end(), ha);
    DKS_HIP(hipMemcpyAsync(sv.idx.p, ha, sizeof(int) * m, hipMemcpyHostToDevice, x.st));
    gather_rows<double>(bk.R.as<double2>(), sv.idx.as<int>(), m, K, row(V, dim), x.st);
    if (use_teter(*x.o)) {
      sv.pE.ensure(sizeof(double2) * n * kTpaMaxBlocks);
      precondition<double>(x.b, x.sys, row(V, dim), m, x.st, x.ncomp, sv.pE.as<double2>());
    }
    if (x.filt) filter_inplace<double>(x, row(V, dim), bk.W.as<double2>(), m);
    apply_h<double>(x.b, x.sys, row(V, dim), row(HV, dim), m, 0.0, 1.0, x.st, sv.ws, x.ncomp);
    if (x.info) x.info->h_applies += m;
    dim += m;
  }
  s.cur = 0;
  return s.converged ? DKS_OK : DKS_WNOTCONV;
}

// One solve of Algorithm 1 on `st` with solver workspace `sv`; returns the
// status and, for a nonzero one, its message.  Throws dks::Error on failures.
static dks_status solve_one(dks_basis *b, int sys, int n, double2 *Xu, double *lambda,
                            double *resnorms, const dks_solve_opts &o, dks_solve_info *info,
                            hipStream_t st, Solver *sv, std::string &msg,
                            bool split_rr = false) {
  {
    const System &s = *b->sys[sys];
    DKS_REQUIRE(o.model == DKS_MODEL_DKS || o.model == DKS_MODEL_KSSO, DKS_EINVAL, "bad model");
    const int ncomp = o.model == DKS_MODEL_KSSO ? 2 : 4;
    DKS_REQUIRE(n >= 1 && n <= 170 && n <= ncomp * s.N, DKS_EINVAL,
                "n must be in [1, min(170, ncomp N)] (subspace dimension 3n <= 512)");
    DKS_REQUIRE(o.n_init >= 0 && o.n_iter >= 0 && o.tol > 0, DKS_EINVAL, "bad options");
    DKS_REQUIRE(o.mode >= 0 && o.mode <= 2, DKS_EINVAL, "bad mode");
    DKS_REQUIRE(o.n_buffer >= 0 && o.n_buffer < n, DKS_EINVAL, "n_buffer must be in [0, n)");
    dks_solve_info inf{};
    inf.min_ritz = std::numeric_limits<double>::infinity();
    Ctx x;
    x.b = b;
    x.sys = sys;
    x.st = st;
    x.sv = sv;
    x.o = &o;
    x.info = &inf;
    x.N = s.N;
    x.ncomp = ncomp;
    x.K = ncomp * (int64_t)s.N;
    x.split_rr = split_rr;
    // the KSSO operator is solved by standard LOBPCG (the paper's comparison):
    // no filter, no kinetic balance, and (no negative band) the breakdown guard on
    x.filt = o.use_filter != 0 && ncomp == 4;
    x.guard = x.filt || ncomp == 2;
    x.c2 = s.c * s.c;
    double C0, O0;
    dks_filter_constants(b, sys, &C0, &O0);
    x.C = std::isnan(o.C) ? C0 : o.C;
    x.Om = std::isnan(o.Omega) ? O0 : o.Omega;
    DKS_REQUIRE(std::isfinite(x.C) && std::isfinite(x.Om) && x.Om != 0.0, DKS_EINVAL, "bad C or Omega");
    inf.C = x.C;
    inf.Omega = x.Om;
    x.iter_cap = o.n_iter + (o.mode != DKS_MODE_FP64 ? o.mixed_iter : 0);
    x.floor = x.filt ? -x.c2 : -std::numeric_limits<double>::infinity();
    if (o.kinetic_balance && ncomp == 4) kinetic_balance(b, sys, Xu, n, st);
    dks_status rc = DKS_OK;
    LoopState<double> s64;
    DKS_REQUIRE(o.preconditioner == DKS_PRECOND_DEFAULT || o.preconditioner == DKS_PRECOND_NONE ||
                    o.preconditioner == DKS_PRECOND_TETER,
                DKS_EINVAL, "preconditioner must be DKS_PRECOND_DEFAULT, _NONE or _TETER");
    DKS_REQUIRE(o.method == DKS_METHOD_LOBPCG || o.method == DKS_METHOD_DAVIDSON, DKS_EINVAL,
                "bad method");
    if (o.method == DKS_METHOD_DAVIDSON) {
      DKS_REQUIRE(o.mode == DKS_MODE_FP64, DKS_EINVAL, "the Davidson form runs in FP64 only");
      const int max_dim = std::min(510, std::max(2, o.davidson_dim) * n);
      DKS_REQUIRE(max_dim >= 2 * n, DKS_EINVAL, "Davidson subspace too small (davidson_dim n > 510)");
      x.sv->b64.ensure(n, x.K);
      DKS_HIP(hipMemcpyAsync(x.sv->b64.z(0, 0), Xu, sizeof(double2) * x.K * n, hipMemcpyDeviceToDevice, st));
      rc = run_davidson(x, x.sv->b64, s64, n, o.n_init, o.tol, o.n_iter, max_dim);
    } else if (o.mode == DKS_MODE_FP64) {
      x.sv->b64.ensure(n, x.K);
      DKS_HIP(hipMemcpyAsync(x.sv->b64.z(0, 0), Xu, sizeof(double2) * x.K * n, hipMemcpyDeviceToDevice, st));
      rc = run_stage<double>(x, x.sv->b64, s64, n, o.n_init, o.tol, o.n_iter, 1e-10, kStallFp64,
                              kStallRestartFp64);
    } else {
      // reduced-precision stage
      x.sv->b32.ensure(n, x.K);
      LoopState<float> s32;
      convert<double, float>(Xu, x.sv->b32.z(0, 0), x.K * n, st);
      const bool fixed = !(o.mixed_tol > 0);   // mixed_tol <= 0: exactly mixed_iter iterations
      x.bf16_gram = (o.mode == DKS_MODE_MIXED_BF16GRAM);
      run_stage<float>(x, x.sv->b32, s32, n, o.n_init, fixed ? 0.0 : o.mixed_tol, o.mixed_iter, 1e-5,
                       fixed ? 0 : kStallFp32, 0);
      inf.iters_reduced = s32.iters;
      x.bf16_gram = false;
      // FP64 polish.  The reduced-precision block carries rounding noise of
      // relative size up to ~1e-7 in every direction, including the negative
      // band, where the residual amplifies it by ~2c^2 (the gamma_LOBPCG ~ Delta/w
      // of Sec. 3.1) and where Y and P, being filtered, cannot remove it.  Two
      // filter applications in FP64 (each damping the negative band by
      // ~(w/2c^2)^2) push it far below the FP64 tolerance.
      x.sv->b64.ensure(n, x.K);
      convert<float, double>(x.sv->b32.z(s32.cur, 0), x.sv->b64.z(0, 0), x.K * n, st);
      s64.iters = 0;
      rc = run_stage<double>(x, x.sv->b64, s64, n, kPolishFilters, o.tol, o.n_iter, 1e-10, kStallFp64,
                              kStallRestartFp64);
    }
    Blocks<double> &bk = x.sv->b64;
    DKS_HIP(hipMemcpyAsync(Xu, bk.z(s64.cur, 0), sizeof(double2) * x.K * n, hipMemcpyDeviceToDevice, st));
    DKS_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < n; ++j) lambda[j] = s64.lam[j];
    double mx = 0;
    int nconv = 0;
    const int nwant = n - o.n_buffer;
    for (int j = 0; j < n; ++j) {
      if (resnorms) resnorms[j] = s64.res[j];
      if (j >= nwant) continue;
      mx = std::max(mx, s64.res[j]);
      if (s64.res[j] < o.tol) ++nconv;
    }
    inf.converged = (nconv == nwant);
    inf.n_converged = nconv;
    inf.max_resnorm = mx;
    if (info) *info = inf;
    for (int j = 0; j < n; ++j)
      if (lambda[j] < -x.c2) {
        msg = "a Ritz value fell below -c^2 (variational collapse)";
        return DKS_ECOLLAPSE;
      }
    if (rc != DKS_OK) msg = "iteration limit reached before every residual fell below tol";
    return rc;
  }
}



// ---------------------------------------------------------------------------
// batches: lanes, and the graph-captured lockstep form
// ---------------------------------------------------------------------------
static BatchLanes &lanes_of(dks_basis *b) {
  SolverSet *set = solvers_of(b);
  if (!set->lanes) {
    auto *bl = new BatchLanes();
    set->lanes = bl;
    for (int l = 0; l < batch_lanes(); ++l) {
      DKS_HIP(hipStreamCreateWithFlags(&bl->lane[l].st, hipStreamNonBlocking));
      DKS_HIP(hipEventCreateWithFlags(&bl->lane[l].done, hipEventDisableTiming));
    }
  }
  return *set->lanes;
}

// Solves items[] of a batch on the lanes (a stream and a host thread each; a
// free lane takes the next item, largest 4N n^2 first), item i with options
// opt[i]; the lanes start after the work queued on `cst`, and `cst` waits for
// them.  Statuses and messages go to rc[i], msg[i].
static void run_on_lanes(dks_basis *b, const std::vector<int> &items, const int *sys, const int *n,
                         void *const *X, double *const *lambda, double *const *resnorms,
                         const std::vector<dks_solve_opts> &opt, dks_solve_info *info,
                         hipStream_t cst, std::vector<dks_status> &rc,
                         std::vector<std::string> &msg) {
  const int ni = (int)items.size();
  if (ni == 0) return;
  BatchLanes &bl = lanes_of(b);
  const int L = std::min(batch_lanes(), ni);
  hipEvent_t start;
  DKS_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  DKS_HIP(hipEventRecord(start, cst));
  for (int l = 0; l < L; ++l) DKS_HIP(hipStreamWaitEvent(bl.lane[l].st, start, 0));
  // items are taken in turn by whichever lane is free, the largest first
  // (work ~ K n^2 per iteration), so that uneven sizes even out over lanes
  std::vector<int> order(items);
  auto work = [&](int i) {
    const double K = 4.0 * b->sys[sys[i]]->N;
    return K * (double)n[i] * (double)n[i];
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work(a) > work(c); });
  std::atomic<int> next{0};
  auto run_lane = [&](int l) {
    const bool dev_ok = hipSetDevice(b->device) == hipSuccess;
    for (int q = next++; q < ni; q = next++) {
      const int i = order[q];
      if (!dev_ok) {
        rc[i] = DKS_EHIP;
        continue;
      }
      try {
        rc[i] = solve_one(b, sys[i], n[i], (double2 *)X[i], lambda[i],
                          resnorms ? resnorms[i] : nullptr, opt[i], info ? &info[i] : nullptr,
                          bl.lane[l].st, &bl.lane[l].sv, msg[i]);
      } catch (...) {   // nothing may escape a lane thread
        rc[i] = status_of_current_exception(msg[i]);
      }
    }
  };
  // a lane thread that cannot start leaves its items to the running lanes
  std::vector<std::thread> th;
  for (int l = 1; l < L; ++l) {
    try {
      th.emplace_back(run_lane, l);
    } catch (...) {
      break;
    }
  }
  run_lane(0);
  for (auto &t : th) t.join();
  for (int l = 0; l < L; ++l) {
    DKS_HIP(hipEventRecord(bl.lane[l].done, bl.lane[l].st));
    DKS_HIP(hipStreamWaitEvent(cst, bl.lane[l].done, 0));
  }
  DKS_HIP(hipEventDestroy(start));
}

// ---- the graph-captured lockstep form --------------------------------------
//
// Every item iterates Algorithm 1 on a fixed shape: the subspace is always
// [X, Y, P] of 3n rows (P = 0 in the first step, whose zero columns the
// Rayleigh-Ritz drops as dependent; the Y and P columns of converged columns
// are zero likewise, k_graph_lock), and P is kept orthogonal to X.  Each
// iteration is then the same sequence of launches with the same sizes, so the
// iterations of a group of items can be captured once into one HIP graph on
// the group's stream and replayed (the groups run concurrently).  Two device kernels per iteration make the decisions the host
// makes on the lanes: k_graph_check after the Rayleigh-Ritz (failed
// factorisation, or a Ritz value below its predecessor by more than the block
// residual allows) and k_graph_step after the residual norms (convergence of
// the wanted columns, stagnation, iteration cap).  A decision sets the item's
// skip flag, which every later kernel of the item reads first: a finished item
// costs empty launches.  The host waits once per graph launch, for the flags.

// per-item device flags (ints) and state (doubles)
enum { kGfSkip = 0, kGfStatus, kGfIters, kGfStall, kGfXbuf, kGfBestNact, kGfCount = 8 };
enum { kGsBest = 0, kGsRf, kGsResMax, kGsLam, kGsCount = kGsLam + 172 };

// A broken-down step (the recurrences for H X and H P drifted in an
// ill-conditioned basis, so the projected pencil no longer compresses H) shows
// as Ritz values below the spectrum: the lowest positive-band eigenvalue is at
// least min V_loc - ||V_NL|| (the kinetic part is >= 0 there), `lower`.  (A
// Ritz value may legitimately fall by more than the block residual when the
// subspace finds an eigenvalue the block had missed, which the graph form,
// iterating every column, does often; so the bound is on the spectrum.)
__global__ void k_graph_check(const int *__restrict__ info, const double *__restrict__ theta,
                              int *__restrict__ flags, double *__restrict__ state, int n, int cur,
                              int guard, double lower) {
  if (threadIdx.x != 0 || flags[kGfSkip]) return;
  int status = 0;
  if (info[1] != 0) {
    status = 2;   // too few independent directions, or too few Ritz values above the floor
  } else if (guard && n > 0 && theta[0] < lower) {
    status = 3;
  }
  if (status) {
    flags[kGfStatus] = status;
    flags[kGfXbuf] = cur;   // the last good block is still the one this step read
    flags[kGfSkip] = 1;
  }
}

__global__ void k_graph_step(const double *__restrict__ norm2, const double *__restrict__ theta,
                             int *__restrict__ flags, double *__restrict__ state, int n, int nwant,
                             double tol, int cap, int stall_window, int nxt, int init, int guard) {
  __shared__ double act[kGsCount - kGsLam];
  if (threadIdx.x != 0 || flags[kGfSkip]) return;
  double rf2 = 0, mx = 0;
  int nact = 0;
  bool conv = true;
  for (int j = 0; j < n; ++j) {
    const double r = sqrt(fmax(norm2[j], 0.0));
    rf2 += r * r;
    if (j < nwant) mx = fmax(mx, r);   // buffer columns may rotate between states freely
    if (j < nwant && !(r < tol)) {
      conv = false;
      act[nact++] = r;
    }
  }
  // median of the wanted residuals not yet below tol (insertion sort, n <= 170)
  for (int a = 1; a < nact; ++a) {
    const double v = act[a];
    int c = a - 1;
    while (c >= 0 && act[c] > v) {
      act[c + 1] = act[c];
      --c;
    }
    act[c + 1] = v;
  }
  const double level = nact ? act[nact / 2] : 0.0;
  int status = 0, xbuf = nxt;
  if (!init) {
    flags[kGfIters] += 1;
    if (guard && !(mx <= 1e3 * state[kGsResMax])) {
      status = 6;   // wanted residuals jumped: the step broke down, keep the block it read
      xbuf = 1 - nxt;
    }
  }
  if (!status) {
    for (int j = 0; j < n; ++j) state[kGsLam + j] = theta[j];
    state[kGsRf] = sqrt(rf2);
    state[kGsResMax] = mx;
    if (conv) {
      status = 1;
    } else if (!init && flags[kGfIters] >= cap) {
      status = 5;
    } else if (init || nact < flags[kGfBestNact]) {
      flags[kGfBestNact] = nact;
      state[kGsBest] = level;
      flags[kGfStall] = 0;
    } else if (level < 0.95 * state[kGsBest]) {
      state[kGsBest] = level;
      flags[kGfStall] = 0;
    } else if (stall_window > 0 && ++flags[kGfStall] >= stall_window) {
      status = 4;
    }
  }
  if (status) {
    flags[kGfStatus] = status;
    flags[kGfXbuf] = xbuf;
    flags[kGfSkip] = 1;
  }
}

template <typename T>
__global__ void k_zero_rows(cplx<T> *__restrict__ X, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) X[i] = cplx<T>{0, 0};
}

struct GraphItem {
  int idx = 0;        // batch item
  int sys = 0, n = 0, nwant = 0;
  hipStream_t st = nullptr;
  Solver *sv = nullptr;
  Ctx x;              // operator context (filter constants, component count)
  int *flags = nullptr;
  double *state = nullptr;
  double lower = 0;   // lower bound of the positive band (Ha, shifted)
};

struct GraphPool {
  std::vector<Solver *> solvers;
  std::vector<hipStream_t> streams;
  DevBuf gflags, gstate;
  HostBuf hflags;
  hipStream_t origin = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  ~GraphPool() {
    for (auto *sv : solvers) delete sv;
    for (auto st : streams) (void)hipStreamDestroy(st);
    for (auto e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (origin) (void)hipStreamDestroy(origin);
  }
  void ensure(int count) {
    while ((int)solvers.size() < count) solvers.push_back(new Solver());
    while ((int)streams.size() < count) {
      hipStream_t st;
      DKS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      streams.push_back(st);
    }
    while ((int)join.size() < count) {
      hipEvent_t e;
      DKS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      join.push_back(e);
    }
    if (!origin) DKS_HIP(hipStreamCreateWithFlags(&origin, hipStreamNonBlocking));
    if (!fork) DKS_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  }
};

SolverSet::~SolverSet() {
  delete lanes;
  delete graph;
}

// Buffers of one item in precision T sized for the fixed-shape iteration, so
// that nothing is allocated while it is captured.
template <typename T>
static void graph_reserve(GraphItem &g, Blocks<T> &bk) {
  Solver &sv = *g.sv;
  const int n = g.n, nz = 3 * n;
  const int64_t K = g.x.K;
  bk.ensure(n, K);
  sv.gS.ensure(sizeof(double2) * nz * nz);
  sv.gA.ensure(sizeof(double2) * nz * nz);
  sv.Vz.ensure(sizeof(double2) * nz * n);
  sv.Wxp.ensure(sizeof(double2) * n * n);
  sv.theta.ensure(sizeof(double) * n);
  sv.norms.ensure(sizeof(double) * n);
  sv.lockmask.ensure(sizeof(int) * n);
  sv.pE.ensure(sizeof(double2) * n * kTpaMaxBlocks);
  sv.rinfo.ensure(sizeof(int) * 4);
  sv.rdinfo.ensure(sizeof(double) * 2);
  sv.rrs.ensure(rr_scratch_bytes(nz, n));
  sv.part.ensure(sizeof(double2) * std::max(gemm_ip_part_elems(nz, nz, K, true, true),
                                            gemm_ip_part_elems(n, n, K, false, false)));
  sv.part2.ensure(sizeof(double) * (size_t)n * (size_t)((K + 8191) / 8192));
}

// Soft locking on the fixed shape: columns j whose residual is below tol get
// no search direction, as on the lanes (the active set of Algorithm 1).  Their
// rows of the next Y (the residual, filtered in place next step) and of P and
// H P are cleared; the Rayleigh-Ritz drops zero columns as dependent, as it
// does for P = 0 in the first step.  Without this, converged columns keep
// residual directions made of rounding noise in the basis, whose Gram and
// projected matrix then lose the H-consistency of the H X recurrence and the
// iteration breaks down (Ritz values inside the gap below the positive band).
// `mask[j]` records the decision; the next iteration's grid transforms skip
// the locked bands (their Y rows are zero).
template <typename T>
__global__ void k_graph_lock(cplx<T> *__restrict__ Y, cplx<T> *__restrict__ P,
                             cplx<T> *__restrict__ HP, const double *__restrict__ norm2, int64_t K,
                             double tol2, int *__restrict__ mask, const int *__restrict__ skip) {
  if (skip && *skip) return;
  const int j = blockIdx.y;
  const bool locked = norm2[j] < tol2;
  if (blockIdx.x == 0 && threadIdx.x == 0) mask[j] = locked ? 1 : 0;
  if (!locked) return;   // active: keeps its directions
  const size_t o = (size_t)j * K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < K;
       e += (int64_t)gridDim.x * blockDim.x) {
    Y[o + e] = cplx<T>{0, 0};
    if (P) {
      P[o + e] = cplx<T>{0, 0};
      HP[o + e] = cplx<T>{0, 0};
    }
  }
}
template <typename T>
static void graph_lock(GraphItem &g, Blocks<T> &bk, int q, double tol, bool with_p) {
  const int n = g.n;
  const int64_t K = g.x.K;
  const unsigned gx = (unsigned)std::min<int64_t>(64, (K + 255) / 256);
  DKS_LAUNCH("k_graph_lock", k_graph_lock<T>, dim3(gx, n), dim3(256), 0, g.st, bk.z(q, n),
             with_p ? bk.z(q, 2 * n) : nullptr, with_p ? bk.hz(q, 2 * n) : nullptr,
             g.sv->norms.as<double>(), K, tol * tol, g.sv->lockmask.as<int>(), g.flags + kGfSkip);
  DKS_HIP(hipGetLastError());
}

// One iteration of item g reading Z[p], writing Z[1 - p]; every launch is
// skipped once the item's flag is set.
template <typename T>
static void graph_iteration(GraphItem &g, Blocks<T> &bk, int p, double tol, int cap,
                            int stall_window, double drop_tol) {
  Solver &sv = *g.sv;
  Ctx &x = g.x;
  const int n = g.n, nz = 3 * n, q = 1 - p;
  const int64_t K = x.K;
  const int *skip = g.flags + kGfSkip;
  hipStream_t st = g.st;
  cplx<T> *Y = bk.z(p, n), *HY = bk.hz(p, n);
  // the locked bands' Y rows are zero: their grid transforms are skipped
  const int *lk = sv.lockmask.as<int>();
  if (use_teter(*x.o)) precondition<T>(x.b, x.sys, Y, n, st, x.ncomp, sv.pE.as<double2>(), skip);
  if (x.filt) {
    apply_h<T>(x.b, x.sys, Y, bk.W.template as<cplx<T>>(), n, x.C, 1.0, st, sv.ws, x.ncomp, skip,
               lk);
    apply_h<T>(x.b, x.sys, bk.W.template as<cplx<T>>(), Y, n, x.C, 1.0 / (x.Om * x.Om), st, sv.ws,
               x.ncomp, skip, lk);
  }
  apply_h<T>(x.b, x.sys, Y, HY, n, 0.0, 1.0, st, sv.ws, x.ncomp, skip, lk);
  gemm_ip<T>(bk.z(p, 0), nullptr, nz, bk.z(p, 0), nullptr, nz, bk.hz(p, 0), K, sv.gS.as<double2>(),
             sv.gA.as<double2>(), nz, sv.part, st, /*hermitian=*/true, skip);
  rayleigh_ritz(sv.gA.as<double2>(), sv.gS.as<double2>(), nz, n, drop_tol, x.floor, nullptr,
                sv.Vz.as<double2>(), sv.theta.as<double>(), sv.rinfo.as<int>(),
                sv.rdinfo.as<double>(), sv.rrs, st, nullptr, skip);
  DKS_LAUNCH("k_graph_check", k_graph_check, dim3(1), dim3(64), 0, st, sv.rinfo.as<int>(),
             sv.theta.as<double>(), g.flags, g.state, n, p, x.guard ? 1 : 0, g.lower);
  DKS_HIP(hipGetLastError());
  // X = Z V, H X alike; P = [Y, P] V (the rows of V below the X block); then
  // P and H P made orthogonal to the new X
  gemm_up2<T>(bk.z(p, 0), bk.hz(p, 0), nullptr, nz, sv.Vz.as<double2>(), n, n, K, bk.z(q, 0),
              bk.hz(q, 0), K, 0.0, st, 1.0, nullptr, skip);
  gemm_up2<T>(bk.z(p, n), bk.hz(p, n), nullptr, nz - n, sv.Vz.as<double2>() + (size_t)n * n, n, n,
              K, bk.z(q, 2 * n), bk.hz(q, 2 * n), K, 0.0, st, 1.0, nullptr, skip);
  gemm_ip<T>(bk.z(q, 0), nullptr, n, bk.z(q, 2 * n), nullptr, n, nullptr, K, sv.Wxp.as<double2>(),
             nullptr, n, sv.part, st, false, skip);
  gemm_up2<T>(bk.z(q, 0), bk.hz(q, 0), nullptr, n, sv.Wxp.as<double2>(), n, n, K, bk.z(q, 2 * n),
              bk.hz(q, 2 * n), K, 1.0, st, -1.0,
              sizeof(T) == 8 ? "k_gemm_up.portho.f64" : "k_gemm_up.portho.f32", skip);
  // R = H X - X Lambda, written where the next step's Y goes
  residual<T>(bk.z(q, 0), bk.hz(q, 0), sv.theta.as<double>(), n, K, bk.z(q, n),
              sv.norms.as<double>(), sv.part2, st, skip);
  graph_lock<T>(g, bk, q, tol, true);
  DKS_LAUNCH("k_graph_step", k_graph_step, dim3(1), dim3(64), 0, st, sv.norms.as<double>(),
             sv.theta.as<double>(), g.flags, g.state, n, g.nwant, tol, cap, stall_window, q, 0,
             x.guard ? 1 : 0);
  DKS_HIP(hipGetLastError());
}

// The start of a graph stage for item g, eager on its stream: the block is in
// Z[0] rows [0, n); n_init filter passes, H X, the Rayleigh-Ritz on X alone,
// X = X V into Z[1], P = 0, R into Z[1]'s Y rows, and the first decisions.
template <typename T>
static void graph_start(GraphItem &g, Blocks<T> &bk, int n_init, double tol, double drop_tol) {
  Solver &sv = *g.sv;
  Ctx &x = g.x;
  const int n = g.n;
  const int64_t K = x.K;
  hipStream_t st = g.st;
  if (x.filt)
    for (int k = 0; k < n_init; ++k) filter_inplace<T>(x, bk.z(0, 0), bk.W.template as<cplx<T>>(), n);
  apply_h<T>(x.b, x.sys, bk.z(0, 0), bk.hz(0, 0), n, 0.0, 1.0, st, sv.ws, x.ncomp);
  gemm_ip<T>(bk.z(0, 0), nullptr, n, bk.z(0, 0), nullptr, n, bk.hz(0, 0), K, sv.gS.as<double2>(),
             sv.gA.as<double2>(), n, sv.part, st, true);
  rayleigh_ritz(sv.gA.as<double2>(), sv.gS.as<double2>(), n, n, drop_tol, x.floor, nullptr,
                sv.Vz.as<double2>(), sv.theta.as<double>(), sv.rinfo.as<int>(),
                sv.rdinfo.as<double>(), sv.rrs, st);
  // a failed start leaves the item at status 2 with its block in Z[0]
  DKS_LAUNCH("k_graph_check", k_graph_check, dim3(1), dim3(64), 0, st, sv.rinfo.as<int>(),
             sv.theta.as<double>(), g.flags, g.state, n, 0, 0, g.lower);
  const int *skip = g.flags + kGfSkip;
  gemm_up2<T>(bk.z(0, 0), bk.hz(0, 0), nullptr, n, sv.Vz.as<double2>(), n, n, K, bk.z(1, 0),
              bk.hz(1, 0), K, 0.0, st, 1.0, nullptr, skip);
  const int64_t cnt = (int64_t)n * K;
  DKS_LAUNCH("k_zero_rows", k_zero_rows<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
             bk.z(1, 2 * n), cnt);
  DKS_LAUNCH("k_zero_rows", k_zero_rows<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st,
             bk.hz(1, 2 * n), cnt);
  residual<T>(bk.z(1, 0), bk.hz(1, 0), sv.theta.as<double>(), n, K, bk.z(1, n),
              sv.norms.as<double>(), sv.part2, st, skip);
  graph_lock<T>(g, bk, 1, tol, false);
  DKS_LAUNCH("k_graph_step", k_graph_step, dim3(1), dim3(64), 0, st, sv.norms.as<double>(),
             sv.theta.as<double>(), g.flags, g.state, n, g.nwant, tol, 1 << 30, 0, 1, 1,
             x.guard ? 1 : 0);
  DKS_HIP(hipGetLastError());
}

// Runs one graph stage in precision T for every item: the eager start, one
// eager iteration (which also sizes every buffer), then one graph per group of
// items (the items of a group one after another on the group's stream, which
// every item of the group uses), each holding `chunk` iterations of its items,
// captured once and launched on its stream until every item has left.  The
// groups run concurrently, one stream each.  Returns the iterations each item
// took (through its flags).
template <typename T>
static void graph_stage(GraphPool &pool, std::vector<GraphItem> &items,
                        std::vector<Blocks<T> *> &blk, int n_init, double tol, int cap,
                        int stall_window, double drop_tol, int chunk, int *flags_h,
                        const std::vector<std::vector<int>> &groups) {
  const int ni = (int)items.size();
  const int nf = kGfCount * ni;
  const auto t_begin = std::chrono::steady_clock::now();
  // reset the flags and state of every item
  {
    std::vector<int> f0(nf, 0);
    DKS_HIP(hipMemcpyAsync(pool.gflags.p, f0.data(), sizeof(int) * nf, hipMemcpyHostToDevice,
                           pool.origin));
    DKS_HIP(hipStreamSynchronize(pool.origin));
  }
  for (int i = 0; i < ni; ++i) {
    graph_reserve<T>(items[i], *blk[i]);
    graph_start<T>(items[i], *blk[i], n_init, tol, drop_tol);
    // one eager iteration: Z[1] -> Z[0]
    graph_iteration<T>(items[i], *blk[i], 1, tol, cap, stall_window, drop_tol);
  }
  for (int i = 0; i < ni; ++i) DKS_HIP(hipStreamSynchronize(items[i].st));
  // capture `chunk` iterations of the items of each group (Z[0] -> Z[1] ->
  // Z[0] ...) on the group's stream
  const int ng = (int)groups.size();
  std::vector<hipGraph_t> graphs(ng, nullptr);
  std::vector<hipGraphExec_t> execs(ng, nullptr);
  auto destroy = [&]() {
    for (auto &e : execs)
      if (e) (void)hipGraphExecDestroy(e), e = nullptr;
    for (auto &g : graphs)
      if (g) (void)hipGraphDestroy(g), g = nullptr;
  };
  try {
    ProfPause no_events;
    for (int gi = 0; gi < ng; ++gi) {
      hipStream_t gs = items[groups[gi][0]].st;
      DKS_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
      try {
        for (int i : groups[gi])
          for (int k = 0; k < chunk; ++k)
            graph_iteration<T>(items[i], *blk[i], k & 1, tol, cap, stall_window, drop_tol);
      } catch (...) {
        hipGraph_t dead = nullptr;
        (void)hipStreamEndCapture(gs, &dead);
        if (dead) (void)hipGraphDestroy(dead);
        throw;
      }
      DKS_HIP(hipStreamEndCapture(gs, &graphs[gi]));
    }
  } catch (...) {
    destroy();
    throw;
  }
  const auto t_cap = std::chrono::steady_clock::now();
  try {
    for (int gi = 0; gi < ng; ++gi) DKS_HIP(hipGraphInstantiate(&execs[gi], graphs[gi], nullptr, nullptr, 0));
    int *hf = flags_h;
    // each round runs `chunk` iterations of every item still in the stage
    const auto t_inst = std::chrono::steady_clock::now();
    const int max_launch = cap / chunk + 2;
    int launches = 0;
    for (int l = 0; l < max_launch; ++l, ++launches) {
      DKS_HIP(hipMemcpyAsync(hf, pool.gflags.p, sizeof(int) * nf, hipMemcpyDeviceToHost,
                             pool.origin));
      DKS_HIP(hipStreamSynchronize(pool.origin));
      std::vector<int> live;
      for (int gi = 0; gi < ng; ++gi) {
        bool all = true;
        for (int i : groups[gi]) all = all && hf[kGfCount * i + kGfSkip];
        if (!all) live.push_back(gi);
      }
      if (live.empty()) break;
      for (int gi : live) DKS_HIP(hipGraphLaunch(execs[gi], items[groups[gi][0]].st));
      for (int gi : live) DKS_HIP(hipStreamSynchronize(items[groups[gi][0]].st));
    }
    DKS_HIP(hipStreamSynchronize(pool.origin));
    DKS_HIP(hipMemcpy(hf, pool.gflags.p, sizeof(int) * nf, hipMemcpyDeviceToHost));
    if (log_enabled()) {
      auto ms = [](auto a, auto b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
      std::fprintf(stderr,
                   "{\"graph_stage\": {\"prec\": %d, \"items\": %d, \"groups\": %d, \"chunk\": %d, "
                   "\"start_ms\": %.1f, \"instantiate_ms\": %.1f, \"rounds\": %d, \"run_ms\": %.1f}}\n",
                   (int)sizeof(T), ni, ng, chunk, ms(t_begin, t_cap), ms(t_cap, t_inst), launches,
                   ms(t_inst, std::chrono::steady_clock::now()));
    }
  } catch (...) {
    destroy();
    throw;
  }
  destroy();
}

// dks_lobpcgf_solve_batch with batch_graph = 1.
static void solve_batch_graph(dks_basis *b, int nsys, const int *sys, const int *n, void *const *X,
                              double *const *lambda, double *const *resnorms,
                              const std::vector<dks_solve_opts> &iopt, dks_solve_info *info,
                              hipStream_t cst, std::vector<dks_status> &rc,
                              std::vector<std::string> &msg) {
  const dks_solve_opts &o = iopt[0];   // shared options (n_buffer differs per item)
  SolverSet *set = solvers_of(b);
  if (!set->graph) set->graph = new GraphPool();
  GraphPool &pool = *set->graph;
  pool.ensure(nsys);
  const int chunk = std::max(2, o.graph_chunk + (o.graph_chunk & 1));
  DKS_REQUIRE(o.mode >= 0 && o.mode <= 2, DKS_EINVAL, "bad mode");
  DKS_REQUIRE(o.model == DKS_MODEL_DKS || o.model == DKS_MODEL_KSSO, DKS_EINVAL, "bad model");
  const int ncomp = o.model == DKS_MODEL_KSSO ? 2 : 4;
  pool.gflags.ensure(sizeof(int) * kGfCount * nsys);
  pool.gstate.ensure(sizeof(double) * kGsCount * nsys);
  int *hf = pool.hflags.as<int>((size_t)kGfCount * nsys);
  // the stage starts after the work queued on the caller's stream
  DKS_HIP(hipEventRecord(pool.fork, cst));
  // groups of items, one stream each: largest items first, dealt round-robin
  const int ngroups = std::max(1, std::min(nsys, batch_lanes()));
  std::vector<std::vector<int>> groups(ngroups);
  {
    std::vector<int> order(nsys);
    for (int i = 0; i < nsys; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
      return (int64_t)b->sys[sys[a]]->N * n[a] > (int64_t)b->sys[sys[c]]->N * n[c];
    });
    for (int q = 0; q < nsys; ++q) groups[q % ngroups].push_back(order[q]);
  }
  std::vector<int> group_of(nsys);
  for (int gi = 0; gi < ngroups; ++gi)
    for (int i : groups[gi]) group_of[i] = gi;
  std::vector<GraphItem> items(nsys);
  std::vector<dks_solve_info> inf(nsys);
  for (int i = 0; i < nsys; ++i) {
    const System &s = *b->sys[sys[i]];
    DKS_REQUIRE(n[i] >= 1 && n[i] <= 170 && n[i] <= ncomp * s.N, DKS_EINVAL,
                "batch item " + std::to_string(i) + ": n must be in [1, min(170, ncomp N)]");
    GraphItem &g = items[i];
    g.idx = i;
    g.sys = sys[i];
    g.n = n[i];
    g.nwant = n[i] - iopt[i].n_buffer;
    g.st = pool.streams[group_of[i]];
    g.sv = pool.solvers[i];
    g.flags = pool.gflags.as<int>() + kGfCount * i;
    g.state = pool.gstate.as<double>() + kGsCount * i;
    Ctx &x = g.x;
    x.b = b;
    x.sys = sys[i];
    x.st = g.st;
    x.sv = g.sv;
    x.o = &iopt[i];
    x.info = nullptr;
    x.N = s.N;
    x.ncomp = ncomp;
    x.K = ncomp * (int64_t)s.N;
    x.c2 = s.c * s.c;
    x.filt = o.use_filter != 0 && ncomp == 4;
    x.guard = x.filt || ncomp == 2;
    double C0, O0;
    dks_filter_constants(b, sys[i], &C0, &O0);
    x.C = std::isnan(o.C) ? C0 : o.C;
    x.Om = std::isnan(o.Omega) ? O0 : o.Omega;
    DKS_REQUIRE(std::isfinite(x.C) && std::isfinite(x.Om) && x.Om != 0.0, DKS_EINVAL,
                "bad C or Omega");
    x.floor = x.filt ? -x.c2 : -std::numeric_limits<double>::infinity();
    g.lower = b->pot[s.vsrc]->vmin - s.nl_bound - 1.0;
    inf[i] = dks_solve_info{};
    inf[i].min_ritz = std::numeric_limits<double>::infinity();
    inf[i].C = x.C;
    inf[i].Omega = x.Om;
    DKS_HIP(hipStreamWaitEvent(g.st, pool.fork, 0));
    if (o.kinetic_balance && ncomp == 4) kinetic_balance(b, sys[i], (double2 *)X[i], n[i], g.st);
  }
  std::vector<int> xbuf(nsys, 0), status(nsys, 0);
  const bool mixed = o.mode != DKS_MODE_FP64;
  int n_init64 = o.n_init;
  if (mixed) {
    // reduced-precision stage: FP32 to mixed_tol (or a stall), then FP64
    std::vector<Blocks<float> *> b32(nsys);
    for (int i = 0; i < nsys; ++i) {
      b32[i] = &items[i].sv->b32;
      b32[i]->ensure(n[i], items[i].x.K);
      convert<double, float>((const double2 *)X[i], b32[i]->z(0, 0), items[i].x.K * n[i], items[i].st);
    }
    const double t32 = o.mixed_tol > 0 ? o.mixed_tol : 0.0;
    graph_stage<float>(pool, items, b32, o.n_init, t32, std::max(2, o.mixed_iter), kStallFp32, 1e-5,
                       chunk, hf, groups);
    for (int i = 0; i < nsys; ++i) {
      const int xb = hf[kGfCount * i + kGfXbuf];
      inf[i].iters_reduced = hf[kGfCount * i + kGfIters];
      items[i].sv->b64.ensure(n[i], items[i].x.K);
      convert<float, double>(b32[i]->z(xb, 0), items[i].sv->b64.z(0, 0), items[i].x.K * n[i],
                             items[i].st);
    }
    n_init64 = kPolishFilters;
  } else {
    for (int i = 0; i < nsys; ++i) {
      items[i].sv->b64.ensure(n[i], items[i].x.K);
      DKS_HIP(hipMemcpyAsync(items[i].sv->b64.z(0, 0), X[i], sizeof(double2) * items[i].x.K * n[i],
                             hipMemcpyDeviceToDevice, items[i].st));
    }
  }
  std::vector<Blocks<double> *> b64(nsys);
  for (int i = 0; i < nsys; ++i) b64[i] = &items[i].sv->b64;
  graph_stage<double>(pool, items, b64, n_init64, o.tol, std::max(2, o.n_iter), kStallFp64, 1e-10,
                      chunk, hf, groups);
  // results: converged items straight from the device; the others go back to
  // the lanes from their last good block (a filtered restart)
  std::vector<int> left;
  std::vector<dks_solve_opts> opt(iopt);
  for (int i = 0; i < nsys; ++i) {
    GraphItem &g = items[i];
    const int *f = hf + kGfCount * i;
    status[i] = f[kGfStatus];
    xbuf[i] = f[kGfXbuf];
    inf[i].graph_exit = status[i];
    inf[i].graph_iterations = f[kGfIters] + inf[i].iters_reduced;
    inf[i].iterations = inf[i].graph_iterations;
    const int64_t K = g.x.K;
    DKS_HIP(hipMemcpyAsync(X[i], g.sv->b64.z(xbuf[i], 0), sizeof(double2) * K * n[i],
                           hipMemcpyDeviceToDevice, g.st));
    if (status[i] == 1) {
      std::vector<double> th(n[i]), r2(n[i]);
      DKS_HIP(hipMemcpyAsync(th.data(), g.sv->theta.p, sizeof(double) * n[i], hipMemcpyDeviceToHost, g.st));
      DKS_HIP(hipMemcpyAsync(r2.data(), g.sv->norms.p, sizeof(double) * n[i], hipMemcpyDeviceToHost, g.st));
      DKS_HIP(hipStreamSynchronize(g.st));
      double mx = 0, mn = std::numeric_limits<double>::infinity();
      int nconv = 0;
      for (int j = 0; j < n[i]; ++j) {
        lambda[i][j] = th[j];
        const double r = std::sqrt(std::max(r2[j], 0.0));
        if (resnorms) resnorms[i][j] = r;
        mn = std::min(mn, th[j]);
        if (j < g.nwant) {
          mx = std::max(mx, r);
          if (r < o.tol) ++nconv;
        }
      }
      inf[i].converged = 1;
      inf[i].n_converged = nconv;
      inf[i].max_resnorm = mx;
      inf[i].min_ritz = mn;
      inf[i].h_applies = inf[i].iterations * n[i] * (g.x.filt ? 3 : 1);
      rc[i] = DKS_OK;
    } else {
      DKS_HIP(hipStreamSynchronize(g.st));
      left.push_back(i);
      dks_solve_opts &oi = opt[i];
      oi.mode = DKS_MODE_FP64;
      oi.n_init = kPolishFilters;
      oi.kinetic_balance = 0;
      oi.n_iter = std::max(20, o.n_iter - f[kGfIters]);
    }
  }
  for (int i = 0; i < nsys; ++i) {
    DKS_HIP(hipEventRecord(pool.join[i], items[i].st));
    DKS_HIP(hipStreamWaitEvent(cst, pool.join[i], 0));
  }
  std::vector<dks_solve_info> lane_inf(nsys);
  run_on_lanes(b, left, sys, n, X, lambda, resnorms, opt, lane_inf.data(), cst, rc, msg);
  for (int i : left) {
    const int gi = inf[i].graph_iterations, ge = inf[i].graph_exit, ir = inf[i].iters_reduced;
    inf[i] = lane_inf[i];
    inf[i].graph_iterations = gi;
    inf[i].graph_exit = ge;
    inf[i].iterations += gi;
    inf[i].iters_reduced += ir;
  }
  if (info)
    for (int i = 0; i < nsys; ++i) info[i] = inf[i];
}

}  // namespace dks

using namespace dks;

extern "C" {

void dks_free_solver(dks_basis *b) {
  if (b && b->solver) {
    delete static_cast<SolverSet *>(b->solver);
    b->solver = nullptr;
  }
}

void dks_default_opts(dks_solve_opts *o) {
  if (!o) return;
  o->C = std::numeric_limits<double>::quiet_NaN();
  o->Omega = std::numeric_limits<double>::quiet_NaN();
  o->n_init = 3;
  o->n_iter = 200;
  o->tol = 1e-8;
  o->mode = DKS_MODE_FP64;
  o->mixed_tol = 3e-4;
  o->mixed_iter = 200;
  o->kinetic_balance = 0;
  o->use_filter = 1;
  o->model = DKS_MODEL_DKS;
  o->batch_graph = 0;
  o->graph_chunk = 8;
  o->item_buffer = nullptr;
  o->method = DKS_METHOD_LOBPCG;
  o->davidson_dim = 4;
  o->preconditioner = DKS_PRECOND_DEFAULT;
  o->n_buffer = 0;
}

dks_status dks_apply_H(dks_basis *b, int sys, const void *X, void *HX, int nb, dks_prec prec,
                       void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && X && HX && sys >= 0 && sys < (int)b->sys.size() && nb >= 0, DKS_EINVAL,
                "bad argument");
    DKS_REQUIRE(X != HX, DKS_EINVAL, "X and HX must not overlap");
    DKS_HIP(hipSetDevice(b->device));
    hipStream_t st = (hipStream_t)stream;
    if (prec == DKS_FP64)
      apply_h<double>(b, sys, (const double2 *)X, (double2 *)HX, nb, 0.0, 1.0, st, b->ws);
    else
      apply_h<float>(b, sys, (const float2 *)X, (float2 *)HX, nb, 0.0, 1.0, st, b->ws);
    return DKS_OK;
  });
}

dks_status dks_apply_H_ksso(dks_basis *b, int sys, const void *X, void *HX, int nb, dks_prec prec,
                            void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && X && HX && sys >= 0 && sys < (int)b->sys.size() && nb >= 0, DKS_EINVAL,
                "bad argument");
    DKS_REQUIRE(X != HX, DKS_EINVAL, "X and HX must not overlap");
    DKS_HIP(hipSetDevice(b->device));
    hipStream_t st = (hipStream_t)stream;
    if (prec == DKS_FP64)
      apply_h<double>(b, sys, (const double2 *)X, (double2 *)HX, nb, 0.0, 1.0, st, b->ws, 2);
    else
      apply_h<float>(b, sys, (const float2 *)X, (float2 *)HX, nb, 0.0, 1.0, st, b->ws, 2);
    return DKS_OK;
  });
}

dks_status dks_apply_filter(dks_basis *b, int sys, const void *Y, void *FY, int nb, double C,
                            double Omega, dks_prec prec, void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && Y && FY && sys >= 0 && sys < (int)b->sys.size() && nb >= 0, DKS_EINVAL,
                "bad argument");
    DKS_REQUIRE(Y != FY, DKS_EINVAL, "Y and FY must not overlap");
    DKS_REQUIRE(std::isfinite(C) && std::isfinite(Omega) && Omega != 0.0, DKS_EINVAL,
                "C and Omega must be finite, Omega nonzero");
    DKS_HIP(hipSetDevice(b->device));
    hipStream_t st = (hipStream_t)stream;
    const System &s = *b->sys[sys];
    const size_t K = 4 * (size_t)s.N;
    if (prec == DKS_FP64) {
      b->ftmp64.ensure(sizeof(double2) * K * nb);
      apply_h<double>(b, sys, (const double2 *)Y, b->ftmp64.as<double2>(), nb, C, 1.0, st, b->ws);
      apply_h<double>(b, sys, b->ftmp64.as<double2>(), (double2 *)FY, nb, C, 1.0 / (Omega * Omega), st,
                      b->ws);
    } else {
      b->ftmp32.ensure(sizeof(float2) * K * nb);
      apply_h<float>(b, sys, (const float2 *)Y, b->ftmp32.as<float2>(), nb, C, 1.0, st, b->ws);
      apply_h<float>(b, sys, b->ftmp32.as<float2>(), (float2 *)FY, nb, C, 1.0 / (Omega * Omega), st,
                     b->ws);
    }
    return DKS_OK;
  });
}

dks_status dks_precondition(dks_basis *b, int sys, void *Y, int nb, int model, dks_prec prec,
                            void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && Y && sys >= 0 && sys < (int)b->sys.size() && nb >= 0, DKS_EINVAL,
                "bad argument");
    DKS_REQUIRE(model == DKS_MODEL_DKS || model == DKS_MODEL_KSSO, DKS_EINVAL, "bad model");
    DKS_REQUIRE(prec == DKS_FP64 || prec == DKS_FP32, DKS_EINVAL, "bad precision");
    DKS_HIP(hipSetDevice(b->device));
    if (nb == 0) return DKS_OK;
    hipStream_t st = (hipStream_t)stream;
    const int ncomp = model == DKS_MODEL_DKS ? 4 : 2;
    b->pE.ensure(sizeof(double2) * nb * kTpaMaxBlocks);
    if (prec == DKS_FP64)
      precondition<double>(b, sys, (double2 *)Y, nb, st, ncomp, b->pE.as<double2>());
    else
      precondition<float>(b, sys, (float2 *)Y, nb, st, ncomp, b->pE.as<double2>());
    return DKS_OK;
  });
}

dks_status dks_lobpcgf_solve(dks_basis *b, int sys, int n, void *X, double *lambda,
                             double *resnorms, const dks_solve_opts *opts, dks_solve_info *info,
                             void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && X && lambda && sys >= 0 && sys < (int)b->sys.size(), DKS_EINVAL, "bad argument");
    dks_solve_opts o;
    if (opts) o = *opts; else dks_default_opts(&o);
    DKS_HIP(hipSetDevice(b->device));
    std::string msg;
    const dks_status rc = solve_one(b, sys, n, (double2 *)X, lambda, resnorms, o, info,
                                    (hipStream_t)stream, &solvers_of(b)->main, msg,
                                    /*split_rr=*/true);
    if (rc != DKS_OK) set_error(msg);
    return rc;
  });
}

dks_status dks_lobpcgf_solve_batch(dks_basis *b, int nsys, const int *sys, const int *n,
                                   void *const *X, double *const *lambda,
                                   double *const *resnorms, const dks_solve_opts *opts,
                                   dks_solve_info *info, void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && nsys >= 0 && (nsys == 0 || (sys && n && X && lambda)), DKS_EINVAL,
                "bad argument");
    for (int i = 0; i < nsys; ++i)
      DKS_REQUIRE(sys[i] >= 0 && sys[i] < (int)b->sys.size() && X[i] && lambda[i], DKS_EINVAL,
                  "bad system index or null block in the batch");
    if (nsys == 0) return DKS_OK;
    dks_solve_opts o;
    if (opts) o = *opts; else dks_default_opts(&o);
    o.iter_ms = nullptr;   // per-iteration times are a single-solve feature
    DKS_HIP(hipSetDevice(b->device));
    hipStream_t cst = (hipStream_t)stream;
    std::vector<dks_status> rc(nsys, DKS_OK);
    std::vector<std::string> msg(nsys);
    std::vector<dks_solve_opts> opt(nsys, o);
    for (int i = 0; i < nsys; ++i) {
      if (o.item_buffer) opt[i].n_buffer = o.item_buffer[i];
      opt[i].item_buffer = nullptr;
      DKS_REQUIRE(opt[i].n_buffer >= 0 && opt[i].n_buffer < n[i], DKS_EINVAL,
                  "batch item " + std::to_string(i) + ": n_buffer must be in [0, n)");
    }
    DKS_REQUIRE(!(o.batch_graph && o.method != DKS_METHOD_LOBPCG), DKS_EINVAL,
                "the graph-captured batch runs Algorithm 1 only (method = DKS_METHOD_LOBPCG)");
    if (o.batch_graph) {
      solve_batch_graph(b, nsys, sys, n, X, lambda, resnorms, opt, info, cst, rc, msg);
    } else {
      std::vector<int> all(nsys);
      for (int i = 0; i < nsys; ++i) all[i] = i;
      run_on_lanes(b, all, sys, n, X, lambda, resnorms, opt, info, cst, rc, msg);
    }
    // errors first (most negative), then warnings
    dks_status worst = DKS_OK;
    for (int i = 0; i < nsys; ++i) {
      const bool take = (rc[i] < 0 && (worst >= 0 || rc[i] < worst)) || (worst == DKS_OK && rc[i] > 0);
      if (take) {
        worst = rc[i];
        set_error("batch item " + std::to_string(i) + " (system " + std::to_string(sys[i]) +
                  "): " + msg[i]);
      }
    }
    return worst;
  });
}

}  // extern "C"
