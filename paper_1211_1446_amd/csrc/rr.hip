// Rayleigh-Ritz step of Algorithm 1 (the projected generalized eigenproblem on
// the subspace, sorted ascending) in FP64 on the device.
//
// Solves A v = theta S v for the nkeep lowest theta above `floor_val`, with
// A = Z^H H Z and S = Z^H Z of the current subspace Z = [X, Y, P], in one
// workgroup of 1024 threads:
//   1. symmetric diagonal scaling D S D, D = diag(S)^-1/2;
//   2. left-looking Cholesky D S D = L L^H; a column whose pivot falls below
//      `drop_tol` (its direction is numerically inside the span of the
//      earlier columns) is removed from the subspace instead of failing;
//   3. Li = L^-1 in place, C = Li (D A D) Li^H with LDS-tiled products that
//      skip the zero triangles;
//   4. Householder reduction C = Q T Q^H to a real symmetric tridiagonal T,
//      three workgroup barriers per reflector;
//   5. the wanted eigenvalues of T by multisection on Sturm counts: those
//      below floor_val (the mid-gap -c^2: negative-band Ritz values) are
//      skipped;
//   6. their eigenvectors by inverse iteration, re-orthogonalised inside
//      clusters of (nearly) equal eigenvalues such as Kramers pairs;
//   7. back-transformation v = D Li^H Q y, each column of y held in the
//      registers of a group of lanes while all reflectors are applied.
// Triangular factors and the Hermitian working matrix are packed lower
// triangles in LDS when n_Z <= 120, else full rows in the global scratch area.
#include <algorithm>
#include <cfloat>
#include <mutex>

#include "dks_internal.h"

namespace dks {

constexpr int kRRMax = 512;
constexpr int kRRThreads = 1024;
constexpr int kRRPackedMax = 120;   // packed triangles of up to this order live in LDS
constexpr int kGT = 64;             // workgroup GEMM output tile (2 x 2 outputs per thread)
constexpr int kGK = 32;             // workgroup GEMM k chunk
constexpr int kSturmPts = 1;        // Sturm counts per thread and multisection round
constexpr int kInvIter = 3;         // inverse iteration sweeps

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
// conj(a) * b
__device__ __forceinline__ double2 zcmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// a b + c
__device__ __forceinline__ double2 zfma(double2 a, double2 b, double2 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}

// Lane exchange inside rows of 16 lanes through DPP (a VALU operand modifier,
// no LDS round trip): CTRL 0xB1 swaps neighbours (lane ^ 1), 0x4E swaps pairs
// (lane ^ 2), 0x141 mirrors each half-row (lane i <- 7 - i), 0x140 mirrors the
// row (lane i <- 15 - i).
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Sum over aligned groups of G lanes (G a power of two <= 64); every lane of the
// group gets the sum.  After the xor-1 and xor-2 steps each quad holds its sum,
// the mirrors then pair quads with quads and half-rows with half-rows.
template <int G> __device__ __forceinline__ double gsum(double v) {
  if (G >= 2) v += dpp_d<0xB1>(v);
  if (G >= 4) v += dpp_d<0x4E>(v);
  if (G >= 8) v += dpp_d<0x141>(v);
  if (G >= 16) v += dpp_d<0x140>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}
template <int G> __device__ __forceinline__ double2 gsum2(double2 v) {
  return make_double2(gsum<G>(v.x), gsum<G>(v.y));
}
__device__ __forceinline__ double wave_sum(double v) { return gsum<64>(v); }

// 1/a from the hardware estimate and two Newton steps (a finite and nonzero)
__device__ __forceinline__ double fast_rcp(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(fma(-a, r, 1.0), r, r);
  r = fma(fma(-a, r, 1.0), r, r);
  return r;
}

// Row-group layout of the BLAS2 steps: G lanes per matrix row, kRowsPass rows
// per pass over the workgroup, at most kPasses passes (order <= kRRMax).
constexpr int kRowG = 8;
constexpr int kRowsPass = kRRThreads / kRowG;
constexpr int kPasses = kRRMax / kRowsPass;

// row i of the lower-triangle index e (e = i (i + 1) / 2 + j, j <= i)
__device__ __forceinline__ int tri_row(int e) {
  int i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > e) --i;
  while ((i + 1) * (i + 2) / 2 <= e) ++i;
  return i;
}

// C(i, j) = sum_{k in [kb, ke)} A(i, k) B(k, j) on the 64 x 64 output tiles
// that Tile(i0, j0) admits, with KR(i0, j0, kb, ke) the k range that can be
// nonzero for the tile.  2 x 2 outputs per thread; the next k chunk is fetched
// into registers while the current one is multiplied.  ta: kGT x kGK, tb:
// kGK x kGT LDS tiles.  All threads must call.
template <typename FA, typename FB, typename FC, typename FK, typename FT>
__device__ void wg_gemm(int M, int N, int K, FA A, FB B, FC Cst, FK KR, FT Tile, double2 *ta,
                        double2 *tb) {
  constexpr int kPer = kGT * kGK / kRRThreads;   // tile elements fetched per thread
  const int tid = threadIdx.x;
  const int tx = tid % 32, ty = tid / 32;
  for (int i0 = 0; i0 < M; i0 += kGT)
    for (int j0 = 0; j0 < N; j0 += kGT) {
      if (!Tile(i0, j0)) continue;   // uniform
      int kb, ke;
      KR(i0, j0, kb, ke);
      kb = max(kb, 0);
      ke = min(ke, K);
      double2 acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = make_double2(0, 0);
      double2 ra[kPer], rb[kPer];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int h = 0; h < kPer; ++h) {
          const int e = tid + h * kRRThreads;
          const int ar = e / kGK, ak = e % kGK;
          const int i = i0 + ar, k = k0 + ak;
          ra[h] = (i < M && k < ke) ? A(i, k) : make_double2(0, 0);
          const int bk = e / kGT, bc = e % kGT;
          const int kk = k0 + bk, j = j0 + bc;
          rb[h] = (kk < ke && j < N) ? B(kk, j) : make_double2(0, 0);
        }
      };
      if (kb < ke) fetch(kb);
      for (int k0 = kb; k0 < ke; k0 += kGK) {
#pragma unroll
        for (int h = 0; h < kPer; ++h) {
          ta[tid + h * kRRThreads] = ra[h];
          tb[tid + h * kRRThreads] = rb[h];
        }
        __syncthreads();
        if (k0 + kGK < ke) fetch(k0 + kGK);
#pragma unroll 8
        for (int kk = 0; kk < kGK; ++kk) {
          const double2 a0 = ta[(2 * ty) * kGK + kk], a1 = ta[(2 * ty + 1) * kGK + kk];
          const double2 b0 = tb[kk * kGT + tx], b1 = tb[kk * kGT + tx + 32];
          acc[0][0] = zfma(a0, b0, acc[0][0]);
          acc[0][1] = zfma(a0, b1, acc[0][1]);
          acc[1][0] = zfma(a1, b0, acc[1][0]);
          acc[1][1] = zfma(a1, b1, acc[1][1]);
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int i = i0 + 2 * ty + a, j = j0 + tx + 32 * b;
          if (i < M && j < N) Cst(i, j, acc[a][b]);
        }
    }
}

// Lower triangle of a square matrix: packed rows in LDS, or full rows in global.
struct PackedLower {
  double2 *p;
  __device__ __forceinline__ int idx(int i, int j) const { return i * (i + 1) / 2 + j; }
  __device__ __forceinline__ double2 lo(int i, int j) const { return p[idx(i, j)]; }   // j <= i
  __device__ __forceinline__ void set(int i, int j, double2 v) const { p[idx(i, j)] = v; }
};
struct FullLower {
  double2 *p;
  int ld;
  __device__ __forceinline__ double2 lo(int i, int j) const { return p[(size_t)i * ld + j]; }
  __device__ __forceinline__ void set(int i, int j, double2 v) const { p[(size_t)i * ld + j] = v; }
};

// Left-looking Cholesky with column dropping on the lower triangle of M (n x n).
// Column j: pivot S_jj - sum_{k<j} |L_jk|^2 and L_ij = (S_ij - sum_{k<j} L_ik
// conj(L_jk)) / L_jj.  The dot products of all rows i >= j are formed at once,
// kRowG lanes per row over strided k and reduced inside the lane group; row j's
// is the pivot, passed on through LDS (`sc`).  keep[j] = 0 marks a dropped
// column, whose L column is zero.  Two barriers per column.
template <typename Mat>
__device__ void cholesky_drop(const Mat M, int n, double drop_tol, const double *dsc, int *keep,
                              double *sc) {
  const int tid = threadIdx.x, g = tid % kRowG, rl = tid / kRowG;
  for (int j = 0; j < n; ++j) {
    const int m = n - j;   // rows j..n-1
    double2 dot[kPasses];
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      dot[p] = make_double2(0, 0);
      if (p * kRowsPass < m) {   // uniform
        const int ii = p * kRowsPass + rl;
        double2 s = make_double2(0, 0);
        if (ii < m) {
          const int i = j + ii;
#pragma unroll 4
          for (int k = g; k < j; k += kRowG) s = zfma(M.lo(i, k), zconj(M.lo(j, k)), s);
        }
        dot[p] = gsum2<kRowG>(s);
      }
    }
    if (tid == 0) sc[0] = M.lo(j, j).x - dot[0].x;
    __syncthreads();
    const double piv = sc[0];
    const bool drop = (dsc[j] == 0.0) || !(piv > drop_tol);
    const double ljj = drop ? 0.0 : sqrt(piv);
    const double inv = drop ? 0.0 : 1.0 / ljj;
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      const int ii = p * kRowsPass + rl;
      if (g == 0 && ii >= 1 && ii < m) {
        const int i = j + ii;
        M.set(i, j, drop ? make_double2(0, 0) : zscale(zsub(M.lo(i, j), dot[p]), inv));
      }
    }
    if (tid == 0) {
      M.set(j, j, make_double2(ljj, 0.0));
      keep[j] = drop ? 0 : 1;
    }
    __syncthreads();
  }
}

// In-place inverse of the lower-triangular n x n matrix in M (nonzero real
// diagonal), column by column from the right: for L = [l 0; x L2],
// L^-1 = [1/l 0; -L2^-1 x / l  L2^-1].  Row groups as in the Cholesky; two
// barriers per column.
template <typename Mat>
__device__ void trtri_lower(const Mat M, int n) {
  const int tid = threadIdx.x, g = tid % kRowG, rl = tid / kRowG;
  for (int j = n - 1; j >= 0; --j) {
    const int m = n - j - 1;
    const double inv = 1.0 / M.lo(j, j).x;
    double2 y[kPasses];
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      y[p] = make_double2(0, 0);
      if (p * kRowsPass < m) {   // uniform
        const int ii = p * kRowsPass + rl;
        double2 s = make_double2(0, 0);
        if (ii < m) {
#pragma unroll 4
          for (int k = g; k <= ii; k += kRowG)
            s = zfma(M.lo(j + 1 + ii, j + 1 + k), M.lo(j + 1 + k, j), s);
        }
        y[p] = gsum2<kRowG>(s);
      }
    }
    __syncthreads();   // column j and its diagonal are read everywhere
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      const int ii = p * kRowsPass + rl;
      if (g == 0 && ii < m) M.set(j + 1 + ii, j, zscale(y[p], -inv));
    }
    if (tid == 0) M.set(j, j, make_double2(inv, 0.0));
    __syncthreads();
  }
}

struct TriWork {
  double *dd, *ee;      // diagonal (r), off-diagonal (r-1)
  double2 *tauv;        // reflector scalars (r-1)
  double2 *vv, *xv;     // reflector vector, tau C v (r)
  double *nred, *qred;  // per-wave partial sums (16 each)
};

// Householder tridiagonalisation of the r x r Hermitian matrix held in M's lower
// triangle.  Reflector k (H_k = I - tau_k v v^H, v = [1, M(k+2.., k)]) acts on
// rows k+1..r-1; the column below the subdiagonal keeps v for the
// back-transformation.  With x = tau C22 v and q = v^H C22 v (real), the
// two-sided update is C22 -= v w^H + w v^H, w = x - |tau|^2 q v / 2.  Per
// reflector: (a) every thread forms tau from the per-wave partial sums of the
// column norm and v is written; (b) x by row groups, and q's per-wave partials;
// (c) the rank-2 update by row groups, which also sums the next column's norm.
template <typename Mat>
__device__ void tridiagonalise(const Mat M, int r, TriWork w) {
  constexpr int NW = kRRThreads / 64;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wid = tid >> 6, g = tid % kRowG, rl = tid / kRowG;
  {
    double x = 0;
    for (int i = 2 + tid; i < r; i += nt) {
      const double2 v = M.lo(i, 0);
      x += v.x * v.x + v.y * v.y;
    }
    x = wave_sum(x);
    if (lane == 0) w.nred[wid] = x;
    __syncthreads();
  }
  for (int k = 0; k + 1 < r; ++k) {
    const int m = r - k - 1;   // trailing size, rows/cols k+1..r-1
    // (a) reflector; identical arithmetic on every thread
    double xn2 = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) xn2 += w.nred[q];
    const double2 alpha = M.lo(k + 1, k);
    double2 tau = make_double2(0, 0), scal = make_double2(0, 0);
    double beta = alpha.x;
    if (!(xn2 == 0.0 && alpha.y == 0.0)) {
      const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
      beta = (alpha.x >= 0) ? -nrm : nrm;
      tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
      const double2 den = make_double2(alpha.x - beta, alpha.y);
      const double dn = den.x * den.x + den.y * den.y;
      scal = make_double2(den.x / dn, -den.y / dn);
    }
    if (tid == 0) {
      w.tauv[k] = tau;
      w.ee[k] = beta;
      w.dd[k] = M.lo(k, k).x;
    }
    for (int i = tid; i < m; i += nt) {
      const double2 v = (i == 0) ? make_double2(1, 0) : zmul(M.lo(k + 1 + i, k), scal);
      w.vv[i] = v;
      if (i > 0) M.set(k + 1 + i, k, v);
    }
    __syncthreads();
    // (b) x = tau C22 v, C22 Hermitian from its lower triangle
    double qp = 0;
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      if (p * kRowsPass < m) {   // uniform
        const int ii = p * kRowsPass + rl;
        double2 s = make_double2(0, 0);
        if (ii < m) {
          const int gi = k + 1 + ii;
#pragma unroll 4
          for (int jj = g; jj < m; jj += kRowG) {
            const int gj = k + 1 + jj;
            const double2 c = (jj <= ii) ? M.lo(gi, gj) : zconj(M.lo(gj, gi));
            s = zfma(c, w.vv[jj], s);
          }
        }
        s = gsum2<kRowG>(s);
        if (ii < m && g == 0) {
          w.xv[ii] = zmul(tau, s);
          const double2 vi = w.vv[ii];
          qp += vi.x * s.x + vi.y * s.y;   // Re(conj(v_i) (C22 v)_i)
        }
      }
    }
    qp = wave_sum(qp);
    if (lane == 0) w.qred[wid] = qp;
    __syncthreads();
    // (c) rank-2 update of the lower triangle, row groups over j <= i
    double q = 0;
#pragma unroll
    for (int p = 0; p < NW; ++p) q += w.qred[p];
    const double al = -0.5 * (tau.x * tau.x + tau.y * tau.y) * q;
    double nx = 0;
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      const int ii = p * kRowsPass + rl;
      if (p * kRowsPass < m && ii < m) {
        const double2 vi = w.vv[ii];
        const double2 wi = zadd(w.xv[ii], zscale(vi, al));
        const int gi = k + 1 + ii;
#pragma unroll 4
        for (int jj = g; jj <= ii; jj += kRowG) {
          const double2 vj = w.vv[jj];
          const double2 wj = zadd(w.xv[jj], zscale(vj, al));
          double2 c = M.lo(gi, k + 1 + jj);
          c = zsub(c, zadd(zmul(vi, zconj(wj)), zmul(wi, zconj(vj))));
          if (ii == jj) c.y = 0.0;
          M.set(gi, k + 1 + jj, c);
          if (jj == 0 && ii >= 2) nx += c.x * c.x + c.y * c.y;
        }
      }
    }
    nx = wave_sum(nx);
    if (lane == 0) w.nred[wid] = nx;
    __syncthreads();
  }
  if (tid == 0) w.dd[r - 1] = M.lo(r - 1, r - 1).x;
  __syncthreads();
}

// Uc = Q U with Q = H_0 H_1 ... H_{r-2} (reflectors stored in M's columns),
// U real r x nk stored per column (U[j r + i]), Uc complex r x nk row-major.
// A group of G lanes owns one column, NPL rows per lane in registers, and
// applies every reflector with shuffle reductions only.
template <int G, int NPL, typename Mat>
__device__ void back_transform(const Mat M, int r, int nk, const double2 *tauv, const double *U,
                               double2 *Uc) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int gl = tid % G;
  for (int j0 = 0; j0 < nk; j0 += nt / G) {
    const int j = j0 + tid / G;
    const bool act = j < nk;
    double2 u[NPL];
#pragma unroll
    for (int s = 0; s < NPL; ++s) {
      const int i = gl + G * s;
      u[s] = (act && i < r) ? make_double2(U[(size_t)j * r + i], 0.0) : make_double2(0, 0);
    }
    for (int k = r - 2; k >= 0; --k) {
      const double2 tau = tauv[k];
      if (tau.x == 0.0 && tau.y == 0.0) continue;   // uniform
      double2 acc = make_double2(0, 0);
#pragma unroll
      for (int s = 0; s < NPL; ++s) {
        const int i = gl + G * s;
        if (i > k && i < r) {
          const double2 v = (i == k + 1) ? make_double2(1, 0) : M.lo(i, k);
          acc = zadd(acc, zcmul(v, u[s]));
        }
      }
      acc = zmul(tau, gsum2<G>(acc));
#pragma unroll
      for (int s = 0; s < NPL; ++s) {
        const int i = gl + G * s;
        if (i > k && i < r) {
          const double2 v = (i == k + 1) ? make_double2(1, 0) : M.lo(i, k);
          u[s] = zsub(u[s], zmul(v, acc));
        }
      }
    }
#pragma unroll
    for (int s = 0; s < NPL; ++s) {
      const int i = gl + G * s;
      if (act && i < r) Uc[(size_t)i * nk + j] = u[s];
    }
  }
  __syncthreads();
}

// one step of the Sturm recurrence q_i = (d_i - x) - e_{i-1}^2 / q_{i-1}
__device__ __forceinline__ double sturm_step(double q, double dmx, double e2, double pivmin) {
  if (fabs(q) < pivmin) q = -pivmin;
  return fma(-e2, fast_rcp(q), dmx);
}

// number of eigenvalues of T below x
__device__ int sturm_count(const double *d, const double *e2, int r, double x, double pivmin) {
  double q = d[0] - x;
  int cnt = q < 0 ? 1 : 0;
#pragma unroll 4
  for (int i = 1; i < r; ++i) {
    q = sturm_step(q, d[i] - x, e2[i - 1], pivmin);
    cnt += q < 0 ? 1 : 0;
  }
  return cnt;
}

// deterministic start vector entries in (-1, 1)
__device__ double start_entry(int i, int j) {
  unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)((j + 1) * 2246822519u);
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  h *= 3266489917u;
  h ^= h >> 16;
  return ((double)(h & 0xFFFFFF) / 8388608.0) - 1.0 + 1e-3;
}

// Inverse iteration for one eigenvalue on one thread: LU with partial
// pivoting of T - lm I (per row: 1/u0, u1, u2, multiplier in f, the row swap
// in sw), the start vector's forward elimination fused into the
// factorisation, then kInvIter solves, each followed by normalisation.  The
// solves run over batches of 8 rows whose loads are issued together.
__device__ void inverse_iteration(const double *dd, const double *ee, int r, double lm,
                                  double eps_t, int seed, double *__restrict__ x,
                                  double *__restrict__ f, unsigned char *__restrict__ sw) {
  double a = dd[0] - lm, bsup = (r > 1) ? ee[0] : 0.0;
  double carry = start_entry(0, seed);
  for (int i = 0; i + 1 < r; ++i) {
    const double c = ee[i];
    const double dn = dd[i + 1] - lm;
    const double en = (i + 2 < r) ? ee[i + 1] : 0.0;
    double u0, u1, u2, mm;
    bool swp;
    if (fabs(a) >= fabs(c)) {
      mm = (a != 0.0) ? c * fast_rcp(a) : 0.0;
      u0 = a; u1 = bsup; u2 = 0.0; swp = false;
      a = dn - mm * bsup;
      bsup = en;
    } else {
      mm = a * fast_rcp(c);
      u0 = c; u1 = dn; u2 = en; swp = true;
      a = bsup - mm * dn;
      bsup = -mm * en;
    }
    if (fabs(u0) < eps_t) u0 = (u0 < 0) ? -eps_t : eps_t;
    f[4 * i + 0] = fast_rcp(u0);
    f[4 * i + 1] = u1;
    f[4 * i + 2] = u2;
    f[4 * i + 3] = mm;
    sw[i] = swp ? 1 : 0;
    double bi = carry, bn = start_entry(i + 1, seed);
    if (swp) { const double tt = bi; bi = bn; bn = tt; }
    x[i] = bi;
    carry = bn - mm * bi;
  }
  {
    double u0 = a;
    if (fabs(u0) < eps_t) u0 = (u0 < 0) ? -eps_t : eps_t;
    f[4 * (r - 1) + 0] = fast_rcp(u0);
    f[4 * (r - 1) + 1] = 0.0;
    f[4 * (r - 1) + 2] = 0.0;
    f[4 * (r - 1) + 3] = 0.0;
    sw[r - 1] = 0;
    x[r - 1] = carry;
  }
  constexpr int B = 8;
  for (int iter = 0; iter < kInvIter; ++iter) {
    if (iter > 0) {
      // forward elimination: rows i, i+1 swapped where the factorisation did,
      // then row i+1 -= mm_i row i
      double cr = x[0];
      int i = 0;
      for (; i + B < r; i += B) {
        double xn[B], mv[B], ov[B];
        unsigned char sv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
          xn[u] = x[i + 1 + u];
          mv[u] = f[4 * (i + u) + 3];
          sv[u] = sw[i + u];
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
          double bi = cr, bn = xn[u];
          if (sv[u]) { const double tt = bi; bi = bn; bn = tt; }
          ov[u] = bi;
          cr = bn - mv[u] * bi;
        }
#pragma unroll
        for (int u = 0; u < B; ++u) x[i + u] = ov[u];
      }
      for (; i + 1 < r; ++i) {
        double bi = cr, bn = x[i + 1];
        if (sw[i]) { const double tt = bi; bi = bn; bn = tt; }
        x[i] = bi;
        cr = bn - f[4 * i + 3] * bi;
      }
      x[r - 1] = cr;
    }
    // back substitution with the upper factor (bandwidth 3)
    double x1 = 0.0, x2 = 0.0;
    int i = r - 1;
    for (; i >= B - 1; i -= B) {
      double xb[B], fa[B], fb[B], fc[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int ii = i - u;
        xb[u] = x[ii];
        fa[u] = f[4 * ii + 0];
        fb[u] = f[4 * ii + 1];
        fc[u] = f[4 * ii + 2];
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const double sv = (xb[u] - fb[u] * x1 - fc[u] * x2) * fa[u];
        xb[u] = sv;
        x2 = x1;
        x1 = sv;
      }
#pragma unroll
      for (int u = 0; u < B; ++u) x[i - u] = xb[u];
    }
    for (; i >= 0; --i) {
      const double sv = (x[i] - f[4 * i + 1] * x1 - f[4 * i + 2] * x2) * f[4 * i];
      x[i] = sv;
      x2 = x1;
      x1 = sv;
    }
    double nrm = 0;
#pragma unroll 8
    for (int ii = 0; ii < r; ++ii) nrm += x[ii] * x[ii];
    const double inv = 1.0 / sqrt(nrm);
#pragma unroll 8
    for (int ii = 0; ii < r; ++ii) x[ii] *= inv;
  }
}

// Orthonormalise the vectors U[t..tend) of one cluster (modified Gram-Schmidt,
// two passes)
__device__ void orthonormalise_cluster(int r, int t, int tend, double *__restrict__ U) {
  for (int jv = t + 1; jv < tend; ++jv) {
    double *x = U + (size_t)jv * r;
    for (int pass = 0; pass < 2; ++pass)
      for (int jp = t; jp < jv; ++jp) {
        const double *y = U + (size_t)jp * r;
        double dot = 0;
#pragma unroll 8
        for (int i = 0; i < r; ++i) dot += y[i] * x[i];
#pragma unroll 8
        for (int i = 0; i < r; ++i) x[i] -= dot * y[i];
      }
    double nrm = 0;
    for (int i = 0; i < r; ++i) nrm += x[i] * x[i];
    const double inv = 1.0 / sqrt(nrm);
    for (int i = 0; i < r; ++i) x[i] *= inv;
  }
}

__global__ void __launch_bounds__(kRRThreads) k_rayleigh_ritz(
    const double2 *__restrict__ Ain, const double2 *__restrict__ Sin, int nz, int nkeep,
    double drop_tol, double floor_val, const int *__restrict__ forced, double2 *__restrict__ Vout,
    double *__restrict__ theta, int *__restrict__ info, double *__restrict__ dinfo,
    double2 *__restrict__ ws, long long *__restrict__ tstamp) {
  // no static LDS in this kernel: the dynamic arena then starts at offset 0,
  // 16-byte aligned, as the double2 accesses (ds_read_b128) need for speed
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // optional phase timestamps (constant-rate wall clock), for tuning
#define DKS_RR_STAMP(k) \
  do {                  \
    if (tstamp && threadIdx.x == 0) tstamp[k] = wall_clock64(); \
  } while (0)
  DKS_RR_STAMP(0);
  // ---- LDS arena (sized by nz): partial sums, per-index arrays, then the
  // packed triangle or the GEMM tiles
  const int na = (nz + 1) & ~1;
  double2 *part = reinterpret_cast<double2 *>(smem_raw);   // kRRThreads
  double2 *tauv = part + kRRThreads;
  double2 *vv = tauv + na;
  double2 *xv = vv + na;
  double *dsc = reinterpret_cast<double *>(xv + na);
  double *dd = dsc + na;
  double *ee = dd + na;
  double *e2 = ee + na;
  double *lam = e2 + na;
  double *red = lam + na;                                  // 64: 0-3 scalars, 32-63 sums
  int *kept = reinterpret_cast<int *>(red + 64);
  double2 *big = reinterpret_cast<double2 *>(kept + na);  // packed triangle or GEMM tiles
  double2 *ta = big, *tb = big + kGT * kGK;
  int &s_r = reinterpret_cast<int *>(red)[0];
  int &s_flag = reinterpret_cast<int *>(red)[1];
  int &s_k0 = reinterpret_cast<int *>(red)[2];
  double &s_lmin = red[2];

  const int tid = threadIdx.x, nt = blockDim.x;
  const size_t nn = (size_t)nz * nz;
  double2 *Sg = ws;              // scaled S lower triangle (global path)
  double2 *Am = Sg + nn;         // scaled A (full)
  double2 *Lc = Am + nn;         // L^-1 column-major: Lc[c r + b] = Li[b][c]
  double2 *Mm = Lc + nn;         // A_r Li^H; compaction buffer; C (global path)
  double2 *Cg = Mm + nn;         // C = Li A_r Li^H, lower tiles
  double2 *Uc = Cg + nn;         // r x nkeep complex eigenvectors
  double *U = reinterpret_cast<double *>(Uc + (size_t)nz * nkeep);   // nkeep x r real, per vector
  double *lu = U + (size_t)nz * nkeep;                                // 5 r per cluster leader
  const bool packed = (nz <= kRRPackedMax);

  // ---- 1. scaling and Hermitian parts
  for (int i = tid; i < nz; i += nt) {
    const double s = Sin[(size_t)i * nz + i].x;
    const bool f = forced ? (forced[i] != 0) : false;
    dsc[i] = (!f && s > 0 && isfinite(s)) ? 1.0 / sqrt(s) : 0.0;
  }
  __syncthreads();
#pragma unroll 4
  for (int e = tid; e < (int)nn; e += nt) {
    const int i = e / nz, j = e - (e / nz) * nz;
    const double f = dsc[i] * dsc[j];
    const double2 a1 = Ain[e], a2 = Ain[(size_t)j * nz + i];
    Am[e] = make_double2(0.5 * f * (a1.x + a2.x), 0.5 * f * (a1.y - a2.y));
    if (j <= i) {
      const double2 s1 = Sin[e], s2 = Sin[(size_t)j * nz + i];
      const double2 h = make_double2(0.5 * f * (s1.x + s2.x), 0.5 * f * (s1.y - s2.y));
      if (packed) PackedLower{big}.set(i, j, h); else FullLower{Sg, nz}.set(i, j, h);
    }
  }
  __syncthreads();
  DKS_RR_STAMP(1);

  // ---- 2. Cholesky with column dropping
  if (packed) cholesky_drop(PackedLower{big}, nz, drop_tol, dsc, kept, red + 4);
  else cholesky_drop(FullLower{Sg, nz}, nz, drop_tol, dsc, kept, red + 4);
  if (tid == 0) {
    int r = 0;
    for (int j = 0; j < nz; ++j)
      if (kept[j]) kept[r++] = j;
    s_r = r;
    s_flag = (r < nkeep) ? 1 : 0;
    info[0] = r;
    info[1] = s_flag;
    info[2] = nz - r;
    info[3] = 0;
  }
  __syncthreads();
  const int r = s_r;
  if (s_flag) return;
  DKS_RR_STAMP(2);

  // ---- 3. compact L to the kept indices (through a global copy, since the
  // compacted triangle overlaps the source), invert it in place
  {
    const int tri = r * (r + 1) / 2;
    for (int e = tid; e < tri; e += nt) {
      const int a = tri_row(e), b = e - a * (a + 1) / 2;
      Mm[e] = packed ? PackedLower{big}.lo(kept[a], kept[b]) : FullLower{Sg, nz}.lo(kept[a], kept[b]);
    }
    __syncthreads();
    for (int e = tid; e < tri; e += nt) {
      const int a = tri_row(e), b = e - a * (a + 1) / 2;
      if (packed) PackedLower{big}.set(a, b, Mm[e]); else FullLower{Sg, r}.set(a, b, Mm[e]);
    }
    __syncthreads();
  }
  if (packed) trtri_lower(PackedLower{big}, r); else trtri_lower(FullLower{Sg, r}, r);
  for (int e = tid; e < r * r; e += nt) {
    const int c = e / r, b = e - (e / r) * r;   // Lc[c r + b] = Li[b][c]
    Lc[e] = (b >= c) ? (packed ? PackedLower{big}.lo(b, c) : FullLower{Sg, r}.lo(b, c))
                     : make_double2(0, 0);
  }
  __syncthreads();
  DKS_RR_STAMP(3);
  // Mm[a][b] = sum_{c <= b} A[ka][kc] conj(Li[b][c])
  wg_gemm(
      r, r, r, [&](int i, int k) { return Am[(size_t)kept[i] * nz + kept[k]]; },
      [&](int k, int j) { return zconj(Lc[(size_t)k * r + j]); },
      [&](int i, int j, double2 v) { Mm[(size_t)i * r + j] = v; },
      [&](int, int j0, int &kb, int &ke) { kb = 0; ke = j0 + kGT; },
      [&](int, int) { return true; }, ta, tb);
  __syncthreads();
  DKS_RR_STAMP(9);
  // Cg[a][b] = sum_{c <= a} Li[a][c] Mm[c][b] on the tiles touching the lower triangle
  wg_gemm(
      r, r, r, [&](int i, int k) { return Lc[(size_t)k * r + i]; },
      [&](int k, int j) { return Mm[(size_t)k * r + j]; },
      [&](int i, int j, double2 v) { Cg[(size_t)i * r + j] = v; },
      [&](int i0, int, int &kb, int &ke) { kb = 0; ke = i0 + kGT; },
      [&](int i0, int j0) { return j0 <= i0; }, ta, tb);
  __syncthreads();
  DKS_RR_STAMP(10);
  {
    // Hermitian part of the lower triangle (diagonal tiles hold both halves)
    const int tri = r * (r + 1) / 2;
    for (int e = tid; e < tri; e += nt) {
      const int i = tri_row(e), j = e - i * (i + 1) / 2;
      double2 h = Cg[(size_t)i * r + j];
      if ((i / kGT) == (j / kGT)) {
        const double2 y = Cg[(size_t)j * r + i];
        h = make_double2(0.5 * (h.x + y.x), 0.5 * (h.y - y.y));
      }
      if (i == j) h.y = 0.0;
      if (packed) PackedLower{big}.set(i, j, h); else FullLower{Mm, r}.set(i, j, h);
    }
  }
  __syncthreads();
  DKS_RR_STAMP(4);

  // ---- 4. tridiagonalisation
  {
    TriWork tw{dd, ee, tauv, vv, xv, red + 32, red + 48};
    if (packed) tridiagonalise(PackedLower{big}, r, tw); else tridiagonalise(FullLower{Mm, r}, r, tw);
  }
  for (int i = tid; i + 1 < r; i += nt) e2[i] = ee[i] * ee[i];
  __syncthreads();
  DKS_RR_STAMP(5);

  // ---- 5. multisection for the kept eigenvalues and the smallest one
  double glo = 1e300, ghi = -1e300, emax2 = 0;
#pragma unroll 8
  for (int i = 0; i < r; ++i) {
    const double off = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < r ? fabs(ee[i]) : 0.0);
    glo = fmin(glo, dd[i] - off);
    ghi = fmax(ghi, dd[i] + off);
    if (i + 1 < r) emax2 = fmax(emax2, e2[i]);
  }
  const double tnorm = fmax(fabs(glo), fabs(ghi));
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  const double atol = DBL_EPSILON * tnorm;
  glo -= 2.0 * DBL_EPSILON * tnorm + 2 * pivmin;
  ghi += 2.0 * DBL_EPSILON * tnorm + 2 * pivmin;
  if (tid == 0) {
    const int k0 = (floor_val > glo) ? sturm_count(dd, e2, r, floor_val, pivmin) : 0;
    s_k0 = k0;
    info[3] = k0;
    if (r - k0 < nkeep) {
      s_flag = 2;
      info[1] = 2;
    }
  }
  __syncthreads();
  if (s_flag) return;
  const int k0 = s_k0;
  {
    // target t < nkeep: eigenvalue k0 + t; t == nkeep: the smallest.  Each
    // round, G threads per target count at NP interior points of its bracket
    // [lo, hi) (count(lo) <= index < count(hi)) and the bracket shrinks to the
    // pair of neighbouring points around the index.
    const int ntar = nkeep + 1;
    const int G = max(1, nt / ntar);
    const int NP = G * kSturmPts;
    double *los = reinterpret_cast<double *>(part);
    double *his = los + ntar;
    unsigned short *cnts = reinterpret_cast<unsigned short *>(his + ntar);
    const double inv_np1 = 1.0 / (double)(NP + 1);
    auto narrow = [&](double lo, double hi) {
      return hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + atol + pivmin;
    };
    for (int t = tid; t < ntar; t += nt) {
      los[t] = glo;
      his[t] = ghi;
    }
    __syncthreads();
    for (int round = 0; round < 64; ++round) {
      for (int u = tid; u < ntar * G; u += nt) {
        const int t = u / G, g = u - (u / G) * G;
        const double lo = los[t], hi = his[t];
        if (narrow(lo, hi)) continue;
#pragma unroll
        for (int p = 0; p < kSturmPts; ++p) {
          const double x = lo + (hi - lo) * ((double)(g * kSturmPts + p + 1) * inv_np1);
          cnts[t * NP + g * kSturmPts + p] = (unsigned short)sturm_count(dd, e2, r, x, pivmin);
        }
      }
      __syncthreads();
      int active = 0;
      for (int t = tid; t < ntar; t += nt) {
        const double lo = los[t], hi = his[t];
        if (narrow(lo, hi)) continue;
        const int idx = (t < nkeep) ? k0 + t : 0;
        int a = -1, b = NP;   // count(point a) <= idx < count(point b)
        while (b - a > 1) {
          const int mid = (a + b) >> 1;
          if ((int)cnts[t * NP + mid] <= idx) a = mid; else b = mid;
        }
        const double nlo = (a >= 0) ? lo + (hi - lo) * ((double)(a + 1) * inv_np1) : lo;
        const double nhi = (b < NP) ? lo + (hi - lo) * ((double)(b + 1) * inv_np1) : hi;
        if (nhi > nlo && nhi - nlo < hi - lo) {
          los[t] = nlo;
          his[t] = nhi;
          active |= narrow(nlo, nhi) ? 0 : 1;
        } else {
          // no representable interior point left: the bracket has converged
          const double mid = 0.5 * (lo + hi);
          los[t] = mid;
          his[t] = mid;
        }
      }
      if (!__syncthreads_or(active)) break;
    }
    for (int t = tid; t < ntar; t += nt) {
      const double v = 0.5 * (los[t] + his[t]);
      if (t < nkeep) lam[t] = v; else s_lmin = v;
    }
    __syncthreads();
  }
  DKS_RR_STAMP(6);

  // ---- 6. inverse iteration, one thread per eigenvalue; within a cluster of
  // close eigenvalues the shifts are spread by 10 ulp(T) and the vectors are
  // orthonormalised afterwards
  const double ctol = 1e-7 * fmax(tnorm, 1e-300);
  const double eps_t = DBL_EPSILON * fmax(tnorm, 1e-300);
  for (int t = tid; t < nkeep; t += nt) {
    int t0 = t;
    while (t0 > 0 && lam[t0] - lam[t0 - 1] <= ctol) --t0;
    double *fb = lu + (size_t)t * 5 * r;
    inverse_iteration(dd, ee, r, lam[t] + (double)(t - t0) * 10.0 * eps_t, eps_t, t,
                      U + (size_t)t * r, fb, reinterpret_cast<unsigned char *>(fb + 4 * r));
  }
  __syncthreads();
  for (int t = tid; t < nkeep; t += nt) {
    if (t > 0 && lam[t] - lam[t - 1] <= ctol) continue;   // not a cluster leader
    int tend = t + 1;
    while (tend < nkeep && lam[tend] - lam[tend - 1] <= ctol) ++tend;
    if (tend > t + 1) orthonormalise_cluster(r, t, tend, U);
  }
  __syncthreads();
  DKS_RR_STAMP(7);

  // ---- 7. back-transformation: Uc = Q U, then V = D Li^H Uc
  if (packed) back_transform<16, 8>(PackedLower{big}, r, nkeep, tauv, U, Uc);
  else back_transform<64, 8>(FullLower{Mm, r}, r, nkeep, tauv, U, Uc);
  DKS_RR_STAMP(11);
  for (int e = tid; e < nz * nkeep; e += nt) Vout[e] = make_double2(0, 0);
  __syncthreads();
  // Vout[kb][j] = d_kb sum_{a >= b} conj(Li[a][b]) Uc[a][j]
  wg_gemm(
      r, nkeep, r, [&](int i, int k) { return zconj(Lc[(size_t)i * r + k]); },
      [&](int k, int j) { return Uc[(size_t)k * nkeep + j]; },
      [&](int i, int j, double2 v) {
        const int ki = kept[i];
        Vout[(size_t)ki * nkeep + j] = zscale(v, dsc[ki]);
      },
      [&](int i0, int, int &kb, int &ke) { kb = i0; ke = r; },
      [&](int, int) { return true; }, ta, tb);
  for (int t = tid; t < nkeep; t += nt) theta[t] = lam[t];
  if (tid == 0) dinfo[0] = s_lmin;
  __syncthreads();
  DKS_RR_STAMP(8);
#undef DKS_RR_STAMP
}

// dynamic LDS of one launch with subspace dimension nz (layout of the kernel's arena)
static size_t rr_lds_bytes(int nz) {
  const size_t na = (size_t)((nz + 1) & ~1);
  const size_t arrays = sizeof(double2) * (kRRThreads + 3 * na) + sizeof(double) * (6 * na + 64) +
                        sizeof(int) * na;
  const size_t packed =
      nz <= kRRPackedMax ? sizeof(double2) * (size_t)nz * (nz + 1) / 2 : 0;
  const size_t tiles = sizeof(double2) * 2 * kGT * kGK;
  return ((arrays + 15) & ~(size_t)15) + (packed > tiles ? packed : tiles);
}

void rayleigh_ritz(const double2 *A, const double2 *S, int nz, int nkeep, double drop_tol,
                   double floor_val, const int *forced_drop, double2 *V, double *theta, int *info,
                   double *dinfo, DevBuf &scratch, hipStream_t st, long long *tstamp) {
  DKS_REQUIRE(nz > 0 && nz <= kRRMax && nkeep > 0 && nkeep <= nz, DKS_EINVAL,
              "Rayleigh-Ritz size out of range (subspace dimension must be <= 512)");
  // the multisection brackets and counts share the kRRThreads partial-sum area
  DKS_REQUIRE(sizeof(double) * 2 * (nkeep + 1) +
                      sizeof(unsigned short) * (size_t)kRRThreads * kSturmPts <=
                  sizeof(double2) * kRRThreads,
              DKS_EINVAL, "Rayleigh-Ritz: too many wanted pairs");
  // once per process, also when batch lanes arrive here together
  static std::once_flag attr;
  hipError_t attr_rc = hipSuccess;
  std::call_once(attr, [&] {
    const size_t mx = std::max(rr_lds_bytes(kRRPackedMax), rr_lds_bytes(kRRMax));
    attr_rc = hipFuncSetAttribute((const void *)k_rayleigh_ritz,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx);
  });
  DKS_HIP(attr_rc);
  const size_t lds = rr_lds_bytes(nz);
  const size_t nn = (size_t)nz * nz;
  const size_t bytes = sizeof(double2) * (5 * nn + (size_t)nz * nkeep) +
                       sizeof(double) * (size_t)nz * nkeep * 6;
  scratch.ensure(bytes);
  DKS_LAUNCH("k_rayleigh_ritz", k_rayleigh_ritz, dim3(1), dim3(kRRThreads), lds, st, A, S, nz,
             nkeep, drop_tol, floor_val, forced_drop, V, theta, info, dinfo, scratch.as<double2>(),
             tstamp);
  DKS_HIP(hipGetLastError());
}

}  // namespace dks
