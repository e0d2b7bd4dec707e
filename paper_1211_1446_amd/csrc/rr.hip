// Rayleigh-Ritz step of Algorithm 1 (the projected generalized eigenproblem on
// the subspace, sorted ascending) in FP64 on the device.
//
// Solves A v = theta S v for the nkeep lowest theta above `floor_val`, with
// A = Z^H H Z and S = Z^H Z of the current subspace Z = [X, Y, P], in three
// launches on one stream:
//   k_rr_reduce (one workgroup of 1024 threads; every step depends on the last)
//   1. symmetric diagonal scaling D S D, D = diag(S)^-1/2;
//   2. left-looking Cholesky D S D = L L^H; a column whose pivot falls below
//      `drop_tol` (its direction is numerically inside the span of the
//      earlier columns) is removed from the subspace instead of failing;
//   3. Li = L^-1 in place, C = Li (D A D) Li^H with LDS-tiled products that
//      skip the zero triangles;
//   4. Householder reduction C = Q T Q^H to a real symmetric tridiagonal T,
//      three workgroup barriers per reflector;
//   k_rr_values (one small workgroup per wanted eigenvalue)
//   5. the wanted eigenvalues of T by multisection on Sturm counts: those
//      below floor_val (the mid-gap -c^2: negative-band Ritz values) are
//      skipped;
//   k_rr_vectors (one workgroup per cluster of (nearly) equal eigenvalues)
//   6. their eigenvectors by inverse iteration, re-orthogonalised inside
//      the cluster (Kramers pairs, for one);
//   7. back-transformation v = D Li^H Q y, each y held in the registers of a
//      group of lanes while all reflectors are applied.
// Triangular factors and the Hermitian working matrix are packed lower
// triangles in LDS when n_Z <= 120, else full rows in the global scratch area.
// A caller that has S before A runs steps 1-3 without A (rayleigh_ritz_s:
// k_rr_reduce phase 2) on a stream of its own, and the rest after A is there
// (rayleigh_ritz_a: k_rr_scale_a forms D A D, then steps 3-7 as above).  The
// unbatched solver does so: S = Z^H Z is complete once Y is filtered, and the
// one-workgroup S phase then runs beside the application of H to Y.
#include <algorithm>
#include <cfloat>
#include <mutex>
#include <type_traits>

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

// Left-looking Cholesky with column dropping on the lower triangle of M (n x n),
// two columns per step.  For columns j and j + 1 the dot products
//   a_i = sum_{k<j} L_ik conj(L_jk),  b_i = sum_{k<j} L_ik conj(L_{j+1,k})
// of all rows i >= j are formed in one pass (kRowG lanes per row over strided
// k, reduced inside the lane group).  Thread 0 takes both pivots:
//   L_jj = sqrt(S_jj - a_j),  L_{j+1,j} = (S_{j+1,j} - a_{j+1}) / L_jj,
//   L_{j+1,j+1} = sqrt(S_{j+1,j+1} - b_{j+1} - |L_{j+1,j}|^2),
// passed on through LDS (`sc`), and every row i > j + 1 forms
//   L_ij = (S_ij - a_i) / L_jj,  L_{i,j+1} = (S_{i,j+1} - b_i - L_ij conj(L_{j+1,j})) / L_{j+1,j+1}.
// A pivot not above drop_tol (or a column of zero scale) drops its column: its
// L column is zero and keep[] = 0.  Three barriers per two columns.  Returns,
// in thread 0, the smallest pivot kept (1 in the other threads).
template <typename Mat>
__device__ double cholesky_drop(const Mat M, int n, double drop_tol, const double *dsc, int *keep,
                                double *sc, double2 *rowj, double2 *rowj1) {
  // rows in global memory (n_Z > 120): rows j and j + 1, read by every row
  // group, are staged in LDS first (one more barrier per step)
  constexpr bool kStage = std::is_same<Mat, FullLower>::value;
  const int tid = threadIdx.x, nt = blockDim.x, g = tid % kRowG, rl = tid / kRowG;
  double pmin = 1.0;
  for (int j = 0; j < n; j += 2) {
    const int m = n - j;   // rows j..n-1
    const bool two = m > 1;
    if constexpr (kStage) {
      for (int k = tid; k < j; k += nt) {
        rowj[k] = M.lo(j, k);
        if (two) rowj1[k] = M.lo(j + 1, k);
      }
      __syncthreads();
    }
    auto rowa = [&](int k) {
      if constexpr (kStage) return rowj[k]; else return M.lo(j, k);
    };
    auto rowb = [&](int k) {
      if constexpr (kStage) return rowj1[k]; else return M.lo(j + 1, k);
    };
    double2 da[kPasses], db[kPasses];
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      da[p] = db[p] = make_double2(0, 0);
      if (p * kRowsPass < m) {   // uniform
        const int ii = p * kRowsPass + rl;
        double2 sa = make_double2(0, 0), sb = make_double2(0, 0);
        if (ii < m) {
          const int i = j + ii;
          if (two) {
            for (int k = g; k < j; k += kRowG) {
              const double2 l = M.lo(i, k);
              sa = zfma(l, zconj(rowa(k)), sa);
              sb = zfma(l, zconj(rowb(k)), sb);
            }
          } else {
            for (int k = g; k < j; k += kRowG) sa = zfma(M.lo(i, k), zconj(rowa(k)), sa);
          }
        }
        da[p] = gsum2<kRowG>(sa);
        db[p] = gsum2<kRowG>(sb);
      }
    }
    // row j + 1's products to thread 0 (row j's are its own)
    if (two && rl == 1 && g == 0) {
      sc[2] = da[0].x;
      sc[3] = da[0].y;
      sc[4] = db[0].x;
    }
    __syncthreads();
    // the pivots, square roots and reciprocals by one thread (all 1024
    // repeating the FP64 square root and division cost more than the barrier)
    if (tid == 0) {
      const double piv = M.lo(j, j).x - da[0].x;
      const bool dr = (dsc[j] == 0.0) || !(piv > drop_tol);
      if (!dr) pmin = fmin(pmin, piv);
      const double l = dr ? 0.0 : sqrt(piv);
      const double inv = dr ? 0.0 : 1.0 / l;
      sc[0] = l;
      sc[1] = inv;
      if (two) {
        const double2 s10 = M.lo(j + 1, j);
        const double2 l10 = dr ? make_double2(0, 0)
                               : zscale(make_double2(s10.x - sc[2], s10.y - sc[3]), inv);
        const double piv1 = M.lo(j + 1, j + 1).x - sc[4] - (l10.x * l10.x + l10.y * l10.y);
        const bool dr1 = (dsc[j + 1] == 0.0) || !(piv1 > drop_tol);
        if (!dr1) pmin = fmin(pmin, piv1);
        const double l1 = dr1 ? 0.0 : sqrt(piv1);
        sc[5] = l10.x;
        sc[6] = l10.y;
        sc[7] = l1;
        sc[8] = dr1 ? 0.0 : 1.0 / l1;
      }
    }
    __syncthreads();
    const double ljj = sc[0], inv = sc[1];
    const bool drop = !(ljj > 0.0);
    const double2 l10 = two ? make_double2(sc[5], sc[6]) : make_double2(0, 0);
    const double l11 = two ? sc[7] : 0.0, inv1 = two ? sc[8] : 0.0;
    const bool drop1 = !(l11 > 0.0);
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      const int ii = p * kRowsPass + rl;
      if (g == 0 && ii >= 1 && ii < m) {
        const int i = j + ii;
        const double2 lij = drop ? make_double2(0, 0) : zscale(zsub(M.lo(i, j), da[p]), inv);
        M.set(i, j, lij);
        if (ii >= 2) {
          const double2 t = zsub(zsub(M.lo(i, j + 1), db[p]), zmul(lij, zconj(l10)));
          M.set(i, j + 1, drop1 ? make_double2(0, 0) : zscale(t, inv1));
        }
      }
    }
    if (tid == 0) {
      M.set(j, j, make_double2(ljj, 0.0));
      keep[j] = drop ? 0 : 1;
      if (two) {
        M.set(j + 1, j + 1, make_double2(l11, 0.0));
        keep[j + 1] = drop1 ? 0 : 1;
      }
    }
    __syncthreads();
  }
  return pmin;
}

// In-place inverse of the lower-triangular n x n matrix in M (nonzero real
// diagonal), two columns per step from the right: for the columns a = j - 1,
// b = j and L = [D 0; X L2] with D = [l_a 0; l_ba l_b] and X = [x_a x_b],
//   L^-1 = [D^-1 0; -L2^-1 X D^-1  L2^-1],  D^-1 = [1/l_a 0; -l_ba/(l_a l_b) 1/l_b],
// so that with Y = L2^-1 X (both columns in one pass over the inverted L2)
// column b becomes -Y_b / l_b below the diagonal and column a
// (Y_b l_ba / l_b - Y_a) / l_a.  Row groups as in the Cholesky; two barriers
// per two columns.  `cola`, `colb`: LDS staging of x_a, x_b (n entries each);
// `sl`: two doubles of LDS for l_ba.
template <typename Mat>
__device__ void trtri_lower(const Mat M, int n, double2 *cola, double2 *colb, double *dinv,
                            double *sl) {
  const int tid = threadIdx.x, nt = blockDim.x, g = tid % kRowG, rl = tid / kRowG;
  // reciprocals of the diagonal, all at once (column j only changes its own)
  for (int j = tid; j < n; j += nt) dinv[j] = 1.0 / M.lo(j, j).x;
  // the columns of the first step below their diagonal block: read across rows
  // they are strided accesses, in global memory for large n
  auto stage = [&](int jb) {   // pair (jb - 1, jb), or the single column 0
    const int m = n - jb - 1;
    if (jb >= 1) {
      for (int k = tid; k < m; k += nt) {
        cola[k] = M.lo(jb + 1 + k, jb - 1);
        colb[k] = M.lo(jb + 1 + k, jb);
      }
      if (tid == 0) {
        const double2 v = M.lo(jb, jb - 1);
        sl[0] = v.x;
        sl[1] = v.y;
      }
    } else {
      for (int k = tid; k < m; k += nt) colb[k] = M.lo(jb + 1 + k, jb);
    }
  };
  stage(n - 1);
  __syncthreads();
  for (int j = n - 1; j >= 0; j -= 2) {
    const bool two = j >= 1;
    const int m = n - j - 1;   // rows of the inverted trailing block L2
    const double ib = dinv[j], ia = two ? dinv[j - 1] : 0.0;
    const double2 lba = two ? make_double2(sl[0], sl[1]) : make_double2(0, 0);
    double2 ya[kPasses], yb[kPasses];
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      ya[p] = yb[p] = make_double2(0, 0);
      if (p * kRowsPass < m) {   // uniform
        const int ii = p * kRowsPass + rl;
        double2 sa = make_double2(0, 0), sb = make_double2(0, 0);
        if (ii < m) {
          if (two) {
            for (int k = g; k <= ii; k += kRowG) {
              const double2 l = M.lo(j + 1 + ii, j + 1 + k);
              sa = zfma(l, cola[k], sa);
              sb = zfma(l, colb[k], sb);
            }
          } else {
            for (int k = g; k <= ii; k += kRowG) sb = zfma(M.lo(j + 1 + ii, j + 1 + k), colb[k], sb);
          }
        }
        ya[p] = gsum2<kRowG>(sa);
        yb[p] = gsum2<kRowG>(sb);
      }
    }
    __syncthreads();   // the staged columns and l_ba are read everywhere
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      const int ii = p * kRowsPass + rl;
      if (g == 0 && ii < m) {
        M.set(j + 1 + ii, j, zscale(yb[p], -ib));
        if (two) M.set(j + 1 + ii, j - 1, zscale(zsub(zscale(zmul(yb[p], lba), ib), ya[p]), ia));
      }
    }
    if (tid == 0) {
      M.set(j, j, make_double2(ib, 0.0));
      if (two) {
        M.set(j - 1, j - 1, make_double2(ia, 0.0));
        M.set(j, j - 1, zscale(lba, -ia * ib));
      }
    }
    // the next pair's columns below their diagonal block: rows j - 1.. of
    // columns j - 3, j - 2, untouched so far
    if (j >= 2) stage(j - 2);
    __syncthreads();
  }
}

struct TriWork {
  double *dd, *ee;       // diagonal (r), off-diagonal (r-1)
  double2 *tauv;         // reflector scalars (r-1)
  double2 *vv0, *vv1, *xv;   // reflector vectors (even, odd steps), tau C v (r)
  __device__ double2 *vv(int k) const { return (k & 1) ? vv1 : vv0; }
  double *nred, *qred;   // per-wave partial sums (16 each)
};

// Householder tridiagonalisation of the r x r Hermitian matrix held in M's lower
// triangle.  Reflector k (H_k = I - tau_k v v^H, v = [1, M(k+2.., k)]) acts on
// rows k+1..r-1; the column below the subdiagonal keeps v for the
// back-transformation.  With x = tau C22 v and q = v^H C22 v (real), the
// two-sided update is C22 -= v w^H + w v^H, w = x - |tau|^2 q v / 2.  Per
// reflector, three barriers on full rows in global memory: (b) x by row
// groups of all waves, and q's per-wave partials; (c1) the update of the
// trailing matrix's first column, which also sums that column's norm; (c2)
// waves 1-15 update the rest while wave 0 forms the next reflector from the
// finished column (look-ahead: its scalar arithmetic and the writing of v no
// longer stand between two barriers).  Packed in LDS, two: wave 0 does (c1)
// itself, with the same sums, and goes on to the reflector.
// Reflector vectors alternate between two LDS buffers, since wave 0 writes
// v_{k+1} while the others still read v_k.
template <typename Mat>
__device__ void tridiagonalise(const Mat M, int r, TriWork w) {
  constexpr int NW = kRRThreads / 64;
  // packed (LDS, order <= 120) matrices: wave 0 takes the first column itself
  // (one barrier fewer); full rows in global memory keep it on all threads
  constexpr bool kFusedCol = std::is_same<Mat, PackedLower>::value;
  static_assert(kRRPackedMax <= 128 && kRRThreads >= 128, "wave 0 covers the first column in two rows of lanes");
  constexpr int kUpRows = (kRRThreads - 64) / kRowG;                  // rows per pass, waves 1-15
  constexpr int kUpPasses = (kRRMax + kUpRows - 1) / kUpRows;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wid = tid >> 6, g = tid % kRowG, rl = tid / kRowG;
  const int rlu = (tid - 64) / kRowG;   // row of waves 1-15 in the update
  // reflector k from column k (its norm below the subdiagonal in w.nred), by
  // wave 0: tau, beta and the diagonal entry to LDS, v into w.vv[k & 1] and M
  auto reflector = [&](int k, double xn2) {
    const int m = r - k - 1;
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
    if (lane == 0) {
      w.tauv[k] = tau;
      w.ee[k] = beta;
      w.dd[k] = M.lo(k, k).x;
    }
    double2 *vv = w.vv(k);
    for (int i = lane; i < m; i += 64) {
      const double2 v = (i == 0) ? make_double2(1, 0) : zmul(M.lo(k + 1 + i, k), scal);
      vv[i] = v;
      if (i > 0) M.set(k + 1 + i, k, v);
    }
  };
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
  auto nred_sum = [&]() {
    double xn2 = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) xn2 += w.nred[q];
    return xn2;
  };
  if (r >= 2 && wid == 0) reflector(0, nred_sum());
  __syncthreads();
  for (int k = 0; k + 1 < r; ++k) {
    const int m = r - k - 1;   // trailing size, rows/cols k+1..r-1
    const double2 *vv = w.vv(k);
    const double2 tau = w.tauv[k];
    // (b) x = tau C22 v, C22 Hermitian from its lower triangle
    double qp = 0;
#pragma unroll
    for (int p = 0; p < kPasses; ++p) {
      if (p * kRowsPass < m) {   // uniform
        const int ii = p * kRowsPass + rl;
        double2 s = make_double2(0, 0), s1 = make_double2(0, 0);
        if (ii < m) {
          const int gi = k + 1 + ii;
          // one load from a selected address (a select between two loads
          // would become a branch around each of them)
          auto elem = [&](int jj) {
            const int gj = k + 1 + jj;
            const bool low = jj <= ii;
            double2 c = M.lo(low ? gi : gj, low ? gj : gi);
            if (!low) c.y = -c.y;
            return c;
          };
          int jj = g;
#pragma unroll 2
          for (; jj + kRowG < m; jj += 2 * kRowG) {   // two chains in flight
            s = zfma(elem(jj), vv[jj], s);
            s1 = zfma(elem(jj + kRowG), vv[jj + kRowG], s1);
          }
          if (jj < m) s = zfma(elem(jj), vv[jj], s);
        }
        s = gsum2<kRowG>(zadd(s, s1));
        if (ii < m && g == 0) {
          w.xv[ii] = zmul(tau, s);
          const double2 vi = vv[ii];
          qp += vi.x * s.x + vi.y * s.y;   // Re(conj(v_i) (C22 v)_i)
        }
      }
    }
    qp = wave_sum(qp);
    if (lane == 0) w.qred[wid] = qp;
    __syncthreads();
    double q = 0;
#pragma unroll
    for (int p = 0; p < NW; ++p) q += w.qred[p];
    const double al = -0.5 * (tau.x * tau.x + tau.y * tau.y) * q;
    auto wv = [&](int i) { return zadd(w.xv[i], zscale(vv[i], al)); };
    // one element of the update of the trailing matrix's first column (local
    // column 0) and its share of that column's norm below the subdiagonal
    const double2 v0 = vv[0], w0 = wv(0);
    auto col0 = [&](int ii) {
      const double2 vi = vv[ii], wi = wv(ii);
      double2 c = M.lo(k + 1 + ii, k + 1);
      c = zsub(c, zadd(zmul(vi, zconj(w0)), zmul(wi, zconj(v0))));
      if (ii == 0) c.y = 0.0;
      M.set(k + 1 + ii, k + 1, c);
      return ii >= 2 ? c.x * c.x + c.y * c.y : 0.0;
    };
    // the rest of the update (local columns 1..), waves 1-15, row groups over
    // 1 <= j <= i
    auto update_rest = [&]() {
#pragma unroll
      for (int p = 0; p < kUpPasses; ++p) {
        const int ii = p * kUpRows + rlu;
        if (p * kUpRows < m && ii < m && ii >= 1) {
          const double2 vi = vv[ii];
          const double2 wi = wv(ii);
          const int gi = k + 1 + ii;
#pragma unroll 4
          for (int jj = 1 + g; jj <= ii; jj += kRowG) {
            const double2 vj = vv[jj];
            const double2 wj = wv(jj);
            double2 c = M.lo(gi, k + 1 + jj);
            c = zsub(c, zadd(zmul(vi, zconj(wj)), zmul(wi, zconj(vj))));
            if (ii == jj) c.y = 0.0;
            M.set(gi, k + 1 + jj, c);
          }
        }
      }
    };
    if constexpr (kFusedCol) {
      // (c) wave 0 updates the first column (m <= 119: rows lane and 64 +
      // lane), sums its norm exactly as the per-wave partials of (c1) below
      // would (the same lanes, the same reductions, added in wave order) and
      // forms the next reflector from the values its lanes have just written
      // (the fence orders them); meanwhile waves 1-15 update the rest.  Two
      // barriers per reflector, the same numbers as three.
      if (wid == 0) {
        const double p0 = wave_sum(lane < m ? col0(lane) : 0.0);
        const double p1 = wave_sum(64 + lane < m ? col0(64 + lane) : 0.0);
        double xn2 = 0;
        xn2 += p0;
        xn2 += p1;
        __threadfence_block();
        if (k + 2 < r) reflector(k + 1, xn2);
      } else {
        update_rest();
      }
      __syncthreads();
    } else {
      // (c1) the first column by all threads, its norm from per-wave partials
      {
        double nx = 0;
        for (int ii = tid; ii < m; ii += nt) nx += col0(ii);
        nx = wave_sum(nx);
        if (lane == 0) w.nred[wid] = nx;
      }
      __syncthreads();
      // (c2) the rest, waves 1-15, while wave 0 forms the next reflector from
      // the finished column
      if (wid == 0) {
        if (k + 2 < r) reflector(k + 1, nred_sum());
      } else {
        update_rest();
      }
      __syncthreads();
    }
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

// Global scratch of one Rayleigh-Ritz (n_Z = nz, nkeep wanted pairs): the
// reduction's working matrices and what the three kernels hand on.
struct RRScratch {
  double2 *Sg;     // scaled S lower triangle (full-row path)
  double2 *Am;     // scaled A (full)
  double2 *Lc;     // L^-1 column-major: Lc[c r + b] = Li[b][c]
  double2 *Mm;     // A_r Li^H; compaction buffer; C and its reflectors (full-row path)
  double2 *Cg;     // C = Li A_r Li^H, lower tiles
  double2 *refl;   // packed reflectors (packed path)
  double2 *tau;    // reflector scalars
  double *U;       // nkeep real eigenvectors of T, r each
  double *dd, *ee, *dsc, *lam;
  int *kept;
  __host__ __device__ static size_t bytes(int nz, int nkeep) {
    const size_t nn = (size_t)nz * nz;
    return sizeof(double2) * (5 * nn + (size_t)nz * (nz + 1) / 2 + nz) +
           sizeof(double) * ((size_t)nkeep * nz + 3 * (size_t)nz + nkeep + 1) + sizeof(int) * nz;
  }
  __host__ __device__ static RRScratch at(void *base, int nz, int nkeep) {
    const size_t nn = (size_t)nz * nz;
    RRScratch w;
    w.Sg = static_cast<double2 *>(base);
    w.Am = w.Sg + nn;
    w.Lc = w.Am + nn;
    w.Mm = w.Lc + nn;
    w.Cg = w.Mm + nn;
    w.refl = w.Cg + nn;
    w.tau = w.refl + (size_t)nz * (nz + 1) / 2;
    w.U = reinterpret_cast<double *>(w.tau + nz);
    w.dd = w.U + (size_t)nkeep * nz;
    w.ee = w.dd + nz;
    w.dsc = w.ee + nz;
    w.lam = w.dsc + nz;
    w.kept = reinterpret_cast<int *>(w.lam + nkeep + 1);
    return w;
  }
};

// ---- 1-4 in one workgroup, in two launches around the two products of
// k_rr_gemm: phase 0 scales, factors (Cholesky with dropping), compacts and
// inverts L; phase 1 takes C = Li A Li^H from the products, forms its
// Hermitian part and reduces it to the tridiagonal T.
__global__ void __launch_bounds__(kRRThreads) k_rr_reduce(
    int phase, const double2 *__restrict__ Ain, const double2 *__restrict__ Sin, int nz, int nkeep,
    double drop_tol, const int *__restrict__ forced, int *__restrict__ info,
    double *__restrict__ dinfo, RRScratch W, long long *__restrict__ tstamp,
    const int *__restrict__ skip) {
  // phase 0: scaling, Cholesky and L^-1 (and the scaled A); phase 2: the same
  // without A, which k_rr_scale_a forms once A is there; phase 1: the rest.
  // A finished system of a graph-captured batch: status 3 makes every later
  // Rayleigh-Ritz kernel of the call return at once
  if (phase != 1 && skip && *skip) {
    if (threadIdx.x == 0) {
      info[0] = 0;
      info[1] = 3;
    }
    return;
  }
  // no static LDS in this kernel: the dynamic arena then starts at offset 0,
  // 16-byte aligned, as the double2 accesses (ds_read_b128) need for speed
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // optional phase timestamps (constant-rate wall clock), for tuning
#define DKS_RR_STAMP(k) \
  do {                  \
    if (tstamp && threadIdx.x == 0) tstamp[k] = wall_clock64(); \
  } while (0)
  if (phase != 1) DKS_RR_STAMP(0);
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

  const int tid = threadIdx.x, nt = blockDim.x;
  const size_t nn = (size_t)nz * nz;
  double2 *Sg = W.Sg, *Am = W.Am, *Lc = W.Lc, *Mm = W.Mm, *Cg = W.Cg;
  const bool packed = (nz <= kRRPackedMax);
  if (phase == 1) {
    if (info[1]) return;
    const int r = info[0];
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
      // the second reflector buffer takes the e2 and lam arrays (unused here)
      TriWork tw{dd, ee, tauv, vv, reinterpret_cast<double2 *>(e2), xv, red + 32, red + 48};
      if (packed) tridiagonalise(PackedLower{big}, r, tw); else tridiagonalise(FullLower{Mm, r}, r, tw);
    }
    // ---- hand-off to the eigenvalue and eigenvector kernels
    for (int i = tid; i < r; i += nt) {
      W.dd[i] = dd[i];
      W.ee[i] = (i + 1 < r) ? ee[i] : 0.0;
      W.tau[i] = (i + 1 < r) ? tauv[i] : make_double2(0, 0);
    }
    if (packed)
      for (int e = tid; e < r * (r + 1) / 2; e += nt) W.refl[e] = big[e];
    DKS_RR_STAMP(5);
    return;
  }

  // ---- 1. scaling and Hermitian parts
  for (int i = tid; i < nz; i += nt) {
    const double s = Sin[(size_t)i * nz + i].x;
    const bool f = forced ? (forced[i] != 0) : false;
    dsc[i] = (!f && s > 0 && isfinite(s)) ? 1.0 / sqrt(s) : 0.0;
  }
  __syncthreads();
  // one wave per row, lanes along it (no division of the flat index)
  for (int i = tid >> 6; i < nz; i += nt >> 6) {
    const double di = dsc[i];
#pragma unroll 2
    for (int j = tid & 63; j < nz; j += 64) {
      const size_t e = (size_t)i * nz + j;
      const double f = di * dsc[j];
      if (phase == 0) {
        const double2 a1 = Ain[e], a2 = Ain[(size_t)j * nz + i];
        Am[e] = make_double2(0.5 * f * (a1.x + a2.x), 0.5 * f * (a1.y - a2.y));
      }
      if (j <= i) {
        const double2 s1 = Sin[e], s2 = Sin[(size_t)j * nz + i];
        const double2 h = make_double2(0.5 * f * (s1.x + s2.x), 0.5 * f * (s1.y - s2.y));
        if (packed) PackedLower{big}.set(i, j, h); else FullLower{Sg, nz}.set(i, j, h);
      }
    }
  }
  __syncthreads();
  DKS_RR_STAMP(1);

  // ---- 2. Cholesky with column dropping
  const double pmin = packed ? cholesky_drop(PackedLower{big}, nz, drop_tol, dsc, kept, red + 4, vv, xv)
                             : cholesky_drop(FullLower{Sg, nz}, nz, drop_tol, dsc, kept, red + 4, vv, xv);
  if (tid == 0) {
    dinfo[1] = pmin;
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
  // (dd: free until the tridiagonalisation)
  if (packed) trtri_lower(PackedLower{big}, r, vv, xv, dd, red + 16);
  else trtri_lower(FullLower{Sg, r}, r, vv, xv, dd, red + 16);
  for (int e = tid; e < r * r; e += nt) {
    const int c = e / r, b = e - (e / r) * r;   // Lc[c r + b] = Li[b][c]
    Lc[e] = (b >= c) ? (packed ? PackedLower{big}.lo(b, c) : FullLower{Sg, r}.lo(b, c))
                     : make_double2(0, 0);
  }
  for (int i = tid; i < r; i += nt) W.kept[i] = kept[i];
  for (int i = tid; i < nz; i += nt) W.dsc[i] = dsc[i];
  DKS_RR_STAMP(3);

#undef DKS_RR_STAMP
}

// ---- 1b. the scaled Hermitian part of A, D (A + A^H) D / 2, for a Rayleigh-Ritz
// whose S phase ran without A (phase 2); one wave per row, D from that phase
__global__ void __launch_bounds__(256) k_rr_scale_a(const double2 *__restrict__ Ain, int nz,
                                                    const int *__restrict__ info, RRScratch W) {
  if (info[1]) return;   // the S phase found too few independent columns
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nz) return;
  const double di = W.dsc[i];
  for (int j = threadIdx.x & 63; j < nz; j += 64) {
    const size_t e = (size_t)i * nz + j;
    const double f = di * W.dsc[j];
    const double2 a1 = Ain[e], a2 = Ain[(size_t)j * nz + i];
    W.Am[e] = make_double2(0.5 * f * (a1.x + a2.x), 0.5 * f * (a1.y - a2.y));
  }
}

// ---- 3b. the two products of C = Li (D A D)_kept Li^H, one 64 x 64 output tile
// per workgroup: which = 1: Mm[a][b] = sum_{c <= b} A[ka][kc] conj(Li[b][c]);
// which = 2: Cg[a][b] = sum_{c <= a} Li[a][c] Mm[c][b] on the tiles touching the
// lower triangle.  The zero triangles of Li bound the k range of each tile.
__global__ void __launch_bounds__(kRRThreads) k_rr_gemm(int which, int nz, const int *__restrict__ info,
                                                        RRScratch W) {
  __shared__ double2 ta[kGT * kGK], tb[kGK * kGT];
  if (info[1]) return;
  const int r = info[0];
  const int ti = blockIdx.x * kGT, tj = blockIdx.y * kGT;
  if (ti >= r || tj >= r || (which == 2 && tj > ti)) return;   // uniform
  const int *kept = W.kept;
  const double2 *Am = W.Am, *Lc = W.Lc;
  double2 *Mm = W.Mm, *Cg = W.Cg;
  auto only = [&](int i0, int j0) { return i0 == ti && j0 == tj; };
  if (which == 1)
    wg_gemm(
        r, r, r, [&](int i, int k) { return Am[(size_t)kept[i] * nz + kept[k]]; },
        [&](int k, int j) { return zconj(Lc[(size_t)k * r + j]); },
        [&](int i, int j, double2 v) { Mm[(size_t)i * r + j] = v; },
        [&](int, int j0, int &kb, int &ke) { kb = 0; ke = j0 + kGT; }, only, ta, tb);
  else
    wg_gemm(
        r, r, r, [&](int i, int k) { return Lc[(size_t)k * r + i]; },
        [&](int k, int j) { return Mm[(size_t)k * r + j]; },
        [&](int i, int j, double2 v) { Cg[(size_t)i * r + j] = v; },
        [&](int i0, int, int &kb, int &ke) { kb = 0; ke = i0 + kGT; }, only, ta, tb);
}

// Sturm tolerances and the padded Gershgorin interval [glo, ghi] of T
// (emax2 = the largest squared off-diagonal entry).
struct SturmBounds {
  double glo, ghi, tnorm, pivmin, atol;
};
__device__ SturmBounds sturm_bounds_of(double glo, double ghi, double emax2) {
  SturmBounds b;
  b.tnorm = fmax(fabs(glo), fabs(ghi));
  b.pivmin = DBL_MIN * fmax(1.0, emax2);
  b.atol = DBL_EPSILON * b.tnorm;
  b.glo = glo - (2.0 * DBL_EPSILON * b.tnorm + 2 * b.pivmin);
  b.ghi = ghi + (2.0 * DBL_EPSILON * b.tnorm + 2 * b.pivmin);
  return b;
}

// ---- 5. one wanted eigenvalue of T per workgroup by multisection: target
// t < nkeep is eigenvalue k0 + t (k0 = number below floor_val), target nkeep
// the smallest.  Each round every thread takes a Sturm count at one of
// blockDim.x interior points of the bracket [lo, hi) (count(lo) <= index <
// count(hi)); the counts are monotone in the point, so the number of points
// with count <= index locates the new bracket between two neighbouring points.
// Small workgroups: a round is one Sturm recurrence long, and more points per
// round would cost more than the rounds they save.
constexpr int kValThreads = 128;   // Sturm points per round and target
__global__ void __launch_bounds__(kValThreads) k_rr_values(
    const double *__restrict__ g_dd, const double *__restrict__ g_ee, int nkeep, double floor_val,
    int *__restrict__ info, double *__restrict__ lam, double *__restrict__ theta,
    double *__restrict__ dinfo, long long *__restrict__ tstamp) {
  __shared__ double dd[kRRMax], e2[kRRMax];
  __shared__ double bred[3][kValThreads / 64];
  __shared__ int cnt[2][kValThreads / 64];
  __shared__ int s_k0;
  if (info[1]) return;   // the Cholesky dropped too much: nothing to do
  const int r = info[0];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6;
  const bool stamp = tstamp && blockIdx.x == 0 && tid == 0;
  if (stamp) tstamp[12] = wall_clock64();
  for (int i = tid; i < r; i += nt) {
    dd[i] = g_dd[i];
    e2[i] = g_ee[i] * g_ee[i];
  }
  // Gershgorin interval, one row per thread, reduced over the workgroup
  double glo = 1e300, ghi = -1e300, emax2 = 0;
  for (int i = tid; i < r; i += nt) {
    const double el = (i > 0) ? g_ee[i - 1] : 0.0, er = (i + 1 < r) ? g_ee[i] : 0.0;
    const double off = fabs(el) + fabs(er);
    const double di = g_dd[i];
    glo = fmin(glo, di - off);
    ghi = fmax(ghi, di + off);
    emax2 = fmax(emax2, er * er);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    glo = fmin(glo, __shfl_xor(glo, o));
    ghi = fmax(ghi, __shfl_xor(ghi, o));
    emax2 = fmax(emax2, __shfl_xor(emax2, o));
  }
  if (lane == 0) {
    bred[0][wid] = glo;
    bred[1][wid] = ghi;
    bred[2][wid] = emax2;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kValThreads / 64; ++q) {
    glo = fmin(glo, bred[0][q]);
    ghi = fmax(ghi, bred[1][q]);
    emax2 = fmax(emax2, bred[2][q]);
  }
  const SturmBounds sb = sturm_bounds_of(glo, ghi, emax2);
  if (tid == 0) {
    const int k0 = (floor_val > sb.glo) ? sturm_count(dd, e2, r, floor_val, sb.pivmin) : 0;
    s_k0 = k0;
    if (blockIdx.x == 0) {
      info[3] = k0;
      if (r - k0 < nkeep) info[1] = 2;
    }
  }
  __syncthreads();
  const int k0 = s_k0;
  if (r - k0 < nkeep) return;
  if (stamp) tstamp[13] = wall_clock64();
  const int t = blockIdx.x;
  const int idx = (t < nkeep) ? k0 + t : 0;
  const double inv_np1 = 1.0 / (double)(nt + 1);
  double lo = sb.glo, hi = sb.ghi;
  for (int round = 0; round < 64; ++round) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + sb.atol + sb.pivmin) break;
    const double x = lo + (hi - lo) * ((double)(tid + 1) * inv_np1);
    const int c = sturm_count(dd, e2, r, x, sb.pivmin);
    const unsigned long long bal = __ballot(c <= idx);
    if (lane == 0) cnt[round & 1][wid] = __popcll(bal);
    __syncthreads();
    int a = -1;   // index of the last point with count <= idx
#pragma unroll
    for (int q = 0; q < kValThreads / 64; ++q) a += cnt[round & 1][q];
    const double nlo = (a >= 0) ? lo + (hi - lo) * ((double)(a + 1) * inv_np1) : lo;
    const double nhi = (a + 1 < nt) ? lo + (hi - lo) * ((double)(a + 2) * inv_np1) : hi;
    if (nhi > nlo && nhi - nlo < hi - lo) {
      lo = nlo;
      hi = nhi;
    } else {
      // no representable interior point left: the bracket has converged
      lo = hi = 0.5 * (lo + hi);
    }
  }
  if (tid == 0) {
    const double v = 0.5 * (lo + hi);
    if (t < nkeep) {
      lam[t] = v;
      theta[t] = v;
    } else {
      dinfo[0] = v;
    }
  }
  if (stamp) tstamp[14] = wall_clock64();
}

// LDS of k_rr_vectors: inverse-iteration slots (x, LU factors, swaps), later
// reused for the packed reflectors when n_Z <= kRRPackedMax.
__host__ __device__ inline size_t rr_slot_bytes(int nz) {
  return sizeof(double) * 5 * (size_t)nz + (((size_t)nz + 15) & ~(size_t)15);
}
constexpr int kRRSlots = kRRThreads / 64;
constexpr int kUc = 16;   // eigenvectors back-transformed per pass (LDS copies)
constexpr size_t kRRVecLds = 144 * 1024;
__host__ __device__ inline int rr_slots(int nz) {
  const size_t fixed = sizeof(double) * 2 * (size_t)nz + sizeof(int) * (size_t)nz + 256;
  const size_t s = (kRRVecLds - fixed) / rr_slot_bytes(nz);
  return s < 1 ? 1 : (s > (size_t)kRRSlots ? kRRSlots : (int)s);
}

// sum over the workgroup (every thread gets it); red holds kRRThreads / 64 doubles
__device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int q = 0; q < kRRThreads / 64; ++q) s += red[q];
  return s;
}

// Back-transformation of one eigenvector by a group of G lanes: u = Q x (x
// real, length r), Q = H_0 ... H_{r-2} with reflector k in column k of M below
// the subdiagonal; lane l of the group holds rows l + G s.  u goes to out.
template <int G, int NPL, typename Mat>
__device__ void bt_group(const Mat M, int r, const double2 *tauv, const double *x, double2 *out) {
  const int gl = threadIdx.x % G;
  double2 u[NPL];
#pragma unroll
  for (int s = 0; s < NPL; ++s) {
    const int i = gl + G * s;
    u[s] = (i < r) ? make_double2(x[i], 0.0) : make_double2(0, 0);
  }
  for (int k = r - 2; k >= 0; --k) {
    const double2 tau = tauv[k];
    if (tau.x == 0.0 && tau.y == 0.0) continue;   // uniform
    // every lane loads (rows outside k+2..r-1 read row k+1 and are masked
    // after): conditional loads would be serialised behind branches
    double2 v[NPL];
    double2 acc = make_double2(0, 0);
#pragma unroll
    for (int s = 0; s < NPL; ++s) {
      const int i = gl + G * s;
      const bool on = i > k && i < r;
      const double2 m = M.lo(on ? i : k + 1, k);
      v[s] = on ? (i == k + 1 ? make_double2(1, 0) : m) : make_double2(0, 0);
      acc = zadd(acc, zcmul(v[s], u[s]));
    }
    acc = zmul(tau, gsum2<G>(acc));
#pragma unroll
    for (int s = 0; s < NPL; ++s) u[s] = zsub(u[s], zmul(v[s], acc));
  }
#pragma unroll
  for (int s = 0; s < NPL; ++s) {
    const int i = gl + G * s;
    if (i < r) out[i] = u[s];
  }
}

// V = D Li^H Uc for nc vectors held in LDS (uc[c r + a]): row kept[i] of
// column j0 + c gets d_i sum_{a >= i} conj(Li[a][i]) Uc_c[a], Lc[i r + a] =
// Li[a][i].  One wave per row, lane l takes a = l + 64 s.
template <int NPL>
__device__ void li_rows(const double2 *__restrict__ Lc, int r, const int *kept, const double *dsc,
                        const double2 *uc, int nc, double2 *__restrict__ V, int ldv, int j0) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = wid; i < r; i += kRRThreads / 64) {
    double2 l[NPL];
#pragma unroll
    for (int s = 0; s < NPL; ++s) {
      const int a = lane + 64 * s;
      l[s] = (a >= i && a < r) ? Lc[(size_t)i * r + a] : make_double2(0, 0);
    }
    const int ki = kept[i];
    const double d = dsc[ki];
    for (int c = 0; c < nc; ++c) {
      double2 acc = make_double2(0, 0);
#pragma unroll
      for (int s = 0; s < NPL; ++s) {
        const int a = lane + 64 * s;
        if (a < r) acc = zadd(acc, zcmul(l[s], uc[(size_t)c * r + a]));
      }
      acc = gsum2<64>(acc);
      if (lane == 0) V[(size_t)ki * ldv + j0 + c] = zscale(acc, d);
    }
  }
}

// ---- 6-7. eigenvectors, one cluster of (nearly) equal eigenvalues per
// workgroup (the workgroup of the cluster's first member; the others exit):
// inverse iteration with the shifts spread by 10 ulp(T), one vector per wave
// with its LU factors in LDS; modified Gram-Schmidt (two passes) inside the
// cluster; then each wave back-transforms one vector, v = D Li^H Q x.
// kSmall: n_Z <= 128, so r <= 128 (register columns of 8 rows per 16-lane
// group); the general form keeps 8 rows per lane of a wave.
template <bool kSmall>
__global__ void __launch_bounds__(kRRThreads) k_rr_vectors(
    const double *__restrict__ g_dd, const double *__restrict__ g_ee,
    const double2 *__restrict__ g_tau, const double2 *__restrict__ g_refl,
    const double2 *__restrict__ Mfull, const double2 *__restrict__ Lc, const int *__restrict__ g_kept,
    const double *__restrict__ g_dsc, const double *__restrict__ lam, const int *__restrict__ info,
    int nz, int nkeep, double *__restrict__ U, double2 *__restrict__ Vout,
    long long *__restrict__ tstamp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  if (info[1]) return;
  const int r = info[0];
  const int t = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6;
  const bool stamp = tstamp && t == 0 && tid == 0;
  if (stamp) tstamp[16] = wall_clock64();
  double *dd = reinterpret_cast<double *>(smem_raw);
  double *ee = dd + nz;
  int *kinv = reinterpret_cast<int *>(ee + nz);
  double *red = reinterpret_cast<double *>(kinv + ((nz + 3) & ~3));   // 32
  unsigned char *area = reinterpret_cast<unsigned char *>(red + 32);
  for (int i = tid; i < r; i += nt) {
    dd[i] = g_dd[i];
    ee[i] = g_ee[i];
  }
  __syncthreads();
  // the cluster tolerances, from T's Gershgorin bound (as the values kernel)
  double tn = 0;
  for (int i = 0; i < r; ++i) {
    const double off = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < r ? fabs(ee[i]) : 0.0);
    tn = fmax(tn, fmax(fabs(dd[i] - off), fabs(dd[i] + off)));
  }
  const double ctol = 1e-7 * fmax(tn, 1e-300);
  const double eps_t = DBL_EPSILON * fmax(tn, 1e-300);
  if (t > 0 && lam[t] - lam[t - 1] <= ctol) return;   // not a cluster leader (uniform)
  int tend = t + 1;
  while (tend < nkeep && lam[tend] - lam[tend - 1] <= ctol) ++tend;
  const int csz = tend - t;
  if (stamp) tstamp[17] = wall_clock64();
  // inverse iteration, nslot vectors at a time (lane 0 of waves 0..nslot-1)
  const int nslot = rr_slots(nz);
  const size_t sb = rr_slot_bytes(nz);
  for (int q0 = 0; q0 < csz; q0 += nslot) {
    const int q = q0 + wid;
    unsigned char *slot = area + (size_t)wid * sb;
    double *x = reinterpret_cast<double *>(slot);
    double *f = x + nz;
    unsigned char *sw = reinterpret_cast<unsigned char *>(f + 4 * nz);
    if (wid < nslot && q < csz && lane == 0)
      inverse_iteration(dd, ee, r, lam[t + q] + (double)q * 10.0 * eps_t, eps_t, t + q, x, f, sw);
    __syncthreads();
    for (int e = tid; e < nslot * r; e += nt) {
      const int w = e / r, i = e - (e / r) * r;
      if (q0 + w < csz)
        U[(size_t)(t + q0 + w) * r + i] = reinterpret_cast<const double *>(area + (size_t)w * sb)[i];
    }
    __syncthreads();
  }
  if (stamp) tstamp[18] = wall_clock64();
  // modified Gram-Schmidt inside the cluster, two passes, the whole workgroup
  for (int jv = 1; jv < csz; ++jv) {
    double *xv = U + (size_t)(t + jv) * r;
    for (int pass = 0; pass < 2; ++pass)
      for (int jp = 0; jp < jv; ++jp) {
        const double *yv = U + (size_t)(t + jp) * r;
        double d = 0;
        for (int i = tid; i < r; i += nt) d += yv[i] * xv[i];
        d = block_sum(d, red);
        for (int i = tid; i < r; i += nt) xv[i] -= d * yv[i];
        __syncthreads();
      }
    double nn = 0;
    for (int i = tid; i < r; i += nt) nn += xv[i] * xv[i];
    nn = block_sum(nn, red);
    const double inv = 1.0 / sqrt(nn);
    for (int i = tid; i < r; i += nt) xv[i] *= inv;
    __syncthreads();
  }
  if (stamp) tstamp[19] = wall_clock64();
  // rows of V outside the kept set are zero
  for (int i = tid; i < nz; i += nt) kinv[i] = -1;
  __syncthreads();
  for (int i = tid; i < r; i += nt) kinv[g_kept[i]] = i;
  __syncthreads();
  for (int e = tid; e < nz * csz; e += nt) {
    const int row = e / csz, c = e - (e / csz) * csz;
    if (kinv[row] < 0) Vout[(size_t)row * nkeep + t + c] = make_double2(0, 0);
  }
  // back-transformation and V = D Li^H Uc, kUc vectors at a time
  const bool packed = nz <= kRRPackedMax;
  double2 *tv = reinterpret_cast<double2 *>(area);
  double2 *pk = tv + ((nz + 1) & ~1);
  double2 *ucs = packed ? pk + (size_t)nz * (nz + 1) / 2 : reinterpret_cast<double2 *>(area);
  if (packed) {
    for (int i = tid; i < r; i += nt) tv[i] = g_tau[i];
    const int tri = r * (r + 1) / 2;
    for (int e0 = 0; e0 < tri; e0 += 8 * kRRThreads) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = g_refl[min(e0 + u * kRRThreads + tid, tri - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (e0 + u * kRRThreads + tid < tri) pk[e0 + u * kRRThreads + tid] = v[u];
    }
  }
  __syncthreads();
  if (stamp) tstamp[20] = wall_clock64();
  const FullLower Mf{const_cast<double2 *>(Mfull), r};
  for (int c0 = 0; c0 < csz; c0 += kUc) {
    const int nc = min(kUc, csz - c0);
    if constexpr (kSmall) {
      // 16 lanes per vector, 8 rows each: DPP-only reductions (one wave per
      // vector, 2 rows per lane, was 13 % faster but its other rounding cost
      // the FP32 graph-form batch its close-cluster item)
      const int grp = tid / 16;
      if (grp < nc) {
        const double *xq = U + (size_t)(t + c0 + grp) * r;
        if (packed) bt_group<16, 8>(PackedLower{pk}, r, tv, xq, ucs + (size_t)grp * r);
        else bt_group<16, 8>(Mf, r, g_tau, xq, ucs + (size_t)grp * r);
      }
      __syncthreads();
      if (stamp && c0 == 0) tstamp[22] = wall_clock64();
      li_rows<2>(Lc, r, g_kept, g_dsc, ucs, nc, Vout, nkeep, t + c0);
    } else {
      if (wid < nc)
        bt_group<64, kRRMax / 64>(Mf, r, g_tau, U + (size_t)(t + c0 + wid) * r, ucs + (size_t)wid * r);
      __syncthreads();
      li_rows<kRRMax / 64>(Lc, r, g_kept, g_dsc, ucs, nc, Vout, nkeep, t + c0);
    }
    __syncthreads();
  }
  if (stamp) tstamp[21] = wall_clock64();
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

// dynamic LDS of k_rr_vectors: dd, ee, kinv, red, then the slots or the
// packed reflectors with their scalars
static size_t rr_vec_lds_bytes(int nz) {
  const size_t fixed = sizeof(double) * 2 * (size_t)nz + sizeof(int) * (size_t)((nz + 3) & ~3) +
                       sizeof(double) * 32;
  const size_t slots = (size_t)rr_slots(nz) * rr_slot_bytes(nz);
  const size_t refl = nz <= kRRPackedMax ? sizeof(double2) * ((size_t)((nz + 1) & ~1) +
                                                              (size_t)nz * (nz + 1) / 2)
                                         : 0;
  const size_t ucs = sizeof(double2) * (size_t)kUc * nz;
  return fixed + std::max(slots, refl + ucs);
}

size_t rr_scratch_bytes(int nz, int nkeep) { return RRScratch::bytes(nz, nkeep); }

static void rr_set_attributes();
static void rr_finish(const double2 *A, int nz, int nkeep, double floor_val,
                      const int *forced_drop, double2 *V, double *theta, int *info, double *dinfo,
                      const RRScratch &W, hipStream_t st, long long *tstamp, const int *skip,
                      bool scale_a);

void rayleigh_ritz(const double2 *A, const double2 *S, int nz, int nkeep, double drop_tol,
                   double floor_val, const int *forced_drop, double2 *V, double *theta, int *info,
                   double *dinfo, DevBuf &scratch, hipStream_t st, long long *tstamp,
                   const int *skip) {
  DKS_REQUIRE(nz > 0 && nz <= kRRMax && nkeep > 0 && nkeep <= nz, DKS_EINVAL,
              "Rayleigh-Ritz size out of range (subspace dimension must be <= 512)");
  rr_set_attributes();
  scratch.ensure(RRScratch::bytes(nz, nkeep));
  const RRScratch W = RRScratch::at(scratch.p, nz, nkeep);
  DKS_LAUNCH("k_rr_reduce", k_rr_reduce, dim3(1), dim3(kRRThreads), rr_lds_bytes(nz), st, 0, A, S,
             nz, nkeep, drop_tol, forced_drop, info, dinfo, W, tstamp, skip);
  DKS_HIP(hipGetLastError());
  rr_finish(A, nz, nkeep, floor_val, forced_drop, V, theta, info, dinfo, W, st, tstamp, skip, false);
}

void rayleigh_ritz_s(const double2 *S, int nz, int nkeep, double drop_tol, const int *forced_drop,
                     int *info, double *dinfo, DevBuf &scratch, hipStream_t st) {
  DKS_REQUIRE(nz > 0 && nz <= kRRMax && nkeep > 0 && nkeep <= nz, DKS_EINVAL,
              "Rayleigh-Ritz size out of range (subspace dimension must be <= 512)");
  rr_set_attributes();
  scratch.ensure(RRScratch::bytes(nz, nkeep));
  const RRScratch W = RRScratch::at(scratch.p, nz, nkeep);
  DKS_LAUNCH("k_rr_reduce", k_rr_reduce, dim3(1), dim3(kRRThreads), rr_lds_bytes(nz), st, 2,
             nullptr, S, nz, nkeep, drop_tol, forced_drop, info, dinfo, W, nullptr, nullptr);
  DKS_HIP(hipGetLastError());
}

void rayleigh_ritz_a(const double2 *A, int nz, int nkeep, double floor_val, const int *forced_drop,
                     double2 *V, double *theta, int *info, double *dinfo, DevBuf &scratch,
                     hipStream_t st) {
  const RRScratch W = RRScratch::at(scratch.p, nz, nkeep);
  rr_finish(A, nz, nkeep, floor_val, forced_drop, V, theta, info, dinfo, W, st, nullptr, nullptr,
            true);
}

// kernel attributes, once per process (also when batch lanes arrive together)
static void rr_set_attributes() {
  static std::once_flag attr;
  hipError_t attr_rc = hipSuccess;
  std::call_once(attr, [&] {
    const size_t mx = std::max(rr_lds_bytes(kRRPackedMax), rr_lds_bytes(kRRMax));
    attr_rc = hipFuncSetAttribute((const void *)k_rr_reduce,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx);
    if (attr_rc == hipSuccess) {
      size_t mv = 0;
      for (int z = 1; z <= kRRMax; ++z) mv = std::max(mv, rr_vec_lds_bytes(z));
      attr_rc = hipFuncSetAttribute((const void *)k_rr_vectors<true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)mv);
      if (attr_rc == hipSuccess)
        attr_rc = hipFuncSetAttribute((const void *)k_rr_vectors<false>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)mv);
    }
  });
  DKS_HIP(attr_rc);
}

// everything after the S phase: [the scaled A,] the two products, the
// tridiagonal reduction, eigenvalues, eigenvectors
static void rr_finish(const double2 *A, int nz, int nkeep, double floor_val,
                      const int *forced_drop, double2 *V, double *theta, int *info, double *dinfo,
                      const RRScratch &W, hipStream_t st, long long *tstamp, const int *skip,
                      bool scale_a) {
  const double2 *S = nullptr;   // phase 1 reads neither input matrix
  const double drop_tol = 0.0;
  if (scale_a) {
    DKS_LAUNCH("k_rr_scale_a", k_rr_scale_a, dim3((nz + 3) / 4), dim3(256), 0, st, A, nz, info, W);
    DKS_HIP(hipGetLastError());
  }
  const unsigned tiles = (unsigned)((nz + kGT - 1) / kGT);
  for (int which = 1; which <= 2; ++which) {
    DKS_LAUNCH("k_rr_gemm", k_rr_gemm, dim3(tiles, tiles), dim3(kRRThreads), 0, st, which, nz, info, W);
    DKS_HIP(hipGetLastError());
  }
  DKS_LAUNCH("k_rr_reduce", k_rr_reduce, dim3(1), dim3(kRRThreads), rr_lds_bytes(nz), st, 1, A, S,
             nz, nkeep, drop_tol, forced_drop, info, dinfo, W, tstamp, skip);
  DKS_HIP(hipGetLastError());
  DKS_LAUNCH("k_rr_values", k_rr_values, dim3(nkeep + 1), dim3(kValThreads), 0, st, W.dd, W.ee,
             nkeep, floor_val, info, W.lam, theta, dinfo, tstamp);
  DKS_HIP(hipGetLastError());
  auto kvec = nz <= 128 ? k_rr_vectors<true> : k_rr_vectors<false>;
  DKS_LAUNCH("k_rr_vectors", kvec, dim3(nkeep), dim3(kRRThreads), rr_vec_lds_bytes(nz), st,
             W.dd, W.ee, W.tau, W.refl, W.Mm, W.Lc, W.kept, W.dsc, W.lam, info, nz, nkeep, W.U, V,
             tstamp);
  DKS_HIP(hipGetLastError());
}

}  // namespace dks
