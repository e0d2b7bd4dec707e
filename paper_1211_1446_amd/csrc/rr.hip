// Rayleigh-Ritz step of Algorithm 1 (the projected generalized eigenproblem on
// the subspace, sorted ascending) in FP64 on the device.
//
// Solves A v = theta S v for the nkeep lowest theta above `floor_val`, with
// A = Z^H H Z and S = Z^H Z of the current subspace Z = [X, Y, P], in one
// workgroup of 1024 threads:
//   1. symmetric diagonal scaling D S D, D = diag(S)^-1/2;
//   2. Cholesky D S D = L L^H, column by column; a column whose pivot falls
//      below `drop_tol` (its direction is numerically inside the span of the
//      earlier columns) is removed from the subspace instead of failing;
//   3. Li = L^-1 row by row, C = Li (D A D) Li^H with LDS-tiled products;
//   4. Householder reduction C = Q T Q^H to a real symmetric tridiagonal T,
//      on the lower triangle (packed in LDS when it fits, else in the global
//      scratch area), every matrix-vector product split over all threads;
//   5. the wanted eigenvalues of T by bisection on Sturm counts: those below
//      floor_val (the mid-gap -c^2: negative-band Ritz values) are skipped;
//   6. their eigenvectors by inverse iteration, re-orthogonalised inside
//      clusters of (nearly) equal eigenvalues such as Kramers pairs;
//   7. back-transformation v = D Li^H Q y.
#include <algorithm>
#include <cfloat>

#include "dks_internal.h"

namespace dks {

constexpr int kRRMax = 512;
constexpr int kRRThreads = 1024;
constexpr int kRRPackedMax = 120;   // r(r+1)/2 complex doubles in LDS up to this r
constexpr int kTile = 32;            // workgroup GEMM tile (kTile^2 = kRRThreads)

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

// workgroup sum of one double per thread (all threads must call)
__device__ double wg_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

// row i of the lower-triangle index e (e = i (i + 1) / 2 + j, j <= i)
__device__ __forceinline__ int tri_row(int e) {
  int i = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > e) --i;
  while ((i + 1) * (i + 2) / 2 <= e) ++i;
  return i;
}

// C(i, j) = sum_k A(i, k) B(k, j) for i < M, j < N, k < K, tiled through LDS.
// ta, tb: kTile x kTile LDS tiles.  All threads must call.
template <typename FA, typename FB, typename FC>
__device__ void wg_gemm(int M, int N, int K, FA A, FB B, FC Cst, double2 *ta, double2 *tb) {
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
  for (int i0 = 0; i0 < M; i0 += kTile)
    for (int j0 = 0; j0 < N; j0 += kTile) {
      double2 acc = make_double2(0, 0);
      for (int k0 = 0; k0 < K; k0 += kTile) {
        {
          const int i = i0 + ty, k = k0 + tx;
          ta[ty * kTile + tx] = (i < M && k < K) ? A(i, k) : make_double2(0, 0);
          const int kk = k0 + ty, j = j0 + tx;
          tb[ty * kTile + tx] = (kk < K && j < N) ? B(kk, j) : make_double2(0, 0);
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < kTile; ++kk) acc = zadd(acc, zmul(ta[ty * kTile + kk], tb[kk * kTile + tx]));
        __syncthreads();
      }
      const int i = i0 + ty, j = j0 + tx;
      if (i < M && j < N) Cst(i, j, acc);
    }
}

// Lower triangle of a Hermitian matrix: packed rows in LDS, or full rows in global.
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

struct TriOut {
  double *dd, *ee;      // diagonal (r), off-diagonal (r-1)
  double2 *tauv;        // reflector scalars (r-1)
  double2 *vv, *wv;     // work vectors (r)
  double2 *part;        // kRRThreads partial sums
  double *red;
};

// Householder tridiagonalisation of the r x r Hermitian matrix held in M's lower
// triangle.  Reflector k (H_k = I - tau_k v v^H, v = [1, M(k+2.., k)]) acts on
// rows k+1..r-1; the column below the subdiagonal keeps v for the
// back-transformation.
template <typename Mat>
__device__ void tridiagonalise(const Mat M, int r, TriOut o) {
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double2 s_tau, s_scal, s_alpha;
  for (int k = 0; k + 1 < r; ++k) {
    const int m = r - k - 1;   // trailing size, rows/cols k+1..r-1
    double xn2 = 0;
    for (int i = k + 2 + tid; i < r; i += nt) {
      double2 v = M.lo(i, k);
      xn2 += v.x * v.x + v.y * v.y;
    }
    xn2 = wg_sum(xn2, o.red);
    if (tid == 0) {
      double2 alpha = M.lo(k + 1, k);
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
      s_tau = tau;
      s_scal = scal;
      o.tauv[k] = tau;
      o.ee[k] = beta;
      o.dd[k] = M.lo(k, k).x;
    }
    __syncthreads();
    const double2 tau = s_tau, scal = s_scal;
    if (tau.x == 0.0 && tau.y == 0.0) continue;   // uniform across the workgroup
    // v (length m): v[0] = 1, v[i] = M(k+1+i, k) * scal
    for (int i = tid; i < m; i += nt) {
      double2 v = (i == 0) ? make_double2(1, 0) : zmul(M.lo(k + 1 + i, k), scal);
      o.vv[i] = v;
      if (i > 0) M.set(k + 1 + i, k, v);
    }
    __syncthreads();
    // x = tau C22 v with C22 Hermitian from its lower triangle; P parts per row
    const int P = max(1, min(nt / max(m, 1), 16));
    for (int t = tid; t < m * P; t += nt) {
      const int i = t % m, p = t / m;
      const int j0 = (m * p) / P, j1 = (m * (p + 1)) / P;
      double2 s = make_double2(0, 0);
      const int gi = k + 1 + i;
      for (int j = j0; j < j1; ++j) {
        const int gj = k + 1 + j;
        double2 c = (j <= i) ? M.lo(gi, gj) : zconj(M.lo(gj, gi));
        s = zadd(s, zmul(c, o.vv[j]));
      }
      o.part[p * m + i] = s;
    }
    __syncthreads();
    double pr = 0, pi = 0;
    for (int i = tid; i < m; i += nt) {
      double2 s = make_double2(0, 0);
      for (int p = 0; p < P; ++p) s = zadd(s, o.part[p * m + i]);
      s = zmul(tau, s);
      o.wv[i] = s;
      double2 t2 = zcmul(s, o.vv[i]);   // conj(x_i) v_i
      pr += t2.x;
      pi += t2.y;
    }
    pr = wg_sum(pr, o.red);
    pi = wg_sum(pi, o.red);
    if (tid == 0) {
      double2 t2 = zmul(tau, make_double2(pr, pi));
      s_alpha = make_double2(-0.5 * t2.x, -0.5 * t2.y);
    }
    __syncthreads();
    const double2 al = s_alpha;
    for (int i = tid; i < m; i += nt) o.wv[i] = zadd(o.wv[i], zmul(al, o.vv[i]));
    __syncthreads();
    // C22 -= v w^H + w v^H on the lower triangle
    const int tri = m * (m + 1) / 2;
    for (int e = tid; e < tri; e += nt) {
      const int i = tri_row(e);
      const int j = e - i * (i + 1) / 2;
      const double2 t1 = zmul(o.vv[i], zconj(o.wv[j]));
      const double2 t2 = zmul(o.wv[i], zconj(o.vv[j]));
      double2 c = M.lo(k + 1 + i, k + 1 + j);
      c = zsub(c, zadd(t1, t2));
      if (i == j) c.y = 0.0;
      M.set(k + 1 + i, k + 1 + j, c);
    }
    __syncthreads();
  }
  if (tid == 0) o.dd[r - 1] = M.lo(r - 1, r - 1).x;
  __syncthreads();
}

// Uc = Q Uc with Q = H_0 H_1 ... H_{r-2} (reflectors stored in M), Uc r x nk
template <typename Mat>
__device__ void back_transform(const Mat M, int r, int nk, const double2 *tauv, double2 *Uc,
                               double2 *part, double2 *sv) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = r - 2; k >= 0; --k) {
    const double2 tau = tauv[k];
    if (tau.x == 0.0 && tau.y == 0.0) continue;
    const int m = r - k - 1;
    const int P = max(1, min(nt / max(nk, 1), 32));
    // s_j = v^H u_j over rows k+1.. in P parts
    for (int t = tid; t < nk * P; t += nt) {
      const int j = t % nk, p = t / nk;
      const int i0 = (m * p) / P, i1 = (m * (p + 1)) / P;
      double2 s = make_double2(0, 0);
      for (int i = i0; i < i1; ++i) {
        double2 v = (i == 0) ? make_double2(1, 0) : M.lo(k + 1 + i, k);
        s = zadd(s, zcmul(v, Uc[(size_t)(k + 1 + i) * nk + j]));
      }
      part[p * nk + j] = s;
    }
    __syncthreads();
    for (int j = tid; j < nk; j += nt) {
      double2 s = make_double2(0, 0);
      for (int p = 0; p < P; ++p) s = zadd(s, part[p * nk + j]);
      sv[j] = zmul(tau, s);
    }
    __syncthreads();
    for (int e = tid; e < m * nk; e += nt) {
      const int i = e / nk, j = e - (e / nk) * nk;
      double2 v = (i == 0) ? make_double2(1, 0) : M.lo(k + 1 + i, k);
      double2 *u = Uc + (size_t)(k + 1 + i) * nk + j;
      *u = zsub(*u, zmul(v, sv[j]));
    }
    __syncthreads();
  }
}

__device__ int sturm_count(const double *d, const double *e2, int r, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0) ++cnt;
  for (int i = 1; i < r; ++i) {
    if (fabs(q) < pivmin) q = -pivmin;
    q = (d[i] - x) - e2[i - 1] / q;
    if (q < 0) ++cnt;
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

__global__ void __launch_bounds__(kRRThreads) k_rayleigh_ritz(
    const double2 *__restrict__ Ain, const double2 *__restrict__ Sin, int nz, int nkeep,
    double drop_tol, double floor_val, const int *__restrict__ forced, double2 *__restrict__ Vout,
    double *__restrict__ theta, int *__restrict__ info, double *__restrict__ dinfo,
    double2 *__restrict__ ws, long long *__restrict__ tstamp) {
  extern __shared__ unsigned char smem_raw[];
  // optional phase timestamps (constant-rate wall clock), for tuning
#define DKS_RR_STAMP(k) \
  do {                  \
    if (tstamp && threadIdx.x == 0) tstamp[k] = wall_clock64(); \
  } while (0)
  DKS_RR_STAMP(0);
  // ---- LDS arena (sized by nz): partial sums, per-index arrays, then the
  // packed matrix or the GEMM tiles
  const int na = (nz + 1) & ~1;
  double2 *part = reinterpret_cast<double2 *>(smem_raw);   // kRRThreads
  double2 *tauv = part + kRRThreads;
  double2 *vv = tauv + na;
  double2 *wv = vv + na;
  double *dsc = reinterpret_cast<double *>(wv + na);
  double *dd = dsc + na;
  double *ee = dd + na;
  double *e2 = ee + na;
  double *lam = e2 + na;
  double *red = lam + na;                                  // 32
  int *kept = reinterpret_cast<int *>(red + 32);
  double2 *big = reinterpret_cast<double2 *>(kept + na);  // packed matrix or GEMM tiles
  double2 *ta = big, *tb = big + kTile * kTile;
  __shared__ int s_r, s_flag, s_k0;
  __shared__ double s_ljj, s_lmin;

  const int tid = threadIdx.x, nt = blockDim.x;
  const size_t nn = (size_t)nz * nz;
  double2 *Sm = ws;              // scaled S, Cholesky factor in its lower triangle
  double2 *Am = Sm + nn;         // scaled A
  double2 *Lc = Am + nn;         // L^-1 column-major: Lc[c r + b] = Li[b][c]
  double2 *Mm = Lc + nn;         // A_r Li^H
  double2 *Cg = Mm + nn;         // C
  double2 *Uc = Cg + nn;         // r x nkeep complex eigenvectors
  double *U = reinterpret_cast<double *>(Uc + (size_t)nz * nkeep);   // r x nkeep real
  double *lu = U + (size_t)nz * nkeep;                                // 5 r per cluster leader

  // ---- 1. scaling and Hermitian parts
  for (int i = tid; i < nz; i += nt) {
    double s = Sin[(size_t)i * nz + i].x;
    bool f = forced ? (forced[i] != 0) : false;
    dsc[i] = (!f && s > 0 && isfinite(s)) ? 1.0 / sqrt(s) : 0.0;
  }
  __syncthreads();
  for (size_t e = tid; e < nn; e += nt) {
    int i = (int)(e / nz), j = (int)(e - (e / nz) * nz);
    double f = dsc[i] * dsc[j];
    double2 s1 = Sin[e], s2 = Sin[(size_t)j * nz + i];
    double2 a1 = Ain[e], a2 = Ain[(size_t)j * nz + i];
    Sm[e] = make_double2(0.5 * f * (s1.x + s2.x), 0.5 * f * (s1.y - s2.y));
    Am[e] = make_double2(0.5 * f * (a1.x + a2.x), 0.5 * f * (a1.y - a2.y));
  }
  __syncthreads();

  // ---- 2. Cholesky with column dropping (lower triangle of Sm)
  DKS_RR_STAMP(1);
  for (int j = 0; j < nz; ++j) {
    if (tid == 0) {
      double piv = Sm[(size_t)j * nz + j].x;
      bool drop = (dsc[j] == 0.0) || !(piv > drop_tol);
      s_ljj = drop ? 0.0 : sqrt(piv);
      kept[j] = drop ? 0 : 1;
      Sm[(size_t)j * nz + j] = make_double2(s_ljj, 0.0);
    }
    __syncthreads();
    const double ljj = s_ljj;
    if (ljj > 0.0) {
      const double inv = 1.0 / ljj;
      for (int i = j + 1 + tid; i < nz; i += nt) Sm[(size_t)i * nz + j] = zscale(Sm[(size_t)i * nz + j], inv);
      __syncthreads();
      const int w = nz - j - 1;
      const int tri = w * (w + 1) / 2;
      for (int e = tid; e < tri; e += nt) {
        const int i = tri_row(e);
        const int k = e - i * (i + 1) / 2;   // k <= i
        const int gi = j + 1 + i, gk = j + 1 + k;
        double2 li = Sm[(size_t)gi * nz + j], lk = Sm[(size_t)gk * nz + j];
        double2 s = Sm[(size_t)gi * nz + gk];
        s.x -= li.x * lk.x + li.y * lk.y;
        s.y -= li.y * lk.x - li.x * lk.y;
        Sm[(size_t)gi * nz + gk] = s;
      }
      __syncthreads();
    } else {
      for (int i = j + 1 + tid; i < nz; i += nt) Sm[(size_t)i * nz + j] = make_double2(0, 0);
      __syncthreads();
    }
  }
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

  // ---- 3. Li = L^-1 row by row (column-major Lc), then C = Li A_r Li^H
  DKS_RR_STAMP(2);
  for (int a = 0; a < r; ++a) {
    const int ka = kept[a];
    const double inv_aa = 1.0 / Sm[(size_t)ka * nz + ka].x;
    const int P = max(1, min(nt / max(a, 1), 16));
    for (int t = tid; t < a * P; t += nt) {
      const int b = t % a, p = t / a;
      const int len = a - b;
      const int c0 = b + (len * p) / P, c1 = b + (len * (p + 1)) / P;
      double2 s = make_double2(0, 0);
      for (int c = c0; c < c1; ++c) s = zadd(s, zmul(Sm[(size_t)ka * nz + kept[c]], Lc[(size_t)b * r + c]));
      part[p * a + b] = s;
    }
    __syncthreads();
    for (int b = tid; b <= a; b += nt) {
      if (b == a) {
        Lc[(size_t)a * r + a] = make_double2(inv_aa, 0.0);
      } else {
        double2 s = make_double2(0, 0);
        for (int p = 0; p < P; ++p) s = zadd(s, part[p * a + b]);
        Lc[(size_t)b * r + a] = zscale(s, -inv_aa);
      }
    }
    for (int b = a + 1 + tid; b < r; b += nt) Lc[(size_t)b * r + a] = make_double2(0, 0);
    __syncthreads();
  }
  // Mm[a][b] = sum_c A[ka][kc] conj(Li[b][c])
  DKS_RR_STAMP(3);
  wg_gemm(
      r, r, r, [&](int i, int k) { return Am[(size_t)kept[i] * nz + kept[k]]; },
      [&](int k, int j) { return zconj(Lc[(size_t)k * r + j]); },
      [&](int i, int j, double2 v) { Mm[(size_t)i * r + j] = v; }, ta, tb);
  __syncthreads();
  // Cg[a][b] = sum_c Li[a][c] Mm[c][b]
  wg_gemm(
      r, r, r, [&](int i, int k) { return Lc[(size_t)k * r + i]; },
      [&](int k, int j) { return Mm[(size_t)k * r + j]; },
      [&](int i, int j, double2 v) { Cg[(size_t)i * r + j] = v; }, ta, tb);
  __syncthreads();
  const bool packed = (nz <= kRRPackedMax);   // the arena holds the packed triangle
  const PackedLower PL{big};
  const FullLower FL{Mm, r};   // Mm is free again: hold the lower triangle there
  {
    const int tri = r * (r + 1) / 2;
    for (int e = tid; e < tri; e += nt) {
      const int i = tri_row(e);
      const int j = e - i * (i + 1) / 2;
      double2 x = Cg[(size_t)i * r + j], y = Cg[(size_t)j * r + i];
      double2 h = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
      if (i == j) h.y = 0.0;
      if (packed) PL.set(i, j, h); else FL.set(i, j, h);
    }
  }
  __syncthreads();

  // ---- 4. tridiagonalisation
  DKS_RR_STAMP(4);
  TriOut to{dd, ee, tauv, vv, wv, part, red};
  if (packed) tridiagonalise(PL, r, to); else tridiagonalise(FL, r, to);
  for (int i = tid; i + 1 < r; i += nt) e2[i] = ee[i] * ee[i];
  __syncthreads();

  // ---- 5. bisection (every thread computes the Gershgorin bounds itself)
  DKS_RR_STAMP(5);
  double glo = 1e300, ghi = -1e300, emax2 = 0;
  for (int i = 0; i < r; ++i) {
    double off = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < r ? fabs(ee[i]) : 0.0);
    glo = fmin(glo, dd[i] - off);
    ghi = fmax(ghi, dd[i] + off);
    if (i + 1 < r) emax2 = fmax(emax2, e2[i]);
  }
  const double tnorm = fmax(fabs(glo), fabs(ghi));
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  glo -= 2.0 * DBL_EPSILON * tnorm + 2 * pivmin;
  ghi += 2.0 * DBL_EPSILON * tnorm + 2 * pivmin;
  if (tid == 0) {
    int k0 = (floor_val > glo) ? sturm_count(dd, e2, r, floor_val, pivmin) : 0;
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
  for (int t = tid; t <= nkeep; t += nt) {
    // t < nkeep: kept eigenvalue k0 + t; t == nkeep: the smallest, for monitoring
    const int idx = (t < nkeep) ? k0 + t : 0;
    double lo = glo, hi = ghi;
    for (int it = 0; it < 200; ++it) {
      double mid = 0.5 * (lo + hi);
      if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
      if (mid <= lo || mid >= hi) break;
      if (sturm_count(dd, e2, r, mid, pivmin) <= idx) lo = mid; else hi = mid;
    }
    if (t < nkeep) lam[t] = 0.5 * (lo + hi); else s_lmin = 0.5 * (lo + hi);
  }
  __syncthreads();

  // ---- 6. inverse iteration, clusters handled by one thread each
  DKS_RR_STAMP(6);
  const double ctol = 1e-7 * fmax(tnorm, 1e-300);
  const double eps_t = DBL_EPSILON * fmax(tnorm, 1e-300);
  for (int t = tid; t < nkeep; t += nt) {
    if (t > 0 && lam[t] - lam[t - 1] <= ctol) continue;   // not a cluster leader
    int tend = t + 1;
    while (tend < nkeep && lam[tend] - lam[tend - 1] <= ctol) ++tend;
    double *u0 = lu + (size_t)t * 5 * r;
    double *u1 = u0 + r, *u2 = u1 + r, *ml = u2 + r, *pv = ml + r;
    for (int jv = t; jv < tend; ++jv) {
      const double lm = lam[jv] + (double)(jv - t) * 10.0 * eps_t;
      // LU with partial pivoting of T - lm I
      double a = dd[0] - lm, bsup = (r > 1) ? ee[0] : 0.0;
      for (int i = 0; i + 1 < r; ++i) {
        const double c = ee[i];
        const double dn = dd[i + 1] - lm;
        const double en = (i + 2 < r) ? ee[i + 1] : 0.0;
        if (fabs(a) >= fabs(c)) {
          double mm = (a != 0.0) ? c / a : 0.0;
          u0[i] = a; u1[i] = bsup; u2[i] = 0.0; pv[i] = 0.0; ml[i] = mm;
          a = dn - mm * bsup;
          bsup = en;
        } else {
          double mm = a / c;
          u0[i] = c; u1[i] = dn; u2[i] = en; pv[i] = 1.0; ml[i] = mm;
          a = bsup - mm * dn;
          bsup = -mm * en;
        }
      }
      u0[r - 1] = a;
      for (int i = 0; i < r; ++i)
        if (fabs(u0[i]) < eps_t) u0[i] = (u0[i] < 0) ? -eps_t : eps_t;
      for (int i = 0; i < r; ++i) U[(size_t)i * nkeep + jv] = start_entry(i, jv);
      for (int iter = 0; iter < 4; ++iter) {
        for (int i = 0; i + 1 < r; ++i) {
          double bi = U[(size_t)i * nkeep + jv], bn = U[(size_t)(i + 1) * nkeep + jv];
          if (pv[i] != 0.0) { double tt = bi; bi = bn; bn = tt; }
          bn -= ml[i] * bi;
          U[(size_t)i * nkeep + jv] = bi;
          U[(size_t)(i + 1) * nkeep + jv] = bn;
        }
        for (int i = r - 1; i >= 0; --i) {
          double s = U[(size_t)i * nkeep + jv];
          if (i + 1 < r) s -= u1[i] * U[(size_t)(i + 1) * nkeep + jv];
          if (i + 2 < r) s -= u2[i] * U[(size_t)(i + 2) * nkeep + jv];
          U[(size_t)i * nkeep + jv] = s / u0[i];
        }
        for (int pass = 0; pass < 2; ++pass)
          for (int jp = t; jp < jv; ++jp) {
            double dot = 0;
            for (int i = 0; i < r; ++i) dot += U[(size_t)i * nkeep + jp] * U[(size_t)i * nkeep + jv];
            for (int i = 0; i < r; ++i) U[(size_t)i * nkeep + jv] -= dot * U[(size_t)i * nkeep + jp];
          }
        double nrm = 0;
        for (int i = 0; i < r; ++i) nrm += U[(size_t)i * nkeep + jv] * U[(size_t)i * nkeep + jv];
        const double inv = 1.0 / sqrt(nrm);
        for (int i = 0; i < r; ++i) U[(size_t)i * nkeep + jv] *= inv;
      }
    }
  }
  __syncthreads();

  // ---- 7. back-transformation: Uc = Q U, then V = D Li^H Uc
  DKS_RR_STAMP(7);
  for (int e = tid; e < r * nkeep; e += nt) Uc[e] = make_double2(U[e], 0.0);
  __syncthreads();
  if (packed) back_transform(PL, r, nkeep, tauv, Uc, part, vv);
  else back_transform(FL, r, nkeep, tauv, Uc, part, vv);
  for (int e = tid; e < nz * nkeep; e += nt) Vout[e] = make_double2(0, 0);
  __syncthreads();
  wg_gemm(
      r, nkeep, r, [&](int i, int k) { return zconj(Lc[(size_t)i * r + k]); },
      [&](int k, int j) { return Uc[(size_t)k * nkeep + j]; },
      [&](int i, int j, double2 v) {
        const int ki = kept[i];
        Vout[(size_t)ki * nkeep + j] = zscale(v, dsc[ki]);
      },
      ta, tb);
  for (int t = tid; t < nkeep; t += nt) theta[t] = lam[t];
  if (tid == 0) dinfo[0] = s_lmin;
  __syncthreads();
  DKS_RR_STAMP(8);
#undef DKS_RR_STAMP
}

// dynamic LDS of one launch with subspace dimension nz (layout of the kernel's arena)
static size_t rr_lds_bytes(int nz) {
  const size_t na = (size_t)((nz + 1) & ~1);
  const size_t arrays = sizeof(double2) * (kRRThreads + 3 * na) + sizeof(double) * (6 * na + 32) +
                        sizeof(int) * na;
  const size_t packed =
      nz <= kRRPackedMax ? sizeof(double2) * (size_t)nz * (nz + 1) / 2 : 0;
  const size_t tiles = sizeof(double2) * 2 * kTile * kTile;
  return ((arrays + 15) & ~(size_t)15) + (packed > tiles ? packed : tiles);
}

void rayleigh_ritz(const double2 *A, const double2 *S, int nz, int nkeep, double drop_tol,
                   double floor_val, const int *forced_drop, double2 *V, double *theta, int *info,
                   double *dinfo, DevBuf &scratch, hipStream_t st, long long *tstamp) {
  DKS_REQUIRE(nz > 0 && nz <= kRRMax && nkeep > 0 && nkeep <= nz, DKS_EINVAL,
              "Rayleigh-Ritz size out of range (subspace dimension must be <= 512)");
  static bool attr = false;
  if (!attr) {
    const size_t mx = std::max(rr_lds_bytes(kRRPackedMax), rr_lds_bytes(kRRMax));
    DKS_HIP(hipFuncSetAttribute((const void *)k_rayleigh_ritz,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx));
    attr = true;
  }
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
