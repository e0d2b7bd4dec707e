// Rayleigh-Ritz step of Algorithm 1 (lines 4 and 12-14) in FP64 on the device.
//
// Solves A v = theta S v for the nkeep smallest theta, with A = Z^H H Z and
// S = Z^H Z of the current subspace Z = [X, Y, P], in one workgroup:
//   1. symmetric diagonal scaling D S D, D = diag(S)^-1/2;
//   2. Cholesky D S D = L L^H, column by column; a column whose pivot falls
//      below `drop_tol` (its direction is numerically inside the span of the
//      earlier columns) is removed from the subspace instead of failing;
//   3. C = L^-1 (D A D) L^-H on the kept columns;
//   4. Householder reduction C = Q T Q^H to a real symmetric tridiagonal T;
//   5. the nkeep smallest eigenvalues of T above `floor_val` by bisection on
//      Sturm counts (floor_val = -c^2 discards Ritz values that belong to the
//      negative band; -inf keeps the plain lowest nkeep);
//   6. their eigenvectors by inverse iteration, re-orthogonalised inside
//      clusters of (nearly) equal eigenvalues such as Kramers pairs;
//   7. back-transformation v = D L^-H Q y.
// Matrices live in a global scratch area (they exceed the LDS for nz > ~120).
#include <cfloat>

#include "dks_internal.h"

namespace dks {

constexpr int kRRMax = 512;
constexpr int kRRThreads = 1024;

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
    double2 *__restrict__ ws) {
  __shared__ double dsc[kRRMax];
  __shared__ int kept[kRRMax];
  __shared__ double dd[kRRMax], ee[kRRMax], e2[kRRMax], lam[kRRMax];
  __shared__ double2 tauv[kRRMax], vv[kRRMax], wv[kRRMax];
  __shared__ double red[32];
  __shared__ int s_r, s_flag, s_k0;
  __shared__ double s_lmin;
  __shared__ double s_ljj;
  __shared__ double2 s_tau, s_alpha2;

  const int tid = threadIdx.x, nt = blockDim.x;
  const size_t nn = (size_t)nz * nz;
  double2 *Sm = ws;
  double2 *Am = Sm + nn;
  double2 *Li = Am + nn;
  double2 *Mm = Li + nn;
  double2 *Cm = Mm + nn;
  double2 *Uc = Cm + nn;                       // r x nkeep
  double *U = reinterpret_cast<double *>(Uc + (size_t)nz * nkeep);   // r x nkeep
  double *lu = U + (size_t)nz * nkeep;          // 5 r per cluster leader

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
      for (int i = j + 1 + tid; i < nz; i += nt) {
        double2 v = Sm[(size_t)i * nz + j];
        Sm[(size_t)i * nz + j] = make_double2(v.x * inv, v.y * inv);
      }
      __syncthreads();
      const int w = nz - j - 1;
      for (int e = tid; e < w * w; e += nt) {
        int i = j + 1 + e / w, k = j + 1 + (e - (e / w) * w);
        if (k > i) continue;
        double2 li = Sm[(size_t)i * nz + j], lk = Sm[(size_t)k * nz + j];
        double2 s = Sm[(size_t)i * nz + k];
        // s -= li conj(lk)
        s.x -= li.x * lk.x + li.y * lk.y;
        s.y -= li.y * lk.x - li.x * lk.y;
        Sm[(size_t)i * nz + k] = s;
      }
      __syncthreads();
    } else {
      for (int i = j + 1 + tid; i < nz; i += nt) Sm[(size_t)i * nz + j] = make_double2(0, 0);
      __syncthreads();
    }
  }
  // kept list
  if (tid == 0) {
    int r = 0;
    for (int j = 0; j < nz; ++j)
      if (kept[j]) kept[r++] = j;
    s_r = r;
    s_flag = (r < nkeep) ? 1 : 0;
    info[0] = r;
    info[1] = s_flag;
    info[2] = nz - r;
  }
  __syncthreads();
  const int r = s_r;
  if (s_flag) return;

  // ---- 3. Li = L^-1 (r x r lower), C = Li A_r Li^H
  for (int b = tid; b < r; b += nt) {
    const int kb = kept[b];
    Li[(size_t)b * r + b] = make_double2(1.0 / Sm[(size_t)kb * nz + kb].x, 0.0);
    for (int a = b + 1; a < r; ++a) {
      const int ka = kept[a];
      double2 s = make_double2(0, 0);
      for (int c = b; c < a; ++c) s = zadd(s, zmul(Sm[(size_t)ka * nz + kept[c]], Li[(size_t)c * r + b]));
      double inv = 1.0 / Sm[(size_t)ka * nz + ka].x;
      Li[(size_t)a * r + b] = make_double2(-s.x * inv, -s.y * inv);
    }
    for (int a = 0; a < b; ++a) Li[(size_t)a * r + b] = make_double2(0, 0);
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    int a = e / r, b = e - (e / r) * r;
    const int ka = kept[a];
    double2 s = make_double2(0, 0);
    for (int c = 0; c <= b; ++c) s = zadd(s, zmul(Am[(size_t)ka * nz + kept[c]], zconj(Li[(size_t)b * r + c])));
    Mm[(size_t)a * r + b] = s;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    int a = e / r, b = e - (e / r) * r;
    double2 s = make_double2(0, 0);
    for (int c = 0; c <= a; ++c) s = zadd(s, zmul(Li[(size_t)a * r + c], Mm[(size_t)c * r + b]));
    Cm[(size_t)a * r + b] = s;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    int a = e / r, b = e - (e / r) * r;
    if (a > b) continue;
    double2 x = Cm[(size_t)a * r + b], y = Cm[(size_t)b * r + a];
    double2 h = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    if (a == b) h.y = 0.0;
    Cm[(size_t)a * r + b] = h;
    Cm[(size_t)b * r + a] = zconj(h);
  }
  __syncthreads();

  // ---- 4. Householder tridiagonalisation (lower), C = Q T Q^H
  for (int k = 0; k + 1 < r; ++k) {
    const int m = r - k - 1;   // trailing size
    double xn2 = 0;
    for (int i = k + 2 + tid; i < r; i += nt) {
      double2 v = Cm[(size_t)i * r + k];
      xn2 += v.x * v.x + v.y * v.y;
    }
    xn2 = wg_sum(xn2, red);
    if (tid == 0) {
      double2 alpha = Cm[(size_t)(k + 1) * r + k];
      double2 tau = make_double2(0, 0);
      double beta = alpha.x;
      double2 scal = make_double2(0, 0);
      if (!(xn2 == 0.0 && alpha.y == 0.0)) {
        double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
        beta = (alpha.x >= 0) ? -nrm : nrm;
        tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
        double2 den = make_double2(alpha.x - beta, alpha.y);
        double dn = den.x * den.x + den.y * den.y;
        scal = make_double2(den.x / dn, -den.y / dn);
      }
      s_tau = tau;
      tauv[k] = tau;
      ee[k] = beta;
      dd[k] = Cm[(size_t)k * r + k].x;
      vv[0] = make_double2(1, 0);
      wv[0] = scal;   // stash
    }
    __syncthreads();
    const double2 tau = s_tau;
    const double2 scal = wv[0];
    __syncthreads();
    if (tau.x != 0.0 || tau.y != 0.0) {
      for (int i = 1 + tid; i < m; i += nt) {
        double2 v = zmul(Cm[(size_t)(k + 1 + i) * r + k], scal);
        vv[i] = v;
        Cm[(size_t)(k + 1 + i) * r + k] = v;   // keep v for the back-transformation
      }
      __syncthreads();
      // x = tau C22 v
      for (int i = tid; i < m; i += nt) {
        const double2 *row = Cm + (size_t)(k + 1 + i) * r + (k + 1);
        double2 s = make_double2(0, 0);
        for (int j = 0; j < m; ++j) s = zadd(s, zmul(row[j], vv[j]));
        wv[i] = zmul(tau, s);
      }
      __syncthreads();
      double pr = 0, pi = 0;
      for (int i = tid; i < m; i += nt) {
        double2 t = zcmul(wv[i], vv[i]);   // conj(x_i) v_i
        pr += t.x;
        pi += t.y;
      }
      pr = wg_sum(pr, red);
      pi = wg_sum(pi, red);
      if (tid == 0) {
        double2 t = zmul(tau, make_double2(pr, pi));
        s_alpha2 = make_double2(-0.5 * t.x, -0.5 * t.y);
      }
      __syncthreads();
      const double2 al = s_alpha2;
      for (int i = tid; i < m; i += nt) wv[i] = zadd(wv[i], zmul(al, vv[i]));
      __syncthreads();
      for (int e = tid; e < m * m; e += nt) {
        int i = e / m, j = e - (e / m) * m;
        double2 *c = Cm + (size_t)(k + 1 + i) * r + (k + 1 + j);
        // c -= v_i conj(w_j) + w_i conj(v_j)
        double2 t1 = zmul(vv[i], zconj(wv[j]));
        double2 t2 = zmul(wv[i], zconj(vv[j]));
        *c = zsub(*c, zadd(t1, t2));
      }
      __syncthreads();
    }
  }
  if (tid == 0) dd[r - 1] = Cm[(size_t)(r - 1) * r + (r - 1)].x;
  __syncthreads();
  for (int i = tid; i + 1 < r; i += nt) e2[i] = ee[i] * ee[i];
  __syncthreads();

  // ---- 5. bisection for the nkeep smallest eigenvalues
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
  // Ritz values below floor_val (the mid-gap -c^2) belong to the negative band;
  // the kept pairs are the nkeep lowest above it.
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
    // t < nkeep: kept eigenvalue k0 + t; t == nkeep: the smallest (index 0), for monitoring
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
      // start vector
      double *x = U + (size_t)0;   // placeholder to keep types simple
      (void)x;
      double nrm = 0;
      for (int i = 0; i < r; ++i) {
        double v = start_entry(i, jv);
        U[(size_t)i * nkeep + jv] = v;
        nrm += v * v;
      }
      for (int iter = 0; iter < 4; ++iter) {
        // forward (row swaps + elimination)
        for (int i = 0; i + 1 < r; ++i) {
          double bi = U[(size_t)i * nkeep + jv], bn = U[(size_t)(i + 1) * nkeep + jv];
          if (pv[i] != 0.0) { double tt = bi; bi = bn; bn = tt; }
          bn -= ml[i] * bi;
          U[(size_t)i * nkeep + jv] = bi;
          U[(size_t)(i + 1) * nkeep + jv] = bn;
        }
        // back substitution
        for (int i = r - 1; i >= 0; --i) {
          double s = U[(size_t)i * nkeep + jv];
          if (i + 1 < r) s -= u1[i] * U[(size_t)(i + 1) * nkeep + jv];
          if (i + 2 < r) s -= u2[i] * U[(size_t)(i + 2) * nkeep + jv];
          U[(size_t)i * nkeep + jv] = s / u0[i];
        }
        // orthogonalise against earlier members of the cluster (twice)
        for (int pass = 0; pass < 2; ++pass)
          for (int jp = t; jp < jv; ++jp) {
            double dot = 0;
            for (int i = 0; i < r; ++i) dot += U[(size_t)i * nkeep + jp] * U[(size_t)i * nkeep + jv];
            for (int i = 0; i < r; ++i) U[(size_t)i * nkeep + jv] -= dot * U[(size_t)i * nkeep + jp];
          }
        nrm = 0;
        for (int i = 0; i < r; ++i) nrm += U[(size_t)i * nkeep + jv] * U[(size_t)i * nkeep + jv];
        double inv = 1.0 / sqrt(nrm);
        for (int i = 0; i < r; ++i) U[(size_t)i * nkeep + jv] *= inv;
      }
    }
  }
  __syncthreads();

  // ---- 7. back-transformation: Uc = Q U, then V = D L^-H Uc
  for (int e = tid; e < r * nkeep; e += nt) Uc[e] = make_double2(U[e], 0.0);
  __syncthreads();
  for (int j = tid; j < nkeep; j += nt) {
    for (int k = r - 2; k >= 0; --k) {
      const double2 tau = tauv[k];
      if (tau.x == 0.0 && tau.y == 0.0) continue;
      // v = [1, Cm[k+2.., k]] on rows k+1..r-1
      double2 s = Uc[(size_t)(k + 1) * nkeep + j];
      for (int i = k + 2; i < r; ++i) s = zadd(s, zcmul(Cm[(size_t)i * r + k], Uc[(size_t)i * nkeep + j]));
      double2 ts = zmul(tau, s);
      Uc[(size_t)(k + 1) * nkeep + j] = zsub(Uc[(size_t)(k + 1) * nkeep + j], ts);
      for (int i = k + 2; i < r; ++i)
        Uc[(size_t)i * nkeep + j] = zsub(Uc[(size_t)i * nkeep + j], zmul(Cm[(size_t)i * r + k], ts));
    }
  }
  __syncthreads();
  for (int e = tid; e < nz * nkeep; e += nt) {
    int i = e / nkeep, j = e - (e / nkeep) * nkeep;
    Vout[e] = make_double2(0, 0);
    (void)i;
    (void)j;
  }
  __syncthreads();
  for (int e = tid; e < r * nkeep; e += nt) {
    int b = e / nkeep, j = e - (e / nkeep) * nkeep;
    double2 s = make_double2(0, 0);
    for (int a = b; a < r; ++a) s = zadd(s, zcmul(Li[(size_t)a * r + b], Uc[(size_t)a * nkeep + j]));
    const int kb = kept[b];
    const double f = dsc[kb];
    Vout[(size_t)kb * nkeep + j] = make_double2(f * s.x, f * s.y);
  }
  for (int t = tid; t < nkeep; t += nt) theta[t] = lam[t];
  if (tid == 0) dinfo[0] = s_lmin;
}

void rayleigh_ritz(const double2 *A, const double2 *S, int nz, int nkeep, double drop_tol,
                   double floor_val, const int *forced_drop, double2 *V, double *theta, int *info, double *dinfo,
                   DevBuf &scratch, hipStream_t st) {
  DKS_REQUIRE(nz > 0 && nz <= kRRMax && nkeep > 0 && nkeep <= nz, DKS_EINVAL,
              "Rayleigh-Ritz size out of range (subspace dimension must be <= 512)");
  size_t nn = (size_t)nz * nz;
  size_t bytes = sizeof(double2) * (5 * nn + (size_t)nz * nkeep) + sizeof(double) * (size_t)nz * nkeep +
                 sizeof(double) * 5 * (size_t)nz * nkeep;
  scratch.ensure(bytes);
  DKS_LAUNCH("k_rayleigh_ritz", k_rayleigh_ritz, dim3(1), dim3(kRRThreads), 0, st, A, S, nz, nkeep, drop_tol,
                     floor_val, forced_drop, V, theta, info, dinfo, scratch.as<double2>());
  DKS_HIP(hipGetLastError());
}

}  // namespace dks
