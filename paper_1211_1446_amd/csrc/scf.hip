// The self-consistent field loop around the DKS eigenproblem (Sec. 2.1:
// Eq. density and the Hartree and exchange-correlation parts of V_hxc;
// Sec. 4: finite electronic temperature, Anderson mixing with the Kerker
// preconditioner; Sec. 3.2: N_init = 3 on the first step, then 1).
//
// Real-space fields at the boundary are FP64 on the FFT grid in natural order
// (index j3 fastest).  Inside, a field lives in the transforms' real-space
// order [p3][p1][p2] (that of the potential table); Potential::d_nat maps a
// position p along axis d to its natural index.
//
//   density   the sphere -> real space transforms of the operator (z lines,
//             then planes) write every band-component's real-space plane, and
//             one pass per grid point sums rho and m over the bands;
//   G-space   full-grid filters (Hartree 4 pi / G^2, Kerker G^2 / (G^2 + q0^2))
//             in three LDS passes: planes forward (a1, a2), z lines forward,
//             x kernel(G), inverse (fused, per column tile), planes inverse;
//   LDA       pointwise Perdew-Zunger correlation, Slater exchange, spin
//             interpolation;
//   mixing    dot products and linear combinations of grid vectors on the
//             device; the small Anderson least-squares problem on the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "dks_internal.h"
#include "fft2.h"
#include "fft_device.h"

namespace dks {

// ---------------------------------------------------------------------------
// densities
// ---------------------------------------------------------------------------
// acc[0..3][e] (+)= sum_b f_b (psi^+ psi, and the spin density components) at
// real-space point e of nbc bands whose components R[(b ncomp + c) ng + e] are
// given (ncomp = 4: m = phi^+ sigma phi - chi^+ sigma chi; ncomp = 2:
// m = phi^+ sigma phi).
__global__ void __launch_bounds__(256) k_density_acc(const double2 *__restrict__ R, int nbc, int ncomp,
                                                     int ng, const double *__restrict__ f,
                                                     double *__restrict__ acc, int first) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ng; e += gridDim.x * blockDim.x) {
    double rho = 0, mx = 0, my = 0, mz = 0;
    for (int b = 0; b < nbc; ++b) {
      const double w = f[b];
      if (w == 0.0) continue;   // uniform
      const double2 *r = R + (size_t)b * ncomp * ng + e;
      for (int h = 0; h < ncomp / 2; ++h) {
        const double2 u = r[(size_t)(2 * h) * ng], d = r[(size_t)(2 * h + 1) * ng];
        const double s = (h == 0) ? w : -w;
        const double uu = u.x * u.x + u.y * u.y, dd = d.x * d.x + d.y * d.y;
        rho += w * (uu + dd);
        // conj(u) d
        const double re = u.x * d.x + u.y * d.y, im = u.x * d.y - u.y * d.x;
        mx += 2.0 * s * re;
        my += 2.0 * s * im;
        mz += s * (uu - dd);
      }
    }
    if (first) {
      acc[e] = rho;
      acc[(size_t)ng + e] = mx;
      acc[2 * (size_t)ng + e] = my;
      acc[3 * (size_t)ng + e] = mz;
    } else {
      acc[e] += rho;
      acc[(size_t)ng + e] += mx;
      acc[2 * (size_t)ng + e] += my;
      acc[3 * (size_t)ng + e] += mz;
    }
  }
}

// dst[k][natural] = scale * src[k][e] for nf fields (e in the transforms' order)
__global__ void __launch_bounds__(256) k_to_natural(const double *__restrict__ src, double *__restrict__ dst,
                                                    int nf, int n1, int n2, int n3,
                                                    const int *__restrict__ nat1, const int *__restrict__ nat2,
                                                    const int *__restrict__ nat3, double scale) {
  const int ng = n1 * n2 * n3;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ng; e += gridDim.x * blockDim.x) {
    const int p2 = e % n2, t = e / n2, p1 = t % n1, p3 = t / n1;
    const size_t o = ((size_t)nat1[p1] * n2 + nat2[p2]) * n3 + nat3[p3];
    for (int k = 0; k < nf; ++k) dst[(size_t)k * ng + o] = scale * src[(size_t)k * ng + e];
  }
}

// the potential tables (FP64 and FP32, the transforms' order) from a natural field
__global__ void __launch_bounds__(256) k_potential_tables(const double *__restrict__ v, double *__restrict__ v64,
                                                          float *__restrict__ v32, int n1, int n2, int n3,
                                                          const int *__restrict__ nat1,
                                                          const int *__restrict__ nat2,
                                                          const int *__restrict__ nat3) {
  const int ng = n1 * n2 * n3;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ng; e += gridDim.x * blockDim.x) {
    const int p2 = e % n2, t = e / n2, p1 = t % n1, p3 = t / n1;
    const double x = v[((size_t)nat1[p1] * n2 + nat2[p2]) * n3 + nat3[p3]];
    v64[e] = x;
    v32[e] = (float)x;
  }
}

// ---------------------------------------------------------------------------
// full-grid reciprocal-space filters
// ---------------------------------------------------------------------------
// Work array W[p3][.][.] (complex, one plane of n1 x n2 per z position).
// Planes forward: the natural real field -> W[p3][k1][k2] (both plane axes in
// natural reciprocal order).
template <bool kTab>
__global__ void __launch_bounds__(768) k_grid_plane_fwd(const double *__restrict__ f, double2 *__restrict__ W,
                                                       const int *__restrict__ nat1, const int *__restrict__ nat2,
                                                       const int *__restrict__ nat3,
                                                       const FftPlan *__restrict__ pxy,
                                                       const double2 *__restrict__ twx,
                                                       const double2 *__restrict__ twy) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *pl = reinterpret_cast<double2 *>(smem_raw);
  const int n1 = pxy[0].n, n2 = pxy[1].n, n3 = gridDim.x, p3 = blockIdx.x;
  const int ld = n2 + 1, tid = threadIdx.x, nthr = blockDim.x;
  const int j3 = nat3[p3];
  for (int e = tid; e < n1 * n2; e += nthr) {
    const int p1 = e / n2, p2 = e - (e / n2) * n2;
    pl[p1 * ld + p2] = make_double2(f[((size_t)nat1[p1] * n2 + nat2[p2]) * n3 + j3], 0.0);
  }
  __syncthreads();
  const fft2::Lines Lx{nullptr, 1, ld}, Ly{nullptr, ld, 1};
  if constexpr (kTab) {
    const fft2::Walk Wc = fft2::walk(n2), Wr = fft2::walk(n1);
    fft2::dispatch_plane(n1, [&]<int A, int B>() {
      fft2::fwd_step2<A, B, double>(pl, Wc, Lx, twx);
      __syncthreads();
      fft2::fwd_step1<A, B, double>(pl, Wc, Lx);
    });
    __syncthreads();
    fft2::dispatch_plane(n2, [&]<int A, int B>() {
      fft2::fwd_step2<A, B, double>(pl, Wr, Ly, twy);
      __syncthreads();
      fft2::fwd_step1<A, B, double>(pl, Wr, Ly);
    });
  } else {
    fft_lines<-1, double>(pl, n2, nullptr, 1, ld, pxy[0], twx);
    __syncthreads();
    fft_lines<-1, double>(pl, n1, nullptr, ld, 1, pxy[1], twy);
  }
  __syncthreads();
  double2 *w = W + (size_t)p3 * n1 * n2;
  for (int e = tid; e < n1 * n2; e += nthr) {
    const int k1 = e / n2, k2 = e - (e / n2) * n2;
    w[e] = pl[k1 * ld + k2];
  }
}

// Planes inverse: W[p3][k1][k2] -> the real part, scaled, into the natural field
// (out = scale Re + beta out).
template <bool kTab>
__global__ void __launch_bounds__(768) k_grid_plane_inv(const double2 *__restrict__ W, double *__restrict__ out,
                                                       double scale, double beta,
                                                       const int *__restrict__ nat1, const int *__restrict__ nat2,
                                                       const int *__restrict__ nat3,
                                                       const FftPlan *__restrict__ pxy,
                                                       const double2 *__restrict__ twx,
                                                       const double2 *__restrict__ twy) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *pl = reinterpret_cast<double2 *>(smem_raw);
  const int n1 = pxy[0].n, n2 = pxy[1].n, n3 = gridDim.x, p3 = blockIdx.x;
  const int ld = n2 + 1, tid = threadIdx.x, nthr = blockDim.x;
  const double2 *w = W + (size_t)p3 * n1 * n2;
  for (int e = tid; e < n1 * n2; e += nthr) {
    const int k1 = e / n2, k2 = e - (e / n2) * n2;
    pl[k1 * ld + k2] = w[e];
  }
  __syncthreads();
  const fft2::Lines Lx{nullptr, 1, ld}, Ly{nullptr, ld, 1};
  if constexpr (kTab) {
    const fft2::Walk Wc = fft2::walk(n2), Wr = fft2::walk(n1);
    fft2::dispatch_plane(n2, [&]<int A, int B>() {
      fft2::inv_step1<A, B, double>(pl, Wr, Ly, twy);
      __syncthreads();
      fft2::inv_step2<A, B, double>(pl, Wr, Ly);
    });
    __syncthreads();
    fft2::dispatch_plane(n1, [&]<int A, int B>() {
      fft2::inv_step1<A, B, double>(pl, Wc, Lx, twx);
      __syncthreads();
      fft2::inv_step2<A, B, double>(pl, Wc, Lx);
    });
  } else {
    fft_lines<+1, double>(pl, n1, nullptr, ld, 1, pxy[1], twy);
    __syncthreads();
    fft_lines<+1, double>(pl, n2, nullptr, 1, ld, pxy[0], twx);
  }
  __syncthreads();
  const int j3 = nat3[p3];
  for (int e = tid; e < n1 * n2; e += nthr) {
    const int p1 = e / n2, p2 = e - (e / n2) * n2;
    const size_t o = ((size_t)nat1[p1] * n2 + nat2[p2]) * n3 + j3;
    const double v = scale * pl[p1 * ld + p2].x;
    out[o] = (beta == 0.0) ? v : v + beta * out[o];
  }
}

// The reciprocal-space kernels of the filters
enum GridKernel { kHartree = 0, kKerker = 1 };
struct Recip {
  double b[9];   // rows b1, b2, b3
};

// z lines of `tile` columns (k1, k2) of W: forward along a3 (the transforms'
// order -> natural k3), x kernel(G) / N_g, inverse along a3, in place.
template <bool kTab>
__global__ void __launch_bounds__(256) k_grid_z(double2 *__restrict__ W, int n1, int n2, int tile,
                                               const FftPlan *__restrict__ pzp,
                                               const double2 *__restrict__ twz, int kind, double q02,
                                               Recip rc, double inv_ng) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *lines = reinterpret_cast<double2 *>(smem_raw);
  const FftPlan &pz = *pzp;
  const int n3 = pz.n, ld = n3 + 1, ncol = n1 * n2;
  const int c0 = blockIdx.x * tile, w = min(tile, ncol - c0);
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int e = tid; e < w * n3; e += nthr) {
    const int z = e / w, ci = e - (e / w) * w;
    lines[ci * ld + z] = W[(size_t)z * ncol + c0 + ci];
  }
  __syncthreads();
  const fft2::Lines Lz{nullptr, ld, 1};
  if constexpr (kTab) {
    const fft2::Walk Wz = fft2::walk(w);
    fft2::dispatch_z(n3, [&]<int A, int B>() {
      fft2::fwd_step2<A, B, double>(lines, Wz, Lz, twz);
      __syncthreads();
      fft2::fwd_step1<A, B, double>(lines, Wz, Lz);
    });
  } else {
    fft_lines<-1, double>(lines, w, nullptr, ld, 1, pz, twz);
  }
  __syncthreads();
  for (int e = tid; e < w * n3; e += nthr) {
    const int ci = e / n3, k3 = e - (e / n3) * n3;
    const int c = c0 + ci, k1 = c / n2, k2 = c - (c / n2) * n2;
    const int m1 = k1 < (n1 + 1) / 2 ? k1 : k1 - n1;
    const int m2 = k2 < (n2 + 1) / 2 ? k2 : k2 - n2;
    const int m3 = k3 < (n3 + 1) / 2 ? k3 : k3 - n3;
    const double gx = m1 * rc.b[0] + m2 * rc.b[3] + m3 * rc.b[6];
    const double gy = m1 * rc.b[1] + m2 * rc.b[4] + m3 * rc.b[7];
    const double gz = m1 * rc.b[2] + m2 * rc.b[5] + m3 * rc.b[8];
    const double g2 = gx * gx + gy * gy + gz * gz;
    double k;
    if (kind == kHartree) k = (m1 | m2 | m3) ? 4.0 * M_PI / g2 : 0.0;
    else k = (m1 | m2 | m3) ? g2 / (g2 + q02) : 1.0;
    k *= inv_ng;
    const double2 v = lines[ci * ld + k3];
    lines[ci * ld + k3] = make_double2(k * v.x, k * v.y);
  }
  __syncthreads();
  if constexpr (kTab) {
    const fft2::Walk Wz = fft2::walk(w);
    fft2::dispatch_z(n3, [&]<int A, int B>() {
      fft2::inv_step1<A, B, double>(lines, Wz, Lz, twz);
      __syncthreads();
      fft2::inv_step2<A, B, double>(lines, Wz, Lz);
    });
  } else {
    fft_lines<+1, double>(lines, w, nullptr, ld, 1, pz, twz);
  }
  __syncthreads();
  for (int e = tid; e < w * n3; e += nthr) {
    const int z = e / w, ci = e - (e / w) * w;
    W[(size_t)z * ncol + c0 + ci] = lines[ci * ld + z];
  }
}

// ---------------------------------------------------------------------------
// local spin density approximation (Perdew-Zunger correlation fit of the
// Ceperley-Alder gas, Slater exchange, von Barth-Hedin spin interpolation)
// ---------------------------------------------------------------------------
struct PzParams {
  double g, b1, b2, A, B, C, D;
};
__device__ __constant__ PzParams kPzU = {-0.1423, 1.0529, 0.3334, 0.0311, -0.048, 0.0020, -0.0116};
__device__ __constant__ PzParams kPzP = {-0.0843, 1.3981, 0.2611, 0.01555, -0.0269, 0.0007, -0.0048};
constexpr double kRhoMin = 1e-14;

__device__ void pz_corr(double rs, const PzParams &p, double &e, double &de) {
  if (rs >= 1.0) {
    const double s = sqrt(rs);
    const double den = 1.0 + p.b1 * s + p.b2 * rs;
    e = p.g / den;
    de = -p.g * (0.5 * p.b1 / s + p.b2) / (den * den);
  } else {
    const double lr = log(rs);
    e = p.A * lr + p.B + p.C * rs * lr + p.D * rs;
    de = p.A / rs + p.C * (lr + 1.0) + p.D;
  }
}

// v_xc = (v_up + v_dn) / 2 and b = (v_up - v_dn) / 2 along m / |m|; exc = rho eps_xc
__global__ void __launch_bounds__(256) k_lda(const double *__restrict__ rho, const double *__restrict__ mag,
                                             int ng, double *__restrict__ vxc, double *__restrict__ bxc,
                                             double *__restrict__ exc) {
  const double cx = 0.75 * cbrt(9.0 * M_PI / 4.0) / M_PI;
  const double fden = exp2(4.0 / 3.0) - 2.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ng; e += gridDim.x * blockDim.x) {
    const double r = rho[e];
    double mx = 0, my = 0, mz = 0;
    if (mag) {
      mx = mag[e];
      my = mag[(size_t)ng + e];
      mz = mag[2 * (size_t)ng + e];
    }
    const double mn = sqrt(mx * mx + my * my + mz * mz);
    double v = 0, bm = 0, ed = 0;
    if (r > kRhoMin) {
      const double z = fmin(1.0, mn / r);
      const double rs = cbrt(3.0 / (4.0 * M_PI * r));
      const double zp = 1.0 + z, zm = 1.0 - z;
      const double zp13 = cbrt(zp), zm13 = cbrt(zm);
      // exchange: the unpolarised value times the spin factor
      const double exu = -cx / rs;
      const double sx = 0.5 * (zp * zp13 + zm * zm13);
      const double dsx = (2.0 / 3.0) * (zp13 - zm13);
      const double ex = exu * sx, dex_drs = (cx / (rs * rs)) * sx, dex_dz = exu * dsx;
      // correlation: interpolation between the unpolarised and polarised fits
      double ecu, decu, ecp, decp;
      pz_corr(rs, kPzU, ecu, decu);
      pz_corr(rs, kPzP, ecp, decp);
      const double fz = (zp * zp13 + zm * zm13 - 2.0) / fden;
      const double dfz = (4.0 / 3.0) * (zp13 - zm13) / fden;
      const double ec = ecu + fz * (ecp - ecu);
      const double dec_drs = decu + fz * (decp - decu);
      const double dec_dz = dfz * (ecp - ecu);
      const double eps = ex + ec, de_drs = dex_drs + dec_drs, de_dz = dex_dz + dec_dz;
      const double common = eps - rs / 3.0 * de_drs;
      const double vu = common + (1.0 - z) * de_dz, vd = common - (1.0 + z) * de_dz;
      v = 0.5 * (vu + vd);
      bm = 0.5 * (vu - vd);
      ed = r * eps;
    }
    vxc[e] = v;
    if (exc) exc[e] = ed;
    if (bxc) {
      const double s = (mn > 0) ? bm / mn : 0.0;
      bxc[e] = s * mx;
      bxc[(size_t)ng + e] = s * my;
      bxc[2 * (size_t)ng + e] = s * mz;
    }
  }
}

// ---------------------------------------------------------------------------
// grid vectors: reductions and linear combinations
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 512;
// part[blockIdx] = sum (or max |.|) over the block's share of x (times y if given)
template <bool kMax>
__global__ void __launch_bounds__(256) k_reduce(const double *__restrict__ x, const double *__restrict__ y,
                                                size_t n, double *__restrict__ part) {
  __shared__ double s[256];
  double a = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const double v = y ? x[e] * y[e] : x[e];
    a = kMax ? fmax(a, fabs(v)) : a + v;
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] = kMax ? fmax(s[threadIdx.x], s[threadIdx.x + h]) : s[threadIdx.x] + s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// part[j * gridDim.x + block] = the block's share of x_j . y_j for k pairs
constexpr int kMaxDots = 16;
struct DotPairs {
  const double *x[kMaxDots];
  const double *y[kMaxDots];
  int k;
};
__global__ void __launch_bounds__(256) k_multidot(DotPairs d, size_t n, double *__restrict__ part) {
  __shared__ double s[256];
  for (int j = 0; j < d.k; ++j) {
    double a = 0;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
      a += d.x[j][e] * d.y[j][e];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)j * gridDim.x + blockIdx.x] = s[0];
    __syncthreads();
  }
}

// min, max and sum of x in one pass: part[3 b + {0, 1, 2}]
__global__ void __launch_bounds__(256) k_minmaxsum(const double *__restrict__ x, size_t n,
                                                   double *__restrict__ part) {
  __shared__ double smn[256], smx[256], ssm[256];
  double mn = INFINITY, mx = -INFINITY, sm = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const double v = x[e];
    mn = fmin(mn, v);
    mx = fmax(mx, v);
    sm += v;
  }
  smn[threadIdx.x] = mn;
  smx[threadIdx.x] = mx;
  ssm[threadIdx.x] = sm;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + h]);
      smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + h]);
      ssm[threadIdx.x] += ssm[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = smn[0];
    part[3 * blockIdx.x + 1] = smx[0];
    part[3 * blockIdx.x + 2] = ssm[0];
  }
}

// out = sum_j c_j x_j (up to kMaxTerms vectors)
constexpr int kMaxTerms = 16;
struct Terms {
  const double *x[kMaxTerms];
  double c[kMaxTerms];
  int k;
};
__global__ void __launch_bounds__(256) k_lincomb(double *__restrict__ out, Terms t, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    double a = 0;
    for (int j = 0; j < t.k; ++j) a += t.c[j] * t.x[j][e];
    out[e] = a;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct ScfWork {
  DevBuf t1, R, acc, gridw, part, occ_d;
  DevBuf v_ext, v_in, v_out, vh, vxc, bxc, exc, rho, mag, tmp, xbar, rbar, x_prev, r_prev;
  std::vector<DevBuf *> hx, hr;   // Anderson history: differences of successive inputs, residuals
  std::vector<double> part_h;
  ~ScfWork() {
    for (auto *p : hx) delete p;
    for (auto *p : hr) delete p;
  }
};

static ScfWork &work_of(dks_basis *b) {
  if (!b->scf) b->scf = new ScfWork();
  return *static_cast<ScfWork *>(b->scf);
}

static bool plane_tab(const System &s) { return fft2::plane_has(s.grid[0]) && fft2::plane_has(s.grid[1]); }

static double cell_volume(const System &s) {
  const double *A = s.lattice;
  return std::fabs(A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                   A[2] * (A[3] * A[7] - A[4] * A[6]));
}

static Recip reciprocal_of(const System &s) {
  const double *A = s.lattice;
  const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
  double inv[9];
  inv[0] = (A[4] * A[8] - A[5] * A[7]) / det;
  inv[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  inv[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  inv[3] = (A[5] * A[6] - A[3] * A[8]) / det;
  inv[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  inv[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  inv[6] = (A[3] * A[7] - A[4] * A[6]) / det;
  inv[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  inv[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  Recip r;
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c) r.b[j * 3 + c] = 2.0 * M_PI * inv[c * 3 + j];
  return r;
}

static int grid_blocks(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 4096); }

// sum (or max |.|) of x (times y), synchronising `st`
static double reduce(ScfWork &w, const double *x, const double *y, size_t n, bool mx, hipStream_t st) {
  w.part.ensure(sizeof(double) * kRedBlocks);
  if (mx)
    DKS_LAUNCH("k_reduce.max", k_reduce<true>, dim3(kRedBlocks), dim3(256), 0, st, x, y, n, w.part.as<double>());
  else
    DKS_LAUNCH("k_reduce.sum", k_reduce<false>, dim3(kRedBlocks), dim3(256), 0, st, x, y, n, w.part.as<double>());
  DKS_HIP(hipGetLastError());
  w.part_h.resize(kRedBlocks);
  DKS_HIP(hipMemcpyAsync(w.part_h.data(), w.part.p, sizeof(double) * kRedBlocks, hipMemcpyDeviceToHost, st));
  DKS_HIP(hipStreamSynchronize(st));
  double a = 0;
  for (double v : w.part_h) a = mx ? std::max(a, v) : a + v;
  return a;
}

// x_j . y_j for the given pairs (any number; kMaxDots per launch), synchronising `st`
static std::vector<double> dots(ScfWork &w, const std::vector<std::pair<const double *, const double *>> &pr,
                                size_t n, hipStream_t st) {
  std::vector<double> out(pr.size(), 0.0);
  w.part.ensure(sizeof(double) * kRedBlocks * kMaxDots);
  w.part_h.resize((size_t)kRedBlocks * kMaxDots);
  for (size_t j0 = 0; j0 < pr.size(); j0 += kMaxDots) {
    DotPairs d{};
    d.k = (int)std::min<size_t>(kMaxDots, pr.size() - j0);
    for (int j = 0; j < d.k; ++j) {
      d.x[j] = pr[j0 + j].first;
      d.y[j] = pr[j0 + j].second;
    }
    DKS_LAUNCH("k_multidot", k_multidot, dim3(kRedBlocks), dim3(256), 0, st, d, n, w.part.as<double>());
    DKS_HIP(hipGetLastError());
    DKS_HIP(hipMemcpyAsync(w.part_h.data(), w.part.p, sizeof(double) * kRedBlocks * d.k, hipMemcpyDeviceToHost,
                           st));
    DKS_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < d.k; ++j) {
      double a = 0;
      for (int q = 0; q < kRedBlocks; ++q) a += w.part_h[(size_t)j * kRedBlocks + q];
      out[j0 + j] = a;
    }
  }
  return out;
}

static void lincomb(double *out, const std::vector<const double *> &xs, const std::vector<double> &cs,
                    size_t n, hipStream_t st) {
  DKS_REQUIRE(xs.size() == cs.size() && !xs.empty() && xs.size() <= (size_t)kMaxTerms, DKS_EINTERNAL,
              "bad linear combination");
  Terms t{};
  t.k = (int)xs.size();
  for (int j = 0; j < t.k; ++j) {
    t.x[j] = xs[j];
    t.c[j] = cs[j];
  }
  DKS_LAUNCH("k_lincomb", k_lincomb, dim3(grid_blocks(n)), dim3(256), 0, st, out, t, n);
  DKS_HIP(hipGetLastError());
}

// out = IFFT[kernel(G) FFT[in]] (real part), natural order; in may equal out
static void grid_filter(dks_basis *b, int sysi, const double *in, double *out, int kind, double q0,
                        hipStream_t st) {
  const System &s = *b->sys[sysi];
  const Potential &pot = *b->pot[s.vsrc];
  ScfWork &w = work_of(b);
  const int n1 = s.grid[0], n2 = s.grid[1], n3 = s.grid[2];
  const size_t ng = (size_t)n1 * n2 * n3;
  w.gridw.ensure(sizeof(double2) * ng);
  double2 *W = w.gridw.as<double2>();
  const bool tab = plane_tab(s), ztab = fft2::z_has(n3);
  const size_t smp = sizeof(double2) * (size_t)n1 * (n2 + 1);
  const int *nat1 = pot.d_nat[0].as<int>(), *nat2 = pot.d_nat[1].as<int>(), *nat3 = pot.d_nat[2].as<int>();
  const FftPlan *pl = s.d_plan.as<FftPlan>();
  auto kf = tab ? k_grid_plane_fwd<true> : k_grid_plane_fwd<false>;
  DKS_LAUNCH("k_grid_plane_fwd", kf, dim3(n3), dim3(768), smp, st, in, W, nat1, nat2, nat3, pl,
             pot.d_tw64[0].as<double2>(), pot.d_tw64[1].as<double2>());
  DKS_HIP(hipGetLastError());
  int tile = 1;
  while (tile < 64 && sizeof(double2) * (size_t)(2 * tile) * (n3 + 1) <= 65536) tile *= 2;
  const int ncol = n1 * n2;
  auto kz = ztab ? k_grid_z<true> : k_grid_z<false>;
  DKS_LAUNCH("k_grid_z", kz, dim3((ncol + tile - 1) / tile), dim3(256),
             sizeof(double2) * (size_t)tile * (n3 + 1), st, W, n1, n2, tile, pl + 2, pot.d_tw64[2].as<double2>(),
             kind, q0 * q0, reciprocal_of(s), 1.0 / (double)ng);
  DKS_HIP(hipGetLastError());
  auto ki = tab ? k_grid_plane_inv<true> : k_grid_plane_inv<false>;
  DKS_LAUNCH("k_grid_plane_inv", ki, dim3(n3), dim3(768), smp, st, W, out, 1.0, 0.0, nat1, nat2, nat3,
             pl, pot.d_tw64[0].as<double2>(), pot.d_tw64[1].as<double2>());
  DKS_HIP(hipGetLastError());
}

// the description of sys holds only this k-point (the SCF loop and the
// potential update act on the potential all its k-points share)
static int systems_sharing(const dks_basis *b, int sysi) {
  int c = 0;
  for (auto *s : b->sys)
    if (s->vsrc == b->sys[sysi]->vsrc) ++c;
  return c;
}

static void density_impl(dks_basis *b, int sysi, int ncomp, const double2 *X, int nb, const double *occ,
                         double *rho, double *mag, hipStream_t st) {
  const System &s = *b->sys[sysi];
  const Potential &pot = *b->pot[s.vsrc];
  ScfWork &w = work_of(b);
  const size_t ng = (size_t)s.grid[0] * s.grid[1] * s.grid[2];
  // bands per chunk: real-space planes of at most ~512 MB
  const size_t per_band = sizeof(double2) * ng * ncomp;
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(nb, ((size_t)512 << 20) / per_band));
  w.R.ensure(per_band * chunk);
  w.t1.ensure(real_space_t1_bytes(b, sysi, chunk * ncomp));
  w.acc.ensure(sizeof(double) * 4 * ng);
  w.occ_d.ensure(sizeof(double) * nb);
  DKS_HIP(hipMemcpyAsync(w.occ_d.p, occ, sizeof(double) * nb, hipMemcpyHostToDevice, st));
  bool first = true;
  for (int b0 = 0; b0 < nb; b0 += chunk) {
    const int bc = std::min(chunk, nb - b0);
    bool any = false;
    for (int j = 0; j < bc; ++j) any = any || occ[b0 + j] != 0.0;
    if (!any) continue;
    real_space_planes(b, sysi, X + (size_t)b0 * ncomp * s.N, bc * ncomp, w.t1.p, w.R.as<double2>(), st);
    DKS_LAUNCH("k_density_acc", k_density_acc, dim3(grid_blocks(ng)), dim3(256), 0, st, w.R.as<double2>(),
               bc, ncomp, (int)ng, w.occ_d.as<double>() + b0, w.acc.as<double>(), first ? 1 : 0);
    DKS_HIP(hipGetLastError());
    first = false;
  }
  if (first) DKS_HIP(hipMemsetAsync(w.acc.p, 0, sizeof(double) * 4 * ng, st));
  const double scale = 1.0 / cell_volume(s);
  const int *nat1 = pot.d_nat[0].as<int>(), *nat2 = pot.d_nat[1].as<int>(), *nat3 = pot.d_nat[2].as<int>();
  DKS_LAUNCH("k_to_natural", k_to_natural, dim3(grid_blocks(ng)), dim3(256), 0, st, w.acc.as<double>(), rho, 1,
             s.grid[0], s.grid[1], s.grid[2], nat1, nat2, nat3, scale);
  DKS_HIP(hipGetLastError());
  if (mag) {
    DKS_LAUNCH("k_to_natural", k_to_natural, dim3(grid_blocks(ng)), dim3(256), 0, st, w.acc.as<double>() + ng,
               mag, 3, s.grid[0], s.grid[1], s.grid[2], nat1, nat2, nat3, scale);
    DKS_HIP(hipGetLastError());
  }
}

static void set_potential_impl(dks_basis *b, int sysi, const double *v, hipStream_t st) {
  const System &s = *b->sys[sysi];
  Potential &pot = *b->pot[s.vsrc];
  ScfWork &w = work_of(b);
  const size_t ng = (size_t)s.grid[0] * s.grid[1] * s.grid[2];
  // bounds first (they decide the filter constants), then the tables
  w.part.ensure(sizeof(double) * 3 * kRedBlocks);
  DKS_LAUNCH("k_minmaxsum", k_minmaxsum, dim3(kRedBlocks), dim3(256), 0, st, v, ng, w.part.as<double>());
  DKS_HIP(hipGetLastError());
  w.part_h.resize(3 * kRedBlocks);
  DKS_HIP(hipMemcpyAsync(w.part_h.data(), w.part.p, sizeof(double) * 3 * kRedBlocks, hipMemcpyDeviceToHost, st));
  DKS_HIP(hipStreamSynchronize(st));
  double mn = INFINITY, mx = -INFINITY, sm = 0;
  for (int i = 0; i < kRedBlocks; ++i) {
    mn = std::min(mn, w.part_h[3 * i]);
    mx = std::max(mx, w.part_h[3 * i + 1]);
    sm += w.part_h[3 * i + 2];
  }
  DKS_REQUIRE(std::isfinite(mn) && std::isfinite(mx) && std::isfinite(sm), DKS_EINVAL,
              "the potential has a non-finite value");
  DKS_LAUNCH("k_potential_tables", k_potential_tables, dim3(grid_blocks(ng)), dim3(256), 0, st, v,
             pot.d_v64.as<double>(), pot.d_v32.as<float>(), s.grid[0], s.grid[1], s.grid[2],
             pot.d_nat[0].as<int>(), pot.d_nat[1].as<int>(), pot.d_nat[2].as<int>());
  DKS_HIP(hipGetLastError());
  pot.vmin = mn;
  pot.vmax = mx;
  pot.vmean = sm / (double)ng;
}

static void get_potential_impl(const dks_basis *b, int sysi, double *v, hipStream_t st) {
  const System &s = *b->sys[sysi];
  const Potential &pot = *b->pot[s.vsrc];
  const size_t ng = (size_t)s.grid[0] * s.grid[1] * s.grid[2];
  DKS_LAUNCH("k_to_natural", k_to_natural, dim3(grid_blocks(ng)), dim3(256), 0, st, pot.d_v64.as<double>(), v,
             1, s.grid[0], s.grid[1], s.grid[2], pot.d_nat[0].as<int>(), pot.d_nat[1].as<int>(),
             pot.d_nat[2].as<int>(), 1.0);
  DKS_HIP(hipGetLastError());
}

static void lda_impl(dks_basis *b, int sysi, const double *rho, const double *mag, double *vxc, double *bxc,
                     double *exc, hipStream_t st) {
  const System &s = *b->sys[sysi];
  const size_t ng = (size_t)s.grid[0] * s.grid[1] * s.grid[2];
  DKS_LAUNCH("k_lda", k_lda, dim3(grid_blocks(ng)), dim3(256), 0, st, rho, mag, (int)ng, vxc, bxc, exc);
  DKS_HIP(hipGetLastError());
}

// Fermi-Dirac occupations of eps[0..n) holding n_el electrons (bisection on mu)
static double fermi_occupations(const double *eps, int n, double n_el, double kT, double *f) {
  double lo = eps[0], hi = eps[0];
  for (int i = 1; i < n; ++i) {
    lo = std::min(lo, eps[i]);
    hi = std::max(hi, eps[i]);
  }
  lo -= 50.0 * kT + 1.0;
  hi += 50.0 * kT + 1.0;
  auto fill = [&](double mu) {
    double sum = 0;
    for (int i = 0; i < n; ++i) {
      const double x = std::min(700.0, std::max(-700.0, (eps[i] - mu) / kT));
      f[i] = 1.0 / (1.0 + std::exp(x));
      sum += f[i];
    }
    return sum;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (fill(mid) < n_el) lo = mid; else hi = mid;
  }
  const double mu = 0.5 * (lo + hi);
  fill(mu);
  return mu;
}

// argmin |r - dR g| from the normal equations (k x k, relative Tikhonov 1e-12)
static std::vector<double> small_lsq(std::vector<double> A, std::vector<double> rhs, int k) {
  double tr = 0;
  for (int i = 0; i < k; ++i) tr += A[i * k + i];
  for (int i = 0; i < k; ++i) A[i * k + i] += 1e-12 * std::max(tr, 1e-300);
  // Cholesky of the symmetric positive definite A
  for (int j = 0; j < k; ++j) {
    double d = A[j * k + j];
    for (int p = 0; p < j; ++p) d -= A[j * k + p] * A[j * k + p];
    DKS_REQUIRE(d > 0, DKS_ECHOL, "Anderson history matrix is not positive definite");
    d = std::sqrt(d);
    A[j * k + j] = d;
    for (int i = j + 1; i < k; ++i) {
      double v = A[i * k + j];
      for (int p = 0; p < j; ++p) v -= A[i * k + p] * A[j * k + p];
      A[i * k + j] = v / d;
    }
  }
  for (int i = 0; i < k; ++i) {
    double v = rhs[i];
    for (int p = 0; p < i; ++p) v -= A[i * k + p] * rhs[p];
    rhs[i] = v / A[i * k + i];
  }
  for (int i = k - 1; i >= 0; --i) {
    double v = rhs[i];
    for (int p = i + 1; p < k; ++p) v -= A[p * k + i] * rhs[p];
    rhs[i] = v / A[i * k + i];
  }
  return rhs;
}

void init_scf_kernel_attributes() {
  const void *fs[] = {(const void *)k_grid_plane_fwd<true>, (const void *)k_grid_plane_fwd<false>,
                      (const void *)k_grid_plane_inv<true>, (const void *)k_grid_plane_inv<false>};
  for (const void *f : fs) DKS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
}

}  // namespace dks

using namespace dks;

void free_scf_work(dks_basis *b) {
  delete static_cast<ScfWork *>(b->scf);
  b->scf = nullptr;
}

extern "C" {

dks_status dks_density(dks_basis *b, int sys, int model, const void *X, int nb, const double *occ,
                       double *rho, double *mag, void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && X && occ && rho && sys >= 0 && sys < (int)b->sys.size() && nb > 0, DKS_EINVAL,
                "bad argument");
    DKS_REQUIRE(model == DKS_MODEL_DKS || model == DKS_MODEL_KSSO, DKS_EINVAL, "bad model");
    for (int i = 0; i < nb; ++i)
      DKS_REQUIRE(std::isfinite(occ[i]) && occ[i] >= 0.0, DKS_EINVAL, "occupations must be finite and >= 0");
    DKS_HIP(hipSetDevice(b->device));
    const int ncomp = model == DKS_MODEL_DKS ? 4 : 2;
    density_impl(b, sys, ncomp, static_cast<const double2 *>(X), nb, occ, rho, mag, (hipStream_t)stream);
    return DKS_OK;
  });
}

dks_status dks_hartree(dks_basis *b, int sys, const double *rho, double *vh, void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && rho && vh && sys >= 0 && sys < (int)b->sys.size(), DKS_EINVAL, "bad argument");
    DKS_HIP(hipSetDevice(b->device));
    grid_filter(b, sys, rho, vh, kHartree, 0.0, (hipStream_t)stream);
    return DKS_OK;
  });
}

dks_status dks_kerker(dks_basis *b, int sys, const double *in, double *out, double q0, void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && in && out && sys >= 0 && sys < (int)b->sys.size(), DKS_EINVAL, "bad argument");
    DKS_REQUIRE(std::isfinite(q0) && q0 > 0, DKS_EINVAL, "q0 must be positive");
    DKS_HIP(hipSetDevice(b->device));
    grid_filter(b, sys, in, out, kKerker, q0, (hipStream_t)stream);
    return DKS_OK;
  });
}

dks_status dks_lda_xc(dks_basis *b, int sys, const double *rho, const double *mag, double *vxc, double *bxc,
                      double *exc, void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && rho && vxc && sys >= 0 && sys < (int)b->sys.size(), DKS_EINVAL, "bad argument");
    DKS_HIP(hipSetDevice(b->device));
    lda_impl(b, sys, rho, mag, vxc, bxc, exc, (hipStream_t)stream);
    return DKS_OK;
  });
}

dks_status dks_get_local_potential(const dks_basis *b, int sys, double *v, void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && v && sys >= 0 && sys < (int)b->sys.size(), DKS_EINVAL, "bad argument");
    DKS_HIP(hipSetDevice(b->device));
    get_potential_impl(b, sys, v, (hipStream_t)stream);
    return DKS_OK;
  });
}

dks_status dks_set_local_potential(dks_basis *b, int sys, const double *v, void *stream) {
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && v && sys >= 0 && sys < (int)b->sys.size(), DKS_EINVAL, "bad argument");
    DKS_HIP(hipSetDevice(b->device));
    set_potential_impl(b, sys, v, (hipStream_t)stream);
    return DKS_OK;
  });
}

void dks_scf_default_opts(dks_scf_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->n_electrons = 0.0;
  o->temperature = 5000.0;
  o->max_scf = 60;
  o->tol = 1e-8;
  o->eig_iters = 3;
  o->n_init_first = 3;
  o->n_init_next = 1;
  o->anderson_depth = 6;
  o->alpha = 0.5;
  o->kerker_q0 = 0.8;
  o->max_bxc = 1e-6;
  o->history = nullptr;
  o->eig_history = nullptr;
}

dks_status dks_scf(dks_basis *b, int sys, int n, void *X, double *lambda, double *occ,
                   const dks_scf_opts *sopts, const dks_solve_opts *eopts, dks_scf_info *info,
                   void *stream) {
  std::string msg;
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && X && lambda && sys >= 0 && sys < (int)b->sys.size(), DKS_EINVAL, "bad argument");
    dks_scf_opts so;
    if (sopts) so = *sopts; else dks_scf_default_opts(&so);
    dks_solve_opts eo;
    if (eopts) eo = *eopts; else dks_default_opts(&eo);
    DKS_REQUIRE(eo.model == DKS_MODEL_DKS || eo.model == DKS_MODEL_KSSO, DKS_EINVAL, "bad model");
    const int nwant = n - eo.n_buffer;
    DKS_REQUIRE(eo.n_buffer >= 0 && nwant >= 1, DKS_EINVAL, "n_buffer must be in [0, n)");
    DKS_REQUIRE(so.n_electrons > 0 && so.n_electrons < nwant, DKS_EINVAL,
                "n_electrons must lie strictly between 0 and the number of wanted bands");
    DKS_REQUIRE(so.temperature > 0 && so.max_scf >= 1 && so.tol > 0 && so.eig_iters >= 1 &&
                    so.n_init_first >= 0 && so.n_init_next >= 0 && so.anderson_depth >= 0 &&
                    so.anderson_depth + 1 <= kMaxTerms && so.alpha > 0 && so.kerker_q0 > 0 &&
                    so.max_bxc > 0,
                DKS_EINVAL, "bad SCF options");
    DKS_REQUIRE(systems_sharing(b, sys) == 1, DKS_EINVAL,
                "the SCF loop runs on a description with a single k-point");
    DKS_HIP(hipSetDevice(b->device));
    hipStream_t st = (hipStream_t)stream;
    const System &s = *b->sys[sys];
    const int ncomp = eo.model == DKS_MODEL_DKS ? 4 : 2;
    const size_t ng = (size_t)s.grid[0] * s.grid[1] * s.grid[2];
    const size_t gb = sizeof(double) * ng;
    ScfWork &w = work_of(b);
    for (DevBuf *d : {&w.v_ext, &w.v_in, &w.v_out, &w.vh, &w.vxc, &w.exc, &w.rho, &w.tmp, &w.xbar, &w.rbar,
                      &w.x_prev, &w.r_prev})
      d->ensure(gb);
    w.mag.ensure(3 * gb);
    w.bxc.ensure(3 * gb);
    const int depth = so.anderson_depth;
    while ((int)w.hx.size() < depth) {
      w.hx.push_back(new DevBuf());
      w.hr.push_back(new DevBuf());
    }
    for (int j = 0; j < depth; ++j) {
      w.hx[j]->ensure(gb);
      w.hr[j]->ensure(gb);
    }
    double *v_ext = w.v_ext.as<double>(), *v_in = w.v_in.as<double>(), *v_out = w.v_out.as<double>();
    get_potential_impl(b, sys, v_ext, st);
    DKS_HIP(hipMemcpyAsync(v_in, v_ext, gb, hipMemcpyDeviceToDevice, st));
    const double kT = 3.166811563e-6 * so.temperature;
    const double dv = cell_volume(s) / (double)ng;
    std::vector<double> f(n, 0.0), res(n);
    // Anderson history: the slots of the stored differences in order of age,
    // their Gram matrix G[slot][slot'] = dR_slot . dR_slot'
    std::vector<int> order;
    std::vector<double> G((size_t)std::max(depth, 1) * std::max(depth, 1), 0.0);
    bool have_prev = false;
    dks_scf_info inf{};
    inf.residual = INFINITY;
    dks_status out = DKS_WNOTCONV;
    // once the measure is below tol while the last solve has not converged,
    // the next step keeps V_in and solves to the eigensolver's own tolerance
    bool polish = false;
    for (int it = 0; it < so.max_scf; ++it) {
      // eigenpairs of H[V_in]: a few LOBPCG-F iterations from the last block
      dks_solve_opts o = eo;
      o.n_iter = polish ? eo.n_iter : so.eig_iters;
      o.n_init = it == 0 ? so.n_init_first : so.n_init_next;
      o.kinetic_balance = it == 0 ? eo.kinetic_balance : 0;
      dks_solve_info si{};
      const dks_status rc = dks_lobpcgf_solve(b, sys, n, X, lambda, res.data(), &o, &si, stream);
      if (rc < 0) throw Error{rc, std::string("eigensolver: ") + dks_last_error()};
      inf.eig_iterations += si.iterations;
      // occupations of the wanted bands
      inf.fermi = fermi_occupations(lambda, nwant, so.n_electrons, kT, f.data());
      for (int i = nwant; i < n; ++i) f[i] = 0.0;
      // densities and the potential they produce
      double *rho = w.rho.as<double>(), *mag = w.mag.as<double>();
      density_impl(b, sys, ncomp, static_cast<const double2 *>(X), n, f.data(), rho, mag, st);
      grid_filter(b, sys, rho, w.vh.as<double>(), kHartree, 0.0, st);
      lda_impl(b, sys, rho, mag, w.vxc.as<double>(), w.bxc.as<double>(), w.exc.as<double>(), st);
      lincomb(v_out, {v_ext, w.vh.as<double>(), w.vxc.as<double>()}, {1.0, 1.0, 1.0}, ng, st);
      inf.max_mag = reduce(w, mag, nullptr, 3 * ng, true, st);
      inf.max_bxc = reduce(w, w.bxc.as<double>(), nullptr, 3 * ng, true, st);
      // residual and its measure ||V_out - V_in|| / ||V_in||
      double *r = w.rbar.as<double>();
      lincomb(r, {v_out, v_in}, {1.0, -1.0}, ng, st);
      const double rn = std::sqrt(reduce(w, r, r, ng, false, st));
      const double vn = std::sqrt(reduce(w, v_in, v_in, ng, false, st));
      inf.residual = rn / std::max(vn, 1e-300);
      if (so.history) so.history[it] = inf.residual;
      if (so.eig_history) so.eig_history[it] = si.max_resnorm;
      // energies: band energy - double counting + E_H + E_xc - T S
      double eband = 0, ent = 0;
      for (int i = 0; i < nwant; ++i) {
        eband += f[i] * lambda[i];
        const double a = std::min(std::max(f[i], 1e-300), 1.0), c = std::min(std::max(1.0 - f[i], 1e-300), 1.0);
        ent -= a * std::log(a) + c * std::log(c);
      }
      lincomb(w.tmp.as<double>(), {v_in, v_ext}, {1.0, -1.0}, ng, st);
      const double dc = reduce(w, w.tmp.as<double>(), rho, ng, false, st) * dv;
      inf.e_hartree = 0.5 * reduce(w, w.vh.as<double>(), rho, ng, false, st) * dv;
      inf.e_xc = reduce(w, w.exc.as<double>(), nullptr, ng, false, st) * dv;
      inf.free_energy = eband - dc + inf.e_hartree + inf.e_xc - kT * ent;
      inf.iterations = it + 1;
      inf.eig_converged = si.converged;
      if (inf.residual < so.tol && si.converged) {
        // the iterates may carry a spin density on the way; the fixed point
        // must not, since H leaves out the sigma.B_xc term
        DKS_REQUIRE(inf.max_bxc <= so.max_bxc, DKS_EINVAL,
                    "spin-polarised self-consistent density (|B_xc| = " + std::to_string(inf.max_bxc) +
                        " Ha): the sigma.B_xc term is not applied by this operator");
        out = DKS_OK;
        break;
      }
      if (it + 1 == so.max_scf) break;
      if (inf.residual < so.tol && !polish) {
        polish = true;
        continue;
      }
      polish = false;
      // Anderson: the differences to the last pair go into the oldest slot
      // (dX = x_k - x_{k-1}, dR = r_k - r_{k-1}), then
      // gamma = argmin |r_k - dR gamma|, xbar = x_k - dX gamma, rbar = r_k - dR gamma
      if (have_prev && depth > 0) {
        int slot;
        if ((int)order.size() < depth) {
          slot = (int)order.size();
        } else {
          slot = order.front();
          order.erase(order.begin());
        }
        lincomb(w.hx[slot]->as<double>(), {v_in, w.x_prev.as<double>()}, {1.0, -1.0}, ng, st);
        lincomb(w.hr[slot]->as<double>(), {r, w.r_prev.as<double>()}, {1.0, -1.0}, ng, st);
        order.push_back(slot);
        std::vector<std::pair<const double *, const double *>> pr;
        for (int j : order) pr.push_back({w.hr[slot]->as<double>(), w.hr[j]->as<double>()});
        const std::vector<double> g = dots(w, pr, ng, st);
        for (size_t q = 0; q < order.size(); ++q) {
          G[(size_t)slot * depth + order[q]] = g[q];
          G[(size_t)order[q] * depth + slot] = g[q];
        }
      }
      DKS_HIP(hipMemcpyAsync(w.x_prev.p, v_in, gb, hipMemcpyDeviceToDevice, st));
      DKS_HIP(hipMemcpyAsync(w.r_prev.p, r, gb, hipMemcpyDeviceToDevice, st));
      have_prev = true;
      const int k = (int)order.size();
      std::vector<const double *> xs{v_in}, rs{r};
      std::vector<double> a{1.0};
      if (k > 0) {
        std::vector<std::pair<const double *, const double *>> pr;
        for (int j : order) pr.push_back({w.hr[j]->as<double>(), r});
        const std::vector<double> rhs = dots(w, pr, ng, st);
        std::vector<double> A((size_t)k * k);
        for (int i = 0; i < k; ++i)
          for (int j = 0; j < k; ++j) A[(size_t)i * k + j] = G[(size_t)order[i] * depth + order[j]];
        const std::vector<double> gam = small_lsq(A, rhs, k);
        for (int i = 0; i < k; ++i) {
          xs.push_back(w.hx[order[i]]->as<double>());
          rs.push_back(w.hr[order[i]]->as<double>());
          a.push_back(-gam[i]);
        }
      }
      lincomb(w.xbar.as<double>(), xs, a, ng, st);
      lincomb(w.tmp.as<double>(), rs, a, ng, st);
      grid_filter(b, sys, w.tmp.as<double>(), w.tmp.as<double>(), kKerker, so.kerker_q0, st);
      lincomb(v_in, {w.xbar.as<double>(), w.tmp.as<double>()}, {1.0, so.alpha}, ng, st);
      set_potential_impl(b, sys, v_in, st);
    }
    if (occ)
      for (int i = 0; i < n; ++i) occ[i] = f[i];
    inf.converged = out == DKS_OK ? 1 : 0;
    if (info) *info = inf;
    DKS_HIP(hipStreamSynchronize(st));
    if (out != DKS_OK) {
      msg = "SCF iteration limit reached";
      set_error(msg);
    }
    return out;
  });
}

}  // extern "C"
