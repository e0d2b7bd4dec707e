// The block DKS operator H X (shifted by -c^2) on gfx950.
//
// For every band and component the local potential goes through the grid in
// three passes over a column-pruned layout T1[column][z][xy-column] that holds
// only the xy-columns (n1, n2) crossing the planewave sphere:
//   zfft_inv   sphere -> z lines (inverse FFT along a3)       -> T1
//   plane      per z plane: inverse FFT along a2 (sphere rows only), inverse
//              FFT along a1, x V(r), forward FFT along a1, forward FFT along a2
//              (sphere rows only); the whole plane stays in LDS
//   zfft_fwd   T1 -> forward FFT along a3 -> sphere, / N_g, added to HX
// The projectors and the free-Dirac block are done first:
//   C = B^H X (matrix-core inner products), C' = W C per (atom, l) and
//   two-spinor, HX = B C' + kinetic(X) - shift X.
#include <algorithm>
#include <atomic>
#include <string>

#include "dks_internal.h"
#include "fft2.h"
#include "fft_device.h"

namespace dks {

// Early exit of the grid transforms, by item and by band: `item` (optional) is
// a finished system of a graph-captured batch; `band` (optional) flags bands
// whose input block rows are zero and whose output the kinetic and nonlocal
// kernel has already written (zero), the locked columns of the fixed-shape
// batch iteration.  The block index y of these kernels is the band-component.
struct BandSkip {
  const int *item;
  const int *band;
  int cshift;   // band = band-component >> cshift
  __device__ __forceinline__ bool done(int cc) const {
    return (item && *item) || (band && band[cc >> cshift]);
  }
};

// ---------------------------------------------------------------------------
// z transforms of the sphere columns
// ---------------------------------------------------------------------------
// Global reads are issued kZU per thread before any of them is waited for, so
// that a wave keeps several HBM requests in flight.  kTab: n3 has a compiled
// two-step split; the generic transforms run in a kernel of their own.
constexpr int kZU = 4;
template <typename T, bool kTab>
__global__ void __launch_bounds__(256) k_zfft_inv(const typename CT<T>::c *__restrict__ X, int N,
                                                  const int *__restrict__ col_off,
                                                  const int2 *__restrict__ gmap, int ncol,
                                                  int tile, const FftPlan *__restrict__ pzp,
                                                  const typename CT<T>::c *__restrict__ twz,
                                                  typename CT<T>::c *__restrict__ T1,
                                                  BandSkip skip) {
  if (skip.done(blockIdx.y)) return;   // a finished system, or a locked band
  using C = typename CT<T>::c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *lines = reinterpret_cast<C *>(smem_raw);
  const FftPlan &pz = *pzp;
  const int n3 = pz.n;
  const int ld = n3 + 1;
  const int c0 = blockIdx.x * tile;
  const int w = min(tile, ncol - c0);
  const int cc = blockIdx.y;
  const C *x = X + (size_t)cc * N;
  const int g0 = col_off[c0], g1 = col_off[c0 + w];
  const int nthr = blockDim.x;
  for (int b = g0; b < g1; b += kZU * nthr) {
    T vr[kZU], vi[kZU];
    int pos[kZU];
#pragma unroll
    for (int u = 0; u < kZU; ++u) {
      const int g = b + u * nthr + (int)threadIdx.x;
      const int gl = min(g, g1 - 1);
      const int2 m = gmap[gl];
      const C v = x[gl];
      vr[u] = v.x;
      vi[u] = v.y;
      pos[u] = g < g1 ? (m.x - c0) * ld + m.y : -1;
    }
    if (b == g0) {   // the first reads are in flight while the lines are cleared
      for (int e = threadIdx.x; e < w * ld; e += nthr) lines[e] = C{0, 0};
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kZU; ++u)
      if (pos[u] >= 0) lines[pos[u]] = C{vr[u], vi[u]};
  }
  if (g1 <= g0)
    for (int e = threadIdx.x; e < w * ld; e += nthr) lines[e] = C{0, 0};
  __syncthreads();
  const fft2::Lines Lz{nullptr, ld, 1};
  if constexpr (kTab) {
    const fft2::Walk Wz = fft2::walk(w);
    fft2::dispatch_z(n3, [&]<int A, int B>() {
      fft2::inv_step1<A, B, T>(lines, Wz, Lz, twz);
      __syncthreads();
      fft2::inv_step2<A, B, T>(lines, Wz, Lz);
    });
  } else {
    fft_lines<+1, T>(lines, w, nullptr, ld, 1, pz, twz);
  }
  __syncthreads();
  C *t = T1 + (size_t)cc * n3 * ncol;
  for (int e = threadIdx.x; e < w * n3; e += blockDim.x) {
    int z = e / w, ci = e - (e / w) * w;
    t[(size_t)z * ncol + c0 + ci] = lines[ci * ld + z];
  }
}

template <typename T, bool kTab>
__global__ void __launch_bounds__(256) k_zfft_fwd(const typename CT<T>::c *__restrict__ T1,
                                                  typename CT<T>::c *__restrict__ HX, int N,
                                                  const int *__restrict__ col_off,
                                                  const int2 *__restrict__ gmap, int ncol,
                                                  int tile, const FftPlan *__restrict__ pzp,
                                                  const typename CT<T>::c *__restrict__ twz,
                                                  T inv_ng, T scale,
                                                  BandSkip skip) {
  if (skip.done(blockIdx.y)) return;   // a finished system, or a locked band
  using C = typename CT<T>::c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *lines = reinterpret_cast<C *>(smem_raw);
  const FftPlan &pz = *pzp;
  const int n3 = pz.n;
  const int ld = n3 + 1;
  const int c0 = blockIdx.x * tile;
  const int w = min(tile, ncol - c0);
  const int cc = blockIdx.y;
  const C *t = T1 + (size_t)cc * n3 * ncol;
  const int nthr = blockDim.x;
  const int ne = w * n3;
  for (int b = 0; b < ne; b += kZU * nthr) {
    T vr[kZU], vi[kZU];
#pragma unroll
    for (int u = 0; u < kZU; ++u) {
      const int e = min(b + u * nthr + (int)threadIdx.x, ne - 1);
      const int z = e / w, ci = e - (e / w) * w;
      const C v = t[(size_t)z * ncol + c0 + ci];
      vr[u] = v.x;
      vi[u] = v.y;
    }
#pragma unroll
    for (int u = 0; u < kZU; ++u) {
      const int e = b + u * nthr + (int)threadIdx.x;
      if (e < ne) {
        const int z = e / w, ci = e - (e / w) * w;
        lines[ci * ld + z] = C{vr[u], vi[u]};
      }
    }
  }
  __syncthreads();
  const fft2::Lines Lz{nullptr, ld, 1};
  if constexpr (kTab) {
    const fft2::Walk Wz = fft2::walk(w);
    fft2::dispatch_z(n3, [&]<int A, int B>() {
      fft2::fwd_step2<A, B, T>(lines, Wz, Lz, twz);
      __syncthreads();
      fft2::fwd_step1<A, B, T>(lines, Wz, Lz);
    });
  } else {
    fft_lines<-1, T>(lines, w, nullptr, ld, 1, pz, twz);
  }
  __syncthreads();
  C *hx = HX + (size_t)cc * N;
  const int g0 = col_off[c0], g1 = col_off[c0 + w];
  for (int b = g0; b < g1; b += kZU * nthr) {
    T hr[kZU], hi[kZU];
    int pos[kZU];
#pragma unroll
    for (int u = 0; u < kZU; ++u) {
      const int gl = min(b + u * nthr + (int)threadIdx.x, g1 - 1);
      const int2 m = gmap[gl];
      const C h = hx[gl];
      hr[u] = h.x;
      hi[u] = h.y;
      pos[u] = (m.x - c0) * ld + m.y;
    }
#pragma unroll
    for (int u = 0; u < kZU; ++u) {
      const int g = b + u * nthr + (int)threadIdx.x;
      if (g < g1) {
        const C v = lines[pos[u]];
        hx[g] = C{scale * (hr[u] + inv_ng * v.x), scale * (hi[u] + inv_ng * v.y)};
      }
    }
  }
}

// ---------------------------------------------------------------------------
// one z plane: 2D inverse FFT, x V, 2D forward FFT, all in LDS
// ---------------------------------------------------------------------------
// One plane per workgroup.  FP64: the plane fills the LDS, one workgroup per
// CU, 768 threads (three waves per SIMD).  FP32: two workgroups of 512 threads
// per CU (two planes in LDS, 128 VGPRs per lane), so that one workgroup's
// barriers and column loads overlap the other's transforms.
// Small planes (a few thousand points, e.g. 48 x 48) leave most of those
// threads idle and fit several times into LDS: 256 threads, several
// workgroups per CU (kSmall).
template <typename T> constexpr int kPlaneThreads = sizeof(T) == 8 ? 768 : 512;
template <typename T> constexpr int kPlaneWaves = sizeof(T) == 8 ? 3 : 4;
constexpr int kSmallPlaneThreads = 256;
constexpr size_t kSmallPlaneLds = 40 * 1024;
template <typename T, bool kSmall>
constexpr int kPlaneThr = kSmall ? kSmallPlaneThreads : kPlaneThreads<T>;
// The list of rows that hold sphere columns sits in LDS behind the plane; so
// do the twiddle tables in FP32.  FP64 reads its twiddles through the vector
// cache: in LDS they slow the FP64 transforms, whose LDS traffic binds.
template <typename T> constexpr bool kPlaneTwLds = sizeof(T) == 4;
template <typename T>
size_t plane_lds_bytes(int n1, int n2) {
  using C = typename CT<T>::c;
  return sizeof(C) * ((size_t)n1 * (n2 + 1) + (kPlaneTwLds<T> ? n1 + n2 : 0)) +
         sizeof(int) * (size_t)((n1 + 3) & ~3);
}
// kTab: both plane axes have a compiled two-step split (fft2.h); otherwise the
// generic radix transforms run, in a kernel of their own so that their calls
// and registers stay out of the table kernel.
// kWaveLines: the line passes of the plane are split between waves by whole
// lines instead of between all threads by tasks (fewer workgroup barriers).
// kLite: both axes have lite lengths (fft2::plane_lite_has); only their
// codelets are compiled in (fewer registers, more waves per SIMD).
template <typename T, bool kTab, bool kSmall = false, bool kWaveLines = false, bool kLite = false>
__global__ void __launch_bounds__((kPlaneThr<T, kSmall>), kPlaneWaves<T>) k_plane(typename CT<T>::c *__restrict__ T1, int ncol,
                                                const int4 *__restrict__ col_info,
                                                const int *__restrict__ rows, int nrows,
                                                const FftPlan *__restrict__ pxy,
                                                const typename CT<T>::c *__restrict__ twx,
                                                const typename CT<T>::c *__restrict__ twy,
                                                const T *__restrict__ V,
                                                BandSkip skip) {
  if (skip.done(blockIdx.y)) return;   // a finished system, or a locked band
  using C = typename CT<T>::c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *pl = reinterpret_cast<C *>(smem_raw);
  const FftPlan &px = pxy[0], &py = pxy[1];
  const int n1 = px.n, n2 = py.n;
  const int ld = n2 + 1;
  const int z = blockIdx.x;
  const int cc = blockIdx.y;
  const int n3 = gridDim.x;
  int *rows_s = reinterpret_cast<int *>(pl + n1 * ld);
  C *twx_s = reinterpret_cast<C *>(rows_s + ((n1 + 3) & ~3)), *twy_s = twx_s + n1;
  const C *tx = kPlaneTwLds<T> ? twx_s : twx;
  const C *ty = kPlaneTwLds<T> ? twy_s : twy;
  auto stage = [&]() {
    for (int e = threadIdx.x; e < n1 * ld; e += blockDim.x) pl[e] = C{0, 0};
    for (int e = threadIdx.x; e < nrows; e += blockDim.x) rows_s[e] = rows[e];
    if constexpr (kPlaneTwLds<T>) {
      for (int e = threadIdx.x; e < n1; e += blockDim.x) twx_s[e] = twx[e];
      for (int e = threadIdx.x; e < n2; e += blockDim.x) twy_s[e] = twy[e];
    }
  };
  auto dispatch = [](int n, auto &&f) {
    if constexpr (kLite)
      return fft2::dispatch_plane_lite(n, f);
    else
      return fft2::dispatch_plane(n, f);
  };
  C *t = T1 + ((size_t)cc * n3 + z) * ncol;
  // The column values are fetched kPre per thread at a time, all loads in
  // flight together; the first batch is in flight while the plane is cleared.
  constexpr int kPre = 4;
  const int nthr = blockDim.x;
  for (int c0 = 0; c0 < ncol; c0 += kPre * nthr) {
    T vr[kPre], vi[kPre];
    int pos[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int c = c0 + u * nthr + (int)threadIdx.x;
      const int cl = min(c, ncol - 1);   // loads unconditional, stores masked
      const int4 ci = col_info[cl];
      const C x = t[cl];
      vr[u] = x.x;
      vi[u] = x.y;
      pos[u] = c < ncol ? ci.x * ld + ci.y : -1;
    }
    if (c0 == 0) {
      stage();
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kPre; ++u)
      if (pos[u] >= 0) pl[pos[u]] = C{vr[u], vi[u]};
  }
  if (ncol <= 0) stage();
  __syncthreads();
  const T *v = V + (size_t)z * n1 * n2;   // potential of this plane, [p1][p2] scrambled
  const fft2::Lines Ly{rows_s, ld, 1};       // rows holding sphere columns, along a2
  const fft2::Lines Lx{nullptr, 1, ld};    // every a2 position, along a1
  if constexpr (kTab && kWaveLines) {
    // Each wave owns whole lines of every axis pass (rows along a2, columns
    // along a1), so the two steps of one axis exchange data only within a
    // wave: a wave-level fence between them, a workgroup barrier only where
    // the axis changes.  Waves drift apart and overlap their LDS waits.
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int r0 = nrows * wave / nw, r1 = nrows * (wave + 1) / nw;
    const int c0 = n2 * wave / nw, c1 = n2 * (wave + 1) / nw;
    const fft2::Lines Lyw{rows_s + r0, ld, 1};
    auto wave_sync = [] {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
    };
    const fft2::Walk Wr = fft2::walk(r1 - r0, lane, 64), Wc = fft2::walk(c1 - c0, lane, 64);
    dispatch(n2, [&]<int A, int B>() {
      fft2::inv_step1<A, B, T>(pl, Wr, Lyw, ty);
      wave_sync();
      fft2::inv_step2<A, B, T>(pl, Wr, Lyw);
    });
    __syncthreads();
    dispatch(n1, [&]<int A, int B>() {
      fft2::inv_step1<A, B, T>(pl + c0, Wc, Lx, tx);
      wave_sync();
      fft2::inv2_mul_fwd2<A, B, T>(pl + c0, Wc, Lx, tx, v + c0, 1, n2);
      wave_sync();
      fft2::fwd_step1<A, B, T>(pl + c0, Wc, Lx);
    });
    __syncthreads();
    dispatch(n2, [&]<int A, int B>() {
      fft2::fwd_step2<A, B, T>(pl, Wr, Lyw, ty);
      wave_sync();
      fft2::fwd_step1<A, B, T>(pl, Wr, Lyw);
    });
    __syncthreads();
  } else {
  // inverse along a2
  const fft2::Walk Wr = fft2::walk(nrows), Wc = fft2::walk(n2);
  if constexpr (kTab) {
    dispatch(n2, [&]<int A, int B>() {
      fft2::inv_step1<A, B, T>(pl, Wr, Ly, ty);
      __syncthreads();
      fft2::inv_step2<A, B, T>(pl, Wr, Ly);
    });
  } else {
    fft_lines<+1, T>(pl, nrows, rows, ld, 1, py, twy);
  }
  __syncthreads();
  // inverse along a1, x V, forward along a1
  if constexpr (kTab) {
    dispatch(n1, [&]<int A, int B>() {
      fft2::inv_step1<A, B, T>(pl, Wc, Lx, tx);
      __syncthreads();
      fft2::inv2_mul_fwd2<A, B, T>(pl, Wc, Lx, tx, v, 1, n2);
      __syncthreads();
      fft2::fwd_step1<A, B, T>(pl, Wc, Lx);
    });
  } else {
    fft_lines<+1, T>(pl, n2, nullptr, 1, ld, px, twx);
    for (int e = threadIdx.x; e < n1 * n2; e += blockDim.x) {
      int i = e / n2, j = e - (e / n2) * n2;
      T s = v[e];
      C a = pl[i * ld + j];
      pl[i * ld + j] = C{a.x * s, a.y * s};
    }
    __syncthreads();
    fft_lines<-1, T>(pl, n2, nullptr, 1, ld, px, twx);
  }
  __syncthreads();
  // forward along a2
  if constexpr (kTab) {
    dispatch(n2, [&]<int A, int B>() {
      fft2::fwd_step2<A, B, T>(pl, Wr, Ly, ty);
      __syncthreads();
      fft2::fwd_step1<A, B, T>(pl, Wr, Ly);
    });
  } else {
    fft_lines<-1, T>(pl, nrows, rows, ld, 1, py, twy);
  }
  __syncthreads();
  }
  for (int c0 = 0; c0 < ncol; c0 += kPre * nthr) {
    T vr[kPre], vi[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int cl = min(c0 + u * nthr + (int)threadIdx.x, ncol - 1);
      const int4 ci = col_info[cl];
      const C x = pl[ci.x * ld + ci.y];
      vr[u] = x.x;
      vi[u] = x.y;
    }
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int c = c0 + u * nthr + (int)threadIdx.x;
      if (c < ncol) t[c] = C{vr[u], vi[u]};
    }
  }
}

// The same plane transform with the column loads and stores folded into the
// first and last steps along a2 (plane form 4): the sphere rows are built in
// registers from the column values (through the column table, zeros where a
// row has no column) and their inverse step 1 runs before anything reaches
// the LDS; the forward step 1' stores the column slots straight from
// registers.  Along a1 only the sphere rows are read (inverse step 1) and
// written back (forward step 1').  No clearing, scattering or gathering pass
// over the LDS plane and three workgroup barriers fewer.
template <typename T>
size_t plane_direct_lds_bytes(int n1, int n2) {
  return plane_lds_bytes<T>(n1, n2) + sizeof(int) * (size_t)((n1 + 3) & ~3);
}
// kSmall: 256-thread workgroups for planes within the small LDS budget, as
// for k_plane (plane form 5).  kLite: both axes have lite lengths (factors at
// most 10); only those codelets are compiled in.
template <typename T, bool kSmall, bool kLite = false>
__global__ void __launch_bounds__((kPlaneThr<T, kSmall>), kPlaneWaves<T>) k_plane_direct(
    typename CT<T>::c *__restrict__ T1, int ncol, const int *__restrict__ ctab,
    const int *__restrict__ rowflag, const int *__restrict__ rows, int nrows,
    const FftPlan *__restrict__ pxy, const typename CT<T>::c *__restrict__ twx,
    const typename CT<T>::c *__restrict__ twy, const T *__restrict__ V,
    BandSkip skip) {
  if (skip.done(blockIdx.y)) return;   // a finished system, or a locked band
  using C = typename CT<T>::c;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *pl = reinterpret_cast<C *>(smem_raw);
  const int n1 = pxy[0].n, n2 = pxy[1].n;
  const int ld = n2 + 1;
  const int z = blockIdx.x;
  const int cc = blockIdx.y;
  const int n3 = gridDim.x;
  const int n1p = (n1 + 3) & ~3;
  int *rows_s = reinterpret_cast<int *>(pl + n1 * ld);
  C *twx_s = reinterpret_cast<C *>(rows_s + n1p), *twy_s = twx_s + n1;
  int *keep_s = reinterpret_cast<int *>(twx_s + (kPlaneTwLds<T> ? n1 + n2 : 0));
  // the tables' LDS copies are written after the first step, whose loads go
  // out first
  auto stage = [&]() {
    for (int e = threadIdx.x; e < nrows; e += blockDim.x) rows_s[e] = rows[e];
    for (int e = threadIdx.x; e < n1; e += blockDim.x) keep_s[e] = rowflag[e];
    if constexpr (kPlaneTwLds<T>) {
      for (int e = threadIdx.x; e < n1; e += blockDim.x) twx_s[e] = twx[e];
      for (int e = threadIdx.x; e < n2; e += blockDim.x) twy_s[e] = twy[e];
    }
  };
  auto dispatch = [](int n, auto &&f) {
    if constexpr (kLite)
      return fft2::dispatch_plane_lite(n, f);
    else
      return fft2::dispatch_plane(n, f);
  };
  const C *tx = kPlaneTwLds<T> ? twx_s : twx;
  const C *ty = kPlaneTwLds<T> ? twy_s : twy;
  C *t = T1 + ((size_t)cc * n3 + z) * ncol;
  const T *v = V + (size_t)z * n1 * n2;   // potential of this plane, [p1][p2] scrambled
  const fft2::Lines Ly{rows_s, ld, 1};      // rows holding sphere columns, along a2
  const fft2::Lines Lx{nullptr, 1, ld};     // every a2 position, along a1
  const fft2::Walk Wr = fft2::walk(nrows), Wc = fft2::walk(n2);
  // inverse along a2 (step 1 from the columns, global twiddles: the LDS copy
  // is not complete before the first barrier)
  dispatch(n2, [&]<int A, int B>() {
    fft2::inv_step1_rows_in<A, B, T>(pl, ld, rows, nrows, n2, ctab, t, twy);
    stage();
    __syncthreads();
    fft2::inv_step2<A, B, T>(pl, Wr, Ly);
  });
  __syncthreads();
  // inverse along a1 (sphere rows in), x V, forward along a1 (sphere rows out)
  dispatch(n1, [&]<int A, int B>() {
    fft2::inv_step1_keep<A, B, T>(pl, Wc, Lx, tx, keep_s);
    __syncthreads();
    fft2::inv2_mul_fwd2<A, B, T>(pl, Wc, Lx, tx, v, 1, n2);
    __syncthreads();
    fft2::fwd_step1_keep<A, B, T>(pl, Wc, Lx, keep_s);
  });
  __syncthreads();
  // forward along a2 (step 1' to the columns)
  dispatch(n2, [&]<int A, int B>() {
    fft2::fwd_step2<A, B, T>(pl, Wr, Ly, ty);
    __syncthreads();
    fft2::fwd_step1_rows_out<A, B, T>(pl, ld, rows_s, nrows, n2, ctab, t);
  });
}

// ---------------------------------------------------------------------------
// projectors: C' = W C, per band, two-spinor and (atom, l) group
// C is [nproj][4 nb] (FP64); W blocks are (2 dim)^2, index (i m, s).
// ---------------------------------------------------------------------------
__global__ void k_apply_w(const double2 *__restrict__ Cin, double2 *__restrict__ Cout, int ldc,
                          int nb, int ncomp, const int4 *__restrict__ winfo, int ngroups,
                          const double2 *__restrict__ W, const int *__restrict__ skip) {
  if (skip && *skip) return;   // a finished system of a graph-captured batch
  // grid: x -> band * (ncomp / 2) + pair, y -> group; threads -> output index (2 dim).
  // ncomp = 4: the large and the small two-spinor of a Dirac spinor; ncomp = 2:
  // the one two-spinor of the two-component (KSSO) operator.
  const int npair = ncomp >> 1;
  const int bp = blockIdx.x;
  const int band = bp / npair, pair = bp - band * npair;
  const int4 gi = winfo[blockIdx.y];
  const int p0 = gi.x, dim = gi.y;
  const double2 *w = W + gi.z;
  const int nd = 2 * dim;
  for (int o = threadIdx.x; o < nd; o += blockDim.x) {
    double re = 0, im = 0;
    for (int k = 0; k < nd; ++k) {
      double2 wv = w[o * nd + k];
      int p = p0 + (k >> 1), s = k & 1;
      double2 cv = Cin[(size_t)p * ldc + band * ncomp + pair * 2 + s];
      re += wv.x * cv.x - wv.y * cv.y;
      im += wv.x * cv.y + wv.y * cv.x;
    }
    int p = p0 + (o >> 1), s = o & 1;
    Cout[(size_t)p * ldc + band * ncomp + pair * 2 + s] = make_double2(re, im);
  }
}

// HX = B C' + kinetic(X) - shift X.  A workgroup takes 256 planewaves of kBT
// bands; the band tiles of one planewave block are neighbouring work items in
// XCD order, so the block's projector rows B[:, g] come from one L2.  B is read
// kPB rows at a time, all loads in flight together.
constexpr int kBT = 4;
constexpr int kPB = 6;
// kPauli: the two-component operator (KSSO): kinetic |q|^2 / 2 on both spin
// components instead of the 4 x 4 free-Dirac block.
template <typename T, bool kPauli = false>
__global__ void __launch_bounds__(256) k_nl_kin(const typename CT<T>::c *__restrict__ X,
                                                typename CT<T>::c *__restrict__ HX, int N, int nb,
                                                const typename CT<T>::c *__restrict__ B, int nproj,
                                                const double2 *__restrict__ Cp, int ldc,
                                                const T *__restrict__ q, T c, T shift,
                                                const int *__restrict__ skip) {
  if (skip && *skip) return;   // a finished system of a graph-captured batch
  using C = typename CT<T>::c;
  constexpr int NC = kPauli ? 2 : 4;   // components per band
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *cs = reinterpret_cast<C *>(smem_raw);  // [nproj][NC kBT]
  const int ntb = (nb + kBT - 1) / kBT;
  const int w = xcd_order(blockIdx.x, gridDim.x);
  const int gb = w / ntb, tb = w - (w / ntb) * ntb;
  const int b0 = tb * kBT;
  const int bw = min(kBT, nb - b0);
  for (int e = threadIdx.x; e < nproj * NC * kBT; e += blockDim.x) {
    int p = e / (NC * kBT), j = e - (e / (NC * kBT)) * (NC * kBT);
    double2 v = (j < NC * bw) ? Cp[(size_t)p * ldc + b0 * NC + j] : make_double2(0, 0);
    cs[e] = C{(T)v.x, (T)v.y};
  }
  __syncthreads();
  const int g = gb * blockDim.x + threadIdx.x;
  if (g >= N) return;
  C acc[NC * kBT];
#pragma unroll
  for (int j = 0; j < NC * kBT; ++j) acc[j] = C{0, 0};
  for (int p0 = 0; p0 < nproj; p0 += kPB) {
    C bv[kPB];
#pragma unroll
    for (int u = 0; u < kPB; ++u) bv[u] = B[(size_t)min(p0 + u, nproj - 1) * N + g];
#pragma unroll
    for (int u = 0; u < kPB; ++u) {
      if (p0 + u < nproj) {
        const C *cr = cs + (p0 + u) * NC * kBT;
#pragma unroll
        for (int j = 0; j < NC * kBT; ++j) {
          const C cv = cr[j];
          acc[j].x += cv.x * bv[u].x - cv.y * bv[u].y;
          acc[j].y += cv.x * bv[u].y + cv.y * bv[u].x;
        }
      }
    }
  }
  const T qx = q[g], qy = q[N + g], qz = q[2 * N + g];
  if constexpr (kPauli) {
    const T kin = T(0.5) * (qx * qx + qy * qy + qz * qz) - shift;
#pragma unroll
    for (int bb = 0; bb < kBT; ++bb) {
      if (bb < bw) {
        const C *x = X + (size_t)(b0 + bb) * 2 * N;
        C *hx = HX + (size_t)(b0 + bb) * 2 * N;
        const C pu = x[g], pd = x[N + g];
        const C o0 = acc[bb * 2 + 0], o1 = acc[bb * 2 + 1];
        hx[g] = C{o0.x + kin * pu.x, o0.y + kin * pu.y};
        hx[N + g] = C{o1.x + kin * pd.x, o1.y + kin * pd.y};
      }
    }
    return;
  }
  const T twoc2 = T(2) * c * c;
#pragma unroll
  for (int bb = 0; bb < kBT; ++bb) {
    if (bb < bw) {
      const C *x = X + (size_t)(b0 + bb) * 4 * N;
      C *hx = HX + (size_t)(b0 + bb) * 4 * N;
      C pu = x[g], pd = x[N + g], cu = x[2 * N + g], cd = x[3 * N + g];
      // sigma.q = [[qz, qx - i qy], [qx + i qy, -qz]]
      C s0 = C{qz * cu.x + qx * cd.x + qy * cd.y, qz * cu.y + qx * cd.y - qy * cd.x};   // (sigma.q chi)_up
      C s1 = C{qx * cu.x - qy * cu.y - qz * cd.x, qx * cu.y + qy * cu.x - qz * cd.y};   // (sigma.q chi)_dn
      C t0 = C{qz * pu.x + qx * pd.x + qy * pd.y, qz * pu.y + qx * pd.y - qy * pd.x};   // (sigma.q phi)_up
      C t1 = C{qx * pu.x - qy * pu.y - qz * pd.x, qx * pu.y + qy * pu.x - qz * pd.y};   // (sigma.q phi)_dn
      C o0 = acc[bb * 4 + 0], o1 = acc[bb * 4 + 1], o2 = acc[bb * 4 + 2], o3 = acc[bb * 4 + 3];
      hx[g] = C{o0.x + c * s0.x - shift * pu.x, o0.y + c * s0.y - shift * pu.y};
      hx[N + g] = C{o1.x + c * s1.x - shift * pd.x, o1.y + c * s1.y - shift * pd.y};
      hx[2 * N + g] = C{o2.x + c * t0.x - (twoc2 + shift) * cu.x, o2.y + c * t0.y - (twoc2 + shift) * cu.y};
      hx[3 * N + g] = C{o3.x + c * t1.x - (twoc2 + shift) * cd.x, o3.y + c * t1.y - (twoc2 + shift) * cd.y};
    }
  }
}

// small component from the large one: chi = c sigma.q phi / (E_q + c^2)  (FP64)
__global__ void k_kinetic_balance(double2 *X, int N, int n, const double *q, double c) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  int b = blockIdx.y;
  if (g >= N || b >= n) return;
  double qx = q[g], qy = q[N + g], qz = q[2 * N + g];
  double q2 = qx * qx + qy * qy + qz * qz;
  double e = sqrt(c * c * q2 + c * c * c * c);
  double f = c / (e + c * c);
  double2 *x = X + (size_t)b * 4 * N;
  double2 pu = x[g], pd = x[N + g];
  double2 t0 = make_double2(qz * pu.x + qx * pd.x + qy * pd.y, qz * pu.y + qx * pd.y - qy * pd.x);
  double2 t1 = make_double2(qx * pu.x - qy * pu.y - qz * pd.x, qx * pu.y + qy * pu.x - qz * pd.y);
  x[2 * N + g] = make_double2(f * t0.x, f * t0.y);
  x[3 * N + g] = make_double2(f * t1.x, f * t1.y);
}

void kinetic_balance(dks_basis *b, int sys, double2 *X, int n, hipStream_t st) {
  System &s = *b->sys[sys];
  dim3 grid((s.N + 255) / 256, n);
  DKS_LAUNCH("k_kinetic_balance", k_kinetic_balance, grid, dim3(256), 0, st, X, s.N, n, s.d_q64.as<double>(),
                     s.c);
  DKS_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
template <typename T> static const typename CT<T>::c *Btab(const System &s);
template <> const double2 *Btab<double>(const System &s) { return s.d_B64.as<double2>(); }
template <> const float2 *Btab<float>(const System &s) { return s.d_B32.as<float2>(); }
template <typename T> static const T *Qtab(const System &s);
template <> const double *Qtab<double>(const System &s) { return s.d_q64.as<double>(); }
template <> const float *Qtab<float>(const System &s) { return s.d_q32.as<float>(); }
template <typename T> static const T *Vtab(const Potential &p);
template <> const double *Vtab<double>(const Potential &p) { return p.d_v64.as<double>(); }
template <> const float *Vtab<float>(const Potential &p) { return p.d_v32.as<float>(); }
template <typename T> static const typename CT<T>::c *Tw(const Potential &p, int d);
template <> const double2 *Tw<double>(const Potential &p, int d) { return p.d_tw64[d].as<double2>(); }
template <> const float2 *Tw<float>(const Potential &p, int d) { return p.d_tw32[d].as<float2>(); }

// ---------------------------------------------------------------------------
// spinor components on the real-space grid (the densities of Eq. density)
// ---------------------------------------------------------------------------
// One z plane of one band-component: the column values the z transform left
// in T1 are placed in the plane, transformed along a2 (sphere rows) and a1
// (every column) to real space, and the whole plane is written to
// R[cc][z][p1][p2] in the transforms' real-space order (that of the potential
// table).  FP64, the thread count of the plane kernel's form 0.
template <bool kTab>
__global__ void __launch_bounds__(kPlaneThreads<double>, kPlaneWaves<double>) k_plane_real(
    const double2 *__restrict__ T1, int ncol, const int4 *__restrict__ col_info,
    const int *__restrict__ rows, int nrows, const FftPlan *__restrict__ pxy,
    const double2 *__restrict__ twx, const double2 *__restrict__ twy, double2 *__restrict__ R) {
  using C = double2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *pl = reinterpret_cast<C *>(smem_raw);
  const FftPlan &px = pxy[0], &py = pxy[1];
  const int n1 = px.n, n2 = py.n;
  const int ld = n2 + 1;
  const int z = blockIdx.x, cc = blockIdx.y, n3 = gridDim.x;
  const int tid = threadIdx.x, nthr = blockDim.x;
  int *rows_s = reinterpret_cast<int *>(pl + n1 * ld);
  for (int e = tid; e < n1 * ld; e += nthr) pl[e] = C{0, 0};
  for (int e = tid; e < nrows; e += nthr) rows_s[e] = rows[e];
  __syncthreads();
  const C *t = T1 + ((size_t)cc * n3 + z) * ncol;
  for (int c = tid; c < ncol; c += nthr) {
    const int4 ci = col_info[c];
    pl[ci.x * ld + ci.y] = t[c];
  }
  __syncthreads();
  const fft2::Lines Ly{rows_s, ld, 1};
  const fft2::Lines Lx{nullptr, 1, ld};
  if constexpr (kTab) {
    const fft2::Walk Wr = fft2::walk(nrows), Wc = fft2::walk(n2);
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
    fft_lines<+1, double>(pl, nrows, rows_s, ld, 1, py, twy);
    __syncthreads();
    fft_lines<+1, double>(pl, n2, nullptr, 1, ld, px, twx);
  }
  __syncthreads();
  C *r = R + ((size_t)cc * n3 + z) * n1 * n2;
  for (int e = tid; e < n1 * n2; e += nthr) {
    const int p1 = e / n2, p2 = e - (e / n2) * n2;
    r[e] = pl[p1 * ld + p2];
  }
}

size_t real_space_t1_bytes(const dks_basis *b, int sysi, int ncols) {
  const System &s = *b->sys[sysi];
  return sizeof(double2) * (size_t)ncols * s.grid[2] * s.ncol;
}

void real_space_planes(dks_basis *b, int sysi, const double2 *X, int ncols, void *t1v,
                       double2 *R, hipStream_t st) {
  const System &s = *b->sys[sysi];
  const Potential &pot = *b->pot[s.vsrc];
  const int N = s.N, n3 = s.grid[2];
  double2 *t1 = static_cast<double2 *>(t1v);
  const int tile = s.tile_z;
  dim3 gz((s.ncol + tile - 1) / tile, ncols);
  const size_t smz = sizeof(double2) * (size_t)tile * (n3 + 1);
  auto kzinv = fft2::z_has(n3) ? k_zfft_inv<double, true> : k_zfft_inv<double, false>;
  DKS_LAUNCH("k_zfft_inv.f64", kzinv, gz, dim3(256), smz, st, X, N, s.d_col_off.as<int>(),
             s.d_gmap.as<int2>(), s.ncol, tile, s.d_plan.as<FftPlan>() + 2, Tw<double>(pot, 2), t1,
             BandSkip{nullptr, nullptr, 0});
  DKS_HIP(hipGetLastError());
  const bool tab = fft2::plane_has(s.grid[0]) && fft2::plane_has(s.grid[1]);
  auto kp = tab ? k_plane_real<true> : k_plane_real<false>;
  DKS_LAUNCH("k_plane_real", kp, dim3(n3, ncols), dim3(kPlaneThreads<double>),
             plane_lds_bytes<double>(s.grid[0], s.grid[1]), st, t1, s.ncol,
             s.d_col_info.as<int4>(), s.d_rows.as<int>(), s.nrows, s.d_plan.as<FftPlan>(),
             Tw<double>(pot, 0), Tw<double>(pot, 1), R);
  DKS_HIP(hipGetLastError());
}

void init_kernel_attributes() {
  static bool done = false;
  if (done) return;
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  for (const void *f : {(const void *)k_plane<double, true, false, false, true>,
                        (const void *)k_plane<float, true, false, false, true>,
                        (const void *)k_plane<double, true, false, true, true>,
                        (const void *)k_plane<float, true, false, true, true>})
    DKS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  for (const void *f : {(const void *)k_plane<double, true, true, false, true>,
                        (const void *)k_plane<float, true, true, false, true>,
                        (const void *)k_plane<double, true, true, true, true>,
                        (const void *)k_plane<float, true, true, true, true>})
    DKS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallPlaneLds));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<double, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallPlaneLds));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<float, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallPlaneLds));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<double, true, false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<float, true, false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<double, true, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallPlaneLds));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane<float, true, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallPlaneLds));
  const void *big_lds[] = {
      (const void *)k_zfft_inv<double, true>, (const void *)k_zfft_inv<double, false>,
      (const void *)k_zfft_inv<float, true>,  (const void *)k_zfft_inv<float, false>,
      (const void *)k_zfft_fwd<double, true>, (const void *)k_zfft_fwd<double, false>,
      (const void *)k_zfft_fwd<float, true>,  (const void *)k_zfft_fwd<float, false>};
  for (const void *f : big_lds)
    DKS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_nl_kin<double>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_nl_kin<float>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_nl_kin<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_nl_kin<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_direct<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_direct<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_direct<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallPlaneLds));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_direct<float, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallPlaneLds));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_direct<double, false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_direct<float, false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_direct<double, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallPlaneLds));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_direct<float, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallPlaneLds));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_real<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  DKS_HIP(hipFuncSetAttribute((const void *)k_plane_real<false>, hipFuncAttributeMaxDynamicSharedMemorySize, 163840));
  init_scf_kernel_attributes();
  done = true;
}

// ---------------------------------------------------------------------------
// preconditioner T of Algorithm 1 (T Y = R), the Teter factor of Sec. 4 on
// spinors: at each planewave, the spectral projectors P+- of the free Dirac
// block [[0, c s.q], [c s.q, -2c^2]] (eigenvalues e+ = sqrt(c^4 + c^2 q^2) - c^2
// and e- = -sqrt(c^4 + c^2 q^2) - c^2), P+ R scaled by K(e+ / E), P- R by
// K(|e-| / E), K(x) = p / (p + 16 x^4), p = 27 + 18x + 12x^2 + 8x^3, E per
// column the mean e+ of the residual's positive part.  Two components (no small
// component): K(|k+G|^2 / 2E).  Blocks [m][ncomp][N].
// ---------------------------------------------------------------------------
constexpr double kTpaEmin = 1e-3;   // floor of E (Ha)

template <typename T>
__device__ __forceinline__ T tpa_factor(T x) {
  const T p = T(27) + x * (T(18) + x * (T(12) + x * T(8)));
  return p / (p + T(16) * (x * x) * (x * x));
}

// P+ of one planewave's four components (phi_up, phi_dn, chi_up, chi_dn);
// returns e+ and |e-|.
template <typename T, typename C>
__device__ __forceinline__ void tpa_split(const C v[4], T qx, T qy, T qz, T c, C pp[4], T &ep,
                                          T &em) {
  const T q2 = qx * qx + qy * qy + qz * qz;
  const T root = sqrt(c * c * c * c + c * c * q2);
  ep = c * c * q2 / (root + c * c);
  em = root + c * c;
  // sigma.q u = [qz u0 + (qx - i qy) u1, (qx + i qy) u0 - qz u1]
  auto sdot = [&](const C &u0, const C &u1, C &o0, C &o1) {
    o0 = C{qz * u0.x + qx * u1.x + qy * u1.y, qz * u0.y + qx * u1.y - qy * u1.x};
    o1 = C{qx * u0.x - qy * u0.y - qz * u1.x, qx * u0.y + qy * u0.x - qz * u1.y};
  };
  C sc0, sc1, sp0, sp1;
  sdot(v[2], v[3], sc0, sc1);
  sdot(v[0], v[1], sp0, sp1);
  const T cc = c * c, h = T(0.5), ir = T(1) / root;
  const C sh[4] = {C{cc * v[0].x + c * sc0.x, cc * v[0].y + c * sc0.y},
                   C{cc * v[1].x + c * sc1.x, cc * v[1].y + c * sc1.y},
                   C{c * sp0.x - cc * v[2].x, c * sp0.y - cc * v[2].y},
                   C{c * sp1.x - cc * v[3].x, c * sp1.y - cc * v[3].y}};
#pragma unroll
  for (int a = 0; a < 4; ++a) pp[a] = C{h * (v[a].x + sh[a].x * ir), h * (v[a].y + sh[a].y * ir)};
}

// Partial sums of E: block (x, j) takes planewaves x*256 + t, step
// gridDim.x*256, of column j and writes (sum e+ |P+ y|^2, sum |P+ y|^2) to
// part[j * gridDim.x + x]; k_tpa_apply adds the partials of its column in a
// fixed order (the result does not depend on scheduling).
template <typename T>
__global__ void __launch_bounds__(256) k_tpa_energy(const cplx<T> *__restrict__ Y, int N,
                                                    const T *__restrict__ q, T c, int ncomp,
                                                    double2 *__restrict__ part,
                                                    const int *__restrict__ skip,
                                                    const int *__restrict__ idx) {
  if (skip && *skip) return;
  using C = cplx<T>;
  const int j = blockIdx.y;
  const C *y = Y + (size_t)(idx ? idx[j] : j) * ncomp * N;
  double num = 0, den = 0;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
    const T qx = q[g], qy = q[N + g], qz = q[2 * N + g];
    if (ncomp == 4) {
      const C v[4] = {y[g], y[N + g], y[2 * N + g], y[3 * N + g]};
      C pp[4];
      T ep, em;
      tpa_split<T>(v, qx, qy, qz, c, pp, ep, em);
      double w = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a) w += (double)pp[a].x * pp[a].x + (double)pp[a].y * pp[a].y;
      num += (double)ep * w;
      den += w;
    } else {
      const C a = y[g], b = y[N + g];
      const double w = (double)a.x * a.x + (double)a.y * a.y + (double)b.x * b.x + (double)b.y * b.y;
      num += 0.5 * ((double)qx * qx + (double)qy * qy + (double)qz * qz) * w;
      den += w;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    num += __shfl_xor(num, o, 64);
    den += __shfl_xor(den, o, 64);
  }
  __shared__ double sn[4], sd[4];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sn[wv] = num;
    sd[wv] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    part[(size_t)j * gridDim.x + blockIdx.x] = make_double2(sn[0] + sn[1] + sn[2] + sn[3],
                                                            sd[0] + sd[1] + sd[2] + sd[3]);
}

template <typename T>
// Src row idx[j] (or j) in, Y row j out: the two coincide in place
__global__ void __launch_bounds__(256) k_tpa_apply(const cplx<T> *Src, cplx<T> *Y, int N,
                                                   const T *__restrict__ q, T c, int ncomp,
                                                   const double2 *__restrict__ part, int nblk,
                                                   const int *__restrict__ skip,
                                                   const int *__restrict__ idx) {
  if (skip && *skip) return;
  using C = cplx<T>;
  const int j = blockIdx.y;
  __shared__ double sE;
  if (threadIdx.x < 64) {
    double num = 0, den = 0;
    for (int k = threadIdx.x; k < nblk; k += 64) {
      const double2 pk = part[(size_t)j * nblk + k];
      num += pk.x;
      den += pk.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
      num += __shfl_xor(num, o, 64);
      den += __shfl_xor(den, o, 64);
    }
    if (threadIdx.x == 0) sE = den > 0 ? fmax(num / den, kTpaEmin) : kTpaEmin;
  }
  __syncthreads();
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  C *y = Y + (size_t)j * ncomp * N;
  const C *src = Src + (size_t)(idx ? idx[j] : j) * ncomp * N;
  const T ie = T(1.0 / sE);
  const T qx = q[g], qy = q[N + g], qz = q[2 * N + g];
  if (ncomp == 4) {
    const C v[4] = {src[g], src[N + g], src[2 * N + g], src[3 * N + g]};
    C pp[4];
    T ep, em;
    tpa_split<T>(v, qx, qy, qz, c, pp, ep, em);
    const T kp = tpa_factor<T>(ep * ie), km = tpa_factor<T>(em * ie);
#pragma unroll
    for (int a = 0; a < 4; ++a)
      y[(size_t)a * N + g] = C{kp * pp[a].x + km * (v[a].x - pp[a].x), kp * pp[a].y + km * (v[a].y - pp[a].y)};
  } else {
    const T k = tpa_factor<T>(T(0.5) * (qx * qx + qy * qy + qz * qz) * ie);
    const C a = src[g], b = src[N + g];
    y[g] = C{k * a.x, k * a.y};
    y[N + g] = C{k * b.x, k * b.y};
  }
}

int tpa_blocks(int N) { return std::min(kTpaMaxBlocks, std::max(1, (N + 2047) / 2048)); }

template <typename T>
void precondition(dks_basis *b, int sysi, cplx<T> *Y, int m, hipStream_t st, int ncomp,
                  double2 *part, const int *skip, const cplx<T> *src, const int *idx) {
  if (m <= 0) return;
  const System &s = *b->sys[sysi];
  const int nblk = tpa_blocks(s.N);
  if (!src) {
    src = Y;
    idx = nullptr;
  }
  DKS_LAUNCH("k_tpa_energy", k_tpa_energy<T>, dim3(nblk, m), dim3(256), 0, st, src, s.N,
             Qtab<T>(s), (T)s.c, ncomp, part, skip, idx);
  DKS_HIP(hipGetLastError());
  DKS_LAUNCH("k_tpa_apply", k_tpa_apply<T>, dim3((s.N + 255) / 256, m), dim3(256), 0, st, src, Y,
             s.N, Qtab<T>(s), (T)s.c, ncomp, part, nblk, skip, idx);
  DKS_HIP(hipGetLastError());
}
template void precondition<double>(dks_basis *, int, double2 *, int, hipStream_t, int, double2 *,
                                   const int *, const double2 *, const int *);
template void precondition<float>(dks_basis *, int, float2 *, int, hipStream_t, int, double2 *,
                                  const int *, const float2 *, const int *);

// Plane form when none is set: the direct forms in FP64 (fewer LDS passes pay
// where the LDS traffic is 16 bytes a point), the LDS-staged ones in FP32;
// the 256-thread forms for planes within the small budget.
template <typename T>
int default_plane_form(const System &s) {
  if (!(fft2::plane_has(s.grid[0]) && fft2::plane_has(s.grid[1]))) return 0;
  if (sizeof(T) == 8) {
    const size_t smd = plane_direct_lds_bytes<T>(s.grid[0], s.grid[1]);
    if (smd > 163840) return 0;
    return smd <= kSmallPlaneLds ? 5 : 4;
  }
  return plane_lds_bytes<T>(s.grid[0], s.grid[1]) <= kSmallPlaneLds ? 1 : 0;
}

template <typename T>
void apply_scratch_bytes(const dks_basis *b, int sysi, int nb, size_t bytes[4], int ncomp) {
  const System &s = *b->sys[sysi];
  const int ncols = ncomp * nb;
  bytes[0] = sizeof(cplx<T>) * (size_t)ncols * s.grid[2] * s.ncol;
  const size_t cbytes = s.nproj > 0 ? sizeof(double2) * (size_t)s.nproj * ncols : 0;
  bytes[1] = cbytes;
  bytes[2] = cbytes;
  bytes[3] = s.nproj > 0 ? sizeof(double2) * gemm_ip_part_elems(s.nproj, ncols, (int64_t)s.N, false,
                                                                 false, s.ip_blocks)
                         : 0;
}

template <typename T>
void apply_h(dks_basis *b, int sysi, const cplx<T> *X, cplx<T> *HX, int nb, double shift,
             double scale, hipStream_t st, Workspace &ws, int ncomp, const int *skip,
             const int *band_skip) {
  if (nb <= 0) return;
  size_t bytes[4];
  apply_scratch_bytes<T>(b, sysi, nb, bytes, ncomp);
  ws.t1.ensure(bytes[0]);
  ws.nlc.ensure(bytes[1]);
  ws.nlc2.ensure(bytes[2]);
  ws.part.ensure(bytes[3]);
  ApplyScratch scr;
  scr.t1 = ws.t1.p;
  scr.nlc = ws.nlc.as<double2>();
  scr.nlc2 = ws.nlc2.as<double2>();
  scr.part = ws.part.as<double2>();
  apply_h_on<T>(b, sysi, X, HX, nb, shift, scale, st, scr, ncomp, skip, band_skip);
}

template <typename T>
void apply_h_on(dks_basis *b, int sysi, const cplx<T> *X, cplx<T> *HX, int nb, double shift,
                double scale, hipStream_t st, const ApplyScratch &scr, int ncomp,
                const int *skip, const int *band_skip) {
  using C = cplx<T>;
  System &s = *b->sys[sysi];
  Potential &pot = *b->pot[s.vsrc];
  if (nb <= 0) return;
  DKS_REQUIRE(ncomp == 4 || ncomp == 2, DKS_EINVAL, "spinor components must be 4 or 2");
  const int N = s.N;
  const int ncols = ncomp * nb;
  // --- projectors and kinetic block: HX = B C' + kin X - shift X
  double2 *Cp = nullptr;
  if (s.nproj > 0) {
    // B rows p*N and X rows cc*N are contiguous: offsets passed as null (stride N)
    gemm_ip_raw<T>(Btab<T>(s), nullptr, s.nproj, X, nullptr, ncols, nullptr, (int64_t)N, scr.nlc,
                   nullptr, ncols, scr.part, st, false, skip, s.ip_blocks);
    dim3 gw(nb * (ncomp / 2), (unsigned)s.groups.size());
    DKS_LAUNCH("k_apply_w", k_apply_w, gw, dim3(64), 0, st, scr.nlc, scr.nlc2, ncols, nb, ncomp,
               s.d_Winfo.as<int4>(), (int)s.groups.size(), s.d_W64.as<double2>(), skip);
    DKS_HIP(hipGetLastError());
    Cp = scr.nlc2;
  }
  {
    dim3 grid((unsigned)(((N + 255) / 256) * ((nb + kBT - 1) / kBT)));
    size_t sm = sizeof(C) * (size_t)s.nproj * ncomp * kBT;
    if (ncomp == 4)
      DKS_LAUNCH((sizeof(T) == 8 ? "k_nl_kin.f64" : "k_nl_kin.f32"), k_nl_kin<T>, grid, dim3(256),
                 sm, st, X, HX, N, nb, Btab<T>(s), s.nproj, Cp, ncols, Qtab<T>(s), (T)s.c, (T)shift,
                 skip);
    else
      DKS_LAUNCH((sizeof(T) == 8 ? "k_nl_kin.pauli.f64" : "k_nl_kin.pauli.f32"), (k_nl_kin<T, true>),
                 grid, dim3(256), sm, st, X, HX, N, nb, Btab<T>(s), s.nproj, Cp, ncols, Qtab<T>(s),
                 (T)s.c, (T)shift, skip);
    DKS_HIP(hipGetLastError());
  }
  // --- local potential through the grid
  const BandSkip gskip{skip, band_skip, ncomp == 4 ? 2 : 1};
  const int n3 = s.grid[2];
  C *t1 = static_cast<C *>(scr.t1);
  const int tile = s.tile_z;
  dim3 gz((s.ncol + tile - 1) / tile, ncols);
  size_t smz = sizeof(C) * (size_t)tile * (n3 + 1);
  const bool ztab = fft2::z_has(n3);
  auto kzinv = ztab ? k_zfft_inv<T, true> : k_zfft_inv<T, false>;
  auto kzfwd = ztab ? k_zfft_fwd<T, true> : k_zfft_fwd<T, false>;
  DKS_LAUNCH((sizeof(T) == 8 ? "k_zfft_inv.f64" : "k_zfft_inv.f32"), kzinv, gz, dim3(256), smz, st, X, N, s.d_col_off.as<int>(),
                     s.d_gmap.as<int2>(), s.ncol, tile, s.d_plan.as<FftPlan>() + 2, Tw<T>(pot, 2), t1,
                     gskip);
  DKS_HIP(hipGetLastError());
  dim3 gp(n3, ncols);
  size_t smp = plane_lds_bytes<T>(s.grid[0], s.grid[1]);
  const bool tab = fft2::plane_has(s.grid[0]) && fft2::plane_has(s.grid[1]);
  const bool fits_small = tab && smp <= kSmallPlaneLds;
  const int form = s.plane_form >= 0 ? s.plane_form : default_plane_form<T>(s);
  if (tab && (form == 4 || form == 5) &&
      plane_direct_lds_bytes<T>(s.grid[0], s.grid[1]) <= 163840) {
    const size_t smd = plane_direct_lds_bytes<T>(s.grid[0], s.grid[1]);
    const bool dsmall = form == 5 && smd <= kSmallPlaneLds;
    const bool lite = fft2::plane_lite_has(s.grid[0]) && fft2::plane_lite_has(s.grid[1]);
    auto kd = dsmall ? (lite ? k_plane_direct<T, true, true> : k_plane_direct<T, true>)
                     : (lite ? k_plane_direct<T, false, true> : k_plane_direct<T, false>);
    DKS_LAUNCH((sizeof(T) == 8 ? "k_plane.f64" : "k_plane.f32"), kd, gp,
               dim3(dsmall ? kSmallPlaneThreads : kPlaneThreads<T>), smd, st, t1,
               s.ncol, s.d_ctab.as<int>(), s.d_rowflag.as<int>(), s.d_rows.as<int>(), s.nrows,
               s.d_plan.as<FftPlan>(), Tw<T>(pot, 0), Tw<T>(pot, 1), Vtab<T>(pot), gskip);
  } else {
  const bool small = fits_small && (form == 1 || form == 3);
  const bool wlines = tab && (form == 2 || form == 3);
  const bool lite = tab && fft2::plane_lite_has(s.grid[0]) && fft2::plane_lite_has(s.grid[1]);
  auto kplane = !tab ? k_plane<T, false>
                : small ? (wlines ? (lite ? k_plane<T, true, true, true, true> : k_plane<T, true, true, true>)
                                  : (lite ? k_plane<T, true, true, false, true> : k_plane<T, true, true>))
                        : (wlines ? (lite ? k_plane<T, true, false, true, true> : k_plane<T, true, false, true>)
                                  : (lite ? k_plane<T, true, false, false, true> : k_plane<T, true>));
  const int pthr = small ? kSmallPlaneThreads : kPlaneThreads<T>;
  DKS_LAUNCH((sizeof(T) == 8 ? "k_plane.f64" : "k_plane.f32"), kplane, gp, dim3(pthr), smp, st, t1, s.ncol,
             s.d_col_info.as<int4>(), s.d_rows.as<int>(), s.nrows, s.d_plan.as<FftPlan>(),
             Tw<T>(pot, 0), Tw<T>(pot, 1), Vtab<T>(pot), gskip);
  }
  DKS_HIP(hipGetLastError());
  DKS_LAUNCH((sizeof(T) == 8 ? "k_zfft_fwd.f64" : "k_zfft_fwd.f32"), kzfwd, gz, dim3(256), smz, st, t1, HX, N, s.d_col_off.as<int>(),
                     s.d_gmap.as<int2>(), s.ncol, tile, s.d_plan.as<FftPlan>() + 2, Tw<T>(pot, 2),
                     (T)(1.0 / s.ng), (T)scale, gskip);
  DKS_HIP(hipGetLastError());
}

template void apply_h<double>(dks_basis *, int, const double2 *, double2 *, int, double, double,
                              hipStream_t, Workspace &, int, const int *, const int *);
template void apply_h<float>(dks_basis *, int, const float2 *, float2 *, int, double, double,
                             hipStream_t, Workspace &, int, const int *, const int *);
template void apply_h_on<double>(dks_basis *, int, const double2 *, double2 *, int, double,
                                 double, hipStream_t, const ApplyScratch &, int, const int *,
                                 const int *);
template void apply_h_on<float>(dks_basis *, int, const float2 *, float2 *, int, double, double,
                                hipStream_t, const ApplyScratch &, int, const int *, const int *);
template void apply_scratch_bytes<double>(const dks_basis *, int, int, size_t[4], int);
template void apply_scratch_bytes<float>(const dks_basis *, int, int, size_t[4], int);

}  // namespace dks

// ---------------------------------------------------------------------------
// H X without allocation: scratch from one file-scope device array
// ---------------------------------------------------------------------------
// The array lives in every GPU the library's code object is loaded on, at a
// per-device address.  The host symbol `scratch` is only a host-side handle:
// kernels are given the device address that hipGetSymbolAddress returns, taken
// once per device at dks_init_basis (with that device current) and kept in
// g_scratch_addr.  Nothing in the array needs to start at zero: every byte a
// kernel of apply_h_on reads is written earlier in the same call (the FFT
// intermediate by the z transform, the projector coefficients by the product
// and its reduction).
namespace dks {

constexpr size_t kNoAllocBytes = size_t(64) << 20;   // DKS_NOALLOC_SCRATCH_BYTES
static_assert(kNoAllocBytes == DKS_NOALLOC_SCRATCH_BYTES, "header and library disagree");
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
static std::atomic<void *> g_scratch_addr[kMaxDevices];

void noalloc_scratch_setup(int device) {
  DKS_REQUIRE(device >= 0 && device < kMaxDevices, DKS_EINVAL, "device index out of range");
  if (g_scratch_addr[device].load() != nullptr) return;
  void *p = nullptr;
  DKS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  DKS_REQUIRE(p != nullptr, DKS_EHIP, "no device address for the scratch array");
  g_scratch_addr[device].store(p);
}

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

template <typename T>
static size_t noalloc_need(const dks_basis *b, int sys, int nb) {
  size_t by[4];
  apply_scratch_bytes<T>(b, sys, nb, by);
  return align256(by[0]) + align256(by[1]) + align256(by[2]) + align256(by[3]);
}

template <typename T>
static void apply_h_noalloc(dks_basis *b, int sys, const cplx<T> *X, cplx<T> *HX, int nb,
                            hipStream_t st) {
  unsigned char *base = static_cast<unsigned char *>(g_scratch_addr[b->device].load());
  DKS_REQUIRE(base != nullptr, DKS_EINVAL, "the scratch array of this device is not set up");
  if (nb <= 0) return;
  const size_t one = noalloc_need<T>(b, sys, 1);
  DKS_REQUIRE(one <= kNoAllocBytes, DKS_EINVAL,
              "one band needs " + std::to_string(one) + " bytes of scratch, more than the " +
                  std::to_string(kNoAllocBytes) + "-byte array");
  // the largest band chunk whose scratch fits (the projector partial sums do
  // not grow linearly with the chunk, so the sizes are checked one by one)
  int chunk = nb;
  while (chunk > 1 && noalloc_need<T>(b, sys, chunk) > kNoAllocBytes) --chunk;
  size_t by[4];
  apply_scratch_bytes<T>(b, sys, chunk, by);
  ApplyScratch scr;
  size_t off = 0;
  scr.t1 = base + off;
  off += align256(by[0]);
  scr.nlc = reinterpret_cast<double2 *>(base + off);
  off += align256(by[1]);
  scr.nlc2 = reinterpret_cast<double2 *>(base + off);
  off += align256(by[2]);
  scr.part = reinterpret_cast<double2 *>(base + off);
  const size_t K = 4 * (size_t)b->sys[sys]->N;
  for (int b0 = 0; b0 < nb; b0 += chunk) {
    const int m = std::min(chunk, nb - b0);
    apply_h_on<T>(b, sys, X + (size_t)b0 * K, HX + (size_t)b0 * K, m, 0.0, 1.0, st, scr);
  }
}

}  // namespace dks

extern "C" dks_status dks_apply_H_noalloc(dks_basis *b, int sys, const void *X, void *HX, int nb,
                                          dks_prec prec, void *stream) {
  using namespace dks;
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && X && HX && sys >= 0 && sys < (int)b->sys.size() && nb >= 0, DKS_EINVAL,
                "bad argument");
    DKS_REQUIRE(X != HX, DKS_EINVAL, "X and HX must not overlap");
    DKS_REQUIRE(prec == DKS_FP64 || prec == DKS_FP32, DKS_EINVAL, "bad precision");
    DKS_HIP(hipSetDevice(b->device));
    ProfPause no_events;   // the optional kernel timing would create events
    hipStream_t st = (hipStream_t)stream;
    if (prec == DKS_FP64)
      apply_h_noalloc<double>(b, sys, (const double2 *)X, (double2 *)HX, nb, st);
    else
      apply_h_noalloc<float>(b, sys, (const float2 *)X, (float2 *)HX, nb, st);
    return DKS_OK;
  });
}

// ---------------------------------------------------------------------------
// launch-shape autotuner
// ---------------------------------------------------------------------------
// For each listed system, H X on nb bands of that system is timed (HIP events,
// median of three calls after a warm-up) for each candidate of one launch
// shape while the others keep their current values, and the fastest is kept:
// first the z-transform tile (xy-columns per workgroup, within the LDS), then
// the plane workgroup form (768/512 or 256 threads, where the plane fits the
// small form's LDS budget), then the split-K target of the projector product.
namespace dks {
template <typename T>
static float time_apply(dks_basis *b, int sys, const cplx<T> *X, cplx<T> *HX, int nb, hipStream_t st,
                        hipEvent_t e0, hipEvent_t e1) {
  apply_h<T>(b, sys, X, HX, nb, 0.0, 1.0, st, b->ws);
  float t[3];
  for (int r = 0; r < 3; ++r) {
    DKS_HIP(hipEventRecord(e0, st));
    apply_h<T>(b, sys, X, HX, nb, 0.0, 1.0, st, b->ws);
    DKS_HIP(hipEventRecord(e1, st));
    DKS_HIP(hipEventSynchronize(e1));
    DKS_HIP(hipEventElapsedTime(&t[r], e0, e1));
  }
  std::sort(t, t + 3);
  return t[1];
}

template <typename T>
static void tune_system(dks_basis *b, int sys, int nb, hipStream_t st, double *ms_out) {
  System &s = *b->sys[sys];
  const size_t K = 4 * (size_t)s.N;
  DevBuf x, hx;
  x.ensure(sizeof(cplx<T>) * K * nb);
  hx.ensure(sizeof(cplx<T>) * K * nb);
  DKS_HIP(hipMemsetAsync(x.p, 0, x.bytes, st));
  hipEvent_t e0, e1;
  DKS_HIP(hipEventCreate(&e0));
  DKS_HIP(hipEventCreate(&e1));
  try {
    const cplx<T> *X = x.as<cplx<T>>();
    cplx<T> *HX = hx.as<cplx<T>>();
    const int n3 = s.grid[2];
    auto best_of = [&](int &knob, const std::vector<int> &cand) {
      int bestv = knob;
      float bestt = 1e30f;
      for (int v : cand) {
        knob = v;
        const float t = time_apply<T>(b, sys, X, HX, nb, st, e0, e1);
        if (t < bestt) {
          bestt = t;
          bestv = v;
        }
      }
      knob = bestv;
      return bestt;
    };
    std::vector<int> tiles;
    for (int t : {2, 4, 8, 16, 32, 64})
      if (sizeof(cplx<T>) * (size_t)t * (n3 + 1) <= 163840 && t <= std::max(1, s.ncol)) tiles.push_back(t);
    float t = best_of(s.tile_z, tiles);
    const bool tab = fft2::plane_has(s.grid[0]) && fft2::plane_has(s.grid[1]);
    if (tab) {
      if (plane_lds_bytes<T>(s.grid[0], s.grid[1]) <= kSmallPlaneLds)
        t = best_of(s.plane_form, {0, 1, 2, 3, 4, 5});
      else
        t = best_of(s.plane_form, {0, 2, 4});
    }
    if (s.nproj > 0) t = best_of(s.ip_blocks, {256, 512, 1024, 2048});
    if (ms_out) *ms_out = t;
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  DKS_HIP(hipEventDestroy(e0));
  DKS_HIP(hipEventDestroy(e1));
}
}  // namespace dks

extern "C" dks_status dks_autotune(dks_basis *b, int nsys, const int *sys, const int *nb,
                                   dks_prec prec, void *stream) {
  using namespace dks;
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && nsys >= 0 && (nsys == 0 || (sys && nb)), DKS_EINVAL, "bad argument");
    for (int i = 0; i < nsys; ++i)
      DKS_REQUIRE(sys[i] >= 0 && sys[i] < (int)b->sys.size() && nb[i] >= 1, DKS_EINVAL,
                  "bad system index or band count");
    DKS_HIP(hipSetDevice(b->device));
    hipStream_t st = (hipStream_t)stream;
    ProfPause no_events;
    for (int i = 0; i < nsys; ++i) {
      if (prec == DKS_FP64)
        tune_system<double>(b, sys[i], nb[i], st, nullptr);
      else
        tune_system<float>(b, sys[i], nb[i], st, nullptr);
    }
    return DKS_OK;
  });
}

extern "C" dks_status dks_get_tuning(const dks_basis *b, int sys, int *tile_z, int *plane_form,
                                     int *ip_blocks) {
  using namespace dks;
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && sys >= 0 && sys < (int)b->sys.size(), DKS_EINVAL, "bad argument");
    const System &s = *b->sys[sys];
    if (tile_z) *tile_z = s.tile_z;
    if (plane_form) *plane_form = s.plane_form >= 0 ? s.plane_form : default_plane_form<double>(s);
    if (ip_blocks) *ip_blocks = s.ip_blocks > 0 ? s.ip_blocks : 1024;
    return DKS_OK;
  });
}

extern "C" dks_status dks_set_tuning(dks_basis *b, int sys, int tile_z, int plane_form,
                                     int ip_blocks) {
  using namespace dks;
  return guarded([&]() -> dks_status {
    DKS_REQUIRE(b && sys >= 0 && sys < (int)b->sys.size(), DKS_EINVAL, "bad argument");
    System &s = *b->sys[sys];
    DKS_REQUIRE(tile_z >= 1 && tile_z <= 64 && sizeof(double2) * (size_t)tile_z * (s.grid[2] + 1) <= 163840,
                DKS_EINVAL, "tile_z out of range for this grid");
    DKS_REQUIRE(plane_form >= -1 && plane_form <= 5, DKS_EINVAL, "plane_form must be in [-1, 5]");
    DKS_REQUIRE(ip_blocks >= 0 && ip_blocks <= 65536, DKS_EINVAL, "ip_blocks out of range");
    s.tile_z = tile_z;
    s.plane_form = plane_form;
    s.ip_blocks = ip_blocks;
    return DKS_OK;
  });
}
