// Block linear algebra on tall spinor blocks (rows of length K = 4N):
//  gemm_ip   small Gram-type products  out[i][j] = sum_k conj(A_i[k]) B_j[k]
//            on the matrix cores (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32),
//            split along k over many workgroups, partial sums reduced in FP64;
//  gemm_up   block updates  out_j[k] = sum_i V[i][j] A_i[k] (+ beta out_j[k]),
//            also on the matrix cores;
//  residuals, column norms, gathers and conversions.
#include "dks_internal.h"
#include "fft_device.h"

namespace dks {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using acc = d4;
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // lane l, slot v holds D[4 v + l / 16][l % 16]
  __device__ static int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct Mfma<float> {
  using acc = f4;
  __device__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // lane l, slot v holds D[4 (l / 16) + v][l % 16]
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int kIpTile = 64;   // output tile per workgroup (4 waves of 32 x 32)
constexpr int kIpKT = 16;     // complex k values staged per step
constexpr int kIpBlocks = 1024;  // split-K: about this many workgroups per product launch

// Output tile (ti, tj) of workgroup x: row-major over all tiles, or over the
// tiles on and above the diagonal when only the upper triangle is wanted.
__device__ __forceinline__ void ip_tile(int x, int tm, bool upper, int &ti, int &tj) {
  if (!upper) {
    ti = x % tm;
    tj = x / tm;
    return;
  }
  ti = 0;
  while (x >= tm - ti) {
    x -= tm - ti;
    ++ti;
  }
  tj = ti + x;
}

// Workgroup L -> (tile t, k split z).  Consecutive workgroups go to the eight
// XCDs in turn, so the tiles of one split are given to workgroups eight apart
// (L, L + 8, ...): they run on one XCD, whose L2 then serves the rows they
// share.  A tail of fewer than eight splits keeps the plain order.
__device__ __forceinline__ void split_map(int L, int tiles, int nsplit, int &t, int &z) {
  const int z8 = nsplit & ~7, full = z8 * tiles;
  if (L < full) {
    const int s = L >> 3;
    t = s % tiles;
    z = (s / tiles) * 8 + (L & 7);
  } else {
    const int r = L - full;
    t = r % tiles;
    z = z8 + r / tiles;
  }
}

// kTwo: B2 is given (the Gram pair S and A); without it the second set of
// accumulators and its LDS tile are not there, which lets a single product
// (projector coefficients, P against X) run at more waves per SIMD.
// kR48 (single products with M <= 48: 36 projectors, P against X of up to 48
// columns): a 48 x 64 output tile, each wave 48 rows x 16 columns, so that no
// 16 x 16 block lies wholly past the 48th row; 64-row tiles spend 28 of 64
// rows on padding at M = 36.
template <typename T, bool kTwo, bool kR48 = false>
__global__ void __launch_bounds__(256) k_gemm_ip(const typename CT<T>::c *__restrict__ A,
                                                 const int64_t *__restrict__ aoff, int M,
                                                 const typename CT<T>::c *__restrict__ B,
                                                 const int64_t *__restrict__ boff, int Nn,
                                                 const typename CT<T>::c *__restrict__ B2,
                                                 int64_t K, int64_t kchunk, int tm, int upper,
                                                 int tiles, int nsplit,
                                                 double2 *__restrict__ part,
                                                 double2 *__restrict__ part2,
                                                 const int *__restrict__ skip) {
  if (skip && *skip) return;   // a finished system of a graph-captured batch
  using C = typename CT<T>::c;
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  static_assert(!(kTwo && kR48), "the 48-row tile is for single products");
  constexpr int LD = kIpKT + 1;
  constexpr int TM = kR48 ? 48 : kIpTile;   // output tile rows
  constexpr int NI = kR48 ? 3 : 2, NJ = kR48 ? 1 : 2;   // 16 x 16 blocks per wave
  __shared__ C As[TM * LD];
  __shared__ C Bs[kIpTile * LD];
  __shared__ C B2s[kTwo ? kIpTile * LD : 1];
  constexpr bool two = kTwo;
  int t_, z, ti, tj;
  split_map(blockIdx.x, tiles, nsplit, t_, z);
  ip_tile(t_, tm, upper != 0, ti, tj);
  const int tm0 = ti * TM, tn0 = tj * kIpTile;
  const int64_t kb = (int64_t)z * kchunk;
  const int64_t ke = min(K, kb + kchunk);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = kR48 ? 0 : (wave >> 1) * 32, wn = kR48 ? wave * 16 : (wave & 1) * 32;
  // loader mapping: 4 threads per row, 4 consecutive complex each
  const int lrow = tid >> 2, lk = (tid & 3) * 4;
  const C *arow = nullptr, *brow = nullptr, *b2row = nullptr;
  if (lrow < TM && tm0 + lrow < M) arow = A + (aoff ? aoff[tm0 + lrow] : (int64_t)(tm0 + lrow) * K);
  if (tn0 + lrow < Nn) {
    int64_t o = boff ? boff[tn0 + lrow] : (int64_t)(tn0 + lrow) * K;
    brow = B + o;
    if (two) b2row = B2 + o;
  }
  // conj(a) b. FP64: four real products, t[0] = re, t[1] = im. FP32: three
  // (Gauss), t[0] = ar br, t[1] = ai bi, t[2] = (ar - ai)(br + bi), so that
  // re = t0 + t1 and im = t2 - t0 + t1; the FP64 form keeps four because six
  // FP64 accumulator sets halve the occupancy and cost more than they save.
  constexpr bool gauss = sizeof(T) == 4;
  constexpr int NT = gauss ? 3 : 2;
  acc_t t[NT][NI][NJ], u[NT][NI][NJ];
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j) t[q][i][j] = u[q][i][j] = acc_t{0, 0, 0, 0};
  // the next k step is fetched into registers while the current one is multiplied
  C ra[4], rb[4], rb2[4];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + lk + u;
      const bool ok = k < ke;
      ra[u] = (arow && ok) ? arow[k] : C{0, 0};
      rb[u] = (brow && ok) ? brow[k] : C{0, 0};
      if (two) rb2[u] = (b2row && ok) ? b2row[k] : C{0, 0};
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kIpKT) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!kR48 || lrow < TM) As[lrow * LD + lk + u] = ra[u];
      Bs[lrow * LD + lk + u] = rb[u];
      if (two) B2s[lrow * LD + lk + u] = rb2[u];
    }
    __syncthreads();
    if (k0 + kIpKT < ke) fetch(k0 + kIpKT);
#pragma unroll
    for (int s = 0; s < kIpKT / 4; ++s) {
      const int kk = s * 4 + (lane >> 4);
      C a[NI], bb[NJ], b2[NJ];
#pragma unroll
      for (int i = 0; i < NI; ++i) a[i] = As[(wm + i * 16 + (lane & 15)) * LD + kk];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        bb[j] = Bs[(wn + j * 16 + (lane & 15)) * LD + kk];
        if (two) b2[j] = B2s[(wn + j * 16 + (lane & 15)) * LD + kk];
      }
      if constexpr (gauss) {
        T ad[NI], bs[NJ], b2s[NJ];
#pragma unroll
        for (int i = 0; i < NI; ++i) ad[i] = a[i].x - a[i].y;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          bs[j] = bb[j].x + bb[j].y;
          if (two) b2s[j] = b2[j].x + b2[j].y;
        }
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            t[0][i][j] = MF::mma(a[i].x, bb[j].x, t[0][i][j]);
            t[1][i][j] = MF::mma(a[i].y, bb[j].y, t[1][i][j]);
            t[NT - 1][i][j] = MF::mma(ad[i], bs[j], t[NT - 1][i][j]);
            if (two) {
              u[0][i][j] = MF::mma(a[i].x, b2[j].x, u[0][i][j]);
              u[1][i][j] = MF::mma(a[i].y, b2[j].y, u[1][i][j]);
              u[NT - 1][i][j] = MF::mma(ad[i], b2s[j], u[NT - 1][i][j]);
            }
          }
      } else {
        // re += ar br + ai bi, im += ar bi - ai br; the .x products of all
        // tiles first so that no accumulator is reused back to back
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            t[0][i][j] = MF::mma(a[i].x, bb[j].x, t[0][i][j]);
            t[1][i][j] = MF::mma(a[i].x, bb[j].y, t[1][i][j]);
            if (two) {
              u[0][i][j] = MF::mma(a[i].x, b2[j].x, u[0][i][j]);
              u[1][i][j] = MF::mma(a[i].x, b2[j].y, u[1][i][j]);
            }
          }
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            t[0][i][j] = MF::mma(a[i].y, bb[j].y, t[0][i][j]);
            t[1][i][j] = MF::mma(-a[i].y, bb[j].x, t[1][i][j]);
            if (two) {
              u[0][i][j] = MF::mma(a[i].y, b2[j].y, u[0][i][j]);
              u[1][i][j] = MF::mma(-a[i].y, b2[j].x, u[1][i][j]);
            }
          }
      }
    }
    __syncthreads();
  }
  double2 *p1 = part + (size_t)z * M * Nn;
  double2 *p2 = two ? part2 + (size_t)z * M * Nn : nullptr;
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int r = tm0 + wm + i * 16 + MF::row(lane, v);
        int c = tn0 + wn + j * 16 + (lane & 15);
        if (r < M && c < Nn) {
          auto val = [&](acc_t (&w)[NT][NI][NJ]) {
            const double x0 = w[0][i][j][v], x1 = w[1][i][j][v];
            if constexpr (gauss) {
              const double x2 = w[NT - 1][i][j][v];
              return make_double2(x0 + x1, x2 - x0 + x1);
            } else {
              return make_double2(x0, x1);
            }
          };
          p1[(size_t)r * Nn + c] = val(t);
          if (two) p2[(size_t)r * Nn + c] = val(u);
        }
      }
}

// out[i][j] = sum over splits of the partial products.  A block takes 64
// consecutive entries of one product; its kRedWaves waves take every
// kRedWaves-th split and the wave sums meet in LDS in a fixed order, so the
// result does not depend on scheduling.  With `upper`, only tiles on or above
// the diagonal were computed: an entry of a tile above it also writes its
// mirror image, conjugated.  Both products (part -> out, part2 -> out2) in one
// launch.
constexpr int kRedWaves = 16;
__global__ void __launch_bounds__(64 * kRedWaves)
    k_reduce_part(const double2 *__restrict__ part, const double2 *__restrict__ part2, int nsplit,
                  int M, int Nn, int upper, double2 *__restrict__ out, double2 *__restrict__ out2,
                  int ldo, const int *__restrict__ skip) {
  __shared__ double2 red[kRedWaves][64];
  if (skip && *skip) return;   // a finished system of a graph-captured batch

  const int nel = M * Nn;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int e = blockIdx.x * 64 + lane;
  const bool second = e >= nel;
  if (second) e -= nel;
  const int i = e / Nn, j = e - (e / Nn) * Nn;
  const bool valid = e < nel && (!second || part2) && !(upper && (i / kIpTile) > (j / kIpTile));
  double re = 0, im = 0;
  if (valid) {
    const double2 *p = (second ? part2 : part) + e;
#pragma unroll 4
    for (int z = w; z < nsplit; z += kRedWaves) {
      const double2 v = p[(size_t)z * nel];
      re += v.x;
      im += v.y;
    }
  }
  red[w][lane] = make_double2(re, im);
  __syncthreads();
  if (w != 0 || !valid) return;
  for (int q = 1; q < kRedWaves; ++q) {
    re += red[q][lane].x;
    im += red[q][lane].y;
  }
  double2 *o = second ? out2 : out;
  o[(size_t)i * ldo + j] = make_double2(re, im);
  if (upper && (i / kIpTile) < (j / kIpTile)) o[(size_t)j * ldo + i] = make_double2(re, -im);
}

static void reduce_parts(const double2 *p1, const double2 *p2, int nsplit, int M, int Nn, bool upper,
                         double2 *out, double2 *out2, int ldo, hipStream_t st,
                         const int *skip = nullptr) {
  const int nel = M * Nn * (p2 ? 2 : 1);
  DKS_LAUNCH("k_reduce_part", k_reduce_part, dim3((nel + 63) / 64), dim3(64 * kRedWaves), 0, st, p1,
             p2, nsplit, M, Nn, (int)upper, out, out2, ldo, skip);
  DKS_HIP(hipGetLastError());
}

// Tiling and split-K of one gemm_ip call: output tiles, k splits and the k
// range of each split.
struct IpShape {
  int tm, tiles;
  bool upper;
  int64_t nsplit, kchunk;
};
static IpShape ip_shape(int M, int Nn, int64_t K, bool hermitian, int blocks) {
  IpShape g;
  g.tm = (M + kIpTile - 1) / kIpTile;
  const int tn = (Nn + kIpTile - 1) / kIpTile;
  g.upper = hermitian && M == Nn;
  g.tiles = g.upper ? g.tm * (g.tm + 1) / 2 : g.tm * tn;
  int64_t maxsplit = (K + kIpKT * 16 - 1) / (kIpKT * 16);
  const int target = blocks > 0 ? blocks : kIpBlocks;
  int64_t nsplit = (target + g.tiles - 1) / g.tiles;
  nsplit = std::max<int64_t>(1, std::min<int64_t>(nsplit, maxsplit));
  int64_t kchunk = (K + nsplit - 1) / nsplit;
  kchunk = (kchunk + kIpKT - 1) / kIpKT * kIpKT;
  if (kchunk < kIpKT) kchunk = kIpKT;
  nsplit = (K + kchunk - 1) / kchunk;
  if (nsplit < 1) nsplit = 1;
  g.nsplit = nsplit;
  g.kchunk = kchunk;
  return g;
}

size_t gemm_ip_part_elems(int M, int Nn, int64_t K, bool two, bool hermitian, int blocks) {
  if (M <= 0 || Nn <= 0) return 0;
  const IpShape g = ip_shape(M, Nn, K, hermitian, blocks);
  return (size_t)g.nsplit * M * Nn * (two ? 2 : 1);
}

template <typename T>
void gemm_ip(const cplx<T> *A, const int64_t *aoff, int M, const cplx<T> *B, const int64_t *boff,
             int Nn, const cplx<T> *B2, int64_t K, double2 *out, double2 *out2, int ldo,
             DevBuf &part, hipStream_t st, bool hermitian, const int *skip) {
  if (M <= 0 || Nn <= 0) return;
  part.ensure(sizeof(double2) * gemm_ip_part_elems(M, Nn, K, B2 != nullptr, hermitian));
  gemm_ip_raw<T>(A, aoff, M, B, boff, Nn, B2, K, out, out2, ldo, part.as<double2>(), st, hermitian,
                 skip);
}

template <typename T>
void gemm_ip_raw(const cplx<T> *A, const int64_t *aoff, int M, const cplx<T> *B, const int64_t *boff,
                 int Nn, const cplx<T> *B2, int64_t K, double2 *out, double2 *out2, int ldo,
                 double2 *part, hipStream_t st, bool hermitian, const int *skip, int blocks) {
  if (M <= 0 || Nn <= 0) return;
  const IpShape g = ip_shape(M, Nn, K, hermitian, blocks);
  const int tm = g.tm, tiles = g.tiles;
  const bool upper = g.upper;
  const int64_t nsplit = g.nsplit, kchunk = g.kchunk;
  double2 *p1 = part;
  double2 *p2 = B2 ? p1 + (size_t)nsplit * M * Nn : nullptr;
  dim3 grid((unsigned)(tiles * nsplit));
  const char *name = upper ? (sizeof(T) == 8 ? "k_gemm_ip.gram.f64" : "k_gemm_ip.gram.f32")
                           : (sizeof(T) == 8 ? "k_gemm_ip.f64" : "k_gemm_ip.f32");
  // single products of at most 48 rows: one 48-row tile (tm = 1 as for 64 rows)
  auto kern = B2 ? k_gemm_ip<T, true> : (M <= 48 ? k_gemm_ip<T, false, true> : k_gemm_ip<T, false>);
  DKS_LAUNCH(name, kern, grid, dim3(256), 0, st, A, aoff, M, B, boff, Nn, B2, K, kchunk, tm,
             (int)upper, tiles, (int)nsplit, p1, p2, skip);
  DKS_HIP(hipGetLastError());
  reduce_parts(p1, p2, (int)nsplit, M, Nn, upper, out, out2, ldo, st, skip);
}

// ---------------------------------------------------------------------------
// Gram products on the BF16 matrix cores with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16).  Each FP32 input is split into two BF16 numbers,
// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to nearest even),
// and a b is taken as hi_a hi_b + hi_a lo_b + lo_a hi_b: about 16 significant
// bits per factor instead of 8, at three BF16 products per real product.
// The split is made once per element, by the thread that stages it: LDS holds
// four BF16 planes per row (hi and lo of the real and the imaginary part).  A
// step stages 32 complex k values; lane l of a 16 x 16 x 32 product holds row
// (or column) l % 16 and the eight values of slot group l / 16.  Thread t
// fetches the pairs k = 2 p, 2 p + 1 with p = t % 4 + 4 u (u < 4: four lanes
// read 64 contiguous bytes of a row per load) and stores them in slots
// 8 (t % 4) + 2 u + {0, 1}; every operand is staged alike, so the k order
// inside a step differs from memory order for all of them together and the
// sums are those of the plain product.
// Same output tiling, k splitting, workgroup order and reduction as k_gemm_ip.
// ---------------------------------------------------------------------------
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
constexpr int kBfKT = 32;                   // complex k values staged per step
constexpr int kBfPlane = kBfKT * 2;         // bytes of one BF16 plane of a row
constexpr int kBfRow = 4 * kBfPlane + 16;   // bytes per staged row (16 B pad: rows l % 16
                                            // of one read fall on distinct banks)
constexpr int kBfBlocks = 512;              // split-K target (fewer partials to reduce)

__device__ __forceinline__ bf8 bf_neg(bf8 x) {
  u4 u = __builtin_bit_cast(u4, x);
  u ^= 0x80008000u;   // flip both BF16 sign bits of each dword
  return __builtin_bit_cast(bf8, u);
}

__global__ void __launch_bounds__(256, 2) k_gemm_ip_bf16(const float2 *__restrict__ A,
                                                      const int64_t *__restrict__ aoff, int M,
                                                      const float2 *__restrict__ B,
                                                      const int64_t *__restrict__ boff, int Nn,
                                                      const float2 *__restrict__ B2, int64_t K,
                                                      int64_t kchunk, int tm, int upper,
                                                      int tiles, int nsplit,
                                                      double2 *__restrict__ part,
                                                      double2 *__restrict__ part2) {
  __shared__ __align__(16) unsigned char As[kIpTile * kBfRow];
  __shared__ __align__(16) unsigned char Bs[kIpTile * kBfRow];
  __shared__ __align__(16) unsigned char B2s[kIpTile * kBfRow];
  const bool two = (B2 != nullptr);
  int t, z, ti, tj;
  split_map(blockIdx.x, tiles, nsplit, t, z);
  ip_tile(t, tm, upper != 0, ti, tj);
  const int tm0 = ti * kIpTile, tn0 = tj * kIpTile;
  const int64_t kb = (int64_t)z * kchunk;
  const int64_t ke = min(K, kb + kchunk);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lrow = tid >> 2, lq = tid & 3;
  // rows past the matrix read the tile's first row and stage zeros: every
  // load is unconditional, its value selected (no branch around each load)
  const bool aval = tm0 + lrow < M, bval = tn0 + lrow < Nn;
  const int ar_ = aval ? tm0 + lrow : tm0, br_ = bval ? tn0 + lrow : tn0;
  const float2 *arow = A + (aoff ? aoff[ar_] : (int64_t)ar_ * K);
  const int64_t bo = boff ? boff[br_] : (int64_t)br_ * K;
  const float2 *brow = B + bo;
  const float2 *b2row = two ? B2 + bo : brow;
  f4 re[2][2], im[2][2], re2[2][2], im2[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      re[i][j] = f4{0, 0, 0, 0};
      im[i][j] = f4{0, 0, 0, 0};
      re2[i][j] = f4{0, 0, 0, 0};
      im2[i][j] = f4{0, 0, 0, 0};
    }
  // 16-byte loads (two complex values) where a row starts 16-byte aligned
  // (kb and k0 are even), two 8-byte loads otherwise
  const bool aal = ((uintptr_t)arow & 15) == 0, bal = ((uintptr_t)brow & 15) == 0,
             b2al = ((uintptr_t)b2row & 15) == 0;
  auto ld2 = [](const float2 *row, bool al, int64_t k) {
    if (al) return *(const float4 *)(row + k);
    const float2 a = row[k], b = row[k + 1];
    return float4{a.x, a.y, b.x, b.y};
  };
  float4 ra[4], rb[4], rb2[4];
  // K is even and every chunk boundary even, so a pair is in range as a whole
  auto fetch = [&](int64_t k0) {   // k0 < ke, so k0 is a valid index
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + 2 * (lq + 4 * u);
      const bool ok = k < ke;
      const int64_t kk = ok ? k : k0;
      const float4 x = ld2(arow, aal, kk), y = ld2(brow, bal, kk);
      ra[u] = (aval && ok) ? x : float4{0, 0, 0, 0};
      rb[u] = (bval && ok) ? y : float4{0, 0, 0, 0};
      if (two) {
        const float4 w = ld2(b2row, b2al, kk);
        rb2[u] = (bval && ok) ? w : float4{0, 0, 0, 0};
      }
    }
  };
  // planes at byte offsets 0 (re hi), 64 (re lo), 128 (im hi), 192 (im lo)
  auto stage = [&](unsigned char *T_, const float4 (&v)[4]) {
    f8 xr, xi;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      xr[2 * u] = v[u].x;
      xi[2 * u] = v[u].y;
      xr[2 * u + 1] = v[u].z;
      xi[2 * u + 1] = v[u].w;
    }
    const bf8 rh = __builtin_convertvector(xr, bf8);
    const bf8 rl = __builtin_convertvector(xr - __builtin_convertvector(rh, f8), bf8);
    const bf8 ih = __builtin_convertvector(xi, bf8);
    const bf8 il = __builtin_convertvector(xi - __builtin_convertvector(ih, f8), bf8);
    unsigned char *p = T_ + lrow * kBfRow + lq * 16;
    *(bf8 *)p = rh;
    *(bf8 *)(p + kBfPlane) = rl;
    *(bf8 *)(p + 2 * kBfPlane) = ih;
    *(bf8 *)(p + 3 * kBfPlane) = il;
  };
  auto frag = [&](const unsigned char *T_, int row, bf8 (&f)[4]) {
    const unsigned char *p = T_ + row * kBfRow + (lane >> 4) * 16;
#pragma unroll
    for (int q = 0; q < 4; ++q) f[q] = *(const bf8 *)(p + q * kBfPlane);
  };
  // acc += x y over the step, x = xh + xl and y = yh + yl: small terms first
  auto prod = [&](f4 (&acc)[2][2], const bf8 (&x)[2][4], int px, const bf8 (&y)[2][4], int py) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[i][px + 1], y[j][py], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[i][px], y[j][py + 1], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x[i][px], y[j][py], acc[i][j], 0, 0, 0);
  };
  if (kb < ke) fetch(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kBfKT) {
    stage(As, ra);
    stage(Bs, rb);
    if (two) stage(B2s, rb2);
    __syncthreads();
    if (k0 + kBfKT < ke) fetch(k0 + kBfKT);
    // a[i] = [re hi, re lo, im hi, im lo], an[i] = [-im hi, -im lo] (slots 2, 3 unused)
    bf8 a[2][4], an[2][4], b[2][4], c[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      frag(As, wm + i * 16 + (lane & 15), a[i]);
      an[i][0] = bf_neg(a[i][2]);
      an[i][1] = bf_neg(a[i][3]);
      frag(Bs, wn + i * 16 + (lane & 15), b[i]);
      if (two) frag(B2s, wn + i * 16 + (lane & 15), c[i]);
    }
    // conj(a) b: re += ar br + ai bi, im += ar bi - ai br
    prod(re, a, 0, b, 0);
    prod(im, a, 0, b, 2);
    prod(re, a, 2, b, 2);
    prod(im, an, 0, b, 0);
    if (two) {
      prod(re2, a, 0, c, 0);
      prod(im2, a, 0, c, 2);
      prod(re2, a, 2, c, 2);
      prod(im2, an, 0, c, 0);
    }
    __syncthreads();
  }
  double2 *p1 = part + (size_t)z * M * Nn;
  double2 *p2 = two ? part2 + (size_t)z * M * Nn : nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // lane l, slot v holds D[4 (l / 16) + v][l % 16]
        const int r = tm0 + wm + i * 16 + 4 * (lane >> 4) + v;
        const int c = tn0 + wn + j * 16 + (lane & 15);
        if (r < M && c < Nn) {
          p1[(size_t)r * Nn + c] = make_double2((double)re[i][j][v], (double)im[i][j][v]);
          if (two) p2[(size_t)r * Nn + c] = make_double2((double)re2[i][j][v], (double)im2[i][j][v]);
        }
      }
}

void gemm_ip_bf16(const float2 *A, const int64_t *aoff, int M, const float2 *B, const int64_t *boff,
                  int Nn, const float2 *B2, int64_t K, double2 *out, double2 *out2, int ldo,
                  DevBuf &part, hipStream_t st, bool hermitian) {
  if (M <= 0 || Nn <= 0) return;
  DKS_REQUIRE(K % 2 == 0, DKS_EINVAL, "BF16 Gram product: the row length must be even");
  const IpShape g = ip_shape(M, Nn, K, hermitian, kBfBlocks);
  const int tm = g.tm, tiles = g.tiles;
  const bool upper = g.upper;
  const int64_t nsplit = g.nsplit, kchunk = g.kchunk;
  part.ensure(sizeof(double2) * gemm_ip_part_elems(M, Nn, K, B2 != nullptr, hermitian, kBfBlocks));
  double2 *p1 = part.as<double2>();
  double2 *p2 = B2 ? p1 + (size_t)nsplit * M * Nn : nullptr;
  dim3 grid((unsigned)(tiles * nsplit));
  DKS_LAUNCH("k_gemm_ip.gram.bf16", k_gemm_ip_bf16, grid, dim3(256), 0, st, A, aoff, M, B, boff, Nn,
             B2, K, kchunk, tm, (int)upper, tiles, (int)nsplit, p1, p2);
  DKS_HIP(hipGetLastError());
  reduce_parts(p1, p2, (int)nsplit, M, Nn, upper, out, out2, ldo, st);
}

template void gemm_ip<double>(const double2 *, const int64_t *, int, const double2 *,
                              const int64_t *, int, const double2 *, int64_t, double2 *,
                              double2 *, int, DevBuf &, hipStream_t, bool, const int *);
template void gemm_ip<float>(const float2 *, const int64_t *, int, const float2 *,
                             const int64_t *, int, const float2 *, int64_t, double2 *, double2 *,
                             int, DevBuf &, hipStream_t, bool, const int *);
template void gemm_ip_raw<double>(const double2 *, const int64_t *, int, const double2 *,
                                  const int64_t *, int, const double2 *, int64_t, double2 *,
                                  double2 *, int, double2 *, hipStream_t, bool, const int *, int);
template void gemm_ip_raw<float>(const float2 *, const int64_t *, int, const float2 *,
                                 const int64_t *, int, const float2 *, int64_t, double2 *,
                                 double2 *, int, double2 *, hipStream_t, bool, const int *, int);

// ---------------------------------------------------------------------------
// block update
// ---------------------------------------------------------------------------
constexpr int kUpICH = 64;   // rows of V staged in LDS at a time

// Block update out_j[k] = sum_i V[i][j] A_i[k] (+ beta out_j[k]) on the matrix
// cores: out (n x K) = V^T (n x m) A (m x K) as
// 16 x 16 x 4 products, V^T the left operand (rows j, reduction over i) and the
// rows of A the right one.  A workgroup of 8 waves covers kUpMK k values of
// kUpMJ columns j: each wave 3 j-tiles x kUpKT k-tile of 16, complex as four
// real products.  One k-tile per wave keeps a wave at <= 80 VGPRs, so that
// three workgroups (six waves per SIMD) share a CU, which the LDS also allows
// (FP64 V chunks of 48 KB); two k-tiles per wave ran at two waves per SIMD in
// FP64 and were 22 % slower.  V comes through LDS in chunks of kUpICH rows;
// the A fragments of the next 4-row step are fetched while the current one is
// multiplied.
constexpr int kUpMJ = 48;
constexpr int kUpMK = 128;
constexpr int kUpKT = 1;
constexpr int kUpThreads = 64 * kUpMK / (16 * kUpKT);
constexpr int kUpWaves = 6;   // minimum waves per SIMD asked of the compiler

template <typename T>
__global__ void __launch_bounds__(kUpThreads, kUpWaves) k_gemm_up_mfma(const typename CT<T>::c *__restrict__ A1,
                                                      const typename CT<T>::c *__restrict__ A2,
                                                      const int64_t *__restrict__ aoff, int m,
                                                      const double2 *__restrict__ V, int ldv,
                                                      int n, int64_t K,
                                                      typename CT<T>::c *__restrict__ out1,
                                                      typename CT<T>::c *__restrict__ out2,
                                                      int64_t ldo, T beta, double alpha,
                                                      const int *__restrict__ skip) {
  if (skip && *skip) return;   // a finished system of a graph-captured batch

  using C = typename CT<T>::c;
  // blockIdx.z selects one of two products with the same V (X and H X alike)
  const typename CT<T>::c *__restrict__ A = blockIdx.z ? A2 : A1;
  typename CT<T>::c *__restrict__ out = blockIdx.z ? out2 : out1;
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  __shared__ T Vr[kUpICH * kUpMJ], Vi[kUpICH * kUpMJ];
  __shared__ int64_t offs[kUpICH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int KT = kUpKT;
  const int j0 = blockIdx.y * kUpMJ;
  const int64_t k0 = (int64_t)blockIdx.x * kUpMK + wave * 16 * KT;
  const int li = lane >> 4, lc = lane & 15;
  acc_t re[3][KT], im[3][KT];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < KT; ++b) {
      re[a][b] = acc_t{0, 0, 0, 0};
      im[a][b] = acc_t{0, 0, 0, 0};
    }
  for (int i0 = 0; i0 < m; i0 += kUpICH) {
    const int ic = min(kUpICH, m - i0);
    for (int e = tid; e < kUpICH * kUpMJ; e += blockDim.x) {
      const int ii = e / kUpMJ, jj = e - (e / kUpMJ) * kUpMJ;
      const double2 v = (ii < ic && j0 + jj < n) ? V[(size_t)(i0 + ii) * ldv + j0 + jj] : make_double2(0, 0);
      Vr[e] = (T)(alpha * v.x);
      Vi[e] = (T)(alpha * v.y);
    }
    for (int e = tid; e < kUpICH; e += blockDim.x)
      offs[e] = (e < ic) ? (aoff ? aoff[i0 + e] : (int64_t)(i0 + e) * K) : 0;
    __syncthreads();
    // A fragments of 4-row step s: row ii = 4 s + li, columns k0 + 16 kt + lc
    C fa[KT], nx[KT];
    auto fetch = [&](int st, C *f) {
      const int ii = 4 * st + li;
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        const int64_t k = k0 + 16 * kt + lc;
        f[kt] = (ii < ic && k < K) ? A[offs[ii] + k] : C{0, 0};
      }
    };
    const int nst = (ic + 3) / 4;
    fetch(0, fa);
    for (int st = 0; st < nst; ++st) {
      if (st + 1 < nst) fetch(st + 1, nx);
      const int ii = 4 * st + li;
#pragma unroll
      for (int jt = 0; jt < 3; ++jt) {
        const T vr = Vr[ii * kUpMJ + jt * 16 + lc], vi = Vi[ii * kUpMJ + jt * 16 + lc];
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          // v a: re += vr ar - vi ai, im += vr ai + vi ar
          re[jt][kt] = MF::mma(vr, fa[kt].x, re[jt][kt]);
          im[jt][kt] = MF::mma(vr, fa[kt].y, im[jt][kt]);
          re[jt][kt] = MF::mma(-vi, fa[kt].y, re[jt][kt]);
          im[jt][kt] = MF::mma(vi, fa[kt].x, im[jt][kt]);
        }
      }
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) fa[kt] = nx[kt];
    }
    __syncthreads();
  }
#pragma unroll
  for (int jt = 0; jt < 3; ++jt)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + jt * 16 + MF::row(lane, v);
        const int64_t k = k0 + 16 * kt + lc;
        if (j < n && k < K) {
          C *o = out + (size_t)j * ldo + k;
          C r{(T)re[jt][kt][v], (T)im[jt][kt][v]};
          if (beta != T(0)) {
            const C ov = *o;
            r.x += beta * ov.x;
            r.y += beta * ov.y;
          }
          *o = r;
        }
      }
}

template <typename T>
void gemm_up(const cplx<T> *A, const int64_t *aoff, int m, const double2 *V, int ldv, int n,
             int64_t K, cplx<T> *out, int64_t ldo, double beta, hipStream_t st, double alpha) {
  gemm_up2<T>(A, nullptr, aoff, m, V, ldv, n, K, out, nullptr, ldo, beta, st, alpha, nullptr);
}

template <typename T>
void gemm_up2(const cplx<T> *A1, const cplx<T> *A2, const int64_t *aoff, int m, const double2 *V,
              int ldv, int n, int64_t K, cplx<T> *out1, cplx<T> *out2, int64_t ldo, double beta,
              hipStream_t st, double alpha, const char *tag, const int *skip) {
  if (n <= 0 || K <= 0) return;
  const char *name = tag ? tag : (sizeof(T) == 8 ? "k_gemm_up.f64" : "k_gemm_up.f32");
  const bool two = A2 != nullptr;
  dim3 grid((unsigned)((K + kUpMK - 1) / kUpMK), (n + kUpMJ - 1) / kUpMJ, two ? 2 : 1);
  DKS_LAUNCH(name, k_gemm_up_mfma<T>, grid, dim3(kUpThreads), 0, st, A1, two ? A2 : A1, aoff, m, V,
             ldv, n, K, out1, two ? out2 : out1, ldo, (T)beta, alpha, skip);
  DKS_HIP(hipGetLastError());
}
template void gemm_up<double>(const double2 *, const int64_t *, int, const double2 *, int, int,
                              int64_t, double2 *, int64_t, double, hipStream_t, double);
template void gemm_up<float>(const float2 *, const int64_t *, int, const double2 *, int, int,
                             int64_t, float2 *, int64_t, double, hipStream_t, double);
template void gemm_up2<double>(const double2 *, const double2 *, const int64_t *, int,
                               const double2 *, int, int, int64_t, double2 *, double2 *, int64_t,
                               double, hipStream_t, double, const char *, const int *);
template void gemm_up2<float>(const float2 *, const float2 *, const int64_t *, int, const double2 *,
                              int, int, int64_t, float2 *, float2 *, int64_t, double, hipStream_t,
                              double, const char *, const int *);

// ---------------------------------------------------------------------------
// residuals and norms
// ---------------------------------------------------------------------------
__device__ double block_sum(double v) {
  __shared__ double red[16];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

constexpr int kRedChunk = 8192;

template <typename T>
__global__ void __launch_bounds__(256) k_residual(const typename CT<T>::c *__restrict__ X,
                                                  const typename CT<T>::c *__restrict__ HX,
                                                  const double *__restrict__ lam, int64_t K,
                                                  typename CT<T>::c *__restrict__ R,
                                                  double *__restrict__ part, int nchunk,
                                                  const int *__restrict__ skip) {
  if (skip && *skip) return;   // a finished system of a graph-captured batch
  using C = typename CT<T>::c;
  const int j = blockIdx.y;
  const T l = (T)lam[j];
  const int64_t b = (int64_t)blockIdx.x * kRedChunk;
  const int64_t e = min(K, b + kRedChunk);
  const C *x = X + (size_t)j * K;
  const C *hx = HX + (size_t)j * K;
  C *r = R + (size_t)j * K;
  double s = 0;
  for (int64_t k = b + threadIdx.x; k < e; k += blockDim.x) {
    C xv = x[k], hv = hx[k];
    C rv = C{hv.x - l * xv.x, hv.y - l * xv.y};
    r[k] = rv;
    s += (double)rv.x * rv.x + (double)rv.y * rv.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[(size_t)j * nchunk + blockIdx.x] = s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_norm2(const typename CT<T>::c *__restrict__ X, int64_t K,
                                               double *__restrict__ part, int nchunk) {
  using C = typename CT<T>::c;
  const int j = blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * kRedChunk;
  const int64_t e = min(K, b + kRedChunk);
  const C *x = X + (size_t)j * K;
  double s = 0;
  for (int64_t k = b + threadIdx.x; k < e; k += blockDim.x) {
    C v = x[k];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[(size_t)j * nchunk + blockIdx.x] = s;
}

__global__ void k_sum_rows(const double *__restrict__ part, int n, int nchunk,
                           double *__restrict__ out, const int *__restrict__ skip) {
  if (skip && *skip) return;   // a finished system of a graph-captured batch
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)j * nchunk + c];
  out[j] = s;
}

template <typename T>
void residual(const cplx<T> *X, const cplx<T> *HX, const double *lam, int n, int64_t K,
              cplx<T> *R, double *norm2, DevBuf &part, hipStream_t st, const int *skip) {
  if (n <= 0) return;
  int nchunk = (int)((K + kRedChunk - 1) / kRedChunk);
  part.ensure(sizeof(double) * (size_t)n * nchunk);
  DKS_LAUNCH((sizeof(T) == 8 ? "k_residual.f64" : "k_residual.f32"), k_residual<T>, dim3(nchunk, n), dim3(256), 0, st, X, HX, lam, K, R,
                     part.as<double>(), nchunk, skip);
  DKS_HIP(hipGetLastError());
  DKS_LAUNCH("k_sum_rows", k_sum_rows, dim3((n + 63) / 64), dim3(64), 0, st, part.as<double>(), n,
                     nchunk, norm2, skip);
  DKS_HIP(hipGetLastError());
}
template void residual<double>(const double2 *, const double2 *, const double *, int, int64_t,
                               double2 *, double *, DevBuf &, hipStream_t, const int *);
template void residual<float>(const float2 *, const float2 *, const double *, int, int64_t,
                              float2 *, double *, DevBuf &, hipStream_t, const int *);

template <typename T>
void col_norm2(const cplx<T> *X, int n, int64_t K, double *norm2, DevBuf &part, hipStream_t st) {
  if (n <= 0) return;
  int nchunk = (int)((K + kRedChunk - 1) / kRedChunk);
  part.ensure(sizeof(double) * (size_t)n * nchunk);
  DKS_LAUNCH((sizeof(T) == 8 ? "k_norm2.f64" : "k_norm2.f32"), k_norm2<T>, dim3(nchunk, n), dim3(256), 0, st, X, K, part.as<double>(),
                     nchunk);
  DKS_HIP(hipGetLastError());
  DKS_LAUNCH("k_sum_rows", k_sum_rows, dim3((n + 63) / 64), dim3(64), 0, st, part.as<double>(), n,
                     nchunk, norm2, nullptr);
  DKS_HIP(hipGetLastError());
}
template void col_norm2<double>(const double2 *, int, int64_t, double *, DevBuf &, hipStream_t);
template void col_norm2<float>(const float2 *, int, int64_t, double *, DevBuf &, hipStream_t);

// ---------------------------------------------------------------------------
// gathers, conversions, scaling
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_gather(const typename CT<T>::c *__restrict__ src, const int *__restrict__ idx,
                         int64_t K, typename CT<T>::c *__restrict__ dst) {
  const int i = blockIdx.y;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  dst[(size_t)i * K + k] = src[(size_t)idx[i] * K + k];
}
template <typename T>
void gather_rows(const cplx<T> *src, const int *idx, int m, int64_t K, cplx<T> *dst,
                 hipStream_t st) {
  if (m <= 0) return;
  DKS_LAUNCH((sizeof(T) == 8 ? "k_gather.f64" : "k_gather.f32"), k_gather<T>, dim3((unsigned)((K + 255) / 256), m), dim3(256), 0, st, src, idx,
                     K, dst);
  DKS_HIP(hipGetLastError());
}
template void gather_rows<double>(const double2 *, const int *, int, int64_t, double2 *, hipStream_t);
template void gather_rows<float>(const float2 *, const int *, int, int64_t, float2 *, hipStream_t);

template <typename Ts, typename Td>
__global__ void k_convert(const typename CT<Ts>::c *__restrict__ s, typename CT<Td>::c *__restrict__ d,
                          int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) d[i] = typename CT<Td>::c{(Td)s[i].x, (Td)s[i].y};
}
template <typename Ts, typename Td>
void convert(const cplx<Ts> *src, cplx<Td> *dst, int64_t count, hipStream_t st) {
  if (count <= 0) return;
  DKS_LAUNCH((sizeof(Ts) == 8 ? "k_convert.f64_f32" : "k_convert.f32_f64"), (k_convert<Ts, Td>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                     src, dst, count);
  DKS_HIP(hipGetLastError());
}
template void convert<double, float>(const double2 *, float2 *, int64_t, hipStream_t);
template void convert<float, double>(const float2 *, double2 *, int64_t, hipStream_t);

template <typename T>
__global__ void k_scale_rows(typename CT<T>::c *X, const double *s, int64_t K) {
  const int i = blockIdx.y;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  T f = (T)s[i];
  typename CT<T>::c v = X[(size_t)i * K + k];
  X[(size_t)i * K + k] = typename CT<T>::c{v.x * f, v.y * f};
}
template <typename T>
void scale_rows(cplx<T> *X, const double *s, int n, int64_t K, hipStream_t st) {
  if (n <= 0) return;
  DKS_LAUNCH((sizeof(T) == 8 ? "k_scale_rows.f64" : "k_scale_rows.f32"), k_scale_rows<T>, dim3((unsigned)((K + 255) / 256), n), dim3(256), 0, st, X, s, K);
  DKS_HIP(hipGetLastError());
}
template void scale_rows<double>(double2 *, const double *, int, int64_t, hipStream_t);
template void scale_rows<float>(float2 *, const double *, int, int64_t, hipStream_t);

}  // namespace dks
