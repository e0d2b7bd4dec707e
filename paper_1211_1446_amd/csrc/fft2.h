// In-place two-step FFTs on LDS lines for the local-potential convolution.
//
// A length n = A * B transform is split as
//   inverse (natural k-space -> scrambled real space):
//     step 1  for every b < B: DFT_A over x[b + B a], twiddle w_n^{b k_a},
//             result back at b + B k_a                       (same positions)
//     step 2  for every k_a < A: DFT_B over the contiguous block at B k_a,
//             result X[k_a + A k_b] stored at B k_a + k_b    (same positions)
//   forward (scrambled real space -> natural k-space) undoes the two steps:
//     step 2' DFT_B over the block at B k_a, twiddle w_n^{-b k_a}
//     step 1' DFT_A over y[b + B k_a], result at b + B a.
// Every thread reads and writes only the positions it owns, so no register
// staging is needed across barriers, and the real-space order is a fixed
// permutation that the potential is stored in.  Step 2, the multiplication by
// V(r) and step 2' touch the same block and run fused in registers.
//
// Codelets DFT_R are unrolled at compile time from radix-2/3/4/5 kernels, with
// constant twiddles between the factors, or none when the two factors are
// coprime (prime-factor index maps); R = 1 is the identity (single-step
// transforms, n = B).
#pragma once

#include "dks_internal.h"
#include "fft_device.h"
#include "fft_split.h"

namespace dks {
namespace fft2 {

// ---- compile-time trigonometry (long double series, |error| < 1e-18) -------
constexpr long double kPi = 3.141592653589793238462643383279502884L;
constexpr long double reduce(long double x) {
  while (x > kPi) x -= 2 * kPi;
  while (x < -kPi) x += 2 * kPi;
  return x;
}
constexpr long double csin(long double x) {
  x = reduce(x);
  long double term = x, sum = x;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr long double ccos(long double x) {
  x = reduce(x);
  long double term = 1, sum = 1;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

// multiply v by exp(S 2 pi i m / R) with compile-time m, R
template <int S, int M, int R, typename T, typename C>
__device__ __forceinline__ C twc(C v) {
  constexpr int m = ((M % R) + R) % R;
  if constexpr (m == 0) {
    return v;
  } else if constexpr (4 * m == R) {
    return cmul_si<S>(v);
  } else if constexpr (2 * m == R) {
    return C{-v.x, -v.y};
  } else if constexpr (4 * m == 3 * R) {
    return cmul_si<-S>(v);
  } else {
    constexpr long double ang = 2.0L * kPi * (long double)m / (long double)R;
    constexpr T c = (T)ccos(ang);
    constexpr T s = (T)((long double)S * csin(ang));
    return C{v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

template <int R> struct Split {
  static constexpr int P = (R % 4 == 0 && R > 4) ? 4 : (R % 2 == 0 ? 2 : (R % 3 == 0 ? 3 : 5));
  static constexpr int Q = R / P;
};

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
// the k in [0, P Q) with k = kp (mod P) and k = kq (mod Q), P and Q coprime
constexpr int crt(int kp, int kq, int P, int Q) {
  int k = kq;
  while (k % P != kp) k += Q;
  return k;
}

// y_k = sum_j v_j exp(S 2 pi i j k / R), in place
template <int R, int S, typename T> struct Codelet {
  template <typename C> __device__ __forceinline__ static void run(C *v) {
    if constexpr (R == 1) {
      return;
    } else if constexpr (R == 2 || R == 3 || R == 4 || R == 5) {
      Dft<R, S, T>::run(v);
    } else if constexpr (cgcd(Split<R>::P, Split<R>::Q) == 1) {
      // coprime factors (Good-Thomas): with j = (Q p + P q) mod R and
      // k = crt(kp, kq), j k = Q p kp + P q kq (mod R), so
      // y[crt(kp, kq)] = sum_p w_P^{p kp} sum_q w_Q^{q kq} v[(Q p + P q) mod R]:
      // two passes of short transforms and no twiddle factors in between
      constexpr int P = Split<R>::P, Q = Split<R>::Q;
      C t[R];
#pragma unroll
      for (int p = 0; p < P; ++p) {
        C u[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) u[q] = v[(Q * p + P * q) % R];
        Codelet<Q, S, T>::run(u);
#pragma unroll
        for (int kq = 0; kq < Q; ++kq) t[p * Q + kq] = u[kq];
      }
#pragma unroll
      for (int kq = 0; kq < Q; ++kq) {
        C u[P];
#pragma unroll
        for (int p = 0; p < P; ++p) u[p] = t[p * Q + kq];
        Codelet<P, S, T>::run(u);
#pragma unroll
        for (int kp = 0; kp < P; ++kp) v[crt(kp, kq, P, Q)] = u[kp];
      }
    } else {
      constexpr int P = Split<R>::P, Q = Split<R>::Q;
      C t[R];
      // y[kp + P kq] = sum_q w_Q^{q kq} [ w_R^{q kp} sum_p x[q + Q p] w_P^{p kp} ]
      unroll_q<0, P, Q>(v, t);
#pragma unroll
      for (int kp = 0; kp < P; ++kp) {
        C u[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) u[q] = t[q + Q * kp];
        Codelet<Q, S, T>::run(u);
#pragma unroll
        for (int kq = 0; kq < Q; ++kq) v[kp + P * kq] = u[kq];
      }
    }
  }
  template <int q, int P, int Q, typename C>
  __device__ __forceinline__ static void unroll_q(const C *v, C *t) {
    if constexpr (q < Q) {
      C u[P];
#pragma unroll
      for (int p = 0; p < P; ++p) u[p] = v[q + Q * p];
      Codelet<P, S, T>::run(u);
      unroll_kp<0, q, P, Q>(u, t);
      unroll_q<q + 1, P, Q>(v, t);
    }
  }
  template <int kp, int q, int P, int Q, typename C>
  __device__ __forceinline__ static void unroll_kp(const C *u, C *t) {
    if constexpr (kp < P) {
      t[q + Q * kp] = twc<S, q * kp, R, T>(u[kp]);
      unroll_kp<kp + 1, q, P, Q>(u, t);
    }
  }
};

// ---- line geometry: element e of line l at base(l) + e * stride --------------
struct Lines {
  const int *rows;   // optional list of line indices
  int ld;            // base(l) = (rows ? rows[l] : l) * ld
  int stride;
  __device__ __forceinline__ int base(int l) const { return (rows ? rows[l] : l) * ld; }
};

// A thread's walk over the tasks t = tid, tid + nthr, ... of a step on nl
// lines, task t standing for (outer index t / nl, line t % nl).  The quotient
// and remainder are carried from task to task (one division per walk, none
// per task; an integer division costs some twenty instructions).
struct Walk {
  int nl, q0, r0, dq, dr, tid, nthr;
};
__device__ __forceinline__ Walk walk(int nl, int tid = threadIdx.x, int nthr = blockDim.x) {
  if (nl <= 0) return Walk{nl, 0, 0, 0, 0, tid, nthr};   // no tasks
  const int q0 = tid / nl, dq = nthr / nl;
  return Walk{nl, q0, tid - q0 * nl, dq, nthr - dq * nl, tid, nthr};
}
// runs body(outer, line) over the walk's tasks below `tasks`
template <typename F>
__device__ __forceinline__ void for_tasks(const Walk &w, int tasks, F &&body) {
  int q = w.q0, l = w.r0;
  for (int t = w.tid; t < tasks; t += w.nthr) {
    body(q, l);
    q += w.dq;
    l += w.dr;
    if (l >= w.nl) {
      l -= w.nl;
      ++q;
    }
  }
}

// twiddle w_n^{S e} from the table tw[t] = exp(-2 pi i t / n)
template <int S, typename C>
__device__ __forceinline__ C twt(const C *tw, int e) {
  C w = tw[e];
  if (S > 0) w.y = -w.y;
  return w;
}

// inverse step 1 on nl lines (in place); `w` walks nl lines
template <int A, int B, typename T>
__device__ __forceinline__ void inv_step1(typename CT<T>::c *buf, const Walk &w, Lines L,
                                          const typename CT<T>::c *tw) {
  using C = typename CT<T>::c;
  if constexpr (A > 1) {
    for_tasks(w, w.nl * B, [&](int b, int l) {
      const int base = L.base(l) + b * L.stride;
      C v[A];
#pragma unroll
      for (int a = 0; a < A; ++a) v[a] = buf[base + B * a * L.stride];
      Codelet<A, +1, T>::run(v);
#pragma unroll
      for (int ka = 1; ka < A; ++ka) v[ka] = cmul(v[ka], twt<+1>(tw, b * ka));
#pragma unroll
      for (int a = 0; a < A; ++a) buf[base + B * a * L.stride] = v[a];
    });
  }
}

// forward step 1' on nl lines (in place): DFT_A over k_a, natural output
template <int A, int B, typename T>
__device__ __forceinline__ void fwd_step1(typename CT<T>::c *buf, const Walk &w, Lines L) {
  using C = typename CT<T>::c;
  if constexpr (A > 1) {
    for_tasks(w, w.nl * B, [&](int b, int l) {
      const int base = L.base(l) + b * L.stride;
      C v[A];
#pragma unroll
      for (int a = 0; a < A; ++a) v[a] = buf[base + B * a * L.stride];
      Codelet<A, -1, T>::run(v);
#pragma unroll
      for (int a = 0; a < A; ++a) buf[base + B * a * L.stride] = v[a];
    });
  }
}

// inverse step 2 on the blocks (in place)
template <int A, int B, typename T>
__device__ __forceinline__ void inv_step2(typename CT<T>::c *buf, const Walk &w, Lines L) {
  using C = typename CT<T>::c;
  for_tasks(w, w.nl * A, [&](int ka, int l) {
    const int base = L.base(l) + B * ka * L.stride;
    C v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = buf[base + b * L.stride];
    Codelet<B, +1, T>::run(v);
#pragma unroll
    for (int b = 0; b < B; ++b) buf[base + b * L.stride] = v[b];
  });
}

// forward step 2' on the blocks (in place), including the w_n^{-b k_a} twiddle
template <int A, int B, typename T>
__device__ __forceinline__ void fwd_step2(typename CT<T>::c *buf, const Walk &w, Lines L,
                                          const typename CT<T>::c *tw) {
  using C = typename CT<T>::c;
  for_tasks(w, w.nl * A, [&](int ka, int l) {
    const int base = L.base(l) + B * ka * L.stride;
    C v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = buf[base + b * L.stride];
    Codelet<B, -1, T>::run(v);
    if constexpr (A > 1) {
#pragma unroll
      for (int b = 1; b < B; ++b) v[b] = cmul(v[b], twt<-1>(tw, b * ka));
    }
#pragma unroll
    for (int b = 0; b < B; ++b) buf[base + b * L.stride] = v[b];
  });
}

// inverse step 2, x V (scrambled layout, element-wise), forward step 2' fused.
// V for line l, position p is Vp[l * vls + p * vps].
template <int A, int B, typename T>
__device__ __forceinline__ void inv2_mul_fwd2(typename CT<T>::c *buf, const Walk &w, Lines L,
                                              const typename CT<T>::c *tw, const T *__restrict__ Vp,
                                              int vls, int vps) {
  using C = typename CT<T>::c;
  for_tasks(w, w.nl * A, [&](int ka, int l) {
    const int base = L.base(l) + B * ka * L.stride;
    const T *vl = Vp + (size_t)l * vls + (size_t)(B * ka) * vps;
    C v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = buf[base + b * L.stride];
    Codelet<B, +1, T>::run(v);
#pragma unroll
    for (int b = 0; b < B; ++b) {
      T s = vl[(size_t)b * vps];
      v[b] = C{v[b].x * s, v[b].y * s};
    }
    Codelet<B, -1, T>::run(v);
    if constexpr (A > 1) {
#pragma unroll
      for (int b = 1; b < B; ++b) v[b] = cmul(v[b], twt<-1>(tw, b * ka));
    }
#pragma unroll
    for (int b = 0; b < B; ++b) buf[base + b * L.stride] = v[b];
  });
}

// Steps that touch only part of a line.  `keep[e]` (LDS) is nonzero for the
// natural-order elements e that carry data: the inverse step 1 reads those and
// takes the others as zero (they are never written before it), and writes the
// whole line; the forward step 1' writes only those (the others are not read
// again).  With A = 1 the inverse form still clears the rest of the line.
template <int A, int B, typename T>
__device__ __forceinline__ void inv_step1_keep(typename CT<T>::c *buf, const Walk &w, Lines L,
                                               const typename CT<T>::c *tw, const int *keep) {
  using C = typename CT<T>::c;
  for_tasks(w, w.nl * B, [&](int b, int l) {
    const int base = L.base(l) + b * L.stride;
    int kb[A];
#pragma unroll
    for (int a = 0; a < A; ++a) kb[a] = keep[b + B * a];   // all flags first: no wait between reads
    C v[A];
#pragma unroll
    for (int a = 0; a < A; ++a) {
      v[a] = C{0, 0};
      if (kb[a]) v[a] = buf[base + B * a * L.stride];
    }
    if constexpr (A > 1) {
      Codelet<A, +1, T>::run(v);
#pragma unroll
      for (int ka = 1; ka < A; ++ka) v[ka] = cmul(v[ka], twt<+1>(tw, b * ka));
    }
#pragma unroll
    for (int a = 0; a < A; ++a) buf[base + B * a * L.stride] = v[a];
  });
}
template <int A, int B, typename T>
__device__ __forceinline__ void fwd_step1_keep(typename CT<T>::c *buf, const Walk &w, Lines L,
                                               const int *keep) {
  using C = typename CT<T>::c;
  if constexpr (A > 1) {
    for_tasks(w, w.nl * B, [&](int b, int l) {
      const int base = L.base(l) + b * L.stride;
      int kb[A];
      C v[A];
#pragma unroll
      for (int a = 0; a < A; ++a) kb[a] = keep[b + B * a];
#pragma unroll
      for (int a = 0; a < A; ++a) v[a] = buf[base + B * a * L.stride];
      Codelet<A, -1, T>::run(v);
#pragma unroll
      for (int a = 0; a < A; ++a)
        if (kb[a]) buf[base + B * a * L.stride] = v[a];
    });
  }
}

// Steps 1 and 1' of the sphere rows against global memory.  Row r of the
// plane holds, at n2 slot p, column ctab[r n2 + p] of the plane's column
// values `t` (-1: no column, zero).  Tasks run b fastest, so that the lanes of
// a wave read and write neighbouring slots of one row.  The inverse step
// writes whole rows to the LDS plane at row_of(r) * ld; the forward step reads
// them there and stores the column slots only.  Loads are unconditional (a
// missing column reads column 0 and is replaced by zero), so that all of a
// task's loads are in flight together.
template <int A, int B, typename T>
__device__ __forceinline__ void inv_step1_rows_in(typename CT<T>::c *pl, int ld, const int *rows,
                                                  int nrows, int n2, const int *__restrict__ ctab,
                                                  const typename CT<T>::c *t,
                                                  const typename CT<T>::c *tw) {
  using C = typename CT<T>::c;
  for_tasks(walk(B), nrows * B, [&](int r, int b) {
    const int *cr = ctab + (size_t)r * n2 + b;
    const int row = rows[r];
    int c[A];
#pragma unroll
    for (int a = 0; a < A; ++a) c[a] = cr[B * a];
    C v[A];
#pragma unroll
    for (int a = 0; a < A; ++a) v[a] = t[c[a] > 0 ? c[a] : 0];
#pragma unroll
    for (int a = 0; a < A; ++a)
      if (c[a] < 0) v[a] = C{0, 0};
    if constexpr (A > 1) {
      Codelet<A, +1, T>::run(v);
#pragma unroll
      for (int ka = 1; ka < A; ++ka) v[ka] = cmul(v[ka], twt<+1>(tw, b * ka));
    }
    C *dst = pl + row * ld + b;
#pragma unroll
    for (int a = 0; a < A; ++a) dst[B * a] = v[a];
  });
}
template <int A, int B, typename T>
__device__ __forceinline__ void fwd_step1_rows_out(const typename CT<T>::c *pl, int ld,
                                                   const int *rows, int nrows, int n2,
                                                   const int *__restrict__ ctab,
                                                   typename CT<T>::c *t) {
  using C = typename CT<T>::c;
  for_tasks(walk(B), nrows * B, [&](int r, int b) {
    const int *cr = ctab + (size_t)r * n2 + b;
    int c[A];
#pragma unroll
    for (int a = 0; a < A; ++a) c[a] = cr[B * a];   // in flight during the LDS reads
    const C *src = pl + rows[r] * ld + b;
    C v[A];
#pragma unroll
    for (int a = 0; a < A; ++a) v[a] = src[B * a];
    if constexpr (A > 1) Codelet<A, -1, T>::run(v);
#pragma unroll
    for (int a = 0; a < A; ++a)
      if (c[a] >= 0) t[c[a]] = v[a];
  });
}

// ---- supported lengths and their (A, B) split --------------------------------
// Plane axes (n <= 128) and z lines (n <= 400) have separate tables so that the
// register budget of each kernel is set by its own largest codelet.  Returns
// false for lengths without a compiled split (the caller falls back).
#define DKS_FFT_PLANE_CASES(X)                                                              \
  X(8, 1, 8) X(9, 1, 9) X(10, 1, 10) X(12, 1, 12) X(15, 1, 15) X(16, 1, 16) X(18, 3, 6)      \
  X(20, 4, 5) X(24, 4, 6) X(25, 5, 5) X(27, 3, 9) X(30, 5, 6) X(32, 4, 8) X(36, 6, 6)        \
  X(40, 5, 8) X(45, 5, 9) X(48, 6, 8) X(50, 5, 10) X(54, 6, 9) X(60, 6, 10) X(64, 8, 8)      \
  X(72, 8, 9) X(75, 5, 15) X(80, 8, 10) X(90, 9, 10) X(96, 8, 12) X(100, 10, 10)            \
  X(120, 10, 12) X(128, 8, 16)
#define DKS_FFT_Z_CASES(X)                                                                  \
  DKS_FFT_PLANE_CASES(X) X(144, 12, 12) X(160, 10, 16) X(180, 12, 15) X(192, 12, 16)        \
  X(200, 10, 20) X(240, 15, 16) X(256, 16, 16) X(288, 16, 18) X(320, 16, 20) X(360, 18, 20) \
  X(400, 20, 20)

// The plane lengths whose two factors are both at most 8: a kernel that
// dispatches only these holds the registers of its own codelets, not of the
// 9- to 16-point ones (fewer VGPRs, more waves per SIMD).
#define DKS_FFT_PLANE_LITE_CASES(X)                                                          \
  X(8, 1, 8) X(18, 3, 6) X(20, 4, 5) X(24, 4, 6) X(25, 5, 5) X(30, 5, 6) X(32, 4, 8)        \
  X(36, 6, 6) X(40, 5, 8) X(48, 6, 8) X(64, 8, 8)

#define DKS_FFT_CASE(N_, A_, B_)     \
  case N_:                           \
    f.template operator()<A_, B_>(); \
    return true;

#define DKS_FFT_HAS(N_, A_, B_) case N_:
// whether plane axis length n has a compiled split (host and device)
__host__ __device__ constexpr bool plane_has(int n) {
  switch (n) {
    DKS_FFT_PLANE_CASES(DKS_FFT_HAS)
    return true;
    default:
      return false;
  }
}
// whether plane axis length n is one of the lite lengths (host and device)
__host__ __device__ constexpr bool plane_lite_has(int n) {
  switch (n) {
    DKS_FFT_PLANE_LITE_CASES(DKS_FFT_HAS)
    return true;
    default:
      return false;
  }
}
// whether z length n has a compiled split (host and device)
__host__ __device__ constexpr bool z_has(int n) {
  switch (n) {
    DKS_FFT_Z_CASES(DKS_FFT_HAS)
    return true;
    default:
      return false;
  }
}
#undef DKS_FFT_HAS

template <typename F>
__device__ __forceinline__ bool dispatch_plane(int n, F &&f) {
  switch (n) {
    DKS_FFT_PLANE_CASES(DKS_FFT_CASE)
    default:
      return false;
  }
}
template <typename F>
__device__ __forceinline__ bool dispatch_plane_lite(int n, F &&f) {
  switch (n) {
    DKS_FFT_PLANE_LITE_CASES(DKS_FFT_CASE)
    default:
      return false;
  }
}
template <typename F>
__device__ __forceinline__ bool dispatch_z(int n, F &&f) {
  switch (n) {
    DKS_FFT_Z_CASES(DKS_FFT_CASE)
    default:
      return false;
  }
}
#undef DKS_FFT_CASE

}  // namespace fft2
}  // namespace dks
