// Batched mixed-radix Stockham FFT passes on lines held in LDS.
//
// A "line" is n complex values at LDS offsets base(l) + e * stride.  Every
// pass of radix R reads the R inputs of each butterfly into registers, waits
// for the whole workgroup, then writes the R outputs: the transform runs in
// place, so a 96 x 96 FP64 plane (147 KB) fits the 160 KB LDS of a CU.
// Twiddles come from a table tw[t] = exp(-2 pi i t / n) built on the host in
// extended precision; the inverse transform uses their conjugates.
#pragma once

#include "dks_internal.h"

namespace dks {

template <typename T> struct CT;
template <> struct CT<double> {
  using c = double2;
  __device__ static c mk(double r, double i) { return make_double2(r, i); }
};
template <> struct CT<float> {
  using c = float2;
  __device__ static c mk(float r, float i) { return make_float2(r, i); }
};

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by s*i (s = +1 or -1)
template <int S, typename C> __device__ __forceinline__ C cmul_si(C a) {
  return S > 0 ? C{-a.y, a.x} : C{a.y, -a.x};
}
template <typename C, typename T> __device__ __forceinline__ C cscale(C a, T s) { return C{a.x * s, a.y * s}; }

// y_k = sum_j a_j exp(S 2 pi i j k / R), in place on v[0..R)
template <int R, int S, typename T> struct Dft;

template <int S, typename T> struct Dft<2, S, T> {
  template <typename C> __device__ static void run(C *v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};
template <int S, typename T> struct Dft<3, S, T> {
  template <typename C> __device__ static void run(C *v) {
    const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
    C t = cadd(v[1], v[2]);
    C u = cmul_si<S>(cscale(csub(v[1], v[2]), h));
    C m = C{v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, u);
    v[2] = csub(m, u);
  }
};
template <int S, typename T> struct Dft<4, S, T> {
  template <typename C> __device__ static void run(C *v) {
    C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    C t2 = cadd(v[1], v[3]), t3 = cmul_si<S>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};
template <int S, typename T> struct Dft<5, S, T> {
  template <typename C> __device__ static void run(C *v) {
    const T c1 = T(0.30901699437494742410229341718282);   // cos(2pi/5)
    const T c2 = T(-0.80901699437494742410229341718282);  // cos(4pi/5)
    const T s1 = T(0.95105651629515357211643933337938);   // sin(2pi/5)
    const T s2 = T(0.58778525229247312916870595463907);   // sin(4pi/5)
    C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    C t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    C b1 = C{v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
    C b2 = C{v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
    C d1 = cmul_si<S>(C{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y});
    C d2 = cmul_si<S>(C{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y});
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(b1, d1);
    v[4] = csub(b1, d1);
    v[2] = cadd(b2, d2);
    v[3] = csub(b2, d2);
  }
};
template <int S, typename T> struct Dft<6, S, T> {
  template <typename C> __device__ static void run(C *v) {
    C e[3] = {v[0], v[2], v[4]};
    C o[3] = {v[1], v[3], v[5]};
    Dft<3, S, T>::run(e);
    Dft<3, S, T>::run(o);
    const T h = T(0.86602540378443864676372317075294);
    // w6 = 1/2 + S i sqrt(3)/2, w6^2 = -1/2 + S i sqrt(3)/2
    C w1 = C{T(0.5), T(S) * h}, w2 = C{T(-0.5), T(S) * h};
    C o1 = cmul(o[1], w1), o2 = cmul(o[2], w2);
    v[0] = cadd(e[0], o[0]);
    v[3] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[4] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[5] = csub(e[2], o2);
  }
};
template <int S, typename T> struct Dft<8, S, T> {
  template <typename C> __device__ static void run(C *v) {
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, S, T>::run(e);
    Dft<4, S, T>::run(o);
    const T r = T(0.70710678118654752440084436210485);
    // w8 = (1 + S i)/sqrt2, w8^2 = S i, w8^3 = (-1 + S i)/sqrt2
    C o1 = cmul(o[1], C{r, T(S) * r});
    C o2 = cmul_si<S>(o[2]);
    C o3 = cmul(o[3], C{-r, T(S) * r});
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// Elements of one pass that a thread may hold; the host checks
// nlines * n <= kMaxElems * blockDim.x for every transform it launches.
constexpr int kMaxElems = 16;

// One Stockham pass of radix R over `nlines` lines (in place, register staged).
// S = -1: forward exp(-i...), S = +1: inverse exp(+i...).
template <int R, int S, typename T>
__device__ void fft_pass(typename CT<T>::c *buf, int nlines, const int *rowlist, int ld,
                         int stride, int n, int Ns, const typename CT<T>::c *tw) {
  using C = typename CT<T>::c;
  constexpr int MB = (kMaxElems + R - 1) / R;
  const int nb = n / R;
  const int total = nlines * nb;
  const int nt = blockDim.x;
  const int tstep = n / (Ns * R);
  C v[MB][R];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    int bi = threadIdx.x + b * nt;
    if (bi < total) {
      int line = bi / nb, j = bi - (bi / nb) * nb;
      int base = (rowlist ? rowlist[line] : line) * ld;
      int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[base + (j + r * nb) * stride];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = tw[r * k * tstep];
        if (S > 0) w.y = -w.y;
        v[b][r] = cmul(v[b][r], w);
      }
      Dft<R, S, T>::run(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    int bi = threadIdx.x + b * nt;
    if (bi < total) {
      int line = bi / nb, j = bi - (bi / nb) * nb;
      int base = (rowlist ? rowlist[line] : line) * ld;
      int k = j % Ns;
      int o = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + (o + r * Ns) * stride] = v[b][r];
    }
  }
  __syncthreads();
}

// Full 1D transform of length plan.n on every line (natural order in and
// out), lines processed in chunks that fit kMaxElems per thread.  Caller
// synchronises before.
template <int S, typename T>
__device__ void fft_lines(typename CT<T>::c *buf, int nlines, const int *rowlist, int ld,
                          int stride, const FftPlan &plan, const typename CT<T>::c *tw) {
  const int chunk = max(1, (int)(kMaxElems * blockDim.x) / plan.n);
  for (int l0 = 0; l0 < nlines; l0 += chunk) {
    const int nl = min(chunk, nlines - l0);
    const int *rl = rowlist ? rowlist + l0 : nullptr;
    typename CT<T>::c *bb = rowlist ? buf : buf + (size_t)l0 * ld;
    int Ns = 1;
    for (int p = 0; p < plan.npass; ++p) {
      int R = plan.radix[p];
      switch (R) {
        case 8: fft_pass<8, S, T>(bb, nl, rl, ld, stride, plan.n, Ns, tw); break;
        case 6: fft_pass<6, S, T>(bb, nl, rl, ld, stride, plan.n, Ns, tw); break;
        case 5: fft_pass<5, S, T>(bb, nl, rl, ld, stride, plan.n, Ns, tw); break;
        case 4: fft_pass<4, S, T>(bb, nl, rl, ld, stride, plan.n, Ns, tw); break;
        case 3: fft_pass<3, S, T>(bb, nl, rl, ld, stride, plan.n, Ns, tw); break;
        default: fft_pass<2, S, T>(bb, nl, rl, ld, stride, plan.n, Ns, tw); break;
      }
      Ns *= R;
    }
  }
}

}  // namespace dks
