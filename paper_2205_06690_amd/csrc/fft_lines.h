// Small-radix DFT codelets and LDS line transforms for gfx950.
//
// A line of length N = N1*N2 is transformed in three stages on data held in
// LDS (the four-step factorisation, index j = j1*N2 + j2, k = k1 + N1*k2):
//   stage A  (per j2): DFT_N1 over j1, times twiddle w_N^(j2*k1); the result
//            for k1 is written to slot k1*N2 + j2.
//   stage B  (per k1): the N2 values in slots k1*N2 + [0, N2) get DFT_N2,
//            giving X[k1 + N1*k2] in slot k1*N2 + k2 ("scrambled" order);
//            optionally a diagonal multiplier and the inverse DFT_N2 follow
//            in registers, then the conjugate twiddle.
//   stage C  (per j2): inverse DFT_N1 over k1 back to natural order.
// A forward transform leaves the spectrum scrambled (stage A + forward half
// of B); an inverse takes scrambled input (inverse half of B + C); the
// kinetic propagator exp(-i k^2 dt/2) along one axis is A + full B + C with
// the phase applied between the two register DFTs, so it costs two LDS
// exchanges and never leaves registers between the forward and inverse
// halves.
#pragma once
#include <hip/hip_runtime.h>

namespace bse {

// ---------------------------------------------------------------- complex
template <typename T> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename T> using cplx = typename cplx_t<T>::type;

template <typename C> __device__ __forceinline__ C cmk(decltype(C::x) a, decltype(C::x) b) {
  C r; r.x = a; r.y = b; return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return cmk<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return cmk<C>(a.x * s, a.y * s); }
// multiply by DIR * i
template <int DIR, typename C> __device__ __forceinline__ C cmul_i(C a) {
  return DIR > 0 ? cmk<C>(-a.y, a.x) : cmk<C>(a.y, -a.x);
}

// ------------------------------------------------- compile-time twiddles
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int i = 1; i < 24; ++i) { term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i)); sum += term; }
  return sum;
}
constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int i = 1; i < 24; ++i) { term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0)); sum += term; }
  return sum;
}
// cos(2 pi m / R), sin(2 pi m / R); exact at quarter turns
constexpr double tw_cos(int m, int R) {
  m = ((m % R) + R) % R;
  if ((4 * m) % R == 0) { int q = 4 * m / R; return q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0); }
  double a = 2.0 * kPi * m / R;
  if (a > kPi) a -= 2.0 * kPi;
  return taylor_cos(a);
}
constexpr double tw_sin(int m, int R) {
  m = ((m % R) + R) % R;
  if ((4 * m) % R == 0) { int q = 4 * m / R; return q == 1 ? 1.0 : (q == 3 ? -1.0 : 0.0); }
  double a = 2.0 * kPi * m / R;
  if (a > kPi) a -= 2.0 * kPi;
  return taylor_sin(a);
}
template <int R> struct TwTab {
  double c[R > 0 ? R : 1];
  double s[R > 0 ? R : 1];
  constexpr TwTab() : c(), s() {
    for (int m = 0; m < R; ++m) { c[m] = tw_cos(m, R); s[m] = tw_sin(m, R); }
  }
};
template <int R> struct TwConst { static constexpr TwTab<R> t{}; };

// w_R^(DIR*m) = cos(2 pi m/R) + DIR i sin(2 pi m/R), applied to a
template <int R, int DIR, typename C> __device__ __forceinline__ C twiddle_const(C a, int m) {
  using T = decltype(C::x);
  const int mm = ((m % R) + R) % R;
  const T c = (T)TwConst<R>::t.c[mm];
  const T s = (T)(DIR * TwConst<R>::t.s[mm]);
  if ((4 * mm) % R == 0) {
    const int q = 4 * mm / R;
    if (q == 0) return a;
    if (q == 2) return cmk<C>(-a.x, -a.y);
    return (q == 1) == (DIR > 0) ? cmk<C>(-a.y, a.x) : cmk<C>(a.y, -a.x);
  }
  return cmk<C>(a.x * c - a.y * s, a.x * s + a.y * c);
}

// ------------------------------------------------------------ codelets
// In-register DFT of length R, X_k = sum_j x_j w_R^(DIR j k), natural order.
template <int R, int DIR, typename C> struct Dft;

template <int DIR, typename C> struct Dft<1, DIR, C> {
  static __device__ __forceinline__ void run(C*) {}
};
template <int DIR, typename C> struct Dft<2, DIR, C> {
  static __device__ __forceinline__ void run(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
  }
};
template <int DIR, typename C> struct Dft<4, DIR, C> {
  static __device__ __forceinline__ void run(C* v) {
    C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    C s13 = cadd(v[1], v[3]), d13 = cmul_i<DIR>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13); v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13); v[3] = csub(d02, d13);
  }
};
// odd prime lengths: pair j with R - j
template <int R, int DIR, typename C> struct DftOdd {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(C::x);
    constexpr int H = (R - 1) / 2;
    C sp[H], sm[H];
#pragma unroll
    for (int j = 1; j <= H; ++j) { sp[j - 1] = cadd(v[j], v[R - j]); sm[j - 1] = csub(v[j], v[R - j]); }
    C x0 = v[0];
    C tot = x0;
#pragma unroll
    for (int j = 0; j < H; ++j) tot = cadd(tot, sp[j]);
    v[0] = tot;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      C a = x0, b = cmk<C>(0, 0);
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const T c = (T)TwConst<R>::t.c[(j * k) % R];
        const T s = (T)TwConst<R>::t.s[(j * k) % R];
        a = cadd(a, cscale(sp[j - 1], c));
        b = cadd(b, cscale(sm[j - 1], s));
      }
      C ib = cmul_i<DIR>(b);
      v[k] = cadd(a, ib);
      v[R - k] = csub(a, ib);
    }
  }
};
template <int DIR, typename C> struct Dft<3, DIR, C> : DftOdd<3, DIR, C> {};
template <int DIR, typename C> struct Dft<5, DIR, C> : DftOdd<5, DIR, C> {};
template <int DIR, typename C> struct Dft<7, DIR, C> : DftOdd<7, DIR, C> {};

// composite R = R1 * R2 in registers (j = j1 R2 + j2, k = k1 + R1 k2)
template <int R1, int R2, int DIR, typename C> struct DftCT {
  static __device__ __forceinline__ void run(C* v) {
    constexpr int R = R1 * R2;
    C t[R];
#pragma unroll
    for (int j2 = 0; j2 < R2; ++j2) {
      C a[R1];
#pragma unroll
      for (int j1 = 0; j1 < R1; ++j1) a[j1] = v[j1 * R2 + j2];
      Dft<R1, DIR, C>::run(a);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) t[k1 * R2 + j2] = twiddle_const<R, DIR>(a[k1], j2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      C b[R2];
#pragma unroll
      for (int j2 = 0; j2 < R2; ++j2) b[j2] = t[k1 * R2 + j2];
      Dft<R2, DIR, C>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = b[k2];
    }
  }
};
template <int DIR, typename C> struct Dft<6, DIR, C> : DftCT<2, 3, DIR, C> {};
template <int DIR, typename C> struct Dft<8, DIR, C> : DftCT<2, 4, DIR, C> {};
template <int DIR, typename C> struct Dft<12, DIR, C> : DftCT<4, 3, DIR, C> {};
template <int DIR, typename C> struct Dft<14, DIR, C> : DftCT<2, 7, DIR, C> {};
template <int DIR, typename C> struct Dft<16, DIR, C> : DftCT<4, 4, DIR, C> {};

// ------------------------------------------------ grid-size factorisation
// N = N1 * N2 with both factors covered by the codelets above.
template <int N> struct Fac;
template <> struct Fac<8> { static constexpr int N1 = 2, N2 = 4; };
template <> struct Fac<12> { static constexpr int N1 = 3, N2 = 4; };
template <> struct Fac<16> { static constexpr int N1 = 4, N2 = 4; };
template <> struct Fac<20> { static constexpr int N1 = 5, N2 = 4; };
template <> struct Fac<24> { static constexpr int N1 = 3, N2 = 8; };
template <> struct Fac<28> { static constexpr int N1 = 7, N2 = 4; };
template <> struct Fac<32> { static constexpr int N1 = 4, N2 = 8; };
template <> struct Fac<40> { static constexpr int N1 = 5, N2 = 8; };
template <> struct Fac<48> { static constexpr int N1 = 3, N2 = 16; };
template <> struct Fac<56> { static constexpr int N1 = 7, N2 = 8; };
template <> struct Fac<64> { static constexpr int N1 = 8, N2 = 8; };
template <> struct Fac<80> { static constexpr int N1 = 5, N2 = 16; };
template <> struct Fac<96> { static constexpr int N1 = 6, N2 = 16; };
template <> struct Fac<112> { static constexpr int N1 = 7, N2 = 16; };
template <> struct Fac<128> { static constexpr int N1 = 8, N2 = 16; };

// ------------------------------------------------ per-axis device tables
// tw[m] = exp(-2 pi i m / N) (forward twiddles), m < N.
// LDS addressing of a set of lines: element e of line l sits at
//   base(l) + e * estride,  base(l) = l * lstride.

// Stage A (forward): DFT_N1 over j1 for fixed (line, j2), twiddle, write
// back to slots k1*N2 + j2.
template <int N, typename C>
__device__ __forceinline__ void stageA_fwd(C* lds, int nlines, int lstride, int estride,
                                           const C* __restrict__ tw, int tid, int nthr,
                                           bool line_fast) {
  constexpr int N1 = Fac<N>::N1, N2 = Fac<N>::N2;
  const int items = nlines * N2;
  for (int w = tid; w < items; w += nthr) {
    const int line = line_fast ? (w % nlines) : (w / N2);
    const int j2 = line_fast ? (w / nlines) : (w % N2);
    C* p = lds + line * lstride;
    C a[N1];
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) a[j1] = p[(j1 * N2 + j2) * estride];
    Dft<N1, -1, C>::run(a);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      C v = a[k1];
      if (k1 > 0 && j2 > 0) v = cmul(v, tw[(j2 * k1) % N]);
      p[(k1 * N2 + j2) * estride] = v;
    }
  }
}

// Stage C (inverse): conj-DFT_N1 over k1 for fixed (line, j2), natural order.
template <int N, typename C>
__device__ __forceinline__ void stageC_inv(C* lds, int nlines, int lstride, int estride,
                                           int tid, int nthr, bool line_fast) {
  constexpr int N1 = Fac<N>::N1, N2 = Fac<N>::N2;
  const int items = nlines * N2;
  for (int w = tid; w < items; w += nthr) {
    const int line = line_fast ? (w % nlines) : (w / N2);
    const int j2 = line_fast ? (w / nlines) : (w % N2);
    C* p = lds + line * lstride;
    C a[N1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) a[k1] = p[(k1 * N2 + j2) * estride];
    Dft<N1, +1, C>::run(a);
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) p[(j1 * N2 + j2) * estride] = a[j1];
  }
}

// Stage B.  MODE 0: forward half only (DFT_N2; leaves scrambled spectrum).
// MODE 1: inverse half only (scrambled spectrum -> conj DFT_N2, conj
// twiddle).  MODE 2: forward DFT_N2, multiply by mul(line, k), inverse
// DFT_N2, conj twiddle.  k = k1 + N1*k2 is the natural frequency index.
template <int N, int MODE, typename C, typename Mul>
__device__ __forceinline__ void stageB(C* lds, int nlines, int lstride, int estride,
                                       const C* __restrict__ tw, int tid, int nthr,
                                       bool line_fast, Mul mul) {
  constexpr int N1 = Fac<N>::N1, N2 = Fac<N>::N2;
  const int items = nlines * N1;
  for (int w = tid; w < items; w += nthr) {
    const int line = line_fast ? (w % nlines) : (w / N1);
    const int k1 = line_fast ? (w / nlines) : (w % N1);
    C* p = lds + line * lstride;
    C b[N2];
#pragma unroll
    for (int j = 0; j < N2; ++j) b[j] = p[(k1 * N2 + j) * estride];
    if (MODE == 0 || MODE == 2) Dft<N2, -1, C>::run(b);
    if (MODE == 2) {
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) b[k2] = mul(line, b[k2], k1 + N1 * k2);
    }
    if (MODE == 1 || MODE == 2) {
      Dft<N2, +1, C>::run(b);
#pragma unroll
      for (int j2 = 0; j2 < N2; ++j2)
        if (k1 > 0 && j2 > 0) b[j2] = cmulc(b[j2], tw[(j2 * k1) % N]);
    }
#pragma unroll
    for (int j = 0; j < N2; ++j) p[(k1 * N2 + j) * estride] = b[j];
  }
}

// natural frequency index of scrambled slot p (p = k1*N2 + k2)
template <int N> __device__ __forceinline__ int scr2k(int p) {
  constexpr int N1 = Fac<N>::N1, N2 = Fac<N>::N2;
  return (p / N2) + N1 * (p % N2);
}

struct NoMul {
  template <typename C> __device__ __forceinline__ C operator()(int, C v, int) const { return v; }
};

}  // namespace bse
