// Complex helpers, exact twiddle factors and fully unrolled small DFTs held in registers.
//
// The 3-D transforms of the Galerkin operator (Sec. 2.1, eq. 2) are built from length-n
// line transforms, each split as n = A * B (four-step): B-point DFTs in one thread's
// registers, a twiddle by W_n^(a c), an exchange through LDS, then A-point DFTs.  This
// header holds the register part.  Twiddles are evaluated at compile time (device) or
// in long double (host tables) from a Taylor series after an exact octant reduction, so
// no math-library constant tables are involved.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <utility>

namespace ghom {

template <typename T> struct cx { T re, im; };

// Streamed global memory: when a context's CG working set exceeds the last-level cache (256
// MB; a float32 CG iteration touches about 184 B per voxel, 386 MB at 128^3) every field and
// spectrum value is read and written once per pass with no reuse, so the passes load and store
// them with the nontemporal hint.  Measured on this chip: a plain copy 6.29 -> 6.73 TB/s,
// three reads and two writes per element 5.71 -> 6.04 TB/s, a 256^3 CG iteration -7%, the
// 384-problem batch +6% throughput; a single 32^3..96^3 problem, whose iteration fits in the
// cache, runs 6-10% slower with it.  Kernels of transform length >= GHOM_NT_MIN are built
// with the hint only (their problems never fit); shorter ones both ways, chosen per context.
// A complex value moves as one 2-vector (spectra are aligned to a whole complex value).
#ifndef GHOM_NT_MIN
#define GHOM_NT_MIN 128
#endif
constexpr bool stream_nt_always(int n) { return n >= GHOM_NT_MIN; }
template <typename T> using vec2_t = T __attribute__((ext_vector_type(2)));
template <bool NT, typename T> __device__ __forceinline__ cx<T> ld_cx(const cx<T>* p) {
  if constexpr (NT) {
    const vec2_t<T> v = __builtin_nontemporal_load(reinterpret_cast<const vec2_t<T>*>(p));
    return cx<T>{v.x, v.y};
  } else {
    return *p;
  }
}
template <bool NT, typename T> __device__ __forceinline__ void st_cx(cx<T>* p, cx<T> z) {
  if constexpr (NT) {
    vec2_t<T> v;
    v.x = z.re;
    v.y = z.im;
    __builtin_nontemporal_store(v, reinterpret_cast<vec2_t<T>*>(p));
  } else {
    *p = z;
  }
}
template <bool NT, typename T> __device__ __forceinline__ T ld_s(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T> __device__ __forceinline__ void st_s(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <typename T> __host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> w) {
  return {a.re * w.re - a.im * w.im, a.re * w.im + a.im * w.re};
}
// a * conj(w)
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> w) {
  return {a.re * w.re + a.im * w.im, a.im * w.re - a.re * w.im};
}
template <typename T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// multiply by s*i, s = +1 or -1
template <int S, typename T> __device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  if constexpr (S > 0) return {-a.im, a.re};
  else return {a.im, -a.re};
}

// ---------------------------------------------------------------------------------
// cos/sin of 2*pi*k/n, exact octant reduction + Taylor series on [0, pi/4]
// ---------------------------------------------------------------------------------
struct CosSin { long double c, s; };

constexpr long double kPi = 3.14159265358979323846264338327950288L;

__host__ __device__ constexpr long double taylor_sin(long double x) {
  long double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
__host__ __device__ constexpr long double taylor_cos(long double x) {
  long double term = 1, sum = 1;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

// (cos, sin) of the angle 2*pi*k/n for any integer k and n > 0.
__host__ __device__ constexpr CosSin cossin_2pi(long long k, long long n) {
  k %= n;
  if (k < 0) k += n;
  const long long q = (8 * k) / n;       // octant 0..7
  const long long rem = 8 * k - q * n;   // angle = (pi/4) (q + rem/n)
  long double c = 0, s = 0;
  long long turns = 0;
  if ((q & 1) == 0) {                    // q pi/4 + phi, phi in [0, pi/4)
    const long double phi = (kPi / 4) * (long double)rem / (long double)n;
    c = taylor_cos(phi);
    s = taylor_sin(phi);
    turns = q / 2;
  } else {                               // (q+1) pi/4 - phi', phi' in (0, pi/4]
    const long double phi = (kPi / 4) * (long double)(n - rem) / (long double)n;
    c = taylor_cos(phi);
    s = -taylor_sin(phi);
    turns = (q + 1) / 2;
  }
  for (long long t = 0; t < (turns & 3); ++t) {  // rotate by quarter turns: (c,s) -> (-s,c)
    const long double nc = -s;
    s = c;
    c = nc;
  }
  return CosSin{c, s};
}

// ---------------------------------------------------------------------------------
// compile-time loops
// ---------------------------------------------------------------------------------
template <int I> using ic = std::integral_constant<int, I>;

template <int Begin, int End, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (Begin < End) {
    f(ic<Begin>{});
    static_for<Begin + 1, End>(f);
  }
}

// multiply by W_R^(K*DIR) = exp(DIR * 2 pi i K / R), K and R known at compile time
template <int K, int R, int DIR, typename T>
__device__ __forceinline__ cx<T> twiddle_c(cx<T> v) {
  constexpr int k = ((K % R) + R) % R;
  if constexpr (k == 0) {
    return v;
  } else if constexpr ((4 * k) % R == 0) {   // multiples of a quarter turn: exact
    constexpr int qt = (4 * k) / R;          // 1, 2, 3
    if constexpr (qt == 2) return cx<T>{-v.re, -v.im};
    else if constexpr ((qt == 1) == (DIR > 0)) return mul_i<+1>(v);
    else return mul_i<-1>(v);
  } else {
    constexpr CosSin cs = cossin_2pi(k, R);
    constexpr T c = (T)cs.c;
    constexpr T s = (T)(DIR > 0 ? cs.s : -cs.s);
    return cmul(v, cx<T>{c, s});
  }
}

constexpr int smallest_radix(int R) {
  return (R % 4 == 0 && R != 8) ? 4 : (R % 2 == 0 ? 2 : (R % 3 == 0 ? 3 : R));
}

// In-place R-point DFT of v[0..R) in natural order:
//   X[k] = sum_m v[m] exp(DIR * 2 pi i m k / R),  DIR = -1 forward, +1 inverse (no scaling).
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    const cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 3) {
    constexpr T h = (T)0.866025403784438646763723170752936183L;  // sin(pi/3)
    const cx<T> a = v[0], s = v[1] + v[2], d = v[1] - v[2];
    const cx<T> t = a - s * (T)0.5;
    const cx<T> r = mul_i<DIR>(d) * h;
    v[0] = a + s;
    v[1] = t + r;
    v[2] = t - r;
  } else if constexpr (R == 4) {
    const cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
    const cx<T> s13 = v[1] + v[3], d13 = mul_i<DIR>(v[1] - v[3]);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + d13;
    v[3] = d02 - d13;
  } else {
    // R = P * Q: input m = a + P b, output k = c + Q d
    constexpr int P = smallest_radix(R);
    constexpr int Q = R / P;
    static_assert(P * Q == R && P > 1 && Q > 1, "unsupported DFT length");
    cx<T> y[R];
    static_for<0, P>([&](auto a_) {
      constexpr int a = decltype(a_)::value;
      cx<T> t[Q];
      static_for<0, Q>([&](auto b_) { t[decltype(b_)::value] = v[a + P * decltype(b_)::value]; });
      dft<Q, DIR>(t);
      static_for<0, Q>([&](auto c_) {
        constexpr int c = decltype(c_)::value;
        y[a * Q + c] = twiddle_c<a * c, R, DIR>(t[c]);
      });
    });
    static_for<0, Q>([&](auto c_) {
      constexpr int c = decltype(c_)::value;
      cx<T> t[P];
      static_for<0, P>([&](auto a_) { t[decltype(a_)::value] = y[decltype(a_)::value * Q + c]; });
      dft<P, DIR>(t);
      static_for<0, P>([&](auto d_) { v[c + Q * decltype(d_)::value] = t[decltype(d_)::value]; });
    });
  }
}

// ---------------------------------------------------------------------------------
// supported line lengths: n = A * B with A | B; A threads per line, B values each
// ---------------------------------------------------------------------------------
template <int A_, int B_> struct Split {
  static constexpr int A = A_, B = B_, N = A_ * B_;
  static_assert(B_ % A_ == 0, "A must divide B");
};

// Calls f(Split<A,B>{}) for a supported n; returns false otherwise.
template <typename F> bool with_split(int n, F&& f) {
  switch (n) {
    case 4: f(Split<2, 2>{}); return true;
    case 6: f(Split<1, 6>{}); return true;
    case 8: f(Split<2, 4>{}); return true;
    case 9: f(Split<3, 3>{}); return true;
    case 12: f(Split<2, 6>{}); return true;
    case 16: f(Split<4, 4>{}); return true;
    case 18: f(Split<3, 6>{}); return true;
    case 24: f(Split<2, 12>{}); return true;
    case 27: f(Split<3, 9>{}); return true;
    case 32: f(Split<4, 8>{}); return true;
    case 36: f(Split<6, 6>{}); return true;
    case 48: f(Split<4, 12>{}); return true;
    case 64: f(Split<8, 8>{}); return true;
    case 72: f(Split<6, 12>{}); return true;
    case 96: f(Split<4, 24>{}); return true;
    case 128: f(Split<8, 16>{}); return true;
    case 144: f(Split<12, 12>{}); return true;
    case 192: f(Split<8, 24>{}); return true;
    case 256: f(Split<16, 16>{}); return true;
    case 512: f(Split<16, 32>{}); return true;
    default: return false;
  }
}

inline bool supported_length(int n) {
  return with_split(n, [](auto) {});
}

// ---------------------------------------------------------------------------------
// three-stage lines: n = B * A1 * A2 with B = A2; A = A1 * A2 threads per line, B values each
// ---------------------------------------------------------------------------------
// Stage 1: B-point DFTs in registers over x[q + A b]; stage 2: A2-point DFTs after an LDS
// exchange (one per thread); stage 3: A1-point DFTs after a second exchange (B / A1 per
// thread).  Half the values per thread of the two-stage split of the same length, for passes
// whose registers limit how many waves a SIMD holds.
template <int B_, int A1_, int A2_> struct Split3 {
  static constexpr int B = B_, A1 = A1_, A2 = A2_, A = A1_ * A2_, N = B_ * A1_ * A2_;
  static_assert(A2_ == B_ && B_ % A1_ == 0, "three-stage split: A2 = B and A1 | B");
};

// Calls f(Split3<...>{}) for a length with a three-stage schedule; returns false otherwise.
template <typename F> bool with_split3(int n, F&& f) {
  switch (n) {
    case 128: f(Split3<8, 2, 8>{}); return true;
    case 256: f(Split3<8, 4, 8>{}); return true;
    case 512: f(Split3<8, 8, 8>{}); return true;
    default: return false;
  }
}

inline bool has_split3(int n) {
  return with_split3(n, [](auto) {});
}

}  // namespace ghom
