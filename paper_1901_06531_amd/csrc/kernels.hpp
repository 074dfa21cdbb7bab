// HIP kernels (gfx950) of the Galerkin-FFT Newton / conjugate-gradient solver with
// stress and mixed control.
//
// Field layout: a tensor field is 9 planes of N = nx*ny*nz values, plane c = 3*i + j
// holds entry (i, j); within a plane the voxel (x, y, z) sits at (x*ny + y)*nz + z.
// Spectrum layout: after the real-to-complex transform along z only the wave numbers
// kz in [0, nzh) are kept (nzh = nz/2 for even nz: the Nyquist plane is zeroed by the
// projection, eq. 10; nzh = (nz+1)/2 for odd nz).  Plane c of the spectrum holds
// Nh = nx*ny*nzh complex values at (x*ny + y)*nzh + kz; passes along y and x transform
// in place, so after the x pass the entry (kx, ky, kz) sits at (kx*ny + ky)*nzh + kz.
//
// One application of the operator of eq. (20), A(v) = G*(K : v), is five passes:
//   zfwd  : K : v per voxel (or a plain copy), real-to-complex along z
//   yfwd  : complex transform along y
//   xproj : transform along x, the projection G* of eq. (22) at each frequency,
//           inverse transform along x
//   yinv  : inverse along y
//   zinv  : complex-to-real along z, fused dot products for CG
#pragma once

#include <cstdint>
#include <type_traits>

#include "cg_stop.hpp"
#include "dft.hpp"

namespace ghom {

struct Geo {
  int nx, ny, nz, nzh;
  long long N;    // voxels
  long long Nh;   // spectrum points per component
  double invL[3];
};

// A range of kz planes of the spectrum: the y and x passes can run slab by slab so that
// the slab's intermediate results stay in the on-chip caches between the passes.
struct Slab {
  int kz0, nkz;
};

enum { MAT_NH = 1, MAT_SVK = 2, MAT_VISCO = 3 };
constexpr int kNHState = 12;     // F^-T (9), a = s mu, b = s lam, c = s (mu - lam ln J)
constexpr int kSVKState = 10;    // H = F - I (9), s (1)
constexpr int kViscoState = 16;  // H = F - I (9), S in Voigt order (6), s (1)
constexpr int kStatePlanes = kViscoState;
static_assert(kStatePlanes >= kNHState && kStatePlanes >= kSVKState, "state planes");
// viscoelastic law: per phase Cinf (36), C1 (36), a = exp(-dt/tau), b = tau (1 - a) / dt
constexpr int kViscoTable = 74;
// internal variables of the viscoelastic law, float64 planes: E_n (6, Voigt with engineering
// shears), Q_n (6, Voigt)
constexpr int kViscoIV = 12;

// scalars shared by the CG kernels (device memory)
struct CGScalars {
  double rr;       // r.r of the current iterate
  double pAp;
  double alpha;
  double beta;
  double thresh;   // stop when rr <= thresh (= tol^2 N)
  double best;     // smallest r.r of the solve so far (stall test)
  int it;          // iterations done
  int max_it;
  int done;        // 1: stop (converged, breakdown, cap or stall)
  int status;      // CG_RUNNING, CG_CONVERGED, CG_BREAKDOWN, CG_CAP or CG_STALLED (cg_stop.hpp)
  int since;       // iterations since best was last lowered
};

// After a CG solve: whether the step of the last completed iteration still has to reach the
// iterate (the forward pass of the iteration after it applies it, and none ran after a stop by
// convergence, cap or stall): 0 no (x is complete; x = 0 when the solve stopped before its
// first step), 1 x = alpha p (a single step: x was never written), 2 x = x + alpha p.
__device__ __forceinline__ int cg_pending_mode(const CGScalars* sc) {
  const int st = sc->status;
  if (sc->it < 1 || (st != CG_CONVERGED && st != CG_CAP && st != CG_STALLED)) return 0;
  return sc->it >= 2 ? 2 : 1;
}

constexpr int kRedThreads = 1024;
constexpr int kRedFlag = 31;  // slot of the det F <= 0 flag in a problem's 32 reduced values

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Deterministic block sum (fixed order): valid in thread 0 only.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  constexpr int NW = (NT + 63) / 64;
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NW; ++i) s += sh[i];
  }
  __syncthreads();
  return s;
}
template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) {
  constexpr int NW = (NT + 63) / 64;
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NW; ++i) s = fmax(s, sh[i]);
  }
  __syncthreads();
  return s;
}

// K block reductions at once, in the order of block_sum / block_max (so the results are
// the same bits): columns k < NMAX take the max, the others the sum.  sh holds K * NW
// doubles; thread k < K calls out(k, value).  Ends the block's use of sh (no barrier
// after it).
template <int NT, int K, int NMAX = 0, typename Out>
__device__ __forceinline__ void block_reduce_cols(const double* v, double* sh, Out&& out) {
  constexpr int NW = (NT + 63) / 64;
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = k < NMAX ? wave_max(v[k]) : wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) sh[k * NW + w] = s;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    const int k = threadIdx.x;
    double s = 0.0;
    for (int i = 0; i < NW; ++i) s = k < NMAX ? fmax(s, sh[k * NW + i]) : s + sh[k * NW + i];
    out(k, s);
  }
}

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}

// LDS budget of a column-pass workgroup (KiB) per precision: 32 KiB in float32 leaves room
// for several workgroups per CU on short lines (n = 96, 192) without changing n = 256
#ifndef GHOM_CLDS_KB_F32
#define GHOM_CLDS_KB_F32 32
#endif
#ifndef GHOM_CLDS_KB_F64
#define GHOM_CLDS_KB_F64 64
#endif
template <typename T> constexpr int lds_cx() {
  return (sizeof(T) == 8 ? GHOM_CLDS_KB_F64 : GHOM_CLDS_KB_F32) * 1024 / (2 * (int)sizeof(T));
}

// column passes: A threads per line, TC lines per workgroup (at most TCMAX)
template <typename T, int A, int B, int TCMAX = 64, int MAXT = 256> struct ColCfg {
  static constexpr int N = A * B;
  static constexpr int TC = pow2_floor(cmax(1, cmin(TCMAX, cmin(MAXT / A, lds_cx<T>() / N))));
  static constexpr int NT = A * TC;
  // LDS stride between the exchange rows of consecutive c: one extra row of TC values
  // moves lanes of neighbouring c to the other half of the banks (float32)
  static constexpr int RS = A * TC + TC;
  static constexpr int LDS = B * RS;
};

// A column-pass configuration widened on lines of length >= MIN_N where its segments would be
// shorter than SEG bytes (more columns per workgroup, up to 512 threads and 80 KiB of LDS).
template <typename T, int A, int B, int MAXT, int SEG, int MIN_N> struct WideColCfg {
  using Base = ColCfg<T, A, B, 64, MAXT>;
  static constexpr int want = A * B >= MIN_N ? SEG / (int)sizeof(cx<T>) : 0;
  static constexpr int lds_cap = 80 * 1024 / (int)sizeof(cx<T>) / (A * B + B);  // columns in 80 KiB
  static constexpr int wide = pow2_floor(cmax(1, cmin(want, cmin(512 / A, lds_cap))));
  static constexpr int TC = Base::TC >= want || wide <= Base::TC ? Base::TC : wide;
  static constexpr int NT = A * TC;
  static constexpr int RS = A * TC + TC;
  static constexpr int LDS = B * RS;
};

// y passes: widened to 256-B segments on lines >= 256.  Measured, float32: 256^3 y pass 0.217
// -> 0.206 ms with 32 columns instead of 16; 192^3 0.092 -> 0.099 ms, so shorter lines keep
// theirs.  (The x pass gains nothing from it: its register-capped "rows" build, the fastest
// at 256^3, runs 0.259 -> 0.264 ms with 32 columns.)
#ifndef GHOM_YSEG
#define GHOM_YSEG 256
#endif
#ifndef GHOM_YSEG_MIN_N
#define GHOM_YSEG_MIN_N 256
#endif
template <typename T, int A, int B> using YCfg = WideColCfg<T, A, B, 256, GHOM_YSEG, GHOM_YSEG_MIN_N>;

// z passes: LP pairs of real lines (9 components each) per workgroup.  LP is at least
// GHOM_ZLP (or enough for ~256 threads on short lines), bounded by 1024 threads and an
// LDS budget of 80 KB.
#ifndef GHOM_ZLP
#define GHOM_ZLP 1
#endif
// LDS budget of a z-pass workgroup (KiB) per precision (bounds the lines per workgroup)
#ifndef GHOM_ZLDS_KB_F32
#define GHOM_ZLDS_KB_F32 24
#endif
#ifndef GHOM_ZLDS_KB_F64
#define GHOM_ZLDS_KB_F64 80
#endif
template <typename T> constexpr int zlds_cx() {
  return (sizeof(T) == 8 ? GHOM_ZLDS_KB_F64 : GHOM_ZLDS_KB_F32) * 1024 / (2 * (int)sizeof(T));
}
// NTMIN: a larger thread count for the per-voxel stages of the CG-step z passes (zfwd_ntmin /
// zinv_ntmin), taken when it leaves fewer thread slots idle in the last round
template <typename T, int A, int B, int NTMIN = 0> struct ZCfg {
  static constexpr int N = A * B;
  static constexpr int R = N + B;  // LDS complex values per line: exchange rows padded to A + 1
  static constexpr int LP =
      cmax(1, cmin(cmax(GHOM_ZLP, 256 / (9 * A)), cmin(1024 / (9 * A), zlds_cx<T>() / (9 * R))));
  static constexpr int NF = 9 * LP * A;           // threads of the transform phase
  static constexpr int NT0 = (NF + 63) / 64 * 64;  // whole wavefronts
  // share of thread slots the per-voxel stage uses (2 LP N voxels over whole rounds of nt)
  static constexpr int slot_use(int nt) { return 1000 * (2 * LP * N) / (((2 * LP * N + nt - 1) / nt) * nt); }
  static constexpr int NT = (NTMIN > NT0 && slot_use(NTMIN) > slot_use(NT0)) ? NTMIN : NT0;
};

// ---------------------------------------------------------------------------------
// four-step building blocks (n = A*B; thread q in [0, A) of a line)
// ---------------------------------------------------------------------------------
// Forward half: v[b] = x[q + A b] (b < B)  ->  v[c] = W_n^(q c) * DFT_B(v)[c]
template <int A, int B, int DIR, typename T>
__device__ __forceinline__ void four_step_first(cx<T>* v, int q, const cx<T>* __restrict__ tw) {
  dft<B, DIR>(v);
#pragma unroll
  for (int c = 1; c < B; ++c) {
    const cx<T> w = tw[q * c];
    v[c] = DIR < 0 ? cmul(v[c], w) : cmulc(v[c], w);
  }
}

// second half, reading the exchanged values: thread q owns c = q + A i (i < B/A);
// for each, t[a] = Y[a][c] (a < A) -> DFT_A -> X[c + B d], stored in v[i + (B/A) d]
// (so v[e] = X[q + A e]).  'get(c, a)' returns Y[a][c].
template <int A, int B, int DIR, typename T, typename Get>
__device__ __forceinline__ void four_step_second(cx<T>* v, int q, Get&& get) {
  constexpr int R = B / A;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int c = q + A * i;
    cx<T> t[A];
#pragma unroll
    for (int a = 0; a < A; ++a) t[a] = get(c, a);
    dft<A, DIR>(t);
#pragma unroll
    for (int d = 0; d < A; ++d) v[i + R * d] = t[d];
  }
}

// inverse of the second half for data held as v[e] = X[q + A e]: for each c = q + A i,
// DFT_A^(DIR) over d of X[c + B d], twiddle by W_n^(-DIR... ) and hand Z[c][a] to put(c, a, z)
template <int A, int B, int DIR, typename T, typename Put>
__device__ __forceinline__ void four_step_second_inv(const cx<T>* v, int q, const cx<T>* __restrict__ tw,
                                                     Put&& put) {
  constexpr int R = B / A;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int c = q + A * i;
    cx<T> t[A];
#pragma unroll
    for (int d = 0; d < A; ++d) t[d] = v[i + R * d];
    dft<A, DIR>(t);
#pragma unroll
    for (int a = 0; a < A; ++a) {
      const cx<T> w = tw[a * c];
      put(c, a, DIR < 0 ? cmul(t[a], w) : cmulc(t[a], w));
    }
  }
}

// ---------------------------------------------------------------------------------
// three-stage line transforms (Split3): n = B * A1 * A2, A = A1 * A2 threads per line
// ---------------------------------------------------------------------------------
// slot(h, l) is this thread's reference to slot h A + l (h < B, l < A) of its line's LDS
// exchange area; sync() a barrier of every thread sharing that area.
//
// Forward (DIR = -1; the inverse with DIR = +1 is three_stage_inv) from v[b] = x[q + A b]:
//   stage 1: Y[q][c] = W_n^(q c) DFT_B(x[q + A .])[c]                      (registers)
//   stage 2: thread q takes (c, q1) = (q % B, q / B):
//            U[c][q1][d1] = W_A^(q1 d1) DFT_A2(Y[q1 + A1 .][c])[d1]
//   stage 3: task t = q + A i (i < B / A1) takes (c, d1) = (t % B, t / B):
//            X[c + B (d1 + A2 d2)] = DFT_A1(U[c][.][d1])[d2], kept in v[i A1 + d2]
// (an A-point DFT over q = q1 + A1 q2, d = d1 + A2 d2, splits as W_A^(q d) =
// W_A1^(q1 d2) W_A^(q1 d1) W_A2^(q2 d1)).  three_stage_freq gives the frequency of v[e].
template <typename S>
__device__ __forceinline__ int three_stage_freq(int q, int e) {
  const int i = e / S::A1, d2 = e % S::A1;
  const int t = q + S::A * i;
  return t % S::B + S::B * (t / S::B + S::A2 * d2);
}

template <typename S, int DIR, typename T, typename Slot, typename Sync>
__device__ __forceinline__ void three_stage_fwd(cx<T>* v, int q, const cx<T>* __restrict__ tw, Slot&& slot,
                                                Sync&& sync) {
  constexpr int B = S::B, A1 = S::A1, A2 = S::A2, A = S::A;
  dft<B, DIR>(v);
#pragma unroll
  for (int c = 1; c < B; ++c) {
    const cx<T> w = tw[q * c];
    v[c] = DIR < 0 ? cmul(v[c], w) : cmulc(v[c], w);
  }
  sync();  // earlier readers of the area are done
#pragma unroll
  for (int c = 0; c < B; ++c) slot(c, q) = v[c];
  sync();
  {
    const int c = q % B, q1 = q / B;
    cx<T> t[A2];
#pragma unroll
    for (int q2 = 0; q2 < A2; ++q2) t[q2] = slot(c, q1 + A1 * q2);
    dft<A2, DIR>(t);
#pragma unroll
    for (int d1 = 1; d1 < A2; ++d1) {
      const cx<T> w = tw[B * q1 * d1];  // W_A^(q1 d1) = W_n^(B q1 d1)
      t[d1] = DIR < 0 ? cmul(t[d1], w) : cmulc(t[d1], w);
    }
    sync();
#pragma unroll
    for (int d1 = 0; d1 < A2; ++d1) slot(c, d1 * A1 + q1) = t[d1];
  }
  sync();
#pragma unroll
  for (int i = 0; i < B / A1; ++i) {
    const int t3 = q + A * i;
    const int c = t3 % B, d1 = t3 / B;
    cx<T> u[A1];
#pragma unroll
    for (int q1 = 0; q1 < A1; ++q1) u[q1] = slot(c, d1 * A1 + q1);
    dft<A1, DIR>(u);
#pragma unroll
    for (int d2 = 0; d2 < A1; ++d2) v[i * A1 + d2] = u[d2];
  }
}

// Inverse of three_stage_fwd (DIR = +1: conjugate twiddles, unnormalized) from the frequency
// layout of three_stage_fwd back to v[b] = x[q + A b].
template <typename S, int DIR, typename T, typename Slot, typename Sync>
__device__ __forceinline__ void three_stage_inv(cx<T>* v, int q, const cx<T>* __restrict__ tw, Slot&& slot,
                                                Sync&& sync) {
  constexpr int B = S::B, A1 = S::A1, A2 = S::A2, A = S::A;
  sync();  // earlier readers of the area are done
#pragma unroll
  for (int i = 0; i < B / A1; ++i) {
    const int t3 = q + A * i;
    const int c = t3 % B, d1 = t3 / B;
    cx<T> u[A1];
#pragma unroll
    for (int d2 = 0; d2 < A1; ++d2) u[d2] = v[i * A1 + d2];
    dft<A1, DIR>(u);
#pragma unroll
    for (int q1 = 0; q1 < A1; ++q1) slot(c, d1 * A1 + q1) = u[q1];
  }
  sync();
  {
    const int c = q % B, q1 = q / B;
    cx<T> t[A2];
#pragma unroll
    for (int d1 = 0; d1 < A2; ++d1) {
      const cx<T> z = slot(c, d1 * A1 + q1);
      const cx<T> w = tw[B * q1 * d1];
      t[d1] = DIR < 0 ? cmul(z, w) : cmulc(z, w);
    }
    dft<A2, DIR>(t);
    sync();
#pragma unroll
    for (int q2 = 0; q2 < A2; ++q2) slot(c, q1 + A1 * q2) = t[q2];
  }
  sync();
#pragma unroll
  for (int c = 0; c < B; ++c) {
    const cx<T> w = tw[q * c];
    const cx<T> z = slot(c, q);
    v[c] = DIR < 0 ? cmul(z, w) : cmulc(z, w);
  }
  dft<B, DIR>(v);
}

// ---------------------------------------------------------------------------------
// y pass: in-place complex transform along y of every spectrum line (c, x, kz)
// ---------------------------------------------------------------------------------
// the y pass's column configuration: WIDE the widened one (YCfg), else the plain one
template <typename T, int A, int B> using YNarrowCfg = ColCfg<T, A, B, 64, 256>;
template <typename T, int A, int B, bool WIDE> using YPassCfg =
    typename std::conditional<WIDE, YCfg<T, A, B>, YNarrowCfg<T, A, B>>::type;

template <typename T, int A, int B, int DIR, bool NTS, bool WIDE = true>
__device__ __forceinline__ void ypass_body(const Geo& g, Slab sl, cx<T>* __restrict__ H, const cx<T>* __restrict__ tw,
                                           const CGScalars* __restrict__ sc, int bx) {
  constexpr bool kNT = NTS;  // nontemporal streamed accesses
  using Cfg = YPassCfg<T, A, B, WIDE>;
  constexpr int TC = Cfg::TC;
  constexpr int RS = Cfg::RS;
  __shared__ cx<T> lds[Cfg::LDS];
  if (sc && sc->done) return;
  const int j = threadIdx.x % TC;
  const int q = threadIdx.x / TC;
  const long long ncols = 9LL * g.nx * sl.nkz;
  const long long col = (long long)bx * TC + j;
  const bool ok = col < ncols;
  const long long grp = col / sl.nkz;  // (c, x)
  const long long base = grp * ((long long)g.ny * g.nzh) + sl.kz0 + (col - grp * sl.nkz);
  const long long rs = g.nzh;
  cx<T> v[B];
#pragma unroll
  for (int e = 0; e < B; ++e) v[e] = ok ? ld_cx<kNT>(&H[base + (long long)(q + A * e) * rs]) : cx<T>{0, 0};
  four_step_first<A, B, DIR>(v, q, tw);
#pragma unroll
  for (int c = 0; c < B; ++c) lds[c * RS + q * TC + j] = v[c];
  __syncthreads();
  four_step_second<A, B, DIR>(v, q, [&](int c, int a) { return lds[c * RS + a * TC + j]; });
  if (ok) {
#pragma unroll
    for (int e = 0; e < B; ++e) st_cx<kNT>(&H[base + (long long)(q + A * e) * rs], v[e]);
  }
}

// y pass with the three-stage schedule (Split3): A threads per line holding B values, TC
// lines per workgroup, LDS of n slots per line with one padding row per A slots.  The forward
// pass writes X[k] where the three-stage layout leaves it; the inverse reads it from there.
template <typename T, typename S> struct Y3Cfg {
  static constexpr int TC = S::A >= 64 ? 8 : 16;  // at most 512 threads per workgroup
  static constexpr int NT = S::A * TC;
  static constexpr int LDS = (S::N + S::N / S::A) * TC;
};

template <typename T, typename S, int DIR, bool NTS>
__device__ __forceinline__ void ypass3_body(const Geo& g, Slab sl, cx<T>* __restrict__ H, const cx<T>* __restrict__ tw,
                                            const CGScalars* __restrict__ sc, int bx) {
  constexpr bool kNT = NTS;
  using Cfg = Y3Cfg<T, S>;
  constexpr int TC = Cfg::TC, A = S::A, B = S::B;
  __shared__ cx<T> lds[Cfg::LDS];
  if (sc && sc->done) return;
  const int j = threadIdx.x % TC;
  const int q = threadIdx.x / TC;
  const long long ncols = 9LL * g.nx * sl.nkz;
  const long long col = (long long)bx * TC + j;
  const bool ok = col < ncols;
  const long long grp = col / sl.nkz;  // (c, x)
  const long long base = grp * ((long long)g.ny * g.nzh) + sl.kz0 + (col - grp * sl.nkz);
  const long long rs = g.nzh;
  auto slot = [&](int h, int l) -> cx<T>& { return lds[(h * (A + 1) + l) * TC + j]; };
  auto sync = [] { __syncthreads(); };
  cx<T> v[B];
  if constexpr (DIR < 0) {
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = ok ? ld_cx<kNT>(&H[base + (long long)(q + A * b) * rs]) : cx<T>{0, 0};
    three_stage_fwd<S, -1>(v, q, tw, slot, sync);
    if (ok) {
#pragma unroll
      for (int e = 0; e < B; ++e) st_cx<kNT>(&H[base + (long long)three_stage_freq<S>(q, e) * rs], v[e]);
    }
  } else {
#pragma unroll
    for (int e = 0; e < B; ++e)
      v[e] = ok ? ld_cx<kNT>(&H[base + (long long)three_stage_freq<S>(q, e) * rs]) : cx<T>{0, 0};
    three_stage_inv<S, +1>(v, q, tw, slot, sync);
    if (ok) {
#pragma unroll
      for (int b = 0; b < B; ++b) st_cx<kNT>(&H[base + (long long)(q + A * b) * rs], v[b]);
    }
  }
}

// ---------------------------------------------------------------------------------
// x pass with the modified projection (eq. 22), for one tensor row per blockIdx.y
// ---------------------------------------------------------------------------------
// No array indexed at run time lives in this struct or in the x-pass bodies: such an array
// is placed in per-lane scratch memory, which every thread would write at kernel start.
struct ProjParams {
  unsigned mask;        // bit c set: component c is stress-controlled (IJ)
  double post;          // output factor (scale / N: fixes the unnormalized transforms)
  const double* pbar;   // nullable: N * pbar[c] is subtracted at xi = 0 (stress-controlled c)
  double n;             // N
  __device__ double off(int c) const { return pbar ? n * pbar[c] : 0.0; }
};

__device__ __forceinline__ int signed_k(int k, int n) { return k <= (n - 1) / 2 ? k : k - n; }

// x pass with the modified projection.  Row i of eq. (9) is B_ij = s xi_j with
// s = (sum_l A_il xi_l) / (xi.xi), so the forward transforms of a row's three components
// only meet in s.  Two variants (the faster one is picked per precision and grid at run
// time):
//  "groups": a workgroup takes TC columns (ky, kz) of one tensor row; thread group l in
//    {0, 1, 2} transforms component 3i + l along x, the groups form s through LDS, then
//    each transforms s xi_l back;
//  "rows": one thread transforms all three components of its columns in turn.
#ifndef XPROJ_TC
#define XPROJ_TC 0
#endif
#ifndef XPROJ_TCMAX
#define XPROJ_TCMAX 16
#endif
template <typename T, int A, int B> struct XCfg {
  static constexpr int N = A * B;
  // three groups share the LDS budget: TC columns per group, power of two
  static constexpr int fit(int tc) {  // largest power of two <= tc whose LDS stays under 100 KB
    while (tc > 1 && 3 * B * (A * tc + tc) * (int)sizeof(cx<T>) > 100 * 1024) tc /= 2;
    return tc;
  }
  static constexpr int TC_AUTO = fit(pow2_floor(cmax(1, cmin(XPROJ_TCMAX, 128 / A))));
  static constexpr int TC = XPROJ_TC > 0 ? fit(XPROJ_TC) : TC_AUTO;
  static constexpr int RS = A * TC + TC;   // padded stride between exchange rows
  static constexpr int REG = B * RS;       // LDS complex values per group
  static constexpr int NG = A * TC;        // threads per group
  static constexpr int NT = 3 * NG;
};

template <typename T, int A, int B, bool NTS>
__device__ __forceinline__ void xproj_groups_body(const Geo& g, Slab sl, cx<T>* __restrict__ H,
                                                  const cx<T>* __restrict__ tw, const ProjParams& pp,
                                                  const CGScalars* __restrict__ sc, int bx, int by) {
  constexpr bool kNT = NTS;  // nontemporal streamed accesses
  using Cfg = XCfg<T, A, B>;
  constexpr int TC = Cfg::TC, RS = Cfg::RS, REG = Cfg::REG;
  __shared__ cx<T> lds[3 * REG];
  if (sc && sc->done) return;
  const int l = threadIdx.x / Cfg::NG;          // component of the row handled by this thread
  const int tl = threadIdx.x - l * Cfg::NG;
  const int j = tl % TC;
  const int q = tl / TC;
  const int row = by;
  const int comp = 3 * row + l;
  cx<T>* E = lds + l * REG;                     // this group's exchange region
  const long long ncols = (long long)g.ny * sl.nkz;
  const long long col = (long long)bx * TC + j;  // column (ky, kz - kz0) of the slab
  const bool ok = col < ncols;
  const long long rs = (long long)g.ny * g.nzh;  // stride between x rows
  const int ky = ok ? (int)(col / sl.nkz) : 0;
  const int kz = ok ? sl.kz0 + (int)(col - (long long)ky * sl.nkz) : 0;
  const long long gcol = (long long)ky * g.nzh + kz;  // column (ky, kz) of the spectrum plane
  const bool nyq_yz = ((g.ny % 2 == 0) && ky == g.ny / 2);
  const T xy = (T)(signed_k(ky, g.ny) * g.invL[1]);
  const T xz = (T)(kz * g.invL[2]);
  const T post = (T)pp.post;
  auto xi_x = [&](int e) { return (T)(signed_k(q + A * e, g.nx) * g.invL[0]); };
  const long long cbase = (long long)comp * g.Nh + gcol;
  cx<T> v[B];
#pragma unroll
  for (int e = 0; e < B; ++e) v[e] = ok ? ld_cx<kNT>(&H[cbase + (long long)(q + A * e) * rs]) : cx<T>{0, 0};
  // forward transform along x of this group's component
  four_step_first<A, B, -1>(v, q, tw);
#pragma unroll
  for (int c = 0; c < B; ++c) E[c * RS + q * TC + j] = v[c];
  __syncthreads();
  four_step_second<A, B, -1>(v, q, [&](int c, int a) { return E[c * RS + a * TC + j]; });
  const cx<T> a0 = v[0];  // value at kx = q (= 0 for q = 0)
  // publish xi_l X_l at this thread's frequencies (kx = q + A e)
  __syncthreads();
#pragma unroll
  for (int e = 0; e < B; ++e) E[e * RS + q * TC + j] = v[e] * (l == 0 ? xi_x(e) : (l == 1 ? xy : xz));
  __syncthreads();
  // s at each frequency, then this group's component of the projection
#pragma unroll
  for (int e = 0; e < B; ++e) {
    const int pos = e * RS + q * TC + j;
    cx<T> s = lds[pos] + lds[REG + pos] + lds[2 * REG + pos];
    const int kx = q + A * e;
    const bool nyq = nyq_yz || ((g.nx % 2 == 0) && kx == g.nx / 2);
    const T xx = xi_x(e);
    const T xi2 = xx * xx + xy * xy + xz * xz;
    s = (nyq || xi2 == (T)0) ? cx<T>{0, 0} : s * (post / xi2);
    v[e] = s * (l == 0 ? xx : (l == 1 ? xy : xz));
  }
  if (ok && ky == 0 && kz == 0 && q == 0) {  // xi = 0: eq. (22) keeps stress-controlled components
    v[0] = ((pp.mask >> comp) & 1u) ? cx<T>{(a0.re - (T)pp.off(comp)) * post, a0.im * post} : cx<T>{0, 0};
  }
  __syncthreads();
  four_step_second_inv<A, B, +1>(v, q, tw, [&](int c, int a, cx<T> z) { E[c * RS + a * TC + j] = z; });
  __syncthreads();
#pragma unroll
  for (int b = 0; b < B; ++b) v[b] = E[b * RS + q * TC + j];
  dft<B, +1>(v);
  if (ok) {
#pragma unroll
    for (int e = 0; e < B; ++e) st_cx<kNT>(&H[cbase + (long long)(q + A * e) * rs], v[e]);
  }
}

// Variant "rows": one thread transforms all three components of its columns in turn and
// carries only the scalar s between the forward and the inverse transforms.
// GHOM_XPF: prefetch of the next component in the "rows" x pass; -1 = float32 only (in
// float64 the second register set would spill)
#ifndef GHOM_XPF
#define GHOM_XPF -1
#endif
#ifndef GHOM_XROWS_MAXT
#define GHOM_XROWS_MAXT 256
#endif
template <typename T, int A, int B> using XRowsCfg = ColCfg<T, A, B, 64, GHOM_XROWS_MAXT>;
template <typename T, int A, int B, bool NTS, bool XPF = (GHOM_XPF < 0 ? sizeof(T) == 4 : GHOM_XPF != 0)>
__device__ __forceinline__ void xproj_rows_body(const Geo& g, Slab sl, cx<T>* __restrict__ H,
                                                const cx<T>* __restrict__ tw, const ProjParams& pp,
                                                const CGScalars* __restrict__ sc, int bx, int by) {
  constexpr bool kNT = NTS;  // nontemporal streamed accesses
  using Cfg = XRowsCfg<T, A, B>;
  constexpr int TC = Cfg::TC;
  constexpr int RS = Cfg::RS;
  __shared__ cx<T> lds[Cfg::LDS];
  if (sc && sc->done) return;
  const int j = threadIdx.x % TC;
  const int q = threadIdx.x / TC;
  const int row = by;  // tensor row i: components 3i, 3i+1, 3i+2
  const long long ncols = (long long)g.ny * sl.nkz;
  const long long col = (long long)bx * TC + j;  // column (ky, kz - kz0) of the slab
  const bool ok = col < ncols;
  const long long rs = (long long)g.ny * g.nzh;  // stride between x rows
  const int ky = ok ? (int)(col / sl.nkz) : 0;
  const int kz = ok ? sl.kz0 + (int)(col - (long long)ky * sl.nkz) : 0;
  const long long gcol = (long long)ky * g.nzh + kz;  // column (ky, kz) of the spectrum plane
  const bool nyq_yz = ((g.ny % 2 == 0) && ky == g.ny / 2);
  const T xy = (T)(signed_k(ky, g.ny) * g.invL[1]);
  const T xz = (T)(kz * g.invL[2]);
  const T post = (T)pp.post;
  // the thread holding kx = 0 (q = 0, e = 0) of column (ky, kz) = (0, 0) holds xi = 0
  const bool hold0 = ok && ky == 0 && kz == 0 && q == 0;
  auto xi_x = [&](int e) { return (T)(signed_k(q + A * e, g.nx) * g.invL[0]); };
  cx<T> s[B];
  __shared__ cx<T> a0s[3];  // values at xi = 0, written and read by the thread that holds it
#pragma unroll
  for (int e = 0; e < B; ++e) s[e] = cx<T>{0, 0};
  auto load_comp = [&](int l, cx<T>* v) {
    const cx<T>* src = H + (long long)(3 * row + l) * g.Nh + gcol;
#pragma unroll
    for (int e = 0; e < B; ++e) v[e] = ok ? ld_cx<kNT>(&src[(long long)(q + A * e) * rs]) : cx<T>{0, 0};
  };
  // XPF: the loads of the next component are in flight during this component's transform
  cx<T> nxt[XPF ? B : 1];
  if constexpr (XPF) load_comp(0, nxt);
#pragma nounroll
  for (int l = 0; l < 3; ++l) {
    cx<T> v[B];
    if constexpr (XPF) {
#pragma unroll
      for (int e = 0; e < B; ++e) v[e] = nxt[e];
      if (l < 2) load_comp(l + 1, nxt);
    } else {
      load_comp(l, v);
    }
    four_step_first<A, B, -1>(v, q, tw);
    if (l) __syncthreads();
#pragma unroll
    for (int c = 0; c < B; ++c) lds[c * RS + q * TC + j] = v[c];
    __syncthreads();
    four_step_second<A, B, -1>(v, q, [&](int c, int a) { return lds[c * RS + a * TC + j]; });
#pragma unroll
    for (int e = 0; e < B; ++e) s[e] = s[e] + v[e] * (l == 0 ? xi_x(e) : (l == 1 ? xy : xz));
    if (hold0) a0s[l] = v[0];
  }
#pragma unroll
  for (int e = 0; e < B; ++e) {
    const int kx = q + A * e;
    const bool nyq = nyq_yz || ((g.nx % 2 == 0) && kx == g.nx / 2);
    const T xx = xi_x(e);
    const T xi2 = xx * xx + xy * xy + xz * xz;
    s[e] = (nyq || xi2 == (T)0) ? cx<T>{0, 0} : s[e] * (post / xi2);
  }
#pragma nounroll
  for (int l = 0; l < 3; ++l) {
    cx<T> v[B];
#pragma unroll
    for (int e = 0; e < B; ++e) v[e] = s[e] * (l == 0 ? xi_x(e) : (l == 1 ? xy : xz));
    if (hold0) {  // xi = 0: eq. (22) keeps stress-controlled components (minus P-bar)
      const int c = 3 * row + l;
      const cx<T> a0 = a0s[l];
      v[0] = ((pp.mask >> c) & 1u) ? cx<T>{(a0.re - (T)pp.off(c)) * post, a0.im * post} : cx<T>{0, 0};
    }
    __syncthreads();
    four_step_second_inv<A, B, +1>(v, q, tw, [&](int c, int a, cx<T> z) { lds[c * RS + a * TC + j] = z; });
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = lds[b * RS + q * TC + j];
    dft<B, +1>(v);
    if (ok) {
      cx<T>* dst = H + (long long)(3 * row + l) * g.Nh + gcol;
#pragma unroll
      for (int e = 0; e < B; ++e) st_cx<kNT>(&dst[(long long)(q + A * e) * rs], v[e]);
    }
  }
}

// x pass with the three-stage schedule ("rows3"): as "rows", one thread takes the three
// components of a tensor row in turn, but a line has A = 32 (n = 256) threads holding 8
// values each, so a thread's registers hold 8 values and 8 projection accumulators instead
// of 16 + 16.  TC columns (ky, kz) per workgroup; LDS exchange area of n slots per column
// with one padding row per A slots.
template <typename T, typename S> struct XRows3Cfg {
  static constexpr int TC = S::A >= 64 ? 8 : 16;  // at most 512 threads per workgroup
  static constexpr int NT = S::A * TC;
  static constexpr int SLOTS = S::N + S::N / S::A;
  static constexpr int LDS = SLOTS * TC;
};

template <typename T, typename S, bool NTS>
__device__ __forceinline__ void xproj_rows3_body(const Geo& g, Slab sl, cx<T>* __restrict__ H,
                                                 const cx<T>* __restrict__ tw, const ProjParams& pp,
                                                 const CGScalars* __restrict__ sc, int bx, int by) {
  constexpr bool kNT = NTS;
  using Cfg = XRows3Cfg<T, S>;
  constexpr int TC = Cfg::TC, A = S::A, B = S::B;
  __shared__ cx<T> lds[Cfg::LDS];
  __shared__ cx<T> a0s[3];
  if (sc && sc->done) return;
  const int j = threadIdx.x % TC;
  const int q = threadIdx.x / TC;
  const int row = by;
  const long long ncols = (long long)g.ny * sl.nkz;
  const long long col = (long long)bx * TC + j;
  const bool ok = col < ncols;
  const long long rs = (long long)g.ny * g.nzh;
  const int ky = ok ? (int)(col / sl.nkz) : 0;
  const int kz = ok ? sl.kz0 + (int)(col - (long long)ky * sl.nkz) : 0;
  const long long gcol = (long long)ky * g.nzh + kz;
  const bool nyq_yz = ((g.ny % 2 == 0) && ky == g.ny / 2);
  const T xy = (T)(signed_k(ky, g.ny) * g.invL[1]);
  const T xz = (T)(kz * g.invL[2]);
  const T post = (T)pp.post;
  const bool hold0 = ok && ky == 0 && kz == 0 && q == 0;  // v[0] of thread 0 holds kx = 0
  auto slot = [&](int h, int l) -> cx<T>& { return lds[(h * (A + 1) + l) * TC + j]; };
  auto sync = [] { __syncthreads(); };
  auto xi_x = [&](int e) { return (T)(signed_k(three_stage_freq<S>(q, e), g.nx) * g.invL[0]); };
  cx<T> s[B];
#pragma unroll
  for (int e = 0; e < B; ++e) s[e] = cx<T>{0, 0};
#pragma nounroll
  for (int l = 0; l < 3; ++l) {
    const cx<T>* src = H + (long long)(3 * row + l) * g.Nh + gcol;
    cx<T> v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = ok ? ld_cx<kNT>(&src[(long long)(q + A * b) * rs]) : cx<T>{0, 0};
    three_stage_fwd<S, -1>(v, q, tw, slot, sync);
#pragma unroll
    for (int e = 0; e < B; ++e) s[e] = s[e] + v[e] * (l == 0 ? xi_x(e) : (l == 1 ? xy : xz));
    if (hold0) a0s[l] = v[0];
  }
#pragma unroll
  for (int e = 0; e < B; ++e) {
    const int kx = three_stage_freq<S>(q, e);
    const bool nyq = nyq_yz || ((g.nx % 2 == 0) && kx == g.nx / 2);
    const T xx = xi_x(e);
    const T xi2 = xx * xx + xy * xy + xz * xz;
    s[e] = (nyq || xi2 == (T)0) ? cx<T>{0, 0} : s[e] * (post / xi2);
  }
#pragma nounroll
  for (int l = 0; l < 3; ++l) {
    cx<T> v[B];
#pragma unroll
    for (int e = 0; e < B; ++e) v[e] = s[e] * (l == 0 ? xi_x(e) : (l == 1 ? xy : xz));
    if (hold0) {  // xi = 0: eq. (22) keeps stress-controlled components (minus P-bar)
      const int c = 3 * row + l;
      const cx<T> a0 = a0s[l];
      v[0] = ((pp.mask >> c) & 1u) ? cx<T>{(a0.re - (T)pp.off(c)) * post, a0.im * post} : cx<T>{0, 0};
    }
    three_stage_inv<S, +1>(v, q, tw, slot, sync);
    if (ok) {
      cx<T>* dst = H + (long long)(3 * row + l) * g.Nh + gcol;
#pragma unroll
      for (int b = 0; b < B; ++b) st_cx<kNT>(&dst[(long long)(q + A * b) * rs], v[b]);
    }
  }
}

// ---------------------------------------------------------------------------------
// pointwise tangents K : dF
// ---------------------------------------------------------------------------------
// neo-Hookean: K:dF = a dF + b (G:dF) G + c G dF^T G with G = F^-T
template <typename T>
__device__ __forceinline__ void tangent_nh(const T* st, const T* d, T* out) {
  const T* G = st;
  const T a = st[9], b = st[10], c = st[11];
  T tr = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) tr += G[k] * d[k];
  // M = dF^T G : M_kj = sum_l dF_lk G_lj
  T M[9];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) M[3 * k + jj] = d[k] * G[jj] + d[3 + k] * G[3 + jj] + d[6 + k] * G[6 + jj];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      const T gm = G[3 * i] * M[jj] + G[3 * i + 1] * M[3 + jj] + G[3 * i + 2] * M[6 + jj];
      out[3 * i + jj] = a * d[3 * i + jj] + b * tr * G[3 * i + jj] + c * gm;
    }
}

// Saint Venant-Kirchhoff: K:dF = dF S + F (s C : sym(F^T dF)), C in 6x6 Voigt form
// SVK tangent K : d = d S + F (C : sym(F^T d)) with F = I + H and S = s C : E(H),
// E = (H + H^T + H^T H) / 2.  Only H and s are stored: S is rebuilt here from the grain's
// stiffness, which the tangent needs anyway, and forming E from H (not F^T F - I) keeps
// the small strains free of cancellation in the CG type.
template <typename T>
__device__ __forceinline__ void tangent_svk(const T* H, T s, const T* __restrict__ C6, const T* d, T* out) {
  auto hth = [&](int i, int j) { return H[i] * H[j] + H[3 + i] * H[3 + j] + H[6 + i] * H[6 + j]; };
  // (F^T d)_ij = d_ij + sum_k H_ki d_kj
  auto ftd = [&](int i, int j) { return d[3 * i + j] + H[i] * d[j] + H[3 + i] * d[3 + j] + H[6 + i] * d[6 + j]; };
  T E[6], dE[6];  // Voigt 11 22 33 23 13 12, engineering shears
  E[0] = H[0] + (T)0.5 * hth(0, 0);
  E[1] = H[4] + (T)0.5 * hth(1, 1);
  E[2] = H[8] + (T)0.5 * hth(2, 2);
  E[3] = H[5] + H[7] + hth(1, 2);
  E[4] = H[2] + H[6] + hth(0, 2);
  E[5] = H[1] + H[3] + hth(0, 1);
  dE[0] = ftd(0, 0);
  dE[1] = ftd(1, 1);
  dE[2] = ftd(2, 2);
  dE[3] = ftd(1, 2) + ftd(2, 1);
  dE[4] = ftd(0, 2) + ftd(2, 0);
  dE[5] = ftd(0, 1) + ftd(1, 0);
  T S[6], dS[6];
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    T a = 0, b = 0;
#pragma unroll
    for (int J = 0; J < 6; ++J) {
      const T c = C6[6 * I + J];
      a += c * E[J];
      b += c * dE[J];
    }
    S[I] = s * a;
    dS[I] = s * b;
  }
  const T Sm[9] = {S[0], S[5], S[4], S[5], S[1], S[3], S[4], S[3], S[2]};
  const T dSm[9] = {dS[0], dS[5], dS[4], dS[5], dS[1], dS[3], dS[4], dS[3], dS[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T acc = dSm[3 * i + j];
#pragma unroll
      for (int k = 0; k < 3; ++k) acc += d[3 * i + k] * Sm[3 * k + j] + H[3 * i + k] * dSm[3 * k + j];
      out[3 * i + j] = acc;
    }
}

// tangent of the viscoelastic law: K : d = d S + F (s C : sym(F^T d)), F = I + H, with the
// stress S taken from the state and C the algorithmic stiffness Cinf + b C1 of the increment
template <typename T>
__device__ __forceinline__ void tangent_visco(const T* H, const T* S, T s, const T* __restrict__ C6, const T* d, T* out) {
  auto ftd = [&](int i, int j) { return d[3 * i + j] + H[i] * d[j] + H[3 + i] * d[3 + j] + H[6 + i] * d[6 + j]; };
  T dE[6];
  dE[0] = ftd(0, 0);
  dE[1] = ftd(1, 1);
  dE[2] = ftd(2, 2);
  dE[3] = ftd(1, 2) + ftd(2, 1);
  dE[4] = ftd(0, 2) + ftd(2, 0);
  dE[5] = ftd(0, 1) + ftd(1, 0);
  T dS[6];
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    T acc = 0;
#pragma unroll
    for (int J = 0; J < 6; ++J) acc += C6[6 * I + J] * dE[J];
    dS[I] = s * acc;
  }
  const T Sm[9] = {S[0], S[5], S[4], S[5], S[1], S[3], S[4], S[3], S[2]};
  const T dSm[9] = {dS[0], dS[5], dS[4], dS[5], dS[1], dS[3], dS[4], dS[3], dS[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T acc = dSm[3 * i + j];
#pragma unroll
      for (int k = 0; k < 3; ++k) acc += d[3 * i + k] * Sm[3 * k + j] + H[3 * i + k] * dSm[3 * k + j];
      out[3 * i + j] = acc;
    }
}

// Constitutive update of one voxel in float64 (neo-Hookean or SVK, modulus scale s):
// P(F) into p, the tangent state into planes of N values at voxel v (CG type TS).
// Returns false when det F <= 0.
template <typename TS, int KIND>
__device__ __forceinline__ bool constitutive_point(const double* f, int ph, double s, bool has_scale,
                                                   const double* __restrict__ mat, double* p, TS* __restrict__ state,
                                                   long long N, long long v, const double* __restrict__ iv = nullptr) {
  const double cf0 = f[4] * f[8] - f[5] * f[7];
  const double cf1 = f[5] * f[6] - f[3] * f[8];
  const double cf2 = f[3] * f[7] - f[4] * f[6];
  const double J = f[0] * cf0 + f[1] * cf1 + f[2] * cf2;
  if constexpr (KIND == MAT_NH) {
    const double mu = s * mat[2 * ph], lam = s * mat[2 * ph + 1];
    // G = F^-T = cofactor(F) / J
    const double iJ = 1.0 / J;
    double G[9];
    G[0] = cf0 * iJ;
    G[1] = cf1 * iJ;
    G[2] = cf2 * iJ;
    G[3] = (f[2] * f[7] - f[1] * f[8]) * iJ;
    G[4] = (f[0] * f[8] - f[2] * f[6]) * iJ;
    G[5] = (f[1] * f[6] - f[0] * f[7]) * iJ;
    G[6] = (f[1] * f[5] - f[2] * f[4]) * iJ;
    G[7] = (f[2] * f[3] - f[0] * f[5]) * iJ;
    G[8] = (f[0] * f[4] - f[1] * f[3]) * iJ;
    const double lnJ = J > 0.0 ? log(J) : 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) p[c] = mu * (f[c] - G[c]) + lam * lnJ * G[c];
#pragma unroll
    for (int c = 0; c < 9; ++c) state[c * N + v] = (TS)G[c];
    state[9 * N + v] = (TS)mu;
    state[10 * N + v] = (TS)lam;
    state[11 * N + v] = (TS)(mu - lam * lnJ);
  } else if constexpr (KIND == MAT_VISCO) {
    // S = s Cinf : E + Q, Q = a Q_n + b s C1 : (E - E_n) (exact over the increment for E
    // linear in time); the tangent state keeps S, since it is not a function of F alone
    const double* t = mat + kViscoTable * ph;
    const double a = t[72], b = t[73];
    auto ftf = [&](int i, int j) { return f[i] * f[j] + f[3 + i] * f[3 + j] + f[6 + i] * f[6 + j]; };
    double E[6];
    E[0] = 0.5 * (ftf(0, 0) - 1.0);
    E[1] = 0.5 * (ftf(1, 1) - 1.0);
    E[2] = 0.5 * (ftf(2, 2) - 1.0);
    E[3] = ftf(1, 2);
    E[4] = ftf(0, 2);
    E[5] = ftf(0, 1);
    double dE[6];
#pragma unroll
    for (int J = 0; J < 6; ++J) dE[J] = E[J] - iv[J * N + v];
    double S[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) {
      double ci = 0.0, c1 = 0.0;
#pragma unroll
      for (int J = 0; J < 6; ++J) {
        ci += t[6 * I + J] * E[J];
        c1 += t[36 + 6 * I + J] * dE[J];
      }
      S[I] = s * ci + a * iv[(6 + I) * N + v] + b * s * c1;
    }
    const double Sm[9] = {S[0], S[5], S[4], S[5], S[1], S[3], S[4], S[3], S[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        p[3 * i + j] = f[3 * i] * Sm[j] + f[3 * i + 1] * Sm[3 + j] + f[3 * i + 2] * Sm[6 + j];
#pragma unroll
    for (int c = 0; c < 9; ++c) state[c * N + v] = (TS)(c % 4 == 0 ? f[c] - 1.0 : f[c]);
#pragma unroll
    for (int I = 0; I < 6; ++I) state[(9 + I) * N + v] = (TS)S[I];
    if (has_scale) state[15 * N + v] = (TS)s;
  } else {
    const double* C6 = mat + 36 * ph;
    // E = (F^T F - I)/2 in Voigt with engineering shears
    auto ftf = [&](int i, int j) { return f[i] * f[j] + f[3 + i] * f[3 + j] + f[6 + i] * f[6 + j]; };
    double E[6];
    E[0] = 0.5 * (ftf(0, 0) - 1.0);
    E[1] = 0.5 * (ftf(1, 1) - 1.0);
    E[2] = 0.5 * (ftf(2, 2) - 1.0);
    E[3] = ftf(1, 2);
    E[4] = ftf(0, 2);
    E[5] = ftf(0, 1);
    double S[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) {
      double acc = 0.0;
#pragma unroll
      for (int J2 = 0; J2 < 6; ++J2) acc += C6[6 * I + J2] * E[J2];
      S[I] = s * acc;
    }
    const double Sm[9] = {S[0], S[5], S[4], S[5], S[1], S[3], S[4], S[3], S[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        p[3 * i + j] = f[3 * i] * Sm[j] + f[3 * i + 1] * Sm[3 + j] + f[3 * i + 2] * Sm[6 + j];
#pragma unroll
    for (int c = 0; c < 9; ++c) state[c * N + v] = (TS)(c % 4 == 0 ? f[c] - 1.0 : f[c]);
    if (has_scale) state[9 * N + v] = (TS)s;
  }
  return J > 0.0;
}

// ---------------------------------------------------------------------------------
// z forward pass: per voxel input (plain copy or K : p), real-to-complex along z
// ---------------------------------------------------------------------------------
// Z_CONST_*: the forward pass of the Newton residual with the constitutive update fused
// in: F -> P (written), tangent state (written, CG type TIN), sums of F and P per block,
// and P goes into the transform.
enum { Z_PLAIN = 0, Z_NH = 1, Z_SVK = 2, Z_CONST_NH = 3, Z_CONST_SVK = 4, Z_VISCO = 5, Z_CONST_VISCO = 6 };

// Threads per workgroup of the z passes: the CG-step passes (zfwd_ntmin here, zinv_ntmin with
// the inverse pass) take GHOM_ZNT_MIN_CG threads where that fills the last round of the staged
// per-voxel loop better (at 256^3: 512 voxels, 2 per thread instead of 2.67 with 192 threads;
// float32 inverse pass 0.598 -> 0.574 ms, float64 CG passes -3%; 48^3 and 128^3 gain too, 96^3
// and 192^3, which fill 128 threads exactly, would lose 2-3%); the Newton-level passes run
// 6-10% slower with more threads and keep the transform's own count.
#ifndef GHOM_ZNT_MIN_CG
#define GHOM_ZNT_MIN_CG 256
#endif
template <int MODE> constexpr int zfwd_ntmin() {
  return (MODE == Z_NH || MODE == Z_SVK || MODE == Z_VISCO) ? GHOM_ZNT_MIN_CG : 0;
}

template <typename T, typename TIN>
struct ZfwdArgs {
  const TIN* in;              // Z_PLAIN: field to transform (9 planes)
  const TIN* pend;            // Z_PLAIN, Newton re-projection: the CG direction whose pending step
  TIN pend_alpha;             //   pend_alpha pend is added to `in` (pend_mode 2) or replaces it (1)
  int pend_mode;
  T* p;                       // Z_NH/Z_SVK: CG direction (updated in place when update_p)
  T* r;                       // CG residual
  T* x;                       // CG iterate: update_p == 1 applies the previous step's alpha p to it
  int x_mode;                 // update_p == 1: 1 x <- alpha p (x not yet written), 2 x <- x + alpha p
  T alpha;                    // the previous CG step's alpha
  const double* b;            // update_p == 2: the Newton right-hand side
  int update_p;               // 0: p as is; 1: x <- x + alpha p, p <- r + beta p; 2 (CG start): r <- b, p <- b;
                              // 3 (CG start, right-hand side already in r): p <- r
  const T* state;             // tangent state planes
  const uint16_t* phase;      // SVK: phase of each voxel
  const T* C6;                // SVK: per-phase 6x6 Voigt stiffness in the CG type
  int has_scale;              // SVK: state plane 9 holds s(x) (else s = 1)
  double* partials;           // nullable: per-block partials (p : K : p, or the Z_CONST sums)
  cx<T>* H;                   // spectrum out
  const cx<T>* tw;            // z twiddles
  const CGScalars* sc;        // early exit / beta (nullable)
  // Z_CONST_*
  const double* F;            // deformation gradient
  double* P;                  // stress out (viscoelastic law only)
  TIN* state_out;             // tangent state out
  const double* scale;        // per-voxel modulus scale (nullable)
  const double* mat;          // per-phase material table (float64)
  const double* iv;           // viscoelastic law: internal variables of the last increment
  int* flag;                  // set when det F <= 0 somewhere
  int pstride;                // Z_CONST sums: column k of block bx at partials[k * pstride + bx]
};

// Staged per-voxel loops in the z passes: every load of a chunk of a thread's voxels is
// issued before the first of them is used (in a plain loop the stores of one voxel hold back
// the loads of the next, since the compiler cannot rule out that they alias).  It costs
// registers; measured at 256^3: float32 CG passes (all voxels in one chunk) forward 0.651 ->
// 0.578 ms, inverse 0.676 -> 0.664 ms; float64 CG passes forward (one chunk) 1.270 -> 1.173
// ms, inverse (chunks of two: one chunk loses occupancy) 1.333 -> 1.308 ms; float64 Newton
// update 0.998 -> 0.755 ms.  The residual pass (constitutive update fused) runs slower staged.
#ifndef GHOM_ZPF_DEPTH64_FWD
#define GHOM_ZPF_DEPTH64_FWD 8
#endif
#ifndef GHOM_ZPF_DEPTH64_INV
#define GHOM_ZPF_DEPTH64_INV 2
#endif
// voxels per chunk of a staged CG loop of trip count it: all of them in float32, at most
// GHOM_ZPF_DEPTH64_FWD / _INV in float64 (twice the registers per value)
template <typename T, bool FWD> constexpr int zpf_depth(int it) {
  return sizeof(T) == 4 ? it : cmin(it, FWD ? GHOM_ZPF_DEPTH64_FWD : GHOM_ZPF_DEPTH64_INV);
}

// CG forward pass, per-voxel stage: p update and K : p of this thread's voxels into LDS, in
// chunks of SD voxels whose loads are all issued first; returns this thread's share of p : K : p
template <typename T, int LP, int NT, int NZ, int R, int MODE, typename TIN, int SD, bool NTS>
__device__ __forceinline__ double zfwd_cg_fill(const Geo& g, const ZfwdArgs<T, TIN>& args, long long line0,
                                               long long nlines, T beta, T* __restrict__ ldsr) {
  constexpr bool kNT = NTS;  // nontemporal streamed accesses
  constexpr int IT = (2 * LP * NZ + NT - 1) / NT;
  constexpr int KS = MODE == Z_NH ? kNHState : (MODE == Z_SVK ? 9 : 15);
  // with one thread per z (NT == NZ) item k of a thread is line k at z = threadIdx.x, so a
  // chunk of an even number of items holds whole line pairs: each component goes to LDS as one
  // complex store (re: line 2m, im: line 2m + 1) instead of two real stores 8 B apart, which
  // take two passes through the LDS banks
  constexpr bool kLdsPairs = NT == NZ && SD % 2 == 0 && IT % SD == 0;
  const long long N = g.N;
  double pkp = 0.0;
#pragma unroll
  for (int c0 = 0; c0 < IT; c0 += SD) {
    long long vx[SD];
    bool ok[SD];
#pragma unroll
    for (int k = 0; k < SD; ++k) {
      const int t = threadIdx.x + (c0 + k) * NT;
      const int lp = t / NZ, z = t - lp * NZ;
      ok[k] = c0 + k < IT && t < 2 * LP * NZ && line0 + lp < nlines;
      vx[k] = ok[k] ? (line0 + lp) * NZ + z : 0;  // voxel 0 stands in (in bounds) for idle slots
    }
    T dv[SD][9];
    if (args.update_p == 2) {
#pragma unroll
      for (int k = 0; k < SD; ++k)
#pragma unroll
        for (int c = 0; c < 9; ++c) dv[k][c] = (T)ld_s<kNT>(&args.b[c * N + vx[k]]);
    } else if (args.update_p == 3) {
#pragma unroll
      for (int k = 0; k < SD; ++k)
#pragma unroll
        for (int c = 0; c < 9; ++c) dv[k][c] = ld_s<kNT>(&args.r[c * N + vx[k]]);
    } else if (args.update_p == 1) {
      // the CG iterate takes the previous step's alpha p here, where p is read anyway (so the
      // inverse pass reads neither x nor p); p <- r + beta p
      T rv[SD][9], xv[SD][9];
      const bool xadd = args.x_mode == 2;
#pragma unroll
      for (int k = 0; k < SD; ++k)
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          rv[k][c] = ld_s<kNT>(&args.r[c * N + vx[k]]);
          dv[k][c] = ld_s<kNT>(&args.p[c * N + vx[k]]);
          xv[k][c] = xadd ? ld_s<kNT>(&args.x[c * N + vx[k]]) : (T)0;
        }
#pragma unroll
      for (int k = 0; k < SD; ++k) {
        if (!ok[k]) continue;
#pragma unroll
        for (int c = 0; c < 9; ++c) st_s<kNT>(&args.x[c * N + vx[k]], xv[k][c] + args.alpha * dv[k][c]);
      }
#pragma unroll
      for (int k = 0; k < SD; ++k)
#pragma unroll
        for (int c = 0; c < 9; ++c) dv[k][c] = rv[k][c] + beta * dv[k][c];
    } else {
#pragma unroll
      for (int k = 0; k < SD; ++k)
#pragma unroll
        for (int c = 0; c < 9; ++c) dv[k][c] = ld_s<kNT>(&args.p[c * N + vx[k]]);
    }
    T st[SD][KS];
    T sv[SD];
    int ph[SD];
#pragma unroll
    for (int k = 0; k < SD; ++k) {
#pragma unroll
      for (int j = 0; j < KS; ++j) st[k][j] = ld_s<kNT>(&args.state[j * N + vx[k]]);
      if constexpr (MODE != Z_NH) {
        ph[k] = ld_s<kNT>(&args.phase[vx[k]]);
        sv[k] = args.has_scale ? ld_s<kNT>(&args.state[KS * N + vx[k]]) : (T)1;
      }
    }
    T pv[kLdsPairs ? SD : 1][9];  // kLdsPairs: the chunk's values, stored a line pair at a time
#pragma unroll
    for (int k = 0; k < SD; ++k) {
      const int t = threadIdx.x + (c0 + k) * NT;
      if (c0 + k >= IT || t >= 2 * LP * NZ) break;
      const int lp = t / NZ, z = t - lp * NZ;
      T* val = pv[kLdsPairs ? k : 0];
      if (ok[k]) {
        const T* d = dv[k];
        if (args.update_p == 2) {
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            st_s<kNT>(&args.r[c * N + vx[k]], d[c]);
            st_s<kNT>(&args.p[c * N + vx[k]], d[c]);
          }
        } else if (args.update_p == 1 || args.update_p == 3) {
#pragma unroll
          for (int c = 0; c < 9; ++c) st_s<kNT>(&args.p[c * N + vx[k]], d[c]);
        }
        if constexpr (MODE == Z_NH) tangent_nh(st[k], d, val);
        else if constexpr (MODE == Z_SVK) tangent_svk(st[k], sv[k], args.C6 + 36 * ph[k], d, val);
        else tangent_visco(st[k], st[k] + 9, sv[k], args.C6 + 36 * ph[k], d, val);
        if (args.partials) {
#pragma unroll
          for (int c = 0; c < 9; ++c) pkp += (double)d[c] * (double)val[c];
        }
      } else {
#pragma unroll
        for (int c = 0; c < 9; ++c) val[c] = 0;
      }
      if constexpr (!kLdsPairs) {
        const int pair = lp >> 1, part = lp & 1;
#pragma unroll
        for (int c = 0; c < 9; ++c) ldsr[2 * ((c * LP + pair) * R + z) + part] = val[c];
      }
    }
    if constexpr (kLdsPairs) {
#pragma unroll
      for (int k = 0; k < SD; k += 2) {
        const int pair = (c0 + k) >> 1;  // lines c0 + k and c0 + k + 1 at z = threadIdx.x
        cx<T>* L = reinterpret_cast<cx<T>*>(ldsr);
#pragma unroll
        for (int c = 0; c < 9; ++c) L[(c * LP + pair) * R + threadIdx.x] = cx<T>{pv[k][c], pv[k + 1][c]};
      }
    }
  }
  return pkp;
}

template <typename T, int A, int B, int MODE, typename TIN, bool NTS>
__device__ __forceinline__ void zfwd_body(const Geo& g, const ZfwdArgs<T, TIN>& args, int bx) {
  constexpr bool kNT = NTS;  // nontemporal streamed accesses
  using Cfg = ZCfg<T, A, B, zfwd_ntmin<MODE>()>;
  constexpr int LP = Cfg::LP, NT = Cfg::NT, NZ = A * B, R = Cfg::R;
  __shared__ cx<T> lds[9 * LP * R];
  __shared__ double red[(NT + 63) / 64];
  constexpr bool CONST = MODE == Z_CONST_NH || MODE == Z_CONST_SVK || MODE == Z_CONST_VISCO;
  constexpr bool CG = MODE == Z_NH || MODE == Z_SVK || MODE == Z_VISCO;
  constexpr int KIND = MODE == Z_CONST_NH ? MAT_NH : (MODE == Z_CONST_SVK ? MAT_SVK : MAT_VISCO);
  if (args.sc && args.sc->done) return;
  const long long nlines = (long long)g.nx * g.ny;
  const long long line0 = (long long)bx * (2 * LP);
  T* ldsr = reinterpret_cast<T*>(lds);
  double pkp = 0.0;
  double cs[CONST ? 18 : 1];  // Z_CONST: sums of F and P
#pragma unroll
  for (int k = 0; k < (CONST ? 18 : 1); ++k) cs[k] = 0.0;
  int bad = 0;
  const T beta = (CG && args.update_p == 1) ? (T)args.sc->beta : (T)0;

  // phase 1: per-voxel values into LDS, line pair (2m, 2m+1) -> (re, im)
  if constexpr (CG) {
    constexpr int SD = zpf_depth<T, true>((2 * LP * NZ + NT - 1) / NT);
    pkp = zfwd_cg_fill<T, LP, NT, NZ, R, MODE, TIN, SD, NTS>(g, args, line0, nlines, beta, ldsr);
  } else
  for (int t = threadIdx.x; t < 2 * LP * NZ; t += NT) {
    const int lp = t / NZ, z = t - lp * NZ;
    const long long line = line0 + lp;
    T val[9];
    if (line < nlines) {
      const long long vox = line * NZ + z;
      if constexpr (MODE == Z_PLAIN) {
        if (args.pend_mode) {
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const TIN xin = args.pend_mode == 2 ? ld_s<kNT>(&args.in[c * g.N + vox]) : (TIN)0;
            val[c] = (T)(xin + args.pend_alpha * ld_s<kNT>(&args.pend[c * g.N + vox]));
          }
        } else {
#pragma unroll
          for (int c = 0; c < 9; ++c) val[c] = (T)ld_s<kNT>(&args.in[c * g.N + vox]);
        }
      } else {  // fused residual: constitutive update
        double f[9], pv[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) f[c] = ld_s<kNT>(&args.F[c * g.N + vox]);
        const double sv = args.scale ? args.scale[vox] : 1.0;
        if (!constitutive_point<TIN, KIND>(f, args.phase[vox], sv, args.scale != nullptr, args.mat, pv, args.state_out,
                                           g.N, vox, args.iv))
          bad = 1;
        // the elastic laws' P field is not stored: it is a function of F, recomputed where it
        // is read; the viscoelastic law's P depends on internal variables that the increment's
        // commit replaces, so its P field is stored here
        if constexpr (MODE == Z_CONST_VISCO) {
#pragma unroll
          for (int c = 0; c < 9; ++c) st_s<kNT>(&args.P[c * g.N + vox], pv[c]);
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          val[c] = (T)pv[c];
          cs[c] += f[c];
          cs[9 + c] += pv[c];
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) val[c] = 0;
    }
    const int pair = lp >> 1, part = lp & 1;
#pragma unroll
    for (int c = 0; c < 9; ++c) ldsr[2 * ((c * LP + pair) * R + z) + part] = val[c];
  }
  __syncthreads();
  // phase 2: 9*LP complex transforms of length NZ (A threads each)
  constexpr int DIRZ = -1;
  const bool ft = threadIdx.x < Cfg::NF;
  const int f = ft ? threadIdx.x / A : 0, q = threadIdx.x - (threadIdx.x / A) * A;
  cx<T>* L = lds + f * R;
  cx<T> v[B];
  if (ft) {
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = L[q + A * b];
    four_step_first<A, B, DIRZ>(v, q, args.tw);
  }
  __syncthreads();
  if (ft) {
#pragma unroll
    for (int c = 0; c < B; ++c) L[c * (A + 1) + q] = v[c];
  }
  __syncthreads();
  if (ft) four_step_second<A, B, DIRZ>(v, q, [&](int c, int a) { return L[c * (A + 1) + a]; });
  __syncthreads();
  if (ft) {
#pragma unroll
    for (int e = 0; e < B; ++e) L[q + A * e] = v[e];
  }
  __syncthreads();
  // phase 3: split the two real lines' spectra, store kz < nzh
  const int nzh = g.nzh;
  for (int t = threadIdx.x; t < 9 * LP * nzh; t += NT) {
    const int ff = t / nzh, kz = t - ff * nzh;
    const int c = ff / LP, pair = ff - c * LP;
    const cx<T> Zk = lds[ff * R + kz];
    const cx<T> Zm = conj(lds[ff * R + (kz == 0 ? 0 : NZ - kz)]);
    const cx<T> Ak = (Zk + Zm) * (T)0.5;
    const cx<T> Bk = mul_i<-1>(Zk - Zm) * (T)0.5;
    const long long l0 = line0 + 2 * pair;
    if (l0 < nlines) st_cx<kNT>(&args.H[c * g.Nh + l0 * nzh + kz], Ak);
    if (l0 + 1 < nlines) st_cx<kNT>(&args.H[c * g.Nh + (l0 + 1) * nzh + kz], Bk);
  }
  if constexpr (CONST) {
    if (bad) atomicOr(args.flag, 1);
    __shared__ double sh[18 * ((NT + 63) / 64)];
    block_reduce_cols<NT, 18>(cs, sh, [&](int k, double t) { args.partials[(long long)k * args.pstride + bx] = t; });
  } else if (args.partials) {
    const double t = block_sum<NT>(pkp, red);
    if (threadIdx.x == 0) args.partials[bx] = t;
  }
}

// ---------------------------------------------------------------------------------
// z inverse pass: complex-to-real along z, write the field, fused partial dot products
// ---------------------------------------------------------------------------------
// ZI_PLAIN: the field goes to `out`; ZI_CG: CG update x += alpha p (x = alpha p on the
// first iteration), r -= alpha A p, partial r.r; ZI_NEWTON: Newton update F += field with
// the partials of max_x |dF(x)|^2 and of the sums of the new F (float64)
enum { ZI_PLAIN = 0, ZI_CG = 1, ZI_NEWTON = 2 };
template <int ZM> constexpr int zinv_ntmin() { return ZM == ZI_CG ? GHOM_ZNT_MIN_CG : 0; }

template <typename T, typename TOUT>
struct ZinvArgs {
  const cx<T>* H;
  TOUT* out;                  // ZI_PLAIN: 9 planes
  TOUT* r;                    // ZI_CG: r <- r - alpha Ap (the iterate is updated by the next forward pass)
  double* F;                  // ZI_NEWTON
  int self_dot;               // ZI_PLAIN: partial sum of out . out per block
  double* partials;           // ZI_CG / self_dot: one per block; ZI_NEWTON: 10 columns
  int pstride;                // ZI_NEWTON: column k of block bx at partials[k * pstride + bx]
  const cx<T>* tw;
  const CGScalars* sc;        // early exit (nullable)
};

template <typename T, int A, int B, typename TOUT, int ZM, bool NTS>
__device__ __forceinline__ void zinv_body(const Geo& g, const ZinvArgs<T, TOUT>& args, int bx) {
  constexpr bool kNT = NTS;  // nontemporal streamed accesses
  using Cfg = ZCfg<T, A, B, zinv_ntmin<ZM>()>;
  constexpr int LP = Cfg::LP, NT = Cfg::NT, NZ = A * B, R = Cfg::R;
  __shared__ cx<T> lds[9 * LP * R];
  __shared__ double red[(NT + 63) / 64];
  if (args.sc && args.sc->done) return;
  const long long nlines = (long long)g.nx * g.ny;
  const long long line0 = (long long)bx * (2 * LP);
  const int nzh = g.nzh;
  // phase 1: Z[k] = A[k] + i B[k] with Hermitian completion; Nyquist (even NZ) is zero
  // (all of a thread's spectrum loads are issued before its LDS stores: measured faster in
  // every inverse pass, e.g. the float64 residual's 0.465 -> 0.414 ms at 256^3)
  {
    constexpr int IT1 = (9 * LP * (NZ / 2 + 1) + NT - 1) / NT;  // nzh <= NZ / 2 + 1
    const int total = 9 * LP * nzh;
    cx<T> av[IT1], bv[IT1];
#pragma unroll
    for (int it = 0; it < IT1; ++it) {
      const int t = threadIdx.x + it * NT;
      const int tt = t < total ? t : 0;
      const int ff = tt / nzh, kz = tt - ff * nzh;
      const int c = ff / LP, pair = ff - c * LP;
      const long long l0 = line0 + 2 * pair;
      av[it] = (t < total && l0 < nlines) ? ld_cx<kNT>(&args.H[c * g.Nh + l0 * nzh + kz]) : cx<T>{0, 0};
      bv[it] = (t < total && l0 + 1 < nlines) ? ld_cx<kNT>(&args.H[c * g.Nh + (l0 + 1) * nzh + kz]) : cx<T>{0, 0};
    }
#pragma unroll
    for (int it = 0; it < IT1; ++it) {
      const int t = threadIdx.x + it * NT;
      if (t >= total) break;
      const int ff = t / nzh, kz = t - ff * nzh;
      const cx<T> a = av[it], b = bv[it];
      lds[ff * R + kz] = a + mul_i<+1>(b);
      if (kz > 0) lds[ff * R + NZ - kz] = conj(a) + mul_i<+1>(conj(b));
      if ((NZ % 2 == 0) && kz == 0) lds[ff * R + NZ / 2] = cx<T>{0, 0};
    }
  }
  __syncthreads();
  constexpr int DIRZ = +1;
  const bool ft = threadIdx.x < Cfg::NF;
  const int f = ft ? threadIdx.x / A : 0, q = threadIdx.x - (threadIdx.x / A) * A;
  cx<T>* L = lds + f * R;
  cx<T> v[B];
  if (ft) {
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = L[q + A * b];
    four_step_first<A, B, DIRZ>(v, q, args.tw);
  }
  __syncthreads();
  if (ft) {
#pragma unroll
    for (int c = 0; c < B; ++c) L[c * (A + 1) + q] = v[c];
  }
  __syncthreads();
  if (ft) four_step_second<A, B, DIRZ>(v, q, [&](int c, int a) { return L[c * (A + 1) + a]; });
  __syncthreads();
  if (ft) {
#pragma unroll
    for (int e = 0; e < B; ++e) L[q + A * e] = v[e];
  }
  __syncthreads();
  // phase 3: real lines out
  const T* ldsr = reinterpret_cast<const T*>(lds);
  double acc = 0.0;
  double fs[ZM == ZI_NEWTON ? 9 : 1];
#pragma unroll
  for (int c = 0; c < (ZM == ZI_NEWTON ? 9 : 1); ++c) fs[c] = 0.0;
  const TOUT alpha = ZM == ZI_CG ? (TOUT)args.sc->alpha : (TOUT)0;
  if constexpr (ZM == ZI_CG || ZM == ZI_NEWTON) {
    // every load of a chunk of this thread's voxels first, then the updates and stores (the
    // CG update in chunks of zpf_depth voxels, the Newton update all at once)
    constexpr int IT = (2 * LP * NZ + NT - 1) / NT;
    const long long N = g.N;
    long long vx[IT];
    bool ok[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int t = threadIdx.x + it * NT;
      const int lp = t / NZ, z = t - lp * NZ;
      ok[it] = t < 2 * LP * NZ && line0 + lp < nlines;
      vx[it] = ok[it] ? (line0 + lp) * NZ + z : 0;  // voxel 0 stands in (in bounds) for idle slots
    }
    if constexpr (ZM == ZI_CG) {
      constexpr int SD = zpf_depth<TOUT, false>(IT);
#pragma unroll
      for (int c0 = 0; c0 < IT; c0 += SD) {
        TOUT rv[SD][9];
#pragma unroll
        for (int k = 0; k < SD; ++k) {
          const long long v = c0 + k < IT ? vx[c0 + k] : 0;
#pragma unroll
          for (int c = 0; c < 9; ++c) rv[k][c] = ld_s<kNT>(&args.r[c * N + v]);
        }
        // one thread per z (NT == NZ): a chunk of an even number of items holds whole line
        // pairs, read from LDS as one complex value per component (see zfwd_cg_fill)
        constexpr bool kLdsPairs = NT == NZ && SD % 2 == 0 && IT % SD == 0;
        T lv[kLdsPairs ? SD : 1][9];
        if constexpr (kLdsPairs) {
          const cx<T>* L = reinterpret_cast<const cx<T>*>(ldsr);
#pragma unroll
          for (int k = 0; k < SD; k += 2) {
            const int pair = (c0 + k) >> 1;
#pragma unroll
            for (int c = 0; c < 9; ++c) {
              const cx<T> w = L[(c * LP + pair) * R + threadIdx.x];
              lv[k][c] = w.re;
              lv[k + 1][c] = w.im;
            }
          }
        }
#pragma unroll
        for (int k = 0; k < SD; ++k) {
          const int it = c0 + k;
          if (it >= IT) break;
          if (!ok[it]) continue;
          const int t = threadIdx.x + it * NT;
          const int lp = t / NZ, z = t - lp * NZ;
          const int pair = lp >> 1, part = lp & 1;
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const TOUT o = kLdsPairs ? (TOUT)lv[kLdsPairs ? k : 0][c] : (TOUT)ldsr[2 * ((c * LP + pair) * R + z) + part];
            const TOUT rn = rv[k][c] - alpha * o;
            st_s<kNT>(&args.r[c * N + vx[it]], rn);
            acc += (double)rn * (double)rn;
          }
        }
      }
    } else {
      double fv[IT][9];
#pragma unroll
      for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int c = 0; c < 9; ++c) fv[it][c] = ld_s<kNT>(&args.F[c * N + vx[it]]);
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int t = threadIdx.x + it * NT;
        if (!ok[it]) continue;
        const int lp = t / NZ, z = t - lp * NZ;
        const int pair = lp >> 1, part = lp & 1;
        double n2 = 0.0;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const double o = (double)ldsr[2 * ((c * LP + pair) * R + z) + part];
          const double fn = fv[it][c] + o;
          st_s<kNT>(&args.F[c * N + vx[it]], fn);
          n2 += o * o;
          fs[c] += fn;
        }
        acc = fmax(acc, n2);
      }
    }
  } else
  for (int t = threadIdx.x; t < 2 * LP * NZ; t += NT) {
    const int lp = t / NZ, z = t - lp * NZ;
    const long long line = line0 + lp;
    if (line >= nlines) continue;
    const long long vox = line * NZ + z;
    const int pair = lp >> 1, part = lp & 1;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const T o = ldsr[2 * ((c * LP + pair) * R + z) + part];
      st_s<kNT>(&args.out[c * g.N + vox], (TOUT)o);
      if (args.self_dot) acc += (double)o * (double)o;  // of the value before a narrowing store
    }
  }
  if constexpr (ZM == ZI_NEWTON) {
    __shared__ double sh[10 * ((NT + 63) / 64)];
    double v[10];
    v[0] = acc;
#pragma unroll
    for (int c = 0; c < 9; ++c) v[1 + c] = fs[c];
    block_reduce_cols<NT, 10, 1>(v, sh, [&](int k, double t) { args.partials[(long long)k * args.pstride + bx] = t; });
  } else if (ZM == ZI_CG || args.self_dot) {
    const double s = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) args.partials[bx] = s;
  }
}

// ---------------------------------------------------------------------------------
// constitutive update (FP64): P(F), tangent state, partial sums of F and P
// ---------------------------------------------------------------------------------
constexpr int kVoxThreads = 256;

template <typename TS, int KIND>
__device__ __forceinline__ void constitutive_body(const Geo& g, const double* __restrict__ F, double* __restrict__ P,
                                                  TS* __restrict__ state, const uint16_t* __restrict__ phase,
                                                  const double* __restrict__ scale, const double* __restrict__ mat,
                                                  const double* __restrict__ iv, double* __restrict__ partials,
                                                  int* __restrict__ flag, int bx, int gx) {
  double sums[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) sums[k] = 0.0;
  int bad = 0;
  for (long long v = (long long)bx * kVoxThreads + threadIdx.x; v < g.N;
       v += (long long)gx * kVoxThreads) {
    double f[9], p[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) f[c] = F[c * g.N + v];
    if (!constitutive_point<TS, KIND>(f, phase[v], scale ? scale[v] : 1.0, scale != nullptr, mat, p, state, g.N, v, iv))
      bad = 1;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      P[c * g.N + v] = p[c];
      sums[c] += f[c];
      sums[9 + c] += p[c];
    }
  }
  if (bad) atomicOr(flag, 1);
  __shared__ double sh[18 * (kVoxThreads / 64)];
  block_reduce_cols<kVoxThreads, 18>(sums, sh, [&](int k, double t) { partials[(long long)bx * 18 + k] = t; });
}

// ---------------------------------------------------------------------------------
// CG vector kernels
// ---------------------------------------------------------------------------------

// sum of nparts partials in a fixed order, by one block; four independent loads in
// flight per thread, so the block is not bound by one memory latency per partial
__device__ __forceinline__ double reduce_partials(const double* __restrict__ base, int nparts, long long stride,
                                                  double* red) {
  constexpr int NT = kRedThreads;
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 0.0;
  int i = threadIdx.x;
  for (; i + 7 * NT < nparts; i += 8 * NT) {  // eight loads in flight per thread
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += base[(long long)(i + k * NT) * stride];
  }
  for (; i < nparts; i += NT) a[0] += base[(long long)i * stride];
  return block_sum<NT>(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])), red);
}

// beta = r'.r' / r.r from the inverse z pass's partials, the iteration count and the stop
// test (one block); then the scalars are copied to sc_host, which the host reads (also when
// the step was skipped: a breakdown set in the step's y pass reaches the host this way)
__device__ __forceinline__ void cg_beta_body(CGScalars* sc, CGScalars* sc_host, const double* __restrict__ partials,
                                             int nparts) {
  __shared__ double red[kRedThreads / 64];
  if (!sc->done) {  // the same for every thread: only thread 0 below writes sc
    const double s = reduce_partials(partials, nparts, 1, red);
    if (threadIdx.x == 0) {
      sc->beta = s / sc->rr;
      sc->rr = s;
      sc->it += 1;
      double best = sc->best;
      int since = sc->since;
      const int st = cg_status_after_iteration(s, sc->thresh, sc->it, sc->max_it, best, since);
      sc->best = best;
      sc->since = since;
      if (st != CG_RUNNING) {
        sc->done = 1;
        sc->status = st;
      }
    }
  }
  if (threadIdx.x == 0) *sc_host = *sc;
}

// alpha = rr / p.Ap by one block of NT threads with
// eight partials in flight per thread.  It is run by the first block of the first y pass of
// a CG step, which starts after the forward z pass has written every partial; the inverse z
// pass, the first reader of alpha, starts after the y pass has ended.
template <int NT>
__device__ __forceinline__ void cg_alpha_block(CGScalars* sc, const double* __restrict__ partials, int nparts) {
  static_assert(NT % 64 == 0, "whole wavefronts (block_sum)");
  __shared__ double red[NT / 64];
  if (sc->done) return;  // no other block writes sc during this kernel: the same for all threads
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 0.0;
  int i = threadIdx.x;
  for (; i + 7 * NT < nparts; i += 8 * NT) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += partials[i + k * NT];
  }
  for (; i < nparts; i += NT) a[0] += partials[i];
  const double s = block_sum<NT>(((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7])), red);
  if (threadIdx.x == 0) {
    sc->pAp = s;
    if (!(s > 0.0) || !isfinite(s)) {
      sc->done = 1;
      sc->status = CG_BREAKDOWN;
    } else {
      sc->alpha = sc->rr / s;
    }
  }
}

// column k of a partials table (entry (i, k) at partials[i * si + k * sk], i < nparts) into
// out[k], reduced with max instead of sum if use_max (one block per column, fixed order)
__device__ __forceinline__ void sum_column_body(const double* __restrict__ partials, int nparts, int k, bool use_max,
                                                long long si, long long sk, double* __restrict__ out) {
  __shared__ double red[kRedThreads / 64];
  const double* base = partials + (long long)k * sk;
  double r;
  if (use_max) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 3 * kRedThreads < nparts; i += 4 * kRedThreads) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = fmax(acc[u], base[(long long)(i + u * kRedThreads) * si]);
    }
    for (; i < nparts; i += kRedThreads) acc[0] = fmax(acc[0], base[(long long)i * si]);
    r = block_max<kRedThreads>(fmax(fmax(acc[0], acc[1]), fmax(acc[2], acc[3])), red);
  } else {
    r = reduce_partials(base, nparts, si, red);
  }
  if (threadIdx.x == 0) out[k] = r;
}

// F += dF; partials: max |dF(x)|^2 and sums of F (10 columns).  dF is the CG iterate x with
// the solve's pending step (cg_pending_mode) added here: dF = [x] + alpha p.
template <typename TD>
__device__ __forceinline__ void newton_update_body(const Geo& g, double* __restrict__ F, const TD* __restrict__ x,
                                                   const TD* __restrict__ p, TD alpha, int mode,
                                                   double* __restrict__ partials, int bx, int gx) {
  __shared__ double red[10 * (kVoxThreads / 64)];
  double mx = 0.0;
  double sums[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) sums[c] = 0.0;
  for (long long v = (long long)bx * kVoxThreads + threadIdx.x; v < g.N; v += (long long)gx * kVoxThreads) {
    double n2 = 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const long long i = c * g.N + v;
      const double d = mode == 0 ? (double)x[i] : (double)((mode == 2 ? x[i] : (TD)0) + alpha * p[i]);
      const double fn = F[i] + d;
      F[c * g.N + v] = fn;
      n2 += d * d;
      sums[c] += fn;
    }
    mx = fmax(mx, n2);
  }
  double v[10];
  v[0] = mx;
#pragma unroll
  for (int c = 0; c < 9; ++c) v[1 + c] = sums[c];
  block_reduce_cols<kVoxThreads, 10, 1>(v, red, [&](int k, double t) { partials[(long long)bx * 10 + k] = t; });
}

__device__ __forceinline__ void shift_body(long long N, double* __restrict__ F, const double* s, int bx, int gx) {
  for (long long v = (long long)bx * kVoxThreads + threadIdx.x; v < N; v += (long long)gx * kVoxThreads) {
#pragma unroll
    for (int c = 0; c < 9; ++c)
      if (s[c] != 0.0) F[c * N + v] += s[c];
  }
}

// uniform field value[c] in every voxel (FP64)
__device__ __forceinline__ void fill9_body(long long N, double* __restrict__ out, const double* val, int bx, int gx) {
  for (long long v = (long long)bx * kVoxThreads + threadIdx.x; v < N; v += (long long)gx * kVoxThreads) {
#pragma unroll
    for (int c = 0; c < 9; ++c) out[c * N + v] = val[c];
  }
}

// dJ/ds(x) = -(lam(x) : P(x)) / s(x), lam the adjoint field (already divided by N)
template <typename TL>
__device__ __forceinline__ void adjoint_grad_body(long long N, const TL* __restrict__ lam, const double* __restrict__ P,
                                                  const double* __restrict__ scale, double inv_n,
                                                  double* __restrict__ grad, int bx, int gx) {
  for (long long v = (long long)bx * kVoxThreads + threadIdx.x; v < N; v += (long long)gx * kVoxThreads) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) acc += (double)lam[c * N + v] * P[c * N + v];
    grad[v] = -acc * inv_n / (scale ? scale[v] : 1.0);
  }
}

// =================================================================================
// Batched launches.  Every pass runs over a set of problems of one grid shape: the
// problem is blockIdx.z (through `ids`), the tile inside it blockIdx.x (and .y).  A
// single problem is a batch of one.
// =================================================================================
enum {
  ROLE_OP_CG = 0,     // CG step: zfwd on p (p <- r + beta p), zinv updates x, r
  ROLE_OP_PLAIN = 1,  // operator on `in`, result to `out`
  ROLE_RESID = 2,     // -G*(P - P-bar) into b, with b.b partials
  ROLE_REPROJ = 3,    // G*(x) into dF64 (float64)
  ROLE_PROJ = 4,      // G*(in) into out (float64)
  ROLE_NEWTON = 5,    // F += G*(x) (float64) with the Newton-update partials
  ROLE_ADJ = 6,       // G*(in) into b (float64) with b.b partials: an adjoint right-hand side
  ROLE_RESID_R = 7    // -G*(P - P-bar) into r (the CG type) with b.b partials: the Newton
                      // right-hand side where the solve starts from it (CG start mode 3)
};

struct ProbDesc {
  Geo g;
  int kind;          // MAT_NH or MAT_SVK
  int has_scale;
  unsigned mask;     // bit c: component c stress-controlled
  int active;        // nonzero while this problem takes part in the current solve
  double pbar[9];    // stress target of the current increment (stress-controlled comps)
  double shift[9];   // uniform shift of the deformation-controlled means
  double fill[9];    // value of a uniform fill
  double cg_thresh;  // CG stop: r.r <= cg_thresh
  double rr0;        // b.b of the right-hand side the next CG solve starts from
  int max_cg;
  double *F, *P, *b, *dF64;
  void *x, *r, *p, *state, *H;
  const uint16_t* phase;
  const double* scale;
  const double* mat;   // tangent table (float64): neo-Hookean (mu, lam), SVK / viscoelastic 6x6 Voigt
  const float* mat32;  // the 6x6 tables in float32
  const double* visc;  // viscoelastic law: per-phase Cinf, C1, a, b (kViscoTable each)
  double* iv;          // viscoelastic law: E_n, Q_n planes (kViscoIV x N)
  const cx<double>* tw64[3];
  const cx<float>* tw32[3];
  double* partials;  // this problem's partial sums
  CGScalars* sc;
  CGScalars* sc_host;  // the same scalars in mapped host memory (written after each CG step)
  double* red;       // reduced values (32)
  int* flag;         // det F <= 0 flag
  const void* in;    // ROLE_OP_PLAIN / ROLE_PROJ input
  void* out;         // ROLE_OP_PLAIN / ROLE_PROJ output; adjoint gradient
};

template <typename T> __device__ __forceinline__ const cx<T>* twd(const ProbDesc& d, int axis);
template <> __device__ __forceinline__ const cx<double>* twd<double>(const ProbDesc& d, int axis) { return d.tw64[axis]; }
template <> __device__ __forceinline__ const cx<float>* twd<float>(const ProbDesc& d, int axis) { return d.tw32[axis]; }

__device__ __forceinline__ bool resid_role(int role) { return role == ROLE_RESID || role == ROLE_RESID_R; }

__device__ __forceinline__ ProjParams proj_params(const ProbDesc& d, int role) {
  ProjParams pp;
  pp.mask = d.mask;
  const double n = (double)d.g.N;
  pp.post = (resid_role(role) ? -1.0 : 1.0) / n;
  pp.pbar = resid_role(role) ? d.pbar : nullptr;
  pp.n = n;
  return pp;
}

// NTS (this and the pass kernels below): nontemporal loads and stores of the streamed data
template <typename T, int A, int B, int MODE, typename TIN, bool NTS>
__global__ void __launch_bounds__((ZCfg<T, A, B, zfwd_ntmin<MODE>()>::NT))
zfwd_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int role, int update_p) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  ZfwdArgs<T, TIN> a{};
  if constexpr (MODE == Z_CONST_NH || MODE == Z_CONST_SVK || MODE == Z_CONST_VISCO) {
    a.F = d.F;
    a.P = d.P;
    a.state_out = reinterpret_cast<TIN*>(d.state);
    a.phase = d.phase;
    a.scale = d.has_scale ? d.scale : nullptr;
    a.mat = MODE == Z_CONST_VISCO ? d.visc : d.mat;
    a.iv = d.iv;
    a.flag = d.flag;
    a.partials = d.partials;
    a.pstride = (int)gridDim.x;
  } else if constexpr (MODE == Z_PLAIN) {
    a.in = resid_role(role) ? reinterpret_cast<const TIN*>(d.P)
                              : ((role == ROLE_REPROJ || role == ROLE_NEWTON) ? reinterpret_cast<const TIN*>(d.x)
                                                     : reinterpret_cast<const TIN*>(d.in));
    if (role == ROLE_NEWTON) {  // the Newton correction: the CG iterate with the solve's pending step
      a.pend = reinterpret_cast<const TIN*>(d.p);
      a.pend_alpha = (TIN)d.sc->alpha;
      a.pend_mode = cg_pending_mode(d.sc);
    }
  } else {
    const bool cg = role == ROLE_OP_CG;
    a.p = cg ? reinterpret_cast<T*>(d.p) : const_cast<T*>(reinterpret_cast<const T*>(d.in));
    a.r = reinterpret_cast<T*>(d.r);
    a.x = cg ? reinterpret_cast<T*>(d.x) : nullptr;
    a.b = d.b;
    a.update_p = cg ? update_p : 0;
    a.state = reinterpret_cast<const T*>(d.state);
    a.phase = d.phase;
    if constexpr (sizeof(T) == 8) a.C6 = reinterpret_cast<const T*>(d.mat);
    else a.C6 = reinterpret_cast<const T*>(d.mat32);
    a.has_scale = d.has_scale;
    a.partials = cg ? d.partials : nullptr;
    a.sc = cg ? d.sc : nullptr;
    if (cg && update_p == 1) {  // sc->it steps are done: the pending iterate update is step it - 1's
      a.x_mode = d.sc->it == 1 ? 1 : 2;
      a.alpha = (T)d.sc->alpha;
    }
  }
  a.H = reinterpret_cast<cx<T>*>(d.H);
  a.tw = twd<T>(d, 2);
  zfwd_body<T, A, B, MODE, TIN, NTS>(d.g, a, blockIdx.x);
}

// alpha_nparts > 0: block 0 of each problem first sets the CG step's alpha from that many
// partials of the forward z pass
template <typename T, int A, int B, int DIR, bool NTS, bool WIDE = true>
__global__ void __launch_bounds__((YPassCfg<T, A, B, WIDE>::NT))
ypass_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int role, Slab sl, int alpha_nparts) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  if (alpha_nparts > 0 && blockIdx.x == 0) {
    cg_alpha_block<YPassCfg<T, A, B, WIDE>::NT>(d.sc, d.partials, alpha_nparts);
    __syncthreads();  // a breakdown (done = 1) is seen by every thread of the block below
  }
  ypass_body<T, A, B, DIR, NTS, WIDE>(d.g, sl, reinterpret_cast<cx<T>*>(d.H), twd<T>(d, 1),
                                      role == ROLE_OP_CG ? d.sc : nullptr, blockIdx.x);
}

template <typename T, typename S, int DIR, bool NTS>
__global__ void __launch_bounds__((Y3Cfg<T, S>::NT))
ypass3_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int role, Slab sl, int alpha_nparts) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  if (alpha_nparts > 0 && blockIdx.x == 0) {
    cg_alpha_block<Y3Cfg<T, S>::NT>(d.sc, d.partials, alpha_nparts);
    __syncthreads();
  }
  ypass3_body<T, S, DIR, NTS>(d.g, sl, reinterpret_cast<cx<T>*>(d.H), twd<T>(d, 1), role == ROLE_OP_CG ? d.sc : nullptr,
                              blockIdx.x);
}

// WAVES > 1: at least that many waves per SIMD, a register cap (the "rows, capped" variant;
// it pays where the uncapped kernel runs one wave per SIMD and spills little when capped).
// The cap is lowered to what the workgroup's LDS allows (160 KiB per CU, 4 SIMDs).
template <typename T, int A, int B, int WAVES> constexpr int xrows_waves() {
  using Cfg = XRowsCfg<T, A, B>;
  constexpr int lds = Cfg::LDS * (int)sizeof(cx<T>) + 64;
  constexpr int per_simd = (160 * 1024 / lds) * (Cfg::NT / 64) / 4;
  return cmax(1, cmin(WAVES, per_simd));
}
template <typename T, int A, int B, int WAVES, bool NTS>
__global__ void __launch_bounds__((XRowsCfg<T, A, B>::NT), (xrows_waves<T, A, B, WAVES>()))
xproj_rows_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int role, Slab sl) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  const ProjParams pp = proj_params(d, role);
  xproj_rows_body<T, A, B, NTS>(d.g, sl, reinterpret_cast<cx<T>*>(d.H), twd<T>(d, 0), pp,
                           role == ROLE_OP_CG ? d.sc : nullptr, blockIdx.x, blockIdx.y);
}

template <typename T, int A, int B, bool NTS>
__global__ void __launch_bounds__((XCfg<T, A, B>::NT))
xproj_groups_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int role, Slab sl) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  const ProjParams pp = proj_params(d, role);
  xproj_groups_body<T, A, B, NTS>(d.g, sl, reinterpret_cast<cx<T>*>(d.H), twd<T>(d, 0), pp,
                             role == ROLE_OP_CG ? d.sc : nullptr, blockIdx.x, blockIdx.y);
}

template <typename T, typename S, bool NTS>
__global__ void __launch_bounds__((XRows3Cfg<T, S>::NT))
xproj_rows3_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int role, Slab sl) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  const ProjParams pp = proj_params(d, role);
  xproj_rows3_body<T, S, NTS>(d.g, sl, reinterpret_cast<cx<T>*>(d.H), twd<T>(d, 0), pp,
                              role == ROLE_OP_CG ? d.sc : nullptr, blockIdx.x, blockIdx.y);
}

template <typename T, int A, int B, typename TOUT, int ZM, bool NTS>
__global__ void __launch_bounds__((ZCfg<T, A, B, zinv_ntmin<ZM>()>::NT))
zinv_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int role, int first) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  ZinvArgs<T, TOUT> a{};
  a.H = reinterpret_cast<const cx<T>*>(d.H);
  a.tw = twd<T>(d, 2);
  a.partials = d.partials;
  if constexpr (ZM == ZI_CG) {
    a.r = reinterpret_cast<TOUT*>(d.r);
    a.sc = d.sc;
  } else if constexpr (ZM == ZI_NEWTON) {
    a.F = d.F;
    a.pstride = (int)gridDim.x;
  } else {
    a.out = role == ROLE_RESID_R ? reinterpret_cast<TOUT*>(d.r)
            : (role == ROLE_RESID || role == ROLE_ADJ)
                ? reinterpret_cast<TOUT*>(d.b)
                : (role == ROLE_REPROJ ? reinterpret_cast<TOUT*>(d.dF64) : reinterpret_cast<TOUT*>(d.out));
    a.self_dot = resid_role(role) || role == ROLE_ADJ;
  }
  zinv_body<T, A, B, TOUT, ZM, NTS>(d.g, a, blockIdx.x);
}

template <typename TS, int KIND>
__global__ void __launch_bounds__(kVoxThreads)
constitutive_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  constitutive_body<TS, KIND>(d.g, d.F, d.P, reinterpret_cast<TS*>(d.state), d.phase, d.has_scale ? d.scale : nullptr,
                              KIND == MAT_VISCO ? d.visc : d.mat, d.iv, d.partials, d.flag, blockIdx.x, gridDim.x);
}

// End of an accepted increment of the viscoelastic law: E_n <- E(F), Q_n <- a Q_n +
// b s C1 : (E - E_n) at the converged F
__global__ void __launch_bounds__(kVoxThreads)
visco_commit_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  const long long N = d.g.N;
  for (long long v = (long long)blockIdx.x * kVoxThreads + threadIdx.x; v < N; v += (long long)gridDim.x * kVoxThreads) {
    double f[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) f[c] = d.F[c * N + v];
    const double s = d.has_scale ? d.scale[v] : 1.0;
    const double* t = d.visc + kViscoTable * d.phase[v];
    auto ftf = [&](int i, int j) { return f[i] * f[j] + f[3 + i] * f[3 + j] + f[6 + i] * f[6 + j]; };
    double E[6];
    E[0] = 0.5 * (ftf(0, 0) - 1.0);
    E[1] = 0.5 * (ftf(1, 1) - 1.0);
    E[2] = 0.5 * (ftf(2, 2) - 1.0);
    E[3] = ftf(1, 2);
    E[4] = ftf(0, 2);
    E[5] = ftf(0, 1);
    double dE[6];
#pragma unroll
    for (int J = 0; J < 6; ++J) dE[J] = E[J] - d.iv[J * N + v];
#pragma unroll
    for (int I = 0; I < 6; ++I) {
      double c1 = 0.0;
#pragma unroll
      for (int J = 0; J < 6; ++J) c1 += t[36 + 6 * I + J] * dE[J];
      d.iv[(6 + I) * N + v] = t[72] * d.iv[(6 + I) * N + v] + t[73] * s * c1;
    }
#pragma unroll
    for (int J = 0; J < 6; ++J) d.iv[J * N + v] = E[J];
  }
}


// CG start for every problem of a launch (one thread each): stop rule, iteration cap and
// r.r = b.b from the descriptor.  The first iteration's passes take r = p = b and x = 0
// themselves.  A problem that needs no iteration (or takes no part) starts finished.
__global__ void cg_start_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int np) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const ProbDesc& d = D[ids[i]];
  CGScalars* sc = d.sc;
  sc->thresh = d.cg_thresh;
  sc->max_it = d.max_cg;
  sc->it = 0;
  sc->rr = d.rr0;
  sc->best = d.rr0;
  sc->since = 0;
  const int stop = !d.active || !(d.rr0 > d.cg_thresh);
  sc->done = stop;
  sc->status = stop ? CG_CONVERGED : CG_RUNNING;
  *d.sc_host = *sc;
}

// one block per problem
__global__ void __launch_bounds__(kRedThreads)
cg_beta_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int nparts) {
  const ProbDesc& d = D[ids[blockIdx.x]];
  if (!d.active) return;
  cg_beta_body(d.sc, d.sc_host, d.partials, nparts);
}

// End of a CG solve: the step the last iteration completed (converged, cap or stall, with
// at least one step) has not yet moved the iterate, since the forward pass of the following
// iteration applies it: x <- x + alpha p (x <- alpha p after a single step).  After a
// breakdown the forward pass of the breaking iteration has applied it already.
template <typename T>
__global__ void __launch_bounds__(kVoxThreads)
cg_finish_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  const int mode = cg_pending_mode(d.sc);
  if (!mode) return;
  const T alpha = (T)d.sc->alpha;
  T* x = reinterpret_cast<T*>(d.x);
  const T* p = reinterpret_cast<const T*>(d.p);
  const long long n = 9 * d.g.N;
  for (long long i = (long long)blockIdx.x * kVoxThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kVoxThreads)
    x[i] = (mode == 2 ? x[i] : (T)0) + alpha * p[i];
}

// layout 0: entry (i, k) at i * K + k; layout 1: at k * nparts + i.  Results go to
// red[off .. off + K); the first nmax columns are maxima.  Grid: (problems, K), one block per
// column of a problem.
__global__ void __launch_bounds__(kRedThreads)
sum_columns_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int nparts, int K, int nmax,
                  int layout, int off, int with_flag) {
  const ProbDesc& d = D[ids[blockIdx.x]];
  if (!d.active) return;
  const int k = blockIdx.y;
  sum_column_body(d.partials, nparts, k, k < nmax, layout ? 1 : K, layout ? nparts : 1, d.red + off);
  // the det F <= 0 flag of the constitutive update (set by device atomics) rides along
  if (with_flag && k == 0 && threadIdx.x == 0) d.red[kRedFlag] = (double)*d.flag;
}

// F += x in FP64 mode (in FP32-split mode the re-projection's inverse pass applies the
// update itself, zinv_batch<..., ZI_NEWTON>)
__global__ void __launch_bounds__(kVoxThreads)
newton_update_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  newton_update_body<double>(d.g, d.F, reinterpret_cast<const double*>(d.x), reinterpret_cast<const double*>(d.p),
                             d.sc->alpha, cg_pending_mode(d.sc), d.partials, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kVoxThreads)
shift_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  shift_body(d.g.N, d.F, d.shift, blockIdx.x, gridDim.x);
}

// which: 0 = F (reset to the fill value), 1 = b (uniform right-hand side)
__global__ void __launch_bounds__(kVoxThreads)
fill9_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int which) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  fill9_body(d.g.N, which == 0 ? d.F : d.b, d.fill, blockIdx.x, gridDim.x);
}

__global__ void zero_flag_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *D[ids[i]].flag = 0;
}

// dJ/ds from the adjoint solution (float64: x in FP64 mode, re-projected dF64 in split mode)
__global__ void __launch_bounds__(kVoxThreads)
adjoint_grad_batch(const ProbDesc* __restrict__ D, const int* __restrict__ ids) {
  const ProbDesc& d = D[ids[blockIdx.z]];
  if (!d.active) return;
  const double* lam = d.dF64 ? d.dF64 : reinterpret_cast<const double*>(d.x);
  adjoint_grad_body<double>(d.g.N, lam, d.P, d.has_scale ? d.scale : nullptr, 1.0 / (double)d.g.N,
                            reinterpret_cast<double*>(d.out), blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------------
// Adjoint through a viscoelastic history (one problem; the backward sweep of the history
// adjoint).  Symmetric tensors are 6 tensor components (11 22 33 23 13 12); contractions
// carry the weights (1, 1, 1, 2, 2, 2); the Voigt tables act on engineering strains.
// mu holds mE (6 planes) then mQ (6 planes).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double voigt_w(int I) { return I < 3 ? 1.0 : 2.0; }

// h = F (mE + b s C1 : mQ), plus the uniform abar when given (the last increment)
__global__ void __launch_bounds__(kVoxThreads)
visco_adj_rhs_kernel(long long N, const double* __restrict__ F, const uint16_t* __restrict__ phase,
                     const double* __restrict__ scale, const double* __restrict__ visc, const double* __restrict__ mu,
                     double* __restrict__ h, const double* __restrict__ abar) {
  for (long long v = (long long)blockIdx.x * kVoxThreads + threadIdx.x; v < N; v += (long long)gridDim.x * kVoxThreads) {
    const double* t = visc + kViscoTable * phase[v];
    const double bs = t[73] * (scale ? scale[v] : 1.0);
    double M[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) {
      double c = 0.0;
#pragma unroll
      for (int J = 0; J < 6; ++J) c += t[36 + 6 * I + J] * voigt_w(J) * mu[(6 + J) * N + v];
      M[I] = mu[I * N + v] + bs * c;
    }
    const double Mm[9] = {M[0], M[5], M[4], M[5], M[1], M[3], M[4], M[3], M[2]};
    double f[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) f[c] = F[c * N + v];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double acc = abar ? abar[3 * i + j] : 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc += f[3 * i + k] * Mm[3 * k + j];
        h[(3 * i + j) * N + v] = acc;
      }
  }
}

// With L = sym(F^T lam): grad += b mQ : C1 : (E - E_prev) - L : (Cinf : E + b C1 : (E - E_prev)),
// mE <- b s C1 : (L - mQ), mQ <- a (mQ - L).  E from F; E_prev from iv (engineering shears).
__global__ void __launch_bounds__(kVoxThreads)
visco_adj_update_kernel(long long N, const double* __restrict__ F, const double* __restrict__ iv,
                        const uint16_t* __restrict__ phase, const double* __restrict__ scale,
                        const double* __restrict__ visc, const double* __restrict__ lam, double* __restrict__ mu,
                        double* __restrict__ grad) {
  for (long long v = (long long)blockIdx.x * kVoxThreads + threadIdx.x; v < N; v += (long long)gridDim.x * kVoxThreads) {
    const double* t = visc + kViscoTable * phase[v];
    const double a = t[72], b = t[73];
    const double s = scale ? scale[v] : 1.0;
    double f[9], l[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      f[c] = F[c * N + v];
      l[c] = lam[c * N + v];
    }
    // (F^T lam)_ij = sum_k F_ki lam_kj
    auto ftl = [&](int i, int j) { return f[i] * l[j] + f[3 + i] * l[3 + j] + f[6 + i] * l[6 + j]; };
    double L[6];
    L[0] = ftl(0, 0);
    L[1] = ftl(1, 1);
    L[2] = ftl(2, 2);
    L[3] = 0.5 * (ftl(1, 2) + ftl(2, 1));
    L[4] = 0.5 * (ftl(0, 2) + ftl(2, 0));
    L[5] = 0.5 * (ftl(0, 1) + ftl(1, 0));
    auto ftf = [&](int i, int j) { return f[i] * f[j] + f[3 + i] * f[3 + j] + f[6 + i] * f[6 + j]; };
    double E[6];
    E[0] = 0.5 * (ftf(0, 0) - 1.0);
    E[1] = 0.5 * (ftf(1, 1) - 1.0);
    E[2] = 0.5 * (ftf(2, 2) - 1.0);
    E[3] = ftf(1, 2);
    E[4] = ftf(0, 2);
    E[5] = ftf(0, 1);
    double mQ[6], dE[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) {
      mQ[I] = mu[(6 + I) * N + v];
      dE[I] = E[I] - iv[I * N + v];
    }
    double g = 0.0;
#pragma unroll
    for (int I = 0; I < 6; ++I) {
      double c1 = 0.0, ci = 0.0, cl = 0.0;
#pragma unroll
      for (int J = 0; J < 6; ++J) {
        c1 += t[36 + 6 * I + J] * dE[J];
        ci += t[6 * I + J] * E[J];
        cl += t[36 + 6 * I + J] * voigt_w(J) * (L[J] - mQ[J]);
      }
      g += voigt_w(I) * (b * mQ[I] * c1 - L[I] * (ci + b * c1));
      mu[I * N + v] = b * s * cl;
    }
#pragma unroll
    for (int I = 0; I < 6; ++I) mu[(6 + I) * N + v] = a * (mQ[I] - L[I]);
    grad[v] += g;
  }
}

}  // namespace ghom
