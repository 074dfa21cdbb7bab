// libghom.so: host runtime and C ABI (include/ghom.h) of the Galerkin-FFT solver with
// stress / mixed control.  Every step of the method runs in the kernels of kernels.hpp on
// the context's HIP stream; the host only sequences launches, moves a few scalars and
// applies the stopping rules.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/ghom.h"
#include "kernels.hpp"

using namespace ghom;

namespace {

constexpr int kMaxVoxBlocks = 8192;

struct ProfRec {
  int launches = 0;
  double ms = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

}  // namespace

struct ghom_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int prec = GHOM_FP64;
  Geo g{};
  size_t tsz = 8;  // bytes of the CG type

  // fields (FP64 master copies)
  double* F = nullptr;
  double* P = nullptr;
  double* b = nullptr;
  double* dF64 = nullptr;  // split mode: re-projected Newton correction
  // CG vectors and tangent state in the CG type
  void* x = nullptr;
  void* r = nullptr;
  void* p = nullptr;
  void* state = nullptr;
  void* H = nullptr;  // spectrum, FP64 capacity
  // material
  int kind = 0;
  int nphase = 0;
  uint16_t* phase = nullptr;
  double* scale = nullptr;
  double* mat = nullptr;  // NH: (mu, lam) per phase; SVK: 36 Voigt values per phase
  float* mat32 = nullptr; // SVK: the Voigt table in float32 (tangent of the FP32 CG)
  bool state_valid = false;
  // twiddles W_n^k = exp(-2 pi i k / n) per axis
  cx<double>* tw64[3] = {nullptr, nullptr, nullptr};
  cx<float>* tw32[3] = {nullptr, nullptr, nullptr};
  // reductions
  double* partials = nullptr;
  size_t npartials = 0;
  CGScalars* sc = nullptr;
  int* flag = nullptr;
  double* red = nullptr;   // 32 reduced values
  double* host_red = nullptr;  // pinned mirror
  CGScalars* host_sc = nullptr;
  // control / history
  uint8_t mask[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  bool mask_set = false;
  std::vector<double> target;
  int nsteps = 0;
  int k = 0;
  double newton_tol = 1e-6, cg_tol = 1e-8, cg_forcing = 0.0;
  int max_newton = 50, max_cg = 5000;
  double Favg[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double Pavg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  std::string err;
  // x-pass variant per precision ([0] float64, [1] float32): 0 untuned, 1 rows, 2 groups
  int xproj_var[2] = {0, 0};
  // kz slabs of the middle passes (1 = whole spectrum per pass)
  int zslabs = 1;
  // profiling
  bool prof = false;
  std::map<std::string, ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

struct HipFail {
  hipError_t e;
  const char* what;
};

#define HIPCALL(expr)                          \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) throw HipFail{_e, #expr}; \
  } while (0)

struct ApiError {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg) { throw ApiError{code, msg}; }

template <typename F>
int guard(ghom_ctx* c, F&& f) {
  if (!c) return GHOM_EINVAL;
  try {
    c->err.clear();
    HIPCALL(hipSetDevice(c->device));
    return f();
  } catch (const ApiError& e) {
    c->err = e.msg;
    return e.code;
  } catch (const HipFail& e) {
    c->err = std::string("HIP error '") + hipGetErrorString(e.e) + "' in " + e.what;
    return e.e == hipErrorOutOfMemory ? GHOM_ENOMEM : GHOM_EHIP;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return GHOM_ENOMEM;
  }
}

hipEvent_t get_event(ghom_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCALL(hipEventCreate(&e));
  return e;
}

// Runs `launch` on the context stream, bracketed by events when profiling.
template <typename L>
void timed(ghom_ctx* c, const char* name, L&& launch) {
  if (!c->prof) {
    launch();
    HIPCALL(hipGetLastError());
    return;
  }
  hipEvent_t a = get_event(c), b = get_event(c);
  HIPCALL(hipEventRecord(a, c->stream));
  launch();
  HIPCALL(hipGetLastError());
  HIPCALL(hipEventRecord(b, c->stream));
  c->prof_recs[name].pending.emplace_back(a, b);
}

void prof_collect(ghom_ctx* c) {
  HIPCALL(hipStreamSynchronize(c->stream));
  for (auto& kv : c->prof_recs) {
    for (auto& pr : kv.second.pending) {
      float ms = 0.f;
      HIPCALL(hipEventElapsedTime(&ms, pr.first, pr.second));
      kv.second.ms += ms;
      kv.second.launches += 1;
      c->ev_pool.push_back(pr.first);
      c->ev_pool.push_back(pr.second);
    }
    kv.second.pending.clear();
  }
}

template <typename T> const char* tname();
template <> const char* tname<double>() { return "f64"; }
template <> const char* tname<float>() { return "f32"; }

template <typename T> const T* mat_table(ghom_ctx* c);
template <> const double* mat_table<double>(ghom_ctx* c) { return c->mat; }
template <> const float* mat_table<float>(ghom_ctx* c) { return c->mat32; }

template <typename T> cx<T>* twid(ghom_ctx* c, int axis);
template <> cx<double>* twid<double>(ghom_ctx* c, int axis) { return c->tw64[axis]; }
template <> cx<float>* twid<float>(ghom_ctx* c, int axis) { return c->tw32[axis]; }

int vox_blocks(long long n) {
  long long b = (n + kVoxThreads - 1) / kVoxThreads;
  return (int)(b < kMaxVoxBlocks ? (b < 1 ? 1 : b) : kMaxVoxBlocks);
}

// ------------------------------------------------------------------ pass launchers ----
template <typename T, int MODE, typename TIN>
int launch_zfwd(ghom_ctx* c, const ZfwdArgs<T, TIN>& a, const char* name) {
  int grid = 0;
  with_split(c->g.nz, [&](auto s) {
    using S = decltype(s);
    using Cfg = ZCfg<T, S::A, S::B>;
    const long long nlines = (long long)c->g.nx * c->g.ny;
    grid = (int)((nlines + 2 * Cfg::LP - 1) / (2 * Cfg::LP));
    timed(c, name, [&] {
      hipLaunchKernelGGL((zfwd_kernel<T, S::A, S::B, MODE, TIN>), dim3(grid), dim3(Cfg::NT), 0, c->stream, c->g, a);
    });
  });
  return grid;
}

template <typename T, typename TOUT, bool CGU = false>
int launch_zinv(ghom_ctx* c, const ZinvArgs<T, TOUT>& a, const char* name) {
  int grid = 0;
  with_split(c->g.nz, [&](auto s) {
    using S = decltype(s);
    using Cfg = ZCfg<T, S::A, S::B>;
    const long long nlines = (long long)c->g.nx * c->g.ny;
    grid = (int)((nlines + 2 * Cfg::LP - 1) / (2 * Cfg::LP));
    timed(c, name, [&] {
      hipLaunchKernelGGL((zinv_kernel<T, S::A, S::B, TOUT, CGU>), dim3(grid), dim3(Cfg::NT), 0, c->stream, c->g, a);
    });
  });
  return grid;
}

template <typename T, int DIR>
void launch_ypass(ghom_ctx* c, Slab sl, const CGScalars* sc, const char* name) {
  with_split(c->g.ny, [&](auto s) {
    using S = decltype(s);
    using Cfg = ColCfg<T, S::A, S::B>;
    const long long ncols = 9LL * c->g.nx * sl.nkz;
    const int grid = (int)((ncols + Cfg::TC - 1) / Cfg::TC);
    timed(c, name, [&] {
      hipLaunchKernelGGL((ypass_kernel<T, S::A, S::B, DIR>), dim3(grid), dim3(Cfg::NT), 0, c->stream, c->g, sl,
                         reinterpret_cast<cx<T>*>(c->H), twid<T>(c, 1), sc);
    });
  });
}

enum { XPROJ_TUNED = 0, XPROJ_ROWS = 1, XPROJ_GROUPS = 2 };

template <typename T> int& xproj_choice(ghom_ctx* c) { return c->xproj_var[sizeof(T) == 8 ? 0 : 1]; }

template <typename T>
void launch_xproj_variant(ghom_ctx* c, int variant, Slab sl, const ProjParams& pp, const CGScalars* sc) {
  with_split(c->g.nx, [&](auto s) {
    using S = decltype(s);
    const long long ncols = (long long)c->g.ny * sl.nkz;
    if (variant == XPROJ_ROWS) {
      using Cfg = ColCfg<T, S::A, S::B>;
      const int grid = (int)((ncols + Cfg::TC - 1) / Cfg::TC);
      hipLaunchKernelGGL((xproj_rows_kernel<T, S::A, S::B>), dim3(grid, 3), dim3(Cfg::NT), 0, c->stream, c->g, sl,
                         reinterpret_cast<cx<T>*>(c->H), twid<T>(c, 0), pp, sc);
    } else {
      using Cfg = XCfg<T, S::A, S::B>;
      const int grid = (int)((ncols + Cfg::TC - 1) / Cfg::TC);
      hipLaunchKernelGGL((xproj_groups_kernel<T, S::A, S::B>), dim3(grid, 3), dim3(Cfg::NT), 0, c->stream, c->g, sl,
                         reinterpret_cast<cx<T>*>(c->H), twid<T>(c, 0), pp, sc);
    }
  });
}

template <typename T>
void launch_xproj(ghom_ctx* c, Slab sl, const ProjParams& pp, const CGScalars* sc, const char* name) {
  const int v = xproj_choice<T>(c);
  timed(c, name, [&] { launch_xproj_variant<T>(c, v == XPROJ_TUNED ? XPROJ_ROWS : v, sl, pp, sc); });
}

// The three middle passes (y forward, x with the projection, y inverse), kz-slab by slab.
template <typename T>
void middle_passes(ghom_ctx* c, const ProjParams& pp, const CGScalars* sc, const std::string& pre) {
  const std::string t = tname<T>();
  const std::string n2 = pre + "yfwd_" + t, n3 = pre + "xproj_" + t, n4 = pre + "yinv_" + t;
  const int ns = std::max(1, std::min(c->zslabs, c->g.nzh));
  const int per = (c->g.nzh + ns - 1) / ns;
  for (int kz0 = 0; kz0 < c->g.nzh; kz0 += per) {
    const Slab sl{kz0, std::min(per, c->g.nzh - kz0)};
    launch_ypass<T, -1>(c, sl, sc, n2.c_str());
    launch_xproj<T>(c, sl, pp, sc, n3.c_str());
    launch_ypass<T, +1>(c, sl, sc, n4.c_str());
  }
}

// Autotuner: times both x-pass variants on the (scratch) spectrum buffer with HIP events
// and keeps the faster one for this precision and grid.  Runs at context creation, when the
// spectrum holds no data; the result is reported by ghom_get_option.
template <typename T>
void tune_xproj(ghom_ctx* c) {
  ProjParams pp{};
  pp.post = 1.0 / (double)c->g.N;
  hipEvent_t e0 = get_event(c), e1 = get_event(c);
  float best = 0.f;
  int best_v = XPROJ_ROWS;
  for (int v : {XPROJ_ROWS, XPROJ_GROUPS}) {
    const Slab full{0, c->g.nzh};
    launch_xproj_variant<T>(c, v, full, pp, nullptr);  // warm-up
    HIPCALL(hipGetLastError());
    float tmin = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      HIPCALL(hipEventRecord(e0, c->stream));
      launch_xproj_variant<T>(c, v, full, pp, nullptr);
      HIPCALL(hipGetLastError());
      HIPCALL(hipEventRecord(e1, c->stream));
      HIPCALL(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCALL(hipEventElapsedTime(&ms, e0, e1));
      if (rep == 0 || ms < tmin) tmin = ms;
    }
    if (v == XPROJ_ROWS || tmin < best) {
      best = tmin;
      best_v = v;
    }
  }
  c->ev_pool.push_back(e0);
  c->ev_pool.push_back(e1);
  xproj_choice<T>(c) = best_v;
}

ProjParams make_proj(ghom_ctx* c, double scale, const double* Pbar) {
  ProjParams pp{};
  pp.mask = 0;
  for (int i = 0; i < 9; ++i)
    if (c->mask[i]) pp.mask |= 1u << i;
  pp.post = scale / (double)c->g.N;
  for (int i = 0; i < 9; ++i) pp.off[i] = Pbar ? (double)c->g.N * Pbar[i] : 0.0;
  return pp;
}

// out = scale * G*(in - Pbar) on FP64 output; `in` of type TIN; optional self dot
template <typename TIN>
int project64(ghom_ctx* c, const TIN* in, double* out, double scale, const double* Pbar, bool self_dot,
              const char* tag) {
  ZfwdArgs<double, TIN> za{};
  za.in = in;
  za.H = reinterpret_cast<cx<double>*>(c->H);
  za.tw = c->tw64[2];
  std::string n1 = std::string(tag) + "_zfwd_f64", n2 = std::string(tag) + "_yfwd_f64",
              n3 = std::string(tag) + "_xproj_f64", n4 = std::string(tag) + "_yinv_f64",
              n5 = std::string(tag) + "_zinv_f64";
  launch_zfwd<double, Z_PLAIN, TIN>(c, za, n1.c_str());
  middle_passes<double>(c, make_proj(c, scale, Pbar), nullptr, std::string(tag) + "_");
  ZinvArgs<double, double> zi{};
  zi.H = reinterpret_cast<cx<double>*>(c->H);
  zi.out = out;
  zi.dot_with = self_dot ? out : nullptr;
  zi.partials = c->partials;
  zi.tw = c->tw64[2];
  return launch_zinv<double, double>(c, zi, n5.c_str());
}

// The operator A(v) = G*(K : v) in the CG type.
//  plain (cg == false): Av written to `Av`.
//  CG step (cg == true): v is the direction p (first updated to r + beta p when update_p);
//    zfwd leaves per-block partials of p : K : p (= p . A p, p lying in the range of G*) for
//    the alpha kernel, and zinv applies x += alpha p, r -= alpha A p with partials of r.r.
template <typename T>
void operator_apply(ghom_ctx* c, T* v, T* Av, bool cg, bool update_p, const CGScalars* sc, int* grid_out) {
  ZfwdArgs<T, T> za{};
  za.p = v;
  za.r = reinterpret_cast<const T*>(c->r);
  za.update_p = update_p ? 1 : 0;
  za.state = reinterpret_cast<const T*>(c->state);
  za.phase = c->phase;
  za.C6 = mat_table<T>(c);
  za.has_scale = c->scale != nullptr;
  za.partials = cg ? c->partials : nullptr;
  za.H = reinterpret_cast<cx<T>*>(c->H);
  za.tw = twid<T>(c, 2);
  za.sc = sc;
  const std::string t = tname<T>();
  const std::string n1 = "op_zfwd_" + t, n2 = "op_yfwd_" + t, n3 = "op_xproj_" + t, n4 = "op_yinv_" + t,
                    n5 = "op_zinv_" + t;
  int gz;
  if (c->kind == MAT_NH) gz = launch_zfwd<T, Z_NH, T>(c, za, n1.c_str());
  else gz = launch_zfwd<T, Z_SVK, T>(c, za, n1.c_str());
  if (grid_out) *grid_out = gz;
  if (cg) {
    timed(c, "cg_scalar", [&] {
      hipLaunchKernelGGL(cg_scalar_kernel, dim3(1), dim3(kRedThreads), 0, c->stream, c->sc, c->partials, gz, 1);
    });
  }
  middle_passes<T>(c, make_proj(c, 1.0, nullptr), sc, "op_");
  ZinvArgs<T, T> zi{};
  zi.H = reinterpret_cast<cx<T>*>(c->H);
  zi.partials = c->partials;
  zi.tw = twid<T>(c, 2);
  zi.sc = sc;
  if (cg) {
    zi.x = reinterpret_cast<T*>(c->x);
    zi.r = reinterpret_cast<T*>(c->r);
    zi.p = v;
    launch_zinv<T, T, true>(c, zi, n5.c_str());
  } else {
    zi.out = Av;
    launch_zinv<T, T, false>(c, zi, n5.c_str());
  }
}

void sync(ghom_ctx* c) { HIPCALL(hipStreamSynchronize(c->stream)); }

__global__ void zero_int_kernel(int* f) { *f = 0; }

__global__ void fill_zero_kernel(long long n, double* p) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// ------------------------------------------------------------------ method steps -------
// constitutive update: P, tangent state, <F>, <P>; EDOMAIN if det F <= 0 anywhere
void constitutive(ghom_ctx* c) {
  const int grid = vox_blocks(c->g.N);
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, c->stream, c->flag);
  HIPCALL(hipGetLastError());
  timed(c, "constitutive", [&] {
    if (c->kind == MAT_NH) {
      if (c->prec == GHOM_FP64)
        hipLaunchKernelGGL((constitutive_kernel<double, MAT_NH>), dim3(grid), dim3(kVoxThreads), 0, c->stream, c->g,
                           c->F, c->P, (double*)c->state, c->phase, c->scale, c->mat, c->partials, c->flag);
      else
        hipLaunchKernelGGL((constitutive_kernel<float, MAT_NH>), dim3(grid), dim3(kVoxThreads), 0, c->stream, c->g,
                           c->F, c->P, (float*)c->state, c->phase, c->scale, c->mat, c->partials, c->flag);
    } else {
      if (c->prec == GHOM_FP64)
        hipLaunchKernelGGL((constitutive_kernel<double, MAT_SVK>), dim3(grid), dim3(kVoxThreads), 0, c->stream, c->g,
                           c->F, c->P, (double*)c->state, c->phase, c->scale, c->mat, c->partials, c->flag);
      else
        hipLaunchKernelGGL((constitutive_kernel<float, MAT_SVK>), dim3(grid), dim3(kVoxThreads), 0, c->stream, c->g,
                           c->F, c->P, (float*)c->state, c->phase, c->scale, c->mat, c->partials, c->flag);
    }
  });
  timed(c, "reduce", [&] {
    hipLaunchKernelGGL(sum_columns_kernel, dim3(1), dim3(kRedThreads), 0, c->stream, c->partials, grid, 18, 0,
                       c->red);
  });
  HIPCALL(hipMemcpyAsync(c->host_red, c->red, 18 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCALL(hipMemcpyAsync(c->host_red + 24, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  int bad = 0;
  std::memcpy(&bad, c->host_red + 24, sizeof(int));
  for (int i = 0; i < 9; ++i) {
    c->Favg[i] = c->host_red[i] / (double)c->g.N;
    c->Pavg[i] = c->host_red[9 + i] / (double)c->g.N;
  }
  c->state_valid = true;
  if (bad) {
    c->state_valid = false;
    fail(GHOM_EDOMAIN, "det F <= 0 at some voxel");
  }
}

// b = -G*(P - Pbar) in FP64; returns rms(b)
double residual(ghom_ctx* c, const double* Pbar) {
  const int grid = project64<double>(c, c->P, c->b, -1.0, Pbar, true, "res");
  timed(c, "reduce", [&] {
    hipLaunchKernelGGL(sum_columns_kernel, dim3(1), dim3(kRedThreads), 0, c->stream, c->partials, grid, 1, 0, c->red);
  });
  HIPCALL(hipMemcpyAsync(c->host_red, c->red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return std::sqrt(c->host_red[0] / (double)c->g.N);
}

__global__ void cg_setup_kernel(CGScalars* sc, double thresh, int max_it) {
  sc->thresh = thresh;
  sc->max_it = max_it;
  sc->it = 0;
  sc->done = 0;
  sc->status = 0;
}

struct CGResult {
  int iters;
  int status;
};

// conjugate gradients on A dF = b from dF = 0 (x holds the result); stop rule of Sec. 4
template <typename T>
CGResult cg_solve(ghom_ctx* c, double rms_b, double* t_ms) {
  const auto t0 = std::chrono::steady_clock::now();
  const double tol = std::max(c->cg_tol, c->cg_forcing * rms_b);
  const long long n9 = 9 * c->g.N;
  T* x = reinterpret_cast<T*>(c->x);
  T* r = reinterpret_cast<T*>(c->r);
  T* p = reinterpret_cast<T*>(c->p);
  hipLaunchKernelGGL(cg_setup_kernel, dim3(1), dim3(1), 0, c->stream, c->sc, tol * tol * (double)c->g.N, c->max_cg);
  HIPCALL(hipGetLastError());
  const int gi = vox_blocks(n9);
  timed(c, "cg_init", [&] {
    hipLaunchKernelGGL((cg_init_kernel<T>), dim3(gi), dim3(kVoxThreads), 0, c->stream, n9, c->b, x, r, p, c->partials);
  });
  timed(c, "cg_scalar", [&] {
    hipLaunchKernelGGL(cg_scalar_kernel, dim3(1), dim3(kRedThreads), 0, c->stream, c->sc, c->partials, gi, 0);
  });
  int enqueued = 0;
  int chunk = c->g.N >= (1LL << 21) ? 1 : (c->g.N >= (1LL << 18) ? 2 : 8);
  for (;;) {
    for (int i = 0; i < chunk; ++i, ++enqueued) {
      int gz = 0;
      operator_apply<T>(c, p, nullptr, true, enqueued > 0, c->sc, &gz);
      timed(c, "cg_scalar", [&] {
        hipLaunchKernelGGL(cg_scalar_kernel, dim3(1), dim3(kRedThreads), 0, c->stream, c->sc, c->partials, gz, 2);
      });
    }
    HIPCALL(hipMemcpyAsync(c->host_sc, c->sc, sizeof(CGScalars), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    if (c->host_sc->done) break;
    if (chunk < 8 && c->g.N < (1LL << 21)) chunk *= 2;
  }
  if (t_ms) *t_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return CGResult{c->host_sc->it, c->host_sc->status};
}

// F += dF (dF in FP64 or the CG type); returns crit = max |dF| / |<F>|
template <typename TD>
double newton_update(ghom_ctx* c, const TD* dF) {
  const int grid = vox_blocks(c->g.N);
  timed(c, "newton_update", [&] {
    hipLaunchKernelGGL((newton_update_kernel<TD>), dim3(grid), dim3(kVoxThreads), 0, c->stream, c->g, c->F, dF,
                       c->partials);
  });
  timed(c, "reduce", [&] {
    hipLaunchKernelGGL(sum_columns_kernel, dim3(1), dim3(kRedThreads), 0, c->stream, c->partials, grid, 10, 1, c->red);
  });
  HIPCALL(hipMemcpyAsync(c->host_red, c->red, 10 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  double nf = 0.0;
  for (int i = 0; i < 9; ++i) {
    const double m = c->host_red[1 + i] / (double)c->g.N;
    nf += m * m;
  }
  c->state_valid = false;
  return std::sqrt(c->host_red[0]) / std::sqrt(nf);
}

// One Newton solve (eq. 20) at the current increment with stress target Pbar.
int newton(ghom_ctx* c, const double* Pbar, ghom_step_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  ghom_step_info loc{};
  loc.crit = INFINITY;
  int rc = GHOM_ENOTCONVERGED;
  try {
    for (int it = 0; it < c->max_newton; ++it) {
      loc.newton_iters += 1;
      constitutive(c);
      const double rms_b = residual(c, Pbar);
      loc.res_rms = rms_b;
      if (!std::isfinite(rms_b)) fail(GHOM_EDOMAIN, "non-finite Newton residual");
      if (rms_b <= c->cg_tol) {
        rc = GHOM_OK;
        break;
      }
      CGResult cr = c->prec == GHOM_FP64 ? cg_solve<double>(c, rms_b, &loc.t_cg_ms)
                                         : cg_solve<float>(c, rms_b, &loc.t_cg_ms);
      loc.cg_iters_total += cr.iters;
      if (cr.status == 2) {
        if (cr.iters == 0) fail(GHOM_ESINGULAR, "CG breakdown (p.Ap <= 0) at its first iteration");
        loc.cg_breakdowns += 1;
      } else if (cr.status == 3) {
        fail(GHOM_ENOTCONVERGED, "CG reached max_cg");
      }
      double crit;
      if (c->prec == GHOM_FP64) {
        crit = newton_update<double>(c, reinterpret_cast<const double*>(c->x));
      } else {
        project64<float>(c, reinterpret_cast<const float*>(c->x), c->dF64, 1.0, nullptr, false, "reproj");
        crit = newton_update<double>(c, c->dF64);
      }
      loc.crit = crit;
      if (!std::isfinite(crit)) fail(GHOM_EDOMAIN, "non-finite Newton correction");
      if (crit < c->newton_tol) {
        rc = GHOM_OK;
        break;
      }
    }
    constitutive(c);  // P and the averages of the final F
  } catch (const ApiError& e) {
    loc.status = e.code;
    loc.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = loc;
    throw;
  }
  if (rc != GHOM_OK) c->err = "Newton reached max_newton";
  loc.status = rc;
  loc.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = loc;
  return rc;
}

void target_split(ghom_ctx* c, int k, double* Pbar) {
  for (int i = 0; i < 9; ++i) Pbar[i] = (k >= 1 && c->mask[i]) ? c->target[(size_t)(k - 1) * 9 + i] : 0.0;
}

void reset_state(ghom_ctx* c) {
  Shift9 id{};
  for (int i = 0; i < 9; ++i) id.d[i] = (i % 4 == 0) ? 1.0 : 0.0;
  hipLaunchKernelGGL(fill9_kernel, dim3(vox_blocks(c->g.N)), dim3(kVoxThreads), 0, c->stream, c->g.N, c->F, id);
  HIPCALL(hipGetLastError());
  c->k = 0;
  c->state_valid = false;
  for (int i = 0; i < 9; ++i) {
    c->Favg[i] = id.d[i];
    c->Pavg[i] = 0.0;
  }
}

template <typename T>
void dev_alloc(T** p, size_t count) {
  void* q = nullptr;
  HIPCALL(hipMalloc(&q, count * sizeof(T) > 0 ? count * sizeof(T) : 1));
  *p = reinterpret_cast<T*>(q);
}

void free_all(ghom_ctx* c) {
  void* ptrs[] = {c->F, c->P, c->b, c->dF64, c->x, c->r, c->p, c->state, c->H, c->phase, c->scale,
                  c->mat, c->mat32, c->partials, c->sc, c->flag, c->red, c->tw64[0], c->tw64[1], c->tw64[2],
                  c->tw32[0], c->tw32[1], c->tw32[2]};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (c->host_red) (void)hipHostFree(c->host_red);
  if (c->host_sc) (void)hipHostFree(c->host_sc);
  for (auto& kv : c->prof_recs)
    for (auto& pr : kv.second.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

void require_ready(ghom_ctx* c) {
  if (!c->kind) fail(GHOM_ESTATE, "no material set");
  if (!c->mask_set) fail(GHOM_ESTATE, "no control mask set");
}

}  // namespace

// =====================================================================================
// C ABI
// =====================================================================================
extern "C" {

int ghom_create(ghom_ctx** out, int nx, int ny, int nz, double Lx, double Ly, double Lz, int precision, int device,
                void* hip_stream) {
  if (!out) return GHOM_EINVAL;
  *out = nullptr;
  if (!supported_length(nx) || !supported_length(ny) || !supported_length(nz)) return GHOM_EINVAL;
  if (!(Lx > 0 && Ly > 0 && Lz > 0)) return GHOM_EINVAL;
  if (precision != GHOM_FP64 && precision != GHOM_FP32_SPLIT) return GHOM_EINVAL;
  ghom_ctx* c = new (std::nothrow) ghom_ctx();
  if (!c) return GHOM_ENOMEM;
  c->device = device;
  c->prec = precision;
  c->tsz = precision == GHOM_FP64 ? 8 : 4;
  c->g.nx = nx;
  c->g.ny = ny;
  c->g.nz = nz;
  c->g.nzh = (nz % 2 == 0) ? nz / 2 : (nz + 1) / 2;
  c->g.N = (long long)nx * ny * nz;
  c->g.Nh = (long long)nx * ny * c->g.nzh;
  c->g.invL[0] = 1.0 / Lx;
  c->g.invL[1] = 1.0 / Ly;
  c->g.invL[2] = 1.0 / Lz;
  const int rc = guard(c, [&]() -> int {
    if (hip_stream) {
      c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    } else {
      HIPCALL(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    const size_t n9 = 9 * (size_t)c->g.N;
    dev_alloc(&c->F, n9);
    dev_alloc(&c->P, n9);
    dev_alloc(&c->b, n9);
    if (precision == GHOM_FP32_SPLIT) dev_alloc(&c->dF64, n9);
    HIPCALL(hipMalloc(&c->x, n9 * c->tsz));
    HIPCALL(hipMalloc(&c->r, n9 * c->tsz));
    HIPCALL(hipMalloc(&c->p, n9 * c->tsz));
    HIPCALL(hipMalloc(&c->state, (size_t)kSVKState * c->g.N * c->tsz));
    HIPCALL(hipMalloc(&c->H, 9 * (size_t)c->g.Nh * sizeof(cx<double>)));
    dev_alloc(&c->phase, (size_t)c->g.N);
    // partials: the largest block count of any reducing launch
    size_t np = (size_t)kMaxVoxBlocks * 18;
    const long long nlines = (long long)nx * ny;
    np = std::max(np, (size_t)nlines + 64);
    c->npartials = np;
    dev_alloc(&c->partials, np);
    dev_alloc(&c->sc, 1);
    dev_alloc(&c->flag, 4);
    dev_alloc(&c->red, 32);
    HIPCALL(hipHostMalloc((void**)&c->host_red, 32 * sizeof(double), hipHostMallocDefault));
    HIPCALL(hipHostMalloc((void**)&c->host_sc, sizeof(CGScalars), hipHostMallocDefault));
    const int ns[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      std::vector<cx<double>> t64(ns[a]);
      std::vector<cx<float>> t32(ns[a]);
      for (int k = 0; k < ns[a]; ++k) {
        const CosSin cs = cossin_2pi(k, ns[a]);
        t64[k] = cx<double>{(double)cs.c, (double)-cs.s};
        t32[k] = cx<float>{(float)cs.c, (float)-cs.s};
      }
      dev_alloc(&c->tw64[a], ns[a]);
      dev_alloc(&c->tw32[a], ns[a]);
      HIPCALL(hipMemcpy(c->tw64[a], t64.data(), ns[a] * sizeof(cx<double>), hipMemcpyHostToDevice));
      HIPCALL(hipMemcpy(c->tw32[a], t32.data(), ns[a] * sizeof(cx<float>), hipMemcpyHostToDevice));
    }
    reset_state(c);
    // zero spectrum, then pick the x-pass variants by timing them on it
    hipLaunchKernelGGL(fill_zero_kernel, dim3(vox_blocks(18 * c->g.Nh)), dim3(kVoxThreads), 0, c->stream,
                       18 * c->g.Nh, reinterpret_cast<double*>(c->H));
    HIPCALL(hipGetLastError());
    tune_xproj<double>(c);
    if (precision == GHOM_FP32_SPLIT) tune_xproj<float>(c);
    sync(c);
    return GHOM_OK;
  });
  if (rc != GHOM_OK) {
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return GHOM_OK;
}

void ghom_destroy(ghom_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}

const char* ghom_last_error(const ghom_ctx* c) { return c ? c->err.c_str() : "null context"; }

int ghom_set_material_neohookean(ghom_ctx* c, const uint16_t* phase, int nphase, const double* mu,
                                 const double* lambda) {
  return guard(c, [&]() -> int {
    if (!phase || !mu || !lambda || nphase < 1 || nphase > 65536) fail(GHOM_EINVAL, "bad neo-Hookean arguments");
    for (long long v = 0; v < c->g.N; ++v)
      if (phase[v] >= nphase) fail(GHOM_EINVAL, "phase index out of range");
    std::vector<double> tab(2 * (size_t)nphase);
    for (int i = 0; i < nphase; ++i) {
      tab[2 * i] = mu[i];
      tab[2 * i + 1] = lambda[i];
    }
    if (c->mat) HIPCALL(hipFree(c->mat));
    c->mat = nullptr;
    dev_alloc(&c->mat, tab.size());
    HIPCALL(hipMemcpy(c->mat, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCALL(hipMemcpy(c->phase, phase, (size_t)c->g.N * sizeof(uint16_t), hipMemcpyHostToDevice));
    c->kind = MAT_NH;
    c->nphase = nphase;
    reset_state(c);
    sync(c);
    return GHOM_OK;
  });
}

int ghom_set_material_svk(ghom_ctx* c, const uint16_t* phase, int nphase, const double* C) {
  return guard(c, [&]() -> int {
    if (!phase || !C || nphase < 1 || nphase > 65536) fail(GHOM_EINVAL, "bad Saint Venant-Kirchhoff arguments");
    for (long long v = 0; v < c->g.N; ++v)
      if (phase[v] >= nphase) fail(GHOM_EINVAL, "phase index out of range");
    // Voigt order 11 22 33 23 13 12
    static const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
    std::vector<double> tab(36 * (size_t)nphase);
    for (int ph = 0; ph < nphase; ++ph) {
      const double* Cp = C + 81 * (size_t)ph;
      auto at = [&](int i, int j, int k, int l) { return Cp[((i * 3 + j) * 3 + k) * 3 + l]; };
      double scale = 0.0;
      for (int q = 0; q < 81; ++q) scale = std::max(scale, std::fabs(Cp[q]));
      const double tol = 1e-12 * (scale > 0 ? scale : 1.0);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
              const double v = at(i, j, k, l);
              if (std::fabs(v - at(j, i, k, l)) > tol || std::fabs(v - at(i, j, l, k)) > tol ||
                  std::fabs(v - at(k, l, i, j)) > tol)
                fail(GHOM_EINVAL, "stiffness lacks minor or major symmetry");
            }
      for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) tab[36 * (size_t)ph + 6 * I + J] = at(vi[I], vj[I], vi[J], vj[J]);
    }
    if (c->mat) HIPCALL(hipFree(c->mat));
    if (c->mat32) HIPCALL(hipFree(c->mat32));
    c->mat = nullptr;
    c->mat32 = nullptr;
    dev_alloc(&c->mat, tab.size());
    HIPCALL(hipMemcpy(c->mat, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    std::vector<float> tab32(tab.begin(), tab.end());
    dev_alloc(&c->mat32, tab32.size());
    HIPCALL(hipMemcpy(c->mat32, tab32.data(), tab32.size() * sizeof(float), hipMemcpyHostToDevice));
    HIPCALL(hipMemcpy(c->phase, phase, (size_t)c->g.N * sizeof(uint16_t), hipMemcpyHostToDevice));
    c->kind = MAT_SVK;
    c->nphase = nphase;
    reset_state(c);
    sync(c);
    return GHOM_OK;
  });
}

int ghom_set_stiffness_scale(ghom_ctx* c, const double* s) {
  return guard(c, [&]() -> int {
    if (!s) {
      if (c->scale) HIPCALL(hipFree(c->scale));
      c->scale = nullptr;
    } else {
      for (long long v = 0; v < c->g.N; ++v)
        if (!(s[v] > 0.0)) fail(GHOM_EINVAL, "stiffness scale must be > 0");
      if (!c->scale) dev_alloc(&c->scale, (size_t)c->g.N);
      HIPCALL(hipMemcpy(c->scale, s, (size_t)c->g.N * sizeof(double), hipMemcpyHostToDevice));
    }
    c->state_valid = false;
    return GHOM_OK;
  });
}

int ghom_set_control(ghom_ctx* c, const uint8_t mask[9]) {
  return guard(c, [&]() -> int {
    if (!mask) fail(GHOM_EINVAL, "null mask");
    for (int i = 0; i < 9; ++i) {
      if (mask[i] > 1) fail(GHOM_EINVAL, "mask entries must be 0 or 1");
      c->mask[i] = mask[i];
    }
    c->mask_set = true;
    return GHOM_OK;
  });
}

int ghom_set_history(ghom_ctx* c, int nsteps, const double* target) {
  return guard(c, [&]() -> int {
    if (nsteps < 1 || !target) fail(GHOM_EINVAL, "bad history");
    c->target.assign(target, target + 9 * (size_t)nsteps);
    c->nsteps = nsteps;
    return GHOM_OK;
  });
}

int ghom_set_tolerances(ghom_ctx* c, double newton_tol, double cg_tol, double cg_forcing, int max_newton,
                        int max_cg) {
  return guard(c, [&]() -> int {
    if (!(newton_tol > 0) || !(cg_tol > 0) || !(cg_forcing >= 0) || max_newton < 1 || max_cg < 1)
      fail(GHOM_EINVAL, "bad tolerances");
    c->newton_tol = newton_tol;
    c->cg_tol = cg_tol;
    c->cg_forcing = cg_forcing;
    c->max_newton = max_newton;
    c->max_cg = max_cg;
    return GHOM_OK;
  });
}

int ghom_step(ghom_ctx* c, ghom_step_info* info) {
  return guard(c, [&]() -> int {
    require_ready(c);
    if (c->nsteps == 0) fail(GHOM_ESTATE, "no history set");
    if (c->k >= c->nsteps) fail(GHOM_ESTATE, "history exhausted");
    const int k1 = c->k + 1;
    Shift9 sh{};
    bool any = false;
    for (int i = 0; i < 9; ++i) {
      if (c->mask[i]) continue;
      const double prev = (k1 == 1) ? ((i % 4 == 0) ? 1.0 : 0.0) : c->target[(size_t)(k1 - 2) * 9 + i];
      sh.d[i] = c->target[(size_t)(k1 - 1) * 9 + i] - prev;
      any = any || sh.d[i] != 0.0;
    }
    if (any) {
      timed(c, "shift", [&] {
        hipLaunchKernelGGL(shift_kernel, dim3(vox_blocks(c->g.N)), dim3(kVoxThreads), 0, c->stream, c->g.N, c->F, sh);
      });
      c->state_valid = false;
    }
    double Pbar[9];
    target_split(c, k1, Pbar);
    int rc;
    try {
      rc = newton(c, Pbar, info);
    } catch (const ApiError& e) {
      if (e.code == GHOM_ENOTCONVERGED) c->k = k1;
      throw;
    }
    c->k = k1;
    return rc;
  });
}

int ghom_resolve(ghom_ctx* c, ghom_step_info* info) {
  return guard(c, [&]() -> int {
    require_ready(c);
    double Pbar[9];
    target_split(c, c->k, Pbar);
    return newton(c, Pbar, info);
  });
}

int ghom_get_averages(ghom_ctx* c, double Fbar[9], double Pbar[9]) {
  return guard(c, [&]() -> int {
    if (!Fbar || !Pbar) fail(GHOM_EINVAL, "null output");
    if (!c->state_valid && c->kind) constitutive(c);
    for (int i = 0; i < 9; ++i) {
      Fbar[i] = c->Favg[i];
      Pbar[i] = c->Pavg[i];
    }
    return GHOM_OK;
  });
}

int ghom_get_field(ghom_ctx* c, int which, double* host_out) {
  return guard(c, [&]() -> int {
    if (!host_out || (which != GHOM_FIELD_F && which != GHOM_FIELD_P)) fail(GHOM_EINVAL, "bad field request");
    if (which == GHOM_FIELD_P) {
      require_ready(c);
      if (!c->state_valid) constitutive(c);
    }
    sync(c);
    HIPCALL(hipMemcpy(host_out, which == GHOM_FIELD_F ? c->F : c->P, 9 * (size_t)c->g.N * sizeof(double),
                      hipMemcpyDeviceToHost));
    return GHOM_OK;
  });
}

int ghom_get_field_device(ghom_ctx* c, int which, double* dev_out) {
  return guard(c, [&]() -> int {
    if (!dev_out || (which != GHOM_FIELD_F && which != GHOM_FIELD_P)) fail(GHOM_EINVAL, "bad field request");
    if (which == GHOM_FIELD_P) {
      require_ready(c);
      if (!c->state_valid) constitutive(c);
    }
    HIPCALL(hipMemcpyAsync(dev_out, which == GHOM_FIELD_F ? c->F : c->P, 9 * (size_t)c->g.N * sizeof(double),
                           hipMemcpyDeviceToDevice, c->stream));
    sync(c);
    return GHOM_OK;
  });
}

int ghom_save_state(ghom_ctx* c, double* F_out, int* step_out) {
  return guard(c, [&]() -> int {
    if (!F_out) fail(GHOM_EINVAL, "null output");
    sync(c);
    HIPCALL(hipMemcpy(F_out, c->F, 9 * (size_t)c->g.N * sizeof(double), hipMemcpyDeviceToHost));
    if (step_out) *step_out = c->k;
    return GHOM_OK;
  });
}

int ghom_load_state(ghom_ctx* c, const double* F_in, int step) {
  return guard(c, [&]() -> int {
    if (!F_in || step < 0 || (c->nsteps > 0 && step > c->nsteps) || (c->nsteps == 0 && step != 0))
      fail(GHOM_EINVAL, "bad state");
    sync(c);
    HIPCALL(hipMemcpy(c->F, F_in, 9 * (size_t)c->g.N * sizeof(double), hipMemcpyHostToDevice));
    c->k = step;
    c->state_valid = false;
    return GHOM_OK;
  });
}

int ghom_adjoint_grad_scale(ghom_ctx* c, const double a[9], double* grad_out) {
  return guard(c, [&]() -> int {
    require_ready(c);
    if (!a || !grad_out) fail(GHOM_EINVAL, "null argument");
    constitutive(c);
    // right-hand side G*(a) for a uniform a: only xi = 0 content, kept on stress-controlled
    // components (the 1/N of G*(a/N) is applied to the solution)
    Shift9 rhs{};
    double rr = 0.0;
    for (int i = 0; i < 9; ++i) {
      rhs.d[i] = c->mask[i] ? a[i] : 0.0;
      rr += rhs.d[i] * rhs.d[i];
    }
    if (rr == 0.0) {
      std::vector<double> zero((size_t)c->g.N, 0.0);
      std::memcpy(grad_out, zero.data(), zero.size() * sizeof(double));
      return GHOM_OK;
    }
    hipLaunchKernelGGL(fill9_kernel, dim3(vox_blocks(c->g.N)), dim3(kVoxThreads), 0, c->stream, c->g.N, c->b, rhs);
    HIPCALL(hipGetLastError());
    const double rms_b = std::sqrt(rr);
    double tcg = 0.0;
    CGResult cr = c->prec == GHOM_FP64 ? cg_solve<double>(c, rms_b, &tcg) : cg_solve<float>(c, rms_b, &tcg);
    if (cr.status == 2 && cr.iters == 0) fail(GHOM_ESINGULAR, "adjoint CG breakdown at its first iteration");
    if (cr.status == 3) fail(GHOM_ENOTCONVERGED, "adjoint CG reached max_cg");
    double* grad_dev = nullptr;
    dev_alloc(&grad_dev, (size_t)c->g.N);
    const int grid = vox_blocks(c->g.N);
    if (c->prec == GHOM_FP64) {
      hipLaunchKernelGGL((adjoint_grad_kernel<double>), dim3(grid), dim3(kVoxThreads), 0, c->stream, c->g.N,
                         (const double*)c->x, c->P, c->scale, 1.0 / (double)c->g.N, grad_dev);
    } else {
      project64<float>(c, reinterpret_cast<const float*>(c->x), c->dF64, 1.0, nullptr, false, "reproj");
      hipLaunchKernelGGL((adjoint_grad_kernel<double>), dim3(grid), dim3(kVoxThreads), 0, c->stream, c->g.N,
                         (const double*)c->dF64, c->P, c->scale, 1.0 / (double)c->g.N, grad_dev);
    }
    const hipError_t le = hipGetLastError();
    const hipError_t se = hipStreamSynchronize(c->stream);
    const hipError_t ce = hipMemcpy(grad_out, grad_dev, (size_t)c->g.N * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(grad_dev);
    HIPCALL(le);
    HIPCALL(se);
    HIPCALL(ce);
    return GHOM_OK;
  });
}

int ghom_apply_operator(ghom_ctx* c, const void* v_dev, void* Av_dev) {
  return guard(c, [&]() -> int {
    require_ready(c);
    if (!v_dev || !Av_dev || v_dev == Av_dev) fail(GHOM_EINVAL, "bad operator buffers");
    if (!c->state_valid) constitutive(c);
    if (c->prec == GHOM_FP64)
      operator_apply<double>(c, (double*)v_dev, (double*)Av_dev, false, false, nullptr, nullptr);
    else
      operator_apply<float>(c, (float*)v_dev, (float*)Av_dev, false, false, nullptr, nullptr);
    sync(c);
    return GHOM_OK;
  });
}

int ghom_apply_projection(ghom_ctx* c, const double* in_dev, double* out_dev) {
  return guard(c, [&]() -> int {
    if (!c->mask_set) fail(GHOM_ESTATE, "no control mask set");
    if (!in_dev || !out_dev) fail(GHOM_EINVAL, "null buffer");
    project64<double>(c, in_dev, out_dev, 1.0, nullptr, false, "proj");
    sync(c);
    return GHOM_OK;
  });
}

int ghom_residual(ghom_ctx* c, const double Pbar[9], double* out_dev) {
  return guard(c, [&]() -> int {
    require_ready(c);
    if (!Pbar || !out_dev) fail(GHOM_EINVAL, "null argument");
    double pb[9];
    for (int i = 0; i < 9; ++i) pb[i] = c->mask[i] ? Pbar[i] : 0.0;
    constitutive(c);
    project64<double>(c, c->P, out_dev, -1.0, pb, false, "res");
    sync(c);
    return GHOM_OK;
  });
}

int ghom_set_option(ghom_ctx* c, int key, int value) {
  return guard(c, [&]() -> int {
    if (key == GHOM_OPT_XPROJ_F64 || key == GHOM_OPT_XPROJ_F32) {
      if (value < XPROJ_TUNED || value > XPROJ_GROUPS) fail(GHOM_EINVAL, "x-pass variant must be 0, 1 or 2");
      int& slot = c->xproj_var[key == GHOM_OPT_XPROJ_F64 ? 0 : 1];
      if (value == XPROJ_TUNED) {
        slot = XPROJ_TUNED;
        sync(c);
        hipLaunchKernelGGL(fill_zero_kernel, dim3(vox_blocks(18 * c->g.Nh)), dim3(kVoxThreads), 0, c->stream,
                           18 * c->g.Nh, reinterpret_cast<double*>(c->H));
        HIPCALL(hipGetLastError());
        if (key == GHOM_OPT_XPROJ_F64) tune_xproj<double>(c);
        else tune_xproj<float>(c);
        sync(c);
      } else {
        slot = value;
      }
      return GHOM_OK;
    }
    if (key == GHOM_OPT_ZSLABS) {
      if (value < 1 || value > 4096) fail(GHOM_EINVAL, "slab count must be in [1, 4096]");
      c->zslabs = value;
      return GHOM_OK;
    }
    fail(GHOM_EINVAL, "unknown option");
  });
}

int ghom_get_option(ghom_ctx* c, int key, int* value) {
  return guard(c, [&]() -> int {
    if (!value) fail(GHOM_EINVAL, "null output");
    if (key == GHOM_OPT_XPROJ_F64) *value = c->xproj_var[0];
    else if (key == GHOM_OPT_XPROJ_F32) *value = c->xproj_var[1];
    else if (key == GHOM_OPT_ZSLABS) *value = c->zslabs;
    else fail(GHOM_EINVAL, "unknown option");
    return GHOM_OK;
  });
}

int ghom_set_profiling(ghom_ctx* c, int on) {
  return guard(c, [&]() -> int {
    c->prof = on != 0;
    return GHOM_OK;
  });
}

int ghom_profile_count(ghom_ctx* c) {
  if (!c) return GHOM_EINVAL;
  return (int)c->prof_recs.size();
}

int ghom_profile_get(ghom_ctx* c, int i, char* name_out, int name_cap, int* launches, double* total_ms) {
  return guard(c, [&]() -> int {
    if (i < 0 || i >= (int)c->prof_recs.size()) fail(GHOM_EINVAL, "record index out of range");
    prof_collect(c);
    auto it = c->prof_recs.begin();
    std::advance(it, i);
    if (name_out && name_cap > 0) {
      std::strncpy(name_out, it->first.c_str(), (size_t)name_cap - 1);
      name_out[name_cap - 1] = 0;
    }
    if (launches) *launches = it->second.launches;
    if (total_ms) *total_ms = it->second.ms;
    return GHOM_OK;
  });
}

int ghom_profile_reset(ghom_ctx* c) {
  return guard(c, [&]() -> int {
    prof_collect(c);
    c->prof_recs.clear();
    return GHOM_OK;
  });
}

}  // extern "C"
