// libghom.so: host runtime and C ABI (include/ghom.h) of the Galerkin-FFT solver with
// stress / mixed control.  Every step of the method runs in the kernels of kernels.hpp on
// the stream of the engine; the host only sequences launches, moves a few scalars and
// applies the stopping rules.
//
// An engine holds any number of independent problems.  Problems with the same grid and
// material law form a shape class; every pass is one launch per class covering all of its
// problems (blockIdx.z = problem), so a batch of hundreds of cells costs a handful of
// launches per pass.  A ghom_ctx is an engine with one problem.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ghom.h"
#include "kernels.hpp"
#include "control.hpp"
#include "substep.hpp"

using namespace ghom;

namespace {

constexpr int kMaxVoxBlocks = 8192;

struct HipFail {
  hipError_t e;
  const char* what;
};

#define HIPCALL(expr)                                 \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) throw HipFail{_e, #expr};   \
  } while (0)

struct ApiError {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg) { throw ApiError{code, msg}; }

struct ProfRec {
  int launches = 0;
  double ms = 0.0;
  std::vector<float> samples;  // each launch's time, in launch order
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

enum { XPROJ_TUNED = 0, XPROJ_ROWS = 1, XPROJ_GROUPS = 2, XPROJ_ROWS_CAPPED = 3, XPROJ_ROWS3 = 4 };
enum { YPASS_TUNED = 0, YPASS_WIDE = 1, YPASS_NARROW = 2, YPASS_THREE = 3 };

struct ShapeClass {
  int nx = 0, ny = 0, nz = 0, kind = 0;
  Geo g{};
  std::vector<int> probs;  // problem indices
  int* ids = nullptr;      // device copy of probs
  cx<double>* tw64[3] = {nullptr, nullptr, nullptr};
  cx<float>* tw32[3] = {nullptr, nullptr, nullptr};
  int xproj_var[2] = {XPROJ_TUNED, XPROJ_TUNED};  // [0] float64, [1] float32
  int ypass_var[2] = {YPASS_TUNED, YPASS_TUNED};  // [0] float64, [1] float32
  bool tuned_x[2] = {false, false}, tuned_y[2] = {false, false};  // picked by timing (or the tuning cache)
  int vb = 1;                                     // voxel-kernel blocks per problem
};

struct Prob {
  int cls = -1;
  int kind = 0;
  int nphase = 0;
  uint8_t mask[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};       // the mask the solver uses
  uint8_t user_mask[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // the mask as set
  bool mask_set = false;
  int gauge_axis = -1;  // axis of the rotation gauge of full stress control, or -1
  std::vector<double> target;
  int nsteps = 0;
  int k = 0;
  double Favg[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double Pavg[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  bool state_valid = false;
  // the P field matches F (the residual pass of the elastic laws does not store it)
  bool p_field_valid = false;
  double adapt_fraction = 1.0;  // adaptive stepping: fraction the next increment starts with
  // solve bookkeeping
  bool running = false;
  int status = GHOM_OK;
  std::string msg;
  double rms_b = 0.0;
  ghom_step_info info{};
  // viscoelastic law: Voigt tables of Cinf and C1 and tau per phase, increment length
  std::vector<double> vinf, v1, vtau;
  double dt = 1.0;
  // device buffers owned outside the arena
  double* scale = nullptr;
  double* mat = nullptr;
  float* mat32 = nullptr;
  double* visc = nullptr;  // viscoelastic law: Cinf, C1, a, b per phase
  double* iv = nullptr;    // viscoelastic law: internal variables (kViscoIV x N)
  // viscoelastic law with checkpoints on: per accepted increment, F at convergence and the
  // internal variables it started from ((9 + kViscoIV) x N float64 each), and its length
  std::vector<double*> ckpt;
  std::vector<double> ckpt_dt;
  int ckpt_k0 = -1;  // increment index of the first checkpoint (0: the history is complete)
};

struct Engine {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int prec = GHOM_FP64;
  size_t tsz = 8;
  std::vector<Prob> P;
  std::vector<ShapeClass> C;
  ProbDesc* hdesc = nullptr;  // pinned host mirror
  ProbDesc* ddesc = nullptr;
  // descriptor uploads without a stream synchronisation: the mirror is staged in a ring of
  // pinned slots, each reused after its copy has completed; an unchanged mirror is not sent
  static constexpr int kDescSlots = 4;
  ProbDesc* desc_stage[kDescSlots] = {};
  hipEvent_t desc_ev[kDescSlots] = {};
  bool desc_pending[kDescSlots] = {};
  int desc_next = 0;
  std::vector<ProbDesc> desc_sent;  // what the device holds (empty: not known)
  char* arena = nullptr;
  size_t np = 0;              // partials per problem
  CGScalars* sc = nullptr;    // device, one per problem
  double* red = nullptr;      // device address of host_red (mapped), 32 per problem
  int* flags = nullptr;       // device, one per problem
  double* ckpt = nullptr;        // adaptive stepping: F at the start of the sub-increment and of the increment
  CGScalars* host_sc = nullptr;  // one entry per problem, mapped: written by the CG kernels
  CGScalars* host_sc_dev = nullptr;  // its device address
  hipEvent_t sc_ev[2] = {nullptr, nullptr};
  double* host_red = nullptr;
  double newton_tol = 1e-6, cg_tol = 1e-8, cg_forcing = 0.0;
  int max_newton = 50, max_cg = 5000;
  int zslabs = 1;
  bool stream_nt = false;  // nontemporal builds of the short-line pass kernels (set at creation)
  bool graphs = false;  // replay captured HIP graphs of CG iterations (not while profiling)
  bool checkpoints = false;  // keep per-increment states of path-dependent laws (adjoint)
  bool rot_gauge = true;     // rotation gauge of full stress control (control.hpp)
  std::map<long long, hipGraphExec_t> graph_cache;  // key: CG type size, start mode, first-iteration flag, iterations
  bool prof = false;
  std::string prof_only;  // time only launches of this name (empty: all)
  int prof_every = 1;     // time every prof_every-th launch of each timed name
  std::map<std::string, long long> prof_seen;  // launches of each timed name so far
  std::map<std::string, ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_pool;
  std::string err;
};

// ------------------------------------------------------------------ plumbing ----------
template <typename F>
int guarded(Engine* e, F&& f) {
  if (!e) return GHOM_EINVAL;
  try {
    e->err.clear();
    HIPCALL(hipSetDevice(e->device));
    return f();
  } catch (const ApiError& x) {
    e->err = x.msg;
    return x.code;
  } catch (const HipFail& x) {
    e->err = std::string("HIP error '") + hipGetErrorString(x.e) + "' in " + x.what;
    return x.e == hipErrorOutOfMemory ? GHOM_ENOMEM : GHOM_EHIP;
  } catch (const std::bad_alloc&) {
    e->err = "host allocation failed";
    return GHOM_ENOMEM;
  }
}

void sync(Engine& e) { HIPCALL(hipStreamSynchronize(e.stream)); }

hipEvent_t get_event(Engine& e) {
  if (!e.ev_pool.empty()) {
    hipEvent_t ev = e.ev_pool.back();
    e.ev_pool.pop_back();
    return ev;
  }
  hipEvent_t ev;
  HIPCALL(hipEventCreate(&ev));
  return ev;
}

// Runs `launch` on the engine stream, bracketed by events when profiling.
template <typename L>
void timed(Engine& e, const std::string& name, L&& launch) {
  if (!e.prof || (!e.prof_only.empty() && name != e.prof_only)) {
    launch();
    HIPCALL(hipGetLastError());
    return;
  }
  if (e.prof_every > 1 && e.prof_seen[name]++ % e.prof_every != 0) {
    launch();
    HIPCALL(hipGetLastError());
    return;
  }
  hipEvent_t a = get_event(e), b = get_event(e);
  HIPCALL(hipEventRecord(a, e.stream));
  launch();
  HIPCALL(hipGetLastError());
  HIPCALL(hipEventRecord(b, e.stream));
  e.prof_recs[name].pending.emplace_back(a, b);
}

void prof_collect(Engine& e) {
  sync(e);
  for (auto& kv : e.prof_recs) {
    for (auto& pr : kv.second.pending) {
      float ms = 0.f;
      HIPCALL(hipEventElapsedTime(&ms, pr.first, pr.second));
      kv.second.ms += ms;
      kv.second.launches += 1;
      kv.second.samples.push_back(ms);
      e.ev_pool.push_back(pr.first);
      e.ev_pool.push_back(pr.second);
    }
    kv.second.pending.clear();
  }
}

template <typename T> const char* tname();
template <> const char* tname<double>() { return "f64"; }
template <> const char* tname<float>() { return "f32"; }

int vox_blocks(long long n) {
  const long long b = (n + kVoxThreads - 1) / kVoxThreads;
  return (int)std::max(1LL, std::min<long long>(b, kMaxVoxBlocks));
}

// The device descriptors take the host mirror's values for every kernel enqueued after this
// call; the host may change the mirror again at once.
void upload_descs(Engine& e) {
  const size_t n = e.P.size();
  const size_t bytes = n * sizeof(ProbDesc);
  if (!e.desc_stage[0]) {  // no staging slots (a one-call engine): copy, then wait
    HIPCALL(hipMemcpyAsync(e.ddesc, e.hdesc, bytes, hipMemcpyHostToDevice, e.stream));
    sync(e);
    return;
  }
  if (e.desc_sent.size() == n && std::memcmp(e.desc_sent.data(), e.hdesc, bytes) == 0) return;
  const int k = e.desc_next;
  e.desc_next = (k + 1) % Engine::kDescSlots;
  if (e.desc_pending[k]) HIPCALL(hipEventSynchronize(e.desc_ev[k]));
  std::memcpy(e.desc_stage[k], e.hdesc, bytes);
  HIPCALL(hipMemcpyAsync(e.ddesc, e.desc_stage[k], bytes, hipMemcpyHostToDevice, e.stream));
  HIPCALL(hipEventRecord(e.desc_ev[k], e.stream));
  e.desc_pending[k] = true;
  e.desc_sent.assign(e.hdesc, e.hdesc + n);
}

bool class_active(Engine& e, const ShapeClass& c) {
  for (int p : c.probs)
    if (e.hdesc[p].active) return true;
  return false;
}

// ------------------------------------------------------------------ pass launchers ----
// Calls f with std::true_type when the pass kernels of transform length N are to use their
// nontemporal build: always for long lines, else as chosen for the context.
template <int N, typename F> void with_nt(const Engine& e, F&& f) {
  if constexpr (stream_nt_always(N)) f(std::true_type{});
  else if (e.stream_nt) f(std::true_type{});
  else f(std::false_type{});
}

// the forward z pass's grid (its block count: the partials of its reductions)
template <typename T, int MODE>
int zfwd_grid(const ShapeClass& c) {
  int grid = 0;
  with_split(c.nz, [&](auto s) {
    using S = decltype(s);
    using Cfg = ZCfg<T, S::A, S::B, zfwd_ntmin<MODE>()>;
    grid = (int)(((long long)c.nx * c.ny + 2 * Cfg::LP - 1) / (2 * Cfg::LP));
  });
  return grid;
}

template <typename T, int MODE, typename TIN>
int launch_zfwd(Engine& e, ShapeClass& c, int role, int update_p, const std::string& name) {
  const int grid = zfwd_grid<T, MODE>(c);
  with_split(c.nz, [&](auto s) {
    using S = decltype(s);
    using Cfg = ZCfg<T, S::A, S::B, zfwd_ntmin<MODE>()>;
    with_nt<S::A * S::B>(e, [&](auto nt) {
      timed(e, name, [&] {
        hipLaunchKernelGGL((zfwd_batch<T, S::A, S::B, MODE, TIN, decltype(nt)::value>),
                           dim3(grid, 1, (unsigned)c.probs.size()), dim3(Cfg::NT), 0, e.stream, e.ddesc, c.ids, role,
                           update_p);
      });
    });
  });
  return grid;
}

template <typename T, typename TOUT, int ZM>
int launch_zinv(Engine& e, ShapeClass& c, int role, const std::string& name, int first = 0) {
  int grid = 0;
  with_split(c.nz, [&](auto s) {
    using S = decltype(s);
    using Cfg = ZCfg<T, S::A, S::B, zinv_ntmin<ZM>()>;
    const long long nlines = (long long)c.nx * c.ny;
    grid = (int)((nlines + 2 * Cfg::LP - 1) / (2 * Cfg::LP));
    with_nt<S::A * S::B>(e, [&](auto nt) {
      timed(e, name, [&] {
        hipLaunchKernelGGL((zinv_batch<T, S::A, S::B, TOUT, ZM, decltype(nt)::value>),
                           dim3(grid, 1, (unsigned)c.probs.size()), dim3(Cfg::NT), 0, e.stream, e.ddesc, c.ids, role,
                           first);
      });
    });
  });
  return grid;
}

template <typename T> int& ypass_choice(ShapeClass& c) { return c.ypass_var[sizeof(T) == 8 ? 0 : 1]; }

// whether y-pass variant v exists for line length n (the narrow one only where it differs from
// the wide one, the three-stage one for lengths with a three-stage schedule)
template <typename T> bool ypass_has(int v, int n) {
  if (v == YPASS_WIDE) return true;
  if (v == YPASS_THREE) return has_split3(n);
  bool differs = false;
  with_split(n, [&](auto s) {
    using S = decltype(s);
    differs = YCfg<T, S::A, S::B>::TC != YNarrowCfg<T, S::A, S::B>::TC;
  });
  return v == YPASS_NARROW && differs;
}

template <typename T, int DIR>
void launch_ypass_variant(Engine& e, ShapeClass& c, int v, int role, Slab sl, const std::string& name,
                          int alpha_nparts) {
  const long long ncols = 9LL * c.nx * sl.nkz;
  if (v == YPASS_THREE && with_split3(c.ny, [&](auto s3) {
        using S3 = decltype(s3);
        using Cfg = Y3Cfg<T, S3>;
        const int grid = (int)((ncols + Cfg::TC - 1) / Cfg::TC);
        with_nt<S3::N>(e, [&](auto nt) {
          timed(e, name, [&] {
            hipLaunchKernelGGL((ypass3_batch<T, S3, DIR, decltype(nt)::value>), dim3(grid, 1, (unsigned)c.probs.size()),
                               dim3(Cfg::NT), 0, e.stream, e.ddesc, c.ids, role, sl, alpha_nparts);
          });
        });
      }))
    return;
  with_split(c.ny, [&](auto s) {
    using S = decltype(s);
    auto go = [&](auto wide) {
      constexpr bool W = decltype(wide)::value;
      using Cfg = YPassCfg<T, S::A, S::B, W>;
      const int grid = (int)((ncols + Cfg::TC - 1) / Cfg::TC);
      with_nt<S::A * S::B>(e, [&](auto nt) {
        timed(e, name, [&] {
          hipLaunchKernelGGL((ypass_batch<T, S::A, S::B, DIR, decltype(nt)::value, W>),
                             dim3(grid, 1, (unsigned)c.probs.size()), dim3(Cfg::NT), 0, e.stream, e.ddesc, c.ids, role,
                             sl, alpha_nparts);
        });
      });
    };
    if constexpr (YCfg<T, S::A, S::B>::TC != YNarrowCfg<T, S::A, S::B>::TC) {
      if (v == YPASS_NARROW) {
        go(std::false_type{});
        return;
      }
    }
    go(std::true_type{});
  });
}

template <typename T, int DIR>
void launch_ypass(Engine& e, ShapeClass& c, int role, Slab sl, const std::string& name, int alpha_nparts = 0) {
  const int v = ypass_choice<T>(c) == YPASS_TUNED ? YPASS_WIDE : ypass_choice<T>(c);
  launch_ypass_variant<T, DIR>(e, c, v, role, sl, name, alpha_nparts);
}

template <typename T>
void launch_xproj_variant(Engine& e, ShapeClass& c, int variant, int role, Slab sl) {
  if (variant == XPROJ_ROWS3 && with_split3(c.nx, [&](auto s3) {
        using S3 = decltype(s3);
        using Cfg = XRows3Cfg<T, S3>;
        const long long ncols = (long long)c.ny * sl.nkz;
        const int grid = (int)((ncols + Cfg::TC - 1) / Cfg::TC);
        with_nt<S3::N>(e, [&](auto nt) {
          hipLaunchKernelGGL((xproj_rows3_batch<T, S3, decltype(nt)::value>), dim3(grid, 3, (unsigned)c.probs.size()),
                             dim3(Cfg::NT), 0, e.stream, e.ddesc, c.ids, role, sl);
        });
      }))
    return;
  with_split(c.nx, [&](auto s) {
    using S = decltype(s);
    const long long ncols = (long long)c.ny * sl.nkz;
    with_nt<S::A * S::B>(e, [&](auto nt) {
      constexpr bool NTS = decltype(nt)::value;
      if (variant == XPROJ_ROWS || variant == XPROJ_ROWS_CAPPED) {
        using Cfg = XRowsCfg<T, S::A, S::B>;
        const int grid = (int)((ncols + Cfg::TC - 1) / Cfg::TC);
        const dim3 gd(grid, 3, (unsigned)c.probs.size());
        if (variant == XPROJ_ROWS)
          hipLaunchKernelGGL((xproj_rows_batch<T, S::A, S::B, 1, NTS>), gd, dim3(Cfg::NT), 0, e.stream, e.ddesc, c.ids,
                             role, sl);
        else
          hipLaunchKernelGGL((xproj_rows_batch<T, S::A, S::B, 2, NTS>), gd, dim3(Cfg::NT), 0, e.stream, e.ddesc, c.ids,
                             role, sl);
      } else {
        using Cfg = XCfg<T, S::A, S::B>;
        const int grid = (int)((ncols + Cfg::TC - 1) / Cfg::TC);
        hipLaunchKernelGGL((xproj_groups_batch<T, S::A, S::B, NTS>), dim3(grid, 3, (unsigned)c.probs.size()),
                           dim3(Cfg::NT), 0, e.stream, e.ddesc, c.ids, role, sl);
      }
    });
  });
}

template <typename T> int& xproj_choice(ShapeClass& c) { return c.xproj_var[sizeof(T) == 8 ? 0 : 1]; }

// y forward, x with the projection, y inverse; kz-slab by slab.  alpha_nparts > 0 (a CG
// step): the first y pass also sets alpha from the forward pass's partials.
template <typename T>
void middle_passes(Engine& e, ShapeClass& c, int role, const std::string& pre, int alpha_nparts = 0) {
  const std::string t = tname<T>();
  const std::string n2 = pre + "yfwd_" + t, n3 = pre + "xproj_" + t, n4 = pre + "yinv_" + t;
  const int nzh = c.g.nzh;
  const int ns = std::max(1, std::min(e.zslabs, nzh));
  const int per = (nzh + ns - 1) / ns;
  const int v = xproj_choice<T>(c) == XPROJ_TUNED ? XPROJ_ROWS : xproj_choice<T>(c);
  for (int kz0 = 0; kz0 < nzh; kz0 += per) {
    const Slab sl{kz0, std::min(per, nzh - kz0)};
    launch_ypass<T, -1>(e, c, role, sl, n2, kz0 == 0 ? alpha_nparts : 0);
    timed(e, n3, [&] { launch_xproj_variant<T>(e, c, v, role, sl); });
    launch_ypass<T, +1>(e, c, role, sl, n4);
  }
}

// ---- autotuner --------------------------------------------------------------------------
// The x pass (transform along x with the projection) and the y passes have several
// schedules: radix splits (two-stage n = A x B with B values per thread, or three-stage
// n = B x A1 x A2 with 8 values per thread), register budgets and column counts per
// workgroup.  At context creation each shape class times the candidates of each pass and
// precision on its own (zeroed) spectra with HIP events (best of three after a warm-up) and
// keeps the fastest, timing each candidate inside the y-forward, x, y-inverse sequence the
// pipeline runs.  Choices are cached for the process, keyed by GPU architecture, pass,
// precision, grid, problem count and streaming build; with the environment variable
// GHOM_TUNE_CACHE naming a file, the cache is read from it at the first tuning and every new
// choice is appended to it.
constexpr float kTuneMargin = 0.98f;  // a variant replaces the one kept so far only if 2% faster
std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;
bool g_tune_loaded = false;

std::string tune_key(const Engine& e, const ShapeClass& c, const char* pass, int prec64) {
  hipDeviceProp_t prop{};
  std::string arch = hipGetDeviceProperties(&prop, e.device) == hipSuccess ? std::string(prop.gcnArchName) : "?";
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s:%s:%s:%dx%dx%d:p%zu:nt%d", arch.c_str(), pass, prec64 ? "f64" : "f32", c.nx, c.ny,
                c.nz, c.probs.size(), e.stream_nt ? 1 : 0);
  return buf;
}

bool tune_lookup(const std::string& key, int* v) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (!g_tune_loaded) {
    g_tune_loaded = true;
    if (const char* f = std::getenv("GHOM_TUNE_CACHE"))
      if (FILE* fp = std::fopen(f, "r")) {
        char k[200];
        int val = 0;
        while (std::fscanf(fp, "%199s %d", k, &val) == 2) g_tune_cache[k] = val;
        std::fclose(fp);
      }
  }
  auto it = g_tune_cache.find(key);
  if (it == g_tune_cache.end()) return false;
  *v = it->second;
  return true;
}

void tune_store(const std::string& key, int v) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache[key] = v;
  if (const char* f = std::getenv("GHOM_TUNE_CACHE"))
    if (FILE* fp = std::fopen(f, "a")) {
      std::fprintf(fp, "%s %d\n", key.c_str(), v);
      std::fclose(fp);
    }
}

// best of five timed launches of `launch` after a warm-up (ms)
template <typename L> float time_best(Engine& e, L&& launch) {
  hipEvent_t e0 = get_event(e), e1 = get_event(e);
  launch();
  HIPCALL(hipGetLastError());
  float tmin = 0.f;
  for (int rep = 0; rep < 5; ++rep) {
    HIPCALL(hipEventRecord(e0, e.stream));
    launch();
    HIPCALL(hipGetLastError());
    HIPCALL(hipEventRecord(e1, e.stream));
    HIPCALL(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCALL(hipEventElapsedTime(&ms, e0, e1));
    if (rep == 0 || ms < tmin) tmin = ms;
  }
  e.ev_pool.push_back(e0);
  e.ev_pool.push_back(e1);
  return tmin;
}

template <typename T>
void tune_xproj(Engine& e, ShapeClass& c, bool use_cache) {
  const std::string key = tune_key(e, c, "x", sizeof(T) == 8);
  int v_cached = 0;
  if (use_cache && tune_lookup(key, &v_cached) && v_cached >= XPROJ_ROWS && v_cached <= XPROJ_ROWS3 &&
      (v_cached != XPROJ_ROWS3 || has_split3(c.nx))) {
    xproj_choice<T>(c) = v_cached;
    c.tuned_x[sizeof(T) == 8 ? 0 : 1] = true;
    return;
  }
  float best = 0.f;
  int best_v = XPROJ_ROWS;
  const Slab full{0, c.g.nzh};
  // timed in context: the y passes around it as the pipeline runs them
  const int yv = ypass_choice<T>(c) == YPASS_TUNED ? YPASS_WIDE : ypass_choice<T>(c);
  for (int v : {XPROJ_ROWS, XPROJ_GROUPS, XPROJ_ROWS_CAPPED, XPROJ_ROWS3}) {
    if (v == XPROJ_ROWS3 && !has_split3(c.nx)) continue;
    const float t = time_best(e, [&] {
      launch_ypass_variant<T, -1>(e, c, yv, ROLE_PROJ, full, "tune", 0);
      launch_xproj_variant<T>(e, c, v, ROLE_PROJ, full);
      launch_ypass_variant<T, +1>(e, c, yv, ROLE_PROJ, full, "tune", 0);
    });
    if (v == XPROJ_ROWS || t < kTuneMargin * best) {  // a challenger must win by the margin
      best = t;
      best_v = v;
    }
  }
  xproj_choice<T>(c) = best_v;
  c.tuned_x[sizeof(T) == 8 ? 0 : 1] = true;
  tune_store(key, best_v);
}

template <typename T>
void tune_ypass(Engine& e, ShapeClass& c, bool use_cache) {
  const std::string key = tune_key(e, c, "y", sizeof(T) == 8);
  int v_cached = 0;
  if (use_cache && tune_lookup(key, &v_cached) && v_cached >= YPASS_WIDE && v_cached <= YPASS_THREE &&
      ypass_has<T>(v_cached, c.ny)) {
    ypass_choice<T>(c) = v_cached;
    c.tuned_y[sizeof(T) == 8 ? 0 : 1] = true;
    return;
  }
  float best = 0.f;
  int best_v = YPASS_WIDE;
  const Slab full{0, c.g.nzh};
  const int xv = xproj_choice<T>(c) == XPROJ_TUNED ? XPROJ_ROWS : xproj_choice<T>(c);
  for (int v : {YPASS_WIDE, YPASS_NARROW, YPASS_THREE}) {
    if (!ypass_has<T>(v, c.ny)) continue;
    const float t = time_best(e, [&] {
      launch_ypass_variant<T, -1>(e, c, v, ROLE_PROJ, full, "tune", 0);
      launch_xproj_variant<T>(e, c, xv, ROLE_PROJ, full);
      launch_ypass_variant<T, +1>(e, c, v, ROLE_PROJ, full, "tune", 0);
    });
    if (v == YPASS_WIDE || t < kTuneMargin * best) {
      best = t;
      best_v = v;
    }
  }
  ypass_choice<T>(c) = best_v;
  c.tuned_y[sizeof(T) == 8 ? 0 : 1] = true;
  tune_store(key, best_v);
}

__global__ void fill_zero_kernel(long long n, double* p) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// which: -1 both precisions, 0 float64 only, 1 float32 only; passes whose choice is
// XPROJ_TUNED / YPASS_TUNED are timed (or taken from the tuning cache when use_cache)
void tune_class(Engine& e, ShapeClass& c, int which, bool use_cache = true) {
  for (size_t p = 0; p < e.P.size(); ++p) e.hdesc[p].active = 0;
  for (int p : c.probs) {
    e.hdesc[p].active = 1;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, e.stream, 18 * c.g.Nh,
                       reinterpret_cast<double*>(e.hdesc[p].H));
    HIPCALL(hipGetLastError());
  }
  upload_descs(e);
  if (which != 1) {
    if (xproj_choice<double>(c) == XPROJ_TUNED) tune_xproj<double>(e, c, use_cache);
    if (ypass_choice<double>(c) == YPASS_TUNED) tune_ypass<double>(e, c, use_cache);
  }
  if (e.prec == GHOM_FP32_SPLIT && which != 0) {
    if (xproj_choice<float>(c) == XPROJ_TUNED) tune_xproj<float>(e, c, use_cache);
    if (ypass_choice<float>(c) == YPASS_TUNED) tune_ypass<float>(e, c, use_cache);
  }
  sync(e);
}

// Column sums (first nmax columns: maxima) of every problem's partials table into red[off ..
// off + K): one block per problem and column.
void launch_sum_columns(Engine& e, const int* ids, int np, int nparts, int K, int nmax, int layout, int off,
                        int with_flag) {
  hipLaunchKernelGGL(sum_columns_batch, dim3(np, K), dim3(kRedThreads), 0, e.stream, e.ddesc, ids, nparts, K, nmax,
                     layout, off, with_flag);
  HIPCALL(hipGetLastError());
}

// out = scale * G*(in - Pbar) in float64 for every active problem of a class
// role: ROLE_RESID (P -> b, with b.b partials), ROLE_RESID_R (the same into r in the CG type),
// ROLE_REPROJ (x -> dF64), ROLE_PROJ (in -> out),
// ROLE_NEWTON (F += G*(x), Newton-update partials)
int project64(Engine& e, ShapeClass& c, int role, const std::string& tag) {
  const std::string pre = tag + "_";
  const bool from_x = role == ROLE_REPROJ || role == ROLE_NEWTON;
  if (from_x && e.prec == GHOM_FP32_SPLIT) launch_zfwd<double, Z_PLAIN, float>(e, c, role, 0, pre + "zfwd_f64");
  else launch_zfwd<double, Z_PLAIN, double>(e, c, role, 0, pre + "zfwd_f64");
  middle_passes<double>(e, c, role, pre);
  if (role == ROLE_NEWTON) return launch_zinv<double, double, ZI_NEWTON>(e, c, role, pre + "zinv_f64");
  return launch_zinv<double, double, ZI_PLAIN>(e, c, role, pre + "zinv_f64");
}

// A(v) = G*(K : v) in the CG type.  ROLE_OP_CG: one CG step (see the kernels); returns the
// z-pass grid (the partial count of its reductions).  ROLE_OP_PLAIN: in -> out.
// update_p: 0 p as is, 1 p <- r + beta p, 2 CG start (r = p = b, x not read), 3 CG start
// from r (p = r: the Newton residual was written into r)
// part: 0 the whole operator, 1 its forward z pass only, 2 the passes after it (a CG step
// queued in two parts, see cg_solve)
template <typename T>
int operator_apply(Engine& e, ShapeClass& c, int role, int update_p, int part = 0) {
  const std::string t = tname<T>();
  int gz;
  if (part == 2) {
    gz = c.kind == MAT_NH ? zfwd_grid<T, Z_NH>(c) : (c.kind == MAT_SVK ? zfwd_grid<T, Z_SVK>(c) : zfwd_grid<T, Z_VISCO>(c));
  } else if (c.kind == MAT_NH) {
    gz = launch_zfwd<T, Z_NH, T>(e, c, role, update_p, "op_zfwd_" + t);
  } else if (c.kind == MAT_SVK) {
    gz = launch_zfwd<T, Z_SVK, T>(e, c, role, update_p, "op_zfwd_" + t);
  } else {
    gz = launch_zfwd<T, Z_VISCO, T>(e, c, role, update_p, "op_zfwd_" + t);
  }
  if (part == 1) return gz;
  middle_passes<T>(e, c, role, "op_", role == ROLE_OP_CG ? gz : 0);
  if (role == ROLE_OP_CG) launch_zinv<T, T, ZI_CG>(e, c, role, "op_zinv_" + t, update_p >= 2 ? 1 : 0);
  else launch_zinv<T, T, ZI_PLAIN>(e, c, role, "op_zinv_" + t);
  return gz;
}

// ------------------------------------------------------------------ method steps -------
// Constitutive update of every active problem: P, tangent state, <F>, <P> (the averages are
// left as they are if !averages).  Problems with det F <= 0 get EDOMAIN and stop.
void constitutive(Engine& e, bool averages = true) {
  for (auto& c : e.C) {
    if (!class_active(e, c)) continue;
    const int np = (int)c.probs.size();
    hipLaunchKernelGGL(zero_flag_batch, dim3((np + 255) / 256), dim3(256), 0, e.stream, e.ddesc, c.ids, np);
    HIPCALL(hipGetLastError());
    timed(e, "constitutive", [&] {
      const dim3 grid(c.vb, 1, np);
      if (c.kind == MAT_NH) {
        if (e.prec == GHOM_FP64)
          hipLaunchKernelGGL((constitutive_batch<double, MAT_NH>), grid, dim3(kVoxThreads), 0, e.stream, e.ddesc, c.ids);
        else
          hipLaunchKernelGGL((constitutive_batch<float, MAT_NH>), grid, dim3(kVoxThreads), 0, e.stream, e.ddesc, c.ids);
      } else if (c.kind == MAT_SVK) {
        if (e.prec == GHOM_FP64)
          hipLaunchKernelGGL((constitutive_batch<double, MAT_SVK>), grid, dim3(kVoxThreads), 0, e.stream, e.ddesc, c.ids);
        else
          hipLaunchKernelGGL((constitutive_batch<float, MAT_SVK>), grid, dim3(kVoxThreads), 0, e.stream, e.ddesc, c.ids);
      } else {
        if (e.prec == GHOM_FP64)
          hipLaunchKernelGGL((constitutive_batch<double, MAT_VISCO>), grid, dim3(kVoxThreads), 0, e.stream, e.ddesc,
                             c.ids);
        else
          hipLaunchKernelGGL((constitutive_batch<float, MAT_VISCO>), grid, dim3(kVoxThreads), 0, e.stream, e.ddesc,
                             c.ids);
      }
    });
    timed(e, "reduce", [&] {
      launch_sum_columns(e, c.ids, np, c.vb, 18, 0, 0, 0, 1);
    });
  }
  const size_t n = e.P.size();
  sync(e);  // the reduced values are written to mapped host memory
  for (size_t p = 0; p < n; ++p) {
    if (!e.hdesc[p].active) continue;
    Prob& q = e.P[p];
    const double N = (double)e.C[q.cls].g.N;
    if (averages) {
      for (int i = 0; i < 9; ++i) {
        q.Favg[i] = e.host_red[32 * p + i] / N;
        q.Pavg[i] = e.host_red[32 * p + 9 + i] / N;
      }
    }
    q.state_valid = true;
    q.p_field_valid = true;
    if (e.host_red[32 * p + kRedFlag] != 0.0) {
      q.state_valid = false;
      q.status = GHOM_EDOMAIN;
      q.msg = "det F <= 0 at some voxel";
      q.running = false;
    }
  }
}

// One Newton evaluation for every active problem: the constitutive update (P, tangent
// state, <F>, <P>; det F <= 0 gives EDOMAIN) fused into the forward pass of the FP64
// residual b = -G*(P - Pbar); sets rms_b and the r.r the next CG solve starts from.  The P
// field itself is stored for the viscoelastic law only (ensure_P_field recomputes it for the
// elastic laws where it is read).
void constitutive_residual(Engine& e) {
  constexpr int kRedB = 20;  // red[0..18): sums of F and P; red[20]: b.b
  for (auto& c : e.C) {
    if (!class_active(e, c)) continue;
    const int np = (int)c.probs.size();
    hipLaunchKernelGGL(zero_flag_batch, dim3((np + 255) / 256), dim3(256), 0, e.stream, e.ddesc, c.ids, np);
    HIPCALL(hipGetLastError());
    int gz = 0;
    if (c.kind == MAT_NH) {
      if (e.prec == GHOM_FP64) gz = launch_zfwd<double, Z_CONST_NH, double>(e, c, ROLE_RESID_R, 0, "res_zfwd_f64");
      else gz = launch_zfwd<double, Z_CONST_NH, float>(e, c, ROLE_RESID_R, 0, "res_zfwd_f64");
    } else if (c.kind == MAT_SVK) {
      if (e.prec == GHOM_FP64) gz = launch_zfwd<double, Z_CONST_SVK, double>(e, c, ROLE_RESID_R, 0, "res_zfwd_f64");
      else gz = launch_zfwd<double, Z_CONST_SVK, float>(e, c, ROLE_RESID_R, 0, "res_zfwd_f64");
    } else {
      if (e.prec == GHOM_FP64) gz = launch_zfwd<double, Z_CONST_VISCO, double>(e, c, ROLE_RESID_R, 0, "res_zfwd_f64");
      else gz = launch_zfwd<double, Z_CONST_VISCO, float>(e, c, ROLE_RESID_R, 0, "res_zfwd_f64");
    }
    timed(e, "reduce", [&] {
      launch_sum_columns(e, c.ids, np, gz, 18, 0, 1, 0, 1);
    });
    middle_passes<double>(e, c, ROLE_RESID_R, "res_");
    // b = -G*(P - Pbar) goes straight into the CG residual r in the CG type (the solve starts
    // from it with p = r); its square sum is taken before the narrowing store
    const int gi = e.prec == GHOM_FP64 ? launch_zinv<double, double, ZI_PLAIN>(e, c, ROLE_RESID_R, "res_zinv_f64")
                                       : launch_zinv<double, float, ZI_PLAIN>(e, c, ROLE_RESID_R, "res_zinv_f64");
    timed(e, "reduce", [&] {
      launch_sum_columns(e, c.ids, np, gi, 1, 0, 0, kRedB, 0);
    });
  }
  const size_t n = e.P.size();
  sync(e);  // the reduced values are written to mapped host memory
  for (size_t p = 0; p < n; ++p) {
    if (!e.hdesc[p].active) continue;
    Prob& q = e.P[p];
    const double N = (double)e.C[q.cls].g.N;
    for (int i = 0; i < 9; ++i) {
      q.Favg[i] = e.host_red[32 * p + i] / N;
      q.Pavg[i] = e.host_red[32 * p + 9 + i] / N;
    }
    q.state_valid = true;
    q.p_field_valid = q.kind == MAT_VISCO;
    const double bb = e.host_red[32 * p + kRedB];
    q.rms_b = std::sqrt(bb / N);
    e.hdesc[p].rr0 = bb;
    if (e.host_red[32 * p + kRedFlag] != 0.0) {
      q.state_valid = false;
      q.status = GHOM_EDOMAIN;
      q.msg = "det F <= 0 at some voxel";
      q.running = false;
    }
  }
}

// Conjugate gradients on A dF = b from dF = 0 for every active problem; the stop test of
// each problem is set in its descriptor (cg_thresh, max_cg).  Returns when all are done.
// finish: apply the step of the last completed iteration to x here (the Newton update, which
// reads x anyway, applies it itself and passes false).  rhs_in_r: b is already in r (in the CG
// type), as the Newton residual writes it; else it is read from the float64 buffer b.
template <typename T>
void cg_solve(Engine& e, double* t_ms, bool finish = true, bool rhs_in_r = false) {
  const auto t0 = std::chrono::steady_clock::now();
  long long vox = 0;
  for (auto& c : e.C) {
    const int np = (int)c.probs.size();
    for (int p : c.probs)
      if (e.hdesc[p].active) vox += c.g.N;
    hipLaunchKernelGGL(cg_start_batch, dim3((np + 63) / 64), dim3(64), 0, e.stream, e.ddesc, c.ids, np);
    HIPCALL(hipGetLastError());
  }
  // The host reads the stop flags one chunk behind: the CG kernels write every problem's
  // scalars into mapped host memory, and while the host waits for the event after chunk k,
  // chunk k+1 is already queued, so the GPU never idles on the round trip.  Iterations queued
  // after every problem has stopped find their done flag set and return at once; they change
  // nothing.
  int enqueued = 0;
  int chunk = vox >= (1LL << 21) ? 1 : (vox >= (1LL << 18) ? 2 : 8);
  const size_t n = e.P.size();
  int it_cap = 0;  // no problem runs more CG steps than its max_cg
  for (size_t p = 0; p < n; ++p)
    if (e.hdesc[p].active) it_cap = std::max(it_cap, e.hdesc[p].max_cg);
  // k CG iterations of every class (the first one starts the solve when `first`); in graph
  // mode every class is included, since a problem's activity is read by the kernels
  auto launch_iters = [&](int k, bool first, bool all_classes) {
    for (int i = 0; i < k; ++i) {
      for (auto& c : e.C) {
        if (!all_classes && !class_active(e, c)) continue;
        const int gz = operator_apply<T>(e, c, ROLE_OP_CG, (first && i == 0) ? (rhs_in_r ? 3 : 2) : 1);
        timed(e, "cg_beta", [&] {
          hipLaunchKernelGGL(cg_beta_batch, dim3((unsigned)c.probs.size()), dim3(kRedThreads), 0, e.stream, e.ddesc,
                             c.ids, gz);
        });
      }
    }
  };
  auto enqueue_chunk = [&](int k) {
    const bool first = enqueued == 0;
    if (e.graphs && !e.prof) {
      const long long key = ((long long)sizeof(T) << 40) | ((long long)rhs_in_r << 33) | ((long long)first << 32) |
                            (long long)k;
      auto it = e.graph_cache.find(key);
      if (it == e.graph_cache.end()) {
        hipGraph_t g = nullptr;
        HIPCALL(hipStreamBeginCapture(e.stream, hipStreamCaptureModeThreadLocal));
        launch_iters(k, first, true);
        HIPCALL(hipStreamEndCapture(e.stream, &g));
        hipGraphExec_t x = nullptr;
        const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCALL(ie);
        it = e.graph_cache.emplace(key, x).first;
      }
      HIPCALL(hipGraphLaunch(it->second, e.stream));
    } else {
      launch_iters(k, first, false);
    }
    enqueued += k;
  };
  auto mark = [&](int slot) { HIPCALL(hipEventRecord(e.sc_ev[slot], e.stream)); };
  auto all_done = [&](int slot) {
    HIPCALL(hipEventSynchronize(e.sc_ev[slot]));
    const volatile CGScalars* hs = e.host_sc;
    for (size_t p = 0; p < n; ++p)
      if (e.hdesc[p].active && !hs[p].done) return false;
    return true;
  };
  // One iteration per chunk (large problems) and no graphs: the next iteration is queued in two
  // parts, its forward z pass before the host waits for the current iteration's flags and the
  // passes after it once the flags say go on (the forward pass runs meanwhile), so that a
  // solve that has stopped leaves one forward pass to return at once instead of a whole
  // iteration.
  const bool split = chunk == 1 && !(e.graphs && !e.prof);
  auto launch_part = [&](bool first, int part) {
    for (auto& c : e.C) {
      if (!class_active(e, c)) continue;
      const int gz = operator_apply<T>(e, c, ROLE_OP_CG, first ? (rhs_in_r ? 3 : 2) : 1, part);
      if (part == 2)
        timed(e, "cg_beta", [&] {
          hipLaunchKernelGGL(cg_beta_batch, dim3((unsigned)c.probs.size()), dim3(kRedThreads), 0, e.stream, e.ddesc,
                             c.ids, gz);
        });
    }
  };
  int slot = 0;
  if (split) {
    launch_part(true, 1);
    launch_part(true, 2);
    mark(0);
    launch_part(false, 1);
    enqueued = 1;
    for (;;) {
      if (enqueued > it_cap + 64) fail(GHOM_EHIP, "CG stop flags not seen by the host");
      if (all_done(slot)) break;
      launch_part(false, 2);
      mark(1 - slot);
      launch_part(false, 1);
      enqueued += 1;
      slot = 1 - slot;
    }
  } else {
    enqueue_chunk(chunk);
    mark(0);
    for (;;) {
      if (enqueued > it_cap + 64) fail(GHOM_EHIP, "CG stop flags not seen by the host");
      if (chunk < 8 && vox < (1LL << 21)) chunk *= 2;
      enqueue_chunk(chunk);
      mark(1 - slot);
      if (all_done(slot)) break;
      slot = 1 - slot;
    }
    // the chunk queued last returns at once; wait for it, so that the scalars are final
    HIPCALL(hipEventSynchronize(e.sc_ev[1 - slot]));
  }
  // a problem that stopped before its first step gets x = 0
  for (auto& c : e.C)
    for (int p : c.probs)
      if (e.hdesc[p].active && e.host_sc[p].it == 0 && e.host_sc[p].status == CG_CONVERGED) {
        const long long nd = (9LL * c.g.N * (long long)sizeof(T) + 7) / 8;  // arena buffers are padded
        hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, e.stream, nd, reinterpret_cast<double*>(e.hdesc[p].x));
        HIPCALL(hipGetLastError());
      }
  // the step the last completed iteration took reaches the iterate here (the forward pass of
  // the iteration after it would have applied it)
  for (auto& c : e.C) {
    if (!finish || !class_active(e, c)) continue;
    timed(e, "cg_finish", [&] {
      hipLaunchKernelGGL(cg_finish_batch<T>, dim3(c.vb, 1, (unsigned)c.probs.size()), dim3(kVoxThreads), 0, e.stream,
                         e.ddesc, c.ids);
    });
  }
  sync(e);
  if (t_ms) *t_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// F += dF for every active problem; sets crit = max |dF| / |<F>|.  FP64: dF = x.
// FP32-split: dF = G*(x) by one float64 transform pair, added to F by its last pass.
void newton_update(Engine& e, std::vector<double>& crit) {
  for (auto& c : e.C) {
    if (!class_active(e, c)) continue;
    const int np = (int)c.probs.size();
    if (e.prec == GHOM_FP32_SPLIT) {
      const int gi = project64(e, c, ROLE_NEWTON, "reproj");
      timed(e, "reduce", [&] {
        launch_sum_columns(e, c.ids, np, gi, 10, 1, 1, 0, 0);
      });
      continue;
    }
    timed(e, "newton_update", [&] {
      hipLaunchKernelGGL(newton_update_batch, dim3(c.vb, 1, np), dim3(kVoxThreads), 0, e.stream, e.ddesc, c.ids);
    });
    timed(e, "reduce", [&] {
      launch_sum_columns(e, c.ids, np, c.vb, 10, 1, 0, 0, 0);
    });
  }
  const size_t n = e.P.size();
  sync(e);  // the reduced values are written to mapped host memory
  crit.assign(n, 0.0);
  for (size_t p = 0; p < n; ++p) {
    if (!e.hdesc[p].active) continue;
    const double N = (double)e.C[e.P[p].cls].g.N;
    double nf = 0.0;
    for (int i = 0; i < 9; ++i) {
      const double m = e.host_red[32 * p + 1 + i] / N;
      nf += m * m;
    }
    crit[p] = std::sqrt(e.host_red[32 * p]) / std::sqrt(nf);
    e.P[p].state_valid = false;
  }
}

// Relative CG forcing.  Float32 CG cannot take its residual much below 1e-6 of the
// right-hand side, so in FP32-split mode the stop is never tighter than 1e-5 of it; the
// float64 Newton residual still drives the solution to the Newton tolerance.
constexpr double kSplitMinForcing = 1e-5;
double forcing(const Engine& e) {
  return e.prec == GHOM_FP32_SPLIT ? std::max(e.cg_forcing, kSplitMinForcing) : e.cg_forcing;
}

void set_active_from_running(Engine& e, const std::vector<int>& set) {
  for (size_t p = 0; p < e.P.size(); ++p) e.hdesc[p].active = 0;
  for (int p : set) e.hdesc[p].active = e.P[p].running ? 1 : 0;
  upload_descs(e);
}

bool any_running(Engine& e, const std::vector<int>& set) {
  for (int p : set)
    if (e.P[p].running) return true;
  return false;
}

// Newton (eq. 20) for the problems in `set`, each at its own stress target (descriptor
// pbar).  Per-problem outcome in P[p].status / info.
void newton(Engine& e, const std::vector<int>& set) {
  const auto t0 = std::chrono::steady_clock::now();
  for (int p : set) {
    Prob& q = e.P[p];
    q.running = true;
    q.status = GHOM_ENOTCONVERGED;
    q.msg = "Newton reached max_newton";
    q.info = ghom_step_info{};
    q.info.crit = INFINITY;
  }
  std::vector<double> crit;
  for (int it = 0; it < e.max_newton && any_running(e, set); ++it) {
    set_active_from_running(e, set);
    for (int p : set)
      if (e.P[p].running) e.P[p].info.newton_iters += 1;
    constitutive_residual(e);
    for (int p : set) {
      Prob& q = e.P[p];
      if (!q.running) continue;
      q.info.res_rms = q.rms_b;
      if (!std::isfinite(q.rms_b)) {
        q.status = GHOM_EDOMAIN;
        q.msg = "non-finite Newton residual";
        q.running = false;
      } else if (q.rms_b <= e.cg_tol) {
        q.status = GHOM_OK;
        q.running = false;
      } else {
        const double tol = std::max(e.cg_tol, forcing(e) * q.rms_b);
        e.hdesc[p].cg_thresh = tol * tol * (double)e.C[q.cls].g.N;
        e.hdesc[p].max_cg = e.max_cg;
      }
    }
    set_active_from_running(e, set);
    if (!any_running(e, set)) break;
    double tcg = 0.0;
    // newton_update applies the pending step; the residual left the right-hand side in r
    if (e.prec == GHOM_FP64) cg_solve<double>(e, &tcg, false, true);
    else cg_solve<float>(e, &tcg, false, true);
    for (int p : set) {
      Prob& q = e.P[p];
      if (!q.running) continue;
      q.info.t_cg_ms += tcg;
      const CGScalars& s = e.host_sc[p];
      q.info.cg_iters_total += s.it;
      if (s.status == CG_BREAKDOWN) {
        if (s.it == 0) {
          q.status = GHOM_ESINGULAR;
          q.msg = "CG breakdown (p.Ap <= 0) at its first iteration";
          q.running = false;
        } else {
          q.info.cg_breakdowns += 1;
        }
      } else if (s.status == CG_STALLED) {
        q.info.cg_stalls += 1;  // Newton continues with the iterate
      } else if (s.status == CG_CAP) {
        q.status = GHOM_ENOTCONVERGED;
        q.msg = "CG reached max_cg";
        q.running = false;
      }
    }
    set_active_from_running(e, set);
    if (!any_running(e, set)) break;
    newton_update(e, crit);
    for (int p : set) {
      Prob& q = e.P[p];
      if (!q.running) continue;
      q.info.crit = crit[p];
      if (!std::isfinite(crit[p])) {
        q.status = GHOM_EDOMAIN;
        q.msg = "non-finite Newton correction";
        q.running = false;
      } else if (crit[p] < e.newton_tol) {
        q.status = GHOM_OK;
        q.running = false;
      }
    }
  }
  for (int p : set) e.P[p].running = false;
  // P and the averages at the final F of every problem of the solve (not after EDOMAIN;
  // a problem whose last Newton evaluation was at its final F has them already)
  for (size_t p = 0; p < e.P.size(); ++p) e.hdesc[p].active = 0;
  bool need = false;
  for (int p : set) {
    e.hdesc[p].active = (e.P[p].status == GHOM_EDOMAIN || e.P[p].state_valid) ? 0 : 1;
    need = need || e.hdesc[p].active;
  }
  upload_descs(e);
  std::vector<int> keep_status(e.P.size());
  std::vector<std::string> keep_msg(e.P.size());
  for (int p : set) {
    keep_status[p] = e.P[p].status;
    keep_msg[p] = e.P[p].msg;
  }
  if (need) constitutive(e);
  for (int p : set)
    if (keep_status[p] != GHOM_EDOMAIN && e.P[p].state_valid) {
      e.P[p].status = keep_status[p];
      e.P[p].msg = keep_msg[p];
    }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int p : set) {
    e.P[p].info.t_total_ms = ms;
    e.P[p].info.status = e.P[p].status;
  }
}

// The mask problem p is solved with: the mask as set, with the rotation gauge of full
// stress control applied when it is on and the history is uniaxial (control.hpp); mirrored
// into the descriptor.
void apply_control(Engine& e, int p) {
  Prob& q = e.P[p];
  if (!q.mask_set) return;
  uint8_t m[9];
  q.gauge_axis = effective_mask(q.user_mask, q.target.empty() ? nullptr : q.target.data(), q.nsteps, e.rot_gauge, m);
  unsigned bits = 0;
  for (int i = 0; i < 9; ++i) {
    q.mask[i] = m[i];
    if (m[i]) bits |= 1u << i;
  }
  e.hdesc[p].mask = bits;
}

// Prescribed values of increment k (row k-1 of the history); increment 0 is F = I, P = 0.
void target_row(const Prob& q, int k, double* out) {
  for (int i = 0; i < 9; ++i)
    out[i] = k == 0 ? ((!q.mask[i] && i % 4 == 0) ? 1.0 : 0.0) : q.target[(size_t)(k - 1) * 9 + i];
}

// Moves problem p's prescribed values from `from` to `to`: the deformation-controlled means
// shift uniformly by to - from, the stress targets become `to`.  Returns whether F moves.
bool set_targets(Engine& e, int p, const double* from, const double* to) {
  Prob& q = e.P[p];
  ProbDesc& d = e.hdesc[p];
  bool any = false;
  for (int i = 0; i < 9; ++i) {
    d.shift[i] = 0.0;
    d.pbar[i] = 0.0;
    if (q.mask[i]) {
      d.pbar[i] = to[i];
    } else {
      d.shift[i] = to[i] - from[i];
      any = any || d.shift[i] != 0.0;
    }
  }
  if (any) q.state_valid = false;
  return any;
}

// Shift the deformation-controlled means to increment k+1 and set the stress targets.
void begin_increment(Engine& e, const std::vector<int>& set) {
  for (size_t p = 0; p < e.P.size(); ++p) e.hdesc[p].active = 0;
  for (int p : set) {
    Prob& q = e.P[p];
    double from[9], to[9];
    target_row(q, q.k, from);
    target_row(q, q.k + 1, to);
    e.hdesc[p].active = set_targets(e, p, from, to) ? 1 : 0;
  }
  upload_descs(e);
  for (auto& c : e.C) {
    if (!class_active(e, c)) continue;
    timed(e, "shift", [&] {
      hipLaunchKernelGGL(shift_batch, dim3(c.vb, 1, (unsigned)c.probs.size()), dim3(kVoxThreads), 0, e.stream, e.ddesc,
                         c.ids);
    });
  }
}

void set_pbar_current(Engine& e, int p) {
  Prob& q = e.P[p];
  for (int i = 0; i < 9; ++i)
    e.hdesc[p].pbar[i] = (q.k >= 1 && q.mask[i]) ? q.target[(size_t)(q.k - 1) * 9 + i] : 0.0;
}

// F = I for the given problems
void drop_checkpoints(Engine& e, int p) {
  Prob& q = e.P[p];
  if (q.ckpt.empty()) return;
  sync(e);
  for (double* b : q.ckpt) (void)hipFree(b);
  q.ckpt.clear();
  q.ckpt_dt.clear();
  q.ckpt_k0 = -1;
}

// Viscoelastic law with checkpoints on: keep F at convergence and the internal variables the
// increment started from (call before the commit), with the increment's length.
void visco_checkpoint(Engine& e, int p, double dt_eff) {
  Prob& q = e.P[p];
  if (!e.checkpoints || q.kind != MAT_VISCO) return;
  const size_t N = (size_t)e.C[q.cls].g.N;
  double* buf = nullptr;
  HIPCALL(hipMalloc((void**)&buf, (9 + kViscoIV) * N * sizeof(double)));
  if (q.ckpt.empty()) q.ckpt_k0 = q.k;
  q.ckpt.push_back(buf);
  q.ckpt_dt.push_back(dt_eff);
  HIPCALL(hipMemcpyAsync(buf, e.hdesc[p].F, 9 * N * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
  HIPCALL(hipMemcpyAsync(buf + 9 * N, q.iv, kViscoIV * N * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
}

void reset_state(Engine& e, const std::vector<int>& set) {
  for (size_t p = 0; p < e.P.size(); ++p) e.hdesc[p].active = 0;
  for (int p : set) {
    e.hdesc[p].active = 1;
    for (int i = 0; i < 9; ++i) e.hdesc[p].fill[i] = (i % 4 == 0) ? 1.0 : 0.0;
    Prob& q = e.P[p];
    q.k = 0;
    q.state_valid = false;
    drop_checkpoints(e, p);
    for (int i = 0; i < 9; ++i) {
      q.Favg[i] = e.hdesc[p].fill[i];
      q.Pavg[i] = 0.0;
    }
  }
  upload_descs(e);
  for (auto& c : e.C) {
    if (!class_active(e, c)) continue;
    hipLaunchKernelGGL(fill9_batch, dim3(c.vb, 1, (unsigned)c.probs.size()), dim3(kVoxThreads), 0, e.stream, e.ddesc,
                       c.ids, 0);
    HIPCALL(hipGetLastError());
  }
  for (int p : set)
    if (e.P[p].iv) {
      hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, e.stream, (long long)kViscoIV * e.C[e.P[p].cls].g.N,
                         e.P[p].iv);
      HIPCALL(hipGetLastError());
    }
  sync(e);
}

// ------------------------------------------------------------------ construction -------
struct ProbSpec {
  int nx, ny, nz;
  double L[3];
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

void destroy_engine(Engine* e) {
  if (!e) return;
  (void)hipSetDevice(e->device);
  if (e->stream) (void)hipStreamSynchronize(e->stream);
  for (auto& q : e->P) {
    if (q.scale) (void)hipFree(q.scale);
    if (q.mat) (void)hipFree(q.mat);
    if (q.mat32) (void)hipFree(q.mat32);
    if (q.visc) (void)hipFree(q.visc);
    if (q.iv) (void)hipFree(q.iv);
    for (double* b : q.ckpt) (void)hipFree(b);
  }
  for (auto& c : e->C) {
    if (c.ids) (void)hipFree(c.ids);
    for (int a = 0; a < 3; ++a) {
      if (c.tw64[a]) (void)hipFree(c.tw64[a]);
      if (c.tw32[a]) (void)hipFree(c.tw32[a]);
    }
  }
  void* ptrs[] = {e->arena, e->ddesc, e->sc, e->flags, e->ckpt};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (e->hdesc) (void)hipHostFree(e->hdesc);
  for (int k = 0; k < Engine::kDescSlots; ++k) {
    if (e->desc_stage[k]) (void)hipHostFree(e->desc_stage[k]);
    if (e->desc_ev[k]) (void)hipEventDestroy(e->desc_ev[k]);
  }
  if (e->host_sc) (void)hipHostFree(e->host_sc);
  if (e->host_red) (void)hipHostFree(e->host_red);
  for (auto& kv : e->prof_recs)
    for (auto& pr : kv.second.pending) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t ev : e->ev_pool) (void)hipEventDestroy(ev);
  for (auto& kv : e->graph_cache) (void)hipGraphExecDestroy(kv.second);
  for (hipEvent_t ev : e->sc_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
  delete e;
}

// Allocates every problem's buffers (one arena), the descriptors and the shape classes.
void build_engine(Engine& e, const std::vector<ProbSpec>& specs, const std::vector<int>& kinds) {
  const size_t n = specs.size();
  e.P.resize(n);
  // shape classes keyed by (nx, ny, nz, kind, cell lengths)
  for (size_t p = 0; p < n; ++p) {
    const ProbSpec& s = specs[p];
    int found = -1;
    for (size_t c = 0; c < e.C.size(); ++c) {
      const ShapeClass& k = e.C[c];
      if (k.nx == s.nx && k.ny == s.ny && k.nz == s.nz && k.kind == kinds[p] && k.g.invL[0] == 1.0 / s.L[0] &&
          k.g.invL[1] == 1.0 / s.L[1] && k.g.invL[2] == 1.0 / s.L[2])
        found = (int)c;
    }
    if (found < 0) {
      ShapeClass k;
      k.nx = s.nx;
      k.ny = s.ny;
      k.nz = s.nz;
      k.kind = kinds[p];
      k.g.nx = s.nx;
      k.g.ny = s.ny;
      k.g.nz = s.nz;
      k.g.nzh = (s.nz % 2 == 0) ? s.nz / 2 : (s.nz + 1) / 2;
      k.g.N = (long long)s.nx * s.ny * s.nz;
      k.g.Nh = (long long)s.nx * s.ny * k.g.nzh;
      for (int a = 0; a < 3; ++a) k.g.invL[a] = 1.0 / s.L[a];
      k.vb = vox_blocks(k.g.N);
      e.C.push_back(k);
      found = (int)e.C.size() - 1;
    }
    e.C[found].probs.push_back((int)p);
    e.P[p].cls = found;
    e.P[p].kind = kinds[p];
  }
  // partials per problem: the largest block count of any reducing launch
  size_t np = 64;
  for (auto& c : e.C) {
    // z passes: at most ceil(nx ny / 2) blocks, up to 18 partials each (fused residual
    // pass); voxel kernels: c.vb blocks with up to 18 partials each
    np = std::max(np, 18 * (((size_t)c.nx * c.ny + 1) / 2) + 64);
    np = std::max(np, (size_t)c.vb * 18);
  }
  e.np = np;
  // arena layout
  auto sizes = [&](const Geo& g) {
    const size_t N = (size_t)g.N;
    size_t b = 0;
    b += 3 * align256(9 * N * 8);                                       // F, P, b
    if (e.prec == GHOM_FP32_SPLIT) b += align256(9 * N * 8);            // dF64
    b += 3 * align256(9 * N * e.tsz);                                   // x, r, p
    b += align256((size_t)kStatePlanes * N * e.tsz);                    // state (either law)
    b += align256(9 * (size_t)g.Nh * sizeof(cx<double>));               // spectrum
    b += align256(N * sizeof(uint16_t));                                // phase
    b += align256(np * sizeof(double));                                 // partials
    return b;
  };
  std::vector<size_t> off(n);
  size_t total = 0;
  double cg_bytes = 0.0;  // bytes one CG iteration of every problem touches
  for (size_t p = 0; p < n; ++p) {
    off[p] = total;
    total += sizes(e.C[e.P[p].cls].g);
    cg_bytes += (double)e.C[e.P[p].cls].g.N * (45.0 * (double)e.tsz + 2.0);
  }
  e.stream_nt = cg_bytes > 256.0 * 1024 * 1024;  // beyond the last-level cache
  HIPCALL(hipMalloc((void**)&e.arena, total));
  HIPCALL(hipMalloc((void**)&e.ddesc, n * sizeof(ProbDesc)));
  HIPCALL(hipMalloc((void**)&e.sc, n * sizeof(CGScalars)));
  HIPCALL(hipMalloc((void**)&e.flags, n * sizeof(int)));
  HIPCALL(hipHostMalloc((void**)&e.hdesc, n * sizeof(ProbDesc), hipHostMallocDefault));
  for (int k = 0; k < Engine::kDescSlots; ++k) {
    HIPCALL(hipHostMalloc((void**)&e.desc_stage[k], n * sizeof(ProbDesc), hipHostMallocDefault));
    HIPCALL(hipEventCreateWithFlags(&e.desc_ev[k], hipEventDisableTiming));
  }
  // coherent mapped memory: the CG kernels' stores reach the host without a copy
  HIPCALL(hipHostMalloc((void**)&e.host_sc, n * sizeof(CGScalars), hipHostMallocMapped | hipHostMallocCoherent));
  HIPCALL(hipHostGetDevicePointer((void**)&e.host_sc_dev, e.host_sc, 0));
  std::fill(e.host_sc, e.host_sc + n, CGScalars{});
  for (auto& ev : e.sc_ev) HIPCALL(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  // reduced values (sums, maxima, the det F flag) are stored by the reduction kernels into
  // coherent mapped host memory: the host reads them after a stream synchronisation
  HIPCALL(hipHostMalloc((void**)&e.host_red, n * 32 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
  HIPCALL(hipHostGetDevicePointer((void**)&e.red, e.host_red, 0));
  std::fill(e.host_red, e.host_red + 32 * n, 0.0);
  // twiddles W_n^k = exp(-2 pi i k / n) and device id lists per class
  for (auto& c : e.C) {
    const int ns[3] = {c.nx, c.ny, c.nz};
    for (int a = 0; a < 3; ++a) {
      std::vector<cx<double>> t64(ns[a]);
      std::vector<cx<float>> t32(ns[a]);
      for (int k = 0; k < ns[a]; ++k) {
        const CosSin cs = cossin_2pi(k, ns[a]);
        t64[k] = cx<double>{(double)cs.c, (double)-cs.s};
        t32[k] = cx<float>{(float)cs.c, (float)-cs.s};
      }
      HIPCALL(hipMalloc((void**)&c.tw64[a], ns[a] * sizeof(cx<double>)));
      HIPCALL(hipMalloc((void**)&c.tw32[a], ns[a] * sizeof(cx<float>)));
      HIPCALL(hipMemcpy(c.tw64[a], t64.data(), ns[a] * sizeof(cx<double>), hipMemcpyHostToDevice));
      HIPCALL(hipMemcpy(c.tw32[a], t32.data(), ns[a] * sizeof(cx<float>), hipMemcpyHostToDevice));
    }
    HIPCALL(hipMalloc((void**)&c.ids, c.probs.size() * sizeof(int)));
    HIPCALL(hipMemcpy(c.ids, c.probs.data(), c.probs.size() * sizeof(int), hipMemcpyHostToDevice));
  }
  // descriptors
  for (size_t p = 0; p < n; ++p) {
    const ShapeClass& c = e.C[e.P[p].cls];
    const size_t N = (size_t)c.g.N;
    ProbDesc& d = e.hdesc[p];
    std::memset(&d, 0, sizeof(ProbDesc));
    d.g = c.g;
    d.kind = e.P[p].kind;
    char* q = e.arena + off[p];
    auto take = [&](size_t bytes) {
      char* r = q;
      q += align256(bytes);
      return (void*)r;
    };
    d.F = (double*)take(9 * N * 8);
    d.P = (double*)take(9 * N * 8);
    d.b = (double*)take(9 * N * 8);
    d.dF64 = e.prec == GHOM_FP32_SPLIT ? (double*)take(9 * N * 8) : nullptr;
    d.x = take(9 * N * e.tsz);
    d.r = take(9 * N * e.tsz);
    d.p = take(9 * N * e.tsz);
    d.state = take((size_t)kStatePlanes * N * e.tsz);
    d.H = take(9 * (size_t)c.g.Nh * sizeof(cx<double>));
    d.phase = (const uint16_t*)take(N * sizeof(uint16_t));
    d.partials = (double*)take(np * sizeof(double));
    for (int a = 0; a < 3; ++a) {
      d.tw64[a] = c.tw64[a];
      d.tw32[a] = c.tw32[a];
    }
    d.sc = e.sc + p;
    d.sc_host = e.host_sc_dev + p;
    d.red = e.red + 32 * p;
    d.flag = e.flags + p;
  }
  std::vector<int> all(n);
  for (size_t p = 0; p < n; ++p) all[p] = (int)p;
  reset_state(e, all);
  for (auto& c : e.C) tune_class(e, c, -1);
}

void check_material(const Prob& q) {
  if (!q.kind) fail(GHOM_ESTATE, "no material set");
  if (!q.mask_set) fail(GHOM_ESTATE, "no control mask set");
}

// Voigt table (36 per phase, order 11 22 33 23 13 12) from C_ijkl, with symmetry checks
std::vector<double> voigt_table(const double* C, int nphase) {
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
  return tab;
}

// Sets the material of problem p (kind, phase map, tables) and resets it to F = I.
void set_material(Engine& e, int p, int kind, const uint16_t* phase, int nphase, const std::vector<double>& tab) {
  Prob& q = e.P[p];
  ShapeClass& c = e.C[q.cls];
  const long long N = c.g.N;
  for (long long v = 0; v < N; ++v)
    if (phase[v] >= nphase) fail(GHOM_EINVAL, "phase index out of range");
  if (c.probs.size() > 1 && c.kind != kind) fail(GHOM_EINVAL, "problems of one shape class need one material law");
  sync(e);
  if (q.mat) HIPCALL(hipFree(q.mat));
  if (q.mat32) HIPCALL(hipFree(q.mat32));
  q.mat = nullptr;
  q.mat32 = nullptr;
  HIPCALL(hipMalloc((void**)&q.mat, tab.size() * sizeof(double)));
  HIPCALL(hipMemcpy(q.mat, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
  if (kind != MAT_NH) {
    std::vector<float> t32(tab.begin(), tab.end());
    HIPCALL(hipMalloc((void**)&q.mat32, t32.size() * sizeof(float)));
    HIPCALL(hipMemcpy(q.mat32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  HIPCALL(hipMemcpy(const_cast<uint16_t*>(e.hdesc[p].phase), phase, (size_t)N * sizeof(uint16_t),
                    hipMemcpyHostToDevice));
  q.kind = kind;
  q.nphase = nphase;
  e.hdesc[p].kind = kind;
  e.hdesc[p].mat = q.mat;
  e.hdesc[p].mat32 = q.mat32;
  c.kind = kind;
  reset_state(e, {p});
}

// Viscoelastic law, increment of length dt_eff: the per-phase device table (Cinf, C1,
// a = exp(-dt/tau), b = tau (1 - a) / dt) and the algorithmic stiffness Cinf + b C1 the
// tangent uses (float64 and float32 copies).
void visco_tables(Engine& e, int p, double dt_eff) {
  Prob& q = e.P[p];
  const int np = q.nphase;
  std::vector<double> vt((size_t)kViscoTable * np), calg(36 * (size_t)np);
  for (int ph = 0; ph < np; ++ph) {
    const double x = dt_eff / q.vtau[ph];
    const double a = std::exp(-x);
    const double b = x > 0.0 ? -std::expm1(-x) / x : 1.0;
    double* t = &vt[(size_t)kViscoTable * ph];
    for (int k = 0; k < 36; ++k) {
      t[k] = q.vinf[36 * (size_t)ph + k];
      t[36 + k] = q.v1[36 * (size_t)ph + k];
      calg[36 * (size_t)ph + k] = t[k] + b * t[36 + k];
    }
    t[72] = a;
    t[73] = b;
  }
  std::vector<float> c32(calg.begin(), calg.end());
  sync(e);
  HIPCALL(hipMemcpy(q.visc, vt.data(), vt.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCALL(hipMemcpy(q.mat, calg.data(), calg.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPCALL(hipMemcpy(q.mat32, c32.data(), c32.size() * sizeof(float), hipMemcpyHostToDevice));
  q.state_valid = false;
}

// End of an accepted increment of the viscoelastic law for problem p (F converged).
void visco_commit(Engine& e, int p) {
  for (size_t i = 0; i < e.P.size(); ++i) e.hdesc[i].active = (int)i == p ? 1 : 0;
  upload_descs(e);
  ShapeClass& c = e.C[e.P[p].cls];
  hipLaunchKernelGGL(visco_commit_batch, dim3(c.vb, 1, (unsigned)c.probs.size()), dim3(kVoxThreads), 0, e.stream,
                     e.ddesc, c.ids);
  HIPCALL(hipGetLastError());
  // P and the averages stay those of the converged increment
}

void refresh_averages(Engine& e, int p) {
  if (e.P[p].state_valid || !e.P[p].kind) return;
  for (size_t i = 0; i < e.P.size(); ++i) e.hdesc[i].active = (int)i == p ? 1 : 0;
  upload_descs(e);
  const int keep = e.P[p].status;
  constitutive(e);
  if (!e.P[p].state_valid) fail(GHOM_EDOMAIN, "det F <= 0 at some voxel");
  e.P[p].status = keep;
}

// P(F) of problem p in its P field, for a reader of that field; the averages and the status
// stay those of the last evaluation
void ensure_P_field(Engine& e, int p) {
  refresh_averages(e, p);
  if (e.P[p].p_field_valid) return;
  for (size_t i = 0; i < e.P.size(); ++i) e.hdesc[i].active = (int)i == p ? 1 : 0;
  upload_descs(e);
  const int keep = e.P[p].status;
  const std::string keep_msg = e.P[p].msg;
  constitutive(e, false);
  if (!e.P[p].state_valid) fail(GHOM_EDOMAIN, "det F <= 0 at some voxel");
  e.P[p].status = keep;
  e.P[p].msg = keep_msg;
}

void copy_field(Engine& e, int p, int which, double* dst, hipMemcpyKind kind) {
  if (which != GHOM_FIELD_F && which != GHOM_FIELD_P) fail(GHOM_EINVAL, "bad field request");
  if (which == GHOM_FIELD_P) {
    check_material(e.P[p]);
    ensure_P_field(e, p);
  }
  sync(e);
  const size_t bytes = 9 * (size_t)e.C[e.P[p].cls].g.N * sizeof(double);
  HIPCALL(hipMemcpy(dst, which == GHOM_FIELD_F ? e.hdesc[p].F : e.hdesc[p].P, bytes, kind));
}

int finish_solve(Engine& e, int p, ghom_step_info* info) {
  Prob& q = e.P[p];
  if (info) *info = q.info;
  if (q.status != GHOM_OK) fail(q.status, q.msg);
  return GHOM_OK;
}

}  // namespace

// =====================================================================================
// Single-problem context = engine with one problem
// =====================================================================================
struct ghom_ctx {
  Engine* e = nullptr;
};

struct ghom_batch {
  Engine* e = nullptr;
};

namespace {

template <typename F>
int guard(ghom_ctx* c, F&& f) {
  if (!c || !c->e) return GHOM_EINVAL;
  return guarded(c->e, std::forward<F>(f));
}

template <typename F>
int guard(ghom_batch* b, F&& f) {
  if (!b || !b->e) return GHOM_EINVAL;
  return guarded(b->e, std::forward<F>(f));
}

Engine* new_engine(int precision, int device, void* hip_stream) {
  Engine* e = new (std::nothrow) Engine();
  if (!e) return nullptr;
  e->device = device;
  e->prec = precision;
  e->tsz = precision == GHOM_FP64 ? 8 : 4;
  return e;
}

void open_stream(Engine& e, void* hip_stream) {
  if (hip_stream) {
    e.stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    HIPCALL(hipStreamCreateWithFlags(&e.stream, hipStreamNonBlocking));
    e.own_stream = true;
  }
}

}  // namespace

extern "C" {

namespace {
// message of the last failed ghom_create / ghom_batch_create of this thread
thread_local std::string g_create_err;
int create_fail(int code, const std::string& msg) {
  g_create_err = msg;
  return code;
}
const char* kLengths = "4, 6, 8, 9, 12, 16, 18, 24, 27, 32, 36, 48, 64, 72, 96, 128, 144, 192, 256, 512";
}  // namespace

int ghom_create(ghom_ctx** out, int nx, int ny, int nz, double Lx, double Ly, double Lz, int precision, int device,
                void* hip_stream) {
  g_create_err.clear();
  if (!out) return create_fail(GHOM_EINVAL, "null output");
  *out = nullptr;
  if (!supported_length(nx) || !supported_length(ny) || !supported_length(nz))
    return create_fail(GHOM_EINVAL, std::string("grid lengths must be among ") + kLengths);
  if (!(Lx > 0 && Ly > 0 && Lz > 0)) return create_fail(GHOM_EINVAL, "cell lengths must be > 0");
  if (precision != GHOM_FP64 && precision != GHOM_FP32_SPLIT) return create_fail(GHOM_EINVAL, "unknown precision");
  Engine* e = new_engine(precision, device, hip_stream);
  if (!e) return create_fail(GHOM_ENOMEM, "host allocation failed");
  const int rc = guarded(e, [&]() -> int {
    open_stream(*e, hip_stream);
    build_engine(*e, {ProbSpec{nx, ny, nz, {Lx, Ly, Lz}}}, {0});
    return GHOM_OK;
  });
  ghom_ctx* c = rc == GHOM_OK ? new (std::nothrow) ghom_ctx() : nullptr;
  if (!c) {
    g_create_err = rc != GHOM_OK ? e->err : std::string("host allocation failed");
    destroy_engine(e);
    return rc != GHOM_OK ? rc : GHOM_ENOMEM;
  }
  c->e = e;
  *out = c;
  return GHOM_OK;
}

void ghom_destroy(ghom_ctx* c) {
  if (!c) return;
  destroy_engine(c->e);
  delete c;
}

const char* ghom_last_error(const ghom_ctx* c) {
  if (!c) return g_create_err.empty() ? "null context" : g_create_err.c_str();
  return c->e ? c->e->err.c_str() : "null context";
}

int ghom_set_material_neohookean(ghom_ctx* c, const uint16_t* phase, int nphase, const double* mu,
                                 const double* lambda) {
  return guard(c, [&]() -> int {
    if (!phase || !mu || !lambda || nphase < 1 || nphase > 65536) fail(GHOM_EINVAL, "bad neo-Hookean arguments");
    std::vector<double> tab(2 * (size_t)nphase);
    for (int i = 0; i < nphase; ++i) {
      tab[2 * i] = mu[i];
      tab[2 * i + 1] = lambda[i];
    }
    set_material(*c->e, 0, MAT_NH, phase, nphase, tab);
    return GHOM_OK;
  });
}

int ghom_set_material_svk(ghom_ctx* c, const uint16_t* phase, int nphase, const double* C) {
  return guard(c, [&]() -> int {
    if (!phase || !C || nphase < 1 || nphase > 65536) fail(GHOM_EINVAL, "bad Saint Venant-Kirchhoff arguments");
    set_material(*c->e, 0, MAT_SVK, phase, nphase, voigt_table(C, nphase));
    return GHOM_OK;
  });
}

int ghom_set_material_visco(ghom_ctx* c, const uint16_t* phase, int nphase, const double* Cinf, const double* C1,
                            const double* tau) {
  return guard(c, [&]() -> int {
    if (!phase || !Cinf || !C1 || !tau || nphase < 1 || nphase > 65536)
      fail(GHOM_EINVAL, "bad viscoelastic arguments");
    for (int i = 0; i < nphase; ++i)
      if (!(tau[i] > 0.0) || !std::isfinite(tau[i])) fail(GHOM_EINVAL, "relaxation times must be finite and > 0");
    Engine& e = *c->e;
    Prob& q = e.P[0];
    std::vector<double> vinf = voigt_table(Cinf, nphase), v1 = voigt_table(C1, nphase);
    const size_t N = (size_t)e.C[q.cls].g.N;
    sync(e);
    if (q.visc) HIPCALL(hipFree(q.visc));
    q.visc = nullptr;
    HIPCALL(hipMalloc((void**)&q.visc, (size_t)kViscoTable * nphase * sizeof(double)));
    if (!q.iv) HIPCALL(hipMalloc((void**)&q.iv, (size_t)kViscoIV * N * sizeof(double)));
    q.vinf = vinf;
    q.v1 = v1;
    q.vtau.assign(tau, tau + nphase);
    e.hdesc[0].visc = q.visc;
    e.hdesc[0].iv = q.iv;
    set_material(e, 0, MAT_VISCO, phase, nphase, vinf);  // also zeroes F - I and the internal variables
    visco_tables(e, 0, q.dt);
    return GHOM_OK;
  });
}

int ghom_set_time_step(ghom_ctx* c, double dt) {
  return guard(c, [&]() -> int {
    if (!(dt > 0.0) || !std::isfinite(dt)) fail(GHOM_EINVAL, "the time step must be finite and > 0");
    Engine& e = *c->e;
    e.P[0].dt = dt;
    if (e.P[0].kind == MAT_VISCO) visco_tables(e, 0, dt);
    return GHOM_OK;
  });
}

int ghom_set_stiffness_scale(ghom_ctx* c, const double* s) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    Prob& q = e.P[0];
    const long long N = e.C[q.cls].g.N;
    if (!s) {
      sync(e);
      if (q.scale) HIPCALL(hipFree(q.scale));
      q.scale = nullptr;
    } else {
      for (long long v = 0; v < N; ++v)
        if (!(s[v] > 0.0)) fail(GHOM_EINVAL, "stiffness scale must be > 0");
      if (!q.scale) HIPCALL(hipMalloc((void**)&q.scale, (size_t)N * sizeof(double)));
      sync(e);
      HIPCALL(hipMemcpy(q.scale, s, (size_t)N * sizeof(double), hipMemcpyHostToDevice));
    }
    e.hdesc[0].scale = q.scale;
    e.hdesc[0].has_scale = q.scale != nullptr;
    q.state_valid = false;
    return GHOM_OK;
  });
}

int ghom_set_control(ghom_ctx* c, const uint8_t mask[9]) {
  return guard(c, [&]() -> int {
    if (!mask) fail(GHOM_EINVAL, "null mask");
    Prob& q = c->e->P[0];
    unsigned bits = 0;
    for (int i = 0; i < 9; ++i)
      if (mask[i] > 1) fail(GHOM_EINVAL, "mask entries must be 0 or 1");
    for (int i = 0; i < 9; ++i) q.user_mask[i] = mask[i];
    q.mask_set = true;
    apply_control(*c->e, 0);
    return GHOM_OK;
  });
}

int ghom_set_history(ghom_ctx* c, int nsteps, const double* target) {
  return guard(c, [&]() -> int {
    if (nsteps < 1 || !target) fail(GHOM_EINVAL, "bad history");
    Prob& q = c->e->P[0];
    q.target.assign(target, target + 9 * (size_t)nsteps);
    q.nsteps = nsteps;
    q.adapt_fraction = 1.0;
    apply_control(*c->e, 0);
    return GHOM_OK;
  });
}

static int set_tolerances(Engine& e, double newton_tol, double cg_tol, double cg_forcing, int max_newton, int max_cg) {
  if (!(newton_tol > 0) || !(cg_tol > 0) || !(cg_forcing >= 0 && cg_forcing < 1) || max_newton < 1 || max_cg < 1)
    fail(GHOM_EINVAL, "bad tolerances");
  e.newton_tol = newton_tol;
  e.cg_tol = cg_tol;
  e.cg_forcing = cg_forcing;
  e.max_newton = max_newton;
  e.max_cg = max_cg;
  return GHOM_OK;
}

int ghom_set_tolerances(ghom_ctx* c, double newton_tol, double cg_tol, double cg_forcing, int max_newton,
                        int max_cg) {
  return guard(c, [&]() -> int { return set_tolerances(*c->e, newton_tol, cg_tol, cg_forcing, max_newton, max_cg); });
}

int ghom_step(ghom_ctx* c, ghom_step_info* info) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    Prob& q = e.P[0];
    check_material(q);
    if (q.nsteps == 0) fail(GHOM_ESTATE, "no history set");
    if (q.k >= q.nsteps) fail(GHOM_ESTATE, "history exhausted");
    if (q.kind == MAT_VISCO) visco_tables(e, 0, q.dt);
    begin_increment(e, {0});
    newton(e, {0});
    if (q.status == GHOM_OK || q.status == GHOM_ENOTCONVERGED) {
      if (q.kind == MAT_VISCO) {
        visco_checkpoint(e, 0, q.dt);
        visco_commit(e, 0);
      }
      q.k += 1;
    }
    return finish_solve(e, 0, info);
  });
}

int ghom_step_adaptive(ghom_ctx* c, int max_cuts, int grow_below, ghom_step_info* info, int* substeps,
                       int* cuts) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    Prob& q = e.P[0];
    check_material(q);
    if (q.nsteps == 0) fail(GHOM_ESTATE, "no history set");
    if (q.k >= q.nsteps) fail(GHOM_ESTATE, "history exhausted");
    if (max_cuts < 0 || max_cuts > 30 || grow_below < 0) fail(GHOM_EINVAL, "bad adaptive stepping parameters");
    const size_t bytes = 9 * (size_t)e.C[q.cls].g.N * sizeof(double);
    if (!e.ckpt) HIPCALL(hipMalloc((void**)&e.ckpt, 2 * bytes));
    double* sub0 = e.ckpt;
    double* inc0 = reinterpret_cast<double*>(reinterpret_cast<char*>(e.ckpt) + bytes);
    double* F = e.hdesc[0].F;
    HIPCALL(hipMemcpyAsync(inc0, F, bytes, hipMemcpyDeviceToDevice, e.stream));
    double from[9], to[9];
    target_row(q, q.k, from);
    target_row(q, q.k + 1, to);
    SubstepClock clk(max_cuts, grow_below, q.adapt_fraction);
    ghom_step_info tot{};
    int subs = 0;
    const auto t0 = std::chrono::steady_clock::now();
    while (!clk.done()) {
      double a[9], b[9];
      lerp9(from, to, clk.theta, a);
      lerp9(from, to, clk.next_end(), b);
      HIPCALL(hipMemcpyAsync(sub0, F, bytes, hipMemcpyDeviceToDevice, e.stream));
      if (q.kind == MAT_VISCO) visco_tables(e, 0, (clk.next_end() - clk.theta) * q.dt);
      e.hdesc[0].active = set_targets(e, 0, a, b) ? 1 : 0;
      upload_descs(e);
      if (e.hdesc[0].active) {
        ShapeClass& cl = e.C[q.cls];
        hipLaunchKernelGGL(shift_batch, dim3(cl.vb, 1, 1), dim3(kVoxThreads), 0, e.stream, e.ddesc, cl.ids);
        HIPCALL(hipGetLastError());
      }
      newton(e, {0});
      tot.newton_iters += q.info.newton_iters;
      tot.cg_iters_total += q.info.cg_iters_total;
      tot.cg_breakdowns += q.info.cg_breakdowns;
      tot.cg_stalls += q.info.cg_stalls;
      tot.t_cg_ms += q.info.t_cg_ms;
      tot.crit = q.info.crit;
      tot.res_rms = q.info.res_rms;
      if (q.status == GHOM_OK) {
        if (q.kind == MAT_VISCO) {
          visco_checkpoint(e, 0, (clk.next_end() - clk.theta) * q.dt);
          visco_commit(e, 0);
        }
        clk.accept(q.info.newton_iters);
        ++subs;
        continue;
      }
      const bool retry = (q.status == GHOM_ENOTCONVERGED || q.status == GHOM_ESINGULAR || q.status == GHOM_EDOMAIN) &&
                         clk.reject();
      if (retry) {
        HIPCALL(hipMemcpyAsync(F, sub0, bytes, hipMemcpyDeviceToDevice, e.stream));
        q.state_valid = false;
        continue;
      }
      // out of cuts: back to the start of the increment
      const int st = q.status;
      const std::string msg = q.msg;
      HIPCALL(hipMemcpyAsync(F, inc0, bytes, hipMemcpyDeviceToDevice, e.stream));
      q.state_valid = false;
      tot.status = st;
      tot.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (info) *info = tot;
      if (substeps) *substeps = subs;
      if (cuts) *cuts = clk.cuts;
      fail(st, msg + " (adaptive stepping: " + std::to_string(clk.cuts) + " cuts spent; state restored to the start "
                     "of the increment)");
    }
    q.k += 1;
    q.adapt_fraction = clk.dtheta;
    tot.status = GHOM_OK;
    tot.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = tot;
    if (substeps) *substeps = subs;
    if (cuts) *cuts = clk.cuts;
    return GHOM_OK;
  });
}

int ghom_resolve(ghom_ctx* c, ghom_step_info* info) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    check_material(e.P[0]);
    if (e.P[0].kind == MAT_VISCO)
      fail(GHOM_EINVAL, "re-solving an increment needs a path-independent law (the viscoelastic state has moved on)");
    set_pbar_current(e, 0);
    newton(e, {0});
    return finish_solve(e, 0, info);
  });
}

int ghom_get_averages(ghom_ctx* c, double Fbar[9], double Pbar[9]) {
  return guard(c, [&]() -> int {
    if (!Fbar || !Pbar) fail(GHOM_EINVAL, "null output");
    Engine& e = *c->e;
    refresh_averages(e, 0);
    for (int i = 0; i < 9; ++i) {
      Fbar[i] = e.P[0].Favg[i];
      Pbar[i] = e.P[0].Pavg[i];
    }
    return GHOM_OK;
  });
}

int ghom_get_field(ghom_ctx* c, int which, double* host_out) {
  return guard(c, [&]() -> int {
    if (!host_out) fail(GHOM_EINVAL, "null output");
    copy_field(*c->e, 0, which, host_out, hipMemcpyDeviceToHost);
    return GHOM_OK;
  });
}

int ghom_get_field_device(ghom_ctx* c, int which, double* dev_out) {
  return guard(c, [&]() -> int {
    if (!dev_out) fail(GHOM_EINVAL, "null output");
    copy_field(*c->e, 0, which, dev_out, hipMemcpyDeviceToDevice);
    return GHOM_OK;
  });
}

int ghom_save_state(ghom_ctx* c, double* F_out, int* step_out) {
  return guard(c, [&]() -> int {
    if (!F_out) fail(GHOM_EINVAL, "null output");
    Engine& e = *c->e;
    sync(e);
    HIPCALL(hipMemcpy(F_out, e.hdesc[0].F, 9 * (size_t)e.C[e.P[0].cls].g.N * sizeof(double), hipMemcpyDeviceToHost));
    if (step_out) *step_out = e.P[0].k;
    return GHOM_OK;
  });
}

int ghom_load_state(ghom_ctx* c, const double* F_in, int step) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    Prob& q = e.P[0];
    if (!F_in || step < 0 || (q.nsteps > 0 && step > q.nsteps) || (q.nsteps == 0 && step != 0))
      fail(GHOM_EINVAL, "bad state");
    if (q.kind == MAT_VISCO && step != 0)
      fail(GHOM_EINVAL, "the viscoelastic law's internal variables are not part of a saved state: only step 0 loads");
    sync(e);
    HIPCALL(hipMemcpy(e.hdesc[0].F, F_in, 9 * (size_t)e.C[q.cls].g.N * sizeof(double), hipMemcpyHostToDevice));
    if (q.kind == MAT_VISCO) {
      hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, e.stream, (long long)kViscoIV * e.C[q.cls].g.N, q.iv);
      HIPCALL(hipGetLastError());
      drop_checkpoints(e, 0);
    }
    q.k = step;
    q.state_valid = false;
    q.adapt_fraction = 1.0;
    return GHOM_OK;
  });
}

namespace {

// Gradient of J = a : <F> at the end of a viscoelastic history with respect to s(x): the
// backward sweep over the checkpointed increments.  For increment n (last to first), with
// that increment's state (F_n, the internal variables it started from, its length) restored:
// h = F_n (mE + b s C1 : mQ) (+ a/N at the last increment), lam solves A_n lam = G*(h) by CG
// with the increment's operator, then the gradient and (mE, mQ) are updated from
// L = sym(F_n^T lam) (visco_adj_update_kernel).  The state of the end of the history is
// restored afterwards: F, the committed internal variables, and P, the tangent state and
// the averages of the last increment's converged evaluation.
void visco_history_adjoint(Engine& e, const double* a, double* grad_out) {
  Prob& q = e.P[0];
  ShapeClass& cl = e.C[q.cls];
  const long long N = cl.g.N;
  if (q.ckpt.empty() || q.ckpt_k0 != 0)
    fail(GHOM_ESTATE, "the adjoint of a viscoelastic history needs checkpoints (GHOM_OPT_CHECKPOINTS) from increment 0");
  const size_t M = q.ckpt.size();
  refresh_averages(e, 0);
  double Fa[9], Pa[9];
  std::copy(q.Favg, q.Favg + 9, Fa);
  std::copy(q.Pavg, q.Pavg + 9, Pa);
  sync(e);
  double* buf = nullptr;
  const size_t nd = (size_t)(9 + kViscoIV + 1 + 9 + kViscoIV) * N + 16;
  HIPCALL(hipMalloc((void**)&buf, nd * sizeof(double)));
  double* h = buf;
  double* mu = h + 9 * N;
  double* gd = mu + kViscoIV * N;
  double* Fkeep = gd + N;
  double* ivkeep = Fkeep + 9 * N;
  double* abar = ivkeep + kViscoIV * N;
  double* F = e.hdesc[0].F;
  const size_t fb = 9 * (size_t)N * sizeof(double), ib = kViscoIV * (size_t)N * sizeof(double);
  bool restored = false;
  auto restore = [&]() {
    if (restored) return;
    restored = true;
    (void)hipMemcpyAsync(F, Fkeep, fb, hipMemcpyDeviceToDevice, e.stream);
    (void)hipMemcpyAsync(q.iv, ivkeep, ib, hipMemcpyDeviceToDevice, e.stream);
    (void)hipStreamSynchronize(e.stream);
    (void)hipFree(buf);
    e.hdesc[0].in = nullptr;
    q.state_valid = false;
  };
  try {
    HIPCALL(hipMemcpyAsync(Fkeep, F, fb, hipMemcpyDeviceToDevice, e.stream));
    HIPCALL(hipMemcpyAsync(ivkeep, q.iv, ib, hipMemcpyDeviceToDevice, e.stream));
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, e.stream, (long long)(kViscoIV + 1) * N, mu);
    HIPCALL(hipGetLastError());
    double ab[9];
    for (int i = 0; i < 9; ++i) ab[i] = a[i] / (double)N;
    HIPCALL(hipMemcpyAsync(abar, ab, sizeof(ab), hipMemcpyHostToDevice, e.stream));
    const dim3 vg(cl.vb), vt(kVoxThreads);
    const double* scale = e.hdesc[0].has_scale ? e.hdesc[0].scale : nullptr;
    for (size_t n = M; n >= 1; --n) {
      double* ck = q.ckpt[n - 1];
      HIPCALL(hipMemcpyAsync(F, ck, fb, hipMemcpyDeviceToDevice, e.stream));
      HIPCALL(hipMemcpyAsync(q.iv, ck + 9 * N, ib, hipMemcpyDeviceToDevice, e.stream));
      visco_tables(e, 0, q.ckpt_dt[n - 1]);
      refresh_averages(e, 0);  // P and the tangent state of increment n
      hipLaunchKernelGGL(visco_adj_rhs_kernel, vg, vt, 0, e.stream, N, F, e.hdesc[0].phase, scale, q.visc, mu, h,
                         n == M ? abar : nullptr);
      HIPCALL(hipGetLastError());
      e.hdesc[0].in = h;
      e.hdesc[0].active = 1;
      upload_descs(e);
      const int gi = project64(e, cl, ROLE_ADJ, "adj");
      launch_sum_columns(e, cl.ids, 1, gi, 1, 0, 0, 20, 0);
      HIPCALL(hipGetLastError());
      sync(e);
      const double rr = e.host_red[20];
      const double tol = std::max(e.cg_tol, forcing(e) * std::sqrt(rr / (double)N));
      e.hdesc[0].cg_thresh = tol * tol * (double)N;
      e.hdesc[0].rr0 = rr;
      e.hdesc[0].max_cg = e.max_cg;
      upload_descs(e);
      double tcg = 0.0;
      if (e.prec == GHOM_FP64) cg_solve<double>(e, &tcg);
      else cg_solve<float>(e, &tcg);
      const CGScalars st = e.host_sc[0];
      if (st.status == CG_BREAKDOWN && st.it == 0) fail(GHOM_ESINGULAR, "adjoint CG breakdown at its first iteration");
      if (st.status == CG_CAP) fail(GHOM_ENOTCONVERGED, "adjoint CG reached max_cg");
      if (st.status == CG_STALLED) fail(GHOM_ENOTCONVERGED, "adjoint CG stalled above its threshold");
      const double* lam = reinterpret_cast<const double*>(e.hdesc[0].x);
      if (e.prec == GHOM_FP32_SPLIT) {
        project64(e, cl, ROLE_REPROJ, "reproj");
        lam = e.hdesc[0].dF64;
      }
      hipLaunchKernelGGL(visco_adj_update_kernel, vg, vt, 0, e.stream, N, F, q.iv, e.hdesc[0].phase, scale, q.visc,
                         lam, mu, gd);
      HIPCALL(hipGetLastError());
    }
    sync(e);
    HIPCALL(hipMemcpy(grad_out, gd, (size_t)N * sizeof(double), hipMemcpyDeviceToHost));
    // the last increment's converged evaluation (its starting internal variables and length),
    // then the committed internal variables
    HIPCALL(hipMemcpyAsync(F, Fkeep, fb, hipMemcpyDeviceToDevice, e.stream));
    HIPCALL(hipMemcpyAsync(q.iv, q.ckpt[M - 1] + 9 * N, ib, hipMemcpyDeviceToDevice, e.stream));
    visco_tables(e, 0, q.ckpt_dt[M - 1]);
    refresh_averages(e, 0);
  } catch (...) {
    restore();
    visco_tables(e, 0, q.dt);
    throw;
  }
  restore();
  q.state_valid = true;
  std::copy(Fa, Fa + 9, q.Favg);
  std::copy(Pa, Pa + 9, q.Pavg);
}

}  // namespace

int ghom_adjoint_grad_scale(ghom_ctx* c, const double a[9], double* grad_out) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    Prob& q = e.P[0];
    check_material(q);
    if (!a || !grad_out) fail(GHOM_EINVAL, "null argument");
    if (q.kind == MAT_VISCO) {
      visco_history_adjoint(e, a, grad_out);
      return GHOM_OK;
    }
    const long long N = e.C[q.cls].g.N;
    // right-hand side G*(a) of a uniform a: only xi = 0 content, kept on the
    // stress-controlled components (the 1/N of G*(a/N) is applied to the solution)
    double rr = 0.0;
    for (int i = 0; i < 9; ++i) {
      e.hdesc[0].fill[i] = q.mask[i] ? a[i] : 0.0;
      rr += e.hdesc[0].fill[i] * e.hdesc[0].fill[i];
    }
    if (rr == 0.0) {
      std::fill(grad_out, grad_out + N, 0.0);
      return GHOM_OK;
    }
    q.state_valid = false;
    refresh_averages(e, 0);
    ShapeClass& cl = e.C[q.cls];
    e.hdesc[0].active = 1;
    const double tol = std::max(e.cg_tol, forcing(e) * std::sqrt(rr));
    e.hdesc[0].cg_thresh = tol * tol * (double)N;
    e.hdesc[0].rr0 = rr * (double)N;
    e.hdesc[0].max_cg = e.max_cg;
    upload_descs(e);
    hipLaunchKernelGGL(fill9_batch, dim3(cl.vb, 1, 1), dim3(kVoxThreads), 0, e.stream, e.ddesc, cl.ids, 1);
    HIPCALL(hipGetLastError());
    double tcg = 0.0;
    if (e.prec == GHOM_FP64) cg_solve<double>(e, &tcg);
    else cg_solve<float>(e, &tcg);
    const CGScalars s = e.host_sc[0];
    if (s.status == CG_BREAKDOWN && s.it == 0) fail(GHOM_ESINGULAR, "adjoint CG breakdown at its first iteration");
    if (s.status == CG_CAP) fail(GHOM_ENOTCONVERGED, "adjoint CG reached max_cg");
    if (s.status == CG_STALLED) fail(GHOM_ENOTCONVERGED, "adjoint CG stalled above its threshold");
    if (e.prec == GHOM_FP32_SPLIT) project64(e, cl, ROLE_REPROJ, "reproj");
    double* grad_dev = nullptr;
    HIPCALL(hipMalloc((void**)&grad_dev, (size_t)N * sizeof(double)));
    e.hdesc[0].out = grad_dev;
    const hipError_t ue = hipMemcpyAsync(e.ddesc, e.hdesc, sizeof(ProbDesc), hipMemcpyHostToDevice, e.stream);
    e.desc_sent.clear();  // the device copy differs from the last upload's
    if (ue == hipSuccess)
      hipLaunchKernelGGL(adjoint_grad_batch, dim3(cl.vb, 1, 1), dim3(kVoxThreads), 0, e.stream, e.ddesc, cl.ids);
    const hipError_t le = hipGetLastError();
    const hipError_t se = hipStreamSynchronize(e.stream);
    const hipError_t ce = hipMemcpy(grad_out, grad_dev, (size_t)N * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(grad_dev);
    e.hdesc[0].out = nullptr;
    HIPCALL(ue);
    HIPCALL(le);
    HIPCALL(se);
    HIPCALL(ce);
    return GHOM_OK;
  });
}

int ghom_apply_operator(ghom_ctx* c, const void* v_dev, void* Av_dev) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    check_material(e.P[0]);
    if (!v_dev || !Av_dev || v_dev == Av_dev) fail(GHOM_EINVAL, "bad operator buffers");
    refresh_averages(e, 0);
    e.hdesc[0].in = v_dev;
    e.hdesc[0].out = Av_dev;
    e.hdesc[0].active = 1;
    upload_descs(e);
    ShapeClass& cl = e.C[e.P[0].cls];
    if (e.prec == GHOM_FP64) operator_apply<double>(e, cl, ROLE_OP_PLAIN, 0);
    else operator_apply<float>(e, cl, ROLE_OP_PLAIN, 0);
    sync(e);
    e.hdesc[0].in = nullptr;
    e.hdesc[0].out = nullptr;
    return GHOM_OK;
  });
}

int ghom_apply_projection(ghom_ctx* c, const double* in_dev, double* out_dev) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    if (!e.P[0].mask_set) fail(GHOM_ESTATE, "no control mask set");
    if (!in_dev || !out_dev) fail(GHOM_EINVAL, "null buffer");
    e.hdesc[0].in = in_dev;
    e.hdesc[0].out = out_dev;
    e.hdesc[0].active = 1;
    upload_descs(e);
    project64(e, e.C[e.P[0].cls], ROLE_PROJ, "proj");
    sync(e);
    e.hdesc[0].in = nullptr;
    e.hdesc[0].out = nullptr;
    return GHOM_OK;
  });
}

int ghom_residual(ghom_ctx* c, const double Pbar[9], double* out_dev) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    Prob& q = e.P[0];
    check_material(q);
    if (!Pbar || !out_dev) fail(GHOM_EINVAL, "null argument");
    q.state_valid = false;
    refresh_averages(e, 0);
    double* b_keep = e.hdesc[0].b;
    for (int i = 0; i < 9; ++i) e.hdesc[0].pbar[i] = q.mask[i] ? Pbar[i] : 0.0;
    e.hdesc[0].b = out_dev;
    e.hdesc[0].active = 1;
    upload_descs(e);
    project64(e, e.C[q.cls], ROLE_RESID, "res");
    sync(e);
    e.hdesc[0].b = b_keep;
    upload_descs(e);
    return GHOM_OK;
  });
}

// captured graphs hold the kernel variants and slab count they were made with
static void drop_graphs(Engine& e) {
  if (!e.graph_cache.empty()) sync(e);
  for (auto& kv : e.graph_cache) (void)hipGraphExecDestroy(kv.second);
  e.graph_cache.clear();
}

static int set_option(Engine& e, int key, int value) {
  if (key == GHOM_OPT_XPROJ_F64 || key == GHOM_OPT_XPROJ_F32) {
    if (value < XPROJ_TUNED || value > XPROJ_ROWS3) fail(GHOM_EINVAL, "x-pass variant must be 0, 1, 2, 3 or 4");
    if (value == XPROJ_ROWS3)
      for (auto& cl : e.C)
        if (!has_split3(cl.nx)) fail(GHOM_EINVAL, "x-pass variant 4 needs x lengths 128, 256 or 512");
    for (auto& cl : e.C) {
      const int i = key == GHOM_OPT_XPROJ_F64 ? 0 : 1;
      cl.xproj_var[i] = value;
      cl.tuned_x[i] = false;
      if (value == XPROJ_TUNED) tune_class(e, cl, i, false);
    }
    drop_graphs(e);
    return GHOM_OK;
  }
  if (key == GHOM_OPT_YPASS_F64 || key == GHOM_OPT_YPASS_F32) {
    if (value < YPASS_TUNED || value > YPASS_THREE) fail(GHOM_EINVAL, "y-pass variant must be 0, 1, 2 or 3");
    const bool f64 = key == GHOM_OPT_YPASS_F64;
    for (auto& cl : e.C)
      if (value != YPASS_TUNED && !(f64 ? ypass_has<double>(value, cl.ny) : ypass_has<float>(value, cl.ny)))
        fail(GHOM_EINVAL, "this y-pass variant does not exist for the grid's y length");
    for (auto& cl : e.C) {
      const int i = f64 ? 0 : 1;
      cl.ypass_var[i] = value;
      cl.tuned_y[i] = false;
      if (value == YPASS_TUNED) tune_class(e, cl, i, false);
    }
    drop_graphs(e);
    return GHOM_OK;
  }
  if (key == GHOM_OPT_ZSLABS) {
    if (value < 1 || value > 4096) fail(GHOM_EINVAL, "slab count must be in [1, 4096]");
    e.zslabs = value;
    drop_graphs(e);
    return GHOM_OK;
  }
  if (key == GHOM_OPT_CHECKPOINTS) {
    if (value != 0 && value != 1) fail(GHOM_EINVAL, "checkpoint option must be 0 or 1");
    e.checkpoints = value != 0;
    if (!e.checkpoints)
      for (size_t p = 0; p < e.P.size(); ++p) drop_checkpoints(e, (int)p);
    return GHOM_OK;
  }
  if (key == GHOM_OPT_GRAPHS) {
    if (value != 0 && value != 1) fail(GHOM_EINVAL, "graph option must be 0 or 1");
    e.graphs = value != 0;
    drop_graphs(e);
    return GHOM_OK;
  }
  if (key == GHOM_OPT_STREAM_NT) {
    if (value != 0 && value != 1) fail(GHOM_EINVAL, "streaming option must be 0 or 1");
    e.stream_nt = value != 0;
    drop_graphs(e);
    return GHOM_OK;
  }
  if (key == GHOM_OPT_PROFILE_EVERY) {
    if (value < 1 || value > 1000000) fail(GHOM_EINVAL, "profiling stride must be in [1, 1000000]");
    e.prof_every = value;
    e.prof_seen.clear();
    return GHOM_OK;
  }
  if (key == GHOM_OPT_ROTATION_GAUGE) {
    if (value != 0 && value != 1) fail(GHOM_EINVAL, "rotation gauge option must be 0 or 1");
    e.rot_gauge = value != 0;
    for (size_t p = 0; p < e.P.size(); ++p) apply_control(e, (int)p);
    upload_descs(e);
    return GHOM_OK;
  }
  fail(GHOM_EINVAL, "unknown option");
}

static int get_option(Engine& e, int key, int* value) {
  if (!value) fail(GHOM_EINVAL, "null output");
  if (key == GHOM_OPT_XPROJ_F64) *value = e.C[0].xproj_var[0];
  else if (key == GHOM_OPT_XPROJ_F32) *value = e.C[0].xproj_var[1];
  else if (key == GHOM_OPT_ZSLABS) *value = e.zslabs;
  else if (key == GHOM_OPT_GRAPHS) *value = e.graphs ? 1 : 0;
  else if (key == GHOM_OPT_CHECKPOINTS) *value = e.checkpoints ? 1 : 0;
  else if (key == GHOM_OPT_STREAM_NT) *value = e.stream_nt ? 1 : 0;
  else if (key == GHOM_OPT_ROTATION_GAUGE) *value = e.rot_gauge ? 1 : 0;
  else if (key == GHOM_OPT_YPASS_F64) *value = e.C[0].ypass_var[0];
  else if (key == GHOM_OPT_YPASS_F32) *value = e.C[0].ypass_var[1];
  else if (key == GHOM_OPT_PROFILE_EVERY) *value = e.prof_every;
  else fail(GHOM_EINVAL, "unknown option");
  return GHOM_OK;
}

}  // extern "C"

namespace {
// "AxB" of a two-stage split or "BxA1xA2" of a three-stage one
std::string split_text(int n, bool three) {
  char buf[32] = "?";
  if (three) with_split3(n, [&](auto s) { std::snprintf(buf, sizeof buf, "%dx%dx%d", decltype(s)::B, decltype(s)::A1, decltype(s)::A2); });
  else with_split(n, [&](auto s) { std::snprintf(buf, sizeof buf, "%dx%d", decltype(s)::A, decltype(s)::B); });
  return buf;
}

// the schedule class c runs: per precision in use, the x-pass and y-pass variants with their
// radix splits and whether the autotuner picked them
std::string schedule_text(const Engine& e, const ShapeClass& c) {
  static const char* xn[] = {"untuned", "rows", "groups", "rows-capped", "rows3"};
  static const char* yn[] = {"untuned", "wide", "narrow", "three-stage"};
  std::string out = std::to_string(c.nx) + "x" + std::to_string(c.ny) + "x" + std::to_string(c.nz) + " (" +
                    std::to_string(c.probs.size()) + " problem" + (c.probs.size() > 1 ? "s" : "") + ")";
  for (int i = 0; i < 2; ++i) {
    if (i == 1 && e.prec != GHOM_FP32_SPLIT) break;
    const int xv = c.xproj_var[i] == XPROJ_TUNED ? XPROJ_ROWS : c.xproj_var[i];
    const int yv = c.ypass_var[i] == YPASS_TUNED ? YPASS_WIDE : c.ypass_var[i];
    out += std::string(i == 0 ? "; f64" : "; f32") + ": x " + xn[xv] + " " + split_text(c.nx, xv == XPROJ_ROWS3) +
           (c.tuned_x[i] ? " (tuned)" : " (set)") + ", y " + yn[yv] + " " + split_text(c.ny, yv == YPASS_THREE) +
           (c.tuned_y[i] ? " (tuned)" : " (set)");
  }
  return out;
}

int copy_text(const std::string& t, char* out, int cap) {
  if (out && cap > 0) {
    std::strncpy(out, t.c_str(), (size_t)cap - 1);
    out[cap - 1] = 0;
  }
  return (int)t.size();
}
}  // namespace

extern "C" {

int ghom_get_schedule(ghom_ctx* c, char* out, int cap) {
  if (!c || !c->e || cap < 0) return GHOM_EINVAL;
  return copy_text(schedule_text(*c->e, c->e->C[0]), out, cap);
}

int ghom_get_control(ghom_ctx* c, uint8_t mask_out[9], int* gauge_axis) {
  return guard(c, [&]() -> int {
    const Prob& q = c->e->P[0];
    if (!q.mask_set) fail(GHOM_ESTATE, "no control mask set");
    if (mask_out)
      for (int i = 0; i < 9; ++i) mask_out[i] = q.mask[i];
    if (gauge_axis) *gauge_axis = q.gauge_axis;
    return GHOM_OK;
  });
}

int ghom_set_option(ghom_ctx* c, int key, int value) {
  return guard(c, [&]() -> int { return set_option(*c->e, key, value); });
}

int ghom_get_option(ghom_ctx* c, int key, int* value) {
  return guard(c, [&]() -> int { return get_option(*c->e, key, value); });
}

int ghom_set_profiling(ghom_ctx* c, int on) {
  return guard(c, [&]() -> int {
    c->e->prof = on != 0;
    return GHOM_OK;
  });
}

int ghom_set_profiling_filter(ghom_ctx* c, const char* name) {
  return guard(c, [&]() -> int {
    c->e->prof_only = name ? std::string(name) : std::string();
    return GHOM_OK;
  });
}

int ghom_profile_count(ghom_ctx* c) {
  if (!c || !c->e) return GHOM_EINVAL;
  return (int)c->e->prof_recs.size();
}

int ghom_profile_get(ghom_ctx* c, int i, char* name_out, int name_cap, int* launches, double* total_ms) {
  return guard(c, [&]() -> int {
    Engine& e = *c->e;
    if (i < 0 || i >= (int)e.prof_recs.size()) fail(GHOM_EINVAL, "record index out of range");
    prof_collect(e);
    auto it = e.prof_recs.begin();
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

int ghom_profile_samples(ghom_ctx* c, int i, float* ms_out, int cap) {
  if (!c || !c->e) return GHOM_EINVAL;
  int n = 0;
  const int rc = guard(c, [&]() -> int {
    Engine& e = *c->e;
    if (i < 0 || i >= (int)e.prof_recs.size() || cap < 0 || (cap > 0 && !ms_out))
      fail(GHOM_EINVAL, "bad record index or output");
    prof_collect(e);
    auto it = e.prof_recs.begin();
    std::advance(it, i);
    const std::vector<float>& v = it->second.samples;
    n = (int)v.size();
    std::copy(v.begin(), v.begin() + std::min(n, cap), ms_out);
    return GHOM_OK;
  });
  return rc == GHOM_OK ? n : rc;
}

int ghom_profile_reset(ghom_ctx* c) {
  return guard(c, [&]() -> int {
    prof_collect(*c->e);
    c->e->prof_recs.clear();
    c->e->prof_seen.clear();
    return GHOM_OK;
  });
}

// =====================================================================================
// Batch of independent problems
// =====================================================================================
int ghom_batch_create(ghom_batch** out, const ghom_problem* probs, int nprob, int precision, int device,
                      void* hip_stream) {
  g_create_err.clear();
  if (!out) return create_fail(GHOM_EINVAL, "null output");
  *out = nullptr;
  if (!probs || nprob < 1 || nprob > 65535) return create_fail(GHOM_EINVAL, "need 1..65535 problems");
  if (precision != GHOM_FP64 && precision != GHOM_FP32_SPLIT) return create_fail(GHOM_EINVAL, "unknown precision");
  for (int i = 0; i < nprob; ++i) {
    const ghom_problem& p = probs[i];
    const std::string at = " (problem " + std::to_string(i) + ")";
    if (!supported_length(p.nx) || !supported_length(p.ny) || !supported_length(p.nz))
      return create_fail(GHOM_EINVAL, std::string("grid lengths must be among ") + kLengths + at);
    if (!p.phase || p.nphase < 1 || p.nphase > 65536 || p.nsteps < 1 || !p.target)
      return create_fail(GHOM_EINVAL, "bad phase map, phase count or history" + at);
    if (p.kind == GHOM_MATERIAL_NEOHOOKEAN) {
      if (!p.mu || !p.lambda) return create_fail(GHOM_EINVAL, "missing neo-Hookean moduli" + at);
    } else if (p.kind == GHOM_MATERIAL_SVK) {
      if (!p.C) return create_fail(GHOM_EINVAL, "missing stiffness tensors" + at);
    } else {
      return create_fail(GHOM_EINVAL, "unknown material kind" + at);
    }
    for (int c = 0; c < 9; ++c)
      if (p.mask[c] > 1) return create_fail(GHOM_EINVAL, "mask entries must be 0 or 1" + at);
  }
  Engine* e = new_engine(precision, device, hip_stream);
  if (!e) return create_fail(GHOM_ENOMEM, "host allocation failed");
  const int rc = guarded(e, [&]() -> int {
    open_stream(*e, hip_stream);
    std::vector<ProbSpec> specs(nprob);
    std::vector<int> kinds(nprob);
    for (int i = 0; i < nprob; ++i) {
      specs[i] = ProbSpec{probs[i].nx, probs[i].ny, probs[i].nz, {1.0, 1.0, 1.0}};
      kinds[i] = probs[i].kind == GHOM_MATERIAL_NEOHOOKEAN ? MAT_NH : MAT_SVK;
    }
    build_engine(*e, specs, kinds);
    for (int i = 0; i < nprob; ++i) {
      const ghom_problem& p = probs[i];
      std::vector<double> tab;
      if (kinds[i] == MAT_NH) {
        tab.resize(2 * (size_t)p.nphase);
        for (int k = 0; k < p.nphase; ++k) {
          tab[2 * k] = p.mu[k];
          tab[2 * k + 1] = p.lambda[k];
        }
      } else {
        tab = voigt_table(p.C, p.nphase);
      }
      set_material(*e, i, kinds[i], p.phase, p.nphase, tab);
      Prob& q = e->P[i];
      for (int c = 0; c < 9; ++c) q.user_mask[c] = p.mask[c];
      q.mask_set = true;
      q.target.assign(p.target, p.target + 9 * (size_t)p.nsteps);
      q.nsteps = p.nsteps;
      apply_control(*e, i);
    }
    upload_descs(*e);
    return GHOM_OK;
  });
  ghom_batch* b = rc == GHOM_OK ? new (std::nothrow) ghom_batch() : nullptr;
  if (!b) {
    g_create_err = rc != GHOM_OK ? e->err : std::string("host allocation failed");
    destroy_engine(e);
    return rc != GHOM_OK ? rc : GHOM_ENOMEM;
  }
  b->e = e;
  *out = b;
  return GHOM_OK;
}

void ghom_batch_destroy(ghom_batch* b) {
  if (!b) return;
  destroy_engine(b->e);
  delete b;
}

const char* ghom_batch_last_error(const ghom_batch* b) {
  if (!b) return g_create_err.empty() ? "null batch" : g_create_err.c_str();
  return b->e ? b->e->err.c_str() : "null batch";
}

int ghom_batch_set_tolerances(ghom_batch* b, double newton_tol, double cg_tol, double cg_forcing, int max_newton,
                              int max_cg) {
  return guard(b, [&]() -> int { return set_tolerances(*b->e, newton_tol, cg_tol, cg_forcing, max_newton, max_cg); });
}

int ghom_batch_step(ghom_batch* b, ghom_step_info* info) {
  return guard(b, [&]() -> int {
    Engine& e = *b->e;
    std::vector<int> set;
    for (size_t p = 0; p < e.P.size(); ++p)
      if (e.P[p].k < e.P[p].nsteps) set.push_back((int)p);
    if (set.empty()) fail(GHOM_ESTATE, "every history is exhausted");
    begin_increment(e, set);
    newton(e, set);
    int rc = GHOM_OK;
    std::vector<char> in(e.P.size(), 0);
    for (int p : set) in[p] = 1;
    for (size_t p = 0; p < e.P.size(); ++p) {
      Prob& q = e.P[p];
      if (in[p] && (q.status == GHOM_OK || q.status == GHOM_ENOTCONVERGED)) q.k += 1;
      if (info) {
        info[p] = in[p] ? q.info : ghom_step_info{};
        if (!in[p]) info[p].status = GHOM_ESTATE;
      }
      if (in[p] && q.status != GHOM_OK && rc == GHOM_OK) {
        rc = q.status;
        e.err = "problem " + std::to_string(p) + ": " + q.msg;
      }
    }
    return rc;
  });
}

int ghom_batch_get_averages(ghom_batch* b, int iprob, double Fbar[9], double Pbar[9]) {
  return guard(b, [&]() -> int {
    Engine& e = *b->e;
    if (iprob < 0 || iprob >= (int)e.P.size() || !Fbar || !Pbar) fail(GHOM_EINVAL, "bad problem index or output");
    refresh_averages(e, iprob);
    for (int i = 0; i < 9; ++i) {
      Fbar[i] = e.P[iprob].Favg[i];
      Pbar[i] = e.P[iprob].Pavg[i];
    }
    return GHOM_OK;
  });
}

int ghom_batch_get_field(ghom_batch* b, int iprob, int which, double* host_out) {
  return guard(b, [&]() -> int {
    Engine& e = *b->e;
    if (iprob < 0 || iprob >= (int)e.P.size() || !host_out) fail(GHOM_EINVAL, "bad problem index or output");
    copy_field(e, iprob, which, host_out, hipMemcpyDeviceToHost);
    return GHOM_OK;
  });
}

int ghom_batch_set_option(ghom_batch* b, int key, int value) {
  return guard(b, [&]() -> int { return set_option(*b->e, key, value); });
}

int ghom_batch_num_classes(ghom_batch* b) {
  if (!b || !b->e) return GHOM_EINVAL;
  return (int)b->e->C.size();
}

int ghom_batch_get_schedule(ghom_batch* b, int cls, char* out, int cap) {
  if (!b || !b->e || cls < 0 || cls >= (int)b->e->C.size() || cap < 0) return GHOM_EINVAL;
  return copy_text(schedule_text(*b->e, b->e->C[cls]), out, cap);
}

}  // extern "C"

// =====================================================================================
// G* without a context and without device allocation
// =====================================================================================
namespace {

// Capacity of the static scratch array on each device: the half spectrum of a 64^3 grid
// (9 x 64 x 64 x 32 complex doubles, 18 MiB) with the descriptor and twiddle tables.
constexpr size_t kScratchBytes = (size_t)24 << 20;

}  // namespace

// Device memory of ghom_apply_projection_static, one copy per GPU, held until the process
// ends.  Host code never passes this name to a kernel or a copy (on the host it is a
// stand-in, not a device address): it uses the address scratch_address() looked up.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxScratchDevices] = {};

// This device's address of `scratch`, looked up once per device with the device current.
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    HIPCALL(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw HipFail{hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)"};
    g_scratch_dev[device] = ptr;
  }
  return g_scratch_dev[device];
}

// Byte offsets in the scratch for one grid: descriptor, problem id, three twiddle tables,
// spectrum (9 x nx ny nzh complex doubles).
struct ScratchLayout {
  size_t desc, ids, tw[3], spec, total;
};

ScratchLayout scratch_layout(int nx, int ny, int nz) {
  ScratchLayout L{};
  size_t at = 0;
  L.desc = at;
  at += align256(sizeof(ProbDesc));
  L.ids = at;
  at += align256(sizeof(int));
  const int ns[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a) {
    L.tw[a] = at;
    at += align256((size_t)ns[a] * sizeof(cx<double>));
  }
  const size_t nzh = (nz % 2 == 0) ? nz / 2 : (nz + 1) / 2;
  L.spec = at;
  at += align256(9 * (size_t)nx * ny * nzh * sizeof(cx<double>));
  L.total = at;
  return L;
}

int static_fail(int code, const std::string& msg) {
  g_create_err = msg;
  return code;
}

}  // namespace

extern "C" int ghom_apply_projection_static(int nx, int ny, int nz, double Lx, double Ly, double Lz,
                                            const uint8_t mask[9], const double* in_dev, double* out_dev,
                                            int device, void* hip_stream) {
  g_create_err.clear();
  if (!supported_length(nx) || !supported_length(ny) || !supported_length(nz))
    return static_fail(GHOM_EINVAL, std::string("grid lengths must be among ") + kLengths);
  if (!(Lx > 0 && Ly > 0 && Lz > 0)) return static_fail(GHOM_EINVAL, "cell lengths must be > 0");
  if (!mask || !in_dev || !out_dev) return static_fail(GHOM_EINVAL, "null mask or buffer");
  unsigned bits = 0;
  for (int c = 0; c < 9; ++c) {
    if (mask[c] > 1) return static_fail(GHOM_EINVAL, "mask entries must be 0 or 1");
    if (mask[c]) bits |= 1u << c;
  }
  const ScratchLayout L = scratch_layout(nx, ny, nz);
  if (L.total > kScratchBytes)
    return static_fail(GHOM_EINVAL, "grid needs " + std::to_string(L.total) + " bytes of scratch; the static scratch holds " +
                                        std::to_string(kScratchBytes) + " (24 MiB: up to 64^3 voxels)");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev || device >= kMaxScratchDevices)
    return static_fail(GHOM_EINVAL, "no such device");
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  int rc = GHOM_OK;
  try {
    HIPCALL(hipSetDevice(device));
    char* base = static_cast<char*>(scratch_address(device));
    // a host-side engine of one problem whose device memory is all in the scratch
    Engine e;
    e.device = device;
    e.stream = static_cast<hipStream_t>(hip_stream);
    e.prec = GHOM_FP64;
    e.tsz = 8;
    e.P.resize(1);
    ShapeClass c;
    c.nx = nx;
    c.ny = ny;
    c.nz = nz;
    c.g.nx = nx;
    c.g.ny = ny;
    c.g.nz = nz;
    c.g.nzh = (nz % 2 == 0) ? nz / 2 : (nz + 1) / 2;
    c.g.N = (long long)nx * ny * nz;
    c.g.Nh = (long long)nx * ny * c.g.nzh;
    c.g.invL[0] = 1.0 / Lx;
    c.g.invL[1] = 1.0 / Ly;
    c.g.invL[2] = 1.0 / Lz;
    c.probs = {0};
    c.ids = reinterpret_cast<int*>(base + L.ids);
    c.xproj_var[0] = XPROJ_ROWS;
    ProbDesc hd;
    std::memset(&hd, 0, sizeof(ProbDesc));
    hd.g = c.g;
    hd.mask = bits;
    hd.active = 1;
    hd.H = base + L.spec;
    hd.in = in_dev;
    hd.out = out_dev;
    // twiddles W_n^k = exp(-2 pi i k / n), as the contexts build them
    const int ns[3] = {nx, ny, nz};
    std::vector<cx<double>> tw[3];
    for (int a = 0; a < 3; ++a) {
      tw[a].resize(ns[a]);
      for (int k = 0; k < ns[a]; ++k) {
        const CosSin cs = cossin_2pi(k, ns[a]);
        tw[a][k] = cx<double>{(double)cs.c, (double)-cs.s};
      }
      c.tw64[a] = reinterpret_cast<cx<double>*>(base + L.tw[a]);
      hd.tw64[a] = c.tw64[a];
      HIPCALL(hipMemcpyAsync(c.tw64[a], tw[a].data(), ns[a] * sizeof(cx<double>), hipMemcpyHostToDevice, e.stream));
    }
    const int id0 = 0;
    HIPCALL(hipMemcpyAsync(c.ids, &id0, sizeof(int), hipMemcpyHostToDevice, e.stream));
    e.hdesc = &hd;
    e.ddesc = reinterpret_cast<ProbDesc*>(base + L.desc);
    upload_descs(e);  // waits for the stream: the host tables above are copied
    project64(e, c, ROLE_PROJ, "proj");
    HIPCALL(hipStreamSynchronize(e.stream));
  } catch (const HipFail& f) {
    rc = static_fail(GHOM_EHIP, std::string(f.what) + ": " + hipGetErrorString(f.e));
  } catch (const ApiError& a) {
    rc = static_fail(a.code, a.msg);
  } catch (const std::exception& x) {
    rc = static_fail(GHOM_EHIP, x.what());
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  return rc;
}
