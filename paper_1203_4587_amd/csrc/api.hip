// C ABI entry points of libcsmri (declared in include/csmri.h).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>

#include "internal.hpp"

namespace csmri {

static thread_local std::string g_last_error;

int set_error(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return set_error(CS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void* DeviceAlloc::get(size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (custom) return a.alloc(bytes, a.ctx);
  void* ptr = nullptr;
  if (hipMalloc(&ptr, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return ptr;
}

void DeviceAlloc::put(void* ptr) {
  if (!ptr) return;
  if (custom) {
    if (a.free) a.free(ptr, a.ctx);
  } else {
    (void)hipFree(ptr);
  }
}

int ensure_dynamic_lds(const void* kernel, size_t bytes) {
  if (bytes <= 65536) return CS_OK;
  int dev = 0;
  CS_HIP(hipGetDevice(&dev));
  static std::mutex mutex;
  static std::map<std::pair<const void*, int>, size_t> enabled;
  std::lock_guard<std::mutex> lock(mutex);
  size_t& have = enabled[{kernel, dev}];
  if (have >= bytes) return CS_OK;
  CS_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  have = bytes;
  return CS_OK;
}

int objective_partial_count();

static bool smooth_23(int n) {
  if (n < 2) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

template <typename T>
static int plan_alloc(cs_plan* p, T** out, size_t count, const char* what) {
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  void* ptr = p->alloc.get(bytes);
  if (!ptr) return set_error(CS_ENOMEM, std::string("allocator returned NULL for ") + what);
  p->owned.push_back(ptr);
  p->bytes += bytes;
  *out = static_cast<T*>(ptr);
  return CS_OK;
}

static void plan_release(cs_plan* p) {
  if (!p) return;
  if (p->jhost) (void)hipHostFree(p->jhost);
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  for (void* ptr : p->owned) p->alloc.put(ptr);
  p->owned.clear();
  delete p;
}

static constexpr uint32_t kAllFlags = CS_FLAG_NO_REFACTOR | CS_FLAG_GRAPH | CS_FLAG_COLUMN_RESIDENT |
                                      CS_FLAG_XU_WAVE | CS_FLAG_XU_GROUP | CS_FLAG_EIGEN | CS_FLAG_CHECK_FINITE;

static int validate_flags(uint32_t f) {
  if (f & ~kAllFlags) return set_error(CS_EINVAL, "unknown flag bits");
  if ((f & CS_FLAG_XU_WAVE) && (f & CS_FLAG_XU_GROUP))
    return set_error(CS_EINVAL, "CS_FLAG_XU_WAVE and CS_FLAG_XU_GROUP are exclusive");
  return CS_OK;
}

static int validate_desc(const cs_plan_desc* d) {
  if (d->nv < 2 || d->nh < 2 || d->nt < 1 || d->nc < 1)
    return set_error(CS_EINVAL, "nv, nh must be >= 2 and nt, nc >= 1");
  if (d->prior != CS_PRIOR_TEMPORAL_TV && d->prior != CS_PRIOR_TEMPORAL_DFT && d->prior != CS_PRIOR_TEMPORAL_FRAME)
    return set_error(CS_EINVAL, "unknown prior");
  if (d->prior == CS_PRIOR_TEMPORAL_TV && d->nt < 2)
    return set_error(CS_EINVAL, "the temporal TV prior needs nt >= 2");
  if (d->prior == CS_PRIOR_TEMPORAL_TV && !(d->mu_ratio > 0.f && std::isfinite(d->mu_ratio)))
    return set_error(CS_EINVAL, "mu_ratio (mu2/mu1) must be finite and > 0");
  if (!smooth_23(d->nv) || !smooth_23(d->nh) || d->nv > 512 || d->nh > 512)
    return set_error(CS_EUNSUPPORTED, "nv and nh must be of the form 2^a 3^b and at most 512");
  if (d->nt > 64) return set_error(CS_EUNSUPPORTED, "nt must be at most 64");
  if (d->nc > 64) return set_error(CS_EUNSUPPORTED, "nc must be at most 64");
  return validate_flags(d->flags);
}

static inline hipStream_t S(cs_stream s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- timing
enum KernelKind { kKindTV = 0, kKindDFT = 1, kKindX = 2, kKindJ = 3, kKindColumn = 4, kKindFrameFinish = 5,
                  kKinds = 6 };
static const char* kKindNames[kKinds] = {"tv_step", "dft_step", "x_update", "objective", "column_solve",
                                         "frame_finish"};

static hipEvent_t pool_event(cs_plan* p) {
  if (p->pool_next == p->event_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->event_pool.push_back(e);
  }
  return p->event_pool[p->pool_next++];
}

// runs launch() bracketed by events when timing is on
template <typename F>
static int timed_launch(cs_plan* p, int kind, hipStream_t s, F launch) {
  if (!p->timing) return launch();
  hipEvent_t a = pool_event(p), b = pool_event(p);
  if (!a || !b) return set_error(CS_EDEVICE, "hipEventCreate failed");
  CS_HIP(hipEventRecord(a, s));
  int st = launch();
  if (st != CS_OK) return st;
  CS_HIP(hipEventRecord(b, s));
  p->timed.push_back({kind, a, b});
  return CS_OK;
}

static int run_phase_loop(cs_plan* p, int32_t iters, float lambda, float mu, float* J_trace,
                          const float2* wgiven, hipStream_t s, bool cont = false);

// CS_FLAG_GRAPH: the phase-kernel loop is captured once per distinct key and
// replayed from the plan's cache.  The key holds everything the recorded
// launches bake in: iters, lambda, mu, J_trace, wgiven, the FFT tiles of the
// objective's SENSE pass and, for the overcomplete frame prior, whether the
// first pass starts from a completed w (after a set-up or an objective
// evaluation) or from the deferred state an iteration leaves.
static int run_phase_graph(cs_plan* p, int32_t iters, float lambda, float mu, float* J_trace,
                           const float2* wgiven, hipStream_t s) {
  float lm[2] = {lambda, mu};
  const bool frame = p->desc.prior == CS_PRIOR_TEMPORAL_FRAME;
  const intptr_t tiles = (intptr_t)(((uint64_t)(uint32_t)p->fft_cw << 32) | (uint32_t)p->fft_rb);
  void* key[8] = {reinterpret_cast<void*>((intptr_t)iters), nullptr, J_trace, const_cast<float2*>(wgiven),
                  reinterpret_cast<void*>((intptr_t)(wgiven != nullptr)),
                  reinterpret_cast<void*>((intptr_t)(frame && p->frame_w_ready ? 1 : 0)),
                  reinterpret_cast<void*>(tiles), nullptr};
  std::memcpy(&key[1], lm, sizeof(lm));
  if (!p->graph || std::memcmp(key, p->graph_key, sizeof(key)) != 0) {
    if (p->graph) {
      CS_HIP(hipStreamSynchronize(s));  // the cached graph may still run on this stream
      CS_HIP(hipGraphExecDestroy(p->graph));
      p->graph = nullptr;
    }
    // recording runs nothing, so it happens on a private stream: the caller's
    // stream may be the null stream, which cannot be captured
    if (!p->capture_stream) CS_HIP(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = p->capture_stream;
    CS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int st = run_phase_loop(p, iters, lambda, mu, J_trace, wgiven, cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (st != CS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      p->graph = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    std::memcpy(p->graph_key, key, sizeof(key));
  }
  CS_HIP(hipGraphLaunch(p->graph, s));
  return CS_OK;
}

int run_iterations(cs_plan* p, int32_t iters, float lambda, float mu, float* J_trace,
                          const float2* wgiven, hipStream_t s) {
  if (!J_trace && (p->desc.flags & CS_FLAG_COLUMN_RESIDENT) && column_solve_supported(p)) {
    if (iters == 0) return CS_OK;
    return timed_launch(p, kKindColumn, s, [&] { return launch_column_solve(p, iters, lambda, mu, wgiven, s); });
  }
  // inside a caller's stream capture (a batch, or the caller's own graph) the
  // plain loop is recorded into that graph instead of a cached one
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  CS_HIP(hipStreamIsCapturing(s, &cap));
  if ((p->desc.flags & CS_FLAG_GRAPH) && cap == hipStreamCaptureStatusNone && !p->timing && iters > 0) {
    const int st = run_phase_graph(p, iters, lambda, mu, J_trace, wgiven, s);
    // a replay runs no host code: the frame state is what the captured loop
    // leaves, completed exactly when its last iteration evaluated J
    p->frame_w_ready = J_trace != nullptr;
    return st;
  }
  return run_phase_loop(p, iters, lambda, mu, J_trace, wgiven, s);
}

// cont: these iterations continue a loop of the same solve, so the temporal
// DFT step's first pass also completes the previous iteration's deferred dual
// update (instead of treating the pass as the solve's first)
static int run_phase_loop(cs_plan* p, int32_t iters, float lambda, float mu, float* J_trace,
                          const float2* wgiven, hipStream_t s, bool cont) {
  const bool tv = p->desc.prior == CS_PRIOR_TEMPORAL_TV;
  int st = CS_OK;
  for (int k = 0; k < iters && st == CS_OK; ++k) {
    if (tv) {
      st = timed_launch(p, kKindTV, s, [&] { return launch_tv_step(p, lambda, mu, s); });
      if (st == CS_OK)
        st = timed_launch(p, kKindX, s,
                          [&] { return launch_xupdate(p, kSolveTV, p->hy, p->s0, p->s3, p->s2, mu, s); });
    } else if (p->desc.prior == CS_PRIOR_TEMPORAL_FRAME) {
      // a pass after the set-up or after an objective evaluation starts from
      // the completed w held in img_tmp
      const bool from_w = p->frame_w_ready;
      st = timed_launch(p, kKindDFT, s, [&] { return launch_frame_step(p, lambda, mu, from_w ? 1 : 0, s); });
      p->frame_w_ready = false;
      if (st == CS_OK)
        st = timed_launch(p, kKindX, s,
                          [&] { return launch_xupdate(p, kSolveDFT, p->hy, p->s3, nullptr, p->s2, mu, s); });
      if (st == CS_OK && J_trace) {
        // J(k) is taken at w_k (eq. L1unconst), which the next pass would
        // otherwise complete in registers: complete it (and d_k) here
        st = timed_launch(p, kKindFrameFinish, s, [&] { return launch_frame_finish(p, s); });
        p->frame_w_ready = true;
      }
    } else {
      st = timed_launch(p, kKindDFT, s, [&] {
        const bool first = k == 0 && !cont;
        return launch_dft_step(p, lambda, mu, first ? 1 : 0, first ? wgiven : nullptr, s);
      });
      if (st == CS_OK)
        st = timed_launch(p, kKindX, s,
                          [&] { return launch_xupdate(p, kSolveDFT, p->hy, p->s3, nullptr, p->s2, mu, s); });
    }
    if (st == CS_OK && J_trace)
      st = timed_launch(p, kKindJ, s, [&] { return launch_objective(p, p->s2, lambda, J_trace + k, s); });
  }
  return st;
}


int run_iterations_cont(cs_plan* p, int32_t iters, float lambda, float mu, bool cont, hipStream_t s) {
  return run_phase_loop(p, iters, lambda, mu, nullptr, nullptr, s, cont);
}

// ---------------------------------------------------------------- solve pieces

static int solve_check(cs_plan* p, float lambda, float mu, const cs_state* state) {
  if (!(lambda >= 0.f && std::isfinite(lambda))) return set_error(CS_EINVAL, "lambda must be finite and >= 0");
  if (!(mu > 0.f && std::isfinite(mu))) return set_error(CS_EINVAL, "mu must be finite and > 0");
  const bool tv = p->desc.prior == CS_PRIOR_TEMPORAL_TV;
  if (state && (!state->s0 || !state->s1 || !state->s2 || (tv && !state->s3)))
    return set_error(CS_EINVAL, "state arrays must not be NULL");
  if (state && state->iter < 0) return set_error(CS_EINVAL, "state->iter must be >= 0");
  return CS_OK;
}

// refactor if mu changed; H'y (and the hybrid data kept for the objective);
// the algorithm's initial state or the caller's warm state.  *wgiven is the
// saved w a warm DFT start hands to its first pass.
static int solve_setup(cs_plan* p, const cs_c64* y, float mu, const cs_state* state, const float2** wgiven,
                       hipStream_t s) {
  const bool tv = p->desc.prior == CS_PRIOR_TEMPORAL_TV;
  const bool warm = state && state->iter > 0;
  int st = check_finite_kspace(p, reinterpret_cast<const float2*>(y), s, "y");
  if (st != CS_OK) return st;
  if (p->desc.flags & CS_FLAG_EIGEN) {
    p->mu = mu;  // the eigen form takes mu at apply time
  } else if (mu != p->mu) {
    if (p->desc.flags & CS_FLAG_NO_REFACTOR) return set_error(CS_EMU_MISMATCH, "mu differs from the plan's mu");
    if ((st = build_factor(p, mu, s)) != CS_OK) return st;
  }
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt;
  const size_t nimg = (size_t)nv * nh * nt;
  const float2 zero = make_float2(0.f, 0.f);
  auto in_t = [&](const cs_c64* src, float2* dst, int frames) {
    return launch_transpose(reinterpret_cast<const float2*>(src), dst, frames, nv, nh, s);
  };
#define CK(expr)                           \
  do {                                     \
    if ((st = (expr)) != CS_OK) return st; \
  } while (0)
  CK(launch_adjoint_rows(p, reinterpret_cast<const float2*>(y), s));
  CK(launch_adjoint_image(p, p->hy, true, s));
  *wgiven = nullptr;
  if (tv) {
    if (warm) {
      CK(in_t(state->s0, p->s0, nt));
      CK(in_t(state->s1, p->s1, nt - 1));
      CK(in_t(state->s2, p->s2, nt));
      CK(in_t(state->s3, p->s3, nt));
    } else {
      CK(launch_copy(p->hy, p->s0, nimg, s));  // m = x
      CK(launch_copy(p->hy, p->s2, nimg, s));  // x = H'y
      CK(launch_fill(p->s1, nimg, zero, s));
      CK(launch_fill(p->s3, nimg, zero, s));
    }
  } else if (p->desc.prior == CS_PRIOR_TEMPORAL_FRAME) {
    if (warm) {
      CK(in_t(state->s0, p->img_tmp, 2 * nt));  // w, used as is by the first pass
      CK(in_t(state->s1, p->s1, 2 * nt));       // v
      CK(in_t(state->s2, p->s0, 2 * nt));       // d
      CK(launch_frame_adjoint(p, p->img_tmp, p->s2, s));  // x = Psi' w (x_out if iters == 0)
    } else {
      CK(launch_copy(p->hy, p->s2, nimg, s));              // x = H'y
      CK(launch_frame_forward(p, p->hy, p->img_tmp, s));   // w_0 = Psi H'y
      CK(launch_fill(p->s0, 2 * nimg, zero, s));           // d_0 = 0
      CK(launch_fill(p->s1, 2 * nimg, zero, s));           // v_0 = 0
    }
    p->frame_w_ready = true;
  } else {
    if (warm) {
      CK(in_t(state->s0, p->img_tmp, nt));                 // w, used as is by the first pass
      CK(launch_dft_apply(p, p->img_tmp, p->s2, nullptr, nullptr, 1, s));  // z = Psi' w (x_out if iters == 0)
      CK(in_t(state->s1, p->s1, nt));                      // v
      CK(in_t(state->s2, p->s0, nt));                      // d
      *wgiven = p->img_tmp;
    } else {
      CK(launch_copy(p->hy, p->s2, nimg, s));  // Psi' w_0 = H'y
      CK(launch_fill(p->s0, nimg, zero, s));
      CK(launch_fill(p->s1, nimg, zero, s));
    }
  }
#undef CK
  return CS_OK;
}

// x_out and the returned state after `iters` iterations of this call
static int solve_finish(cs_plan* p, int32_t iters, cs_c64* x_out, cs_state* state, hipStream_t s) {
  const bool tv = p->desc.prior == CS_PRIOR_TEMPORAL_TV;
  const bool warm = state && state->iter > 0;
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt;
  auto out_t = [&](const float2* src, cs_c64* dst, int frames) {
    return launch_transpose(src, reinterpret_cast<float2*>(dst), frames, nh, nv, s);
  };
  int st = CS_OK;
#define CK(expr)                           \
  do {                                     \
    if ((st = (expr)) != CS_OK) return st; \
  } while (0)
  CK(out_t(p->s2, x_out, nt));
  if (state) {
    if (tv) {
      CK(out_t(p->s0, state->s0, nt));
      CK(out_t(p->s1, state->s1, nt - 1));
      CK(out_t(p->s2, state->s2, nt));
      CK(out_t(p->s3, state->s3, nt));
    } else if (p->desc.prior == CS_PRIOR_TEMPORAL_FRAME) {
      if (iters > 0 || !warm) {
        // w and d of the last iteration (the pass that follows an iteration
        // completes them); a fresh start with no iteration returns w_0 = Psi H'y
        if (!p->frame_w_ready) CK(launch_frame_finish(p, s));
        p->frame_w_ready = true;
        CK(out_t(p->img_tmp, state->s0, 2 * nt));
        CK(out_t(p->s1, state->s1, 2 * nt));
        CK(out_t(p->s0, state->s2, 2 * nt));
      }
    } else if (iters > 0 || !warm) {
      // w = Psi z; after iterations this also completes the deferred dual
      // update d <- d - (w - v) of the last one.  A warm start with no
      // iteration leaves the caller's state untouched.
      CK(launch_dft_apply(p, p->s2, p->img_tmp, iters > 0 ? p->s0 : nullptr, p->s1, 0, s));
      CK(out_t(p->img_tmp, state->s0, nt));
      CK(out_t(p->s1, state->s1, nt));
      CK(out_t(p->s0, state->s2, nt));
    }
    state->iter += iters;
  }
#undef CK
  return CS_OK;
}

}  // namespace csmri

using namespace csmri;

extern "C" {

int cs_version(void) { return 10000; }

const char* cs_status_string(int status) {
  switch (status) {
    case CS_OK: return "CS_OK";
    case CS_EINVAL: return "CS_EINVAL: invalid argument";
    case CS_EUNSUPPORTED: return "CS_EUNSUPPORTED: unsupported size";
    case CS_ENOMEM: return "CS_ENOMEM: device allocation failed";
    case CS_EDEVICE: return "CS_EDEVICE: HIP runtime error";
    case CS_EMU_MISMATCH: return "CS_EMU_MISMATCH: mu differs from the plan's and refactoring is disabled";
    default: return "unknown cs_status";
  }
}

const char* cs_last_error(void) { return g_last_error.c_str(); }

int cs_plan_create(const cs_plan_desc* desc, const cs_c64* coil, const uint8_t* mask, float mu,
                   const cs_allocator* alloc, cs_stream stream, cs_plan** out) {
  if (!out) return set_error(CS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc || !coil || !mask) return set_error(CS_EINVAL, "desc, coil and mask must not be NULL");
  if (!(mu > 0.f && std::isfinite(mu))) return set_error(CS_EINVAL, "mu must be finite and > 0");
  if (alloc && !alloc->alloc) return set_error(CS_EINVAL, "allocator without an alloc callback");
  int st = validate_desc(desc);
  if (st != CS_OK) return st;
  cs_plan* p = new (std::nothrow) cs_plan();
  if (!p) return set_error(CS_ENOMEM, "host allocation of the plan failed");
  p->desc = *desc;
  p->alloc.custom = alloc != nullptr;
  if (alloc) p->alloc.a = *alloc;
  const int nv = desc->nv, nh = desc->nh, nt = desc->nt, nc = desc->nc;
  const size_t npix = (size_t)nv * nh;
  const size_t nimg = npix * nt;
  // coefficient arrays (d, v, w) of the overcomplete frame prior hold 2 nt frames
  const size_t ncoef = desc->prior == CS_PRIOR_TEMPORAL_FRAME ? 2 * nimg : nimg;
  hipStream_t s = S(stream);
  auto fail = [&](int status) {
    plan_release(p);
    return status;
  };
  // the factor is by far the largest buffer; take it before any device work
  p->flayout = make_factor_layout(nv, (size_t)nt * nh);
  if (desc->flags & CS_FLAG_EIGEN) {
    const size_t ublk = (size_t)nt * nh * nv * nv;
    if ((st = plan_alloc(p, &p->eig_uh, ublk, "the eigenvector store")) != CS_OK ||
        (st = plan_alloc(p, &p->eig_uc, ublk, "the eigenvector store")) != CS_OK ||
        (st = plan_alloc(p, &p->eig_e, (size_t)nt * nh * nv, "the eigenvalue store")) != CS_OK)
      return fail(st);
  } else if ((st = plan_alloc(p, &p->factor, factor_elems(p->flayout), "the factor store")) != CS_OK) {
    return fail(st);
  }
  if (!make_fft_desc(nv, &p->fft_v) || !make_fft_desc(nh, &p->fft_h))
    return fail(set_error(CS_EUNSUPPORTED, "no FFT plan for this size"));
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) return fail(hip_fail(e, "hipGetDevice"));

  // sampling pattern: rows per frame (host), uploaded as tables
  std::vector<uint8_t> hmask((size_t)nt * nv);
  e = hipMemcpyAsync(hmask.data(), mask, hmask.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(hip_fail(e, "copy of the mask to the host"));
  p->h_mcnt.assign(nt, 0);
  for (int t = 0; t < nt; ++t)
    for (int j = 0; j < nv; ++j) p->h_mcnt[t] += hmask[(size_t)t * nv + j] != 0;
  p->m_max = *std::max_element(p->h_mcnt.begin(), p->h_mcnt.end());
  const int mrow = std::max(p->m_max, 1);
  std::vector<int32_t> hrows((size_t)nt * mrow, -1), hrinv((size_t)nt * nv, -1);
  for (int t = 0; t < nt; ++t) {
    int r = 0;
    for (int j = 0; j < nv; ++j)
      if (hmask[(size_t)t * nv + j]) {
        hrinv[(size_t)t * nv + j] = r;
        hrows[(size_t)t * mrow + r++] = j;
      }
  }
  // FP64 first column of F_v' M_t F_v: p_t[l] = (1/nv) sum_{ky in Omega_t} exp(+2 pi i ky l / nv)
  std::vector<double2> hp((size_t)nt * nv);
  for (int t = 0; t < nt; ++t)
    for (int l = 0; l < nv; ++l) {
      double re = 0, im = 0;
      for (int r = 0; r < p->h_mcnt[t]; ++r) {
        const long long ky = hrows[(size_t)t * mrow + r];
        const double ang = 2.0 * M_PI * (double)((ky * l) % nv) / nv;
        re += std::cos(ang);
        im += std::sin(ang);
      }
      hp[(size_t)t * nv + l] = make_double2(re / nv, im / nv);
    }
  auto twiddles = [](int n) {
    std::vector<float2> w(n);
    for (int q = 0; q < n; ++q) {
      const double ang = -2.0 * M_PI * q / n;
      w[q] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    return w;
  };
  std::vector<float2> htwv = twiddles(nv), htwh = twiddles(nh);
  // unitary temporal DFT: Psi[f][t] = exp(-2 pi i f t / nt) / sqrt(nt)
  // MFMA fragments of the real 2x2-block embedding of Psi (and of Psi'):
  // Psihat[2f + a][2t + b] = [[Re P, -Im P], [Im P, Re P]], P = Psi[f][t],
  // padded to KP = 2 nt rounded up to 16; Psihat' is its transpose.  Lane l of
  // fragment (m, k) holds A[16 m + l % 16][4 k + l / 16].
  const int kp = (2 * nt + 15) / 16 * 16;
  const int kmt = kp / 16, kks = kp / 4;
  std::vector<float> hfrag((size_t)kmt * kks * 64, 0.f);
  {
    std::vector<double> E((size_t)kp * kp, 0.0);
    for (int f = 0; f < nt; ++f)
      for (int t = 0; t < nt; ++t) {
        const double ang = -2.0 * M_PI * (double)((f * t) % nt) / nt, sc = 1.0 / std::sqrt((double)nt);
        const double re = std::cos(ang) * sc, im = std::sin(ang) * sc;
        E[(size_t)(2 * f) * kp + 2 * t] = re;
        E[(size_t)(2 * f) * kp + 2 * t + 1] = -im;
        E[(size_t)(2 * f + 1) * kp + 2 * t] = im;
        E[(size_t)(2 * f + 1) * kp + 2 * t + 1] = re;
      }
    for (int mm = 0; mm < kmt; ++mm)
      for (int kk = 0; kk < kks; ++kk)
        for (int l = 0; l < 64; ++l) {
          const int r = 16 * mm + l % 16, c = 4 * kk + l / 16;
          hfrag[((size_t)mm * kks + kk) * 64 + l] = (float)E[(size_t)r * kp + c];
        }
  }
  // MFMA fragments of T^{-1}, T = rho I + D'D (FP64 Gauss-Jordan; T is symmetric
  // positive definite), padded to KT = nt rounded up to 16, same lane layout
  // as the DFT fragments
  const int kt = (nt + 15) / 16 * 16;
  std::vector<float> htfrag((size_t)(kt / 16) * (kt / 4) * 64, 0.f);
  if (desc->prior == CS_PRIOR_TEMPORAL_TV) {
    const double rho = desc->mu_ratio;
    std::vector<double> A((size_t)nt * 2 * nt, 0.0);  // [T | I]
    for (int t = 0; t < nt; ++t) {
      A[(size_t)t * 2 * nt + t] = rho + ((t == 0 || t == nt - 1) ? 1.0 : 2.0);
      if (t > 0) A[(size_t)t * 2 * nt + t - 1] = -1.0;
      if (t < nt - 1) A[(size_t)t * 2 * nt + t + 1] = -1.0;
      A[(size_t)t * 2 * nt + nt + t] = 1.0;
    }
    for (int c = 0; c < nt; ++c) {
      const double piv = A[(size_t)c * 2 * nt + c];
      for (int j = 0; j < 2 * nt; ++j) A[(size_t)c * 2 * nt + j] /= piv;
      for (int r = 0; r < nt; ++r) {
        if (r == c) continue;
        const double f = A[(size_t)r * 2 * nt + c];
        if (f != 0.0)
          for (int j = 0; j < 2 * nt; ++j) A[(size_t)r * 2 * nt + j] -= f * A[(size_t)c * 2 * nt + j];
      }
    }
    const int tks = kt / 4;
    for (int mm = 0; mm < kt / 16; ++mm)
      for (int kk = 0; kk < tks; ++kk)
        for (int l = 0; l < 64; ++l) {
          const int r = 16 * mm + l % 16, c = 4 * kk + l / 16;
          if (r < nt && c < nt) htfrag[((size_t)mm * tks + kk) * 64 + l] = (float)A[(size_t)r * 2 * nt + nt + c];
        }
  }

  const size_t ksz = (size_t)nt * nc * mrow * nh;
  if ((st = plan_alloc(p, &p->rows, hrows.size(), "rows")) ||
      (st = plan_alloc(p, &p->mcnt, (size_t)nt, "mcnt")) ||
      (st = plan_alloc(p, &p->rinv, hrinv.size(), "rinv")) ||
      (st = plan_alloc(p, &p->mask, hmask.size(), "mask")) ||
      (st = plan_alloc(p, &p->pcol, hp.size(), "pcol")) ||
      (st = plan_alloc(p, &p->tw_v, (size_t)nv, "tw_v")) ||
      (st = plan_alloc(p, &p->tw_h, (size_t)nh, "tw_h")) ||
      (st = plan_alloc(p, &p->dft_frags, hfrag.size(), "psi fragments")) ||
      (st = plan_alloc(p, &p->tv_frags, htfrag.size(), "tv fragments")) ||
      (st = plan_alloc(p, &p->coil_cm, npix * nc, "coil")) ||
      (st = plan_alloc(p, &p->ktmp, ksz, "ktmp")) ||
      (st = plan_alloc(p, &p->ftmp, ksz, "ftmp")) ||
      (st = plan_alloc(p, &p->hy, nimg, "hy")) ||
      (st = plan_alloc(p, &p->s0, ncoef, "state")) ||
      (st = plan_alloc(p, &p->s1, ncoef, "state")) ||
      (st = plan_alloc(p, &p->s2, nimg, "state")) ||
      (st = plan_alloc(p, &p->s3, nimg, "state")) ||
      (st = plan_alloc(p, &p->img_tmp, ncoef, "image workspace")) ||
      (st = plan_alloc(p, &p->jpart, (size_t)objective_partial_count(), "objective partials")) ||
      (st = plan_alloc(p, &p->jdev, 2, "objective values")) ||
      (st = plan_alloc(p, &p->check_flag, 1, "check flag")))
    return fail(st);
  p->jpart_len = objective_partial_count();

#define UP(dst, src, bytes)                                                                     \
  do {                                                                                          \
    hipError_t _e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);                  \
    if (_e != hipSuccess) return fail(hip_fail(_e, "upload of plan tables"));                   \
  } while (0)
  UP(p->rows, hrows.data(), hrows.size() * sizeof(int32_t));
  UP(p->mcnt, p->h_mcnt.data(), (size_t)nt * sizeof(int32_t));
  UP(p->rinv, hrinv.data(), hrinv.size() * sizeof(int32_t));
  UP(p->mask, hmask.data(), hmask.size());
  UP(p->pcol, hp.data(), hp.size() * sizeof(double2));
  UP(p->tw_v, htwv.data(), htwv.size() * sizeof(float2));
  UP(p->tw_h, htwh.data(), htwh.size() * sizeof(float2));
  UP(p->dft_frags, hfrag.data(), hfrag.size() * sizeof(float));
  UP(p->tv_frags, htfrag.data(), htfrag.size() * sizeof(float));
#undef UP
  if ((st = check_finite_values(p, reinterpret_cast<const float2*>(coil), npix * nc, s, "coil")) != CS_OK)
    return fail(st);
  // coil maps [c][j][i] -> column-major [c][i][j]
  if ((st = launch_transpose(reinterpret_cast<const float2*>(coil), p->coil_cm, nc, nv, nh, s)) != CS_OK)
    return fail(st);
  if (desc->flags & CS_FLAG_EIGEN) {
    if ((st = build_factor_eigen(p, s)) != CS_OK) return fail(st);
    p->mu = mu;
  } else if ((st = build_factor(p, mu, s)) != CS_OK) {
    return fail(st);
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(hip_fail(e, "hipStreamSynchronize(plan)"));
  *out = p;
  return CS_OK;
}

int cs_plan_destroy(cs_plan* plan) {
  if (!plan) return CS_OK;
  (void)hipSetDevice(plan->device);
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : plan->event_pool) (void)hipEventDestroy(e);
  plan_release(plan);
  return CS_OK;
}

int cs_kernel_timing(cs_plan* plan, int enable) {
  if (!plan) return set_error(CS_EINVAL, "plan is NULL");
  plan->timing = enable != 0;
  plan->timed.clear();
  plan->pool_next = 0;
  return CS_OK;
}

int cs_kernel_times(cs_plan* plan, cs_kernel_time* out, int max, int* count) {
  if (!plan || !count || (max > 0 && !out)) return set_error(CS_EINVAL, "plan, out and count must not be NULL");
  CS_HIP(hipSetDevice(plan->device));
  double ms[kKinds] = {};
  int n[kKinds] = {};
  for (const auto& t : plan->timed) {
    CS_HIP(hipEventSynchronize(t.stop));
    float e = 0.f;
    CS_HIP(hipEventElapsedTime(&e, t.start, t.stop));
    ms[t.kind] += e;
    n[t.kind] += 1;
  }
  int c = 0;
  for (int k = 0; k < kKinds; ++k) {
    if (!n[k]) continue;
    if (c < max) {
      std::memset(out[c].name, 0, sizeof(out[c].name));
      std::strncpy(out[c].name, kKindNames[k], sizeof(out[c].name) - 1);
      out[c].launches = n[k];
      out[c].ms = ms[k];
    }
    ++c;
  }
  *count = c;
  plan->timed.clear();
  plan->pool_next = 0;
  return CS_OK;
}

int cs_plan_bytes(const cs_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return set_error(CS_EINVAL, "plan and bytes must not be NULL");
  *bytes = plan->bytes;
  return CS_OK;
}

static size_t image_values(const cs_plan* p) { return (size_t)p->desc.nv * p->desc.nh * p->desc.nt; }

int cs_apply_A(cs_plan* p, const cs_c64* x, cs_c64* y, cs_stream stream) {
  if (!p || !x || !y) return set_error(CS_EINVAL, "plan, x and y must not be NULL");
  CS_HIP(hipSetDevice(p->device));
  int st = check_finite_values(p, reinterpret_cast<const float2*>(x), image_values(p), S(stream), "x");
  if (st != CS_OK) return st;
  return launch_forward(p, reinterpret_cast<const float2*>(x), false, reinterpret_cast<float2*>(y), S(stream));
}

int cs_apply_AH(cs_plan* p, const cs_c64* y, cs_c64* x, cs_stream stream) {
  if (!p || !x || !y) return set_error(CS_EINVAL, "plan, x and y must not be NULL");
  CS_HIP(hipSetDevice(p->device));
  int st = check_finite_kspace(p, reinterpret_cast<const float2*>(y), S(stream), "y");
  if (st != CS_OK) return st;
  st = launch_adjoint_rows(p, reinterpret_cast<const float2*>(y), S(stream));
  if (st != CS_OK) return st;
  return launch_adjoint_image(p, reinterpret_cast<float2*>(x), false, S(stream));
}

int cs_apply_block_inverse(cs_plan* p, const cs_c64* b, cs_c64* x, cs_stream stream) {
  if (!p || !b || !x) return set_error(CS_EINVAL, "plan, b and x must not be NULL");
  CS_HIP(hipSetDevice(p->device));
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt;
  hipStream_t s = S(stream);
  int st = check_finite_values(p, reinterpret_cast<const float2*>(b), image_values(p), s, "b");
  if (st == CS_OK) st = launch_transpose(reinterpret_cast<const float2*>(b), p->img_tmp, nt, nv, nh, s);
  if (st == CS_OK) st = launch_xupdate(p, kSolvePlain, p->img_tmp, nullptr, nullptr, p->img_tmp, p->mu, s);
  if (st == CS_OK) st = launch_transpose(p->img_tmp, reinterpret_cast<float2*>(x), nt, nh, nv, s);
  return st;
}

int cs_admm_solve(cs_plan* p, const cs_c64* y, float lambda, float mu, int32_t iters, cs_c64* x_out,
                  cs_state* state, float* J_trace, cs_stream stream) {
  if (!p || !y || !x_out) return set_error(CS_EINVAL, "plan, y and x_out must not be NULL");
  if (iters < 0) return set_error(CS_EINVAL, "iters must be >= 0");
  int st = solve_check(p, lambda, mu, state);
  if (st != CS_OK) return st;
  CS_HIP(hipSetDevice(p->device));
  hipStream_t s = S(stream);
  const float2* wgiven = nullptr;
  if ((st = solve_setup(p, y, mu, state, &wgiven, s)) != CS_OK) return st;
  if ((st = run_iterations(p, iters, lambda, mu, J_trace, wgiven, s)) != CS_OK) return st;
  return solve_finish(p, iters, x_out, state, s);
}

int cs_admm_solve_until(cs_plan* p, const cs_c64* y, float lambda, float mu, int32_t max_iters, float tol,
                        int32_t check_every, cs_c64* x_out, cs_state* state, int32_t* iters_done, float* delta,
                        cs_stream stream) {
  if (!p || !y || !x_out || !iters_done) return set_error(CS_EINVAL, "plan, y, x_out and iters_done must not be NULL");
  if (max_iters < 1) return set_error(CS_EINVAL, "max_iters must be >= 1");
  if (check_every < 1) return set_error(CS_EINVAL, "check_every must be >= 1");
  if (!std::isfinite(tol)) return set_error(CS_EINVAL, "tol must be finite");
  int st = solve_check(p, lambda, mu, state);
  if (st != CS_OK) return st;
  CS_HIP(hipSetDevice(p->device));
  hipStream_t s = S(stream);
  if (!p->jhost) {
    void* h = nullptr;
    CS_HIP(hipHostMalloc(&h, 2 * sizeof(float), hipHostMallocDefault));
    p->jhost = static_cast<float*>(h);
  }
  const float2* wgiven = nullptr;
  if ((st = solve_setup(p, y, mu, state, &wgiven, s)) != CS_OK) return st;
  // blocks of check_every iterations; the last two iterations of a block also
  // evaluate J, and the solve stops after the first block whose Delta(k) (eq.
  // r_ratio) falls below tol.  With check_every == 1 every iteration is
  // checked against the previous one (J(0) is taken at the initial iterate).
  int32_t k = 0;
  double last_delta = std::numeric_limits<double>::quiet_NaN();
  float jprev = 0.f;
  bool stop = false;
  while (k < max_iters && !stop && st == CS_OK) {
    const int32_t n = std::min(check_every, max_iters - k);
    const float2* wg = k == 0 ? wgiven : nullptr;
    const bool cont = k > 0;
    bool have_j0 = true;
    if (n >= 2) {
      st = run_phase_loop(p, n - 2, lambda, mu, nullptr, wg, s, cont);
      if (st == CS_OK) st = run_phase_loop(p, 1, lambda, mu, p->jdev, n > 2 ? nullptr : wg, s, cont || n > 2);
      if (st == CS_OK) st = run_phase_loop(p, 1, lambda, mu, p->jdev + 1, nullptr, s, true);
    } else if (k == 0) {
      st = launch_objective(p, p->s2, lambda, p->jdev, s);
      if (st == CS_OK) st = run_phase_loop(p, 1, lambda, mu, p->jdev + 1, wg, s, false);
    } else {
      st = run_phase_loop(p, 1, lambda, mu, p->jdev + 1, nullptr, s, true);
      have_j0 = false;  // J(k - 1) is the previous block's J
    }
    if (st != CS_OK) break;
    k += n;
    hipError_t e = hipMemcpyAsync(p->jhost, p->jdev, 2 * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      st = hip_fail(e, "reading J back");
      break;
    }
    const double j0 = have_j0 ? p->jhost[0] : jprev, j1 = p->jhost[1];
    jprev = p->jhost[1];
    last_delta = (j0 - j1) / j1;
    // converged when the relative change of J is small either way: ADMM does
    // not decrease J monotonically, and a block in which J rose by more than
    // tol is not a stall
    stop = std::fabs(last_delta) < (double)tol;
  }
  if (st != CS_OK) return st;
  *iters_done = k;
  if (delta) *delta = (float)last_delta;
  return solve_finish(p, k, x_out, state, s);
}

}  // extern "C"

// ---------------------------------------------------------------- flags and tuning

static void drop_graph(cs_plan* p) {
  if (p->graph) {
    (void)hipDeviceSynchronize();  // the cached graph may still run
    (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
  }
}

static void set_plan_flags(cs_plan* p, uint32_t flags) {
  if (flags == p->desc.flags) return;
  drop_graph(p);  // the cached graph holds the kernels of the old form
  p->desc.flags = flags;
}

extern "C" {

int cs_plan_flags(const cs_plan* p, uint32_t* flags) {
  if (!p || !flags) return set_error(CS_EINVAL, "plan and flags must not be NULL");
  *flags = p->desc.flags;
  return CS_OK;
}

int cs_plan_set_flags(cs_plan* p, uint32_t flags) {
  if (!p) return set_error(CS_EINVAL, "plan is NULL");
  int st = validate_flags(flags);
  if (st != CS_OK) return st;
  CS_HIP(hipSetDevice(p->device));
  // the factor's form is fixed when the plan is built
  set_plan_flags(p, (flags & ~(uint32_t)CS_FLAG_EIGEN) | (p->desc.flags & CS_FLAG_EIGEN));
  return CS_OK;
}

int cs_plan_fft_tiles(const cs_plan* p, int32_t* cols, int32_t* rows) {
  if (!p || !cols || !rows) return set_error(CS_EINVAL, "plan, cols and rows must not be NULL");
  *cols = fft_cols_per_group(p);
  *rows = fft_rows_per_group(p);
  return CS_OK;
}

int cs_plan_set_fft_tiles(cs_plan* p, int32_t cols, int32_t rows) {
  if (!p) return set_error(CS_EINVAL, "plan is NULL");
  if (cols < 0 || rows < 0) return set_error(CS_EINVAL, "tile sizes must be >= 0 (0 selects the largest)");
  p->fft_cw = cols;
  p->fft_rb = rows;
  return CS_OK;
}

// FFT tiles of the SENSE passes: every (columns per wave, rows per
// workgroup) pair from the largest down to 1/16 (columns) and 1/4 (rows) of
// it is timed on H'y of y (the adjoint passes) followed by the vertical
// forward pass, which the objective uses; the fastest is kept in the plan.
// The register passes (n = 16 M) have fixed tiles, so a knob they ignore is not swept.
static int tune_fft_tiles(cs_plan* p, const cs_c64* y, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int save_cw = p->fft_cw, save_rb = p->fft_rb;
  p->fft_cw = 0;
  p->fft_rb = 0;
  const int cw_default = fft_cols_per_group(p);
  const int cw_full = fft_cols_limit(p), rb_full = fft_rows_per_group(p);
  std::vector<int> cws, rbs;
  const int cw_div = reg16_size(p->desc.nv) ? 1 : 16, rb_div = reg16_size(p->desc.nh) ? 1 : 4;
  for (int d = 1; d <= cw_div; d *= 2)
    if (cw_full / d >= 1 && (cws.empty() || cws.back() != cw_full / d)) cws.push_back(cw_full / d);
  for (int d = 1; d <= rb_div; d *= 2)
    if (rb_full / d >= 1 && (rbs.empty() || rbs.back() != rb_full / d)) rbs.push_back(rb_full / d);
  float best = -1.f;
  int bcw = cw_full, brb = rb_full, st = CS_OK;
  for (int cw : cws)
    for (int rb : rbs) {
      p->fft_cw = cw;
      p->fft_rb = rb;
      auto run = [&]() {
        int r = launch_adjoint_rows(p, reinterpret_cast<const float2*>(y), s);
        if (r == CS_OK) r = launch_adjoint_image(p, p->img_tmp, true, s);
        if (r == CS_OK) r = launch_forward(p, p->img_tmp, true, nullptr, s);
        return r;
      };
      if ((st = run()) != CS_OK) break;  // warm-up
      hipError_t e = hipEventRecord(e0, s);
      for (int rep = 0; rep < 3 && e == hipSuccess && st == CS_OK; ++rep) st = run();
      if (e == hipSuccess && st == CS_OK) e = hipEventRecord(e1, s);
      if (e == hipSuccess && st == CS_OK) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess && st == CS_OK) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) st = hip_fail(e, "timing an FFT tile candidate");
      if (st != CS_OK) break;
      if (best < 0.f || ms < best) {
        best = ms;
        bcw = cw;
        brb = rb;
      }
    }
  if (st != CS_OK) {
    p->fft_cw = save_cw;
    p->fft_rb = save_rb;
    return st;
  }
  p->fft_cw = bcw == cw_default ? 0 : bcw;
  p->fft_rb = brb == rb_full ? 0 : brb;
  return CS_OK;
}

int cs_plan_tune(cs_plan* p, const cs_c64* y, float lambda, int32_t iters, cs_tune_entry* entries, int32_t cap,
                 int32_t* count, cs_stream stream) {
  if (!p || !y) return set_error(CS_EINVAL, "plan and y must not be NULL");
  if (iters < 1) return set_error(CS_EINVAL, "iters must be >= 1");
  if (!(lambda >= 0.f && std::isfinite(lambda))) return set_error(CS_EINVAL, "lambda must be finite and >= 0");
  if (cap < 0) return set_error(CS_EINVAL, "cap must be >= 0");
  if (p->timing) return set_error(CS_EINVAL, "kernel timing is on; switch it off before tuning");
  CS_HIP(hipSetDevice(p->device));
  hipStream_t s = S(stream);
  const uint32_t keep = p->desc.flags & CS_FLAG_NO_REFACTOR;
  const uint32_t forms = CS_FLAG_GRAPH | CS_FLAG_COLUMN_RESIDENT | CS_FLAG_XU_WAVE | CS_FLAG_XU_GROUP;
  const uint32_t original = p->desc.flags;
  std::vector<uint32_t> cand;
  if (p->desc.nv % 2 == 0) {
    cand.push_back(CS_FLAG_GRAPH | CS_FLAG_XU_WAVE);
    cand.push_back(CS_FLAG_GRAPH | CS_FLAG_XU_GROUP);
  } else {
    cand.push_back(CS_FLAG_GRAPH);
  }
  if (column_solve_supported(p)) cand.push_back(CS_FLAG_COLUMN_RESIDENT);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CS_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return set_error(CS_EDEVICE, "hipEventCreate failed");
  }
  int st = tune_fft_tiles(p, y, s, e0, e1);
  // a fresh start on y: the algorithm's initial state in the plan's
  // workspaces (no image is written out, so img_tmp keeps the frame prior's w_0)
  const float2* wgiven = nullptr;
  if (st == CS_OK) st = solve_setup(p, y, p->mu, nullptr, &wgiven, s);
  if (st != CS_OK) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
  }
  // kTuneRounds interleaved rounds over the candidates, each keeping its
  // fastest time, so that no candidate pays alone for the clocks ramping up or
  // for whatever ran before; every timed run follows an untimed one in the
  // same form (a form change records the plan's graph again)
  constexpr int kTuneRounds = 3;
  std::vector<float> per(cand.size(), -1.f);
  std::vector<uint32_t> used(cand.size(), 0);
  for (int round = 0; round < kTuneRounds && st == CS_OK; ++round) {
    for (size_t i = 0; i < cand.size(); ++i) {
      set_plan_flags(p, keep | cand[i] | (original & ~(forms | keep)));
      used[i] = p->desc.flags;
      // two untimed runs: the first may start from the set-up's state, which
      // the frame prior's first pass records differently, so the timed run
      // replays the graph the second one recorded
      if ((st = run_iterations(p, iters, lambda, p->mu, nullptr, nullptr, s)) != CS_OK) break;
      if ((st = run_iterations(p, iters, lambda, p->mu, nullptr, nullptr, s)) != CS_OK) break;
      hipError_t e = hipEventRecord(e0, s);
      if (e == hipSuccess) st = run_iterations(p, iters, lambda, p->mu, nullptr, nullptr, s);
      if (e == hipSuccess && st == CS_OK) e = hipEventRecord(e1, s);
      if (e == hipSuccess && st == CS_OK) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess && st == CS_OK) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) st = hip_fail(e, "timing a tuning candidate");
      if (st != CS_OK) break;
      const float v = ms / (float)iters;
      if (per[i] < 0.f || v < per[i]) per[i] = v;
    }
  }
  uint32_t best = original;
  float best_ms = 0.f;
  int32_t n = 0;
  for (size_t i = 0; i < cand.size() && st == CS_OK; ++i) {
    if (entries && n < cap) entries[n] = cs_tune_entry{used[i], per[i]};
    ++n;
    if (n == 1 || per[i] < best_ms) {
      best_ms = per[i];
      best = used[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  set_plan_flags(p, st == CS_OK ? best : original);
  // the cached graph was recorded mid-solve, from the tuning runs' state
  drop_graph(p);
  if (count) *count = n;
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------- batches

// Branches of the batch graph: the slices are dealt to this many chains in
// LPT order (the largest factor first, each to the chain with the least work
// so far), and the chains run concurrently.  Two chains let one slice's
// temporal steps and set-up run beside another's factor stream; more of them
// only make the streams compete (24 uneven slices, slice-iterations/s against
// plain solves: 1 chain x1.00, 2 x1.034-1.037, 3 x1.012, 4 x0.996, one per
// slice x0.993).
constexpr size_t kBatchBranches = 2;

struct cs_batch {
  std::vector<cs_plan*> plans;
  std::vector<hipStream_t> streams;  // one per branch, used only while recording
  std::vector<hipEvent_t> joins;
  hipEvent_t fork = nullptr;
  hipStream_t capture = nullptr;
  hipGraphExec_t graph = nullptr;
  std::vector<const void*> key;
};

// the private recording streams and events (recreated by the next recording)
static void batch_drop_streams(cs_batch* b) {
  for (hipEvent_t e : b->joins) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  b->joins.clear();
  b->streams.clear();
  b->fork = nullptr;
  b->capture = nullptr;
}

// all of them or none: a failure part way leaves nothing behind
static int batch_make_streams(cs_batch* b, size_t n) {
  hipError_t e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (size_t i = 0; i < n && e == hipSuccess; ++i) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) b->streams.push_back(st);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->joins.push_back(ev);
  }
  if (e != hipSuccess) {
    batch_drop_streams(b);
    return hip_fail(e, "creating the batch's recording streams");
  }
  return CS_OK;
}

static void batch_release(cs_batch* b) {
  if (!b) return;
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  batch_drop_streams(b);
  for (cs_plan* p : b->plans) (void)cs_plan_destroy(p);
  delete b;
}

extern "C" {

int cs_batch_create(const cs_slice_desc* slices, int32_t count, const cs_allocator* alloc, cs_stream stream,
                    cs_batch** out) {
  if (!out) return set_error(CS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!slices || count <= 0) return set_error(CS_EINVAL, "slices must be a non-empty array");
  cs_batch* b = new (std::nothrow) cs_batch();
  if (!b) return set_error(CS_ENOMEM, "host allocation of the batch failed");
  for (int32_t i = 0; i < count; ++i) {
    cs_plan_desc d = slices[i].desc;
    d.flags &= ~(uint32_t)CS_FLAG_GRAPH;  // the batch records its own graph
    cs_plan* p = nullptr;
    const int st = cs_plan_create(&d, slices[i].coil, slices[i].mask, slices[i].mu, alloc, stream, &p);
    if (st != CS_OK) {
      const std::string msg = "slice " + std::to_string(i) + ": " + g_last_error;
      batch_release(b);
      return set_error(st, msg);
    }
    b->plans.push_back(p);
  }
  *out = b;
  return CS_OK;
}

int cs_batch_destroy(cs_batch* b) {
  if (!b) return CS_OK;
  if (!b->plans.empty()) {
    (void)hipSetDevice(b->plans[0]->device);
    (void)hipDeviceSynchronize();
  }
  batch_release(b);
  return CS_OK;
}

int cs_batch_size(const cs_batch* b, int32_t* count) {
  if (!b || !count) return set_error(CS_EINVAL, "batch and count must not be NULL");
  *count = (int32_t)b->plans.size();
  return CS_OK;
}

int cs_batch_plan(cs_batch* b, int32_t index, cs_plan** plan) {
  if (!b || !plan) return set_error(CS_EINVAL, "batch and plan must not be NULL");
  if (index < 0 || (size_t)index >= b->plans.size()) return set_error(CS_EINVAL, "slice index out of range");
  *plan = b->plans[(size_t)index];
  return CS_OK;
}

int cs_batch_solve(cs_batch* b, const cs_c64* const* y, const float* lambda, int32_t iters, cs_c64* const* x_out,
                   cs_stream stream) {
  if (!b || !y || !lambda || !x_out) return set_error(CS_EINVAL, "batch, y, lambda and x_out must not be NULL");
  if (iters < 0) return set_error(CS_EINVAL, "iters must be >= 0");
  const size_t n = b->plans.size();
  for (size_t i = 0; i < n; ++i) {
    if (!y[i] || !x_out[i]) return set_error(CS_EINVAL, "slice " + std::to_string(i) + ": NULL array");
    if (!(lambda[i] >= 0.f && std::isfinite(lambda[i])))
      return set_error(CS_EINVAL, "slice " + std::to_string(i) + ": lambda must be finite and >= 0");
  }
  CS_HIP(hipSetDevice(b->plans[0]->device));
  hipStream_t s = S(stream);
  for (size_t i = 0; i < n; ++i) {
    const int st = check_finite_kspace(b->plans[i], reinterpret_cast<const float2*>(y[i]), s, "y");
    if (st != CS_OK) return set_error(st, "slice " + std::to_string(i) + ": " + g_last_error);
  }
  std::vector<const void*> key;
  key.push_back(reinterpret_cast<const void*>((intptr_t)iters));
  for (size_t i = 0; i < n; ++i) {
    uint32_t lb;
    std::memcpy(&lb, &lambda[i], sizeof(lb));
    key.push_back(y[i]);
    key.push_back(x_out[i]);
    key.push_back(reinterpret_cast<const void*>((intptr_t)lb));
    key.push_back(reinterpret_cast<const void*>((intptr_t)b->plans[i]->desc.flags));
    // a slice's plan may be used on its own in between: a solve at another mu
    // refactors it (the recorded kernels carry mu), and new FFT tiles change
    // the recorded SENSE launches
    uint32_t mb;
    std::memcpy(&mb, &b->plans[i]->mu, sizeof(mb));
    key.push_back(reinterpret_cast<const void*>((intptr_t)mb));
    key.push_back(reinterpret_cast<const void*>((intptr_t)b->plans[i]->fft_cw));
    key.push_back(reinterpret_cast<const void*>((intptr_t)b->plans[i]->fft_rb));
  }
  if (!b->graph || key != b->key) {
    if (b->graph) {
      CS_HIP(hipStreamSynchronize(s));
      CS_HIP(hipGraphExecDestroy(b->graph));
      b->graph = nullptr;
    }
    const size_t nb = std::min(n, kBatchBranches);
    if (!b->capture) {
      const int ms = batch_make_streams(b, nb);
      if (ms != CS_OK) return ms;
    }
    // record: fork each branch's stream off the capture stream, run its
    // slices' solves one after another on it, join the branches back.  The
    // slices go out in decreasing order of factor size, each to the branch
    // with the least factor work so far (LPT scheduling), so the branches end
    // close together and the largest solves are the first to reach the GPU.
    std::vector<size_t> order(n);
    for (size_t i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) {
      return factor_elems(b->plans[a]->flayout) > factor_elems(b->plans[c]->flayout);
    });
    CS_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    int st = CS_OK;
    hipError_t e = hipEventRecord(b->fork, b->capture);
    std::vector<char> forked(nb, 0);  // branch streams inside the capture
    std::vector<double> load(nb, 0.0);
    for (size_t oi = 0; oi < n && st == CS_OK && e == hipSuccess; ++oi) {
      const size_t i = order[oi];
      const size_t j = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
      load[j] += (double)factor_elems(b->plans[i]->flayout);
      if (!forked[j]) {
        e = hipStreamWaitEvent(b->streams[j], b->fork, 0);
        if (e != hipSuccess) break;
        forked[j] = 1;
      }
      cs_plan* p = b->plans[i];
      const bool saved_timing = p->timing;
      const uint32_t saved_flags = p->desc.flags;
      p->timing = false;
      // recorded straight into the batch graph; y was checked above
      p->desc.flags &= ~(uint32_t)(CS_FLAG_GRAPH | CS_FLAG_CHECK_FINITE);
      st = cs_admm_solve(p, y[i], lambda[i], p->mu, iters, x_out[i], nullptr, nullptr, b->streams[j]);
      p->timing = saved_timing;
      p->desc.flags = saved_flags;
    }
    // every forked branch is joined back before the capture ends (also after
    // a failure, so that no stream stays attached to an abandoned capture)
    for (size_t j = 0; j < nb; ++j) {
      if (!forked[j]) continue;
      hipError_t ej = hipEventRecord(b->joins[j], b->streams[j]);
      if (ej == hipSuccess) ej = hipStreamWaitEvent(b->capture, b->joins[j], 0);
      if (e == hipSuccess) e = ej;
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->capture, &g);
    if (st != CS_OK || e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      // the recording streams are not reused after a failed recording
      (void)hipGetLastError();
      batch_drop_streams(b);
      if (st != CS_OK) return st;
      return hip_fail(e != hipSuccess ? e : e2, "recording the batch graph");
    }
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->graph = nullptr;
      return hip_fail(e, "hipGraphInstantiate(batch)");
    }
    b->key = key;
  }
  CS_HIP(hipGraphLaunch(b->graph, s));
  return CS_OK;
}

}  // extern "C"
