// Reverse-mode differentiation of unrolled Algorithm 2 (temporal TV) and
// Algorithm 1 (temporal DFT): the checkpointed forward and the adjoint sweep
// behind cs_admm_forward_ckpt / cs_admm_backward.  The Algorithm 1 reverse
// step is the x-update kernel applying W followed by k_dft_adjoint
// (iterate.hip), which carries its derivation; what follows is Algorithm 2's.
//
// One iteration of Algorithm 2 (Sec. IV-B), with D = D_t (eq. TV),
// T = rho I + D'D, W = (mu I + H'H)^{-1} (eq. eigen_mu), tau = lambda/(2 mu1):
//     a = D m + d1;  v = soft(a, tau);  m' = T^{-1}[D'(v - d1) + rho (x + d2)]
//     x' = W [H'y + mu (m' - d2)];  d1' = d1 - (v - D m');  d2' = d2 - (m' - x')
// Its transposed Jacobian, given the adjoints (mb', d1b', d2b', xb') of the
// state after it (gradients in the dL/dRe + i dL/dIm convention):
//     bb  = W (xb' + d2b')                          W Hermitian
//     q   = mb' - d2b' + D' d1b' + mu bb           adjoint of m', T^{-1} applied next
//     rb  = T^{-1} q                                T real symmetric
//     vb  = D rb - d1b'
//     ab  = (dsoft/da)^T vb                         real 2x2 Jacobian on |a| > tau
//     mb  = D' ab;  d1b = d1b' - D rb + ab;  xb = rho rb;  d2b = d2b' - mu bb + rho rb
//     dL/dH'y += bb;  dL/dtau += -sum_{|a|>tau} Re(conj(a/|a|) vb)
//     dL/dmu  += Re<bb, m' - d2 - x'> = -Re<bb, d2'>     (the rhs term plus dW/dmu = -W^2)
// and at the end x_0 = m_0 = H'y adds mb + xb to dL/dH'y, tau = lambda rho/(2 mu)
// turns dL/dtau into dL/dlambda and dL/dmu, and dL/dy = A(dL/dH'y).
//
// Kernels: the x-update kernel applies W (bb = W e with e = xb' + d2b');
// k_tv_adjoint_tiles (iterate.hip) does everything else, 16 pixels per wave,
// with T^{-1} applied on the matrix cores, and accumulates per-workgroup FP64
// partial sums of dL/dtau and dL/dmu in its own slot (no atomics; summed in a
// fixed order at the end).
#include <algorithm>
#include <new>

#include "internal.hpp"

namespace csmri {

int run_iterations(cs_plan* p, int32_t iters, float lambda, float mu, float* J_trace, const float2* wgiven,
                   hipStream_t s);

// partial sums: one FP64 pair per 64 pixels (a workgroup of the reverse-step kernels)
constexpr int kAdjPixels = 64;

// dL/dlambda and dL/dmu from the accumulated dL/dtau and direct dL/dmu
__global__ __launch_bounds__(256) void k_grad_finish(const double* __restrict__ partial, int nslots,
                                                     float* __restrict__ out, double lambda, double mu,
                                                     double rho) {
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nslots; i += 256) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double gtau = red[0][0], gmu = red[1][0];
    out[0] = (float)(gtau * rho / (2.0 * mu));
    out[1] = (float)(gmu - gtau * lambda * rho / (2.0 * mu * mu));
  }
}

}  // namespace csmri

using namespace csmri;

struct cs_grad {
  cs_plan* plan = nullptr;
  int iters = 0, every = 1, nseg = 0;
  size_t nimg = 0, npix = 0;
  float lambda = 0.f, mu = 0.f;
  bool ready = false;
  std::vector<void*> owned;
  float2* hy = nullptr;
  std::vector<float2*> ck;          // [nseg][4]: m, d1, x, d2 at the start of each segment
  bool dft = false;                   // Algorithm 1 (temporal DFT) instead of Algorithm 2
  // the tape of one segment.  TV: m_j, d1_j (before step j+1), d2_j.  DFT
  // (same arrays): z_j (tm, j <= L), d_j completed by step j+1 (td1), u_{j+1} (td2)
  std::vector<float2*> tm, td1, td2;  // [every + 1]
  int taped_seg = -1;                 // segment whose tape the forward left in tm/td1/td2, or -1
  float2 *mb = nullptr, *d1b = nullptr, *d2b = nullptr, *e = nullptr, *bb = nullptr, *hyb = nullptr;
  double* partial = nullptr;
  int nslots = 0;
};

static void grad_release(cs_grad* g) {
  if (!g) return;
  for (void* ptr : g->owned) g->plan->alloc.put(ptr);
  delete g;
}

static int grad_alloc(cs_grad* g, float2** out, size_t count) {
  void* ptr = g->plan->alloc.get(std::max<size_t>(count * sizeof(float2), 256));
  if (!ptr) return set_error(CS_ENOMEM, "allocator returned NULL for the gradient workspace");
  g->owned.push_back(ptr);
  *out = static_cast<float2*>(ptr);
  return CS_OK;
}

// one Algorithm 2 iteration on the plan's state, exactly as cs_admm_solve runs it
static int one_iteration(cs_plan* p, float lambda, float mu, hipStream_t s) {
  return run_iterations(p, 1, lambda, mu, nullptr, nullptr, s);
}

// L iterations of Algorithm 2 on the plan's state (m = s0, d1 = s1, x = s2,
// d2 = s3), one at a time, keeping m_j and d1_j before step j + 1 and d2 after it
static int tv_segment_tape(cs_grad* g, int L, float lambda, float mu, hipStream_t s) {
  cs_plan* p = g->plan;
  const size_t n = g->nimg;
  int st = launch_copy_multi(CopyPairs{{p->s0, p->s1}, {g->tm[0], g->td1[0]}, 2}, n, s);
  for (int j = 0; j < L && st == CS_OK; ++j) {
    st = one_iteration(p, lambda, mu, s);
    if (st != CS_OK) break;
    if (j + 1 < L)
      st = launch_copy_multi(CopyPairs{{p->s3, p->s0, p->s1}, {g->td2[j + 1], g->tm[j + 1], g->td1[j + 1]}, 3}, n, s);
    else
      st = launch_copy(p->s3, g->td2[j + 1], n, s);
  }
  return st;
}

// L iterations of Algorithm 1 on the plan's state (z = s2, d = s0, v = s1),
// one at a time, keeping z before each and the completed d and u after it;
// cont: the first of them continues the solve (completes the deferred d)
static int dft_segment_tape(cs_grad* g, int L, float lambda, float mu, bool cont, hipStream_t s) {
  cs_plan* p = g->plan;
  const size_t n = g->nimg;
  int st = CS_OK;
  st = launch_copy(p->s2, g->tm[0], n, s);
  for (int j = 0; j < L && st == CS_OK; ++j) {
    st = run_iterations_cont(p, 1, lambda, mu, cont || j > 0, s);
    // d and u after step j, and z before step j + 1 (= after step j)
    if (st == CS_OK) st = launch_copy_multi(CopyPairs{{p->s0, p->s3, p->s2}, {g->td1[j], g->td2[j], g->tm[j + 1]}, 3},
                                            n, s);
  }
  return st;
}

static int ensure_mu(cs_plan* p, float mu, hipStream_t s) {
  if (p->desc.flags & CS_FLAG_EIGEN) {
    p->mu = mu;  // the eigen form takes mu at apply time
    return CS_OK;
  }
  if (mu == p->mu) return CS_OK;
  if (p->desc.flags & CS_FLAG_NO_REFACTOR) return set_error(CS_EMU_MISMATCH, "mu differs from the plan's mu");
  return build_factor(p, mu, s);
}

// Algorithm 1: with x_K = Psi' w_K, the adjoints after the last iteration are
// wb_K = Psi g, db_K = 0, so the adjoint reaching z_K is Psi'(wb_K - db_K) = g
static int dft_backward(cs_grad* g, const cs_c64* grad_x, cs_c64* grad_y, float* grad_lambda_mu, hipStream_t s) {
  cs_plan* p = g->plan;
  const float lambda = g->lambda, mu = g->mu;
  const float tau = lambda / (2.0f * mu);  // as the forward step computes it
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt;
  const size_t n = g->nimg;
  const float2 zero = make_float2(0.f, 0.f);
  int st = CS_OK;
#define CK(expr)                              \
  do {                                        \
    if (st == CS_OK) st = (expr);             \
  } while (0)
  float2* zb = g->e;   // adjoint reaching z (image)
  float2* db = g->d1b; // adjoint of d (frequency)
  CK(launch_transpose(reinterpret_cast<const float2*>(grad_x), zb, nt, nv, nh, s));
  CK(launch_fill(db, n, zero, s));
  CK(launch_fill(g->hyb, n, zero, s));
  CK(launch_fill(reinterpret_cast<float2*>(g->partial), (size_t)g->nslots * 2, zero, s));
  CK(launch_copy(g->hy, p->hy, n, s));  // the plan may have solved something else since
  for (int seg = g->nseg - 1; seg >= 0 && st == CS_OK; --seg) {
    const int L = std::min(g->every, g->iters - seg * g->every);
    if (seg != g->taped_seg) {
      CK(launch_copy_multi(CopyPairs{{g->ck[(size_t)seg * 4 + 0], g->ck[(size_t)seg * 4 + 1],
                                      g->ck[(size_t)seg * 4 + 2]}, {p->s2, p->s0, p->s1}, 3}, n, s));
      CK(dft_segment_tape(g, L, lambda, mu, seg > 0, s));
    }
    g->taped_seg = -1;  // the tape now holds (or will hold) another segment
    for (int j = L - 1; j >= 0 && st == CS_OK; --j) {
      CK(launch_xupdate(p, kSolvePlain, zb, nullptr, nullptr, g->bb, mu, s));  // bb = W zb
      const int last = (seg == 0 && j == 0) ? 1 : 0;
      CK(launch_dft_adjoint(p, (unsigned)g->nslots, g->bb, db, zb, g->hyb, g->tm[j], g->td1[j], g->td2[j],
                            g->tm[j + 1], g->partial, tau, mu, last, s));
    }
  }
  if (g->iters == 0) CK(launch_copy(zb, g->hyb, n, s));  // x_K = x_0 = H'y
  if (st == CS_OK) {
    hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(256), 0, s, g->partial, g->nslots, grad_lambda_mu,
                       (double)lambda, (double)mu, 1.0);  // tau = lambda / (2 mu)
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) st = hip_fail(e, "k_grad_finish");
  }
  CK(launch_forward(p, g->hyb, true, reinterpret_cast<float2*>(grad_y), s));  // dL/dy = A(dL/dH'y)
#undef CK
  return st;
}

extern "C" {

int cs_grad_create(cs_plan* p, int32_t iters, int32_t every, cs_grad** out) {
  if (!out) return set_error(CS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return set_error(CS_EINVAL, "plan is NULL");
  if (p->desc.prior == CS_PRIOR_TEMPORAL_FRAME)
    return set_error(CS_EUNSUPPORTED, "differentiation is implemented for the temporal TV and DFT priors");
  if (iters < 0) return set_error(CS_EINVAL, "iters must be >= 0");
  if (every < 1) return set_error(CS_EINVAL, "ckpt_every must be >= 1");
  cs_grad* g = new (std::nothrow) cs_grad();
  if (!g) return set_error(CS_ENOMEM, "host allocation failed");
  g->plan = p;
  g->dft = p->desc.prior == CS_PRIOR_TEMPORAL_DFT;
  g->iters = iters;
  g->every = std::min(every, std::max(iters, 1));
  g->nseg = (iters + g->every - 1) / g->every;
  g->npix = (size_t)p->desc.nv * p->desc.nh;
  g->nimg = g->npix * p->desc.nt;
  g->nslots = (int)((g->npix + kAdjPixels - 1) / kAdjPixels);
  int st = CS_OK;
  auto A = [&](float2** q) {
    if (st == CS_OK) st = grad_alloc(g, q, g->nimg);
  };
  CS_HIP(hipSetDevice(p->device));
  A(&g->hy);
  g->ck.assign((size_t)g->nseg * 4, nullptr);
  for (auto& q : g->ck) A(&q);
  g->tm.assign(g->every + 1, nullptr);
  g->td1.assign(g->every + 1, nullptr);
  g->td2.assign(g->every + 1, nullptr);
  for (int j = 0; j <= g->every; ++j) {
    if (j < g->every || g->dft) A(&g->tm[j]);
    if (j < g->every) A(&g->td1[j]);
    if (j > 0 || g->dft) A(&g->td2[j]);
  }
  A(&g->mb);
  A(&g->d1b);
  A(&g->d2b);
  A(&g->e);
  A(&g->bb);
  A(&g->hyb);
  if (st == CS_OK) {
    float2* part = nullptr;
    st = grad_alloc(g, &part, (size_t)g->nslots * 2);  // 2 doubles per slot
    g->partial = reinterpret_cast<double*>(part);
  }
  if (st != CS_OK) {
    grad_release(g);
    return st;
  }
  *out = g;
  return CS_OK;
}

int cs_grad_destroy(cs_grad* g) {
  if (!g) return CS_OK;
  (void)hipSetDevice(g->plan->device);
  (void)hipDeviceSynchronize();
  grad_release(g);
  return CS_OK;
}

int cs_admm_forward_ckpt(cs_grad* g, const cs_c64* y, float lambda, float mu, cs_c64* x_out, cs_stream stream) {
  if (!g || !y || !x_out) return set_error(CS_EINVAL, "grad, y and x_out must not be NULL");
  if (!(lambda >= 0.f && std::isfinite(lambda))) return set_error(CS_EINVAL, "lambda must be finite and >= 0");
  if (!(mu > 0.f && std::isfinite(mu))) return set_error(CS_EINVAL, "mu must be finite and > 0");
  cs_plan* p = g->plan;
  CS_HIP(hipSetDevice(p->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  g->ready = false;
  int st = check_finite_kspace(p, reinterpret_cast<const float2*>(y), s, "y");
  if (st == CS_OK) st = ensure_mu(p, mu, s);
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt;
  const size_t n = g->nimg;
  const float2 zero = make_float2(0.f, 0.f);
#define CK(expr)                              \
  do {                                        \
    if (st == CS_OK) st = (expr);             \
  } while (0)
  CK(launch_adjoint_rows(p, reinterpret_cast<const float2*>(y), s));
  CK(launch_adjoint_image(p, p->hy, true, s));
  CK(launch_copy(p->hy, g->hy, n, s));
  if (g->dft) {
    // Algorithm 1's initial state as cs_admm_solve sets it: z = Psi' w_0 = H'y, d = v = 0
    CK(launch_copy(p->hy, p->s2, n, s));
    CK(launch_fill(p->s0, n, zero, s));
    CK(launch_fill(p->s1, n, zero, s));
    g->taped_seg = -1;
    for (int seg = 0; seg < g->nseg && st == CS_OK; ++seg) {
      CK(launch_copy_multi(CopyPairs{{p->s2, p->s0, p->s1}, {g->ck[(size_t)seg * 4 + 0], g->ck[(size_t)seg * 4 + 1],
                                                             g->ck[(size_t)seg * 4 + 2]}, 3}, n, s));
      const int L = std::min(g->every, g->iters - seg * g->every);
      if (seg + 1 < g->nseg) {
        CK(run_iterations_cont(p, L, lambda, mu, seg > 0, s));
      } else {
        CK(dft_segment_tape(g, L, lambda, mu, seg > 0, s));
        if (st == CS_OK) g->taped_seg = seg;
      }
    }
    CK(launch_transpose(p->s2, reinterpret_cast<float2*>(x_out), nt, nh, nv, s));
    if (st != CS_OK) return st;
    g->lambda = lambda;
    g->mu = mu;
    g->ready = true;
    return CS_OK;
  }
  CK(launch_copy_multi(CopyPairs{{p->hy, p->hy}, {p->s0, p->s2}, 2}, n, s));  // m = x = H'y
  CK(launch_fill(p->s1, n, zero, s));
  CK(launch_fill(p->s3, n, zero, s));
  float2* state[4] = {p->s0, p->s1, p->s2, p->s3};
  g->taped_seg = -1;
  for (int seg = 0; seg < g->nseg && st == CS_OK; ++seg) {
    CK(launch_copy_multi(CopyPairs{{state[0], state[1], state[2], state[3]},
                                   {g->ck[(size_t)seg * 4 + 0], g->ck[(size_t)seg * 4 + 1], g->ck[(size_t)seg * 4 + 2],
                                    g->ck[(size_t)seg * 4 + 3]}, 4}, n, s));
    const int L = std::min(g->every, g->iters - seg * g->every);
    if (seg + 1 < g->nseg) {
      CK(run_iterations(p, L, lambda, mu, nullptr, nullptr, s));
    } else {
      // the last segment is the first one the backward sweeps: keep its tape
      // now, so that the backward need not recompute it (with ckpt_every >= K
      // nothing is recomputed at all)
      CK(tv_segment_tape(g, L, lambda, mu, s));
      if (st == CS_OK) g->taped_seg = seg;
    }
  }
  CK(launch_transpose(p->s2, reinterpret_cast<float2*>(x_out), nt, nh, nv, s));
#undef CK
  if (st != CS_OK) return st;
  g->lambda = lambda;
  g->mu = mu;
  g->ready = true;
  return CS_OK;
}

int cs_admm_backward(cs_grad* g, const cs_c64* grad_x, cs_c64* grad_y, float* grad_lambda_mu, cs_stream stream) {
  if (!g || !grad_x || !grad_y || !grad_lambda_mu)
    return set_error(CS_EINVAL, "grad, grad_x, grad_y and grad_lambda_mu must not be NULL");
  if (!g->ready) return set_error(CS_EINVAL, "cs_admm_backward needs a preceding cs_admm_forward_ckpt");
  cs_plan* p = g->plan;
  CS_HIP(hipSetDevice(p->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const float lambda = g->lambda, mu = g->mu, rho = p->desc.mu_ratio;
  const float tau = lambda * rho / (2.0f * mu);  // as the forward step computes it
  int st = check_finite_values(p, reinterpret_cast<const float2*>(grad_x),
                               (size_t)p->desc.nv * p->desc.nh * p->desc.nt, s, "grad_x");
  if (st == CS_OK) st = ensure_mu(p, mu, s);
  if (st != CS_OK) return st;
  if (g->dft) return dft_backward(g, grad_x, grad_y, grad_lambda_mu, s);
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt;
  const size_t n = g->nimg;
  const float2 zero = make_float2(0.f, 0.f);
#define CK(expr)                              \
  do {                                        \
    if (st == CS_OK) st = (expr);             \
  } while (0)
  CK(launch_transpose(reinterpret_cast<const float2*>(grad_x), g->e, nt, nv, nh, s));  // e = xb_K + d2b_K
  CK(launch_fill(g->mb, n, zero, s));
  CK(launch_fill(g->d1b, n, zero, s));
  CK(launch_fill(g->d2b, n, zero, s));
  CK(launch_fill(g->hyb, n, zero, s));
  CK(launch_fill(reinterpret_cast<float2*>(g->partial), (size_t)g->nslots * 2, zero, s));
  CK(launch_copy(g->hy, p->hy, n, s));  // the plan may have solved something else since
  float2* state[4] = {p->s0, p->s1, p->s2, p->s3};
  const unsigned blocks = (unsigned)g->nslots;
  for (int seg = g->nseg - 1; seg >= 0 && st == CS_OK; --seg) {
    const int L = std::min(g->every, g->iters - seg * g->every);
    if (seg != g->taped_seg) {
      CK(launch_copy_multi(CopyPairs{{g->ck[(size_t)seg * 4 + 0], g->ck[(size_t)seg * 4 + 1],
                                      g->ck[(size_t)seg * 4 + 2], g->ck[(size_t)seg * 4 + 3]},
                                     {state[0], state[1], state[2], state[3]}, 4}, n, s));
      CK(tv_segment_tape(g, L, lambda, mu, s));  // recompute the segment, keeping what the adjoint needs
    }
    g->taped_seg = -1;  // the tape now holds (or will hold) another segment
    for (int j = L - 1; j >= 0 && st == CS_OK; --j) {
      CK(launch_xupdate(p, kSolvePlain, g->e, nullptr, nullptr, g->bb, mu, s));  // bb = W e
      if (st != CS_OK) break;
      const int last = (seg == 0 && j == 0) ? 1 : 0;
      CK(launch_tv_adjoint(p, blocks, g->mb, g->d1b, g->d2b, g->e, g->bb, g->hyb, g->tm[j], g->td1[j],
                           g->td2[j + 1], g->partial, tau, rho, mu, last, s));
    }
  }
  if (g->iters == 0) CK(launch_copy(g->e, g->hyb, n, s));  // x_K = x_0 = H'y
  if (st == CS_OK) {
    hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(256), 0, s, g->partial, g->nslots, grad_lambda_mu,
                       (double)lambda, (double)mu, (double)rho);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) st = hip_fail(e, "k_grad_finish");
  }
  CK(launch_forward(p, g->hyb, true, reinterpret_cast<float2*>(grad_y), s));  // dL/dy = A(dL/dH'y)
#undef CK
  return st;
}

}  // extern "C"
