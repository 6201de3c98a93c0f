// Per-iteration kernels of Algorithms 1 and 2 (Sec. IV-A/B).
//
// Solver arrays use the paper's column stacking (eq. x_def): frame-major,
// then column i, then row j fastest, so one (column, frame) block of the
// x-update is nv contiguous values and one pixel's time series is a stride-
// (nv*nh) sequence read coalesced across neighbouring pixels.
#include "internal.hpp"

namespace csmri {

// ---------------------------------------------------------------- x-update
//
// x = (mu I + G_{i,t})^{-1} b for one (column, frame) block per workgroup,
// with W = (mu I + G)^{-1} stored as wrapped diagonals c_s[k] = W[k, k+s]
// (see FactorLayout):
//   (W b)_k = c_0[k] b_k + sum_{s=1}^{F-1} ( c_s[k] b_{k+s} + conj(c_s[k-s]) b_{k-s} )
//             (+ c_{n/2}[k] b_{k+n/2} or conj(c_{n/2}[k-n/2]) b_{k-n/2} for even n),
// indices mod n.  The right-hand side and the dual update are fused around
// the product:
//   TV  (Algorithm 2):  b = H'y + mu2 (m - d2);  x = W b;  d2 <- d2 - (m - x)
//   DFT (Algorithm 1):  b = H'y + mu u,  u = Psi'(v + d) from the temporal step
//   plain:              x = W b
// Every factor value is read from HBM exactly once per launch.

typedef float v4f __attribute__((ext_vector_type(4)));

// streaming (non-temporal) 16-byte load: the factor is read once per
// iteration and is far larger than the caches, so it should not evict the
// iterates, which are reused by the next kernel
__device__ inline float4 ld_stream4(const float2* p) {
  const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

template <int MODE>
__device__ inline float2 rhs_value(const float2* hy, const float2* m, const float2* d2, size_t q, float mu,
                                   float2& mk, float2& dk) {
  const float2 h = hy[q];
  if (MODE == kSolvePlain) return h;
  if (MODE == kSolveTV) {
    mk = m[q];
    dk = d2[q];
    return make_float2(fmaf(mu, mk.x - dk.x, h.x), fmaf(mu, mk.y - dk.y, h.y));
  }
  const float2 u = m[q];
  return make_float2(fmaf(mu, u.x, h.x), fmaf(mu, u.y, h.y));
}

// Even n: lane l owns rows 2l and 2l+1 and streams each diagonal as one
// 16-byte load per lane.  The rotated values c_s[k-s] belong to other lanes;
// UNR diagonals at a time are staged in LDS and read back rotated.
template <int MODE, int UNR>
__global__ __launch_bounds__(256) void k_xupdate_pairs(const float2* __restrict__ W, FactorLayout L,
                                                       const float2* hy, const float2* __restrict__ m,
                                                       float2* __restrict__ d2, float2* x, float mu) {
  extern __shared__ float2 lds[];
  const int n = L.n, h = n >> 1, F = L.F;
  float2* bsh = lds;      // [n]   right-hand side
  float2* dsh = lds + n;  // [UNR][n] staged diagonals
  const int l = threadIdx.x;
  const bool act = l < h;
  const size_t blk = blockIdx.x;
  const size_t base = blk * (size_t)n;
  const int k0 = 2 * l, k1 = 2 * l + 1;
  float2 b0 = make_float2(0.f, 0.f), b1 = b0, m0 = b0, m1 = b0, e0 = b0, e1 = b0;
  if (act) {
    b0 = rhs_value<MODE>(hy, m, d2, base + k0, mu, m0, e0);
    b1 = rhs_value<MODE>(hy, m, d2, base + k1, mu, m1, e1);
    bsh[k0] = b0;
    bsh[k1] = b1;
  }
  __syncthreads();
  float2 a0 = make_float2(0.f, 0.f), a1 = a0;
  if (act) {
    const float4 c = ld_stream4(W + diag_offset(L, blk, 0) + k0);
    a0 = cmul(make_float2(c.x, c.y), b0);
    a1 = cmul(make_float2(c.z, c.w), b1);
  }
  for (int s0 = 1; s0 < F; s0 += UNR) {
    float4 c[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      c[u] = (act && s0 + u < F) ? ld_stream4(W + diag_offset(L, blk, s0 + u) + k0) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      if (act) *reinterpret_cast<float4*>(dsh + u * n + k0) = c[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int s = s0 + u;
      if (act && s < F) {
        int p0 = k0 + s, p1 = k1 + s, q0 = k0 - s, q1 = k1 - s;
        p0 -= p0 >= n ? n : 0;
        p1 -= p1 >= n ? n : 0;
        q0 += q0 < 0 ? n : 0;
        q1 += q1 < 0 ? n : 0;
        const float2* d = dsh + u * n;
        a0 = cfma(make_float2(c[u].x, c[u].y), bsh[p0], a0);
        a1 = cfma(make_float2(c[u].z, c[u].w), bsh[p1], a1);
        a0 = cfmac(d[q0], bsh[q0], a0);
        a1 = cfmac(d[q1], bsh[q1], a1);
      }
    }
    __syncthreads();
  }
  if (!act) return;
  const float2* hd = W + half_offset(L, blk);
  a0 = k0 < h ? cfma(hd[k0], bsh[k0 + h], a0) : cfmac(hd[k0 - h], bsh[k0 - h], a0);
  a1 = k1 < h ? cfma(hd[k1], bsh[k1 + h], a1) : cfmac(hd[k1 - h], bsh[k1 - h], a1);
  x[base + k0] = a0;
  x[base + k1] = a1;
  if (MODE == kSolveTV) {
    d2[base + k0] = make_float2(e0.x - (m0.x - a0.x), e0.y - (m0.y - a0.y));
    d2[base + k1] = make_float2(e1.x - (m1.x - a1.x), e1.y - (m1.y - a1.y));
  }
}

// Odd n: lane k owns row k; the rotated c_s[k-s] is re-read from the same
// diagonal run, which the vector cache serves.
template <int MODE>
__global__ __launch_bounds__(512) void k_xupdate_rows(const float2* __restrict__ W, FactorLayout L,
                                                      const float2* hy, const float2* __restrict__ m,
                                                      float2* __restrict__ d2, float2* x, float mu) {
  extern __shared__ float2 bsh[];
  const int n = L.n;
  const int k = threadIdx.x;
  const size_t blk = blockIdx.x;
  const size_t base = blk * (size_t)n;
  float2 bk = make_float2(0.f, 0.f), mk = bk, dk = bk;
  if (k < n) {
    bk = rhs_value<MODE>(hy, m, d2, base + k, mu, mk, dk);
    bsh[k] = bk;
  }
  __syncthreads();
  if (k >= n) return;
  float2 acc = cmul(W[diag_offset(L, blk, 0) + k], bk);
#pragma unroll 8
  for (int s = 1; s < L.F; ++s) {
    const float2* dg = W + diag_offset(L, blk, s);
    int kp = k + s;
    kp -= kp >= n ? n : 0;
    int km = k - s;
    km += km < 0 ? n : 0;
    acc = cfma(dg[k], bsh[kp], acc);
    acc = cfmac(dg[km], bsh[km], acc);
  }
  x[base + k] = acc;
  if (MODE == kSolveTV) d2[base + k] = make_float2(dk.x - (mk.x - acc.x), dk.y - (mk.y - acc.y));
}

constexpr int kXUnroll = 8;

template <int MODE>
static void xupdate_launch(cs_plan* p, const float2* hy, const float2* m, float2* d2, float2* x, float mu,
                           hipStream_t s) {
  const FactorLayout& L = p->flayout;
  const int n = L.n;
  const unsigned nblk = (unsigned)L.nblk;
  if ((n & 1) == 0) {
    const int wg = (std::max(n / 2, 1) + 63) / 64 * 64;
    const size_t lds = (size_t)(1 + kXUnroll) * n * sizeof(float2);
    hipLaunchKernelGGL((k_xupdate_pairs<MODE, kXUnroll>), dim3(nblk), dim3(wg), lds, s, p->factor, L, hy, m, d2,
                       x, mu);
  } else {
    const int wg = (n + 63) / 64 * 64;
    hipLaunchKernelGGL(k_xupdate_rows<MODE>, dim3(nblk), dim3(wg), (size_t)n * sizeof(float2), s, p->factor, L,
                       hy, m, d2, x, mu);
  }
}

int launch_block_solve(cs_plan* p, int mode, const float2* hy, const float2* m, float2* d2, float2* x,
                       float mu, hipStream_t s) {
  if (mode == kSolveTV) xupdate_launch<kSolveTV>(p, hy, m, d2, x, mu, s);
  else if (mode == kSolveDFT) xupdate_launch<kSolveDFT>(p, hy, m, d2, x, mu, s);
  else xupdate_launch<kSolvePlain>(p, hy, m, d2, x, mu, s);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// ---------------------------------------------------------------- TV step
//
// Algorithm 2, lines v, m and d1 with R = D_t, one pixel per thread over all
// frames (D_t couples frames only):
//   v   = soft(D m + d1, tau),  tau = lambda / (2 mu1)
//   m   = (rho I + D'D)^{-1} [ D'(v - d1) + rho (x + d2) ],  rho = mu2 / mu1
//   d1 <- d1 - (v - D m)
// rho I + D'D is tridiagonal (diagonal rho+1, rho+2, ..., rho+2, rho+1; off-
// diagonals -1) and is solved exactly by the Thomas recurrence with the
// pivots' reciprocals invden[t] precomputed in FP64.  v never reaches memory:
// e_t = d1_t - v_t is kept in registers for the dual update.
// The time series of a pixel (4 arrays x nt frames) is loaded before any
// arithmetic so that all its loads are in flight together: a 256x256 image
// has only one wave per SIMD, so latency has to be hidden inside the wave.
template <int NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_tv_step(
    float2* __restrict__ m, float2* __restrict__ d1, const float2* __restrict__ x, const float2* __restrict__ d2,
    const float* __restrict__ invden, int nt, size_t npix, float tau, float rho) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  float2 M[NT], E[NT], R[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    M[t] = t < nt ? m[(size_t)t * npix + p] : make_float2(0.f, 0.f);
    E[t] = t < nt - 1 ? d1[(size_t)t * npix + p] : make_float2(0.f, 0.f);
    if (t < nt) {
      const float2 xt = x[(size_t)t * npix + p], d2t = d2[(size_t)t * npix + p];
      R[t] = make_float2(rho * (xt.x + d2t.x), rho * (xt.y + d2t.y));
    } else {
      R[t] = make_float2(0.f, 0.f);
    }
  }
  // v_t = soft(m_{t+1} - m_t + d1_t); e_t = d1_t - v_t (kept in E);
  // r_t = rho (x_t + d2_t) + e_t - e_{t-1}; forward Thomas sweep in place (R)
  float2 eprev = make_float2(0.f, 0.f), dprev = make_float2(0.f, 0.f);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t < nt) {
      float2 dtu = make_float2(0.f, 0.f);
      if (t < nt - 1) {
        const float2 a = make_float2(M[t + 1].x - M[t].x + E[t].x, M[t + 1].y - M[t].y + E[t].y);
        const float2 v = soft_threshold(a, tau);
        E[t] = csub(E[t], v);
        dtu = E[t];
      }
      if (t > 0) dtu = csub(dtu, eprev);
      if (t < nt - 1) eprev = E[t];
      const float iv = invden[t];
      dprev = make_float2((R[t].x + dtu.x + dprev.x) * iv, (R[t].y + dtu.y + dprev.y) * iv);
      R[t] = dprev;
    }
  }
  // back substitution m_t = r'_t + invden_t m_{t+1}; d1 <- e_t + m_{t+1} - m_t
  float2 mnext = make_float2(0.f, 0.f);
#pragma unroll
  for (int t = NT - 1; t >= 0; --t) {
    if (t < nt) {
      float2 mt = R[t];
      if (t < nt - 1) {
        const float iv = invden[t];
        mt = make_float2(fmaf(iv, mnext.x, mt.x), fmaf(iv, mnext.y, mt.y));
        d1[(size_t)t * npix + p] = make_float2(E[t].x + mnext.x - mt.x, E[t].y + mnext.y - mt.y);
      }
      m[(size_t)t * npix + p] = mt;
      mnext = mt;
    }
  }
}

template <int NT>
static void tv_launch(cs_plan* p, float tau, float rho, hipStream_t s) {
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  hipLaunchKernelGGL(k_tv_step<NT>, dim3((unsigned)((npix + 63) / 64)), dim3(64), 0, s, p->s0, p->s1, p->s2,
                     p->s3, p->tv_invden, p->desc.nt, npix, tau, rho);
}

int launch_tv_step(cs_plan* p, float lambda, float mu, hipStream_t s) {
  const float rho = p->desc.mu_ratio;
  const float tau = lambda * rho / (2.0f * mu);  // lambda / (2 mu1), mu1 = mu / rho
  const int nt = p->desc.nt;
  if (nt <= 8) tv_launch<8>(p, tau, rho, s);
  else if (nt <= 16) tv_launch<16>(p, tau, rho, s);
  else if (nt <= 24) tv_launch<24>(p, tau, rho, s);
  else if (nt <= 32) tv_launch<32>(p, tau, rho, s);
  else if (nt <= 40) tv_launch<40>(p, tau, rho, s);
  else if (nt <= 48) tv_launch<48>(p, tau, rho, s);
  else tv_launch<64>(p, tau, rho, s);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// ---------------------------------------------------------------- DFT step
//
// Algorithm 1 with Psi = unitary DFT along frames, one pixel per thread.
// The iteration is split around the x-update so that each half is one pass:
//   this kernel:  w = Psi z  (z = the last x-update output)
//                 d <- d - (w - v)       (dual update of the previous
//                                          iteration; skipped on the first)
//                 v <- soft(w - d, tau),  tau = lambda / (2 mu)
//                 u <- Psi'(v + d)
//   x-update:     z <- (mu I + H'H)^{-1} (H'y + mu u)
// which is the algorithm's order (v, w, d) with the d-update deferred to the
// start of the next pass.  For an orthonormal Psi the frame term
// (1/mu)(I - Psi Psi')[.] of the w-update vanishes.
// On a warm start the saved w is passed as `wgiven` and used as is on the
// first pass (it is the value an uninterrupted run computes there), so a
// resumed solve reproduces the uninterrupted one bit for bit.
template <int NT>
__global__ __launch_bounds__(256) void k_dft_step(const float2* __restrict__ z, float2* __restrict__ d,
                                                  float2* __restrict__ v, float2* __restrict__ u,
                                                  const float2* __restrict__ psi,
                                                  const float2* __restrict__ wgiven, int nt, size_t npix,
                                                  float tau, int first) {
  __shared__ float2 ps[NT * NT];
  for (int q = threadIdx.x; q < nt * nt; q += blockDim.x) ps[q] = psi[q];
  __syncthreads();
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  float2 zz[NT], uu[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    zz[t] = (t < nt && !wgiven) ? z[(size_t)t * npix + p] : make_float2(0.f, 0.f);
    uu[t] = make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int f = 0; f < NT; ++f) {
    if (f < nt) {
      const float2* row = ps + f * nt;
      float2 w = make_float2(0.f, 0.f);
      if (wgiven) {
        w = wgiven[(size_t)f * npix + p];
      } else {
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (t < nt) w = cfma(row[t], zz[t], w);
      }
      float2 df = d[(size_t)f * npix + p];
      if (!first) {
        const float2 vp = v[(size_t)f * npix + p];
        df = make_float2(df.x - (w.x - vp.x), df.y - (w.y - vp.y));
      }
      const float2 vf = soft_threshold(csub(w, df), tau);
      d[(size_t)f * npix + p] = df;
      v[(size_t)f * npix + p] = vf;
      const float2 q = cadd(vf, df);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        if (t < nt) uu[t] = cfmac(row[t], q, uu[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
    if (t < nt) u[(size_t)t * npix + p] = uu[t];
}

// out = Psi in (adjoint = 0) or Psi' in (adjoint = 1); with dual != nullptr
// (forward only) also completes the deferred dual update d <- d - (out - v).
template <int NT>
__global__ __launch_bounds__(256) void k_dft_apply(const float2* __restrict__ in, float2* __restrict__ out,
                                                   float2* __restrict__ dual, const float2* __restrict__ v,
                                                   const float2* __restrict__ psi, int nt, size_t npix,
                                                   int adjoint) {
  __shared__ float2 ps[NT * NT];
  for (int q = threadIdx.x; q < nt * nt; q += blockDim.x) ps[q] = psi[q];
  __syncthreads();
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  float2 a[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) a[t] = t < nt ? in[(size_t)t * npix + p] : make_float2(0.f, 0.f);
#pragma unroll
  for (int f = 0; f < NT; ++f) {
    if (f < nt) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t < nt) {
          // Psi[f][t] is symmetric in (f, t); Psi'[f][t] = conj(Psi[t][f]) = conj(Psi[f][t])
          acc = adjoint ? cfmac(ps[f * nt + t], a[t], acc) : cfma(ps[f * nt + t], a[t], acc);
        }
      }
      out[(size_t)f * npix + p] = acc;
      if (dual) {
        const float2 vf = v[(size_t)f * npix + p];
        float2 df = dual[(size_t)f * npix + p];
        dual[(size_t)f * npix + p] = make_float2(df.x - (acc.x - vf.x), df.y - (acc.y - vf.y));
      }
    }
  }
}

template <int NT>
static void dft_step_launch(cs_plan* p, float tau, int first, const float2* wgiven, hipStream_t s) {
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  hipLaunchKernelGGL(k_dft_step<NT>, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s, p->s2, p->s0,
                     p->s1, p->s3, p->psi_t, wgiven, p->desc.nt, npix, tau, first);
}

template <int NT>
static void dft_apply_launch(cs_plan* p, const float2* in, float2* out, float2* dual, const float2* v,
                             int adjoint, hipStream_t s) {
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  hipLaunchKernelGGL(k_dft_apply<NT>, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s, in, out, dual,
                     v, p->psi_t, p->desc.nt, npix, adjoint);
}

#define CS_DISPATCH_NT(nt, FN, ...)            \
  do {                                         \
    if ((nt) <= 8) FN<8>(__VA_ARGS__);         \
    else if ((nt) <= 16) FN<16>(__VA_ARGS__);  \
    else if ((nt) <= 24) FN<24>(__VA_ARGS__);  \
    else if ((nt) <= 32) FN<32>(__VA_ARGS__);  \
    else if ((nt) <= 40) FN<40>(__VA_ARGS__);  \
    else if ((nt) <= 48) FN<48>(__VA_ARGS__);  \
    else FN<64>(__VA_ARGS__);                  \
  } while (0)

int launch_dft_step(cs_plan* p, float lambda, float mu, int first, const float2* wgiven, hipStream_t s) {
  const float tau = lambda / (2.0f * mu);
  CS_DISPATCH_NT(p->desc.nt, dft_step_launch, p, tau, first, wgiven, s);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_dft_apply(cs_plan* p, const float2* in, float2* out, float2* dual, const float2* v, int adjoint,
                     hipStream_t s) {
  CS_DISPATCH_NT(p->desc.nt, dft_apply_launch, p, in, out, dual, v, adjoint, s);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// ---------------------------------------------------------------- fill

__global__ void k_fill(float2* __restrict__ ptr, size_t n, float2 v) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
    ptr[q] = v;
}

int launch_fill(float2* ptr, size_t n, float2 v, hipStream_t s) {
  if (n == 0) return CS_OK;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, ptr, n, v);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// ---------------------------------------------------------------- objective
//
// J = lambda * l1 + ||y - H x||^2 (eqs. L1an_pri / L1unconst), evaluated in
// hybrid (ky, i) space: F_h is unitary, so the data term equals
// sum_{t,c,r,i} |(M_t F_v (s_c . x))[r, i] - (F_h' y)[r, i]|^2 over sampled
// rows r.  l1 = sum |D_t x| (TV) or sum |Psi x| (DFT), moduli of complex
// values.  Partial sums are FP64 and reduced in a fixed order, so the value
// is bit-reproducible run to run.
constexpr int kJBlocks = 512;
constexpr int kJThreads = 256;

__device__ inline void block_reduce_store(double v, double* out) {
  __shared__ double red[kJThreads];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kJThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

__global__ __launch_bounds__(kJThreads) void k_resid_partial(const float2* __restrict__ f,
                                                             const float2* __restrict__ g,
                                                             const int32_t* __restrict__ mcnt, int nc,
                                                             int m_max, int nh, int nt, double* __restrict__ part) {
  const size_t per_frame = (size_t)nc * m_max * nh;
  const size_t total = per_frame * nt;
  double acc = 0.0;
  for (size_t q = (size_t)blockIdx.x * kJThreads + threadIdx.x; q < total; q += (size_t)kJBlocks * kJThreads) {
    const int t = (int)(q / per_frame);
    const int r = (int)((q / nh) % m_max);
    if (r < mcnt[t]) {
      const float2 a = f[q], b = g[q];
      const double dx = (double)a.x - b.x, dy = (double)a.y - b.y;
      acc += dx * dx + dy * dy;
    }
  }
  block_reduce_store(acc, part + blockIdx.x);
}

__global__ __launch_bounds__(kJThreads) void k_l1_tv_partial(const float2* __restrict__ x, int nt, size_t npix,
                                                             double* __restrict__ part) {
  const size_t total = (size_t)(nt - 1) * npix;
  double acc = 0.0;
  for (size_t q = (size_t)blockIdx.x * kJThreads + threadIdx.x; q < total; q += (size_t)kJBlocks * kJThreads) {
    const float2 a = x[q + npix], b = x[q];
    const double dx = (double)a.x - b.x, dy = (double)a.y - b.y;
    acc += sqrt(dx * dx + dy * dy);
  }
  block_reduce_store(acc, part + blockIdx.x);
}

template <int NT>
__global__ __launch_bounds__(kJThreads) void k_l1_dft_partial(const float2* __restrict__ x,
                                                              const float2* __restrict__ psi, int nt, size_t npix,
                                                              double* __restrict__ part) {
  __shared__ float2 ps[NT * NT];
  for (int q = threadIdx.x; q < nt * nt; q += blockDim.x) ps[q] = psi[q];
  __syncthreads();
  double acc = 0.0;
  for (size_t p = (size_t)blockIdx.x * kJThreads + threadIdx.x; p < npix; p += (size_t)kJBlocks * kJThreads) {
    float2 a[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) a[t] = t < nt ? x[(size_t)t * npix + p] : make_float2(0.f, 0.f);
#pragma unroll
    for (int f = 0; f < NT; ++f) {
      if (f < nt) {
        float2 w = make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (t < nt) w = cfma(ps[f * nt + t], a[t], w);
        acc += sqrt((double)w.x * w.x + (double)w.y * w.y);
      }
    }
  }
  block_reduce_store(acc, part + blockIdx.x);
}

__global__ void k_j_final(const double* __restrict__ part, float lambda, float* __restrict__ out) {
  __shared__ double r[2];
  if (threadIdx.x < 2) {
    double acc = 0.0;
    for (int q = 0; q < kJBlocks; ++q) acc += part[threadIdx.x * kJBlocks + q];
    r[threadIdx.x] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) *out = (float)((double)lambda * r[1] + r[0]);
}

template <int NT>
static void l1_dft_launch(cs_plan* p, const float2* x, hipStream_t s) {
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  hipLaunchKernelGGL(k_l1_dft_partial<NT>, dim3(kJBlocks), dim3(kJThreads), 0, s, x, p->psi_t, p->desc.nt,
                     npix, p->jpart + kJBlocks);
}

// x in solver layout; the plan's ktmp must hold F_h' y (set by the solve setup)
int launch_objective(cs_plan* p, const float2* x, float lambda, float* out, hipStream_t s) {
  const int nh = p->desc.nh, nt = p->desc.nt, nc = p->desc.nc;
  const size_t npix = (size_t)p->desc.nv * nh;
  int st = launch_forward(p, x, true, nullptr, s);
  if (st != CS_OK) return st;
  hipLaunchKernelGGL(k_resid_partial, dim3(kJBlocks), dim3(kJThreads), 0, s, p->ftmp, p->ktmp, p->mcnt, nc,
                     p->m_max, nh, nt, p->jpart);
  if (p->desc.prior == CS_PRIOR_TEMPORAL_TV) {
    hipLaunchKernelGGL(k_l1_tv_partial, dim3(kJBlocks), dim3(kJThreads), 0, s, x, nt, npix,
                       p->jpart + kJBlocks);
  } else {
    CS_DISPATCH_NT(nt, l1_dft_launch, p, x, s);
  }
  hipLaunchKernelGGL(k_j_final, dim3(1), dim3(64), 0, s, p->jpart, lambda, out);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int objective_partial_count() { return 2 * kJBlocks; }

}  // namespace csmri
