// Measurement operator H and its adjoint (Sec. II-A, eqs. mri_mcoil2,
// mri_csmcoill2, H_2):   y_{t,c} = F_h M_t F_v (s_c . x_t).
//
// Forward: a vertical pass (length-nv FFT of every column of s_c . x_t, only
// the sampled ky rows kept) followed by a horizontal pass over the sampled
// rows only, so the horizontal work is 1/R of a full 2D FFT.  Rows ky that a
// frame does not sample are zero-filled by a third, store-only kernel.  The
// adjoint runs the same passes in reverse order.
//
// The vertical passes work on the solver's column-major image layout
// [t][i][j]: one wave owns a group of adjacent columns of one frame, keeps
// them in registers, and runs every coil's transform in an LDS region of its
// own, so no workgroup barrier is involved and each image value is read once
// for all coils (the adjoint sums conj(s_c) . (.) over coils in registers
// before its single store).  Between the two passes the sampled rows live in
// hybrid (ky, i) space as [t][c][i][r] (r < m_max fastest), so the rows of one
// column are contiguous for the vertical passes.  The row-major [t][j][i]
// layout of the boundary goes through a tiled transpose.  Lengths n = 16 M
// (M = 4, 6, 8, 9, 12, 16) take register passes instead of the LDS Stockham
// FFT: a length-M and a length-16 DFT in registers around one LDS transpose.
#include "fft.hpp"
#include "tdft.hpp"

namespace csmri {

bool make_fft_desc(int n, FftDesc* d) {
  if (n < 2 || n > 512) return false;
  int m = n, np = 0;
  // radix-4 passes first (keeping one factor 4 for the tail when possible),
  // then radix 3, then the remaining 4s and at most one 2
  while (m % 4 == 0 && m > 4) { d->radix[np++] = 4; m /= 4; }
  while (m % 3 == 0) { d->radix[np++] = 3; m /= 3; }
  while (m % 4 == 0) { d->radix[np++] = 4; m /= 4; }
  while (m % 2 == 0) { d->radix[np++] = 2; m /= 2; }
  if (m != 1 || np > kMaxFftPasses) return false;
  d->n = n;
  d->npass = np;
  return true;
}

// ---------------------------------------------------------------- kernels

constexpr int kVWaves = 4;  // waves per workgroup of the vertical passes
// A column group holds at most WE = 256 or 512 values (WE / 64 per lane); the
// kernels are compiled for both so that groups of up to 256 values carry half
// the registers.

// Per-lane part of a column group: element e = lane + 64 q of the group's
// ncol * nv values, which sit contiguously in the column-major image.
struct ColGroup {
  int t, i0, ncol, tot;
};

__device__ __forceinline__ ColGroup col_group(int u, int ngrp, int cw, int nv, int nh) {
  ColGroup g;
  g.t = u / ngrp;
  g.i0 = (u - g.t * ngrp) * cw;
  g.ncol = min(cw, nh - g.i0);
  g.tot = g.ncol * nv;
  return g;
}

// MODE kFwdStore:    hyb[t][c][i][r] = (1/sqrt nv) (F_v (s_c . x_t))[rows[t][r], i]
// MODE kFwdResidual: sum over (t, c, i, r < mcnt[t]) of |that value - ref[t][c][i][r]|^2,
//                    one FP64 partial per workgroup (grid-stride over column
//                    groups with a fixed grid, so the sum is reproducible);
//                    with tvl > 0 the partials also hold tvl * sum |x[t+1] - x[t]|
//                    over the group's pixels (t < nt - 1), from the image values
//                    the pass holds anyway
constexpr int kFwdStore = 0, kFwdResidual = 1;

// FP64 |a - b| of complex values
__device__ __forceinline__ double cabs_diff(float2 a, float2 b) {
  const double dx = (double)a.x - b.x, dy = (double)a.y - b.y;
  return sqrt(dx * dx + dy * dy);
}

// one FP64 partial per workgroup: fixed tree over its threads
template <int NT>
__device__ __forceinline__ void store_block_partial(double v, double* __restrict__ part) {
  __shared__ double red[NT];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

template <int MODE, int WE>
__global__ __launch_bounds__(64 * kVWaves) void k_fwd_vertical(
    const float2* __restrict__ x, const float2* __restrict__ coil_cm, float2* __restrict__ hyb,
    const float2* __restrict__ ref, const int32_t* __restrict__ rows, const int32_t* __restrict__ mcnt,
    FftDesc fv, const float2* __restrict__ twv, int nv, int nh, int nt, int nc, int m_max, int cw, float scale,
    float tvl, double* __restrict__ part) {
  constexpr int kVE = WE / 64;  // image values per lane of one column group
  extern __shared__ float2 lds[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float2* tw = lds;
  float2* buf = lds + nv + (size_t)wv * cw * nv;
  for (int q = threadIdx.x; q < nv; q += blockDim.x) tw[q] = twv[q];
  __syncthreads();
  const int ngrp = (nh + cw - 1) / cw;
  const int units = nt * ngrp;
  double acc = 0.0, l1 = 0.0;
  for (int u = blockIdx.x * kVWaves + wv; u < units; u += gridDim.x * kVWaves) {
    const ColGroup g = col_group(u, ngrp, cw, nv, nh);
    const float2* xs = x + ((size_t)g.t * nh + g.i0) * nv;
    float2 xv[kVE], cv[kVE];
#pragma unroll
    for (int q = 0; q < kVE; ++q) {
      const int e = lane + 64 * q;
      xv[q] = e < g.tot ? xs[e] : make_float2(0.f, 0.f);
      cv[q] = e < g.tot ? coil_cm[(size_t)g.i0 * nv + e] : make_float2(0.f, 0.f);
    }
    if (MODE == kFwdResidual && tvl > 0.f && g.t + 1 < nt) {
      const float2* xn = xs + (size_t)nh * nv;
#pragma unroll
      for (int q = 0; q < kVE; ++q) {
        const int e = lane + 64 * q;
        if (e < g.tot) l1 += cabs_diff(xn[e], xv[q]);
      }
    }
    const int m = mcnt[g.t];
    const int32_t* rw = rows + (size_t)g.t * m_max;
    const float inv_m = 1.0f / (float)max(m, 1);
    for (int c = 0; c < nc; ++c) {
#pragma unroll
      for (int q = 0; q < kVE; ++q) {
        const int e = lane + 64 * q;
        if (e < g.tot) buf[e] = cmul(cv[q], xv[q]);
      }
      // the next coil's values are requested before this coil's transform
      if (c + 1 < nc) {
        const float2* cs = coil_cm + ((size_t)(c + 1) * nh + g.i0) * nv;
#pragma unroll
        for (int q = 0; q < kVE; ++q) {
          const int e = lane + 64 * q;
          if (e < g.tot) cv[q] = cs[e];
        }
      }
      __builtin_amdgcn_wave_barrier();
      fft_wave<-1, WE>(buf, fv, tw, g.ncol, nv, lane);
      const size_t ob = (((size_t)g.t * nc + c) * nh + g.i0) * m_max;
      for (int e = lane; e < g.ncol * m; e += 64) {
        int r;
        const int col = fast_div(e, m, inv_m, r);
        const float2 v = cscale(buf[col * nv + rw[r]], scale);
        if constexpr (MODE == kFwdStore) {
          hyb[ob + (size_t)col * m_max + r] = v;
        } else {
          const float2 b = ref[ob + (size_t)col * m_max + r];
          const double dx = (double)v.x - b.x, dy = (double)v.y - b.y;
          acc += dx * dx + dy * dy;
        }
      }
      __builtin_amdgcn_wave_barrier();  // the next coil overwrites buf
    }
  }
  if constexpr (MODE == kFwdResidual) store_block_partial<64 * kVWaves>(acc + (double)tvl * l1, part);
}

// y[t][c][rows[t][r]][:] = (1/sqrt nh) F_h hyb[t][c][:][r]
__global__ __launch_bounds__(kFftThreads) void k_fwd_horizontal(
    const float2* __restrict__ hyb, float2* __restrict__ y, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ mcnt, FftDesc fh, const float2* __restrict__ twh, int nv, int nh,
    int nc, int m_max, int rb, float scale) {
  extern __shared__ float2 lds[];
  float2* tw = lds;
  float2* buf = lds + nh;
  const int stride = nh + 1;
  const int r0 = blockIdx.x * rb, t = blockIdx.y, c = blockIdx.z;
  const int nrow = min(rb, mcnt[t] - r0);
  if (nrow <= 0) return;  // uniform over the workgroup
  const float inv_nh = 1.0f / (float)nh, inv_nrow = 1.0f / (float)nrow;
  for (int q = threadIdx.x; q < nh; q += kFftThreads) tw[q] = twh[q];
  const float2* src = hyb + ((size_t)(t * nc + c) * nh) * m_max + r0;
  for (int e = threadIdx.x; e < nrow * nh; e += kFftThreads) {
    int rr;
    const int i = fast_div(e, nrow, inv_nrow, rr);
    buf[rr * stride + i] = src[(size_t)i * m_max + rr];
  }
  __syncthreads();
  fft_lds<-1>(buf, fh, tw, nrow, stride);
  const int32_t* rw = rows + (size_t)t * m_max + r0;
  for (int e = threadIdx.x; e < nrow * nh; e += kFftThreads) {
    int i;
    const int rr = fast_div(e, nh, inv_nh, i);
    y[((size_t)(t * nc + c) * nv + rw[rr]) * nh + i] = cscale(buf[rr * stride + i], scale);
  }
}

// zero the rows ky that frame t does not sample
__global__ void k_zero_unsampled(float2* __restrict__ y, const uint8_t* __restrict__ mask, int nv,
                                 int nh, int nc) {
  const int ky = blockIdx.x, t = blockIdx.y, c = blockIdx.z;
  if (mask[(size_t)t * nv + ky]) return;
  float2* line = y + ((size_t)(t * nc + c) * nv + ky) * nh;
  for (int i = threadIdx.x; i < nh; i += blockDim.x) line[i] = make_float2(0.f, 0.f);
}

// hyb[t][c][:][r] = (1/sqrt nh) F_h' y[t][c][rows[t][r]][:]   (hybrid space)
__global__ __launch_bounds__(kFftThreads) void k_adj_horizontal(
    const float2* __restrict__ y, float2* __restrict__ hyb, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ mcnt, FftDesc fh, const float2* __restrict__ twh, int nv, int nh,
    int nc, int m_max, int rb, float scale) {
  extern __shared__ float2 lds[];
  float2* tw = lds;
  float2* buf = lds + nh;
  const int stride = nh + 1;
  const int r0 = blockIdx.x * rb, t = blockIdx.y, c = blockIdx.z;
  const int nrow = min(rb, mcnt[t] - r0);
  if (nrow <= 0) return;
  const float inv_nh = 1.0f / (float)nh, inv_nrow = 1.0f / (float)nrow;
  for (int q = threadIdx.x; q < nh; q += kFftThreads) tw[q] = twh[q];
  const int32_t* rw = rows + (size_t)t * m_max + r0;
  for (int e = threadIdx.x; e < nrow * nh; e += kFftThreads) {
    int i;
    const int rr = fast_div(e, nh, inv_nh, i);
    buf[rr * stride + i] = y[((size_t)(t * nc + c) * nv + rw[rr]) * nh + i];
  }
  __syncthreads();
  fft_lds<+1>(buf, fh, tw, nrow, stride);
  float2* dst = hyb + ((size_t)(t * nc + c) * nh) * m_max + r0;
  for (int e = threadIdx.x; e < nrow * nh; e += kFftThreads) {
    int rr;
    const int i = fast_div(e, nrow, inv_nrow, rr);
    dst[(size_t)i * m_max + rr] = cscale(buf[rr * stride + i], scale);
  }
}

// x_t[:, i] = (1/sqrt nv) sum_c conj(s_c[:, i]) . F_v' (column i of hyb[t][c],
// zero-filled at the rows the frame does not sample); x column-major
template <int WE>
__global__ __launch_bounds__(64 * kVWaves) void k_adj_vertical(
    const float2* __restrict__ hyb, const float2* __restrict__ coil_cm, float2* __restrict__ x,
    const int32_t* __restrict__ rows, const int32_t* __restrict__ mcnt, FftDesc fv,
    const float2* __restrict__ twv, int nv, int nh, int nt, int nc, int m_max, int cw, float scale) {
  constexpr int kVE = WE / 64;  // image values per lane of one column group
  extern __shared__ float2 lds[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float2* tw = lds;
  float2* buf = lds + nv + (size_t)wv * cw * nv;
  for (int q = threadIdx.x; q < nv; q += blockDim.x) tw[q] = twv[q];
  __syncthreads();
  const int ngrp = (nh + cw - 1) / cw;
  const int units = nt * ngrp;
  for (int u = blockIdx.x * kVWaves + wv; u < units; u += gridDim.x * kVWaves) {
    const ColGroup g = col_group(u, ngrp, cw, nv, nh);
    const int m = mcnt[g.t];
    const int32_t* rw = rows + (size_t)g.t * m_max;
    const float inv_m = 1.0f / (float)max(m, 1);
    float2 acc[kVE];
#pragma unroll
    for (int q = 0; q < kVE; ++q) acc[q] = make_float2(0.f, 0.f);
    for (int c = 0; c < nc; ++c) {
      const float2* cs = coil_cm + ((size_t)c * nh + g.i0) * nv;
      float2 cv[kVE];
#pragma unroll
      for (int q = 0; q < kVE; ++q) {
        const int e = lane + 64 * q;
        cv[q] = e < g.tot ? cs[e] : make_float2(0.f, 0.f);
        if (e < g.tot) buf[e] = make_float2(0.f, 0.f);
      }
      __builtin_amdgcn_wave_barrier();
      const float2* src = hyb + (((size_t)g.t * nc + c) * nh + g.i0) * m_max;
      for (int e = lane; e < g.ncol * m; e += 64) {
        int r;
        const int col = fast_div(e, m, inv_m, r);
        buf[col * nv + rw[r]] = src[(size_t)col * m_max + r];
      }
      __builtin_amdgcn_wave_barrier();
      fft_wave<+1, WE>(buf, fv, tw, g.ncol, nv, lane);
#pragma unroll
      for (int q = 0; q < kVE; ++q) {
        const int e = lane + 64 * q;
        if (e < g.tot) acc[q] = cfmac(cv[q], buf[e], acc[q]);
      }
      __builtin_amdgcn_wave_barrier();  // the next coil overwrites buf
    }
    float2* xs = x + ((size_t)g.t * nh + g.i0) * nv;
#pragma unroll
    for (int q = 0; q < kVE; ++q) {
      const int e = lane + 64 * q;
      if (e < g.tot) xs[e] = cscale(acc[q], scale);
    }
  }
}

// ---------------------------------------------------------------- register passes, n = 16 M
//
// n = 16 M (M <= 16 a product of 2, 3 and 5; n_v for the vertical passes, n_h
// for the horizontal ones): input index 16 n1 + q (q < 16, n1 < M), output
// index k1 + M k2 (k1 < M, k2 < 16).  Lane q of a 16-lane line holds the M
// inputs 16 n1 + q, runs the length-M DFT over n1 in registers, multiplies
// by exp(SIGN 2 pi i q k1 / n) (the workgroup's LDS copy of the table), and
// after one transpose through LDS (rows padded to 17 values) lane k1 < M holds
// the 16 values of k1 over q, which a length-16 DFT transforms into the
// outputs k1 + M k2 (lanes k1 >= M carry no output).  A wave holds 4 lines.
// For the vertical passes the sampled rows move between hybrid storage and the
// lanes through the frame's row index rinv[t][ky] (r, or -1 for an unsampled
// ky), so no zero-filled buffer is built.  Results agree with the generic
// mixed-radix passes to rounding (not bit for bit: another butterfly order).
constexpr int kV256Cols = 4;                   // lines (readout columns or sampled rows) per wave
constexpr int kV256Lds = kV256Cols * 16 * 17;  // transpose buffer values per wave

constexpr bool reg16_ok(int n) { return n % 16 == 0 && tdft_len_ok(n / 16); }

struct Lane256 {
  int b, q;
};
__device__ __forceinline__ Lane256 lane256(int lane) { return Lane256{lane >> 4, lane & 15}; }

// the workgroup's copy of the table exp(-2 pi i m / n), m < n, at the start
// of its LDS (all threads; ends with a barrier)
__device__ __forceinline__ void stage_twiddles(float2* twl, const float2* __restrict__ tw, int n) {
  for (int m = threadIdx.x; m < n; m += blockDim.x) twl[m] = tw[m];
  __syncthreads();
}

// v[n1] (n1 < M): inputs 16 n1 + q in; v[k2] (k2 < 16) on lanes q < M: the
// outputs q + M k2 of the transform (unnormalised); the twiddles exp(SIGN 2
// pi i q k1 / 16 M) come from the LDS table.  Every lane of the wave takes
// part (lanes q >= M read a real lane's buffer row and hold no output).
template <int M, int SIGN>
__device__ __forceinline__ void fft16m_lanes(float2 (&v)[16], const float2* twl, float2* tbuf, Lane256 L) {
  if constexpr (M == 16) {
    dft16_regs<SIGN>(v);
  } else {
    float2 a[M];
#pragma unroll
    for (int n = 0; n < M; ++n) a[n] = v[n];
    dft_reg<M, SIGN>(a);
#pragma unroll
    for (int n = 0; n < M; ++n) v[n] = a[n];
  }
#pragma unroll
  for (int k1 = 1; k1 < M; ++k1) {
    const float2 t = twl[L.q * k1];  // q k1 < 16 M
    v[k1] = SIGN < 0 ? cmul(v[k1], t) : cmulc(t, v[k1]);
  }
  float2* tb = tbuf + L.b * (16 * 17);
#pragma unroll
  for (int k1 = 0; k1 < M; ++k1) tb[k1 * 17 + L.q] = v[k1];
  __builtin_amdgcn_wave_barrier();
  const int r = min(L.q, M - 1);
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) v[n2] = tb[r * 17 + n2];
  __builtin_amdgcn_wave_barrier();  // the buffer is rewritten by the next transform
  dft16_regs<SIGN>(v);
}

// adjoint vertical pass at n_v = 16 M (as k_adj_vertical).  With csplit > 1
// (1, 2 or 4) the csplit waves of a workgroup slot share one column group and
// take contiguous coil ranges each; their sums meet in LDS and are added in
// wave order, so the result depends on csplit but not on the launch.
template <int M>
__global__ __launch_bounds__(64 * kVWaves) void k_adj_vertical16m(
    const float2* __restrict__ hyb, const float2* __restrict__ coil_cm, float2* __restrict__ x,
    const int32_t* __restrict__ rinv, const float2* __restrict__ twv, int nh, int nt, int nc, int m_max,
    int csplit, float scale) {
  constexpr int NV = 16 * M;
  extern __shared__ float2 lds[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const Lane256 L = lane256(lane);
  const bool owner = L.q < M;        // the lane holds output rows L.q + M k2
  const int qo = min(L.q, M - 1);    // a valid row for the lanes that hold none
  float2* twl = lds;
  float2* tbuf = lds + NV + (size_t)wv * kV256Lds;
  stage_twiddles(twl, twv, NV);
  const int upb = kVWaves / csplit;  // column groups per workgroup pass
  const int slot = wv / csplit, part = wv - slot * csplit;
  const int c0 = part * nc / csplit, c1 = (part + 1) * nc / csplit;
  const int ngrp = (nh + kV256Cols - 1) / kV256Cols;
  const int units = nt * ngrp;
  // the trip count is uniform over the workgroup (the reduction's barriers)
  for (int ub = blockIdx.x * upb; ub < units; ub += gridDim.x * upb) {
    const int u = ub + slot;
    const int t = min(u, units - 1) / ngrp;
    const int i = (u - t * ngrp) * kV256Cols + L.b;
    const bool active = u < units && i < nh;
    int rr[M];
#pragma unroll
    for (int n1 = 0; n1 < M; ++n1) rr[n1] = active ? rinv[(size_t)t * NV + 16 * n1 + L.q] : -1;
    float2 acc[16];
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) acc[k2] = make_float2(0.f, 0.f);
    // coil c + 1's hybrid rows are requested before coil c is transformed,
    // and coil c's map values (used after the transform) at its start: the
    // latency hides behind the transform (two waves per SIMD cannot hide it
    // otherwise)
    const int ic = active ? i : 0;
    float2 hn[M];
    auto fetch_rows = [&](int c) {
      const float2* src = hyb + (((size_t)t * nc + c) * nh + ic) * m_max;
#pragma unroll
      for (int n = 0; n < M; ++n) hn[n] = rr[n] >= 0 ? src[rr[n]] : make_float2(0.f, 0.f);
    };
    if (c0 < c1) fetch_rows(c0);
    for (int c = c0; c < c1; ++c) {
      float2 v[16], sv[16];
#pragma unroll
      for (int n = 0; n < M; ++n) v[n] = hn[n];
      if (c + 1 < c1) fetch_rows(c + 1);
      const float2* cs = coil_cm + ((size_t)c * nh + ic) * NV + qo;
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) sv[k2] = active ? cs[M * k2] : make_float2(0.f, 0.f);
      fft16m_lanes<M, +1>(v, twl, tbuf, L);
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) acc[k2] = cfmac(sv[k2], v[k2], acc[k2]);
    }
    if (csplit == 1) {
      if (active && owner) {
        float2* xs = x + ((size_t)t * nh + i) * NV + L.q;
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) xs[M * k2] = cscale(acc[k2], scale);
      }
      continue;
    }
    // 64 x 16 partial sums per wave in its own transpose buffer (free after
    // the last transform); wave `part` of the slot adds outputs k2 in
    // [part * 16 / csplit, (part + 1) * 16 / csplit) over the slot's waves
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) tbuf[k2 * 64 + lane] = acc[k2];
    __syncthreads();
    const int kq = 16 / csplit, k0 = part * kq;
    if (active && owner) {
      const float2* red = lds + NV + (size_t)(slot * csplit) * kV256Lds;
      float2* xs = x + ((size_t)t * nh + i) * NV + L.q;
      for (int k2 = k0; k2 < k0 + kq; ++k2) {
        float2 a = red[k2 * 64 + lane];
        for (int w = 1; w < csplit; ++w) a = cadd(a, red[(size_t)w * kV256Lds + k2 * 64 + lane]);
        xs[M * k2] = cscale(a, scale);
      }
    }
    __syncthreads();  // the next pass rewrites the buffers
  }
}

// forward vertical pass at n_v = 16 M (as k_fwd_vertical, both modes).  After
// each transform the lanes drop their sampled outputs into the (then free)
// transpose buffer at slot r of their column, and the wave walks the m
// sampled values of its columns in r order: hybrid rows are stored (or
// compared with the reference rows) contiguously, and the FP64 residual is
// formed for the sampled values only.  A unit of work is a column group of
// one frame and one of csplit contiguous coil ranges (each coil's rows are
// its own, so the stored rows do not depend on csplit).
template <int M, int MODE>
__global__ __launch_bounds__(64 * kVWaves) void k_fwd_vertical16m(
    const float2* __restrict__ x, const float2* __restrict__ coil_cm, float2* __restrict__ hyb,
    const float2* __restrict__ ref, const int32_t* __restrict__ rinv, const int32_t* __restrict__ mcnt,
    const float2* __restrict__ twv, int nh, int nt, int nc, int m_max, int csplit, float scale, float tvl,
    double* __restrict__ part) {
  constexpr int NV = 16 * M;
  extern __shared__ float2 lds[];
  const int wv = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const Lane256 L = lane256(lane);
  const bool owner = L.q < M;  // the lane holds output rows L.q + M k2
  float2* twl = lds;
  float2* tbuf = lds + NV + (size_t)wv * kV256Lds;
  stage_twiddles(twl, twv, NV);
  const int ngrp = (nh + kV256Cols - 1) / kV256Cols;
  const int units = nt * ngrp * csplit;  // (frame, column group, coil range)
  double acc = 0.0, l1 = 0.0;
  for (int u = blockIdx.x * kVWaves + wv; u < units; u += gridDim.x * kVWaves) {
    const int g = u / csplit, cp = u - g * csplit;
    const int c0 = cp * nc / csplit, c1 = (cp + 1) * nc / csplit;
    const int t = g / ngrp;
    const int i0 = (g - t * ngrp) * kV256Cols;  // first column of the group
    const int i = i0 + L.b;
    const bool active = i < nh;
    const int m = mcnt[t];
    const int ncol = min(kV256Cols, nh - i0);
    // image rows 16 n1 + q of column i; hybrid row index of the output rows q + M k2
    float2 xv[M];
    int ro[16];
    const float2* xs = x + ((size_t)t * nh + (active ? i : 0)) * NV + L.q;
#pragma unroll
    for (int n1 = 0; n1 < M; ++n1) xv[n1] = active ? xs[16 * n1] : make_float2(0.f, 0.f);
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) ro[k2] = (active && owner) ? rinv[(size_t)t * NV + L.q + M * k2] : -1;
    if (MODE == kFwdResidual && tvl > 0.f && active && cp == 0 && t + 1 < nt) {
      const float2* xn = xs + (size_t)nh * NV;
#pragma unroll
      for (int n1 = 0; n1 < M; ++n1) l1 += cabs_diff(xn[16 * n1], xv[n1]);
    }
    // coil c + 1's map values are requested before coil c is transformed
    const int ic = active ? i : 0;
    float2 sn[M];
    auto fetch_coil = [&](int c) {
      const float2* cs = coil_cm + ((size_t)c * nh + ic) * NV + L.q;
#pragma unroll
      for (int n = 0; n < M; ++n) sn[n] = active ? cs[16 * n] : make_float2(0.f, 0.f);
    };
    if (c0 < c1) fetch_coil(c0);
    for (int c = c0; c < c1; ++c) {
      float2 v[16];
#pragma unroll
      for (int n = 0; n < M; ++n) v[n] = cmul(sn[n], xv[n]);
      if (c + 1 < c1) fetch_coil(c + 1);
      fft16m_lanes<M, -1>(v, twl, tbuf, L);
      float2* slots = tbuf + L.b * (16 * 17);
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2)
        if (ro[k2] >= 0) slots[ro[k2]] = cscale(v[k2], scale);
      __builtin_amdgcn_wave_barrier();
      const size_t ob0 = ((size_t)t * nc + c) * nh + i0;
      for (int e = lane; e < ncol * m; e += 64) {
        const int b = e / m, r = e - b * m;
        const float2 val = tbuf[b * (16 * 17) + r];
        const size_t o = (ob0 + b) * m_max + r;
        if constexpr (MODE == kFwdStore) {
          hyb[o] = val;
        } else {
          const float2 bref = ref[o];
          const double dx = (double)val.x - bref.x, dy = (double)val.y - bref.y;
          acc += dx * dx + dy * dy;
        }
      }
      __builtin_amdgcn_wave_barrier();  // the next transform rewrites the buffer
    }
  }
  if constexpr (MODE == kFwdResidual) store_block_partial<64 * kVWaves>(acc + (double)tvl * l1, part);
}

// Horizontal passes at n_h = 16 M: a workgroup of 4 waves owns 16 sampled rows
// of one (frame, coil); lane (b, q) of wave w holds row 4 w + b.  The hybrid
// side [i][r] goes through a workgroup LDS tile of 16 rows x (n_h + 1) values,
// so hybrid rows move as 16 contiguous values per readout column.
constexpr int kH256Rows = 16;  // sampled rows per workgroup
constexpr size_t kLds16m = (256 + (size_t)kVWaves * kV256Lds) * sizeof(float2);  // any M <= 16
static_assert(kH256Rows * 257 <= kVWaves * kV256Lds, "the row tile reuses the transform buffers");

// hyb[t][c][i][r] = (1/sqrt nh) F_h' y[t][c][rows[t][r]][i]
template <int M>
__global__ __launch_bounds__(64 * kVWaves) void k_adj_horizontal16m(
    const float2* __restrict__ y, float2* __restrict__ hyb, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ mcnt, const float2* __restrict__ twh, int nv, int nc, int m_max, float scale) {
  constexpr int NH = 16 * M, STRIDE = NH + 1;
  extern __shared__ float2 lds[];
  const int r0 = blockIdx.x * kH256Rows, t = blockIdx.y, c = blockIdx.z;
  const int m = mcnt[t];
  if (r0 >= m) return;  // uniform over the workgroup
  const int wv = threadIdx.x >> 6;
  const Lane256 L = lane256(threadIdx.x & 63);
  float2* twl = lds;
  float2* tiles = lds + NH;
  float2* tbuf = tiles + (size_t)wv * kV256Lds;
  stage_twiddles(twl, twh, NH);
  const int R = 4 * wv + L.b;  // row of the tile
  const bool active = r0 + R < m;
  float2 v[16];
  {
    const int ky = active ? rows[(size_t)t * m_max + r0 + R] : 0;
    const float2* src = y + ((size_t)(t * nc + c) * nv + ky) * NH + L.q;
#pragma unroll
    for (int n1 = 0; n1 < M; ++n1) v[n1] = active ? src[16 * n1] : make_float2(0.f, 0.f);
  }
  fft16m_lanes<M, +1>(v, twl, tbuf, L);
  __syncthreads();  // every wave is done with its transform buffer
  if (L.q < M) {
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) tiles[R * STRIDE + L.q + M * k2] = cscale(v[k2], scale);
  }
  __syncthreads();
  const int nrow = min(kH256Rows, m - r0);
  float2* dst = hyb + ((size_t)(t * nc + c) * NH) * m_max + r0;
  for (int e = threadIdx.x; e < NH * kH256Rows; e += 64 * kVWaves) {
    const int rr = e & (kH256Rows - 1), i = e >> 4;
    if (rr < nrow) dst[(size_t)i * m_max + rr] = tiles[rr * STRIDE + i];
  }
}

// y[t][c][rows[t][r]][:] = (1/sqrt nh) F_h hyb[t][c][:][r]
template <int M>
__global__ __launch_bounds__(64 * kVWaves) void k_fwd_horizontal16m(
    const float2* __restrict__ hyb, float2* __restrict__ y, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ mcnt, const float2* __restrict__ twh, int nv, int nc, int m_max, float scale) {
  constexpr int NH = 16 * M, STRIDE = NH + 1;
  extern __shared__ float2 lds[];
  const int r0 = blockIdx.x * kH256Rows, t = blockIdx.y, c = blockIdx.z;
  const int m = mcnt[t];
  if (r0 >= m) return;  // uniform over the workgroup
  const int wv = threadIdx.x >> 6;
  const Lane256 L = lane256(threadIdx.x & 63);
  float2* twl = lds;
  float2* tiles = lds + NH;
  float2* tbuf = tiles + (size_t)wv * kV256Lds;
  for (int q = threadIdx.x; q < NH; q += blockDim.x) twl[q] = twh[q];
  const int nrow = min(kH256Rows, m - r0);
  const float2* src = hyb + ((size_t)(t * nc + c) * NH) * m_max + r0;
  for (int e = threadIdx.x; e < NH * kH256Rows; e += 64 * kVWaves) {
    const int rr = e & (kH256Rows - 1), i = e >> 4;
    tiles[rr * STRIDE + i] = rr < nrow ? src[(size_t)i * m_max + rr] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int R = 4 * wv + L.b;
  float2 v[16];
#pragma unroll
  for (int n1 = 0; n1 < M; ++n1) v[n1] = tiles[R * STRIDE + 16 * n1 + L.q];
  __syncthreads();  // the transform buffers overlay the tile
  fft16m_lanes<M, -1>(v, twl, tbuf, L);
  if (R < nrow && L.q < M) {
    float2* dst = y + ((size_t)(t * nc + c) * nv + rows[(size_t)t * m_max + r0 + R]) * NH + L.q;
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) dst[M * k2] = cscale(v[k2], scale);
  }
}

// out[f][c][r] = in[f][r][c]
__global__ void k_transpose(const float2* __restrict__ in, float2* __restrict__ out, int R, int C) {
  __shared__ float2 tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const size_t f = blockIdx.z;
  const float2* src = in + f * (size_t)R * C;
  float2* dst = out + f * (size_t)R * C;
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    const int r = r0 + yy, c = c0 + threadIdx.x;
    if (r < R && c < C) tile[yy][threadIdx.x] = src[(size_t)r * C + c];
  }
  __syncthreads();
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    const int c = c0 + yy, r = r0 + threadIdx.x;
    if (r < R && c < C) dst[(size_t)c * R + r] = tile[threadIdx.x][yy];
  }
}

// ---------------------------------------------------------------- launchers

static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// columns per wave of the vertical passes: by default the most that fit 256
// values (one column when nv > 256), or the plan's tuned choice of at most
// fft_cols_limit; sampled rows per workgroup of the horizontal passes: the
// most that fit kFftElems values, or the plan's tuned (smaller) choice
int fft_cols_limit(const cs_plan* p) { return std::max(1, std::min(p->desc.nh, kWaveElems / p->desc.nv)); }
int fft_cols_per_group(const cs_plan* p) {
  if (p->fft_cw > 0) return std::min(p->fft_cw, fft_cols_limit(p));
  return std::max(1, std::min(p->desc.nh, 256 / p->desc.nv));
}
int fft_rows_per_group(const cs_plan* p) {
  const int full = std::max(1, std::min(p->m_max, kFftElems / p->desc.nh));
  return p->fft_rb > 0 ? std::min(p->fft_rb, full) : full;
}

int launch_transpose(const float2* in, float2* out, int frames, int rows, int cols, hipStream_t s) {
  if (frames <= 0) return CS_OK;
  dim3 grid(ceil_div(cols, 32), ceil_div(rows, 32), frames);
  hipLaunchKernelGGL(k_transpose, grid, dim3(32, 8), 0, s, in, out, rows, cols);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

static size_t vertical_lds(const cs_plan* p, int cw) {
  return (size_t)(p->desc.nv + kVWaves * cw * p->desc.nv) * sizeof(float2);
}

// one wave per column group: enough workgroups for every group, at most 65535
static unsigned vertical_grid(const cs_plan* p, int cw) {
  const size_t units = (size_t)p->desc.nt * ceil_div(p->desc.nh, cw);
  return (unsigned)std::min<size_t>((units + kVWaves - 1) / kVWaves, 65535);
}

// register passes (n = 16 M): blocks of kVWaves waves, one wave per group of
// kV256Cols columns of one frame and one of csplit coil ranges (at most 65535
// blocks; the kernels loop over further groups)
static unsigned grid16m(int nh, int nt, int csplit) {
  const size_t units = (size_t)nt * ((nh + kV256Cols - 1) / kV256Cols) * csplit;
  return (unsigned)std::min<size_t>((units + kVWaves - 1) / kVWaves, 65535);
}

// Coil ranges per column group of the register vertical passes.  A lone wave
// per column group walking all coils leaves the chip short of waves when
// there are many coils and few frames or columns; then 2 or 4 waves share a
// group's coil loop (each keeping at least 2 coils).  A function of the shape
// only, so every caller of a pass on one shape gets the same split and the
// same rounding.  The thresholds are measured (A, A', J, same box):
//   groups x coils -> split: effect
//   384 x 8, 512 x 16, 704 x 32 -> 4: 25-55% faster;  1024 x 16 -> 2: 17-33% faster;
//   1152 x 12 -> 2: A' 7% slower;  1920 x 12 -> 4, 2048 x 8 -> 2: 5-25% slower
// (the extra image loads and the LDS reduction cost more than the waves gain).
constexpr int kSplitMaxGroups = 1024, kSplit4MaxGroups = 767;
int coil_split16(int nh, int nt, int nc) {
  const size_t groups = (size_t)nt * ((nh + kV256Cols - 1) / kV256Cols);
  if (groups > (size_t)kSplitMaxGroups || nc < 4) return 1;
  return groups <= (size_t)kSplit4MaxGroups && nc >= 8 ? 4 : 2;
}

// the sizes that take the register passes: n = 16 M for M = 4, 6, 8, 9, 12,
// 16 (n = 64 ... 256 among the supported sizes; smaller M would leave most
// lanes of the second transform idle)
bool reg16_size(int n) {
  const int m = n / 16;
  return n % 16 == 0 && (m == 4 || m == 6 || m == 8 || m == 9 || m == 12 || m == 16);
}
template <class F>
static void reg16_switch(int n, F&& f) {
  switch (n / 16) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 12: f(std::integral_constant<int, 12>{}); break;
    default: f(std::integral_constant<int, 16>{}); break;
  }
}

int launch_forward(cs_plan* p, const float2* x, bool x_colmajor, float2* y, hipStream_t s) {
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt, nc = p->desc.nc;
  if (p->m_max > 0) {
    if (!x_colmajor) {
      int st = launch_transpose(x, p->img_tmp, nt, nv, nh, s);
      if (st != CS_OK) return st;
      x = p->img_tmp;
    }
    const int cw = fft_cols_per_group(p);
    const float sv = 1.0f / std::sqrt((float)nv), sh = 1.0f / std::sqrt((float)nh);
    if (reg16_size(nv)) {
      reg16_switch(nv, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        const int cs = coil_split16(nh, nt, nc);
        hipLaunchKernelGGL((k_fwd_vertical16m<M, kFwdStore>), dim3(grid16m(nh, nt, cs)), dim3(64 * kVWaves), kLds16m,
                           s, x, p->coil_cm, p->ftmp, nullptr, p->rinv, p->mcnt, p->tw_v, nh, nt, nc, p->m_max, cs, sv,
                           0.f, nullptr);
      });
    } else {
      auto k = cw * nv <= 256 ? k_fwd_vertical<kFwdStore, 256> : k_fwd_vertical<kFwdStore, 512>;
      hipLaunchKernelGGL(k, dim3(vertical_grid(p, cw)), dim3(64 * kVWaves), vertical_lds(p, cw), s, x, p->coil_cm,
                         p->ftmp, nullptr, p->rows, p->mcnt, p->fft_v, p->tw_v, nv, nh, nt, nc, p->m_max, cw, sv,
                         0.f, nullptr);
    }
    CS_HIP(hipGetLastError());
    if (y && reg16_size(nh)) {
      reg16_switch(nh, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        hipLaunchKernelGGL((k_fwd_horizontal16m<M>), dim3(ceil_div(p->m_max, kH256Rows), nt, nc), dim3(64 * kVWaves),
                           kLds16m, s, p->ftmp, y, p->rows, p->mcnt, p->tw_h, nv, nc, p->m_max, sh);
      });
      CS_HIP(hipGetLastError());
    } else if (y) {
      const int rb = fft_rows_per_group(p);
      const size_t lds2 = (size_t)(nh + rb * (nh + 1)) * sizeof(float2);
      dim3 g2(ceil_div(p->m_max, rb), nt, nc);
      hipLaunchKernelGGL(k_fwd_horizontal, g2, dim3(kFftThreads), lds2, s, p->ftmp, y, p->rows, p->mcnt,
                         p->fft_h, p->tw_h, nv, nh, nc, p->m_max, rb, sh);
      CS_HIP(hipGetLastError());
    }
  }
  if (y) {
    hipLaunchKernelGGL(k_zero_unsampled, dim3(nv, nt, nc), dim3(128), 0, s, y, p->mask, nv, nh, nc);
    CS_HIP(hipGetLastError());
  }
  return CS_OK;
}

int launch_forward_residual(cs_plan* p, const float2* x, double* part, int nblocks, float tv_lambda,
                            hipStream_t s) {
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt, nc = p->desc.nc;
  const int cw = fft_cols_per_group(p);
  if (reg16_size(nv)) {
    reg16_switch(nv, [&](auto mc) {
      constexpr int M = decltype(mc)::value;
      hipLaunchKernelGGL((k_fwd_vertical16m<M, kFwdResidual>), dim3(nblocks), dim3(64 * kVWaves), kLds16m, s, x,
                         p->coil_cm, nullptr, p->ktmp, p->rinv, p->mcnt, p->tw_v, nh, nt, nc, p->m_max,
                         coil_split16(nh, nt, nc), 1.0f / std::sqrt((float)nv), tv_lambda, part);
    });
    CS_HIP(hipGetLastError());
    return CS_OK;
  }
  auto k = cw * nv <= 256 ? k_fwd_vertical<kFwdResidual, 256> : k_fwd_vertical<kFwdResidual, 512>;
  hipLaunchKernelGGL(k, dim3(nblocks), dim3(64 * kVWaves), vertical_lds(p, cw), s, x, p->coil_cm, nullptr,
                     p->ktmp, p->rows, p->mcnt, p->fft_v, p->tw_v, nv, nh, nt, nc, p->m_max, cw,
                     1.0f / std::sqrt((float)nv), tv_lambda, part);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_adjoint_rows_raw(const float2* y, float2* hyb, const int32_t* rows, const int32_t* mcnt, const FftDesc& fh,
                            const float2* twh, int nv, int nh, int nt, int nc, int m_max, int rb, hipStream_t s) {
  if (reg16_size(nh)) {
    reg16_switch(nh, [&](auto mc) {
      constexpr int M = decltype(mc)::value;
      hipLaunchKernelGGL((k_adj_horizontal16m<M>), dim3(ceil_div(m_max, kH256Rows), nt, nc), dim3(64 * kVWaves),
                         kLds16m, s, y, hyb, rows, mcnt, twh, nv, nc, m_max, 1.0f / std::sqrt((float)nh));
    });
    CS_HIP(hipGetLastError());
    return CS_OK;
  }
  const size_t lds = (size_t)(nh + rb * (nh + 1)) * sizeof(float2);
  dim3 g(ceil_div(m_max, rb), nt, nc);
  hipLaunchKernelGGL(k_adj_horizontal, g, dim3(kFftThreads), lds, s, y, hyb, rows, mcnt, fh, twh, nv, nh, nc,
                     m_max, rb, 1.0f / std::sqrt((float)nh));
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_adjoint_vertical_raw(const float2* hyb, const float2* coil_cm, float2* x, const int32_t* rows,
                                const int32_t* mcnt, const int32_t* rinv, const FftDesc& fv, const float2* twv,
                                int nv, int nh, int nt, int nc, int m_max, int cw, int csplit, hipStream_t s) {
  if (reg16_size(nv)) {
    if (csplit != 1 && csplit != 2 && csplit != 4) return CS_EINVAL;
    reg16_switch(nv, [&](auto mc) {
      constexpr int M = decltype(mc)::value;
      // csplit waves per column group: kVWaves / csplit groups per block
      const size_t units = (size_t)nt * ((nh + kV256Cols - 1) / kV256Cols);
      const unsigned grid = (unsigned)std::min<size_t>((units * csplit + kVWaves - 1) / kVWaves, 65535);
      hipLaunchKernelGGL((k_adj_vertical16m<M>), dim3(grid), dim3(64 * kVWaves), kLds16m, s, hyb, coil_cm, x, rinv,
                         twv, nh, nt, nc, m_max, csplit, 1.0f / std::sqrt((float)nv));
    });
    CS_HIP(hipGetLastError());
    return CS_OK;
  }
  auto k = cw * nv <= 256 ? k_adj_vertical<256> : k_adj_vertical<512>;
  const size_t units = (size_t)nt * ceil_div(nh, cw);
  const unsigned grid = (unsigned)std::min<size_t>((units + kVWaves - 1) / kVWaves, 65535);
  const size_t lds = (size_t)(nv + kVWaves * cw * nv) * sizeof(float2);
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * kVWaves), lds, s, hyb, coil_cm, x, rows, mcnt, fv, twv, nv, nh, nt,
                     nc, m_max, cw, 1.0f / std::sqrt((float)nv));
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_adjoint_rows(cs_plan* p, const float2* y, hipStream_t s) {
  if (p->m_max == 0) return CS_OK;
  return launch_adjoint_rows_raw(y, p->ktmp, p->rows, p->mcnt, p->fft_h, p->tw_h, p->desc.nv, p->desc.nh,
                                 p->desc.nt, p->desc.nc, p->m_max, fft_rows_per_group(p), s);
}

int launch_adjoint_image(cs_plan* p, float2* x, bool x_colmajor, hipStream_t s) {
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt;
  float2* xo = x_colmajor ? x : p->img_tmp;
  int st = launch_adjoint_vertical_raw(p->ktmp, p->coil_cm, xo, p->rows, p->mcnt, p->rinv, p->fft_v, p->tw_v, nv,
                                       nh, nt, p->desc.nc, p->m_max, fft_cols_per_group(p),
                                       coil_split16(nh, nt, p->desc.nc), s);
  if (st != CS_OK) return st;
  if (!x_colmajor) return launch_transpose(p->img_tmp, x, nt, nh, nv, s);
  return CS_OK;
}

// ---------------------------------------------------------------- finite-value checks
//
// CS_FLAG_CHECK_FINITE: an input holding a NaN or an infinity is rejected
// before any work.  Each kernel stores 1 into *flag when it meets one (every
// writer stores the same value, so the stores need no ordering).

// one workgroup per sampled line (t, c, r): the rows of k-space a solve reads
__global__ void k_nonfinite_rows(const float2* __restrict__ y, const int32_t* __restrict__ rows, int mrow, int nc,
                                 int nv, int nh, int* __restrict__ flag) {
  const int line = blockIdx.x;  // (t * nc + c) * mrow + r
  const int r = line % mrow, tc = line / mrow, t = tc / nc;
  const int ky = rows[(size_t)t * mrow + r];
  if (ky < 0) return;
  const float2* src = y + ((size_t)tc * nv + ky) * nh;
  bool bad = false;
  for (int i = threadIdx.x; i < nh; i += blockDim.x) {
    const float2 v = src[i];
    bad |= !(isfinite(v.x) && isfinite(v.y));
  }
  if (bad) *flag = 1;
}

__global__ void k_nonfinite(const float2* __restrict__ x, size_t n, int* __restrict__ flag) {
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float2 v = x[i];
    bad |= !(isfinite(v.x) && isfinite(v.y));
  }
  if (bad) *flag = 1;
}

// clears *flag, runs the check, reads the flag back (synchronises s)
template <typename F>
static int run_finite_check(cs_plan* p, hipStream_t s, const char* what, F launch) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  CS_HIP(hipStreamIsCapturing(s, &cap));
  if (cap != hipStreamCaptureStatusNone)
    return set_error(CS_EINVAL, "CS_FLAG_CHECK_FINITE reads its result back and cannot run under stream capture");
  CS_HIP(hipMemsetAsync(p->check_flag, 0, sizeof(int), s));
  launch();
  CS_HIP(hipGetLastError());
  int h = 0;
  CS_HIP(hipMemcpyAsync(&h, p->check_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  CS_HIP(hipStreamSynchronize(s));
  if (h) return set_error(CS_EINVAL, std::string(what) + " holds a non-finite value (CS_FLAG_CHECK_FINITE)");
  return CS_OK;
}

int check_finite_kspace(cs_plan* p, const float2* y, hipStream_t s, const char* what) {
  if (!(p->desc.flags & CS_FLAG_CHECK_FINITE) || p->m_max == 0) return CS_OK;
  const int mrow = std::max(p->m_max, 1);
  const unsigned lines = (unsigned)((size_t)p->desc.nt * p->desc.nc * mrow);
  return run_finite_check(p, s, what, [&] {
    hipLaunchKernelGGL(k_nonfinite_rows, dim3(lines), dim3(256), 0, s, y, p->rows, mrow, p->desc.nc, p->desc.nv,
                       p->desc.nh, p->check_flag);
  });
}

int check_finite_values(cs_plan* p, const float2* x, size_t n, hipStream_t s, const char* what) {
  if (!(p->desc.flags & CS_FLAG_CHECK_FINITE) || n == 0) return CS_OK;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  return run_finite_check(p, s, what, [&] {
    hipLaunchKernelGGL(k_nonfinite, dim3(blocks), dim3(256), 0, s, x, n, p->check_flag);
  });
}

}  // namespace csmri
