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
// layout of the boundary goes through a tiled transpose.
#include "fft.hpp"

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
//                    groups with a fixed grid, so the sum is reproducible)
constexpr int kFwdStore = 0, kFwdResidual = 1;

template <int MODE, int WE>
__global__ __launch_bounds__(64 * kVWaves) void k_fwd_vertical(
    const float2* __restrict__ x, const float2* __restrict__ coil_cm, float2* __restrict__ hyb,
    const float2* __restrict__ ref, const int32_t* __restrict__ rows, const int32_t* __restrict__ mcnt,
    FftDesc fv, const float2* __restrict__ twv, int nv, int nh, int nt, int nc, int m_max, int cw, float scale,
    double* __restrict__ part) {
  constexpr int kVE = WE / 64;  // image values per lane of one column group
  extern __shared__ float2 lds[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float2* tw = lds;
  float2* buf = lds + nv + (size_t)wv * cw * nv;
  for (int q = threadIdx.x; q < nv; q += blockDim.x) tw[q] = twv[q];
  __syncthreads();
  const int ngrp = (nh + cw - 1) / cw;
  const int units = nt * ngrp;
  double acc = 0.0;
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
  if constexpr (MODE == kFwdResidual) {
    __shared__ double red[64 * kVWaves];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 32 * kVWaves; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
  }
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
    auto k = cw * nv <= 256 ? k_fwd_vertical<kFwdStore, 256> : k_fwd_vertical<kFwdStore, 512>;
    hipLaunchKernelGGL(k, dim3(vertical_grid(p, cw)), dim3(64 * kVWaves), vertical_lds(p, cw), s, x, p->coil_cm,
                       p->ftmp, nullptr, p->rows, p->mcnt, p->fft_v, p->tw_v, nv, nh, nt, nc, p->m_max, cw, sv,
                       nullptr);
    CS_HIP(hipGetLastError());
    if (y) {
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

int launch_forward_residual(cs_plan* p, const float2* x, double* part, int nblocks, hipStream_t s) {
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt, nc = p->desc.nc;
  const int cw = fft_cols_per_group(p);
  auto k = cw * nv <= 256 ? k_fwd_vertical<kFwdResidual, 256> : k_fwd_vertical<kFwdResidual, 512>;
  hipLaunchKernelGGL(k, dim3(nblocks), dim3(64 * kVWaves), vertical_lds(p, cw), s, x, p->coil_cm, nullptr,
                     p->ktmp, p->rows, p->mcnt, p->fft_v, p->tw_v, nv, nh, nt, nc, p->m_max, cw,
                     1.0f / std::sqrt((float)nv), part);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_adjoint_rows_raw(const float2* y, float2* hyb, const int32_t* rows, const int32_t* mcnt, const FftDesc& fh,
                            const float2* twh, int nv, int nh, int nt, int nc, int m_max, int rb, hipStream_t s) {
  const size_t lds = (size_t)(nh + rb * (nh + 1)) * sizeof(float2);
  dim3 g(ceil_div(m_max, rb), nt, nc);
  hipLaunchKernelGGL(k_adj_horizontal, g, dim3(kFftThreads), lds, s, y, hyb, rows, mcnt, fh, twh, nv, nh, nc,
                     m_max, rb, 1.0f / std::sqrt((float)nh));
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_adjoint_vertical_raw(const float2* hyb, const float2* coil_cm, float2* x, const int32_t* rows,
                                const int32_t* mcnt, const FftDesc& fv, const float2* twv, int nv, int nh, int nt,
                                int nc, int m_max, int cw, hipStream_t s) {
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
  int st = launch_adjoint_vertical_raw(p->ktmp, p->coil_cm, xo, p->rows, p->mcnt, p->fft_v, p->tw_v, nv, nh, nt,
                                       p->desc.nc, p->m_max, fft_cols_per_group(p), s);
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
