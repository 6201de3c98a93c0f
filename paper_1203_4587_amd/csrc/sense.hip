// Measurement operator H and its adjoint (Sec. II-A, eqs. mri_mcoil2,
// mri_csmcoill2, H_2):   y_{t,c} = F_h M_t F_v (s_c . x_t).
//
// Forward: a vertical pass (coil multiply fused into the load, length-nv FFT
// of every column, only the sampled ky rows kept) followed by a horizontal
// pass over the sampled rows only, so the horizontal work is 1/R of a full
// 2D FFT.  Rows ky that a frame does not sample are zero-filled by a third,
// store-only kernel.  The adjoint runs the same passes in reverse order and
// sums conj(s_c) . (.) over coils in registers before the single store.
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

// ktmp[t][c][r][i] = (1/sqrt nv) * (F_v (s_c . x_t))[rows[t][r], i]
template <bool COLMAJOR>
__global__ __launch_bounds__(kFftThreads) void k_fwd_vertical(
    const float2* __restrict__ x, const float2* __restrict__ coil_cm, float2* __restrict__ ktmp,
    const int32_t* __restrict__ rows, const int32_t* __restrict__ mcnt, FftDesc fv,
    const float2* __restrict__ twv, int nv, int nh, int nc, int m_max, int cw, float scale) {
  extern __shared__ float2 lds[];
  float2* tw = lds;
  float2* buf = lds + nv;
  const int stride = nv + 1;
  const int i0 = blockIdx.x * cw, t = blockIdx.y, c = blockIdx.z;
  const int ncol = min(cw, nh - i0);
  for (int q = threadIdx.x; q < nv; q += kFftThreads) tw[q] = twv[q];
  const int tot = ncol * nv;
  const float inv_nv = 1.0f / (float)nv, inv_ncol = 1.0f / (float)ncol;
  for (int e = threadIdx.x; e < tot; e += kFftThreads) {
    int j, col;
    float2 xv;
    if (COLMAJOR) {
      col = fast_div(e, nv, inv_nv, j);
      xv = x[((size_t)t * nh + i0 + col) * nv + j];
    } else {
      j = fast_div(e, ncol, inv_ncol, col);
      xv = x[((size_t)t * nv + j) * nh + i0 + col];
    }
    const float2 sv = coil_cm[((size_t)c * nh + i0 + col) * nv + j];
    buf[col * stride + j] = cmul(sv, xv);
  }
  __syncthreads();
  fft_lds<-1>(buf, fv, tw, ncol, stride);
  const int m = mcnt[t];
  const int32_t* rw = rows + (size_t)t * m_max;
  float2* out = ktmp + ((size_t)(t * nc + c) * m_max) * nh + i0;
  for (int e = threadIdx.x; e < m * ncol; e += kFftThreads) {
    int col;
    const int r = fast_div(e, ncol, inv_ncol, col);
    out[(size_t)r * nh + col] = cscale(buf[col * stride + rw[r]], scale);
  }
}

// y[t][c][rows[t][r]][:] = (1/sqrt nh) F_h ktmp[t][c][r][:]
__global__ __launch_bounds__(kFftThreads) void k_fwd_horizontal(
    const float2* __restrict__ ktmp, float2* __restrict__ y, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ mcnt, FftDesc fh, const float2* __restrict__ twh, int nv, int nh,
    int nc, int m_max, int rb, float scale) {
  extern __shared__ float2 lds[];
  float2* tw = lds;
  float2* buf = lds + nh;
  const int stride = nh + 1;
  const int r0 = blockIdx.x * rb, t = blockIdx.y, c = blockIdx.z;
  const int nrow = min(rb, mcnt[t] - r0);
  if (nrow <= 0) return;  // uniform over the workgroup
  const float inv_nh = 1.0f / (float)nh;
  for (int q = threadIdx.x; q < nh; q += kFftThreads) tw[q] = twh[q];
  const float2* src = ktmp + ((size_t)(t * nc + c) * m_max + r0) * nh;
  for (int e = threadIdx.x; e < nrow * nh; e += kFftThreads) {
    int i;
    const int rr = fast_div(e, nh, inv_nh, i);
    buf[rr * stride + i] = src[(size_t)rr * nh + i];
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

// ktmp[t][c][r][:] = (1/sqrt nh) F_h' y[t][c][rows[t][r]][:]   (hybrid space)
__global__ __launch_bounds__(kFftThreads) void k_adj_horizontal(
    const float2* __restrict__ y, float2* __restrict__ ktmp, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ mcnt, FftDesc fh, const float2* __restrict__ twh, int nv, int nh,
    int nc, int m_max, int rb, float scale) {
  extern __shared__ float2 lds[];
  float2* tw = lds;
  float2* buf = lds + nh;
  const int stride = nh + 1;
  const int r0 = blockIdx.x * rb, t = blockIdx.y, c = blockIdx.z;
  const int nrow = min(rb, mcnt[t] - r0);
  if (nrow <= 0) return;
  const float inv_nh = 1.0f / (float)nh;
  for (int q = threadIdx.x; q < nh; q += kFftThreads) tw[q] = twh[q];
  const int32_t* rw = rows + (size_t)t * m_max + r0;
  for (int e = threadIdx.x; e < nrow * nh; e += kFftThreads) {
    int i;
    const int rr = fast_div(e, nh, inv_nh, i);
    buf[rr * stride + i] = y[((size_t)(t * nc + c) * nv + rw[rr]) * nh + i];
  }
  __syncthreads();
  fft_lds<+1>(buf, fh, tw, nrow, stride);
  float2* dst = ktmp + ((size_t)(t * nc + c) * m_max + r0) * nh;
  for (int e = threadIdx.x; e < nrow * nh; e += kFftThreads) {
    int i;
    const int rr = fast_div(e, nh, inv_nh, i);
    dst[(size_t)rr * nh + i] = cscale(buf[rr * stride + i], scale);
  }
}

// x_t[:, i] = (1/sqrt nv) sum_c conj(s_c[:, i]) . F_v' (zero-filled column of ktmp[t][c][:, i])
// The coil sum lives in registers across the coil loop; two waves per SIMD
// (instead of the one an unconstrained allocation leaves) measured 1.4x faster.
template <bool COLMAJOR>
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_adj_vertical(
    const float2* __restrict__ ktmp, const float2* __restrict__ coil_cm, float2* __restrict__ x,
    const int32_t* __restrict__ rows, const int32_t* __restrict__ mcnt, FftDesc fv,
    const float2* __restrict__ twv, int nv, int nh, int nc, int m_max, int cw, float scale) {
  constexpr int kEPT = kFftElems / kFftThreads;
  extern __shared__ float2 lds[];
  float2* tw = lds;
  float2* buf = lds + nv;
  const int stride = nv + 1;
  const int i0 = blockIdx.x * cw, t = blockIdx.y;
  const int ncol = min(cw, nh - i0);
  const int tot = ncol * nv;
  const int m = mcnt[t];
  const float inv_nv = 1.0f / (float)nv, inv_ncol = 1.0f / (float)ncol;
  // element e = threadIdx.x + q kFftThreads of the accumulation is the pair
  // (column, row); the split is recomputed where it is used rather than held
  // in registers across the coil loop
  auto split = [&](int e, int& j, int& col) {
    if (COLMAJOR) col = fast_div(e, nv, inv_nv, j);
    else j = fast_div(e, ncol, inv_ncol, col);
  };
  const int32_t* rw = rows + (size_t)t * m_max;
  for (int q = threadIdx.x; q < nv; q += kFftThreads) tw[q] = twv[q];
  float2 acc[kEPT];
#pragma unroll
  for (int q = 0; q < kEPT; ++q) acc[q] = make_float2(0.f, 0.f);
  for (int c = 0; c < nc; ++c) {
    for (int e = threadIdx.x; e < ncol * stride; e += kFftThreads) buf[e] = make_float2(0.f, 0.f);
    __syncthreads();
    const float2* src = ktmp + ((size_t)(t * nc + c) * m_max) * nh + i0;
    for (int e = threadIdx.x; e < m * ncol; e += kFftThreads) {
      int col;
      const int r = fast_div(e, ncol, inv_ncol, col);
      buf[col * stride + rw[r]] = src[(size_t)r * nh + col];
    }
    __syncthreads();
    fft_lds<+1>(buf, fv, tw, ncol, stride);
#pragma unroll
    for (int q = 0; q < kEPT; ++q) {
      const int e = threadIdx.x + q * kFftThreads;
      if (e < tot) {
        int j, col;
        split(e, j, col);
        const float2 sv = coil_cm[((size_t)c * nh + i0 + col) * nv + j];
        acc[q] = cfmac(sv, buf[col * stride + j], acc[q]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kEPT; ++q) {
    const int e = threadIdx.x + q * kFftThreads;
    if (e < tot) {
      int j, col;
      split(e, j, col);
      if (COLMAJOR) x[((size_t)t * nh + i0 + col) * nv + j] = cscale(acc[q], scale);
      else x[((size_t)t * nv + j) * nh + i0 + col] = cscale(acc[q], scale);
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

// columns per workgroup of the vertical passes and sampled rows per workgroup
// of the horizontal passes: the largest that fit kFftElems values, or the
// plan's tuned (smaller) choice
int fft_cols_per_group(const cs_plan* p) {
  const int full = std::min(p->desc.nh, kFftElems / p->desc.nv);
  return p->fft_cw > 0 ? std::min(p->fft_cw, full) : full;
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

int launch_forward(cs_plan* p, const float2* x, bool x_colmajor, float2* y, hipStream_t s) {
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt, nc = p->desc.nc;
  if (p->m_max > 0) {
    const int cw = fft_cols_per_group(p);
    const size_t lds1 = (size_t)(nv + cw * (nv + 1)) * sizeof(float2);
    dim3 g1(ceil_div(nh, cw), nt, nc);
    const float sv = 1.0f / std::sqrt((float)nv), sh = 1.0f / std::sqrt((float)nh);
    if (x_colmajor)
      hipLaunchKernelGGL(k_fwd_vertical<true>, g1, dim3(kFftThreads), lds1, s, x, p->coil_cm, p->ftmp,
                         p->rows, p->mcnt, p->fft_v, p->tw_v, nv, nh, nc, p->m_max, cw, sv);
    else
      hipLaunchKernelGGL(k_fwd_vertical<false>, g1, dim3(kFftThreads), lds1, s, x, p->coil_cm, p->ftmp,
                         p->rows, p->mcnt, p->fft_v, p->tw_v, nv, nh, nc, p->m_max, cw, sv);
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

int launch_adjoint_rows(cs_plan* p, const float2* y, hipStream_t s) {
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt, nc = p->desc.nc;
  if (p->m_max == 0) return CS_OK;
  const int rb = fft_rows_per_group(p);
  const size_t lds = (size_t)(nh + rb * (nh + 1)) * sizeof(float2);
  dim3 g(ceil_div(p->m_max, rb), nt, nc);
  hipLaunchKernelGGL(k_adj_horizontal, g, dim3(kFftThreads), lds, s, y, p->ktmp, p->rows, p->mcnt,
                     p->fft_h, p->tw_h, nv, nh, nc, p->m_max, rb, 1.0f / std::sqrt((float)nh));
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_adjoint_image(cs_plan* p, float2* x, bool x_colmajor, hipStream_t s) {
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt, nc = p->desc.nc;
  const int cw = fft_cols_per_group(p);
  const size_t lds = (size_t)(nv + cw * (nv + 1)) * sizeof(float2);
  dim3 g(ceil_div(nh, cw), nt);
  const float sv = 1.0f / std::sqrt((float)nv);
  if (x_colmajor)
    hipLaunchKernelGGL(k_adj_vertical<true>, g, dim3(kFftThreads), lds, s, p->ktmp, p->coil_cm, x, p->rows,
                       p->mcnt, p->fft_v, p->tw_v, nv, nh, nc, p->m_max, cw, sv);
  else
    hipLaunchKernelGGL(k_adj_vertical<false>, g, dim3(kFftThreads), lds, s, p->ktmp, p->coil_cm, x, p->rows,
                       p->mcnt, p->fft_v, p->tw_v, nv, nh, nc, p->m_max, cw, sv);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

}  // namespace csmri
