// LDS-resident mixed-radix (2, 3, 4) Stockham FFT used by the SENSE operator
// kernels.  A workgroup transforms `nbatch` independent length-n sequences
// stored at buf[b * stride + q]; the passes run in place with a register
// stage between two barriers, so one LDS buffer suffices.
//
// Pass with radix r after a span p of earlier radices: butterfly k in
// [0, n/r) reads u_m = x[k + m n/r] (m < r), multiplies u_m by
// w^(i m n/(p r)) with i = k mod p and w = exp(SIGN 2 pi i / n), takes the
// r-point DFT and writes v_m to y[(k - i) r + i + m p].  After all passes the
// sequence holds the unnormalised DFT sum_q x_q exp(SIGN 2 pi i k q / n).
#pragma once

#include "internal.hpp"

namespace csmri {

constexpr int kFftThreads = 256;      // workgroup size of every FFT kernel
constexpr int kFftElems = 4096;       // nbatch * n handled by one workgroup
constexpr int kFftMaxBfly = 8;        // kFftElems / 2 / kFftThreads: butterflies per thread in
                                      // a radix-2 pass, the most of any radix

template <int SIGN>
__device__ __forceinline__ float2 twiddle(float2 u, float2 w) {
  // w = exp(-2 pi i q / n) from the table; the inverse transform uses conj(w)
  return SIGN < 0 ? cmul(u, w) : cmulc(w, u);
}

// Loads one butterfly's inputs, applies twiddles and the r-point DFT.
template <int SIGN>
__device__ __forceinline__ void fft_butterfly(const float2* s, int nr, int r, int tq, const float2* tw,
                                     float2* v) {
  if (r == 4) {
    float2 u0 = s[0], u1 = s[nr], u2 = s[2 * nr], u3 = s[3 * nr];
    if (tq) {
      u1 = twiddle<SIGN>(u1, tw[tq]);
      u2 = twiddle<SIGN>(u2, tw[2 * tq]);
      u3 = twiddle<SIGN>(u3, tw[3 * tq]);
    }
    float2 t0 = cadd(u0, u2), t1 = csub(u0, u2), t2 = cadd(u1, u3), t3 = csub(u1, u3);
    // omega = exp(SIGN i pi/2) = SIGN * i ; omega * t3
    float2 wt3 = SIGN < 0 ? make_float2(t3.y, -t3.x) : make_float2(-t3.y, t3.x);
    v[0] = cadd(t0, t2);
    v[1] = cadd(t1, wt3);
    v[2] = csub(t0, t2);
    v[3] = csub(t1, wt3);
  } else if (r == 3) {
    float2 u0 = s[0], u1 = s[nr], u2 = s[2 * nr];
    if (tq) {
      u1 = twiddle<SIGN>(u1, tw[tq]);
      u2 = twiddle<SIGN>(u2, tw[2 * tq]);
    }
    const float h = 0.86602540378443864676f;  // sqrt(3)/2
    float2 sm = cadd(u1, u2), df = csub(u1, u2);
    float2 base = make_float2(u0.x - 0.5f * sm.x, u0.y - 0.5f * sm.y);
    // SIGN * i * h * df
    float2 rot = SIGN < 0 ? make_float2(h * df.y, -h * df.x) : make_float2(-h * df.y, h * df.x);
    v[0] = cadd(u0, sm);
    v[1] = cadd(base, rot);
    v[2] = csub(base, rot);
  } else {  // r == 2
    float2 u0 = s[0], u1 = s[nr];
    if (tq) u1 = twiddle<SIGN>(u1, tw[tq]);
    v[0] = cadd(u0, u1);
    v[1] = csub(u0, u1);
  }
}

// q = a / b and a - q b for 0 <= a < 16384, 1 <= b <= 4096 (checked
// exhaustively): a float estimate of the quotient, off by at most one, then
// corrected.  A general integer division costs tens of instructions; every
// index split of the FFT kernels (a < 2 kFftElems, b <= 512) uses this.
__device__ __forceinline__ int fast_div(int a, int b, float inv_b, int& rem) {
  int q = (int)((float)a * inv_b);
  int r = a - q * b;
  if (r < 0) {
    --q;
    r += b;
  } else if (r >= b) {
    ++q;
    r -= b;
  }
  rem = r;
  return q;
}

// In-place transform of nbatch sequences; all threads of the (1-D, kFftThreads
// wide) workgroup must call it.  Ends with a barrier.
template <int SIGN>
__device__ void fft_lds(float2* buf, const FftDesc& d, const float2* tw, int nbatch, int stride) {
  const int tid = threadIdx.x;
  const int n = d.n;
  int p = 1;
  for (int ps = 0; ps < d.npass; ++ps) {
    const int r = d.radix[ps];
    const int nr = n / r;
    const int tstep = n / (p * r);
    const int total = nbatch * nr;
    const float inv_nr = 1.0f / (float)nr, inv_p = 1.0f / (float)p;
    // butterfly g of the pass: sequence bt = g / nr, index k = g mod nr, i = k mod p
    int bt_q[kFftMaxBfly], k_q[kFftMaxBfly], i_q[kFftMaxBfly];
    float2 v[kFftMaxBfly][4];
#pragma unroll
    for (int q = 0; q < kFftMaxBfly; ++q) {
      const int g = tid + q * kFftThreads;
      bt_q[q] = k_q[q] = i_q[q] = 0;
      if (g < total) {
        int k, i;
        const int bt = fast_div(g, nr, inv_nr, k);
        (void)fast_div(k, p, inv_p, i);
        bt_q[q] = bt;
        k_q[q] = k;
        i_q[q] = i;
        fft_butterfly<SIGN>(buf + bt * stride + k, nr, r, i * tstep, tw, v[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kFftMaxBfly; ++q) {
      const int g = tid + q * kFftThreads;
      if (g < total) {
        const int bt = bt_q[q], k = k_q[q], i = i_q[q];
        float2* o = buf + bt * stride + (k - i) * r + i;
        o[0] = v[q][0];
        o[p] = v[q][1];
        if (r > 2) o[2 * p] = v[q][2];
        if (r > 3) o[3 * p] = v[q][3];
      }
    }
    __syncthreads();
    p *= r;
  }
}

}  // namespace csmri
