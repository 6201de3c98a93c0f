// LDS-resident mixed-radix (2, 3, 4) Stockham FFT used by the SENSE operator
// kernels.  A group of threads (a workgroup, or a single wave working in its
// own LDS region) transforms `nbatch` independent length-n sequences stored
// at buf[b * stride + q]; the passes run in place with a register stage
// between two barriers, so one LDS buffer suffices.
//
// Pass with radix r after a span p of earlier radices: butterfly k in
// [0, n/r) reads u_m = x[k + m n/r] (m < r), multiplies u_m by
// w^(i m n/(p r)) with i = k mod p and w = exp(SIGN 2 pi i / n), takes the
// r-point DFT and writes v_m to y[(k - i) r + i + m p].  After all passes the
// sequence holds the unnormalised DFT sum_q x_q exp(SIGN 2 pi i k q / n).
#pragma once

#include "internal.hpp"

namespace csmri {

constexpr int kFftThreads = 256;      // workgroup size of the horizontal FFT kernels
constexpr int kFftElems = 4096;       // nbatch * n handled by one such workgroup
constexpr int kWaveElems = 512;       // nbatch * n handled by one wave (vertical passes)

template <int SIGN>
__device__ __forceinline__ float2 twiddle(float2 u, float2 w) {
  // w = exp(-2 pi i q / n) from the table; the inverse transform uses conj(w)
  return SIGN < 0 ? cmul(u, w) : cmulc(w, u);
}

// Loads one butterfly's inputs, applies twiddles and the R-point DFT.
template <int SIGN, int R>
__device__ __forceinline__ void fft_butterfly(const float2* s, int nr, int tq, const float2* tw, float2 (&v)[R]) {
  if constexpr (R == 4) {
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
  } else if constexpr (R == 3) {
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
  } else {
    static_assert(R == 2, "radix 2, 3 or 4");
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

// Barrier between the read and write halves of a pass: the whole workgroup,
// or only the wave when the buffer is private to it (a wave's LDS accesses
// complete in issue order, so only code motion has to be fenced).
template <bool WAVE>
__device__ __forceinline__ void fft_sync() {
  if constexpr (WAVE) __builtin_amdgcn_wave_barrier();
  else __syncthreads();
}

// One radix-R pass after a span p of earlier radices, in place, by THREADS
// threads (thread index tid) over at most ELEMS values: every thread first
// computes its butterflies into registers, then all store after a barrier.
// R is a template argument so that the staging arrays are indexed with
// constants only and stay in registers (a radix chosen at run time made them
// a private-memory array).
template <int SIGN, int R, int THREADS, int ELEMS, bool WAVE>
__device__ __forceinline__ void fft_pass(float2* buf, const float2* tw, int n, int p, int nbatch, int stride,
                                         int tid) {
  constexpr int kB = (ELEMS / R + THREADS - 1) / THREADS;  // butterflies per thread
  const int nr = n / R;
  const int tstep = n / (p * R);
  const int total = nbatch * nr;
  const float inv_nr = 1.0f / (float)nr, inv_p = 1.0f / (float)p;
  float2 v[kB][R];
  int dst[kB];
#pragma unroll
  for (int q = 0; q < kB; ++q) {
    // butterfly g: sequence bt = g / nr, index k = g mod nr, i = k mod p
    const int g = tid + q * THREADS;
    dst[q] = -1;
    if (g < total) {
      int k, i;
      const int bt = fast_div(g, nr, inv_nr, k);
      (void)fast_div(k, p, inv_p, i);
      fft_butterfly<SIGN, R>(buf + bt * stride + k, nr, i * tstep, tw, v[q]);
      dst[q] = bt * stride + (k - i) * R + i;
    }
  }
  fft_sync<WAVE>();
#pragma unroll
  for (int q = 0; q < kB; ++q) {
    if (dst[q] >= 0) {
      float2* o = buf + dst[q];
#pragma unroll
      for (int m = 0; m < R; ++m) o[m * p] = v[q][m];
    }
  }
  fft_sync<WAVE>();
}

template <int SIGN, int THREADS, int ELEMS, bool WAVE>
__device__ __forceinline__ void fft_passes(float2* buf, const FftDesc& d, const float2* tw, int nbatch, int stride,
                                           int tid) {
  const int n = d.n;
  int p = 1;
  for (int ps = 0; ps < d.npass; ++ps) {
    const int r = d.radix[ps];
    if (r == 4) fft_pass<SIGN, 4, THREADS, ELEMS, WAVE>(buf, tw, n, p, nbatch, stride, tid);
    else if (r == 3) fft_pass<SIGN, 3, THREADS, ELEMS, WAVE>(buf, tw, n, p, nbatch, stride, tid);
    else fft_pass<SIGN, 2, THREADS, ELEMS, WAVE>(buf, tw, n, p, nbatch, stride, tid);
    p *= r;
  }
}

// In-place transform of nbatch sequences (nbatch * n <= kFftElems) by the
// whole (1-D, kFftThreads wide) workgroup; all threads must call it.  Ends
// with a barrier.
template <int SIGN>
__device__ void fft_lds(float2* buf, const FftDesc& d, const float2* tw, int nbatch, int stride) {
  fft_passes<SIGN, kFftThreads, kFftElems, false>(buf, d, tw, nbatch, stride, threadIdx.x);
}

// In-place transform of nbatch sequences (nbatch * n <= WE <= kWaveElems) in
// a buffer private to the calling wave; all 64 lanes must call it.  Ends with
// a wave barrier.
template <int SIGN, int WE>
__device__ __forceinline__ void fft_wave(float2* buf, const FftDesc& d, const float2* tw, int nbatch, int stride,
                                         int lane) {
  static_assert(WE <= kWaveElems, "wave transform larger than its buffer bound");
  fft_passes<SIGN, 64, WE, true>(buf, d, tw, nbatch, stride, lane);
}

// ---------------------------------------------------------------- register DFTs
//
// Length-16 DFT of values held by one lane, v[k] <- sum_n v[n] exp(SIGN 2 pi i
// n k / 16), as 4 x 4 Cooley-Tukey: n = 4 n1 + n2, k = k1 + 4 k2.  Four
// length-4 DFTs over n1, the twiddles exp(SIGN 2 pi i n2 k1 / 16), four
// length-4 DFTs over n2; every index is a compile-time constant, so the whole
// transform stays in registers.

template <int SIGN>
__device__ __forceinline__ void dft4_regs(float2& a, float2& b, float2& c, float2& d) {
  const float2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
  // (SIGN i) t3
  const float2 wt3 = SIGN < 0 ? make_float2(t3.y, -t3.x) : make_float2(-t3.y, t3.x);
  a = cadd(t0, t2);
  b = cadd(t1, wt3);
  c = csub(t0, t2);
  d = csub(t1, wt3);
}

// exp(SIGN 2 pi i m / 16) * u for the m that occur (m = n2 k1 <= 9)
template <int SIGN, int M>
__device__ __forceinline__ float2 w16_mul(float2 u) {
  constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;  // cos, sin (pi / 8)
  constexpr float h = 0.70710678118654752440f;                                 // cos (pi / 4)
  constexpr int m = M % 16;
  // (c + SIGN i s) u with c = cos(2 pi m / 16), s = sin(2 pi m / 16)
  auto rot = [](float2 v, float c, float sn) {
    const float ss = SIGN < 0 ? -sn : sn;
    return make_float2(fmaf(c, v.x, -(ss * v.y)), fmaf(c, v.y, ss * v.x));
  };
  if constexpr (m == 0) return u;
  else if constexpr (m == 4) return SIGN < 0 ? make_float2(u.y, -u.x) : make_float2(-u.y, u.x);
  else if constexpr (m == 8) return make_float2(-u.x, -u.y);
  else if constexpr (m == 1) return rot(u, c1, s1);
  else if constexpr (m == 2) return rot(u, h, h);
  else if constexpr (m == 3) return rot(u, s1, c1);
  else if constexpr (m == 6) return rot(u, -h, h);
  else {
    static_assert(m == 9, "twiddle index of the 4 x 4 split");
    return rot(u, -c1, -s1);
  }
}

template <int SIGN>
__device__ __forceinline__ void dft16_regs(float2 (&v)[16]) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4_regs<SIGN>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // v[4 k1 + n2] now holds the length-4 DFT over n1 at frequency k1
  v[5] = w16_mul<SIGN, 1>(v[5]);
  v[6] = w16_mul<SIGN, 2>(v[6]);
  v[7] = w16_mul<SIGN, 3>(v[7]);
  v[9] = w16_mul<SIGN, 2>(v[9]);
  v[10] = w16_mul<SIGN, 4>(v[10]);
  v[11] = w16_mul<SIGN, 6>(v[11]);
  v[13] = w16_mul<SIGN, 3>(v[13]);
  v[14] = w16_mul<SIGN, 6>(v[14]);
  v[15] = w16_mul<SIGN, 9>(v[15]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4_regs<SIGN>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // v[4 k1 + k2] holds frequency k1 + 4 k2: reorder to natural order
  float2 o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = o[k];
}

}  // namespace csmri
