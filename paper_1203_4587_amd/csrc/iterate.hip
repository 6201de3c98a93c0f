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
__device__ __forceinline__ float4 ld_stream4(const float2* p) {
  const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

template <int MODE>
__device__ __forceinline__ float2 rhs_value(const float2* hy, const float2* m, const float2* d2, size_t q, float mu,
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

// Pair form (even n, one block per workgroup of round_up(n/2, 64) lanes):
// lane l owns rows 2l and 2l+1 and streams each diagonal as one 16-byte load;
// UNR diagonals at a time are staged in LDS behind workgroup barriers.  Used
// when n/2 is not a multiple of 64, where the wave-per-block form below would
// leave part of a wave idle on every load.
// Columns [i0, i0 + w) of an image with nh columns: the launch's block b
// solves factor/image block (t, i) = (b / w, i0 + b % w), index t * nh + i.
// The full image is i0 = 0, w = nh, where the mapping is the identity.
struct ColRange {
  int i0, w, nh;
};
__device__ __forceinline__ size_t range_block(const ColRange& c, unsigned b) {
  return (size_t)(b / (unsigned)c.w) * c.nh + c.i0 + b % (unsigned)c.w;
}

template <int MODE, int UNR>
__global__ __launch_bounds__(256) void k_xupdate_pairs(const float2* __restrict__ W, FactorLayout L, ColRange cr,
                                                       const float2* hy, const float2* __restrict__ m,
                                                       float2* __restrict__ d2, float2* x, float mu) {
  extern __shared__ float2 lds[];
  const int n = L.n, h = n >> 1, F = L.F;
  float2* bsh = lds;      // [n]   right-hand side
  float2* dsh = lds + n;  // [UNR][n] staged diagonals
  const int l = threadIdx.x;
  const bool act = l < h;
  const size_t blk = range_block(cr, blockIdx.x);
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

// Wave-per-block form (even n): one wave solves a block alone, so no
// workgroup barrier is needed.  Lane l owns the row pairs (2q, 2q+1),
// q = l + 64 r, r < RP; each diagonal is one 16-byte non-temporal load per
// pair.  Diagonals are handled UNR at a time through wave-private LDS (the
// rotated operand c_s[k-s] of the Hermitian mirror belongs to another lane),
// and the next UNR diagonals are already in flight while the current ones
// are staged and multiplied (two register buffers, alternated by hand so
// that no copy forces an early wait).  LDS needs (1 + UNR) n values.
template <int UNR, int RP>
struct DiagChunk {
  float4 c[UNR][RP];
};

template <int UNR, int RP>
__device__ __forceinline__ void load_chunk(DiagChunk<UNR, RP>& ch, const float2* __restrict__ W, const FactorLayout& L,
                                  size_t blk, int s0, int lane) {
  const int h = L.n >> 1;
#pragma unroll
  for (int u = 0; u < UNR; ++u)
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int q = lane + 64 * r;
      ch.c[u][r] = (q < h && s0 + u < L.F) ? ld_stream4(W + diag_offset(L, blk, s0 + u) + 2 * q)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

template <int UNR, int RP>
__device__ __forceinline__ void apply_chunk(const DiagChunk<UNR, RP>& ch, const FactorLayout& L, int s0, int lane,
                                   const float2* bsh, float2* dsh, float2 (&a0)[RP], float2 (&a1)[RP]) {
  const int n = L.n, h = n >> 1;
#pragma unroll
  for (int u = 0; u < UNR; ++u)
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int q = lane + 64 * r;
      if (q < h) *reinterpret_cast<float4*>(dsh + u * n + 2 * q) = ch.c[u][r];
    }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int u = 0; u < UNR; ++u) {
    const int s = s0 + u;
    if (s < L.F) {
      const float2* d = dsh + u * n;
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const int q = lane + 64 * r;
        if (q < h) {
          const int k0 = 2 * q, k1 = 2 * q + 1;
          int p0 = k0 + s, p1 = k1 + s, q0 = k0 - s, q1 = k1 - s;
          p0 -= p0 >= n ? n : 0;
          p1 -= p1 >= n ? n : 0;
          q0 += q0 < 0 ? n : 0;
          q1 += q1 < 0 ? n : 0;
          a0[r] = cfma(make_float2(ch.c[u][r].x, ch.c[u][r].y), bsh[p0], a0[r]);
          a1[r] = cfma(make_float2(ch.c[u][r].z, ch.c[u][r].w), bsh[p1], a1[r]);
          a0[r] = cfmac(d[q0], bsh[q0], a0[r]);
          a1[r] = cfmac(d[q1], bsh[q1], a1[r]);
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
}

template <int MODE, int UNR, int RP>
__device__ __forceinline__ void xupdate_wave_block(const float2* __restrict__ W, const FactorLayout& L, size_t blk, int lane,
                                          float2* bsh, float2* dsh, const float2* hy, const float2* __restrict__ m,
                                          float2* __restrict__ d2, float2* x, float mu) {
  const int n = L.n, h = n >> 1, F = L.F;
  const size_t base = blk * (size_t)n;
  DiagChunk<UNR, RP> A, B;
  if (F > 1) load_chunk<UNR, RP>(A, W, L, blk, 1, lane);
  float2 b0[RP], b1[RP], m0[RP], m1[RP], e0[RP], e1[RP], a0[RP], a1[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int q = lane + 64 * r;
    b0[r] = b1[r] = m0[r] = m1[r] = e0[r] = e1[r] = a0[r] = a1[r] = make_float2(0.f, 0.f);
    if (q < h) {
      b0[r] = rhs_value<MODE>(hy, m, d2, base + 2 * q, mu, m0[r], e0[r]);
      b1[r] = rhs_value<MODE>(hy, m, d2, base + 2 * q + 1, mu, m1[r], e1[r]);
      const float4 c = ld_stream4(W + diag_offset(L, blk, 0) + 2 * q);
      a0[r] = cmul(make_float2(c.x, c.y), b0[r]);
      a1[r] = cmul(make_float2(c.z, c.w), b1[r]);
    }
  }
  // a previous block's epilogue of this wave may still be reading bsh; the
  // wave executes in order, so a compiler barrier is all that is needed
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int q = lane + 64 * r;
    if (q < h) *reinterpret_cast<float4*>(bsh + 2 * q) = make_float4(b0[r].x, b0[r].y, b1[r].x, b1[r].y);
  }
  __builtin_amdgcn_wave_barrier();
  for (int s0 = 1; s0 < F; s0 += 2 * UNR) {
    if (s0 + UNR < F) load_chunk<UNR, RP>(B, W, L, blk, s0 + UNR, lane);
    apply_chunk<UNR, RP>(A, L, s0, lane, bsh, dsh, a0, a1);
    if (s0 + 2 * UNR < F) load_chunk<UNR, RP>(A, W, L, blk, s0 + 2 * UNR, lane);
    if (s0 + UNR < F) apply_chunk<UNR, RP>(B, L, s0 + UNR, lane, bsh, dsh, a0, a1);
  }
  const float2* hd = W + half_offset(L, blk);
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int q = lane + 64 * r;
    if (q < h) {
      const int k0 = 2 * q, k1 = 2 * q + 1;
      a0[r] = k0 < h ? cfma(hd[k0], bsh[k0 + h], a0[r]) : cfmac(hd[k0 - h], bsh[k0 - h], a0[r]);
      a1[r] = k1 < h ? cfma(hd[k1], bsh[k1 + h], a1[r]) : cfmac(hd[k1 - h], bsh[k1 - h], a1[r]);
      *reinterpret_cast<float4*>(x + base + k0) = make_float4(a0[r].x, a0[r].y, a1[r].x, a1[r].y);
      if (MODE == kSolveTV)
        *reinterpret_cast<float4*>(d2 + base + k0) =
            make_float4(e0[r].x - (m0[r].x - a0[r].x), e0[r].y - (m0[r].y - a0[r].y),
                        e1[r].x - (m1[r].x - a1[r].x), e1[r].y - (m1[r].y - a1[r].y));
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// The same wave-per-block solve with n a compile-time constant N, the only
// sizes the phase form runs it at being N = 128, 256, 384, 512 (N/2 row pairs
// fill RP = N/128 lanes per wave exactly).  Every guard then disappears: the
// chunks of UNR diagonals tile s = 0 .. F-1 (F = N/2, a multiple of UNR) with
// diagonal 0 peeled into the first one, and the right-hand side is staged
// twice in LDS (b[k] = b[k + N]) so that b_{k+s} and b_{k-s} (mod N) are read
// at k + s and k - s + N without a wrap, as pairs with constant offsets.  The
// FMAs and their order are those of xupdate_wave_block, so the results are
// bit-identical.  LDS: 2N right-hand side values, UNR N staged diagonals.
template <int MODE, int N, int UNR>
struct WaveSolveN {
  static constexpr int H = N / 2, F = N / 2, RP = N / 128, NCH = F / UNR;
  static_assert(N % 128 == 0 && F % UNR == 0, "wave solve sizes");
  static constexpr size_t kLdsValues = (size_t)(2 + UNR) * N;

  static __device__ __forceinline__ void load(float4 (&c)[UNR][RP], const float2* __restrict__ W,
                                               const FactorLayout& L, size_t blk, int s0, int lane) {
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int r = 0; r < RP; ++r) c[u][r] = ld_stream4(W + diag_offset(L, blk, s0 + u) + 2 * (lane + 64 * r));
  }

  // diagonals s0 .. s0 + UNR - 1 (FIRST: s0 = 0, whose diagonal 0 starts the sums)
  template <bool FIRST>
  static __device__ __forceinline__ void apply(const float4 (&c)[UNR][RP], int s0, int lane, const float2* bsh,
                                                float2* dsh, float2 (&a0)[RP], float2 (&a1)[RP]) {
#pragma unroll
    for (int u = FIRST ? 1 : 0; u < UNR; ++u)
#pragma unroll
      for (int r = 0; r < RP; ++r) *reinterpret_cast<float4*>(dsh + u * N + 2 * (lane + 64 * r)) = c[u][r];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int k0 = 2 * (lane + 64 * r);
      const float2* bp = bsh + k0 + s0;                  // b_{k0+s} = bp[u]
      const float2* bm = bsh + k0 + N - s0 - (UNR - 1);  // b_{k0-s} = bm[UNR - 1 - u]
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        if (FIRST && u == 0) {
          a0[r] = cmul(make_float2(c[0][r].x, c[0][r].y), bp[0]);
          a1[r] = cmul(make_float2(c[0][r].z, c[0][r].w), bp[1]);
          continue;
        }
        const int s = s0 + u;
        const float2* d = dsh + u * N;
        int q0 = k0 - s, q1 = k0 + 1 - s;
        q0 += q0 < 0 ? N : 0;
        q1 += q1 < 0 ? N : 0;
        a0[r] = cfma(make_float2(c[u][r].x, c[u][r].y), bp[u], a0[r]);
        a1[r] = cfma(make_float2(c[u][r].z, c[u][r].w), bp[u + 1], a1[r]);
        a0[r] = cfmac(d[q0], bm[UNR - 1 - u], a0[r]);
        a1[r] = cfmac(d[q1], bm[UNR - u], a1[r]);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }

  static __device__ __forceinline__ void solve(const float2* __restrict__ W, const FactorLayout& L, size_t blk,
                                                int lane, float2* bsh, float2* dsh, const float2* hy,
                                                const float2* __restrict__ m, float2* __restrict__ d2, float2* x,
                                                float mu) {
    const size_t base = blk * (size_t)N;
    float4 A[UNR][RP], B[UNR][RP];
    load(A, W, L, blk, 0, lane);
    float2 m0[RP], m1[RP], e0[RP], e1[RP], a0[RP], a1[RP];
    // a previous block's epilogue of this wave may still be reading bsh; the
    // wave executes in order, so a compiler barrier is all that is needed
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int q = lane + 64 * r;
      const float2 b0 = rhs_value<MODE>(hy, m, d2, base + 2 * q, mu, m0[r], e0[r]);
      const float2 b1 = rhs_value<MODE>(hy, m, d2, base + 2 * q + 1, mu, m1[r], e1[r]);
      const float4 bb = make_float4(b0.x, b0.y, b1.x, b1.y);
      *reinterpret_cast<float4*>(bsh + 2 * q) = bb;
      *reinterpret_cast<float4*>(bsh + N + 2 * q) = bb;
    }
    __builtin_amdgcn_wave_barrier();
    // chunk c covers s = c UNR .. c UNR + UNR - 1: A holds the even chunks and
    // B the odd ones, the next chunk's loads in flight during this one's work
    if (NCH > 1) load(B, W, L, blk, UNR, lane);
    apply<true>(A, 0, lane, bsh, dsh, a0, a1);
    for (int c = 1; c + 1 < NCH; c += 2) {
      load(A, W, L, blk, (c + 1) * UNR, lane);
      apply<false>(B, c * UNR, lane, bsh, dsh, a0, a1);
      if (c + 2 < NCH) load(B, W, L, blk, (c + 2) * UNR, lane);
      apply<false>(A, (c + 1) * UNR, lane, bsh, dsh, a0, a1);
    }
    if (NCH % 2 == 0) apply<false>(B, (NCH - 1) * UNR, lane, bsh, dsh, a0, a1);
    const float2* hd = W + half_offset(L, blk);
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int k0 = 2 * (lane + 64 * r), k1 = k0 + 1;
      a0[r] = k0 < H ? cfma(hd[k0], bsh[k0 + H], a0[r]) : cfmac(hd[k0 - H], bsh[k0 - H], a0[r]);
      a1[r] = k1 < H ? cfma(hd[k1], bsh[k1 + H], a1[r]) : cfmac(hd[k1 - H], bsh[k1 - H], a1[r]);
      *reinterpret_cast<float4*>(x + base + k0) = make_float4(a0[r].x, a0[r].y, a1[r].x, a1[r].y);
      if (MODE == kSolveTV)
        *reinterpret_cast<float4*>(d2 + base + k0) =
            make_float4(e0[r].x - (m0[r].x - a0[r].x), e0[r].y - (m0[r].y - a0[r].y),
                        e1[r].x - (m1[r].x - a1[r].x), e1[r].y - (m1[r].y - a1[r].y));
    }
    __builtin_amdgcn_wave_barrier();
  }
};

template <int MODE, int N, int UNR>
__global__ __launch_bounds__(64) void k_xupdate_wave(const float2* __restrict__ W, FactorLayout L, ColRange cr,
                                                     const float2* hy, const float2* __restrict__ m,
                                                     float2* __restrict__ d2, float2* x, float mu) {
  extern __shared__ float2 lds[];
  WaveSolveN<MODE, N, UNR>::solve(W, L, range_block(cr, blockIdx.x), threadIdx.x, lds, lds + 2 * N, hy, m, d2, x,
                                  mu);
}

// Odd n: lane k owns row k; the rotated c_s[k-s] is re-read from the same
// diagonal run, which the vector cache serves.
template <int MODE>
__global__ __launch_bounds__(512) void k_xupdate_rows(const float2* __restrict__ W, FactorLayout L, ColRange cr,
                                                      const float2* hy, const float2* __restrict__ m,
                                                      float2* __restrict__ d2, float2* x, float mu) {
  extern __shared__ float2 bsh[];
  const int n = L.n;
  const int k = threadIdx.x;
  const size_t blk = range_block(cr, blockIdx.x);
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

// diagonals per chunk of the phase-form x-update: 4 streams faster than 8 on
// gfx950 (256-row blocks: 353 vs 373 us per 2.24 GB launch), 16 starves occupancy
constexpr int kXUnroll = 4;
constexpr int kXUnrollCol = 4;  // diagonals per chunk, column-resident solve (8 waves share a CU's LDS)

// row pairs per lane: nv/2 pairs over 64 lanes
inline int pairs_per_lane(int n) { return ((n >> 1) + 63) / 64; }

// diagonals per chunk of the compile-time-n wave solve: 2.  Measured at n = 256
// (256x256x32 blocks, one box, two interleaved rounds): 355.1-356.8 us with 2,
// 358.9-359.9 us with 4 and 356.2-358.9 us with 8, against 363.4-365.5 us for
// the run-time-n form above; a loads-only stream of the same factor layout
// takes 308.7-309.3 us.  Neither loading the half diagonal with the first
// chunk nor persistent waves that prefetch the next block changed the time.
template <int N>
constexpr int wave_unroll() { return 2; }

template <int MODE, int N>
static void xupdate_wave_launch(cs_plan* p, const ColRange& cr, const float2* hy, const float2* m, float2* d2,
                                float2* x, float mu, hipStream_t s) {
  constexpr int UNR = wave_unroll<N>();
  using K = WaveSolveN<MODE, N, UNR>;
  const size_t lds = K::kLdsValues * sizeof(float2);
  const unsigned grid = (unsigned)cr.w * (unsigned)p->desc.nt;
  hipLaunchKernelGGL((k_xupdate_wave<MODE, N, UNR>), dim3(grid), dim3(64), lds, s, p->factor, p->flayout, cr, hy,
                     m, d2, x, mu);
}

template <int MODE>
static void xupdate_launch(cs_plan* p, const ColRange& cr, const float2* hy, const float2* m, float2* d2, float2* x,
                           float mu, hipStream_t s) {
  const FactorLayout& L = p->flayout;
  const int n = L.n;
  const uint32_t f = p->desc.flags;
  const unsigned grid = (unsigned)cr.w * (unsigned)p->desc.nt;
  // the wave form runs at n = 128, 256, 384, 512 (n/2 a multiple of 64); the
  // workgroup form covers every other even n (n = 64 and 192 normally take the
  // two-blocks-per-wave form before reaching here)
  const bool wave = n % 128 == 0 && !(f & CS_FLAG_XU_GROUP);
  if (wave) {
    if (n == 128) xupdate_wave_launch<MODE, 128>(p, cr, hy, m, d2, x, mu, s);
    else if (n == 256) xupdate_wave_launch<MODE, 256>(p, cr, hy, m, d2, x, mu, s);
    else if (n == 384) xupdate_wave_launch<MODE, 384>(p, cr, hy, m, d2, x, mu, s);
    else xupdate_wave_launch<MODE, 512>(p, cr, hy, m, d2, x, mu, s);
  } else if ((n & 1) == 0) {
    const int wg = (std::max(n / 2, 1) + 63) / 64 * 64;
    const size_t lds = (size_t)(1 + kXUnroll) * n * sizeof(float2);
    hipLaunchKernelGGL((k_xupdate_pairs<MODE, kXUnroll>), dim3(grid), dim3(wg), lds, s, p->factor, L, cr, hy, m, d2,
                       x, mu);
  } else {
    const int wg = (n + 63) / 64 * 64;
    hipLaunchKernelGGL(k_xupdate_rows<MODE>, dim3(grid), dim3(wg), (size_t)n * sizeof(float2), s, p->factor, L, cr,
                       hy, m, d2, x, mu);
  }
}

int launch_block_solve_cols(cs_plan* p, int mode, const float2* hy, const float2* m, float2* d2, float2* x,
                            float mu, int i0, int i1, hipStream_t s) {
  if (i1 <= i0) return CS_OK;
  const ColRange cr{i0, i1 - i0, p->desc.nh};
  if (mode == kSolveTV) xupdate_launch<kSolveTV>(p, cr, hy, m, d2, x, mu, s);
  else if (mode == kSolveDFT) xupdate_launch<kSolveDFT>(p, cr, hy, m, d2, x, mu, s);
  else xupdate_launch<kSolvePlain>(p, cr, hy, m, d2, x, mu, s);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_block_solve(cs_plan* p, int mode, const float2* hy, const float2* m, float2* d2, float2* x,
                       float mu, hipStream_t s) {
  return launch_block_solve_cols(p, mode, hy, m, d2, x, mu, 0, p->desc.nh, s);
}

// ---------------------------------------------------------------- TV step
// (defined after the MFMA tile helpers of the temporal DFT, which it shares)

}  // namespace csmri
#include "tdft.hpp"  // the temporal DFT as a register FFT over lane groups
namespace csmri {

// ---------------------------------------------------------------- temporal DFT on MFMA
//
// The temporal DFT of 16 pixels at a time is a dense real contraction: with a
// complex series written as interleaved real rows (re z_t, im z_t), w = Psi z
// becomes What = Psihat zhat, Psihat the real 2x2-block embedding
//   [[Re P, -Im P], [Im P, Re P]]  of every entry P = Psi[f][t],
// of size 2 nt x 2 nt (zero-padded to KP = a multiple of 16).  One wave runs it
// as (KP/16) x (KP/4) v_mfma_f32_16x16x4f32 steps: A = a 16x4 block of Psihat
// (lane l holds A[l % 16][l / 16]), B = 4 rows x 16 pixels of zhat staged in
// LDS (lane l holds B[l / 16][l % 16]), accumulator lane l holds
// D[4 (l / 16) + v][l % 16], v < 4, i.e. the real and imaginary parts of two
// consecutive frequencies of pixel l % 16.  The A fragments of Psihat are
// built on the host in FP64 and held in LDS; the adjoint reuses them (see
// tile_gemm).

typedef float mfma_v4 __attribute__((ext_vector_type(4)));

template <int KP>
struct DftTile {
  static constexpr int MT = KP / 16;  // 16-row output tiles
  static constexpr int KS = KP / 4;   // 4-deep contraction steps
  static constexpr int FRAG = MT * KS * 64;  // floats per matrix
};

// acc[m] = sum_k Ahat(m, k) Bhat(k), Bhat = tile[KP][16] in LDS.  Only the
// fragments of Psihat are stored: Psi is symmetric, so the embedding of
// Psi' = conj(Psi) is Psihat with its off-diagonal entries of every 2x2 block
// negated, which for the A operand is a per-lane sign (row parity l & 1 against
// column parity (l >> 4) & 1) applied when ADJ.
template <int KP, bool ADJ>
__device__ __forceinline__ void tile_gemm(const float* __restrict__ frag, const float* tile, int lane,
                                          mfma_v4 (&acc)[DftTile<KP>::MT]) {
  constexpr int MT = DftTile<KP>::MT, KS = DftTile<KP>::KS;
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = mfma_v4{0.f, 0.f, 0.f, 0.f};
  const int col = lane & 15, grp = lane >> 4;
  const unsigned flip = (ADJ && ((lane ^ (lane >> 4)) & 1)) ? 0x80000000u : 0u;
#pragma unroll 4
  for (int k = 0; k < KS; ++k) {
    const float b = tile[(4 * k + grp) * 16 + col];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const float a = __uint_as_float(__float_as_uint(frag[(m * KS + k) * 64 + lane]) ^ flip);
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[m], 0, 0, 0);
    }
  }
}

// stage 16 pixels' series (rows 2t, 2t+1 = re, im of frame t) into tile[KP][16]
template <int KP>
__device__ __forceinline__ void tile_stage(float* tile, const float2* __restrict__ src, int nt, size_t npix, size_t p0,
                                  int count, int lane) {
  const int col = lane & 15, grp = lane >> 4;
  constexpr int NK = KP / 8;  // frames t = grp + 4k per lane
  float2 r[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {  // every load in flight before the first LDS store
    const int t = grp + 4 * k;
    r[k] = (t < nt && col < count) ? src[(size_t)t * npix + p0 + col] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int t = grp + 4 * k;
    tile[(2 * t) * 16 + col] = r[k].x;
    tile[(2 * t + 1) * 16 + col] = r[k].y;
  }
  __builtin_amdgcn_wave_barrier();
}

enum DftTileMode { kDftStep = 0, kDftForward = 1, kDftAdjoint = 2 };

// One wave, pixels p0 .. p0 + count - 1 (count <= 16), frame stride npix.
//   kDftStep:    w = Psi z (or w = wgiven); d <- d - (w - v) unless first;
//                v <- soft(w - d, tau); u <- Psi'(v + d).  Writes d, v, u.
//   kDftForward: out = Psi in; with dual != null also dual <- dual - (out - v).
//   kDftAdjoint: out = Psi' in.
template <int KP, int MODE>
__device__ __forceinline__ void dft_tile(const float* __restrict__ frag, float* tile,
                                const float2* __restrict__ in, float2* __restrict__ d, float2* __restrict__ v,
                                float2* __restrict__ out, const float2* __restrict__ wgiven, int nt, size_t npix,
                                size_t p0, int count, float tau, int first, int lane) {
  constexpr int MT = DftTile<KP>::MT;
  const int col = lane & 15, grp = lane >> 4;
  const bool pv = col < count;
  const size_t p = p0 + col;
  mfma_v4 acc[MT];
  // the step's dual and shrinkage operands of this lane's frequencies are
  // loaded up front, so that their latency overlaps the staging and the MFMAs
  float2 dpre[MT][2], vpre[MT][2];
  if (MODE == kDftStep) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f = 8 * m + 2 * grp + h;
        const bool ok = f < nt && pv;
        dpre[m][h] = ok ? d[(size_t)f * npix + p] : make_float2(0.f, 0.f);
        vpre[m][h] = (ok && !first) ? v[(size_t)f * npix + p] : make_float2(0.f, 0.f);
      }
  }
  if (MODE == kDftStep && wgiven) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f = 8 * m + 2 * grp + h;
        const float2 w = (f < nt && pv) ? wgiven[(size_t)f * npix + p] : make_float2(0.f, 0.f);
        acc[m][2 * h] = w.x;
        acc[m][2 * h + 1] = w.y;
      }
  } else {
    tile_stage<KP>(tile, in, nt, npix, p0, count, lane);
    tile_gemm<KP, MODE == kDftAdjoint>(frag, tile, lane, acc);
    __builtin_amdgcn_wave_barrier();
  }
  if (MODE != kDftStep) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f = 8 * m + 2 * grp + h;
        if (f < nt && pv) {
          const float2 w = make_float2(acc[m][2 * h], acc[m][2 * h + 1]);
          out[(size_t)f * npix + p] = w;
          if (MODE == kDftForward && d) {
            const float2 vf = v[(size_t)f * npix + p];
            const float2 df = d[(size_t)f * npix + p];
            d[(size_t)f * npix + p] = make_float2(df.x - (w.x - vf.x), df.y - (w.y - vf.y));
          }
        }
      }
    return;
  }
  // dual update, shrinkage and q = v + d, written back as the rows of qhat
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int f = 8 * m + 2 * grp + h;
      const int row = 16 * m + 4 * grp + 2 * h;
      float2 q = make_float2(0.f, 0.f);
      if (f < nt && pv) {
        const float2 w = make_float2(acc[m][2 * h], acc[m][2 * h + 1]);
        float2 df = dpre[m][h];
        if (!first) {
          const float2 vp = vpre[m][h];
          df = make_float2(df.x - (w.x - vp.x), df.y - (w.y - vp.y));
        }
        const float2 vf = soft_threshold(csub(w, df), tau);
        d[(size_t)f * npix + p] = df;
        v[(size_t)f * npix + p] = vf;
        q = cadd(vf, df);
      }
      tile[row * 16 + col] = q.x;
      tile[(row + 1) * 16 + col] = q.y;
    }
  __builtin_amdgcn_wave_barrier();
  tile_gemm<KP, true>(frag, tile, lane, acc);
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = 8 * m + 2 * grp + h;
      if (t < nt && pv) out[(size_t)t * npix + p] = make_float2(acc[m][2 * h], acc[m][2 * h + 1]);
    }
  __builtin_amdgcn_wave_barrier();
}

// load / store at a wave-uniform base plus a 32-bit per-lane byte offset
__device__ __forceinline__ float2 ld_off(const float2* __restrict__ base, uint32_t off) {
  return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(base) + off);
}
__device__ __forceinline__ void st_off(float2* __restrict__ base, uint32_t off, float2 v) {
  *reinterpret_cast<float2*>(reinterpret_cast<char*>(base) + off) = v;
}

// The same three modes as dft_tile, for nt = L N2 (tdft_lanes(nt) = L), with
// Psi as the lane-group FFT of tdft.hpp: lane l, member j of group g in the
// lane layout GroupLane<L, STRIDED>, on pixel g and frames j + L n2, or
// frequencies k2 + N2 bitrev(j) after the forward transform; 64 / L pixels
// per wave.  No LDS and no matrix cores.  Every lane of the wave runs the
// transforms (the lane exchanges read the partner lanes).  Each pixel goes
// through the same operations in either layout, so both give the same bits.
template <int L, int N2, int MODE, bool STRIDED = false>
__device__ __forceinline__ void dft_fft_tile(const float2* __restrict__ in, float2* __restrict__ d,
                                             float2* __restrict__ v, float2* __restrict__ out,
                                             const float2* __restrict__ wgiven, size_t npix, size_t p0, int count,
                                             float tau, int first, int lane, const GroupRoots<L, N2>& roots) {
  using GL = GroupLane<L, STRIDED>;
  constexpr float kScale = (float)cx_rsqrt(L * N2);  // 1 / sqrt(nt): Psi is unitary
  const int col = GL::group(lane), j = GL::member(lane);
  const int k1 = lane_bitrev<L>(j);
  const bool pv = col < count;
  // Addresses: a wave-uniform base per frame or frequency (from p0) plus one
  // 32-bit byte offset per lane (8 nt npix < 2^32 for every supported size).
  // Lanes past the tile's last pixel read that pixel (a group's lanes share
  // their pixel, so its values never mix with a real pixel's) and store
  // nothing.
  const uint32_t cc = (uint32_t)min(col, count - 1);
  const uint32_t offT = 8u * (cc + (uint32_t)(j * npix)), offF = 8u * (cc + (uint32_t)(N2 * k1 * npix));
  const size_t strideT = (size_t)L * npix;
  float2 x[N2];
  // the step's dual and shrinkage operands of this lane's frequencies are
  // requested first, so that their latency overlaps the transform
  float2 dpre[N2], vpre[N2];
  if (MODE == kDftStep) {
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const size_t bk = p0 + (size_t)k * npix;
      dpre[k] = ld_off(d + bk, offF);
      vpre[k] = first ? make_float2(0.f, 0.f) : ld_off(v + bk, offF);
    }
  }
  if (MODE == kDftStep && wgiven) {
#pragma unroll
    for (int k = 0; k < N2; ++k) x[k] = ld_off(wgiven + p0 + (size_t)k * npix, offF);
  } else if (MODE == kDftAdjoint) {
#pragma unroll
    for (int k = 0; k < N2; ++k) x[k] = ld_off(in + p0 + (size_t)k * npix, offF);
  } else {
#pragma unroll
    for (int n = 0; n < N2; ++n) x[n] = ld_off(in + p0 + (size_t)n * strideT, offT);
    group_fft_time_to_freq<L, N2, -1, GL::LS>(x, j, roots);
#pragma unroll
    for (int k = 0; k < N2; ++k) x[k] = cscale(x[k], kScale);
  }
  if (MODE == kDftForward) {
    if (pv) {
#pragma unroll
      for (int k = 0; k < N2; ++k) {
        const size_t bk = p0 + (size_t)k * npix;
        st_off(out + bk, offF, x[k]);
        if (d) {
          const float2 vf = ld_off(v + bk, offF), df = ld_off(d + bk, offF);
          st_off(d + bk, offF, make_float2(df.x - (x[k].x - vf.x), df.y - (x[k].y - vf.y)));
        }
      }
    }
    return;
  }
  if (MODE == kDftStep) {
    // dual update, shrinkage and q = v + d, in place of w
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const float2 w = x[k];
      float2 df = dpre[k];
      if (!first) df = make_float2(df.x - (w.x - vpre[k].x), df.y - (w.y - vpre[k].y));
      const float2 vf = soft_threshold(csub(w, df), tau);
      if (pv) {
        const size_t bk = p0 + (size_t)k * npix;
        st_off(d + bk, offF, df);
        st_off(v + bk, offF, vf);
      }
      x[k] = cadd(vf, df);
    }
  }
  group_fft_freq_to_time<L, N2, +1, GL::LS>(x, j, roots);
  if (pv) {
#pragma unroll
    for (int n = 0; n < N2; ++n) st_off(out + p0 + (size_t)n * strideT, offT, cscale(x[n], kScale));
  }
}

// phase-kernel form of the group-FFT step: 4 waves per workgroup, one tile of
// 64 / L pixels per wave in a grid-stride loop, the groups' lanes strided so
// that consecutive lanes touch consecutive pixels of one frame (measured on
// 192 x 192 x 40: 15.9 us per launch against 22.8 us with each pixel's lanes
// adjacent, whose loads touch a different frame every lane)
template <int L, int N2, int MODE>
__global__ __launch_bounds__(256) void k_dft_fft(const float2* __restrict__ in, float2* __restrict__ d,
                                                 float2* __restrict__ v, float2* __restrict__ out,
                                                 const float2* __restrict__ wgiven, size_t npix, size_t pix0,
                                                 size_t pix1, float tau, int first) {
  constexpr int P = 64 / L;  // pixels per wave
  // the wave index is uniform over the wave: said so, the tile's base
  // addresses stay in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (pix1 - pix0 + P - 1) / P;
  const GroupRoots<L, N2> roots = group_roots<L, N2>(GroupLane<L, true>::member(lane));
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = pix0 + tl * P;
    const int count = (int)std::min<size_t>(P, pix1 - p0);
    dft_fft_tile<L, N2, MODE, true>(in, d, v, out, wgiven, npix, p0, count, tau, first, lane, roots);
  }
}

// The DFT step of one 16-pixel tile by the group FFT when tdft_lanes(nt) is
// not 0 (for a padded size KP: 8 lanes with N2 = KP / 16, or 4 lanes with an
// odd N2 = KP / 8 - 1), else by the MFMA contraction.  The phase kernels
// choose the same way, so every form computes the step with the same
// arithmetic.  nt is uniform over the wave.
template <int KP, int MODE>
__device__ __forceinline__ void dft_tile_any(const float* __restrict__ frag, float* tile,
                                             const float2* __restrict__ in, float2* __restrict__ d,
                                             float2* __restrict__ v, float2* __restrict__ out,
                                             const float2* __restrict__ wgiven, int nt, size_t npix, size_t p0,
                                             int count, float tau, int first, int lane) {
  constexpr int k8 = KP / 16, k4 = KP / 8 - 1;
  if constexpr (tdft_len_ok(k8)) {
    if (nt == 8 * k8 && tdft_lanes(nt) == 8) {  // two 8-pixel halves
      const GroupRoots<8, k8> roots = group_roots<8, k8>(lane % 8);
      dft_fft_tile<8, k8, MODE>(in, d, v, out, wgiven, npix, p0, std::min(count, 8), tau, first, lane, roots);
      if (count > 8)
        dft_fft_tile<8, k8, MODE>(in, d, v, out, wgiven, npix, p0 + 8, count - 8, tau, first, lane, roots);
      return;
    }
  }
  if constexpr (k4 % 2 == 1 && tdft_len_ok(k4)) {
    if (nt == 4 * k4 && tdft_lanes(nt) == 4) {
      dft_fft_tile<4, k4, MODE>(in, d, v, out, wgiven, npix, p0, count, tau, first, lane, group_roots<4, k4>(lane % 4));
      return;
    }
  }
  dft_tile<KP, MODE>(frag, tile, in, d, v, out, wgiven, nt, npix, p0, count, tau, first, lane);
}

// copy the fragment matrix into LDS (all threads of the workgroup)
// (16-byte aligned on both sides; batches of loads in flight before their stores)
template <int KP>
__device__ __forceinline__ void load_frags(float* dst, const float* __restrict__ src) {
  constexpr int N4 = DftTile<KP>::FRAG / 4;
  constexpr int BATCH = 8;
  const float4* s4 = reinterpret_cast<const float4*>(src);
  float4* d4 = reinterpret_cast<float4*>(dst);
  for (int q0 = threadIdx.x; q0 < N4; q0 += BATCH * blockDim.x) {
    float4 r[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int q = q0 + u * blockDim.x;
      r[u] = q < N4 ? s4[q] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int q = q0 + u * blockDim.x;
      if (q < N4) d4[q] = r[u];
    }
  }
}

// phase-kernel form: blockDim/64 waves per workgroup, pixel tiles of 16 in a grid-stride loop
template <int KP, int MODE>
__global__ __launch_bounds__(256) void k_dft_tiles(const float* __restrict__ frags, const float2* __restrict__ in,
                                                   float2* __restrict__ d, float2* __restrict__ v,
                                                   float2* __restrict__ out, const float2* __restrict__ wgiven,
                                                   int nt, size_t npix, size_t pix0, size_t pix1, float tau,
                                                   int first) {
  extern __shared__ float lds_f[];
  float* frag = lds_f;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* tile = lds_f + DftTile<KP>::FRAG + wv * KP * 16;
  load_frags<KP>(lds_f, frags);
  __syncthreads();
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (pix1 - pix0 + 15) / 16;
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = pix0 + tl * 16;
    const int count = (int)std::min<size_t>(16, pix1 - p0);
    dft_tile<KP, MODE>(frag, tile, in, d, v, out, wgiven, nt, npix, p0, count, tau, first, lane);
  }
}

// padded real dimension of the embedded temporal DFT: 2 nt rounded up to 16
inline int dft_kp(int nt) { return (2 * nt + 15) / 16 * 16; }

// waves per workgroup of the phase kernels: the fragment matrix (4 KP^2
// bytes) and one KP x 16 tile per wave share the workgroup's LDS
inline int dft_waves(int kp) { return kp <= 96 ? 4 : 2; }

inline size_t dft_lds_bytes(int kp, int waves) {
  return ((size_t)(kp / 16) * (kp / 4) * 64 + (size_t)waves * kp * 16) * sizeof(float);
}

template <int L, int N2, int MODE>
static int dft_fft_launch(cs_plan* p, const float2* in, float2* d, float2* v, float2* out, const float2* wgiven,
                          float tau, int first, int i0, int i1, hipStream_t s) {
  constexpr size_t P = 64 / L;
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  const size_t pix0 = (size_t)i0 * p->desc.nv, pix1 = (size_t)i1 * p->desc.nv;
  const size_t ntiles = (pix1 - pix0 + P - 1) / P;
  // one tile per wave: the step is short and gains most from many loads in
  // flight (fewer waves with several tiles each measured slower)
  const unsigned grid = (unsigned)std::min<size_t>((ntiles + 3) / 4, 65535);
  hipLaunchKernelGGL((k_dft_fft<L, N2, MODE>), dim3(grid), dim3(256), 0, s, in, d, v, out, wgiven, npix, pix0,
                     pix1, tau, first);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

template <int KP, int MODE>
static int dft_tiles_launch(cs_plan* p, const float2* in, float2* d, float2* v, float2* out, const float2* wgiven,
                            float tau, int first, int i0, int i1, hipStream_t s) {
  constexpr int k8 = KP / 16, k4 = KP / 8 - 1;  // the group-FFT lengths whose nt has this KP
  const int nt = p->desc.nt, lanes = tdft_lanes(nt);
  if constexpr (tdft_len_ok(k8))
    if (lanes == 8 && nt == 8 * k8) return dft_fft_launch<8, k8, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
  if constexpr (k4 % 2 == 1 && tdft_len_ok(k4))
    if (lanes == 4 && nt == 4 * k4) return dft_fft_launch<4, k4, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  const size_t pix0 = (size_t)i0 * p->desc.nv, pix1 = (size_t)i1 * p->desc.nv;
  const int waves = dft_waves(KP);
  const size_t lds = dft_lds_bytes(KP, waves);
  CS_HIP_STATUS(ensure_dynamic_lds((const void*)k_dft_tiles<KP, MODE>, lds));
  const size_t ntiles = (pix1 - pix0 + 15) / 16;
  // one tile per wave where the grid fits on the chip at once (the grid-stride
  // loop covers larger images)
  const unsigned grid = (unsigned)std::min<size_t>((ntiles + waves - 1) / waves, 2048);
  hipLaunchKernelGGL((k_dft_tiles<KP, MODE>), dim3(grid), dim3(64 * waves), lds, s, p->dft_frags, in, d, v, out,
                     wgiven, p->desc.nt, npix, pix0, pix1, tau, first);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

template <int MODE>
static int dft_tiles_dispatch(cs_plan* p, const float2* in, float2* d, float2* v, float2* out,
                              const float2* wgiven, float tau, int first, int i0, int i1, hipStream_t s) {
  if (i1 <= i0) return CS_OK;
  switch (dft_kp(p->desc.nt)) {
    case 16: return dft_tiles_launch<16, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
    case 32: return dft_tiles_launch<32, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
    case 48: return dft_tiles_launch<48, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
    case 64: return dft_tiles_launch<64, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
    case 80: return dft_tiles_launch<80, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
    case 96: return dft_tiles_launch<96, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
    case 112: return dft_tiles_launch<112, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
    default: return dft_tiles_launch<128, MODE>(p, in, d, v, out, wgiven, tau, first, i0, i1, s);
  }
}

int launch_dft_step_cols(cs_plan* p, float lambda, float mu, int first, const float2* wgiven, int i0, int i1,
                         hipStream_t s) {
  const float tau = lambda / (2.0f * mu);
  return dft_tiles_dispatch<kDftStep>(p, p->s2, p->s0, p->s1, p->s3, wgiven, tau, first, i0, i1, s);
}

int launch_dft_step(cs_plan* p, float lambda, float mu, int first, const float2* wgiven, hipStream_t s) {
  return launch_dft_step_cols(p, lambda, mu, first, wgiven, 0, p->desc.nh, s);
}

int launch_dft_apply(cs_plan* p, const float2* in, float2* out, float2* dual, const float2* v, int adjoint,
                     hipStream_t s) {
  const int nh = p->desc.nh;
  if (adjoint) return dft_tiles_dispatch<kDftAdjoint>(p, in, nullptr, nullptr, out, nullptr, 0.f, 0, 0, nh, s);
  return dft_tiles_dispatch<kDftForward>(p, in, dual, const_cast<float2*>(v), out, nullptr, 0.f, 0, 0, nh, s);
}

// ---------------------------------------------------------------- TV step on MFMA
//
// Algorithm 2, lines v, m and d1 with R = D_t (D_t couples frames only):
//   v   = soft(D m + d1, tau),  tau = lambda / (2 mu1)
//   m   = (rho I + D'D)^{-1} [ D'(v - d1) + rho (x + d2) ],  rho = mu2 / mu1
//   d1 <- d1 - (v - D m)
// T = rho I + D'D is the same for every pixel, so the m-solve of 16 pixels
// is one real contraction m = T^{-1} r of the padded KT x KT inverse (built in
// FP64 on the host) with the KT x 16 real and imaginary parts of r, on
// v_mfma_f32_16x16x4f32 (fragment layout as for the temporal DFT).  The
// pointwise lines run with lane l on pixel l % 16 and frames t = l / 16 + 4 k
// (or, in 8-pixel tiles, pixel l % 8 and frames l / 8 + 8 k); values a lane
// needs from a neighbouring frame pass through the wave's LDS.
// One wave per 16 pixels gives four times the waves of a pixel-per-lane
// recurrence, which is what hides the latency of the streams.
template <int KT, int PX = 16>
__device__ __forceinline__ void tv_tile(const float* __restrict__ frag, float2* buf0, float2* buf1,
                                        float2* __restrict__ m, float2* __restrict__ d1,
                                        const float2* __restrict__ x, const float2* __restrict__ d2, int nt,
                                        size_t npix, size_t p0, int count, float tau, float rho, int lane) {
  // PX = 16 or 8 pixels per wave: lane l on pixel l % PX and frames
  // l / PX + G k (G = 64 / PX); with 8 the contraction's columns 8..15 carry
  // whatever the buffers hold and their results are dropped (each output
  // column of the product depends on its own column only)
  static_assert(PX == 16 || PX == 8, "TV tile width");
  constexpr int MT = DftTile<KT>::MT, G = 64 / PX, NK = KT / G;
  const int col = lane % PX, grp = lane / PX;
  const bool pv = col < count;
  // addresses: a wave-uniform base (p0 and the frame step of the unrolled
  // loop) plus one 32-bit byte offset per lane, the same for every stream
  // (8 nt npix < 2^32 for every supported size); lanes past the tile's last
  // pixel use its last pixel's offset and neither keep nor store a value
  const uint32_t off = 8u * ((uint32_t)min(col, count - 1) + (uint32_t)grp * (uint32_t)npix);
  // the product's output layout: lane l holds frames 16 mm + 4 (l / 16) + j of column l % 16
  const int ocol = lane & 15, ogrp = lane >> 4;
  const bool opv = ocol < PX && ocol < count;
  const uint32_t offm = 8u * ((uint32_t)min(ocol, count - 1) + 4u * (uint32_t)ogrp * (uint32_t)npix);
  // every stream is requested up front (x and d2 are first needed for r):
  // one memory round trip per tile instead of two.  Measured at 256x256x32
  // (one box, three interleaved rounds): 24.4-24.6 us against 25.6-26.1 us
  // with x and d2 loaded after the shrink; a 16-pixel tile per wave stays
  // best (two tiles per wave with the next tile's loads issued inside the
  // current one: 26.2 us at 178 VGPRs)
  float2 xv[NK], zv[NK];
  // m -> buf0, d1 -> buf1 (rows t, 16 pixels)
  {
    float2 mv[NK], dv[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + G * k;
      const bool ok = t < nt && pv;
      const size_t b = p0 + (size_t)(G * k) * npix;
      mv[k] = ok ? ld_off(m + b, off) : make_float2(0.f, 0.f);
      dv[k] = (ok && t < nt - 1) ? ld_off(d1 + b, off) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + G * k;
      const bool ok = t < nt && pv;
      const size_t b = p0 + (size_t)(G * k) * npix;
      xv[k] = ok ? ld_off(x + b, off) : make_float2(0.f, 0.f);
      zv[k] = ok ? ld_off(d2 + b, off) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + G * k;
      buf0[t * 16 + col] = mv[k];
      buf1[t * 16 + col] = dv[k];
    }
  }
  __builtin_amdgcn_wave_barrier();
  // v_t = soft(m_{t+1} - m_t + d1_t, tau); e_t = d1_t - v_t (t < nt - 1), into buf1
  {
    float2 ev[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + G * k;
      ev[k] = make_float2(0.f, 0.f);
      if (t + 1 < KT && t < nt - 1) {
        const float2 m0 = buf0[t * 16 + col], m1 = buf0[(t + 1) * 16 + col], dt = buf1[t * 16 + col];
        const float2 a = make_float2(m1.x - m0.x + dt.x, m1.y - m0.y + dt.y);
        ev[k] = csub(dt, soft_threshold(a, tau));
      }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < NK; ++k) buf1[(grp + G * k) * 16 + col] = ev[k];
  }
  __builtin_amdgcn_wave_barrier();
  // r_t = rho (x_t + d2_t) + e_t - e_{t-1}, split into real and imaginary
  // operand rows (buf0, whose m is no longer needed, as two KT x 16 float tiles)
  float* bre = reinterpret_cast<float*>(buf0);
  float* bim = bre + KT * 16;
  {
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + G * k;
      float2 r = make_float2(0.f, 0.f);
      if (t < nt) {
        const float2 e0 = buf1[t * 16 + col];
        const float2 em1 = t > 0 ? buf1[(t - 1) * 16 + col] : make_float2(0.f, 0.f);
        r = make_float2(rho * (xv[k].x + zv[k].x) + e0.x - em1.x, rho * (xv[k].y + zv[k].y) + e0.y - em1.y);
      }
      bre[t * 16 + col] = r.x;
      bim[t * 16 + col] = r.y;
    }
  }
  __builtin_amdgcn_wave_barrier();
  mfma_v4 are[MT], aim[MT];
  tile_gemm<KT, false>(frag, bre, lane, are);
  tile_gemm<KT, false>(frag, bim, lane, aim);
  __builtin_amdgcn_wave_barrier();
  // new m: accumulator lane l holds frames 16 mm + 4 (l / 16) + j of pixel l % 16
#pragma unroll
  for (int mm = 0; mm < MT; ++mm)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = 16 * mm + 4 * ogrp + j;
      const float2 mv = make_float2(are[mm][j], aim[mm][j]);
      buf0[t * 16 + ocol] = mv;
      if (t < nt && opv) st_off(m + p0 + (size_t)(16 * mm + j) * npix, offm, mv);
    }
  __builtin_amdgcn_wave_barrier();
  // d1_t <- e_t + m_{t+1} - m_t
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int t = grp + G * k;
    if (t + 1 < KT && t < nt - 1 && pv) {
      const float2 e0 = buf1[t * 16 + col], m0 = buf0[t * 16 + col], m1 = buf0[(t + 1) * 16 + col];
      st_off(d1 + p0 + (size_t)(G * k) * npix, off, make_float2(e0.x + m1.x - m0.x, e0.y + m1.y - m0.y));
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// LDS floats of one wave's two KT x 16 complex buffers
constexpr int tv_wave_floats(int kt) { return 4 * kt * 16; }
inline int tv_kt(int nt) { return (nt + 15) / 16 * 16; }

// waves per SIMD the TV kernel is compiled for: its LDS (fragments plus two
// KT x 16 buffers per wave) allows 4 at KT <= 32, where 4 waves of 4096 tiles
// fill the chip at 256 x 256 pixels in one round; larger KT keep the
// compiler's choice
template <int KT>
constexpr int tv_waves_per_eu() { return KT <= 32 ? 4 : 1; }

template <int KT, int PX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(tv_waves_per_eu<KT>()))) void k_tv_tiles(
    const float* __restrict__ frags, float2* __restrict__ m,
                                                  float2* __restrict__ d1, const float2* __restrict__ x,
                                                  const float2* __restrict__ d2, int nt, size_t npix, size_t pix0,
                                                  size_t pix1, float tau, float rho) {
  extern __shared__ float lds_f[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float2* buf0 = reinterpret_cast<float2*>(lds_f + DftTile<KT>::FRAG + wv * tv_wave_floats(KT));
  float2* buf1 = buf0 + KT * 16;
  load_frags<KT>(lds_f, frags);
  __syncthreads();
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (pix1 - pix0 + PX - 1) / PX;
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = pix0 + tl * PX;
    const int count = (int)std::min<size_t>(PX, pix1 - p0);
    tv_tile<KT, PX>(lds_f, buf0, buf1, m, d1, x, d2, nt, npix, p0, count, tau, rho, lane);
  }
}

template <int KT, int PX>
static int tv_tiles_launch_px(cs_plan* p, float tau, float rho, size_t npix, size_t pix0, size_t pix1,
                              hipStream_t s) {
  constexpr int waves = 4;
  const size_t lds = ((size_t)DftTile<KT>::FRAG + (size_t)waves * tv_wave_floats(KT)) * sizeof(float);
  CS_HIP_STATUS(ensure_dynamic_lds((const void*)k_tv_tiles<KT, PX>, lds));
  const size_t ntiles = (pix1 - pix0 + PX - 1) / PX;
  const unsigned grid = (unsigned)std::min<size_t>((ntiles + waves - 1) / waves, 65535);
  hipLaunchKernelGGL((k_tv_tiles<KT, PX>), dim3(grid), dim3(64 * waves), lds, s, p->tv_frags, p->s0, p->s1, p->s2,
                     p->s3, p->desc.nt, npix, pix0, pix1, tau, rho);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// pixels per wave of the TV step: 8 where 16-pixel tiles would leave fewer
// than kTvNarrowTiles waves (small images: twice the waves in flight).
// Measured (event-timed per launch, two rounds): 128 x 128 x 22 frames 9.7 ->
// 9.0-9.2 us with 8; 192 x 192 x 24 13.8 -> 15.1 us and 256 x 256 x 32 21.1 ->
// 23.2 us, so 16 stays above the threshold.
constexpr size_t kTvNarrowTiles = 2048;

template <int KT>
static int tv_tiles_launch(cs_plan* p, float tau, float rho, int i0, int i1, hipStream_t s) {
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  const size_t pix0 = (size_t)i0 * p->desc.nv, pix1 = (size_t)i1 * p->desc.nv;
  if ((pix1 - pix0 + 15) / 16 < kTvNarrowTiles) return tv_tiles_launch_px<KT, 8>(p, tau, rho, npix, pix0, pix1, s);
  return tv_tiles_launch_px<KT, 16>(p, tau, rho, npix, pix0, pix1, s);
}

// pixels of columns [i0, i1): the solver layout puts column i's rows at i*nv .. i*nv + nv - 1
int launch_tv_step_cols(cs_plan* p, float lambda, float mu, int i0, int i1, hipStream_t s) {
  if (i1 <= i0) return CS_OK;
  const float rho = p->desc.mu_ratio;
  const float tau = lambda * rho / (2.0f * mu);  // lambda / (2 mu1), mu1 = mu / rho
  switch (tv_kt(p->desc.nt)) {
    case 16: return tv_tiles_launch<16>(p, tau, rho, i0, i1, s);
    case 32: return tv_tiles_launch<32>(p, tau, rho, i0, i1, s);
    case 48: return tv_tiles_launch<48>(p, tau, rho, i0, i1, s);
    default: return tv_tiles_launch<64>(p, tau, rho, i0, i1, s);
  }
}

int launch_tv_step(cs_plan* p, float lambda, float mu, hipStream_t s) {
  return launch_tv_step_cols(p, lambda, mu, 0, p->desc.nh, s);
}

// ---------------------------------------------------------------- overcomplete temporal frame
//
// Algorithm 1 with the tight frame Psi = [I; F] / sqrt(2) (identity and the
// unitary temporal DFT F; Psi'Psi = I, Psi Psi' != I).  Coefficient arrays
// hold 2 nt frames: the identity part (frames 0..nt-1) over the DFT part
// (frames nt..2nt-1).  With u = Psi'(v + d) and x~ = (mu I + H'H)^{-1}(H'y +
// mu u), the w-update of Algorithm 1 (including its (1/mu)(I - Psi Psi') term,
// Sec. IV-A) is w = (v + d) + Psi (x~ - u), because Psi'q = H'y + mu u for
// q = Psi H'y + mu (v + d); and Psi' w = x~.  So one iteration is one
// per-pixel pass (finish the previous iteration's w and d, shrink, form u)
// plus the x-update with right-hand side H'y + mu u.  Both transforms of a
// pass run on the group FFT where it applies (else on the MFMA DFT tiles); the
// identity part needs no arithmetic.
//   kFrameFirst:   v = soft(w - d, tau), u = Psi'(v + d) from the given w (d kept)
//   kFrameStep:    w = v + d + Psi(x~ - u); d <- d - (w - v); v = soft(w - d, tau);
//                  u = Psi'(v + d)
//   kFrameFinish:  w = v + d + Psi(x~ - u); d <- d - (w - v); writes w, d
//   kFrameForward: w = Psi x
//   kFrameAdjoint: x = Psi' w
enum FrameMode { kFrameFirst = 0, kFrameStep = 1, kFrameFinish = 2, kFrameForward = 3, kFrameAdjoint = 4 };
constexpr float kInvSqrt2 = 0.70710678118654752440f;

template <int KP, int MODE>
__device__ __forceinline__ void frame_tile(const float* __restrict__ frag, float* tile, const float2* __restrict__ xt,
                                           float2* __restrict__ u, float2* __restrict__ v, float2* __restrict__ d,
                                           float2* __restrict__ w, int nt, size_t npix, size_t p0, int count,
                                           float tau, int lane) {
  constexpr int MT = DftTile<KP>::MT;
  const int col = lane & 15, grp = lane >> 4;
  const bool pv = col < count;
  const size_t p = p0 + col;
  mfma_v4 acc[MT];
  if (MODE == kFrameForward) {
    tile_stage<KP>(tile, xt, nt, npix, p0, count, lane);
    tile_gemm<KP, false>(frag, tile, lane, acc);
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f = 8 * m + 2 * grp + h;
        if (f < nt && pv) {
          const float2 xf = make_float2(tile[(2 * f) * 16 + col], tile[(2 * f + 1) * 16 + col]);
          w[(size_t)f * npix + p] = cscale(xf, kInvSqrt2);
          w[(size_t)(nt + f) * npix + p] = cscale(make_float2(acc[m][2 * h], acc[m][2 * h + 1]), kInvSqrt2);
        }
      }
    __builtin_amdgcn_wave_barrier();
    return;
  }
  float2 qI[MT][2];
  if (MODE == kFrameAdjoint) {
    // stage the DFT part of w, keep the identity part for the sum
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f = 8 * m + 2 * grp + h;
        const bool ok = f < nt && pv;
        const float2 wf = ok ? w[(size_t)(nt + f) * npix + p] : make_float2(0.f, 0.f);
        qI[m][h] = ok ? w[(size_t)f * npix + p] : make_float2(0.f, 0.f);
        tile[(2 * f) * 16 + col] = wf.x;
        tile[(2 * f + 1) * 16 + col] = wf.y;
      }
  } else {
    // Psi (x~ - u): the DFT part from the MFMA tile, the identity part from the staged e
    float2 peI[MT][2], peF[MT][2];
    if (MODE != kFrameFirst) {
      constexpr int NK = KP / 8;
      float2 r[NK];
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int t = grp + 4 * k;
        const bool ok = t < nt && pv;
        const float2 a = ok ? xt[(size_t)t * npix + p] : make_float2(0.f, 0.f);
        const float2 b = ok ? u[(size_t)t * npix + p] : make_float2(0.f, 0.f);
        r[k] = csub(a, b);
      }
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int t = grp + 4 * k;
        tile[(2 * t) * 16 + col] = r[k].x;
        tile[(2 * t + 1) * 16 + col] = r[k].y;
      }
      __builtin_amdgcn_wave_barrier();
      tile_gemm<KP, false>(frag, tile, lane, acc);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int f = 8 * m + 2 * grp + h;
          peF[m][h] = cscale(make_float2(acc[m][2 * h], acc[m][2 * h + 1]), kInvSqrt2);
          peI[m][h] = cscale(make_float2(tile[(2 * f) * 16 + col], tile[(2 * f + 1) * 16 + col]), kInvSqrt2);
        }
      __builtin_amdgcn_wave_barrier();
    }
    // coefficient updates, identity part (c = f) and DFT part (c = nt + f)
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f = 8 * m + 2 * grp + h;
        float2 qF = make_float2(0.f, 0.f);
        qI[m][h] = make_float2(0.f, 0.f);
        if (f < nt && pv) {
#pragma unroll
          for (int part = 0; part < 2; ++part) {
            const size_t o = (size_t)(part ? nt + f : f) * npix + p;
            float2 dv = d[o], q;
            if (MODE == kFrameFirst) {
              const float2 vn = soft_threshold(csub(w[o], dv), tau);
              v[o] = vn;
              q = cadd(vn, dv);
            } else {
              const float2 vv = v[o];
              const float2 wv = cadd(cadd(vv, dv), part ? peF[m][h] : peI[m][h]);
              dv = csub(dv, csub(wv, vv));
              if (MODE == kFrameFinish) {
                w[o] = wv;
                d[o] = dv;
                q = make_float2(0.f, 0.f);
              } else {
                const float2 vn = soft_threshold(csub(wv, dv), tau);
                v[o] = vn;
                d[o] = dv;
                q = cadd(vn, dv);
              }
            }
            if (part) qF = q;
            else qI[m][h] = q;
          }
        }
        if (MODE != kFrameFinish) {
          tile[(2 * f) * 16 + col] = qF.x;
          tile[(2 * f + 1) * 16 + col] = qF.y;
        }
      }
    if (MODE == kFrameFinish) return;
  }
  // u = Psi' q = (q_identity + F' q_dft) / sqrt(2)  (x for kFrameAdjoint)
  __builtin_amdgcn_wave_barrier();
  tile_gemm<KP, true>(frag, tile, lane, acc);
  float2* out = MODE == kFrameAdjoint ? const_cast<float2*>(xt) : u;
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = 8 * m + 2 * grp + h;
      if (t < nt && pv)
        out[(size_t)t * npix + p] =
            cscale(cadd(make_float2(acc[m][2 * h], acc[m][2 * h + 1]), qI[m][h]), kInvSqrt2);
    }
  __builtin_amdgcn_wave_barrier();
}

// frame_tile with F as the lane-group FFT (nt = L N2, tdft_lanes(nt) = L):
// 64 / L pixels per wave.  The identity part of the coefficients is handled
// in the frame layout (lane j: frames j + L n2), the DFT part in the
// frequency layout (lane j: k2 + N2 bitrev(j)); each coefficient is updated
// on its own, so only the sum u = (q_I + F' q_F) / sqrt(2) combines them.
template <int L, int N2, int MODE>
__device__ __forceinline__ void frame_fft_tile(const float2* __restrict__ xt, float2* __restrict__ u,
                                               float2* __restrict__ v, float2* __restrict__ d,
                                               float2* __restrict__ w, int nt, size_t npix, size_t p0, int count,
                                               float tau, int lane, const GroupRoots<L, N2>& roots) {
  constexpr float kScale = (float)cx_rsqrt(L * N2);
  using GL = GroupLane<L, true>;  // lanes along the pixels (see k_dft_fft)
  const int col = GL::group(lane), j = GL::member(lane);
  const int k1 = lane_bitrev<L>(j);
  const bool pv = col < count;
  const uint32_t cc = (uint32_t)min(col, count - 1);
  const uint32_t offT = 8u * (cc + (uint32_t)(j * npix)), offF = 8u * (cc + (uint32_t)(N2 * k1 * npix));
  const size_t strideT = (size_t)L * npix;
  const size_t partF = (size_t)nt * npix;  // the DFT part's first coefficient frame
  float2 xI[N2], xF[N2];  // frame layout, frequency layout
  if (MODE == kFrameForward) {
#pragma unroll
    for (int n = 0; n < N2; ++n) xI[n] = ld_off(xt + p0 + (size_t)n * strideT, offT);
#pragma unroll
    for (int n = 0; n < N2; ++n) xF[n] = xI[n];
    group_fft_time_to_freq<L, N2, -1, GL::LS>(xF, j, roots);
    if (pv) {
#pragma unroll
      for (int n = 0; n < N2; ++n) st_off(w + p0 + (size_t)n * strideT, offT, cscale(xI[n], kInvSqrt2));
#pragma unroll
      for (int k = 0; k < N2; ++k)
        st_off(w + partF + p0 + (size_t)k * npix, offF, cscale(cscale(xF[k], kScale), kInvSqrt2));
    }
    return;
  }
  if (MODE == kFrameAdjoint) {
#pragma unroll
    for (int n = 0; n < N2; ++n) xI[n] = ld_off(w + p0 + (size_t)n * strideT, offT);
#pragma unroll
    for (int k = 0; k < N2; ++k) xF[k] = ld_off(w + partF + p0 + (size_t)k * npix, offF);
  } else {
    // every operand is requested before the transform: the identity part's
    // (frame layout) and the DFT part's (frequency layout) d and v, and w or
    // the x~ and u of e = x~ - u
    float2 dI[N2], dF[N2], vI[N2], vF[N2], peI[N2], peF[N2];
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const size_t bI = p0 + (size_t)k * strideT, bF = partF + p0 + (size_t)k * npix;
      dI[k] = ld_off(d + bI, offT);
      dF[k] = ld_off(d + bF, offF);
      if (MODE == kFrameFirst) {  // v <- soft(w - d): w in place of v
        vI[k] = ld_off(w + bI, offT);
        vF[k] = ld_off(w + bF, offF);
      } else {
        vI[k] = ld_off(v + bI, offT);
        vF[k] = ld_off(v + bF, offF);
        peI[k] = csub(ld_off(xt + bI, offT), ld_off(u + bI, offT));
      }
    }
    // Psi (x~ - u): the identity part e / sqrt(2), the DFT part F e / sqrt(2)
    if (MODE != kFrameFirst) {
#pragma unroll
      for (int n = 0; n < N2; ++n) peF[n] = peI[n];
      group_fft_time_to_freq<L, N2, -1, GL::LS>(peF, j, roots);
#pragma unroll
      for (int k = 0; k < N2; ++k) {
        peF[k] = cscale(cscale(peF[k], kScale), kInvSqrt2);
        peI[k] = cscale(peI[k], kInvSqrt2);
      }
    }
    // coefficient updates: part 0 the identity (frame layout), part 1 the DFT
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
      for (int k = 0; k < N2; ++k) {
        const size_t b = part ? partF + p0 + (size_t)k * npix : p0 + (size_t)k * strideT;
        const uint32_t off = part ? offF : offT;
        float2 dv = part ? dF[k] : dI[k], q;
        if (MODE == kFrameFirst) {
          const float2 vn = soft_threshold(csub(part ? vF[k] : vI[k], dv), tau);
          if (pv) st_off(v + b, off, vn);
          q = cadd(vn, dv);
        } else {
          const float2 vv = part ? vF[k] : vI[k];
          const float2 wv = cadd(cadd(vv, dv), part ? peF[k] : peI[k]);
          dv = csub(dv, csub(wv, vv));
          if (MODE == kFrameFinish) {
            if (pv) {
              st_off(w + b, off, wv);
              st_off(d + b, off, dv);
            }
            q = make_float2(0.f, 0.f);
          } else {
            const float2 vn = soft_threshold(csub(wv, dv), tau);
            if (pv) {
              st_off(v + b, off, vn);
              st_off(d + b, off, dv);
            }
            q = cadd(vn, dv);
          }
        }
        if (part) xF[k] = q;
        else xI[k] = q;
      }
    }
    if (MODE == kFrameFinish) return;
  }
  // u = Psi' q = (q_identity + F' q_dft) / sqrt(2)  (x for kFrameAdjoint)
  group_fft_freq_to_time<L, N2, +1, GL::LS>(xF, j, roots);
  float2* out = MODE == kFrameAdjoint ? const_cast<float2*>(xt) : u;
  if (pv) {
#pragma unroll
    for (int n = 0; n < N2; ++n)
      st_off(out + p0 + (size_t)n * strideT, offT, cscale(cadd(cscale(xF[n], kScale), xI[n]), kInvSqrt2));
  }
}

template <int L, int N2, int MODE>
__global__ __launch_bounds__(256) void k_frame_fft(const float2* xt, float2* __restrict__ u, float2* __restrict__ v,
                                                   float2* __restrict__ d, float2* __restrict__ w, int nt,
                                                   size_t npix, float tau) {
  constexpr int P = 64 / L;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (npix + P - 1) / P;
  const GroupRoots<L, N2> roots = group_roots<L, N2>(GroupLane<L, true>::member(lane));
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = tl * P;
    const int count = (int)std::min<size_t>(P, npix - p0);
    frame_fft_tile<L, N2, MODE>(xt, u, v, d, w, nt, npix, p0, count, tau, lane, roots);
  }
}

template <int L, int N2, int MODE>
static int frame_fft_launch(cs_plan* p, const float2* xt, float2* u, float2* v, float2* d, float2* w, float tau,
                            hipStream_t s) {
  constexpr size_t P = 64 / L;
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  const size_t ntiles = (npix + P - 1) / P;
  const unsigned grid = (unsigned)std::min<size_t>((ntiles + 3) / 4, 65535);
  hipLaunchKernelGGL((k_frame_fft<L, N2, MODE>), dim3(grid), dim3(256), 0, s, xt, u, v, d, w, p->desc.nt, npix, tau);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

template <int KP, int MODE>
__global__ __launch_bounds__(256) void k_frame_tiles(const float* __restrict__ frags, const float2* xt,
                                                     float2* __restrict__ u, float2* __restrict__ v,
                                                     float2* __restrict__ d, float2* __restrict__ w, int nt,
                                                     size_t npix, float tau) {
  extern __shared__ float lds_f[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* tile = lds_f + DftTile<KP>::FRAG + wv * KP * 16;
  load_frags<KP>(lds_f, frags);
  __syncthreads();
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (npix + 15) / 16;
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = tl * 16;
    const int count = (int)std::min<size_t>(16, npix - p0);
    frame_tile<KP, MODE>(lds_f, tile, xt, u, v, d, w, nt, npix, p0, count, tau, lane);
  }
}

template <int KP, int MODE>
static int frame_tiles_launch(cs_plan* p, const float2* xt, float2* u, float2* v, float2* d, float2* w, float tau,
                              hipStream_t s) {
  constexpr int k8 = KP / 16, k4 = KP / 8 - 1;  // the group-FFT lengths whose nt has this KP
  const int nt = p->desc.nt, lanes = tdft_lanes(nt);
  if constexpr (tdft_len_ok(k8))
    if (lanes == 8 && nt == 8 * k8) return frame_fft_launch<8, k8, MODE>(p, xt, u, v, d, w, tau, s);
  if constexpr (k4 % 2 == 1 && tdft_len_ok(k4))
    if (lanes == 4 && nt == 4 * k4) return frame_fft_launch<4, k4, MODE>(p, xt, u, v, d, w, tau, s);
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  const int waves = dft_waves(KP);
  const size_t lds = dft_lds_bytes(KP, waves);
  CS_HIP_STATUS(ensure_dynamic_lds((const void*)k_frame_tiles<KP, MODE>, lds));
  const size_t ntiles = (npix + 15) / 16;
  const unsigned grid = (unsigned)std::min<size_t>((ntiles + waves - 1) / waves, 2048);
  hipLaunchKernelGGL((k_frame_tiles<KP, MODE>), dim3(grid), dim3(64 * waves), lds, s, p->dft_frags, xt, u, v, d, w,
                     p->desc.nt, npix, tau);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

template <int MODE>
static int frame_dispatch(cs_plan* p, const float2* xt, float2* u, float2* v, float2* d, float2* w, float tau,
                          hipStream_t s) {
  switch (dft_kp(p->desc.nt)) {
    case 16: return frame_tiles_launch<16, MODE>(p, xt, u, v, d, w, tau, s);
    case 32: return frame_tiles_launch<32, MODE>(p, xt, u, v, d, w, tau, s);
    case 48: return frame_tiles_launch<48, MODE>(p, xt, u, v, d, w, tau, s);
    case 64: return frame_tiles_launch<64, MODE>(p, xt, u, v, d, w, tau, s);
    case 80: return frame_tiles_launch<80, MODE>(p, xt, u, v, d, w, tau, s);
    case 96: return frame_tiles_launch<96, MODE>(p, xt, u, v, d, w, tau, s);
    case 112: return frame_tiles_launch<112, MODE>(p, xt, u, v, d, w, tau, s);
    default: return frame_tiles_launch<128, MODE>(p, xt, u, v, d, w, tau, s);
  }
}

// plan state for the frame prior: s0 = d, s1 = v (2 nt frames each), s2 = x~,
// s3 = u, img_tmp = w (2 nt frames)
int launch_frame_step(cs_plan* p, float lambda, float mu, int first, hipStream_t s) {
  const float tau = lambda / (2.0f * mu);
  if (first) return frame_dispatch<kFrameFirst>(p, p->s2, p->s3, p->s1, p->s0, p->img_tmp, tau, s);
  return frame_dispatch<kFrameStep>(p, p->s2, p->s3, p->s1, p->s0, p->img_tmp, tau, s);
}

int launch_frame_finish(cs_plan* p, hipStream_t s) {
  return frame_dispatch<kFrameFinish>(p, p->s2, p->s3, p->s1, p->s0, p->img_tmp, 0.f, s);
}

int launch_frame_forward(cs_plan* p, const float2* x, float2* w, hipStream_t s) {
  return frame_dispatch<kFrameForward>(p, x, nullptr, nullptr, nullptr, w, 0.f, s);
}

int launch_frame_adjoint(cs_plan* p, const float2* w, float2* x, hipStream_t s) {
  return frame_dispatch<kFrameAdjoint>(p, x, nullptr, nullptr, nullptr, const_cast<float2*>(w), 0.f, s);
}

// Frame-count instantiations of the remaining per-pixel kernel (objective).
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

// ---------------------------------------------------------------- column-resident solve
//
// Temporal priors never couple readout columns: the temporal step couples the
// frames of one pixel and the x-update the rows of one (column, frame) block.
// Every column is therefore an independent ADMM problem for all iterations
// (the paper's remark that the reconstruction separates along the horizontal
// axis, Sec. V), and one workgroup can own column i for the whole solve:
//   repeat iters times:
//     temporal step (TV or DFT) for the nv pixels of column i
//     x-update of the nt blocks (t, i), ngroups blocks at a time
// with only workgroup barriers between the phases -- no grid-wide
// synchronisation and no per-iteration launch.  The per-column state stays
// in L2 / the memory-side cache while the factor streams past it with
// non-temporal loads.
struct ColumnSolveArgs {
  const float2* W;
  FactorLayout L;
  const float2* hy;
  float2 *s0, *s1, *s2, *s3;
  const float* frags;    // MFMA fragments: T^{-1} (TV prior) or the embedded temporal DFT (DFT prior)
  const float2* wgiven;  // DFT warm start: w for the first pass, or null
  int nh, nt, iters;
  int wave_floats;       // LDS floats per wave
  float mu, tau, rho;
};

// NT: the padded MFMA size, KT of the TV step (TV prior) or KP of the
// embedded DFT (DFT prior).  Per-wave LDS: `wave_floats` floats (x-update
// staging, reused as the temporal step's tiles), then the fragment matrix.
template <int PRIOR, int NT, int RP>
__global__ __launch_bounds__(512) void k_column_solve(ColumnSolveArgs a) {
  extern __shared__ float2 lds[];
  const int n = a.L.n;
  const int nwaves = blockDim.x >> 6;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float2* bsh = lds + (size_t)w * (a.wave_floats / 2);
  float2* dsh = bsh + n;
  float* frags = reinterpret_cast<float*>(lds + (size_t)nwaves * (a.wave_floats / 2));
  load_frags<NT>(frags, a.frags);
  __syncthreads();
  const int i = blockIdx.x;
  const size_t npix = (size_t)n * a.nh;
  for (int k = 0; k < a.iters; ++k) {
    if constexpr (PRIOR == CS_PRIOR_TEMPORAL_TV) {
      for (int tl = w; tl * 16 < n; tl += nwaves)
        tv_tile<NT>(frags, bsh, bsh + NT * 16, a.s0, a.s1, a.s2, a.s3, a.nt, npix, (size_t)i * n + 16 * tl,
                    std::min(16, n - 16 * tl), a.tau, a.rho, lane);
    } else {
      for (int tl = w; tl * 16 < n; tl += nwaves)
        dft_tile_any<NT, kDftStep>(frags, reinterpret_cast<float*>(bsh), a.s2, a.s0, a.s1, a.s3,
                                   k == 0 ? a.wgiven : nullptr, a.nt, npix, (size_t)i * n + 16 * tl,
                                   std::min(16, n - 16 * tl), a.tau, k == 0, lane);
    }
    __syncthreads();
    // x-update: wave w solves the blocks (t, i), t = w, w + nwaves, ...; no
    // barrier is needed between them
    for (int t = w; t < a.nt; t += nwaves) {
      const size_t blk = (size_t)t * a.nh + i;
      if (PRIOR == CS_PRIOR_TEMPORAL_TV)
        xupdate_wave_block<kSolveTV, kXUnrollCol, RP>(a.W, a.L, blk, lane, bsh, dsh, a.hy, a.s0, a.s3, a.s2, a.mu);
      else
        xupdate_wave_block<kSolveDFT, kXUnrollCol, RP>(a.W, a.L, blk, lane, bsh, dsh, a.hy, a.s3, nullptr, a.s2,
                                                       a.mu);
    }
    __syncthreads();
  }
}

template <int PRIOR, int NT, int RP>
static int column_launch_rp(cs_plan* p, const ColumnSolveArgs& a, int threads, size_t lds, hipStream_t s) {
  CS_HIP_STATUS(ensure_dynamic_lds((const void*)k_column_solve<PRIOR, NT, RP>, lds));
  hipLaunchKernelGGL((k_column_solve<PRIOR, NT, RP>), dim3(p->desc.nh), dim3(threads), lds, s, a);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

template <int PRIOR, int NT>
static int column_launch(cs_plan* p, const ColumnSolveArgs& a, int threads, size_t lds, hipStream_t s) {
  const int rp = pairs_per_lane(p->desc.nv);
  if (rp == 1) return column_launch_rp<PRIOR, NT, 1>(p, a, threads, lds, s);
  if (rp == 2) return column_launch_rp<PRIOR, NT, 2>(p, a, threads, lds, s);
  return column_launch_rp<PRIOR, NT, 4>(p, a, threads, lds, s);
}

bool column_solve_supported(const cs_plan* p) {
  return (p->desc.nv & 1) == 0 && p->desc.prior != CS_PRIOR_TEMPORAL_FRAME && !(p->desc.flags & CS_FLAG_EIGEN);
}

int launch_column_solve(cs_plan* p, int iters, float lambda, float mu, const float2* wgiven, hipStream_t s) {
  const int n = p->desc.nv, nt = p->desc.nt;
  if (iters <= 0) return CS_OK;
  const bool tv = p->desc.prior == CS_PRIOR_TEMPORAL_TV;
  ColumnSolveArgs a;
  a.W = p->factor;
  a.L = p->flayout;
  a.hy = p->hy;
  a.s0 = p->s0;
  a.s1 = p->s1;
  a.s2 = p->s2;
  a.s3 = p->s3;
  a.frags = tv ? p->tv_frags : p->dft_frags;
  a.wgiven = wgiven;
  a.nh = p->desc.nh;
  a.nt = nt;
  a.iters = iters;
  a.mu = mu;
  a.rho = p->desc.mu_ratio;
  a.tau = tv ? lambda * a.rho / (2.0f * mu) : lambda / (2.0f * mu);
  const int max_threads = 512;  // the launch bound of k_column_solve
  const int kp = tv ? tv_kt(nt) : dft_kp(nt);
  const size_t frag_bytes = (size_t)(kp / 16) * (kp / 4) * 64 * sizeof(float);
  a.wave_floats = std::max(2 * (1 + kXUnrollCol) * n, tv ? tv_wave_floats(kp) : kp * 16);
  a.wave_floats = (a.wave_floats + 3) / 4 * 4;  // keep every wave's region 16-byte aligned
  const size_t per_wave = (size_t)a.wave_floats * sizeof(float);
  const size_t lds_budget = 160 * 1024;
  const int nwaves = (int)std::max<size_t>(1, std::min<size_t>(max_threads / 64, (lds_budget - frag_bytes) / per_wave));
  const int threads = nwaves * 64;
  const size_t lds = nwaves * per_wave + frag_bytes;
  if (tv) {
    switch (kp) {
      case 16: return column_launch<CS_PRIOR_TEMPORAL_TV, 16>(p, a, threads, lds, s);
      case 32: return column_launch<CS_PRIOR_TEMPORAL_TV, 32>(p, a, threads, lds, s);
      case 48: return column_launch<CS_PRIOR_TEMPORAL_TV, 48>(p, a, threads, lds, s);
      default: return column_launch<CS_PRIOR_TEMPORAL_TV, 64>(p, a, threads, lds, s);
    }
  }
  switch (kp) {
    case 16: return column_launch<CS_PRIOR_TEMPORAL_DFT, 16>(p, a, threads, lds, s);
    case 32: return column_launch<CS_PRIOR_TEMPORAL_DFT, 32>(p, a, threads, lds, s);
    case 48: return column_launch<CS_PRIOR_TEMPORAL_DFT, 48>(p, a, threads, lds, s);
    case 64: return column_launch<CS_PRIOR_TEMPORAL_DFT, 64>(p, a, threads, lds, s);
    case 80: return column_launch<CS_PRIOR_TEMPORAL_DFT, 80>(p, a, threads, lds, s);
    case 96: return column_launch<CS_PRIOR_TEMPORAL_DFT, 96>(p, a, threads, lds, s);
    case 112: return column_launch<CS_PRIOR_TEMPORAL_DFT, 112>(p, a, threads, lds, s);
    default: return column_launch<CS_PRIOR_TEMPORAL_DFT, 128>(p, a, threads, lds, s);
  }
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

__global__ void k_copy(const float2* __restrict__ src, float2* __restrict__ dst, size_t n) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
    dst[q] = src[q];
}

// up to kCopyMax independent copies of n values each in one launch (no
// destination may overlap a source); 16-byte accesses when every pointer is
// 16-byte aligned and n is even
__global__ void k_copy_multi(CopyPairs c, size_t n, int vec) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t first = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vec) {
    const size_t n4 = n / 2;
    for (int a = 0; a < c.count; ++a) {
      const float4* src = reinterpret_cast<const float4*>(c.src[a]);
      float4* dst = reinterpret_cast<float4*>(c.dst[a]);
      for (size_t q = first; q < n4; q += stride) dst[q] = src[q];
    }
  } else {
    for (int a = 0; a < c.count; ++a)
      for (size_t q = first; q < n; q += stride) c.dst[a][q] = c.src[a][q];
  }
}

int launch_copy_multi(const CopyPairs& c, size_t n, hipStream_t s) {
  if (n == 0 || c.count == 0) return CS_OK;
  bool aligned = (n % 2) == 0;
  for (int a = 0; a < c.count; ++a)
    aligned = aligned && (reinterpret_cast<uintptr_t>(c.src[a]) % 16 == 0) &&
              (reinterpret_cast<uintptr_t>(c.dst[a]) % 16 == 0);
  const size_t units = aligned ? n / 2 : n;
  const unsigned blocks = (unsigned)std::min<size_t>((units + 255) / 256, 8192);
  hipLaunchKernelGGL(k_copy_multi, dim3(blocks), dim3(256), 0, s, c, n, aligned ? 1 : 0);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_copy(const float2* src, float2* dst, size_t n, hipStream_t s) {
  if (n == 0) return CS_OK;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, src, dst, n);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// ---------------------------------------------------------------- Algorithm 2 reverse step
//
// The per-pixel part of the transposed Jacobian of one Algorithm 2 iteration
// (the x-update kernel applies W before it: bb = W e), given the adjoints
// (mb', d1b', d2b') of the state after the iteration and the stored m, d1 of
// its start and d2 after it (T = rho I + D'D, D = D_t):
//   q   = mb' - d2b' + D' d1b' + mu bb;   rb = T^{-1} q
//   vb  = D rb - d1b';   ab = (dsoft/da)^T vb  (real 2x2 Jacobian on |a| > tau)
//   mb  = D' ab;   d1b = d1b' - D rb + ab;   xb = rho rb;   d2b = d2b' - mu bb + xb;   e = xb + d2b
//   dL/dH'y += bb (+ mb + xb for the first iteration, x_0 = m_0 = H'y)
//   dL/dtau += -sum_{|a| > tau} Re(conj(a/|a|) vb);   dL/dmu += -Re<bb, d2'>
// As in the forward TV step, 16 pixels per wave: lane l holds pixel l % 16
// and frames l / 16 + 4 k, neighbouring frames pass through the wave's LDS,
// and T^{-1} (symmetric, so its own transpose) is applied as the contraction
// of the forward's fragments.  a = D m + d1 is formed with the forward's own
// arithmetic, so every |a| > tau decision is the forward's.  A fixed grid
// with a grid-stride loop; one FP64 slot pair per workgroup.
template <int KT>
__global__ __launch_bounds__(256) void k_tv_adjoint_tiles(
    const float* __restrict__ frags, float2* __restrict__ mb, float2* __restrict__ d1b, float2* __restrict__ d2b,
    float2* __restrict__ e, const float2* __restrict__ bb, float2* __restrict__ hyb, const float2* __restrict__ m,
    const float2* __restrict__ d1, const float2* __restrict__ d2n, double* __restrict__ partial, int nt,
    size_t npix, float tau, float rho, float mu, int last) {
  constexpr int MT = DftTile<KT>::MT, NK = KT / 4;
  extern __shared__ float lds_f[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  float2* bufA = reinterpret_cast<float2*>(lds_f + DftTile<KT>::FRAG + wv * tv_wave_floats(KT));
  float2* bufB = bufA + KT * 16;
  float* bre = reinterpret_cast<float*>(bufB);
  float* bim = bre + KT * 16;
  load_frags<KT>(lds_f, frags);
  __syncthreads();
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (npix + 15) / 16;
  double tsum = 0.0, msum = 0.0;
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = tl * 16;
    const bool pv = col < (int)std::min<size_t>(16, npix - p0);
    const size_t p = p0 + col;
    float2 w[NK], bv[NK];
    // d1b' of this lane's frames, shared for the D' d1b' term
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + 4 * k;
      w[k] = (t < nt - 1 && pv) ? d1b[(size_t)t * npix + p] : make_float2(0.f, 0.f);
      bufA[t * 16 + col] = w[k];
    }
    __builtin_amdgcn_wave_barrier();
    // q, as the real and imaginary operand rows
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + 4 * k;
      const bool ok = t < nt && pv;
      const size_t o = (size_t)t * npix + p;
      float2 q = make_float2(0.f, 0.f);
      bv[k] = ok ? bb[o] : make_float2(0.f, 0.f);
      if (ok) {
        const float2 a = mb[o], z = d2b[o];
        const float2 wprev = t > 0 ? bufA[(t - 1) * 16 + col] : make_float2(0.f, 0.f);
        q = make_float2(fmaf(mu, bv[k].x, (a.x - z.x) + (wprev.x - w[k].x)),
                        fmaf(mu, bv[k].y, (a.y - z.y) + (wprev.y - w[k].y)));
      }
      bre[t * 16 + col] = q.x;
      bim[t * 16 + col] = q.y;
    }
    __builtin_amdgcn_wave_barrier();
    mfma_v4 rre[MT], rim[MT];
    tile_gemm<KT, false>(lds_f, bre, lane, rre);
    tile_gemm<KT, false>(lds_f, bim, lane, rim);
    __builtin_amdgcn_wave_barrier();
    // rb into bufB (accumulator lane l holds frames 16 mm + 4 (l / 16) + j), m into bufA
#pragma unroll
    for (int mm = 0; mm < MT; ++mm)
#pragma unroll
      for (int j = 0; j < 4; ++j) bufB[(16 * mm + 4 * grp + j) * 16 + col] = make_float2(rre[mm][j], rim[mm][j]);
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + 4 * k;
      bufA[t * 16 + col] = (t < nt && pv) ? m[(size_t)t * npix + p] : make_float2(0.f, 0.f);
    }
    __builtin_amdgcn_wave_barrier();
    float2 ab[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + 4 * k;
      ab[k] = make_float2(0.f, 0.f);
      if (t < nt - 1 && pv) {
        const size_t o = (size_t)t * npix + p;
        const float2 dr = csub(bufB[(t + 1) * 16 + col], bufB[t * 16 + col]);
        const float2 vb = csub(dr, w[k]);
        const float2 m0 = bufA[t * 16 + col], m1 = bufA[(t + 1) * 16 + col], dd = d1[o];
        // same arithmetic as the forward step, so the same |a| > tau decision
        const float2 a = make_float2(m1.x - m0.x + dd.x, m1.y - m0.y + dd.y);
        const float mag = sqrtf(fmaf(a.x, a.x, a.y * a.y));
        if (mag > tau) {
          const float sdot = fmaf(a.x, vb.x, a.y * vb.y) / mag;  // Re(conj(a/|a|) vb)
          const float kk = tau / mag;
          const float ks = kk * sdot / mag;
          ab[k] = make_float2(fmaf(1.f - kk, vb.x, ks * a.x), fmaf(1.f - kk, vb.y, ks * a.y));
          tsum -= (double)sdot;
        }
        d1b[o] = cadd(csub(w[k], dr), ab[k]);
      }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < NK; ++k) bufA[(grp + 4 * k) * 16 + col] = ab[k];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int t = grp + 4 * k;
      if (t < nt && pv) {
        const size_t o = (size_t)t * npix + p;
        const float2 abprev = t > 0 ? bufA[(t - 1) * 16 + col] : make_float2(0.f, 0.f);
        const float2 mnew = csub(abprev, ab[k]);  // (D' ab)_t = ab_{t-1} - ab_t
        const float2 r = bufB[t * 16 + col], b = bv[k], z = d2b[o], dn = d2n[o];
        const float2 xb = make_float2(rho * r.x, rho * r.y);
        const float2 z2 = make_float2(fmaf(-mu, b.x, z.x) + xb.x, fmaf(-mu, b.y, z.y) + xb.y);
        d2b[o] = z2;
        e[o] = cadd(xb, z2);
        mb[o] = mnew;
        float2 h = cadd(hyb[o], b);
        if (last) h = cadd(h, cadd(mnew, xb));
        hyb[o] = h;
        msum -= (double)fmaf(b.x, dn.x, b.y * dn.y);
      }
    }
    __builtin_amdgcn_wave_barrier();  // the next tile overwrites this wave's buffers
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = tsum;
  red[1][threadIdx.x] = msum;
  __syncthreads();
  for (int k = (int)blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      red[0][threadIdx.x] += red[0][threadIdx.x + k];
      red[1][threadIdx.x] += red[1][threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] += red[0][0];
    partial[2 * blockIdx.x + 1] += red[1][0];
  }
}

template <int KT>
static int tv_adjoint_launch(cs_plan* p, unsigned nblocks, float2* mb, float2* d1b, float2* d2b, float2* e,
                             const float2* bb, float2* hyb, const float2* m, const float2* d1, const float2* d2n,
                             double* partial, float tau, float rho, float mu, int last, hipStream_t s) {
  constexpr int waves = 4;
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  const size_t lds = ((size_t)DftTile<KT>::FRAG + (size_t)waves * tv_wave_floats(KT)) * sizeof(float);
  CS_HIP_STATUS(ensure_dynamic_lds((const void*)k_tv_adjoint_tiles<KT>, lds));
  hipLaunchKernelGGL(k_tv_adjoint_tiles<KT>, dim3(nblocks), dim3(64 * waves), lds, s, p->tv_frags, mb, d1b, d2b, e,
                     bb, hyb, m, d1, d2n, partial, p->desc.nt, npix, tau, rho, mu, last);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_tv_adjoint(cs_plan* p, unsigned nblocks, float2* mb, float2* d1b, float2* d2b, float2* e,
                      const float2* bb, float2* hyb, const float2* m, const float2* d1, const float2* d2n,
                      double* partial, float tau, float rho, float mu, int last, hipStream_t s) {
  switch (tv_kt(p->desc.nt)) {
    case 16: return tv_adjoint_launch<16>(p, nblocks, mb, d1b, d2b, e, bb, hyb, m, d1, d2n, partial, tau, rho, mu, last, s);
    case 32: return tv_adjoint_launch<32>(p, nblocks, mb, d1b, d2b, e, bb, hyb, m, d1, d2n, partial, tau, rho, mu, last, s);
    case 48: return tv_adjoint_launch<48>(p, nblocks, mb, d1b, d2b, e, bb, hyb, m, d1, d2n, partial, tau, rho, mu, last, s);
    default: return tv_adjoint_launch<64>(p, nblocks, mb, d1b, d2b, e, bb, hyb, m, d1, d2n, partial, tau, rho, mu, last, s);
  }
}

// ---------------------------------------------------------------- Algorithm 1 reverse step
//
// Transposed Jacobian of one iteration of Algorithm 1 with Psi the unitary
// temporal DFT (a = w - d, v = soft(a, tau), u = Psi'(v + d),
// z = W (H'y + mu u), w' = Psi z, d' = d - (w' - v)), given
//   bb = W zb   (zb = Psi'(wb' - db'), the adjoint reaching z; W Hermitian)
// and the adjoint db' of d':
//   s   = Psi (mu bb)                        adjoint of u, taken to (v, d)
//   vb  = db' + s
//   ab  = (dsoft/da)^T vb                    real 2x2 Jacobian on |a| > tau
//   wb  = ab;  db = db' + s - ab
//   zb  <- Psi'(wb - db)                     the next (earlier) step's zb
//   dL/dH'y += bb;  dL/dtau += -sum Re(conj(a/|a|) vb);  dL/dmu += Re<bb, u - z>
// For the first iteration (last = 1) the state before it is w_0 = Psi H'y,
// d_0 = 0, so Psi' wb is added to dL/dH'y instead of forming zb.  a is formed
// again from the stored z_{k-1} and d_{k-1} with the forward step's own
// contraction and subtraction, so every |a| > tau decision is the forward's.
// One wave per 16 pixels, three contractions on the fragments of Psihat; a
// fixed grid with a grid-stride loop and one FP64 slot pair per workgroup.
template <int KP>
__global__ __launch_bounds__(256) void k_dft_adjoint(const float* __restrict__ frags, const float2* __restrict__ bb,
                                                     float2* __restrict__ db, float2* __restrict__ zb,
                                                     float2* __restrict__ hyb, const float2* __restrict__ zprev,
                                                     const float2* __restrict__ dprev,
                                                     const float2* __restrict__ u, const float2* __restrict__ z,
                                                     double* __restrict__ partial, int nt, size_t npix, float tau,
                                                     float mu, int last) {
  constexpr int MT = DftTile<KP>::MT, NK = KP / 8;
  extern __shared__ float lds_f[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  float* tile = lds_f + DftTile<KP>::FRAG + wv * KP * 16;
  load_frags<KP>(lds_f, frags);
  __syncthreads();
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (npix + 15) / 16;
  double tsum = 0.0, msum = 0.0;
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = tl * 16;
    const int count = (int)std::min<size_t>(16, npix - p0);
    const bool pv = col < count;
    const size_t p = p0 + col;
    // s = Psi (mu bb)
    {
      float2 r[NK];
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int t = grp + 4 * k;
        r[k] = (t < nt && pv) ? cscale(bb[(size_t)t * npix + p], mu) : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int t = grp + 4 * k;
        tile[(2 * t) * 16 + col] = r[k].x;
        tile[(2 * t + 1) * 16 + col] = r[k].y;
      }
    }
    __builtin_amdgcn_wave_barrier();
    mfma_v4 S[MT], A[MT];
    tile_gemm<KP, false>(lds_f, tile, lane, S);
    __builtin_amdgcn_wave_barrier();
    // w_{k-1} = Psi z_{k-1}, as the forward step formed it
    tile_stage<KP>(tile, zprev, nt, npix, p0, count, lane);
    tile_gemm<KP, false>(lds_f, tile, lane, A);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f = 8 * m + 2 * grp + h;
        const int row = 16 * m + 4 * grp + 2 * h;
        float2 q = make_float2(0.f, 0.f);
        if (f < nt && pv) {
          const size_t o = (size_t)f * npix + p;
          const float2 dk = db[o];
          const float2 a = csub(make_float2(A[m][2 * h], A[m][2 * h + 1]), dprev[o]);
          const float2 sv = make_float2(S[m][2 * h], S[m][2 * h + 1]);
          const float2 vb = cadd(dk, sv);
          float2 ab = make_float2(0.f, 0.f);
          const float mag = sqrtf(fmaf(a.x, a.x, a.y * a.y));
          if (mag > tau) {
            const float sdot = fmaf(a.x, vb.x, a.y * vb.y) / mag;  // Re(conj(a/|a|) vb)
            const float kk = tau / mag;
            const float ks = kk * sdot / mag;
            ab = make_float2(fmaf(1.f - kk, vb.x, ks * a.x), fmaf(1.f - kk, vb.y, ks * a.y));
            tsum -= (double)sdot;
          }
          const float2 dn = csub(vb, ab);
          db[o] = dn;
          q = last ? ab : csub(ab, dn);
        }
        tile[row * 16 + col] = q.x;
        tile[(row + 1) * 16 + col] = q.y;
      }
    __builtin_amdgcn_wave_barrier();
    tile_gemm<KP, true>(lds_f, tile, lane, A);  // Psi'(wb - db), or Psi' wb for the first iteration
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = 8 * m + 2 * grp + h;
        if (t < nt && pv) {
          const size_t o = (size_t)t * npix + p;
          const float2 r = make_float2(A[m][2 * h], A[m][2 * h + 1]);
          const float2 b = bb[o], uu = u[o], zz = z[o];
          msum += (double)b.x * ((double)uu.x - zz.x) + (double)b.y * ((double)uu.y - zz.y);
          float2 hv = cadd(hyb[o], b);
          if (last) hv = cadd(hv, r);
          else zb[o] = r;
          hyb[o] = hv;
        }
      }
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = tsum;
  red[1][threadIdx.x] = msum;
  __syncthreads();
  for (int k = (int)blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      red[0][threadIdx.x] += red[0][threadIdx.x + k];
      red[1][threadIdx.x] += red[1][threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] += red[0][0];
    partial[2 * blockIdx.x + 1] += red[1][0];
  }
}

// k_dft_adjoint with Psi as the lane-group FFT (nt = L N2): the same three
// transforms and the same per-frequency and per-frame lines, 64 / L pixels
// per wave (lane l on pixel l / L).  w_{k-1} = Psi z_{k-1} is formed by the
// forward step's own transform and scaling, so every |a| > tau decision is
// the forward's.
template <int L, int N2>
__global__ __launch_bounds__(256) void k_dft_adjoint_fft(const float2* __restrict__ bb, float2* __restrict__ db,
                                                         float2* __restrict__ zb, float2* __restrict__ hyb,
                                                         const float2* __restrict__ zprev,
                                                         const float2* __restrict__ dprev,
                                                         const float2* __restrict__ u, const float2* __restrict__ z,
                                                         double* __restrict__ partial, size_t npix, float tau,
                                                         float mu, int last) {
  constexpr float kScale = (float)cx_rsqrt(L * N2);
  constexpr int P = 64 / L;  // pixels per wave
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  using GL = GroupLane<L, true>;  // lanes along the pixels (see k_dft_fft)
  const int col = GL::group(lane), j = GL::member(lane);
  const int k1 = lane_bitrev<L>(j);
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (npix + P - 1) / P;
  const GroupRoots<L, N2> roots = group_roots<L, N2>(j);
  double tsum = 0.0, msum = 0.0;
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = tl * P;
    const int count = (int)std::min<size_t>(P, npix - p0);
    const bool pv = col < count;
    const size_t p = p0 + col;
    // s = Psi (mu bb) and w_{k-1} = Psi z_{k-1}
    float2 S[N2], A[N2];
#pragma unroll
    for (int n = 0; n < N2; ++n) {
      const size_t o = (size_t)(j + L * n) * npix + p;
      S[n] = pv ? cscale(bb[o], mu) : make_float2(0.f, 0.f);
      A[n] = pv ? zprev[o] : make_float2(0.f, 0.f);
    }
    group_fft_time_to_freq<L, N2, -1, GL::LS>(S, j, roots);
    group_fft_time_to_freq<L, N2, -1, GL::LS>(A, j, roots);
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      S[k] = cscale(S[k], kScale);
      A[k] = cscale(A[k], kScale);
    }
    float2 Q[N2];
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      float2 q = make_float2(0.f, 0.f);
      if (pv) {
        const size_t o = (size_t)(k + N2 * k1) * npix + p;
        const float2 dk = db[o];
        const float2 a = csub(A[k], dprev[o]);
        const float2 vb = cadd(dk, S[k]);
        float2 ab = make_float2(0.f, 0.f);
        const float mag = sqrtf(fmaf(a.x, a.x, a.y * a.y));
        if (mag > tau) {
          const float sdot = fmaf(a.x, vb.x, a.y * vb.y) / mag;  // Re(conj(a/|a|) vb)
          const float kk = tau / mag;
          const float ks = kk * sdot / mag;
          ab = make_float2(fmaf(1.f - kk, vb.x, ks * a.x), fmaf(1.f - kk, vb.y, ks * a.y));
          tsum -= (double)sdot;
        }
        const float2 dn = csub(vb, ab);
        db[o] = dn;
        q = last ? ab : csub(ab, dn);
      }
      Q[k] = q;
    }
    group_fft_freq_to_time<L, N2, +1, GL::LS>(Q, j, roots);  // Psi'(wb - db), or Psi' wb for the first iteration
    if (pv) {
#pragma unroll
      for (int n = 0; n < N2; ++n) {
        const size_t o = (size_t)(j + L * n) * npix + p;
        const float2 r = cscale(Q[n], kScale);
        const float2 b = bb[o], uu = u[o], zz = z[o];
        msum += (double)b.x * ((double)uu.x - zz.x) + (double)b.y * ((double)uu.y - zz.y);
        float2 hv = cadd(hyb[o], b);
        if (last) hv = cadd(hv, r);
        else zb[o] = r;
        hyb[o] = hv;
      }
    }
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = tsum;
  red[1][threadIdx.x] = msum;
  __syncthreads();
  for (int k = (int)blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      red[0][threadIdx.x] += red[0][threadIdx.x + k];
      red[1][threadIdx.x] += red[1][threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] += red[0][0];
    partial[2 * blockIdx.x + 1] += red[1][0];
  }
}

template <int L, int N2>
static int dft_adjoint_fft_launch(cs_plan* p, unsigned nblocks, const float2* bb, float2* db, float2* zb,
                                  float2* hyb, const float2* zprev, const float2* dprev, const float2* u,
                                  const float2* z, double* partial, float tau, float mu, int last, hipStream_t s) {
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  hipLaunchKernelGGL((k_dft_adjoint_fft<L, N2>), dim3(nblocks), dim3(256), 0, s, bb, db, zb, hyb, zprev, dprev, u, z,
                     partial, npix, tau, mu, last);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

template <int KP>
static int dft_adjoint_launch(cs_plan* p, unsigned nblocks, const float2* bb, float2* db, float2* zb, float2* hyb,
                              const float2* zprev, const float2* dprev, const float2* u, const float2* z,
                              double* partial, float tau, float mu, int last, hipStream_t s) {
  constexpr int k8 = KP / 16, k4 = KP / 8 - 1;  // the group-FFT lengths whose nt has this KP
  const int nt = p->desc.nt, lanes = tdft_lanes(nt);
  if constexpr (tdft_len_ok(k8))
    if (lanes == 8 && nt == 8 * k8)
      return dft_adjoint_fft_launch<8, k8>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
  if constexpr (k4 % 2 == 1 && tdft_len_ok(k4))
    if (lanes == 4 && nt == 4 * k4)
      return dft_adjoint_fft_launch<4, k4>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  const int waves = dft_waves(KP);
  const size_t lds = dft_lds_bytes(KP, waves);
  CS_HIP_STATUS(ensure_dynamic_lds((const void*)k_dft_adjoint<KP>, lds));
  hipLaunchKernelGGL(k_dft_adjoint<KP>, dim3(nblocks), dim3(64 * waves), lds, s, p->dft_frags, bb, db, zb, hyb,
                     zprev, dprev, u, z, partial, p->desc.nt, npix, tau, mu, last);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int launch_dft_adjoint(cs_plan* p, unsigned nblocks, const float2* bb, float2* db, float2* zb, float2* hyb,
                       const float2* zprev, const float2* dprev, const float2* u, const float2* z, double* partial,
                       float tau, float mu, int last, hipStream_t s) {
  switch (dft_kp(p->desc.nt)) {
    case 16: return dft_adjoint_launch<16>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
    case 32: return dft_adjoint_launch<32>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
    case 48: return dft_adjoint_launch<48>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
    case 64: return dft_adjoint_launch<64>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
    case 80: return dft_adjoint_launch<80>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
    case 96: return dft_adjoint_launch<96>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
    case 112:
      return dft_adjoint_launch<112>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
    default:
      return dft_adjoint_launch<128>(p, nblocks, bb, db, zb, hyb, zprev, dprev, u, z, partial, tau, mu, last, s);
  }
}

// ---------------------------------------------------------------- objective
//
// J = lambda * l1 + ||y - H x||^2 (eqs. L1an_pri / L1unconst), evaluated in
// hybrid (ky, i) space: F_h is unitary, so the data term equals
// sum_{t,c,r,i} |(M_t F_v (s_c . x))[r, i] - (F_h' y)[r, i]|^2 over sampled
// rows r.  l1 = sum |D_t x| (TV), sum |Psi x| (DFT) or, for the overcomplete
// frame, sum |w| over the completed coefficients (moduli of complex values).
// For TV the data-term pass adds lambda |D_t x| to its own partials (it holds
// the image values anyway); the other priors have an l1 kernel of their own.
// Partial sums are FP64 and reduced in a fixed order, so the value is
// bit-reproducible run to run.
constexpr int kJBlocks = 1024;
constexpr int kJThreads = 256;

__device__ __forceinline__ void block_reduce_store(double v, double* out) {
  __shared__ double red[kJThreads];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kJThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// l1 of the coefficients w themselves (overcomplete frame prior: 2 nt frames)
__global__ __launch_bounds__(kJThreads) void k_l1_abs_partial(const float2* __restrict__ w, size_t count,
                                                              double* __restrict__ part) {
  double acc = 0.0;
  for (size_t q = (size_t)blockIdx.x * kJThreads + threadIdx.x; q < count; q += (size_t)kJBlocks * kJThreads) {
    const float2 a = w[q];
    acc += sqrt((double)a.x * a.x + (double)a.y * a.y);
  }
  block_reduce_store(acc, part + blockIdx.x);
}

// l1 of Psi x for the temporal-DFT prior: the same MFMA contraction as the
// DFT step (16 pixels per wave), then sum |w| over this lane's frequencies in
// FP64; a fixed grid with a grid-stride loop keeps the partials reproducible
template <int KP>
__global__ __launch_bounds__(256) void k_l1_dft_tiles(const float* __restrict__ frags, const float2* __restrict__ x,
                                                      int nt, size_t npix, double* __restrict__ part) {
  constexpr int MT = DftTile<KP>::MT;
  extern __shared__ float lds_f[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  float* tile = lds_f + DftTile<KP>::FRAG + wv * KP * 16;
  load_frags<KP>(lds_f, frags);
  __syncthreads();
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (npix + 15) / 16;
  double acc = 0.0;
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = tl * 16;
    const int count = (int)std::min<size_t>(16, npix - p0);
    mfma_v4 w[MT];
    tile_stage<KP>(tile, x, nt, npix, p0, count, lane);
    tile_gemm<KP, false>(lds_f, tile, lane, w);
    __builtin_amdgcn_wave_barrier();  // the next tile overwrites this wave's staging rows
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f = 8 * m + 2 * grp + h;
        if (f < nt && col < count) {
          const double a = w[m][2 * h], b = w[m][2 * h + 1];
          acc += sqrt(a * a + b * b);
        }
      }
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = (int)blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// the same sum with Psi as the lane-group FFT (nt = L N2): 64 / L pixels per
// wave, the forward step's own transform and scaling
template <int L, int N2>
__global__ __launch_bounds__(256) void k_l1_dft_fft(const float2* __restrict__ x, size_t npix,
                                                    double* __restrict__ part) {
  constexpr float kScale = (float)cx_rsqrt(L * N2);
  constexpr int P = 64 / L;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  using GL = GroupLane<L, true>;  // lanes along the pixels (see k_dft_fft)
  const int col = GL::group(lane), j = GL::member(lane);
  const int nw = blockDim.x >> 6;
  const size_t ntiles = (npix + P - 1) / P;
  const GroupRoots<L, N2> roots = group_roots<L, N2>(j);
  double acc = 0.0;
  for (size_t tl = (size_t)blockIdx.x * nw + wv; tl < ntiles; tl += (size_t)gridDim.x * nw) {
    const size_t p0 = tl * P;
    const int count = (int)std::min<size_t>(P, npix - p0);
    const uint32_t cc = (uint32_t)min(col, count - 1);
    const uint32_t offT = 8u * (cc + (uint32_t)(j * npix));
    float2 w[N2];
#pragma unroll
    for (int n = 0; n < N2; ++n) w[n] = ld_off(x + p0 + (size_t)n * L * npix, offT);
    group_fft_time_to_freq<L, N2, -1, GL::LS>(w, j, roots);
    if (col < count) {
#pragma unroll
      for (int k = 0; k < N2; ++k) {
        const double a = cscale(w[k], kScale).x, b = cscale(w[k], kScale).y;
        acc += sqrt(a * a + b * b);
      }
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = (int)blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

template <int KP>
static int l1_dft_launch(cs_plan* p, const float2* x, double* part, hipStream_t s) {
  const size_t npix = (size_t)p->desc.nv * p->desc.nh;
  constexpr int k8 = KP / 16, k4 = KP / 8 - 1;  // the group-FFT lengths whose nt has this KP
  const int nt = p->desc.nt, lanes = tdft_lanes(nt);
  if constexpr (tdft_len_ok(k8))
    if (lanes == 8 && nt == 8 * k8) {
      hipLaunchKernelGGL((k_l1_dft_fft<8, k8>), dim3(kJBlocks), dim3(256), 0, s, x, npix, part);
      CS_HIP(hipGetLastError());
      return CS_OK;
    }
  if constexpr (k4 % 2 == 1 && tdft_len_ok(k4))
    if (lanes == 4 && nt == 4 * k4) {
      hipLaunchKernelGGL((k_l1_dft_fft<4, k4>), dim3(kJBlocks), dim3(256), 0, s, x, npix, part);
      CS_HIP(hipGetLastError());
      return CS_OK;
    }
  const int waves = dft_waves(KP);
  const size_t lds = dft_lds_bytes(KP, waves);
  CS_HIP_STATUS(ensure_dynamic_lds((const void*)k_l1_dft_tiles<KP>, lds));
  hipLaunchKernelGGL(k_l1_dft_tiles<KP>, dim3(kJBlocks), dim3(64 * waves), lds, s, p->dft_frags, x, p->desc.nt, npix,
                     part);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

// J = lambda * l1 + data from the two halves of the partials (l1_half: the
// second half holds l1; otherwise the first holds all of J): each of the
// kJThreads threads sums a fixed run of each half, then a fixed tree; the
// order never changes, so J is reproducible
__global__ __launch_bounds__(kJThreads) void k_j_final(const double* __restrict__ part, float lambda, int l1_half,
                                                       float* __restrict__ out) {
  constexpr int kRun = kJBlocks / kJThreads;
  static_assert(kJBlocks % kJThreads == 0, "partials split evenly over the threads");
  __shared__ double r0[kJThreads], r1[kJThreads];
  double a = 0.0, b = 0.0;
#pragma unroll
  for (int q = 0; q < kRun; ++q) {
    a += part[threadIdx.x * kRun + q];
    if (l1_half) b += part[kJBlocks + threadIdx.x * kRun + q];
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int w = kJThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (float)((double)lambda * r1[0] + r0[0]);
}

// x in solver layout; the plan's ktmp must hold F_h' y (set by the solve setup)
int launch_objective(cs_plan* p, const float2* x, float lambda, float* out, hipStream_t s) {
  const int nh = p->desc.nh, nt = p->desc.nt;
  const size_t npix = (size_t)p->desc.nv * nh;
  const bool tv = p->desc.prior == CS_PRIOR_TEMPORAL_TV;
  // data term, fused with the vertical pass (and, for TV, lambda |D_t x|)
  int st = launch_forward_residual(p, x, p->jpart, kJBlocks, tv ? lambda : 0.f, s);
  if (st != CS_OK) return st;
  if (p->desc.prior == CS_PRIOR_TEMPORAL_FRAME) {
    // J at the completed coefficients w (img_tmp); x = Psi' w for the data term
    hipLaunchKernelGGL(k_l1_abs_partial, dim3(kJBlocks), dim3(kJThreads), 0, s, p->img_tmp, 2 * (size_t)nt * npix,
                       p->jpart + kJBlocks);
  } else if (!tv) {
    switch (dft_kp(nt)) {
      case 16: st = l1_dft_launch<16>(p, x, p->jpart + kJBlocks, s); break;
      case 32: st = l1_dft_launch<32>(p, x, p->jpart + kJBlocks, s); break;
      case 48: st = l1_dft_launch<48>(p, x, p->jpart + kJBlocks, s); break;
      case 64: st = l1_dft_launch<64>(p, x, p->jpart + kJBlocks, s); break;
      case 80: st = l1_dft_launch<80>(p, x, p->jpart + kJBlocks, s); break;
      case 96: st = l1_dft_launch<96>(p, x, p->jpart + kJBlocks, s); break;
      case 112: st = l1_dft_launch<112>(p, x, p->jpart + kJBlocks, s); break;
      default: st = l1_dft_launch<128>(p, x, p->jpart + kJBlocks, s); break;
    }
    if (st != CS_OK) return st;
  }
  hipLaunchKernelGGL(k_j_final, dim3(1), dim3(kJThreads), 0, s, p->jpart, lambda, tv ? 0 : 1, out);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

int objective_partial_count() { return 2 * kJBlocks; }

// ---------------------------------------------------------------- x-update, eigen form
//
// The paper's form of the exact x-update (Sec. IV-C, eq. eigen_mu): with
// G = U diag(e) U' stored per block, x = U diag(1/(mu + e)) U' b, for the
// same right-hand sides and fused dual update as the packed-inverse forms.
// One wave per block; lane l owns indices l + 64 r, r < R.
//   pass 1: t_k = sum_j conj(U[j, k]) b_j   (row j of U, conjugated, is the
//           contiguous uh[j][.]; b_j is broadcast from wave-private LDS)
//   s_k = t_k / (mu + e_k)
//   pass 2: x_j = sum_k U[j, k] s_k          (column k read as uc[k][.])
// Neither pass needs a cross-lane reduction; each reads its n x n values
// once, front to back, so a launch streams 2 n^2 complex64 values per block
// (four times the packed inverse's n (n + 1) / 2).

typedef float v2f __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 ld_stream2(const float2* p) {
  const v2f v = __builtin_nontemporal_load(reinterpret_cast<const v2f*>(p));
  return make_float2(v.x, v.y);
}

// acc[r] += sum_j M[j][lane + 64 r] v_j for an n x n row-major M, v in LDS.
// JC rows are loaded before any is used, so each lane keeps JC * R loads in
// flight.
template <int R>
__device__ __forceinline__ void stream_matvec(const float2* __restrict__ M, const float2* v, int n, int lane,
                                              float2 (&acc)[R]) {
  constexpr int JC = R >= 8 ? 2 : 16 / R;
  for (int j0 = 0; j0 < n; j0 += JC) {
    float2 c[JC][R];
#pragma unroll
    for (int u = 0; u < JC; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int k = lane + 64 * r;
        c[u][r] = (k < n && j0 + u < n) ? ld_stream2(M + (size_t)(j0 + u) * n + k) : make_float2(0.f, 0.f);
      }
#pragma unroll
    for (int u = 0; u < JC; ++u) {
      if (j0 + u < n) {
        const float2 vj = v[j0 + u];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = cfma(c[u][r], vj, acc[r]);
      }
    }
  }
}

// Even n: the same product with lane l owning the index pairs (2q, 2q+1),
// q = l + 64 r, r < RP, one 16-byte load per pair and row.
template <int RP>
__device__ __forceinline__ void stream_matvec2(const float2* __restrict__ M, const float2* v, int n, int lane,
                                               float2 (&a0)[RP], float2 (&a1)[RP]) {
  constexpr int JC = RP >= 4 ? 4 : (RP == 3 ? 5 : 16 / RP);
  const int h = n >> 1;
  for (int j0 = 0; j0 < n; j0 += JC) {
    float4 c[JC][RP];
#pragma unroll
    for (int u = 0; u < JC; ++u)
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const int q = lane + 64 * r;
        c[u][r] = (q < h && j0 + u < n) ? ld_stream4(M + (size_t)(j0 + u) * n + 2 * q)
                                        : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
    for (int u = 0; u < JC; ++u) {
      if (j0 + u < n) {
        const float2 vj = v[j0 + u];
#pragma unroll
        for (int r = 0; r < RP; ++r) {
          a0[r] = cfma(make_float2(c[u][r].x, c[u][r].y), vj, a0[r]);
          a1[r] = cfma(make_float2(c[u][r].z, c[u][r].w), vj, a1[r]);
        }
      }
    }
  }
}

template <int MODE, int R>
__global__ __launch_bounds__(64) void k_xupdate_eigen(const float2* __restrict__ uh, const float2* __restrict__ uc,
                                                      const float* __restrict__ ev, int n, ColRange cr,
                                                      const float2* hy, const float2* __restrict__ m,
                                                      float2* __restrict__ d2, float2* x, float mu) {
  extern __shared__ float2 lds[];
  float2* bsh = lds;      // [n] right-hand side
  float2* ssh = lds + n;  // [n] scaled coefficients s
  const int lane = threadIdx.x;
  const size_t blk = range_block(cr, blockIdx.x);
  const size_t base = blk * (size_t)n;
  const size_t nn = (size_t)n * n;
  float2 mk[R], dk[R], acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = lane + 64 * r;
    mk[r] = dk[r] = acc[r] = make_float2(0.f, 0.f);
    if (j < n) bsh[j] = rhs_value<MODE>(hy, m, d2, base + j, mu, mk[r], dk[r]);
  }
  __builtin_amdgcn_wave_barrier();
  stream_matvec<R>(uh + blk * nn, bsh, n, lane, acc);  // t = U' b
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = lane + 64 * r;
    if (k < n) {
      const float inv = 1.0f / (mu + ev[blk * n + k]);
      ssh[k] = make_float2(acc[r].x * inv, acc[r].y * inv);
    }
    acc[r] = make_float2(0.f, 0.f);
  }
  __builtin_amdgcn_wave_barrier();
  stream_matvec<R>(uc + blk * nn, ssh, n, lane, acc);  // x = U s
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = lane + 64 * r;
    if (j < n) {
      x[base + j] = acc[r];
      if (MODE == kSolveTV) d2[base + j] = make_float2(dk[r].x - (mk[r].x - acc[r].x), dk[r].y - (mk[r].y - acc[r].y));
    }
  }
}

template <int MODE, int RP>
__global__ __launch_bounds__(64) void k_xupdate_eigen2(const float2* __restrict__ uh, const float2* __restrict__ uc,
                                                       const float* __restrict__ ev, int n, ColRange cr,
                                                       const float2* hy, const float2* __restrict__ m,
                                                       float2* __restrict__ d2, float2* x, float mu) {
  extern __shared__ float2 lds[];
  float2* bsh = lds;      // [n] right-hand side
  float2* ssh = lds + n;  // [n] scaled coefficients s
  const int lane = threadIdx.x;
  const int h = n >> 1;
  const size_t blk = range_block(cr, blockIdx.x);
  const size_t base = blk * (size_t)n;
  const size_t nn = (size_t)n * n;
  float2 m0[RP], m1[RP], e0[RP], e1[RP], a0[RP], a1[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int q = lane + 64 * r;
    m0[r] = m1[r] = e0[r] = e1[r] = a0[r] = a1[r] = make_float2(0.f, 0.f);
    if (q < h) {
      bsh[2 * q] = rhs_value<MODE>(hy, m, d2, base + 2 * q, mu, m0[r], e0[r]);
      bsh[2 * q + 1] = rhs_value<MODE>(hy, m, d2, base + 2 * q + 1, mu, m1[r], e1[r]);
    }
  }
  __builtin_amdgcn_wave_barrier();
  stream_matvec2<RP>(uh + blk * nn, bsh, n, lane, a0, a1);  // t = U' b
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int q = lane + 64 * r;
    if (q < h) {
      const float i0 = 1.0f / (mu + ev[blk * n + 2 * q]), i1 = 1.0f / (mu + ev[blk * n + 2 * q + 1]);
      ssh[2 * q] = make_float2(a0[r].x * i0, a0[r].y * i0);
      ssh[2 * q + 1] = make_float2(a1[r].x * i1, a1[r].y * i1);
    }
    a0[r] = a1[r] = make_float2(0.f, 0.f);
  }
  __builtin_amdgcn_wave_barrier();
  stream_matvec2<RP>(uc + blk * nn, ssh, n, lane, a0, a1);  // x = U s
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int q = lane + 64 * r;
    if (q < h) {
      *reinterpret_cast<float4*>(x + base + 2 * q) = make_float4(a0[r].x, a0[r].y, a1[r].x, a1[r].y);
      if (MODE == kSolveTV)
        *reinterpret_cast<float4*>(d2 + base + 2 * q) =
            make_float4(e0[r].x - (m0[r].x - a0[r].x), e0[r].y - (m0[r].y - a0[r].y),
                        e1[r].x - (m1[r].x - a1[r].x), e1[r].y - (m1[r].y - a1[r].y));
    }
  }
}

template <int MODE, int RP>
static void eigen_launch_p(cs_plan* p, const float2* hy, const float2* m, float2* d2, float2* x, float mu,
                           hipStream_t s) {
  const int n = p->desc.nv, nh = p->desc.nh;
  const ColRange cr{0, nh, nh};
  const unsigned grid = (unsigned)nh * (unsigned)p->desc.nt;
  hipLaunchKernelGGL((k_xupdate_eigen2<MODE, RP>), dim3(grid), dim3(64), 2 * (size_t)n * sizeof(float2), s,
                     p->eig_uh, p->eig_uc, p->eig_e, n, cr, hy, m, d2, x, mu);
}

template <int MODE, int R>
static void eigen_launch_r(cs_plan* p, const float2* hy, const float2* m, float2* d2, float2* x, float mu,
                           hipStream_t s) {
  const int n = p->desc.nv, nh = p->desc.nh;
  const ColRange cr{0, nh, nh};
  const unsigned grid = (unsigned)nh * (unsigned)p->desc.nt;
  hipLaunchKernelGGL((k_xupdate_eigen<MODE, R>), dim3(grid), dim3(64), 2 * (size_t)n * sizeof(float2), s, p->eig_uh,
                     p->eig_uc, p->eig_e, n, cr, hy, m, d2, x, mu);
}

template <int MODE>
static void eigen_launch(cs_plan* p, const float2* hy, const float2* m, float2* d2, float2* x, float mu,
                         hipStream_t s) {
  const int n = p->desc.nv;  // <= 512
  if ((n & 1) == 0) {
    const int rp = pairs_per_lane(n);
    if (rp == 1) eigen_launch_p<MODE, 1>(p, hy, m, d2, x, mu, s);
    else if (rp == 2) eigen_launch_p<MODE, 2>(p, hy, m, d2, x, mu, s);
    else if (rp == 3) eigen_launch_p<MODE, 3>(p, hy, m, d2, x, mu, s);
    else eigen_launch_p<MODE, 4>(p, hy, m, d2, x, mu, s);
    return;
  }
  const int r = (n + 63) / 64;
  if (r == 1) eigen_launch_r<MODE, 1>(p, hy, m, d2, x, mu, s);
  else if (r == 2) eigen_launch_r<MODE, 2>(p, hy, m, d2, x, mu, s);
  else if (r == 3) eigen_launch_r<MODE, 3>(p, hy, m, d2, x, mu, s);
  else if (r == 4) eigen_launch_r<MODE, 4>(p, hy, m, d2, x, mu, s);
  else if (r <= 6) eigen_launch_r<MODE, 6>(p, hy, m, d2, x, mu, s);
  else eigen_launch_r<MODE, 8>(p, hy, m, d2, x, mu, s);
}

// ---------------------------------------------------------------- x-update, two blocks per wave
//
// The packed-inverse product of the wave form (same wrapped diagonals, same
// operations in the same order, so bit-identical results) for even n whose
// n/2 row pairs do not fill whole waves but whose 2 (n/2) do: n = 64 and
// n = 192.  Wave w solves blocks 2w and 2w + 1; slot r of lane l is the pair
// index P = l + 64 r over both blocks, block b = [P >= n/2], rows
// 2 (P - b n/2) and 2 (P - b n/2) + 1.  Every lane is busy on every load,
// where one block per wave would leave a quarter (n = 192) or half (n = 64)
// of the slots idle.  Each block keeps its own right-hand side and staged
// diagonals in the wave's LDS.

template <int UNR, int RP>
struct Diag2Chunk {
  float4 c[UNR][RP];
};

template <int UNR, int RP>
__device__ __forceinline__ void load_chunk2(Diag2Chunk<UNR, RP>& ch, const float2* __restrict__ W,
                                            const FactorLayout& L, const size_t (&blk)[RP], const int (&q)[RP],
                                            const bool (&act)[RP], int s0) {
#pragma unroll
  for (int u = 0; u < UNR; ++u)
#pragma unroll
    for (int r = 0; r < RP; ++r)
      ch.c[u][r] = (act[r] && s0 + u < L.F) ? ld_stream4(W + diag_offset(L, blk[r], s0 + u) + 2 * q[r])
                                            : make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int UNR, int RP>
__device__ __forceinline__ void apply_chunk2(const Diag2Chunk<UNR, RP>& ch, const FactorLayout& L, int s0,
                                             const int (&boff)[RP], const int (&q)[RP], const bool (&act)[RP],
                                             const float2* bsh, float2* dsh, float2 (&a0)[RP], float2 (&a1)[RP]) {
  const int n = L.n, n2 = 2 * L.n;
#pragma unroll
  for (int u = 0; u < UNR; ++u)
#pragma unroll
    for (int r = 0; r < RP; ++r)
      if (act[r]) *reinterpret_cast<float4*>(dsh + u * n2 + boff[r] + 2 * q[r]) = ch.c[u][r];
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int u = 0; u < UNR; ++u) {
    const int s = s0 + u;
    if (s < L.F) {
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        if (act[r]) {
          const float2* bb = bsh + boff[r];
          const float2* d = dsh + u * n2 + boff[r];
          const int k0 = 2 * q[r], k1 = k0 + 1;
          int p0 = k0 + s, p1 = k1 + s, q0 = k0 - s, q1 = k1 - s;
          p0 -= p0 >= n ? n : 0;
          p1 -= p1 >= n ? n : 0;
          q0 += q0 < 0 ? n : 0;
          q1 += q1 < 0 ? n : 0;
          a0[r] = cfma(make_float2(ch.c[u][r].x, ch.c[u][r].y), bb[p0], a0[r]);
          a1[r] = cfma(make_float2(ch.c[u][r].z, ch.c[u][r].w), bb[p1], a1[r]);
          a0[r] = cfmac(d[q0], bb[q0], a0[r]);
          a1[r] = cfmac(d[q1], bb[q1], a1[r]);
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
}

template <int MODE, int UNR, int RP>
__global__ __launch_bounds__(64) void k_xupdate_wave2(const float2* __restrict__ W, FactorLayout L, const float2* hy,
                                                      const float2* __restrict__ m, float2* __restrict__ d2,
                                                      float2* x, float mu) {
  extern __shared__ float2 lds[];
  const int n = L.n, h = n >> 1, F = L.F;
  float2* bsh = lds;          // [2][n] right-hand sides
  float2* dsh = lds + 2 * n;  // [UNR][2][n] staged diagonals
  const int lane = threadIdx.x;
  size_t blk[RP];
  int q[RP], boff[RP];
  bool act[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int P = lane + 64 * r;  // < 2 h = 64 RP
    const int b = P >= h ? 1 : 0;
    q[r] = P - b * h;
    boff[r] = b * n;
    blk[r] = 2 * (size_t)blockIdx.x + b;
    act[r] = blk[r] < L.nblk;
  }
  Diag2Chunk<UNR, RP> A, B;
  if (F > 1) load_chunk2<UNR, RP>(A, W, L, blk, q, act, 1);
  float2 b0[RP], b1[RP], m0[RP], m1[RP], e0[RP], e1[RP], a0[RP], a1[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    b0[r] = b1[r] = m0[r] = m1[r] = e0[r] = e1[r] = a0[r] = a1[r] = make_float2(0.f, 0.f);
    if (act[r]) {
      const size_t base = blk[r] * (size_t)n;
      b0[r] = rhs_value<MODE>(hy, m, d2, base + 2 * q[r], mu, m0[r], e0[r]);
      b1[r] = rhs_value<MODE>(hy, m, d2, base + 2 * q[r] + 1, mu, m1[r], e1[r]);
      const float4 c = ld_stream4(W + diag_offset(L, blk[r], 0) + 2 * q[r]);
      a0[r] = cmul(make_float2(c.x, c.y), b0[r]);
      a1[r] = cmul(make_float2(c.z, c.w), b1[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < RP; ++r)
    if (act[r])
      *reinterpret_cast<float4*>(bsh + boff[r] + 2 * q[r]) = make_float4(b0[r].x, b0[r].y, b1[r].x, b1[r].y);
  __builtin_amdgcn_wave_barrier();
  for (int s0 = 1; s0 < F; s0 += 2 * UNR) {
    if (s0 + UNR < F) load_chunk2<UNR, RP>(B, W, L, blk, q, act, s0 + UNR);
    apply_chunk2<UNR, RP>(A, L, s0, boff, q, act, bsh, dsh, a0, a1);
    if (s0 + 2 * UNR < F) load_chunk2<UNR, RP>(A, W, L, blk, q, act, s0 + 2 * UNR);
    if (s0 + UNR < F) apply_chunk2<UNR, RP>(B, L, s0 + UNR, boff, q, act, bsh, dsh, a0, a1);
  }
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    if (act[r]) {
      const float2* hd = W + half_offset(L, blk[r]);
      const float2* bb = bsh + boff[r];
      const int k0 = 2 * q[r], k1 = k0 + 1;
      a0[r] = k0 < h ? cfma(hd[k0], bb[k0 + h], a0[r]) : cfmac(hd[k0 - h], bb[k0 - h], a0[r]);
      a1[r] = k1 < h ? cfma(hd[k1], bb[k1 + h], a1[r]) : cfmac(hd[k1 - h], bb[k1 - h], a1[r]);
      const size_t base = blk[r] * (size_t)n;
      *reinterpret_cast<float4*>(x + base + k0) = make_float4(a0[r].x, a0[r].y, a1[r].x, a1[r].y);
      if (MODE == kSolveTV)
        *reinterpret_cast<float4*>(d2 + base + k0) =
            make_float4(e0[r].x - (m0[r].x - a0[r].x), e0[r].y - (m0[r].y - a0[r].y),
                        e1[r].x - (m1[r].x - a1[r].x), e1[r].y - (m1[r].y - a1[r].y));
    }
  }
}

// diagonals per chunk: with two blocks the wave's LDS holds (1 + UNR) 2n
// values, and 4 (15 KB at n = 192) limits a CU to 10 such waves; 2 measured
// 182.6 us per 192x192x40 launch against 214.6 us for 4 and 196.8 us for
// the one-block-per-workgroup pairs form
constexpr int kWave2Unroll = 2;

// n = 64 or 192: the two-blocks-per-wave form replaces the one-block wave form and is the default there
static bool wave2_shape(int n) { return n % 64 == 0 && (n / 2) % 64 != 0; }

template <int MODE, int RP>
static void wave2_launch(cs_plan* p, const float2* hy, const float2* m, float2* d2, float2* x, float mu,
                         hipStream_t s) {
  const FactorLayout& L = p->flayout;
  constexpr int UNR = kWave2Unroll;
  const size_t lds = (size_t)(1 + UNR) * 2 * L.n * sizeof(float2);
  const unsigned grid = (unsigned)((L.nblk + 1) / 2);
  hipLaunchKernelGGL((k_xupdate_wave2<MODE, UNR, RP>), dim3(grid), dim3(64), lds, s, p->factor, L, hy, m, d2, x, mu);
}

template <int MODE>
static void wave2_dispatch(cs_plan* p, const float2* hy, const float2* m, float2* d2, float2* x, float mu,
                           hipStream_t s) {
  if (p->desc.nv == 64) wave2_launch<MODE, 1>(p, hy, m, d2, x, mu, s);
  else wave2_launch<MODE, 3>(p, hy, m, d2, x, mu, s);
}

int launch_xupdate(cs_plan* p, int mode, const float2* hy, const float2* m, float2* d2, float2* x, float mu,
                   hipStream_t s) {
  const uint32_t f = p->desc.flags;
  if (!(f & CS_FLAG_EIGEN)) {
    // n = 64, 192: two blocks per wave unless the workgroup form is asked for
    if ((f & CS_FLAG_XU_GROUP) || !wave2_shape(p->desc.nv)) return launch_block_solve(p, mode, hy, m, d2, x, mu, s);
    if (mode == kSolveTV) wave2_dispatch<kSolveTV>(p, hy, m, d2, x, mu, s);
    else if (mode == kSolveDFT) wave2_dispatch<kSolveDFT>(p, hy, m, d2, x, mu, s);
    else wave2_dispatch<kSolvePlain>(p, hy, m, d2, x, mu, s);
    CS_HIP(hipGetLastError());
    return CS_OK;
  }
  if (mode == kSolveTV) eigen_launch<kSolveTV>(p, hy, m, d2, x, mu, s);
  else if (mode == kSolveDFT) eigen_launch<kSolveDFT>(p, hy, m, d2, x, mu, s);
  else eigen_launch<kSolvePlain>(p, hy, m, d2, x, mu, s);
  CS_HIP(hipGetLastError());
  return CS_OK;
}

}  // namespace csmri
