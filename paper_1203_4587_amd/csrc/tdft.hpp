// The unitary temporal DFT Psi (Algorithm 1: Psi = the DFT along frames,
// Psi[f][t] = exp(-2 pi i f t / nt) / sqrt(nt)) as a register FFT over a group
// of L = 8 or 4 lanes per pixel, for nt = L N2 with N2 <= 16 a product of 2,
// 3 and 5 (8 lanes whenever nt / 8 is such a length).
//
// Lane j (= lane % L) of a group holds the frames t = j + L n2, n2 < N2, of
// one pixel.  Forward: a length-N2 DFT over n2 in the lane's registers, a
// multiplication by exp(-2 pi i j k2 / nt), then a length-L DFT over j across
// the group (radix-2 stages through lane exchanges), after which lane j holds
// the frequencies f = k2 + N2 bitrev(j).  The inverse runs the same steps
// backwards with the conjugate roots.  Against the dense product this takes
// O(nt log nt) instead of O(nt^2) operations per pixel and needs neither LDS
// nor matrix cores; more lanes per pixel give more waves for the same image.
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace csmri {

// ---- compile-time roots of unity (double, rounded to float where used)
constexpr double kTwoPi = 6.283185307179586476925286766559;

// sin and cos of x in [-2 pi, 2 pi] by their Taylor series (error far below a
// float's rounding at these arguments)
constexpr double cx_sin(double x) {
  if (x > kTwoPi / 2) x -= kTwoPi;
  if (x < -kTwoPi / 2) x += kTwoPi;
  double term = x, sum = x;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos(double x) {
  if (x > kTwoPi / 2) x -= kTwoPi;
  if (x < -kTwoPi / 2) x += kTwoPi;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
constexpr double cx_rsqrt(int n) {  // 1 / sqrt(n), n >= 1, by Newton's iteration from below
  double y = 1.0 / n;  // below 1 / sqrt(n): every step stays below it and increases
  for (int k = 0; k < 200; ++k) y = y * (1.5 - 0.5 * n * y * y);
  return y;
}

// a length (2, 3, 5 only) factorisation test for the per-lane DFT length
constexpr bool tdft_len_ok(int n) {
  if (n < 1 || n > 16) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  return n == 1;
}
// lanes per pixel of the group FFT for nt frames: 8 when nt / 8 is a
// supported length, else 4 when nt / 4 is, else 0 (the dense product is used)
constexpr int tdft_lanes(int nt) {
  return (nt % 8 == 0 && tdft_len_ok(nt / 8)) ? 8 : (nt % 4 == 0 && tdft_len_ok(nt / 4)) ? 4 : 0;
}

// f(std::integral_constant<int, K>) for K = B .. E-1, unrolled at compile time
template <int B, int E>
struct StaticFor {
  template <class F>
  __device__ __forceinline__ static void run(F&& f) {
    if constexpr (B < E) {
      f(std::integral_constant<int, B>{});
      StaticFor<B + 1, E>::run(f);
    }
  }
};

// v * exp(SIGN 2 pi i E / N), the multiples of pi/2 exact
template <int N, int E, int SIGN>
__device__ __forceinline__ float2 root_mul(float2 v) {
  constexpr int e = ((E % N) + N) % N;
  if constexpr (e == 0) {
    return v;
  } else if constexpr (2 * e == N) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * e == N) {  // * (SIGN i)
    return SIGN > 0 ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
  } else if constexpr (4 * e == 3 * N) {  // * (-SIGN i)
    return SIGN > 0 ? make_float2(v.y, -v.x) : make_float2(-v.y, v.x);
  } else {
    constexpr float c = (float)cx_cos(kTwoPi * e / N);
    constexpr float s = (float)(SIGN * cx_sin(kTwoPi * e / N));
    return make_float2(fmaf(v.x, c, -(v.y * s)), fmaf(v.x, s, v.y * c));
  }
}

// in-register DFT of length N (2, 3, 5 factors): x[k] <- sum_n x[n] exp(SIGN 2 pi i n k / N)
template <int N, int SIGN>
__device__ __forceinline__ void dft_reg(float2 (&x)[N]) {
  if constexpr (N == 1) {
    return;
  } else if constexpr (N == 2) {
    const float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (N == 3) {
    constexpr float h = (float)(SIGN * cx_sin(kTwoPi / 3));  // SIGN sqrt(3) / 2
    const float2 s = cadd(x[1], x[2]), d = csub(x[1], x[2]);
    const float2 base = make_float2(fmaf(-0.5f, s.x, x[0].x), fmaf(-0.5f, s.y, x[0].y));
    const float2 rot = make_float2(-h * d.y, h * d.x);  // SIGN i (sqrt 3 / 2) d
    x[0] = cadd(x[0], s);
    x[1] = cadd(base, rot);
    x[2] = csub(base, rot);
  } else if constexpr (N == 4) {
    const float2 t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
    const float2 t2 = cadd(x[1], x[3]), t3 = csub(x[1], x[3]);
    const float2 r = SIGN > 0 ? make_float2(-t3.y, t3.x) : make_float2(t3.y, -t3.x);  // SIGN i t3
    x[0] = cadd(t0, t2);
    x[2] = csub(t0, t2);
    x[1] = cadd(t1, r);
    x[3] = csub(t1, r);
  } else if constexpr (N == 5) {
    constexpr float c1 = (float)cx_cos(kTwoPi / 5), c2 = (float)cx_cos(2 * kTwoPi / 5);
    constexpr float s1 = (float)(SIGN * cx_sin(kTwoPi / 5)), s2 = (float)(SIGN * cx_sin(2 * kTwoPi / 5));
    const float2 a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
    const float2 a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
    const float2 x0 = x[0];
    // real parts of the pairs, and SIGN i (sin-weighted differences)
    const float2 p1 = make_float2(fmaf(c1, a1.x, fmaf(c2, a2.x, x0.x)), fmaf(c1, a1.y, fmaf(c2, a2.y, x0.y)));
    const float2 p2 = make_float2(fmaf(c2, a1.x, fmaf(c1, a2.x, x0.x)), fmaf(c2, a1.y, fmaf(c1, a2.y, x0.y)));
    const float2 q1 = make_float2(fmaf(s1, b1.x, s2 * b2.x), fmaf(s1, b1.y, s2 * b2.y));
    const float2 q2 = make_float2(fmaf(s2, b1.x, -(s1 * b2.x)), fmaf(s2, b1.y, -(s1 * b2.y)));
    const float2 r1 = make_float2(-q1.y, q1.x), r2 = make_float2(-q2.y, q2.x);  // i q
    x[0] = cadd(x0, cadd(a1, a2));
    x[1] = cadd(p1, r1);
    x[4] = csub(p1, r1);
    x[2] = cadd(p2, r2);
    x[3] = csub(p2, r2);
  } else {
    // decimation in time: N = R M, sub-sequences x[r + R m] transformed over m,
    // then a length-R DFT across r for every k < M (outputs k + M q)
    constexpr int R = (N % 4 == 0) ? 4 : (N % 2 == 0) ? 2 : (N % 3 == 0) ? 3 : 5;
    constexpr int M = N / R;
    float2 sub[R][M];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int m = 0; m < M; ++m) sub[r][m] = x[r + R * m];
#pragma unroll
    for (int r = 0; r < R; ++r) dft_reg<M, SIGN>(sub[r]);
    StaticFor<0, M>::run([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      float2 t[R];
      StaticFor<0, R>::run([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        t[q] = root_mul<N, q * k, SIGN>(sub[q][k]);
      });
      dft_reg<R, SIGN>(t);
#pragma unroll
      for (int q = 0; q < R; ++q) x[k + M * q] = t[q];
    });
  }
}

// Exchanges between lanes l and l ^ XOR.  A lane group of L = 4 or 8 lanes
// per pixel has its members 1 apart (XOR = 1, 2, 4) or 64 / L apart (XOR = 8,
// 16, 32 for L = 8; 16, 32 for L = 4).  xor 1 and xor 2 are DPP quad
// permutes, xor 4 a bitmask-mode swizzle (lanes exchanged within 32), xor 8
// a DPP rotation by 8 within each row of 16 lanes, xor 16 and xor 32 the
// permlane swaps of rows of 16 and halves of 32 lanes (each returns the
// swapped pair; a lane takes the copy that came from its partner).
template <int XOR>
__device__ __forceinline__ float lane_xor(float v) {
  if constexpr (XOR == 1) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
  } else if constexpr (XOR == 2) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
  } else if constexpr (XOR == 4) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), (XOR << 10) | 0x1F));
  } else if constexpr (XOR == 8) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xF, 0xF, false));  // row_ror:8
  } else if constexpr (XOR == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float((__lane_id() & 16) ? r[0] : r[1]);
  } else {
    static_assert(XOR == 32, "lane exchange distance");
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float((__lane_id() & 32) ? r[0] : r[1]);
  }
}
// butterfly between partner lanes: the lane whose bit is clear gets v + w,
// the other w - v (w the partner's value), as w + sgn v with sgn = -1 on the
// high lane (exact: one rounding either way)
template <int XOR>
__device__ __forceinline__ float2 lane_butterfly(float2 v, float sgn) {
  const float2 w = make_float2(lane_xor<XOR>(v.x), lane_xor<XOR>(v.y));
  return make_float2(fmaf(sgn, v.x, w.x), fmaf(sgn, v.y, w.y));
}

// Where a pixel's L lanes sit in the wave: STRIDED = false puts group g on
// lanes L g + j (member j), STRIDED = true on lanes g + (64 / L) j, so that
// lanes 0, 1, 2, ... hold consecutive groups (pixels) of one frame and a
// wave's memory accesses run along the pixels.  LS is the distance between
// members j and j + 1.
template <int L, bool STRIDED>
struct GroupLane {
  static constexpr int G = 64 / L;  // groups per wave
  static constexpr int LS = STRIDED ? G : 1;
  static __device__ __forceinline__ int member(int lane) { return STRIDED ? lane / G : lane % L; }
  static __device__ __forceinline__ int group(int lane) { return STRIDED ? lane % G : lane / L; }
};

// The lane's roots, computed once per kernel (they depend only on the lane):
// exp(-2 pi i j k / nt) for k < N2, and exp(-2 pi i (j mod 4) / 8) for the
// first stage of an 8-lane group.  The forward transform uses them, the
// inverse their conjugates.  Each is a compile-time value chosen by j.
template <int L, int N2>
struct GroupRoots {
  float c[N2], s[N2];
  float c8, s8;          // 1, 0 on the lanes of the first stage's low half
  float sg1, sg2, sg4;   // butterfly signs of the stages between members j ^ 1, j ^ 2, j ^ 4
};

// the roots of every lane of a group, as a compile-time table in device
// memory (read once per kernel: one load per root instead of a chain of
// selects between compile-time values)
struct RootPair {
  float c, s;
};
template <int L, int N2>
struct RootTable {
  RootPair r[L][N2 + 1];  // [j][k]: exp(-2 pi i j k / nt); [j][N2]: exp(-2 pi i (j mod 4) / 8)
  constexpr RootTable() : r() {
    for (int j = 0; j < L; ++j) {
      for (int k = 0; k < N2; ++k)
        r[j][k] = RootPair{(float)cx_cos(kTwoPi * ((j * k) % (L * N2)) / (L * N2)),
                           (float)(-cx_sin(kTwoPi * ((j * k) % (L * N2)) / (L * N2)))};
      r[j][N2] = (j & 4) ? RootPair{(float)cx_cos(kTwoPi * (j & 3) / 8), (float)(-cx_sin(kTwoPi * (j & 3) / 8))}
                         : RootPair{1.f, 0.f};
    }
  }
};
template <int L, int N2>
__device__ constexpr RootTable<L, N2> kRootTable{};

template <int L, int N2>
__device__ __forceinline__ GroupRoots<L, N2> group_roots(int j) {
  GroupRoots<L, N2> r;
  const RootPair* t = kRootTable<L, N2>.r[j];
#pragma unroll
  for (int k = 0; k < N2; ++k) {
    r.c[k] = t[k].c;
    r.s[k] = t[k].s;
  }
  r.c8 = t[N2].c;
  r.s8 = t[N2].s;
  r.sg1 = (j & 1) ? -1.f : 1.f;
  r.sg2 = (j & 2) ? -1.f : 1.f;
  r.sg4 = (j & 4) ? -1.f : 1.f;
  return r;
}

// v * (c + i SIGN' s) with SIGN' = +1 (forward roots) or -1 (their conjugates)
template <int SIGN>
__device__ __forceinline__ float2 root_apply(float2 v, float c, float s) {
  const float t = SIGN < 0 ? s : -s;
  return make_float2(fmaf(v.x, c, -(v.y * t)), fmaf(v.x, t, v.y * c));
}

// bit reversal of j < L
template <int L>
__device__ __forceinline__ int lane_bitrev(int j) {
  if constexpr (L == 4) return ((j & 1) << 1) | (j >> 1);
  else return ((j & 1) << 2) | (j & 2) | (j >> 2);
}

// forward transform of a lane group (SIGN = -1 for Psi; LS the lane distance
// between members, GroupLane): frames j + L n2 in, frequencies k2 + N2
// bitrev(j) out, unnormalised.  A length-N2 DFT in the lane's registers, the
// twiddles exp(SIGN 2 pi i j k2 / nt), then a length-L DFT across the group by
// decimation in frequency (stages between members j ^ L/2 .. j ^ 1, i.e.
// lanes LS L/2 .. LS apart; the difference of a stage of half-size h
// multiplied by exp(SIGN 2 pi i (j mod h) / 2h)).  Every lane of the wave must
// take part.
template <int L, int N2, int SIGN, int LS = 1>
__device__ __forceinline__ void group_fft_time_to_freq(float2 (&x)[N2], int j, const GroupRoots<L, N2>& r) {
  dft_reg<N2, SIGN>(x);
#pragma unroll
  for (int k = 1; k < N2; ++k) x[k] = root_apply<SIGN>(x[k], r.c[k], r.s[k]);
#pragma unroll
  for (int k = 0; k < N2; ++k) {
    float2 v = x[k];
    if constexpr (L == 8) {
      v = lane_butterfly<4 * LS>(v, r.sg4);
      v = root_apply<SIGN>(v, r.c8, r.s8);  // exp(SIGN 2 pi i (j mod 4) / 8) on the high half, else 1
    }
    v = lane_butterfly<2 * LS>(v, r.sg2);
    if ((j & 3) == 3) v = SIGN > 0 ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);  // * (SIGN i)
    x[k] = lane_butterfly<LS>(v, r.sg1);
  }
}

// the reverse steps (decimation in time): frequencies k2 + N2 bitrev(j) in,
// frames j + L n2 out, unnormalised (SIGN = +1 for Psi')
template <int L, int N2, int SIGN, int LS = 1>
__device__ __forceinline__ void group_fft_freq_to_time(float2 (&x)[N2], int j, const GroupRoots<L, N2>& r) {
#pragma unroll
  for (int k = 0; k < N2; ++k) {
    float2 v = lane_butterfly<LS>(x[k], r.sg1);
    if ((j & 3) == 3) v = SIGN > 0 ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);  // * (SIGN i)
    v = lane_butterfly<2 * LS>(v, r.sg2);
    if constexpr (L == 8) {
      v = root_apply<SIGN>(v, r.c8, r.s8);
      v = lane_butterfly<4 * LS>(v, r.sg4);
    }
    x[k] = v;
  }
#pragma unroll
  for (int k = 1; k < N2; ++k) x[k] = root_apply<SIGN>(x[k], r.c[k], r.s[k]);
  dft_reg<N2, SIGN>(x);
}

}  // namespace csmri
