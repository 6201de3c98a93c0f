// Internal declarations shared by the HIP translation units of libcsmri.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "csmri.h"

namespace csmri {

// ---------------------------------------------------------------- complex
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// complex products with explicit FMAs (the library is built without implicit
// contraction, so these round identically in every kernel)
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// conj(a) * b
__host__ __device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.x, b.y, -(a.y * b.x)));
}
// acc + a * b
__host__ __device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 acc) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a) * b
__host__ __device__ __forceinline__ float2 cfmac(float2 a, float2 b, float2 acc) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(-a.y, b.x, acc.y);
  return acc;
}
__host__ __device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x));
}
__host__ __device__ __forceinline__ double2 zfma(double2 a, double2 b, double2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc - a * b
__host__ __device__ __forceinline__ double2 zfms(double2 a, double2 b, double2 acc) {
  acc.x = fma(-a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(-a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
__host__ __device__ __forceinline__ double2 zrecip(double2 a) {
  double d = fma(a.x, a.x, a.y * a.y);
  return make_double2(a.x / d, -a.y / d);
}

// Complex soft threshold: (|a| - tau) a / |a| if |a| > tau, else 0.
__device__ __forceinline__ float2 soft_threshold(float2 a, float tau) {
  float mag = sqrtf(fmaf(a.x, a.x, a.y * a.y));
  if (!(mag > tau)) return make_float2(0.f, 0.f);
  float s = (mag - tau) / mag;
  return make_float2(a.x * s, a.y * s);
}

// ---------------------------------------------------------------- factor layout
//
// Storage of the per-(column, frame) inverses W = (mu I + G)^{-1}, n = nv.
// Block b = t*nh + i holds its wrapped diagonals c_s[k] = W[k, (k+s) mod n]:
// F = ceil(n/2) full diagonals s = 0..F-1 of n values, plus for even n the
// half diagonal s = n/2 of n/2 values -- n(n+1)/2 values per block in all.
// Full diagonals are grouped G = 2^glog at a time across blocks,
//     [s / G][block][s % G][k],
// so that the workgroups streaming neighbouring blocks read a compact
// address window; the half diagonals of all blocks follow, [block][k].
struct FactorLayout {
  int n;
  int F;
  int glog;
  size_t nblk;
};
__host__ __device__ __forceinline__ size_t diag_offset(const FactorLayout& L, size_t blk, int s) {
  return ((((size_t)(s >> L.glog) * L.nblk + blk) << L.glog) + (size_t)(s & ((1 << L.glog) - 1))) * L.n;
}
__host__ __device__ __forceinline__ size_t half_offset(const FactorLayout& L, size_t blk) {
  return (size_t)L.F * L.n * L.nblk + blk * (size_t)(L.n / 2);
}
inline FactorLayout make_factor_layout(int n, size_t nblk) {
  FactorLayout L;
  L.n = n;
  L.F = (n + 1) / 2;
  L.glog = 3;
  while (L.glog > 0 && (L.F % (1 << L.glog)) != 0) --L.glog;
  L.nblk = nblk;
  return L;
}
inline size_t factor_elems(const FactorLayout& L) { return L.nblk * (size_t)L.n * (L.n + 1) / 2; }

// ---------------------------------------------------------------- FFT plan
constexpr int kMaxFftPasses = 12;
struct FftDesc {
  int n;
  int npass;
  int radix[kMaxFftPasses];
};
bool make_fft_desc(int n, FftDesc* d);  // false if n is not 2^a 3^b in [2, 512]

// ---------------------------------------------------------------- errors
int set_error(int status, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
#define CS_HIP(expr)                                   \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return hip_fail(_e, #expr);  \
  } while (0)
// returns from the enclosing function on a cs_status other than CS_OK
#define CS_HIP_STATUS(expr)             \
  do {                                  \
    const int _st = (expr);             \
    if (_st != CS_OK) return _st;       \
  } while (0)

// Raise `kernel`'s dynamic-LDS limit on the current device to at least
// `bytes` when they exceed the default 64 KiB.  The attribute belongs to a
// (kernel, device) pair, so the sizes already set are kept per pair in a
// mutex-guarded table; repeated calls cost a lookup.
int ensure_dynamic_lds(const void* kernel, size_t bytes);

// ---------------------------------------------------------------- plan
struct DeviceAlloc {
  cs_allocator a;
  bool custom;
  void* get(size_t bytes);
  void put(void* p);
};

}  // namespace csmri

struct cs_plan {
  cs_plan_desc desc;
  int device = 0;
  float mu = 0.f;
  csmri::DeviceAlloc alloc;
  std::vector<void*> owned;
  size_t bytes = 0;

  // FFT tiles of the SENSE passes (0: the largest that fit; cs_plan_tune may pick smaller)
  int fft_cw = 0;  // columns per workgroup, vertical passes
  int fft_rb = 0;  // sampled rows per workgroup, horizontal passes

  // sampling pattern
  int m_max = 0;
  std::vector<int32_t> h_mcnt;  // sampled rows per frame
  int32_t* rows = nullptr;      // [nt][m_max] sampled ky, padded with -1
  int32_t* mcnt = nullptr;      // [nt]
  int32_t* rinv = nullptr;      // [nt][nv] r with rows[t][r] = ky, or -1 for an unsampled ky
  uint8_t* mask = nullptr;      // [nt][nv]
  double2* pcol = nullptr;      // [nt][nv] first column of F_v' M_t F_v (FP64)

  // tables
  csmri::FftDesc fft_v{}, fft_h{};
  float2* tw_v = nullptr;       // exp(-2 pi i q / nv), q < nv
  float2* tw_h = nullptr;
  float* dft_frags = nullptr;   // MFMA A-operand fragments of the embedded Psi and Psi' (DFT prior)
  float* tv_frags = nullptr;    // MFMA A-operand fragments of (rho I + D'D)^{-1}, padded to 16 (TV step)

  // coil maps in the solver's column-major layout [c][i][j]
  float2* coil_cm = nullptr;

  // factor: nt*nh blocks (t, i), block index t*nh + i, layout csmri::FactorLayout
  float2* factor = nullptr;     // packed inverses (not allocated with CS_FLAG_EIGEN)
  float2* eig_uh = nullptr;     // CS_FLAG_EIGEN: [block][j][k] conj(U[j, k]) (rows of U, conjugated)
  float2* eig_uc = nullptr;     // CS_FLAG_EIGEN: [block][k][j] U[j, k] (columns of U)
  float* eig_e = nullptr;       // CS_FLAG_EIGEN: [block][k] eigenvalue k of G (mu not included)
  csmri::FactorLayout flayout{};

  // workspaces (solver layout [t][i][j], i.e. column-contiguous)
  float2* ktmp = nullptr;       // [nt][nc][nh][m_max] hybrid-space rows of the data, F_h' y
  float2* ftmp = nullptr;       // [nt][nc][nh][m_max] forward intermediate, M_t F_v (s_c . x)
  float2* hy = nullptr;         // H'y
  float2* s0 = nullptr;         // TV: m   DFT: d
  float2* s1 = nullptr;         // TV: d1  DFT: v
  float2* s2 = nullptr;         // TV: x   DFT: z (image-domain iterate)
  float2* s3 = nullptr;         // TV: d2  DFT: u
  float2* img_tmp = nullptr;    // one image, layout conversions
  double* jpart = nullptr;      // objective partial sums
  float* jdev = nullptr;        // [2] objective values read back by the Delta-driven solve
  float* jhost = nullptr;       // [2] pinned host copy (hipHostMalloc, on first use)
  int* check_flag = nullptr;    // CS_FLAG_CHECK_FINITE: set to 1 by a check that meets a non-finite value
  int jpart_len = 0;

  hipGraphExec_t graph = nullptr;  // cached iteration graph
  void* graph_key[8] = {};
  hipStream_t capture_stream = nullptr;  // private stream used only to record graphs

  // per-kernel event timing (cs_kernel_timing)
  bool timing = false;
  // overcomplete frame prior: img_tmp holds a completed w (and s0 the
  // completed d) -- after the set-up of a solve and after launch_frame_finish --
  // rather than the deferred state an iteration leaves for the next frame pass
  bool frame_w_ready = false;
  struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
  };
  std::vector<TimedLaunch> timed;   // event pairs recorded since the last read
  std::vector<hipEvent_t> event_pool;
  size_t pool_next = 0;
};

namespace csmri {

// sense.hip
int launch_forward(cs_plan* p, const float2* x, bool x_colmajor, float2* y, hipStream_t s);
int build_factor_eigen(cs_plan* p, hipStream_t s);  // CS_FLAG_EIGEN plans: U and e of every block
// reverse step of one Algorithm 1 iteration (temporal DFT prior): see iterate.hip
// reverse step of one Algorithm 2 iteration (temporal TV prior), after bb = W e: see iterate.hip
int launch_tv_adjoint(cs_plan* p, unsigned nblocks, float2* mb, float2* d1b, float2* d2b, float2* e,
                      const float2* bb, float2* hyb, const float2* m, const float2* d1, const float2* d2n,
                      double* partial, float tau, float rho, float mu, int last, hipStream_t s);
int launch_dft_adjoint(cs_plan* p, unsigned nblocks, const float2* bb, float2* db, float2* zb, float2* hyb,
                       const float2* zprev, const float2* dprev, const float2* u, const float2* z, double* partial,
                       float tau, float mu, int last, hipStream_t s);
// `iters` phase-form iterations without objective; cont: they continue a loop of
// the same solve (the temporal DFT step completes the previous deferred update)
int run_iterations_cont(cs_plan* p, int32_t iters, float lambda, float mu, bool cont, hipStream_t s);
int launch_adjoint_rows(cs_plan* p, const float2* y, hipStream_t s);  // y -> p->ktmp
// sum |M_t F_v (s_c . x) - ktmp|^2, one FP64 partial per workgroup of an nblocks grid (x column-major);
// tv_lambda > 0 adds tv_lambda * sum_{t < nt-1} |x[t + 1] - x[t]| (the temporal-TV l1) to the partials
int launch_forward_residual(cs_plan* p, const float2* x, double* part, int nblocks, float tv_lambda,
                            hipStream_t s);
int launch_adjoint_image(cs_plan* p, float2* x, bool x_colmajor, hipStream_t s);  // p->ktmp -> x
// the two adjoint passes on explicit buffers (the plan launchers above call
// these): hyb is [nt][nc][nh][m_max], rows [nt][m_max] padded with -1, mcnt
// [nt] (rows r >= mcnt[t] are neither written nor read), x column-major
int launch_adjoint_rows_raw(const float2* y, float2* hyb, const int32_t* rows, const int32_t* mcnt, const FftDesc& fh,
                            const float2* twh, int nv, int nh, int nt, int nc, int m_max, int rb, hipStream_t s);
// rinv [nt][nv]: r of each sampled ky (-1 for the others), read by the nv = 16 M kernels;
// csplit (1, 2 or 4): coil ranges per column group of those kernels, from
// coil_split16 of the whole series' shape (frame chunks keep the series' split)
int launch_adjoint_vertical_raw(const float2* hyb, const float2* coil_cm, float2* x, const int32_t* rows,
                                const int32_t* mcnt, const int32_t* rinv, const FftDesc& fv, const float2* twv,
                                int nv, int nh, int nt, int nc, int m_max, int cw, int csplit, hipStream_t s);
int coil_split16(int nh, int nt, int nc);
int launch_transpose(const float2* in, float2* out, int frames, int rows, int cols, hipStream_t s);
// CS_FLAG_CHECK_FINITE (no-ops without it): CS_EINVAL if the sampled rows of
// k-space y, or the n values at x, hold a NaN or an infinity; synchronise s
int check_finite_kspace(cs_plan* p, const float2* y, hipStream_t s, const char* what);
int check_finite_values(cs_plan* p, const float2* x, size_t n, hipStream_t s, const char* what);
int fft_cols_per_group(const cs_plan* p);
int fft_cols_limit(const cs_plan* p);
// sizes (n_v or n_h) that take the 16 x M register passes (fixed tiles)
bool reg16_size(int n);
int fft_rows_per_group(const cs_plan* p);

// factor.hip
int build_factor(cs_plan* p, float mu, hipStream_t s);

// iterate.hip
// the x-update of every block in the plan's form: the packed inverse
// (launch_block_solve), or U diag(1/(mu + e)) U' for CS_FLAG_EIGEN plans
int launch_xupdate(cs_plan* p, int mode, const float2* hy, const float2* m, float2* d2, float2* x, float mu,
                   hipStream_t s);
int launch_block_solve(cs_plan* p, int mode, const float2* hy, const float2* m, float2* d2,
                       float2* x, float mu, hipStream_t s);
int launch_tv_step(cs_plan* p, float lambda, float mu, hipStream_t s);
// the same kernels restricted to the readout columns [i0, i1) (columns never interact under a temporal prior)
int launch_block_solve_cols(cs_plan* p, int mode, const float2* hy, const float2* m, float2* d2, float2* x,
                            float mu, int i0, int i1, hipStream_t s);
int launch_tv_step_cols(cs_plan* p, float lambda, float mu, int i0, int i1, hipStream_t s);
int launch_dft_step_cols(cs_plan* p, float lambda, float mu, int first, const float2* wgiven, int i0, int i1,
                         hipStream_t s);
// first != 0 skips the deferred dual update; wgiven (nullable) replaces Psi z on this pass
int launch_dft_step(cs_plan* p, float lambda, float mu, int first, const float2* wgiven, hipStream_t s);
// out = Psi in (adjoint == 0) or Psi' in (adjoint == 1); with dual != nullptr (forward only)
// also d <- d - (out - v)
int launch_dft_apply(cs_plan* p, const float2* in, float2* out, float2* dual, const float2* v, int adjoint,
                     hipStream_t s);
// overcomplete temporal frame prior (state: s0 = d, s1 = v, s2 = x~, s3 = u, img_tmp = w)
int launch_frame_step(cs_plan* p, float lambda, float mu, int first, hipStream_t s);
int launch_frame_finish(cs_plan* p, hipStream_t s);
int launch_frame_forward(cs_plan* p, const float2* x, float2* w, hipStream_t s);
int launch_frame_adjoint(cs_plan* p, const float2* w, float2* x, hipStream_t s);
int launch_fill(float2* ptr, size_t n, float2 v, hipStream_t s);
int launch_copy(const float2* src, float2* dst, size_t n, hipStream_t s);
constexpr int kCopyMax = 4;
struct CopyPairs {
  const float2* src[kCopyMax];
  float2* dst[kCopyMax];
  int count;
};
// the copies of `c` (n values each, disjoint) in one launch
int launch_copy_multi(const CopyPairs& c, size_t n, hipStream_t s);
// all iterations in one launch, one workgroup per readout column (even nv)
bool column_solve_supported(const cs_plan* p);
int launch_column_solve(cs_plan* p, int iters, float lambda, float mu, const float2* wgiven, hipStream_t s);
int launch_objective(cs_plan* p, const float2* x, float lambda, float* out, hipStream_t s);

enum BlockSolveMode { kSolvePlain = 0, kSolveTV = 1, kSolveDFT = 2 };

}  // namespace csmri
