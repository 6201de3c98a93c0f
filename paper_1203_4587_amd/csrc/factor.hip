// Plan-time factor of the exact x-update (Sec. IV-C).
//
// H'H is block diagonal with one nv x nv block per (column i, frame t)
// (eqs. HconjH, separate_x):
//     G_{i,t}[j,k] = p_t[(j - k) mod nv] * sum_c conj(s_{c,j,i}) s_{c,k,i},
// where p_t is the first column of the circulant F_v' M_t F_v,
//     p_t[l] = (1/nv) sum_{ky sampled in frame t} exp(+2 pi i ky l / nv).
// (The coil product is conj(s_j) s_k; the printed Hadamard form s s' is its
// conjugate, which is not the block for complex maps.)
//
// The paper applies (mu I + G)^{-1} = U diag(1/(e + mu)) U' through an
// eigendecomposition of every block.  Here the inverse W = (mu I + G)^{-1} is
// formed once, in FP64, by blocked in-place Gauss-Jordan elimination without
// pivoting (mu I + G is Hermitian positive definite, so every pivot block is
// too), and stored in complex64 as nv(nv+1)/2 values per block in
// "circulant-diagonal" order: for s = 0 .. floor(nv/2),
//     c_s[k] = W[k, (k + s) mod nv],   k < nv   (k < nv/2 when s = nv/2).
// Those wrapped diagonals hold every entry of the Hermitian W exactly once,
// and the per-iteration product W b then reads them as contiguous runs.
#include "internal.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

namespace csmri {

// ws block (column-major, A(r, c) at c * nv + r) = mu I + G_{i,t}
__global__ __launch_bounds__(512) void k_gram_assemble(double2* __restrict__ ws,
                                                       const float2* __restrict__ coil_cm,
                                                       const double2* __restrict__ pcol, int nv, int nh,
                                                       int nc, int blk0, double mu) {
  constexpr int kCoilChunk = 16;
  extern __shared__ float2 sc[];  // [kCoilChunk][nv]
  const int blk = blk0 + blockIdx.x;
  const int t = blk / nh, i = blk - t * nh;
  const int j = threadIdx.x;  // row
  double2* A = ws + (size_t)blockIdx.x * nv * nv;
  const double2* pt = pcol + (size_t)t * nv;
  for (int c0 = 0; c0 < nc; c0 += kCoilChunk) {
    const int cn = min(kCoilChunk, nc - c0);
    const bool last = c0 + kCoilChunk >= nc;
    __syncthreads();
    for (int e = threadIdx.x; e < cn * nv; e += blockDim.x) {
      const int cc = e / nv, q = e - cc * nv;
      sc[cc * nv + q] = coil_cm[((size_t)(c0 + cc) * nh + i) * nv + q];
    }
    __syncthreads();
    if (j < nv) {
      double2 sj[kCoilChunk];
#pragma unroll
      for (int cc = 0; cc < kCoilChunk; ++cc) {
        float2 v = cc < cn ? sc[cc * nv + j] : make_float2(0.f, 0.f);
        sj[cc] = make_double2(v.x, -(double)v.y);  // conj(s_j)
      }
      for (int k = 0; k < nv; ++k) {
        double2 g = c0 == 0 ? make_double2(0.0, 0.0) : A[(size_t)k * nv + j];
#pragma unroll
        for (int cc = 0; cc < kCoilChunk; ++cc) {
          if (cc < cn) {
            const float2 v = sc[cc * nv + k];
            g = zfma(sj[cc], make_double2(v.x, v.y), g);
          }
        }
        if (last) {
          int l = j - k;
          l += l < 0 ? nv : 0;
          g = zmul(pt[l], g);
          if (j == k) g.x += mu;
        }
        A[(size_t)k * nv + j] = g;
      }
    }
  }
}

// In-place inverse of each column-major n x n block (Hermitian positive
// definite) by blocked Gauss-Jordan with panels of NB columns:
//   D = A_PP^{-1};  A_PQ <- D A_PQ;  A_QQ <- A_QQ - A_QP A_PQ;  A_QP <- -A_QP D;  A_PP <- D
// Thread i owns row i; the new row panel sits in LDS as Rl[j * NB + k].
template <int NB>
__global__ __launch_bounds__(512) void k_gj_inverse(double2* __restrict__ ws, int n) {
  extern __shared__ double2 lds2[];
  double2* Rl = lds2;                   // [n][NB]
  double2* Dl = lds2 + (size_t)n * NB;  // [NB][NB + 1]
  constexpr int LD = NB + 1;
  double2* A = ws + (size_t)blockIdx.x * n * n;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int i = tid;
  for (int p0 = 0; p0 < n; p0 += NB) {
    const int nb = min(NB, n - p0);
    const bool in_panel = i >= p0 && i < p0 + nb;
    double2 C[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k)
      C[k] = (i < n && k < nb) ? A[(size_t)(p0 + k) * n + i] : make_double2(0.0, 0.0);
    if (in_panel) {
#pragma unroll
      for (int k = 0; k < NB; ++k)
        if (k < nb) Dl[(i - p0) * LD + k] = C[k];
    }
    __syncthreads();
    // unblocked Gauss-Jordan on the nb x nb diagonal block; every thread
    // computes up to kPer entries from the old block, then all write
    {
      constexpr int kPer = (NB * NB + 63) / 64;  // the workgroup has >= 64 threads
      for (int q = 0; q < nb; ++q) {
        double2 val[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int e = tid + u * nthr;
          val[u] = make_double2(0.0, 0.0);
          if (e < nb * nb) {
            const int r = e / nb, cc = e - (e / nb) * nb;
            const double2 pinv = zrecip(Dl[q * LD + q]);
            if (r == q && cc == q) {
              val[u] = pinv;
            } else if (r == q) {
              val[u] = zmul(Dl[q * LD + cc], pinv);
            } else if (cc == q) {
              const double2 v = zmul(Dl[r * LD + q], pinv);
              val[u] = make_double2(-v.x, -v.y);
            } else {
              val[u] = zfms(zmul(Dl[r * LD + q], pinv), Dl[q * LD + cc], Dl[r * LD + cc]);
            }
          }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int e = tid + u * nthr;
          if (e < nb * nb) Dl[(e / nb) * LD + (e - (e / nb) * nb)] = val[u];
        }
        __syncthreads();
      }
    }
    // new row panel R = D A_PQ
    for (int e = tid; e < n * NB; e += nthr) {
      const int j = e / NB, k = e - j * NB;
      if (k < nb && (j < p0 || j >= p0 + nb)) {
        const double2* col = A + (size_t)j * n + p0;
        double2 acc = make_double2(0.0, 0.0);
        for (int l = 0; l < nb; ++l) acc = zfma(Dl[k * LD + l], col[l], acc);
        Rl[j * NB + k] = acc;
      }
    }
    __syncthreads();
    for (int e = tid; e < n * NB; e += nthr) {
      const int j = e / NB, k = e - j * NB;
      if (k < nb && (j < p0 || j >= p0 + nb)) A[(size_t)j * n + p0 + k] = Rl[j * NB + k];
    }
    if (i < n) {
      if (!in_panel) {
        // columns outside the panel: [0, p0) and [p0 + nb, n)
        auto update = [&](int j) {
          double2 a = A[(size_t)j * n + i];
#pragma unroll
          for (int k = 0; k < NB; ++k)
            if (k < nb) a = zfms(C[k], Rl[j * NB + k], a);
          A[(size_t)j * n + i] = a;
        };
        for (int j = 0; j < p0; ++j) update(j);
        for (int j = p0 + nb; j < n; ++j) update(j);
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          if (k < nb) {
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll
            for (int l = 0; l < NB; ++l)
              if (l < nb) acc = zfma(C[l], Dl[l * LD + k], acc);
            A[(size_t)(p0 + k) * n + i] = make_double2(-acc.x, -acc.y);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < NB; ++k)
          if (k < nb) A[(size_t)(p0 + k) * n + i] = Dl[(i - p0) * LD + k];
      }
    }
    __syncthreads();
  }
}

// packing into the wrapped-diagonal layout: c_s[k] = W[k, (k + s) mod n]
__global__ void k_pack_circdiag(const double2* __restrict__ ws, float2* __restrict__ factor, FactorLayout L,
                                int blk0) {
  const int s = blockIdx.y;
  const int k = threadIdx.x;
  const int n = L.n;
  if (k >= n) return;
  const bool half = s == L.F;  // only launched for even n
  if (half && k >= n / 2) return;
  const double2* W = ws + (size_t)blockIdx.x * n * n;
  int col = k + s;
  col -= col >= n ? n : 0;
  const double2 w = W[(size_t)col * n + k];
  const size_t blk = (size_t)blk0 + blockIdx.x;
  const size_t off = half ? half_offset(L, blk) : diag_offset(L, blk, s);
  factor[off + k] = make_float2((float)w.x, (float)w.y);
}

static inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

int build_factor(cs_plan* p, float mu, hipStream_t s) {
  const int nv = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt, nc = p->desc.nc;
  const size_t nblocks = (size_t)nt * nh;
  const size_t blk_bytes = (size_t)nv * nv * sizeof(double2);
  const size_t ws_limit = (size_t)1 << 30;
  const size_t chunk = std::max<size_t>(1, std::min(nblocks, ws_limit / blk_bytes));
  double2* ws = static_cast<double2*>(p->alloc.get(chunk * blk_bytes));
  if (!ws) return set_error(CS_ENOMEM, "allocator returned NULL for the FP64 factor workspace");
  const int wg = round_up(nv, 64);
  const int nb = nv <= 256 ? 16 : 8;
  const size_t lds_gj = ((size_t)nv * nb + (size_t)nb * (nb + 1)) * sizeof(double2);
  const int ndiag = (nv & 1) ? (nv + 1) / 2 : nv / 2 + 1;
  if (lds_gj > 65536) {
    hipError_t ea = nb == 16 ? hipFuncSetAttribute((const void*)k_gj_inverse<16>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_gj)
                             : hipFuncSetAttribute((const void*)k_gj_inverse<8>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_gj);
    if (ea != hipSuccess) {
      p->alloc.put(ws);
      return hip_fail(ea, "hipFuncSetAttribute(k_gj_inverse)");
    }
  }
  int st = CS_OK;
  for (size_t b0 = 0; b0 < nblocks && st == CS_OK; b0 += chunk) {
    const int nblk = (int)std::min(chunk, nblocks - b0);
    hipLaunchKernelGGL(k_gram_assemble, dim3(nblk), dim3(wg), (size_t)16 * nv * sizeof(float2), s, ws,
                       p->coil_cm, p->pcol, nv, nh, nc, (int)b0, (double)mu);
    if (nb == 16)
      hipLaunchKernelGGL(k_gj_inverse<16>, dim3(nblk), dim3(wg), lds_gj, s, ws, nv);
    else
      hipLaunchKernelGGL(k_gj_inverse<8>, dim3(nblk), dim3(wg), lds_gj, s, ws, nv);
    hipLaunchKernelGGL(k_pack_circdiag, dim3(nblk, ndiag), dim3(wg), 0, s, ws, p->factor, p->flayout, (int)b0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) st = hip_fail(e, "factor kernels");
  }
  hipError_t e = hipStreamSynchronize(s);
  p->alloc.put(ws);
  if (st != CS_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(factor)");
  p->mu = mu;
  return CS_OK;
}

// ---------------------------------------------------------------- eigen form
//
// The paper's own factor (Sec. IV-C, eq. eigen_mu): G_{i,t} = U diag(e) U'
// once per plan, after which (mu I + G)^{-1} b = U diag(1/(mu + e)) U' b for
// any mu.  G is assembled in FP64 as above (mu = 0) and decomposed by the
// batched Hermitian divide-and-conquer eigensolver of rocSOLVER (ascending
// e, orthonormal eigenvectors in the columns).  Stored per block, in
// complex64 / float:
//   uh[j][k] = conj(U[j, k])  (row j of U, conjugated: the U' b pass reads a
//                              contiguous row per right-hand-side value)
//   uc[k][j] = U[j, k]        (column k of U: the U s pass reads a
//                              contiguous column per coefficient)
//   e[k]
// so both passes of the apply stream their n x n values front to back.

__global__ void k_pack_eigen(const double2* __restrict__ ws, const double* __restrict__ ev,
                             float2* __restrict__ uh, float2* __restrict__ uc, float* __restrict__ eo, int n,
                             int blk0) {
  const int k = blockIdx.y;  // eigenvector
  const int j = threadIdx.x;
  if (j >= n) return;
  const size_t nn = (size_t)n * n;
  const size_t blk = (size_t)blk0 + blockIdx.x;
  const double2 u = ws[(size_t)blockIdx.x * nn + (size_t)k * n + j];
  uc[blk * nn + (size_t)k * n + j] = make_float2((float)u.x, (float)u.y);
  uh[blk * nn + (size_t)j * n + k] = make_float2((float)u.x, (float)-u.y);
  if (j == 0) eo[blk * n + k] = (float)ev[(size_t)blockIdx.x * n + k];
}

static int rocsolver_fail(rocblas_status r, const char* what) {
  return set_error(CS_EDEVICE, std::string(what) + ": " + rocblas_status_to_string(r));
}

int build_factor_eigen(cs_plan* p, hipStream_t s) {
  const int n = p->desc.nv, nh = p->desc.nh, nt = p->desc.nt, nc = p->desc.nc;
  const size_t nblocks = (size_t)nt * nh;
  const size_t nn = (size_t)n * n;
  // per block: the matrix (overwritten by U), e, the tridiagonal off-diagonal, info
  const size_t blk_bytes = nn * sizeof(double2) + 2 * (size_t)n * sizeof(double) + sizeof(rocblas_int);
  const size_t ws_limit = (size_t)1 << 30;
  const size_t chunk = std::max<size_t>(1, std::min(nblocks, ws_limit / blk_bytes));
  double2* ws = static_cast<double2*>(p->alloc.get(chunk * nn * sizeof(double2)));
  double* dv = static_cast<double*>(p->alloc.get(chunk * 2 * (size_t)n * sizeof(double)));
  rocblas_int* info = static_cast<rocblas_int*>(p->alloc.get(std::max<size_t>(chunk * sizeof(rocblas_int), 256)));
  rocblas_handle h = nullptr;
  void* lib_ws = nullptr;  // the solver's internal workspace, also from the plan's allocator
  auto done = [&](int status) {
    if (h) (void)rocblas_destroy_handle(h);
    if (lib_ws) p->alloc.put(lib_ws);
    if (ws) p->alloc.put(ws);
    if (dv) p->alloc.put(dv);
    if (info) p->alloc.put(info);
    return status;
  };
  if (!ws || !dv || !info) return done(set_error(CS_ENOMEM, "allocator returned NULL for the eigensolver workspace"));
  rocblas_status r = rocblas_create_handle(&h);
  if (r != rocblas_status_success) {
    h = nullptr;
    return done(rocsolver_fail(r, "rocblas_create_handle"));
  }
  if ((r = rocblas_set_stream(h, s)) != rocblas_status_success) return done(rocsolver_fail(r, "rocblas_set_stream"));
  // the solver's device workspace: its size for the largest chunk comes from
  // rocBLAS's size query (no kernel runs in query mode), the memory from the
  // plan's allocator, and the handle is switched to that user-owned workspace
  // so that it allocates none of its own
  {
    if ((r = rocblas_start_device_memory_size_query(h)) != rocblas_status_success)
      return done(rocsolver_fail(r, "rocblas_start_device_memory_size_query"));
    (void)rocsolver_zheevd_strided_batched(h, rocblas_evect_original, rocblas_fill_lower, n,
                                           reinterpret_cast<rocblas_double_complex*>(ws), n, (rocblas_stride)nn,
                                           dv, n, dv + (size_t)chunk * n, n, info, (rocblas_int)chunk);
    size_t lib_bytes = 0;
    if ((r = rocblas_stop_device_memory_size_query(h, &lib_bytes)) != rocblas_status_success)
      return done(rocsolver_fail(r, "rocblas_stop_device_memory_size_query"));
    lib_bytes = std::max<size_t>(lib_bytes, 256);
    lib_ws = p->alloc.get(lib_bytes);
    if (!lib_ws) return done(set_error(CS_ENOMEM, "allocator returned NULL for the eigensolver's library workspace"));
    if ((r = rocblas_set_workspace(h, lib_ws, lib_bytes)) != rocblas_status_success)
      return done(rocsolver_fail(r, "rocblas_set_workspace"));
    if (rocblas_is_managing_device_memory(h))
      return done(set_error(CS_EDEVICE, "the rocBLAS handle did not take the caller-allocated workspace"));
  }
  const int wg = round_up(n, 64);
  std::vector<rocblas_int> hinfo(chunk);
  for (size_t b0 = 0; b0 < nblocks; b0 += chunk) {
    const int nblk = (int)std::min(chunk, nblocks - b0);
    double* ev = dv;
    double* offd = dv + (size_t)chunk * n;
    hipLaunchKernelGGL(k_gram_assemble, dim3(nblk), dim3(wg), (size_t)16 * n * sizeof(float2), s, ws, p->coil_cm,
                       p->pcol, n, nh, nc, (int)b0, 0.0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return done(hip_fail(e, "k_gram_assemble"));
    r = rocsolver_zheevd_strided_batched(h, rocblas_evect_original, rocblas_fill_lower, n,
                                         reinterpret_cast<rocblas_double_complex*>(ws), n, (rocblas_stride)nn, ev,
                                         n, offd, n, info, nblk);
    if (r != rocblas_status_success) return done(rocsolver_fail(r, "rocsolver_zheevd_strided_batched"));
    hipLaunchKernelGGL(k_pack_eigen, dim3(nblk, n), dim3(wg), 0, s, ws, ev, p->eig_uh, p->eig_uc, p->eig_e, n,
                       (int)b0);
    if ((e = hipGetLastError()) != hipSuccess) return done(hip_fail(e, "k_pack_eigen"));
    if ((e = hipMemcpyAsync(hinfo.data(), info, nblk * sizeof(rocblas_int), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return done(hip_fail(e, "eigensolver status copy"));
    for (int b = 0; b < nblk; ++b)
      if (hinfo[b] != 0)
        return done(set_error(CS_EDEVICE, "the eigensolver did not converge for block " + std::to_string(b0 + b)));
  }
  return done(CS_OK);
}

}  // namespace csmri
