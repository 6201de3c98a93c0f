// cs_read_stream: the HBM read rate this chip sustains for a pure read
// stream, a yardstick for the HBM-bound kernels (the x-update reads its packed
// inverse factor once per iteration and is limited by exactly this rate).
// Not part of the method; callers time a launch themselves.
//
// Each workgroup reads one contiguous tile of 256 x 8 16-byte values (32 KB)
// per step with non-temporal loads, eight in flight per thread, and moves on
// by the grid's width in tiles; a sum of everything read is stored to *sink
// only when it equals a value no real buffer produces, so the loads stay live
// and nothing is written in practice.  (Contiguous tiles per workgroup hold
// about 7.1 TB/s on MI355X at any grid from 1024 to 16384 workgroups; a
// thread-strided grid loop with the same loads in flight stays near 6.2.)
#include "internal.hpp"

namespace csmri {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kReadThreads = 256;
constexpr int kReadUnroll = 8;
constexpr int kReadDefaultBlocks = 8192;

__global__ __launch_bounds__(kReadThreads) void k_read_stream(const v4f* __restrict__ p, size_t n4,
                                                              float* __restrict__ sink) {
  constexpr size_t kTile = (size_t)kReadThreads * kReadUnroll;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  const size_t full = n4 / kTile;
  for (size_t t = blockIdx.x; t < full; t += gridDim.x) {
    const v4f* q = p + t * kTile + threadIdx.x;
    v4f v[kReadUnroll];
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) v[u] = __builtin_nontemporal_load(q + u * kReadThreads);
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) acc += v[u];
  }
  for (size_t i = full * kTile + (size_t)blockIdx.x * kReadThreads + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * kReadThreads)
    acc += __builtin_nontemporal_load(p + i);
  const float s = acc.x + acc.y + acc.z + acc.w;
  if (s == -1.2345e-37f) *sink = s;
}

}  // namespace csmri

using namespace csmri;

extern "C" int cs_read_stream(const void* buf, size_t bytes, int32_t blocks, float* sink, cs_stream stream) {
  if (!buf || !sink) return set_error(CS_EINVAL, "buf and sink must not be NULL");
  if (bytes == 0 || bytes % 16 != 0) return set_error(CS_EINVAL, "bytes must be a positive multiple of 16");
  if (reinterpret_cast<uintptr_t>(buf) % 16 != 0) return set_error(CS_EINVAL, "buf must be 16-byte aligned");
  if (blocks < 0 || blocks > 65535) return set_error(CS_EINVAL, "blocks must be in [0, 65535] (0: default)");
  const unsigned grid = blocks ? (unsigned)blocks : (unsigned)kReadDefaultBlocks;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_read_stream, dim3(grid), dim3(kReadThreads), 0, s, static_cast<const v4f*>(buf), bytes / 16,
                     sink);
  CS_HIP(hipGetLastError());
  return CS_OK;
}
