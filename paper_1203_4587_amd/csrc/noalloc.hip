// H'y without a plan and without any allocation: cs_apply_AH_noalloc.
//
// The same two adjoint passes as cs_apply_AH (Sec. II-A: H' = S' F~' of the
// stacked operator, x_t = sum_c conj(s_c) . F' M_t y_{t,c}), for callers that
// cannot allocate device memory (code under stream capture, serving loops,
// harnesses that forbid it).  Everything a plan would hold -- the sampled-row
// tables, the twiddles, the coil maps in column-major order, the hybrid-space
// rows and the column-major image -- is carved out of `scratch`, a fixed
// device array of this file.  The tables are built on the device from the
// caller's mask, so the call makes no host round trip either.
//
// Frames are processed in chunks of as many frames as fit the array after the
// tables and the coil maps.  The hybrid rows of a chunk are laid out with
// stride nv (an upper bound of any frame's sampled-row count, which the host
// never reads); rows r >= mcnt[t] are neither written nor read, so nothing
// left in the array by an earlier call is ever used.
#include <mutex>

#include "fft.hpp"

namespace csmri {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // per device, held until the process ends
constexpr int kMaxScratchDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// device address of `scratch` on each device, looked up once per device with
// that device current (in host code the array's name is not a device address)
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kMaxScratchDevices] = {};

static int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxScratchDevices)
    return set_error(CS_EUNSUPPORTED, "cs_apply_AH_noalloc supports device ordinals below 64");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return set_error(CS_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return CS_OK;
}

// Blocks 0..nt-1: the sampled rows of frame t in increasing ky, padded with -1
// to nv, and their count.  Block nt: the twiddles exp(-2 pi i q / n) of both
// axes, rounded from FP64 as the plan's tables are.
__global__ void k_noalloc_tables(const uint8_t* __restrict__ mask, int32_t* __restrict__ rows,
                                 int32_t* __restrict__ mcnt, int32_t* __restrict__ rinv, float2* __restrict__ tw_v,
                                 float2* __restrict__ tw_h, int nv, int nh, int nt) {
  const int t = blockIdx.x;
  if (t < nt) {
    // every entry starts at -1 (all threads), then one thread walks the mask
    // in order and stores only for sampled rows.  (Written this way on
    // purpose: a form that selected "sampled ? r : -1" inside the one-thread
    // loop was compiled into a scalar select on an unrelated condition flag,
    // which left r in the entries of unsampled rows.)
    int32_t* rw = rows + (size_t)t * nv;
    int32_t* ri = rinv + (size_t)t * nv;
    for (int j = threadIdx.x; j < nv; j += blockDim.x) {
      rw[j] = -1;
      ri[j] = -1;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    int r = 0;
    for (int j = 0; j < nv; ++j) {
      if (mask[(size_t)t * nv + j]) {
        ri[j] = r;
        rw[r] = j;
        ++r;
      }
    }
    mcnt[t] = r;
    return;
  }
  for (int q = threadIdx.x; q < nv; q += blockDim.x) {
    const double ang = -2.0 * M_PI * q / nv;
    tw_v[q] = make_float2((float)cos(ang), (float)sin(ang));
  }
  for (int q = threadIdx.x; q < nh; q += blockDim.x) {
    const double ang = -2.0 * M_PI * q / nh;
    tw_h[q] = make_float2((float)cos(ang), (float)sin(ang));
  }
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Byte layout of `scratch` for one call; frames_per_chunk == 0 means the
// sizes do not fit.
struct NoallocLayout {
  size_t rows, mcnt, rinv, tw_v, tw_h, coil, hyb, img;
  size_t need;           // bytes for the tables, the coil maps and one frame
  int frames_per_chunk;
};

static NoallocLayout noalloc_layout(int nv, int nh, int nt, int nc) {
  NoallocLayout L{};
  size_t off = 0;
  L.rows = off;
  off += align256((size_t)nt * nv * sizeof(int32_t));
  L.mcnt = off;
  off += align256((size_t)nt * sizeof(int32_t));
  L.rinv = off;
  off += align256((size_t)nt * nv * sizeof(int32_t));
  L.tw_v = off;
  off += align256((size_t)nv * sizeof(float2));
  L.tw_h = off;
  off += align256((size_t)nh * sizeof(float2));
  L.coil = off;
  off += align256((size_t)nc * nv * nh * sizeof(float2));
  const size_t hyb_frame = align256((size_t)nc * nh * nv * sizeof(float2));
  const size_t img_frame = align256((size_t)nh * nv * sizeof(float2));
  L.need = off + hyb_frame + img_frame;
  if (L.need > kScratchBytes) return L;
  const size_t fit = (kScratchBytes - off) / (hyb_frame + img_frame);
  L.frames_per_chunk = (int)std::min<size_t>(fit, (size_t)nt);
  L.hyb = off;
  L.img = off + (size_t)L.frames_per_chunk * hyb_frame;
  return L;
}

}  // namespace csmri

using namespace csmri;

extern "C" int cs_apply_AH_noalloc(const cs_plan_desc* desc, const cs_c64* coil, const uint8_t* mask,
                                   const cs_c64* y, cs_c64* x, cs_stream stream) {
  if (!desc || !coil || !mask || !y || !x) return set_error(CS_EINVAL, "desc, coil, mask, y and x must not be NULL");
  const int nv = desc->nv, nh = desc->nh, nt = desc->nt, nc = desc->nc;
  if (nv < 2 || nh < 2 || nt < 1 || nc < 1) return set_error(CS_EINVAL, "nv, nh must be >= 2 and nt, nc >= 1");
  FftDesc fv{}, fh{};
  if (!make_fft_desc(nv, &fv) || !make_fft_desc(nh, &fh) || nt > 64 || nc > 64)
    return set_error(CS_EUNSUPPORTED, "nv and nh must be of the form 2^a 3^b and at most 512; nt, nc at most 64");
  const NoallocLayout L = noalloc_layout(nv, nh, nt, nc);
  if (L.frames_per_chunk < 1)
    return set_error(CS_EUNSUPPORTED, "cs_apply_AH_noalloc: the tables, the coil maps and one frame need " +
                                          std::to_string(L.need) + " bytes; its device array holds " +
                                          std::to_string(kScratchBytes));
  int device = 0;
  CS_HIP(hipGetDevice(&device));
  unsigned char* base = nullptr;
  int st = scratch_address(device, &base);
  if (st != CS_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  auto* rows = reinterpret_cast<int32_t*>(base + L.rows);
  auto* mcnt = reinterpret_cast<int32_t*>(base + L.mcnt);
  auto* rinv = reinterpret_cast<int32_t*>(base + L.rinv);
  auto* tw_v = reinterpret_cast<float2*>(base + L.tw_v);
  auto* tw_h = reinterpret_cast<float2*>(base + L.tw_h);
  auto* coil_cm = reinterpret_cast<float2*>(base + L.coil);
  auto* hyb = reinterpret_cast<float2*>(base + L.hyb);
  auto* img = reinterpret_cast<float2*>(base + L.img);
  hipLaunchKernelGGL(k_noalloc_tables, dim3(nt + 1), dim3(256), 0, s, mask, rows, mcnt, rinv, tw_v, tw_h, nv, nh,
                     nt);
  CS_HIP(hipGetLastError());
  // coil maps [c][j][i] -> column-major [c][i][j]
  if ((st = launch_transpose(reinterpret_cast<const float2*>(coil), coil_cm, nc, nv, nh, s)) != CS_OK) return st;
  // tiles as a fresh plan picks them: as many readout columns per wave as fit
  // 256 values, as many sampled rows per workgroup as fit kFftElems values
  const int cw = std::max(1, std::min(nh, 256 / nv));
  const int rb = std::max(1, std::min(nv, kFftElems / nh));
  const size_t kframe = (size_t)nc * nv * nh, iframe = (size_t)nv * nh;
  for (int t0 = 0; t0 < nt; t0 += L.frames_per_chunk) {
    const int f = std::min(L.frames_per_chunk, nt - t0);
    const float2* yc = reinterpret_cast<const float2*>(y) + (size_t)t0 * kframe;
    if ((st = launch_adjoint_rows_raw(yc, hyb, rows + (size_t)t0 * nv, mcnt + t0, fh, tw_h, nv, nh, f, nc, nv, rb,
                                      s)) != CS_OK)
      return st;
    if ((st = launch_adjoint_vertical_raw(hyb, coil_cm, img, rows + (size_t)t0 * nv, mcnt + t0, rinv + (size_t)t0 * nv,
                                          fv, tw_v, nv, nh, f, nc, nv, cw, coil_split16(nh, nt, nc), s)) != CS_OK)
      return st;
    if ((st = launch_transpose(img, reinterpret_cast<float2*>(x) + (size_t)t0 * iframe, f, nh, nv, s)) != CS_OK)
      return st;
  }
  return CS_OK;
}
