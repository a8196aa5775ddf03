// api_core.hip -- the staged entry points of include/dctcodec.h (the paper's
// separate DCT, quantizer and IDCT stages, Sec. 3.2, and PSNR, Sec. 4.1), the
// recipe constants, status strings and the library's shared host state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <mutex>

#include "dctcodec.h"
#include "host.hpp"
#include "kernels.hpp"
#include "staged.hpp"

namespace dct {
namespace host {

namespace {
std::array<int, kMaxDevices> g_arch_ok{};  // 0 unknown, 1 gfx950, -1 other
}  // namespace

std::mutex &lock() {
  static std::mutex m;
  return m;
}

int check_device(int *dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DCT_ERR_DEVICE;
  if (dev < 0 || dev >= kMaxDevices) return DCT_ERR_UNSUPPORTED;
  int ok = __atomic_load_n(&g_arch_ok[dev], __ATOMIC_ACQUIRE);
  if (ok == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return DCT_ERR_DEVICE;
    ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : -1;
    __atomic_store_n(&g_arch_ok[dev], ok, __ATOMIC_RELEASE);
  }
  if (ok < 0) return DCT_ERR_UNSUPPORTED;
  if (dev_out) *dev_out = dev;
  return DCT_OK;
}

// The smallest float r >= 1/Q makes trunc(float(m) r) = floor(m / Q) for every
// m < 2^14 (the lemma the CPU tests check for every table entry); half is the
// rounding offset after the pre-shift max(F - 12, 0).
CodecQuant codec_quant(int qs, int F, int G) {
  CodecQuant qa{};
  const int pre = F > 12 ? F - 12 : 0;
  for (int s = 0; s < 15; ++s) {
    const int32_t Q = 1 + (1 + s) * qs;
    float r = static_cast<float>(1.0 / Q);
    if (static_cast<double>(r) < 1.0 / Q) r = std::nextafter(r, std::numeric_limits<float>::infinity());
    qa.rcp[s] = r;
    qa.qscale[s] = static_cast<float>(Q) * static_cast<float>(1 << G);
    qa.half[s] = Q << (F + 2 - pre);
  }
  return qa;
}

}  // namespace host
}  // namespace dct

namespace {

using namespace dct::host;

// per device: {sse, max pixel}, then {sum, max} of each SSE workgroup
constexpr int kSseMaxGroups = 1024;
std::array<unsigned long long *, kMaxDevices> g_scratch{};  // guarded by lock()
std::array<unsigned long long *, kMaxDevices> g_pinned{};   // per device: pinned host copy of the result

// Scratch of dct_psnr_noalloc: the per-workgroup {sum, max} partials of the SSE
// pass, 16 KiB, in the code object's own data (one copy per device, held until
// the process ends).  Host code must not pass this name to a kernel: it is a
// host-side stand-in; the device address comes from hipGetSymbolAddress and is
// kept per device in g_static_scratch.
__device__ __align__(256) unsigned long long scratch[2 * kSseMaxGroups];
std::array<unsigned long long *, kMaxDevices> g_static_scratch{};  // guarded by lock()

dct::DequantTable dequant_table(int qs) {
  dct::DequantTable dq{};
  for (int s = 0; s < 15; ++s) dq.Q[s] = 1 + (1 + s) * qs;
  return dq;
}

// eq. (23)-(24): 20 log10(MAX / sqrt(SSE / npix)), +inf for SSE = 0
double psnr_of(uint64_t sse, double npix, double peak) {
  if (sse == 0) return std::numeric_limits<double>::infinity();
  const double mse = static_cast<double>(sse) / npix;
  return 20.0 * std::log10(peak / std::sqrt(mse));
}

}  // namespace

extern "C" {

int dct_forward(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t *coef, void *stream) {
  if (!plane_ok(src, W, H, src_stride) || coef == nullptr || !aligned(coef, 16)) return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int bw = (W + 7) / 8, nblocks = bw * ((H + 7) / 8);
  dct::forward_kernel<<<grid_for(nblocks, dct::kBlockThreads), dct::kBlockThreads, 0, as_stream(stream)>>>(
      src, W, H, src_stride, bw, nblocks, coef);
  return launched();
}

int dct_quantize(const int32_t *coef, int64_t nblocks, int32_t qs, int16_t *qcoef, void *stream) {
  if (nblocks < 0 || nblocks > (int64_t{1} << 28) || !qs_ok(qs)) return DCT_ERR_INVALID;
  if (nblocks == 0) return DCT_OK;
  if (coef == nullptr || qcoef == nullptr || !aligned(coef, 16) || !aligned(qcoef, 16)) return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int64_t nrows = nblocks * 8;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(grid_for(nrows), 1 << 20));
  dct::quantize_kernel<<<grid, dct::kWg, 0, as_stream(stream)>>>(coef, nrows, qs, qcoef);
  return launched();
}

int dct_inverse(const int16_t *qcoef, int32_t qs, int32_t W, int32_t H, uint8_t *dst, int32_t dst_stride,
                void *stream) {
  if (!plane_ok(dst, W, H, dst_stride) || qcoef == nullptr || !aligned(qcoef, 16) || !qs_ok(qs))
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int bw = (W + 7) / 8, nblocks = bw * ((H + 7) / 8);
  dct::inverse_kernel<<<grid_for(nblocks, dct::kBlockThreads), dct::kBlockThreads, 0, as_stream(stream)>>>(
      qcoef, dequant_table(qs), W, H, bw, nblocks, dst, dst_stride);
  return launched();
}

int dct_psnr(const uint8_t *a, int32_t a_stride, const uint8_t *b, int32_t b_stride, int32_t W, int32_t H,
             double peak, double *psnr_host, uint64_t *sse_host, void *stream) {
  if (!plane_ok(a, W, H, a_stride) || !plane_ok(b, W, H, b_stride) || psnr_host == nullptr || !(peak >= 0.0) ||
      std::isinf(peak))
    return DCT_ERR_INVALID;
  int dev = 0;
  if (int st = check_device(&dev)) return st;
  std::lock_guard<std::mutex> guard(lock());
  if (g_scratch[dev] == nullptr) {
    void *p = nullptr;
    if (hipMalloc(&p, (2 + 2 * kSseMaxGroups) * sizeof(unsigned long long)) != hipSuccess) return DCT_ERR_NOMEM;
    g_scratch[dev] = static_cast<unsigned long long *>(p);
  }
  if (g_pinned[dev] == nullptr) {
    void *p = nullptr;
    if (hipHostMalloc(&p, 2 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) return DCT_ERR_NOMEM;
    g_pinned[dev] = static_cast<unsigned long long *>(p);
  }
  unsigned long long *acc = g_scratch[dev];
  unsigned long long *host = g_pinned[dev];
  hipStream_t s = as_stream(stream);
  // grid.x covers a row's 8-byte segments, grid.y strides over rows: at most
  // kSseMaxGroups workgroups, each writing its own partial (every one is written)
  const int segs = (W + 7) / 8;
  const unsigned gx = static_cast<unsigned>(std::min((segs + dct::kWg - 1) / dct::kWg, 16));
  const unsigned gy = static_cast<unsigned>(std::max(1, std::min<int>(H, kSseMaxGroups / static_cast<int>(gx))));
  unsigned long long *partial = acc + 2;
  dct::sse_kernel<<<dim3(gx, gy), dct::kWg, 0, s>>>(a, a_stride, b, b_stride, W, H, partial);
  if (launched()) return DCT_ERR_DEVICE;
  dct::sse_reduce_kernel<<<1, dct::kWg, 0, s>>>(partial, static_cast<int>(gx * gy), acc);
  if (launched()) return DCT_ERR_DEVICE;
  // the 16-byte result comes back through a pinned buffer: no staging copy
  if (hipMemcpyAsync(host, acc, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s) != hipSuccess)
    return DCT_ERR_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return DCT_ERR_DEVICE;
  const uint64_t sse = host[0];
  const double mx = peak > 0.0 ? peak : static_cast<double>(static_cast<uint32_t>(host[1]));
  if (sse_host) *sse_host = sse;
  *psnr_host = psnr_of(sse, static_cast<double>(W) * static_cast<double>(H), mx);
  return DCT_OK;
}

int dct_psnr_noalloc(const uint8_t *a, int32_t a_stride, const uint8_t *b, int32_t b_stride, int32_t W, int32_t H,
                     uint64_t *result_dev, void *stream) {
  if (!plane_ok(a, W, H, a_stride) || !plane_ok(b, W, H, b_stride) || result_dev == nullptr ||
      !aligned(result_dev, 8))
    return DCT_ERR_INVALID;
  int dev = 0;
  if (int st = check_device(&dev)) return st;
  unsigned long long *partial = nullptr;
  {
    std::lock_guard<std::mutex> guard(lock());
    if (g_static_scratch[dev] == nullptr) {
      // once per device, with that device current: the address of this device's copy
      void *p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return DCT_ERR_DEVICE;
      g_static_scratch[dev] = static_cast<unsigned long long *>(p);
    }
    partial = g_static_scratch[dev];
  }
  // the same grid as dct_psnr: at most kSseMaxGroups workgroups, each of which
  // writes its own {sum, max} pair, so nothing in the scratch needs clearing
  const int segs = (W + 7) / 8;
  const unsigned gx = static_cast<unsigned>(std::min((segs + dct::kWg - 1) / dct::kWg, 16));
  const unsigned gy = static_cast<unsigned>(std::max(1, std::min<int>(H, kSseMaxGroups / static_cast<int>(gx))));
  if (gx * gy > static_cast<unsigned>(kSseMaxGroups)) return DCT_ERR_INVALID;  // beyond the scratch (never, by the grid rule)
  hipStream_t s = as_stream(stream);
  dct::sse_kernel<<<dim3(gx, gy), dct::kWg, 0, s>>>(a, a_stride, b, b_stride, W, H, partial);
  if (launched()) return DCT_ERR_DEVICE;
  dct::sse_reduce_kernel<<<1, dct::kWg, 0, s>>>(partial, static_cast<int>(gx * gy),
                                                 reinterpret_cast<unsigned long long *>(result_dev));
  return launched();
}

int dct_psnr_from_sse(uint64_t sse, int64_t npix, double peak, double *psnr_host) {
  if (npix < 1 || !(peak > 0.0) || std::isinf(peak) || psnr_host == nullptr) return DCT_ERR_INVALID;
  *psnr_host = psnr_of(sse, static_cast<double>(npix), peak);
  return DCT_OK;
}

int dct_recipe_info(int32_t *n_iter, int32_t *frac_bits, int32_t *comp_bits) {
  if (n_iter == nullptr || frac_bits == nullptr || comp_bits == nullptr) return DCT_ERR_INVALID;
  *n_iter = dct::kIter;
  *frac_bits = dct::kFrac;
  *comp_bits = dct::kComp;
  return DCT_OK;
}

int dct_recipe_tables(int32_t *directions, int32_t *gains) { return dct_recipe_tables_n(dct::kIter, directions, gains); }

const char *dct_status_string(int status) {
  switch (status) {
    case DCT_OK: return "ok";
    case DCT_ERR_INVALID: return "invalid argument";
    case DCT_ERR_UNSUPPORTED: return "unsupported device (gfx950 required) or recipe not built";
    case DCT_ERR_DEVICE: return "HIP runtime error";
    case DCT_ERR_NOMEM: return "out of device memory";
    default: return "unknown status";
  }
}

int dct_shutdown(void) {
  std::lock_guard<std::mutex> guard(lock());
  int rc = DCT_OK;
  for (auto &p : g_scratch) {
    if (p != nullptr) {
      if (hipFree(p) != hipSuccess) rc = DCT_ERR_DEVICE;
      p = nullptr;
    }
  }
  for (auto &p : g_pinned) {
    if (p != nullptr) {
      if (hipHostFree(p) != hipSuccess) rc = DCT_ERR_DEVICE;
      p = nullptr;
    }
  }
  return rc;
}

}  // extern "C"
