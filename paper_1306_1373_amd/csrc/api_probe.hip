// A plain device copy: the HBM bandwidth that a pure read-once, write-once
// stream reaches on the device, the practical ceiling beside which the codec
// kernels' bandwidth is read (their fractions are quoted against the 8 TB/s
// peak).  Not an operation of the codec.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dctcodec.h"
#include "host.hpp"

namespace {

using namespace dct::host;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kCopyThreads = 256;

// One 16-byte word per lane per pass, both accesses non-temporal; every access
// is guarded by i < n.
__global__ __launch_bounds__(kCopyThreads) void copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                            size_t n) {
  const size_t step = static_cast<size_t>(gridDim.x) * kCopyThreads;
  for (size_t i = static_cast<size_t>(blockIdx.x) * kCopyThreads + threadIdx.x; i < n; i += step)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" {

DCT_API int dct_probe_copy(const void *src, void *dst, int64_t bytes, void *stream) {
  if (bytes < 0 || bytes % 16 != 0) return DCT_ERR_INVALID;
  if (bytes == 0) return DCT_OK;  // nothing to do, whatever the pointers
  if (src == nullptr || dst == nullptr || !aligned(src, 16) || !aligned(dst, 16)) return DCT_ERR_INVALID;
  const auto a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
  const auto n = static_cast<uint64_t>(bytes);
  if (a < b + n && b < a + n) return DCT_ERR_INVALID;  // overlapping buffers
  int dev = 0;
  if (int st = check_device(&dev)) return st;
  const uint64_t words = n / 16;
  // one word per lane up to 2^31 - 1 workgroups; the loop takes the rest
  const auto grid = static_cast<unsigned>(
      std::min<uint64_t>((words + kCopyThreads - 1) / kCopyThreads, uint64_t{0x7fffffff}));
  copy_kernel<<<grid, kCopyThreads, 0, as_stream(stream)>>>(static_cast<const u32x4 *>(src),
                                                            static_cast<u32x4 *>(dst), words);
  return launched();
}

}  // extern "C"
