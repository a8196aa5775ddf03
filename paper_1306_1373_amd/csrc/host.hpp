// host.hpp -- host-side helpers shared by the translation units of the C ABI:
// argument checks, device check, launch-status mapping and the library lock.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "dctcodec.h"
#include "kernels.hpp"

namespace dct {
namespace host {

inline constexpr int kMaxDevices = 64;
inline constexpr int kMaxW = 65535;
inline constexpr int kMaxH = 1 << 24;  // a stack of images coded as one plane; the 2^32 offset rule binds first
inline constexpr int kMaxQs = 1024;

inline bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// The kernels address a plane with 32-bit offsets: (H - 1) stride + W < 2^32.
inline bool plane_ok(const void *p, int32_t W, int32_t H, int32_t stride) {
  return p != nullptr && aligned(p, 8) && W >= 1 && W <= kMaxW && H >= 1 && H <= kMaxH && stride >= W &&
         stride % 8 == 0 &&
         static_cast<uint64_t>(H - 1) * static_cast<uint64_t>(stride) + static_cast<uint64_t>(W) <
             (uint64_t{1} << 32);
}

// an interleaved RGB image of W x H pixels with row pitch rgb_stride
inline bool rgb_ok(const void *rgb, int32_t W, int32_t H, int32_t rgb_stride) {
  return rgb != nullptr && W >= 1 && W <= kMaxW && H >= 1 && H <= kMaxH && rgb_stride >= 3 * W &&
         static_cast<uint64_t>(H - 1) * static_cast<uint64_t>(rgb_stride) + 3u * static_cast<uint64_t>(W) <
             (uint64_t{1} << 32);
}

inline bool qs_ok(int32_t qs) { return qs >= 1 && qs <= kMaxQs; }

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// DCT_OK when the current device is a gfx950 part (its index to *dev_out).
int check_device(int *dev_out);

inline int launched() { return hipGetLastError() == hipSuccess ? DCT_OK : DCT_ERR_DEVICE; }

inline unsigned grid_for(int64_t items, int threads = kWg) {
  return static_cast<unsigned>((items + threads - 1) / threads);
}

// Quantizer of the fused codec for Q[u][v] = 1 + (1 + u + v) qs under F forward
// and G inverse fractional bits.
CodecQuant codec_quant(int qs, int F, int G);

// Guards the library's shared host state (scratch tables, batch plans).
std::mutex &lock();

}  // namespace host
}  // namespace dct
