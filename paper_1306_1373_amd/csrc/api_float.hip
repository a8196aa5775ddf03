// api_float.hip -- the floating-point forms of include/dctcodec.h (the exact
// DCT of Sec. 2.5.1 that Sec. 4.1 compares against: FP32 Loeffler, FP16 / BF16
// matrix form on the matrix cores) and the integer YCbCr conversion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "dctcodec.h"
#include "host.hpp"
#include "matrix_form.hpp"

namespace {

using namespace dct::host;

dct::FloatQuant float_quant(int qs) {
  dct::FloatQuant fq{};
  for (int s = 0; s < 15; ++s) {
    const int32_t Q = 1 + (1 + s) * qs;
    fq.Q[s] = static_cast<float>(Q);
    fq.rcp[s] = static_cast<float>(1.0 / Q);
  }
  return fq;
}

bool form_ok(int form) {
  return form == dct::kFormF32Loeffler || form == dct::kFormMfmaF16 || form == dct::kFormMfmaBf16;
}


}  // namespace

extern "C" {

int dct_forward_float(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t form,
                      float *coef, void *stream) {
  if (!plane_ok(src, W, H, src_stride) || coef == nullptr || !aligned(coef, 16) || !form_ok(form))
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int bw = (W + 7) / 8, nblocks = bw * ((H + 7) / 8);
  const int ntiles = (nblocks + 15) / 16;
  hipStream_t s = as_stream(stream);
  const dct::FloatQuant fq{};
  const unsigned kgrid = static_cast<unsigned>(std::min<int64_t>((ntiles + dct::kMfmaWaves - 1) / dct::kMfmaWaves, 4096));
  if (form == dct::kFormF32Loeffler)
    dct::loeffler_f32_kernel<false><<<grid_for(nblocks), dct::kWg, 0, s>>>(src, W, H, src_stride, bw, nblocks, coef,
                                                                           fq, nullptr, 0, nullptr);
  else if (form == dct::kFormMfmaF16)
    dct::kron_kernel<false, false><<<kgrid, 64 * dct::kMfmaWaves, 0, s>>>(src, W, H, src_stride, bw, nblocks, ntiles,
                                                                          coef, fq, nullptr, 0, nullptr);
  else
    dct::kron_kernel<true, false><<<kgrid, 64 * dct::kMfmaWaves, 0, s>>>(src, W, H, src_stride, bw, nblocks, ntiles,
                                                                         coef, fq, nullptr, 0, nullptr);
  return launched();
}

int dct_codec_float(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t form, int32_t qs,
                    uint8_t *dst, int32_t dst_stride, uint64_t *sse_dev, void *stream) {
  if (!plane_ok(src, W, H, src_stride) || !plane_ok(dst, W, H, dst_stride) || !form_ok(form) || qs < 1 ||
      qs > kMaxQs || sse_dev == nullptr || !aligned(sse_dev, 8))
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int bw = (W + 7) / 8, nblocks = bw * ((H + 7) / 8);
  const int ntiles = (nblocks + 15) / 16;
  hipStream_t s = as_stream(stream);
  auto *acc = reinterpret_cast<unsigned long long *>(sse_dev);
  dct::fill_zero_kernel<<<1, 64, 0, s>>>(acc, 1);
  if (launched()) return DCT_ERR_DEVICE;
  const dct::FloatQuant fq = float_quant(qs);
  // one wave per group of kKronCodecTiles tiles, at most 4096 workgroups
  const int64_t ngroups = (ntiles + dct::kKronCodecTiles - 1) / dct::kKronCodecTiles;
  const unsigned kgrid = static_cast<unsigned>(std::min<int64_t>((ngroups + dct::kMfmaWaves - 1) / dct::kMfmaWaves, 4096));
  if (form == dct::kFormF32Loeffler)
    dct::loeffler_f32_kernel<true><<<grid_for(nblocks), dct::kWg, 0, s>>>(src, W, H, src_stride, bw, nblocks, nullptr,
                                                                          fq, dst, dst_stride, acc);
  else if (form == dct::kFormMfmaF16)
    dct::kron_kernel<false, true><<<kgrid, 64 * dct::kMfmaWaves, 0, s>>>(src, W, H, src_stride, bw, nblocks, ntiles,
                                                                         nullptr, fq, dst, dst_stride, acc);
  else
    dct::kron_kernel<true, true><<<kgrid, 64 * dct::kMfmaWaves, 0, s>>>(src, W, H, src_stride, bw, nblocks, ntiles,
                                                                        nullptr, fq, dst, dst_stride, acc);
  return launched();
}

int dct_codec_rgb_float(const uint8_t *rgb, int32_t W, int32_t H, int32_t rgb_stride, int32_t form, int32_t qs,
                        uint8_t *y, uint8_t *cb, uint8_t *cr, int32_t plane_stride, uint64_t *sse_dev,
                        void *stream) {
  if (rgb == nullptr || W < 1 || W > kMaxW || H < 1 || H > kMaxH || rgb_stride < 3 * W ||
      static_cast<uint64_t>(H - 1) * static_cast<uint64_t>(rgb_stride) + 3u * static_cast<uint64_t>(W) >=
          (uint64_t{1} << 32) ||
      !plane_ok(y, W, H, plane_stride) || !plane_ok(cb, W, H, plane_stride) || !plane_ok(cr, W, H, plane_stride) ||
      (form != dct::kFormMfmaF16 && form != dct::kFormMfmaBf16) || qs < 1 || qs > kMaxQs || sse_dev == nullptr ||
      !aligned(sse_dev, 8))
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int bw = (W + 7) / 8, nblocks = bw * ((H + 7) / 8);
  const int ntiles = (nblocks + 15) / 16;
  hipStream_t s = as_stream(stream);
  auto *acc = reinterpret_cast<unsigned long long *>(sse_dev);
  dct::fill_zero_kernel<<<1, 64, 0, s>>>(acc, 3);
  if (launched()) return DCT_ERR_DEVICE;
  const dct::FloatQuant fq = float_quant(qs);
  const bool vec_ok = aligned(rgb, 4) && rgb_stride % 4 == 0;
  const unsigned kgrid =
      static_cast<unsigned>(std::min<int64_t>((ntiles + dct::kMfmaWaves - 1) / dct::kMfmaWaves, 4096));
  if (form == dct::kFormMfmaF16)
    dct::kron_rgb_kernel<false><<<kgrid, 64 * dct::kMfmaWaves, 0, s>>>(rgb, W, H, rgb_stride, vec_ok, bw, nblocks,
                                                                       ntiles, fq, y, cb, cr, plane_stride, acc);
  else
    dct::kron_rgb_kernel<true><<<kgrid, 64 * dct::kMfmaWaves, 0, s>>>(rgb, W, H, rgb_stride, vec_ok, bw, nblocks,
                                                                      ntiles, fq, y, cb, cr, plane_stride, acc);
  return launched();
}

int dct_rgb_to_ycbcr(const uint8_t *rgb, int32_t W, int32_t H, int32_t rgb_stride, uint8_t *y, uint8_t *cb,
                     uint8_t *cr, int32_t plane_stride, void *stream) {
  if (rgb == nullptr || W < 1 || W > kMaxW || H < 1 || H > kMaxH || rgb_stride < 3 * W ||
      static_cast<uint64_t>(H - 1) * static_cast<uint64_t>(rgb_stride) + 3u * static_cast<uint64_t>(W) >=
          (uint64_t{1} << 32) ||
      !plane_ok(y, W, H, plane_stride) || !plane_ok(cb, W, H, plane_stride) || !plane_ok(cr, W, H, plane_stride))
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int64_t total = static_cast<int64_t>((W + 7) / 8) * H;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(grid_for(total), 16384));
  const bool vec_ok = aligned(rgb, 8) && rgb_stride % 8 == 0;
  dct::ycbcr_kernel<<<grid, dct::kWg, 0, as_stream(stream)>>>(rgb, W, H, rgb_stride, y, cb, cr, plane_stride,
                                                              vec_ok);
  return launched();
}

}  // extern "C"
