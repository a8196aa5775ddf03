// api_codec.hip -- the fused codec entry points of include/dctcodec.h (steps
// a1-a9 in one pass) under the default recipe and under the built family.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "codec_launch.hpp"
#include "dctcodec.h"
#include "host.hpp"
#include "rows.hpp"

namespace dct {
namespace host {

int recipes_default(const RecipeEntry **out) {
  static constexpr RecipeEntry k[] = {entry<kIter, kFrac, kFrac>()};
  *out = k;
  return 1;
}

}  // namespace host
}  // namespace dct

namespace {

using namespace dct::host;

// Calls f on each built recipe in list order (the default first) until it returns true.
template <class Fn>
void for_each_recipe(Fn &&f) {
  int (*const parts[])(const RecipeEntry **) = {recipes_default, recipes_n4_n6, recipes_n8_n10, recipes_n12};
  for (auto part : parts) {
    const RecipeEntry *e = nullptr;
    const int n = part(&e);
    for (int i = 0; i < n; ++i)
      if (f(e[i])) return;
  }
}

const RecipeEntry *find_recipe(int n, int F, int G) {
  const RecipeEntry *found = nullptr;
  for_each_recipe([&](const RecipeEntry &r) {
    if (r.n == n && r.F == F && r.G == G) found = &r;
    return found != nullptr;
  });
  return found;
}

// The default recipe with one lane per block row (rows.hpp), after zeroing the
// SSE word unless zero_sse is false.
int codec_rows(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t qs, uint8_t *dst,
               int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream, bool zero_sse) {
  if (int st = check_device(nullptr)) return st;
  using RC = dct::DefaultRecipe;
  const int bw = (W + 7) / 8, nblocks = bw * ((H + 7) / 8);
  const unsigned grid = dct::rows::launch_groups((nblocks + 7) / 8);
  auto *sse = reinterpret_cast<unsigned long long *>(sse_dev);
  hipStream_t s = as_stream(stream);
  if (zero_sse) {
    dct::fill_zero_kernel<<<1, 64, 0, s>>>(sse, 1);
    if (launched()) return DCT_ERR_DEVICE;
  }
  const dct::CodecQuant qa = codec_quant(qs, RC::frac, RC::inv_frac);
  if (qcoef_or_null)
    dct::rows::codec_rows_kernel<RC, true><<<grid, dct::rows::kThreads, 0, s>>>(
        src, W, H, src_stride, bw, nblocks, qa, dst, dst_stride, qcoef_or_null, sse);
  else
    dct::rows::codec_rows_kernel<RC, false><<<grid, dct::rows::kThreads, 0, s>>>(
        src, W, H, src_stride, bw, nblocks, qa, dst, dst_stride, nullptr, sse);
  return launched();
}

// The lane-per-block kernel under recipe rc; zero_sse: overwrite *sse_dev rather than add to it
int codec_common(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, const RecipeEntry &rc, int32_t qs,
                 uint8_t *dst, int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream,
                 bool zero_sse = true) {
  if (int st = check_device(nullptr)) return st;
  CodecArgs a{};
  a.src = src;
  a.W = W;
  a.H = H;
  a.src_stride = src_stride;
  a.bw = (W + 7) / 8;
  a.nblocks = a.bw * ((H + 7) / 8);
  a.qa = codec_quant(qs, rc.F, rc.G);
  a.dst = dst;
  a.dst_stride = dst_stride;
  a.qcoef = qcoef_or_null;
  a.sse = reinterpret_cast<unsigned long long *>(sse_dev);
  hipStream_t s = as_stream(stream);
  if (zero_sse) {
    dct::fill_zero_kernel<<<1, 64, 0, s>>>(a.sse, 1);
    if (launched()) return DCT_ERR_DEVICE;
  }
  rc.launch(a, s);
  return launched();
}

bool codec_args_ok(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t qs, const uint8_t *dst,
                   int32_t dst_stride, const int16_t *qcoef_or_null, const uint64_t *sse_dev) {
  return plane_ok(src, W, H, src_stride) && plane_ok(dst, W, H, dst_stride) && qs_ok(qs) && sse_dev != nullptr &&
         aligned(sse_dev, 8) && (qcoef_or_null == nullptr || aligned(qcoef_or_null, 16));
}

}  // namespace

extern "C" {

int dct_codec(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t qs, uint8_t *dst,
              int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream) {
  if (!codec_args_ok(src, W, H, src_stride, qs, dst, dst_stride, qcoef_or_null, sse_dev)) return DCT_ERR_INVALID;
  return codec_rows(src, W, H, src_stride, qs, dst, dst_stride, qcoef_or_null, sse_dev, stream, true);
}

int dct_codec_accumulate(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t qs, uint8_t *dst,
                         int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream) {
  if (!codec_args_ok(src, W, H, src_stride, qs, dst, dst_stride, qcoef_or_null, sse_dev)) return DCT_ERR_INVALID;
  return codec_rows(src, W, H, src_stride, qs, dst, dst_stride, qcoef_or_null, sse_dev, stream, false);
}

int dct_codec_blocks(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t qs, uint8_t *dst,
                     int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream) {
  if (!codec_args_ok(src, W, H, src_stride, qs, dst, dst_stride, qcoef_or_null, sse_dev)) return DCT_ERR_INVALID;
  const RecipeEntry *rc = nullptr;
  recipes_default(&rc);
  return codec_common(src, W, H, src_stride, *rc, qs, dst, dst_stride, qcoef_or_null, sse_dev, stream);
}

int dct_codec_recipe(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t n_iter,
                     int32_t frac_bits, int32_t inv_frac_bits, int32_t qs, uint8_t *dst, int32_t dst_stride,
                     int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream) {
  if (!codec_args_ok(src, W, H, src_stride, qs, dst, dst_stride, qcoef_or_null, sse_dev)) return DCT_ERR_INVALID;
  const RecipeEntry *rc = find_recipe(n_iter, frac_bits, inv_frac_bits);
  if (rc == nullptr) return DCT_ERR_UNSUPPORTED;
  return codec_common(src, W, H, src_stride, *rc, qs, dst, dst_stride, qcoef_or_null, sse_dev, stream);
}

int dct_recipe_supported(int32_t n_iter, int32_t frac_bits, int32_t inv_frac_bits) {
  return find_recipe(n_iter, frac_bits, inv_frac_bits) != nullptr ? 1 : 0;
}

int dct_recipe_list(int32_t *recipes, int32_t capacity) {
  int count = 0;
  for_each_recipe([&](const RecipeEntry &) {
    ++count;
    return false;
  });
  if (recipes == nullptr) return count;
  if (capacity < 0) return DCT_ERR_INVALID;
  int i = 0;
  for_each_recipe([&](const RecipeEntry &r) {
    if (i >= capacity) return true;
    recipes[3 * i] = r.n;
    recipes[3 * i + 1] = r.F;
    recipes[3 * i + 2] = r.G;
    ++i;
    return false;
  });
  return count;
}

int dct_recipe_tables_n(int32_t n_iter, int32_t *directions, int32_t *gains) {
  if (directions == nullptr || gains == nullptr) return DCT_ERR_INVALID;
  const RecipeEntry *found = nullptr;
  for_each_recipe([&](const RecipeEntry &r) {
    if (r.n == n_iter) found = &r;
    return found != nullptr;
  });
  if (found == nullptr) return DCT_ERR_UNSUPPORTED;
  found->tables(directions, gains);
  return DCT_OK;
}

}  // extern "C"
