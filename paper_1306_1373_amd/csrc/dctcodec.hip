// dctcodec.hip -- the C ABI of include/dctcodec.h: argument checks, quantizer
// constants, launch shapes, and error mapping.  The kernels are in kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <mutex>

#include <unordered_map>
#include <vector>

#include "batch.hpp"
#include "deblock.hpp"
#include "dctcodec.h"
#include "kernels.hpp"
#include "matrix_form.hpp"

namespace {

constexpr int kMaxDevices = 64;
constexpr int kMaxW = 65535;
constexpr int kMaxH = 1 << 24;  // a stack of images coded as one plane; the 2^32 offset rule binds first
constexpr int kMaxQs = 1024;

std::mutex g_lock;                                   // guards the scratch table and dct_psnr
// per device: {sse, max pixel}, then {sum, max} of each SSE workgroup
constexpr int kSseMaxGroups = 1024;
std::array<unsigned long long *, kMaxDevices> g_scratch{};
std::array<unsigned long long *, kMaxDevices> g_pinned{};   // per device: pinned host copy of the same
std::array<int, kMaxDevices> g_arch_ok{};            // 0 unknown, 1 gfx950, -1 other

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// The kernels address a plane with 32-bit offsets: (H - 1) stride + W < 2^32.
bool plane_ok(const void *p, int32_t W, int32_t H, int32_t stride) {
  return p != nullptr && aligned(p, 8) && W >= 1 && W <= kMaxW && H >= 1 && H <= kMaxH &&
         stride >= W && stride % 8 == 0 &&
         static_cast<uint64_t>(H - 1) * static_cast<uint64_t>(stride) + static_cast<uint64_t>(W) <
             (uint64_t{1} << 32);
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// The current device must be a gfx950 part.
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

int launched() { return hipGetLastError() == hipSuccess ? DCT_OK : DCT_ERR_DEVICE; }

// Quantizer of the fused codec for Q[u][v] = 1 + (1 + u + v) qs, indexed by u + v,
// under F forward and G inverse fractional bits: the smallest float r >= 1/Q
// makes trunc(float(m) r) = floor(m / Q) for every m < 2^14 (the lemma the CPU
// tests check for every table entry); half is the rounding offset after the
// pre-shift max(F - 12, 0).
dct::CodecQuant codec_quant(int qs, int F, int G) {
  dct::CodecQuant qa{};
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

// The fused codec under one recipe.
struct CodecArgs {
  const uint8_t *src;
  int W, H, src_stride, bw, nblocks;
  dct::CodecQuant qa;
  uint8_t *dst;
  int dst_stride;
  int16_t *qcoef;
  unsigned long long *sse;
};

template <class RC>
void launch_codec(const CodecArgs &a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>((a.nblocks + dct::kBlockThreads - 1) / dct::kBlockThreads);
  if (a.qcoef)
    dct::codec_kernel<RC, true><<<grid, dct::kBlockThreads, 0, s>>>(a.src, a.W, a.H, a.src_stride, a.bw, a.nblocks,
                                                                   a.qa, a.dst, a.dst_stride, a.qcoef, a.sse);
  else
    dct::codec_kernel<RC, false><<<grid, dct::kBlockThreads, 0, s>>>(a.src, a.W, a.H, a.src_stride, a.bw, a.nblocks,
                                                                    a.qa, a.dst, a.dst_stride, nullptr, a.sse);
}

struct RecipeEntry {
  int n, F, G;
  void (*launch)(const CodecArgs &, hipStream_t);
  void (*tables)(int32_t *, int32_t *);
};

template <int N>
void copy_tables(int32_t *directions, int32_t *gains) {
  for (int r = 0; r < 3; ++r)
    for (int i = 0; i < N; ++i) directions[r * N + i] = dct::kTablesN<N>.dir[r][i];
  for (int r = 0; r < 3; ++r) gains[r] = dct::kTablesN<N>.gain[r];
  gains[3] = dct::kTablesN<N>.sqrt2;
}

template <int N, int F, int G>
constexpr RecipeEntry entry() {
  return {N, F, G, &launch_codec<dct::Recipe<N, F, G>>, &copy_tables<N>};
}

// The recipes the library is built with: n in {4, 6, 8, 10, 12} micro-rotations,
// (F, G) in {(8, 8), (12, 12), (16, 12)}.  The first is the default.
constexpr RecipeEntry kRecipes[] = {
    entry<10, 12, 12>(), entry<4, 8, 8>(),   entry<4, 12, 12>(), entry<4, 16, 12>(), entry<6, 8, 8>(),
    entry<6, 12, 12>(),  entry<6, 16, 12>(), entry<8, 8, 8>(),   entry<8, 12, 12>(), entry<8, 16, 12>(),
    entry<10, 8, 8>(),   entry<10, 16, 12>(), entry<12, 8, 8>(), entry<12, 12, 12>(), entry<12, 16, 12>(),
};

const RecipeEntry *find_recipe(int n, int F, int G) {
  for (const RecipeEntry &r : kRecipes)
    if (r.n == n && r.F == F && r.G == G) return &r;
  return nullptr;
}

int codec_common(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, const RecipeEntry &rc, int32_t qs,
                 uint8_t *dst, int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream);

// workgroups of a weight-gradient pass at most (each writes one partial row)
constexpr int kGradGroups = 2048;

struct DeblockLayout {
  size_t wq, wh, sq, a1, a2, a3, g4, ga, gb, part, bytes;
};
DeblockLayout deblock_layout(int64_t npix, bool training);
int deblock_forward(const dct::db::ImageSet &set, int64_t npix, const float *params, uint8_t *ws,
                    const DeblockLayout &L, uint8_t *out, int out_stride, float *y, float *grad, double *loss,
                    hipStream_t s);
int deblock_backward(const dct::db::ImageSet &set, int64_t npix, uint8_t *ws, const DeblockLayout &L, float *grad,
                     hipStream_t s);

// Batches planned into a workspace: the host keeps what a run needs to launch
// safely, so dct_batch_run never trusts sizes it is handed.
struct BatchPlan {
  int64_t total_chunks;
  int32_t n_images, chunk;
  int64_t images_offset, table_offset;
};
std::unordered_map<const void *, BatchPlan> g_batches;  // guarded by g_lock

bool chunk_ok(int chunk) { return chunk == 256 || chunk == 512; }

// Chunks of each image and the workspace layout; false if an image is invalid.
bool batch_layout(const dct_image *images, int32_t n, int32_t chunk, BatchPlan &plan, size_t &bytes) {
  if (images == nullptr || n < 1 || n > (1 << 24) || !chunk_ok(chunk)) return false;
  int64_t chunks = 0;
  for (int32_t k = 0; k < n; ++k) {
    const dct_image &im = images[k];
    if (!plane_ok(im.src, im.W, im.H, im.src_stride) || !plane_ok(im.dst, im.W, im.H, im.dst_stride) ||
        im.qs < 1 || im.qs > kMaxQs)
      return false;
    const int64_t nb = static_cast<int64_t>((im.W + 7) / 8) * ((im.H + 7) / 8);
    chunks += (nb + chunk - 1) / chunk;
  }
  if (chunks >= (int64_t{1} << 31)) return false;
  plan.total_chunks = chunks;
  plan.n_images = n;
  plan.chunk = chunk;
  plan.images_offset = 256;
  plan.table_offset = plan.images_offset + ((static_cast<int64_t>(n) * sizeof(dct::BatchImage) + 255) / 256) * 256;
  bytes = static_cast<size_t>(plan.table_offset + chunks * static_cast<int64_t>(sizeof(int32_t)));
  return true;
}

dct::DequantTable dequant_table(int qs) {
  dct::DequantTable dq{};
  for (int s = 0; s < 15; ++s) dq.Q[s] = 1 + (1 + s) * qs;
  return dq;
}

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

unsigned grid_for(int64_t items, int threads = dct::kWg) {
  return static_cast<unsigned>((items + threads - 1) / threads);
}

}  // namespace

extern "C" {

int dct_forward(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t *coef,
                void *stream) {
  if (!plane_ok(src, W, H, src_stride) || coef == nullptr || !aligned(coef, 16)) return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int bw = (W + 7) / 8, nblocks = bw * ((H + 7) / 8);
  dct::forward_kernel<<<grid_for(nblocks, dct::kBlockThreads), dct::kBlockThreads, 0, as_stream(stream)>>>(
      src, W, H, src_stride, bw, nblocks, coef);
  return launched();
}

int dct_quantize(const int32_t *coef, int64_t nblocks, int32_t qs, int16_t *qcoef, void *stream) {
  if (nblocks < 0 || nblocks > (int64_t{1} << 28) || qs < 1 || qs > kMaxQs) return DCT_ERR_INVALID;
  if (nblocks == 0) return DCT_OK;
  if (coef == nullptr || qcoef == nullptr || !aligned(coef, 16) || !aligned(qcoef, 16))
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int64_t nrows = nblocks * 8;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(grid_for(nrows), 1 << 20));
  dct::quantize_kernel<<<grid, dct::kWg, 0, as_stream(stream)>>>(coef, nrows, qs, qcoef);
  return launched();
}

int dct_inverse(const int16_t *qcoef, int32_t qs, int32_t W, int32_t H, uint8_t *dst,
                int32_t dst_stride, void *stream) {
  if (!plane_ok(dst, W, H, dst_stride) || qcoef == nullptr || !aligned(qcoef, 16) || qs < 1 ||
      qs > kMaxQs)
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const int bw = (W + 7) / 8, nblocks = bw * ((H + 7) / 8);
  dct::inverse_kernel<<<grid_for(nblocks, dct::kBlockThreads), dct::kBlockThreads, 0, as_stream(stream)>>>(
      qcoef, dequant_table(qs), W, H, bw, nblocks, dst, dst_stride);
  return launched();
}

int dct_psnr(const uint8_t *a, int32_t a_stride, const uint8_t *b, int32_t b_stride, int32_t W,
             int32_t H, double peak, double *psnr_host, uint64_t *sse_host, void *stream) {
  if (!plane_ok(a, W, H, a_stride) || !plane_ok(b, W, H, b_stride) || psnr_host == nullptr ||
      !(peak >= 0.0) || std::isinf(peak))
    return DCT_ERR_INVALID;
  int dev = 0;
  if (int st = check_device(&dev)) return st;
  std::lock_guard<std::mutex> guard(g_lock);
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
  if (sse == 0) {
    *psnr_host = std::numeric_limits<double>::infinity();
  } else {
    const double mse = static_cast<double>(sse) / (static_cast<double>(W) * static_cast<double>(H));
    *psnr_host = 20.0 * std::log10(mx / std::sqrt(mse));
  }
  return DCT_OK;
}

int dct_codec(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t qs, uint8_t *dst,
              int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream) {
  if (!plane_ok(src, W, H, src_stride) || !plane_ok(dst, W, H, dst_stride) || qs < 1 || qs > kMaxQs ||
      sse_dev == nullptr || !aligned(sse_dev, 8) ||
      (qcoef_or_null != nullptr && !aligned(qcoef_or_null, 16)))
    return DCT_ERR_INVALID;
  return codec_common(src, W, H, src_stride, kRecipes[0], qs, dst, dst_stride, qcoef_or_null, sse_dev, stream);
}

int dct_codec_recipe(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t n_iter,
                     int32_t frac_bits, int32_t inv_frac_bits, int32_t qs, uint8_t *dst, int32_t dst_stride,
                     int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream) {
  if (!plane_ok(src, W, H, src_stride) || !plane_ok(dst, W, H, dst_stride) || qs < 1 || qs > kMaxQs ||
      sse_dev == nullptr || !aligned(sse_dev, 8) ||
      (qcoef_or_null != nullptr && !aligned(qcoef_or_null, 16)))
    return DCT_ERR_INVALID;
  const RecipeEntry *rc = find_recipe(n_iter, frac_bits, inv_frac_bits);
  if (rc == nullptr) return DCT_ERR_UNSUPPORTED;
  return codec_common(src, W, H, src_stride, *rc, qs, dst, dst_stride, qcoef_or_null, sse_dev, stream);
}

int dct_recipe_supported(int32_t n_iter, int32_t frac_bits, int32_t inv_frac_bits) {
  return find_recipe(n_iter, frac_bits, inv_frac_bits) != nullptr ? 1 : 0;
}

int dct_recipe_list(int32_t *recipes, int32_t capacity) {
  const int count = static_cast<int>(sizeof(kRecipes) / sizeof(kRecipes[0]));
  if (recipes == nullptr) return count;
  if (capacity < 0) return DCT_ERR_INVALID;
  for (int i = 0; i < count && i < capacity; ++i) {
    recipes[3 * i] = kRecipes[i].n;
    recipes[3 * i + 1] = kRecipes[i].F;
    recipes[3 * i + 2] = kRecipes[i].G;
  }
  return count;
}

int dct_recipe_tables_n(int32_t n_iter, int32_t *directions, int32_t *gains) {
  if (directions == nullptr || gains == nullptr) return DCT_ERR_INVALID;
  for (const RecipeEntry &r : kRecipes)
    if (r.n == n_iter) {
      r.tables(directions, gains);
      return DCT_OK;
    }
  return DCT_ERR_UNSUPPORTED;
}

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
  const unsigned kgrid = static_cast<unsigned>(std::min<int64_t>((ntiles + dct::kMfmaWaves - 1) / dct::kMfmaWaves, 4096));
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

size_t dct_batch_workspace_size(const dct_image *images, int32_t n_images, int32_t chunk) {
  BatchPlan plan{};
  size_t bytes = 0;
  return batch_layout(images, n_images, chunk, plan, bytes) ? bytes : 0;
}

int dct_batch_plan(const dct_image *images, int32_t n_images, int32_t chunk, void *workspace,
                   size_t workspace_bytes, int64_t *total_chunks, void *stream) {
  BatchPlan plan{};
  size_t bytes = 0;
  if (!batch_layout(images, n_images, chunk, plan, bytes) || workspace == nullptr || !aligned(workspace, 256) ||
      workspace_bytes < bytes)
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  std::vector<uint8_t> host(bytes, 0);
  dct::BatchHeader hdr{plan.total_chunks, plan.n_images, plan.chunk, plan.images_offset, plan.table_offset};
  std::memcpy(host.data(), &hdr, sizeof(hdr));
  auto *imgs = reinterpret_cast<dct::BatchImage *>(host.data() + plan.images_offset);
  auto *table = reinterpret_cast<int32_t *>(host.data() + plan.table_offset);
  int64_t next = 0;
  for (int32_t k = 0; k < n_images; ++k) {
    const dct_image &im = images[k];
    dct::BatchImage &d = imgs[k];
    d.src = im.src;
    d.dst = im.dst;
    d.W = im.W;
    d.H = im.H;
    d.src_stride = im.src_stride;
    d.dst_stride = im.dst_stride;
    d.bw = (im.W + 7) / 8;
    d.nblocks = d.bw * ((im.H + 7) / 8);
    d.first_chunk = next;
    d.qa = codec_quant(im.qs, dct::kFrac, dct::kFrac);
    const int64_t c = (d.nblocks + chunk - 1) / chunk;
    for (int64_t j = 0; j < c; ++j) table[next + j] = k;
    next += c;
  }
  hipStream_t s = as_stream(stream);
  if (hipMemcpyAsync(workspace, host.data(), bytes, hipMemcpyHostToDevice, s) != hipSuccess) return DCT_ERR_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return DCT_ERR_DEVICE;
  {
    std::lock_guard<std::mutex> guard(g_lock);
    g_batches[workspace] = plan;
  }
  if (total_chunks) *total_chunks = plan.total_chunks;
  return DCT_OK;
}

int dct_batch_run(const void *workspace, int32_t grid, uint64_t *sse_dev, void *stream) {
  if (workspace == nullptr || sse_dev == nullptr || !aligned(sse_dev, 8) || grid < 0) return DCT_ERR_INVALID;
  BatchPlan plan{};
  {
    std::lock_guard<std::mutex> guard(g_lock);
    auto it = g_batches.find(workspace);
    if (it == g_batches.end()) return DCT_ERR_INVALID;
    plan = it->second;
  }
  if (int st = check_device(nullptr)) return st;
  hipStream_t s = as_stream(stream);
  auto *acc = reinterpret_cast<unsigned long long *>(sse_dev);
  dct::fill_zero_kernel<<<grid_for(plan.n_images, 256), 256, 0, s>>>(acc, plan.n_images);
  if (launched()) return DCT_ERR_DEVICE;
  const auto *base = static_cast<const uint8_t *>(workspace);
  const auto *imgs = reinterpret_cast<const dct::BatchImage *>(base + plan.images_offset);
  const auto *table = reinterpret_cast<const int32_t *>(base + plan.table_offset);
  const unsigned g = static_cast<unsigned>(grid == 0 ? plan.total_chunks : std::min<int64_t>(grid, plan.total_chunks));
  if (plan.chunk == 512)
    dct::batch_codec_kernel<512><<<g, 512, 0, s>>>(imgs, table, plan.total_chunks, acc);
  else
    dct::batch_codec_kernel<256><<<g, 256, 0, s>>>(imgs, table, plan.total_chunks, acc);
  return launched();
}

int dct_batch_release(const void *workspace) {
  std::lock_guard<std::mutex> guard(g_lock);
  return g_batches.erase(workspace) ? DCT_OK : DCT_ERR_INVALID;
}

int32_t dct_deblock_nparam(void) { return dct::db::kNParam; }

size_t dct_deblock_workspace_size(int64_t npix, int32_t training) {
  if (npix < 1 || npix >= (int64_t{1} << 31)) return 0;
  const DeblockLayout L = deblock_layout(npix, training != 0);
  return L.bytes;
}

int dct_deblock_apply(const uint8_t *decoded, int32_t W, int32_t H, int32_t stride, const float *params,
                      uint8_t *out, int32_t out_stride, void *workspace, size_t workspace_bytes, void *stream) {
  if (!plane_ok(decoded, W, H, stride) || !plane_ok(out, W, H, out_stride) || params == nullptr ||
      !aligned(params, 4))
    return DCT_ERR_INVALID;
  const int64_t npix = static_cast<int64_t>(W) * H;
  const DeblockLayout L = deblock_layout(npix, false);
  if (npix >= (int64_t{1} << 31) || workspace == nullptr || !aligned(workspace, 256) || workspace_bytes < L.bytes)
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  dct::db::ImageSet set{decoded, nullptr, stride, W, H, nullptr, 1, H, W};
  return deblock_forward(set, npix, params, static_cast<uint8_t *>(workspace), L, out, out_stride, nullptr,
                         nullptr, nullptr, as_stream(stream));
}

int dct_deblock_forward(const uint8_t *decoded, int32_t plane_w, int32_t plane_h, int32_t stride, const int32_t *pos,
                        int32_t n, int32_t h, int32_t w, const float *params, float *y, void *workspace,
                        size_t workspace_bytes, void *stream) {
  if (!plane_ok(decoded, plane_w, plane_h, stride) || n < 1 || h < 1 || w < 1 || params == nullptr ||
      y == nullptr || !aligned(y, 4) || (pos == nullptr && n != 1))
    return DCT_ERR_INVALID;
  const int64_t npix = static_cast<int64_t>(n) * h * w;
  const DeblockLayout L = deblock_layout(npix, true);
  if (npix >= (int64_t{1} << 31) || workspace == nullptr || !aligned(workspace, 256) || workspace_bytes < L.bytes)
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  dct::db::ImageSet set{decoded, decoded, stride, plane_w, plane_h, pos, n, h, w};
  return deblock_forward(set, npix, params, static_cast<uint8_t *>(workspace), L, nullptr, 0, y, nullptr, nullptr,
                         as_stream(stream));
}

int dct_deblock_grad(const uint8_t *decoded, const uint8_t *original, int32_t plane_w, int32_t plane_h,
                     int32_t stride, const int32_t *pos, int32_t n, int32_t h, int32_t w, const float *params,
                     float *grad, double *loss, void *workspace, size_t workspace_bytes, void *stream) {
  if (!plane_ok(decoded, plane_w, plane_h, stride) || !plane_ok(original, plane_w, plane_h, stride) || n < 1 ||
      h < 1 || w < 1 || params == nullptr || grad == nullptr || !aligned(grad, 4) || loss == nullptr ||
      !aligned(loss, 8) || (pos == nullptr && n != 1))
    return DCT_ERR_INVALID;
  const int64_t npix = static_cast<int64_t>(n) * h * w;
  const DeblockLayout L = deblock_layout(npix, true);
  if (npix >= (int64_t{1} << 31) || workspace == nullptr || !aligned(workspace, 256) || workspace_bytes < L.bytes)
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  dct::db::ImageSet set{decoded, original, stride, plane_w, plane_h, pos, n, h, w};
  hipStream_t s = as_stream(stream);
  auto *ws = static_cast<uint8_t *>(workspace);
  int st = deblock_forward(set, npix, params, ws, L, nullptr, 0, nullptr, grad, loss, s);
  if (st) return st;
  return deblock_backward(set, npix, ws, L, grad, s);
}

int dct_deblock_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr, float beta1,
                     float beta2, float eps, void *stream) {
  if (params == nullptr || m == nullptr || v == nullptr || grad == nullptr || step < 1 || !(lr > 0.0f) ||
      !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  const float c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta1), step));
  const float c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta2), step));
  dct::db::adam_kernel<<<grid_for(dct::db::kNParam), dct::db::kThreads, 0, as_stream(stream)>>>(
      params, m, v, grad, dct::db::kNParam, lr, beta1, beta2, eps, c1, c2);
  return launched();
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
  std::lock_guard<std::mutex> guard(g_lock);
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

namespace {

int codec_common(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, const RecipeEntry &rc, int32_t qs,
                 uint8_t *dst, int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream) {
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
  dct::fill_zero_kernel<<<1, 64, 0, s>>>(a.sse, 1);
  if (launched()) return DCT_ERR_DEVICE;
  rc.launch(a, s);
  return launched();
}

}  // namespace

namespace {

// Workspace of the deblocking network: FP16-rounded weights (FP32 and FP16), the
// loss accumulator, three activation buffers (two for inference) and, for
// training, dL/dy and two FP32 gradient buffers.  Every part 256-byte aligned.
size_t align256(size_t v) { return (v + 255) / 256 * 256; }

DeblockLayout deblock_layout(int64_t npix, bool training) {
  DeblockLayout L{};
  size_t o = 0;
  L.wq = o;
  o += align256(sizeof(float) * dct::db::kNParam);
  L.wh = o;
  o += align256(sizeof(_Float16) * dct::db::kNParam);
  L.sq = o;
  o += 256;
  const size_t act = align256(sizeof(_Float16) * dct::db::kC * static_cast<size_t>(npix));
  L.a1 = o;
  o += act;
  L.a2 = o;
  o += act;
  L.a3 = training ? o : L.a1;  // inference writes the third activation over the first
  if (training) o += act;
  L.g4 = o;
  if (training) o += align256(sizeof(float) * static_cast<size_t>(npix));
  const size_t gsz = align256(sizeof(float) * dct::db::kC * static_cast<size_t>(npix));
  L.ga = o;
  if (training) o += gsz;
  L.gb = o;
  if (training) o += gsz;
  // per-workgroup partial weight gradients: at most kGradGroups workgroups x the largest layer
  L.part = o;
  if (training) o += align256(sizeof(float) * kGradGroups * (dct::db::kC * dct::db::kC * 9 + dct::db::kC));
  L.bytes = o;
  return L;
}

unsigned px_grid(int64_t npix) {
  return static_cast<unsigned>(std::min<int64_t>((npix + dct::db::kThreads - 1) / dct::db::kThreads, 1 << 16));
}

// Forward pass.  out != null: inference to the output plane.  Otherwise y (may be
// null) gets y; with grad != null the loss terms and dL/dy are formed too.
int deblock_forward(const dct::db::ImageSet &set, int64_t npix, const float *params, uint8_t *ws,
                    const DeblockLayout &L, uint8_t *out, int out_stride, float *y, float *grad, double *loss,
                    hipStream_t s) {
  using namespace dct::db;
  auto *wq = reinterpret_cast<float *>(ws + L.wq);
  auto *wh = reinterpret_cast<_Float16 *>(ws + L.wh);
  auto *sq = reinterpret_cast<double *>(ws + L.sq);
  auto *a1 = reinterpret_cast<_Float16 *>(ws + L.a1);
  auto *a2 = reinterpret_cast<_Float16 *>(ws + L.a2);
  auto *a3 = reinterpret_cast<_Float16 *>(ws + L.a3);
  auto *g4 = reinterpret_cast<float *>(ws + L.g4);
  prep_kernel<<<grid_for(kNParam), kThreads, 0, s>>>(params, wq, wh);
  // layer 1 and layer 4: one thread per kRows vertically adjacent pixels of a column
  const int64_t ngroups = static_cast<int64_t>(set.n) * ((set.h + kRows - 1) / kRows) * set.w;
  layer1_kernel<<<px_grid(ngroups), kThreads, 0, s>>>(set, wq, a1, ngroups);
  // tiles of kRows rows x 16 pixels of one image: ceil(h / kRows) x ceil(w / 16) per image
  const int64_t ntiles = static_cast<int64_t>(set.n) * ((set.h + kRows - 1) / kRows) * ((set.w + 15) / 16);
  const unsigned mgrid = static_cast<unsigned>(std::min<int64_t>((ntiles + 3) / 4, 8192));
  mid_kernel<<<mgrid, kThreads, 0, s>>>(set, a1, wh + kW2, wq + kB2, a2, npix, ntiles);
  mid_kernel<<<mgrid, kThreads, 0, s>>>(set, a2, wh + kW3, wq + kB3, a3, npix, ntiles);
  if (out != nullptr) {
    layer4_kernel<false><<<px_grid(ngroups), kThreads, 0, s>>>(set, a3, wq, ngroups, out, out_stride, nullptr,
                                                               nullptr, nullptr, 0.0f);
    return launched();
  }
  zero_f32_kernel<<<1, kThreads, 0, s>>>(reinterpret_cast<float *>(sq), 2);
  layer4_kernel<true><<<px_grid(ngroups), kThreads, 0, s>>>(set, a3, wq, ngroups, nullptr, 0, y, g4, sq,
                                                            2.0f / static_cast<float>(npix));
  if (grad != nullptr) mean_kernel<<<1, 64, 0, s>>>(sq, loss, 1.0 / static_cast<double>(npix));
  return launched();
}

// Backward pass after deblock_forward with grad: writes the gradient of the mean
// squared error with respect to all 19105 parameters into grad.
int deblock_backward(const dct::db::ImageSet &set, int64_t npix, uint8_t *ws, const DeblockLayout &L, float *grad,
                     hipStream_t s) {
  using namespace dct::db;
  auto *wq = reinterpret_cast<float *>(ws + L.wq);
  auto *a1 = reinterpret_cast<_Float16 *>(ws + L.a1);
  auto *a2 = reinterpret_cast<_Float16 *>(ws + L.a2);
  auto *a3 = reinterpret_cast<_Float16 *>(ws + L.a3);
  auto *g4 = reinterpret_cast<float *>(ws + L.g4);
  auto *ga = reinterpret_cast<float *>(ws + L.ga);
  auto *gb = reinterpret_cast<float *>(ws + L.gb);
  auto *part = reinterpret_cast<float *>(ws + L.part);
  // at least 64 pixels and at most kGradGroups workgroups per weight-gradient
  // pass, so the partials fit the workspace
  const int per_wg = static_cast<int>(std::max<int64_t>(64, (npix + kGradGroups - 1) / kGradGroups));
  const int wg = static_cast<int>((npix + per_wg - 1) / per_wg);
  const unsigned pg = px_grid(npix);
  auto reduce = [&](int nw, int nb, float *dW, float *db) {
    reduce_kernel<<<static_cast<unsigned>((nw + nb + 63) / 64), kThreads, 0, s>>>(part, wg, nw, nb, dW, db);
  };
  // layer 4
  wgrad_kernel<kC, 1><<<wg, kThreads, 0, s>>>(set, g4, a3, part, npix, per_wg);
  reduce(kC * 9, 1, grad + kW4, grad + kB4);
  bwd4_kernel<<<pg, kThreads, 0, s>>>(set, g4, a3, wq, ga, npix);
  // layer 3: ga = dL/d(pre-activation 3)
  wgrad_kernel<kC, kC><<<wg, kThreads, 0, s>>>(set, ga, a2, part, npix, per_wg);
  reduce(kC * kC * 9, kC, grad + kW3, grad + kB3);
  bwd_mid_kernel<<<pg, kThreads, 0, s>>>(set, ga, a2, wq + kW3, gb, npix);
  // layer 2
  wgrad_kernel<kC, kC><<<wg, kThreads, 0, s>>>(set, gb, a1, part, npix, per_wg);
  reduce(kC * kC * 9, kC, grad + kW2, grad + kB2);
  bwd_mid_kernel<<<pg, kThreads, 0, s>>>(set, gb, a1, wq + kW2, ga, npix);
  // layer 1
  wgrad_kernel<1, kC><<<wg, kThreads, 0, s>>>(set, ga, nullptr, part, npix, per_wg);
  reduce(kC * 9, kC, grad + kW1, grad + kB1);
  return launched();
}

}  // namespace
