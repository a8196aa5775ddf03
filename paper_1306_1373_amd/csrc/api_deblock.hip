// api_deblock.hip -- the learned deblocking post-filter of include/dctcodec.h:
// inference, training gradient and Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "dctcodec.h"
#include "host.hpp"
#include "deblock.hpp"

namespace {

using namespace dct::host;

// workgroups of a weight-gradient pass at most (each writes one partial row)
constexpr int kGradGroups = 2048;
// chunks (32 pixels of a row) per workgroup of the 32 -> 32 weight-gradient pass
// and of the layer 1 / layer 4 passes
constexpr int kMidChunks = 8;
constexpr int kEdgeChunks = 8;
// workgroups of the training output layer (each writes one partial loss sum)
constexpr int kLossGroups = 1024;

struct DeblockLayout {
  size_t wq, wh, ops, sq, a1, a2, a3, g4, ga, gb, part, bytes;
};
DeblockLayout deblock_layout(int64_t npix, bool training);
int deblock_forward(const dct::db::ImageSet &set, int64_t npix, const float *params, uint8_t *ws,
                    const DeblockLayout &L, uint8_t *out, int out_stride, float *y, float *grad, double *loss,
                    hipStream_t s);
int deblock_backward(const dct::db::ImageSet &set, int64_t npix, uint8_t *ws, const DeblockLayout &L, float *grad,
                     hipStream_t s);

}  // namespace

extern "C" {

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

int dct_deblock_apply_stack(const uint8_t *decoded, int32_t W, int32_t H, int32_t n, int32_t stride,
                            const float *params, uint8_t *out, int32_t out_stride, void *workspace,
                            size_t workspace_bytes, void *stream) {
  if (n < 1 || H < 1 || static_cast<int64_t>(n) * H > std::numeric_limits<int32_t>::max()) return DCT_ERR_INVALID;
  const int32_t rows = n * H;
  if (!plane_ok(decoded, W, rows, stride) || !plane_ok(out, W, rows, out_stride) || params == nullptr ||
      !aligned(params, 4))
    return DCT_ERR_INVALID;
  const int64_t npix = static_cast<int64_t>(W) * rows;
  const DeblockLayout L = deblock_layout(static_cast<int64_t>(W) * H, false);
  if (npix >= (int64_t{1} << 31) || workspace == nullptr || !aligned(workspace, 256) || workspace_bytes < L.bytes)
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  dct::db::ImageSet set{decoded, nullptr, stride, W, rows, nullptr, n, H, W};
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

int dct_deblock_init(uint64_t seed, float *params, void *stream) {
  if (params == nullptr || !aligned(params, 4)) return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  dct::db::init_kernel<<<grid_for(dct::db::kNParam, dct::db::kThreads), dct::db::kThreads, 0, as_stream(stream)>>>(
      params, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  return launched();
}

int dct_deblock_select(const uint64_t *sse_plain, const uint64_t *sse_filtered, int32_t n, float *params,
                       double *mean_gain_host, int32_t *kept_host, void *stream) {
  if (sse_plain == nullptr || sse_filtered == nullptr || n < 1 || n > (1 << 24) || params == nullptr ||
      !aligned(params, 4) || !aligned(sse_plain, 8) || !aligned(sse_filtered, 8))
    return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  hipStream_t s = as_stream(stream);
  std::vector<uint64_t> host(2 * static_cast<size_t>(n));
  if (hipMemcpyAsync(host.data(), sse_plain, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(host.data() + n, sse_filtered, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DCT_ERR_DEVICE;
  // The PSNR gain of image k, eq. (23) of the filtered output minus that of the
  // decoded one: the image's size and peak cancel, leaving 10 log10 of the ratio
  // of the two SSEs (+inf when the filter makes the image exact, 0 when both are).
  double sum = 0.0;
  for (int32_t k = 0; k < n; ++k) {
    const uint64_t a = host[k], b = host[n + k];
    if (b == 0)
      sum += a == 0 ? 0.0 : std::numeric_limits<double>::infinity();
    else if (a == 0)
      sum -= std::numeric_limits<double>::infinity();
    else
      sum += 10.0 * std::log10(static_cast<double>(a) / static_cast<double>(b));
  }
  const double mean = sum / n;  // NaN only if both infinities occur; then the filter is not kept
  const bool keep = mean > 0.0;
  if (!keep) {
    dct::db::zero_output_layer_kernel<<<grid_for(dct::db::kNParam - dct::db::kW4, dct::db::kThreads),
                                        dct::db::kThreads, 0, s>>>(params);
    if (launched()) return DCT_ERR_DEVICE;
  }
  if (mean_gain_host) *mean_gain_host = mean;
  if (kept_host) *kept_host = keep ? 1 : 0;
  return DCT_OK;
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

}  // extern "C"

namespace {

// Workspace of the deblocking network: FP16-rounded weights (FP32 and FP16), the
// loss partial sums, three activation buffers (two for inference) and, for
// training, the scaled FP16 dL/dy, two scaled FP16 backward-signal buffers and
// the partial weight-gradient rows.  Every part 256-byte aligned.
size_t align256(size_t v) { return (v + 255) / 256 * 256; }

DeblockLayout deblock_layout(int64_t npix, bool training) {
  DeblockLayout L{};
  size_t o = 0;
  L.wq = o;
  o += align256(sizeof(float) * dct::db::kNParam);
  L.wh = o;
  o += align256(sizeof(_Float16) * dct::db::kNParam);
  L.ops = o;
  if (!training) o += align256(sizeof(dct::db::WeightOps));
  L.sq = o;
  o += align256(sizeof(double) * kLossGroups);
  const size_t act = align256(sizeof(_Float16) * dct::db::kC * static_cast<size_t>(npix));
  // inference runs in one launch with its activations in LDS: only the weights
  L.a1 = o;
  if (training) o += act;
  L.a2 = o;
  if (training) o += act;
  L.a3 = o;
  if (training) o += act;
  L.g4 = o;
  if (training) o += align256(sizeof(_Float16) * static_cast<size_t>(npix));
  const size_t gsz = act;  // scaled FP16 backward signals, 32 channels
  L.ga = o;
  if (training) o += gsz;
  L.gb = o;
  if (training) o += gsz;
  // per-workgroup partial weight gradients: at most kGradGroups workgroups x the largest layer
  L.part = o;
  if (training) o += align256(sizeof(float) * kGradGroups * dct::db::kNWMid);
  L.bytes = o;
  return L;
}

// S = 2^(floor(log2 npix) + 8), the scale of the FP16 backward signals
float signal_scale(int64_t npix) {
  int e = 0;
  while ((int64_t{2} << e) <= npix) ++e;  // 2^e <= npix < 2^(e+1)
  return std::ldexp(1.0f, e + 8);
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
  auto *g4 = reinterpret_cast<_Float16 *>(ws + L.g4);
  if (out != nullptr) {
    // inference: the operands prepared once, then workgroups that each keep a
    // 28 x 28 output tile in LDS, one per CU, looping over the tiles
    constexpr int lds = kLdsA1 + kLdsA2 + kLdsX;
    static const hipError_t attr =
        hipFuncSetAttribute(reinterpret_cast<const void *>(&fused_apply_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (attr != hipSuccess) return DCT_ERR_DEVICE;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      return DCT_ERR_DEVICE;
    auto *ops = reinterpret_cast<WeightOps *>(ws + L.ops);
    prep_ops_kernel<<<grid_for(kPrepOpsThreads), kThreads, 0, s>>>(params, ops);
    // the n images of the set stacked vertically, set.h rows each
    const int64_t tiles = static_cast<int64_t>(set.n) * ((set.w + kTW - 1) / kTW) * ((set.h + kTH - 1) / kTH);
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>(tiles, cus));
    fused_apply_kernel<<<grid, kFThreads, lds, s>>>(set.plane, set.w, set.h, set.stride, set.n, ops, out,
                                                    out_stride);
    return launched();
  }
  prep_kernel<<<grid_for(kNParam), kThreads, 0, s>>>(params, wq, wh);
  // layers 1 to 3 in tiles of kRows rows x 16 pixels of one image, ceil(h / kRows) x ceil(w / 16) per
  // image; layer 4 in tiles of kRows rows x kL4Cols pixels
  const int64_t ntiles = static_cast<int64_t>(set.n) * ((set.h + kRows - 1) / kRows) * ((set.w + 15) / 16);
  const unsigned mgrid = static_cast<unsigned>(std::min<int64_t>((ntiles + 3) / 4, 8192));
  layer1_kernel<<<mgrid, kThreads, 0, s>>>(set, wq, wh, a1, ntiles);
  mid_kernel<false><<<mgrid, kThreads, 0, s>>>(set, a1, wh + kW2, wq + kB2, nullptr, a2, npix, ntiles);
  mid_kernel<false><<<mgrid, kThreads, 0, s>>>(set, a2, wh + kW3, wq + kB3, nullptr, a3, npix, ntiles);
  const int64_t ntiles4 =
      static_cast<int64_t>(set.n) * ((set.h + kRows - 1) / kRows) * ((set.w + kL4Cols - 1) / kL4Cols);
  const unsigned lgrid = static_cast<unsigned>(std::min<int64_t>((ntiles4 + 3) / 4, kLossGroups));
  layer4_kernel<<<lgrid, kThreads, 0, s>>>(set, a3, wq, wh, ntiles4, y, g4, sq, 2.0f / static_cast<float>(npix),
                                          signal_scale(npix));
  if (grad != nullptr) loss_reduce_kernel<<<1, kThreads, 0, s>>>(sq, static_cast<int>(lgrid), loss,
                                                                 1.0 / static_cast<double>(npix));
  return launched();
}

// Backward pass after deblock_forward with grad: writes the gradient of the mean
// squared error with respect to all 19105 parameters into grad.
int deblock_backward(const dct::db::ImageSet &set, int64_t npix, uint8_t *ws, const DeblockLayout &L, float *grad,
                     hipStream_t s) {
  using namespace dct::db;
  auto *wq = reinterpret_cast<float *>(ws + L.wq);
  auto *wh = reinterpret_cast<_Float16 *>(ws + L.wh);
  auto *a1 = reinterpret_cast<_Float16 *>(ws + L.a1);
  auto *a2 = reinterpret_cast<_Float16 *>(ws + L.a2);
  auto *a3 = reinterpret_cast<_Float16 *>(ws + L.a3);
  auto *g4 = reinterpret_cast<_Float16 *>(ws + L.g4);
  auto *ga = reinterpret_cast<_Float16 *>(ws + L.ga);
  auto *gb = reinterpret_cast<_Float16 *>(ws + L.gb);
  auto *part = reinterpret_cast<float *>(ws + L.part);
  const float inv_s = 1.0f / signal_scale(npix);  // exact: a power of two
  // chunks of 32 pixels of one image row; each pass's workgroups take a fixed
  // number of them, at most kGradGroups workgroups (the partial rows' room)
  const uint32_t nchunks = static_cast<uint32_t>(static_cast<int64_t>(set.n) * set.h * ((set.w + 31) / 32));
  auto per_group = [&](uint32_t want) {
    return std::max<uint32_t>(want, (nchunks + kGradGroups - 1) / kGradGroups);
  };
  const uint32_t cpw_mid = per_group(kMidChunks), cpw_edge = per_group(kEdgeChunks);
  const unsigned wg_mid = (nchunks + cpw_mid - 1) / cpw_mid, wg_edge = (nchunks + cpw_edge - 1) / cpw_edge;
  auto reduce = [&](bool mid_rows, unsigned nwg, int nw, int nb, float *dW, float *db, float wscale) {
    const unsigned grid = static_cast<unsigned>((nw + nb + 63) / 64);
    if (mid_rows)
      reduce_kernel<true><<<grid, 64 * kRedWaves, 0, s>>>(part, static_cast<int>(nwg), nw, nb, dW, db, wscale,
                                                          inv_s);
    else
      reduce_kernel<false><<<grid, 64 * kRedWaves, 0, s>>>(part, static_cast<int>(nwg), nw, nb, dW, db, wscale,
                                                           inv_s);
  };
  const int64_t ntiles = static_cast<int64_t>(set.n) * ((set.h + kRows - 1) / kRows) * ((set.w + 15) / 16);
  const unsigned mgrid = static_cast<unsigned>(std::min<int64_t>((ntiles + 3) / 4, 8192));
  // layer 4
  wgrad_edge_kernel<false><<<wg_edge, kEdgeGradThreads, 0, s>>>(set, a3, g4, part, nchunks, cpw_edge);
  reduce(false, wg_edge, kC * 9, 1, grad + kW4, grad + kB4, inv_s);
  bwd4_kernel<<<px_grid(npix), kThreads, 0, s>>>(set, g4, a3, wq, ga, npix);
  // layer 3: ga = S dL/d(pre-activation 3)
  wgrad_mid_kernel<<<wg_mid, kMidGradThreads, 0, s>>>(set, ga, a2, part, nchunks, cpw_mid);
  reduce(true, wg_mid, kC * kC * 9, kC, grad + kW3, grad + kB3, inv_s);
  mid_kernel<true><<<mgrid, kThreads, 0, s>>>(set, ga, wh + kW3, nullptr, a2, gb, npix, ntiles);
  // layer 2
  wgrad_mid_kernel<<<wg_mid, kMidGradThreads, 0, s>>>(set, gb, a1, part, nchunks, cpw_mid);
  reduce(true, wg_mid, kC * kC * 9, kC, grad + kW2, grad + kB2, inv_s);
  mid_kernel<true><<<mgrid, kThreads, 0, s>>>(set, gb, wh + kW2, nullptr, a1, ga, npix, ntiles);
  // layer 1: the pixel values' 1/255 joins the scale of the weight gradients
  wgrad_edge_kernel<true><<<wg_edge, kEdgeGradThreads, 0, s>>>(set, ga, nullptr, part, nchunks, cpw_edge);
  reduce(false, wg_edge, kC * 9, kC, grad + kW1, grad + kB1, inv_s * kInv255);
  return launched();
}

}  // namespace
