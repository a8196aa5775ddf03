// api_batch.hip -- the batched fused codec of include/dctcodec.h: many images of
// uneven size and quality scale in one capturable launch.
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
#include "batch.hpp"

namespace {

using namespace dct::host;

// Batches planned into a workspace: the host keeps what a run needs to launch
// safely, so dct_batch_run never trusts sizes it is handed.
struct BatchPlan {
  int64_t total_chunks;
  int32_t n_images, chunk;
  int64_t images_offset, table_offset;
};
std::unordered_map<const void *, BatchPlan> g_batches;  // guarded by lock()

bool chunk_ok(int chunk) { return chunk == 256 || chunk == 512 || chunk == 1024 || chunk == 2048; }

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

}  // namespace

extern "C" {

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
    std::lock_guard<std::mutex> guard(lock());
    g_batches[workspace] = plan;
  }
  if (total_chunks) *total_chunks = plan.total_chunks;
  return DCT_OK;
}

int dct_batch_run_threads(const void *workspace, int32_t grid, int32_t threads, uint64_t *sse_dev, void *stream) {
  if (workspace == nullptr || sse_dev == nullptr || !aligned(sse_dev, 8) || grid < 0 ||
      (threads != 256 && threads != 512))
    return DCT_ERR_INVALID;
  BatchPlan plan{};
  {
    std::lock_guard<std::mutex> guard(lock());
    auto it = g_batches.find(workspace);
    if (it == g_batches.end()) return DCT_ERR_INVALID;
    plan = it->second;
  }
  if (threads > plan.chunk) return DCT_ERR_INVALID;
  if (int st = check_device(nullptr)) return st;
  hipStream_t s = as_stream(stream);
  auto *acc = reinterpret_cast<unsigned long long *>(sse_dev);
  dct::fill_zero_kernel<<<grid_for(plan.n_images, 256), 256, 0, s>>>(acc, plan.n_images);
  if (launched()) return DCT_ERR_DEVICE;
  const auto *base = static_cast<const uint8_t *>(workspace);
  const auto *imgs = reinterpret_cast<const dct::BatchImage *>(base + plan.images_offset);
  const auto *table = reinterpret_cast<const int32_t *>(base + plan.table_offset);
  const unsigned g = static_cast<unsigned>(grid == 0 ? plan.total_chunks : std::min<int64_t>(grid, plan.total_chunks));
  if (threads == 512)
    dct::batch_codec_kernel<512><<<g, 512, 0, s>>>(imgs, table, plan.total_chunks, plan.chunk, acc);
  else
    dct::batch_codec_kernel<256><<<g, 256, 0, s>>>(imgs, table, plan.total_chunks, plan.chunk, acc);
  return launched();
}

int dct_batch_run(const void *workspace, int32_t grid, uint64_t *sse_dev, void *stream) {
  if (workspace == nullptr) return DCT_ERR_INVALID;
  int32_t chunk = 0;
  {
    std::lock_guard<std::mutex> guard(lock());
    auto it = g_batches.find(workspace);
    if (it == g_batches.end()) return DCT_ERR_INVALID;
    chunk = it->second.chunk;
  }
  return dct_batch_run_threads(workspace, grid, std::min(chunk, 512), sse_dev, stream);
}

int dct_batch_release(const void *workspace) {
  std::lock_guard<std::mutex> guard(lock());
  return g_batches.erase(workspace) ? DCT_OK : DCT_ERR_INVALID;
}

}  // extern "C"
