// batch.hpp -- the fused codec over a batch of images of uneven size in one launch.
//
// Each image's blocks are split into chunks of `chunk` consecutive blocks (the
// last chunk of an image padded with dead lanes), so a chunk, and the
// workgroup that codes it, belongs to one image: the image's quantizer table
// stays workgroup-uniform, exactly as in the single-image kernel, and every
// block is coded by the same device function.  A workgroup of kThreads lanes
// (one block per lane) codes a chunk in chunk / kThreads passes.  A table maps
// each chunk to its image; workgroups walk the chunks with a fixed stride (a
// persistent grid when the launch has fewer workgroups than chunks).  Each
// workgroup adds its SSE to its image's slot with one atomic per chunk.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dct {

// One image of a batch, as the kernel reads it (built by the host).
struct alignas(16) BatchImage {
  const uint8_t *src;
  uint8_t *dst;
  int32_t W, H, src_stride, dst_stride;
  int32_t bw, nblocks;
  int64_t first_chunk;  // index of the image's first chunk
  CodecQuant qa;        // quantizer of the image's qs (default recipe)
};

// Layout of the batch workspace: a header, the images, then the chunk table.
struct BatchHeader {
  int64_t total_chunks;
  int32_t n_images;
  int32_t chunk;  // blocks per chunk
  int64_t images_offset, table_offset;  // bytes from the workspace start
};

template <int kThreads>
__global__ __launch_bounds__(kThreads) DCT_FOUR_WAVES void batch_codec_kernel(const BatchImage *__restrict__ images,
                                                              const int32_t *__restrict__ chunk_image,
                                                              int64_t total_chunks, int chunk,
                                                              unsigned long long *__restrict__ sse) {
  const int wave = wave_index();
  for (int64_t c = blockIdx.x; c < total_chunks; c += gridDim.x) {
    const int im = __builtin_amdgcn_readfirstlane(chunk_image[c]);
    const BatchImage &d = images[im];
    const int chunk_base = static_cast<int>(c - d.first_chunk) * chunk;
    uint32_t err = 0;
    for (int pass = 0; pass < chunk; pass += kThreads)
      err += codec_block<DefaultRecipe, false>(d.src, d.W, d.H, d.src_stride, d.bw, d.nblocks,
                                               chunk_base + pass + wave * 64, d.qa, d.dst, d.dst_stride, nullptr);
    workgroup_add<kThreads>(err, sse + im, wave);
  }
}

}  // namespace dct
