// staged.hpp -- the kernels of the staged entry points: the paper's separate
// DCT, quantizer and IDCT stages (Sec. 3.2) and the standalone PSNR reduction
// (Sec. 4.1, eq. (23)-(24)).  Included by one translation unit only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dct {

// a1..a4: one lane per block; writes 64 int32 coefficients per block.
__global__ __launch_bounds__(kBlockThreads) void forward_kernel(const uint8_t *__restrict__ src, int W, int H,
                                                                int stride, int bw, int nblocks,
                                                                int32_t *__restrict__ coef) {
  const int b = blockIdx.x * kBlockThreads + threadIdx.x;
  const BlockPos p = block_pos(b, W, H, bw, nblocks);
  uint32_t pix[16] = {};
  if (p.live) load_block(src, W, H, stride, p.by, p.bx, p.full, pix);
  int x[64];
  unpack_block<kFrac>(pix, x);
  barrier();
  forward_block<kIter, kFrac>(x);
  if (p.live) {
    int4 *out = reinterpret_cast<int4 *>(coef + static_cast<size_t>(b) * 64);
#pragma unroll
    for (int k = 0; k < 16; ++k) out[k] = make_int4(x[4 * k], x[4 * k + 1], x[4 * k + 2], x[4 * k + 3]);
  }
}

// a5: one thread per block row (8 coefficients); any int32 input.
__global__ __launch_bounds__(kWg) void quantize_kernel(const int32_t *__restrict__ coef, int64_t nrows, int qs,
                                                       int16_t *__restrict__ qcoef) {
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kWg + threadIdx.x; t < nrows;
       t += static_cast<int64_t>(gridDim.x) * kWg) {
    const int u = static_cast<int>(t & 7);
    const int4 *in = reinterpret_cast<const int4 *>(coef + t * 8);
    const int4 c0 = in[0], c1 = in[1];
    const int c[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
    int q[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) q[v] = quantize_any(c[v], 1 + (1 + u + v) * qs);
    int4 o;
    o.x = (q[0] & 0xffff) | (q[1] << 16);
    o.y = (q[2] & 0xffff) | (q[3] << 16);
    o.z = (q[4] & 0xffff) | (q[5] << 16);
    o.w = (q[6] & 0xffff) | (q[7] << 16);
    *reinterpret_cast<int4 *>(qcoef + t * 8) = o;
  }
}

// a6..a8: one lane per block; reads 64 int16, writes the W x H reconstruction.
__global__ __launch_bounds__(kBlockThreads) DCT_FOUR_WAVES void inverse_kernel(const int16_t *__restrict__ qcoef, DequantTable dq,
                                                                int W, int H, int bw, int nblocks,
                                                                uint8_t *__restrict__ dst, int stride) {
  const int b = blockIdx.x * kBlockThreads + threadIdx.x;
  const BlockPos p = block_pos(b, W, H, bw, nblocks);
  int x[64];
  if (p.live) {
    const int4 *in = reinterpret_cast<const int4 *>(qcoef + static_cast<size_t>(b) * 64);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int4 w = in[k];
      const int v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        x[8 * k + 2 * h] = static_cast<int16_t>(v[h] & 0xffff);
        x[8 * k + 2 * h + 1] = v[h] >> 16;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 64; ++k) x[k] = 0;
  }
  // a6: d = clamp(q Q, -2048, 2047) << F (any int16 input)
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int d = __mul24(x[u * 8 + v], dq.Q[u + v]);
      x[u * 8 + v] = min(max(d, -2048), 2047) * (1 << kFrac);
    }
  x[0] += kReconstructDC<kFrac>;
  barrier();
  inverse_block<kIter>(x);
  uint32_t rec[16];
  pack_block<kFrac>(x, rec);
  if (p.live) store_block(dst, W, H, stride, p.by, p.bx, p.full, rec);
}

// a9 standalone, first stage: SSE of b against a (and the largest pixel of a)
// over W x H.  One thread per 8-pixel row segment, strided over rows (grid.y)
// and segments (grid.x); workgroup w writes its sum and maximum to partial[2w]
// and partial[2w + 1] (no atomics: one address shared by thousands of
// workgroups serialises them).
__global__ __launch_bounds__(kWg) void sse_kernel(const uint8_t *__restrict__ a, int a_stride,
                                                  const uint8_t *__restrict__ b, int b_stride, int W, int H,
                                                  unsigned long long *__restrict__ partial) {
  const int segs = (W + 7) / 8;
  uint64_t sum = 0;
  uint32_t mx = 0;
  // rows across grid.y, the row's 8-byte segments across grid.x: 32-bit indices
  for (int y = blockIdx.y; y < H; y += gridDim.y)
  for (int sg = blockIdx.x * kWg + threadIdx.x; sg < segs; sg += gridDim.x * kWg) {
    const int x0 = sg * 8;
    const uint8_t *ra = a + static_cast<size_t>(y) * a_stride + x0;
    const uint8_t *rb = b + static_cast<size_t>(y) * b_stride + x0;
    uint32_t a0, a1, b0, b1;
    if (x0 + 8 <= W) {
      const uint2 wa = *reinterpret_cast<const uint2 *>(ra);
      const uint2 wb = *reinterpret_cast<const uint2 *>(rb);
      a0 = wa.x;
      a1 = wa.y;
      b0 = wb.x;
      b1 = wb.y;
    } else {
      a0 = a1 = b0 = b1 = 0;
      for (int j = 0; j < W - x0; ++j) {
        if (j < 4) {
          a0 |= static_cast<uint32_t>(ra[j]) << (8 * j);
          b0 |= static_cast<uint32_t>(rb[j]) << (8 * j);
        } else {
          a1 |= static_cast<uint32_t>(ra[j]) << (8 * (j - 4));
          b1 |= static_cast<uint32_t>(rb[j]) << (8 * (j - 4));
        }
      }
    }
    uint32_t s = __builtin_amdgcn_udot4(a0, a0, 0u, false);
    s = __builtin_amdgcn_udot4(a1, a1, s, false);
    s = __builtin_amdgcn_udot4(b0, b0, s, false);
    s = __builtin_amdgcn_udot4(b1, b1, s, false);
    uint32_t c = __builtin_amdgcn_udot4(a0, b0, 0u, false);
    c = __builtin_amdgcn_udot4(a1, b1, c, false);
    sum += s - 2u * c;
#pragma unroll
    for (int j = 0; j < 4; ++j) mx = max(mx, max((a0 >> (8 * j)) & 0xffu, (a1 >> (8 * j)) & 0xffu));
  }
  __shared__ unsigned long long wsum[kWg / 64];
  __shared__ uint32_t wmax[kWg / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_xor(sum, off, 64);
    mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), off, 64)));
  }
  if ((threadIdx.x & 63) == 0) {
    wsum[threadIdx.x >> 6] = sum;
    wmax[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    uint32_t m = 0;
#pragma unroll
    for (int w = 0; w < kWg / 64; ++w) {
      t += wsum[w];
      m = max(m, wmax[w]);
    }
    const unsigned wg = blockIdx.y * gridDim.x + blockIdx.x;
    partial[2 * wg] = t;
    partial[2 * wg + 1] = m;
  }
}

// a9 standalone, second stage (one workgroup): acc[0] = the sum of the n
// workgroups' sums, acc[1] = the largest of their maxima.
__global__ __launch_bounds__(kWg) void sse_reduce_kernel(const unsigned long long *__restrict__ partial, int n,
                                                         unsigned long long *__restrict__ acc) {
  unsigned long long sum = 0;
  unsigned long long mx = 0;
  for (int w = threadIdx.x; w < n; w += kWg) {
    sum += partial[2 * w];
    mx = max(mx, partial[2 * w + 1]);
  }
  __shared__ unsigned long long ssum[kWg], smax[kWg];
  ssum[threadIdx.x] = sum;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int h = kWg / 2; h > 0; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) {
      ssum[threadIdx.x] += ssum[threadIdx.x + h];
      smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    acc[0] = ssum[0];
    acc[1] = smax[0];
  }
}

}  // namespace dct
