// kernels.hpp -- gfx950 kernels of the blockwise Cordic-based Loeffler DCT codec.
//
// Mapping.  The transform kernels give each lane one whole 8x8 block and keep
// its 64 samples in VGPRs through both passes: the row-to-column transpose is a
// change of register index, not a data movement, so these kernels need no LDS,
// no barriers and no cross-lane shuffles, and every VALU instruction does useful
// work on all 64 lanes.  Consecutive lanes own horizontally consecutive blocks,
// so the wave's load of one block row is one 8-byte access per lane over 512
// contiguous bytes (fully coalesced), and likewise for the reconstruction
// stores.  The codec is VALU-bound (about a hundred int32 operations per pixel
// against two bytes of HBM traffic), so these choices aim at instruction count.
//
// Steps (Sec. 2.5.2 transform, Sec. 3.2 quantizer, Sec. 4.1 PSNR):
//   a1 load + level shift, a2 row pass, a3 transpose (register renaming),
//   a4 column pass, a5 quantize, a6 dequantize, a7 inverse column and row pass,
//   a8 reconstruct, a9 SSE.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "transform.hpp"

namespace dct {

inline constexpr int kWg = 256;  // threads per workgroup (four waves)

// Quantizer constants of one table Q[u][v] = 1 + (1 + u + v) qs, indexed by
// s = u + v (0..14).  They are wave-uniform in the lane-per-block kernels, so
// they live in SGPRs.
struct QuantArgs {
  int32_t Q[15];       // table entry
  int32_t half[15];    // Q << (F + 2): the rounding offset of the quantizer
  uint32_t magic[15];  // ceil(2^shift / Q): floor(m / Q) = (m magic) >> shift for m < 2^14
  int32_t shift[15];   // 14 + ceil(log2 Q)
};

// ---------------------------------------------------------------------------
// a1: load one block (lane-per-block), with edge replication
// ---------------------------------------------------------------------------

// Packed source pixels of the lane's block: word 2r holds pixels 0..3 of row r,
// word 2r+1 pixels 4..7 (little-endian bytes).  Rows past H repeat row H-1 and
// columns past W repeat column W-1; no byte outside the W x H region is read.
// The full-width case (every block but the last of a block row when W is not a
// multiple of 8) is one branch around eight independent 8-byte loads, so they
// are all in flight together.
__device__ __forceinline__ void load_block(const uint8_t *__restrict__ src, int W, int H, int stride,
                                           int by, int bx, uint32_t (&pix)[16]) {
  const int x0 = bx * 8;
  if (x0 + 8 <= W) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int y = min(by * 8 + r, H - 1);
      const uint2 w = *reinterpret_cast<const uint2 *>(src + static_cast<size_t>(y) * stride + x0);
      pix[2 * r] = w.x;
      pix[2 * r + 1] = w.y;
    }
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint8_t *row = src + static_cast<size_t>(min(by * 8 + r, H - 1)) * stride;
      uint32_t lo = 0, hi = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        lo |= static_cast<uint32_t>(row[min(x0 + j, W - 1)]) << (8 * j);
        hi |= static_cast<uint32_t>(row[min(x0 + 4 + j, W - 1)]) << (8 * j);
      }
      pix[2 * r] = lo;
      pix[2 * r + 1] = hi;
    }
  }
}

// x = (p - 128) << F for every pixel of the block
__device__ __forceinline__ void level_shift(const uint32_t (&pix)[16], int (&x)[64]) {
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int p = static_cast<int>((pix[2 * r + (j >> 2)] >> (8 * (j & 3))) & 0xffu);
      x[r * 8 + j] = (p - 128) * (1 << kFrac);
    }
}

// ---------------------------------------------------------------------------
// a5 + a6: quantize and dequantize one coefficient whose table slot is uniform
// ---------------------------------------------------------------------------

// q = sgn(c) floor((|c| + Q 2^(F+2)) / (Q 2^(F+3))), then d = clamp(q Q, -2048, 2047) << F.
// Valid for |c| < 2^(F+3) (2^14 - Q/2), which every coefficient of a uint8 block meets.
__device__ __forceinline__ int quant_dequant(int c, int32_t Q, int32_t half, uint32_t magic,
                                             int32_t shift, int &q_out) {
  const int sgn = c >> 31;  // 0 or -1
  const uint32_t a = static_cast<uint32_t>((c ^ sgn) - sgn);
  const uint32_t m = (a + static_cast<uint32_t>(half)) >> (kFrac + 3);
  const uint32_t q = __umul24(m, magic) >> shift;
  q_out = (static_cast<int>(q) ^ sgn) - sgn;
  int d = static_cast<int>(__umul24(q, static_cast<uint32_t>(Q)));
  d = min(d, 2047 - sgn);  // magnitude bound 2047 for positive, 2048 for negative values
  d = (d ^ sgn) - sgn;
  return d * (1 << kFrac);
}

// q for any int32 coefficient and any table entry (per-lane Q): exact floor
// division by a reciprocal estimate and one correction step, int16 saturation.
__device__ __forceinline__ int quantize_any(int c, int32_t Q) {
  const int sgn = c >> 31;
  const uint32_t a = static_cast<uint32_t>(c ^ sgn) - static_cast<uint32_t>(sgn);  // |c| <= 2^31
  const uint32_t m = (a + (static_cast<uint32_t>(Q) << (kFrac + 2))) >> (kFrac + 3);  // < 2^17
  const float rq = __builtin_amdgcn_rcpf(static_cast<float>(Q));
  uint32_t q = static_cast<uint32_t>(static_cast<float>(m) * rq);
  const int r = static_cast<int>(m) - static_cast<int>(q * static_cast<uint32_t>(Q));
  if (r < 0)
    q -= 1;
  else if (r >= Q)
    q += 1;
  q = min(q, 32767u - static_cast<uint32_t>(sgn));  // 32767 for positive, 32768 for negative
  return (static_cast<int>(q) ^ sgn) - sgn;
}

// ---------------------------------------------------------------------------
// a8: reconstruction
// ---------------------------------------------------------------------------

// p = clamp(((x + 2^(F+2)) >> (F+3)) + 128, 0, 255)
__device__ __forceinline__ uint32_t reconstruct(int x) {
  const int p = ((x + (1 << (kFrac + 2))) >> (kFrac + 3)) + 128;
  return static_cast<uint32_t>(min(max(p, 0), 255));
}

// Pack the reconstruction of the block into 16 words like load_block.
__device__ __forceinline__ void pack_block(const int (&x)[64], uint32_t (&rec)[16]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      lo |= reconstruct(x[r * 8 + j]) << (8 * j);
      hi |= reconstruct(x[r * 8 + 4 + j]) << (8 * j);
    }
    rec[2 * r] = lo;
    rec[2 * r + 1] = hi;
  }
}

// Store the W x H part of a packed block (one branch for the full-width case).
__device__ __forceinline__ void store_block(uint8_t *__restrict__ dst, int W, int H, int stride,
                                            int by, int bx, const uint32_t (&rec)[16]) {
  const int x0 = bx * 8;
  if (x0 + 8 <= W && by * 8 + 8 <= H) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
      *reinterpret_cast<uint2 *>(dst + static_cast<size_t>(by * 8 + r) * stride + x0) =
          make_uint2(rec[2 * r], rec[2 * r + 1]);
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int y = by * 8 + r;
      if (y < H) {
        uint8_t *row = dst + static_cast<size_t>(y) * stride;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (x0 + j < W) row[x0 + j] = static_cast<uint8_t>(rec[2 * r + (j >> 2)] >> (8 * (j & 3)));
      }
    }
  }
}

// a9: sum of squared differences of the W x H part of the block.  Bytes of
// pixels outside the image are masked to zero in both operands, and the sum is
// taken as sum(p^2) - 2 sum(p r) + sum(r^2) with packed unsigned dot products,
// exact in 32 bits (at most 64 * 255^2 per term).
__device__ __forceinline__ uint32_t block_sse(const uint32_t (&pix)[16], const uint32_t (&rec)[16], int W,
                                              int H, int by, int bx) {
  const int x0 = bx * 8;
  const int cols = min(W - x0, 8);
  const uint32_t mlo = cols >= 4 ? 0xffffffffu : (0xffffffffu >> (8 * (4 - cols)));
  const uint32_t mhi = cols >= 8 ? 0xffffffffu : (cols <= 4 ? 0u : (0xffffffffu >> (8 * (8 - cols))));
  uint32_t pp = 0, pr = 0, rr = 0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const bool in = by * 8 + r < H;
    const uint32_t a0 = in ? pix[2 * r] & mlo : 0u, a1 = in ? pix[2 * r + 1] & mhi : 0u;
    const uint32_t b0 = in ? rec[2 * r] & mlo : 0u, b1 = in ? rec[2 * r + 1] & mhi : 0u;
    pp = __builtin_amdgcn_udot4(a0, a0, pp, false);
    pp = __builtin_amdgcn_udot4(a1, a1, pp, false);
    pr = __builtin_amdgcn_udot4(a0, b0, pr, false);
    pr = __builtin_amdgcn_udot4(a1, b1, pr, false);
    rr = __builtin_amdgcn_udot4(b0, b0, rr, false);
    rr = __builtin_amdgcn_udot4(b1, b1, rr, false);
  }
  return pp - 2u * pr + rr;
}

// Sum of v over the workgroup, then one 64-bit atomic add to *acc.
__device__ __forceinline__ void workgroup_add(uint64_t v, unsigned long long *acc) {
  __shared__ unsigned long long partial[kWg / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) partial[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kWg / 64; ++w) t += partial[w];
    if (t) atomicAdd(acc, t);
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Zero n 64-bit words (a fill kernel, so the library enqueues no memset).
__global__ void fill_zero_kernel(unsigned long long *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// a1..a4: one lane per block; writes 64 int32 coefficients per block.
__global__ __launch_bounds__(kWg) void forward_kernel(const uint8_t *__restrict__ src, int W, int H,
                                                      int stride, int bw, int nblocks,
                                                      int32_t *__restrict__ coef) {
  const int b = blockIdx.x * kWg + threadIdx.x;
  if (b >= nblocks) return;
  const int by = b / bw, bx = b - by * bw;
  uint32_t pix[16];
  int x[64];
  load_block(src, W, H, stride, by, bx, pix);
  level_shift(pix, x);
  forward_block(x);
  int4 *out = reinterpret_cast<int4 *>(coef + static_cast<size_t>(b) * 64);
#pragma unroll
  for (int k = 0; k < 16; ++k) out[k] = make_int4(x[4 * k], x[4 * k + 1], x[4 * k + 2], x[4 * k + 3]);
}

// a5: one thread per block row (8 coefficients); any int32 input.
__global__ __launch_bounds__(kWg) void quantize_kernel(const int32_t *__restrict__ coef, int64_t nrows,
                                                       int qs, int16_t *__restrict__ qcoef) {
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
__global__ __launch_bounds__(kWg) void inverse_kernel(const int16_t *__restrict__ qcoef, QuantArgs qa,
                                                      int W, int H, int bw, int nblocks,
                                                      uint8_t *__restrict__ dst, int stride) {
  const int b = blockIdx.x * kWg + threadIdx.x;
  if (b >= nblocks) return;
  const int by = b / bw, bx = b - by * bw;
  int x[64];
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
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int d = __mul24(x[u * 8 + v], qa.Q[u + v]);
      x[u * 8 + v] = min(max(d, -2048), 2047) * (1 << kFrac);
    }
  inverse_block(x);
  uint32_t rec[16];
  pack_block(x, rec);
  store_block(dst, W, H, stride, by, bx, rec);
}

// a1..a9 fused: one lane per block, only pixels (and optionally the int16
// quantized values) touch memory; the SSE goes to *sse by one atomic per
// workgroup.
template <bool kEmitQ>
__global__ __launch_bounds__(kWg) void codec_kernel(const uint8_t *__restrict__ src, int W, int H,
                                                    int src_stride, int bw, int nblocks, QuantArgs qa,
                                                    uint8_t *__restrict__ dst, int dst_stride,
                                                    int16_t *__restrict__ qcoef,
                                                    unsigned long long *__restrict__ sse) {
  const int b = blockIdx.x * kWg + threadIdx.x;
  uint32_t err = 0;
  if (b < nblocks) {
    const int by = b / bw, bx = b - by * bw;
    uint32_t pix[16];
    int x[64];
    load_block(src, W, H, src_stride, by, bx, pix);
    level_shift(pix, x);
    forward_block(x);
    int q[64];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int s = u + v;
        x[u * 8 + v] = quant_dequant(x[u * 8 + v], qa.Q[s], qa.half[s], qa.magic[s], qa.shift[s], q[u * 8 + v]);
      }
    if constexpr (kEmitQ) {
      int4 *out = reinterpret_cast<int4 *>(qcoef + static_cast<size_t>(b) * 64);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        out[k] = make_int4((q[8 * k] & 0xffff) | (q[8 * k + 1] << 16), (q[8 * k + 2] & 0xffff) | (q[8 * k + 3] << 16),
                           (q[8 * k + 4] & 0xffff) | (q[8 * k + 5] << 16), (q[8 * k + 6] & 0xffff) | (q[8 * k + 7] << 16));
    }
    inverse_block(x);
    uint32_t rec[16];
    pack_block(x, rec);
    store_block(dst, W, H, dst_stride, by, bx, rec);
    err = block_sse(pix, rec, W, H, by, bx);
  }
  workgroup_add(err, sse);
}

// a9 standalone: SSE of b against a (and the largest pixel of a) over W x H.
// One thread per 8-pixel row segment, grid-stride.
__global__ __launch_bounds__(kWg) void sse_kernel(const uint8_t *__restrict__ a, int a_stride,
                                                  const uint8_t *__restrict__ b, int b_stride, int W, int H,
                                                  unsigned long long *__restrict__ acc) {
  const int segs = (W + 7) / 8;
  const int64_t total = static_cast<int64_t>(segs) * H;
  uint64_t sum = 0;
  uint32_t mx = 0;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kWg + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * kWg) {
    const int y = static_cast<int>(t / segs);
    const int x0 = static_cast<int>(t - static_cast<int64_t>(y) * segs) * 8;
    const uint8_t *ra = a + static_cast<size_t>(y) * a_stride + x0;
    const uint8_t *rb = b + static_cast<size_t>(y) * b_stride + x0;
    uint32_t a0, a1, b0, b1;
    if (x0 + 8 <= W) {
      const uint2 wa = *reinterpret_cast<const uint2 *>(ra);
      const uint2 wb = *reinterpret_cast<const uint2 *>(rb);
      a0 = wa.x; a1 = wa.y; b0 = wb.x; b1 = wb.y;
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
  workgroup_add(sum, acc);
  // largest pixel: reduce in the wave, one atomic per wave
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), off, 64)));
  if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned int *>(acc + 1), mx);
}

}  // namespace dct
