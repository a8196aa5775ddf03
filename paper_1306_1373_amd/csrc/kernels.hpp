// kernels.hpp -- gfx950 kernels of the blockwise Cordic-based Loeffler DCT codec.
//
// Mapping.  The transform kernels give each lane one whole 8x8 block and keep
// its 64 samples in VGPRs through both passes: the row-to-column transpose is
// a change of register index, not a data movement, so no LDS or cross-lane
// traffic is needed for it.  Consecutive lanes own horizontally consecutive
// blocks, so a wave's load of one block row is one 8-byte access per lane over
// 512 contiguous bytes, and likewise for the reconstruction stores.
//
// Issue.  The codec is bound by VALU issue (about a hundred int32 operations
// per pixel against two bytes of HBM traffic).  gfx950 issues two plain 32-bit
// VALU instructions per SIMD per cycle pair when two waves on that SIMD are at
// the same instruction, so the kernels are written for waves in lockstep:
// large workgroups (kBlockThreads), a workgroup barrier between phases, and
// passes whose plain add/sub/shift runs are separated from the 64-bit
// multiply-adds (transform.hpp).
//
// Steps (Sec. 2.5.2 transform, Sec. 3.2 quantizer and IDCT, Sec. 4.1 PSNR):
//   a1 load + level shift, a2 row pass, a3 transpose (register renaming),
//   a4 column pass, a5 quantize, a6 dequantize, a7 inverse column and row pass,
//   a8 reconstruct, a9 SSE.
//
// Exact rewrites used (each gives the same bits as the recipe as written):
//   * The level shift x = (p - 128) 2^F only changes the DC coefficient: in the
//     graph a constant added to all eight inputs reaches Z0 alone, through
//     butterflies only.  The kernels transform p 2^F and subtract
//     64 * 128 * 2^F = 2^(F+13) from the DC coefficient.
//   * Likewise the reconstruction's + 2^(G+2) rounding and + 128 level shift,
//     added to every output, equal adding 2^(G+2) + 2^(G+10) to the
//     dequantized DC coefficient before the inverse.
//   * The fused kernel's quantizer forms m = (|c| + Q 2^(F+2)) >> (F+3) as
//     ((|c| >> s) + Q 2^(F+2-s)) >> (F+3-s) with s = max(F - 12, 0), equal
//     because Q 2^(F+2) is a multiple of 2^s, and which keeps the sum inside
//     32 bits; it divides m (< 2^14) by Q as trunc(float(m) * r) with r the
//     smallest float >= 1/Q, exact for every table entry and m (checked
//     exhaustively on the CPU); it omits the dequantization clamp, which no
//     coefficient of a uint8 block can reach (|qQ| <= 2041; also checked).
//
// The staged kernels run the default recipe R(10, 12, 12); the fused codec
// kernel is instantiated for each recipe R(n, F, G) the library offers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "transform.hpp"

namespace dct {

inline constexpr int kBlockThreads = 256;  // workgroup of the transform kernels (4 waves)
inline constexpr int kWg = 256;            // workgroup of the elementwise kernels

// Quantizer of the fused codec, indexed by s = u + v (0..14), wave-uniform (SGPRs).
struct CodecQuant {
  float rcp[15];     // smallest float >= 1/Q
  float qscale[15];  // Q 2^G (exact in float)
  int32_t half[15];  // Q 2^(F+2-s), the quantizer's rounding offset after the pre-shift s
};

// pre-shift of the fused quantizer: s = max(F - 12, 0)
template <int F>
inline constexpr int kQuantPreShift = F > 12 ? F - 12 : 0;

// Dequantizer of the staged inverse: the table entries Q, indexed by s = u + v.
struct DequantTable {
  int32_t Q[15];
};

__device__ __forceinline__ void barrier() { __syncthreads(); }

// Cap a transform kernel at 128 VGPRs, four waves per SIMD.  With 256-thread
// workgroups in lockstep that occupancy is worth more than the few values (a
// few dozen bytes per lane) the compiler then keeps in scratch: measured on the
// fused codec, 5% faster than the spill-free build at three waves, and faster
// also than a spill-free build at four waves whose phases were pinned apart.
#define DCT_FOUR_WAVES __attribute__((amdgpu_waves_per_eu(4)))

// ---------------------------------------------------------------------------
// a1: load one block (lane-per-block)
// ---------------------------------------------------------------------------

// Packed source pixels of the lane's block: word 2r holds pixels 0..3 of row r,
// word 2r+1 pixels 4..7 (little-endian).  A full block (inside W x H) is eight
// 8-byte loads at 32-bit offsets from the plane base; an edge block repeats the
// last row / column for positions past H / W and reads byte by byte.  No byte
// outside the W x H region is read.
__device__ __forceinline__ void load_block(const uint8_t *__restrict__ src, int W, int H, int stride,
                                           int by, int bx, bool full, uint32_t (&pix)[16]) {
  const int x0 = bx * 8, y0 = by * 8;
  if (full) {
    const uint32_t off = static_cast<uint32_t>(y0) * static_cast<uint32_t>(stride) + static_cast<uint32_t>(x0);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint2 w = *reinterpret_cast<const uint2 *>(src + (off + static_cast<uint32_t>(r * stride)));
      pix[2 * r] = w.x;
      pix[2 * r + 1] = w.y;
    }
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint8_t *row = src + static_cast<size_t>(min(y0 + r, H - 1)) * stride;
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

// x = p 2^F for every pixel (the level shift is applied on DC afterwards)
template <int F>
__device__ __forceinline__ void unpack_block(const uint32_t (&pix)[16], int (&x)[64]) {
  static_assert(F >= 8 && F <= 16, "byte lanes are shifted into place");
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint32_t w = pix[k];
    x[4 * k + 0] = static_cast<int>((w << F) & (0xffu << F));
    x[4 * k + 1] = static_cast<int>((w << (F - 8)) & (0xffu << F));
    x[4 * k + 2] = static_cast<int>((w >> (16 - F)) & (0xffu << F));
    x[4 * k + 3] = static_cast<int>((w >> (24 - F)) & (0xffu << F));
  }
}

template <int F>
inline constexpr int kLevelShiftDC = 64 * 128 * (1 << F);  // 2^(F+13)
template <int G>
inline constexpr int kReconstructDC = (1 << (G + 2)) + (128 << (G + 3));  // 2^(G+2) + 2^(G+10)

// a1..a4 on a register block: transform of p 2^F, then the level shift on DC
template <int N, int F>
__device__ __forceinline__ void forward_block(int (&x)[64]) {
  forward_pass<N, true>(x);
  barrier();
  forward_pass<N, false>(x);
  x[0] -= kLevelShiftDC<F>;
}

// a7 on a register block of dequantized values d 2^G; the caller has already
// added kReconstructDC<G> to the DC value
template <int N>
__device__ __forceinline__ void inverse_block(int (&x)[64]) {
  inverse_pass<N, false>(x);
  barrier();
  inverse_pass<N, true>(x);
}

// ---------------------------------------------------------------------------
// a5 + a6: quantize and dequantize
// ---------------------------------------------------------------------------

// Fused-codec quantizer for a coefficient c of a uint8 block in table slot s:
// returns the dequantized value d 2^G and, through q_out, q itself.
//
// Every step but the truncation is a plain 32-bit instruction, which gfx950 can
// pair: |c| by xor and subtract of the sign word; the float of m < 2^14 by
// setting it into the mantissa of 2^23 and subtracting 2^23; the integer of
// the dequantized q Q 2^G <= 2^23 (the clamp lemma: |q Q| <= 2048) by adding
// 2^23 and subtracting the bits of 2^23.  Each of these is exact.
template <int F>
__device__ __forceinline__ int quant_dequant(int c, float rcp, float qscale, int32_t half, int &q_out) {
  constexpr int s = kQuantPreShift<F>;
  constexpr uint32_t kTwo23Bits = 0x4B000000u;  // the bits of 2^23
  constexpr float kTwo23 = 8388608.0f;
  const int sgn = c >> 31;
  const int a = ((c ^ sgn) - sgn) >> s;
  const uint32_t m = static_cast<uint32_t>(a + half) >> (F + 3 - s);
  const float mf = __builtin_bit_cast(float, m | kTwo23Bits) - kTwo23;
  const float qf = __builtin_truncf(mf * rcp);
  const int d = static_cast<int>(__builtin_bit_cast(uint32_t, qf * qscale + kTwo23) - kTwo23Bits);
  const int q = static_cast<int>(__builtin_bit_cast(uint32_t, qf + kTwo23) - kTwo23Bits);
  q_out = (q ^ sgn) - sgn;
  return (d ^ sgn) - sgn;
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
// a8: reconstruction, packing, storing
// ---------------------------------------------------------------------------

// p = clamp(x >> (G+3), 0, 255) for x that already carries the rounding and +128
template <int G>
__device__ __forceinline__ void pack_block(const int (&x)[64], uint32_t (&rec)[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    uint32_t w = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      w |= static_cast<uint32_t>(min(max(x[4 * k + j] >> (G + 3), 0), 255)) << (8 * j);
    rec[k] = w;
  }
}

// Store the W x H part of a packed block.
__device__ __forceinline__ void store_block(uint8_t *__restrict__ dst, int W, int H, int stride, int by,
                                            int bx, bool full, const uint32_t (&rec)[16]) {
  const int x0 = bx * 8, y0 = by * 8;
  if (full) {
    const uint32_t off = static_cast<uint32_t>(y0) * static_cast<uint32_t>(stride) + static_cast<uint32_t>(x0);
#pragma unroll
    for (int r = 0; r < 8; ++r)
      *reinterpret_cast<uint2 *>(dst + (off + static_cast<uint32_t>(r * stride))) =
          make_uint2(rec[2 * r], rec[2 * r + 1]);
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int y = y0 + r;
      if (y < H) {
        uint8_t *row = dst + static_cast<size_t>(y) * stride;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (x0 + j < W) row[x0 + j] = static_cast<uint8_t>(rec[2 * r + (j >> 2)] >> (8 * (j & 3)));
      }
    }
  }
}

// a9: sum of squared differences of the W x H part of a block, as
// sum(p^2) - 2 sum(p r) + sum(r^2) with packed unsigned dot products, exact in
// 32 bits (at most 64 * 255^2 per term).  Edge blocks mask the bytes of
// positions outside the image to zero in both operands.
__device__ __forceinline__ uint32_t block_sse(const uint32_t (&pix)[16], const uint32_t (&rec)[16], int W,
                                              int H, int by, int bx, bool full) {
  uint32_t pp = 0, pr = 0, rr = 0;
  if (full) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      pp = __builtin_amdgcn_udot4(pix[k], pix[k], pp, false);
      pr = __builtin_amdgcn_udot4(pix[k], rec[k], pr, false);
      rr = __builtin_amdgcn_udot4(rec[k], rec[k], rr, false);
    }
  } else {
    const int cols = min(W - bx * 8, 8);
    const uint32_t mlo = cols >= 4 ? 0xffffffffu : (0xffffffffu >> (8 * (4 - cols)));
    const uint32_t mhi = cols >= 8 ? 0xffffffffu : (cols <= 4 ? 0u : (0xffffffffu >> (8 * (8 - cols))));
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
  }
  return pp - 2u * pr + rr;
}

// Sum of v over the workgroup, then one 64-bit atomic add to *acc; `wave` is
// this wave's index in the workgroup (wave-uniform).
template <int kThreads>
__device__ __forceinline__ void workgroup_add(uint64_t v, unsigned long long *acc, int wave) {
  __shared__ unsigned long long partial[kThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const bool leader = __lane_id() == 0;
  if (leader) partial[wave] = v;
  __syncthreads();
  if (leader && wave == 0) {
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += partial[w];
    if (t) atomicAdd(acc, t);
  }
}

template <int kThreads>
__device__ __forceinline__ void workgroup_add(uint64_t v, unsigned long long *acc) {
  workgroup_add<kThreads>(v, acc, static_cast<int>(threadIdx.x >> 6));
}

// This wave's index in its workgroup as an SGPR value, taken at kernel entry so
// that threadIdx.x need not stay live in a VGPR until the final reduction.
__device__ __forceinline__ int wave_index() {
  int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x)) >> 6;
  asm volatile("" : "+s"(w));
  return w;
}

// The lane's index in its wave, computed afresh at each call (the mask is
// opaque to the compiler, so two calls are never merged into one live value).
__device__ __forceinline__ int lane_index() {
  unsigned m = ~0u;
  asm volatile("" : "+s"(m));
  return static_cast<int>(__builtin_amdgcn_mbcnt_hi(m, __builtin_amdgcn_mbcnt_lo(m, 0u)));
}

// Position of this lane's block.  Lanes past the last block run the same
// instructions on zeros (so every lane reaches every barrier) and touch no memory.
struct BlockPos {
  int by, bx;
  bool live, full;
};

__device__ __forceinline__ BlockPos block_pos(int b, int W, int H, int bw, int nblocks) {
  // computed on every lane and zeroed by selects on dead ones: no branch, so no
  // constant has to be carried to a join point
  const bool live = b < nblocks;
  const int by = b / bw, bx = b - (b / bw) * bw;
  BlockPos p;
  p.live = live;
  p.by = live ? by : 0;
  p.bx = live ? bx : 0;
  p.full = live && bx * 8 + 8 <= W && by * 8 + 8 <= H;
  return p;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Zero n words (a fill kernel, so the library enqueues no memset).
template <class T>
__global__ void fill_zero_kernel(T *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

// a1..a9 on block b = wave_base + lane of one plane under recipe RC, one lane
// per block (wave_base is wave-uniform): returns the block's SSE (0 for a lane
// past the last block).  Every lane of the workgroup must call it together (it
// contains workgroup barriers).  The block index is formed twice, at the load
// and again at the store, so no VGPR carries it through the transforms.
template <class RC, bool kEmitQ>
__device__ __forceinline__ uint32_t codec_block(const uint8_t *__restrict__ src, int W, int H, int src_stride,
                                                int bw, int nblocks, int wave_base, const CodecQuant &qa,
                                                uint8_t *__restrict__ dst, int dst_stride,
                                                int16_t *__restrict__ qcoef) {
  const int b = wave_base + lane_index();
  const BlockPos p = block_pos(b, W, H, bw, nblocks);
  uint32_t pix[16] = {};
  if (p.live) load_block(src, W, H, src_stride, p.by, p.bx, p.full, pix);
  int x[64];
  unpack_block<RC::frac>(pix, x);
  barrier();
  forward_block<RC::n, RC::frac>(x);
  barrier();
  int q[64];
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int s = u + v;
      x[u * 8 + v] = quant_dequant<RC::frac>(x[u * 8 + v], qa.rcp[s], qa.qscale[s], qa.half[s], q[u * 8 + v]);
    }
  if constexpr (kEmitQ) {
    if (p.live) {
      int4 *out = reinterpret_cast<int4 *>(qcoef + static_cast<size_t>(b) * 64);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        out[k] = make_int4((q[8 * k] & 0xffff) | (q[8 * k + 1] << 16), (q[8 * k + 2] & 0xffff) | (q[8 * k + 3] << 16),
                           (q[8 * k + 4] & 0xffff) | (q[8 * k + 5] << 16), (q[8 * k + 6] & 0xffff) | (q[8 * k + 7] << 16));
    }
  }
  x[0] += kReconstructDC<RC::inv_frac>;
  barrier();
  inverse_block<RC::n>(x);
  barrier();
  uint32_t rec[16];
  pack_block<RC::inv_frac>(x, rec);
  const BlockPos p2 = block_pos(wave_base + lane_index(), W, H, bw, nblocks);
  uint32_t pix2[16] = {};
  if (p2.live) {
    store_block(dst, W, H, dst_stride, p2.by, p2.bx, p2.full, rec);
    load_block(src, W, H, src_stride, p2.by, p2.bx, p2.full, pix2);  // again, for the SSE (cache hit)
  }
  // every lane forms a sum (a select, not a branch, discards the dead lanes')
  const uint32_t err = block_sse(pix2, rec, W, H, p2.by, p2.bx, p2.full);
  return p2.live ? err : 0u;
}

// a1..a9 fused under recipe RC: one lane per block; only pixels (and optionally
// the int16 quantized values) touch memory; the SSE goes to *sse by one atomic
// per workgroup.
template <class RC, bool kEmitQ>
__global__ __launch_bounds__(kBlockThreads) DCT_FOUR_WAVES void codec_kernel(const uint8_t *__restrict__ src, int W, int H,
                                                              int src_stride, int bw, int nblocks, CodecQuant qa,
                                                              uint8_t *__restrict__ dst, int dst_stride,
                                                              int16_t *__restrict__ qcoef,
                                                              unsigned long long *__restrict__ sse) {
  const int wave = wave_index();
  const int wave_base = static_cast<int>(blockIdx.x) * kBlockThreads + wave * 64;
  const uint32_t err =
      codec_block<RC, kEmitQ>(src, W, H, src_stride, bw, nblocks, wave_base, qa, dst, dst_stride, qcoef);
  workgroup_add<kBlockThreads>(err, sse, wave);
}

}  // namespace dct
