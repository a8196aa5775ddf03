// deblock.hpp -- the learned deblocking post-filter: a 1-32-32-32-1 network of
// 3x3 convolutions applied to decoded planes, its training gradient and Adam.
//
// The paper's decoded images show the blocking of 8x8 transform coding (Sec. 4);
// this network reduces it.  With x = p / 255 for the decoded pixels p:
//   a1 = relu(conv(x; W1, b1)), a2 = relu(conv(a1; W2, b2)), a3 = relu(conv(a2; W3, b3)),
//   y  = x + conv(a3; W4, b4),
// conv a 3x3 cross-correlation with zero padding outside each image.  The output
// pixel is clamp(floor(255 y + 1/2), 0, 255).  Weights are used as FP16 values
// (rounded from the FP32 master copy), activations are stored as FP16,
// accumulation is FP32; gradients are FP32.
//
// Data layout: activations are pixel-major with the 32 channels of a pixel in
// 64 contiguous bytes (FP16).  Pixels are numbered image by image, row-major.
// An "image set" is n images of h x w whose top-left corners sit at given
// (row, col) positions of one uint8 plane (training crops), or one image at the
// origin (inference).
//
// Backward signals.  The training pass keeps g_l = dL/dz_l (z_l the layer's
// pre-activation) as FP16 values times an exact power of two S (kept in the
// same pixel-major layout), so that every product of the backward pass runs on
// the matrix cores with FP16 operands and FP32 sums.  S = 2^(floor(log2 N) + 8)
// for N pixels puts dL/dy = 2 (y - t) / N at 2^8 .. 2^9 times (y - t), inside
// FP16's normal range for |y - t| between about 2^-22 and 2^7; the weight and
// bias gradients are divided by S (exactly) when their partial sums are added.
//
// Kernels (a wave per tile of 3 rows x 16 pixels unless stated):
//   layer1_kernel      x -> a1 on the matrix cores: the nine taps as the K of
//                      v_mfma_f32_16x16x16_f16 over the decoded pixel values
//                      0..255 (exact in FP16), the 1/255 and the bias after the sum
//   mid_kernel<false>  a -> relu(conv(a)) for the 32 -> 32 layers on the matrix
//                      cores: per wave, 16 pixels x 32 output channels, K = 9 taps
//                      x 32 input channels as nine v_mfma_f32_16x16x32_f16 per
//                      16-channel half; lane (i, g) loads 8 channels (16 bytes)
//                      of its pixel's neighbour and gets 4 output channels.
//   mid_kernel<true>   g_l from g_(l+1) through a 32 -> 32 layer: the same
//                      implicit GEMM with the layer's weights transposed (input
//                      and output channels swapped) and the taps mirrored, and
//                      the ReLU mask of a_l in place of bias and ReLU
//   layer4_kernel      a3 -> y (training), the loss terms and S dL/dy: the
//                      32 -> 1 layer as one GEMM per input row with the nine
//                      taps as its rows, then each pixel's nine tap sums added
//   fused_apply_kernel inference in one launch: all four layers of a 28 x 28
//                      output tile with x, a1, a2 and layer 4's tap sums in LDS
//   bwd4_kernel        g3 from dL/dy through layer 4 and the ReLU of a3 (VALU,
//                      one thread per pixel)
//   wgrad_mid_kernel   weight and bias gradients of a 32 -> 32 layer as a GEMM
//                      over pixels, K = 32 pixels of one image row per
//                      instruction: three waves per workgroup, one per tap row
//   wgrad_edge_kernel  the same for layer 1 (x against g1) and layer 4 (a3
//                      against dL/dy), with the nine taps as the GEMM's columns
//   reduce_kernel      second stage of the weight gradients: adds the partial
//                      rows of all workgroups in a fixed order and scales them
//   loss_reduce_kernel the training loss from per-workgroup partial sums, in a
//                      fixed order
//   adam_kernel        Adam with bias correction
//   init_kernel        the initial parameters from a seed (Philox4x32-10)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dct {
namespace db {

inline constexpr int kC = 32;
inline constexpr int kNParam = 19105;
inline constexpr int kW1 = 0, kB1 = 288, kW2 = 320, kB2 = 9536, kW3 = 9568, kB3 = 18784, kW4 = 18816, kB4 = 19104;
inline constexpr int kThreads = 256;

struct ImageSet {
  const uint8_t *plane;  // decoded pixels
  const uint8_t *orig;   // original pixels at the same positions (training), or null
  int32_t stride, plane_w, plane_h;
  const int32_t *pos;  // [n][2] top-left (row, col) per image, or null for one image at (0, 0)
  int32_t n, h, w;
};

struct Pix {
  int b, r, c;
};

// pixel id -> (image, row, column); ids stay below 2^31 (checked on the host), so
// the divisions are 32-bit
__device__ __forceinline__ Pix pix_of(const ImageSet &s, int64_t p) {
  const uint32_t u = static_cast<uint32_t>(p), hw = static_cast<uint32_t>(s.h) * static_cast<uint32_t>(s.w);
  Pix q;
  q.b = static_cast<int>(u / hw);
  const uint32_t rem = u - static_cast<uint32_t>(q.b) * hw;
  q.r = static_cast<int>(rem / static_cast<uint32_t>(s.w));
  q.c = static_cast<int>(rem - static_cast<uint32_t>(q.r) * static_cast<uint32_t>(s.w));
  return q;
}

// pixel (r, c) of image b of a plane; 0 outside the image or the plane
__device__ __forceinline__ float plane_px(const ImageSet &s, const uint8_t *__restrict__ plane, int b, int r, int c) {
  if (r < 0 || r >= s.h || c < 0 || c >= s.w) return 0.0f;
  const int R = (s.pos ? s.pos[2 * b] : 0) + r, Cc = (s.pos ? s.pos[2 * b + 1] : 0) + c;
  if (R < 0 || R >= s.plane_h || Cc < 0 || Cc >= s.plane_w) return 0.0f;
  return static_cast<float>(plane[static_cast<size_t>(R) * s.stride + Cc]);
}

// pixel id of neighbour (r + dr, c + dc) of image b, or -1 outside the image
__device__ __forceinline__ int64_t nb_id(const ImageSet &s, const Pix &q, int dr, int dc) {
  const int r = q.r + dr, c = q.c + dc;
  if (r < 0 || r >= s.h || c < 0 || c >= s.w) return -1;
  return (static_cast<int64_t>(q.b) * s.h + r) * s.w + c;
}

inline constexpr float kInv255 = 1.0f / 255.0f;

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// FP32 master -> FP16-rounded weights, as FP32 (VALU kernels) and FP16 (matrix cores)
__global__ __launch_bounds__(kThreads) void prep_kernel(const float *__restrict__ p, float *__restrict__ wq,
                                                        _Float16 *__restrict__ wh) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k < kNParam) {
    const _Float16 h = static_cast<_Float16>(p[k]);
    wh[k] = h;
    wq[k] = static_cast<float>(h);
  }
}

// pixel rows a wave's tile computes
inline constexpr int kRows = 3;

// The inference operands: the matrix-core A operands of every lane, laid out so
// that a lane loads its whole set with 16-byte accesses, consecutive lanes at
// consecutive addresses, and the biases, all from the FP16-rounded weights
// (prepared once per call from the FP32 master copy):
//   mid[layer][m][t][lane]  layers 2 and 3: W[16m + i][8g + e][t], e = 0..7
//   l4[lane]                layer 4: W4[4g + e][i] (e < 4), W4[12 + 4g + e][i] (e >= 4) for
//                           taps i < 9, zero for i >= 9
//   l1[m][lane]             layer 1: W1[16m + i][4g + e], e = 0..3 (taps 9.. zero)
//   bias[l]                 b1, b2, b3; b4 in b4
struct WeightOps {
  h8 mid[2][2][9][64];
  h8 l4[64];
  _Float16 l1[2][64][4];
  float bias[3][kC];
  float b4;
};

__global__ __launch_bounds__(kThreads) void prep_ops_kernel(const float *__restrict__ p, WeightOps *__restrict__ ops) {
  const int k = blockIdx.x * kThreads + threadIdx.x;  // one thread per operand slot
  constexpr int kMid = 2 * 2 * 9 * 64, kL4 = 64, kL1 = 2 * 64, kBias = 3 * kC + 1;
  const _Float16 zero = static_cast<_Float16>(0.0f);
  auto h = [&](int idx) { return static_cast<_Float16>(p[idx]); };
  if (k < kMid) {
    const int lane = k % 64, t = (k / 64) % 9, m = (k / (64 * 9)) % 2, layer = k / (64 * 9 * 2);
    const int i = lane & 15, g = lane >> 4;
    const int w = layer == 0 ? kW2 : kW3;
    h8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = h(w + ((16 * m + i) * kC + 8 * g + e) * 9 + t);
    ops->mid[layer][m][t][lane] = v;
  } else if (k < kMid + kL4) {
    const int lane = k - kMid;
    const int i = lane & 15, g = lane >> 4;
    h8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = i < 9 ? h(kW4 + (e < 4 ? 4 * g + e : 12 + 4 * g + e) * 9 + i) : zero;
    ops->l4[lane] = v;
  } else if (k < kMid + kL4 + kL1) {
    const int lane = (k - kMid - kL4) % 64, m = (k - kMid - kL4) / 64;
    const int i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int t = 4 * g + e;
      ops->l1[m][lane][e] = t < 9 ? h(kW1 + (16 * m + i) * 9 + t) : zero;
    }
  } else if (k < kMid + kL4 + kL1 + kBias) {
    const int j = k - kMid - kL4 - kL1;
    const int base[3] = {kB1, kB2, kB3};
    if (j < 3 * kC)
      ops->bias[j / kC][j % kC] = static_cast<float>(h(base[j / kC] + j % kC));
    else
      ops->b4 = static_cast<float>(h(kB4));
  }
}
inline constexpr int kPrepOpsThreads = 2 * 2 * 9 * 64 + 64 + 2 * 64 + 3 * kC + 1;

typedef _Float16 h4 __attribute__((ext_vector_type(4)));

// Layer 1 on the matrix cores, v_mfma_f32_16x16x16_f16 with the nine taps as K
// (taps 9..15 zero): z[co] = sum_t W1[co][t] P[pixel + offset(t)] with P the
// decoded pixel values 0..255 (exact in FP16, so every product is exact), then
// a1 = relu(z / 255 + b1) from the FP32 sum.  Operands of output half m, lane
// (i, g): A[i][4g+e] = W1[16m + i][4g + e], B[4g+e][i] = P of pixel i at tap
// 4g + e, D[4g + r][i] = z[16m + 4g + r] of pixel i.
struct L1Consts {
  h4 wa[2];
  float bv[2][4];
};

__device__ __forceinline__ void l1_consts(const _Float16 *__restrict__ wh, const float *__restrict__ wq,
                                          L1Consts &c) {
  const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int t = 4 * g + e;
      c.wa[m][e] = t < 9 ? wh[kW1 + (16 * m + i) * 9 + t] : static_cast<_Float16>(0.0f);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) c.bv[m][r] = wq[kB1 + 16 * m + 4 * g + r];
  }
}

typedef float f2 __attribute__((ext_vector_type(2)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// relu(z) for four FP32 sums as FP16, two to a word.  The conversion rounds to
// nearest and keeps the sign, so taking the ReLU after it gives the same
// values (a negative sum may leave -0, which counts as zero everywhere).
__device__ __forceinline__ uint2 relu_pack(f4 z) {
  const h2 zero = {static_cast<_Float16>(0.0f), static_cast<_Float16>(0.0f)};
  const h2 lo = __builtin_elementwise_max(__builtin_convertvector(f2{z[0], z[1]}, h2), zero);
  const h2 hi = __builtin_elementwise_max(__builtin_convertvector(f2{z[2], z[3]}, h2), zero);
  return make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
}

// The lane's four channels 16m + 4g .. + 3 of a1 for its pixel, as two packed
// words per half m, from the B operand bp (the pixel's taps 4g .. 4g + 3)
__device__ __forceinline__ void l1_pixel(const L1Consts &c, h4 bp, uint2 (&out)[2]) {
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const f4 d = __builtin_amdgcn_mfma_f32_16x16x16f16(c.wa[m], bp, f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    f4 z;
#pragma unroll
    for (int r = 0; r < 4; ++r) z[r] = d[r] * kInv255 + c.bv[m][r];
    out[m] = relu_pack(z);
  }
}

// Layer 4 on the matrix cores with the taps as the M dimension.  For 16
// consecutive pixels p of an a3 row, one v_mfma_f32_16x16x32_f16 forms the
// per-tap sums D[t][p] = sum_ci W4[ci][t] a3[p][ci] (A row t holds tap t's
// weights, rows 9 .. 15 zero).  Its K index 8g + e stands for channel 4g + e
// (e < 4) or 16 + 4g + e - 4 (e >= 4), so that a lane's B operand is exactly the
// two packed words a 32 -> 32 layer leaves in lane (i, g) for pixel i (channels
// 16m + 4g .. + 3 for m = 0, 1).  Output pixel (r, c) then adds its nine taps in
// the order t = 3 dy + dx = 0 .. 8, D_t taken at a3 pixel (r + dy, c + dx):
//   net = ((D_0 + D_1) + ...) + D_8,   y = p / 255 + (net + b4).
// Every kernel that forms y uses l4_sums and l4_net, so the sums are the same
// everywhere.
struct L4Consts {
  h8 wa;  // A[i][8g + e] = W4[channel(g, e)][i] for taps i < 9
  float b4;
};

__device__ __forceinline__ int l4_channel(int g, int e) { return e < 4 ? 4 * g + e : 16 + 4 * g + e - 4; }

__device__ __forceinline__ void l4_consts(const _Float16 *__restrict__ wh, const float *__restrict__ wq,
                                          L4Consts &c) {
  const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
#pragma unroll
  for (int e = 0; e < 8; ++e)
    c.wa[e] = i < 9 ? wh[kW4 + l4_channel(g, e) * 9 + i] : static_cast<_Float16>(0.0f);
  c.b4 = wq[kB4];
}

// the per-tap sums of the lane's pixel from its packed channels (w[m]: channels
// 16m + 4g .. + 3): lane (i, g) gets taps 4g .. 4g + 3 of pixel i
__device__ __forceinline__ f4 l4_sums(const h8 &wa, uint2 w0, uint2 w1) {
  const h8 bx = __builtin_bit_cast(h8, make_uint4(w0.x, w0.y, w1.x, w1.y));
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(wa, bx, f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
}

// net of one output pixel from its nine per-tap sums, D(dy, dx, t)
template <class Fetch>
__device__ __forceinline__ float l4_net(Fetch D) {
  float net = D(0, 0, 0);
#pragma unroll
  for (int t = 1; t < 9; ++t) net += D(t / 3, t % 3, t);
  return net;
}

// every lane's LDS stores before any lane's loads (and loads before the next
// stores) in a buffer private to the wave
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The training pass's layer-4 tiles: kRows output rows x kL4Cols columns, whose
// sums come from kRows + 2 input rows of 16 columns, through a buffer per wave.
// With these pitches the 48 lanes of a buffer store (lanes (i, g < 3), tap
// 4g + r) and the 42 lanes of a gather (lanes (j, o)) each meet different banks.
inline constexpr int kL4Cols = 14;
inline constexpr int kL4TapPitch = 20;                        // floats per tap: 16 pixels + 4
inline constexpr int kL4RowPitch = 12 * kL4TapPitch + 32;     // floats per input row (taps 0 .. 11)
inline constexpr int kL4Buf = (kRows + 2) * kL4RowPitch;      // floats per wave

// a1 = relu(conv(x; W1, b1)): a wave computes kRows rows x 16 columns of one image
__global__ __launch_bounds__(kThreads) void layer1_kernel(ImageSet s, const float *__restrict__ wq,
                                                          const _Float16 *__restrict__ wh,
                                                          _Float16 *__restrict__ a1, int64_t ntiles) {
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
  L1Consts k1;
  l1_consts(wh, wq, k1);
  const uint32_t col_tiles = (static_cast<uint32_t>(s.w) + 15u) / 16u;
  const uint32_t row_groups = (static_cast<uint32_t>(s.h) + kRows - 1u) / kRows;
  const uint32_t step = gridDim.x * (kThreads / 64);
  for (uint32_t tile = blockIdx.x * (kThreads / 64) + wave; tile < static_cast<uint32_t>(ntiles); tile += step) {
    const uint32_t gid = tile / col_tiles;
    const int b = static_cast<int>(gid / row_groups);
    const int r0 = static_cast<int>(gid - static_cast<uint32_t>(b) * row_groups) * kRows;
    const int c = static_cast<int>((tile - gid * col_tiles) * 16u) + i;
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int r = r0 + j;
      h4 bp;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int t = 4 * g + e;
        bp[e] = static_cast<_Float16>(t < 9 ? plane_px(s, s.plane, b, r + t / 3 - 1, c + t % 3 - 1) : 0.0f);
      }
      uint2 out[2];
      l1_pixel(k1, bp, out);
      if (r < s.h && c < s.w) {
        const int64_t p = (static_cast<int64_t>(b) * s.h + r) * s.w + c;
#pragma unroll
        for (int m = 0; m < 2; ++m) *reinterpret_cast<uint2 *>(a1 + p * kC + 16 * m + 4 * g) = out[m];
      }
    }
  }
}

// aout = relu(conv(ain; W, b)) for a 32 -> 32 layer on the matrix cores
// (kBwd = false), or the backward signal of its input (kBwd = true):
//   aout[q][ci] = (mask[q][ci] > 0) sum_t sum_co W[co][ci][t] ain[q - offset(t)][co],
// which is the same convolution with input and output channels swapped and the
// taps mirrored (offset(8 - t) = -offset(t)), applied to the scaled FP16 signal
// `ain` of the layer above; `mask` is the layer's input activation.
// Operands of v_mfma_f32_16x16x32_f16 for tap t and output half m (lane i, g):
//   A[i][8g+e] = W'[16m + i][8g + e][t], B[8g+e][i] = ain[neighbour t of pixel i][8g + e],
//   D[4g+r][i] = output channel 16m + 4g + r of pixel i,
// with W' = W forward and W'[o][c][t] = W[c][o][8 - t] backward.
// A wave computes kRows vertically adjacent tiles of 16 pixels (rows r0 .. r0 +
// kRows - 1, columns c0 .. c0 + 15 of one image): each of the kRows + 2 input rows
// x 3 column offsets is loaded once and feeds every output row whose 3x3 window
// covers it, so a tile needs (kRows + 2) * 3 / kRows loads instead of 9.  The
// image, row and column of a tile are the same for the whole wave.
template <bool kBwd>
__global__ __launch_bounds__(kThreads) void mid_kernel(ImageSet s, const _Float16 *__restrict__ ain,
                                                       const _Float16 *__restrict__ wh_layer,
                                                       const float *__restrict__ bias,
                                                       const _Float16 *__restrict__ mask,
                                                       _Float16 *__restrict__ aout, int64_t npix, int64_t ntiles) {
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
  h8 wa[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        wa[t][m][e] = kBwd ? wh_layer[((8 * g + e) * kC + 16 * m + i) * 9 + (8 - t)]
                           : wh_layer[((16 * m + i) * kC + 8 * g + e) * 9 + t];
  float bv[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) bv[m][r] = kBwd ? 0.0f : bias[16 * m + 4 * g + r];
  const uint32_t col_tiles = (static_cast<uint32_t>(s.w) + 15u) / 16u;
  const uint32_t row_groups = (static_cast<uint32_t>(s.h) + kRows - 1u) / kRows;
  const uint32_t step = gridDim.x * (kThreads / 64);
  for (uint32_t tile = blockIdx.x * (kThreads / 64) + wave; tile < static_cast<uint32_t>(ntiles); tile += step) {
    const uint32_t gid = tile / col_tiles;  // (image, row group) over the whole set
    const int b = static_cast<int>(gid / row_groups);
    const int r0 = static_cast<int>(gid - static_cast<uint32_t>(b) * row_groups) * kRows;
    const int c = static_cast<int>((tile - gid * col_tiles) * 16u) + i;
    // forward: the bias is the addend of each sum's first product
    f4 acc[kRows][2];
#pragma unroll
    for (int j = 0; j < kRows; ++j)
#pragma unroll
      for (int m = 0; m < 2; ++m) acc[j][m] = f4{bv[m][0], bv[m][1], bv[m][2], bv[m][3]};
#pragma unroll
    for (int k = 0; k < kRows + 2; ++k) {  // input row r0 - 1 + k
      // one input row's loads in flight at a time (the accumulators pass through
      // an empty asm, so no later row's loads are hoisted above this point): 128
      // VGPRs and four waves per SIMD instead of 132 and three
      static_assert(kRows == 3, "the fence names the three rows' accumulators");
      asm volatile("" : "+v"(acc[0][0]), "+v"(acc[0][1]), "+v"(acc[1][0]), "+v"(acc[1][1]), "+v"(acc[2][0]),
                   "+v"(acc[2][1]));
      const int rr = r0 - 1 + k;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int cc = c + dx - 1;
        h8 bx;
        if (rr >= 0 && rr < s.h && cc >= 0 && cc < s.w && c < s.w) {
          const int64_t nb = (static_cast<int64_t>(b) * s.h + rr) * s.w + cc;
          bx = *reinterpret_cast<const h8 *>(ain + nb * kC + 8 * g);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) bx[e] = static_cast<_Float16>(0.0f);
        }
        // output row j uses input row r0 - 1 + k as tap row dy = k - j
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
          const int dy = k - j;
          if (dy >= 0 && dy <= 2) {
#pragma unroll
            for (int m = 0; m < 2; ++m)
              acc[j][m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wa[dy * 3 + dx][m], bx, acc[j][m], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int r = r0 + j;
      if (r < s.h && c < s.w) {
        const int64_t p = (static_cast<int64_t>(b) * s.h + r) * s.w + c;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          uint2 w;
          if constexpr (kBwd) {
            const uint2 mw = *reinterpret_cast<const uint2 *>(mask + p * kC + 16 * m + 4 * g);
            const uint32_t mv[4] = {mw.x & 0xffffu, mw.x >> 16, mw.y & 0xffffu, mw.y >> 16};
            uint32_t hb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float a = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(mv[q])));
              hb[q] = __builtin_bit_cast(uint16_t, static_cast<_Float16>(a > 0.0f ? acc[j][m][q] : 0.0f));
            }
            w = make_uint2(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16));
          } else {
            w = relu_pack(acc[j][m]);
          }
          *reinterpret_cast<uint2 *>(aout + p * kC + 16 * m + 4 * g) = w;
        }
      }
    }
  }
}

// y = p / 255 + net for a decoded pixel p: the quotient rounded on its own, then
// the sum (no fused multiply-add), identically in every kernel that forms y
__device__ __forceinline__ float residual(float p, float net) {
#pragma clang fp contract(off)
  return p * kInv255 + net;
}

// Training forward of layer 4: y = x + conv(a3; W4, b4) on the matrix cores
// (l4_sums / l4_net, a wave per kRows rows x kL4Cols columns of one image), then
// y to y_out (if not null), the scaled signal S dL/dy = fp16(fp32(grad_scale
// (y - t)) S) to g4, and the workgroup's sum of (y - t)^2 to sq[blockIdx.x]
// (summed in a fixed order).
__global__ __launch_bounds__(kThreads) void layer4_kernel(ImageSet s, const _Float16 *__restrict__ a3,
                                                          const float *__restrict__ wq,
                                                          const _Float16 *__restrict__ wh, int64_t ntiles,
                                                          float *__restrict__ y_out, _Float16 *__restrict__ g4,
                                                          double *__restrict__ sq, float grad_scale, float S) {
  __shared__ float bufs[kThreads / 64][kL4Buf];
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
  float *buf = bufs[wave];
  L4Consts k4;
  l4_consts(wh, wq, k4);
  double local = 0.0;
  const uint32_t col_tiles = (static_cast<uint32_t>(s.w) + kL4Cols - 1u) / kL4Cols;
  const uint32_t row_groups = (static_cast<uint32_t>(s.h) + kRows - 1u) / kRows;
  const uint32_t step = gridDim.x * (kThreads / 64);
  for (uint32_t tile = blockIdx.x * (kThreads / 64) + wave; tile < static_cast<uint32_t>(ntiles); tile += step) {
    const uint32_t gid = tile / col_tiles;
    const int b = static_cast<int>(gid / row_groups);
    const int r0 = static_cast<int>(gid - static_cast<uint32_t>(b) * row_groups) * kRows;
    const int c0 = static_cast<int>((tile - gid * col_tiles) * kL4Cols);
    const int cc = c0 - 1 + i;  // this lane's input column
#pragma unroll
    for (int k = 0; k < kRows + 2; ++k) {
      const int rr = r0 - 1 + k;
      uint2 w[2] = {make_uint2(0u, 0u), make_uint2(0u, 0u)};
      if (rr >= 0 && rr < s.h && cc >= 0 && cc < s.w) {
        const _Float16 *px = a3 + ((static_cast<int64_t>(b) * s.h + rr) * s.w + cc) * kC + 4 * g;
        w[0] = *reinterpret_cast<const uint2 *>(px);
        w[1] = *reinterpret_cast<const uint2 *>(px + 16);
      }
      const f4 d = l4_sums(k4.wa, w[0], w[1]);
      if (g < 3) {
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[k * kL4RowPitch + (4 * g + r) * kL4TapPitch + i] = d[r];
      }
    }
    wave_sync();
    if (l < kRows * kL4Cols) {
      const int j = l / kL4Cols, o = l - j * kL4Cols;
      const int r = r0 + j, c = c0 + o;
      const float *src = buf + j * kL4RowPitch + o;
      const float net = l4_net([&](int dy, int dx, int t) { return src[dy * kL4RowPitch + t * kL4TapPitch + dx]; });
      if (r < s.h && c < s.w) {
        const float y = residual(plane_px(s, s.plane, b, r, c), net + k4.b4);
        const int64_t p = (static_cast<int64_t>(b) * s.h + r) * s.w + c;
        const float e = y - plane_px(s, s.orig, b, r, c) * kInv255;
        if (y_out) y_out[p] = y;
        const float gv = grad_scale * e;
        g4[p] = static_cast<_Float16>(gv * S);
        local += static_cast<double>(e) * e;
      }
    }
    wave_sync();
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) local += __shfl_xor(local, off, 64);
  __shared__ double wsum[kThreads / 64];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += wsum[w];
    sq[blockIdx.x] = t;
  }
}

// S g3 = (a3 > 0) S dL/da3 with S dL/da3[q][ci] = sum_t W4[ci][t] (S g4)[q - offset(t)]
// (FP32 sums of the FP16 signal), stored as FP16
__global__ __launch_bounds__(kThreads) void bwd4_kernel(ImageSet s, const _Float16 *__restrict__ g4,
                                                        const _Float16 *__restrict__ a3,
                                                        const float *__restrict__ wq, _Float16 *__restrict__ g3,
                                                        int64_t npix) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; p < npix;
       p += static_cast<int64_t>(gridDim.x) * kThreads) {
    const Pix q = pix_of(s, p);
    float gv[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int64_t nb = nb_id(s, q, 1 - t / 3, 1 - t % 3);
      gv[t] = nb >= 0 ? static_cast<float>(g4[nb]) : 0.0f;
    }
    const uint4 *ap = reinterpret_cast<const uint4 *>(a3 + p * kC);
    uint4 *dst = reinterpret_cast<uint4 *>(g3 + p * kC);
#pragma unroll
    for (int k = 0; k < kC / 8; ++k) {
      const h8 av = __builtin_bit_cast(h8, ap[k]);
      h8 o;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int ci = 8 * k + j;
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += wq[kW4 + ci * 9 + t] * gv[t];
        o[j] = static_cast<_Float16>(static_cast<float>(av[j]) > 0.0f ? acc : 0.0f);
      }
      dst[k] = __builtin_bit_cast(uint4, o);
    }
  }
}

// Weight and bias gradients as GEMMs over pixels on the matrix cores, first
// stage.  The contraction runs over "chunks": 32 consecutive pixels of one image
// row (columns c0 .. c0 + 31, c0 a multiple of 32; columns past the image width
// contribute zeros).  Lane (j, g) of a wave (j = lane % 16, g = lane / 16)
// supplies pixels c0 + 8g .. c0 + 8g + 7 of the chunk to both operands of
// v_mfma_f32_16x16x32_f16, whose D[4g + r][j] it then holds.  Workgroup w takes
// chunks w cpw .. w cpw + cpw - 1 and writes one partial row of FP32 sums (of the
// scaled signals) to part[w]; reduce_kernel adds the rows.  A 32 -> 32 layer's
// row holds its weights in accumulator order (mid_slot), so that each of a
// wave's stores covers 64 consecutive floats; reduce_kernel puts them back in
// the [co][ci][t] order of the parameters.
inline constexpr int kNWMid = kC * kC * 9 + kC;  // partial row of a 32 -> 32 layer
inline constexpr int kNWEdge = kC * 9 + kC;      // partial row of layer 1 (layer 4 uses 9 kC + 1)

// Slot of D[4 gq + r][j] of tile (m, n) of tap t in a 32 -> 32 layer's partial
// row, and the weight (co, ci, t) = (16 m + 4 gq + r, 16 n + j, t) it belongs to.
__host__ __device__ constexpr int mid_slot(int t, int m, int n, int r, int gq, int j) {
  return ((((t * 2 + m) * 2 + n) * 4 + r) * 4 + gq) * 16 + j;
}
__host__ __device__ constexpr int mid_weight_of_slot(int k) {
  const int j = k & 15, gq = (k >> 4) & 3, r = (k >> 6) & 3, n = (k >> 8) & 1, m = (k >> 9) & 1, t = k >> 10;
  return ((16 * m + 4 * gq + r) * kC + 16 * n + j) * 9 + t;
}
constexpr bool mid_slots_invert() {
  for (int t = 0; t < 9; ++t)
    for (int m = 0; m < 2; ++m)
      for (int n = 0; n < 2; ++n)
        for (int r = 0; r < 4; ++r)
          for (int gq = 0; gq < 4; ++gq)
            for (int j = 0; j < 16; ++j) {
              const int k = mid_slot(t, m, n, r, gq, j);
              if (k < 0 || k >= kC * kC * 9 ||
                  mid_weight_of_slot(k) != ((16 * m + 4 * gq + r) * kC + 16 * n + j) * 9 + t)
                return false;
            }
  return true;
}
static_assert(mid_slots_invert(), "mid_slot is a bijection onto the weights, undone by mid_weight_of_slot");

struct Chunk {
  int b, r, c;  // image, row, first column of this lane's eight pixels
};

__device__ __forceinline__ Chunk chunk_of(const ImageSet &s, uint32_t chunk, int g) {
  const uint32_t segs = (static_cast<uint32_t>(s.w) + 31u) / 32u;
  const uint32_t row = chunk / segs;
  Chunk k;
  k.b = static_cast<int>(row / static_cast<uint32_t>(s.h));
  k.r = static_cast<int>(row - static_cast<uint32_t>(k.b) * static_cast<uint32_t>(s.h));
  k.c = static_cast<int>((chunk - row * segs) * 32u) + 8 * g;
  return k;
}

// 32 -> 32 layer: dW[co][ci][t] = sum_p g[p][co] a[p + offset(t)][ci], db[co] = sum_p g[p][co]
// (g the scaled FP16 signal of the layer's pre-activation, a its FP16 input).
// A[j][8g+e] = g[pixel e][16m + j], B[8g+e][j] = a[pixel e + offset(t)][16n + j].
// Three waves per chunk stream; wave dy computes the taps (dy, 0..2) for all four
// 16 x 16 (co, ci) tiles: the ten input pixels c - 1 .. c + 8 of its tap row give
// the three column offsets' operands.  Wave 0 of a stream also sums the bias
// gradients.  A workgroup runs kMidSplit streams, stream h taking every kMidSplit-th
// of its chunks from the h-th on; the other streams' sums are added to stream 0's
// through LDS in stream order, so the partial row does not depend on timing.
inline constexpr int kMidSplit = 2;
inline constexpr int kMidGradThreads = 3 * 64 * kMidSplit;
__global__ __launch_bounds__(kMidGradThreads) void wgrad_mid_kernel(ImageSet s, const _Float16 *__restrict__ g,
                                                                     const _Float16 *__restrict__ a,
                                                                     float *__restrict__ part, uint32_t nchunks,
                                                                     uint32_t cpw) {
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int dy = wave % 3, stream = wave / 3;
  const int l = threadIdx.x & 63, j = l & 15, gq = l >> 4;
  f4 acc[3][2][2];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx)
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n) acc[dx][m][n] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum[2] = {0.0f, 0.0f};
  const uint32_t first = blockIdx.x * cpw, last = min(first + cpw, nchunks);
  const _Float16 zero = static_cast<_Float16>(0.0f);
  for (uint32_t chunk = first + stream; chunk < last; chunk += kMidSplit) {
    const Chunk k = chunk_of(s, chunk, gq);
    const int64_t row = static_cast<int64_t>(k.b) * s.h + k.r;
    h8 A[2];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        A[m][e] = k.c + e < s.w ? g[(row * s.w + k.c + e) * kC + 16 * m + j] : zero;
    if (dy == 0) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int e = 0; e < 8; ++e) bsum[m] += static_cast<float>(A[m][e]);
    }
    const int rr = k.r + dy - 1;
    const bool row_ok = rr >= 0 && rr < s.h;
    const int64_t nrow = static_cast<int64_t>(k.b) * s.h + rr;
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      _Float16 v[10];
#pragma unroll
      for (int e = 0; e < 10; ++e) {
        const int cc = k.c - 1 + e;
        v[e] = row_ok && cc >= 0 && cc < s.w ? a[(nrow * s.w + cc) * kC + 16 * n + j] : zero;
      }
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        h8 B;
#pragma unroll
        for (int e = 0; e < 8; ++e) B[e] = v[dx + e];
#pragma unroll
        for (int m = 0; m < 2; ++m)
          acc[dx][m][n] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[m], B, acc[dx][m][n], 0, 0, 0);
      }
    }
  }
  // [stream - 1][dy][value][lane]: 48 accumulator values, then the two bias sums
  __shared__ float other[kMidSplit - 1][3][50][64];
  if (stream > 0) {
    float *o = &other[stream - 1][dy][0][l];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int r = 0; r < 4; ++r) o[64 * (((dx * 2 + m) * 2 + n) * 4 + r)] = acc[dx][m][n][r];
    o[64 * 48] = bsum[0];
    o[64 * 49] = bsum[1];
  }
  __syncthreads();
  if (stream > 0) return;
#pragma unroll
  for (int h = 0; h < kMidSplit - 1; ++h) {
    const float *o = &other[h][dy][0][l];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[dx][m][n][r] += o[64 * (((dx * 2 + m) * 2 + n) * 4 + r)];
    bsum[0] += o[64 * 48];
    bsum[1] += o[64 * 49];
  }
  float *dst = part + static_cast<size_t>(blockIdx.x) * kNWMid;
#pragma unroll
  for (int dx = 0; dx < 3; ++dx)
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          dst[mid_slot(dy * 3 + dx, m, n, r, gq, j)] = acc[dx][m][n][r];
  if (dy == 0) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      float t = bsum[m];
      t += __shfl_xor(t, 16, 64);
      t += __shfl_xor(t, 32, 64);
      if (gq == 0) dst[kC * kC * 9 + 16 * m + j] = t;
    }
  }
}

// Layers 1 and 4, with the nine taps as the GEMM's columns (j < 9; columns 9 .. 15
// are zero):
//   kFirst: dW1[co][t] = sum_p g1[p][co] P[p + offset(t)], db1[co] = sum_p g1[p][co],
//           A[j][8g+e] = g1[pixel e][16m + j], B[8g+e][t] = P[pixel e + offset(t)],
//           with P the decoded pixel values 0..255 (exact in FP16; reduce_kernel
//           applies the 1/255 of x = P / 255);
//   else:   dW4[ci][t] = sum_q a3[q][ci] g4[q - offset(t)], db4 = sum_q g4[q],
//           A[j][8g+e] = a3[pixel e][16m + j], B[8g+e][t] = g4[pixel e - offset(t)].
// kEdgeSplit waves per workgroup, wave h taking every kEdgeSplit-th of its chunks
// from the h-th on; the other waves' sums are added to wave 0's through LDS in
// wave order.
inline constexpr int kEdgeSplit = 4;
inline constexpr int kEdgeGradThreads = 64 * kEdgeSplit;
template <bool kFirst>
__global__ __launch_bounds__(kEdgeGradThreads) void wgrad_edge_kernel(ImageSet s, const _Float16 *__restrict__ act,
                                                                       const _Float16 *__restrict__ g4,
                                                                       float *__restrict__ part, uint32_t nchunks,
                                                                       uint32_t cpw) {
  constexpr int NW = kFirst ? kNWEdge : kC * 9 + 1;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int l = threadIdx.x & 63, j = l & 15, gq = l >> 4;
  const int tdy = j / 3 - 1, tdx = j % 3 - 1;  // this lane's tap offset (j < 9)
  f4 acc[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
  float bsum[2] = {0.0f, 0.0f};
  const uint32_t first = blockIdx.x * cpw, last = min(first + cpw, nchunks);
  const _Float16 zero = static_cast<_Float16>(0.0f);
  for (uint32_t chunk = first + wave; chunk < last; chunk += kEdgeSplit) {
    const Chunk k = chunk_of(s, chunk, gq);
    const int64_t row = static_cast<int64_t>(k.b) * s.h + k.r;
    h8 A[2], B;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        A[m][e] = k.c + e < s.w ? act[(row * s.w + k.c + e) * kC + 16 * m + j] : zero;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if constexpr (kFirst) {
        // plane_px is 0 outside the image and the plane; pixels past the row's
        // end meet A = 0
        B[e] = j < 9 ? static_cast<_Float16>(plane_px(s, s.plane, k.b, k.r + tdy, k.c + e + tdx)) : zero;
      } else {
        const int rr = k.r - tdy, cc = k.c + e - tdx;
        B[e] = j < 9 && k.c + e < s.w && rr >= 0 && rr < s.h && cc >= 0 && cc < s.w
                   ? g4[(static_cast<int64_t>(k.b) * s.h + rr) * s.w + cc]
                   : zero;
      }
    }
    if constexpr (kFirst) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int e = 0; e < 8; ++e) bsum[m] += static_cast<float>(A[m][e]);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) bsum[0] += j == 4 ? static_cast<float>(B[e]) : 0.0f;  // centre tap: g4[q]
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[m], B, acc[m], 0, 0, 0);
  }
  // [wave - 1][value][lane]: eight accumulator values, then the two bias sums
  __shared__ float other[kEdgeSplit - 1][10][64];
  if (wave > 0) {
#pragma unroll
    for (int v = 0; v < 8; ++v) other[wave - 1][v][l] = acc[v >> 2][v & 3];
    other[wave - 1][8][l] = bsum[0];
    other[wave - 1][9][l] = bsum[1];
  }
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int h = 0; h < kEdgeSplit - 1; ++h) {
#pragma unroll
    for (int v = 0; v < 8; ++v) acc[v >> 2][v & 3] += other[h][v][l];
    bsum[0] += other[h][8][l];
    bsum[1] += other[h][9][l];
  }
  float *dst = part + static_cast<size_t>(blockIdx.x) * NW;
  if (j < 9) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[(16 * m + 4 * gq + r) * 9 + j] = acc[m][r];
  }
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    float t = bsum[m];
    t += __shfl_xor(t, 16, 64);
    t += __shfl_xor(t, 32, 64);
    bsum[m] = t;
  }
  if constexpr (kFirst) {
    if (gq == 0) {
#pragma unroll
      for (int m = 0; m < 2; ++m) dst[kC * 9 + 16 * m + j] = bsum[m];
    }
  } else {
    if (l == 4) dst[kC * 9] = bsum[0];
  }
}

// Second stage: dW[k] = wscale * (sum over workgroups of part[w][k]) for the nw
// weights, db[k] likewise with bscale for the nb biases stored after them.  A
// workgroup reduces 64 consecutive entries; its kRedWaves waves take every
// kRedWaves-th partial row each (the loads of a lane are independent, so many are
// in flight), then add their sums in LDS: a fixed order, so the result is
// deterministic.
// kMidRows: the rows hold a 32 -> 32 layer's weights in mid_slot order.
inline constexpr int kRedWaves = 16;
template <bool kMidRows>
__global__ __launch_bounds__(64 * kRedWaves) void reduce_kernel(const float *__restrict__ part, int nwg, int nw,
                                                                int nb, float *__restrict__ dW,
                                                                float *__restrict__ db, float wscale, float bscale) {
  constexpr int kWaves = kRedWaves;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = nw + nb;
  const int k = blockIdx.x * 64 + lane;
  float acc = 0.0f;
  if (k < n) {
#pragma unroll 8
    for (int w = wave; w < nwg; w += kWaves) acc += part[static_cast<size_t>(w) * n + k];
  }
  __shared__ float sums[kWaves][64];
  sums[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && k < n) {
    float t = 0.0f;
#pragma unroll
    for (int j = 0; j < kWaves; ++j) t += sums[j][lane];
    if (k < nw)
      dW[kMidRows ? mid_weight_of_slot(k) : k] = t * wscale;
    else
      db[k - nw] = t * bscale;
  }
}

// ---------------------------------------------------------------------------
// Inference in one launch: the four layers of a tile with every activation in LDS
// ---------------------------------------------------------------------------
//
// A workgroup of kFThreads threads computes an output tile of kTW x kTH pixels
// of one image.  Each layer is computed on the region the next one reads (one
// pixel more on every side), so the tile's decoded pixels and activations never
// leave LDS and only the decoded and the output pixels touch HBM.  Positions
// outside the image hold zeros at every layer (the network's zero padding).
// Layer 3's results never reach LDS: the lane that forms them turns them into
// layer 4's per-tap sums at once (l4_sums), and the last phase adds each output
// pixel's nine sums.  Every layer runs on the matrix cores through the same
// functions as the one-layer kernels of the training pass (l1_pixel, relu_pack,
// l4_sums, l4_net), with the same operands in the same order, so the output is
// the rounding of the y those kernels form.
//
// Regions, in rows and columns relative to the tile's top-left output pixel:
//   a3  rows -1 .. 3 kG3 - 2, columns -1 .. 30  (kG3 row groups x two 16-column halves;
//       held only as layer 4's per-tap sums)
//   a2  rows -2 .. 3 kG2 - 3, columns -2 .. 31  (kG2 groups x two halves; columns 30, 31
//       are read only by a3 columns past the tile and are never written)
//   a1  rows -3 .. 3 kG2 - 2, columns -3 .. 30  (its kR1 x kC1 pixels in runs of 16)
//   P   rows -4 .., columns -4 .. 31 (the decoded pixels, FP16)
//
// Activations are stored pixel-major, 64 bytes per pixel, its four 16-byte
// channel groups G permuted within the pixel to slot G ^ ((C >> 1) & 3) for the
// pixel's column C in its region.  The LDS serves a 16-byte access eight lanes
// at a time over 32 four-byte banks; those lanes read eight consecutive columns
// of one row, two pixels share each 128-byte bank row, and the permutation puts
// the four pixels of each parity in different 16-byte bank ranges.  Since the permutation depends on the column only, a
// lane's address for row R is its row-0 address plus R times the row pitch, a
// constant offset of the LDS instruction.
//
// The tasks of the 32 -> 32 layers are (row group, half) pairs dealt to the
// waves in turn; with an even number of waves a wave always gets
// the same half, so its lane addresses are fixed for the whole launch.
inline constexpr int kTW = 28;                          // output columns of a tile
inline constexpr int kTH = 28;                          // output rows of a tile (3 kG3 - 2: no layer-3 row unused)
inline constexpr int kFThreads = 512;                   // eight waves
inline constexpr int kFWaves = kFThreads / 64;
static_assert(kFWaves % 2 == 0, "a wave keeps its half");
inline constexpr int kG3 = (kTH + 2 + kRows - 1) / kRows;      // a3 row groups
inline constexpr int kG2 = (3 * kG3 + 2 + kRows - 1) / kRows;  // a2 row groups (cover a3's rows +- 1)
inline constexpr int kR3 = 3 * kG3, kR2 = 3 * kG2, kR1 = kR2 + 2, kRX = kR1 + 2;  // rows held
static_assert(3 * kG3 == kTH + 2, "the tile height uses every layer-3 row the tile computes");
inline constexpr int kC2 = 34, kC1 = 34, kCX = 36;                                // columns held
inline constexpr int kLdsA1 = kR1 * kC1 * kC * 2;       // bytes; the layer-4 sums later reuse this space
inline constexpr int kLdsA2 = kR2 * kC2 * kC * 2;
inline constexpr int kLdsX = 2 * kRX * kCX * 2;            // two P tiles
// layer 4's per-tap sums of the a3 region: taps 0 .. 11 of kR3 rows x 32 columns
// (taps 9 .. 11 zero); the pitches put the 48 lanes of a store and 64
// consecutive output pixels of a gather in different banks
inline constexpr int kDTap = 36, kDRow = 12 * kDTap + 44;  // floats
static_assert(kR3 * kDRow * 4 <= kLdsA1, "the layer-4 sums fit in a1's space");
static_assert(kLdsA1 + kLdsA2 + kLdsX <= 160 * 1024, "the tile fits in one CU's LDS");

// byte offset of channel group G of the pixel with index q (row-major in its
// region) and column C
__device__ __forceinline__ int act_off(int q, int C, int G) { return q * 64 + 16 * (G ^ ((C >> 1) & 3)); }

// 32 -> 32 layer on a 16-pixel x kRows tile, operands from LDS.  `src` is the
// input region's row one above the tile's row 0 (kCin columns); rd[dx] is the
// lane's offset of its B operand at column offset dx in that row.  w[j][m] gets
// the lane's packed channels 16m + 4g .. + 3 of its pixel in tile row j: zero
// unless row_in[j] and col_in say the pixel lies in the image.
template <int kCin>
__device__ __forceinline__ void fused_mid_tile(const uint8_t *src, const int (&rd)[3], const h8 (&wa)[9][2],
                                               const f4 (&bias)[2], bool col_in, const bool (&row_in)[kRows],
                                               uint2 (&w)[kRows][2]) {
  f4 acc[kRows][2];
#pragma unroll
  for (int j = 0; j < kRows; ++j) acc[j][0] = bias[0], acc[j][1] = bias[1];
#pragma unroll
  for (int k = 0; k < kRows + 2; ++k) {
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const h8 bx = *reinterpret_cast<const h8 *>(src + rd[dx] + k * (kCin * 64));
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const int dy = k - j;
        if (dy >= 0 && dy <= 2) {
#pragma unroll
          for (int m = 0; m < 2; ++m)
            acc[j][m] = __builtin_amdgcn_mfma_f32_16x16x32_f16(wa[dy * 3 + dx][m], bx, acc[j][m], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kRows; ++j) {
    const bool in = col_in && row_in[j];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const uint2 v = relu_pack(acc[j][m]);
      w[j][m] = in ? v : make_uint2(0u, 0u);
    }
  }
}

// a mid layer's A operands (layer 0: W2, 1: W3) and biases for this lane, the
// bias of output half m as the addend of its sums (D row 4g + r = channel 16m + 4g + r)
__device__ __forceinline__ void load_mid_ops(const WeightOps *__restrict__ ops, int layer, h8 (&wa)[9][2],
                                             f4 (&bv)[2]) {
  const int l = threadIdx.x & 63, g = l >> 4;
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m) wa[t][m] = ops->mid[layer][m][t][l];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) bv[m][r] = ops->bias[layer + 1][16 * m + 4 * g + r];
}

// the P tile (decoded pixels on rows R0 - 4 .., columns C0 - 4 .., zero outside the
// image): this thread's entries tid + kFThreads e
inline constexpr int kXs = kRX * kCX;                                   // entries of a P tile
inline constexpr int kXsPer = (kXs + kFThreads - 1) / kFThreads;
__device__ __forceinline__ void fetch_p(const uint8_t *__restrict__ plane, int W, int H, int stride, int R0,
                                        int C0, uint32_t (&v)[kXsPer]) {
#pragma unroll
  for (int e = 0; e < kXsPer; ++e) {
    const int k = static_cast<int>(threadIdx.x) + kFThreads * e;
    const int rr = R0 - 4 + k / kCX, cc = C0 - 4 + k % kCX;
    v[e] = k < kXs && rr >= 0 && rr < H && cc >= 0 && cc < W ? plane[static_cast<size_t>(rr) * stride + cc] : 0u;
  }
}
__device__ __forceinline__ void store_p(_Float16 *xs, const uint32_t (&v)[kXsPer]) {
#pragma unroll
  for (int e = 0; e < kXsPer; ++e) {
    const int k = static_cast<int>(threadIdx.x) + kFThreads * e;
    if (k < kXs) xs[k] = static_cast<_Float16>(static_cast<float>(v[e]));
  }
}

// The deblocked output planes of n decoded W x H images stacked vertically in
// one plane (image k at rows k H .. k H + H - 1, pitch stride; each filtered on
// its own, with zeros outside it).  The tiles of all images form one list:
// each workgroup takes tiles blockIdx.x, + gridDim.x, ..., so the last round of
// one image's tiles does not leave CUs idle when more images follow.  The next
// tile's pixels are fetched while this one's middle layers run, into the other
// of two P buffers, and each layer's weights are loaded while the layer before
// it computes.
__global__ __launch_bounds__(kFThreads) void fused_apply_kernel(const uint8_t *__restrict__ plane, int W, int H,
                                                                int stride, int n, const WeightOps *__restrict__ ops,
                                                                uint8_t *__restrict__ out, int out_stride) {
  extern __shared__ __align__(16) uint8_t lds[];
  uint8_t *a1 = lds;
  float *dsum = reinterpret_cast<float *>(lds);  // layer 4's per-tap sums; a1 is dead once a2 is formed
  uint8_t *a2 = lds + kLdsA1;
  _Float16 *xbuf = reinterpret_cast<_Float16 *>(lds + kLdsA1 + kLdsA2);  // two P tiles
  const int tiles_x = (W + kTW - 1) / kTW, per_image = tiles_x * ((H + kTH - 1) / kTH), ntiles = per_image * n;
  // image of a tile and the tile's first row and column in that image
  auto origin = [&](int t, int &img, int &R0, int &C0) {
    img = t / per_image;
    const int lt = t - img * per_image;
    R0 = lt / tiles_x * kTH;
    C0 = lt % tiles_x * kTW;
  };
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l = tid & 63, i = l & 15, g = l >> 4;
  const int half = wave & 1;
  // the lane's offsets in a row of a region: B operands at columns 16 half + i + dx,
  // results at column 16 half + i (every region is addressed from its column 0)
  int rd[3], wr[2];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) {
    const int C = 16 * half + i + dx;
    rd[dx] = act_off(C, C, g);
  }
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int C = 16 * half + i;
    wr[m] = act_off(C, C, 2 * m + (g >> 1)) + 8 * (g & 1);
  }
  L1Consts k1;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    k1.wa[m] = *reinterpret_cast<const h4 *>(ops->l1[m][l]);
#pragma unroll
    for (int r = 0; r < 4; ++r) k1.bv[m][r] = ops->bias[0][16 * m + 4 * g + r];
  }
  // layer 1's tap offsets in the P tile for taps 4g + e (taps 9 .. 15 have zero
  // weights, so their B entries may read any P value)
  int toff[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int t = 4 * g + e;
    toff[e] = t < 9 ? t / 3 * kCX + t % 3 : 0;
  }
  int tile = static_cast<int>(blockIdx.x);
  if (tile >= ntiles) return;
  {
    uint32_t v[kXsPer];
    int img, r0, c0;
    origin(tile, img, r0, c0);
    fetch_p(plane + static_cast<size_t>(img) * H * stride, W, H, stride, r0, c0, v);
    store_p(xbuf, v);
  }
  __syncthreads();
  for (int cur = 0; tile < ntiles; tile += static_cast<int>(gridDim.x), cur ^= 1) {
    int img, R0, C0;
    origin(tile, img, R0, C0);
    const _Float16 *xs = xbuf + cur * kXs;
    h8 wa2[9][2];
    f4 bv2[2];
    load_mid_ops(ops, 0, wa2, bv2);
    {
      // layer 1 on the a1 region (row 0 = image row R0 - 3, column 0 = C0 - 3) in
      // runs of 16 pixels; tap t = (t / 3, t % 3) of a1 pixel (R, C) is P region
      // pixel (R + t / 3, C + t % 3).  Two runs per pass (u and u + kFWaves), their
      // loads issued together; a run past the region's end computes from clamped
      // positions and stores nothing.
      constexpr int kPx1 = kR1 * kC1, kRuns1 = (kPx1 + 15) / 16;
      for (int u0 = wave; u0 < kRuns1; u0 += 2 * kFWaves) {
        int q[2], R[2], C[2];
        h4 bp[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          q[h] = min(16 * (u0 + h * kFWaves) + i, kPx1 - 1);
          R[h] = static_cast<int>(static_cast<uint32_t>(q[h]) / static_cast<uint32_t>(kC1));
          C[h] = q[h] - R[h] * kC1;
          const _Float16 *px = xs + R[h] * kCX + C[h];
#pragma unroll
          for (int e = 0; e < 4; ++e) bp[h][e] = px[toff[e]];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          uint2 o[2];
          l1_pixel(k1, bp[h], o);
          if (16 * (u0 + h * kFWaves) + i < kPx1) {
            const int ir = R0 - 3 + R[h], ic = C0 - 3 + C[h];
            const bool in = static_cast<uint32_t>(ir) < static_cast<uint32_t>(H) &&
                            static_cast<uint32_t>(ic) < static_cast<uint32_t>(W);
#pragma unroll
            for (int m = 0; m < 2; ++m)
              *reinterpret_cast<uint2 *>(a1 + act_off(q[h], C[h], 2 * m + (g >> 1)) + 8 * (g & 1)) =
                  in ? o[m] : make_uint2(0u, 0u);
          }
        }
      }
    }
    __syncthreads();
    // the next tile's pixels, in flight through layers 2 and 3
    const int next = tile + static_cast<int>(gridDim.x);
    uint32_t pv[kXsPer];
    if (next < ntiles) {
      int nimg, nr0, nc0;
      origin(next, nimg, nr0, nc0);
      fetch_p(plane + static_cast<size_t>(nimg) * H * stride, W, H, stride, nr0, nc0, pv);
    }
    h8 wa3[9][2];
    f4 bv3[2];
    load_mid_ops(ops, 1, wa3, bv3);
    {
      // layer 2: a2 rows -2 .., columns -2 .. 29 from a1 (a1 region row 0 = image row
      // R0 - 3; a2 region row 0 = image row R0 - 2, column 0 = C0 - 2)
      const bool col_in = static_cast<uint32_t>(C0 - 2 + 16 * half + i) < static_cast<uint32_t>(W);
      for (int grp = wave >> 1; grp < kG2; grp += kFWaves / 2) {
        const int ro = grp * kRows;
        bool row_in[kRows];
#pragma unroll
        for (int j = 0; j < kRows; ++j) row_in[j] = static_cast<uint32_t>(R0 - 2 + ro + j) < static_cast<uint32_t>(H);
        uint2 w[kRows][2];
        fused_mid_tile<kC1>(a1 + ro * (kC1 * 64), rd, wa2, bv2, col_in, row_in, w);
        uint8_t *dst = a2 + ro * (kC2 * 64);
#pragma unroll
        for (int j = 0; j < kRows; ++j)
#pragma unroll
          for (int m = 0; m < 2; ++m) *reinterpret_cast<uint2 *>(dst + wr[m] + j * (kC2 * 64)) = w[j][m];
      }
    }
    __syncthreads();
    const h8 wa4 = ops->l4[l];
    const float b4 = ops->b4;
    {
      // layer 3: a3 rows -1 .., columns -1 .. 30 from a2 (a3 region row 0 = image row
      // R0 - 1, column 0 = C0 - 1)
      const bool col_in = static_cast<uint32_t>(C0 - 1 + 16 * half + i) < static_cast<uint32_t>(W);
      for (int grp = wave >> 1; grp < kG3; grp += kFWaves / 2) {
        const int ro = grp * kRows;
        bool row_in[kRows];
#pragma unroll
        for (int j = 0; j < kRows; ++j) row_in[j] = static_cast<uint32_t>(R0 - 1 + ro + j) < static_cast<uint32_t>(H);
        uint2 w[kRows][2];
        fused_mid_tile<kC2>(a2 + ro * (kC2 * 64), rd, wa3, bv3, col_in, row_in, w);
        // layer 4's per-tap sums of these a3 pixels, taps 4g .. 4g + 3 in lane (i, g)
        float *drow = dsum + ro * kDRow + 4 * g * kDTap + 16 * half + i;
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
          const f4 d = l4_sums(wa4, w[j][0], w[j][1]);
          if (g < 3) {
#pragma unroll
            for (int r = 0; r < 4; ++r) drow[j * kDRow + r * kDTap] = d[r];
          }
        }
      }
    }
    if (next < ntiles) store_p(xbuf + (cur ^ 1) * kXs, pv);
    __syncthreads();
    // layer 4: each output pixel adds its nine per-tap sums (a3 region row 0 =
    // image row R0 - 1, column 0 = C0 - 1, so output (r, c) takes tap (dy, dx) at
    // a3 pixel (r + dy, c + dx))
    for (int q = tid; q < kTW * kTH; q += kFThreads) {
      const int r = q / kTW, c = q - r * kTW;
      const float *src = dsum + r * kDRow + c;
      const float net = l4_net([&](int dy, int dx, int t) { return src[dy * kDRow + t * kDTap + dx]; });
      const int ir = R0 + r, ic = C0 + c;
      if (ir < H && ic < W) {
        const float y = residual(static_cast<float>(xs[(r + 4) * kCX + c + 4]), net + b4);
        const float v = fminf(fmaxf(floorf(255.0f * y + 0.5f), 0.0f), 255.0f);
        out[(static_cast<size_t>(img) * H + ir) * out_stride + ic] = static_cast<uint8_t>(v);
      }
    }
    __syncthreads();
  }
}

// Adam with bias correction (c1 = 1 - b1^step, c2 = 1 - b2^step from the host);
// refreshes the FP16-rounded copies.
__global__ __launch_bounds__(kThreads) void adam_kernel(float *__restrict__ p, float *__restrict__ m,
                                                        float *__restrict__ v, const float *__restrict__ g, int n,
                                                        float lr, float b1, float b2, float eps, float c1, float c2) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k < n) {
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  }
}

// loss = inv_n * (sum of the n per-workgroup partial sums), added in a fixed order
__global__ __launch_bounds__(kThreads) void loss_reduce_kernel(const double *__restrict__ sq, int n,
                                                               double *__restrict__ loss, double inv_n) {
  double t = 0.0;
  for (int k = threadIdx.x; k < n; k += kThreads) t += sq[k];
  __shared__ double part[kThreads];
  part[threadIdx.x] = t;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0] * inv_n;
}

// Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and Shaw
// ("Parallel random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of two
// 32 x 32 -> 64-bit products with the multipliers 0xD2511F53 and 0xCD9E8D57,
// the key bumped by the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x, p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
    c = make_uint4(static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0, static_cast<uint32_t>(p1),
                   static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1, static_cast<uint32_t>(p0));
  }
  return c;
}

// Initial parameters: He-normal weights N(0, 2 / (9 C_in)) for the three ReLU
// layers, zero biases and a zero output layer, so that the untrained filter is
// the identity.  Weight k draws counter (k, 0, 0, 0) under key (seed low word,
// seed high word); the first two words give u1 = (x0 + 1) 2^-32 in (0, 1] and
// u2 = x1 2^-32, and the Box-Muller transform sqrt(-2 ln u1) cos(2 pi u2) the
// standard normal value (computed in double, stored as float).
__global__ __launch_bounds__(kThreads) void init_kernel(float *__restrict__ p, uint32_t k0, uint32_t k1) {
  const int k = blockIdx.x * kThreads + threadIdx.x;
  if (k >= kNParam) return;
  double sd = 0.0;
  if (k < kB1)
    sd = 2.0 / 9.0;
  else if ((k >= kW2 && k < kB2) || (k >= kW3 && k < kB3))
    sd = 2.0 / (9.0 * kC);
  float v = 0.0f;
  if (sd > 0.0) {
    const uint4 x = philox4x32_10(make_uint4(static_cast<uint32_t>(k), 0u, 0u, 0u), k0, k1);
    const double u1 = (static_cast<double>(x.x) + 1.0) * 0x1p-32, u2 = static_cast<double>(x.y) * 0x1p-32;
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
    v = static_cast<float>(sqrt(sd) * z);
  }
  p[k] = v;
}

// Zero the output layer (W4, b4) of a parameter array: the filter then returns
// its input bit for bit.
__global__ __launch_bounds__(kThreads) void zero_output_layer_kernel(float *__restrict__ p) {
  const int k = kW4 + static_cast<int>(blockIdx.x * kThreads + threadIdx.x);
  if (k < kNParam) p[k] = 0.0f;
}

}  // namespace db
}  // namespace dct
