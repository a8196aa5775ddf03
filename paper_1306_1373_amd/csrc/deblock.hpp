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
// 64 contiguous bytes (FP16) or 128 bytes (FP32 gradients).  Pixels are numbered
// image by image, row-major.  An "image set" is n images of h x w whose top-left
// corners sit at given (row, col) positions of one uint8 plane (training crops),
// or one image at the origin (inference).
//
// Kernels (one thread per pixel unless stated):
//   layer1_kernel      x -> a1 (VALU, 288 FMA per pixel)
//   mid_kernel         a -> relu(conv(a)) for the 32 -> 32 layers on the matrix
//                      cores: per wave, 16 pixels x 32 output channels, K = 9 taps
//                      x 32 input channels as nine v_mfma_f32_16x16x32_f16 per
//                      16-channel half; lane (i, g) loads 8 channels (16 bytes)
//                      of its pixel's neighbour and gets 4 output channels.
//   layer4_kernel      a3 -> y, and either the output pixel or the loss terms and
//                      dL/dy (training)
//   bwd4_kernel        dL/da3 through layer 4 and the ReLU of a3
//   bwd_mid_kernel     dL/da through a 32 -> 32 layer and the ReLU of its input
//   wgrad_kernel       weight and bias gradients of a layer, first stage: each
//                      workgroup sums its pixels' products into a partial row
//   reduce_kernel      second stage: adds the partial rows (no atomics)
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

// pixel rows a thread (layers 1 and 4) or a wave's tile (layers 2 and 3) computes
inline constexpr int kRows = 3;

// a1 = relu(conv(x; W1, b1))
__global__ __launch_bounds__(kThreads) void layer1_kernel(ImageSet s, const float *__restrict__ wq,
                                                          _Float16 *__restrict__ a1, int64_t ngroups) {
  // a thread computes kRows vertically adjacent pixels of one column: the
  // (kRows + 2) x 3 neighbourhood is read and converted once for all of them
  const uint32_t row_groups = (static_cast<uint32_t>(s.h) + kRows - 1u) / kRows;
  for (int64_t gidx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; gidx < ngroups;
       gidx += static_cast<int64_t>(gridDim.x) * kThreads) {
    const uint32_t u = static_cast<uint32_t>(gidx);
    const uint32_t col_id = u / static_cast<uint32_t>(s.w);
    const int c = static_cast<int>(u - col_id * static_cast<uint32_t>(s.w));
    const int b = static_cast<int>(col_id / row_groups);
    const int r0 = static_cast<int>(col_id - static_cast<uint32_t>(b) * row_groups) * kRows;
    float x[kRows + 2][3];
#pragma unroll
    for (int k = 0; k < kRows + 2; ++k)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) x[k][dx] = plane_px(s, s.plane, b, r0 - 1 + k, c + dx - 1) * kInv255;
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int r = r0 + j;
      if (r >= s.h) break;
      uint32_t words[kC / 2];
#pragma unroll
      for (int co = 0; co < kC; ++co) {
        float acc = wq[kB1 + co];
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += wq[kW1 + co * 9 + t] * x[j + t / 3][t % 3];
        const uint32_t hbits = __builtin_bit_cast(uint16_t, static_cast<_Float16>(fmaxf(acc, 0.0f)));
        words[co >> 1] = (co & 1) ? (words[co >> 1] | (hbits << 16)) : hbits;
      }
      const int64_t p = (static_cast<int64_t>(b) * s.h + r) * s.w + c;
      uint4 *dst = reinterpret_cast<uint4 *>(a1 + p * kC);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        dst[k] = make_uint4(words[4 * k], words[4 * k + 1], words[4 * k + 2], words[4 * k + 3]);
    }
  }
}

// aout = relu(conv(ain; W, b)) for a 32 -> 32 layer on the matrix cores.
// Operands of v_mfma_f32_16x16x32_f16 for tap t and output half m (lane i, g):
//   A[i][8g+e] = W[16m + i][8g + e][t], B[8g+e][i] = ain[neighbour t of pixel i][8g + e],
//   D[4g+r][i] = output channel 16m + 4g + r of pixel i.
// A wave computes kRows vertically adjacent tiles of 16 pixels (rows r0 .. r0 +
// kRows - 1, columns c0 .. c0 + 15 of one image): each of the kRows + 2 input rows
// x 3 column offsets is loaded once and feeds every output row whose 3x3 window
// covers it, so a tile needs (kRows + 2) * 3 / kRows loads instead of 9.  The
// image, row and column of a tile are the same for the whole wave.
__global__ __launch_bounds__(kThreads) void mid_kernel(ImageSet s, const _Float16 *__restrict__ ain,
                                                       const _Float16 *__restrict__ wh_layer,
                                                       const float *__restrict__ bias,
                                                       _Float16 *__restrict__ aout, int64_t npix, int64_t ntiles) {
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
  const int l = threadIdx.x & 63, i = l & 15, g = l >> 4;
  h8 wa[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int e = 0; e < 8; ++e) wa[t][m][e] = wh_layer[((16 * m + i) * kC + 8 * g + e) * 9 + t];
  float bv[2][4];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) bv[m][r] = bias[16 * m + 4 * g + r];
  const uint32_t col_tiles = (static_cast<uint32_t>(s.w) + 15u) / 16u;
  const uint32_t row_groups = (static_cast<uint32_t>(s.h) + kRows - 1u) / kRows;
  const uint32_t step = gridDim.x * (kThreads / 64);
  for (uint32_t tile = blockIdx.x * (kThreads / 64) + wave; tile < static_cast<uint32_t>(ntiles); tile += step) {
    const uint32_t gid = tile / col_tiles;  // (image, row group) over the whole set
    const int b = static_cast<int>(gid / row_groups);
    const int r0 = static_cast<int>(gid - static_cast<uint32_t>(b) * row_groups) * kRows;
    const int c = static_cast<int>((tile - gid * col_tiles) * 16u) + i;
    f4 acc[kRows][2];
#pragma unroll
    for (int j = 0; j < kRows; ++j) acc[j][0] = acc[j][1] = f4{0.f, 0.f, 0.f, 0.f};
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
          uint32_t hb[4];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            hb[q] = __builtin_bit_cast(uint16_t, static_cast<_Float16>(fmaxf(acc[j][m][q] + bv[m][q], 0.0f)));
          *reinterpret_cast<uint2 *>(aout + p * kC + 16 * m + 4 * g) =
              make_uint2(hb[0] | (hb[1] << 16), hb[2] | (hb[3] << 16));
        }
      }
    }
  }
}

// y = x + conv(a3; W4, b4).  kTrain = false: writes the output pixel to `out`
// (clamp(floor(255 y + 1/2))).  kTrain = true: y to y_out (if not null),
// dL/dy = grad_scale (y - t) to g4, and the sum of (y - t)^2 to *sq (one atomic
// per wave).  A thread computes kRows vertically adjacent pixels of one column:
// each of the kRows + 2 neighbour rows x 3 columns is loaded and converted once.
template <bool kTrain>
__global__ __launch_bounds__(kThreads) void layer4_kernel(ImageSet s, const _Float16 *__restrict__ a3,
                                                          const float *__restrict__ wq, int64_t ngroups,
                                                          uint8_t *__restrict__ out, int out_stride,
                                                          float *__restrict__ y_out, float *__restrict__ g4,
                                                          double *__restrict__ sq, float grad_scale) {
  double local = 0.0;
  const uint32_t row_groups = (static_cast<uint32_t>(s.h) + kRows - 1u) / kRows;
  for (int64_t gidx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; gidx < ngroups;
       gidx += static_cast<int64_t>(gridDim.x) * kThreads) {
    // group id -> (image, row group, column)
    const uint32_t u = static_cast<uint32_t>(gidx);
    const uint32_t col_id = u / static_cast<uint32_t>(s.w);
    const int c = static_cast<int>(u - col_id * static_cast<uint32_t>(s.w));
    const int b = static_cast<int>(col_id / row_groups);
    const int r0 = static_cast<int>(col_id - static_cast<uint32_t>(b) * row_groups) * kRows;
    float acc[kRows];
#pragma unroll
    for (int j = 0; j < kRows; ++j) acc[j] = wq[kB4];
#pragma unroll
    for (int k = 0; k < kRows + 2; ++k) {  // input row r0 - 1 + k
      const int rr = r0 - 1 + k;
      if (rr < 0 || rr >= s.h) continue;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int cc = c + dx - 1;
        if (cc < 0 || cc >= s.w) continue;
        const uint4 *src = reinterpret_cast<const uint4 *>(a3 + ((static_cast<int64_t>(b) * s.h + rr) * s.w + cc) * kC);
        float av[kC];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const h8 hv = __builtin_bit_cast(h8, src[q]);
#pragma unroll
          for (int e = 0; e < 8; ++e) av[8 * q + e] = static_cast<float>(hv[e]);
        }
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
          const int dy = k - j;  // tap row of output row r0 + j
          if (dy >= 0 && dy <= 2) {
#pragma unroll
            for (int ci = 0; ci < kC; ++ci) acc[j] += wq[kW4 + ci * 9 + dy * 3 + dx] * av[ci];
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kRows; ++j) {
      const int r = r0 + j;
      if (r >= s.h) break;
      const float y = plane_px(s, s.plane, b, r, c) * kInv255 + acc[j];
      const int64_t p = (static_cast<int64_t>(b) * s.h + r) * s.w + c;
      if constexpr (!kTrain) {
        const float v = fminf(fmaxf(floorf(255.0f * y + 0.5f), 0.0f), 255.0f);
        out[static_cast<size_t>(r) * out_stride + c] = static_cast<uint8_t>(v);
      } else {
        const float e = y - plane_px(s, s.orig, b, r, c) * kInv255;
        if (y_out) y_out[p] = y;
        g4[p] = grad_scale * e;
        local += static_cast<double>(e) * e;
      }
    }
  }
  if constexpr (kTrain) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) local += __shfl_xor(local, off, 64);
    if ((threadIdx.x & 63) == 0 && local != 0.0) atomicAdd(sq, local);
  }
}

// g3 = (a3 > 0) * dL/da3, dL/da3[q][ci] = sum_t W4[ci][t] g4[q - offset(t)]
__global__ __launch_bounds__(kThreads) void bwd4_kernel(ImageSet s, const float *__restrict__ g4,
                                                        const _Float16 *__restrict__ a3,
                                                        const float *__restrict__ wq, float *__restrict__ g3,
                                                        int64_t npix) {
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; p < npix;
       p += static_cast<int64_t>(gridDim.x) * kThreads) {
    const Pix q = pix_of(s, p);
    float gv[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int64_t nb = nb_id(s, q, 1 - t / 3, 1 - t % 3);
      gv[t] = nb >= 0 ? g4[nb] : 0.0f;
    }
    const _Float16 *ap = a3 + p * kC;
    float4 *dst = reinterpret_cast<float4 *>(g3 + p * kC);
#pragma unroll
    for (int k = 0; k < kC / 4; ++k) {
      float o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ci = 4 * k + j;
        float acc = 0.0f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc += wq[kW4 + ci * 9 + t] * gv[t];
        o[j] = static_cast<float>(ap[ci]) > 0.0f ? acc : 0.0f;
      }
      dst[k] = make_float4(o[0], o[1], o[2], o[3]);
    }
  }
}

// gin = (ain > 0) * dL/dain through a 32 -> 32 layer:
//   dL/dain[q][ci] = sum_t sum_co W[co][ci][t] gout[q - offset(t)][co]
__global__ __launch_bounds__(kThreads) void bwd_mid_kernel(ImageSet s, const float *__restrict__ gout,
                                                           const _Float16 *__restrict__ ain,
                                                           const float *__restrict__ wq_layer,
                                                           float *__restrict__ gin, int64_t npix) {
  __shared__ float wl[kC * kC * 9];  // [t][co][ci]
  for (int k = threadIdx.x; k < kC * kC * 9; k += kThreads) {
    const int t = k / (kC * kC), co = (k / kC) % kC, ci = k % kC;
    wl[k] = wq_layer[(co * kC + ci) * 9 + t];
  }
  __syncthreads();
  for (int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; p < npix;
       p += static_cast<int64_t>(gridDim.x) * kThreads) {
    const Pix q = pix_of(s, p);
    float acc[kC];
#pragma unroll
    for (int ci = 0; ci < kC; ++ci) acc[ci] = 0.0f;
    for (int t = 0; t < 9; ++t) {
      const int64_t nb = nb_id(s, q, 1 - t / 3, 1 - t % 3);
      if (nb < 0) continue;
      const float4 *gp = reinterpret_cast<const float4 *>(gout + nb * kC);
      for (int c4 = 0; c4 < kC / 4; ++c4) {
        const float4 gg = gp[c4];
        const float gvals[4] = {gg.x, gg.y, gg.z, gg.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float *wrow = wl + (t * kC + 4 * c4 + j) * kC;
#pragma unroll
          for (int ci = 0; ci < kC; ++ci) acc[ci] += wrow[ci] * gvals[j];
        }
      }
    }
    const _Float16 *ap = ain + p * kC;
    float4 *dst = reinterpret_cast<float4 *>(gin + p * kC);
#pragma unroll
    for (int k = 0; k < kC / 4; ++k) {
      float o[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] = static_cast<float>(ap[4 * k + j]) > 0.0f ? acc[4 * k + j] : 0.0f;
      dst[k] = make_float4(o[0], o[1], o[2], o[3]);
    }
  }
}

// Weight and bias gradients of one layer, first stage:
//   dW[co][ci][t] = sum_p gout[p][co] in[p + offset(t)][ci],  db[co] = sum_p gout[p][co],
// with `in` the FP16 activations (CI = 32) or the decoded plane / 255 (CI = 1).
// Workgroup w sums `per_wg` consecutive pixels and writes its partial sums to
// part[w][0 .. CO CI 9 + CO) (weights, then biases); reduce_kernel adds the
// partials of all workgroups.  Thread k owns co = k / GROUPS and CPT = CI / GROUPS
// input channels.
template <int CI, int CO>
__global__ __launch_bounds__(kThreads) void wgrad_kernel(ImageSet s, const float *__restrict__ gout,
                                                         const _Float16 *__restrict__ ain, float *__restrict__ part,
                                                         int64_t npix, int per_wg) {
  constexpr int GROUPS = CI >= 4 ? (kThreads / CO < CI / 4 ? kThreads / CO : CI / 4) : 1;
  constexpr int CPT = CI / GROUPS;
  constexpr int NW = CO * CI * 9 + CO;
  static_assert(CO * GROUPS <= kThreads, "one thread per (co, group)");
  const int k = threadIdx.x;
  const bool active = k < CO * GROUPS;
  const int co = active ? k / GROUPS : 0, grp = active ? k % GROUPS : 0;
  float acc[CPT][9];
  float accb = 0.0f;
#pragma unroll
  for (int j = 0; j < CPT; ++j)
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[j][t] = 0.0f;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * per_wg;
  const int64_t p1 = p0 + per_wg < npix ? p0 + per_wg : npix;
  if (active) {
    for (int64_t p = p0; p < p1; ++p) {
      const float gv = gout[p * CO + co];
      accb += gv;
      const Pix q = pix_of(s, p);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        if constexpr (CI == 1) {
          acc[0][t] += gv * plane_px(s, s.plane, q.b, q.r + t / 3 - 1, q.c + t % 3 - 1) * kInv255;
        } else {
          const int64_t nb = nb_id(s, q, t / 3 - 1, t % 3 - 1);
          if (nb >= 0) {
            const _Float16 *ap = ain + nb * CI + grp * CPT;
#pragma unroll
            for (int j = 0; j < CPT; ++j) acc[j][t] += gv * static_cast<float>(ap[j]);
          }
        }
      }
    }
    float *dst = part + static_cast<size_t>(blockIdx.x) * NW;
#pragma unroll
    for (int j = 0; j < CPT; ++j)
#pragma unroll
      for (int t = 0; t < 9; ++t) dst[(co * CI + grp * CPT + j) * 9 + t] = acc[j][t];
    if (grp == 0) dst[CO * CI * 9 + co] = accb;
  }
}

// Second stage: dW[k] = sum over workgroups of part[w][k] for the nw weights,
// db[k] likewise for the nb biases stored after them.  A workgroup reduces 64
// consecutive entries; its four waves take every fourth partial row each (the
// loads of a lane are independent, so many are in flight), then add their
// four sums in LDS.
__global__ __launch_bounds__(kThreads) void reduce_kernel(const float *__restrict__ part, int nwg, int nw, int nb,
                                                          float *__restrict__ dW, float *__restrict__ db) {
  constexpr int kWaves = kThreads / 64;
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
      dW[k] = t;
    else
      db[k - nw] = t;
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

__global__ __launch_bounds__(kThreads) void zero_f32_kernel(float *__restrict__ a, int64_t n) {
  for (int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; k < n;
       k += static_cast<int64_t>(gridDim.x) * kThreads)
    a[k] = 0.0f;
}

__global__ void mean_kernel(const double *__restrict__ sq, double *__restrict__ loss, double inv_n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *loss = *sq * inv_n;
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
