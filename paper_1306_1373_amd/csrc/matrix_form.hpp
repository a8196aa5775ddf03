// matrix_form.hpp -- floating-point forms of the 8x8 DCT codec.
//
// The exact DCT the paper compares its Cordic-based Loeffler codec against
// (Sec. 4.1, Tables 3-4, the "DCT" rows) computed in floating point on the GPU:
//
//   * kFormF32Loeffler: the same four-stage Loeffler graph (Sec. 2.5.2) in FP32
//     with exact rotation constants; one lane per block, like the integer codec.
//   * kFormMfmaF16 / kFormMfmaBf16: the 2-D DCT-II of eq. (6) as one matrix
//     product per block, vec(F) = (C (x) C) vec(X) with C the orthonormal 8-point
//     DCT-II matrix, batched over blocks into a GEMM [blocks x 64] x [64 x 64] on
//     the matrix cores (v_mfma_f32_16x16x32_f16 / _bf16): pixels X = p - 128 and
//     C (x) C rounded once to FP16 or BF16, products accumulated in FP32.  The
//     inverse is the transposed product with the same matrix.
//
// Every form runs the same codec around its transform: quantize
// q = sgn(F) floor(|F| / Q + 1/2) with Q[u][v] = 1 + (1 + u + v) qs, dequantize
// q Q, inverse transform, reconstruct clamp(floor(x + 128 + 1/2), 0, 255), SSE.
// These results are within stated tolerances of the FP64 definition, not bit
// for bit: a coefficient whose exact value lies within the form's error of a
// quantizer tie may quantize to either side.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "recipe.hpp"

namespace dct {

enum Form : int { kFormF32Loeffler = 1, kFormMfmaF16 = 2, kFormMfmaBf16 = 3 };

namespace mf {

constexpr double cosine(double x) {
  const double pi = detail::kPi;
  while (x > pi) x -= 2 * pi;
  while (x < -pi) x += 2 * pi;
  double t = 1.0, s = 1.0;
  const double x2 = x * x;
  for (int k = 1; k < 30; ++k) {
    t *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    s += t;
  }
  return s;
}

constexpr double sine(double x) { return cosine(x - detail::kPi / 2); }

// orthonormal 8-point DCT-II matrix C[u][i] = alpha(u) sqrt(2/8) cos((2i+1) u pi / 16)
constexpr double basis(int u, int i) {
  return (u == 0 ? detail::sqrt_newton(0.125) : 0.5) * cosine((2 * i + 1) * u * detail::kPi / 16.0);
}

// round-to-nearest-even of a normal double to the bits of a binary16 / bfloat16
constexpr uint16_t round_bits(double v, int frac_bits, int bias) {
  const uint16_t sign = v < 0 ? 0x8000 : 0;
  if (v < 0) v = -v;
  int e = 0;
  while (v >= 2.0) {
    v /= 2.0;
    ++e;
  }
  while (v < 1.0) {
    v *= 2.0;
    --e;
  }
  const double one = static_cast<double>(1LL << frac_bits);
  const double sc = v * one;
  long long m = static_cast<long long>(sc);
  const double fr = sc - static_cast<double>(m);
  if (fr > 0.5 || (fr == 0.5 && (m & 1))) ++m;
  if (m == 2 * (1LL << frac_bits)) {
    m = 1LL << frac_bits;
    ++e;
  }
  return static_cast<uint16_t>(sign | ((e + bias) << frac_bits) | (m - (1LL << frac_bits)));
}

// K[j][k] = C[u][i] C[v][jj] with j = 8u + v (coefficient), k = 8i + jj (pixel)
struct KTable {
  uint16_t v[64 * 64];
};

template <bool kBf16>
constexpr KTable make_k() {
  KTable t{};
  for (int j = 0; j < 64; ++j)
    for (int k = 0; k < 64; ++k) {
      const double val = basis(j / 8, k / 8) * basis(j % 8, k % 8);
      t.v[j * 64 + k] = kBf16 ? round_bits(val, 7, 127) : round_bits(val, 10, 15);
    }
  return t;
}

// FP32 constants of the Loeffler graph with exact rotations
struct LoefflerConsts {
  float c1, s1, c3, s3, c6r2, s6r2, r2;
};

constexpr LoefflerConsts make_loeffler() {
  const double pi = detail::kPi, r2 = detail::sqrt_newton(2.0);
  return {static_cast<float>(cosine(pi / 16)),       static_cast<float>(sine(pi / 16)),
          static_cast<float>(cosine(3 * pi / 16)),   static_cast<float>(sine(3 * pi / 16)),
          static_cast<float>(r2 * cosine(6 * pi / 16)), static_cast<float>(r2 * sine(6 * pi / 16)),
          static_cast<float>(r2)};
}

}  // namespace mf

__device__ constexpr mf::KTable kKronF16 = mf::make_k<false>();
__device__ constexpr mf::KTable kKronBf16 = mf::make_k<true>();
inline constexpr mf::LoefflerConsts kLf = mf::make_loeffler();

// Quantizer of the floating-point forms: the table entries and their reciprocals,
// indexed by s = u + v.
struct FloatQuant {
  float Q[15];
  float rcp[15];  // 1/Q rounded to nearest
};

// q = sgn(F) floor(|F| / Q + 1/2); returns the dequantized q Q
__device__ __forceinline__ float fquant(float F, float Q, float rcp) {
  const float q = __builtin_floorf(__builtin_fabsf(F) * rcp + 0.5f);
  return __builtin_copysignf(q * Q, F);
}

// clamp(floor(x + 128 + 1/2), 0, 255)
__device__ __forceinline__ uint32_t freconstruct(float x) {
  const float p = __builtin_floorf(x + 128.5f);
  return static_cast<uint32_t>(__builtin_fminf(__builtin_fmaxf(p, 0.0f), 255.0f));
}

// ---------------------------------------------------------------------------
// FP32 Loeffler form (one lane per block)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void frot(float &a, float &b, float c, float s) {
  const float x = a, y = b;
  a = x * c + y * s;
  b = y * c - x * s;
}

template <bool kRows>
__device__ __forceinline__ float &fat(float (&x)[64], int line, int k) {
  return kRows ? x[line * 8 + k] : x[k * 8 + line];
}

template <bool kRows>
__device__ __forceinline__ void floeffler_fwd(float (&x)[64]) {
#pragma unroll
  for (int L = 0; L < 8; ++L) {
    const float s0 = fat<kRows>(x, L, 0) + fat<kRows>(x, L, 7), d0 = fat<kRows>(x, L, 0) - fat<kRows>(x, L, 7);
    const float s1 = fat<kRows>(x, L, 1) + fat<kRows>(x, L, 6), d1 = fat<kRows>(x, L, 1) - fat<kRows>(x, L, 6);
    const float s2 = fat<kRows>(x, L, 2) + fat<kRows>(x, L, 5), d2 = fat<kRows>(x, L, 2) - fat<kRows>(x, L, 5);
    const float s3 = fat<kRows>(x, L, 3) + fat<kRows>(x, L, 4), d3 = fat<kRows>(x, L, 3) - fat<kRows>(x, L, 4);
    const float e0 = s0 + s3, e3 = s0 - s3, e1 = s1 + s2;
    float e2 = s1 - s2, e3r = e3;
    float u4 = d3, u7 = d0, u5 = d2, u6 = d1;
    frot(u4, u7, kLf.c3, kLf.s3);
    frot(u5, u6, kLf.c1, kLf.s1);
    frot(e2, e3r, kLf.c6r2, kLf.s6r2);
    const float v4 = u4 + u6, v6 = u4 - u6, v7 = u7 + u5, v5 = u7 - u5;
    fat<kRows>(x, L, 0) = e0 + e1;
    fat<kRows>(x, L, 4) = e0 - e1;
    fat<kRows>(x, L, 2) = e2;
    fat<kRows>(x, L, 6) = e3r;
    fat<kRows>(x, L, 1) = v7 + v4;
    fat<kRows>(x, L, 7) = v7 - v4;
    fat<kRows>(x, L, 3) = kLf.r2 * v5;
    fat<kRows>(x, L, 5) = kLf.r2 * v6;
  }
}

template <bool kRows>
__device__ __forceinline__ void floeffler_inv(float (&x)[64]) {
#pragma unroll
  for (int L = 0; L < 8; ++L) {
    const float z0 = fat<kRows>(x, L, 0), z1 = fat<kRows>(x, L, 1), z4 = fat<kRows>(x, L, 4), z7 = fat<kRows>(x, L, 7);
    const float v7 = z1 + z7, v4 = z1 - z7, v5 = kLf.r2 * fat<kRows>(x, L, 3), v6 = kLf.r2 * fat<kRows>(x, L, 5);
    const float e0 = z0 + z4, e1 = z0 - z4;
    float e2 = fat<kRows>(x, L, 2), e3 = fat<kRows>(x, L, 6);
    frot(e2, e3, kLf.c6r2, -kLf.s6r2);
    float u4 = v4 + v6, u6 = v4 - v6, u7 = v7 + v5, u5 = v7 - v5;
    frot(u4, u7, kLf.c3, -kLf.s3);
    frot(u5, u6, kLf.c1, -kLf.s1);
    const float s0 = e0 + e3, s3 = e0 - e3, s1 = e1 + e2, s2 = e1 - e2;
    fat<kRows>(x, L, 0) = s0 + u7;
    fat<kRows>(x, L, 7) = s0 - u7;
    fat<kRows>(x, L, 1) = s1 + u6;
    fat<kRows>(x, L, 6) = s1 - u6;
    fat<kRows>(x, L, 2) = s2 + u5;
    fat<kRows>(x, L, 5) = s2 - u5;
    fat<kRows>(x, L, 3) = s3 + u4;
    fat<kRows>(x, L, 4) = s3 - u4;
  }
}

// kCodec = false: write FP32 orthonormal coefficients; true: whole codec + SSE
template <bool kCodec>
__global__ __launch_bounds__(kWg) void loeffler_f32_kernel(const uint8_t *__restrict__ src, int W, int H, int stride,
                                                          int bw, int nblocks, float *__restrict__ coef,
                                                          FloatQuant fq, uint8_t *__restrict__ dst, int dst_stride,
                                                          unsigned long long *__restrict__ sse) {
  const int b = blockIdx.x * kWg + threadIdx.x;
  const BlockPos p = block_pos(b, W, H, bw, nblocks);
  uint32_t pix[16] = {};
  if (p.live) load_block(src, W, H, stride, p.by, p.bx, p.full, pix);
  float x[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) x[k] = static_cast<float>(static_cast<int>((pix[k >> 2] >> (8 * (k & 3))) & 0xffu) - 128);
  floeffler_fwd<true>(x);
  floeffler_fwd<false>(x);
#pragma unroll
  for (int k = 0; k < 64; ++k) x[k] *= 0.125f;  // two passes scale by 8
  if constexpr (!kCodec) {
    if (p.live) {
      float4 *out = reinterpret_cast<float4 *>(coef + static_cast<size_t>(b) * 64);
#pragma unroll
      for (int k = 0; k < 16; ++k) out[k] = make_float4(x[4 * k], x[4 * k + 1], x[4 * k + 2], x[4 * k + 3]);
    }
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = 0; v < 8; ++v) x[u * 8 + v] = fquant(x[u * 8 + v], fq.Q[u + v], fq.rcp[u + v]);
    floeffler_inv<false>(x);
    floeffler_inv<true>(x);
    uint32_t rec[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      uint32_t w = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) w |= freconstruct(x[4 * k + j] * 0.125f) << (8 * j);
      rec[k] = w;
    }
    uint32_t err = 0;
    if (p.live) {
      store_block(dst, W, H, dst_stride, p.by, p.bx, p.full, rec);
      err = block_sse(pix, rec, W, H, p.by, p.bx, p.full);
    }
    workgroup_add<kWg>(err, sse);
  }
}

// ---------------------------------------------------------------------------
// Kronecker form on the matrix cores
// ---------------------------------------------------------------------------

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool kBf16>
struct MfmaTraits;

template <>
struct MfmaTraits<false> {
  typedef f16x8 vec;
  typedef _Float16 elem;
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
  __device__ static const uint16_t *table() { return kKronF16.v; }
};

template <>
struct MfmaTraits<true> {
  typedef bf16x8 vec;
  typedef __bf16 elem;
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
  __device__ static const uint16_t *table() { return kKronBf16.v; }
};

inline constexpr int kMfmaWaves = 4;  // waves per workgroup; each wave codes 16 blocks per step

// One 8-byte row of block (by, bx), row r of the block, clamped at the edges.
__device__ __forceinline__ uint2 load_row(const uint8_t *__restrict__ src, int W, int H, int stride, int by, int bx,
                                          int r, bool full) {
  const int x0 = bx * 8;
  if (full) {
    const uint32_t off = static_cast<uint32_t>(by * 8 + r) * static_cast<uint32_t>(stride) + static_cast<uint32_t>(x0);
    return *reinterpret_cast<const uint2 *>(src + off);
  }
  const uint8_t *row = src + static_cast<size_t>(min(by * 8 + r, H - 1)) * stride;
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    lo |= static_cast<uint32_t>(row[min(x0 + j, W - 1)]) << (8 * j);
    hi |= static_cast<uint32_t>(row[min(x0 + 4 + j, W - 1)]) << (8 * j);
  }
  return make_uint2(lo, hi);
}

// Lane layouts of v_mfma_f32_16x16x32 (lane l, i = l % 16, g = l / 16):
//   A[i][8g + e], B[8g + e][i], D[4g + r][i]  (e = 0..7, r = 0..3).
// Forward, K-step s, N-tile t:  A = pixels of block i, row 4s + g;
//   B[k][j] = K[j][k] for k = 32s + 8g + e, j = 16t + i.
// D[4g + r][16t + i] = F of block 4g + r, coefficient 16t + i.
// Inverse: A[i][j = 32s + 8g + e] = dequantized F of block i; B[j][k] = K[j][k]
// for k = 16t + i; D[4g + r][16t + i] = pixel 16t + i of block 4g + r.
template <bool kBf16, bool kCodec>
__global__ __launch_bounds__(64 * kMfmaWaves) void kron_kernel(const uint8_t *__restrict__ src, int W, int H,
                                                              int stride, int bw, int nblocks, int ntiles,
                                                              float *__restrict__ coef, FloatQuant fq,
                                                              uint8_t *__restrict__ dst, int dst_stride,
                                                              unsigned long long *__restrict__ sse) {
  using T = MfmaTraits<kBf16>;
  typedef typename T::vec vec;
  typedef typename T::elem elem;
  __shared__ uint16_t lds_coef[kMfmaWaves][16 * 64];
  __shared__ uint8_t lds_pix[kMfmaWaves][16 * 64];
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, g = l >> 4;
  const uint16_t *K = T::table();

  // constant B operands (each lane: 2 K-steps x 4 N-tiles x 8 elements, per direction)
  vec bf[2][4], bi[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        bf[s][t][e] = __builtin_bit_cast(elem, K[(16 * t + i) * 64 + 32 * s + 8 * g + e]);
        bi[s][t][e] = __builtin_bit_cast(elem, K[(32 * s + 8 * g + e) * 64 + 16 * t + i]);
      }

  uint64_t err = 0;
  // workgroup-uniform loop over groups of kMfmaWaves tiles of 16 blocks
  for (int base = blockIdx.x * kMfmaWaves; base < ntiles; base += gridDim.x * kMfmaWaves) {
    const int tile = base + wave;
    // a1: this lane's block i of the tile: rows g and 4 + g
    const int b = tile * 16 + i;
    const BlockPos p = block_pos(b, W, H, bw, nblocks);
    uint2 raw[2] = {make_uint2(0, 0), make_uint2(0, 0)};
    if (p.live) {
      raw[0] = load_row(src, W, H, stride, p.by, p.bx, g, p.full);
      raw[1] = load_row(src, W, H, stride, p.by, p.bx, 4 + g, p.full);
    }
    vec a[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t w = e < 4 ? raw[s].x : raw[s].y;
        a[s][e] = static_cast<elem>(static_cast<float>(static_cast<int>((w >> (8 * (e & 3))) & 0xffu) - 128));
      }
    // forward product
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 2; ++s) acc[t] = T::mma(a[s], bf[s][t], acc[t]);
    }
    if constexpr (!kCodec) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int bo = tile * 16 + 4 * g + r;
        if (bo < nblocks) {
#pragma unroll
          for (int t = 0; t < 4; ++t) coef[static_cast<size_t>(bo) * 64 + 16 * t + i] = acc[t][r];
        }
      }
    } else {
      // quantize, dequantize, and lay the block's values out for the inverse
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = 16 * t + i, sidx = (j >> 3) + (j & 7);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float d = fquant(acc[t][r], fq.Q[sidx], fq.rcp[sidx]);
          lds_coef[wave][(4 * g + r) * 64 + j] = __builtin_bit_cast(uint16_t, static_cast<elem>(d));
        }
      }
      __syncthreads();
      vec ai[2];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          ai[s][e] = __builtin_bit_cast(elem, lds_coef[wave][i * 64 + 32 * s + 8 * g + e]);
      f32x4 rx[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        rx[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s) rx[t] = T::mma(ai[s], bi[s][t], rx[t]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          lds_pix[wave][(4 * g + r) * 64 + 16 * t + i] = static_cast<uint8_t>(freconstruct(rx[t][r]));
      __syncthreads();
      // rows g and 4 + g of block i back to the lane that loaded them
      uint32_t rec[16] = {}, pix[16] = {};
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int r = 4 * s + g;
        const uint2 w = *reinterpret_cast<const uint2 *>(&lds_pix[wave][i * 64 + 8 * r]);
        rec[2 * r] = w.x;
        rec[2 * r + 1] = w.y;
        pix[2 * r] = raw[s].x;
        pix[2 * r + 1] = raw[s].y;
      }
      if (p.live) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int r = 4 * s + g, y = p.by * 8 + r;
          if (p.full) {
            const uint32_t off = static_cast<uint32_t>(y) * static_cast<uint32_t>(dst_stride) +
                                 static_cast<uint32_t>(p.bx * 8);
            *reinterpret_cast<uint2 *>(dst + off) = make_uint2(rec[2 * r], rec[2 * r + 1]);
          } else if (y < H) {
            uint8_t *row = dst + static_cast<size_t>(y) * dst_stride;
#pragma unroll
            for (int jj = 0; jj < 8; ++jj)
              if (p.bx * 8 + jj < W) row[p.bx * 8 + jj] = static_cast<uint8_t>(rec[2 * r + (jj >> 2)] >> (8 * (jj & 3)));
          }
        }
        // SSE of the two rows this lane holds (the other rows are zero in both)
        err += block_sse(pix, rec, W, H, p.by, p.bx, p.full);
      }
      __syncthreads();
    }
  }
  if constexpr (kCodec) workgroup_add<64 * kMfmaWaves>(err, sse);
}

}  // namespace dct

namespace dct {

// Integer full-range YCbCr of interleaved RGB (JFIF weights rounded to 2^-16):
//   Y  = (19595 R + 38470 G + 7471 B + 2^15) >> 16
//   Cb = ((-11058 R - 21710 G + 32768 B + 2^15) >> 16) + 128
//   Cr = ((32768 R - 27439 G - 5329 B + 2^15) >> 16) + 128, each clamped to [0, 255].
__global__ __launch_bounds__(kWg) void ycbcr_kernel(const uint8_t *__restrict__ rgb, int W, int H, int rgb_stride,
                                                    uint8_t *__restrict__ y, uint8_t *__restrict__ cb,
                                                    uint8_t *__restrict__ cr, int plane_stride) {
  const int64_t total = static_cast<int64_t>(W) * H;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kWg + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * kWg) {
    const int row = static_cast<int>(t / W), col = static_cast<int>(t - static_cast<int64_t>(row) * W);
    const uint8_t *px = rgb + static_cast<size_t>(row) * rgb_stride + 3 * col;
    const int R = px[0], G = px[1], B = px[2];
    const int yy = (19595 * R + 38470 * G + 7471 * B + (1 << 15)) >> 16;
    const int bb = ((-11058 * R - 21710 * G + 32768 * B + (1 << 15)) >> 16) + 128;
    const int rr = ((32768 * R - 27439 * G - 5329 * B + (1 << 15)) >> 16) + 128;
    const size_t o = static_cast<size_t>(row) * plane_stride + col;
    y[o] = static_cast<uint8_t>(min(max(yy, 0), 255));
    cb[o] = static_cast<uint8_t>(min(max(bb, 0), 255));
    cr[o] = static_cast<uint8_t>(min(max(rr, 0), 255));
  }
}

}  // namespace dct
