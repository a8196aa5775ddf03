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

// q = sgn(F) floor(|F| / Q + 1/2); returns the dequantized q Q (the sign is put
// on q first: the same value, one instruction fewer when the product is then
// rounded to a 16-bit operand)
__device__ __forceinline__ float fquant(float F, float Q, float rcp) {
  const float q = __builtin_floorf(__builtin_fabsf(F) * rcp + 0.5f);
  return __builtin_copysignf(q, F) * Q;
}

// The matrix form's quantizer in three instructions: t = F (1/Q) + 1.5 2^23 (one
// FMA) lies in [2^23, 2^24), where the last place is 1, so t holds 1.5 2^23 + q
// with q the integer nearest the exact product F (1/Q) (ties to even, either
// sign; needs |F / Q| < 2^22, which |F| <= 1024 gives); t - 1.5 2^23 = q and
// q Q (< 2^24) are exact.  It differs from sgn(F) floor(|F| / Q + 1/2) only when
// the product is an exact half-integer, within the form's error of the rounding
// boundary.
inline constexpr float kRoundMagic = 12582912.0f;  // 1.5 2^23
__device__ __forceinline__ float fquant_rne(float F, float rcp, float Q) {
  return (__builtin_fmaf(F, rcp, kRoundMagic) - kRoundMagic) * Q;
}

// clamp(floor(x + 128 + 1/2), 0, 255)
__device__ __forceinline__ uint32_t freconstruct(float x) {
  const float p = __builtin_floorf(x + 128.5f);
  return static_cast<uint32_t>(__builtin_fminf(__builtin_fmaxf(p, 0.0f), 255.0f));
}

// The same into byte k of acc for the matrix form, given x + 128 (the inverse
// product starts its accumulation there): the byte conversion rounds to the
// nearest integer, ties to even, and saturates to [0, 255] (checked on the
// device), so one instruction rounds and clamps; it differs from floor(x + 128 +
// 1/2) only when the computed x + 128 is an exact tie, within the form's error
// of the rounding boundary.
__device__ __forceinline__ uint32_t pack_reconstruct(float x_offset, uint32_t k, uint32_t acc) {
  return __builtin_amdgcn_cvt_pk_u8_f32(x_offset, k, acc);
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

inline constexpr int kMfmaWaves = 4;  // waves per workgroup; a tile is the 16 blocks of one product
inline constexpr int kKronCodecTiles = 2;  // tiles the codec kernel codes per wave step, sharing operand reads

// Register-only layout of the matrix form.  With blocks as the N dimension,
// the forward product is F^T = K X^T (M = coefficient, K = pixel) and the
// inverse X^T = K^T F^T (M = pixel, K = coefficient).  The inner dimension of a
// product may be taken in any order, so both use the order
//     sigma(s, g, e) = 16 (2 s + e / 4) + 4 g + e % 4
// for K-step s, lane group g = lane / 16 and element e of the 8-element operand.
// Then, for lane (i = lane % 16, g):
//   * the forward B operand is pixels sigma(s, g, 0..7) of block i: the four
//     4-byte words w[t] = row 2t + g/2, columns 4(g%2)..4(g%2)+3 (t = 0..3),
//     loaded straight from the plane;
//   * the forward result D[4g + r] of M-tile t is coefficient 16t + 4g + r of
//     block i, which is element e = 4(t % 2) + r of the inverse B operand of
//     K-step s = t / 2, so the quantized values never leave the lane;
//   * the inverse result D[4g + r] of M-tile t is pixel 16t + 4g + r of block
//     i, byte r of the lane's own word w[t], so it is stored where it was
//     loaded and the SSE needs no second read.
// No LDS and no barrier is involved.  The A operands are the constant matrix
// K[j][k] (coefficient j, pixel k) in that order, held in registers.
__device__ __forceinline__ int sigma_index(int s, int g, int e) { return 16 * (2 * s + (e >> 2)) + 4 * g + (e & 3); }

// the four words of lane group g of a block: row 2t + g/2, bytes 4(g%2)..+3
__device__ __forceinline__ void load_words(const uint8_t *__restrict__ src, int W, int H, int stride, int by,
                                           int bx, int g, bool full, uint32_t (&w)[4]) {
  const int x0 = bx * 8 + 4 * (g & 1), y0 = by * 8 + (g >> 1);
  if (full) {
    const uint32_t off = static_cast<uint32_t>(y0) * static_cast<uint32_t>(stride) + static_cast<uint32_t>(x0);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      w[t] = *reinterpret_cast<const uint32_t *>(src + (off + static_cast<uint32_t>(2 * t * stride)));
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint8_t *row = src + static_cast<size_t>(min(y0 + 2 * t, H - 1)) * stride;
      uint32_t v = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) v |= static_cast<uint32_t>(row[min(x0 + r, W - 1)]) << (8 * r);
      w[t] = v;
    }
  }
}

// the same for stores; a block inside the image is stored non-temporally (its
// bytes are not read again), an edge block byte by byte
__device__ __forceinline__ void store_words(uint8_t *__restrict__ dst, int W, int H, int stride, int by, int bx,
                                            int g, bool full, const uint32_t (&w)[4]) {
  const int x0 = bx * 8 + 4 * (g & 1), y0 = by * 8 + (g >> 1);
  if (full) {
    const uint32_t off = static_cast<uint32_t>(y0) * static_cast<uint32_t>(stride) + static_cast<uint32_t>(x0);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      __builtin_nontemporal_store(w[t], reinterpret_cast<uint32_t *>(dst + (off + static_cast<uint32_t>(2 * t * stride))));
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int y = y0 + 2 * t;
      if (y < H) {
        uint8_t *row = dst + static_cast<size_t>(y) * stride;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (x0 + r < W) row[x0 + r] = static_cast<uint8_t>(w[t] >> (8 * r));
      }
    }
  }
}

// SSE of the lane's four words of a block inside the image
__device__ __forceinline__ uint32_t words_sse_full(const uint32_t (&a)[4], const uint32_t (&b)[4]) {
  uint32_t pp = 0, pr = 0, rr = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    pp = __builtin_amdgcn_udot4(a[t], a[t], pp, false);
    pr = __builtin_amdgcn_udot4(a[t], b[t], pr, false);
    rr = __builtin_amdgcn_udot4(b[t], b[t], rr, false);
  }
  return pp - 2u * pr + rr;
}

// SSE of the lane's four words; edge blocks count only pixels inside W x H
__device__ __forceinline__ uint32_t words_sse(const uint32_t (&a)[4], const uint32_t (&b)[4], int W, int H, int by,
                                              int bx, int g, bool full) {
  uint32_t mask = 0xffffffffu;
  int rows = 8;
  if (!full) {
    const int cols = min(max(W - (bx * 8 + 4 * (g & 1)), 0), 4);
    mask = cols >= 4 ? 0xffffffffu : (1u << (8 * cols)) - 1u;
    rows = H - by * 8 - (g >> 1);
  }
  uint32_t pp = 0, pr = 0, rr = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bool in = full || 2 * t < rows;
    const uint32_t x = in ? a[t] & mask : 0u, y = in ? b[t] & mask : 0u;
    pp = __builtin_amdgcn_udot4(x, x, pp, false);
    pr = __builtin_amdgcn_udot4(x, y, pr, false);
    rr = __builtin_amdgcn_udot4(y, y, rr, false);
  }
  return pp - 2u * pr + rr;
}

// The workgroup's constants of the matrix form, in LDS: the A operands of every
// lane, forward fa[t][s][lane][e] = K[16t + i][sigma(s, g, e)] and inverse
// ia[t][s][lane][e] = K[sigma(s, g, e)][16t + i] (one 16-byte read per operand,
// consecutive lanes at consecutive addresses), and the quantizer entries of the
// coefficients 16t + 4g + r that lane group g holds, qv[t][g][r] = Q and
// rq[t][g][r] = 1/Q (one 16-byte read that the group's lanes share).  Keeping
// them out of registers leaves the plane kernel at about 60 VGPRs.
template <bool kBf16>
struct OperandTable {
  typename MfmaTraits<kBf16>::vec fa[4][2][64];
  typename MfmaTraits<kBf16>::vec ia[4][2][64];
  f32x4 qv[4][4], rq[4][4];
};

// Fills (wave 0) the workgroup's operand table, the inverse half and the
// quantizer entries only when kCodec; the caller synchronizes the workgroup after.
template <bool kBf16, bool kCodec>
__device__ __forceinline__ void kron_setup(OperandTable<kBf16> *inv, const FloatQuant &fq, int wave, int i, int g) {
  using T = MfmaTraits<kBf16>;
  typedef typename T::elem elem;
  const uint16_t *K = T::table();
  const int lane = 16 * g + i;
  if (wave != 0) return;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      typename T::vec fa, ia;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        fa[e] = __builtin_bit_cast(elem, K[(16 * t + i) * 64 + sigma_index(s, g, e)]);
        if constexpr (kCodec) ia[e] = __builtin_bit_cast(elem, K[sigma_index(s, g, e) * 64 + 16 * t + i]);
      }
      inv->fa[t][s][lane] = fa;
      if constexpr (kCodec) inv->ia[t][s][lane] = ia;
    }
  if constexpr (kCodec) {
    if (i < 4) {
      // lane (i < 4, g) fills entries t = i: coefficient 16t + 4g + r has u + v = 2t + r + g/2 + 4(g%2)
      const int t = i;
      f32x4 qq, rr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int sidx = 2 * t + r + (g >> 1) + 4 * (g & 1);
        qq[r] = fq.Q[0];
        rr[r] = fq.rcp[0];
#pragma unroll
        for (int k = 1; k < 15; ++k) {
          qq[r] = sidx == k ? fq.Q[k] : qq[r];
          rr[r] = sidx == k ? fq.rcp[k] : rr[r];
        }
      }
      inv->qv[t][g] = qq;
      inv->rq[t][g] = rr;
    }
  }
}

// forward products of kN tiles, the lane's 16 pixels (four words) of each:
// acc[n][t][r] = coefficient 16t + 4g + r of tile n.  Each operand read from LDS
// serves the kN tiles' products.
template <bool kBf16, int kN>
__device__ __forceinline__ void kron_forward(const OperandTable<kBf16> *tab, int lane, const uint32_t (&w)[kN][4],
                                             f32x4 (&acc)[kN][4]) {
  // the table is read afresh at every call (an opaque index keeps the reads in the loop)
  asm volatile("" : "+v"(lane));
  using T = MfmaTraits<kBf16>;
  typedef typename T::vec vec;
  typedef typename T::elem elem;
  vec bx[kN][2];
#pragma unroll
  for (int n = 0; n < kN; ++n) {
    if constexpr (!kBf16) {
      // FP16 of b - 128 for two bytes at once: 0x6400 | b is 1024 + b, exact with
      // 11 significant bits, and 1024 + b - 1152 is exact too
      typedef _Float16 h2 __attribute__((ext_vector_type(2)));
      const h2 off = {static_cast<_Float16>(1152.0f), static_cast<_Float16>(1152.0f)};
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const uint32_t word = w[n][2 * s + (h >> 1)];
          const uint32_t sel = (h & 1) ? 0x04030402u : 0x04010400u;  // bytes 2, 3 or 0, 1 under 0x64
          const h2 v = __builtin_bit_cast(h2, __builtin_amdgcn_perm(0x64646464u, word, sel)) - off;
          bx[n][s][2 * h] = v[0];
          bx[n][s][2 * h + 1] = v[1];
        }
    } else {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t word = w[n][2 * s + (e >> 2)];
          bx[n][s][e] = static_cast<elem>(static_cast<float>((word >> (8 * (e & 3))) & 0xffu) - 128.0f);
        }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const vec fa0 = tab->fa[t][0][lane], fa1 = tab->fa[t][1][lane];
#pragma unroll
    for (int n = 0; n < kN; ++n) {
      acc[n][t] = T::mma(fa0, bx[n][0], f32x4{0.f, 0.f, 0.f, 0.f});
      acc[n][t] = T::mma(fa1, bx[n][1], acc[n][t]);
    }
  }
}

// quantize, dequantize, inverse product and reconstruction of kN tiles: the four
// output words of each; each operand and quantizer read serves the kN tiles
template <bool kBf16, int kN>
__device__ __forceinline__ void kron_code(const OperandTable<kBf16> *inv, int lane, const f32x4 (&acc)[kN][4],
                                          uint32_t (&rec)[kN][4]) {
  // the table is read afresh at every call: an opaque index keeps the compiler
  // from hoisting the reads out of the tile loop into registers
  asm volatile("" : "+v"(lane));
  using T = MfmaTraits<kBf16>;
  typedef typename T::vec vec;
  typedef typename T::elem elem;
  const int g = lane >> 4;
  // element e = 4(t % 2) + r of inverse step t / 2
  vec bq[kN][2];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const f32x4 qv = inv->qv[t][g], rq = inv->rq[t][g];
#pragma unroll
    for (int n = 0; n < kN; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        bq[n][t >> 1][4 * (t & 1) + r] = static_cast<elem>(fquant_rne(acc[n][t][r], rq[r], qv[r]));
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const vec ia0 = inv->ia[t][0][lane], ia1 = inv->ia[t][1][lane];
#pragma unroll
    for (int n = 0; n < kN; ++n) {
      f32x4 x = T::mma(ia0, bq[n][0], f32x4{128.0f, 128.0f, 128.0f, 128.0f});
      x = T::mma(ia1, bq[n][1], x);
      uint32_t v = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) v = pack_reconstruct(x[r], r, v);
      rec[n][t] = v;
    }
  }
}

// Position of block 16 tile + i.  tile is wave-uniform, so the division by bw is
// one scalar division per tile; a lane then wraps at most once into the next
// block row when the row holds at least 16 blocks (else each lane divides).
__device__ __forceinline__ BlockPos tile_pos(int tile, int i, int W, int H, int bw, int nblocks) {
  const int b0 = tile * 16;
  int by, bx;
  if (bw >= 16) {
    const int by0 = b0 / bw;
    bx = b0 - by0 * bw + i;
    const bool wrap = bx >= bw;
    bx = wrap ? bx - bw : bx;
    by = by0 + (wrap ? 1 : 0);
  } else {
    by = (b0 + i) / bw;
    bx = b0 + i - by * bw;
  }
  const bool live = b0 + i < nblocks;
  BlockPos p;
  p.live = live;
  p.by = live ? by : 0;
  p.bx = live ? bx : 0;
  p.full = live && bx * 8 + 8 <= W && by * 8 + 8 <= H;
  return p;
}

// kCodec = false: FP32 coefficients only; true: quantize, inverse, reconstruct, SSE.
template <bool kBf16, bool kCodec>
__global__ __launch_bounds__(64 * kMfmaWaves) void kron_kernel(const uint8_t *__restrict__ src, int W, int H,
                                                              int stride, int bw, int nblocks, int ntiles,
                                                              float *__restrict__ coef, FloatQuant fq,
                                                              uint8_t *__restrict__ dst, int dst_stride,
                                                              unsigned long long *__restrict__ sse) {
  const int wave = wave_index(), l = threadIdx.x & 63, i = l & 15, g = l >> 4;
  __shared__ OperandTable<kBf16> inv;
  kron_setup<kBf16, kCodec>(&inv, fq, wave, i, g);
  __syncthreads();
  uint64_t err = 0;
  // A wave codes kN consecutive tiles per step (the codec: two, 32 blocks, so
  // that each operand read from LDS serves two tiles' products) and walks its
  // steps with the words of the next kDepth steps in flight, in a ring of
  // kDepth + 1 slots that the unrolled loop rotates: no register of a load in
  // flight is copied, which would wait for the load.  A tile's block positions
  // are found once, when its words are loaded.
  constexpr int kN = kCodec ? kKronCodecTiles : 1;
  constexpr int kDepth = kCodec ? 1 : 2;
  constexpr int kSlots = kDepth + 1;
  const int ngroups = (ntiles + kN - 1) / kN;
  const int step = gridDim.x * kMfmaWaves;
  int grp = blockIdx.x * kMfmaWaves + wave;
  uint32_t ring[kSlots][kN][4];
  BlockPos rpos[kSlots][kN];
  // The prefetch is four unconditional buffer loads per lane and tile: the words
  // of a block inside the image, and for every other lane the plane's first
  // words (a load past the plane's bytes returns zero).  With no branch around
  // the loads the compiler keeps them in flight until their tile is coded; an
  // edge block reloads its words then, with edge replication.  The loads (cache
  // policy 2) and the stores of whole blocks are non-temporal: every byte of the
  // planes is read once and written once.
  const __amdgpu_buffer_rsrc_t plane =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(src), 0,
                                        static_cast<int>(static_cast<uint32_t>(H - 1) * static_cast<uint32_t>(stride) +
                                                         static_cast<uint32_t>(W)),
                                        0x00020000);
  auto fetch = [&](int gi, uint32_t(&w)[kN][4], BlockPos(&p)[kN]) {
#pragma unroll
    for (int n = 0; n < kN; ++n) {
      p[n] = tile_pos(gi * kN + n, i, W, H, bw, nblocks);
      const uint32_t off = p[n].full ? static_cast<uint32_t>(p[n].by * 8 + (g >> 1)) * static_cast<uint32_t>(stride) +
                                           static_cast<uint32_t>(p[n].bx * 8 + 4 * (g & 1))
                                     : 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        w[n][k] = static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b32(
            plane, static_cast<int>(off + static_cast<uint32_t>(2 * k * stride)), 0, 2));
    }
  };
#pragma unroll
  for (int d = 0; d < kDepth; ++d) fetch(grp + d * step, ring[d], rpos[d]);
  while (grp < ngroups) {
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      if (grp < ngroups) {
        fetch(grp + kDepth * step, ring[(k + kDepth) % kSlots], rpos[(k + kDepth) % kSlots]);
        uint32_t(&w)[kN][4] = ring[k];
        const BlockPos(&p)[kN] = rpos[k];
#pragma unroll
        for (int n = 0; n < kN; ++n)
          if (!p[n].full && p[n].live) load_words(src, W, H, stride, p[n].by, p[n].bx, g, false, w[n]);
        f32x4 acc[kN][4];
        kron_forward<kBf16, kN>(&inv, l, w, acc);
        if constexpr (!kCodec) {
          if (p[0].live) {
            const size_t b = static_cast<size_t>(grp) * 16 + i;
#pragma unroll
            for (int t = 0; t < 4; ++t)
              *reinterpret_cast<float4 *>(coef + b * 64 + 16 * t + 4 * g) =
                  make_float4(acc[0][t][0], acc[0][t][1], acc[0][t][2], acc[0][t][3]);
          }
        } else {
          uint32_t rec[kN][4];
          kron_code<kBf16, kN>(&inv, l, acc, rec);
#pragma unroll
          for (int n = 0; n < kN; ++n) {
            if (p[n].full) {
              store_words(dst, W, H, dst_stride, p[n].by, p[n].bx, g, true, rec[n]);
              err += words_sse_full(w[n], rec[n]);
            } else if (p[n].live) {
              store_words(dst, W, H, dst_stride, p[n].by, p[n].bx, g, false, rec[n]);
              err += words_sse(w[n], rec[n], W, H, p[n].by, p[n].bx, g, false);
            }
          }
        }
        grp += step;
      }
    }
  }
  if constexpr (kCodec) workgroup_add<64 * kMfmaWaves>(err, sse, wave);
}

// JFIF YCbCr of one RGB pixel (integer, 2^-16 weights).  The luma weights sum to
// 2^16, so Y lies in [0, 255] without a clamp; Cb and Cr are clamped.  (Written
// without the luma clamp on purpose: with it, hipcc for gfx950 packs pairs of
// clamped shifts into v_ashr_pk_u8_i32 and then ORs more bytes into the upper
// half of that register without clearing it, which corrupts byte 2.)
// Every product of an 8-bit sample and a weight below 2^16 fits 24 bits, so the
// products use the full-rate 24-bit multiplier; the sums are the same integers.
__device__ __forceinline__ void ycc_pixel(int R, int G, int B, uint32_t &y, uint32_t &cb, uint32_t &cr) {
  const uint32_t r = static_cast<uint32_t>(R), g = static_cast<uint32_t>(G), b = static_cast<uint32_t>(B);
  y = (__umul24(19595u, r) + __umul24(38470u, g) + __umul24(7471u, b) + (1u << 15)) >> 16;
  const int tb = static_cast<int>((b << 15) + (1u << 15)) - static_cast<int>(__umul24(11058u, r) + __umul24(21710u, g));
  const int tr = static_cast<int>((r << 15) + (1u << 15)) - static_cast<int>(__umul24(27439u, g) + __umul24(5329u, b));
  cb = static_cast<uint32_t>(min(max((tb >> 16) + 128, 0), 255));
  cr = static_cast<uint32_t>(min(max((tr >> 16) + 128, 0), 255));
}

// The lane's four pixel words of each of the Y, Cb, Cr planes of an RGB block,
// converted on the fly (positions as load_words).  A full block with 4-aligned
// RGB rows reads three 4-byte words per 4 pixels; other blocks go byte by byte
// with edge replication.
// The Y, Cb and Cr words of four RGB pixels given as twelve bytes (R, G, B each)
__device__ __forceinline__ void ycc_words(const uint32_t (&bytes)[12], uint32_t &y, uint32_t &cb, uint32_t &cr) {
  uint32_t wy = 0, wb = 0, wr = 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    uint32_t vy, vb, vr;
    ycc_pixel(static_cast<int>(bytes[3 * r]), static_cast<int>(bytes[3 * r + 1]), static_cast<int>(bytes[3 * r + 2]),
              vy, vb, vr);
    wy |= vy << (8 * r);
    wb |= vb << (8 * r);
    wr |= vr << (8 * r);
  }
  y = wy;
  cb = wb;
  cr = wr;
}

__device__ __forceinline__ void load_rgb_words(const uint8_t *__restrict__ rgb, int W, int H, int rgb_stride,
                                               int by, int bx, int g, bool full, bool vec_ok, uint32_t (&y)[4],
                                               uint32_t (&cb)[4], uint32_t (&cr)[4]) {
  const int x0 = bx * 8 + 4 * (g & 1), y0 = by * 8 + (g >> 1);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    uint32_t bytes[12];
    if (full && vec_ok) {
      const uint32_t off = static_cast<uint32_t>(y0 + 2 * t) * static_cast<uint32_t>(rgb_stride) +
                           static_cast<uint32_t>(3 * x0);
      const uint32_t *src = reinterpret_cast<const uint32_t *>(rgb + off);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const uint32_t v = src[k];
#pragma unroll
        for (int j = 0; j < 4; ++j) bytes[4 * k + j] = (v >> (8 * j)) & 0xffu;
      }
    } else {
      const uint8_t *row = rgb + static_cast<size_t>(min(y0 + 2 * t, H - 1)) * rgb_stride;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int xx = min(x0 + r, W - 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) bytes[3 * r + c] = row[3 * xx + c];
      }
    }
    ycc_words(bytes, y[t], cb[t], cr[t]);
  }
}

// The same from the lane's twelve words of a block inside the image, loaded
// beforehand: words 3t .. 3t + 2 hold the twelve RGB bytes of its row 2t + g/2.
__device__ __forceinline__ void rgb_words_from_raw(const uint32_t (&raw)[12], uint32_t (&y)[4], uint32_t (&cb)[4],
                                                   uint32_t (&cr)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    uint32_t bytes[12];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) bytes[4 * k + j] = (raw[3 * t + k] >> (8 * j)) & 0xffu;
    ycc_words(bytes, y[t], cb[t], cr[t]);
  }
}

// RGB in, three coded planes out: the YCbCr conversion fused with the matrix-form
// codec of each plane, the SSE of each plane against its converted values into
// sse[0..2].  Bit for bit what dct_rgb_to_ycbcr followed by the matrix-form codec
// of each plane gives, with 6 bytes of HBM traffic per RGB pixel instead of 12.
template <bool kBf16>
__global__ __launch_bounds__(64 * kMfmaWaves) void kron_rgb_kernel(const uint8_t *__restrict__ rgb, int W, int H,
                                                                  int rgb_stride, bool vec_ok, int bw, int nblocks,
                                                                  int ntiles, FloatQuant fq,
                                                                  uint8_t *__restrict__ out_y,
                                                                  uint8_t *__restrict__ out_cb,
                                                                  uint8_t *__restrict__ out_cr, int plane_stride,
                                                                  unsigned long long *__restrict__ sse) {
  const int wave = wave_index(), l = threadIdx.x & 63, i = l & 15, g = l >> 4;
  __shared__ OperandTable<kBf16> inv;
  kron_setup<kBf16, true>(&inv, fq, wave, i, g);
  __syncthreads();
  uint64_t err[3] = {0, 0, 0};
  // The next tile's RGB words are loaded while the current tile is coded, in a
  // ring of two slots that the unrolled loop rotates: twelve unconditional,
  // non-temporal buffer loads per lane (a block inside the image, else the
  // image's first words; the buffer's bounds check returns zero past its end).
  // Edge blocks, and images whose rows are not 4-byte aligned, gather their bytes
  // when they are coded.
  constexpr int kSlots = 2;
  const int step = gridDim.x * kMfmaWaves;
  int tile = blockIdx.x * kMfmaWaves + wave;
  uint32_t ring[kSlots][12];
  BlockPos rpos[kSlots];
  const __amdgpu_buffer_rsrc_t image = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(rgb), 0,
      static_cast<int>(static_cast<uint32_t>(H - 1) * static_cast<uint32_t>(rgb_stride) + 3u * static_cast<uint32_t>(W)),
      0x00020000);
  auto fetch = [&](int t, uint32_t(&raw)[12], BlockPos &p) {
    p = tile_pos(t, i, W, H, bw, nblocks);
    const uint32_t off =
        p.full && vec_ok ? static_cast<uint32_t>(p.by * 8 + (g >> 1)) * static_cast<uint32_t>(rgb_stride) +
                               3u * static_cast<uint32_t>(p.bx * 8 + 4 * (g & 1))
                         : 0u;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        raw[3 * r + k] = static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b32(
            image, static_cast<int>(off + static_cast<uint32_t>(2 * r * rgb_stride + 4 * k)), 0, 2));
  };
  fetch(tile, ring[0], rpos[0]);
  uint8_t *outs[3] = {out_y, out_cb, out_cr};
  while (tile < ntiles) {
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
      if (tile < ntiles) {
        fetch(tile + step, ring[(k + 1) % kSlots], rpos[(k + 1) % kSlots]);
        const BlockPos &p = rpos[k];
        uint32_t w[3][4] = {};
        if (p.full && vec_ok)
          rgb_words_from_raw(ring[k], w[0], w[1], w[2]);
        else if (p.live)
          load_rgb_words(rgb, W, H, rgb_stride, p.by, p.bx, g, p.full, vec_ok, w[0], w[1], w[2]);
        // the three planes' products share each operand read
        f32x4 acc[3][4];
        kron_forward<kBf16, 3>(&inv, l, w, acc);
        uint32_t rec[3][4];
        kron_code<kBf16, 3>(&inv, l, acc, rec);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (p.live) {
            store_words(outs[c], W, H, plane_stride, p.by, p.bx, g, p.full, rec[c]);
            err[c] += words_sse(w[c], rec[c], W, H, p.by, p.bx, g, p.full);
          }
        }
        tile += step;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    workgroup_add<64 * kMfmaWaves>(err[c], sse + c, wave);
    __syncthreads();
  }
}

}  // namespace dct

namespace dct {

// Integer full-range YCbCr of interleaved RGB (JFIF weights rounded to 2^-16):
//   Y  = (19595 R + 38470 G + 7471 B + 2^15) >> 16
//   Cb = ((-11058 R - 21710 G + 32768 B + 2^15) >> 16) + 128
//   Cr = ((32768 R - 27439 G - 5329 B + 2^15) >> 16) + 128, each clamped to [0, 255].
__device__ __forceinline__ uint32_t ycc_byte(int v) { return static_cast<uint32_t>(min(max(v, 0), 255)); }

// One pixel: (Y, Cb, Cr) as three bytes.
__device__ __forceinline__ void ycc(int R, int G, int B, uint32_t &y, uint32_t &cb, uint32_t &cr) {
  y = static_cast<uint32_t>((19595 * R + 38470 * G + 7471 * B + (1 << 15)) >> 16);  // in [0, 255]: weights sum to 2^16
  cb = ycc_byte(((-11058 * R - 21710 * G + 32768 * B + (1 << 15)) >> 16) + 128);
  cr = ycc_byte(((32768 * R - 27439 * G - 5329 * B + (1 << 15)) >> 16) + 128);
}

// One thread per group of 8 pixels of a row, grid-stride.  A group inside the
// row of an 8-byte-aligned RGB row (rgb_stride % 8 == 0 and base aligned) reads
// three 8-byte words and writes one 8-byte word per plane; other groups go byte
// by byte.
__global__ __launch_bounds__(kWg) void ycbcr_kernel(const uint8_t *__restrict__ rgb, int W, int H, int rgb_stride,
                                                    uint8_t *__restrict__ y, uint8_t *__restrict__ cb,
                                                    uint8_t *__restrict__ cr, int plane_stride, bool vec_ok) {
  const int groups = (W + 7) / 8;
  const int64_t total = static_cast<int64_t>(groups) * H;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * kWg + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * kWg) {
    const int row = static_cast<int>(t / groups), x0 = static_cast<int>(t - static_cast<int64_t>(row) * groups) * 8;
    const uint8_t *px = rgb + static_cast<size_t>(row) * rgb_stride + 3 * x0;
    const size_t o = static_cast<size_t>(row) * plane_stride + x0;
    if (vec_ok && x0 + 8 <= W) {
      const uint2 a = reinterpret_cast<const uint2 *>(px)[0], b2 = reinterpret_cast<const uint2 *>(px)[1],
                  c = reinterpret_cast<const uint2 *>(px)[2];
      const uint32_t wv[6] = {a.x, a.y, b2.x, b2.y, c.x, c.y};
      uint32_t yy[2] = {0u, 0u}, bb[2] = {0u, 0u}, rr[2] = {0u, 0u};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int R = (wv[(3 * k) >> 2] >> (8 * ((3 * k) & 3))) & 0xff;
        const int G = (wv[(3 * k + 1) >> 2] >> (8 * ((3 * k + 1) & 3))) & 0xff;
        const int B = (wv[(3 * k + 2) >> 2] >> (8 * ((3 * k + 2) & 3))) & 0xff;
        uint32_t vy, vb, vr;
        ycc(R, G, B, vy, vb, vr);
        yy[k >> 2] |= vy << (8 * (k & 3));
        bb[k >> 2] |= vb << (8 * (k & 3));
        rr[k >> 2] |= vr << (8 * (k & 3));
      }
      *reinterpret_cast<uint2 *>(y + o) = make_uint2(yy[0], yy[1]);
      *reinterpret_cast<uint2 *>(cb + o) = make_uint2(bb[0], bb[1]);
      *reinterpret_cast<uint2 *>(cr + o) = make_uint2(rr[0], rr[1]);
    } else {
      for (int k = 0; k < 8 && x0 + k < W; ++k) {
        uint32_t vy, vb, vr;
        ycc(px[3 * k], px[3 * k + 1], px[3 * k + 2], vy, vb, vr);
        y[o + k] = static_cast<uint8_t>(vy);
        cb[o + k] = static_cast<uint8_t>(vb);
        cr[o + k] = static_cast<uint8_t>(vr);
      }
    }
  }
}

}  // namespace dct
