// transform.hpp -- device-side Cordic-based Loeffler flow graphs on register blocks.
//
// The forward graph is the four-stage Loeffler 8-point DCT of Sec. 2.5.2:
//   stage 1  butterflies s_i = x_i + x_{7-i}, d_i = x_i - x_{7-i};
//   stage 2  even half: e0 = s0 + s3, e3 = s0 - s3, e1 = s1 + s2, e2 = s1 - s2;
//            odd half: (u4, u7) = R(d3, d0; 3pi/16), (u5, u6) = R(d2, d1; pi/16);
//   stage 3  Z0 = e0 + e1, Z4 = e0 - e1, (Z2, Z6) = sqrt2 R(e2, e3; 6pi/16);
//            v4 = u4 + u6, v6 = u4 - u6, v7 = u7 + u5, v5 = u7 - u5;
//   stage 4  Z1 = v7 + v4, Z7 = v7 - v4, Z3 = sqrt2 v5, Z5 = sqrt2 v6,
// with R(a, b; t) = (a cos t + b sin t, -a sin t + b cos t).  Its output is
// 2 sqrt(2) times the orthonormal DCT-II of its input, in the same fixed point.
// The inverse graph is the transpose: the stages in reverse order with every
// rotation by -t.
//
// Every rotation block is N micro-rotations a' = a + d_i (b >> i),
// b' = b - d_i (a >> i), directions resolved at compile time, followed by the
// gain compensation (v M + 2^(P-1)) >> P of each output.  All shifts are
// arithmetic; no value leaves int32 (the largest magnitude any step stores is
// below 2^30 for every input a uint8 plane or a clamped dequantized block gives).
//
// The compensation is computed as the high word of a 64-bit multiply-add:
//   (v M + 2^14) >> 15 = ((v 2^k) (M 2^(17-k)) + 2^31) >> 32,
// an identity of integers, with k = 1 for M < 2^15 and k = 2 for M < 2^16 so
// that M 2^(17-k) fits int32; v 2^k fits int32 because every compensated value
// of every recipe stays below 2^(31-k) in magnitude (bounded on the CPU through
// the flow graph's linear forms and truncation errors: at most 2^30.4 after the
// shift).  The shift is a plain instruction; the funnel shift the direct form
// needs to extract bits 15..46 is not.
//
// A pass transforms all eight lines (rows or columns) of a register block at
// once and keeps the instruction kinds apart: the butterflies and micro-
// rotations of all lines are plain 32-bit adds, subtracts and shifts, which
// gfx950 can issue two at a time across waves, while the 64-bit multiply-adds
// of the gain compensations, which it cannot, each cost far more when they
// stand alone between plain instructions than inside a run.  They are written
// as runs of eight in one asm statement (the compiler's scheduler otherwise
// interleaves them with the shifts that feed them), and scheduling barriers
// keep the regions apart.
#pragma once

#include <hip/hip_runtime.h>

#include "recipe.hpp"

namespace dct {

// keep the compiler from moving instructions across this point
__device__ __forceinline__ void region() { __builtin_amdgcn_sched_barrier(0); }

// one micro-rotation step I of rotation block R; S = +1 rotates by +theta, -1 by -theta
template <int N, int R, int S, int I>
__device__ __forceinline__ void cordic_step(int &a, int &b) {
  constexpr int d = S * kTablesN<N>.dir[R][I];
  const int sa = a >> I;
  const int sb = b >> I;
  if constexpr (d > 0) {
    a = a + sb;
    b = b - sa;
  } else {
    a = a - sb;
    b = b + sa;
  }
}

// the gain compensation's pre-shift k and multiplier M 2^(17-k) (P = 15)
template <int32_t M>
inline constexpr int kCompShift = M < (1 << 15) ? 1 : 2;
template <int32_t M>
inline constexpr int32_t kCompMul = M << (17 - kCompShift<M>);
static_assert(kComp == 15, "the high-word form of the compensation assumes P = 15");

// high words of v_i M 2^(17-k) + 2^31 for eight pre-shifted values v_i = v 2^k:
// one run of eight 64-bit multiply-adds
template <int32_t M>
__device__ __forceinline__ void comp_mul8(int *v) {
  static_assert(M > 0 && M < (1 << 16), "multiplier range");
  const int32_t m = kCompMul<M>;
  const long long r = 1LL << 31;
  long long p0, p1, p2, p3, p4, p5, p6, p7;
  unsigned long long carry;
  asm("v_mad_i64_i32 %0, %8, %9, %17, %18\n\t"
      "v_mad_i64_i32 %1, %8, %10, %17, %18\n\t"
      "v_mad_i64_i32 %2, %8, %11, %17, %18\n\t"
      "v_mad_i64_i32 %3, %8, %12, %17, %18\n\t"
      "v_mad_i64_i32 %4, %8, %13, %17, %18\n\t"
      "v_mad_i64_i32 %5, %8, %14, %17, %18\n\t"
      "v_mad_i64_i32 %6, %8, %15, %17, %18\n\t"
      "v_mad_i64_i32 %7, %8, %16, %17, %18"
      : "=&v"(p0), "=&v"(p1), "=&v"(p2), "=&v"(p3), "=&v"(p4), "=&v"(p5), "=&v"(p6), "=&v"(p7), "=&s"(carry)
      : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]), "s"(m), "v"(r));
  v[0] = static_cast<int>(p0 >> 32);
  v[1] = static_cast<int>(p1 >> 32);
  v[2] = static_cast<int>(p2 >> 32);
  v[3] = static_cast<int>(p3 >> 32);
  v[4] = static_cast<int>(p4 >> 32);
  v[5] = static_cast<int>(p5 >> 32);
  v[6] = static_cast<int>(p6 >> 32);
  v[7] = static_cast<int>(p7 >> 32);
}

// multiply sixteen values by M / 2^P, rounding half up: (v M + 2^(P-1)) >> P
template <int32_t M>
__device__ __forceinline__ void compensate(int (&a)[8], int (&b)[8]) {
#pragma unroll
  for (int L = 0; L < 8; ++L) {
    a[L] = static_cast<int>(static_cast<uint32_t>(a[L]) << kCompShift<M>);
    b[L] = static_cast<int>(static_cast<uint32_t>(b[L]) << kCompShift<M>);
  }
  comp_mul8<M>(a);
  comp_mul8<M>(b);
}

// the micro-rotations of the three rotation blocks of all eight lines, step by step
template <int N, int S, int I = 0>
__device__ __forceinline__ void cordic_lines(int (&a1)[8], int (&b1)[8], int (&a3)[8], int (&b3)[8],
                                             int (&a6)[8], int (&b6)[8]) {
  if constexpr (I < N) {
#pragma unroll
    for (int L = 0; L < 8; ++L) {
      cordic_step<N, kRot1, S, I>(a1[L], b1[L]);
      cordic_step<N, kRot3, S, I>(a3[L], b3[L]);
      cordic_step<N, kRot6, S, I>(a6[L], b6[L]);
    }
    cordic_lines<N, S, I + 1>(a1, b1, a3, b3, a6, b6);
  }
}

// the gain compensations of the three rotation blocks of all eight lines
template <int N>
__device__ __forceinline__ void gains_lines(int (&a1)[8], int (&b1)[8], int (&a3)[8], int (&b3)[8],
                                            int (&a6)[8], int (&b6)[8]) {
  compensate<kTablesN<N>.gain[kRot1]>(a1, b1);
  compensate<kTablesN<N>.gain[kRot3]>(a3, b3);
  compensate<kTablesN<N>.gain[kRot6]>(a6, b6);
}

// element k of line L: rows when kRows, columns otherwise
template <bool kRows>
__device__ __forceinline__ int &at(int (&x)[64], int line, int k) {
  return kRows ? x[line * 8 + k] : x[k * 8 + line];
}

// forward graph on the eight rows (kRows) or columns of a block, in place
template <int N, bool kRows>
__device__ __forceinline__ void forward_pass(int (&x)[64]) {
  int e0[8], e1[8], a6[8], b6[8], a3[8], b3[8], a1[8], b1[8];
#pragma unroll
  for (int L = 0; L < 8; ++L) {
    int v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = at<kRows>(x, L, k);
    // stage 1
    const int s0 = v[0] + v[7], s1 = v[1] + v[6], s2 = v[2] + v[5], s3 = v[3] + v[4];
    const int d0 = v[0] - v[7], d1 = v[1] - v[6], d2 = v[2] - v[5], d3 = v[3] - v[4];
    // stage 2, even half; the rotation inputs
    e0[L] = s0 + s3;
    e1[L] = s1 + s2;
    a6[L] = s1 - s2;  // e2
    b6[L] = s0 - s3;  // e3
    a3[L] = d3;       // (u4, u7) = R(d3, d0; 3pi/16)
    b3[L] = d0;
    a1[L] = d2;       // (u5, u6) = R(d2, d1; pi/16)
    b1[L] = d1;
  }
  cordic_lines<N, +1>(a1, b1, a3, b3, a6, b6);
  region();
  gains_lines<N>(a1, b1, a3, b3, a6, b6);
  region();
  int v5[8], v6[8];
#pragma unroll
  for (int L = 0; L < 8; ++L) {
    // stage 3
    const int v4 = a3[L] + b1[L], v7 = b3[L] + a1[L];
    v6[L] = a3[L] - b1[L];
    v5[L] = b3[L] - a1[L];
    at<kRows>(x, L, 0) = e0[L] + e1[L];
    at<kRows>(x, L, 4) = e0[L] - e1[L];
    at<kRows>(x, L, 2) = a6[L];
    at<kRows>(x, L, 6) = b6[L];
    // stage 4, butterfly
    at<kRows>(x, L, 1) = v7 + v4;
    at<kRows>(x, L, 7) = v7 - v4;
  }
  region();
  // stage 4, the two sqrt(2) factors
  compensate<kTablesN<N>.sqrt2>(v5, v6);
#pragma unroll
  for (int L = 0; L < 8; ++L) {
    at<kRows>(x, L, 3) = v5[L];
    at<kRows>(x, L, 5) = v6[L];
  }
  region();
}

// inverse (transposed) graph on the eight columns or rows of a block, in place
template <int N, bool kRows>
__device__ __forceinline__ void inverse_pass(int (&x)[64]) {
  // stage 4 transposed: v5 = sqrt2 Z3, v6 = sqrt2 Z5
  int v5[8], v6[8];
#pragma unroll
  for (int L = 0; L < 8; ++L) {
    v5[L] = at<kRows>(x, L, 3);
    v6[L] = at<kRows>(x, L, 5);
  }
  compensate<kTablesN<N>.sqrt2>(v5, v6);
  region();
  int e0[8], e1[8], a6[8], b6[8], a3[8], b3[8], a1[8], b1[8];
#pragma unroll
  for (int L = 0; L < 8; ++L) {
    const int z0 = at<kRows>(x, L, 0), z1 = at<kRows>(x, L, 1), z2 = at<kRows>(x, L, 2);
    const int z4 = at<kRows>(x, L, 4), z6 = at<kRows>(x, L, 6), z7 = at<kRows>(x, L, 7);
    const int v7 = z1 + z7, v4 = z1 - z7;
    // stage 3 transposed
    e0[L] = z0 + z4;
    e1[L] = z0 - z4;
    a6[L] = z2;  // (e2, e3) = sqrt2 R(Z2, Z6; -6pi/16)
    b6[L] = z6;
    a3[L] = v4 + v6[L];  // u4
    b3[L] = v7 + v5[L];  // u7: (t4, t7) = R(u4, u7; -3pi/16)
    a1[L] = v7 - v5[L];  // u5
    b1[L] = v4 - v6[L];  // u6: (t5, t6) = R(u5, u6; -pi/16)
  }
  cordic_lines<N, -1>(a1, b1, a3, b3, a6, b6);
  region();
  gains_lines<N>(a1, b1, a3, b3, a6, b6);
  region();
#pragma unroll
  for (int L = 0; L < 8; ++L) {
    // stage 2 and stage 1 transposed: d0 = t7, d1 = t6, d2 = t5, d3 = t4
    const int s0 = e0[L] + b6[L], s3 = e0[L] - b6[L], s1 = e1[L] + a6[L], s2 = e1[L] - a6[L];
    at<kRows>(x, L, 0) = s0 + b3[L];
    at<kRows>(x, L, 7) = s0 - b3[L];
    at<kRows>(x, L, 1) = s1 + b1[L];
    at<kRows>(x, L, 6) = s1 - b1[L];
    at<kRows>(x, L, 2) = s2 + a1[L];
    at<kRows>(x, L, 5) = s2 - a1[L];
    at<kRows>(x, L, 3) = s3 + a3[L];
    at<kRows>(x, L, 4) = s3 - a3[L];
  }
  region();
}

}  // namespace dct
