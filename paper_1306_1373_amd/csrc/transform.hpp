// transform.hpp -- device-side 8-point Cordic-based Loeffler flow graphs.
//
// One call transforms eight int32 values held in registers.  The forward graph
// is the four-stage Loeffler 8-point DCT of Sec. 2.5.2 (stage 1 butterflies;
// stage 2 even butterflies and the odd 3pi/16 and pi/16 rotations; stage 3 the
// DC/Nyquist butterfly, the sqrt(2)-scaled 6pi/16 rotation and the odd
// butterflies; stage 4 the last odd butterfly and two sqrt(2) factors).  Its
// output is 2 sqrt(2) times the orthonormal DCT-II of the input, in the same
// fixed point.  The inverse graph is its transpose: stages in reverse order,
// every rotation by -theta.
//
// Every rotation block is kIter micro-rotations with the directions of
// recipe.hpp resolved at compile time (so each step is two shifts and two
// adds), followed by the gain compensation (v M + 2^(P-1)) >> P with a 64-bit
// product.  All shifts are arithmetic; the values never leave int32 (the
// largest magnitude any step stores is below 2^29 for every input a uint8 plane
// or a clamped dequantized block can produce).
#pragma once

#include <hip/hip_runtime.h>

#include "recipe.hpp"

namespace dct {

// kIter micro-rotations, step I onwards; S = +1 rotates by +theta, S = -1 by -theta
template <int R, int S, int I = 0>
__device__ __forceinline__ void cordic_steps(int &a, int &b) {
  if constexpr (I < kIter) {
    constexpr int d = S * kTables.dir[R][I];
    const int sa = a >> I;
    const int sb = b >> I;
    if constexpr (d > 0) {
      a = a + sb;
      b = b - sa;
    } else {
      a = a - sb;
      b = b + sa;
    }
    cordic_steps<R, S, I + 1>(a, b);
  }
}

// multiply by M / 2^P, rounding half up
template <int32_t M>
__device__ __forceinline__ int compensate(int v) {
  return static_cast<int>((static_cast<long long>(v) * M + (1LL << (kComp - 1))) >> kComp);
}

// rotation block R(a, b; S theta_R) = (a cos + b sin, -a sin + b cos), scaled
// by sqrt(2) for the 6pi/16 block
template <int R, int S>
__device__ __forceinline__ void rotate(int &a, int &b) {
  cordic_steps<R, S>(a, b);
  a = compensate<kTables.gain[R]>(a);
  b = compensate<kTables.gain[R]>(b);
}

// forward 8-point graph, in place: x0..x7 -> Z0..Z7
__device__ __forceinline__ void loeffler_fwd(int &x0, int &x1, int &x2, int &x3, int &x4, int &x5,
                                             int &x6, int &x7) {
  // stage 1
  const int s0 = x0 + x7, s1 = x1 + x6, s2 = x2 + x5, s3 = x3 + x4;
  const int d0 = x0 - x7, d1 = x1 - x6, d2 = x2 - x5, d3 = x3 - x4;
  // stage 2
  const int e0 = s0 + s3, e3 = s0 - s3, e1 = s1 + s2, e2 = s1 - s2;
  int u4 = d3, u7 = d0, u5 = d2, u6 = d1;
  rotate<kRot3, +1>(u4, u7);
  rotate<kRot1, +1>(u5, u6);
  // stage 3
  int z2 = e2, z6 = e3;
  rotate<kRot6, +1>(z2, z6);
  const int v4 = u4 + u6, v6 = u4 - u6, v7 = u7 + u5, v5 = u7 - u5;
  // stage 4
  x0 = e0 + e1;
  x4 = e0 - e1;
  x2 = z2;
  x6 = z6;
  x1 = v7 + v4;
  x7 = v7 - v4;
  x3 = compensate<kTables.sqrt2>(v5);
  x5 = compensate<kTables.sqrt2>(v6);
}

// inverse (transposed) 8-point graph, in place: Z0..Z7 -> x0..x7
__device__ __forceinline__ void loeffler_inv(int &z0, int &z1, int &z2, int &z3, int &z4, int &z5,
                                             int &z6, int &z7) {
  // stage 4 transposed
  const int v7 = z1 + z7, v4 = z1 - z7;
  const int v5 = compensate<kTables.sqrt2>(z3), v6 = compensate<kTables.sqrt2>(z5);
  // stage 3 transposed
  const int e0 = z0 + z4, e1 = z0 - z4;
  int e2 = z2, e3 = z6;
  rotate<kRot6, -1>(e2, e3);
  int u4 = v4 + v6, u6 = v4 - v6, u7 = v7 + v5, u5 = v7 - v5;
  // stage 2 transposed
  rotate<kRot3, -1>(u4, u7);
  rotate<kRot1, -1>(u5, u6);
  const int s0 = e0 + e3, s3 = e0 - e3, s1 = e1 + e2, s2 = e1 - e2;
  // stage 1 transposed (d0 = u7, d1 = u6, d2 = u5, d3 = u4)
  z0 = s0 + u7;
  z7 = s0 - u7;
  z1 = s1 + u6;
  z6 = s1 - u6;
  z2 = s2 + u5;
  z5 = s2 - u5;
  z3 = s3 + u4;
  z4 = s3 - u4;
}

// 2-D forward on a register block x[i*8 + j]: row pass, then column pass.
// Input (p - 128) << F; output c[u*8 + v] with coefficient = c / 2^(F+3).
__device__ __forceinline__ void forward_block(int (&x)[64]) {
#pragma unroll
  for (int i = 0; i < 8; ++i)
    loeffler_fwd(x[i * 8 + 0], x[i * 8 + 1], x[i * 8 + 2], x[i * 8 + 3], x[i * 8 + 4], x[i * 8 + 5],
                 x[i * 8 + 6], x[i * 8 + 7]);
#pragma unroll
  for (int j = 0; j < 8; ++j)
    loeffler_fwd(x[0 * 8 + j], x[1 * 8 + j], x[2 * 8 + j], x[3 * 8 + j], x[4 * 8 + j], x[5 * 8 + j],
                 x[6 * 8 + j], x[7 * 8 + j]);
}

// 2-D inverse on a register block: column pass, then row pass.
__device__ __forceinline__ void inverse_block(int (&x)[64]) {
#pragma unroll
  for (int j = 0; j < 8; ++j)
    loeffler_inv(x[0 * 8 + j], x[1 * 8 + j], x[2 * 8 + j], x[3 * 8 + j], x[4 * 8 + j], x[5 * 8 + j],
                 x[6 * 8 + j], x[7 * 8 + j]);
#pragma unroll
  for (int i = 0; i < 8; ++i)
    loeffler_inv(x[i * 8 + 0], x[i * 8 + 1], x[i * 8 + 2], x[i * 8 + 3], x[i * 8 + 4], x[i * 8 + 5],
                 x[i * 8 + 6], x[i * 8 + 7]);
}

}  // namespace dct
