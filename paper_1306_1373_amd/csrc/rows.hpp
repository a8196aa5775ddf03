// rows.hpp -- the fused codec with one lane per block row and the row-to-column
// transposes staged through LDS (the mapping of the paper's Sec. 2.4 shared-
// memory design): the kernel of dct_codec and dct_codec_accumulate.  The
// lane-per-block kernel of kernels.hpp, which keeps a block in one lane's
// registers, serves the recipe family, the batch and dct_codec_blocks.
//
// A wave codes eight horizontally consecutive blocks; lane (j, r) = (lane % 8,
// lane / 8) owns row r of block j for the row passes and column r of block j
// for the column passes, and the two transposes go through a wave-private LDS
// tile of the eight blocks (64 int32 each, laid out so that neither the stores
// nor the loads of a transpose meet in a bank).  Lanes with the same r read
// and write 64 contiguous bytes of the plane.  Every value is the same integer
// as in the lane-per-block kernel: the 1-D graphs below perform the same
// operations as forward_pass / inverse_pass on one line.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "transform.hpp"

namespace dct {
namespace rows {

// the high word of (v 2^k)(M 2^(17-k)) + 2^31, i.e. (v M + 2^14) >> 15
template <int32_t M>
__device__ __forceinline__ int comp1(int v) {
  const long long p = static_cast<long long>(static_cast<int>(static_cast<uint32_t>(v) << kCompShift<M>)) *
                          static_cast<long long>(kCompMul<M>) +
                      (1LL << 31);
  return static_cast<int>(p >> 32);
}

template <int N, int S, int I = 0>
__device__ __forceinline__ void cordic_line(int &a1, int &b1, int &a3, int &b3, int &a6, int &b6) {
  if constexpr (I < N) {
    cordic_step<N, kRot1, S, I>(a1, b1);
    cordic_step<N, kRot3, S, I>(a3, b3);
    cordic_step<N, kRot6, S, I>(a6, b6);
    cordic_line<N, S, I + 1>(a1, b1, a3, b3, a6, b6);
  }
}

template <int N>
__device__ __forceinline__ void gains_line(int &a1, int &b1, int &a3, int &b3, int &a6, int &b6) {
  a1 = comp1<kTablesN<N>.gain[kRot1]>(a1);
  b1 = comp1<kTablesN<N>.gain[kRot1]>(b1);
  a3 = comp1<kTablesN<N>.gain[kRot3]>(a3);
  b3 = comp1<kTablesN<N>.gain[kRot3]>(b3);
  a6 = comp1<kTablesN<N>.gain[kRot6]>(a6);
  b6 = comp1<kTablesN<N>.gain[kRot6]>(b6);
}

// forward graph on one line, in place (natural output order Z0 .. Z7)
template <int N>
__device__ __forceinline__ void forward_line(int (&v)[8]) {
  const int s0 = v[0] + v[7], s1 = v[1] + v[6], s2 = v[2] + v[5], s3 = v[3] + v[4];
  const int d0 = v[0] - v[7], d1 = v[1] - v[6], d2 = v[2] - v[5], d3 = v[3] - v[4];
  const int e0 = s0 + s3, e1 = s1 + s2;
  int a6 = s1 - s2, b6 = s0 - s3, a3 = d3, b3 = d0, a1 = d2, b1 = d1;
  cordic_line<N, +1>(a1, b1, a3, b3, a6, b6);
  gains_line<N>(a1, b1, a3, b3, a6, b6);
  const int v4 = a3 + b1, v7 = b3 + a1, v6 = a3 - b1, v5 = b3 - a1;
  v[0] = e0 + e1;
  v[4] = e0 - e1;
  v[2] = a6;
  v[6] = b6;
  v[1] = v7 + v4;
  v[7] = v7 - v4;
  v[3] = comp1<kTablesN<N>.sqrt2>(v5);
  v[5] = comp1<kTablesN<N>.sqrt2>(v6);
}

// inverse (transposed) graph on one line, in place
template <int N>
__device__ __forceinline__ void inverse_line(int (&z)[8]) {
  const int v5 = comp1<kTablesN<N>.sqrt2>(z[3]), v6 = comp1<kTablesN<N>.sqrt2>(z[5]);
  const int v7 = z[1] + z[7], v4 = z[1] - z[7];
  const int e0 = z[0] + z[4], e1 = z[0] - z[4];
  int a6 = z[2], b6 = z[6], a3 = v4 + v6, b3 = v7 + v5, a1 = v7 - v5, b1 = v4 - v6;
  cordic_line<N, -1>(a1, b1, a3, b3, a6, b6);
  gains_line<N>(a1, b1, a3, b3, a6, b6);
  const int s0 = e0 + b6, s3 = e0 - b6, s1 = e1 + a6, s2 = e1 - a6;
  z[0] = s0 + b3;
  z[7] = s0 - b3;
  z[1] = s1 + b1;
  z[6] = s1 - b1;
  z[2] = s2 + a1;
  z[5] = s2 - a1;
  z[3] = s3 + a3;
  z[4] = s3 - a3;
}

inline constexpr int kThreads = 256;               // four waves

// Workgroups of a launch over ngroups groups of eight blocks.  A wave that codes
// one group spends much of its life starting up, so waves take four groups
// each once the image is large enough to fill the device that way; smaller images
// give each wave one group (their time is one wave's latency).  Measured at
// 8192 x 8192: one group per wave 245 us, four 143 us, sixteen 145 us.
inline unsigned launch_groups(int ngroups) {
  const int one = (ngroups + 3) / 4, four = (ngroups + 15) / 16;
  if (one <= 1024) return static_cast<unsigned>(one);
  return static_cast<unsigned>(four > 8192 ? 8192 : (four < 1024 ? 1024 : four));
}
// LDS layout of a wave's tile: element (a, b) of block j (a the pass's output
// index, b the line) at word 76 j + 9 a + b.  The LDS takes a wave's 64 accesses
// as two halves of 32 lanes (j = 0..7, b or a = 0..3 and 4..7) over 32 banks: a
// row-pass store (fixed a, lanes (j, b)) hits banks 12 j + b + 9 a (mod 32) and a
// column-pass load (fixed b, lanes (j, a)) hits 12 j + 9 a + b (mod 32), 32
// different banks in each half both ways (a 72-word block, conflict-free for 64
// banks, collides blocks j and j + 4).
inline constexpr int kPitch = 9;                   // LDS words per line of a block tile
inline constexpr int kTile = 76;                   // words per block

// a1..a9 under recipe RC, one lane per block row; each wave codes groups of
// eight blocks, group g = blockIdx.x * 4 + wave, g += gridDim.x * 4
template <class RC, bool kEmitQ>
__global__ __launch_bounds__(kThreads) void codec_rows_kernel(const uint8_t *__restrict__ src, int W, int H,
                                                              int src_stride, int bw, int nblocks, CodecQuant qa,
                                                              uint8_t *__restrict__ dst, int dst_stride,
                                                              int16_t *__restrict__ qcoef,
                                                              unsigned long long *__restrict__ sse) {
  constexpr int F = RC::frac, G = RC::inv_frac, N = RC::n;
  __shared__ int tile[kThreads / 64][8 * kTile];
  __shared__ float q_rcp[15], q_scale[15];
  __shared__ int q_half[15];
  if (threadIdx.x < 15) {
    q_rcp[threadIdx.x] = qa.rcp[threadIdx.x];
    q_scale[threadIdx.x] = qa.qscale[threadIdx.x];
    q_half[threadIdx.x] = qa.half[threadIdx.x];
  }
  __syncthreads();
  const int wave = wave_index();
  const int l = static_cast<int>(threadIdx.x & 63), j = l & 7, r = l >> 3;
  int *T = tile[wave] + j * kTile;
  // the quantizer of column r: entries s = u + r for u = 0..7
  float rcp[8], qsc[8];
  int half[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    rcp[u] = q_rcp[u + r];
    qsc[u] = q_scale[u + r];
    half[u] = q_half[u + r];
  }
  uint64_t err = 0;
  const int ngroups = (nblocks + 7) / 8;
  for (int grp = blockIdx.x * (kThreads / 64) + wave; grp < ngroups; grp += gridDim.x * (kThreads / 64)) {
    // block grp * 8 + j: one scalar division per group (grp is wave-uniform); a
    // lane wraps at most once into the next block row when a row holds at least
    // eight blocks, else it divides
    const int b0 = grp * 8, b = b0 + j;
    const bool live = b < nblocks;
    int by, bx;
    if (bw >= 8) {
      const int by0 = b0 / bw;
      bx = b0 - by0 * bw + j;
      const bool wrap = bx >= bw;
      bx = wrap ? bx - bw : bx;
      by = by0 + (wrap ? 1 : 0);
    } else {
      by = b / bw;
      bx = b - by * bw;
    }
    by = live ? by : 0;
    bx = live ? bx : 0;
    const int x0 = bx * 8, y = by * 8 + r;
    const bool full = live && x0 + 8 <= W && by * 8 + 8 <= H;
    // a1: this lane's row (edge rows and columns repeat the last pixel)
    uint32_t w0 = 0, w1 = 0;
    if (full) {
      const uint2 w = *reinterpret_cast<const uint2 *>(src + (static_cast<uint32_t>(y) * static_cast<uint32_t>(src_stride) +
                                                              static_cast<uint32_t>(x0)));
      w0 = w.x;
      w1 = w.y;
    } else if (live) {
      const uint8_t *row = src + static_cast<size_t>(min(y, H - 1)) * src_stride;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        w0 |= static_cast<uint32_t>(row[min(x0 + k, W - 1)]) << (8 * k);
        w1 |= static_cast<uint32_t>(row[min(x0 + 4 + k, W - 1)]) << (8 * k);
      }
    }
    int x[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[k] = static_cast<int>((w0 >> (8 * k)) & 0xffu) << F;
      x[4 + k] = static_cast<int>((w1 >> (8 * k)) & 0xffu) << F;
    }
    // a2 row pass, a3 transpose: T[v][r] = row r's coefficient v
    forward_line<N>(x);
#pragma unroll
    for (int v = 0; v < 8; ++v) T[v * kPitch + r] = x[v];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // a4 column pass on column r
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = T[r * kPitch + u];
    forward_line<N>(x);
    if (r == 0) x[0] -= kLevelShiftDC<F>;
    // a5, a6
    int q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = quant_dequant<F>(x[u], rcp[u], qsc[u], half[u], q[u]);
    if constexpr (kEmitQ) {
      if (live) {
        int16_t *out = qcoef + static_cast<size_t>(b) * 64 + r;
#pragma unroll
        for (int u = 0; u < 8; ++u) out[u * 8] = static_cast<int16_t>(q[u]);
      }
    }
    if (r == 0) x[0] += kReconstructDC<G>;
    // a7 inverse column pass, transpose back: T[i][r] = row i's value in column r
    inverse_line<N>(x);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < 8; ++i) T[i * kPitch + r] = x[i];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = T[r * kPitch + k];
    inverse_line<N>(x);
    // a8: pack and store this lane's row; a9: its SSE against the loaded pixels
    uint32_t o0 = 0, o1 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      o0 |= static_cast<uint32_t>(min(max(x[k] >> (G + 3), 0), 255)) << (8 * k);
      o1 |= static_cast<uint32_t>(min(max(x[4 + k] >> (G + 3), 0), 255)) << (8 * k);
    }
    if (full) {
      *reinterpret_cast<uint2 *>(dst + (static_cast<uint32_t>(y) * static_cast<uint32_t>(dst_stride) +
                                        static_cast<uint32_t>(x0))) = make_uint2(o0, o1);
      uint32_t e = __builtin_amdgcn_udot4(w0, w0, 0u, false);
      e = __builtin_amdgcn_udot4(w1, w1, e, false);
      e = __builtin_amdgcn_udot4(o0, o0, e, false);
      e = __builtin_amdgcn_udot4(o1, o1, e, false);
      const uint32_t c = __builtin_amdgcn_udot4(w1, o1, __builtin_amdgcn_udot4(w0, o0, 0u, false), false);
      err += static_cast<uint32_t>(e - 2u * c);
    } else if (live && y < H) {
      uint8_t *row = dst + static_cast<size_t>(y) * dst_stride;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (x0 + k < W) {
          const uint32_t pv = ((k < 4 ? o0 : o1) >> (8 * (k & 3))) & 0xffu;
          const uint32_t sv = ((k < 4 ? w0 : w1) >> (8 * (k & 3))) & 0xffu;
          row[x0 + k] = static_cast<uint8_t>(pv);
          err += (pv - sv) * (pv - sv);
        }
      }
    }
    // the next group's row-pass writes must not overtake this group's reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  workgroup_add<kThreads>(err, sse, wave);
}

}  // namespace rows
}  // namespace dct
