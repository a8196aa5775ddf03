// recipe.hpp -- compile-time constants of the integer Cordic-based Loeffler recipe.
//
// The Loeffler 8-point flow graph (Sec. 2.5.2) has three rotation blocks, by
// pi/16, 3pi/16 and 6pi/16; the last one also carries a factor sqrt(2), and two
// odd outputs are scaled by sqrt(2).  Each rotation block is computed as
// n CORDIC micro-rotations
//     a' = a + d_i (b >> i),   b' = b - d_i (a >> i)
// followed by one gain-compensation multiply (v M + 2^(P-1)) >> P.  A recipe
// R(n, F, G) also fixes F, the fractional bits of the forward transform's
// samples, and G, those of the inverse's; the default is R(10, 12, 12).
//
// Everything here is derived at compile time from first principles so that the
// kernels carry the directions and gains as immediates:
//   * pi from Machin's formula pi/4 = 4 atan(1/5) - atan(1/239);
//   * atan(x) for |x| <= 1/2 from its Taylor series;
//   * sqrt from Newton's iteration;
//   * d_i from the greedy CORDIC rule: z_0 = theta, d_i = +1 if z_i >= 0 else -1,
//     z_{i+1} = z_i - d_i atan(2^-i)  (the smallest |z_i| at a decision is
//     5.7e-4 rad, far above any rounding of this derivation);
//   * the gain K_n = prod_{i<n} sqrt(1 + 2^-2i) and M = round(k 2^P / K_n).
#pragma once

#include <cstdint>

namespace dct {

inline constexpr int kIter = 10;     // default CORDIC micro-rotations per rotation block (n)
inline constexpr int kFrac = 12;     // default fractional bits of the samples (F = G)
inline constexpr int kComp = 15;     // fractional bits of the gain constants (P)
inline constexpr int kMaxIter = 16;

namespace detail {

// atan(x) by its Taylor series; converges geometrically for |x| <= 1/2
constexpr double atan_series(double x) {
  double term = x, sum = 0.0, x2 = x * x;
  for (int k = 0; k < 60; ++k) {
    sum += (k % 2 == 0 ? term : -term) / (2 * k + 1);
    term *= x2;
  }
  return sum;
}

// atan(1/q) for q >= 2
constexpr double atan_inv(double q) { return atan_series(1.0 / q); }

constexpr double kPi = 4.0 * (4.0 * atan_inv(5.0) - atan_inv(239.0));

// atan(2^-i); i = 0 is pi/4
constexpr double atan_pow2(int i) {
  if (i == 0) return kPi / 4.0;
  double x = 1.0;
  for (int k = 0; k < i; ++k) x *= 0.5;
  return atan_series(x);
}

constexpr double sqrt_newton(double a) {
  double x = a > 1.0 ? a : 1.0;
  for (int k = 0; k < 100; ++k) x = 0.5 * (x + a / x);
  return x;
}

constexpr double pow2(int e) {
  double v = 1.0;
  for (int k = 0; k < (e < 0 ? -e : e); ++k) v = e < 0 ? v * 0.5 : v * 2.0;
  return v;
}

constexpr int32_t round_pos(double v) { return static_cast<int32_t>(v + 0.5); }

}  // namespace detail

// rotation blocks of the graph
enum Rot : int { kRot1 = 0, kRot3 = 1, kRot6 = 2 };

template <int N>
struct Tables {
  int dir[3][N];    // CORDIC directions of the pi/16, 3pi/16, 6pi/16 blocks
  int32_t gain[3];  // M of each block; the 6pi/16 block includes sqrt(2)
  int32_t sqrt2;    // round(sqrt(2) 2^P) for the odd sqrt(2) factors
};

template <int N>
constexpr Tables<N> make_tables() {
  static_assert(N >= 1 && N <= kMaxIter, "micro-rotation count");
  Tables<N> t{};
  const double theta[3] = {detail::kPi / 16.0, 3.0 * detail::kPi / 16.0, 6.0 * detail::kPi / 16.0};
  const double k[3] = {1.0, 1.0, detail::sqrt_newton(2.0)};
  double K = 1.0;
  for (int i = 0; i < N; ++i) K *= detail::sqrt_newton(1.0 + detail::pow2(-2 * i));
  for (int r = 0; r < 3; ++r) {
    double z = theta[r];
    for (int i = 0; i < N; ++i) {
      const int d = z >= 0.0 ? 1 : -1;
      t.dir[r][i] = d;
      z -= d * detail::atan_pow2(i);
    }
    t.gain[r] = detail::round_pos(k[r] * detail::pow2(kComp) / K);
  }
  t.sqrt2 = detail::round_pos(detail::sqrt_newton(2.0) * detail::pow2(kComp));
  return t;
}

template <int N>
inline constexpr Tables<N> kTablesN = make_tables<N>();

inline constexpr Tables<kIter> kTables = kTablesN<kIter>;

// A recipe R(n, F, G).  F and G bound what int32 holds: the forward transform
// of p 2^F stores at most 2^(F + 14) (the DC path of a 255 block) and the
// inverse of clamped dequantized values at most 2^(G + 16.9).
template <int N, int F, int G>
struct Recipe {
  static constexpr int n = N;
  static constexpr int frac = F;
  static constexpr int inv_frac = G;
  static_assert(F >= 8 && F <= 16, "forward fractional bits");
  static_assert(G >= 8 && G <= 12, "inverse fractional bits");
};

using DefaultRecipe = Recipe<kIter, kFrac, kFrac>;

// the gains stay within the operand range the kernels rely on
static_assert(kTables.gain[kRot1] > 0 && kTables.gain[kRot1] < (1 << 16), "gain range");
static_assert(kTables.gain[kRot6] > 0 && kTables.gain[kRot6] < (1 << 16), "gain range");
static_assert(kTables.sqrt2 > 0 && kTables.sqrt2 < (1 << 16), "gain range");
static_assert(kTablesN<4>.gain[kRot6] < (1 << 16) && kTablesN<16>.gain[kRot1] > 0, "gain range");

}  // namespace dct
