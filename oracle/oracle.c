/*
 * oracle.c -- CPU reference for the blockwise 8x8 Cordic-based Loeffler DCT codec.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle: a plain, slow,
 * obviously correct C implementation of what the codec computes.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.  The
 * product library (the HIP kernels behind include/dctcodec.h) never links,
 * includes or calls anything here, and nothing here includes or calls the
 * product library: the two share no source, header, table or constant.
 *
 * Contents, each following the paper (Modieginyane, Ncube, Gasela, "CUDA based
 * performance evaluation of the computational efficiency of the DCT image
 * compression technique on both the CPU and GPU"):
 *
 *   O1  exact 2-D DCT-II of an 8x8 block in FP64, straight from the definition
 *       (Sec. 2.5.1, eq. (6)-(7), read as the orthonormal DCT-II; O(N^4) sums).
 *   O2  exact 2-D inverse (orthonormal DCT-III), the F^-1 that Sec. 2.5.1 names
 *       but does not print.
 *   O3-O5  exact FP64 codec: table quantizer (Sec. 3.2 names a quantizer kernel),
 *       dequantizer, inverse, level shift back, round and clamp.
 *   O6  SSE / MSE / PSNR (Sec. 4.1, eq. (23)-(24)).
 *   O7  the integer Cordic-based Loeffler recipe R(n, F, G) with P = 15: the
 *       Loeffler 8-point flow graph in four stages (Sec. 2.5.2) with every
 *       rotation block done as n fixed-point CORDIC shift-add micro-rotations
 *       plus one gain-compensation multiply; F fractional bits in the forward
 *       transform, G in the inverse.  The default recipe is R(10, 12, 12).  The figure with the flow graph is
 *       missing from the paper; the graph here is derived from the DCT-II
 *       definition and pinned against it by the tests.
 *   An FP64 version of the same Loeffler graph with exact rotations, used by the
 *   tests to pin the graph's structure against 2*sqrt(2)*C.
 *
 * Arithmetic conventions of the recipe (fixed here because the paper gives none):
 *   * all recipe values are held in int64 so that nothing can wrap; every value
 *     the recipe stores is reported through *peak so tests can check that an
 *     int32 implementation never overflows;
 *   * every right shift is a floor division by a power of two, written out with
 *     truncating C division and an explicit correction for negative operands.
 *
 * Parity status: O1, O2, O3-O6 and the structure of O7 are pinned by closed
 * forms, library routines and invariants in tests/.  The exact bit pattern of
 * the O7 integer recipe (where each floor falls) has no independent printed
 * value to check against; the tests pin it by exactness on constant blocks,
 * error bounds against O1, the overflow bound, and an exhaustive check of the
 * quantizer division.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_NITER 10 /* default CORDIC micro-rotations per rotation block (n) */
#define OR_FRAC 12  /* default fractional bits of the fixed-point samples (F = G) */
#define OR_PBITS 15 /* fractional bits of the gain-compensation constants (P) */
#define OR_MAX_NITER 16

/* ------------------------------------------------------------------------- */
/* helpers                                                                    */
/* ------------------------------------------------------------------------- */

static double or_pi(void) { return acos(-1.0); }

/* floor(v / 2^s) for any sign of v, written as the textbook floor division. */
static int64_t floor_div_pow2(int64_t v, int s) {
  const int64_t d = (int64_t)1 << s;
  int64_t q = v / d; /* C division truncates toward zero */
  if (v % d != 0 && v < 0) q -= 1;
  return q;
}

static int64_t i64_abs(int64_t v) { return v < 0 ? -v : v; }

static void track(int64_t *peak, int64_t v) {
  if (peak && i64_abs(v) > *peak) *peak = i64_abs(v);
}

/* pixel (y, x) of a plane, replicating the last row / column for positions
   beyond the image (the block grid is ceil(H/8) x ceil(W/8)) */
static int pixel_at(const uint8_t *p, int W, int H, int stride, int y, int x) {
  if (y > H - 1) y = H - 1;
  if (x > W - 1) x = W - 1;
  return p[(int64_t)y * stride + x];
}

/* ------------------------------------------------------------------------- */
/* O1 / O2: the definition of the 2-D DCT-II and its inverse, N = M = 8        */
/* ------------------------------------------------------------------------- */

/* normalising factor alpha of eq. (4)/(7), indexed by the frequency */
static double alpha(int k) { return k == 0 ? 1.0 / sqrt(2.0) : 1.0; }

/* F(u,v) = sqrt(2/8) sqrt(2/8) alpha(u) alpha(v)
 *          sum_i sum_j cos[pi u (2i+1) / 16] cos[pi v (2j+1) / 16] f(i,j)
 * f and F are row-major 8x8; i, u index rows, j, v index columns. */
void or_fdct8x8_f64(const double *f, double *F) {
  const double pi = or_pi();
  for (int u = 0; u < 8; ++u) {
    for (int v = 0; v < 8; ++v) {
      double s = 0.0;
      for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j)
          s += cos(pi * u * (2 * i + 1) / 16.0) * cos(pi * v * (2 * j + 1) / 16.0) *
               f[i * 8 + j];
      F[u * 8 + v] = sqrt(2.0 / 8.0) * sqrt(2.0 / 8.0) * alpha(u) * alpha(v) * s;
    }
  }
}

/* f(i,j) = sqrt(2/8) sqrt(2/8) sum_u sum_v alpha(u) alpha(v)
 *          cos[pi u (2i+1) / 16] cos[pi v (2j+1) / 16] F(u,v) */
void or_idct8x8_f64(const double *F, double *f) {
  const double pi = or_pi();
  for (int i = 0; i < 8; ++i) {
    for (int j = 0; j < 8; ++j) {
      double s = 0.0;
      for (int u = 0; u < 8; ++u)
        for (int v = 0; v < 8; ++v)
          s += alpha(u) * alpha(v) * cos(pi * u * (2 * i + 1) / 16.0) *
               cos(pi * v * (2 * j + 1) / 16.0) * F[u * 8 + v];
      f[i * 8 + j] = sqrt(2.0 / 8.0) * sqrt(2.0 / 8.0) * s;
    }
  }
}

/* Image-level exact forward transform: level shift p - 128, then O1 on every
 * block.  coef is [ceil(H/8) * ceil(W/8)][64], blocks in row-major block order. */
void or_exact_forward(const uint8_t *src, int W, int H, int stride, double *coef) {
  const int bw = (W + 7) / 8, bh = (H + 7) / 8;
  double f[64];
  for (int by = 0; by < bh; ++by)
    for (int bx = 0; bx < bw; ++bx) {
      for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j)
          f[i * 8 + j] = pixel_at(src, W, H, stride, by * 8 + i, bx * 8 + j) - 128.0;
      or_fdct8x8_f64(f, coef + ((int64_t)by * bw + bx) * 64);
    }
}

/* Quantization table Q[u][v] = 1 + (1 + u + v) * qs.  qs = 0 gives Q = 1. */
static int64_t qtable(int u, int v, int qs) { return 1 + (int64_t)(1 + u + v) * qs; }

/* O3: q = sgn(F) * floor(|F| / Q + 1/2)   (round half away from zero) */
static double quantize_f64(double F, int64_t Q) {
  const double m = floor(fabs(F) / (double)Q + 0.5);
  return F < 0 ? -m : m;
}

/* O5: round half up, then clamp to the 8-bit range */
static int reconstruct_f64(double f) {
  double p = floor(f + 128.0 + 0.5);
  if (p < 0) p = 0;
  if (p > 255) p = 255;
  return (int)p;
}

/* Exact FP64 codec (O1 -> O3 -> O4 -> O2 -> O5) on every block.  Writes the
 * W x H reconstruction; when qcoef is non-NULL it receives the quantized values
 * (as doubles, integral) in the coefficient layout. */
void or_exact_codec(const uint8_t *src, int W, int H, int stride, int qs, uint8_t *dst,
                    int dst_stride, double *qcoef) {
  const int bw = (W + 7) / 8, bh = (H + 7) / 8;
  double f[64], F[64], R[64];
  for (int by = 0; by < bh; ++by)
    for (int bx = 0; bx < bw; ++bx) {
      for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j)
          f[i * 8 + j] = pixel_at(src, W, H, stride, by * 8 + i, bx * 8 + j) - 128.0;
      or_fdct8x8_f64(f, F);
      for (int u = 0; u < 8; ++u)
        for (int v = 0; v < 8; ++v) {
          const int64_t Q = qtable(u, v, qs);
          const double q = quantize_f64(F[u * 8 + v], Q);
          if (qcoef) qcoef[((int64_t)by * bw + bx) * 64 + u * 8 + v] = q;
          F[u * 8 + v] = q * (double)Q; /* O4 */
        }
      or_idct8x8_f64(F, R);
      for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
          const int y = by * 8 + i, x = bx * 8 + j;
          if (y < H && x < W) dst[(int64_t)y * dst_stride + x] = (uint8_t)reconstruct_f64(R[i * 8 + j]);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* O6: SSE, MSE, PSNR (eq. (23)-(24))                                         */
/* ------------------------------------------------------------------------- */

/* SSE = sum over the W x H region of (O - C)^2, exact in 64-bit integers */
uint64_t or_sse(const uint8_t *a, int a_stride, const uint8_t *b, int b_stride, int W, int H) {
  uint64_t s = 0;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int64_t d = (int64_t)a[(int64_t)y * a_stride + x] - (int64_t)b[(int64_t)y * b_stride + x];
      s += (uint64_t)(d * d);
    }
  return s;
}

/* largest pixel value of plane a over W x H (the "MAX" of eq. (23) read as max(O)) */
int or_max_pixel(const uint8_t *a, int a_stride, int W, int H) {
  int m = 0;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      if (a[(int64_t)y * a_stride + x] > m) m = a[(int64_t)y * a_stride + x];
  return m;
}

/* PSNR = 20 log10(MAX / sqrt(MSE)),  MSE = SSE / (N M);  SSE = 0 gives +inf */
double or_psnr_from_sse(uint64_t sse, int W, int H, double peak) {
  if (sse == 0) return INFINITY;
  const double mse = (double)sse / ((double)W * (double)H);
  return 20.0 * log10(peak / sqrt(mse));
}

/* ------------------------------------------------------------------------- */
/* O7: the integer Cordic-based Loeffler recipe                                */
/* ------------------------------------------------------------------------- */

/* Rotation blocks of the Loeffler graph, in the order pi/16, 3pi/16, 6pi/16. */
enum { ROT_1 = 0, ROT_3 = 1, ROT_6 = 2 };

/* One recipe R(n, F, G): n micro-rotations per rotation block, F fractional
 * bits of the forward samples, G of the inverse samples, and its constants. */
typedef struct {
  int n, F, G;
  int dir[3][OR_MAX_NITER]; /* CORDIC direction d_i of each rotation block */
  int64_t gain[3];          /* gain compensation M of each rotation block */
  int64_t sqrt2;            /* round(sqrt(2) * 2^P) for the two odd sqrt(2) factors */
} recipe_t;

/* Directions: z_0 = theta, d_i = +1 if z_i >= 0 else -1, z_{i+1} = z_i - d_i atan(2^-i).
 * Gain: n micro-rotations scale a vector by K_n = prod_i sqrt(1 + 2^-2i); the
 * compensation constant is M = round(k 2^P / K_n), with k = sqrt(2) for the
 * even-part rotation that carries the sqrt(2) factor and k = 1 otherwise. */
static void recipe_make(recipe_t *R, int n, int F, int G) {
  const double pi = or_pi();
  const double theta[3] = {pi / 16.0, 3.0 * pi / 16.0, 6.0 * pi / 16.0};
  const double k[3] = {1.0, 1.0, sqrt(2.0)};
  R->n = n;
  R->F = F;
  R->G = G;
  double K = 1.0;
  for (int i = 0; i < n; ++i) K *= sqrt(1.0 + ldexp(1.0, -2 * i));
  for (int r = 0; r < 3; ++r) {
    double z = theta[r];
    for (int i = 0; i < n; ++i) {
      const int d = z >= 0.0 ? 1 : -1;
      R->dir[r][i] = d;
      z -= d * atan(ldexp(1.0, -i));
    }
    R->gain[r] = llround(k[r] * ldexp(1.0, OR_PBITS) / K);
  }
  R->sqrt2 = llround(sqrt(2.0) * ldexp(1.0, OR_PBITS));
}

static recipe_t g_default;
static pthread_once_t g_once = PTHREAD_ONCE_INIT;
static void default_init(void) { recipe_make(&g_default, OR_NITER, OR_FRAC, OR_FRAC); }
static const recipe_t *default_recipe(void) {
  pthread_once(&g_once, default_init);
  return &g_default;
}

/* recipes the oracle accepts: 1 <= n <= 16, 1 <= F <= 16, 1 <= G <= 12 */
int or_recipe_valid(int n, int F, int G) {
  return n >= 1 && n <= OR_MAX_NITER && F >= 1 && F <= 16 && G >= 1 && G <= 12;
}

void or_recipe_info(int *n_iter, int *frac_bits, int *comp_bits) {
  *n_iter = OR_NITER;
  *frac_bits = OR_FRAC;
  *comp_bits = OR_PBITS;
}

/* directions: 3 * n values, rotation blocks in the order pi/16, 3pi/16, 6pi/16;
 * gain: M(pi/16), M(3pi/16), M(6pi/16) (the last includes sqrt(2)), M_sqrt2 */
void or_recipe_tables_n(int n, int *directions, int64_t *gain) {
  recipe_t R;
  recipe_make(&R, n, OR_FRAC, OR_FRAC);
  for (int r = 0; r < 3; ++r)
    for (int i = 0; i < n; ++i) directions[r * n + i] = R.dir[r][i];
  for (int r = 0; r < 3; ++r) gain[r] = R.gain[r];
  gain[3] = R.sqrt2;
}

void or_recipe_tables(int *directions, int64_t *gain) { or_recipe_tables_n(OR_NITER, directions, gain); }

/* multiply by M / 2^P, rounding half up:  (v M + 2^(P-1)) floor/ 2^P */
static int64_t compensate(int64_t v, int64_t M) {
  return floor_div_pow2(v * M + ((int64_t)1 << (OR_PBITS - 1)), OR_PBITS);
}

/* Rotation block R(a,b;theta) = (a cos + b sin, -a sin + b cos) of the given
 * block, by n micro-rotations  a' = a + d_i (b >> i),  b' = b - d_i (a >> i)
 * (both from the old a, b), then the gain compensation of both outputs.
 * sense = +1 rotates by +theta; sense = -1 negates every d_i and so rotates by
 * -theta, which is the transpose used by the inverse graph. */
static void cordic_rotate(const recipe_t *R, int64_t *a, int64_t *b, int rot, int sense, int64_t *peak) {
  int64_t x = *a, y = *b;
  for (int i = 0; i < R->n; ++i) {
    const int64_t d = (int64_t)sense * R->dir[rot][i];
    const int64_t xn = x + d * floor_div_pow2(y, i);
    const int64_t yn = y - d * floor_div_pow2(x, i);
    x = xn;
    y = yn;
    track(peak, x);
    track(peak, y);
  }
  *a = compensate(x, R->gain[rot]);
  *b = compensate(y, R->gain[rot]);
  track(peak, *a);
  track(peak, *b);
}

/* One 8-point forward Loeffler flow graph, four stages (Sec. 2.5.2).  Output
 * Z[k] = 2 sqrt(2) times the orthonormal 1-D DCT-II, in the same fixed point
 * as the input.  Stage 1: butterflies.  Stage 2: the even half (a 4-point DCT)
 * gets butterflies, the odd half gets the 3pi/16 and pi/16 rotations.  Stage 3:
 * the even half splits again into the DC/Nyquist butterfly and the sqrt(2)
 * rotation by 6pi/16; the odd half gets butterflies.  Stage 4: the last odd
 * butterfly and the two sqrt(2) factors. */
static void loeffler_forward_int(const recipe_t *R, int64_t *x, int64_t *peak) {
  /* stage 1 */
  const int64_t s0 = x[0] + x[7], s1 = x[1] + x[6], s2 = x[2] + x[5], s3 = x[3] + x[4];
  int64_t d0 = x[0] - x[7], d1 = x[1] - x[6], d2 = x[2] - x[5], d3 = x[3] - x[4];
  track(peak, s0); track(peak, s1); track(peak, s2); track(peak, s3);
  track(peak, d0); track(peak, d1); track(peak, d2); track(peak, d3);
  /* stage 2 */
  const int64_t e0 = s0 + s3, e3 = s0 - s3, e1 = s1 + s2, e2 = s1 - s2;
  track(peak, e0); track(peak, e1); track(peak, e2); track(peak, e3);
  int64_t u4 = d3, u7 = d0, u5 = d2, u6 = d1;
  cordic_rotate(R, &u4, &u7, ROT_3, +1, peak); /* (u4, u7) = R(d3, d0; 3pi/16) */
  cordic_rotate(R, &u5, &u6, ROT_1, +1, peak); /* (u5, u6) = R(d2, d1;  pi/16) */
  /* stage 3 */
  const int64_t Z0 = e0 + e1, Z4 = e0 - e1;
  int64_t Z2 = e2, Z6 = e3;
  cordic_rotate(R, &Z2, &Z6, ROT_6, +1, peak); /* (Z2, Z6) = sqrt2 R(e2, e3; 6pi/16) */
  const int64_t v4 = u4 + u6, v6 = u4 - u6, v7 = u7 + u5, v5 = u7 - u5;
  track(peak, Z0); track(peak, Z4);
  track(peak, v4); track(peak, v5); track(peak, v6); track(peak, v7);
  /* stage 4 */
  const int64_t Z1 = v7 + v4, Z7 = v7 - v4;
  const int64_t Z3 = compensate(v5, R->sqrt2), Z5 = compensate(v6, R->sqrt2);
  track(peak, Z1); track(peak, Z7); track(peak, Z3); track(peak, Z5);
  x[0] = Z0; x[1] = Z1; x[2] = Z2; x[3] = Z3;
  x[4] = Z4; x[5] = Z5; x[6] = Z6; x[7] = Z7;
}

/* The transposed graph: every stage of loeffler_forward_int run backwards with
 * each butterfly transposed and each rotation by -theta.  Output = 2 sqrt(2)
 * times the orthonormal 1-D DCT-III of the input. */
static void loeffler_inverse_int(const recipe_t *R, int64_t *Z, int64_t *peak) {
  /* stage 4 transposed */
  const int64_t v7 = Z[1] + Z[7], v4 = Z[1] - Z[7];
  const int64_t v5 = compensate(Z[3], R->sqrt2), v6 = compensate(Z[5], R->sqrt2);
  track(peak, v7); track(peak, v4); track(peak, v5); track(peak, v6);
  /* stage 3 transposed */
  const int64_t e0 = Z[0] + Z[4], e1 = Z[0] - Z[4];
  int64_t e2 = Z[2], e3 = Z[6];
  cordic_rotate(R, &e2, &e3, ROT_6, -1, peak); /* (e2, e3) = sqrt2 R(Z2, Z6; -6pi/16) */
  int64_t u4 = v4 + v6, u6 = v4 - v6, u7 = v7 + v5, u5 = v7 - v5;
  track(peak, e0); track(peak, e1);
  track(peak, u4); track(peak, u5); track(peak, u6); track(peak, u7);
  /* stage 2 transposed */
  cordic_rotate(R, &u4, &u7, ROT_3, -1, peak); /* (d3, d0) = R(u4, u7; -3pi/16) */
  cordic_rotate(R, &u5, &u6, ROT_1, -1, peak); /* (d2, d1) = R(u5, u6;  -pi/16) */
  const int64_t d0 = u7, d1 = u6, d2 = u5, d3 = u4;
  const int64_t s0 = e0 + e3, s3 = e0 - e3, s1 = e1 + e2, s2 = e1 - e2;
  track(peak, s0); track(peak, s1); track(peak, s2); track(peak, s3);
  /* stage 1 transposed */
  Z[0] = s0 + d0; Z[7] = s0 - d0;
  Z[1] = s1 + d1; Z[6] = s1 - d1;
  Z[2] = s2 + d2; Z[5] = s2 - d2;
  Z[3] = s3 + d3; Z[4] = s3 - d3;
  for (int k = 0; k < 8; ++k) track(peak, Z[k]);
}

/* Forward recipe on one block of already level-shifted, scaled samples
 * x[i*8+j] = (p - 128) << F: row pass, then column pass.  Output c[u*8+v] is
 * 8 times the orthonormal coefficient in the input's fixed point, i.e. the
 * coefficient equals c / 2^(F+3). */
static void recipe_forward_block(const recipe_t *R, const int64_t *x, int64_t *c, int64_t *peak) {
  int64_t t[8];
  int64_t m[64];
  for (int i = 0; i < 8; ++i) { /* rows */
    for (int j = 0; j < 8; ++j) t[j] = x[i * 8 + j];
    loeffler_forward_int(R, t, peak);
    for (int j = 0; j < 8; ++j) m[i * 8 + j] = t[j];
  }
  for (int j = 0; j < 8; ++j) { /* columns */
    for (int i = 0; i < 8; ++i) t[i] = m[i * 8 + j];
    loeffler_forward_int(R, t, peak);
    for (int i = 0; i < 8; ++i) c[i * 8 + j] = t[i];
  }
}

/* Inverse recipe on one block: column pass, then row pass. */
static void recipe_inverse_block(const recipe_t *R, const int64_t *d, int64_t *x, int64_t *peak) {
  int64_t t[8];
  int64_t m[64];
  for (int j = 0; j < 8; ++j) { /* columns */
    for (int i = 0; i < 8; ++i) t[i] = d[i * 8 + j];
    loeffler_inverse_int(R, t, peak);
    for (int i = 0; i < 8; ++i) m[i * 8 + j] = t[i];
  }
  for (int i = 0; i < 8; ++i) { /* rows */
    for (int j = 0; j < 8; ++j) t[j] = m[i * 8 + j];
    loeffler_inverse_int(R, t, peak);
    for (int j = 0; j < 8; ++j) x[i * 8 + j] = t[j];
  }
}

/* quantizer of the recipe: q = sgn(c) * floor((|c| + Q 2^(F+2)) / (Q 2^(F+3))),
 * i.e. c / (Q 2^(F+3)) rounded half away from zero */
static int64_t recipe_quantize(int F, int64_t c, int64_t Q) {
  const int64_t D = Q << (F + 3);
  const int64_t m = (i64_abs(c) + (Q << (F + 2))) / D;
  return c < 0 ? -m : m;
}

/* dequantizer of the recipe: clamp(q Q, -2048, 2047) << G */
static int64_t recipe_dequantize(int G, int64_t q, int64_t Q) {
  int64_t d = q * Q;
  if (d < -2048) d = -2048;
  if (d > 2047) d = 2047;
  return d * ((int64_t)1 << G);
}

/* reconstruction: clamp(floor((x + 2^(G+2)) / 2^(G+3)) + 128, 0, 255) */
static int recipe_reconstruct(int G, int64_t x) {
  int64_t p = floor_div_pow2(x + ((int64_t)1 << (G + 2)), G + 3) + 128;
  if (p < 0) p = 0;
  if (p > 255) p = 255;
  return (int)p;
}

/* ---- image-level entry points of the recipe (mirror the codec's stages) ---- */

static int64_t forward_image(const recipe_t *R, const uint8_t *src, int W, int H, int stride, int32_t *coef) {
  const int bw = (W + 7) / 8, bh = (H + 7) / 8;
  int64_t peak = 0, x[64], c[64];
  for (int by = 0; by < bh; ++by)
    for (int bx = 0; bx < bw; ++bx) {
      for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j)
          x[i * 8 + j] = ((int64_t)pixel_at(src, W, H, stride, by * 8 + i, bx * 8 + j) - 128) *
                         ((int64_t)1 << R->F);
      recipe_forward_block(R, x, c, &peak);
      int32_t *out = coef + ((int64_t)by * bw + bx) * 64;
      for (int k = 0; k < 64; ++k) out[k] = (int32_t)c[k];
    }
  return peak;
}

static void quantize_image(const recipe_t *R, const int32_t *coef, int64_t nblocks, int qs, int16_t *qcoef) {
  for (int64_t b = 0; b < nblocks; ++b)
    for (int u = 0; u < 8; ++u)
      for (int v = 0; v < 8; ++v) {
        const int64_t k = b * 64 + u * 8 + v;
        int64_t q = recipe_quantize(R->F, coef[k], qtable(u, v, qs));
        if (q > 32767) q = 32767;
        if (q < -32768) q = -32768;
        qcoef[k] = (int16_t)q;
      }
}

static int64_t inverse_image(const recipe_t *R, const int16_t *qcoef, int qs, int W, int H, uint8_t *dst,
                             int dst_stride) {
  const int bw = (W + 7) / 8, bh = (H + 7) / 8;
  int64_t peak = 0, d[64], x[64];
  for (int by = 0; by < bh; ++by)
    for (int bx = 0; bx < bw; ++bx) {
      const int16_t *q = qcoef + ((int64_t)by * bw + bx) * 64;
      for (int u = 0; u < 8; ++u)
        for (int v = 0; v < 8; ++v) d[u * 8 + v] = recipe_dequantize(R->G, q[u * 8 + v], qtable(u, v, qs));
      recipe_inverse_block(R, d, x, &peak);
      for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
          const int y = by * 8 + i, xx = bx * 8 + j;
          if (y < H && xx < W) dst[(int64_t)y * dst_stride + xx] = (uint8_t)recipe_reconstruct(R->G, x[i * 8 + j]);
        }
    }
  return peak;
}

static uint64_t codec_image(const recipe_t *R, const uint8_t *src, int W, int H, int stride, int qs, uint8_t *dst,
                            int dst_stride, int16_t *qcoef) {
  const int64_t nblocks = (int64_t)((W + 7) / 8) * ((H + 7) / 8);
  int32_t *coef = (int32_t *)malloc((size_t)nblocks * 64 * sizeof(int32_t));
  int16_t *q = qcoef ? qcoef : (int16_t *)malloc((size_t)nblocks * 64 * sizeof(int16_t));
  if (!coef || !q) {
    free(coef);
    if (!qcoef) free(q);
    return UINT64_MAX;
  }
  forward_image(R, src, W, H, stride, coef);
  quantize_image(R, coef, nblocks, qs, q);
  inverse_image(R, q, qs, W, H, dst, dst_stride);
  free(coef);
  if (!qcoef) free(q);
  return or_sse(src, stride, dst, dst_stride, W, H);
}

/* a1..a4: uint8 plane -> int32 coefficients [ceil(H/8)*ceil(W/8)][64].
 * Returns the largest |value| the recipe stored (for overflow tests). */
int64_t or_cordic_forward(const uint8_t *src, int W, int H, int stride, int32_t *coef) {
  return forward_image(default_recipe(), src, W, H, stride, coef);
}

/* a5: int32 coefficients -> int16 quantized values, same layout.  The int16
 * container saturates; coefficients of a uint8 plane give |q| <= 1024 and never
 * reach the limits, only arbitrary int32 input can. */
void or_cordic_quantize(const int32_t *coef, int64_t nblocks, int qs, int16_t *qcoef) {
  quantize_image(default_recipe(), coef, nblocks, qs, qcoef);
}

/* a6..a8: int16 quantized values -> uint8 plane (only the W x H region is
 * written).  Returns the largest |value| the recipe stored. */
int64_t or_cordic_inverse(const int16_t *qcoef, int qs, int W, int H, uint8_t *dst, int dst_stride) {
  return inverse_image(default_recipe(), qcoef, qs, W, H, dst, dst_stride);
}

/* a1..a9 in one call: forward, quantize, dequantize, inverse, reconstruct and
 * SSE against the source.  qcoef may be NULL.  Returns the SSE. */
uint64_t or_cordic_codec(const uint8_t *src, int W, int H, int stride, int qs, uint8_t *dst,
                         int dst_stride, int16_t *qcoef) {
  return codec_image(default_recipe(), src, W, H, stride, qs, dst, dst_stride, qcoef);
}

/* The same stages under recipe R(n, F, G) (UINT64_MAX / -1 for an invalid recipe).
 * The *peak outputs of the forward and inverse report the largest |value| stored. */
uint64_t or_recipe_codec(int n, int F, int G, const uint8_t *src, int W, int H, int stride, int qs, uint8_t *dst,
                         int dst_stride, int16_t *qcoef) {
  if (!or_recipe_valid(n, F, G)) return UINT64_MAX;
  recipe_t R;
  recipe_make(&R, n, F, G);
  return codec_image(&R, src, W, H, stride, qs, dst, dst_stride, qcoef);
}

int64_t or_recipe_forward_block(int n, int F, int G, const int64_t *x, int64_t *c) {
  if (!or_recipe_valid(n, F, G)) return -1;
  recipe_t R;
  recipe_make(&R, n, F, G);
  int64_t peak = 0;
  recipe_forward_block(&R, x, c, &peak);
  return peak;
}

int64_t or_recipe_inverse_block(int n, int F, int G, const int64_t *d, int64_t *x) {
  if (!or_recipe_valid(n, F, G)) return -1;
  recipe_t R;
  recipe_make(&R, n, F, G);
  int64_t peak = 0;
  recipe_inverse_block(&R, d, x, &peak);
  return peak;
}

/* forward and inverse peaks of recipe R(n, F, G) on a whole image at quality
 * scale qs (for the int32 headroom tests of each recipe); -1 if invalid */
int or_recipe_peaks(int n, int F, int G, const uint8_t *src, int W, int H, int stride, int qs, int64_t *fwd_peak,
                    int64_t *inv_peak) {
  if (!or_recipe_valid(n, F, G)) return -1;
  recipe_t R;
  recipe_make(&R, n, F, G);
  const int64_t nblocks = (int64_t)((W + 7) / 8) * ((H + 7) / 8);
  int32_t *coef = (int32_t *)malloc((size_t)nblocks * 64 * sizeof(int32_t));
  int16_t *q = (int16_t *)malloc((size_t)nblocks * 64 * sizeof(int16_t));
  uint8_t *dst = (uint8_t *)malloc((size_t)W * H);
  if (!coef || !q || !dst) {
    free(coef);
    free(q);
    free(dst);
    return -1;
  }
  *fwd_peak = forward_image(&R, src, W, H, stride, coef);
  quantize_image(&R, coef, nblocks, qs, q);
  *inv_peak = inverse_image(&R, q, qs, W, H, dst, W);
  free(coef);
  free(q);
  free(dst);
  return 0;
}

/* Block-level access for tests: forward / inverse recipe on one block of raw
 * fixed-point samples (no level shift, no quantizer).  Return the peak |value|. */
int64_t or_cordic_forward_block(const int64_t *x, int64_t *c) {
  int64_t peak = 0;
  recipe_forward_block(default_recipe(), x, c, &peak);
  return peak;
}

int64_t or_cordic_inverse_block(const int64_t *d, int64_t *x) {
  int64_t peak = 0;
  recipe_inverse_block(default_recipe(), d, x, &peak);
  return peak;
}

/* One CORDIC rotation block alone (for tests of the rotation itself). */
void or_cordic_rotate_pair(int64_t *a, int64_t *b, int rot, int sense) {
  cordic_rotate(default_recipe(), a, b, rot, sense, NULL);
}

/* The recipe's scalar quantizer and dequantizer (for exhaustive tests). */
int64_t or_recipe_quantize(int64_t c, int64_t Q) { return recipe_quantize(OR_FRAC, c, Q); }
int64_t or_recipe_dequantize(int64_t q, int64_t Q) { return recipe_dequantize(OR_FRAC, q, Q); }
int or_recipe_reconstruct(int64_t x) { return recipe_reconstruct(OR_FRAC, x); }

/* ------------------------------------------------------------------------- */
/* Colour conversion for three-channel inputs (not in the paper, which works  */
/* on grayscale images; the precision workload codes the Y, Cb and Cr planes  */
/* of RGB images)                                                             */
/* ------------------------------------------------------------------------- */

/* Integer full-range YCbCr (the JPEG File Interchange Format definition with
 * the BT.601 luma weights 0.299, 0.587, 0.114), each weight rounded to
 * round(w 2^16) so that the luma weights sum to 2^16 and the chroma weights to 0:
 *   Y  = (19595 R + 38470 G +  7471 B + 2^15) >> 16
 *   Cb = ((-11058 R - 21710 G + 32768 B + 2^15) >> 16) + 128
 *   Cr = (( 32768 R - 27439 G -  5329 B + 2^15) >> 16) + 128
 * (floor shifts), each clamped to [0, 255].  rgb is interleaved R, G, B bytes
 * with row pitch rgb_stride; the three output planes share plane_stride. */
static int clamp255(int64_t v) { return v < 0 ? 0 : (v > 255 ? 255 : (int)v); }

void or_rgb_to_ycbcr(const uint8_t *rgb, int W, int H, int rgb_stride, uint8_t *y, uint8_t *cb,
                     uint8_t *cr, int plane_stride) {
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j) {
      const uint8_t *p = rgb + (int64_t)i * rgb_stride + 3 * (int64_t)j;
      const int64_t R = p[0], G = p[1], B = p[2];
      const int64_t half = (int64_t)1 << 15;
      const int64_t yy = floor_div_pow2(19595 * R + 38470 * G + 7471 * B + half, 16);
      const int64_t bb = floor_div_pow2(-11058 * R - 21710 * G + 32768 * B + half, 16) + 128;
      const int64_t rr = floor_div_pow2(32768 * R - 27439 * G - 5329 * B + half, 16) + 128;
      const int64_t o = (int64_t)i * plane_stride + j;
      y[o] = (uint8_t)clamp255(yy);
      cb[o] = (uint8_t)clamp255(bb);
      cr[o] = (uint8_t)clamp255(rr);
    }
}

/* ------------------------------------------------------------------------- */
/* The same Loeffler graph in FP64 with exact rotations (structure pin)       */
/* ------------------------------------------------------------------------- */

static void rot_f64(double *a, double *b, double theta, double scale) {
  const double x = *a, y = *b;
  *a = scale * (x * cos(theta) + y * sin(theta));
  *b = scale * (-x * sin(theta) + y * cos(theta));
}

/* Z = 2 sqrt(2) C x with C the orthonormal 8-point DCT-II matrix */
void or_loeffler_forward_f64(const double *x, double *Z) {
  const double pi = or_pi(), r2 = sqrt(2.0);
  const double s0 = x[0] + x[7], s1 = x[1] + x[6], s2 = x[2] + x[5], s3 = x[3] + x[4];
  const double d0 = x[0] - x[7], d1 = x[1] - x[6], d2 = x[2] - x[5], d3 = x[3] - x[4];
  const double e0 = s0 + s3, e3 = s0 - s3, e1 = s1 + s2, e2 = s1 - s2;
  double u4 = d3, u7 = d0, u5 = d2, u6 = d1;
  rot_f64(&u4, &u7, 3 * pi / 16, 1.0);
  rot_f64(&u5, &u6, pi / 16, 1.0);
  double Z2 = e2, Z6 = e3;
  rot_f64(&Z2, &Z6, 6 * pi / 16, r2);
  const double v4 = u4 + u6, v6 = u4 - u6, v7 = u7 + u5, v5 = u7 - u5;
  Z[0] = e0 + e1; Z[4] = e0 - e1; Z[2] = Z2; Z[6] = Z6;
  Z[1] = v7 + v4; Z[7] = v7 - v4; Z[3] = r2 * v5; Z[5] = r2 * v6;
}

/* x = (2 sqrt(2) C)^T Z */
void or_loeffler_inverse_f64(const double *Z, double *x) {
  const double pi = or_pi(), r2 = sqrt(2.0);
  const double v7 = Z[1] + Z[7], v4 = Z[1] - Z[7], v5 = r2 * Z[3], v6 = r2 * Z[5];
  const double e0 = Z[0] + Z[4], e1 = Z[0] - Z[4];
  double e2 = Z[2], e3 = Z[6];
  rot_f64(&e2, &e3, -6 * pi / 16, r2);
  double u4 = v4 + v6, u6 = v4 - v6, u7 = v7 + v5, u5 = v7 - v5;
  rot_f64(&u4, &u7, -3 * pi / 16, 1.0);
  rot_f64(&u5, &u6, -pi / 16, 1.0);
  const double d0 = u7, d1 = u6, d2 = u5, d3 = u4;
  const double s0 = e0 + e3, s3 = e0 - e3, s1 = e1 + e2, s2 = e1 - e2;
  x[0] = s0 + d0; x[7] = s0 - d0;
  x[1] = s1 + d1; x[6] = s1 - d1;
  x[2] = s2 + d2; x[5] = s2 - d2;
  x[3] = s3 + d3; x[4] = s3 - d3;
}
