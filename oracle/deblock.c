/*
 * deblock.c -- CPU reference for the learned deblocking network applied to
 * decoded images.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; it shares nothing with the
 * HIP library.
 *
 * The paper reports blocking artefacts in the decoded images of its CORDIC
 * codec (Sec. 4, the PSNR tables 3-4 and the reconstructed images) but does not
 * remove them; this is the post-filter that reduces them.  The network, its loss
 * and its optimiser are fixed here (the paper has none):
 *
 *   x = p / 255 for the decoded pixels p of one image (or crop);
 *   a1 = relu(conv(x; W1, b1))       1 -> 32 channels
 *   a2 = relu(conv(a1; W2, b2))      32 -> 32
 *   a3 = relu(conv(a2; W3, b3))      32 -> 32
 *   y  = x + conv(a3; W4, b4)        32 -> 1, residual
 * with conv a 3x3 cross-correlation with zero padding outside the image:
 *   conv(a; W, b)[o][r][c] = b[o] + sum_i sum_{dy,dx in 0..2} W[o][i][dy][dx] a[i][r+dy-1][c+dx-1].
 * The loss of a batch of B images is the mean of (y - t)^2 over all B H W
 * pixels, t = original / 255.  Gradients are the exact derivatives of that loss
 * (ReLU'(0) = 0); the optimiser is Adam with bias correction.
 *
 * Parameters are one flat array of 19105 values in the order W1 [32][1][3][3],
 * b1 [32], W2 [32][32][3][3], b2 [32], W3 [32][32][3][3], b3 [32],
 * W4 [1][32][3][3], b4 [1].  Everything is FP64.
 *
 * Parity status: pinned by SciPy's correlate2d, closed forms (identity and
 * shift kernels, the zero network, Adam's first step) and central finite
 * differences of the loss in the tests.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define DB_C 32
#define DB_NPARAM (32 * 9 + 32 + 2 * (32 * 32 * 9 + 32) + 32 * 9 + 1)

int or_db_nparam(void) { return DB_NPARAM; }

/* offsets of the layers in the flat parameter array */
static void layer_offsets(long *w, long *b) {
  const long sizes_w[4] = {32 * 9, 32 * 32 * 9, 32 * 32 * 9, 32 * 9};
  const long sizes_b[4] = {32, 32, 32, 1};
  long o = 0;
  for (int l = 0; l < 4; ++l) {
    w[l] = o;
    o += sizes_w[l];
    b[l] = o;
    o += sizes_b[l];
  }
}

static const int CIN[4] = {1, DB_C, DB_C, DB_C};
static const int COUT[4] = {DB_C, DB_C, DB_C, 1};

/* y[co][r][c] = b[co] + sum W[co][ci][dy][dx] x[ci][r+dy-1][c+dx-1], zero outside */
void or_conv3x3(const double *x, int ci_n, int H, int W, const double *w, const double *b, int co_n, double *y) {
  for (int co = 0; co < co_n; ++co)
    for (int r = 0; r < H; ++r)
      for (int c = 0; c < W; ++c) {
        double s = b ? b[co] : 0.0;
        for (int ci = 0; ci < ci_n; ++ci)
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              const int rr = r + dy - 1, cc = c + dx - 1;
              if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
              s += w[((long)co * ci_n + ci) * 9 + dy * 3 + dx] * x[((long)ci * H + rr) * W + cc];
            }
        y[((long)co * H + r) * W + c] = s;
      }
}

/* Gradients of a conv layer given dL/dy: gx (may be NULL) = dL/dx, and gw, gb
 * are ADDED to (so a batch accumulates). */
void or_conv3x3_bwd(const double *x, int ci_n, int H, int W, const double *w, int co_n, const double *gy, double *gx,
                    double *gw, double *gb) {
  if (gx) memset(gx, 0, sizeof(double) * (size_t)ci_n * H * W);
  for (int co = 0; co < co_n; ++co)
    for (int r = 0; r < H; ++r)
      for (int c = 0; c < W; ++c) {
        const double g = gy[((long)co * H + r) * W + c];
        if (gb) gb[co] += g;
        for (int ci = 0; ci < ci_n; ++ci)
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              const int rr = r + dy - 1, cc = c + dx - 1;
              if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
              const long wi = ((long)co * ci_n + ci) * 9 + dy * 3 + dx, xi = ((long)ci * H + rr) * W + cc;
              if (gw) gw[wi] += g * x[xi];
              if (gx) gx[xi] += g * w[wi];
            }
      }
}

/* Forward pass of one image; acts (may be NULL) receives a1, a2, a3 (each
 * 32 H W, in that order). */
void or_db_forward(const double *params, const double *x, int H, int W, double *y, double *acts) {
  long wo[4], bo[4];
  layer_offsets(wo, bo);
  const long n = (long)H * W;
  double *a = malloc(sizeof(double) * 3 * DB_C * n);
  const double *in = x;
  for (int l = 0; l < 3; ++l) {
    double *out = a + (long)l * DB_C * n;
    or_conv3x3(in, CIN[l], H, W, params + wo[l], params + bo[l], COUT[l], out);
    for (long k = 0; k < DB_C * n; ++k) out[k] = out[k] > 0.0 ? out[k] : 0.0;
    in = out;
  }
  or_conv3x3(in, DB_C, H, W, params + wo[3], params + bo[3], 1, y);
  for (long k = 0; k < n; ++k) y[k] += x[k];
  if (acts) memcpy(acts, a, sizeof(double) * 3 * DB_C * n);
  free(a);
}

/* Loss of a batch of B images (x, t: B H W) and its gradient with respect to the
 * parameters (grad: DB_NPARAM, overwritten).  Returns the mean squared error. */
double or_db_loss_grad(const double *params, const double *x, const double *t, int B, int H, int W, double *grad) {
  long wo[4], bo[4];
  layer_offsets(wo, bo);
  const long n = (long)H * W;
  const double scale = 2.0 / ((double)B * n);
  double *acts = malloc(sizeof(double) * 3 * DB_C * n);
  double *y = malloc(sizeof(double) * n);
  double *g = malloc(sizeof(double) * DB_C * n);
  double *g2 = malloc(sizeof(double) * DB_C * n);
  if (grad) memset(grad, 0, sizeof(double) * DB_NPARAM);
  double loss = 0.0;
  for (int bi = 0; bi < B; ++bi) {
    const double *xb = x + (long)bi * n, *tb = t + (long)bi * n;
    or_db_forward(params, xb, H, W, y, acts);
    for (long k = 0; k < n; ++k) {
      const double e = y[k] - tb[k];
      loss += e * e;
      g[k] = scale * e; /* dL/dy */
    }
    if (!grad) continue;
    /* layer 4: input a3 */
    const double *a3 = acts + 2L * DB_C * n, *a2 = acts + 1L * DB_C * n, *a1 = acts;
    or_conv3x3_bwd(a3, DB_C, H, W, params + wo[3], 1, g, g2, grad + wo[3], grad + bo[3]);
    for (long k = 0; k < DB_C * n; ++k) g2[k] = a3[k] > 0.0 ? g2[k] : 0.0;
    or_conv3x3_bwd(a2, DB_C, H, W, params + wo[2], DB_C, g2, g, grad + wo[2], grad + bo[2]);
    for (long k = 0; k < DB_C * n; ++k) g[k] = a2[k] > 0.0 ? g[k] : 0.0;
    or_conv3x3_bwd(a1, DB_C, H, W, params + wo[1], DB_C, g, g2, grad + wo[1], grad + bo[1]);
    for (long k = 0; k < DB_C * n; ++k) g2[k] = a1[k] > 0.0 ? g2[k] : 0.0;
    or_conv3x3_bwd(xb, 1, H, W, params + wo[0], DB_C, g2, NULL, grad + wo[0], grad + bo[0]);
  }
  free(acts);
  free(y);
  free(g);
  free(g2);
  return loss / ((double)B * n);
}

/* One Adam step (Kingma and Ba), step counted from 1:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
void or_adam_step(double *p, double *m, double *v, const double *g, long n, double lr, double b1, double b2,
                  double eps, int step) {
  const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (long k = 0; k < n; ++k) {
    m[k] = b1 * m[k] + (1.0 - b1) * g[k];
    v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    p[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
  }
}
