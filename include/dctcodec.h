/*
 * dctcodec.h -- C ABI of the blockwise 8x8 Cordic-based Loeffler DCT image codec
 * for AMD Instinct MI355X (gfx950).
 *
 * The codec follows Modieginyane, Ncube and Gasela, "CUDA based performance
 * evaluation of the computational efficiency of the DCT image compression
 * technique on both the CPU and GPU":
 *   - the transform is the 2-D DCT-II of Sec. 2.5.1, eq. (6)-(7) (orthonormal
 *     scaling), on 8x8 blocks, computed as row then column 8-point Loeffler
 *     flow graphs (Sec. 2.5.2) whose rotation blocks are fixed-point CORDIC
 *     shift-add rotations;
 *   - the DCT, the quantizer and the IDCT are separate stages (Sec. 3.2);
 *   - reconstruction quality is PSNR, eq. (23)-(24) (Sec. 4.1).
 *
 * Integer recipe R(n, F, P) = R(10, 12, 15), identical bit for bit on every
 * entry point:
 *   samples      x = (p - 128) << F                      (level shift)
 *   rotation     n micro-rotations a' = a + d_i (b >> i), b' = b - d_i (a >> i)
 *                (simultaneous, arithmetic shifts), then a <- (a M + 2^(P-1)) >> P
 *                per output; d_i from the greedy CORDIC rule, M = round(k 2^P / K_n)
 *   forward      row pass then column pass; coefficient = c / 2^(F+3)  (Q16.15)
 *   quantize     Q[u][v] = 1 + (1 + u + v) qs;
 *                q = sgn(c) floor((|c| + Q 2^(F+2)) / (Q 2^(F+3))), saturated to int16
 *   dequantize   clamp(q Q, -2048, 2047) << F
 *   inverse      transposed graph (rotations by -theta), column pass then row pass
 *   reconstruct  clamp(((x + 2^(F+2)) >> (F+3)) + 128, 0, 255)
 * dct_recipe_info / dct_recipe_tables report the parameters and constants.
 *
 * Conventions shared by every entry point:
 *   - Planes are uint8 grayscale, row-major, W x H pixels, rows `stride` bytes
 *     apart.  stride >= W, stride % 8 == 0 and (H - 1) * stride + W < 2^32 (the
 *     kernels address a plane with 32-bit offsets); the plane pointer is 8-byte
 *     aligned.  A source plane must hold (H - 1) * stride + W readable bytes; the
 *     library reads no byte outside the W x H region.  A destination plane gets
 *     exactly its W x H region written; pad bytes are left untouched.
 *   - The block grid is ceil(W/8) x ceil(H/8).  Pixels of edge blocks that lie
 *     outside the image repeat the nearest pixel of the last column / row.
 *   - Coefficient arrays are [nblocks][64]: blocks in row-major block order
 *     (by * ceil(W/8) + bx), each block in natural (not zig-zag) order u * 8 + v
 *     with u the vertical and v the horizontal frequency.  They are 16-byte
 *     aligned.
 *   - Pointers are device pointers unless marked "host".  The caller allocates
 *     and owns every buffer; the library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *     enqueue their kernels on it and return without waiting unless stated.
 *   - Sizes: 1 <= W <= 65535, 1 <= H <= 2^24 (within the 2^32 rule above);
 *     1 <= qs <= 1024.  Blocks never span two images stacked vertically in one
 *     plane when each image's height is a multiple of 8, so such a stack codes
 *     exactly like its images one by one.
 *   - Every call returns a dct_status.  Arguments are checked before anything is
 *     enqueued (DCT_ERR_INVALID); a failed launch gives DCT_ERR_DEVICE.  The
 *     library never aborts and never throws across this interface.
 *   - Thread safety: calls on different streams may run concurrently, except
 *     dct_psnr, which serialises on a library lock (it uses a per-device scratch
 *     word on the device and a pinned host copy of it, and waits for its stream).
 */
#ifndef DCTCODEC_H
#define DCTCODEC_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define DCT_API __attribute__((visibility("default")))
#else
#define DCT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DCT_OK = 0,
  DCT_ERR_INVALID = -1,     /* an argument violates the preconditions above */
  DCT_ERR_UNSUPPORTED = -2, /* no gfx950 device is current, or the recipe is not built */
  DCT_ERR_DEVICE = -3,      /* the HIP runtime reported an error */
  DCT_ERR_NOMEM = -4        /* the library could not allocate its scratch word */
} dct_status;

/* Forward transform, steps a1-a4 (level shift, row pass, transpose, column pass):
 * the Loeffler flow graph of Sec. 2.5.2 with CORDIC rotation blocks, applied to
 * every 8x8 block (2-D DCT-II of Sec. 2.5.1, eq. (6)).
 *   src   W x H uint8 plane, row pitch src_stride.
 *   coef  out: int32 [ceil(H/8) * ceil(W/8)][64]; coefficient = value / 2^15. */
DCT_API int dct_forward(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t *coef,
                void *stream);

/* Table quantizer, step a5 (the quantizer stage of Sec. 3.2).
 *   coef     int32 [nblocks][64] as written by dct_forward (any int32 accepted).
 *   nblocks  number of blocks, >= 0 (0 enqueues nothing).
 *   qs       quality scale of the table Q[u][v] = 1 + (1 + u + v) qs.
 *   qcoef    out: int16 [nblocks][64], nearest integer to coefficient / Q with
 *            ties away from zero, saturated to [-32768, 32767]. */
DCT_API int dct_quantize(const int32_t *coef, int64_t nblocks, int32_t qs, int16_t *qcoef, void *stream);

/* Dequantize and inverse transform, steps a6-a8 (the IDCT stage of Sec. 3.2; the
 * inverse of eq. (6) named in Sec. 2.5.1).  Any int16 input is accepted: the
 * dequantized value is clamped to [-2048, 2047] before the inverse.
 *   qcoef  int16 [ceil(H/8) * ceil(W/8)][64].
 *   qs     the quality scale the values were quantized with.
 *   dst    out: W x H uint8 plane, row pitch dst_stride. */
DCT_API int dct_inverse(const int16_t *qcoef, int32_t qs, int32_t W, int32_t H, uint8_t *dst,
                int32_t dst_stride, void *stream);

/* PSNR of plane b against plane a, step a9 (Sec. 4.1, eq. (23)-(24)).
 *   peak       MAX of eq. (23): > 0 uses that value; 0 uses the largest pixel of a.
 *   psnr_host  host out: 20 log10(MAX / sqrt(SSE / (W H))); +inf when SSE = 0.
 *   sse_host   host out, may be NULL: the exact sum of squared differences.
 * Waits for `stream` before returning. */
DCT_API int dct_psnr(const uint8_t *a, int32_t a_stride, const uint8_t *b, int32_t b_stride, int32_t W,
             int32_t H, double peak, double *psnr_host, uint64_t *sse_host, void *stream);

/* PSNR of eq. (23)-(24) (Sec. 4.1) from an exact sum of squared differences, as
 * dct_psnr computes it: 20 log10(peak / sqrt(sse / npix)), +inf when sse = 0.
 * For the SSE that dct_codec and the other fused entry points leave in device
 * memory, once the caller has it on the host.
 *   sse        the sum of squared differences over npix pixels.
 *   npix       number of pixels, >= 1 (W H of the image).
 *   peak       MAX of eq. (23), > 0 (255 for 8-bit planes).
 *   psnr_host  host out.
 * Host arithmetic only: enqueues nothing, touches no device. */
DCT_API int dct_psnr_from_sse(uint64_t sse, int64_t npix, double peak, double *psnr_host);

/* dct_psnr's SSE pass for callers that cannot allocate: code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc.  It enqueues the
 * same SSE kernels as dct_psnr (step a9, the sum of eq. (23)) but calls no
 * allocating routine, does not wait, and leaves its result in device memory:
 *   result_dev  out: two uint64 in device memory (8-byte aligned), overwritten
 *               with {SSE of b against a over W x H, largest pixel of a}; the
 *               PSNR then follows from dct_psnr_from_sse with npix = W H and
 *               peak 255 (or the largest pixel, dct_psnr's peak = 0 reading).
 * Its partial sums live in a fixed 16 KiB scratch array inside the library, one
 * per device, resolved on the first call on each device and held until the
 * process ends.  The grid never needs more than that array, so every plane
 * the conventions above accept fits (the call still returns DCT_ERR_INVALID if
 * a launch would need more).  Every workgroup overwrites its own partials, so
 * nothing is cleared between calls.  Calls that overlap on one device (on
 * different streams, or from different threads without ordering) share that
 * array and race: serialise them. */
DCT_API int dct_psnr_noalloc(const uint8_t *a, int32_t a_stride, const uint8_t *b, int32_t b_stride, int32_t W,
                             int32_t H, uint64_t *result_dev, void *stream);

/* The whole codec in one pass, steps a1-a9: forward, quantize, dequantize,
 * inverse, reconstruct, and the SSE of the reconstruction against the source.
 * Bit-identical to dct_forward + dct_quantize + dct_inverse + dct_psnr.
 *   dst            out: W x H uint8 reconstruction, row pitch dst_stride.
 *   qcoef_or_null  out, optional: the int16 quantized values, as dct_quantize.
 *   sse_dev        out: one uint64 in device memory, overwritten with the SSE
 *                  (PSNR = 10 log10(255^2 W H / SSE)). */
DCT_API int dct_codec(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t qs, uint8_t *dst,
              int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream);

/* dct_codec that adds the block SSEs to *sse_dev instead of overwriting it: one
 * kernel launch and nothing else.  The caller zeroes *sse_dev once; calls on
 * the bands or tiles of one image (each a plane of its own, block-aligned), on
 * the frames of a sequence, or on the images of a set then leave the SSE of the
 * whole in it, whose PSNR (eq. (23), Sec. 4.1) is over all their pixels
 * (dct_psnr_from_sse with npix their total).  Calls that add into one word
 * may overlap: the additions are atomic.  Arguments and every other output as
 * dct_codec. */
DCT_API int dct_codec_accumulate(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t qs,
                                 uint8_t *dst, int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev,
                                 void *stream);

/* dct_codec with the other thread mapping: one lane per 8x8 block, the block's
 * 64 samples kept in that lane's registers through both passes, the
 * row-to-column transpose a change of register index.  dct_codec and
 * dct_codec_accumulate give each lane one block row and stage the transposes
 * through LDS (the shared-memory design of Sec. 2.4); the recipe family and the
 * batch use this mapping.  Bit-identical to dct_codec (arguments and outputs as
 * dct_codec); kept so that the two mappings can be measured against each other. */
DCT_API int dct_codec_blocks(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t qs,
                             uint8_t *dst, int32_t dst_stride, int16_t *qcoef_or_null, uint64_t *sse_dev,
                             void *stream);

/* Floating-point forms of the transform (the exact DCT of Sec. 2.5.1, eq. (6),
 * that Sec. 4.1 compares the Cordic-based codec against), for dct_forward_float
 * and dct_codec_float:
 *   DCT_FORM_F32_LOEFFLER  the four-stage Loeffler graph in FP32, exact rotations;
 *   DCT_FORM_MFMA_F16      vec(F) = (C (x) C) vec(p - 128) as a GEMM over blocks on
 *                          the matrix cores, FP16 inputs (C (x) C rounded once to
 *                          FP16), FP32 accumulation;
 *   DCT_FORM_MFMA_BF16     the same with BF16 inputs. */
typedef enum { DCT_FORM_F32_LOEFFLER = 1, DCT_FORM_MFMA_F16 = 2, DCT_FORM_MFMA_BF16 = 3 } dct_form;

/* Orthonormal 2-D DCT-II coefficients of every 8x8 block in a floating-point form.
 *   src   W x H uint8 plane (level shift p - 128 applied).
 *   form  a dct_form value.
 *   coef  out: float [ceil(H/8) * ceil(W/8)][64], layout as dct_forward, 16-byte aligned. */
DCT_API int dct_forward_float(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t form,
                              float *coef, void *stream);

/* The codec with a floating-point transform: forward in `form`, quantize
 * q = sgn(F) floor(|F| / Q + 1/2) with the table of dct_quantize, dequantize q Q,
 * inverse in `form`, reconstruct clamp(floor(x + 128 + 1/2), 0, 255), and the SSE
 * against the source into *sse_dev (one uint64 in device memory, overwritten).
 * Results are within the form's stated tolerance of the FP64 codec, not bit-exact. */
DCT_API int dct_codec_float(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t form, int32_t qs,
                            uint8_t *dst, int32_t dst_stride, uint64_t *sse_dev, void *stream);

/* Integer full-range YCbCr planes of an interleaved RGB image (JFIF / BT.601 luma
 * weights rounded to 2^-16: Y = (19595 R + 38470 G + 7471 B + 2^15) >> 16,
 * Cb = ((-11058 R - 21710 G + 32768 B + 2^15) >> 16) + 128,
 * Cr = ((32768 R - 27439 G - 5329 B + 2^15) >> 16) + 128, clamped to [0, 255]),
 * so that three-channel images can be coded plane by plane.
 *   rgb           W x H pixels of 3 bytes, row pitch rgb_stride >= 3 W.
 *   y, cb, cr     out: W x H planes with row pitch plane_stride. */
DCT_API int dct_rgb_to_ycbcr(const uint8_t *rgb, int32_t W, int32_t H, int32_t rgb_stride, uint8_t *y, uint8_t *cb,
                             uint8_t *cr, int32_t plane_stride, void *stream);

/* The fused codec of dct_codec under another recipe R(n, F, G) of the family
 * the paper's Sec. 2.5.2 leaves open (its flow-graph figure, with the CORDIC
 * iteration count and word length, is missing): n micro-rotations per rotation
 * block, F fractional bits in the forward transform (x = (p - 128) << F,
 * coefficient = c / 2^(F+3), q = sgn(c) floor((|c| + Q 2^(F+2)) / (Q 2^(F+3)))),
 * G in the inverse (dequantize clamp(q Q, -2048, 2047) << G, reconstruct
 * clamp(((x + 2^(G+2)) >> (G+3)) + 128, 0, 255)); P = 15.  R(10, 12, 12) is
 * dct_codec itself.  The library is built with n in {4, 6, 8, 10, 12} and
 * (F, G) in {(8, 8), (12, 12), (16, 12)}; other recipes give DCT_ERR_UNSUPPORTED.
 * Arguments and outputs as dct_codec. */
DCT_API int dct_codec_recipe(const uint8_t *src, int32_t W, int32_t H, int32_t src_stride, int32_t n_iter,
                             int32_t frac_bits, int32_t inv_frac_bits, int32_t qs, uint8_t *dst, int32_t dst_stride,
                             int16_t *qcoef_or_null, uint64_t *sse_dev, void *stream);

/* 1 if dct_codec_recipe accepts R(n_iter, frac_bits, inv_frac_bits), else 0. */
DCT_API int dct_recipe_supported(int32_t n_iter, int32_t frac_bits, int32_t inv_frac_bits);

/* The built recipes: returns their count; when `recipes` (host) is not NULL,
 * also writes up to `capacity` triples (n, F, G), the default first. */
DCT_API int dct_recipe_list(int32_t *recipes, int32_t capacity);

/* Constants of the built recipes with n_iter micro-rotations (host outs), as
 * dct_recipe_tables; DCT_ERR_UNSUPPORTED if no built recipe has that n. */
DCT_API int dct_recipe_tables_n(int32_t n_iter, int32_t *directions, int32_t *gains);

/* One image of a batch (host struct): planes and quality scale as for dct_codec. */
typedef struct {
  const uint8_t *src; /* W x H source plane, row pitch src_stride */
  uint8_t *dst;       /* W x H reconstruction, row pitch dst_stride */
  int32_t W, H, src_stride, dst_stride;
  int32_t qs;         /* quality scale of this image, 1..1024 */
  int32_t reserved;   /* set to 0 */
} dct_image;

/* The fused codec of dct_codec over a batch of images of any sizes and quality
 * scales in one kernel launch (the paper codes one image per run, Sec. 3.2 and
 * Sec. 4; this is the same per-image computation, bit for bit, for many images).
 * Planning and running are separate so that the run can be captured in a HIP
 * graph and replayed:
 *
 * dct_batch_workspace_size: bytes of device workspace the batch needs with
 *   `chunk` blocks per work item, the tile a workgroup codes at a time (256,
 *   512, 1024 or 2048); 0 if any image or argument is invalid.
 * dct_batch_plan: validates the images (host array of n_images), writes the
 *   batch description into `workspace` (device memory, 256-byte aligned, at
 *   least the size above, owned by the caller), waits for `stream`, and
 *   remembers the plan under the workspace address; *total_chunks (host, may be
 *   NULL) gets the number of workgroup chunks.  Planning a workspace again
 *   replaces its plan.  Not capturable (it copies from host memory and waits).
 * dct_batch_run: codes every image of the plan in `workspace`: writes each dst
 *   plane and overwrites sse_dev[k] (device, n_images uint64) with image k's
 *   SSE.  grid = 0 launches one workgroup per chunk; grid > 0 launches that many
 *   workgroups, each walking the chunks with a fixed stride.  Enqueues two
 *   kernels and nothing else, so it can be captured in a graph.  The images'
 *   planes must stay valid and unchanged in place between plan and run.
 *   Each workgroup has min(chunk, 512) lanes, one block per lane.
 *   DCT_ERR_INVALID if the workspace holds no plan.
 * dct_batch_run_threads: dct_batch_run with `threads` lanes per workgroup (256
 *   or 512, at most the plan's chunk), which codes a chunk in chunk / threads
 *   passes.  DCT_ERR_INVALID for another thread count.
 * dct_batch_release: forgets the plan of a workspace (the caller frees it). */
DCT_API size_t dct_batch_workspace_size(const dct_image *images, int32_t n_images, int32_t chunk);
DCT_API int dct_batch_plan(const dct_image *images, int32_t n_images, int32_t chunk, void *workspace,
                           size_t workspace_bytes, int64_t *total_chunks, void *stream);
DCT_API int dct_batch_run(const void *workspace, int32_t grid, uint64_t *sse_dev, void *stream);
DCT_API int dct_batch_run_threads(const void *workspace, int32_t grid, int32_t threads, uint64_t *sse_dev,
                                  void *stream);
DCT_API int dct_batch_release(const void *workspace);

/* Learned deblocking post-filter for decoded planes.  The paper's decoded images
 * carry the blocking of 8x8 transform coding (Sec. 4, Tables 3-4); this network
 * reduces it after dct_codec.  With x = p / 255 for the decoded pixels p:
 *   a1 = relu(conv(x; W1, b1))  1 -> 32 channels,  a2 = relu(conv(a1; W2, b2))  32 -> 32,
 *   a3 = relu(conv(a2; W3, b3)) 32 -> 32,          y = x + conv(a3; W4, b4)     32 -> 1,
 * conv a 3x3 cross-correlation, zero outside each image; output pixel
 * clamp(floor(255 y + 1/2), 0, 255).  Parameters: 19105 float32 in the order W1
 * [32][1][3][3], b1 [32], W2 [32][32][3][3], b2 [32], W3 [32][32][3][3], b3 [32],
 * W4 [1][32][3][3], b4 [1] (device memory, caller-owned); kernels use them rounded
 * to FP16, store activations as FP16 and accumulate in FP32.  With W4 and b4 zero
 * the filter returns its input bit for bit.
 *
 * Training works on an image set: n images (crops) of h x w whose top-left corners
 * are pos[2k], pos[2k+1] (row, col; int32 device array) in planes of plane_w x
 * plane_h pixels and pitch `stride`; pos = NULL means one image at (0, 0).  Pixels
 * of a crop outside the plane read as 0.  The loss is the mean over all n h w
 * pixels of (y - original / 255)^2.
 *
 * dct_deblock_nparam: 19105.
 * dct_deblock_workspace_size: device workspace bytes for npix = n h w pixels
 *   (training != 0: for dct_deblock_forward / dct_deblock_grad; 0: for
 *   dct_deblock_apply with npix = W H); 0 if npix is out of range.
 * dct_deblock_apply: filters one decoded W x H plane into `out`.
 * dct_deblock_apply_stack: the same for n decoded W x H images stacked
 *   vertically in one plane (image k at rows k H .. k H + H - 1 of `decoded` and
 *   of `out`), each filtered on its own (zeros outside it), in one launch whose
 *   tiles run over all n images; bit for bit n dct_deblock_apply calls.  Its
 *   workspace is dct_deblock_apply's for npix = W H.
 * dct_deblock_forward: y (float32 device array [n][h][w]) of an image set.
 * dct_deblock_grad: the gradient of the loss (float32 device array [19105],
 *   overwritten) and the loss (*loss, one double in device memory).
 * dct_deblock_adam: one Adam step (bias-corrected, step counted from 1) on the
 *   parameters with moments m, v (float32 device arrays [19105]) and `grad`.
 * Workspaces are 256-byte aligned device memory owned by the caller. */
DCT_API int32_t dct_deblock_nparam(void);
DCT_API size_t dct_deblock_workspace_size(int64_t npix, int32_t training);
DCT_API int dct_deblock_apply(const uint8_t *decoded, int32_t W, int32_t H, int32_t stride, const float *params,
                              uint8_t *out, int32_t out_stride, void *workspace, size_t workspace_bytes, void *stream);
DCT_API int dct_deblock_apply_stack(const uint8_t *decoded, int32_t W, int32_t H, int32_t n, int32_t stride,
                                    const float *params, uint8_t *out, int32_t out_stride, void *workspace,
                                    size_t workspace_bytes, void *stream);
DCT_API int dct_deblock_forward(const uint8_t *decoded, int32_t plane_w, int32_t plane_h, int32_t stride,
                                const int32_t *pos, int32_t n, int32_t h, int32_t w, const float *params, float *y,
                                void *workspace, size_t workspace_bytes, void *stream);
DCT_API int dct_deblock_grad(const uint8_t *decoded, const uint8_t *original, int32_t plane_w, int32_t plane_h,
                             int32_t stride, const int32_t *pos, int32_t n, int32_t h, int32_t w,
                             const float *params, float *grad, double *loss, void *workspace,
                             size_t workspace_bytes, void *stream);
DCT_API int dct_deblock_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr,
                             float beta1, float beta2, float eps, void *stream);

/* Initial parameters of the deblocking network from a seed (params: float32
 * device array [19105], overwritten): He-normal weights, N(0, 2 / (9 C_in)), for
 * the three ReLU layers, zero biases, and a zero output layer, so that the
 * untrained filter returns its input bit for bit.  The normal values come from
 * the counter-based generator Philox4x32-10 (Salmon et al., SC 2011) with key
 * (seed mod 2^32, seed >> 32) and counter (k, 0, 0, 0) for parameter k, through
 * the Box-Muller transform of its first two words: u1 = (x0 + 1) 2^-32,
 * u2 = x1 2^-32, z = sqrt(-2 ln u1) cos(2 pi u2).  The same seed gives the same
 * parameters on every device. */
DCT_API int dct_deblock_init(uint64_t seed, float *params, void *stream);

/* The fallback rule of the learned filter: the trained filter is kept only if it
 * raises the mean PSNR (eq. (23), Sec. 4.1) of a validation set over the plain
 * decoded images.  sse_plain[k] and sse_filtered[k] (device, n uint64 each) are
 * the SSEs of image k's decoded and filtered planes against its original; the
 * gain of image k is 10 log10(sse_plain[k] / sse_filtered[k]) (its size and peak
 * cancel; +inf when the filtered SSE is 0, 0 when both are).  If the mean gain
 * is not above 0, the output layer of params (device) is zeroed, so that the
 * filter returns the decoded image bit for bit.  mean_gain_host and kept_host
 * (host, each may be NULL) get the mean gain in dB and 1 if the filter was kept.
 * Waits for `stream` (it reads the SSEs back to the host). */
DCT_API int dct_deblock_select(const uint64_t *sse_plain, const uint64_t *sse_filtered, int32_t n, float *params,
                               double *mean_gain_host, int32_t *kept_host, void *stream);

/* Three-channel images through the matrix-form codec in one pass: each pixel of
 * the interleaved RGB image is converted as dct_rgb_to_ycbcr does, each of the
 * three planes is coded as dct_codec_float does (form DCT_FORM_MFMA_F16 or
 * DCT_FORM_MFMA_BF16 only), and the reconstructions are written to y, cb, cr
 * (W x H planes, row pitch plane_stride).  sse_dev (device, three uint64) is
 * overwritten with each plane's SSE against its converted values.  Bit for bit
 * the result of dct_rgb_to_ycbcr followed by dct_codec_float on each plane,
 * without writing or reading the converted planes. */
DCT_API int dct_codec_rgb_float(const uint8_t *rgb, int32_t W, int32_t H, int32_t rgb_stride, int32_t form, int32_t qs,
                                uint8_t *y, uint8_t *cb, uint8_t *cr, int32_t plane_stride, uint64_t *sse_dev,
                                void *stream);

/* Recipe parameters (host outs): CORDIC micro-rotations n, fractional bits F of
 * the samples, fractional bits P of the gain constants. */
DCT_API int dct_recipe_info(int32_t *n_iter, int32_t *frac_bits, int32_t *comp_bits);

/* Recipe constants (host outs), derived by the library at compile time:
 *   directions  3 * n values in {-1, +1}: the CORDIC directions d_i of the
 *               pi/16, 3pi/16 and 6pi/16 rotation blocks, in that order;
 *   gains       4 values: M(pi/16), M(3pi/16), M(6pi/16) (including the sqrt(2)
 *               of the even rotation), and round(sqrt(2) 2^P). */
DCT_API int dct_recipe_tables(int32_t *directions, int32_t *gains);

/* Not an operation of the codec, a measurement aid: copies `bytes` bytes from
 * src to dst (device, 16-byte aligned, not overlapping; bytes a non-negative
 * multiple of 16), one 16-byte word per lane with non-temporal loads and stores,
 * enqueued on `stream`.  Timed, it gives the HBM bandwidth that a pure
 * read-once, write-once stream reaches, the practical ceiling beside which the
 * codec kernels' bandwidth is read.  DCT_ERR_INVALID for a null, misaligned or
 * overlapping buffer or a bad size; 0 bytes is DCT_OK with nothing enqueued,
 * whatever the pointers. */
DCT_API int dct_probe_copy(const void *src, void *dst, int64_t bytes, void *stream);

/* Human-readable name of a dct_status value (static storage). */
DCT_API const char *dct_status_string(int status);

/* Releases the library's per-device scratch words (device and pinned host).
 * Optional; later calls allocate them again. */
DCT_API int dct_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* DCTCODEC_H */
