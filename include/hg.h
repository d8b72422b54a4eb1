/*
 * hg.h -- C ABI of the MI355X (gfx950) hash-grid secondary-ray renderer.
 *
 * The library implements the hash-grid renderer of "Baking Relightable NeRF
 * for Real-time Direct/Indirect Illumination Rendering" (arXiv 2409.10327):
 * a multi-resolution hash-grid encoder H, a BRDF decoder B and an implicit
 * ray tracer I (Sec. 3.2), one recursive bounce at the secondary point
 * x' = x + t w (Sec. 3.1), and the Monte Carlo rendering equation over an
 * equirectangular environment map (Eq. 1, Eq. 2, Sec. 2.2), plus the
 * hand-written backward, L2 loss and Adam used to distil it (Sec. 3.3).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers (HBM), caller-allocated,
 *     contiguous, row-major, at least 16-byte aligned (FP16/BF16 tables and
 *     weights included; only the shadow written by hg_adam_step needs just
 *     8 bytes).  Descriptor structs are HOST memory, read only during the
 *     call.  The one host array argument is hg_env_build_sampling's map.
 *   - Work is enqueued asynchronously on `stream`; nothing synchronises
 *     except hg_env_build_sampling (once per environment map).
 *   - No call allocates device memory; gradients are accumulated (+=) into
 *     caller buffers, so the caller zeroes them between steps.
 *   - Return value: HG_OK, or an error code with no work enqueued
 *     (HG_E_INVALID / HG_E_UNSUPPORTED: argument validation on the host) or
 *     HG_E_HIP (a launch failed).  hg_last_error() gives a message for the
 *     calling thread's last failure.  n == 0 is a valid no-op.
 *   - Supported shapes: F = 2 features per level, L = 16 levels, hidden
 *     width 64, decoder 32->64->64->5, tracer 35->64->64->2 (the decoder and
 *     tracer of Sec. 3.2 with 3 layers of width 64, Sec. 4.1), log2_T in
 *     [10, 24], per-level resolutions strictly increasing in [2, 2^20],
 *     box extent a power of two, n_dirs and n_dirs2 powers of two in
 *     [1, 1024] and [1, 64].
 *   - Precision pairs: FP32 tables with FP32 MLP weights (plain path); FP16
 *     tables with BF16 MLP weights (mixed path: BF16 matrix-core products,
 *     FP32 accumulation, FP32 interpolation, compensated FP32 sums over light
 *     directions).  The backward also accepts FP16 tables with FP32 weights.
 */
#ifndef HG_H
#define HG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HG_OK = 0,
    HG_E_INVALID = 1,     /* malformed argument (NULL, size, alignment, shape) */
    HG_E_UNSUPPORTED = 2, /* well-formed but not built (shape, dtype pair) */
    HG_E_WORKSPACE = 3,   /* a workspace cannot hold what the call needs */
    HG_E_HIP = 4          /* a HIP launch or runtime call failed */
} hg_status;

typedef enum { HG_F32 = 0, HG_F16 = 1, HG_BF16 = 2 } hg_dtype;

/* hg_sampling.flags */
#define HG_DIFFUSE_ONLY 1u /* f_r = albedo/pi (furnace tests) */
#define HG_HARD_VIS 2u     /* binary visibility v = [o0 > 0]; the bounce runs only for shadow
                              rays and sums visible secondary rays only (Sec. 3.2 "Overview");
                              forward only */
#define HG_MIS 4u          /* shade mode: the n_dirs = 2M primary directions are M light-importance
                              rays and M GGX visible-normal rays, weighted by the balance heuristic
                              (Sec. 4.1); needs hg_env.dist; forward only */

/* Multi-resolution hash grid (Sec. 3.2, InstantNGP layout).
 * L in [1, 16] levels (16 in the benchmark model, 14 in the paper's, Sec. 4.1),
 * F = 2, table: [L][T][F], T = 2^log2_T, entries FP32 or FP16.
 * res[l]: resolution N_l of level l (host-computed integers).
 * A position x maps to u = clamp((x - box_lo) / box_extent, 0, 1); the
 * subtraction is rounded to FP32 and box_extent is a power of two.  Level l
 * uses cell c = min(floor(u N_l), N_l - 1), fractional weights w = u N_l - c
 * (cell chosen from the exact product), vertex index dense row-major when
 * (N_l+1)^3 <= T, else the spatial hash of Mueller et al. 2022 (Eq. 4),
 * primes (1, 2654435761, 805459861) masked to T.  Features are trilinear
 * blends, concatenated level-major: f[l*F + k]. */
typedef struct {
    int32_t L, F, log2_T;
    int32_t res[32];
    float box_lo, box_extent;
    hg_dtype dtype;
    const void *table;
} hg_grid;

/* Three-layer ReLU MLP n_in -> n_hidden -> n_hidden -> n_out (n_hidden = 64).
 * W[k]: [out][in] (FP32 or BF16), b[k]: [out] FP32.
 * Input layout: the renderer feeds the MLPs 16 level slots of F = 2 features
 * whatever L is, so the decoder has n_in = 32 and the tracer n_in = 35
 * (slots, then the direction).  With L < 16 the slots of levels L..15 carry
 * zero features: the weight columns of those slots have no effect (callers
 * store zeros there) and receive zero gradients. */
typedef struct {
    int32_t n_in, n_hidden, n_out;
    hg_dtype dtype;
    const void *W[3];
    const float *b[3];
} hg_mlp;

/* The hash renderer: grid, BRDF decoder B (outputs: albedo logits 0..2,
 * roughness logit 3 -> 0.09 + 0.91 sigmoid, metallic logit 4 -> sigmoid;
 * n_out = 8 adds the paper's normal head, outputs 5..7 -> n / |n|, which
 * orients the bounce point's hemisphere and BRDF, forward only) and
 * tracer I (input [f, w]; output 0 -> visibility sigmoid, output 1 -> depth
 * d = min(softplus, 1), t = t_near + (t_far - t_near) d).  f0 is the
 * dielectric Fresnel reflectance (0.04 in the paper, Sec. 5). */
typedef struct {
    hg_grid grid;
    hg_mlp brdf, irt;
    float t_near, t_far, f0;
} hg_model;

/* Equirectangular HDR map [H][W][3] FP32; y is up, row 0 at the zenith,
 * azimuth atan2(w_z, w_x) from -pi at column 0; bilinear lookup at texel
 * centres, columns wrap, rows clamp (Sec. 2.2, image-based lighting).
 * dist: the map's light-sampling distribution written by
 * hg_env_build_sampling (device memory); read only under HG_MIS, may be NULL
 * otherwise. */
typedef struct {
    int32_t H, W;
    const float *rgb;
    const void *dist;
} hg_env;

/* Light-importance distribution of an environment map for HG_MIS (Sec. 4.1:
 * one light-importance ray per primary point).  Piecewise constant in solid
 * angle: texel (y, x) covers theta in [pi y/H, pi (y+1)/H] and phi in
 * [-pi + 2 pi x/W, -pi + 2 pi (x+1)/W]; its probability is proportional to
 * its Rec. 709 luminance times its solid angle, and inside a texel the
 * direction is uniform in solid angle.  An all-black map gives the uniform
 * sphere.  Built once per map on the HOST in double precision from
 * rgb_host (host memory, [H][W][3] FP32, the same values as hg_env.rgb),
 * then copied to `dist` (device memory, 16-byte aligned, at least
 * hg_env_sampling_size(H, W) bytes) on `stream`; the call waits for that
 * copy (it synchronises `stream`) and must be repeated when the map
 * changes.  Device layout, all single precision: per row float4 (cos theta
 * at the top edge, 1 - that cosine, 1 + the cosine at the bottom edge,
 * top minus bottom cosine) [H]; marginal CDF over rows [H+1] and
 * conditional CDFs over the columns of each row [H][W+1] as float2
 * (hi, lo) with hi + lo the double value to 2^-48 relative; texel densities
 * per steradian [H][W].  Errors (HG_E_INVALID, nothing copied): NULL
 * pointers, H or W < 1 or above 8192, dist not 16-byte aligned, bytes too
 * small; HG_E_HIP if the copy fails. */
size_t hg_env_sampling_size(int32_t H, int32_t W);
hg_status hg_env_build_sampling(const float *rgb_host, int32_t H, int32_t W, void *dist, size_t bytes,
                                hipStream_t stream);

/* Light sampling: n_dirs stratified cosine-weighted directions per primary
 * point and n_dirs2 per secondary point (8 in the paper's renderer,
 * supplementary "Rendering Details").  The uniforms come from
 * Philox4x32-10 (key = seed, counter = (point, primary direction index or 0,
 * sample >> 2, 0 primary / 1 secondary), 16-bit halves of word sample & 3).
 * Under HG_MIS, primary direction i < M is light sample k = i (counter tag
 * 2) and direction i >= M GGX sample k = i - M (tag 3), each strategy
 * stratified over its M samples like the cosine sampler; direction i
 * carries the weight 2 f_r (n.w_i) / (p_env(w_i) + p_ggx(w_i)) in place of
 * pi f_r.  The GGX rays sample the visible normals of the decoder's
 * roughness (alpha = r^2; Heitz, JCGT 2018) for the view w_o with its
 * normal component clamped to 1e-4. */
typedef struct {
    int32_t n_dirs, n_dirs2;
    uint64_t seed;
    uint32_t flags;
} hg_sampling;

/* Points, each [n][3] FP32 on the device.
 * Shade mode (dir == NULL): pos, nrm (unit normal), wo (unit direction to
 * the viewer) of primary surface points.
 * Query mode (dir != NULL): pos and a unit direction per query; nrm and wo
 * are ignored. */
typedef struct {
    int64_t n;
    const float *pos, *nrm, *wo, *dir;
} hg_points;

/* f = H(x) (Sec. 3.2, "Indirect Illumination Renderer").
 * pos [n][3] FP32 -> feat [n][L*F] FP32. */
hg_status hg_encode(const hg_grid *grid, const float *pos, int64_t n, float *feat,
                    hipStream_t stream);

/* Index stage of H for inspection and bit-exact testing: for each point and
 * level, the table indices of the 8 cell corners (corner bit 0 = +x, bit 1 =
 * +y, bit 2 = +z) and the in-cell weights w = u N_l - c.
 * pos [n][3] FP32 -> idx [n][L][8] uint32, w [n][L][3] FP32 (w may be NULL). */
hg_status hg_encode_index(const hg_grid *grid, const float *pos, int64_t n, uint32_t *idx, float *w,
                          hipStream_t stream);

/* Direct illumination with shadows ("d" rows of Table 3): Eq. (1) with the
 * incoming radiance V(x, w_i) L_env(w_i), V from the tracer.
 * Shade mode: rgb [n][3] = 1/N sum_i pi f_r(x; w_i, w_o) V_i L_env(w_i);
 *   vis, depth (optional, may be NULL) [n][n_dirs] receive V_i and d_i.
 * Query mode: rgb [n][3] = V L_env(dir), vis [n] = V, depth [n] = d. */
hg_status hg_render_direct(const hg_model *model, const hg_env *env, const hg_sampling *samp,
                           const hg_points *pts, float *rgb, float *vis, float *depth,
                           hipStream_t stream);

/* Direct + one indirect bounce ("d+id" rows of Table 3): the incoming
 * radiance of Eq. (2), L_in = V L_env(w) + (1 - V) L'_o, with
 * L'_o = 1/N' sum_j pi f_r(x'; w'_j, -w) V'_j L_env(w'_j) at
 * x' = x + t w, (a', r', m') = B(H(x')), normal n' = -w (facing) or the
 * decoder's normal head, view -w,
 * V'_j = sigmoid(I(H(x'), w'_j)_0) (Sec. 3.1, Sec. 3.2 "Overview").
 * Outputs as for hg_render_direct; in query mode rgb = L_in. */
hg_status hg_render_indirect(const hg_model *model, const hg_env *env, const hg_sampling *samp,
                             const hg_points *pts, float *rgb, float *vis, float *depth,
                             hipStream_t stream);

/* Workspace bytes hg_backward needs for n queries: per encoding the loss
 * depends on (x, and with the bounce also x') one record of 160 bytes
 * (the point, the feature gradient there, a sort key and an index, and
 * their sorted copies), plus the radix sort's temporary storage, the
 * BF16 weight tiles of the mixed backward (66 KiB) and 128 replicated
 * accumulators of the MLP gradients (6.5 MiB).  0 for n <= 0, n >= 2^30 or
 * indirect not 0/1. */
size_t hg_backward_workspace_size(int32_t indirect, int64_t n);

/* Backward of query mode (the distillation forward, Sec. 3.3), with the
 * bounce activations recomputed, not stored.  Given upstream gradients
 * g_rgb [n][3], g_vis [n], g_depth [n], ADDS the gradients of
 * sum_p (g_rgb.rgb + g_vis vis + g_depth depth) to
 *   g_table [L][T][F] FP32 (atomic scatter-add through the trilinear weights),
 *   g_brdf[6], g_irt[6]: FP32 W0,b0,W1,b1,W2,b2 of decoder and tracer,
 * and WRITES d/dpos into g_pos [n][3] if it is not NULL.
 * indirect selects the query mode of hg_render_indirect (1) or
 * hg_render_direct (0).  Precisions (table, MLP weights): (FP32, FP32);
 * (FP16, FP32): the FP32 MLP arithmetic on FP16 tables; (FP16, BF16): the
 * mixed path, the MLP products in BF16 on the matrix cores with FP32
 * accumulation (weights the BF16 shadows, activations and deltas packed to
 * BF16), the gradient arrays FP32 in every case.  Biases are FP32 in all.
 * Accumulation order of the atomics is unspecified.  Each wave first adds
 * its MLP weight gradients into one of 128 copies in the workspace (so that
 * the waves' atomics do not all meet on one address); the copies' sum is
 * then added to g_brdf / g_irt on the same stream.
 * ws: device workspace of at least hg_backward_workspace_size(indirect, n)
 * bytes, 256-byte aligned; its contents on entry are ignored.  The table
 * gradient is scattered after sorting the encodings' points by a Morton
 * key, so that a wave's contributions share cells and merge before the
 * atomics (all of it on `stream`).  Errors: HG_E_INVALID for a missing,
 * misaligned or small workspace; HG_E_WORKSPACE if the sort would need more
 * temporary storage than the size query reserved. */
hg_status hg_backward(const hg_model *model, const hg_env *env, const hg_sampling *samp,
                      const hg_points *pts, int32_t indirect, const float *g_rgb,
                      const float *g_vis, const float *g_depth, float *g_table,
                      float *const g_brdf[6], float *const g_irt[6], float *g_pos,
                      void *ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes hg_morton_order needs for n points: two 8-byte keys and a
 * 4-byte index per point, plus the radix sort's temporary storage.  0 for
 * n <= 0 or n >= 2^31. */
size_t hg_morton_order_workspace_size(int64_t n);

/* Order of n points along a Z-order (Morton) curve over the grid's domain
 * box: a locality aid for the random batches of the distillation step
 * (Sec. 3.3), not part of the method.  A batch rendered and differentiated
 * in this order gives each wave neighbouring points, whose table gathers and
 * gradient adds share cells and cache lines.  pos [n][3] FP32 device; the
 * cell along an axis is trunc((p - box_lo) * 2^21 / box_extent) clamped to
 * [0, 2^21 - 1] (FP32 arithmetic; a NaN coordinate takes cell 0), the key
 * interleaves the bits of the x, y, z cells (x lowest), and the sort is
 * stable.  Writes perm [n] (int32): perm[i] is the index of the i-th point
 * in key order, equal keys in ascending index.  box_lo, box_extent as in
 * hg_grid (extent a power of two).  ws: device workspace of at least
 * hg_morton_order_workspace_size(n) bytes, 256-byte aligned, contents on
 * entry ignored.  Errors: HG_E_INVALID for n outside [0, 2^31 - 1], a bad
 * box, a missing or misaligned pointer or a small workspace; HG_E_WORKSPACE
 * if the sort would need more temporary storage than the size query
 * reserved.  n = 0 returns HG_OK without touching the pointers. */
hg_status hg_morton_order(const float *pos, int64_t n, float box_lo, float box_extent, int32_t *perm,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/* L2 distillation loss (squared-error reading of Sec. 3.3's losses):
 *   loss = 1/n sum_p [ |rgb_p - t_p[0:3]|^2 + (vis_p - t_p[3])^2 +
 *                      (depth_p - t_p[4])^2 ],
 * tgt [n][5].  Writes loss [1] (FP32 sum order unspecified) and the
 * gradients g_rgb [n][3], g_vis [n], g_depth [n] (elementwise, exact
 * order). */
hg_status hg_l2_loss(const float *rgb, const float *vis, const float *depth, const float *tgt,
                     int64_t n, float *loss, float *g_rgb, float *g_vis, float *g_depth,
                     hipStream_t stream);

/* One Adam step (Kingma & Ba) with bias correction, weight decay added to
 * the gradient (the paper trains with Adam, lr 2e-3, weight decay 1e-6 on
 * the MLPs; supplementary training details).  step >= 1.  Updates param,
 * m, v in place (FP32).  If shadow != NULL, also writes the updated
 * parameters rounded to nearest-even in shadow_dtype (HG_F16 for tables,
 * HG_BF16 for MLP weights). */
hg_status hg_adam_step(float *param, const float *grad, float *m, float *v, int64_t n,
                       int32_t step, float lr, float beta1, float beta2, float eps,
                       float weight_decay, void *shadow, hg_dtype shadow_dtype,
                       hipStream_t stream);

/* One tensor of hg_adam_step_multi: the arrays and size of one
 * hg_adam_step call, its weight decay and optional shadow. */
#define HG_ADAM_MAX_TENSORS 16
typedef struct hg_adam_tensor {
    float *param;
    float *grad;
    float *m;
    float *v;
    int64_t n;
    float weight_decay;
    hg_dtype shadow_dtype; /* HG_F16 or HG_BF16 when shadow is not NULL */
    void *shadow;
} hg_adam_tensor;

/* The Adam step of hg_adam_step for up to HG_ADAM_MAX_TENSORS tensors (the
 * table and the twelve MLP arrays of a model) in one launch, with the same
 * arithmetic per element (bit-identical results).  With zero_grad = 1 each
 * gradient is cleared after it is read, so the next hg_backward can add
 * into it without a separate clearing pass.  tensors: HOST array of count
 * descriptors.  Errors: HG_E_INVALID for count outside [0, 16], zero_grad
 * not 0/1, step < 1, betas outside [0, 1), a non-finite hyper-parameter or
 * weight decay, n outside [0, 2^36], a missing or misaligned array, a bad
 * shadow dtype.  count = 0 returns HG_OK. */
hg_status hg_adam_step_multi(const hg_adam_tensor *tensors, int32_t count, int32_t step, float lr,
                             float beta1, float beta2, float eps, int32_t zero_grad,
                             hipStream_t stream);

/* Spatial variance-guided a-trous filter of a rendered frame: SVGF without
 * its temporal parts, as the paper applies it to the Monte Carlo result
 * (Sec. 4.1); the depth gradient for the edge-stopping weight is a finite
 * difference of the depth map (supplementary "Rendering Details").
 * rgb, out [H][W][3]; depth [H][W]; nrm [H][W][3] (unit normals).
 * Iteration k uses a 5x5 B3-spline footprint with step 2^k and weights
 *   exp(-|z_p - z_q| / (sigma_z |grad z_p . (p - q)| + 1e-6))
 *   * max(0, n_p . n_q)^sigma_n
 *   * exp(-|l_p - l_q| / (sigma_l sqrt(g3(var)_p) + 1e-10)),
 * luminance l with Rec. 709 weights, variance initialised from 7x7
 * luminance moments and propagated with the squared weights; taps outside
 * the image are dropped.  work: device scratch of at least
 * hg_denoise_workspace_size(H, W) bytes, 16-byte aligned; its contents on
 * entry are ignored.  iterations = 0 copies rgb to out.  Errors
 * (HG_E_INVALID, nothing launched): NULL pointers, H or W < 1,
 * H * W >= 2^28, H > 1048560, iterations outside [0, 10], negative or
 * non-finite sigmas, work_bytes below the workspace size. */
typedef struct {
    int32_t iterations;
    float sigma_z, sigma_n, sigma_l;
} hg_denoise_params;

size_t hg_denoise_workspace_size(int32_t H, int32_t W);
hg_status hg_denoise(const float *rgb, const float *depth, const float *nrm, int32_t H, int32_t W,
                     const hg_denoise_params *params, float *out, void *work, size_t work_bytes,
                     hipStream_t stream);

/* hg_denoise for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same filter and the same kernels as hg_denoise, bit for bit, with the
 * workspace taken from a static device array of the library instead of a
 * caller buffer.  The array holds HG_DENOISE_NOALLOC_MAX_PIXELS pixels
 * (48 MiB); each GPU the call runs on holds its own copy until the process
 * ends.  The call allocates nothing (no hipMalloc, no library allocation);
 * its first call on a device looks up that device's copy of the array.
 * Arguments and errors as hg_denoise, plus HG_E_INVALID (nothing launched)
 * for H * W > HG_DENOISE_NOALLOC_MAX_PIXELS.  The array needs no clearing
 * (every pass writes what the next one reads), but all calls on one GPU
 * share it: calls that overlap in time on one GPU (different streams, or
 * threads without ordering) race and give undefined results. */
#define HG_DENOISE_NOALLOC_MAX_PIXELS 1048576
hg_status hg_denoise_noalloc(const float *rgb, const float *depth, const float *nrm, int32_t H, int32_t W,
                             const hg_denoise_params *params, float *out, hipStream_t stream);

/* Message describing the calling thread's last failed call ("" if none). */
const char *hg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HG_H */
